"""The continuous-batching server on the GPU (paper_2511_10363_amd.serving):
a job's results are bit-identical when it runs alone and when it runs inside
a mix of jobs that arrive while batches are in flight on two streams, and
they match the CPU FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle
import kf_workloads as W
from tests.gpu_common import TOL, gpu_available, kfscan, normwise, oracle_inputs_for, torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _jobs(nx, ny, n, seed, lo=6.0, hi=11.5):
    rng = np.random.default_rng(seed)
    out = []
    for T in W.log_uniform_lengths(n, lo, hi, rng):
        m = W.random_stable_model(nx, ny, 0.98, 0.05, 0.2, rng)
        out.append((m, W.simulate(m, T, rng)))
    return out


@pytest.mark.parametrize("nx,ny,prec", [(4, 2, "f32"), (16, 8, "mixed"), (8, 4, "f32")])
def test_alone_and_in_the_mix_are_identical(nx, ny, prec):
    from paper_2511_10363_amd import serving as S
    k = kfscan()
    _say("serving identity", nx, ny, prec)
    jobs = _jobs(nx, ny, 24, seed=nx)
    dt = k.dtype_for(prec)
    ex = S.GpuExecutor(nstreams=2)
    srv = S.Server(ex, rows_per_class=12000, slots_per_class=64, max_batch=8)
    dev_jobs = [(ex.flat_model(m.arrays(), prec), torch.as_tensor(y).to("cuda", dt).contiguous())
                for m, y in jobs]

    def finish(jid):
        while srv.jobs[jid].finished < 0:
            srv.step()
        out = [o.clone() for o in srv.result(jid)]
        srv.release(jid)
        return out

    probe = [3, 10, 17]
    alone = {}
    for i in probe:
        alone[i] = finish(srv.submit(*dev_jobs[i], entry="rts", precision=prec))
    torch.cuda.synchronize()
    # the mix: jobs submitted a few at a time while earlier batches run; the
    # arena (12000 rows) forces admission to wait for rows to free up
    ids = {}
    for s0 in range(0, len(jobs), 5):
        for i in range(s0, min(len(jobs), s0 + 5)):
            ids[srv.submit(*dev_jobs[i], entry="rts", precision=prec)] = i
        srv.step()
        for jid in [j for j in ids if srv.jobs[j].finished >= 0]:
            i = ids.pop(jid)
            out = [o.clone() for o in srv.result(jid)]
            srv.release(jid)
            if i in alone:
                for a, b in zip(alone[i], out):
                    assert torch.equal(a, b), ("job", i)
            alone.setdefault(("mix", i), out)
    while ids:
        srv.step()
        for jid in [j for j in ids if srv.jobs[j].finished >= 0]:
            i = ids.pop(jid)
            out = [o.clone() for o in srv.result(jid)]
            srv.release(jid)
            if i in alone:
                for a, b in zip(alone[i], out):
                    assert torch.equal(a, b), ("job", i)
            alone.setdefault(("mix", i), out)
    batches = {srv.done[-1].batch}
    assert len({j.batch for j in srv.done}) > 3
    del batches
    # and the results are the oracle's
    for i in probe:
        m, y = jobs[i]
        arrs, yy = oracle_inputs_for(m, y, prec)
        ref = oracle.smooth_rts(*arrs, yy)
        for g, r in zip(alone[i], ref):
            assert normwise(g.double().cpu().numpy(), r) <= TOL[prec]
