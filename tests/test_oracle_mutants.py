"""Planted mistakes in the oracle must be caught by its pins.

Each case copies kf_oracle.c, plants one plausible mistake (a dropped term, a
wrong sign, a transposed operand, a wrong index), builds it with gcc into a
temporary library and checks that at least one independent pin fails:
brute-force joint-Gaussian conditioning, the Riccati steady state, RTS = two-
filter agreement, or associativity/fold of the paper's operators.  The
mutants run on the CPU only.
"""
import os
import subprocess

import numpy as np
import pytest
import scipy.linalg

import oracle
import kf_workloads as W
from tests.bruteforce import posteriors
from tests.test_oracle_pins import _rand_model

MUTANTS = {
    "kf_drop_Q": ("for (int i = 0; i < n * n; ++i) Pp[i] += Qk[i];", "(void)Qk;"),
    "kf_innovation_sign": ("v[i] = yk[i] - v[i] - (dk ? dk[i] : 0.0);",
                           "v[i] = yk[i] + v[i] - (dk ? dk[i] : 0.0);"),
    "rts_gain_transposed": ("G[i * n + j] = tmp[j * n + i];", "G[i * n + j] = tmp[i * n + j];"),
    "binfo_IQJ_order": ("mat_mul(n, n, n, J, Qk1, Mi);", "mat_mul(n, n, n, Qk1, J, Mi);"),
    "tf_drop_Peta": ("mat_vec(n, n, Pf, eta + k * n, v);", "memset(v, 0, sizeof(double) * n);"),
    "lemma1_drop_Ci_etaj": ("mat_vec(n, n, Ci, nj, v);", "memset(v, 0, sizeof(double) * n);"),
    "lemma1_untransposed_solve": ("lu_solve_t(n, 1, Mm, piv, w);", "lu_solve(n, 1, Mm, piv, w);"),
    "lemma1_operand_order": ("mat_mul(n, n, n, Aj, X, Ao);", "mat_mul(n, n, n, X, Aj, Ao);"),
    "lemma2_missing_transpose": ("mat_mul_bt(n, n, n, X, Ei, Lo);", "mat_mul(n, n, n, X, Ei, Lo);"),
    "pkf_init1_drop_u": ("bk[i] = (uk1 ? uk1[i] : 0.0) + tv[i];", "bk[i] = tv[i];"),
    "lu_transpose_pivot_order": ("for (int k = n - 1; k >= 0; --k)", "for (int k = 0; k < n; ++k)"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(oracle.source_path()).read()
    assert src.count(old) == 1, name
    path = tmp_path / ("%s.c" % name)
    path.write_text(src.replace(old, new))
    so = tmp_path / ("lib%s.so" % name)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-w", "-o", str(so),
                           str(path), "-lm"])
    return str(so)


def wild_filter_element(rng, n, scale=1.0):
    """A valid filtering element far from identity: random A, b, eta and
    random full-rank PSD C, J, so that I + C_i J_j is far from diagonal and
    its LU factorisation pivots (often with overlapping row swaps)."""
    X = scale * rng.standard_normal((n, n))
    Y = scale * rng.standard_normal((n, n))
    return (rng.standard_normal((n, n)), rng.standard_normal(n), X @ X.T,
            rng.standard_normal(n), Y @ Y.T)


def _pins_pass():
    """Run a compact set of pins; return False as soon as one fails."""
    def close(a, b, tol):
        return np.max(np.abs(np.asarray(a) - np.asarray(b))) <= tol * max(1.0, np.max(np.abs(b)))
    try:
        rng = np.random.default_rng(77)
        T = 7
        F, Q, H, R, m0, P0, u, d = _rand_model(rng, 3, 2, tv=True, T=T, inputs=True)
        y = rng.standard_normal((T, 2))
        bf = posteriors(F, Q, H, R, m0, P0, y, u, d)
        m_f, P_f, m_p, P_p = oracle.kf_filter(F, Q, H, R, m0, P0, y, u, d)
        m_s, P_s = oracle.rts(F, m_f, P_f, m_p, P_p)
        eta, J = oracle.backward_info(F, Q, H, R, y, u, d)
        m_t, P_t = oracle.tf_combine(m_f, P_f, eta, J)
        for a, b in ((m_f, bf["m_f"]), (P_f, bf["P_f"]), (m_s, bf["m_s"]), (P_s, bf["P_s"]),
                     (eta, bf["eta"]), (J, bf["J"]), (m_t, bf["m_s"]), (P_t, bf["P_s"])):
            if not close(a, b, 1e-8):
                return False
        # Riccati steady state on a stable model
        mdl = W.random_stable_model(3, 2, 0.9, 0.2, 0.5, rng)
        yy = W.simulate(mdl, 800, rng)
        _, _, _, Pp = oracle.kf_filter(*mdl.arrays(), yy)
        if not close(Pp[400], scipy.linalg.solve_discrete_are(mdl.F.T, mdl.H.T, mdl.Q, mdl.R), 1e-8):
            return False
        # paper-form fold equals the sequential recursions, with inputs
        pf = oracle.prts(F, Q, H, R, m0, P0, y, u, d)
        if not (close(pf[0], m_f, 1e-9) and close(pf[2], m_s, 1e-9) and close(pf[3], P_s, 1e-9)):
            return False
        pt = oracle.ptfs(F, Q, H, R, m0, P0, y, u, d)
        if not (close(pt[2], m_s, 1e-9) and close(pt[3], P_s, 1e-9)):
            return False
        # a tree-shaped scan combines aggregates on both sides (A, b, C of the
        # right operand matter), which a left or right fold never does
        from oracle import scans
        tree = oracle.prts(F, Q, H, R, m0, P0, y, u, d, scan=scans.ladner_fischer)
        if not all(close(a, b, 1e-9) for a, b in zip(tree, (m_f, P_f, m_s, P_s))):
            return False
        tf = oracle.ptfs(F, Q, H, R, m0, P0, y, u, d, scan=scans.blelloch)
        if not (close(tf[2], m_s, 1e-9) and close(tf[3], P_s, 1e-9)):
            return False
        # associativity on wild elements (large PSD C, J) whose solves pivot
        for n in (3, 4, 4, 4):
            a, b, c = (wild_filter_element(rng, n) for _ in range(3))
            left = oracle.filter_combine(oracle.filter_combine(a, b), c)
            right = oracle.filter_combine(a, oracle.filter_combine(b, c))
            if not all(close(x, z, 1e-10) for x, z in zip(left, right)):
                return False
    except (np.linalg.LinAlgError, ValueError, FloatingPointError):
        return False
    return True


def test_unmutated_oracle_passes_compact_pins():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    so = _build_mutant(tmp_path, name, old, new)
    with oracle.use_library(so):
        caught = not _pins_pass()
    os.remove(so)
    assert caught, "planted mistake %s went unnoticed" % name
