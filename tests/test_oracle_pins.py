"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* closed forms: scalar random walk steady state (derived from the Kalman and
  RTS recursions of Sec. III and the two-filter combination);
* library routines: scipy's discrete algebraic Riccati and Lyapunov solvers;
* brute force: dense joint-Gaussian conditioning for short series;
* special cases: Bayesian linear regression (F = I, Q = 0), pure prediction (H = 0);
* invariants: smoother = filter at T, RTS = two-filter, chunked filtering,
  cross-axis independence of the constant-velocity model.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
import kf_workloads as W
from tests.bruteforce import posteriors

RNG_SEED = 7


def _rand_model(rng, n, m, tv=False, T=None, inputs=False):
    def spd(k):
        X = rng.standard_normal((k, k))
        return X @ X.T + 0.3 * np.eye(k)
    if tv:
        F = np.stack([0.9 * np.linalg.qr(rng.standard_normal((n, n)))[0] for _ in range(T)])
        Q = np.stack([spd(n) for _ in range(T)])
        H = rng.standard_normal((T, m, n))
        R = np.stack([spd(m) for _ in range(T)])
    else:
        F = rng.standard_normal((n, n)) * 0.5
        Q = spd(n)
        H = rng.standard_normal((m, n))
        R = spd(m)
    u = d = None
    if inputs:
        u = rng.standard_normal((T, n)) if tv else rng.standard_normal(n)
        d = rng.standard_normal((T, m)) if tv else rng.standard_normal(m)
    m0 = rng.standard_normal(n)
    P0 = spd(n)
    return F, Q, H, R, m0, P0, u, d


def _close(a, b, tol=1e-10):
    a, b = np.asarray(a), np.asarray(b)
    scale = max(1.0, np.max(np.abs(b)))
    assert np.max(np.abs(a - b)) <= tol * scale, np.max(np.abs(a - b)) / scale


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("q,r", [(1.0, 1.0), (0.3, 2.0), (2.5, 0.1)])
def test_scalar_random_walk_steady_state(q, r):
    """F = H = 1: P^-_inf = (q + sqrt(q^2 + 4qr))/2, P_inf = P^-_inf - q,
    interior smoother P_inf P^-_inf / (P_inf + P^-_inf), backward J = 1/P^-_inf."""
    T = 400
    rng = np.random.default_rng(1)
    y = np.cumsum(rng.standard_normal(T)).reshape(T, 1)
    one = np.ones((1, 1))
    args = (one, q * one, one, r * one, np.zeros(1), np.eye(1), y)
    m_f, P_f, m_p, P_p = oracle.kf_filter(*args)
    m_s, P_s = oracle.rts(one, m_f, P_f, m_p, P_p)
    eta, J = oracle.backward_info(one, q * one, one, r * one, y)
    Pm = 0.5 * (q + math.sqrt(q * q + 4 * q * r))
    Pf = Pm - q
    Ps = Pf * Pm / (Pf + Pm)
    mid = slice(T // 4, 3 * T // 4)
    assert np.allclose(P_p[mid, 0, 0], Pm, rtol=1e-12, atol=0)
    assert np.allclose(P_f[mid, 0, 0], Pf, rtol=1e-12, atol=0)
    assert np.allclose(P_s[mid, 0, 0], Ps, rtol=1e-12, atol=0)
    assert np.allclose(J[mid, 0, 0], 1.0 / Pm, rtol=1e-12, atol=0)


def test_golden_ratio_fixture():
    """q = r = 1 gives the golden-ratio constants stored in tests/golden."""
    import json, os
    with open(os.path.join(os.path.dirname(__file__), "golden", "scalar_random_walk.json")) as f:
        g = json.load(f)
    T = 300
    y = np.linspace(0, 1, T).reshape(T, 1)
    one = np.ones((1, 1))
    m_f, P_f, m_p, P_p = oracle.kf_filter(one, one, one, one, np.zeros(1), np.eye(1), y)
    m_s, P_s = oracle.rts(one, m_f, P_f, m_p, P_p)
    k = T // 2
    assert abs(P_p[k, 0, 0] - g["P_pred"]) < 1e-12
    assert abs(P_f[k, 0, 0] - g["P_filt"]) < 1e-12
    assert abs(P_s[k, 0, 0] - g["P_smooth"]) < 1e-12


# --------------------------------------------------------------------------
# library routines
# --------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["cv", "stable4", "stable3x3"])
def test_riccati_and_lyapunov_steady_state(which):
    rng = np.random.default_rng(3)
    if which == "cv":
        mdl = W.cv_model()
    elif which == "stable4":
        mdl = W.random_stable_model(4, 2, 0.95, 0.1, 0.5, rng)
    else:
        mdl = W.random_stable_model(3, 3, 0.9, 0.2, 0.3, rng)
    T = 3000
    y = W.simulate(mdl, T, rng)
    m_f, P_f, m_p, P_p = oracle.kf_filter(*mdl.arrays(), y)
    m_s, P_s = oracle.rts(mdl.F, m_f, P_f, m_p, P_p)
    Pm = scipy.linalg.solve_discrete_are(mdl.F.T, mdl.H.T, mdl.Q, mdl.R)
    _close(P_p[T // 2], Pm, 1e-9)
    # filtered steady state from the predicted one
    S = mdl.H @ Pm @ mdl.H.T + mdl.R
    Pf = Pm - Pm @ mdl.H.T @ np.linalg.solve(S, mdl.H @ Pm)
    _close(P_f[T // 2], Pf, 1e-9)
    # interior smoother covariance solves X = G X G^T + (Pf - G Pm G^T)
    G = Pf @ mdl.F.T @ np.linalg.inv(Pm)
    Xs = scipy.linalg.solve_discrete_lyapunov(G, Pf - G @ Pm @ G.T)
    _close(P_s[T // 2], Xs, 1e-9)


def test_cv_model_steady_state_values():
    """Reading C10 of the tracking model: steady filtered and interior RTS
    variances match the Riccati/Lyapunov solutions to 6 digits."""
    mdl = W.cv_model()
    T = 2000
    y = W.simulate(mdl, T, np.random.default_rng(0))
    m_f, P_f, m_s, P_s = oracle.smooth_rts(*mdl.arrays(), y)
    assert np.allclose(np.diag(P_f[T // 2]), [0.074821, 0.074821, 0.515309, 0.515309], atol=2e-6)
    assert np.allclose(np.diag(P_s[T // 2]), [0.022228, 0.022228, 0.140590, 0.140590], atol=2e-6)


# --------------------------------------------------------------------------
# brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,m,tv,inputs,T", [
    (1, 1, False, False, 6), (2, 1, False, True, 9), (3, 2, True, True, 8),
    (4, 2, False, False, 12), (4, 4, True, False, 7), (2, 3, True, True, 5),
    (3, 1, False, True, 1), (2, 2, True, False, 2)])
def test_bruteforce_joint_gaussian(n, m, tv, inputs, T):
    rng = np.random.default_rng(100 + 10 * n + m + T)
    F, Q, H, R, m0, P0, u, d = _rand_model(rng, n, m, tv, T, inputs)
    y = rng.standard_normal((T, m)) * 2.0
    bf = posteriors(F, Q, H, R, m0, P0, y, u, d)
    m_f, P_f, m_p, P_p = oracle.kf_filter(F, Q, H, R, m0, P0, y, u, d)
    m_s, P_s = oracle.rts(F, m_f, P_f, m_p, P_p)
    eta, J = oracle.backward_info(F, Q, H, R, y, u, d)
    m_t, P_t = oracle.tf_combine(m_f, P_f, eta, J)
    _close(m_f, bf["m_f"], 1e-9); _close(P_f, bf["P_f"], 1e-9)
    _close(m_s, bf["m_s"], 1e-9); _close(P_s, bf["P_s"], 1e-9)
    _close(J, bf["J"], 1e-8); _close(eta, bf["eta"], 1e-8)
    _close(m_t, bf["m_s"], 1e-9); _close(P_t, bf["P_s"], 1e-9)


# --------------------------------------------------------------------------
# special cases
# --------------------------------------------------------------------------

def test_bayesian_linear_regression():
    """F = I, Q = 0: P_k = (P0^-1 + k H^T R^-1 H)^-1,
    m_k = P_k (P0^-1 m0 + H^T R^-1 sum_{i<=k} y_i); smoother = filter at T for all k."""
    rng = np.random.default_rng(11)
    n, m, T = 3, 2, 40
    H = rng.standard_normal((m, n))
    R = np.diag([0.5, 2.0])
    m0 = rng.standard_normal(n)
    P0 = np.diag([3.0, 1.0, 0.5])
    y = rng.standard_normal((T, m))
    m_f, P_f, m_p, P_p = oracle.kf_filter(np.eye(n), np.zeros((n, n)), H, R, m0, P0, y)
    Ri = np.linalg.inv(R)
    csum = np.cumsum(y, axis=0)
    for k in range(1, T + 1):
        Pk = np.linalg.inv(np.linalg.inv(P0) + k * H.T @ Ri @ H)
        mk = Pk @ (np.linalg.solve(P0, m0) + H.T @ Ri @ csum[k - 1])
        _close(P_f[k - 1], Pk, 1e-11)
        _close(m_f[k - 1], mk, 1e-11)
    # Q = 0 makes P_{k+1|k} = P_{k|k}, so RTS reduces to the final posterior everywhere
    m_s, P_s = oracle.rts(np.eye(n), m_f, P_f, m_p, P_p)
    for k in range(T):
        _close(m_s[k], m_f[-1], 1e-9)
        _close(P_s[k], P_f[-1], 1e-9)


def test_pure_prediction():
    """H = 0: the filter only predicts, m_k = F^k m0, P_k = F P_{k-1} F^T + Q,
    and the smoother equals the filter."""
    rng = np.random.default_rng(12)
    n, m, T = 3, 2, 25
    F = 0.9 * np.linalg.qr(rng.standard_normal((n, n)))[0]
    Q = np.diag([0.2, 0.1, 0.3])
    m0 = rng.standard_normal(n)
    P0 = np.eye(n)
    y = rng.standard_normal((T, m))
    m_f, P_f, m_s, P_s = oracle.smooth_rts(F, Q, np.zeros((m, n)), np.eye(m), m0, P0, y)
    x, P = m0.copy(), P0.copy()
    for k in range(T):
        x = F @ x
        P = F @ P @ F.T + Q
        _close(m_f[k], x, 1e-12); _close(P_f[k], P, 1e-12)
    _close(m_s, m_f, 1e-10); _close(P_s, P_f, 1e-10)
    m_f2, P_f2, m_t, P_t = oracle.smooth_twofilter(F, Q, np.zeros((m, n)), np.eye(m), m0, P0, y)
    _close(m_t, m_f, 1e-10); _close(P_t, P_f, 1e-10)


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("inputs", [False, True])
def test_rts_equals_two_filter_and_end_agreement(inputs):
    rng = np.random.default_rng(21)
    T = 300
    F, Q, H, R, m0, P0, u, d = _rand_model(rng, 4, 2, tv=True, T=T, inputs=inputs)
    y = rng.standard_normal((T, 2))
    m_f, P_f, m_s, P_s = oracle.smooth_rts(F, Q, H, R, m0, P0, y, u, d)
    _, _, m_t, P_t = oracle.smooth_twofilter(F, Q, H, R, m0, P0, y, u, d)
    _close(m_t, m_s, 1e-9); _close(P_t, P_s, 1e-9)
    assert np.array_equal(m_s[-1], m_f[-1]) and np.array_equal(P_s[-1], P_f[-1])


def test_chunked_filtering_equals_one_pass():
    """Restarting the filter from (x_{t|t}, P_{t|t}) as the new prior continues it
    exactly (predict-first convention of reading C1)."""
    mdl, y = W.tracking(500, seed=5)
    m_f, P_f, _, _ = oracle.kf_filter(*mdl.arrays(), y)
    t = 173
    m2, P2, _, _ = oracle.kf_filter(mdl.F, mdl.Q, mdl.H, mdl.R, m_f[t - 1], P_f[t - 1], y[t:])
    _close(m2, m_f[t:], 1e-12); _close(P2, P_f[t:], 1e-12)


def test_cv_cross_axis_blocks_are_zero():
    mdl, y = W.tracking(200, seed=9)
    m_f, P_f, m_s, P_s = oracle.smooth_rts(*mdl.arrays(), y)
    for P in (P_f, P_s):
        for i, j in [(0, 1), (0, 3), (1, 2), (2, 3)]:
            assert np.max(np.abs(P[:, i, j])) == 0.0


def test_time_varying_and_shared_model_agree():
    """A per-step model array whose steps are all equal gives the shared-model result."""
    rng = np.random.default_rng(31)
    T = 50
    F, Q, H, R, m0, P0, u, d = _rand_model(rng, 3, 2, tv=False, T=T, inputs=True)
    y = rng.standard_normal((T, 2))
    a = oracle.smooth_rts(F, Q, H, R, m0, P0, y, u, d)
    tile = lambda M: np.repeat(M[None], T, axis=0)           # noqa: E731
    b = oracle.smooth_rts(tile(F), tile(Q), tile(H), tile(R), m0, P0, y, tile(u), tile(d))
    for x1, x2 in zip(a, b):
        assert np.array_equal(x1, x2)


def test_bad_arguments_raise():
    with pytest.raises(ValueError):
        oracle.kf_filter(np.eye(2), np.eye(3), np.eye(2), np.eye(2), np.zeros(2), np.eye(2),
                         np.zeros((5, 2)))
    with pytest.raises(np.linalg.LinAlgError):
        oracle.kf_filter(np.eye(2), np.eye(2), np.eye(2), -np.eye(2), np.zeros(2), np.eye(2),
                         np.zeros((5, 2)))
