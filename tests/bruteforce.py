"""Brute-force posteriors from the dense joint Gaussian of a short series.

Written independently of the oracle: the linear-Gaussian model of Sec. III-A
(transition and measurement densities) is unrolled into one linear map from the
independent Gaussian sources (x_0, process noises, measurement noises) to all
states and measurements, and every posterior is read off by plain Gaussian
conditioning.  Only for tiny T (the matrices are dense).
"""
from __future__ import annotations

import numpy as np


def _per_step(a, T, shape):
    a = np.asarray(a, dtype=np.float64)
    if a.shape == shape:
        return [a] * T
    return [a[k] for k in range(T)]


def joint(F, Q, H, R, m0, P0, T, u=None, d=None):
    """Mean and covariance of (x_0..x_T, y_1..y_T), stacked state-major."""
    n = np.asarray(m0).shape[0]
    m = np.asarray(H).shape[-2]
    Fs = _per_step(F, T, (n, n)); Qs = _per_step(Q, T, (n, n))
    Hs = _per_step(H, T, (m, n)); Rs = _per_step(R, T, (m, m))
    us = [np.zeros(n)] * T if u is None else _per_step(u, T, (n,))
    ds = [np.zeros(m)] * T if d is None else _per_step(d, T, (m,))
    nz = n + T * n + T * m                       # sources: x0, w_1..w_T, v_1..v_T
    src_cov = np.zeros((nz, nz))
    src_mean = np.zeros(nz)
    src_cov[:n, :n] = P0
    src_mean[:n] = m0
    for k in range(T):
        o = n + k * n
        src_cov[o:o + n, o:o + n] = Qs[k]
        src_mean[o:o + n] = us[k]                # w_k carries the input u_{k-1}
        o = n + T * n + k * m
        src_cov[o:o + m, o:o + m] = Rs[k]
        src_mean[o:o + m] = ds[k]                # v_k carries the offset d_k
    nv = (T + 1) * n + T * m
    Mx = np.zeros((nv, nz))
    Mx[:n, :n] = np.eye(n)                       # x_0
    for k in range(1, T + 1):                    # x_k = F_{k-1} x_{k-1} + w_k
        rows = slice(k * n, (k + 1) * n)
        Mx[rows] = Fs[k - 1] @ Mx[(k - 1) * n:k * n]
        Mx[rows, n + (k - 1) * n:n + k * n] += np.eye(n)
    for k in range(1, T + 1):                    # y_k = H_k x_k + v_k
        rows = slice((T + 1) * n + (k - 1) * m, (T + 1) * n + k * m)
        Mx[rows] = Hs[k - 1] @ Mx[k * n:(k + 1) * n]
        o = n + T * n + (k - 1) * m
        Mx[rows, o:o + m] += np.eye(m)
    return Mx @ src_mean, Mx @ src_cov @ Mx.T, n, m


def _condition(mu, S, idx_a, idx_b, yb):
    Sab = S[np.ix_(idx_a, idx_b)]
    Sbb = S[np.ix_(idx_b, idx_b)]
    K = np.linalg.solve(Sbb, Sab.T).T
    mean = mu[idx_a] + K @ (yb - mu[idx_b])
    cov = S[np.ix_(idx_a, idx_a)] - K @ Sab.T
    return mean, 0.5 * (cov + cov.T)


def posteriors(F, Q, H, R, m0, P0, y, u=None, d=None):
    """Brute-force filter, smoother and backward-information results.

    Returns dict with m_f, P_f (x_k | y_{1:k}), m_s, P_s (x_k | y_{1:T}) and
    eta, J (information form of p(y_{k+1:T} | x_k), zero at k = T), k = 1..T.
    """
    y = np.asarray(y, dtype=np.float64)
    T = y.shape[0]
    mu, S, n, m = joint(F, Q, H, R, m0, P0, T, u, d)
    xi = lambda k: np.arange(k * n, (k + 1) * n)                      # noqa: E731
    yi = lambda k: np.arange((T + 1) * n + (k - 1) * m, (T + 1) * n + k * m)  # noqa: E731
    out = {key: [] for key in ("m_f", "P_f", "m_s", "P_s", "eta", "J")}
    all_y = np.concatenate([yi(k) for k in range(1, T + 1)])
    for k in range(1, T + 1):
        obs = np.concatenate([yi(j) for j in range(1, k + 1)])
        mf, Pf = _condition(mu, S, xi(k), obs, y[:k].ravel())
        ms, Ps = _condition(mu, S, xi(k), all_y, y.ravel())
        out["m_f"].append(mf); out["P_f"].append(Pf)
        out["m_s"].append(ms); out["P_s"].append(Ps)
        if k == T:
            out["eta"].append(np.zeros(n)); out["J"].append(np.zeros((n, n)))
            continue
        fut = np.concatenate([yi(j) for j in range(k + 1, T + 1)])
        # y_fut | x_k ~ N(a + B x_k, Sigma): regression of y_fut on x_k
        Sxx = S[np.ix_(xi(k), xi(k))]
        Syx = S[np.ix_(fut, xi(k))]
        B = np.linalg.solve(Sxx, Syx.T).T
        a = mu[fut] - B @ mu[xi(k)]
        Sig = S[np.ix_(fut, fut)] - B @ Syx.T
        W = np.linalg.solve(Sig, B)
        out["J"].append(B.T @ W)
        out["eta"].append(W.T @ (y[k:].ravel() - a))
    return {key: np.array(v) for key, v in out.items()}
