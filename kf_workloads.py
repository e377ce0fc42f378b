"""Seeded synthetic inputs for the Kalman filter/smoother workloads.

This module holds model definitions and data simulation only -- none of the
filtering or smoothing arithmetic.  Both the CPU oracle (through the tests and
the benchmark) and the GPU path consume the arrays it returns; neither side
imports the other.

The paper (Sarkka & Garcia-Fernandez, arXiv 2511.10363, Sec. VI-A) evaluates
on synthetic data simulated from the model; no public dataset is involved.
Model readings (stated in the design notes):

* ``cv_model``      -- constant-velocity 2-D tracking, state (x, y, vx, vy),
  F = [[I, dt I], [0, I]], continuous white-noise-acceleration
  Q = q [[dt^3/3, dt^2/2], [dt^2/2, dt]] (x) I_2, position-only H = [I 0],
  R = r I, m0 = 0, P0 = I.
* ``random_stable_model`` -- F = rho G / spectral_radius(G) with G standard
  Gaussian, H standard Gaussian (ny x nx), Q = q I, R = r I, m0 = 0, P0 = I.
* ``paper_tv_model`` -- the time-varying model of Sec. VI-A: per step Gaussian
  F_k replaced by 0.99 times the Q factor of its QR factorisation, Gaussian u_k,
  H_k, d_k, and Q_k = Xi Xi^T, R_k = Xi Xi^T with Gaussian Xi; random m0, P0.
* ``simulate``      -- x_0 ~ N(m0, P0), x_k = F x_{k-1} + u_{k-1} + q_k,
  y_k = H x_k + d_k + r_k for k = 1..T.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Model:
    F: np.ndarray
    Q: np.ndarray
    H: np.ndarray
    R: np.ndarray
    m0: np.ndarray
    P0: np.ndarray
    u: np.ndarray | None = None
    d: np.ndarray | None = None
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def nx(self) -> int:
        return self.F.shape[-1]

    @property
    def ny(self) -> int:
        return self.H.shape[-2]

    def arrays(self):
        return self.F, self.Q, self.H, self.R, self.m0, self.P0


def cv_model(dt: float = 0.1, q: float = 1.0, r: float = 0.25) -> Model:
    I2 = np.eye(2)
    Z2 = np.zeros((2, 2))
    F = np.block([[I2, dt * I2], [Z2, I2]])
    Q = q * np.kron(np.array([[dt ** 3 / 3.0, dt ** 2 / 2.0], [dt ** 2 / 2.0, dt]]), I2)
    H = np.hstack([I2, Z2])
    R = r * I2
    return Model(F, Q, H, R, np.zeros(4), np.eye(4), name="cv2d",
                 extra=dict(dt=dt, q=q, r=r))


def random_stable_model(nx: int, ny: int, rho: float, q: float, r: float,
                        rng: np.random.Generator) -> Model:
    G = rng.standard_normal((nx, nx))
    rad = max(abs(np.linalg.eigvals(G)))
    F = rho * G / rad
    H = rng.standard_normal((ny, nx))
    return Model(F, q * np.eye(nx), H, r * np.eye(ny), np.zeros(nx), np.eye(nx),
                 name="stable_rho%g" % rho, extra=dict(rho=rho, q=q, r=r))


def _rand_spd(rng, n, count=None):
    shape = (n, n) if count is None else (count, n, n)
    Xi = rng.standard_normal(shape)
    return Xi @ np.swapaxes(Xi, -1, -2)


def paper_tv_model(T: int, rng: np.random.Generator, nx: int = 4, ny: int = 2) -> Model:
    G = rng.standard_normal((T, nx, nx))
    Qf, _ = np.linalg.qr(G)
    F = 0.99 * Qf
    u = rng.standard_normal((T, nx))
    H = rng.standard_normal((T, ny, nx))
    d = rng.standard_normal((T, ny))
    Q = _rand_spd(rng, nx, T)
    R = _rand_spd(rng, ny, T)
    m0 = rng.standard_normal(nx)
    P0 = _rand_spd(rng, nx)
    return Model(F, Q, H, R, m0, P0, u=u, d=d, name="paper_tv")


def _chol(S):
    return np.linalg.cholesky(S + 0.0 * np.eye(S.shape[-1]))


def simulate(model: Model, T: int, rng: np.random.Generator, return_states: bool = False):
    """Simulate y_{1:T} (and optionally x_{0:T}) from ``model``."""
    nx, ny = model.nx, model.ny
    x0 = model.m0 + _chol(model.P0) @ rng.standard_normal(nx)
    tv = model.F.ndim == 3
    if tv:
        x = np.empty((T + 1, nx))
        x[0] = x0
        LQ = np.linalg.cholesky(model.Q[:T])
        LR = np.linalg.cholesky(model.R[:T])
        wq = np.einsum("kij,kj->ki", LQ, rng.standard_normal((T, nx)))
        wr = np.einsum("kij,kj->ki", LR, rng.standard_normal((T, ny)))
        for k in range(1, T + 1):
            x[k] = model.F[k - 1] @ x[k - 1] + model.u[k - 1] + wq[k - 1]
        y = np.einsum("kij,kj->ki", model.H[:T], x[1:]) + model.d[:T] + wr
    else:
        w = np.empty((T + 1, nx))
        w[0] = x0
        w[1:] = rng.standard_normal((T, nx)) @ _chol(model.Q).T
        if model.u is not None:
            w[1:] += model.u if model.u.ndim == 1 else model.u[:T]
        # x_k = sum_j F^{k-j} w_j by recursive doubling (vectorised, exact up to rounding)
        x = w.copy()
        Fp = model.F.copy()
        s = 1
        while s <= T:
            x[s:] = x[s:] + x[:-s] @ Fp.T
            Fp = Fp @ Fp
            s *= 2
        y = x[1:] @ model.H.T + rng.standard_normal((T, ny)) @ _chol(model.R).T
        if model.d is not None:
            y += model.d if model.d.ndim == 1 else model.d[:T]
    return (y, x) if return_states else y


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def tracking(T: int, seed: int = 20251110):
    """Constant-velocity tracking model with T simulated measurements."""
    rng = np.random.default_rng(seed)
    model = cv_model()
    y = simulate(model, T, rng)
    return model, y


def ragged_batch(nseq: int = 4096, log2_lo: float = 6.0, log2_hi: float = 14.0,
                 nx_choices=(2, 4, 8), rho: float = 0.95, q: float = 0.1, r: float = 0.5,
                 seed: int = 4096):
    """Uneven batch: T_i = round(2^U), U ~ Uniform[log2_lo, log2_hi]; nx_i uniform
    on ``nx_choices`` with ny = nx/2; one random stable model per sequence."""
    rng = np.random.default_rng(seed)
    seqs = []
    for _ in range(nseq):
        T = int(round(2.0 ** rng.uniform(log2_lo, log2_hi)))
        nx = int(rng.choice(nx_choices))
        ny = max(1, nx // 2)
        model = random_stable_model(nx, ny, rho, q, r, rng)
        y = simulate(model, T, rng)
        seqs.append((model, y))
    return seqs


def log_uniform_lengths(count: int, log2_lo: float, log2_hi: float, rng) -> list[int]:
    return [int(round(2.0 ** rng.uniform(log2_lo, log2_hi))) for _ in range(count)]


def poisson_arrivals(count: int, rate_hz: float, rng) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=count))


def steps_log2(T: int) -> float:
    return math.log2(T)
