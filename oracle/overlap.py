"""The Neuberger-Dirac operator -- oracle (test infrastructure only).

Eq. 4 (Sec. 2.2): D_N = (1 + gamma5 sign(Q)) / abar with Q = gamma5 (a D_W - 1 - s).
With a = 1, this Q is the Q = gamma5 D_W of Eq. 1 at Wilson mass m = -1 - s
(s = 0.4 for m = -1.4; |s| < 1 as the paper requires).

abar is not defined in the text.  Eq. 12 fixes it: the bound
(2/a)(1 + s - a m/2)(kappa_+ + kappa_-) equals (1/abar - m/2) times the
error of sign(Q) only for abar = a / (1 + s).  The massive operator used in
Eq. 12 is read as

    D_N^m = (1 - abar m / 2) D_N + m,

with m the quark mass (distinct from the Wilson mass of Eq. 1).
The Ginsparg-Wilson relation gamma5 D + D gamma5 = abar D gamma5 D holds for
D_N exactly when sign(Q)^2 = 1.
"""
from __future__ import annotations

import numpy as np

from .dirac import gamma5


def abar(s: float, a: float = 1.0) -> float:
    return a / (1.0 + s)


def s_of_wilson_mass(m: float) -> float:
    return -1.0 - m


def apply_DN(apply_sign, psi: np.ndarray, s: float, mq: float = 0.0) -> np.ndarray:
    """D_N^m psi = (1 - abar mq/2) (psi + gamma5 sign(Q) psi) / abar + mq psi."""
    ab = abar(s)
    return (1.0 - ab * mq / 2.0) * (psi + gamma5(apply_sign(psi))) / ab + mq * psi


def gamma5_dense(volume: int) -> np.ndarray:
    """gamma5 as a dense diagonal matrix on the canonical [V, 4, 3] layout."""
    d = np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), volume)
    return np.diag(d).astype(np.complex128)


def dense_DN(sign_dense: np.ndarray, s: float, mq: float = 0.0) -> np.ndarray:
    n = sign_dense.shape[0]
    g5 = gamma5_dense(n // 12)
    ab = abar(s)
    return (1.0 - ab * mq / 2.0) * (np.eye(n) + g5 @ sign_dense) / ab + mq * np.eye(n)


def gw_residual(d_dense: np.ndarray, s: float) -> float:
    """|gamma5 D + D gamma5 - abar D gamma5 D| (spectral norm) for the massless D_N."""
    n = d_dense.shape[0]
    g5 = gamma5_dense(n // 12)
    r = g5 @ d_dense + d_dense @ g5 - abar(s) * d_dense @ g5 @ d_dense
    return float(np.linalg.norm(r, 2))


def cgne(apply_d, apply_ddag, b: np.ndarray, tol: float = 1e-10, max_iter: int = 100000):
    """Textbook CG on the normal equations D^H D x = D^H b.

    Stops on the true residual |b - D x| <= tol |b|, checked every step
    through the recursive residual of D x.  Returns (x, iterations).
    """
    x = np.zeros_like(b)
    r = b.copy()                     # b - D x
    z = apply_ddag(r)                # D^H r
    p = z.copy()
    zz = np.vdot(z.ravel(), z.ravel()).real
    bnorm = np.linalg.norm(b.ravel())
    for it in range(1, max_iter + 1):
        dp = apply_d(p)
        alpha = zz / np.vdot(dp.ravel(), dp.ravel()).real
        x = x + alpha * p
        r = r - alpha * dp
        if np.linalg.norm(r.ravel()) <= tol * bnorm:
            return x, it
        z = apply_ddag(r)
        zz_new = np.vdot(z.ravel(), z.ravel()).real
        p = z + (zz_new / zz) * p
        zz = zz_new
    raise RuntimeError("CGNE did not converge")
