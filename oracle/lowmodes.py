"""Low modes of Q and the projector diagnostics -- oracle (test infrastructure only).

Sec. 2.3 of the paper:

* V = span of l approximate eigenvectors, P its orthogonal projector, and the
  Rayleigh-Ritz vectors u_k in V with P Q u_k = nu_k u_k;
* P_+ / P_- = sum of u_k u_k^H over nu_k > 0 / nu_k < 0 (Eq. 7);
* residues rho_k = |(Q - nu_k) u_k| (Eq. 8);
* kappa_+-^2 = sum_{+-nu_k > 0} rho_k^2 / d_k^2 (Eq. 9), where d_k is the
  distance of nu_k from the exact spectrum of Q on the subspace orthogonal to
  the exact projector of the same sign (the printed sentence is garbled; its
  second "if" is read as "or");
* |P_+- - (P_+-)_exact| <= kappa (1 + 2 kappa) / (1 - 2 kappa (1 + 2 kappa)) (Eq. 10);
* |D_N^m(approx) - D_N^m| <= (2/a)(1 + s - a m / 2)(kappa_+ + kappa_-) (Eq. 12).

The paper finds V by minimising the Ritz functional of Q^2; ``ritz_lowmodes``
does that literally (conjugate gradients on the Rayleigh quotient with exact
line minimisation, one mode after the other, each kept orthogonal to the
modes already found), ``dense_lowmodes`` takes V from a dense
eigen-decomposition (small lattices).
"""
from __future__ import annotations

import numpy as np


def dense_lowmodes(q_dense: np.ndarray, l: int, eig=None):
    """The l eigenpairs of smallest |lambda| of a dense Hermitian Q.

    Returns (nu[l], modes[l, N]) sorted by |lambda| (stable on ties);
    ``eig`` = (lambda, W) if already known.
    """
    lam, w = np.linalg.eigh(q_dense) if eig is None else eig
    order = np.argsort(np.abs(lam), kind="stable")[:l]
    return lam[order], w[:, order].T.copy()


def rayleigh_ritz(apply_q, basis: np.ndarray):
    """Rayleigh-Ritz of Q in span(basis): orthonormalise, form M = V^H Q V,
    diagonalise.  Returns (nu ascending, u[l, ...]) with P Q u_k = nu_k u_k."""
    shape = basis.shape[1:]
    v = basis.reshape(basis.shape[0], -1).T
    v, _ = np.linalg.qr(v)
    qv = np.stack([apply_q(v[:, k].reshape(shape)).ravel() for k in range(v.shape[1])], axis=1)
    m = v.conj().T @ qv
    m = 0.5 * (m + m.conj().T)
    nu, w = np.linalg.eigh(m)
    u = (v @ w).T.reshape((-1,) + shape)
    return nu, u


def residues(apply_q, modes: np.ndarray, nu: np.ndarray) -> np.ndarray:
    """rho_k = |(Q - nu_k) u_k| (Eq. 8)."""
    return np.array([np.linalg.norm((apply_q(u) - n * u).ravel()) for u, n in zip(modes, nu)])


def gap_distances(nu: np.ndarray, lam_next: float) -> np.ndarray:
    """Estimate of d_k (Sec. 2.3): distance of nu_k from the exact spectrum of Q
    restricted to the complement of the exact projector of the same sign.

    That spectrum holds the opposite-sign low modes and every eigenvalue of
    modulus >= lam_next (the first |eigenvalue| outside V):
    d_k = min(lam_next - |nu_k|, |nu_k| + min_{sign(nu_j) != sign(nu_k)} |nu_j|).
    """
    nu = np.asarray(nu, dtype=np.float64)
    d = np.empty_like(nu)
    for k, n in enumerate(nu):
        opp = np.abs(nu[np.sign(nu) != np.sign(n)])
        cand = [lam_next - abs(n)]
        if opp.size:
            cand.append(abs(n) + opp.min())
        d[k] = min(cand)
    return d


def kappas(nu: np.ndarray, rho: np.ndarray, d: np.ndarray):
    """(kappa_+, kappa_-) of Eq. 9."""
    pos = nu > 0
    kp = float(np.sqrt(np.sum((rho[pos] / d[pos]) ** 2)))
    km = float(np.sqrt(np.sum((rho[~pos] / d[~pos]) ** 2)))
    return kp, km


def projector_bound(kappa: float) -> float:
    """Eq. 10: kappa (1 + 2 kappa) / (1 - 2 kappa (1 + 2 kappa)); inf when the
    denominator is not positive."""
    q = kappa * (1.0 + 2.0 * kappa)
    den = 1.0 - 2.0 * q
    return q / den if den > 0 else float("inf")


def dn_bound(kappa_p: float, kappa_m: float, s: float, mq: float, a: float = 1.0) -> float:
    """Eq. 12: (2/a)(1 + s - a m / 2)(kappa_+ + kappa_-)."""
    return (2.0 / a) * (1.0 + s - a * mq / 2.0) * (kappa_p + kappa_m)


def _vdot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def ritz_minimise(apply_a, x0, lower, tol: float, max_iter: int = 10000):
    """Minimise the Ritz functional mu(x) = <x, A x> / <x, x> of a Hermitian
    positive A over x orthogonal to the orthonormal vectors ``lower``.

    Conjugate gradients on the unit sphere: the gradient direction is
    g = (A x - mu x) with the components along ``lower`` removed; each step
    minimises mu exactly on span(x, p) (the smaller eigenvalue of the 2 x 2
    Rayleigh-quotient matrix of that plane); the next direction is
    g + beta p with beta = |g_new|^2 / |g_old|^2.  Stops when |g| <= tol.
    Returns (x unit, mu, |g|, iterations).
    """
    def proj(v):
        for u in lower:
            v = v - _vdot(u, v) * u
        return v

    x = proj(np.array(x0, dtype=np.complex128))
    x = x / np.linalg.norm(x.ravel())
    y = apply_a(x)
    mu = _vdot(x, y).real
    g = proj(y - mu * x)
    g2 = _vdot(g, g).real
    p = g.copy()
    it = 0
    while np.sqrt(g2) > tol and it < max_iter:
        pp = p - _vdot(x, p) * x
        ph = pp / np.linalg.norm(pp.ravel())
        z = apply_a(ph)
        a, b, c = mu, _vdot(x, z).real, _vdot(ph, z).real
        # mu(t) = a cos^2 t + 2 b sin t cos t + c sin^2 t is smallest at
        # (cos 2t, sin 2t) proportional to ((c - a) / 2, -b)
        t = 0.5 * np.arctan2(-b, 0.5 * (c - a))
        cs, sn = np.cos(t), np.sin(t)
        x = cs * x + sn * ph
        y = cs * y + sn * z
        x = proj(x)
        nx = np.linalg.norm(x.ravel())
        x, y = x / nx, y / nx
        mu = _vdot(x, y).real
        g_new = proj(y - mu * x)
        g2_new = _vdot(g_new, g_new).real
        p = g_new + (g2_new / g2) * pp
        g, g2 = g_new, g2_new
        it += 1
    return x, mu, float(np.sqrt(g2)), it


def ritz_lowmodes(apply_a, starts, nev: int, tol: float, max_iter: int = 10000):
    """The nev lowest eigenpairs of A (Sec. 2.3: the Ritz functional of Q^2),
    one after the other, mode k minimised orthogonally to modes 0..k-1 from the
    start vector starts[k].  Returns (mu[nev] ascending, x[nev, ...], |g|[nev])."""
    modes, mus, gs = [], [], []
    for k in range(nev):
        x, mu, gn, _ = ritz_minimise(apply_a, starts[k], modes, tol, max_iter)
        modes.append(x)
        mus.append(mu)
        gs.append(gn)
    return np.array(mus), np.stack(modes), np.array(gs)

