"""Derivatives of Q with respect to the spinor and the links -- oracle (test
infrastructure only).  Not in the paper; follows from Eq. 1.

Link perturbations are taken along su(3): U_mu(x) -> exp(i w T_a) U_mu(x)
with T_a = lambda_a / 2 (Gell-Mann).  For a cotangent g of y = Q psi, the
link force is

    F^a_mu(x) = d/dw Re<g, Q[U(w)] psi> at w = 0
              = 1/2 Re[ -i chi(x)^H T_a U_mu(x) (1 - gamma_mu) psi(x + mu)
                        + i chi(x + mu)^H U_mu(x)^H T_a (1 + gamma_mu) psi(x) ],
    chi = gamma5 g,

because U_mu(x) enters D_W through the forward hop at x and the backward hop
at x + mu, each with weight -1/2.  For S = |Q psi|^2 the cotangent is
g = 2 Q psi (chi = 2 D_W psi), and dS/dpsi-bar = Q^2 psi.
"""
from __future__ import annotations

import numpy as np

from . import geometry
from .dirac import apply_Q, gamma5, gamma_matrices


def su3_generators() -> np.ndarray:
    """T_a = lambda_a / 2."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam / 2


_T = su3_generators()
_G, _ = gamma_matrices()
_I4 = np.eye(4, dtype=np.complex128)


def action(U, psi, m, dims) -> float:
    """S = psi^H Q^2 psi = |Q psi|^2."""
    q = apply_Q(U, psi, m, dims)
    return float(np.vdot(q.ravel(), q.ravel()).real)


def grad_psi_action(U, psi, m, dims) -> np.ndarray:
    """Gradient of S in the convention 2 dS/d(psi-bar) = 2 Q^2 psi."""
    return 2.0 * apply_Q(U, apply_Q(U, psi, m, dims), m, dims)


def force_vjp(U, psi, g, dims) -> np.ndarray:
    """F[V, 4, 8] = d Re<g, Q psi> / d w^a_mu(x) (see module docstring)."""
    dims = geometry.check_dims(dims)
    v = geometry.volume(dims)
    nb = geometry.neighbour_table(dims)
    chi = gamma5(g)
    f = np.empty((v, 4, 8))
    for mu in range(4):
        fwd = nb[:, mu]
        u = U[:, mu]                                             # [V,3,3]
        hm = np.einsum("st,vtc->vsc", _I4 - _G[mu], psi[fwd])    # (1-g) psi(x+mu)
        hp = np.einsum("st,vtc->vsc", _I4 + _G[mu], psi)         # (1+g) psi(x)
        for a in range(8):
            t1 = np.einsum("vsa,ab,vbc,vsc->v", chi.conj(), _T[a], u, hm)
            t2 = np.einsum("vsa,vba,bc,vsc->v", chi[fwd].conj(), u.conj(), _T[a], hp)
            f[:, mu, a] = 0.5 * (-1j * t1 + 1j * t2).real
    return f


def force_action(U, psi, m, dims) -> np.ndarray:
    """dS/dw for S = |Q psi|^2."""
    return force_vjp(U, psi, 2.0 * apply_Q(U, psi, m, dims), dims)


def perturb_links(U, omega, t: float) -> np.ndarray:
    """U_mu(x) -> exp(i t sum_a omega^a_mu(x) T_a) U_mu(x), omega [V, 4, 8]."""
    h = t * np.einsum("vma,aij->vmij", omega, _T)
    e, w = np.linalg.eigh(h)
    ex = np.einsum("...ij,...j,...kj->...ik", w, np.exp(1j * e), w.conj())
    return np.einsum("vmij,vmjk->vmik", ex, U)
