"""The Wilson-Dirac operator D_W and Q = gamma5 D_W -- oracle (test infrastructure only).

Follows Sec. 2.1, Eq. 1 and Eq. 2 of the paper literally:

    D_W phi(x) = (4 + m) phi(x) - 1/2 sum_{mu = +-0..+-3} U_mu(x) (1 - gamma_mu) phi(x + mu-hat),
    U_{-mu}(x) = U_mu(x - mu-hat)^{-1},   gamma_{-mu} = -gamma_mu,   Q = gamma5 D_W.

Spin matrices are full 4x4 matrices and links are full 3x3 matrices; the
backward link is a true matrix inverse (equal to the conjugate transpose for
SU(3) links, which a test checks).  Lattice spacing a = 1.

The paper does not fix a representation of the Dirac matrices; the chiral
(Weyl) representation with Hermitian gamma matrices is used:

    gamma_0 = [[0, -1], [-1, 0]],  gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
    gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 = diag(1, 1, -1, -1).

Fields are canonical arrays: spinor [..., V, 4, 3], gauge [V, 4, 3, 3]
(lexicographic sites, see ``oracle.geometry``).
"""
from __future__ import annotations

import numpy as np

from . import geometry


def gamma_matrices():
    """Return (g[4,4,4], g5[4,4]) in the chiral representation."""
    i2 = np.eye(2, dtype=np.complex128)
    z2 = np.zeros((2, 2), dtype=np.complex128)
    s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    g = np.empty((4, 4, 4), dtype=np.complex128)
    g[0] = np.block([[z2, -i2], [-i2, z2]])
    for k, s in enumerate((s1, s2, s3), start=1):
        g[k] = np.block([[z2, -1j * s], [1j * s, z2]])
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


_G, _G5 = gamma_matrices()
_I4 = np.eye(4, dtype=np.complex128)


def _lattice(psi: np.ndarray, dims) -> np.ndarray:
    return psi.reshape(psi.shape[:-3] + tuple(dims) + (4, 3))


def _canonical(psi_l: np.ndarray) -> np.ndarray:
    return psi_l.reshape(psi_l.shape[:-6] + (-1, 4, 3))


def _spin(mat: np.ndarray, psi: np.ndarray) -> np.ndarray:
    return np.einsum("st,...tc->...sc", mat, psi)


def _colour(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    return np.einsum("...ab,...sb->...sa", u, psi)


def hopping(U: np.ndarray, psi: np.ndarray, dims) -> np.ndarray:
    """H psi(x) = sum over the 8 directions of U_{+-mu}(x)(1 - gamma_{+-mu}) psi(x +- mu-hat).

    So that D_W = (4 + m) - H/2 (Eq. 1).
    """
    dims = geometry.check_dims(dims)
    ul = U.reshape(dims + (4, 3, 3))
    pl = _lattice(psi, dims)
    base = pl.ndim - 6
    out = np.zeros_like(pl, dtype=np.complex128)
    for mu in range(4):
        ax = base + mu
        # +mu: U_mu(x) (1 - gamma_mu) psi(x + mu)
        fwd = np.roll(pl, -1, axis=ax)
        out += _colour(ul[..., mu, :, :], _spin(_I4 - _G[mu], fwd))
        # -mu: U_{-mu}(x) = U_mu(x - mu)^{-1}, gamma_{-mu} = -gamma_mu
        u_back = np.linalg.inv(np.roll(ul[..., mu, :, :], 1, axis=mu))
        bwd = np.roll(pl, 1, axis=ax)
        out += _colour(u_back, _spin(_I4 + _G[mu], bwd))
    return _canonical(out)


def wilson_dirac(U: np.ndarray, psi: np.ndarray, m: float, dims) -> np.ndarray:
    """D_W psi (Eq. 1)."""
    return (4.0 + m) * psi - 0.5 * hopping(U, psi, dims)


def gamma5(psi: np.ndarray) -> np.ndarray:
    return _spin(_G5, psi)


def apply_Q(U: np.ndarray, psi: np.ndarray, m: float, dims) -> np.ndarray:
    """Q psi = gamma5 D_W psi (Eq. 1)."""
    return gamma5(wilson_dirac(U, psi, m, dims))


def apply_Q_at(U: np.ndarray, psi_at, m: float, dims, sites) -> np.ndarray:
    """(Q psi)(y) for the lexicographic sites y in ``sites`` only (Eq. 1 at those sites).

    ``psi_at(idx)`` returns psi at the lexicographic sites ``idx`` as
    [..., len(idx), 4, 3]; so psi never has to exist as a full array (large
    lattices, point sources).  ``U`` is the gauge field [V, 4, 3, 3] or any
    object indexable as U[site, mu].  The neighbours are found from the
    coordinates of each site with periodic wrap-around, independently of
    ``neighbour_table``.
    """
    dims = geometry.check_dims(dims)
    n = np.array(dims)
    sites = np.asarray(sites, dtype=np.int64)
    x = np.stack(np.unravel_index(sites, dims), axis=-1)
    out = (4.0 + m) * psi_at(sites)
    for mu in range(4):
        e = np.zeros(4, dtype=np.int64)
        e[mu] = 1
        fwd = geometry.lex_of(dims, (x + e) % n)
        bwd = geometry.lex_of(dims, (x - e) % n)
        u_f = np.asarray(U[sites, mu])
        u_b = np.linalg.inv(np.asarray(U[bwd, mu]))
        out = out - 0.5 * _colour(u_f, _spin(_I4 - _G[mu], psi_at(fwd)))
        out = out - 0.5 * _colour(u_b, _spin(_I4 + _G[mu], psi_at(bwd)))
    return gamma5(out)


def dslash(U: np.ndarray, psi_in: np.ndarray, dims, out_parity: int) -> np.ndarray:
    """Even/odd hopping block: (H psi)_p for psi living on parity 1-p.

    ``psi_in`` is a half field [..., V/2, 4, 3] of parity 1-p in eo order; the
    result is the half field of parity p.  Defined by embedding into the full
    lattice, applying ``hopping`` and restricting, i.e. the plain definition of
    the off-diagonal block H_{p,1-p} in D_W = [[4+m, -H_eo/2], [-H_oe/2, 4+m]].
    """
    leo = geometry.lex_of_eo(dims)
    v = geometry.volume(dims)
    full = np.zeros(psi_in.shape[:-3] + (v, 4, 3), dtype=np.complex128)
    full[..., leo[1 - out_parity], :, :] = psi_in
    return hopping(U, full, dims)[..., leo[out_parity], :, :]


def qhat_ee(U: np.ndarray, psi_e: np.ndarray, m: float, dims) -> np.ndarray:
    """Even-site Schur complement, gamma5-Hermitian form:

        Qhat_ee = gamma5 [ (4+m) - H_eo H_oe / (4 (4+m)) ],

    the gamma5 times the Schur complement D_ee - D_eo D_oo^{-1} D_oe of
    D_W = [[4+m, -H_eo/2], [-H_oe/2, 4+m]].
    """
    t = dslash(U, psi_e, dims, 1)
    t = dslash(U, t, dims, 0)
    return gamma5((4.0 + m) * psi_e - t / (4.0 * (4.0 + m)))


def dense_Q(U: np.ndarray, m: float, dims, chunk: int = 512) -> np.ndarray:
    """Q as a dense (12V x 12V) matrix, column j = Q e_j (small lattices only)."""
    v = geometry.volume(dims)
    n = 12 * v
    q = np.empty((n, n), dtype=np.complex128)
    for start in range(0, n, chunk):
        stop = min(n, start + chunk)
        e = np.zeros((stop - start, n), dtype=np.complex128)
        e[np.arange(stop - start), np.arange(start, stop)] = 1.0
        q[:, start:stop] = apply_Q(U, e.reshape(-1, v, 4, 3), m, dims).reshape(stop - start, n).T
    return q


def free_field_symbol(p, m: float) -> np.ndarray:
    """D_W in momentum space for U = 1 (closed form, used as a pin):

        D_W(p) = m + sum_mu (1 - cos p_mu) + i sum_mu gamma_mu sin p_mu.
    """
    p = np.asarray(p, dtype=np.float64)
    d = (m + np.sum(1 - np.cos(p))) * _I4
    for mu in range(4):
        d = d + 1j * np.sin(p[mu]) * _G[mu]
    return d


def lambda_max_bound(m: float) -> float:
    """Rigorous bound |Q| <= |4 + m| + 4 used for X = Q/|Q| (Eq. 5).

    Each of the four direction terms (1/2)[U(1-gamma) T_+ + U^-1 (1+gamma) T_-]
    is a norm-1 operator, and the free field at p = (pi, pi, pi, pi) attains
    the bound when 4 + m >= 0.
    """
    return abs(4.0 + m) + 4.0
