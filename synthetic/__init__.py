"""Seeded synthetic inputs for the Neuberger-Dirac hot path.

This module is the only code shared by the FP64 CPU oracle and the GPU path.
It draws random numbers and shapes them into gauge fields, spinor fields,
gauge transformations and perturbation directions; it contains none of the
arithmetic of the operators themselves (no Wilson-Dirac stencil, no sign
function, no projector).

All arrays are numpy, complex128, in the canonical host layout:

* sites in lexicographic order ``lex = ((x0*N1 + x1)*N2 + x2)*N3 + x3`` with
  ``dims = (N0, N1, N2, N3)`` and ``N0`` the time extent;
* gauge field ``[V][4 mu][3 row][3 col]``;
* spinor field ``[V][4 spin][3 colour]`` (a leading ``nrhs`` axis for batches).

Seeds follow one convention: gauge 1001, spinor/source 1002, Haar gauge
transformation 1003, su(3) finite-difference directions 1004, eigensolver
start vector 1005.  Random generators are numpy ``Generator(PCG64(seed))``.
"""
from __future__ import annotations

import numpy as np

SEED_GAUGE = 1001
SEED_SPINOR = 1002
SEED_HAAR = 1003
SEED_DIRECTIONS = 1004
SEED_START = 1005


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def volume(dims) -> int:
    n0, n1, n2, n3 = (int(d) for d in dims)
    return n0 * n1 * n2 * n3


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda_a, shape [8,3,3] complex128."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def su3_generators() -> np.ndarray:
    """T_a = lambda_a / 2 (Hermitian, traceless, tr T_a T_b = delta_ab / 2)."""
    return gell_mann() / 2


def _expi_hermitian(h: np.ndarray) -> np.ndarray:
    """exp(i h) for a stack of Hermitian 3x3 matrices via eigen-decomposition."""
    e, w = np.linalg.eigh(h)
    return np.einsum("...ij,...j,...kj->...ik", w, np.exp(1j * e), w.conj())


def reunitarize(u: np.ndarray) -> np.ndarray:
    """Project a stack of near-unitary 3x3 matrices onto SU(3).

    Column a is normalised, column b is orthogonalised against a and
    normalised, and column c is rebuilt as conj(a x b), which makes det = 1.
    """
    a = u[..., :, 0]
    a = a / np.linalg.norm(a, axis=-1, keepdims=True)
    b = u[..., :, 1]
    b = b - np.sum(a.conj() * b, axis=-1, keepdims=True) * a
    b = b / np.linalg.norm(b, axis=-1, keepdims=True)
    c = np.cross(a, b).conj()
    return np.stack([a, b, c], axis=-1)


def gauge_field(dims, width: float = 0.3, seed: int = SEED_GAUGE) -> np.ndarray:
    """Random SU(3) links U = exp(i sum_a omega_a T_a), omega_a ~ N(0, width^2).

    omega is drawn in C order with shape (N0, N1, N2, N3, 4, 8), one
    independent su(3) vector per link, then exponentiated and
    re-unitarised.  Returns complex128 ``[V, 4, 3, 3]``.
    """
    dims = tuple(int(d) for d in dims)
    omega = _rng(seed).normal(0.0, width, size=dims + (4, 8))
    h = np.einsum("...a,aij->...ij", omega, su3_generators())
    u = reunitarize(_expi_hermitian(h))
    return np.ascontiguousarray(u.reshape(volume(dims), 4, 3, 3))


def cold_gauge(dims) -> np.ndarray:
    """Unit links U = 1 (the free field)."""
    v = volume(dims)
    u = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def spinor(nsites: int, nrhs: int | None = None, seed: int = SEED_SPINOR) -> np.ndarray:
    """Complex Gaussian spinor, Re and Im ~ N(0, 1/2) so that E|z|^2 = 1.

    Drawn as reals of shape (nrhs, nsites, 4, 3, 2) (nrhs omitted if None).
    """
    shape = (nsites, 4, 3, 2) if nrhs is None else (nrhs, nsites, 4, 3, 2)
    r = _rng(seed).normal(0.0, np.sqrt(0.5), size=shape)
    return np.ascontiguousarray(r[..., 0] + 1j * r[..., 1])


def point_sources(nsites: int, site: int = 0) -> np.ndarray:
    """The 12 spin-colour point sources delta_{x,site} delta_{alpha,s} delta_{a,c}.

    Returns ``[12, nsites, 4, 3]`` with rhs index ``3*s + c``.
    """
    out = np.zeros((12, nsites, 4, 3), dtype=np.complex128)
    for s in range(4):
        for c in range(3):
            out[3 * s + c, site, s, c] = 1.0
    return out


def haar_su3(n: int, seed: int = SEED_HAAR) -> np.ndarray:
    """n Haar-distributed SU(3) matrices (QR of a complex Ginibre matrix with
    the phases of R's diagonal removed, then det fixed to 1)."""
    r = _rng(seed).normal(size=(n, 3, 3, 2))
    z = (r[..., 0] + 1j * r[..., 1]) / np.sqrt(2)
    q, rr = np.linalg.qr(z)
    d = np.diagonal(rr, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return q


def su3_directions(nsites: int, ndir: int = 8, seed: int = SEED_DIRECTIONS) -> np.ndarray:
    """Random su(3) directions omega[ndir, V, 4, 8] ~ N(0, 1) for finite differences."""
    return _rng(seed).normal(size=(ndir, nsites, 4, 8))


def start_vector(nsites: int, seed: int = SEED_START) -> np.ndarray:
    """Eigensolver start vector: a complex Gaussian spinor ``[V, 4, 3]``."""
    return spinor(nsites, None, seed)


def flux_gauge_field(dims, q01: int, q23: int, noise: float = 0.0, noise_seed: int = SEED_GAUGE,
                     gauge_seed: int | None = None) -> np.ndarray:
    """SU(3) links carrying quantised U(1) fluxes (a smooth background of known topology).

    U(1) phases with the uniform field strength 2 pi q01 / (N0 N1) on every
    (0,1) plaquette and 2 pi q23 / (N2 N3) on every (2,3) plaquette of the
    periodic lattice:

        phi_0(x) = -2 pi q01 x1 / (N0 N1),   phi_1(x) = 2 pi q01 x0 / N0 if x1 = N1 - 1, else 0,
        phi_2(x) = -2 pi q23 x3 / (N2 N3),   phi_3(x) = 2 pi q23 x2 / N2 if x3 = N3 - 1, else 0,

    embedded as diag(e^{i phi}, e^{-i phi}, 1) (colour charges +1, -1, 0, so the
    continuum topological charge is 2 q01 q23).  With ``noise`` > 0 every link
    is multiplied from the left by a random SU(3) link of that width (drawn as
    ``gauge_field(dims, noise, noise_seed)``); with ``gauge_seed`` the field is
    then gauge transformed, U_mu(x) -> Omega(x) U_mu(x) Omega(x + mu)^H with
    Haar-random Omega = ``haar_su3(V, gauge_seed)``.  Returns ``[V, 4, 3, 3]``.
    """
    dims = tuple(int(d) for d in dims)
    n0, n1, n2, n3 = dims
    v = volume(dims)
    x = np.stack(np.unravel_index(np.arange(v), dims), axis=-1)
    phi = np.zeros((v, 4))
    phi[:, 0] = -2.0 * np.pi * q01 * x[:, 1] / (n0 * n1)
    phi[:, 1] = np.where(x[:, 1] == n1 - 1, 2.0 * np.pi * q01 * x[:, 0] / n0, 0.0)
    phi[:, 2] = -2.0 * np.pi * q23 * x[:, 3] / (n2 * n3)
    phi[:, 3] = np.where(x[:, 3] == n3 - 1, 2.0 * np.pi * q23 * x[:, 2] / n2, 0.0)
    e = np.exp(1j * phi)
    u = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = e
    u[..., 1, 1] = e.conj()
    u[..., 2, 2] = 1.0
    if noise > 0.0:
        u = np.einsum("vmab,vmbc->vmac", gauge_field(dims, noise, noise_seed), u)
    if gauge_seed is not None:
        om = haar_su3(v, gauge_seed)
        u = np.einsum("vab,vmbc->vmac", om, u)
        for mu in range(4):
            shift = [0, 0, 0, 0]
            shift[mu] = 1
            nb = np.ravel_multi_index(tuple((x[:, k] + shift[k]) % dims[k] for k in range(4)), dims)
            u[:, mu] = u[:, mu] @ om[nb].conj().transpose(0, 2, 1)
    return np.ascontiguousarray(u)
