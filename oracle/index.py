"""Index of the massless Neuberger-Dirac operator by zero-mode counting -- oracle
(test infrastructure only).  Dense: small lattices only.

The outlook of Sec. 4 names the index of D_N, found by counting zero modes, as
the next workload.  For the massless operator of Eq. 4,

    D = (1 + gamma5 eps) / abar,   eps = sign(Q),

the kernel of D is invariant under gamma5 (it follows from eps^2 = 1 and the
Ginsparg-Wilson relation that Eq. 4 satisfies), so its zero modes can be taken
chiral: n_+ of chirality +1 and n_- of chirality -1; the index is n_+ - n_-.

Two routes are written out here:

* ``zero_modes_svd``: the definition.  n_s is the dimension of the null space
  of D restricted to the chirality-s subspace, counted from the singular
  values of the columns of D with gamma5 = s;
* ``sector_spectra``: the method the GPU library uses.  On the chirality-s
  subspace, D^H D = (2 / abar^2) A_s with

      A_s = 1 + s P_s eps P_s,   P_s = (1 + s gamma5) / 2,

  (using eps^2 = 1), whose spectrum lies in [0, 2]; n_s is the number of its
  eigenvalues below a cut.  The nonzero eigenvalues of A_+ and A_- coincide
  (chiral pairing), so only zero modes make the two sectors differ.

Pins (tests/test_oracle_index.py): the free field's constant zero modes
(12 of them, 6 per chirality, from the closed-form symbol at p = 0), the index
theorem on flux backgrounds (index = -2 q01 q23 for the embedding of
``synthetic.flux_gauge_field``; the sign flips with the flux), the sum rule
n_+ - n_- = -(1/2) Tr eps = -(1/2) (number of positive minus negative
eigenvalues of Q), agreement of the two routes, and chiral pairing.
"""
from __future__ import annotations

import numpy as np


def chirality(volume: int) -> np.ndarray:
    """gamma5 eigenvalue (+1 or -1) of each component of the canonical
    [V, 4, 3] layout (chiral representation: spins 0, 1 are +1)."""
    return np.tile(np.repeat([1, 1, -1, -1], 3), volume)


def zero_modes_svd(d_dense: np.ndarray, cut: float = 1e-8) -> dict:
    """n_+, n_-, index from the singular values of D on each chirality subspace.

    d_dense: the massless D (any positive normalisation); cut is relative to
    the largest singular value of D."""
    chi = chirality(d_dense.shape[0] // 12)
    smax = np.linalg.norm(d_dense, 2)
    out = {}
    for s, name in ((1, "n_plus"), (-1, "n_minus")):
        sv = np.linalg.svd(d_dense[:, chi == s], compute_uv=False)
        out[name] = int(np.count_nonzero(sv < cut * smax))
        out["sv_plus" if s == 1 else "sv_minus"] = np.sort(sv)
    out["index"] = out["n_plus"] - out["n_minus"]
    return out


def sector_operator(eps_dense: np.ndarray, s: int) -> np.ndarray:
    """A_s = 1 + s P_s eps P_s on the chirality-s subspace (a dense matrix on
    the components with gamma5 = s)."""
    chi = chirality(eps_dense.shape[0] // 12)
    idx = np.flatnonzero(chi == s)
    return np.eye(idx.size) + s * eps_dense[np.ix_(idx, idx)]


def sector_spectra(eps_dense: np.ndarray) -> dict:
    """Ascending eigenvalues of A_+ and A_-."""
    return {s: np.linalg.eigvalsh(sector_operator(eps_dense, s)) for s in (1, -1)}


def count_zero_modes(spectra: dict, cut: float = 1e-8) -> dict:
    """n_+, n_-, index from the sector spectra: eigenvalues of A_s below cut."""
    n_plus = int(np.count_nonzero(spectra[1] < cut))
    n_minus = int(np.count_nonzero(spectra[-1] < cut))
    return {"n_plus": n_plus, "n_minus": n_minus, "index": n_plus - n_minus}


def spectral_asymmetry(lam: np.ndarray) -> int:
    """Number of positive minus number of negative eigenvalues of Q (= Tr eps)."""
    return int(np.count_nonzero(lam > 0)) - int(np.count_nonzero(lam < 0))
