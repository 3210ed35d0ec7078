"""Pins of the zero-mode-counting oracle (index of the massless D_N, outlook of
Sec. 4) on 4^4, against what the mathematics fixes: the free field's constant
zero modes (closed form at p = 0), the index theorem on quantised-flux
backgrounds, the sum rule index = -(1/2) Tr sign(Q), agreement of the
definition (null spaces of D per chirality) with the sector method, and chiral
pairing of the nonzero spectrum."""
import numpy as np
import pytest

import synthetic
from oracle import dirac, index, overlap, sign

M = -1.4
S = overlap.s_of_wilson_mass(M)
DIMS = (4, 4, 4, 4)
V = 256


class Case:
    """Exact sign(Q) of a 4^4 field; with ``definition`` also the dense D and
    the null-space counts of the definition."""

    def __init__(self, u=None, dense=None, definition=True):
        if dense is None:
            q = dirac.dense_Q(u, M, DIMS)
            self.lam, w = sign.dense_eig(q)
        else:
            q, self.lam, w = dense.Q, dense.lam, dense.W
        self.eps = sign.dense_sign_exact(q, eig=(self.lam, w))
        if definition:
            self.d = overlap.dense_DN(self.eps, S)
            self.svd = index.zero_modes_svd(self.d)
        self.spectra = index.sector_spectra(self.eps)
        self.count = index.count_zero_modes(self.spectra)


@pytest.fixture(scope="module")
def free(dense_cold):
    return Case(dense=dense_cold)


@pytest.fixture(scope="module")
def flux_pp():
    return Case(synthetic.flux_gauge_field(DIMS, 1, 1, noise=0.2, gauge_seed=synthetic.SEED_HAAR))


@pytest.fixture(scope="module")
def flux_pm():
    return Case(synthetic.flux_gauge_field(DIMS, 1, -1, noise=0.2, gauge_seed=synthetic.SEED_HAAR), definition=False)


def test_free_field_constant_zero_modes(free):
    """U = 1: D_W(p = 0) = m < 0, so Q = m gamma5 and sign(Q) = -gamma5 on the
    12 constant spinors, where D = (1 - 1)/abar = 0; every other momentum has
    |D| > 0.  Hence 6 zero modes of each chirality, index 0."""
    const = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for k in range(12):
        const[k, :, k // 3, k % 3] = 1.0 / np.sqrt(V)
    dc = free.d @ const.reshape(12, -1).T
    assert np.abs(dc).max() < 1e-12
    for r in (free.svd, free.count):
        assert (r["n_plus"], r["n_minus"], r["index"]) == (6, 6, 0)
    # the next singular value is far from zero
    assert free.svd["sv_plus"][6] > 1e-2 * free.svd["sv_plus"][-1]


@pytest.mark.slow
def test_index_theorem_on_flux_backgrounds(flux_pp, flux_pm):
    """Fluxes (q01, q23) = (1, +-1) in the diag(e^{i phi}, e^{-i phi}, 1)
    embedding: |Q_top| = 2 |q01 q23| = 2, with opposite signs; light noise and a
    gauge transformation leave it unchanged.  With the chirality convention used here the
    index n_+ - n_- is -2 q01 q23."""
    assert flux_pp.svd["index"] == -2
    assert (flux_pp.count["n_plus"], flux_pp.count["n_minus"]) == (flux_pp.svd["n_plus"], flux_pp.svd["n_minus"])
    assert flux_pm.count["index"] == 2
    for case in (flux_pp, flux_pm):
        # all zero modes have one chirality (no accidental pairs at this noise)
        assert min(case.count["n_plus"], case.count["n_minus"]) == 0


@pytest.mark.slow
def test_index_sum_rule(flux_pp, flux_pm, free):
    """n_+ - n_- = -(1/2) Tr sign(Q) (Tr gamma5 = 0 and the Ginsparg-Wilson pairing)."""
    for case in (flux_pp, flux_pm, free):
        assert case.count["index"] == -index.spectral_asymmetry(case.lam) // 2
        assert index.spectral_asymmetry(case.lam) % 2 == 0


@pytest.mark.slow
def test_chiral_pairing(flux_pp):
    """The eigenvalues of A_+ and A_- inside (0, 2) coincide.  The unpaired
    ones are the zero modes and the modes at 2 (D = 2 / abar), whose chirality
    counts balance them (Tr gamma5 = 0): n'_+ - n'_- = -(n_+ - n_-)."""
    c = flux_pp
    inner, top = {}, {}
    for s in (1, -1):
        ev = c.spectra[s]
        inner[s] = ev[(ev > 1e-8) & (ev < 2.0 - 1e-10)]
        top[s] = int(np.count_nonzero(ev >= 2.0 - 1e-10))
    assert inner[1].size == inner[-1].size
    assert np.abs(inner[1] - inner[-1]).max() < 1e-12
    assert top[1] - top[-1] == -(c.count["n_plus"] - c.count["n_minus"])
    # zero modes are zero to rounding; the first nonzero mode is well above the cut
    assert c.spectra[-1][:2].max() < 1e-12 and min(inner[1][0], inner[-1][0]) > 1e-6


@pytest.mark.slow
def test_sector_operator_is_DdagD(flux_pp):
    """On the chirality-s subspace, D^H D = (2 / abar^2) A_s (with eps^2 = 1)."""
    c = flux_pp
    abar = overlap.abar(S)
    chi = index.chirality(V)
    dd = c.d.conj().T @ c.d
    for s in (1, -1):
        idx = np.flatnonzero(chi == s)
        assert np.abs(dd[np.ix_(idx, idx)] - 2.0 / abar ** 2 * index.sector_operator(c.eps, s)).max() < 1e-12


@pytest.mark.slow
def test_massive_normal_operator_on_sectors(flux_pp):
    """The chirality-sector form of the massive normal equations used by the
    sector solver: with D^m = alpha + beta gamma5 eps (Eq. 4 with the massive
    form of Eq. 12: alpha = 1/abar + mq/2, beta = 1/abar - mq/2), on the
    chirality-s subspace (D^m)^H D^m = (alpha - beta)^2 + 2 alpha beta A_s, and
    it maps each sector to itself (zero off-diagonal blocks)."""
    c = flux_pp
    mq = 0.05
    abar = overlap.abar(S)
    alpha, beta = 1.0 / abar + mq / 2, 1.0 / abar - mq / 2
    d = overlap.dense_DN(c.eps, S, mq)
    dd = d.conj().T @ d
    chi = index.chirality(V)
    ip, im = np.flatnonzero(chi == 1), np.flatnonzero(chi == -1)
    assert np.abs(dd[np.ix_(ip, im)]).max() < 1e-12
    for s, idx in ((1, ip), (-1, im)):
        want = (alpha - beta) ** 2 * np.eye(idx.size) + 2 * alpha * beta * index.sector_operator(c.eps, s)
        assert np.abs(dd[np.ix_(idx, idx)] - want).max() < 1e-12
