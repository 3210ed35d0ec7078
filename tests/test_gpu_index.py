"""Index of the massless D_N by zero-mode counting on the GPU (ndq_index_DN),
against the dense FP64 oracle on 4^4 (counts and the lowest eigenvalues of the
sector operators A_s built from the same approximate sign) and, on 8^4 where
no dense oracle fits, against the index theorem for quantised fluxes."""
import numpy as np
import pytest

import synthetic
from oracle import approx, dirac, index, sign

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1010_5636_amd as ndq  # noqa: E402

M = -1.4
LMAX = 6.6
DIMS = (4, 4, 4, 4)
CUT = 1e-7


def cu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


class Dense:
    def __init__(self, u):
        self.u = u
        self.q = dirac.dense_Q(u, M, DIMS)
        self.lam, self.w = sign.dense_eig(self.q)
        self.order = np.argsort(np.abs(self.lam), kind="stable")


@pytest.fixture(scope="module")
def flux():
    return Dense(synthetic.flux_gauge_field(DIMS, 1, 1, noise=0.2, gauge_seed=synthetic.SEED_HAAR))


@pytest.fixture(scope="module")
def free():
    return Dense(synthetic.cold_gauge(DIMS))


def gpu_index(d, dims, nev=0, degree=12, **kw):
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(d.u), ndq.F64, 18)
    if nev:
        k = abs(d.lam[d.order[nev]]) / LMAX
        low = d.w[:, d.order[:nev]].T.reshape(nev, -1, 4, 3)
        modes = ndq.SpinorField.pack(g, cu(low), ndq.F64, ndq.FULL)
        nu = d.lam[d.order[:nev]]
    else:
        k = abs(d.lam[d.order[0]]) / LMAX
        modes, nu = None, None
    ap = ndq.Approx(ndq.ZOLOTAREV, k, degree)
    ov = ndq.Overlap(g, M, ap, LMAX, modes=modes, nu=nu, tol=1e-13)
    start = ndq.SpinorField.pack(g, cu(synthetic.start_vector(g.volume)), ndq.F64, ndq.FULL)
    r = ndq.index_DN(g, U, ov, start, zero_cut=CUT, **kw)
    # the oracle's sector spectra for the same approximate sign
    eps = sign.dense_sign_approx(d.q, approx.zolotarev(k, degree), LMAX, n_low=nev, eig=(d.lam, d.w))
    return r, index.sector_spectra(eps)


def check_against_oracle(r, spectra, nb):
    want = index.count_zero_modes(spectra, CUT)
    assert (r["n_plus"], r["n_minus"], r["index"]) == (want["n_plus"], want["n_minus"], want["index"])
    for s, key in ((1, "plus"), (-1, "minus")):
        theta, res, ev = np.array(r["theta_" + key]), np.array(r["resid_" + key]), spectra[s]
        n = r["n_" + key]
        # the pairs below the cut: converged, on the oracle's lowest eigenvalues
        assert (res[:n] <= 1e-7).all()
        assert np.all(np.abs(theta[:n] - ev[:n]) <= 2 * res[:n] + 1e-12), (key, theta[:n], ev[:n])
        # the first pair above the cut: above the cut, an upper bound of the
        # n-th eigenvalue, within its residue of some eigenvalue
        assert theta[n] - res[n] > CUT
        assert theta[n] >= ev[n] - 1e-12
        assert np.abs(ev - theta[n]).min() <= res[n] + 1e-12


def test_flux_background_vs_oracle(flux):
    r, spectra = gpu_index(flux, DIMS)
    check_against_oracle(r, spectra, 8)
    assert (r["n_plus"], r["n_minus"], r["index"]) == (0, 2, -2)
    assert r["converged"] == [True, True]


def test_flux_background_with_exact_low_modes(flux):
    """The sign with 8 exact low modes of Q (Eq. 11) gives the same count."""
    r, spectra = gpu_index(flux, DIMS, nev=8)
    check_against_oracle(r, spectra, 8)
    assert r["index"] == -2


def test_free_field_degenerate_zero_modes(free):
    """Six-fold degenerate zero modes per chirality (the constant spinors): the
    block of 8 resolves the multiplicity; index 0."""
    r, spectra = gpu_index(free, DIMS)
    check_against_oracle(r, spectra, 8)
    assert (r["n_plus"], r["n_minus"], r["index"]) == (6, 6, 0)


def test_block_too_small(free):
    """A block of 4 cannot hold six zero modes: ENOCONV with the partial result."""
    with pytest.raises(ndq.NdqError) as e:
        gpu_index(free, DIMS, block=4, max_sweeps=40)
    assert e.value.status == -6
    assert e.value.info["theta_plus"][2] < CUT


@pytest.mark.parametrize("q23,want", [(1, -2), (-1, 2)])
def test_index_theorem_8x4(q23, want):
    """8^4 flux backgrounds (no dense oracle): index = -2 q01 q23 in the
    chirality convention used here (the oracle's sign, pinned on 4^4)."""
    dims = (8, 8, 8, 8)
    u = synthetic.flux_gauge_field(dims, 1, q23, noise=0.2, gauge_seed=synthetic.SEED_HAAR)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), ndq.F64, 18)
    start = ndq.SpinorField.pack(g, cu(synthetic.start_vector(g.volume)), ndq.F64, ndq.FULL)
    # 4 exact low modes of Q, the approximant on [lam_next, lam_max] (Sec. 2.3)
    modes, nu, rho, lm = ndq.lowmodes_compute(g, U, M, LMAX, start, 4, tol=1e-10)
    assert lm["lam_next"] > 0.1
    ap = ndq.Approx(ndq.ZOLOTAREV, lm["lam_next"] / LMAX, 12)
    assert ap.delta < 1e-9
    ov = ndq.Overlap(g, M, ap, LMAX, modes=modes, nu=nu, tol=1e-12)
    r = ndq.index_DN(g, U, ov, start, zero_cut=CUT)
    assert r["index"] == want
    assert min(r["n_plus"], r["n_minus"]) == 0
    # the first Ritz value above the cut is the same in both sectors (chiral
    # pairing: a near-zero pair of the noisy background, well above the cut)
    tp, tm = r["theta_plus"][r["n_plus"]], r["theta_minus"][r["n_minus"]]
    assert min(tp, tm) > 10 * CUT
    assert abs(tp - tm) <= 2 * (r["resid_plus"][r["n_plus"]] + r["resid_minus"][r["n_minus"]]) + 1e-12
