"""GPU low-mode solver (Sec. 2.3) against dense diagonalisation and the oracle.

* 4^4 random links, l = 8: eigenvalues vs the dense spectrum of Q, residues
  rho_k recomputed by the oracle, orthonormality, the Eq. 10 bound against the
  true projector deviation, and sign(Q) with these modes vs the oracle's closed
  form with exact modes.
* 8^4 random links, l = 12: residues recomputed by the oracle's stencil.
* 4^4 free field, l = 48 (block method): the exactly 48-fold degenerate
  |lambda| = 0.6 eigenspace, projector against the exact one.
* the block method with an F32 filter phase (4^4 against the dense spectrum, 8^4
  against the FP64-only run and the oracle's residues).
* every run: the library's kappa_+-, Eq. 10 bounds (Eq. 9, Eq. 10) against the
  oracle's gap_distances / kappas / projector_bound evaluated on the library's
  own nu, rho and certified lower gap lam_next - rho_next (relative 1e-10).
All three methods (block subspace iteration, thick-restart Lanczos, and the
paper's Ritz-functional minimisation) are exercised.
"""
import numpy as np
import pytest

import synthetic
from oracle import approx, dirac, geometry, lowmodes, sign

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1010_5636_amd as ndq  # noqa: E402

M = -1.4
LMAX = 6.6


def cu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def run(dims, u, nev, nextra=8, tol=1e-11, basis=0, method=ndq.ndq.LM_SUBSPACE):
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), ndq.F64, 18)
    v = geometry.volume(dims)
    start = ndq.SpinorField.pack(g, cu(synthetic.start_vector(v)), ndq.F64, ndq.FULL)
    modes, nu, rho, info = ndq.lowmodes_compute(g, U, M, LMAX, start, nev, nextra=nextra, tol=tol, basis=basis,
                                                method=method)
    return g, U, modes, nu, rho, info


METHODS = [ndq.ndq.LM_SUBSPACE, ndq.ndq.LM_LANCZOS, ndq.ndq.LM_RITZ]


def check_diagnostics(nu, rho, info):
    """kappa_+- and the Eq. 10 bounds of the library against the oracle's
    formulas on the same nu, rho and lower gap (first nev_used modes)."""
    l = info["nev_used"]
    d = lowmodes.gap_distances(nu[:l], info["lam_next"] - info["rho_next"])
    kp, km = lowmodes.kappas(nu[:l], rho[:l], d)
    for got, ref in ((info["kappa_plus"], kp), (info["kappa_minus"], km),
                     (info["bound_plus"], lowmodes.projector_bound(kp)),
                     (info["bound_minus"], lowmodes.projector_bound(km))):
        assert abs(got - ref) <= 1e-10 * abs(ref) + 1e-300, (got, ref, info)
    assert info["rho_next"] >= 0.0 and info["lam_next"] - info["rho_next"] > np.abs(nu[:l]).max()


@pytest.fixture(scope="module")
def dense4():
    u = synthetic.gauge_field((4, 4, 4, 4))
    q = dirac.dense_Q(u, M, (4, 4, 4, 4))
    lam, w = np.linalg.eigh(q)
    return {"u": u, "q": q, "eig": (lam, w), "order": np.argsort(np.abs(lam), kind="stable")}


@pytest.mark.parametrize("method", METHODS)
def test_lowmodes_random_4c4(dense4, method):
    nev = 8
    g, U, modes, nu, rho, info = run((4, 4, 4, 4), dense4["u"], nev, method=method)
    lam = dense4["eig"][0][dense4["order"]]
    assert np.allclose(np.sort(nu), np.sort(lam[:nev]), atol=1e-10), (nu, lam[:nev + 2])
    assert np.all(rho <= 1e-11 * LMAX)
    um = modes.unpack().cpu().numpy().reshape(nev, -1)
    assert np.abs(um.conj() @ um.T - np.eye(nev)).max() < 1e-12
    # rho_k recomputed with the oracle's stencil
    qu = dirac.apply_Q(dense4["u"], um.reshape(nev, 256, 4, 3), M, (4, 4, 4, 4)).reshape(nev, -1)
    rho_o = np.linalg.norm(qu - nu[:, None] * um, axis=1)
    assert np.allclose(rho, rho_o, rtol=1e-3, atol=1e-13)
    assert abs(info["lam_next"] - abs(lam[nev])) < 1e-6
    assert info["lam_next"] - info["rho_next"] <= abs(lam[nev]) + 1e-12
    check_diagnostics(nu, rho, info)
    # Eq. 10 against the true projector deviation
    nu_ex, m_ex = lowmodes.dense_lowmodes(dense4["q"], nev, eig=dense4["eig"])
    for sgn, bound in ((1, info["bound_plus"]), (-1, info["bound_minus"])):
        pe = m_ex[np.sign(nu_ex) == sgn]
        pg = um[np.sign(nu) == sgn]
        dev = np.linalg.norm(pg.T @ pg.conj() - pe.T @ pe.conj(), 2)
        assert dev <= bound + 1e-12


def test_sign_with_computed_modes(dense4):
    nev = 8
    g, U, modes, nu, rho, info = run((4, 4, 4, 4), dense4["u"], nev)
    k = abs(dense4["eig"][0][dense4["order"][nev]]) / LMAX
    ap, ref_ap = ndq.Approx(ndq.ZOLOTAREV, k, 10), approx.zolotarev(k, 10)
    psi = synthetic.spinor(256, seed=17)
    ov = ndq.Overlap(g, M, ap, LMAX, modes=modes, nu=nu, tol=1e-13)
    x = ndq.SpinorField.pack(g, cu(psi), ndq.F64, ndq.FULL)
    y = x.like()
    ndq.apply_sign(g, U, ov, x, y)
    got = y.unpack().cpu().numpy().ravel()
    ref = sign.dense_sign_approx(dense4["q"], ref_ap, LMAX, n_low=nev, eig=dense4["eig"]) @ psi.ravel()
    assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(psi)


@pytest.mark.parametrize("method", METHODS)
def test_lowmodes_8c4_residuals(method):
    dims = (8, 8, 8, 8)
    u = synthetic.gauge_field(dims, seed=5)
    nev = 12
    g, U, modes, nu, rho, info = run(dims, u, nev, tol=1e-10, method=method)
    v = geometry.volume(dims)
    um = modes.unpack().cpu().numpy()
    qu = dirac.apply_Q(u, um, M, dims).reshape(nev, -1)
    rho_o = np.linalg.norm(qu - nu[:, None] * um.reshape(nev, -1), axis=1)
    assert np.all(rho_o <= 1e-10 * LMAX * 1.01)
    gram = um.reshape(nev, -1).conj() @ um.reshape(nev, -1).T
    assert np.abs(gram - np.eye(nev)).max() < 1e-12
    assert np.all(np.abs(nu) <= info["lam_next"] + 1e-12)
    assert np.all(np.diff(np.abs(nu)) >= -1e-14)
    check_diagnostics(nu, rho, info)


@pytest.mark.parametrize("dims,nev,seed", [((4, 4, 4, 4), 8, None), ((8, 8, 8, 8), 12, 5)])
def test_lowmodes_f32_filter_phase(dense4, dims, nev, seed):
    """The subspace method with F32 links for the early filter restarts reaches the
    same FP64 modes: eigenvalues against the dense spectrum (4^4) or the FP64-only
    run (8^4), residues recomputed by the oracle's stencil, orthonormality."""
    u = dense4["u"] if seed is None else synthetic.gauge_field(dims, seed=seed)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), ndq.F64, 18)
    U32 = ndq.GaugeField.pack(g, cu(u), ndq.F32, 12)
    v = geometry.volume(dims)
    start = ndq.SpinorField.pack(g, cu(synthetic.start_vector(v)), ndq.F64, ndq.FULL)
    tol = 1e-11 if seed is None else 1e-10
    modes, nu, rho, info = ndq.lowmodes_compute(g, U, M, LMAX, start, nev, nextra=8, tol=tol, U_lo=U32)
    assert info["restarts_lo"] >= 1 and info["restarts"] > info["restarts_lo"], info
    if seed is None:
        lam = dense4["eig"][0][dense4["order"]]
        ref = np.sort(lam[:nev])
    else:
        _, _, _, nu64, _, _ = run(dims, u, nev, tol=tol)
        ref = np.sort(nu64)
    assert np.allclose(np.sort(nu), ref, atol=1e-9), (nu, ref)
    um = modes.unpack().cpu().numpy()
    qu = dirac.apply_Q(u, um, M, dims).reshape(nev, -1)
    rho_o = np.linalg.norm(qu - nu[:, None] * um.reshape(nev, -1), axis=1)
    assert np.all(rho_o <= tol * LMAX * 1.01)
    gram = um.reshape(nev, -1).conj() @ um.reshape(nev, -1).T
    assert np.abs(gram - np.eye(nev)).max() < 1e-12
    check_diagnostics(nu, rho, info)


def test_lowmodes_f32_filter_rejects_bad_links():
    """U_lo must be F32 links and needs the subspace method."""
    dims = (4, 4, 4, 4)
    u = synthetic.gauge_field(dims)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), ndq.F64, 18)
    start = ndq.SpinorField.pack(g, cu(synthetic.start_vector(256)), ndq.F64, ndq.FULL)
    with pytest.raises(ndq.NdqError):
        ndq.lowmodes_compute(g, U, M, LMAX, start, 4, U_lo=U)
    U32 = ndq.GaugeField.pack(g, cu(u), ndq.F32, 12)
    with pytest.raises(ndq.NdqError):
        ndq.lowmodes_compute(g, U, M, LMAX, start, 4, U_lo=U32, method=ndq.ndq.LM_LANCZOS)


def test_lowmodes_free_field_degenerate():
    """Block subspace iteration resolves the free field's 48-fold |lambda| = 0.6
    eigenspace (gap to sqrt(1.16)); the projector must equal the exact one."""
    dims = (4, 4, 4, 4)
    u = synthetic.cold_gauge(dims)
    nev = 48
    g, U, modes, nu, rho, info = run(dims, u, nev, nextra=12)
    assert np.allclose(np.abs(nu), 0.6, atol=1e-10)
    assert np.sum(nu > 0) == 24
    assert abs(info["lam_next"] - np.sqrt(1.16)) < 1e-6
    um = modes.unpack().cpu().numpy().reshape(nev, -1)
    q = dirac.dense_Q(u, M, dims)
    lam, w = np.linalg.eigh(q)
    pe = w[:, np.abs(np.abs(lam) - 0.6) < 1e-9]
    assert pe.shape[1] == 48
    assert np.linalg.norm(um.T @ um.conj() - pe @ pe.conj().T, 2) < 1e-9
    check_diagnostics(nu, rho, info)


@pytest.mark.parametrize("method", METHODS)
def test_dynamic_number_of_modes(dense4, method):
    """nev_min: the number l of projected modes is the one in [nev_min, nev]
    with the largest relative gap |nu_(l+1)| / |nu_l| (Sec. 2.3), checked
    against the dense spectrum."""
    nev, nev_min = 10, 4
    g = ndq.Geometry((4, 4, 4, 4))
    U = ndq.GaugeField.pack(g, cu(dense4["u"]), ndq.F64, 18)
    start = ndq.SpinorField.pack(g, cu(synthetic.start_vector(256)), ndq.F64, ndq.FULL)
    modes, nu, rho, info = ndq.lowmodes_compute(g, U, M, LMAX, start, nev, tol=1e-11, method=method,
                                                nev_min=nev_min)
    lam = np.abs(dense4["eig"][0][dense4["order"]])
    ratios = [lam[l] / lam[l - 1] for l in range(nev_min, nev + 1)]
    l_expect = nev_min + int(np.argmax(ratios))
    assert info["nev_used"] == l_expect
    assert abs(info["lam_next"] - lam[l_expect]) < 1e-8
    if l_expect < nev:
        assert info["rho_next"] == rho[l_expect]
    check_diagnostics(nu, rho, info)

