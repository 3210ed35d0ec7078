"""GPU parity of sign(Q) (Eq. 5, Eq. 11) and D_N^m (Eq. 4, Eq. 12) against the
FP64 oracle.

At 4^4 the oracle is the spectral closed form W f(Lambda) W^H with the oracle's
own approximant coefficients (f = sign on the exactly treated modes); on a
ragged 8x4x6x2 lattice it is the operator form (one CG per shift, forward
Chebyshev recurrence).  The GPU path uses the library's own coefficients
(computed independently in C++).
"""
import numpy as np
import pytest

import synthetic
from oracle import approx, dirac, geometry, lowmodes, overlap, sign

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1010_5636_amd as ndq  # noqa: E402

M = -1.4
S = 0.4
LMAX = 6.6
DIMS = (4, 4, 4, 4)


def cu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def dense():
    u = synthetic.gauge_field(DIMS)
    q = dirac.dense_Q(u, M, DIMS)
    lam, w = np.linalg.eigh(q)
    order = np.argsort(np.abs(lam), kind="stable")
    return {"u": u, "q": q, "eig": (lam, w), "order": order, "psi": synthetic.spinor(256, seed=7)}


@pytest.fixture(scope="module")
def gpu(dense):
    g = ndq.Geometry(DIMS)
    return {"g": g, "U64": ndq.GaugeField.pack(g, cu(dense["u"]), ndq.F64, 18),
            "U32": ndq.GaugeField.pack(g, cu(dense["u"]), ndq.F32, 12)}


def run_sign(gpu, dense, ap, prec=ndq.F64, nev=0, form=ndq.LITERAL, tol=1e-13, dn=False, mq=0.0):
    g = gpu["g"]
    U = gpu["U64"] if prec == ndq.F64 else gpu["U32"]
    modes, nu = None, None
    if nev:
        nu, m = lowmodes.dense_lowmodes(dense["q"], nev, eig=dense["eig"])
        modes = ndq.SpinorField.pack(g, cu(m.reshape(nev, 256, 4, 3)), ndq.F64, ndq.FULL)
    ov = ndq.Overlap(g, M, ap, LMAX, modes=modes, nu=nu, mq=mq, form=form, tol=tol)
    x = ndq.SpinorField.pack(g, cu(dense["psi"]), prec, ndq.FULL)
    y = x.like()
    st = (ndq.apply_DN if dn else ndq.apply_sign)(g, U, ov, x, y)
    return y.unpack().cpu().numpy()[0].ravel(), st


def k_low(dense, nev):
    return np.abs(dense["eig"][0][dense["order"][nev]]) / LMAX


@pytest.mark.parametrize("kind", ["rational", "polynomial"])
def test_sign_f64_no_projection(dense, gpu, kind):
    k = k_low(dense, 0)
    if kind == "rational":
        ap, ref_ap = ndq.Approx(ndq.ZOLOTAREV, k, 10), approx.zolotarev(k, 10)
    else:
        ap, ref_ap = ndq.Approx(ndq.MINMAX_POLY, k * k, 120), approx.minimax_polynomial(k * k, 120)
    got, st = run_sign(gpu, dense, ap)
    ref = sign.dense_sign_approx(dense["q"], ref_ap, LMAX, eig=dense["eig"]) @ dense["psi"].ravel()
    assert rel(got, ref) <= 1e-10, (rel(got, ref), st)
    exact = sign.dense_sign_exact(dense["q"], eig=dense["eig"]) @ dense["psi"].ravel()
    assert np.linalg.norm(got - exact) <= ref_ap.delta * np.linalg.norm(dense["psi"]) * 1.01 + 1e-10
    if kind == "polynomial":
        assert st["q_applies"] == 2 * 120 + 1
    else:
        # CG iterations run in blocks of check_every (8) between convergence checks;
        # the ones after convergence leave every vector unchanged but are executed
        assert 2 * st["iterations"] + 1 <= st["q_applies"] <= 2 * (st["iterations"] + 8) + 1


@pytest.mark.parametrize("form", [ndq.LITERAL, ndq.SANDWICH])
@pytest.mark.parametrize("kind", ["rational", "polynomial"])
def test_sign_f64_low_modes(dense, gpu, form, kind):
    nev = 8
    k = k_low(dense, nev)
    if kind == "rational":
        ap, ref_ap = ndq.Approx(ndq.ZOLOTAREV, k, 10), approx.zolotarev(k, 10)
    else:
        ap, ref_ap = ndq.Approx(ndq.MINMAX_POLY, k * k, 120), approx.minimax_polynomial(k * k, 120)
    got, _ = run_sign(gpu, dense, ap, nev=nev, form=form)
    ref = sign.dense_sign_approx(dense["q"], ref_ap, LMAX, n_low=nev, eig=dense["eig"]) @ dense["psi"].ravel()
    assert rel(got, ref) <= 1e-9
    exact = sign.dense_sign_exact(dense["q"], eig=dense["eig"]) @ dense["psi"].ravel()
    assert np.linalg.norm(got - exact) <= ref_ap.delta * np.linalg.norm(dense["psi"]) * 1.01 + 1e-9


@pytest.mark.parametrize("kind", ["rational", "polynomial"])
def test_sign_f32(dense, gpu, kind):
    nev = 8
    k = k_low(dense, nev)
    if kind == "rational":
        ap, ref_ap = ndq.Approx(ndq.ZOLOTAREV, k, 6), approx.zolotarev(k, 6)
    else:
        ap, ref_ap = ndq.Approx(ndq.MINMAX_POLY, k * k, 60), approx.minimax_polynomial(k * k, 60)
    got, _ = run_sign(gpu, dense, ap, prec=ndq.F32, nev=nev, tol=1e-6)
    ref = sign.dense_sign_approx(dense["q"], ref_ap, LMAX, n_low=nev, eig=dense["eig"]) @ dense["psi"].ravel()
    assert rel(got, ref) <= 2e-5


def test_sign_squares_to_one(dense, gpu):
    """sign(sign psi) = psi to O(delta) (projected Zolotarev, FP64)."""
    nev = 8
    k = k_low(dense, nev)
    ap = ndq.Approx(ndq.ZOLOTAREV, k, 10)
    g = gpu["g"]
    nu, m = lowmodes.dense_lowmodes(dense["q"], nev, eig=dense["eig"])
    modes = ndq.SpinorField.pack(g, cu(m.reshape(nev, 256, 4, 3)), ndq.F64, ndq.FULL)
    ov = ndq.Overlap(g, M, ap, LMAX, modes=modes, nu=nu, tol=1e-13)
    x = ndq.SpinorField.pack(g, cu(dense["psi"]), ndq.F64, ndq.FULL)
    y, z = x.like(), x.like()
    ndq.apply_sign(g, gpu["U64"], ov, x, y)
    ndq.apply_sign(g, gpu["U64"], ov, y, z)
    assert rel(z.unpack().cpu().numpy(), dense["psi"]) <= 3 * ap.delta + 1e-10


def test_dn_massive(dense, gpu):
    nev, mq = 8, 0.05
    k = k_low(dense, nev)
    ap, ref_ap = ndq.Approx(ndq.ZOLOTAREV, k, 10), approx.zolotarev(k, 10)
    got, _ = run_sign(gpu, dense, ap, nev=nev, dn=True, mq=mq)
    s_ap = sign.dense_sign_approx(dense["q"], ref_ap, LMAX, n_low=nev, eig=dense["eig"])
    ref = overlap.dense_DN(s_ap, S, mq) @ dense["psi"].ravel()
    assert rel(got, ref) <= 1e-9


def test_sign_ragged_operator_form():
    """8x4x6x2 (V = 384, ragged against 256-lane blocks): library vs the oracle's
    operator-form sign (independent CG per shift) with the same coefficients."""
    dims = (8, 4, 6, 2)
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims, seed=99)
    psi = synthetic.spinor(v, seed=98)
    k = 0.08
    ref_ap = approx.zolotarev(k, 8)
    ap = ndq.Approx.from_coeffs(ndq.ZOLOTAREV, ref_ap.sigma, ref_ap.beta, lo=k, delta=ref_ap.delta)
    ref = sign.sign_rational(lambda w: dirac.apply_Q(u, w, M, dims), psi, ref_ap, LMAX, tol=1e-13)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), ndq.F64, 18)
    ov = ndq.Overlap(g, M, ap, LMAX, tol=1e-13)
    x = ndq.SpinorField.pack(g, cu(psi), ndq.F64, ndq.FULL)
    y = x.like()
    ndq.apply_sign(g, U, ov, x, y)
    assert rel(y.unpack().cpu().numpy()[0], ref) <= 1e-10


def test_sign_errors(dense, gpu):
    g = gpu["g"]
    ap = ndq.Approx(ndq.ZOLOTAREV, 0.08, 6)
    x = ndq.SpinorField.pack(g, cu(dense["psi"]), ndq.F64, ndq.FULL)
    y = x.like()
    ov = ndq.Overlap(g, M, ap, LMAX, tol=1e-13, max_iter=3, check_every=1)
    with pytest.raises(ndq.NdqError) as e:
        ndq.apply_sign(g, gpu["U64"], ov, x, y)
    assert e.value.status == -6
    nu, m = lowmodes.dense_lowmodes(dense["q"], 2, eig=dense["eig"])
    modes = ndq.SpinorField.pack(g, cu(m.reshape(2, 256, 4, 3)), ndq.F64, ndq.FULL)
    ov = ndq.Overlap(g, M, ap, LMAX, modes=modes, nu=np.array([nu[0], 0.0]))
    with pytest.raises(ndq.NdqError) as e:
        ndq.apply_sign(g, gpu["U64"], ov, x, y)
    assert e.value.status == -5


def test_sign_max_modes_and_shifts(dense, gpu):
    """The documented maxima: 64 exactly treated modes and a 32-pole Zolotarev
    approximant, against the spectral closed form."""
    nev = 64
    k = k_low(dense, nev)
    ap, ref_ap = ndq.Approx(ndq.ZOLOTAREV, k, 32), approx.zolotarev(k, 32)
    got, st = run_sign(gpu, dense, ap, nev=nev)
    ref = sign.dense_sign_approx(dense["q"], ref_ap, LMAX, n_low=nev, eig=dense["eig"]) @ dense["psi"].ravel()
    assert rel(got, ref) <= 1e-9, (rel(got, ref), st)
    with pytest.raises(ndq.NdqError):
        ndq.Approx(ndq.ZOLOTAREV, k, 33)
    nu, m = lowmodes.dense_lowmodes(dense["q"], 65, eig=dense["eig"])
    modes = ndq.SpinorField.pack(gpu["g"], cu(m.reshape(65, 256, 4, 3)), ndq.F64, ndq.FULL)
    ov = ndq.Overlap(gpu["g"], M, ap, LMAX, modes=modes, nu=nu)
    x = ndq.SpinorField.pack(gpu["g"], cu(dense["psi"]), ndq.F64, ndq.FULL)
    with pytest.raises(ndq.NdqError):
        ndq.apply_sign(gpu["g"], gpu["U64"], ov, x, x.like())
