"""GPU solve of D_N^m x = b (plain FP64 and mixed precision) checked by the oracle.

4^4: the oracle's dense D_N^m with its own approximant coefficients and the
exact 8 low modes gives both the LU solution and the true residual of the
GPU's x.  8^4: the true residual is recomputed by the oracle's operator-form
D_N^m (forward Chebyshev recurrence), with the low modes the GPU found.
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
MQ = 0.05


def cu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.fixture(scope="module")
def setup4():
    dims = (4, 4, 4, 4)
    u = synthetic.gauge_field(dims)
    q = dirac.dense_Q(u, M, dims)
    eig = np.linalg.eigh(q)
    nev = 8
    nu, m = lowmodes.dense_lowmodes(q, nev, eig=eig)
    order = np.argsort(np.abs(eig[0]), kind="stable")
    k = abs(eig[0][order[nev]]) / LMAX
    g = ndq.Geometry(dims)
    d = {"dims": dims, "u": u, "q": q, "eig": eig, "nu": nu, "k": k, "g": g,
         "U64": ndq.GaugeField.pack(g, cu(u), ndq.F64, 18),
         "U32": ndq.GaugeField.pack(g, cu(u), ndq.F32, 12),
         "U16": ndq.GaugeField.pack(g, cu(u), ndq.F16, 12),
         "modes": ndq.SpinorField.pack(g, cu(m.reshape(nev, 256, 4, 3)), ndq.F64, ndq.FULL),
         "b": synthetic.spinor(256, seed=1002)}
    ref_ap = approx.zolotarev(k, 14)
    s_ap = sign.dense_sign_approx(q, ref_ap, LMAX, n_low=nev, eig=eig)
    d["D"] = overlap.dense_DN(s_ap, S, MQ)
    d["x_lu"] = np.linalg.solve(d["D"], d["b"].ravel())
    return d


def solve(d, inner_prec, kind="rational", sectors=False, b=None):
    g = d["g"]
    ap64 = ndq.Approx(ndq.ZOLOTAREV, d["k"], 14)
    ov64 = ndq.Overlap(g, M, ap64, LMAX, modes=d["modes"], nu=d["nu"], mq=MQ, tol=1e-13)
    if kind == "rational":
        ap_lo = ndq.Approx(ndq.ZOLOTAREV, d["k"], 6)
    else:
        ap_lo = ndq.Approx(ndq.MINMAX_POLY, d["k"] ** 2, 70)
    ov_lo = ndq.Overlap(g, M, ap_lo, LMAX, modes=d["modes"], nu=d["nu"], mq=MQ, tol=1e-6)
    bnp = d["b"] if b is None else b
    b = ndq.SpinorField.pack(g, cu(bnp), ndq.F64, ndq.FULL)
    x = ndq.SpinorField.pack(g, cu(np.zeros_like(bnp)), ndq.F64, ndq.FULL)
    U_lo = {ndq.F64: None, ndq.F32: d["U32"], ndq.F16: d["U16"]}[inner_prec]
    st = ndq.solve_DN(g, d["U64"], ov64, b, x, tol=1e-10, U_lo=U_lo, ov_lo=None if inner_prec == ndq.F64 else ov_lo,
                      inner_prec=inner_prec, inner_tol=0 if inner_prec != ndq.F16 else 2e-3, max_outer=30,
                      sectors=sectors)
    return x.unpack().cpu().numpy().ravel(), st


@pytest.mark.parametrize("inner_prec,kind,sectors", [(ndq.F64, "rational", False), (ndq.F32, "rational", False),
                                                     (ndq.F32, "polynomial", False), (ndq.F16, "polynomial", False),
                                                     (ndq.F64, "rational", True), (ndq.F32, "polynomial", True),
                                                     (ndq.F16, "polynomial", True)])
def test_solve_4c4(setup4, inner_prec, kind, sectors):
    x, st = solve(setup4, inner_prec, kind, sectors)
    b = setup4["b"].ravel()
    true_res = np.linalg.norm(b - setup4["D"] @ x) / np.linalg.norm(b)
    assert true_res <= 1.2e-10, (true_res, st)
    assert st["residual"] <= 1e-10
    assert np.linalg.norm(x - setup4["x_lu"]) <= 1e-8 * np.linalg.norm(setup4["x_lu"])
    if inner_prec != ndq.F64:
        assert st["outer"] >= 2


@pytest.mark.parametrize("inner_prec", [ndq.F64, ndq.F32])
def test_chiral_point_source_one_sector(setup4, inner_prec):
    """A spin-colour point source is chiral (gamma5 is diagonal in the chiral
    basis): the sector solver needs one sector and one sign per iteration.  Both
    solvers reach the LU solution.  In FP64 the sector solver needs well under
    the Q applies of CGNE; in mixed precision the squared conditioning of the
    sector equations costs an extra outer step, which eats the gain."""
    d = setup4
    b = synthetic.point_sources(256)[7]          # spin 2: chirality -1
    x_lu = np.linalg.solve(d["D"], b.ravel())
    out = {}
    for sectors in (False, True):
        x, st = solve(d, inner_prec, "rational", sectors, b=b)
        true_res = np.linalg.norm(b.ravel() - d["D"] @ x) / np.linalg.norm(b)
        assert true_res <= 1.2e-10, (sectors, true_res, st)
        assert np.linalg.norm(x - x_lu) <= 1e-8 * np.linalg.norm(x_lu)
        out[sectors] = st
    if inner_prec == ndq.F64:
        assert out[True]["q_applies"] < 0.7 * out[False]["q_applies"], out
    else:
        assert out[True]["q_applies"] < 1.3 * out[False]["q_applies"], out


def test_solve_8c4_operator_form():
    dims = (8, 8, 8, 8)
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims, seed=11)
    g = ndq.Geometry(dims)
    U64 = ndq.GaugeField.pack(g, cu(u), ndq.F64, 18)
    U32 = ndq.GaugeField.pack(g, cu(u), ndq.F32, 12)
    start = ndq.SpinorField.pack(g, cu(synthetic.start_vector(v)), ndq.F64, ndq.FULL)
    nev = 12
    modes, nu, rho, info = ndq.lowmodes_compute(g, U64, M, LMAX, start, nev, tol=1e-11)
    k = (info["lam_next"] - info["rho_next"]) / LMAX
    ref_poly = approx.minimax_polynomial(k * k, 260)
    assert ref_poly.delta < 1e-13
    ap64 = ndq.Approx.from_coeffs(ndq.MINMAX_POLY, ref_poly.c, lo=k * k, delta=ref_poly.delta)
    ap_lo = ndq.Approx(ndq.MINMAX_POLY, k * k, 90)
    ov64 = ndq.Overlap(g, M, ap64, LMAX, modes=modes, nu=nu, mq=MQ)
    ov_lo = ndq.Overlap(g, M, ap_lo, LMAX, modes=modes, nu=nu, mq=MQ)
    bnp = synthetic.spinor(v, seed=1002)
    b = ndq.SpinorField.pack(g, cu(bnp), ndq.F64, ndq.FULL)
    um = modes.unpack().cpu().numpy()
    apq = lambda w: dirac.apply_Q(u, w, M, dims)
    sgn = lambda w: sign.project_literal(lambda t: sign.sign_polynomial(apq, t, ref_poly, LMAX), um, nu, w)
    for sectors in (False, True):
        x = ndq.SpinorField.pack(g, cu(np.zeros_like(bnp)), ndq.F64, ndq.FULL)
        st = ndq.solve_DN(g, U64, ov64, b, x, tol=1e-10, U_lo=U32, ov_lo=ov_lo, inner_prec=ndq.F32, sectors=sectors)
        xs = x.unpack().cpu().numpy()[0]
        res = bnp - overlap.apply_DN(sgn, xs, S, MQ)
        assert np.linalg.norm(res) / np.linalg.norm(bnp) <= 1.5e-10, (sectors, st)
