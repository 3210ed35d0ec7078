"""GPU solve of D_N^m x = b (plain FP64 and mixed precision) checked by the oracle.

4^4: the oracle's dense D_N^m with its own approximant coefficients and the
exact 8 low modes gives both the LU solution and the true residual of the
GPU's x (also with inexact modes, rho ~ 1e-6).  8x8x8x16: the library's FP64
D_N^m and the true residuals of mixed F32 and F16-storage solves are
recomputed by the oracle's operator-form D_N^m (forward Chebyshev recurrence,
sandwich projection with the low modes the library found).
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


_SETUP4 = {}


@pytest.fixture(scope="module")
def setup4():
    return _setup4_cache()


def _setup4_cache():
    if _SETUP4:
        return _SETUP4
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
    _SETUP4.update(d)
    return _SETUP4


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


def _poly_for(k, target):
    """Oracle minimax polynomial of the smallest degree (in steps of 8) with delta <= target."""
    n = max(8, int(0.8 * np.log(2.0 / target) / (2.0 * k)) - 16)
    while True:
        p = approx.minimax_polynomial(k * k, n)
        if p.delta <= target:
            return p
        n += 8


def test_production_lattice_apply_and_solves():
    """8x8x8x16 (every extent >= 8; the FP64 full Q and the multi-RHS stencil
    take their slice-chunked tile order here, as on 24^3x48).  With 16 low modes
    from the library and an FP64 minimax polynomial (delta <= 1e-4) computed by
    the oracle and handed to the library:

    * the library's FP64 D_N^m psi against the oracle's operator form (forward
      Chebyshev recurrence, sandwich projection with the library's modes),
      element by element;
    * mixed-precision solves (F32 arithmetic on F32 storage, and on F16
      storage) checked by the oracle's true residual |b - D x| / |b| <= 1.5e-10.

    The oracle evaluates D_N^m once on the stack of the three fields (psi and
    the two solutions): about 2 n + 2 stacked Q applies, ~40 s on one core.
    """
    dims = (8, 8, 8, 16)
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims, seed=13)
    g = ndq.Geometry(dims)
    U64 = ndq.GaugeField.pack(g, cu(u), ndq.F64, 18)
    U32 = ndq.GaugeField.pack(g, cu(u), ndq.F32, 12)
    U16 = ndq.GaugeField.pack(g, cu(u), ndq.F16, 12)
    start = ndq.SpinorField.pack(g, cu(synthetic.start_vector(v)), ndq.F64, ndq.FULL)
    nev = 16
    modes, nu, rho, info = ndq.lowmodes_compute(g, U64, M, LMAX, start, nev, nextra=16, tol=1e-11)
    k = (info["lam_next"] - info["rho_next"]) / LMAX
    ref_poly = _poly_for(k, 1e-4)
    ap64 = ndq.Approx.from_coeffs(ndq.MINMAX_POLY, ref_poly.c, lo=k * k, delta=ref_poly.delta)
    ap_lo = ndq.Approx(ndq.MINMAX_POLY, k * k, max(8, len(ref_poly.c) - 1 - 24))
    ov64 = ndq.Overlap(g, M, ap64, LMAX, modes=modes, nu=nu, mq=MQ, form=ndq.ndq.SANDWICH)
    ov_lo = ndq.Overlap(g, M, ap_lo, LMAX, modes=modes, nu=nu, mq=MQ)
    psi = synthetic.spinor(v, seed=21)
    bnp = synthetic.spinor(v, seed=1002)
    b = ndq.SpinorField.pack(g, cu(bnp), ndq.F64, ndq.FULL)
    x_in = ndq.SpinorField.pack(g, cu(psi), ndq.F64, ndq.FULL)
    y = x_in.like()
    ndq.apply_DN(g, U64, ov64, x_in, y)
    dn_gpu = y.unpack().cpu().numpy()[0]
    sols = {}
    for name, prec, Ulo, itol in (("f32", ndq.F32, U32, 0.0), ("f16", ndq.F16, U16, 2e-3)):
        x = ndq.SpinorField.pack(g, cu(np.zeros_like(bnp)), ndq.F64, ndq.FULL)
        st = ndq.solve_DN(g, U64, ov64, b, x, tol=1e-10, U_lo=Ulo, ov_lo=ov_lo, inner_prec=prec, inner_tol=itol,
                          max_outer=30)
        assert st["residual"] <= 1e-10 and st["outer"] >= 2, (name, st)
        sols[name] = x.unpack().cpu().numpy()[0]
    um = modes.unpack().cpu().numpy()
    apq = lambda w: dirac.apply_Q(u, w, M, dims)
    sgn = lambda w: sign.project_sandwich(lambda t: sign.sign_polynomial(apq, t, ref_poly, LMAX), um, nu, w)
    stack = np.stack([psi, sols["f32"], sols["f16"]])
    ref = overlap.apply_DN(sgn, stack, S, MQ)
    err = np.abs(dn_gpu - ref[0]).max() / np.abs(ref[0]).max()
    assert err <= 1e-11, err
    assert np.linalg.norm(dn_gpu - ref[0]) <= 1e-12 * np.linalg.norm(ref[0])
    for j, name in ((1, "f32"), (2, "f16")):
        res = np.linalg.norm(bnp - ref[j]) / np.linalg.norm(bnp)
        assert res <= 1.5e-10, (name, res)


def test_solve_with_loose_modes():
    """Low modes with residues rho ~ 1e-6 (exact modes plus noise, Rayleigh-Ritz
    in their span): the solve's operators use the sandwich projection of
    Eq. 11, exactly Hermitian, so CGNE with D^H = gamma5 D gamma5 is consistent
    and the mixed solve converges in a few outer steps.  The oracle builds the
    same operator (dense approximant of Q on all modes, sandwich projection with
    these modes) and checks the true residual."""
    d = _setup4_cache()
    q, nev = d["q"], 8
    nu_ex, m_ex = lowmodes.dense_lowmodes(q, nev, eig=d["eig"])
    rng = np.random.default_rng(8)
    noisy = m_ex + 4e-9 * (rng.normal(size=m_ex.shape) + 1j * rng.normal(size=m_ex.shape))
    nu, um = lowmodes.rayleigh_ritz(lambda w: q @ w, noisy)
    rho = lowmodes.residues(lambda w: q @ w, um, nu)
    assert 1e-7 < rho.max() < 1e-5
    g = d["g"]
    k = d["k"]
    md = ndq.SpinorField.pack(g, cu(um.reshape(nev, 256, 4, 3)), ndq.F64, ndq.FULL)
    ap64, ap_lo = ndq.Approx(ndq.ZOLOTAREV, k, 14), ndq.Approx(ndq.MINMAX_POLY, k * k, 70)
    ov64 = ndq.Overlap(g, M, ap64, LMAX, modes=md, nu=nu, mq=MQ, tol=1e-13)
    ov_lo = ndq.Overlap(g, M, ap_lo, LMAX, modes=md, nu=nu, mq=MQ)
    b = ndq.SpinorField.pack(g, cu(d["b"]), ndq.F64, ndq.FULL)
    x = ndq.SpinorField.pack(g, cu(np.zeros_like(d["b"])), ndq.F64, ndq.FULL)
    st = ndq.solve_DN(g, d["U64"], ov64, b, x, tol=1e-10, U_lo=d["U32"], ov_lo=ov_lo, inner_prec=ndq.F32,
                      max_outer=30)
    assert st["residual"] <= 1e-10 and 2 <= st["outer"] <= 4, st
    # the approximant of Q on its whole spectrum, r(Q) t = W r(Lambda / lam_max) W^H t
    lam, w_ev = d["eig"]
    f = approx.zolotarev(k, 14)(lam / LMAX)
    apply_r = lambda t: (w_ev @ (f * (w_ev.conj().T @ t.ravel()))).reshape(t.shape)
    um4 = um.reshape(nev, 256, 4, 3)
    sgn = lambda w: sign.project_sandwich(apply_r, um4, nu, w)
    xs = x.unpack().cpu().numpy()[0]
    bb = d["b"]
    res = bb - overlap.apply_DN(sgn, xs, S, MQ)
    assert np.linalg.norm(res) / np.linalg.norm(bb) <= 1.2e-10
