"""GPU parity of the index tables, field packing and the Wilson stencil
(Q = gamma5 D_W, the even/odd dslash and Qhat_ee) against the FP64 oracle.

Tolerances (relative L2 per apply): 1e-13 for FP64, 1e-6 for FP32, 5e-3 for
FP16 storage; index tables bit-exact.
"""
import numpy as np
import pytest

import synthetic
from oracle import dirac, geometry

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1010_5636_amd as ndq  # noqa: E402

M = -1.4
TOL = {ndq.F64: 1e-13, ndq.F32: 1e-6, ndq.F16: 5e-3}
# (spinor precision, link precision, recon)
FORMATS = [(ndq.F64, ndq.F64, 18), (ndq.F64, ndq.F64, 12), (ndq.F64, ndq.F64, 8),
           (ndq.F32, ndq.F32, 18), (ndq.F32, ndq.F32, 12), (ndq.F32, ndq.F32, 8),
           (ndq.F32, ndq.F16, 12), (ndq.F16, ndq.F32, 12), (ndq.F16, ndq.F16, 18), (ndq.F16, ndq.F16, 12)]
DIMS = [(4, 4, 4, 4), (8, 4, 6, 2), (2, 6, 2, 10), (6, 10, 4, 6)]


def tol(sp, lp):
    """F16 storage of either field sets the F16 bound."""
    return TOL[ndq.F16] if ndq.F16 in (sp, lp) else TOL[sp]


def rel_l2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def f16_site_bound(nb_psi_norms, self_norm, out_norm):
    """Per-site error bound of Q (or of the dslash) with F16 storage.

    F16 spinors keep each real as a half of value / m (m the site's largest
    |real|): error <= 2^-12 m per real, so <= sqrt(24) 2^-12 |psi(y)| ~ 1.2e-3 |psi(y)|
    per site; F16 links (entries <= 1): |dU|_2 <= |dU|_F <= sqrt(18) 2^-12 ~ 1.04e-3.
    Each hop U (1 -+ gamma) psi(y) has norm <= 2 |psi(y)| and enters with weight
    1/2 (Q) or 1 (dslash); (4+m) = 2.6 weighs the site term; the output is
    rounded once more (1.2e-3 |out(x)|).  With weight 2 for the dslash hops:
        |err(x)| <= 2.5e-3 (sum_y |psi(y)| + 2.6 |psi(x)| + |out(x)|) * 2,
    FP32 arithmetic (~1e-6) included in the margin.  A wrong link or neighbour
    at a single site would exceed it by orders of magnitude."""
    return 5e-3 * (nb_psi_norms + 2.6 * self_norm + out_norm)


def f16_site_errors_ok(got, ref, psi, nb, self_term=True):
    """Largest ratio of the per-site error to f16_site_bound; nb: [sites, 8]
    indices into psi; self_term: Q (psi and the output on the same sites) or
    the dslash (no same-site term)."""
    pn = np.linalg.norm(psi.reshape(psi.shape[0], -1), axis=1)
    nbn = pn[nb].sum(axis=1)
    selfn = pn if self_term else 0.0
    err = np.linalg.norm((got - ref).reshape(got.shape[0], -1), axis=1)
    bound = f16_site_bound(nbn, selfn, np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1))
    return float((err / bound).max())


_CACHE = {}


def problem(dims, cold=False):
    key = (dims, cold)
    if key not in _CACHE:
        v = geometry.volume(dims)
        u = synthetic.cold_gauge(dims) if cold else synthetic.gauge_field(dims)
        psi = synthetic.spinor(v)
        _CACHE[key] = (u, psi, dirac.apply_Q(u, psi, M, dims))
    return _CACHE[key]


@pytest.mark.parametrize("dims", DIMS + [(32, 16, 16, 16), (48, 24, 24, 24)])
def test_tables_bit_exact(dims):
    g = ndq.Geometry(dims)
    nb, leo, nbe = g.tables()
    torch.cuda.synchronize()
    assert np.array_equal(nb.cpu().numpy(), geometry.neighbour_table(dims))
    assert np.array_equal(leo.cpu().numpy(), geometry.lex_of_eo(dims))
    assert np.array_equal(nbe.cpu().numpy(), geometry.eo_neighbour_table(dims))


@pytest.mark.parametrize("prec,recon,tol", [(ndq.F64, 18, 0.0), (ndq.F64, 12, 1e-15), (ndq.F64, 8, 1e-13),
                                             (ndq.F32, 18, 1e-7), (ndq.F32, 12, 3e-7), (ndq.F32, 8, 1e-5),
                                             (ndq.F16, 18, 1e-3), (ndq.F16, 12, 2e-3)])
def test_gauge_pack_roundtrip(prec, recon, tol):
    dims = (8, 4, 6, 2)
    u = synthetic.gauge_field(dims)
    g = ndq.Geometry(dims)
    back = ndq.GaugeField.pack(g, cu(u), prec, recon).unpack().cpu().numpy()
    err = np.abs(back - u).max()
    assert err <= tol, err


def test_gauge_pack_8_singular_cold():
    dims = (4, 4, 4, 4)
    g = ndq.Geometry(dims)
    with pytest.raises(ndq.NdqError) as e:
        ndq.GaugeField.pack(g, cu(synthetic.cold_gauge(dims)), ndq.F32, 8)
    assert e.value.status == -5


@pytest.mark.parametrize("prec,parity", [(p, q) for p in (ndq.F64, ndq.F32, ndq.F16) for q in (ndq.FULL, ndq.EVEN)])
def test_spinor_pack_roundtrip(prec, parity):
    dims = (6, 10, 4, 6)
    g = ndq.Geometry(dims)
    n = g.volume if parity == ndq.FULL else g.volume // 2
    psi = synthetic.spinor(n, nrhs=3)
    back = ndq.SpinorField.pack(g, cu(psi), prec, parity).unpack().cpu().numpy()
    if prec == ndq.F64:
        assert np.array_equal(back, psi)
    else:
        # F32: componentwise rounding; F16: rounding relative to the site's max |component|
        bound = 6e-8 if prec == ndq.F32 else 2 ** -11
        site_max = np.abs(np.stack([psi.real, psi.imag])).max(axis=(0, 3, 4))
        err = np.abs(back - psi).max(axis=(2, 3))
        assert np.all(err <= bound * (site_max if prec == ndq.F16 else np.abs(psi).max(axis=(2, 3))) * 1.5)


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("fmt", FORMATS)
def test_apply_Q_parity(dims, fmt):
    sp, lp, recon = fmt
    u, psi, ref = problem(dims)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), lp, recon)
    x = ndq.SpinorField.pack(g, cu(psi), sp, ndq.FULL)
    y = x.like()
    ndq.apply_Q(g, U, M, x, y)
    got = y.unpack().cpu().numpy()[0]
    assert rel_l2(got, ref) <= tol(sp, lp)
    if ndq.F16 in (sp, lp):
        assert f16_site_errors_ok(got, ref, psi, geometry.neighbour_table(dims)) <= 1.0


@pytest.mark.parametrize("fmt", [(ndq.F64, ndq.F64, 18), (ndq.F64, ndq.F64, 12), (ndq.F32, ndq.F32, 18),
                                 (ndq.F16, ndq.F16, 18)])
def test_apply_Q_cold_free_field(fmt):
    sp, lp, recon = fmt
    dims = (4, 4, 4, 4)
    u, psi, ref = problem(dims, cold=True)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), lp, recon)
    x = ndq.SpinorField.pack(g, cu(psi), sp, ndq.FULL)
    y = x.like()
    ndq.apply_Q(g, U, M, x, y)
    assert rel_l2(y.unpack().cpu().numpy()[0], ref) <= tol(sp, lp)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 6, 2), (6, 10, 4, 6)])
@pytest.mark.parametrize("fmt", [(ndq.F64, ndq.F64, 18), (ndq.F32, ndq.F32, 12), (ndq.F32, ndq.F32, 8),
                                 (ndq.F16, ndq.F16, 12)])
@pytest.mark.parametrize("out_parity", [0, 1])
def test_dslash_parity(dims, fmt, out_parity):
    sp, lp, recon = fmt
    u, _, _ = problem(dims)
    v = geometry.volume(dims)
    psi = synthetic.spinor(v // 2, seed=31 + out_parity)
    ref = dirac.dslash(u, psi, dims, out_parity)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), lp, recon)
    x = ndq.SpinorField.pack(g, cu(psi), sp, 1 - out_parity)
    y = x.like(parity=out_parity)
    ndq.apply_dslash(g, U, x, y)
    assert rel_l2(y.unpack().cpu().numpy()[0], ref) <= tol(sp, lp)


@pytest.mark.parametrize("fmt", [(ndq.F64, ndq.F64, 18), (ndq.F32, ndq.F32, 18), (ndq.F32, ndq.F32, 12),
                                 (ndq.F32, ndq.F32, 8), (ndq.F16, ndq.F16, 12)])
def test_qhat_ee_parity(fmt):
    sp, lp, recon = fmt
    dims = (8, 4, 6, 2)
    u, _, _ = problem(dims)
    v = geometry.volume(dims)
    psi = synthetic.spinor(v // 2, seed=41)
    ref = dirac.qhat_ee(u, psi, M, dims)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), lp, recon)
    x = ndq.SpinorField.pack(g, cu(psi), sp, ndq.EVEN)
    y = x.like()
    t = x.like(parity=ndq.ODD)
    ndq.apply_Qhat_ee(g, U, M, x, y, t)
    assert rel_l2(y.unpack().cpu().numpy()[0], ref) <= tol(sp, lp)


def test_multi_rhs_equals_single():
    dims = (8, 4, 6, 2)
    u, _, _ = problem(dims)
    v = geometry.volume(dims)
    psi = synthetic.spinor(v, nrhs=3, seed=51)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), ndq.F64, 18)
    x = ndq.SpinorField.pack(g, cu(psi), ndq.F64, ndq.FULL)
    y = x.like()
    ndq.apply_Q(g, U, M, x, y)
    got = y.unpack().cpu().numpy()
    for r in range(3):
        assert rel_l2(got[r], dirac.apply_Q(u, psi[r], M, dims)) <= 1e-13


@pytest.mark.parametrize("fmt", [(ndq.F64, ndq.F64, 18), (ndq.F32, ndq.F32, 18), (ndq.F32, ndq.F32, 12),
                                 (ndq.F32, ndq.F32, 8), (ndq.F16, ndq.F16, 12)])
def test_apply_Q_full_size_16c32(fmt):
    """The 16^3 x 32 lattice of the dslash benchmark, full comparison."""
    sp, lp, recon = fmt
    dims = (32, 16, 16, 16)
    u, psi, ref = problem(dims)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), lp, recon)
    x = ndq.SpinorField.pack(g, cu(psi), sp, ndq.FULL)
    y = x.like()
    ndq.apply_Q(g, U, M, x, y)
    got = y.unpack().cpu().numpy()[0]
    assert rel_l2(got, ref) <= tol(sp, lp)
    if ndq.F16 in (sp, lp):
        assert f16_site_errors_ok(got, ref, psi, geometry.neighbour_table(dims)) <= 1.0


@pytest.mark.parametrize("block,xcd", [(0, 0), (64, 0), (128, 1), (256, 0), (256, 1)])
def test_launch_shapes_agree(block, xcd):
    dims = (6, 10, 4, 6)
    u, psi, ref = problem(dims)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), ndq.F64, 18)
    x = ndq.SpinorField.pack(g, cu(psi), ndq.F64, ndq.FULL)
    y = x.like()
    try:
        ndq.ndq.set_launch(block, xcd)
        ndq.apply_Q(g, U, M, x, y)
    finally:
        ndq.ndq.set_launch(0, True)
    assert rel_l2(y.unpack().cpu().numpy()[0], ref) <= 1e-13


BENCH_FORMATS = [(ndq.F32, ndq.F32, 12), (ndq.F32, ndq.F32, 18), (ndq.F32, ndq.F32, 8), (ndq.F64, ndq.F64, 18),
                 (ndq.F16, ndq.F16, 12)]
_DSLASH_REF = {}


def dslash_ref_16c32(out_parity):
    """Oracle even/odd dslash on the 16^3 x 32 benchmark lattice (cached)."""
    if out_parity not in _DSLASH_REF:
        dims = (32, 16, 16, 16)
        u, _, _ = problem(dims)
        psi = synthetic.spinor(geometry.volume(dims) // 2, seed=91 + out_parity)
        _DSLASH_REF[out_parity] = (u, psi, dirac.dslash(u, psi, dims, out_parity))
    return _DSLASH_REF[out_parity]


@pytest.mark.parametrize("fmt", BENCH_FORMATS)
@pytest.mark.parametrize("block,xcd", [(0, 1), (0, 0), (64, 1), (128, 1), (256, 1), (256, 0)])
@pytest.mark.parametrize("out_parity", [ndq.EVEN, ndq.ODD])
def test_dslash_full_size_16c32_every_shape(fmt, block, xcd, out_parity):
    """The benchmarked operator (even/odd dslash on 16^3 x 32, every format) in every
    launch shape the autotuner can pick, against the oracle over all sites."""
    sp, lp, recon = fmt
    dims = (32, 16, 16, 16)
    u, psi, ref = dslash_ref_16c32(out_parity)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), lp, recon)
    x = ndq.SpinorField.pack(g, cu(psi), sp, 1 - out_parity)
    y = x.like(parity=out_parity)
    try:
        ndq.set_launch_for(sp, lp, recon, block, bool(xcd))
        ndq.apply_dslash(g, U, x, y)
    finally:
        ndq.set_launch(0, True)
    got = y.unpack().cpu().numpy()[0]
    assert rel_l2(got, ref) <= tol(sp, lp)
    if ndq.F16 in (sp, lp):
        nb = geometry.eo_neighbour_table(dims)[out_parity]
        assert f16_site_errors_ok(got, ref, psi, nb, self_term=False) <= 1.0


@pytest.mark.parametrize("fmt", [(ndq.F64, ndq.F64, 18), (ndq.F32, ndq.F32, 12), (ndq.F16, ndq.F16, 12)])
def test_apply_Q_sampled_24c48(fmt):
    """Q on the 24^3 x 48 solve lattice in the solver's formats, checked at 200
    sampled sites (and every face of the lattice) against the oracle's per-site Eq. 1."""
    sp, lp, recon = fmt
    dims = (48, 24, 24, 24)
    v = geometry.volume(dims)
    u, psi, _ = _big_24c48()
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), lp, recon)
    x = ndq.SpinorField.pack(g, cu(psi), sp, ndq.FULL)
    y = x.like()
    ndq.apply_Q(g, U, M, x, y)
    rng = np.random.default_rng(17)
    corners = np.array([[0, 0, 0, 0], [47, 23, 23, 23], [0, 23, 0, 23], [47, 0, 11, 0]])
    sites = np.concatenate([geometry.lex_of(dims, corners), rng.integers(0, v, 200)])
    got = y.unpack()[0][torch.from_numpy(sites).to("cuda")].cpu().numpy()
    ref = dirac.apply_Q_at(u, lambda i: psi[i], M, dims, sites)
    assert rel_l2(got, ref) <= tol(sp, lp)


_BIG = {}


def _big_24c48():
    if "f" not in _BIG:
        dims = (48, 24, 24, 24)
        v = geometry.volume(dims)
        _BIG["f"] = (synthetic.gauge_field(dims), synthetic.spinor(v, seed=1002), None)
    return _BIG["f"]
