"""Batched stencil applies: many right-hand sides on one gauge field in one launch.

Each right-hand side of a batched apply must equal the one-lane-per-site
kernel applied to that right-hand side alone (the same arithmetic in the same
order, so bit for bit), and the FP64 oracle within the format's tolerance.
The full-size case is the 12 spin-colour point sources on 32^3 x 64 at FP32
with 18-real links, checked at every site the oracle can compute one by one
(the source site and its 8 neighbours) and to be exactly zero elsewhere.
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
FORMATS = [(ndq.F64, ndq.F64, 18), (ndq.F64, ndq.F64, 12), (ndq.F64, ndq.F64, 8),
           (ndq.F32, ndq.F32, 18), (ndq.F32, ndq.F32, 12), (ndq.F32, ndq.F32, 8),
           (ndq.F32, ndq.F16, 12), (ndq.F16, ndq.F32, 12), (ndq.F16, ndq.F16, 18), (ndq.F16, ndq.F16, 12)]


def tol(sp, lp):
    return TOL[ndq.F16] if ndq.F16 in (sp, lp) else TOL[sp]


def rel_l2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.fixture
def one_lane_per_site():
    """Route single-right-hand-side applies to the one-lane-per-site kernel."""
    ndq.set_launch(64, 1)
    yield
    ndq.set_launch(0, 1)


def single_rhs_outputs(g, U, psi, sp, apply):
    outs = []
    for r in range(psi.shape[0]):
        x = ndq.SpinorField.pack(g, cu(psi[r]), sp, ndq.FULL)
        y = x.like()
        apply(x, y)
        outs.append(y.buf.clone())
    return outs


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("dims,nrhs", [((8, 4, 6, 2), 12), ((6, 10, 4, 6), 5), ((4, 4, 4, 4), 2)])
def test_batched_Q_equals_single(fmt, dims, nrhs, one_lane_per_site):
    """Ragged cases: nrhs not a multiple of 4, V/2 not a multiple of 64."""
    sp, lp, recon = fmt
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims)
    psi = synthetic.spinor(v, nrhs=nrhs, seed=61)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), lp, recon)
    x = ndq.SpinorField.pack(g, cu(psi), sp, ndq.FULL)
    y = x.like()
    ndq.apply_Q(g, U, M, x, y)
    singles = single_rhs_outputs(g, U, psi, sp, lambda a, b: ndq.apply_Q(g, U, M, a, b))
    rb = g.spinor_bytes(sp, ndq.FULL, 1)
    for r in range(nrhs):
        assert torch.equal(y.buf[r * rb:(r + 1) * rb], singles[r]), f"rhs {r} differs from the single-rhs kernel"
    got = y.unpack().cpu().numpy()
    for r in range(nrhs):
        assert rel_l2(got[r], dirac.apply_Q(u, psi[r], M, dims)) <= tol(sp, lp)


@pytest.mark.parametrize("fmt", [(ndq.F64, ndq.F64, 18), (ndq.F32, ndq.F32, 12), (ndq.F16, ndq.F16, 12)])
@pytest.mark.parametrize("out_parity", [ndq.EVEN, ndq.ODD])
def test_batched_dslash_equals_single(fmt, out_parity, one_lane_per_site):
    sp, lp, recon = fmt
    dims = (8, 4, 6, 2)
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims)
    nrhs = 7
    psi = synthetic.spinor(v // 2, nrhs=nrhs, seed=62)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), lp, recon)
    in_par = ndq.ODD if out_parity == ndq.EVEN else ndq.EVEN
    x = ndq.SpinorField.pack(g, cu(psi), sp, in_par)
    y = x.like(parity=out_parity)
    ndq.apply_dslash(g, U, x, y)
    rb = g.spinor_bytes(sp, out_parity, 1)
    got = y.unpack().cpu().numpy()
    for r in range(nrhs):
        xs = ndq.SpinorField.pack(g, cu(psi[r]), sp, in_par)
        ys = xs.like(parity=out_parity)
        ndq.apply_dslash(g, U, xs, ys)
        assert torch.equal(y.buf[r * rb:(r + 1) * rb], ys.buf)
        ref = dirac.dslash(u, psi[r], dims, out_parity)
        assert rel_l2(got[r], ref) <= tol(sp, lp)


def test_point_sources_32c64():
    """12 point sources on 32^3 x 64, FP32 spinors and 18-real FP32 links, one batched apply."""
    dims = (64, 32, 32, 32)
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), ndq.F32, 18)
    x0 = np.array([63, 0, 31, 17])
    s0 = int(geometry.lex_of(dims, x0))
    canon = torch.zeros((12, v, 4, 3), dtype=torch.complex128, device="cuda")
    for s in range(4):
        for c in range(3):
            canon[3 * s + c, s0, s, c] = 1.0
    x = ndq.SpinorField.pack(g, canon, ndq.F32, ndq.FULL)
    del canon
    y = x.like()
    ndq.apply_Q(g, U, M, x, y)
    out = y.unpack()
    n = np.array(dims)
    near = [s0]
    for mu in range(4):
        e = np.zeros(4, dtype=np.int64)
        e[mu] = 1
        near += [int(geometry.lex_of(dims, (x0 + e) % n)), int(geometry.lex_of(dims, (x0 - e) % n))]
    near = np.array(near)

    def psi_at(idx):
        p = np.zeros((12, len(idx), 4, 3), dtype=np.complex128)
        for k, site in enumerate(idx):
            if site == s0:
                for s in range(4):
                    for c in range(3):
                        p[3 * s + c, k, s, c] = 1.0
        return p

    ref = dirac.apply_Q_at(u, psi_at, M, dims, near)
    got = out[:, torch.from_numpy(near).to("cuda")].cpu().numpy()
    for r in range(12):
        assert rel_l2(got[r], ref[r]) <= TOL[ndq.F32], r
    # nothing leaks beyond the 9 sites: the total norm is the norm at those sites
    total = torch.linalg.vector_norm(out).item()
    assert abs(total - np.linalg.norm(got)) <= 1e-12 * total


@pytest.mark.parametrize("shape", [(0, 0, -1, 1, -1), (1, 1, 0, 1, -1), (3, 1, 2, 0, 1), (5, 0, 4, 1, 0),
                                   (6, 1, 4, 1, -1), (12, 1, 8, 1, 1), (3, 2, 4, 1, -1), (6, 2, 0, 1, -1),
                                   (5, 2, -1, 1, -1)])
def test_work_order_does_not_change_results(shape):
    """Every work order of the multi-RHS stencil (fields per workgroup, group-
    or tile-major order, one group per XCD, tile chunk, XCD remap, link load hint) gives the same
    bits: 12 fields of Q on an 8x8x8x16 lattice (8 tiles of 64 sites per time
    slice; ragged last group for 5 per group), and the even/odd hopping block
    on the same fields."""
    rg, gm, chunk, xcd, nt = shape
    dims = (8, 8, 8, 16)
    g = ndq.Geometry(dims)
    v = g.volume
    U = ndq.GaugeField.pack(g, cu(synthetic.gauge_field(dims, seed=5)), ndq.F32, 12)
    psi = synthetic.spinor(v, nrhs=12, seed=6)
    x = ndq.SpinorField.pack(g, cu(psi), ndq.F32, ndq.FULL)
    xo = ndq.SpinorField.pack(g, cu(psi[:, : v // 2]), ndq.F32, ndq.ODD)
    outs = {}
    for label, sh in (("default", None), ("shape", shape)):
        if sh is not None:
            ndq.ndq.set_mrhs_launch(g, ndq.F32, ndq.F32, 12, 12, 2, rg, gm, chunk, bool(xcd), nt)
            ndq.ndq.set_mrhs_launch(g, ndq.F32, ndq.F32, 12, 12, 1, rg, gm, chunk, bool(xcd), nt)
        y = x.like()
        ndq.apply_Q(g, U, M, x, y)
        ye = xo.like(parity=ndq.EVEN)
        ndq.apply_dslash(g, U, xo, ye)
        torch.cuda.synchronize()
        outs[label] = (y.buf.clone(), ye.buf.clone())
    got = ndq.ndq.get_mrhs_launch(g, ndq.F32, ndq.F32, 12, 12, 2)
    assert (got["rg"], got["group_major"], got["chunk"], got["xcd_remap"]) == (rg, gm, chunk, xcd)
    assert torch.equal(outs["default"][0], outs["shape"][0])
    assert torch.equal(outs["default"][1], outs["shape"][1])
