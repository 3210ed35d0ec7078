"""Multi-shift CG iterations replayed from captured HIP graphs.

The graph holds the same kernels with the same arguments as the eager
launches, so every replay must give the eager result bit for bit.  Each test
replays several times with the program's own eager work and synchronisations
in between (other inputs, other shapes of the captured block, other
precisions), and checks every replay against the eager result; the eager
result itself is checked against the FP64 oracle.
"""
import numpy as np
import pytest

import synthetic
from oracle import approx, dirac, lowmodes, sign

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1010_5636_amd as ndq  # noqa: E402

M = -1.4
LMAX = 6.6
MQ = 0.05
DIMS = (4, 4, 4, 4)
NEV = 8


def cu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.fixture(scope="module")
def setup():
    u = synthetic.gauge_field(DIMS)
    q = dirac.dense_Q(u, M, DIMS)
    eig = np.linalg.eigh(q)
    nu, m = lowmodes.dense_lowmodes(q, NEV, eig=eig)
    order = np.argsort(np.abs(eig[0]), kind="stable")
    k = abs(eig[0][order[NEV]]) / LMAX
    g = ndq.Geometry(DIMS)
    return {"u": u, "q": q, "eig": eig, "nu": nu, "k": k, "g": g,
            "U64": ndq.GaugeField.pack(g, cu(u), ndq.F64, 18),
            "U32": ndq.GaugeField.pack(g, cu(u), ndq.F32, 12),
            "modes": ndq.SpinorField.pack(g, cu(m.reshape(NEV, 256, 4, 3)), ndq.F64, ndq.FULL),
            "psi": [synthetic.spinor(256, seed=s) for s in (31, 32, 33)]}


def overlap(d, graph, every, prec=ndq.F64, degree=12, tol=1e-13):
    ap = ndq.Approx(ndq.ZOLOTAREV, d["k"], degree)
    return ndq.Overlap(d["g"], M, ap, LMAX, modes=d["modes"], nu=d["nu"], mq=MQ, tol=tol, check_every=every,
                       graph=graph)


def sign_of(d, ov, psi, prec=ndq.F64):
    U = d["U64"] if prec == ndq.F64 else d["U32"]
    x = ndq.SpinorField.pack(d["g"], cu(psi), prec, ndq.FULL)
    y = x.like()
    st = ndq.apply_sign(d["g"], U, ov, x, y)
    torch.cuda.synchronize()
    return y.buf.clone(), y.unpack().cpu().numpy().ravel(), st


@pytest.mark.parametrize("every", [1, 3, 8])
def test_graph_replays_equal_eager_f64(setup, every):
    d = setup
    eager = overlap(d, False, every)
    graph = overlap(d, True, every)
    ref = [sign_of(d, eager, p) for p in d["psi"]]
    # the eager result against the oracle's closed form
    ap = approx.zolotarev(d["k"], 12)
    s_ap = sign.dense_sign_approx(d["q"], ap, LMAX, n_low=NEV, eig=d["eig"])
    for (_, y, _), p in zip(ref, d["psi"]):
        assert np.linalg.norm(y - s_ap @ p.ravel()) <= 1e-10 * np.linalg.norm(p)
    for rep in range(3):
        for j, p in enumerate(d["psi"]):
            raw, _, st = sign_of(d, graph, p)
            assert torch.equal(raw, ref[j][0]), (rep, j)
            assert st["iterations"] == ref[j][2]["iterations"]
            # eager work of another shape between replays
            sign_of(d, eager, d["psi"][(j + 1) % 3])


def test_graph_alternating_precisions(setup):
    """F64 and F32 graphs (different kernels) kept side by side, alternated."""
    d = setup
    e64, g64 = overlap(d, False, 4), overlap(d, True, 4)
    e32, g32 = overlap(d, False, 4, ndq.F32, 6, 1e-6), overlap(d, True, 4, ndq.F32, 6, 1e-6)
    p = d["psi"][0]
    r64 = sign_of(d, e64, p)[0]
    r32 = sign_of(d, e32, p, ndq.F32)[0]
    for _ in range(3):
        assert torch.equal(sign_of(d, g64, p)[0], r64)
        assert torch.equal(sign_of(d, g32, p, ndq.F32)[0], r32)


def test_graph_solve_equals_eager(setup):
    d = setup
    b = ndq.SpinorField.pack(d["g"], cu(d["psi"][1]), ndq.F64, ndq.FULL)
    out = {}
    for graph in (False, True, True):
        ov64 = overlap(d, graph, 8)
        ov32 = overlap(d, graph, 8, ndq.F32, 6, 1e-6)
        x = ndq.SpinorField.pack(d["g"], cu(np.zeros_like(d["psi"][1])), ndq.F64, ndq.FULL)
        st = ndq.solve_DN(d["g"], d["U64"], ov64, b, x, tol=1e-10, U_lo=d["U32"], ov_lo=ov32, inner_prec=ndq.F32)
        torch.cuda.synchronize()
        assert st["residual"] <= 1e-10
        if graph not in out:
            out[graph] = x.buf.clone()
        else:
            assert torch.equal(x.buf, out[graph])
    assert torch.equal(out[True], out[False])


def test_graph_after_new_geometry():
    """A kept graph is never replayed for another lattice, even when a new
    geometry or workspace reuses a freed one's address."""
    import gc
    for dims in ((4, 4, 4, 4), (8, 4, 6, 2), (4, 4, 4, 4), (6, 2, 4, 4)):
        g = ndq.Geometry(dims)
        v = g.volume
        u = synthetic.gauge_field(dims)
        U = ndq.GaugeField.pack(g, cu(u), ndq.F64, 18)
        psi = synthetic.spinor(v, seed=5)
        ap = ndq.Approx(ndq.ZOLOTAREV, 0.08, 10)
        outs = []
        for graph in (False, True, True):
            ov = ndq.Overlap(g, M, ap, LMAX, tol=1e-12, check_every=4, graph=graph)
            x = ndq.SpinorField.pack(g, cu(psi), ndq.F64, ndq.FULL)
            y = x.like()
            ndq.apply_sign(g, U, ov, x, y)
            torch.cuda.synchronize()
            outs.append(y.buf.clone())
            del ov, x, y
        assert torch.equal(outs[1], outs[0]) and torch.equal(outs[2], outs[0]), dims
        ref = sign.sign_rational(lambda w: dirac.apply_Q(u, w, M, dims), psi, approx.zolotarev(0.08, 10), LMAX,
                                 tol=1e-13)
        got = ndq.SpinorField(g, ndq.F64, ndq.FULL, buffer=outs[0]).unpack().cpu().numpy()[0]
        assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(psi)
        del g, U
        gc.collect()
