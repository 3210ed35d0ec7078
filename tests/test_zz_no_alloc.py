"""The allocation-free D_N^m entry point (static device scratch) against the
workspace-taking one: same kernels and arguments, so the results must agree
bit for bit.  Two calls in a row, the second on a smaller lattice, so the
second reuses the scratch the first left behind."""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1010_5636_amd.ndq as ndq  # noqa: E402

M = -1.4
LMAX = 6.6


def cu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def random_modes(v, nev, seed):
    """nev orthonormal fields (stand-ins for low modes: the entry points only project on them)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((v * 12, nev)) + 1j * rng.standard_normal((v * 12, nev))
    q, _ = np.linalg.qr(a)
    return q.T.reshape(nev, v, 4, 3)


def case(dims, prec, recon, kind, nev, form, seed):
    g = ndq.Geometry(dims)
    v = g.volume
    u = cu(synthetic.gauge_field(dims, seed=seed))
    U = ndq.GaugeField.pack(g, u, prec, recon)
    if kind == ndq.ZOLOTAREV:
        ap = ndq.Approx(ndq.ZOLOTAREV, 0.08, 8)
    else:
        ap = ndq.Approx(ndq.MINMAX_POLY, 0.01, 40)
    modes, nu = None, None
    if nev:
        modes = ndq.SpinorField.pack(g, cu(random_modes(v, nev, seed + 1)), ndq.F64, ndq.FULL)
        nu = np.array([0.3, -0.25, 0.41, -0.5, 0.2, -0.33][:nev])
    ov = ndq.Overlap(g, M, ap, LMAX, modes=modes, nu=nu, mq=0.05, form=form, tol=1e-10 if prec != ndq.F64 else 1e-12)
    x = ndq.SpinorField.pack(g, cu(synthetic.spinor(v, seed=seed + 2)), prec, ndq.FULL)
    return g, U, ov, x


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_workspace_entry_point(order):
    print("no-alloc D_N: 8^4 F64 Zolotarev 4 modes, then 4^4 F32 polynomial", flush=True)
    cases = [((8, 8, 8, 8), ndq.F64, 18, ndq.ZOLOTAREV, 4, ndq.SANDWICH, 31),
             ((4, 4, 4, 4), ndq.F32, 12, ndq.MINMAX_POLY, 2, ndq.LITERAL, 41)]
    for dims, prec, recon, kind, nev, form, seed in cases:
        g, U, ov, x = case(dims, prec, recon, kind, nev, form, seed)
        need = int(ndq.lib().ndq_workspace_bytes(g.handle, ndq.ctypes.byref(ov.p), prec, ndq.OP_DN))
        assert 0 < need <= ndq.noalloc_scratch_bytes()
        y_ws, y_na = x.like(), x.like()
        st_ws = ndq.apply_DN(g, U, ov, x, y_ws)
        st_na = ndq.apply_DN_noalloc(g, U, ov, x, y_na)
        torch.cuda.synchronize()
        assert st_na["q_applies"] == st_ws["q_applies"]
        assert st_na["iterations"] == st_ws["iterations"]
        assert torch.equal(y_na.buf, y_ws.buf), f"{dims}: results differ"
        assert float(y_na.unpack().abs().max()) > 0


def test_noalloc_rejects_oversize_and_graph():
    dims = (16, 16, 16, 16)   # five FP64 fields of 12.6 MB exceed the static scratch
    g = ndq.Geometry(dims)
    U = ndq.GaugeField(g, ndq.F64, 18)
    x = ndq.SpinorField(g, ndq.F64, ndq.FULL)
    ov = ndq.Overlap(g, M, ndq.Approx(ndq.MINMAX_POLY, 0.01, 20), LMAX, mq=0.05)
    need = int(ndq.lib().ndq_workspace_bytes(g.handle, ndq.ctypes.byref(ov.p), ndq.F64, ndq.OP_DN))
    assert need > ndq.noalloc_scratch_bytes()
    with pytest.raises(ndq.NdqError) as e:
        ndq.apply_DN_noalloc(g, U, ov, x, x.like())
    assert e.value.status == -4 and "static scratch" in str(e.value)
    small = ndq.Geometry((4, 4, 4, 4))
    ov2 = ndq.Overlap(small, M, ndq.Approx(ndq.ZOLOTAREV, 0.08, 6), LMAX, graph=True)
    xs = ndq.SpinorField(small, ndq.F64, ndq.FULL)
    with pytest.raises(ndq.NdqError) as e:
        ndq.apply_DN_noalloc(small, ndq.GaugeField(small, ndq.F64, 18), ov2, xs, xs.like())
    assert e.value.status == -1
