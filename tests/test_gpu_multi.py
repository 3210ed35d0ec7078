"""Persistent launch of Q over several lattices of uneven size, and the
launch-shape autotuner.

Each lattice of a multi-lattice launch must equal its own single-lattice
apply bit for bit (the same per-tile arithmetic) and the FP64 oracle within
the format's tolerance.  The autotuner must leave a launch shape whose
results still match the oracle.
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


def cu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def lattice(dims, nrhs, seed, sp, lp, recon, m=M):
    v = geometry.volume(dims)
    u = synthetic.gauge_field(dims, seed=seed)
    psi = synthetic.spinor(v, nrhs=nrhs, seed=seed + 100)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, cu(u), lp, recon)
    x = ndq.SpinorField.pack(g, cu(psi), sp, ndq.FULL)
    return {"dims": dims, "u": u, "psi": psi, "g": g, "U": U, "x": x, "y": x.like(), "m": m}


@pytest.fixture
def one_lane_per_site():
    ndq.set_launch(64, 1)
    yield
    ndq.set_launch(0, 1)


@pytest.mark.parametrize("fmt", [(ndq.F32, ndq.F32, 12), (ndq.F64, ndq.F64, 18), (ndq.F16, ndq.F16, 12)])
def test_three_uneven_lattices_4_rhs(fmt):
    """8^4, 12^4 and 16^3 x 32 at 4 right-hand sides each, one launch."""
    sp, lp, recon = fmt
    lats = [lattice(d, 4, s, sp, lp, recon) for d, s in (((8, 8, 8, 8), 21), ((12, 12, 12, 12), 22),
                                                        ((32, 16, 16, 16), 23))]
    ndq.apply_Q_multi([(L["g"], L["U"], L["m"], L["x"], L["y"]) for L in lats])
    for L in lats:
        single = L["x"].like()
        ndq.apply_Q(L["g"], L["U"], L["m"], L["x"], single)
        assert torch.equal(L["y"].buf, single.buf), L["dims"]
        got = L["y"].unpack().cpu().numpy()
        tol = TOL[ndq.F16] if ndq.F16 in (sp, lp) else TOL[sp]
        for r in range(4):
            assert rel_l2(got[r], dirac.apply_Q(L["u"], L["psi"][r], L["m"], L["dims"])) <= tol


def test_ragged_jobs(one_lane_per_site):
    """V/2 not a multiple of 64, one right-hand side, nrhs not a multiple of 4,
    different masses; single-rhs jobs compared with the one-lane-per-site kernel."""
    specs = [((6, 10, 4, 6), 1, 31, -1.4), ((4, 4, 4, 4), 3, 32, -1.0), ((8, 4, 6, 2), 5, 33, -1.8),
             ((2, 2, 2, 2), 2, 34, -1.4)]
    lats = [lattice(d, n, s, ndq.F64, ndq.F64, 12, m) for d, n, s, m in specs]
    ndq.apply_Q_multi([(L["g"], L["U"], L["m"], L["x"], L["y"]) for L in lats])
    for L in lats:
        single = L["x"].like()
        ndq.apply_Q(L["g"], L["U"], L["m"], L["x"], single)
        assert torch.equal(L["y"].buf, single.buf), L["dims"]
        got = L["y"].unpack().cpu().numpy()
        for r in range(L["psi"].shape[0]):
            assert rel_l2(got[r], dirac.apply_Q(L["u"], L["psi"][r], L["m"], L["dims"])) <= 1e-13


def test_multi_rejects_mixed_formats():
    a = lattice((4, 4, 4, 4), 1, 41, ndq.F32, ndq.F32, 12)
    b = lattice((4, 4, 4, 4), 1, 42, ndq.F32, ndq.F32, 18)
    with pytest.raises(ndq.NdqError):
        ndq.apply_Q_multi([(a["g"], a["U"], M, a["x"], a["y"]), (b["g"], b["U"], M, b["x"], b["y"])])
    with pytest.raises(ndq.NdqError):
        ndq.apply_Q_multi([])


@pytest.mark.parametrize("fmt", [(ndq.F32, ndq.F32, 12), (ndq.F64, ndq.F64, 18)])
def test_autotune_keeps_parity(fmt):
    sp, lp, recon = fmt
    dims = (32, 16, 16, 16)
    L = lattice(dims, 1, 51, sp, lp, recon)
    try:
        res = ndq.autotune(L["g"], L["U"], sp, reps=50, rotate_bytes=int(6e8))
        assert res["block"] in (0, 64, 128, 256) and res["xcd_remap"] in (0, 1)
        assert res["nsets"] > 1
        assert all(t > 0 for t in res["us"].values())
        # the fastest shape, or the one in use when it is within 3% of the fastest
        assert res["us_best"] <= 1.03 * min(res["us"].values())
        suffix = "_chunked" if res["order"] else ""
        assert res["us_best"] == res["us"][f"block{res['block']}_xcd{res['xcd_remap']}{suffix}"]
        shape = {"block": res["block"], "xcd_remap": res["xcd_remap"]}
        assert ndq.ndq.get_launch_lattice(L["g"], sp, lp, recon, 1) == shape
        # other lattices keep the format's shape
        other = ndq.Geometry((8, 8, 8, 8))
        assert ndq.ndq.get_launch_lattice(other, sp, lp, recon, 1) == ndq.ndq.get_launch(sp, lp, recon)
        resq = ndq.autotune(L["g"], L["U"], sp, reps=20, rotate_bytes=int(6e8), full_q=True)
        assert ndq.ndq.get_launch_lattice(L["g"], sp, lp, recon, 2) == {"block": resq["block"],
                                                                       "xcd_remap": resq["xcd_remap"]}
        ndq.apply_Q(L["g"], L["U"], M, L["x"], L["y"])
        got = L["y"].unpack().cpu().numpy()[0]
        assert rel_l2(got, dirac.apply_Q(L["u"], L["psi"][0], M, dims)) <= TOL[sp]
    finally:
        ndq.set_launch(0, 1)
    assert ndq.ndq.get_launch_lattice(L["g"], sp, lp, recon, 1) == {"block": 0, "xcd_remap": 1}


def test_multi_max_jobs():
    """8 lattices (the maximum) in one launch; 9 are rejected."""
    specs = [((4, 4, 4, 4), 2), ((2, 2, 2, 2), 1), ((8, 4, 6, 2), 3), ((6, 10, 4, 6), 1), ((4, 2, 2, 2), 5),
             ((2, 6, 2, 10), 2), ((8, 8, 8, 8), 4), ((4, 4, 2, 6), 1)]
    lats = [lattice(d, n, 60 + k, ndq.F32, ndq.F32, 18) for k, (d, n) in enumerate(specs)]
    ndq.apply_Q_multi([(L["g"], L["U"], L["m"], L["x"], L["y"]) for L in lats])
    for L in lats:
        got = L["y"].unpack().cpu().numpy()
        for r in range(L["psi"].shape[0]):
            assert rel_l2(got[r], dirac.apply_Q(L["u"], L["psi"][r], L["m"], L["dims"])) <= TOL[ndq.F32]
    extra = lattice((4, 4, 4, 4), 1, 70, ndq.F32, ndq.F32, 18)
    with pytest.raises(ndq.NdqError):
        ndq.apply_Q_multi([(L["g"], L["U"], L["m"], L["x"], L["y"]) for L in lats + [extra]])


def test_multi_grid_factor_and_autotuner():
    """Every grid factor of the persistent launch gives the same bits (the tiles
    are computed alike whichever workgroup walks them); the grid autotuner picks
    one of its factors and leaves the outputs of one apply."""
    lats = [lattice(d, 4, s, ndq.F32, ndq.F32, 12) for d, s in (((8, 8, 8, 8), 81), ((12, 12, 12, 12), 82),
                                                                ((32, 16, 16, 16), 83))]
    jobs = [(L["g"], L["U"], L["m"], L["x"], L["y"]) for L in lats]
    ref = []
    try:
        ndq.ndq.set_multi_grid(4)
        ndq.apply_Q_multi(jobs)
        ref = [L["y"].buf.clone() for L in lats]
        for f in (1, 2, 3, 8, 12, 16):
            ndq.ndq.set_multi_grid(f)
            for L in lats:
                L["y"].buf.zero_()
            ndq.apply_Q_multi(jobs)
            for L, r in zip(lats, ref):
                assert torch.equal(L["y"].buf, r), (f, L["dims"])
        ndq.ndq.set_multi_grid(4)
        for L in lats:
            L["y"].buf.zero_()
        t = ndq.ndq.autotune_multi(jobs, reps=5)
        assert t["factor"] in (1, 2, 3, 4, 6, 8, 12)
        assert ndq.ndq.get_multi_grid() == t["factor"]
        assert len(t["us"]) == 7 and all(v > 0 for v in t["us"].values())
        assert t["us_best"] <= t["us_previous"]
        for L, r in zip(lats, ref):
            assert torch.equal(L["y"].buf, r), L["dims"]
        got = lats[0]["y"].unpack().cpu().numpy()
        L = lats[0]
        assert rel_l2(got[0], dirac.apply_Q(L["u"], L["psi"][0], L["m"], L["dims"])) <= TOL[ndq.F32]
    finally:
        ndq.ndq.set_multi_grid(4)


def test_autotune_mrhs_and_cache(tmp_path, monkeypatch):
    """The work-order autotuner of the multi-RHS stencil picks an order, records
    it for its key, appends it to the NDQ_TUNE_CACHE file, and a second call
    takes it from the file without timing; Q stays at its oracle parity."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("NDQ_TUNE_CACHE", str(cache))
    dims = (8, 8, 8, 16)
    L = lattice(dims, 6, 61, ndq.F32, ndq.F32, 12)
    res = ndq.ndq.autotune_mrhs(L["g"], L["U"], ndq.F32, 6, ny=2, reps=5)
    assert res["cached"] == 0 and res["nshapes"] > 0 and res["us_best"] > 0
    assert res["us_best"] <= res["us_previous"]
    got = ndq.ndq.get_mrhs_launch(L["g"], ndq.F32, ndq.F32, 12, 6, 2)
    assert (got["rg"], got["group_major"], got["chunk"]) == (res["rg"], res["group_major"], res["chunk"])
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and lines[0].startswith("mrhs 8 8 8 16 1 1 12 6 2 ")
    again = ndq.ndq.autotune_mrhs(L["g"], L["U"], ndq.F32, 6, ny=2, reps=5)
    assert again["cached"] == 1 and (again["rg"], again["chunk"]) == (res["rg"], res["chunk"])
    assert len(cache.read_text().strip().splitlines()) == 1
    ndq.apply_Q(L["g"], L["U"], M, L["x"], L["y"])
    got = L["y"].unpack().cpu().numpy()
    for r in range(6):
        assert rel_l2(got[r], dirac.apply_Q(L["u"], L["psi"][r], M, dims)) <= TOL[ndq.F32]
