"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function that include/ndq.h declares, and validates arguments on the
host before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ndq.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ndq_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def ndq():
    import paper_1010_5636_amd as pkg
    try:
        pkg.ndq.lib()
    except RuntimeError as e:  # library not built
        pytest.fail(str(e))
    return pkg.ndq


def test_every_declared_symbol_is_exported(ndq):
    lib = ndq.lib()
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol(ndq):
    assert set(_declared()) <= set(ndq._SIG), set(_declared()) - set(ndq._SIG)


def test_version_and_status_strings(ndq):
    assert "gfx950" in ndq.version()
    assert ndq.status_string(0) == "ok"
    assert ndq.status_string(-2) == "invalid lattice dimensions"


@pytest.mark.parametrize("dims", [(4, 4, 4, 3), (4, 4, 0, 4), (1, 4, 4, 4), (2048, 2048, 2048, 2)])
def test_bad_dims_rejected(ndq, dims):
    with pytest.raises(ndq.NdqError) as e:
        ndq.Geometry(dims)
    assert e.value.status == -2


def test_sizes(ndq):
    g = ndq.Geometry((32, 16, 16, 16))
    v = 131072
    assert g.volume == v
    assert g.gauge_bytes(ndq.F64, 18) == v * 4 * 144
    assert g.gauge_bytes(ndq.F32, 12) == v * 4 * 48
    assert g.gauge_bytes(ndq.F32, 8) == v * 4 * 32 + 256   # links, then the pack's status word
    assert g.gauge_bytes(ndq.F16, 12) == v * 4 * 24
    assert g.spinor_bytes(ndq.F64, ndq.FULL, 1) == v * 192
    assert g.spinor_bytes(ndq.F32, ndq.EVEN, 12) == 12 * v // 2 * 96
    assert g.spinor_bytes(ndq.F16, ndq.ODD, 1) == v // 2 * 52
    assert g.gauge_bytes(7, 18) == 0


def test_set_launch_validation(ndq):
    with pytest.raises(ndq.NdqError):
        ndq.set_launch(96, True)
    ndq.set_launch(0, True)


def test_multi_grid_validation(ndq):
    """The persistent launch's grid factor: 1..16, process-wide, default 4."""
    assert ndq.get_multi_grid() == 4
    for bad in (0, -1, 17):
        with pytest.raises(ndq.NdqError):
            ndq.set_multi_grid(bad)
    try:
        ndq.set_multi_grid(16)
        assert ndq.get_multi_grid() == 16
    finally:
        ndq.set_multi_grid(4)


def test_multi_grid_autotune_validation(ndq):
    """The grid autotuner checks its jobs before any launch (no stream is touched)."""
    import types
    null_stream = types.SimpleNamespace(cuda_stream=0)
    with pytest.raises(ndq.NdqError):
        ndq.autotune_multi([], stream=null_stream)
    with pytest.raises(ndq.NdqError):
        ndq.autotune_multi([], reps=0, stream=null_stream)
    assert ndq.get_multi_grid() == 4


def test_descriptor_validation_before_launch(ndq):
    """Bad descriptors fail on the host (no device memory is touched)."""
    lib = ndq.lib()
    g = ndq.Geometry((4, 4, 4, 4))
    fake = 0x1000  # never dereferenced: validation fails first
    bad_gauge = ndq._Gauge(fake, ndq.F32, 10)
    sp = ndq._Spinor(fake, ndq.F32, ndq.FULL, 1)
    rc = lib.ndq_apply_Q(g.handle, ctypes.byref(bad_gauge), -1.4, ctypes.byref(sp), ctypes.byref(sp), None)
    assert rc == -3
    ok_gauge = ndq._Gauge(fake, ndq.F64, 18)
    rc = lib.ndq_apply_Q(g.handle, ctypes.byref(ok_gauge), -1.4, ctypes.byref(sp), ctypes.byref(sp), None)
    assert rc == -3  # F64 links with F32 spinors
    sp64 = ndq._Spinor(fake, ndq.F64, ndq.FULL, 1)
    rc = lib.ndq_apply_Q(g.handle, ctypes.byref(ok_gauge), -1.4, ctypes.byref(sp64), ctypes.byref(sp64), None)
    assert rc == -1  # in and out alias
    even = ndq._Spinor(fake, ndq.F64, ndq.EVEN, 1)
    rc = lib.ndq_apply_dslash(g.handle, ctypes.byref(ok_gauge), ctypes.byref(even), ctypes.byref(even), None)
    assert rc == -1  # same parity
    f16_8 = ndq._Gauge(fake, ndq.F16, 8)
    rc = lib.ndq_gauge_pack(g.handle, ctypes.c_void_p(fake), ctypes.byref(f16_8), None)
    assert rc == -3
    assert "F16" in lib.ndq_last_error().decode()


@pytest.mark.parametrize("k,n", [(0.0909, 10), (0.05, 6), (0.3, 1), (0.2, 16)])
def test_zolotarev_library_vs_oracle(ndq, k, n):
    """Host-side approximant of the library against the oracle's independent one."""
    from oracle import approx
    a = ndq.Approx(ndq.ZOLOTAREV, k, n)
    sig, beta = a.coeffs()
    ref = approx.zolotarev(k, n)
    assert np.allclose(sig, ref.sigma, rtol=1e-12, atol=0)
    assert np.allclose(beta, ref.beta, rtol=1e-12, atol=0)
    assert abs(a.delta - ref.delta) <= 1e-6 * ref.delta + 1e-14


@pytest.mark.parametrize("eps,n", [(0.0909 ** 2, 40), (0.05 ** 2, 100), (0.01, 0), (0.2 ** 2, 7)])
def test_minmax_library_vs_oracle(ndq, eps, n):
    from oracle import approx
    a = ndq.Approx(ndq.MINMAX_POLY, eps, n)
    c, _ = a.coeffs()
    ref = approx.minimax_polynomial(eps, n)
    assert np.abs(c - ref.c).max() <= 1e-10 * np.abs(ref.c).max()
    assert abs(a.delta - ref.delta) <= 1e-6 * ref.delta + 1e-14


def test_approx_validation(ndq):
    with pytest.raises(ndq.NdqError):
        ndq.Approx(ndq.ZOLOTAREV, 1.5, 4)
    with pytest.raises(ndq.NdqError):
        ndq.Approx(ndq.ZOLOTAREV, 0.1, 0)
    with pytest.raises(ndq.NdqError):
        ndq.Approx(7, 0.1, 3)
    a = ndq.Approx.from_coeffs(ndq.MINMAX_POLY, [1.0, 0.5, 0.25], lo=0.01, delta=0.1)
    assert a.n == 2 and abs(a.delta - 0.1) < 1e-15
    assert np.allclose(a.coeffs()[0], [1.0, 0.5, 0.25])


@pytest.mark.parametrize("n", [1, 3, 17, 64])
def test_host_eigh(ndq, n):
    """The library's host Hermitian eigensolver against numpy's LAPACK eigh."""
    rng = np.random.default_rng(n)
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    a = a + a.conj().T
    w, z = ndq.host_eigh(a)
    assert np.allclose(w, np.linalg.eigvalsh(a), atol=1e-12 * np.abs(w).max())
    assert np.abs(a @ z - z * w).max() < 1e-12 * np.abs(w).max()
    assert np.abs(z.conj().T @ z - np.eye(n)).max() < 1e-12


def test_minmax_library_at_rounding_floor(ndq):
    from oracle import approx
    k, n = 0.0932, 260
    a = ndq.Approx(ndq.MINMAX_POLY, k * k, n)
    c, _ = a.coeffs()
    ref = approx.minimax_polynomial(k * k, n)
    assert a.delta < 1e-13
    assert np.abs(c - ref.c).max() < 1e-12


def test_index_validation_before_launch(ndq):
    """ndq_index_DN rejects bad parameters, precisions and workspaces on the host."""
    lib = ndq.lib()
    g = ndq.Geometry((4, 4, 4, 4))
    fake = 0x1000  # never dereferenced: validation fails first
    a = ndq.Approx(ndq.ZOLOTAREV, 0.09, 8)
    p = ndq._Params(-1.4, 0.0, 6.6, a.handle.value, None, None, 0, 0, 1e-12, 1000, 8, 0)
    U = ndq._Gauge(fake, ndq.F64, 18)
    start = ndq._Spinor(fake, ndq.F64, ndq.FULL, 1)
    info = ndq._IndexInfo()
    by = ctypes.byref
    bad = ndq._IndexParams(65, 8, 10, 0, 1e-7, 1e-7)
    assert lib.ndq_index_workspace_bytes(g.handle, by(p), by(bad)) == 0
    assert lib.ndq_index_DN(g.handle, by(U), by(p), by(bad), by(start), by(info), None, 0, None) == -1
    ok = ndq._IndexParams(0, 0, 0, 0, 0.0, 0.0)
    need = lib.ndq_index_workspace_bytes(g.handle, by(p), by(ok))
    assert need > 3 * 8 * 256 * 192       # three blocks of the default 8 vectors
    start32 = ndq._Spinor(fake, ndq.F32, ndq.FULL, 1)
    assert lib.ndq_index_DN(g.handle, by(U), by(p), by(ok), by(start32), by(info), None, 0, None) == -3
    assert lib.ndq_index_DN(g.handle, by(U), by(p), by(ok), by(start), by(info), None, 0, None) == -4
    assert "workspace" in lib.ndq_last_error().decode()
    assert info.block == 0 and info.index == 0
