"""Python binding of libndq (ctypes).

Argument marshalling only: every operation runs in the HIP kernels of
libndq.so.  PyTorch supplies device memory (uint8 buffers sized by the
library's *_bytes queries) and the current HIP stream.  Function names follow
the C entry points without their ``ndq_`` prefix.

Raises ``NdqError`` for any non-zero status and ``RuntimeError`` when the
library has not been built (no silent fallback).
"""
from __future__ import annotations

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libndq.so")
_lib = None

F64, F32, F16 = 0, 1, 2
EVEN, ODD, FULL = 0, 1, 2
ZOLOTAREV, MINMAX_POLY = 0, 1
LITERAL, SANDWICH = 0, 1
LM_SUBSPACE, LM_LANCZOS, LM_RITZ = 0, 1, 2
OP_SIGN, OP_DN, OP_SOLVE = 0, 1, 2

STATUS = {0: "NDQ_OK", -1: "NDQ_EINVAL", -2: "NDQ_EDIMS", -3: "NDQ_EPREC", -4: "NDQ_ENOMEM",
          -5: "NDQ_ESINGULAR", -6: "NDQ_ENOCONV", -7: "NDQ_ENAN", -8: "NDQ_EHIP"}


class NdqError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _Gauge(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("prec", ctypes.c_int32), ("recon", ctypes.c_int32)]


class _Spinor(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("prec", ctypes.c_int32), ("parity", ctypes.c_int32),
                ("nrhs", ctypes.c_int32)]


class _QJob(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("U", ctypes.POINTER(_Gauge)), ("m", ctypes.c_double),
                ("inp", ctypes.POINTER(_Spinor)), ("out", ctypes.POINTER(_Spinor))]


class _TuneResult(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("xcd_remap", ctypes.c_int32), ("us_best", ctypes.c_double),
                ("us", ctypes.c_double * 8), ("nsets", ctypes.c_int32), ("order", ctypes.c_int32),
                ("us_order", ctypes.c_double * 8)]


class _MrhsTuneResult(ctypes.Structure):
    _fields_ = [("rg", ctypes.c_int32), ("group_major", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("link_nt", ctypes.c_int32), ("nshapes", ctypes.c_int32),
                ("cached", ctypes.c_int32), ("us_best", ctypes.c_double), ("us_previous", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class _MultiTuneResult(ctypes.Structure):
    _fields_ = [("factor", ctypes.c_int32), ("nfactors", ctypes.c_int32), ("us", ctypes.c_double * 8),
                ("us_best", ctypes.c_double), ("us_previous", ctypes.c_double)]

    def as_dict(self):
        facs = (1, 2, 3, 4, 6, 8, 12)
        return {"factor": self.factor, "us": {f: self.us[k] for k, f in enumerate(facs[:self.nfactors])},
                "us_best": self.us_best, "us_previous": self.us_previous}


class _Params(ctypes.Structure):
    _fields_ = [("m", ctypes.c_double), ("mq", ctypes.c_double), ("lam_max", ctypes.c_double),
                ("approx", ctypes.c_void_p), ("modes", ctypes.c_void_p), ("nu", ctypes.POINTER(ctypes.c_double)),
                ("nev", ctypes.c_int32), ("form", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32), ("graph", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("q_applies", ctypes.c_int64), ("iterations", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("inner", ctypes.c_int64), ("residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class _LmParams(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int32), ("nextra", ctypes.c_int32), ("basis", ctypes.c_int32),
                ("cheb_degree", ctypes.c_int32), ("cheb_lo", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_restarts", ctypes.c_int32), ("method", ctypes.c_int32), ("nev_min", ctypes.c_int32),
                ("U_lo", ctypes.c_void_p), ("lo_until", ctypes.c_double)]


class _LmInfo(ctypes.Structure):
    _fields_ = [("lam_next", ctypes.c_double), ("kappa_plus", ctypes.c_double), ("kappa_minus", ctypes.c_double),
                ("bound_plus", ctypes.c_double), ("bound_minus", ctypes.c_double), ("cheb_lo", ctypes.c_double),
                ("cheb_degree", ctypes.c_int32), ("restarts", ctypes.c_int32), ("q_applies", ctypes.c_int64),
                ("max_rho", ctypes.c_double), ("rho_next", ctypes.c_double), ("seconds", ctypes.c_double),
                ("nev_used", ctypes.c_int32), ("restarts_lo", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class _IndexParams(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("degree", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tol", ctypes.c_double), ("zero_cut", ctypes.c_double)]


INDEX_REPORT = 16


class _IndexInfo(ctypes.Structure):
    _fields_ = [("n_plus", ctypes.c_int32), ("n_minus", ctypes.c_int32), ("index", ctypes.c_int32),
                ("block", ctypes.c_int32), ("sweeps", ctypes.c_int32 * 2), ("converged", ctypes.c_int32 * 2),
                ("degree", ctypes.c_int32 * 2),
                ("theta", (ctypes.c_double * INDEX_REPORT) * 2), ("resid", (ctypes.c_double * INDEX_REPORT) * 2),
                ("sign_applies", ctypes.c_int64), ("seconds", ctypes.c_double)]

    def as_dict(self):
        n = min(self.block, INDEX_REPORT)
        return {"n_plus": self.n_plus, "n_minus": self.n_minus, "index": self.index, "block": self.block,
                "sweeps": list(self.sweeps), "converged": [bool(c) for c in self.converged],
                "degree": list(self.degree),
                "theta_plus": list(self.theta[0])[:n], "theta_minus": list(self.theta[1])[:n],
                "resid_plus": list(self.resid[0])[:n], "resid_minus": list(self.resid[1])[:n],
                "sign_applies": self.sign_applies, "seconds": self.seconds}


class _SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("max_inner", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("inner_prec", ctypes.c_int32), ("sectors", ctypes.c_int32)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIG = {
    "ndq_last_error": (ctypes.c_char_p, []),
    "ndq_status_string": (ctypes.c_char_p, [_I]),
    "ndq_version": (ctypes.c_char_p, []),
    "ndq_geom_create": (_I, [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_P)]),
    "ndq_geom_destroy": (None, [_P]),
    "ndq_geom_volume": (ctypes.c_int64, [_P]),
    "ndq_geom_tables": (_I, [_P, _P, _P, _P, _P]),
    "ndq_gauge_bytes": (ctypes.c_size_t, [_P, _I, _I]),
    "ndq_spinor_bytes": (ctypes.c_size_t, [_P, _I, _I, _I]),
    "ndq_gauge_pack": (_I, [_P, _P, ctypes.POINTER(_Gauge), _P]),
    "ndq_gauge_unpack": (_I, [_P, ctypes.POINTER(_Gauge), _P, _P]),
    "ndq_spinor_pack": (_I, [_P, _P, ctypes.POINTER(_Spinor), _P]),
    "ndq_spinor_unpack": (_I, [_P, ctypes.POINTER(_Spinor), _P, _P]),
    "ndq_apply_Q": (_I, [_P, ctypes.POINTER(_Gauge), _D, ctypes.POINTER(_Spinor), ctypes.POINTER(_Spinor), _P]),
    "ndq_get_launch_for": (_I, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]),
    "ndq_autotune_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(_Gauge), ctypes.c_int, ctypes.c_int64]),
    "ndq_autotune": (_I, [_P, ctypes.POINTER(_Gauge), ctypes.c_int, ctypes.c_int, ctypes.c_int64, _P, ctypes.c_size_t,
                          ctypes.POINTER(_TuneResult), _P]),
    "ndq_autotune_q_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(_Gauge), ctypes.c_int, ctypes.c_int64]),
    "ndq_autotune_q": (_I, [_P, ctypes.POINTER(_Gauge), ctypes.c_int, ctypes.c_int, ctypes.c_int64, _P, ctypes.c_size_t,
                            ctypes.POINTER(_TuneResult), _P]),
    "ndq_get_launch_lattice": (_I, [_P, _I, _I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "ndq_autotune_mrhs_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "ndq_autotune_mrhs": (_I, [_P, ctypes.POINTER(_Gauge), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P,
                               ctypes.c_size_t, ctypes.POINTER(_MrhsTuneResult), _P]),
    "ndq_gram_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int, ctypes.c_int]),
    "ndq_spinor_gram": (_I, [_P, ctypes.POINTER(_Spinor), ctypes.POINTER(_Spinor), _P, _P, ctypes.c_size_t, _P]),
    "ndq_apply_Q_multi": (_I, [ctypes.POINTER(_QJob), ctypes.c_int32, _P]),
    "ndq_set_multi_grid": (_I, [_I]),
    "ndq_get_multi_grid": (_I, []),
    "ndq_autotune_multi": (_I, [ctypes.POINTER(_QJob), ctypes.c_int32, _I, ctypes.POINTER(_MultiTuneResult), _P]),
    "ndq_apply_dslash": (_I, [_P, ctypes.POINTER(_Gauge), ctypes.POINTER(_Spinor), ctypes.POINTER(_Spinor), _P]),
    "ndq_apply_Qhat_ee": (_I, [_P, ctypes.POINTER(_Gauge), _D, ctypes.POINTER(_Spinor), ctypes.POINTER(_Spinor),
                               ctypes.POINTER(_Spinor), _P]),
    "ndq_approx_create": (_I, [_I, _D, _I, ctypes.POINTER(_P)]),
    "ndq_approx_from_coeffs": (_I, [_I, _I, ctypes.POINTER(_D), ctypes.POINTER(_D), _D, _D, ctypes.POINTER(_P)]),
    "ndq_approx_info": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "ndq_approx_coeffs": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "ndq_approx_destroy": (None, [_P]),
    "ndq_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(_Params), _I, _I]),
    "ndq_workspace_bytes_nrhs": (ctypes.c_size_t, [_P, ctypes.POINTER(_Params), _I, _I, _I]),
    "ndq_apply_sign": (_I, [_P, ctypes.POINTER(_Gauge), ctypes.POINTER(_Params), ctypes.POINTER(_Spinor),
                            ctypes.POINTER(_Spinor), _P, ctypes.c_size_t, ctypes.POINTER(_Stats), _P]),
    "ndq_apply_DN": (_I, [_P, ctypes.POINTER(_Gauge), ctypes.POINTER(_Params), ctypes.POINTER(_Spinor),
                          ctypes.POINTER(_Spinor), _P, ctypes.c_size_t, ctypes.POINTER(_Stats), _P]),
    "ndq_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "ndq_apply_DN_noalloc": (_I, [_P, ctypes.POINTER(_Gauge), ctypes.POINTER(_Params), ctypes.POINTER(_Spinor),
                                  ctypes.POINTER(_Spinor), ctypes.POINTER(_Stats), _P]),
    "ndq_lowmodes_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(_LmParams)]),
    "ndq_lowmodes_compute": (_I, [_P, ctypes.POINTER(_Gauge), _D, _D, ctypes.POINTER(_LmParams),
                                  ctypes.POINTER(_Spinor), _P, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                  ctypes.POINTER(_LmInfo), _P, ctypes.c_size_t, _P]),
    "ndq_host_eigh": (_I, [_I, _P, _P, _P]),
    "ndq_index_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(_Params), ctypes.POINTER(_IndexParams)]),
    "ndq_index_DN": (_I, [_P, ctypes.POINTER(_Gauge), ctypes.POINTER(_Params), ctypes.POINTER(_IndexParams),
                          ctypes.POINTER(_Spinor), ctypes.POINTER(_IndexInfo), _P, ctypes.c_size_t, _P]),
    "ndq_solve_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(_Params), ctypes.POINTER(_Params),
                                                    ctypes.POINTER(_SolveParams)]),
    "ndq_solve_workspace_bytes_nrhs": (ctypes.c_size_t, [_P, ctypes.POINTER(_Params), ctypes.POINTER(_Params),
                                                         ctypes.POINTER(_SolveParams), _I]),
    "ndq_solve_DN": (_I, [_P, ctypes.POINTER(_Gauge), ctypes.POINTER(_Gauge), ctypes.POINTER(_Params),
                          ctypes.POINTER(_Params), ctypes.POINTER(_SolveParams), ctypes.POINTER(_Spinor),
                          ctypes.POINTER(_Spinor), _P, ctypes.c_size_t, ctypes.POINTER(_Stats), _P]),
    "ndq_gauge_force": (_I, [_P, ctypes.POINTER(_Gauge), ctypes.POINTER(_Spinor), ctypes.POINTER(_Spinor), _P, _P,
                             _P]),
    "ndq_set_launch": (_I, [_I, _I]),
    "ndq_set_mrhs_launch": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _I, _I, _I]),
    "ndq_get_mrhs_launch": (_I, [_P, _I, _I, _I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                                 ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "ndq_set_launch_for": (_I, [_I, _I, _I, _I, _I]),
}


def lib():
    """The loaded libndq.so (loads it on first use; raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with paper_1010_5636_amd.build.build()")
        handle = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in _SIG.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(rc: int):
    if rc != 0:
        raise NdqError(rc, lib().ndq_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def status_string(status: int) -> str:
    return lib().ndq_status_string(status).decode()


def version() -> str:
    return lib().ndq_version().decode()


def set_launch(block: int, xcd_remap: bool = True):
    """Launch shape for every storage format (block 0 = direction split)."""
    _check(lib().ndq_set_launch(block, int(bool(xcd_remap))))


def autotune(geom: "Geometry", U: "GaugeField", sprec: int, reps: int = 100, rotate_bytes: int = 0,
             full_q: bool = False, stream=None) -> dict:
    """Time every stencil launch shape of the dslash (or, with ``full_q``, of Q) on
    this lattice and format, and keep the fastest for them."""
    r = _TuneResult()
    pre = "ndq_autotune_q" if full_q else "ndq_autotune"
    n = int(getattr(lib(), pre + "_workspace_bytes")(geom.handle, ctypes.byref(U.desc), int(sprec), int(rotate_bytes)))
    if n == 0:
        raise NdqError(-1, f"bad arguments for {pre}_workspace_bytes")
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    _check(getattr(lib(), pre)(geom.handle, ctypes.byref(U.desc), int(sprec), int(reps), int(rotate_bytes), _ptr(ws),
                               n, ctypes.byref(r), _stream(stream)))
    del ws
    shapes = {f"block{b}_xcd{x}": r.us[2 * i + x] for i, b in enumerate((0, 64, 128, 256)) for x in (0, 1)}
    shapes.update({f"block{b}_xcd{x}_chunked": r.us_order[2 * i + x] for i, b in enumerate((0, 64, 128, 256))
                   for x in (0, 1)})
    return {"block": r.block, "xcd_remap": r.xcd_remap, "order": r.order, "us_best": r.us_best, "us": shapes,
            "nsets": r.nsets}


def autotune_mrhs(geom: "Geometry", U: "GaugeField", sprec: int, nrhs: int, ny: int = 2, reps: int = 10,
                  stream=None) -> dict:
    """Time the work orders of the multi-RHS stencil for this key and keep the fastest
    (or apply the entry of the NDQ_TUNE_CACHE file)."""
    n = int(lib().ndq_autotune_mrhs_workspace_bytes(geom.handle, int(sprec), int(nrhs), int(ny)))
    if n == 0:
        raise NdqError(-1, "bad arguments for ndq_autotune_mrhs_workspace_bytes")
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    r = _MrhsTuneResult()
    _check(lib().ndq_autotune_mrhs(geom.handle, ctypes.byref(U.desc), int(sprec), int(nrhs), int(ny), int(reps),
                                   _ptr(ws), n, ctypes.byref(r), _stream(stream)))
    return r.as_dict()


def get_launch_lattice(geom: "Geometry", sprec: int, lprec: int, recon: int, ny: int = 1) -> dict:
    """The launch shape used on this lattice (the tuned one, else the format's)."""
    b = ctypes.c_int()
    x = ctypes.c_int()
    _check(lib().ndq_get_launch_lattice(geom.handle, sprec, lprec, recon, ny, ctypes.byref(b), ctypes.byref(x)))
    return {"block": b.value, "xcd_remap": x.value}


def get_launch(sprec: int, lprec: int, recon: int) -> dict:
    """The launch shape currently used for one storage format."""
    b = ctypes.c_int()
    x = ctypes.c_int()
    _check(lib().ndq_get_launch_for(sprec, lprec, recon, ctypes.byref(b), ctypes.byref(x)))
    return {"block": b.value, "xcd_remap": x.value}


def set_mrhs_launch(geom: "Geometry", sprec: int, lprec: int, recon: int, nrhs: int, ny: int, rg: int = 0,
                    group_major: int = 0, chunk: int = -1, xcd_remap: bool = True, link_nt: int = -1):
    """Work order of the multi-right-hand-side stencil for one lattice, format, nrhs and ny
    (group_major: 0 tile-major, 1 group-major, 2 one group per XCD)."""
    _check(lib().ndq_set_mrhs_launch(geom.handle, sprec, lprec, recon, nrhs, ny, rg, int(group_major), chunk,
                                     int(bool(xcd_remap)), int(link_nt)))


def get_mrhs_launch(geom: "Geometry", sprec: int, lprec: int, recon: int, nrhs: int, ny: int) -> dict:
    v = [ctypes.c_int() for _ in range(5)]
    _check(lib().ndq_get_mrhs_launch(geom.handle, sprec, lprec, recon, nrhs, ny, *[ctypes.byref(x) for x in v]))
    return {"rg": v[0].value, "group_major": v[1].value, "chunk": v[2].value, "xcd_remap": v[3].value,
            "link_nt": v[4].value}


def set_launch_for(sprec: int, lprec: int, recon: int, block: int, xcd_remap: bool = True):
    _check(lib().ndq_set_launch_for(sprec, lprec, recon, block, int(bool(xcd_remap))))


class Geometry:
    """Host handle of a periodic N0 x N1 x N2 x N3 lattice (ndq_geom)."""

    def __init__(self, dims):
        self.dims = tuple(int(d) for d in dims)
        arr = (ctypes.c_int32 * 4)(*self.dims)
        h = ctypes.c_void_p()
        _check(lib().ndq_geom_create(arr, ctypes.byref(h)))
        self.handle = h
        self.volume = int(lib().ndq_geom_volume(h))

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.ndq_geom_destroy(self.handle)
            self.handle = None

    def tables(self, stream=None):
        """(nb [V,8], lex_of_eo [2,V/2], nb_eo [2,V/2,8]) int32 device tensors."""
        v = self.volume
        dev = torch.device("cuda")
        nb = torch.empty((v, 8), dtype=torch.int32, device=dev)
        leo = torch.empty((2, v // 2), dtype=torch.int32, device=dev)
        nbe = torch.empty((2, v // 2, 8), dtype=torch.int32, device=dev)
        _check(lib().ndq_geom_tables(self.handle, _ptr(nb), _ptr(leo), _ptr(nbe), _stream(stream)))
        return nb, leo, nbe

    def gauge_bytes(self, prec: int, recon: int) -> int:
        return int(lib().ndq_gauge_bytes(self.handle, prec, recon))

    def spinor_bytes(self, prec: int, parity: int, nrhs: int = 1) -> int:
        return int(lib().ndq_spinor_bytes(self.handle, prec, parity, nrhs))


class GaugeField:
    """A packed gauge field in device memory owned by a torch uint8 buffer."""

    def __init__(self, geom: Geometry, prec: int, recon: int, buffer: torch.Tensor | None = None):
        nbytes = geom.gauge_bytes(prec, recon)
        if nbytes == 0:
            raise NdqError(-3, f"unsupported gauge format prec={prec} recon={recon}")
        self.geom, self.prec, self.recon = geom, prec, recon
        self.buf = buffer if buffer is not None else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.desc = _Gauge(self.buf.data_ptr(), prec, recon)

    @classmethod
    def pack(cls, geom: Geometry, canon: torch.Tensor, prec: int, recon: int, stream=None):
        canon = _canon(canon, (geom.volume, 4, 3, 3))
        u = cls(geom, prec, recon)
        _check(lib().ndq_gauge_pack(geom.handle, _ptr(canon), ctypes.byref(u.desc), _stream(stream)))
        return u

    def unpack(self, stream=None) -> torch.Tensor:
        out = torch.empty((self.geom.volume, 4, 3, 3), dtype=torch.complex128, device="cuda")
        _check(lib().ndq_gauge_unpack(self.geom.handle, ctypes.byref(self.desc), _ptr(out), _stream(stream)))
        return out


class SpinorField:
    """A packed spinor field (nrhs right-hand sides on EVEN, ODD or FULL sites)."""

    def __init__(self, geom: Geometry, prec: int, parity: int, nrhs: int = 1, buffer: torch.Tensor | None = None):
        nbytes = geom.spinor_bytes(prec, parity, nrhs)
        if nbytes == 0:
            raise NdqError(-1, f"bad spinor format prec={prec} parity={parity} nrhs={nrhs}")
        self.geom, self.prec, self.parity, self.nrhs = geom, prec, parity, nrhs
        self.nsites = geom.volume if parity == FULL else geom.volume // 2
        self.buf = buffer if buffer is not None else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.desc = _Spinor(self.buf.data_ptr(), prec, parity, nrhs)

    @classmethod
    def pack(cls, geom: Geometry, canon: torch.Tensor, prec: int, parity: int, stream=None):
        nsites = geom.volume if parity == FULL else geom.volume // 2
        nrhs = 1 if canon.dim() == 3 else canon.shape[0]
        canon = _canon(canon, (nrhs, nsites, 4, 3))
        s = cls(geom, prec, parity, nrhs)
        _check(lib().ndq_spinor_pack(geom.handle, _ptr(canon), ctypes.byref(s.desc), _stream(stream)))
        return s

    def unpack(self, stream=None) -> torch.Tensor:
        out = torch.empty((self.nrhs, self.nsites, 4, 3), dtype=torch.complex128, device="cuda")
        _check(lib().ndq_spinor_unpack(self.geom.handle, ctypes.byref(self.desc), _ptr(out), _stream(stream)))
        return out

    def like(self, parity: int | None = None, prec: int | None = None) -> "SpinorField":
        return SpinorField(self.geom, self.prec if prec is None else prec,
                           self.parity if parity is None else parity, self.nrhs)


def _canon(t: torch.Tensor, shape) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    if t.dtype != torch.complex128:
        t = t.to(torch.complex128)
    if t.device.type != "cuda":
        t = t.to("cuda")
    t = t.reshape(shape)
    return t.contiguous()


def apply_Q(geom: Geometry, U: GaugeField, m: float, inp: SpinorField, out: SpinorField, stream=None):
    _check(lib().ndq_apply_Q(geom.handle, ctypes.byref(U.desc), float(m), ctypes.byref(inp.desc),
                             ctypes.byref(out.desc), _stream(stream)))


def spinor_gram(geom: Geometry, A: SpinorField, B: SpinorField, stream=None) -> torch.Tensor:
    """G[i][j] = <A_i, B_j> for blocks of F64 FULL fields (matrix cores); complex128 [na, nb] on the GPU."""
    n = int(lib().ndq_gram_workspace_bytes(geom.handle, A.nrhs, B.nrhs))
    if n == 0:
        raise NdqError(-1, "bad block sizes for ndq_spinor_gram")
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    G = torch.empty((A.nrhs, B.nrhs), dtype=torch.complex128, device="cuda")
    _check(lib().ndq_spinor_gram(geom.handle, ctypes.byref(A.desc), ctypes.byref(B.desc), _ptr(G), _ptr(ws), n,
                                 _stream(stream)))
    return G


def _q_jobs(jobs):
    arr = (_QJob * len(jobs))()
    for k, (geom, U, m, inp, out) in enumerate(jobs):
        arr[k] = _QJob(geom.handle, ctypes.pointer(U.desc), float(m), ctypes.pointer(inp.desc),
                       ctypes.pointer(out.desc))
    return arr


def apply_Q_multi(jobs, stream=None):
    """Q on several lattices in one persistent launch: ``jobs`` is a list of
    (geom, U, m, inp, out) tuples (NDQ_FULL fields, shared formats)."""
    _check(lib().ndq_apply_Q_multi(_q_jobs(jobs), len(jobs), _stream(stream)))


def set_multi_grid(factor: int):
    """Grid of the persistent multi-lattice launch, in multiples of the resident workgroups."""
    _check(lib().ndq_set_multi_grid(int(factor)))


def get_multi_grid() -> int:
    return int(lib().ndq_get_multi_grid())


def autotune_multi(jobs, reps: int = 20, stream=None) -> dict:
    """Time the multi-lattice launch of ``jobs`` at each grid factor and keep the fastest
    (the jobs' outputs end as one apply_Q_multi leaves them)."""
    r = _MultiTuneResult()
    _check(lib().ndq_autotune_multi(_q_jobs(jobs), len(jobs), int(reps), ctypes.byref(r), _stream(stream)))
    return r.as_dict()


def apply_dslash(geom: Geometry, U: GaugeField, inp: SpinorField, out: SpinorField, stream=None):
    _check(lib().ndq_apply_dslash(geom.handle, ctypes.byref(U.desc), ctypes.byref(inp.desc),
                                  ctypes.byref(out.desc), _stream(stream)))


def apply_Qhat_ee(geom: Geometry, U: GaugeField, m: float, inp: SpinorField, out: SpinorField,
                  tmp: SpinorField, stream=None):
    _check(lib().ndq_apply_Qhat_ee(geom.handle, ctypes.byref(U.desc), float(m), ctypes.byref(inp.desc),
                                   ctypes.byref(out.desc), ctypes.byref(tmp.desc), _stream(stream)))


class Approx:
    """Host handle of a sign approximant (ndq_approx)."""

    def __init__(self, kind: int, lo: float, degree: int, _handle=None):
        if _handle is None:
            h = ctypes.c_void_p()
            _check(lib().ndq_approx_create(kind, float(lo), int(degree), ctypes.byref(h)))
            _handle = h
        self.handle = _handle
        k, n, lo_, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(lib().ndq_approx_info(self.handle, ctypes.byref(k), ctypes.byref(n), ctypes.byref(lo_), ctypes.byref(d)))
        self.kind, self.n, self.lo, self.delta = k.value, n.value, lo_.value, d.value

    @classmethod
    def from_coeffs(cls, kind: int, a, b=None, lo: float = 0.0, delta: float = 0.0):
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float64)
        n = len(a) if kind == ZOLOTAREV else len(a) - 1
        bp = None
        if b is not None:
            b = np.ascontiguousarray(b, dtype=np.float64)
            bp = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        _check(lib().ndq_approx_from_coeffs(kind, n, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), bp,
                                            float(lo), float(delta), ctypes.byref(h)))
        return cls(kind, lo, n, _handle=h)

    def coeffs(self):
        import numpy as np
        na = self.n if self.kind == ZOLOTAREV else self.n + 1
        a = np.zeros(na)
        b = np.zeros(self.n) if self.kind == ZOLOTAREV else None
        _check(lib().ndq_approx_coeffs(self.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       None if b is None else b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return a, b

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.ndq_approx_destroy(self.handle)
            self.handle = None


class Overlap:
    """Parameters of sign(Q) / D_N (ndq_overlap_params) plus the device workspace.

    ``modes``: a SpinorField (F64, FULL, nrhs = nev) of orthonormal Rayleigh-Ritz
    vectors; ``nu``: their eigenvalues."""

    def __init__(self, geom: Geometry, m: float, approx: Approx, lam_max: float, modes: "SpinorField | None" = None,
                 nu=None, mq: float = 0.0, form: int = LITERAL, tol: float = 1e-12, max_iter: int = 100000,
                 check_every: int = 8, graph: bool = False):
        import numpy as np
        self.geom, self.approx, self.modes = geom, approx, modes
        nev = 0 if modes is None else modes.nrhs
        if modes is not None and (modes.prec != F64 or modes.parity != FULL):
            raise NdqError(-1, "low modes must be F64 FULL spinor fields")
        self.nu = np.ascontiguousarray(np.zeros(1) if nu is None else nu, dtype=np.float64)
        self.p = _Params(float(m), float(mq), float(lam_max), approx.handle.value,
                         None if modes is None else modes.buf.data_ptr(),
                         self.nu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nev, form, float(tol),
                         int(max_iter), int(check_every), int(bool(graph)))
        self._ws = {}

    def workspace(self, prec: int, op: int, nrhs: int = 1):
        key = (prec, op, nrhs)
        if key not in self._ws:
            n = int(lib().ndq_workspace_bytes_nrhs(self.geom.handle, ctypes.byref(self.p), prec, op, nrhs))
            if n == 0:
                raise NdqError(-1, "invalid parameters for ndq_workspace_bytes")
            self._ws[key] = torch.empty(n, dtype=torch.uint8, device="cuda")
        return self._ws[key]


def apply_sign(geom: Geometry, U: GaugeField, ov: Overlap, inp: SpinorField, out: SpinorField, stream=None) -> dict:
    ws = ov.workspace(inp.prec, OP_SIGN, inp.nrhs)
    st = _Stats()
    _check(lib().ndq_apply_sign(geom.handle, ctypes.byref(U.desc), ctypes.byref(ov.p), ctypes.byref(inp.desc),
                                ctypes.byref(out.desc), _ptr(ws), ws.numel(), ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def apply_DN(geom: Geometry, U: GaugeField, ov: Overlap, inp: SpinorField, out: SpinorField, stream=None) -> dict:
    ws = ov.workspace(inp.prec, OP_DN, inp.nrhs)
    st = _Stats()
    _check(lib().ndq_apply_DN(geom.handle, ctypes.byref(U.desc), ctypes.byref(ov.p), ctypes.byref(inp.desc),
                              ctypes.byref(out.desc), _ptr(ws), ws.numel(), ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def apply_DN_noalloc(geom: Geometry, U: GaugeField, ov: Overlap, inp: SpinorField, out: SpinorField,
                     stream=None) -> dict:
    """D_N^m inp with the library's static device scratch (no workspace argument)."""
    st = _Stats()
    _check(lib().ndq_apply_DN_noalloc(geom.handle, ctypes.byref(U.desc), ctypes.byref(ov.p), ctypes.byref(inp.desc),
                                      ctypes.byref(out.desc), ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def noalloc_scratch_bytes() -> int:
    return int(lib().ndq_noalloc_scratch_bytes())


def lowmodes_compute(geom: Geometry, U: GaugeField, m: float, lam_max: float, start: SpinorField, nev: int,
                     nextra: int = 8, basis: int = 0, cheb_degree: int = 0, cheb_lo: float = 0.0, tol: float = 1e-10,
                     max_restarts: int = 0, method: int = 0, nev_min: int = 0, U_lo: "GaugeField" = None,
                     lo_until: float = 0.0, stream=None):
    """Low modes of Q: returns (modes SpinorField (F64, FULL, nrhs=nev), nu, rho, info dict).
    U_lo: F32 links of the same field for the filter of the early restarts (subspace method)."""
    import numpy as np
    basis = basis or min(63, nev + nextra + max(12, nev))
    p = _LmParams(nev, nextra, basis, cheb_degree, cheb_lo, tol, max_restarts, method, nev_min,
                  ctypes.cast(ctypes.pointer(U_lo.desc), ctypes.c_void_p) if U_lo is not None else None,
                  float(lo_until))
    nbytes = int(lib().ndq_lowmodes_workspace_bytes(geom.handle, ctypes.byref(p)))
    if nbytes == 0:
        raise NdqError(-1, "bad low-mode parameters")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    modes = SpinorField(geom, F64, FULL, nev)
    nu = np.zeros(nev)
    rho = np.zeros(nev)
    info = _LmInfo()
    rc = lib().ndq_lowmodes_compute(geom.handle, ctypes.byref(U.desc), float(m), float(lam_max), ctypes.byref(p),
                                    ctypes.byref(start.desc), _ptr(modes.buf),
                                    nu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(info),
                                    _ptr(ws), nbytes, _stream(stream))
    _check(rc)
    return modes, nu, rho, info.as_dict()


def index_DN(geom: Geometry, U: GaugeField, ov: Overlap, start: SpinorField, block: int = 8, degree: int = 0,
             max_sweeps: int = 200, tol: float = 1e-7, zero_cut: float = 1e-7, stream=None) -> dict:
    """Index of the massless D_N by zero-mode counting (ndq_index_DN): returns
    {n_plus, n_minus, index, lowest Ritz values and residues per sector, ...}.
    On an error the raised NdqError carries the same dict as ``.info``."""
    p = _IndexParams(int(block), int(degree), int(max_sweeps), 0, float(tol), float(zero_cut))
    nbytes = int(lib().ndq_index_workspace_bytes(geom.handle, ctypes.byref(ov.p), ctypes.byref(p)))
    if nbytes == 0:
        raise NdqError(-1, "bad index parameters")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    info = _IndexInfo()
    rc = lib().ndq_index_DN(geom.handle, ctypes.byref(U.desc), ctypes.byref(ov.p), ctypes.byref(p),
                            ctypes.byref(start.desc), ctypes.byref(info), _ptr(ws), nbytes, _stream(stream))
    try:
        _check(rc)
    except NdqError as e:
        e.info = info.as_dict()
        raise
    return info.as_dict()


def host_eigh(a):
    """The library's host Hermitian eigensolver (for tests): returns (w, z)."""
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.complex128).copy()
    n = a.shape[0]
    w = np.zeros(n)
    z = np.zeros((n, n), dtype=np.complex128)
    _check(lib().ndq_host_eigh(n, a.ctypes.data, w.ctypes.data, z.ctypes.data))
    return w, z


def solve_DN(geom: Geometry, U64: GaugeField, ov64: Overlap, b: SpinorField, x: SpinorField, tol: float = 1e-10,
             U_lo: GaugeField | None = None, ov_lo: Overlap | None = None, inner_prec: int = F64,
             inner_tol: float = 0.0, max_outer: int = 20, max_inner: int = 0, sectors: bool = False,
             stream=None) -> dict:
    """x = (D_N^m)^{-1} b for every right-hand side of b (up to 32, all sharing
    each application of D); x holds the initial guess (e.g. zeros) on entry.
    ``sectors``: CG on the chirality sectors of D^H D instead of CGNE."""
    sp = _SolveParams(float(tol), int(max_outer), int(max_inner), float(inner_tol), int(inner_prec),
                      int(bool(sectors)))
    plo = ctypes.byref(ov_lo.p) if ov_lo is not None else None
    n = int(lib().ndq_solve_workspace_bytes_nrhs(geom.handle, ctypes.byref(ov64.p), plo, ctypes.byref(sp), b.nrhs))
    if n == 0:
        raise NdqError(-1, "bad solve parameters")
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    st = _Stats()
    _check(lib().ndq_solve_DN(geom.handle, ctypes.byref(U64.desc), None if U_lo is None else ctypes.byref(U_lo.desc),
                              ctypes.byref(ov64.p), plo, ctypes.byref(sp), ctypes.byref(b.desc), ctypes.byref(x.desc),
                              _ptr(ws), n, ctypes.byref(st), _stream(stream)))
    return st.as_dict()


def gauge_force(geom: Geometry, U: GaugeField, psi: SpinorField, g: SpinorField, want_force: bool = True,
                want_grad: bool = False, stream=None):
    """(force [V,4,8] float64 or None, tangent gradient [V,4,3,3] complex128 or None) for
    y = Q[U] psi and cotangent g."""
    v = geom.volume
    f = torch.empty((v, 4, 8), dtype=torch.float64, device="cuda") if want_force else None
    gr = torch.empty((v, 4, 3, 3), dtype=torch.complex128, device="cuda") if want_grad else None
    _check(lib().ndq_gauge_force(geom.handle, ctypes.byref(U.desc), ctypes.byref(psi.desc), ctypes.byref(g.desc),
                                 None if f is None else _ptr(f), None if gr is None else _ptr(gr), _stream(stream)))
    return f, gr


class QFunction(torch.autograd.Function):
    """y = Q[U] psi on canonical complex128 GPU tensors (psi [V,4,3], links [V,4,3,3]),
    differentiable in psi (grad = Q g) and in the links (the su(3) tangent-space
    gradient from ndq_gauge_force).  Usage: QFunction.apply(psi, links, geom, m)."""

    @staticmethod
    def forward(ctx, psi, links, geom, m):
        U = GaugeField.pack(geom, links.detach(), F64, 18)
        x = SpinorField.pack(geom, psi.detach(), F64, FULL)
        y = x.like()
        apply_Q(geom, U, m, x, y)
        ctx.geom, ctx.m, ctx.U, ctx.x = geom, m, U, x
        return y.unpack()[0]

    @staticmethod
    def backward(ctx, gy):
        geom = ctx.geom
        gsp = SpinorField.pack(geom, gy.contiguous(), F64, FULL)
        gpsi = glinks = None
        if ctx.needs_input_grad[0]:
            out = gsp.like()
            apply_Q(geom, ctx.U, ctx.m, gsp, out)
            gpsi = out.unpack()[0]
        if ctx.needs_input_grad[1]:
            _, glinks = gauge_force(geom, ctx.U, ctx.x, gsp, want_force=False, want_grad=True)
        return gpsi, glinks, None, None
