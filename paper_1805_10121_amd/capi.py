"""ctypes binding of include/chase.h -- argument marshalling only.

Every call below forwards to the function of the same name in ``libchase.so``; no numerical
step runs in Python.  Device buffers are passed as raw pointers (``tensor.data_ptr()``);
torch supplies device memory and the stream, nothing else.  If the library has not been built
the import raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libchase.so")

CHASE_OK = 0
CHASE_NOT_CONVERGED = 1
CHASE_EINVAL = -1
CHASE_ENOMEM = -2
CHASE_EDEVICE = -3
CHASE_ENUMERIC = -4
CHASE_EBUSY = -5

CHASE_FP64 = 0
CHASE_FP32 = 1
CHASE_MIXED = 2
CHASE_FP32_3M = 3
CHASE_REAL_FP64 = 4
CHASE_REAL_FP32 = 5
CHASE_FP64_3M = 6
CHASE_FP64_LOWER = 7

_i64, _i32, _f64, _u64, _vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p


class chase_config(ctypes.Structure):
    _fields_ = [
        ("n", _i64), ("nev", _i64), ("nex", _i64),
        ("approx", _i32), ("tol", _f64), ("max_iter", _i32), ("optim", _i32),
        ("deg_extra", _i32), ("deg_max", _i32), ("deg", _i32),
        ("lanczos_iter", _i32), ("num_lanczos", _i32),
        ("precision", _i32), ("switch_resid", _f64), ("deg_max_fp32", _i32),
        ("resid_relative", _i32), ("intersperse", _i32), ("dos_sigma", _f64),
        ("seed", _u64), ("lanczos_start", _vp), ("have_mu", _i32),
        ("mu_1", _f64), ("mu_nevnex", _f64), ("verbose", _i32), ("real_symmetric", _i32),
        ("filter_3m", _i32),
    ]


class chase_stats(ctypes.Structure):
    _fields_ = [
        ("status", _i32), ("iterations", _i32), ("nconv", _i32), ("fp32_iterations", _i32),
        ("qr_fallbacks", _i32), ("reserved", _i32),
        ("matvecs", _i64), ("filter_matvecs", _i64), ("filter_flops", _f64),
        ("filter_ms", _f64), ("lanczos_ms", _f64), ("ortho_ms", _f64), ("rr_ms", _f64),
        ("resid_ms", _f64), ("total_ms", _f64),
        ("b_sup", _f64), ("mu_1", _f64), ("mu_nevnex", _f64), ("norm_est", _f64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_PROTOTYPES = {
    "chase_config_init": (None, [ctypes.POINTER(chase_config), _i64, _i64, _i64]),
    "chase_config_init_fp32": (None, [ctypes.POINTER(chase_config), _i64, _i64, _i64]),
    "chase_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _vp]),
    "chase_destroy": (None, [_vp]),
    "chase_last_error": (ctypes.c_char_p, [_vp]),
    "chase_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(chase_config)]),
    "chase_filter": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _i64, _i64, _vp, _vp, _i64, _i64,
                                    ctypes.POINTER(_i32), _f64, _f64, _f64]),
    "chase_filter_noalloc": (ctypes.c_int, [ctypes.c_int, _vp, ctypes.c_int, _vp, _i64, _i64, _vp,
                                            _vp, _i64, _i64, ctypes.POINTER(_i32), _f64, _f64,
                                            _f64, ctypes.c_char_p, ctypes.c_size_t]),
    "chase_hemm_step": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _i64, _i64, _vp, _i64, _vp, _i64,
                                       _i64, _f64, _f64, _f64]),
    "chase_convert_c128_to_c64": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i64, _i64]),
    "chase_convert_c64_to_c128": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i64, _i64]),
    "chase_convert_c128_to_planar32": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i64]),
    "chase_convert_c128_to_planar64": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i64]),
    "chase_solve": (ctypes.c_int, [_vp, ctypes.POINTER(chase_config), _vp, _i64, _vp, _i64,
                                   ctypes.POINTER(_f64), ctypes.POINTER(_f64),
                                   ctypes.POINTER(chase_stats)]),
    "chase_seq_create": (ctypes.c_int, [_vp, ctypes.POINTER(chase_config), ctypes.POINTER(_vp)]),
    "chase_seq_solve": (ctypes.c_int, [_vp, _vp, _i64, ctypes.POINTER(_f64),
                                       ctypes.POINTER(_f64), ctypes.POINTER(chase_stats)]),
    "chase_seq_vectors": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_i64)]),
    "chase_seq_destroy": (None, [_vp]),
    "chase_server_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_size_t,
                                           ctypes.c_int]),
    "chase_server_submit": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(chase_config), _vp,
                                           _i64, ctypes.POINTER(ctypes.c_uint64)]),
    "chase_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_f64),
                                         ctypes.POINTER(_f64), ctypes.POINTER(chase_stats),
                                         ctypes.POINTER(_f64)]),
    "chase_server_vectors": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(_vp),
                                            ctypes.POINTER(_i64)]),
    "chase_server_end_sequence": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "chase_server_info": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "chase_server_last_error": (ctypes.c_char_p, [_vp]),
    "chase_server_destroy": (None, [_vp]),
}

_lib = None


def lib():
    """The loaded ``libchase.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1805_10121_amd.build` "
                "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_PROTOTYPES)


class ChaseError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"chase error {code}: {msg}")
        self.code = code


def _check(ctx, rc):
    if rc < 0:
        raise ChaseError(rc, lib().chase_last_error(ctx).decode())
    return rc


def config(n, nev, nex, **kw) -> chase_config:
    cfg = chase_config()
    lib().chase_config_init(ctypes.byref(cfg), n, nev, nex)
    return _apply(cfg, kw)


def config_fp32(n, nev, nex, **kw) -> chase_config:
    """Table 1's single-precision defaults with precision = CHASE_FP32."""
    cfg = chase_config()
    lib().chase_config_init_fp32(ctypes.byref(cfg), n, nev, nex)
    return _apply(cfg, kw)


def _apply(cfg, kw):
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Context:
    """A chase_ctx bound to a torch CUDA stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        rc = lib().chase_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream))
        if rc != CHASE_OK:
            raise ChaseError(rc, "chase_create failed")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().chase_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----- calls (same names as the C ABI, minus the prefix) -----
    def chase_filter(self, precision, H, ldh, n, V, W, ld, ncols, degrees, b_sup, mu_1, mu_nevnex):
        deg = (_i32 * max(int(ncols), 1))(*[int(x) for x in degrees])
        return _check(self.handle, lib().chase_filter(
            self.handle, precision, _ptr(H), ldh, n, _ptr(V), _ptr(W), ld, ncols, deg,
            float(b_sup), float(mu_1), float(mu_nevnex)))

    def chase_hemm_step(self, precision, H, ldh, n, X, ldx, OUT, ldo, ncols, alpha, beta, gamma):
        return _check(self.handle, lib().chase_hemm_step(
            self.handle, precision, _ptr(H), ldh, n, _ptr(X), ldx, _ptr(OUT), ldo, ncols,
            float(alpha), float(beta), float(gamma)))

    def chase_convert_c128_to_c64(self, src, ld_src, dst, ld_dst, rows, cols):
        return _check(self.handle, lib().chase_convert_c128_to_c64(
            self.handle, _ptr(src), ld_src, _ptr(dst), ld_dst, rows, cols))

    def chase_convert_c128_to_planar64(self, src, ld_src, dst, ld_dst, n):
        return _check(self.handle, lib().chase_convert_c128_to_planar64(
            self.handle, _ptr(src), ld_src, _ptr(dst), ld_dst, n))

    def chase_convert_c128_to_planar32(self, src, ld_src, dst, ld_dst, n):
        return _check(self.handle, lib().chase_convert_c128_to_planar32(
            self.handle, _ptr(src), ld_src, _ptr(dst), ld_dst, n))

    def chase_convert_c64_to_c128(self, src, ld_src, dst, ld_dst, rows, cols):
        return _check(self.handle, lib().chase_convert_c64_to_c128(
            self.handle, _ptr(src), ld_src, _ptr(dst), ld_dst, rows, cols))

    def chase_solve(self, cfg, H, ldh, V, ldv, ritzv, resid):
        """ritzv, resid: numpy float64 arrays of length nev+nex (ritzv read when approx=1)."""
        st = chase_stats()
        rc = lib().chase_solve(
            self.handle, ctypes.byref(cfg), _ptr(H), ldh, _ptr(V), ldv,
            ritzv.ctypes.data_as(ctypes.POINTER(_f64)), resid.ctypes.data_as(ctypes.POINTER(_f64)),
            ctypes.byref(st))
        _check(self.handle, rc)
        return rc, st

    def last_error(self):
        return lib().chase_last_error(self.handle).decode()


class Sequence:
    """chase_seq: a sequence whose state stays on the device between problems."""

    def __init__(self, ctx: Context, cfg: chase_config):
        self.ctx = ctx
        self.cfg = cfg
        h = ctypes.c_void_p()
        _check(ctx.handle, lib().chase_seq_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h

    def chase_seq_solve(self, H, ldh, ritzv, resid):
        st = chase_stats()
        rc = lib().chase_seq_solve(self.handle, _ptr(H), ldh,
                                   ritzv.ctypes.data_as(ctypes.POINTER(_f64)),
                                   resid.ctypes.data_as(ctypes.POINTER(_f64)), ctypes.byref(st))
        _check(self.ctx.handle, rc)
        return rc, st

    def chase_seq_vectors(self):
        p, ld = ctypes.c_void_p(), _i64()
        _check(self.ctx.handle, lib().chase_seq_vectors(self.handle, ctypes.byref(p), ctypes.byref(ld)))
        return p.value, ld.value

    def close(self):
        if getattr(self, "handle", None):
            lib().chase_seq_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """chase_server: continuous batching of solves from many sequences on one device."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 288 << 30, workers: int = 8):
        h = ctypes.c_void_p()
        rc = lib().chase_server_create(ctypes.byref(h), device, mem_budget_bytes, workers)
        if rc != CHASE_OK:
            raise ChaseError(rc, "chase_server_create failed")
        self.handle = h
        self._cfgs = {}

    def _err(self, rc):
        if rc < 0:
            raise ChaseError(rc, lib().chase_server_last_error(self.handle).decode())
        return rc

    def chase_server_submit(self, seq_id, cfg, H, ldh):
        t = ctypes.c_uint64()
        self._err(lib().chase_server_submit(self.handle, seq_id, ctypes.byref(cfg), _ptr(H), ldh,
                                            ctypes.byref(t)))
        self._cfgs[t.value] = cfg.nev + cfg.nex
        return t.value

    def chase_server_poll(self, ticket, wait=False):
        """Returns None while running, else (status, ritzv, resid, stats, latency_s)."""
        import numpy as np

        nb = self._cfgs[ticket]
        done = ctypes.c_int()
        ritzv, resid = np.zeros(nb), np.zeros(nb)
        st, lat = chase_stats(), _f64()
        rc = lib().chase_server_poll(self.handle, ticket, 1 if wait else 0, ctypes.byref(done),
                                     ritzv.ctypes.data_as(ctypes.POINTER(_f64)),
                                     resid.ctypes.data_as(ctypes.POINTER(_f64)), ctypes.byref(st),
                                     ctypes.byref(lat))
        if not done.value:
            self._err(rc)
            return None
        self._cfgs.pop(ticket, None)
        self._err(rc)
        return rc, ritzv, resid, st, lat.value

    def chase_server_vectors(self, seq_id):
        p, ld = ctypes.c_void_p(), _i64()
        self._err(lib().chase_server_vectors(self.handle, seq_id, ctypes.byref(p), ctypes.byref(ld)))
        return p.value, ld.value

    def chase_server_end_sequence(self, seq_id):
        return self._err(lib().chase_server_end_sequence(self.handle, seq_id))

    def chase_server_info(self):
        a, b, c = _i64(), _i64(), ctypes.c_size_t()
        self._err(lib().chase_server_info(self.handle, ctypes.byref(a), ctypes.byref(b),
                                          ctypes.byref(c)))
        return {"grouped_launches": a.value, "grouped_products": b.value, "bytes_in_use": c.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().chase_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chase_filter_noalloc(device, stream, precision, H, ldh, n, V, W, ld, ncols, degrees, b_sup,
                         mu_1, mu_nevnex):
    """chase_filter without a context and without device allocation; ``stream`` is a torch
    CUDA stream on ``device`` (None: the null stream)."""
    deg = (_i32 * max(int(ncols), 1))(*[int(x) for x in degrees])
    err = ctypes.create_string_buffer(512)
    rc = lib().chase_filter_noalloc(
        int(device), ctypes.c_void_p(stream.cuda_stream if stream is not None else 0), precision,
        _ptr(H), ldh, n, _ptr(V), _ptr(W), ld, ncols, deg, float(b_sup), float(mu_1),
        float(mu_nevnex), err, len(err))
    if rc < 0:
        raise ChaseError(rc, err.value.decode())
    return rc


# ----------------------------------------------------------------------------- layout helpers

def to_device(A, device="cuda"):
    """Host column-major matrix (numpy, any order) -> device tensor whose storage is A in
    column-major order (the tensor has shape (cols, rows))."""
    import numpy as np
    import torch

    A = np.asarray(A)
    return torch.from_numpy(np.ascontiguousarray(A.T)).to(device)


def device_block_to_host(ptr, ld, rows, cols, dtype=None):
    """Copy a borrowed device block (column-major, leading dimension ld; complex128 unless
    dtype says otherwise) to a numpy array (rows, cols) -- a hipMemcpy2D through the HIP
    runtime, no arithmetic."""
    import numpy as np

    dtype = np.dtype(dtype or np.complex128)
    es = dtype.itemsize
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy2D.restype = ctypes.c_int
    hip.hipMemcpy2D.argtypes = [_vp, ctypes.c_size_t, _vp, ctypes.c_size_t, ctypes.c_size_t,
                                ctypes.c_size_t, ctypes.c_int]
    out = np.empty((cols, rows), dtype=dtype)
    rc = hip.hipMemcpy2D(out.ctypes.data, rows * es, ptr, ld * es, rows * es, cols, 2)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy2D failed ({rc})")
    return out.T


def from_device(t):
    """Inverse of ``to_device``: device tensor of shape (cols, rows) -> numpy (rows, cols)."""
    return t.detach().cpu().numpy().T
