"""MI355X (gfx950) multiplication of sparse Laurent polynomials and Poisson series.

Thin Python binding over the C ABI in ``include/kp.h`` (``libkp.so``, built
in-tree by ``build.py``).  This module only marshals arguments: torch tensors
provide device memory and the current HIP stream, and every step of a product
-- min/max of the exponents, Kronecker encoding, sorting, the multiply with
dense or hash accumulation, compaction and decoding -- runs in the library's
HIP kernels.  There is no CPU fallback: without the built library every call
raises.

Method: Biscani, "Multiplication of sparse Laurent polynomials and Poisson
series on modern hardware architectures" (ISSAC 2010) -- Kronecker
substitution (Section 2), schoolbook products accumulated by code in a dense
array or a hash table (Section 3), Poisson split by eq. werner with the
factor 1/2.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkp.so")
MAX_VARS = 16

KP_OK, KP_E_ARG, KP_E_RANGE, KP_E_CODE_OVERFLOW, KP_E_NONCANONICAL = 0, 1, 2, 3, 4
KP_E_CAPACITY, KP_E_WORKSPACE, KP_E_DEVICE, KP_E_DTYPE, KP_E_MODE = 5, 6, 7, 8, 9
KP_I64, KP_F64, KP_I128 = 0, 1, 2
KP_AUTO, KP_DENSE, KP_HASH = 0, 1, 2
KP_FLAG_ASYNC = 1
KP_BATCH_GRAPH = 2
KP_PACK_GRAPH = 4
KP_SCRATCH_BYTES = 64 << 20   # the scratch array of kp_mul_laurent_noalloc (include/kp.h)
KP_KIND_LAURENT, KP_KIND_POISSON = 0, 1
MODES = {"auto": KP_AUTO, "dense": KP_DENSE, "hash": KP_HASH}
MODE_NAMES = {v: k for k, v in MODES.items()}

EXPORTED = ["kp_ctx_create", "kp_ctx_destroy", "kp_ctx_get_tune", "kp_ctx_set_tune",
            "kp_ctx_check", "kp_status_str", "kp_last_error", "kp_ctx_timing",
            "kp_ctx_timing_read", "kp_minmax", "kp_layout_product",
            "kp_encode", "kp_mul_bound", "kp_mul_laurent", "kp_mul_poisson", "kp_decode",
            "kp_encode_host", "kp_decode_host", "kp_batch_create", "kp_batch_destroy",
            "kp_batch_add", "kp_batch_clear", "kp_batch_launch", "kp_batch_status",
            "kp_ctx_hash_stats", "kp_ctx_hash_stats_read", "kp_probe_lds_atomic",
            "kp_plan_laurent", "kp_mul_laurent_exps", "kp_plan_poisson", "kp_mul_poisson_exps",
            "kp_mul_laurent_auto", "kp_ctx_set_truncation", "kp_ctx_clear_truncation",
            "kp_mul_laurent_noalloc", "kp_pack_create", "kp_pack_destroy", "kp_pack_plan",
            "kp_pack_run", "kp_pack_wait", "kp_pack_query", "kp_ctx_set_harmonic_truncation"]


class PackTask(C.Structure):
    _fields_ = [("nvars", C.c_int32), ("dtype", C.c_int32), ("a_exps", C.c_void_p),
                ("a_coef", C.c_void_p), ("na", C.c_int64), ("b_exps", C.c_void_p),
                ("b_coef", C.c_void_p), ("nb", C.c_int64)]


class KPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"kp status {status}: {msg}")
        self.status = status


class Layout(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("amin", C.c_int32 * MAX_VARS), ("amax", C.c_int32 * MAX_VARS),
                ("bmin", C.c_int32 * MAX_VARS), ("bmax", C.c_int32 * MAX_VARS),
                ("ha", C.c_int32 * MAX_VARS), ("hb", C.c_int32 * MAX_VARS),
                ("xmin", C.c_int64 * MAX_VARS), ("xw", C.c_int64 * MAX_VARS),
                ("xc", C.c_int64 * MAX_VARS), ("Wx", C.c_int64),
                ("yh", C.c_int64 * MAX_VARS), ("yc", C.c_int64 * MAX_VARS),
                ("Hy", C.c_int64), ("nkeys", C.c_int64)]


class Tune(C.Structure):
    _fields_ = [("window", C.c_int32), ("block", C.c_int32), ("tasks_per_cu", C.c_int32),
                ("hash_load", C.c_double), ("hash_capacity", C.c_int64),
                ("dense_max_keys", C.c_int64), ("dense_keys_per_pair", C.c_double),
                ("hash_rows", C.c_int32), ("hash_partitioned", C.c_int32),
                ("hash_bucket", C.c_int32), ("hash_order", C.c_int32),
                ("hash_bin_slots", C.c_int32), ("hash_grouping", C.c_int32),
                ("hash_max_bin_bits", C.c_int32), ("hash_bin_fill", C.c_int32)]


class MulDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("layout", Layout), ("dtype", C.c_int32),
                ("mode", C.c_int32), ("a_codes", C.c_void_p), ("a_y", C.c_void_p),
                ("a_sin", C.c_void_p), ("a_coef", C.c_void_p), ("na", C.c_int64),
                ("b_codes", C.c_void_p), ("b_y", C.c_void_p), ("b_sin", C.c_void_p),
                ("b_coef", C.c_void_p), ("nb", C.c_int64), ("out_codes", C.c_void_p),
                ("out_coef", C.c_void_p), ("out_cap", C.c_int64), ("out_n", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t)]


_lib = None


def lib():
    """The loaded libkp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_1004_4548_amd/build.py "
                           "(or __graft_entry__.build()) first")
    L = C.CDLL(LIB_PATH)
    p, i32, i64, u32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint, C.c_size_t
    sig = {
        "kp_ctx_create": (i32, [i32, C.POINTER(p)]),
        "kp_ctx_destroy": (i32, [p]),
        "kp_ctx_get_tune": (i32, [p, C.POINTER(Tune)]),
        "kp_ctx_set_tune": (i32, [p, C.POINTER(Tune)]),
        "kp_ctx_check": (i32, [p, p]),
        "kp_status_str": (C.c_char_p, [i32]),
        "kp_last_error": (C.c_char_p, [p]),
        "kp_ctx_timing": (i32, [p, i32]),
        "kp_ctx_timing_read": (i32, [p, C.POINTER(C.c_double), C.POINTER(i64)]),
        "kp_minmax": (i32, [p, i64, i32, p, p, u32, p]),
        "kp_layout_product": (i32, [i32, i32, p, p, p, p, p, p, C.POINTER(Layout)]),
        "kp_encode": (i32, [p, C.POINTER(Layout), i32, i64, p, p, p, p, p, u32, p]),
        "kp_mul_bound": (i32, [p, C.POINTER(Layout), i32, i32, i32, i64, i64, C.POINTER(i32),
                               C.POINTER(i64), C.POINTER(sz)]),
        "kp_mul_laurent": (i32, [p, C.POINTER(Layout), i32, i32, u32, p, p, i64, p, p, i64, p,
                                 p, i64, p, p, sz, p]),
        "kp_mul_laurent_noalloc": (i32, [p, C.POINTER(Layout), i32, i32, u32, p, p, i64, p, p,
                                         i64, p, p, i64, p, p]),
        "kp_mul_poisson": (i32, [p, C.POINTER(Layout), i32, u32, p, p, p, p, i64, p, p, p, p,
                                 i64, p, p, i64, p, p, sz, p]),
        "kp_decode": (i32, [p, C.POINTER(Layout), i32, i64, p, p, p, p, u32, p]),
        "kp_encode_host": (i32, [C.POINTER(Layout), i32, i64, p, p, p, p, p]),
        "kp_decode_host": (i32, [C.POINTER(Layout), i32, i64, p, p, p, p]),
        "kp_batch_create": (i32, [p, i64, C.POINTER(p)]),
        "kp_batch_destroy": (i32, [p]),
        "kp_batch_add": (i32, [p, C.POINTER(MulDesc), C.POINTER(i64)]),
        "kp_batch_clear": (i32, [p]),
        "kp_batch_launch": (i32, [p, u32, p]),
        "kp_batch_status": (i32, [p, i64, C.POINTER(i64)]),
        "kp_ctx_hash_stats": (i32, [p, i32]),
        "kp_ctx_hash_stats_read": (i32, [p, p, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]),
        "kp_probe_lds_atomic": (i32, [p, i32, C.POINTER(C.c_double), p]),
        "kp_plan_laurent": (i32, [p, i32, i32, i32, p, i64, p, i64, C.POINTER(Layout),
                                  C.POINTER(i32), C.POINTER(i64), C.POINTER(sz), p]),
        "kp_mul_laurent_exps": (i32, [p, C.POINTER(Layout), i32, i32, u32, p, p, i64, p, p, i64,
                                      p, p, i64, p, C.POINTER(i64), p, sz, p]),
        "kp_mul_laurent_auto": (i32, [p, i32, i32, i32, u32, p, p, i64, p, p, i64, p, p, i64, p,
                                      C.POINTER(i64), p, sz, C.POINTER(Layout), C.POINTER(i64),
                                      C.POINTER(sz), p]),
        "kp_pack_create": (i32, [p, i32, C.POINTER(p)]),
        "kp_pack_destroy": (i32, [p]),
        "kp_pack_plan": (i32, [p, C.POINTER(PackTask), i32, C.POINTER(i64), C.POINTER(sz), p]),
        "kp_pack_run": (i32, [p, C.POINTER(p), C.POINTER(p), p, sz, u32, p]),
        "kp_pack_wait": (i32, [p, C.POINTER(i64)]),
        "kp_pack_query": (i32, [p, C.POINTER(i32)]),
        "kp_ctx_set_truncation": (i32, [p, i32, C.POINTER(i32), i64]),
        "kp_ctx_set_harmonic_truncation": (i32, [p, i32, C.POINTER(i32), i64]),
        "kp_ctx_clear_truncation": (i32, [p]),
        "kp_plan_poisson": (i32, [p, i32, i32, i32, p, p, i64, p, p, i64, C.POINTER(Layout),
                                  C.POINTER(i32), C.POINTER(i64), C.POINTER(sz), p]),
        "kp_mul_poisson_exps": (i32, [p, C.POINTER(Layout), i32, u32, p, p, p, p, i64, p, p, p, p,
                                      i64, p, p, p, p, i64, p, C.POINTER(i64), p, sz, p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_str(s):
    return lib().kp_status_str(s).decode()


# ------------------------------------------------------------------ host-only
def layout_product(nx, ny, amin, amax, bmin, bmax, ha=None, hb=None) -> Layout:
    """kp_layout_product: the product's coding vectors from the factor boxes."""
    arr = C.c_int32 * MAX_VARS
    def a(v, n):
        v = [] if v is None else [int(x) for x in v]
        assert len(v) == n
        return arr(*v)
    out = Layout()
    st = lib().kp_layout_product(nx, ny, a(amin, nx), a(amax, nx), a(bmin, nx), a(bmax, nx),
                                 a(ha, ny), a(hb, ny), C.byref(out))
    if st != KP_OK:
        raise KPError(st, status_str(st))
    return out


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def encode_host(layout: Layout, which, x, y=None, t=None):
    """kp_encode_host on numpy arrays (same per-term map as the kernel)."""
    import numpy as np
    x = np.ascontiguousarray(x, dtype=np.int32).reshape(-1, max(layout.nx, 1))
    n = x.shape[0]
    kx = np.zeros(n, dtype=np.int64)
    ky = np.zeros(n, dtype=np.int64) if layout.ny else None
    if layout.ny:
        y = np.ascontiguousarray(y, dtype=np.int32).reshape(n, layout.ny)
        t = np.ascontiguousarray(t, dtype=np.uint8).reshape(n)
    st = lib().kp_encode_host(C.byref(layout), which, n, _np_ptr(x), _np_ptr(y), _np_ptr(t),
                              _np_ptr(kx), _np_ptr(ky))
    if st != KP_OK:
        raise KPError(st, status_str(st))
    return kx, ky


def decode_host(layout: Layout, codes, poisson=False):
    import numpy as np
    codes = np.ascontiguousarray(codes, dtype=np.int64).reshape(-1)
    n = codes.shape[0]
    x = np.zeros((n, layout.nx), dtype=np.int32)
    y = np.zeros((n, layout.ny), dtype=np.int32) if poisson else None
    t = np.zeros(n, dtype=np.uint8) if poisson else None
    st = lib().kp_decode_host(C.byref(layout), 1 if poisson else 0, n, _np_ptr(codes),
                              _np_ptr(x), _np_ptr(y), _np_ptr(t))
    if st != KP_OK:
        raise KPError(st, status_str(st))
    return (x, y, t) if poisson else x


# ------------------------------------------------------------------ device
class Context:
    """A kp_ctx on one device (tuning knobs, device status block)."""

    def __init__(self, device=0):
        self.device = device
        h = C.c_void_p()
        st = lib().kp_ctx_create(device, C.byref(h))
        if st != KP_OK:
            raise KPError(st, "kp_ctx_create failed")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.kp_ctx_destroy(h)
            self.h = None

    def check(self, st):
        if st != KP_OK:
            raise KPError(st, f"{status_str(st)}: {lib().kp_last_error(self.h).decode()}")

    @property
    def tune(self) -> Tune:
        t = Tune()
        self.check(lib().kp_ctx_get_tune(self.h, C.byref(t)))
        return t

    def set_tune(self, **kw):
        t = self.tune
        for k, v in kw.items():
            setattr(t, k, v)
        self.check(lib().kp_ctx_set_tune(self.h, C.byref(t)))

    def timing(self, enable=True):
        """Record HIP events around every accumulation kernel launch."""
        self.check(lib().kp_ctx_timing(self.h, 1 if enable else 0))

    def timing_read(self):
        """(summed accumulation-kernel milliseconds, launches) since the last read."""
        ms = C.c_double()
        n = C.c_int64()
        self.check(lib().kp_ctx_timing_read(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def set_truncation(self, weights, max_degree):
        """Keep only product terms with sum(w * e) <= max_degree (Laurent)."""
        w = [int(x) for x in weights]
        arr = (C.c_int32 * len(w))(*w)
        self.check(lib().kp_ctx_set_truncation(self.h, len(w), arr, int(max_degree)))

    def clear_truncation(self):
        self.check(lib().kp_ctx_clear_truncation(self.h))

    def truncation(self, weights, max_degree):
        """Context manager: a truncation for the products inside the block."""
        import contextlib

        @contextlib.contextmanager
        def scope():
            self.set_truncation(weights, max_degree)
            try:
                yield self
            finally:
                self.clear_truncation()
        return scope()

    def set_harmonic_truncation(self, weights, max_order):
        """Keep only Poisson product terms with sum(w * |j|) <= max_order."""
        w = [int(x) for x in weights]
        arr = (C.c_int32 * len(w))(*w)
        self.check(lib().kp_ctx_set_harmonic_truncation(self.h, len(w), arr, int(max_order)))

    def harmonic_truncation(self, weights, max_order):
        """Context manager: a harmonic-order truncation for the Poisson
        products inside the block."""
        import contextlib

        @contextlib.contextmanager
        def scope():
            self.set_harmonic_truncation(weights, max_order)
            try:
                yield self
            finally:
                self.clear_truncation()
        return scope()

    def hash_stats(self, enable=True):
        """Count insertions and extra probe steps of every hash-mode multiply."""
        self.check(lib().kp_ctx_hash_stats(self.h, 1 if enable else 0))

    def hash_stats_read(self, stream=None):
        """(insertions, slots visited beyond the home slots, insertions sent to
        the bucketed table's overflow table) since the last read."""
        n = C.c_int64()
        x = C.c_int64()
        o = C.c_int64()
        self.check(lib().kp_ctx_hash_stats_read(self.h, _stream(stream), C.byref(n), C.byref(x),
                                                C.byref(o)))
        return n.value, x.value, o.value

    def probe_lds_atomic(self, pattern=0, stream=None):
        """Device-wide LDS atomic adds per second: 0/1 = 64-bit counters,
        consecutive (conflict-free) or pseudo-random; 2/3 = 32-bit counters."""
        r = C.c_double()
        self.check(lib().kp_probe_lds_atomic(self.h, pattern, C.byref(r), _stream(stream)))
        return r.value

    def sync_check(self, stream=None):
        self.check(lib().kp_ctx_check(self.h, _stream(stream)))


_contexts = {}


def context(device=None) -> Context:
    import torch
    d = torch.cuda.current_device() if device is None else device
    if d not in _contexts:
        _contexts[d] = Context(d)
    return _contexts[d]


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _raw_stream(device):
    """Handle of the current stream of `device` (a torch.device), as an int."""
    import torch
    return torch._C._cuda_getCurrentRawStream(device.index)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_check(t, dtype, name):
    import torch
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def minmax(vals, ctx=None, flags=0, out=None):
    """kp_minmax: per-column (min, max) of an int32 [n, nv] device tensor
    (into `out`, 2 * nv int32, when given)."""
    import torch
    ctx = ctx or context()
    _dev_check(vals, torch.int32, "vals")
    n, nv = vals.shape
    if out is None:
        out = torch.empty(2 * nv, dtype=torch.int32, device=vals.device)
    ctx.check(lib().kp_minmax(ctx.h, n, nv, _ptr(vals), _ptr(out), flags, _stream()))
    return out


def encode(layout, which, x, y=None, t=None, ctx=None, flags=0):
    """kp_encode: Kronecker codes of one factor (device tensors)."""
    import torch
    ctx = ctx or context()
    _dev_check(x, torch.int32, "x")
    n = x.shape[0]
    kx = torch.empty(n, dtype=torch.int64, device=x.device)
    ky = None
    if layout.ny:
        _dev_check(y, torch.int32, "y")
        _dev_check(t, torch.uint8, "is_sin")
        ky = torch.empty(n, dtype=torch.int64, device=x.device)
    ctx.check(lib().kp_encode(ctx.h, C.byref(layout), which, n, _ptr(x), _ptr(y), _ptr(t),
                              _ptr(kx), _ptr(ky), flags, _stream()))
    return kx, ky


def decode(layout, codes, poisson=False, ctx=None, flags=0, out=None):
    """kp_decode: product codes (or Poisson keys) back to exponents (into
    `out`, int32 [n, nx], when given: Laurent codes only)."""
    import torch
    ctx = ctx or context()
    _dev_check(codes, torch.int64, "codes")
    n = codes.shape[0]
    if out is not None:
        if poisson or tuple(out.shape) != (n, layout.nx) or out.dtype != torch.int32:
            raise ValueError("out must be int32 [n, nx] for Laurent codes")
        x = out
    else:
        x = torch.empty((n, layout.nx), dtype=torch.int32, device=codes.device)
    y = t = None
    if poisson:
        y = torch.empty((n, layout.ny), dtype=torch.int32, device=codes.device)
        t = torch.empty(n, dtype=torch.uint8, device=codes.device)
    ctx.check(lib().kp_decode(ctx.h, C.byref(layout), 1 if poisson else 0, n, _ptr(codes),
                              _ptr(x), _ptr(y), _ptr(t), flags, _stream()))
    return (x, y, t) if poisson else x


def mul_bound(layout, poisson, dtype, mode, na, nb, ctx=None):
    """kp_mul_bound -> (resolved mode name, max result terms, workspace bytes)."""
    ctx = ctx or context()
    m = C.c_int32()
    mo = C.c_int64()
    ws = C.c_size_t()
    ctx.check(lib().kp_mul_bound(ctx.h, C.byref(layout), 1 if poisson else 0, dtype,
                                 MODES[mode] if isinstance(mode, str) else mode, na, nb,
                                 C.byref(m), C.byref(mo), C.byref(ws)))
    return MODE_NAMES[m.value], mo.value, ws.value


class Workspace:
    """Grow-only device scratch for repeated multiplies (torch-owned)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        import torch
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


def _dt(t, exact=False):
    """Library dtype of factor coefficients; `exact` asks for 128-bit sums of
    int64 products (KP_I128)."""
    import torch
    if t.dtype == torch.int64:
        return KP_I128 if exact else KP_I64
    if exact:
        raise ValueError("exact (128-bit) products take int64 coefficients")
    if t.dtype == torch.float64:
        return KP_F64
    raise ValueError(f"coefficients must be int64 or float64, got {t.dtype}")


def _out_coef(n, dt, device):
    """Result coefficient buffer: [n] of the factor type, or int64 [n, 2]
    (low word, high word) for 128-bit results."""
    import torch
    if dt == KP_I128:
        return torch.empty((n, 2), dtype=torch.int64, device=device)
    return torch.empty(n, dtype=torch.float64 if dt == KP_F64 else torch.int64, device=device)


def to_pyint(coef, unsigned=False):
    """Python integers of 128-bit result coefficients (int64 [n, 2] tensor or
    array: low word, high word).  The sums are exact modulo 2^128: read as
    two's complement (default) they are exact while |sum| < 2^127, read as
    unsigned (`unsigned=True`) for nonnegative sums below 2^128."""
    import numpy as np
    w = np.asarray(coef.cpu() if hasattr(coef, "cpu") else coef, dtype=np.int64).reshape(-1, 2)
    out = [(int(lo) & 0xFFFFFFFFFFFFFFFF) | (int(hi) << 64) for lo, hi in w]
    return [v % (1 << 128) for v in out] if unsigned else out


def mul_laurent_codes(layout, a_codes, a_coef, b_codes, b_coef, mode="auto", ctx=None,
                      workspace=None, out=None, flags=0, exact=False):
    """kp_mul_laurent on coded factors.

    Returns (codes, coef, count_tensor).  Without KP_FLAG_ASYNC the outputs
    are trimmed to the result size (one host read of the count).  With
    `exact` (int64 factors) coef is int64 [n, 2]: 128-bit sums.
    """
    import torch
    ctx = ctx or context()
    dev = a_codes.device
    dt = _dt(a_coef, exact)
    for t, nm in ((a_codes, "a_codes"), (b_codes, "b_codes")):
        _dev_check(t, torch.int64, nm)
    _dev_check(a_coef, a_coef.dtype, "a_coef")
    _dev_check(b_coef, a_coef.dtype, "b_coef")
    na, nb = a_codes.shape[0], b_codes.shape[0]
    _, max_out, ws = mul_bound(layout, False, dt, mode, na, nb, ctx)
    if out is None:
        oc = torch.empty(max(max_out, 1), dtype=torch.int64, device=dev)
        ov = _out_coef(max(max_out, 1), dt, dev)
        on = torch.empty(1, dtype=torch.int64, device=dev)
    else:
        oc, ov, on = out
    wbuf = (workspace or Workspace()).get(ws, dev)
    st = lib().kp_mul_laurent(ctx.h, C.byref(layout), dt, MODES[mode] if isinstance(mode, str)
                              else mode, flags | KP_FLAG_ASYNC, _ptr(a_codes), _ptr(a_coef), na,
                              _ptr(b_codes), _ptr(b_coef), nb, _ptr(oc), _ptr(ov), oc.shape[0],
                              _ptr(on), _ptr(wbuf), wbuf.numel(), _stream())
    ctx.check(st)
    if flags & KP_FLAG_ASYNC:
        return oc, ov, on
    n = _count(ctx, on)
    return oc[:n], ov[:n], on


def mul_laurent_noalloc(layout, a_codes, a_coef, b_codes, b_coef, out, mode="auto", ctx=None,
                        flags=0):
    """kp_mul_laurent_noalloc: kp_mul_laurent with the library's per-GPU
    scratch array as workspace.  `out` = (codes int64 [cap], coef [cap],
    count int64 [1]), caller-allocated; nothing is allocated here.  Returns
    the count (without KP_FLAG_ASYNC; one read) or None."""
    import torch
    ctx = ctx or context()
    dt = _dt(a_coef)
    for t, nm in ((a_codes, "a_codes"), (b_codes, "b_codes")):
        _dev_check(t, torch.int64, nm)
    oc, ov, on = out
    ctx.check(lib().kp_mul_laurent_noalloc(
        ctx.h, C.byref(layout), dt, _mode(mode), flags, _ptr(a_codes), _ptr(a_coef),
        a_codes.shape[0], _ptr(b_codes), _ptr(b_coef), b_codes.shape[0], _ptr(oc), _ptr(ov),
        oc.shape[0], _ptr(on), _stream()))
    return None if flags & KP_FLAG_ASYNC else int(on.item())


def _count(ctx, on):
    """Result count of an asynchronous multiply: one synchronising read.  A
    negative count is -(status); the context's latched error is then read
    (and cleared) for the message."""
    n = int(on.item())
    if n < 0:
        ctx.sync_check()
        raise KPError(-n, status_str(-n))
    return n


def mul_poisson_codes(layout, a, b, mode="auto", ctx=None, workspace=None, out=None, flags=0):
    """kp_mul_poisson on coded series a = (x_codes, y_codes, is_sin, coef)."""
    import torch
    ctx = ctx or context()
    ax, ay, at, ac = a
    bx, by, bt, bc = b
    dev = ax.device
    for t, nm in ((ax, "a_x"), (ay, "a_y"), (bx, "b_x"), (by, "b_y")):
        _dev_check(t, torch.int64, nm)
    _dev_check(at, torch.uint8, "a_sin")
    _dev_check(bt, torch.uint8, "b_sin")
    _dev_check(ac, torch.float64, "a_coef")
    _dev_check(bc, torch.float64, "b_coef")
    na, nb = ac.shape[0], bc.shape[0]
    _, max_out, ws = mul_bound(layout, True, KP_F64, mode, na, nb, ctx)
    if out is None:
        ok = torch.empty(max(max_out, 1), dtype=torch.int64, device=dev)
        ov = torch.empty(max(max_out, 1), dtype=torch.float64, device=dev)
        on = torch.empty(1, dtype=torch.int64, device=dev)
    else:
        ok, ov, on = out
    wbuf = (workspace or Workspace()).get(ws, dev)
    st = lib().kp_mul_poisson(ctx.h, C.byref(layout), MODES[mode] if isinstance(mode, str)
                              else mode, flags | KP_FLAG_ASYNC, _ptr(ax), _ptr(ay), _ptr(at), _ptr(ac), na,
                              _ptr(bx), _ptr(by), _ptr(bt), _ptr(bc), nb, _ptr(ok), _ptr(ov),
                              ok.shape[0], _ptr(on), _ptr(wbuf), wbuf.numel(), _stream())
    ctx.check(st)
    if flags & KP_FLAG_ASYNC:
        return ok, ov, on
    n = _count(ctx, on)
    return ok[:n], ov[:n], on


# ------------------------------------------------------------------ high level
@dataclass
class Poly:
    """Sparse Laurent polynomial: exps int32 [n, nv], coef int64 or float64 [n]."""
    exps: "object"
    coef: "object"

    @property
    def nv(self):
        return self.exps.shape[1]


@dataclass
class PoissonSeries:
    """Sparse Poisson series in canonical form: x int32 [n, nx], y int32 [n, ny],
    is_sin uint8 [n], coef float64 [n]."""
    x: "object"
    y: "object"
    is_sin: "object"
    coef: "object"


def _boxes(ctx, *vals):
    """(min, max) lists of every int32 [n, nv] tensor, with one host read."""
    import torch
    widths = [v.shape[1] for v in vals]
    out = torch.empty(max(1, 2 * sum(widths)), dtype=torch.int32, device=vals[0].device)
    off = 0
    for v, nv in zip(vals, widths):
        minmax(v, ctx, KP_FLAG_ASYNC, out[off:off + 2 * nv])
        off += 2 * nv
    mm = out.cpu().tolist()
    res, off = [], 0
    for nv in widths:
        res.append((mm[off:off + nv], mm[off + nv:off + 2 * nv]))
        off += 2 * nv
    return res


def laurent_layout(a: Poly, b: Poly, ctx=None) -> Layout:
    ctx = ctx or context()
    (amin, amax), (bmin, bmax) = _boxes(ctx, a.exps, b.exps)
    return layout_product(a.nv, 0, amin, amax, bmin, bmax)


def _mode(mode):
    return MODES[mode] if isinstance(mode, str) else mode


def plan_laurent(a: Poly, b: Poly, mode="auto", ctx=None, stream=None, exact=False):
    """kp_plan_laurent: boxes of both factors (one launch, one wait) ->
    (Layout, resolved mode name, max result terms, workspace bytes)."""
    import torch
    ctx = ctx or context()
    _dev_check(a.exps, torch.int32, "a.exps")
    _dev_check(b.exps, torch.int32, "b.exps")
    if a.nv != b.nv:
        raise ValueError("factors must have the same number of variables")
    s = _raw_stream(a.exps.device) if stream is None else stream.cuda_stream
    lay, m, mo, ws = Layout(), C.c_int32(), C.c_int64(), C.c_size_t()
    ctx.check(lib().kp_plan_laurent(ctx.h, a.nv, _dt(a.coef, exact), _mode(mode), a.exps.data_ptr(),
                                    a.exps.shape[0], b.exps.data_ptr(), b.exps.shape[0],
                                    C.byref(lay), C.byref(m), C.byref(mo), C.byref(ws), s))
    return lay, MODE_NAMES[m.value], mo.value, ws.value


_SIZE_HINT = {}   # (na, nb, nvars, dtype, mode) -> (result capacity, workspace bytes)


def mul_laurent(a: Poly, b: Poly, mode="auto", ctx=None, workspace=None, exact=False):
    """A * B for device-resident Laurent polynomials; returns (Poly, Layout).

    One library call when the sizes of the last product of the same shape
    still fit (kp_mul_laurent_auto: plan, encode, multiply, decode, wait for
    the count), else the plan's sizes and a second call.  The device count
    slot sits after the multiply's workspace.  With `exact` (int64 factors)
    every product and sum is formed in 128 bits and the result's coef is
    int64 [n, 2] (low word, high word; `to_pyint` converts)."""
    import torch
    ctx = ctx or context()
    _dev_check(a.exps, torch.int32, "a.exps")
    _dev_check(b.exps, torch.int32, "b.exps")
    _dev_check(a.coef, a.coef.dtype, "a.coef")
    _dev_check(b.coef, a.coef.dtype, "b.coef")
    if a.nv != b.nv:
        raise ValueError("factors must have the same number of variables")
    dev = a.exps.device
    s = _raw_stream(dev)
    na, nb, nv, dt, md = a.exps.shape[0], b.exps.shape[0], a.nv, _dt(a.coef, exact), _mode(mode)
    key = (na, nb, nv, dt, md)
    cap, ws = _SIZE_HINT.get(key, (1, 0))
    workspace = workspace or Workspace()
    lay, n, need_cap, need_ws = Layout(), C.c_int64(), C.c_int64(), C.c_size_t()
    for attempt in range(2):
        ox = torch.empty((cap, nv), dtype=torch.int32, device=dev)
        oc = _out_coef(cap, dt, dev)
        ws_al = (ws + 255) & ~255
        w = workspace.get(ws_al + 256, dev).data_ptr()
        if attempt == 0:
            st = lib().kp_mul_laurent_auto(
                ctx.h, nv, dt, md, 0, a.exps.data_ptr(), a.coef.data_ptr(), na,
                b.exps.data_ptr(), b.coef.data_ptr(), nb, ox.data_ptr(), oc.data_ptr(), cap,
                w + ws_al, C.byref(n), w, ws_al, C.byref(lay), C.byref(need_cap),
                C.byref(need_ws), s)
            if st == KP_E_WORKSPACE and (need_cap.value > cap or need_ws.value > ws):
                cap, ws = need_cap.value, need_ws.value
                _SIZE_HINT[key] = (cap, ws)
                continue
        else:
            st = lib().kp_mul_laurent_exps(
                ctx.h, C.byref(lay), dt, md, 0, a.exps.data_ptr(), a.coef.data_ptr(), na,
                b.exps.data_ptr(), b.coef.data_ptr(), nb, ox.data_ptr(), oc.data_ptr(), cap,
                w + ws_al, C.byref(n), w, ws_al, s)
        ctx.check(st)
        break
    n = n.value
    return Poly(ox[:n], oc[:n]), lay


def poisson_layout(a: PoissonSeries, b: PoissonSeries, ctx=None) -> Layout:
    """The product's layout, as kp_plan_poisson computes it."""
    return plan_poisson(a, b, "auto", ctx)[0]


def plan_poisson(a: PoissonSeries, b: PoissonSeries, mode="auto", ctx=None, stream=None):
    """kp_plan_poisson -> (Layout, resolved mode name, max result terms, workspace bytes)."""
    import torch
    ctx = ctx or context()
    for t, nm in ((a.x, "a.x"), (a.y, "a.y"), (b.x, "b.x"), (b.y, "b.y")):
        _dev_check(t, torch.int32, nm)
    nx, ny = a.x.shape[1], a.y.shape[1]
    if (b.x.shape[1], b.y.shape[1]) != (nx, ny):
        raise ValueError("factors must have the same numbers of variables")
    s = _raw_stream(a.y.device) if stream is None else stream.cuda_stream
    lay, m, mo, ws = Layout(), C.c_int32(), C.c_int64(), C.c_size_t()
    ctx.check(lib().kp_plan_poisson(ctx.h, nx, ny, _mode(mode), a.x.data_ptr(), a.y.data_ptr(),
                                    a.y.shape[0], b.x.data_ptr(), b.y.data_ptr(), b.y.shape[0],
                                    C.byref(lay), C.byref(m), C.byref(mo), C.byref(ws), s))
    return lay, MODE_NAMES[m.value], mo.value, ws.value


def mul_poisson(a: PoissonSeries, b: PoissonSeries, mode="auto", ctx=None, workspace=None):
    """A * B for device-resident canonical Poisson series; returns (series, Layout)."""
    import torch
    ctx = ctx or context()
    for t, nm in ((a.is_sin, "a.is_sin"), (b.is_sin, "b.is_sin")):
        _dev_check(t, torch.uint8, nm)
    for t, nm in ((a.coef, "a.coef"), (b.coef, "b.coef")):
        _dev_check(t, torch.float64, nm)
    dev = a.y.device
    s = _raw_stream(dev)
    lay, _, max_out, ws = plan_poisson(a, b, mode, ctx)
    cap = max(max_out, 1)
    nx, ny = a.x.shape[1], a.y.shape[1]
    ox = torch.empty((cap, nx), dtype=torch.int32, device=dev)
    oy = torch.empty((cap, ny), dtype=torch.int32, device=dev)
    ot = torch.empty(cap, dtype=torch.uint8, device=dev)
    oc = torch.empty(cap, dtype=torch.float64, device=dev)
    ws_al = (ws + 255) & ~255
    wbuf = (workspace or Workspace()).get(ws_al + 256, dev)
    w = wbuf.data_ptr()
    n = C.c_int64()
    ctx.check(lib().kp_mul_poisson_exps(
        ctx.h, C.byref(lay), _mode(mode), 0, a.x.data_ptr(), a.y.data_ptr(), a.is_sin.data_ptr(),
        a.coef.data_ptr(), a.y.shape[0], b.x.data_ptr(), b.y.data_ptr(), b.is_sin.data_ptr(),
        b.coef.data_ptr(), b.y.shape[0], ox.data_ptr(), oy.data_ptr(), ot.data_ptr(),
        oc.data_ptr(), cap, w + ws_al, C.byref(n), w, ws_al, s))
    n = n.value
    return PoissonSeries(ox[:n], oy[:n], ot[:n], oc[:n]), lay


# ------------------------------------------------------------------ batches
class Batch:
    """kp_batch: many products queued by one call, optionally captured once
    into a HIP graph and replayed.  Descriptors reference the caller's
    tensors, which this object keeps alive until clear()."""

    def __init__(self, max_tasks, ctx=None):
        self.ctx = ctx or context()
        h = C.c_void_p()
        self.ctx.check(lib().kp_batch_create(self.ctx.h, max_tasks, C.byref(h)))
        self.h = h
        self._keep = []

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.kp_batch_destroy(self.h)
            self.h = None

    def _add(self, d, tensors):
        tid = C.c_int64()
        self.ctx.check(lib().kp_batch_add(self.h, C.byref(d), C.byref(tid)))
        self._keep.append(tensors)
        return tid.value

    def add_laurent(self, layout, a_codes, a_coef, b_codes, b_coef, out, workspace, mode="auto",
                    exact=False):
        """Queue a Laurent product; `out` = (codes, coef, count) device tensors,
        `workspace` a uint8 device tensor of kp_mul_bound's size; `exact` as
        in mul_laurent (coef then int64 [cap, 2])."""
        oc, ov, on = out
        d = MulDesc(kind=KP_KIND_LAURENT, layout=layout, dtype=_dt(a_coef, exact),
                    mode=MODES[mode] if isinstance(mode, str) else mode,
                    a_codes=a_codes.data_ptr(), a_coef=a_coef.data_ptr(), na=a_codes.shape[0],
                    b_codes=b_codes.data_ptr(), b_coef=b_coef.data_ptr(), nb=b_codes.shape[0],
                    out_codes=oc.data_ptr(), out_coef=ov.data_ptr(), out_cap=oc.shape[0],
                    out_n=on.data_ptr(), workspace=workspace.data_ptr(),
                    workspace_bytes=workspace.numel())
        return self._add(d, (a_codes, a_coef, b_codes, b_coef, oc, ov, on, workspace))

    def add_poisson(self, layout, a, b, out, workspace, mode="auto"):
        """Queue a Poisson product of coded series a, b = (x, y, is_sin, coef)."""
        ok, ov, on = out
        d = MulDesc(kind=KP_KIND_POISSON, layout=layout, dtype=KP_F64,
                    mode=MODES[mode] if isinstance(mode, str) else mode,
                    a_codes=a[0].data_ptr(), a_y=a[1].data_ptr(), a_sin=a[2].data_ptr(),
                    a_coef=a[3].data_ptr(), na=a[0].shape[0], b_codes=b[0].data_ptr(),
                    b_y=b[1].data_ptr(), b_sin=b[2].data_ptr(), b_coef=b[3].data_ptr(),
                    nb=b[0].shape[0], out_codes=ok.data_ptr(), out_coef=ov.data_ptr(),
                    out_cap=ok.shape[0], out_n=on.data_ptr(), workspace=workspace.data_ptr(),
                    workspace_bytes=workspace.numel())
        return self._add(d, (*a, *b, ok, ov, on, workspace))

    def launch(self, graph=False, stream=None):
        """Queue every task (replaying the captured graph when `graph`).  A
        graph is captured on a side stream of this batch, ordered after and
        before the current stream's work."""
        import torch
        cur = torch.cuda.current_stream() if stream is None else stream
        if not graph:
            self.ctx.check(lib().kp_batch_launch(self.h, 0, _stream(cur)))
            return
        if getattr(self, "_side", None) is None:
            self._side = torch.cuda.Stream()
        self._side.wait_stream(cur)
        self.ctx.check(lib().kp_batch_launch(self.h, KP_BATCH_GRAPH, _stream(self._side)))
        cur.wait_stream(self._side)

    def status(self, task):
        n = C.c_int64()
        st = lib().kp_batch_status(self.h, task, C.byref(n))
        if st != KP_OK:
            raise KPError(st, status_str(st))
        return n.value

    def clear(self):
        self.ctx.check(lib().kp_batch_clear(self.h))
        self._keep = []


class Pack:
    """kp_pack: many whole Laurent products in one fixed sequence of
    persistent launches over a device task table; with graph=True the
    sequence is a HIP graph captured at the first launch and replayed by
    every later one.  One batch at a time: launch(), then wait()."""

    def __init__(self, max_tasks, ctx=None):
        self.ctx = ctx or context()
        h = C.c_void_p()
        self.ctx.check(lib().kp_pack_create(self.ctx.h, max_tasks, C.byref(h)))
        self.h = h
        self.max_tasks = max_tasks
        self._run = None
        self._side = None

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.kp_pack_destroy(self.h)
            self.h = None

    def launch(self, products, graph=False, stream=None, alloc=None):
        """Plans the products [(Poly a, Poly b), ...] (one host wait for every
        factor's box) and queues them on `stream` (default: the current one).
        `alloc(numel, dtype)` supplies the device buffers (results and arena)
        when given, else they are new tensors."""
        self.plan(products, graph, stream)
        self.run(alloc)

    def plan(self, products, graph=False, stream=None):
        """kp_pack_plan: the products' bounds (list) and the device bytes that
        run() allocates (results and arena), without queueing them."""
        import torch
        n = len(products)
        tasks = (PackTask * max(n, 1))()
        for k, (a, b) in enumerate(products):
            for t, nm in ((a.exps, "a.exps"), (b.exps, "b.exps")):
                _dev_check(t, torch.int32, nm)
            if a.coef.dtype != b.coef.dtype or a.coef.dtype not in (torch.int64, torch.float64):
                raise ValueError("both factors int64 or both float64")
            if a.nv != b.nv:
                raise ValueError("factors must have the same number of variables")
            tasks[k] = PackTask(a.nv, KP_F64 if a.coef.dtype == torch.float64 else KP_I64,
                                a.exps.data_ptr(), a.coef.data_ptr(), a.coef.shape[0],
                                b.exps.data_ptr(), b.coef.data_ptr(), b.coef.shape[0])
        cur = torch.cuda.current_stream() if stream is None else stream
        run_on = cur
        if graph and cur.cuda_stream == 0:   # capture needs a stream of its own
            if self._side is None:
                self._side = torch.cuda.Stream()
            self._side.wait_stream(cur)
            run_on = self._side
        caps = (C.c_int64 * max(n, 1))()
        ab = C.c_size_t()
        self.ctx.check(lib().kp_pack_plan(self.h, tasks, n, caps, C.byref(ab),
                                          C.c_void_p(run_on.cuda_stream)))
        caps = [int(caps[k]) for k in range(n)]
        nx = sum(c * a.nv for c, (a, _) in zip(caps, products))
        al = lambda x: (x + 255) & ~255
        need = al(4 * max(nx, 1)) + al(8 * max(sum(caps), 1)) + al(max(ab.value, 256))
        self._planned = (products, caps, ab.value, nx, graph, cur, run_on)
        return caps, need

    def run(self, alloc=None):
        """kp_pack_run of the planned products."""
        import torch
        products, caps, ab, nx, graph, cur, run_on = self._planned
        n = len(products)
        with torch.cuda.stream(run_on):
            dev = cur.device
            new = alloc or (lambda n_, dt: torch.empty(n_, dtype=dt, device=dev))
            X = new(max(nx, 1), torch.int32)
            V = new(max(sum(caps), 1), torch.int64)
            arena = new(max(ab, 256), torch.uint8)
        ox, oc, views, px, pc = (C.c_void_p * max(n, 1))(), (C.c_void_p * max(n, 1))(), [], 0, 0
        for k, (a, _) in enumerate(products):
            x = X[px:px + caps[k] * a.nv].view(caps[k], a.nv)
            v = V[pc:pc + caps[k]]
            if a.coef.dtype == torch.float64:
                v = v.view(torch.float64)
            ox[k], oc[k] = x.data_ptr(), v.data_ptr()
            views.append((x, v))
            px += caps[k] * a.nv
            pc += caps[k]
        self.ctx.check(lib().kp_pack_run(self.h, ox, oc, C.c_void_p(arena.data_ptr()), ab,
                                         KP_PACK_GRAPH if graph else 0,
                                         C.c_void_p(run_on.cuda_stream)))
        if run_on is not cur:
            cur.wait_stream(run_on)
        self._planned = None
        self._run = (products, views, arena, n)

    def ready(self):
        """True when the last launch's counts are back (no wait)."""
        d = C.c_int32()
        self.ctx.check(lib().kp_pack_query(self.h, C.byref(d)))
        return bool(d.value)

    def wait(self):
        """The last launch's products, as Polys (views of two shared buffers)."""
        _, views, _, n = self._run
        counts = (C.c_int64 * max(n, 1))()
        self._run = None
        self.ctx.check(lib().kp_pack_wait(self.h, counts))
        return [Poly(x[:counts[k]], v[:counts[k]]) for k, (x, v) in enumerate(views)]
