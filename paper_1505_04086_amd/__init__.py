"""Python binding of librsoc (speculative First-Fit graph colouring on MI355X).

Argument marshalling only: every step of the colouring runs in the HIP
kernels of ``librsoc.so`` (built from ``csrc/`` by :func:`build.build`).  The
names mirror the C ABI in ``include/rsoc.h``.  Host arrays are numpy int32;
device arrays are torch tensors on a ROCm device (torch provides device
memory and streams only).

``torch`` is imported before the library is loaded so that the process uses a
single HIP runtime (torch's), which the library then binds to.  If the
library has not been built, importing this package raises ImportError: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import weakref
import os

import numpy as np

try:  # torch first: its HIP runtime is the one the library must share
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the environment
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsoc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("librsoc.so is not built (run paper_1505_04086_amd.build.build() or "
                      "__graft_entry__.build()); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

RSOC_OK = 0
RSOC_EINVAL = -1
RSOC_ECSR = -2
RSOC_ESELFLOOP = -3
RSOC_EASYM = -4
RSOC_ENOMEM = -5
RSOC_EHIP = -6
RSOC_ENOCONV = -7
RSOC_EBUDGET = -8
RSOC_ENOTFOUND = -9
RSOC_EINTERNAL = -10
RSOC_ESCRATCH = -11

RSOC_MODE_OPTIMISTIC = 0
RSOC_MODE_DETERMINISTIC = 1
RSOC_MODE_TWO_PHASE = 2
RSOC_MODE_TWO_PHASE_LIVE = 3
RSOC_TIE_LOWER_KEEPS = 0
RSOC_TIE_HIGHER_KEEPS = 1
RSOC_CHECK_CSR = 1
RSOC_CHECK_SYMMETRY = 2

_MODES = {"optimistic": 0, "opt": 0, "deterministic": 1, "det": 1, "two_phase": 2, "two_phase_live": 3,
          0: 0, 1: 1, 2: 2, 3: 3}
_TIES = {"lower": 0, "higher": 1, 0: 0, 1: 1}


class rsoc_options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tie", ctypes.c_int32), ("max_rounds", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("t_thread", ctypes.c_int32), ("t_wave", ctypes.c_int32),
                ("grid_thread", ctypes.c_int32), ("grid_wave", ctypes.c_int32),
                ("rounds_per_sync", ctypes.c_int32), ("small_cutoff", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("full_sweep", ctypes.c_int32), ("lookahead", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("grid_list", ctypes.c_int32), ("tail", ctypes.c_int32),
                ("distance", ctypes.c_int32), ("grid_bin", ctypes.c_int32), ("hub_first", ctypes.c_int32),
                ("bands", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class rsoc_stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("passes", ctypes.c_int32), ("colors", ctypes.c_int32),
                ("colors_distinct", ctypes.c_int32), ("conflicts", ctypes.c_int64), ("inspected", ctypes.c_int64),
                ("alg_bytes", ctypes.c_int64), ("ms", ctypes.c_double), ("ms_round0", ctypes.c_double),
                ("ms_round1", ctypes.c_double), ("bytes_round0", ctypes.c_int64), ("bytes_round1", ctypes.c_int64),
                ("max_degree", ctypes.c_int32), ("bin_counts", ctypes.c_int32 * 3),
                ("per_round_L", ctypes.POINTER(ctypes.c_int32)), ("per_round_cap", ctypes.c_int32),
                ("worklist0", ctypes.c_int32), ("chunk", ctypes.c_int32), ("small_graphs", ctypes.c_int32),
                ("per_round_U", ctypes.POINTER(ctypes.c_int32))]


_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sig = {
    "rsoc_default_options": (None, [ctypes.POINTER(rsoc_options)]),
    "rsoc_color": (_i32, [_p, _p, _i32, _p]),
    "rsoc_ctx_create": (_i32, [ctypes.POINTER(_p), _i32]),
    "rsoc_ctx_destroy": (None, [_p]),
    "rsoc_color_ex": (_i32, [_p, _p, _p, _i32, _p, ctypes.POINTER(rsoc_options), ctypes.POINTER(rsoc_stats)]),
    "rsoc_color_device": (_i32, [_p, _p, _p, _i32, _p, ctypes.POINTER(rsoc_options), ctypes.POINTER(rsoc_stats), _p]),
    "rsoc_color_batch": (_i32, [_p, _i32, _p, _p, _p, _p, _p, _p, ctypes.POINTER(rsoc_options),
                                ctypes.POINTER(rsoc_stats), _p]),
    "rsoc_pool_create": (_i32, [_p, _i64, _i32, ctypes.POINTER(_p)]),
    "rsoc_pool_destroy": (None, [_p]),
    "rsoc_pool_admit": (_i32, [_p, _p, _p, _i32, _p, ctypes.POINTER(rsoc_options)]),
    "rsoc_pool_admit_recolor": (_i32, [_p, _p, _p, _i32, _p, _p, _i32, ctypes.POINTER(rsoc_options)]),
    "rsoc_pool_step": (_i32, [_p, _p, _p, _i32]),
    "rsoc_pool_step_launch": (_i32, [_p, _p]),
    "rsoc_pool_step_finish": (_i32, [_p, _p, _i32]),
    "rsoc_pool_live": (_i32, [_p]),
    "rsoc_pool_reserved_bytes": (_i64, [_p]),
    "rsoc_pool_result": (_i32, [_p, _i32, ctypes.POINTER(rsoc_stats)]),
    "rsoc_recolor_device": (_i32, [_p, _p, _p, _i32, _p, _p, _i32, ctypes.POINTER(rsoc_options),
                                   ctypes.POINTER(rsoc_stats), _p]),
    "rsoc_color_classes": (_i32, [_p, _p, _i32, _i32, _p, _p, _p]),
    "rsoc_color_classes_noalloc": (_i32, [_p, _i32, _i32, _p, _p, _p]),
    "rsoc_check_csr": (_i32, [_p, _p, _i32, _i32]),
    "rsoc_strerror": (ctypes.c_char_p, [_i32]),
    "rsoc_last_error": (ctypes.c_char_p, []),
}
EXPORTED = tuple(_sig)
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class RsocError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = "%s: %s (%d)" % (where, rsoc_strerror(code), code)
        extra = rsoc_last_error()
        if code == RSOC_EHIP and extra:
            msg += " [" + extra + "]"
        super().__init__(msg)


def rsoc_strerror(code: int) -> str:
    return _lib.rsoc_strerror(code).decode()


def rsoc_last_error() -> str:
    return (_lib.rsoc_last_error() or b"").decode()


def _chk(code, where, ok_noconv=False):
    if code < 0 and not (ok_noconv and code == RSOC_ENOCONV):
        raise RsocError(code, where)
    return code


def make_options(mode="optimistic", tie="lower", max_rounds=0, validate=0, **tuning) -> rsoc_options:
    o = rsoc_options()
    _lib.rsoc_default_options(ctypes.byref(o))
    o.mode = _MODES[mode]
    o.tie = _TIES[tie]
    o.max_rounds = int(max_rounds)
    o.validate = int(validate)
    for k, v in tuning.items():
        if v is not None:
            setattr(o, k, int(v))
    return o


def _per_round_arrays(st: rsoc_stats, cap: int):
    """Caller arrays for |L| per round and |U| per pass (kept alive by the
    returned pair), or None."""
    if not cap:
        return None
    L = np.zeros(cap, dtype=np.int32)
    U = np.zeros(cap, dtype=np.int32)
    st.per_round_L = L.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    st.per_round_U = U.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    st.per_round_cap = cap
    return L, U


def stats_dict(st: rsoc_stats, LU=None) -> dict:
    d = {f: getattr(st, f) for f, _ in rsoc_stats._fields_
         if f not in ("per_round_L", "per_round_U", "reserved", "bin_counts")}
    d["bin_counts"] = list(st.bin_counts)
    if LU is not None:
        L, U = LU
        d["L_sizes"] = L[:min(st.rounds, len(L))].copy()
        d["U_sizes"] = U[:min(st.passes, len(U))].copy()
    return d


def _host_i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, (a.ctypes.data if a.size else None)


def _dev_ptr(t):
    if t is None:
        return None
    if not (hasattr(t, "is_cuda") and t.is_cuda):
        raise TypeError("expected a device tensor")
    if t.dtype not in (torch.int32, torch.int64) or not t.is_contiguous():
        raise TypeError("expected a contiguous int32/int64 device tensor")
    return t.data_ptr() if t.numel() else None


def _stream_ptr(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ API --

def rsoc_color(row_ptr, col_idx, n=None, colors_out=None):
    """Host arrays in, host colours out (default options).  Returns (colors, K)."""
    rp, rpp = _host_i32(row_ptr)
    ci, cip = _host_i32(col_idx)
    n = len(rp) - 1 if n is None else int(n)
    out = np.empty(max(n, 1), dtype=np.int32) if colors_out is None else colors_out
    k = _chk(_lib.rsoc_color(rpp, cip, n, out.ctypes.data), "rsoc_color")
    return out[:n], k


class Context:
    """An rsoc_ctx on one device (rsoc_ctx_create / rsoc_ctx_destroy)."""

    def __init__(self, device: int = 0):
        h = _p()
        _chk(_lib.rsoc_ctx_create(ctypes.byref(h), int(device)), "rsoc_ctx_create")
        self.h = h
        self.device = device
        self._pools = weakref.WeakSet()

    def close(self):
        if self.h:
            # pools hold the context's scratch and streams: they go first
            for pool in list(self._pools):
                pool.close()
            _lib.rsoc_ctx_destroy(self.h)
            self.h = _p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def rsoc_ctx_create(device: int = 0) -> Context:
    return Context(device)


def rsoc_ctx_destroy(ctx: Context):
    ctx.close()


def rsoc_color_ex(ctx: Context, row_ptr, col_idx, n=None, colors_out=None, options=None, per_round_cap=0,
                  allow_noconv=False):
    """Host-pointer colouring.  Returns (colors, K, stats dict)."""
    rp, rpp = _host_i32(row_ptr)
    ci, cip = _host_i32(col_idx)
    n = len(rp) - 1 if n is None else int(n)
    out = np.empty(max(n, 1), dtype=np.int32) if colors_out is None else colors_out
    o = options if options is not None else make_options()
    st = rsoc_stats()
    L = _per_round_arrays(st, per_round_cap)
    k = _chk(_lib.rsoc_color_ex(ctx.h, rpp, cip, n, out.ctypes.data, ctypes.byref(o), ctypes.byref(st)),
             "rsoc_color_ex", ok_noconv=allow_noconv)
    return out[:n], k, stats_dict(st, L)


def rsoc_color_device(ctx: Context, d_row_ptr, d_col_idx, n, d_colors_out, options=None, stream=None,
                      per_round_cap=0, allow_noconv=False):
    """Device-tensor colouring.  Returns (K, stats dict)."""
    o = options if options is not None else make_options()
    st = rsoc_stats()
    L = _per_round_arrays(st, per_round_cap)
    k = _chk(_lib.rsoc_color_device(ctx.h, _dev_ptr(d_row_ptr), _dev_ptr(d_col_idx), int(n), _dev_ptr(d_colors_out),
                                    ctypes.byref(o), ctypes.byref(st), _stream_ptr(stream)),
             "rsoc_color_device", ok_noconv=allow_noconv)
    return k, stats_dict(st, L)


def rsoc_recolor_device(ctx: Context, d_row_ptr, d_col_idx, n, d_colors_inout, d_touched, options=None,
                        stream=None, per_round_cap=0, allow_noconv=False):
    """Recolouring after topology edits: d_colors_inout holds the colouring
    before the edits (negative = none) and receives the result; d_touched
    (device int32, may be None or empty) lists the touched vertices.
    Returns (K, stats dict)."""
    o = options if options is not None else make_options()
    st = rsoc_stats()
    L = _per_round_arrays(st, per_round_cap)
    nt = 0 if d_touched is None else int(d_touched.numel())
    k = _chk(_lib.rsoc_recolor_device(ctx.h, _dev_ptr(d_row_ptr), _dev_ptr(d_col_idx), int(n),
                                      _dev_ptr(d_colors_inout), _dev_ptr(d_touched) if nt else None, nt,
                                      ctypes.byref(o), ctypes.byref(st), _stream_ptr(stream)),
             "rsoc_recolor_device", ok_noconv=allow_noconv)
    return k, stats_dict(st, L)


def rsoc_color_classes(ctx: Context, d_colors, n, K, d_class_ptr, d_class_vtx, stream=None):
    """Colour classes of a device colouring: fills d_class_ptr (K+1) and
    d_class_vtx (n); class k is d_class_vtx[d_class_ptr[k]:d_class_ptr[k+1]]."""
    _chk(_lib.rsoc_color_classes(ctx.h, _dev_ptr(d_colors), int(n), int(K), _dev_ptr(d_class_ptr),
                                 _dev_ptr(d_class_vtx), _stream_ptr(stream)), "rsoc_color_classes")


def rsoc_color_classes_noalloc(d_colors, n, K, d_class_ptr, d_class_vtx, stream=None):
    """rsoc_color_classes without a context and without allocating: runs on the
    current device with the library's fixed per-GPU scratch (n <= 2^30)."""
    _chk(_lib.rsoc_color_classes_noalloc(_dev_ptr(d_colors), int(n), int(K), _dev_ptr(d_class_ptr),
                                         _dev_ptr(d_class_vtx), _stream_ptr(stream)), "rsoc_color_classes_noalloc")


def rsoc_color_batch(ctx: Context, vtx_off, nnz_off, d_row_ptr_cat, d_col_idx_cat, d_colors_cat, options=None,
                     stream=None, per_round_cap=0):
    """Batched colouring.  vtx_off/nnz_off are host int64 arrays (G+1).
    Returns (counts int32[G], max K, stats dict); with per_round_cap the stats
    carry L_sizes, |L| per recolouring round summed over the graphs."""
    vo = np.ascontiguousarray(vtx_off, dtype=np.int64)
    no = np.ascontiguousarray(nnz_off, dtype=np.int64)
    G = len(vo) - 1
    counts = np.zeros(max(G, 1), dtype=np.int32)
    o = options if options is not None else make_options()
    st = rsoc_stats()
    L = _per_round_arrays(st, per_round_cap)
    k = _chk(_lib.rsoc_color_batch(ctx.h, G, vo.ctypes.data, no.ctypes.data, _dev_ptr(d_row_ptr_cat),
                                   _dev_ptr(d_col_idx_cat), _dev_ptr(d_colors_cat), counts.ctypes.data,
                                   ctypes.byref(o), ctypes.byref(st), _stream_ptr(stream)), "rsoc_color_batch")
    d = stats_dict(st, L)
    d.pop("U_sizes", None)  # the batch reports |L| per round only
    return counts[:G], k, d


def rsoc_check_csr(row_ptr, col_idx, n=None, flags=RSOC_CHECK_CSR) -> int:
    rp, rpp = _host_i32(row_ptr)
    ci, cip = _host_i32(col_idx)
    n = len(rp) - 1 if n is None else int(n)
    return _lib.rsoc_check_csr(rpp, cip, n, int(flags))


class Pool:
    """Continuous-batching pool (rsoc_pool_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, max_slots: int = 256):
        h = _p()
        _chk(_lib.rsoc_pool_create(ctx.h, int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)), "rsoc_pool_create")
        self.h = h
        self.ctx = ctx
        ctx._pools.add(self)

    def admit(self, d_row_ptr, d_col_idx, n, d_colors_out, options=None) -> int:
        """Returns a slot id, or raises RsocError (code RSOC_EBUDGET when it does not fit now)."""
        o = options if options is not None else make_options()
        return _chk(_lib.rsoc_pool_admit(self.h, _dev_ptr(d_row_ptr), _dev_ptr(d_col_idx), int(n),
                                         _dev_ptr(d_colors_out), ctypes.byref(o)), "rsoc_pool_admit")

    def try_admit(self, d_row_ptr, d_col_idx, n, d_colors_out, options=None) -> int:
        o = options if options is not None else make_options()
        r = _lib.rsoc_pool_admit(self.h, _dev_ptr(d_row_ptr), _dev_ptr(d_col_idx), int(n), _dev_ptr(d_colors_out),
                                 ctypes.byref(o))
        if r < 0 and r != RSOC_EBUDGET:
            raise RsocError(r, "rsoc_pool_admit")
        return r

    def admit_recolor(self, d_row_ptr, d_col_idx, n, d_colors_inout, d_touched, options=None) -> int:
        """Recolouring after edits (d_colors_inout: the colouring before them,
        negative = none; d_touched: device int32 or None).  Returns a slot id,
        or raises RsocError (RSOC_EBUDGET when it does not fit now)."""
        o = options if options is not None else make_options()
        nt = 0 if d_touched is None else int(d_touched.numel())
        return _chk(_lib.rsoc_pool_admit_recolor(self.h, _dev_ptr(d_row_ptr), _dev_ptr(d_col_idx), int(n),
                                                 _dev_ptr(d_colors_inout), _dev_ptr(d_touched) if nt else None, nt,
                                                 ctypes.byref(o)), "rsoc_pool_admit_recolor")

    def try_admit_recolor(self, d_row_ptr, d_col_idx, n, d_colors_inout, d_touched, options=None) -> int:
        o = options if options is not None else make_options()
        nt = 0 if d_touched is None else int(d_touched.numel())
        r = _lib.rsoc_pool_admit_recolor(self.h, _dev_ptr(d_row_ptr), _dev_ptr(d_col_idx), int(n),
                                         _dev_ptr(d_colors_inout), _dev_ptr(d_touched) if nt else None, nt,
                                         ctypes.byref(o))
        if r < 0 and r != RSOC_EBUDGET:
            raise RsocError(r, "rsoc_pool_admit_recolor")
        return r

    def step(self, stream=None, cap=1024):
        buf = (ctypes.c_int32 * cap)()
        k = _chk(_lib.rsoc_pool_step(self.h, _stream_ptr(stream), buf, cap), "rsoc_pool_step")
        return [buf[i] for i in range(k)]

    def step_launch(self, stream=None):
        """Enqueues one fused round without waiting for it (rsoc_pool_step_launch)."""
        _chk(_lib.rsoc_pool_step_launch(self.h, _stream_ptr(stream)), "rsoc_pool_step_launch")

    def step_finish(self, cap=1024):
        """Waits for the launched round; returns the finished slots (rsoc_pool_step_finish)."""
        buf = (ctypes.c_int32 * cap)()
        k = _chk(_lib.rsoc_pool_step_finish(self.h, buf, cap), "rsoc_pool_step_finish")
        return [buf[i] for i in range(k)]

    def live(self) -> int:
        return _lib.rsoc_pool_live(self.h)

    def reserved_bytes(self) -> int:
        return _lib.rsoc_pool_reserved_bytes(self.h)

    def result(self, slot: int):
        st = rsoc_stats()
        k = _chk(_lib.rsoc_pool_result(self.h, int(slot), ctypes.byref(st)), "rsoc_pool_result")
        return k, stats_dict(st)

    def close(self):
        if self.h:
            _lib.rsoc_pool_destroy(self.h)
            self.h = _p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rsoc_pool_create(ctx, hbm_budget_bytes=0, max_slots=256) -> Pool:
    return Pool(ctx, hbm_budget_bytes, max_slots)
