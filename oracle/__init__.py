"""CPU oracle for speculative First-Fit colouring -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product (``paper_1505_04086_amd``) never does, and
this package imports nothing from it: the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, compiled with gcc); this file
only marshals numpy arrays.  Functions:

* :func:`seq_ff` -- sequential First-Fit in natural id order (Section 2.1,
  Algorithm 1).
* :func:`rsync`  -- Algorithm 3 (Section 3) as a deterministic
  round-synchronous schedule: every read in a round sees the colours of the
  previous barrier; ties go to the lower id by default.
* :func:`cat`    -- Algorithm 2 (Section 2.2) under the same reading.
* :func:`check`  -- validity and the First-Fit bound c(v) <= deg(v).
* :func:`omp_rsoc` -- Algorithm 3 as the paper runs it, on the host's cores
  with OpenMP (``omp_rsoc.c``): live reads, thread-local parts of L.  A CPU
  baseline, not a reference value: its result depends on the interleaving,
  except with one thread, where it equals seq_ff.

Parity status: seq_ff, rsync (both tie rules) and check are pinned by the
``-m "not gpu"`` tests (closed forms, hand-derived worked examples, networkx's
independent greedy colouring, brute-force chromatic numbers, reversal
symmetry and monotonicity of |L|).  cat is pinned by hand-derived examples and
invariants only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

TIE_LOWER_KEEPS = 0
TIE_HIGHER_KEEPS = 1
TIE_NONE = 2
_TIES = {"lower": 0, "higher": 1, "none": 2, 0: 0, 1: 1, 2: 2}

ENOCONV = -7


_OMP_SRC = os.path.join(_HERE, "omp_rsoc.c")
_OMP_LIB = os.path.join(_HERE, "libomprsoc.so")
_omp = None


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile ``oracle.c`` (or another copy of it) into a shared library; the
    default build also compiles the OpenMP baseline ``omp_rsoc.c``."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src], check=True)
        os.replace(tmp, out)
    if src == _SRC and (force or not os.path.exists(_OMP_LIB)):
        tmp = _OMP_LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _OMP_SRC], check=True)
        os.replace(tmp, _OMP_LIB)
    return out


class OracleLib:
    """ctypes view of one compiled copy of ``oracle.c`` (the default build, or a
    test-built variant)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        p = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.orc_seq_ff.argtypes = [i32, p, p, p]
        lib.orc_seq_ff.restype = i32
        for f in (lib.orc_rsync, lib.orc_cat):
            f.argtypes = [i32, p, p, i32, i32, p, ctypes.POINTER(i32), ctypes.POINTER(i64), p, i32]
            f.restype = i32
        lib.orc_check.argtypes = [i32, p, p, p]
        lib.orc_check.restype = i64
        lib.orc_classes.argtypes = [i32, p, i32, p, p]
        lib.orc_classes.restype = i32
        lib.orc_recolor.argtypes = [i32, p, p, i32, i32, p, p, i32, ctypes.POINTER(i32), ctypes.POINTER(i64), p, i32]
        lib.orc_recolor.restype = i32
        lib.orc_square.argtypes = [i32, p, p, p, p, i64]
        lib.orc_square.restype = i64
        self.lib = lib
        self.path = path

    def seq_ff(self, row_ptr, col_idx):
        """Sequential First-Fit (Algorithm 1).  Returns (colors int32[n], K)."""
        rp, ci, n = _csr(row_ptr, col_idx)
        col = np.empty(max(n, 1), dtype=np.int32)
        k = self.lib.orc_seq_ff(n, rp.ctypes.data, ci.ctypes.data, col.ctypes.data)
        if k < 0:
            raise RuntimeError("orc_seq_ff failed: %d" % k)
        return col[:n], int(k)

    def _iterated(self, fn, row_ptr, col_idx, tie, max_rounds, raise_on_noconv):
        rp, ci, n = _csr(row_ptr, col_idx)
        col = np.empty(max(n, 1), dtype=np.int32)
        cap = n + 2
        Ls = np.zeros(cap, dtype=np.int32)
        rounds = ctypes.c_int32(0)
        conflicts = ctypes.c_int64(0)
        k = fn(n, rp.ctypes.data, ci.ctypes.data, _TIES[tie], int(max_rounds or 0), col.ctypes.data,
               ctypes.byref(rounds), ctypes.byref(conflicts), Ls.ctypes.data, cap)
        if k < 0 and (k != ENOCONV or raise_on_noconv):
            raise RuntimeError("oracle failed: %d" % k)
        R = int(rounds.value)
        return {"colors": col[:n], "K": int(k), "rounds": R, "conflicts": int(conflicts.value),
                "L_sizes": Ls[:min(R, cap)].copy(), "status": 0 if k >= 0 else int(k)}

    def rsync(self, row_ptr, col_idx, tie="lower", max_rounds=None, raise_on_noconv=True):
        """Deterministic round-synchronous Algorithm 3.

        Returns dict(colors, K, rounds = recolouring rounds R, conflicts = sum |L|,
        L_sizes = |L| per recolouring round, status)."""
        return self._iterated(self.lib.orc_rsync, row_ptr, col_idx, tie, max_rounds, raise_on_noconv)

    def cat(self, row_ptr, col_idx, tie="lower", max_rounds=None, raise_on_noconv=True):
        """Deterministic round-synchronous Algorithm 2 (tentative colouring, barrier,
        conflict detection, barrier).  rounds = Phase-1 passes; L_sizes = |L| per round."""
        return self._iterated(self.lib.orc_cat, row_ptr, col_idx, tie, max_rounds, raise_on_noconv)

    def check(self, row_ptr, col_idx, colors) -> int:
        """0 iff no edge joins equal colours and 0 <= c(v) <= deg(v) for all v."""
        rp, ci, n = _csr(row_ptr, col_idx)
        c = np.ascontiguousarray(colors, dtype=np.int32)
        if n == 0:
            return 0
        return int(self.lib.orc_check(n, rp.ctypes.data, ci.ctypes.data, c.ctypes.data))


    def recolor(self, row_ptr, col_idx, prev_colors, touched, tie="lower", max_rounds=None, raise_on_noconv=True):
        """Recolouring after topology edits: Algorithm 3 (snapshot reading)
        from the previous colouring with U^0 = touched vertices plus those
        whose colour is negative or above their degree.  Returns the dict of
        rsync (colors, K, rounds, conflicts, L_sizes, status)."""
        rp, ci, n = _csr(row_ptr, col_idx)
        col = np.empty(max(n, 1), dtype=np.int32)
        col[:n] = np.asarray(prev_colors, dtype=np.int32)[:n]
        t = np.ascontiguousarray(touched, dtype=np.int32)
        if len(t) == 0:
            t = np.zeros(1, dtype=np.int32)
            nt = 0
        else:
            nt = len(t)
        cap = n + 2
        Ls = np.zeros(cap, dtype=np.int32)
        rounds = ctypes.c_int32(0)
        conflicts = ctypes.c_int64(0)
        k = self.lib.orc_recolor(n, rp.ctypes.data, ci.ctypes.data, _TIES[tie], int(max_rounds or 0), col.ctypes.data,
                                 t.ctypes.data, nt, ctypes.byref(rounds), ctypes.byref(conflicts), Ls.ctypes.data, cap)
        if k == -1:
            raise ValueError("orc_recolor: bad argument (touched id outside [0, n)?)")
        if k < 0 and (k != ENOCONV or raise_on_noconv):
            raise RuntimeError("oracle failed: %d" % k)
        R = int(rounds.value)
        return {"colors": col[:n], "K": int(k), "rounds": R, "conflicts": int(conflicts.value),
                "L_sizes": Ls[:min(R, cap)].copy(), "status": 0 if k >= 0 else int(k)}

    def square(self, row_ptr, col_idx):
        """G^2 as CSR (row_ptr int64[n+1], col_idx int32, rows ascending,
        no self-loops, no repeats)."""
        rp, ci, n = _csr(row_ptr, col_idx)
        out_rp = np.zeros(n + 1, dtype=np.int64)
        nnz = self.lib.orc_square(n, rp.ctypes.data, ci.ctypes.data, out_rp.ctypes.data, None, 0)
        if nnz < 0:
            raise RuntimeError("orc_square failed: %d" % nnz)
        out_ci = np.empty(max(nnz, 1), dtype=np.int32)
        r = self.lib.orc_square(n, rp.ctypes.data, ci.ctypes.data, out_rp.ctypes.data, out_ci.ctypes.data, nnz)
        if r != nnz:
            raise RuntimeError("orc_square failed: %d" % r)
        return out_rp, out_ci[:nnz]

    def classes(self, colors, K=None):
        """Colour classes: (ptr int32[K+1], vtx int32[n]); class k is
        vtx[ptr[k]:ptr[k+1]], ascending ids.  K defaults to max + 1."""
        c = np.ascontiguousarray(colors, dtype=np.int32)
        n = len(c)
        if K is None:
            K = int(c.max()) + 1 if n else 0
        ptr = np.zeros(K + 1, dtype=np.int32)
        vtx = np.empty(max(n, 1), dtype=np.int32)
        r = self.lib.orc_classes(n, c.ctypes.data if n else None, int(K), ptr.ctypes.data, vtx.ctypes.data)
        if r < 0:
            raise ValueError("orc_classes: colour outside [0, K)")
        return ptr, vtx[:n]


def _csr(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if len(ci) == 0:
        ci = np.zeros(1, dtype=np.int32)
    return rp, ci, len(rp) - 1


def default() -> OracleLib:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            _lib = OracleLib(_LIB)
    return _lib


def seq_ff(row_ptr, col_idx):
    return default().seq_ff(row_ptr, col_idx)


def rsync(row_ptr, col_idx, tie="lower", max_rounds=None, raise_on_noconv=True):
    return default().rsync(row_ptr, col_idx, tie, max_rounds, raise_on_noconv)


def cat(row_ptr, col_idx, tie="lower", max_rounds=None, raise_on_noconv=True):
    return default().cat(row_ptr, col_idx, tie, max_rounds, raise_on_noconv)


def check(row_ptr, col_idx, colors) -> int:
    return default().check(row_ptr, col_idx, colors)


def classes(colors, K=None):
    return default().classes(colors, K)


def square(row_ptr, col_idx):
    return default().square(row_ptr, col_idx)


def seq_ff_d2(row_ptr, col_idx):
    """Distance-2 colouring by Algorithm 1: First-Fit on G^2."""
    rp2, ci2 = square(row_ptr, col_idx)
    return seq_ff(rp2.astype(np.int32), ci2)


def rsync_d2(row_ptr, col_idx, tie="lower", max_rounds=None, raise_on_noconv=True):
    """Distance-2 colouring by Algorithm 3 (snapshot reading) on G^2."""
    rp2, ci2 = square(row_ptr, col_idx)
    return rsync(rp2.astype(np.int32), ci2, tie, max_rounds, raise_on_noconv)


def recolor(row_ptr, col_idx, prev_colors, touched, tie="lower", max_rounds=None, raise_on_noconv=True):
    return default().recolor(row_ptr, col_idx, prev_colors, touched, tie, max_rounds, raise_on_noconv)


def omp_rsoc(row_ptr, col_idx, tie="lower", threads=None, max_rounds=None):
    """Algorithm 3 with OpenMP on `threads` host threads (default: the
    OpenMP default).  Returns dict(colors, K, rounds, conflicts, threads)."""
    global _omp
    with _lock:
        if _omp is None:
            if not os.path.exists(_OMP_LIB) or os.path.getmtime(_OMP_LIB) < os.path.getmtime(_OMP_SRC):
                build(force=True)
            lib = ctypes.CDLL(_OMP_LIB)
            p = ctypes.c_void_p
            lib.omp_rsoc.argtypes = [ctypes.c_int32, p, p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, p,
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
            lib.omp_rsoc.restype = ctypes.c_int32
            lib.omp_get_max_threads.restype = ctypes.c_int
            _omp = lib
    rp, ci, n = _csr(row_ptr, col_idx)
    th = int(threads) if threads else int(_omp.omp_get_max_threads())
    col = np.empty(max(n, 1), dtype=np.int32)
    rounds = ctypes.c_int32(0)
    conflicts = ctypes.c_int64(0)
    k = _omp.omp_rsoc(n, rp.ctypes.data, ci.ctypes.data, _TIES[tie], th, int(max_rounds or 0), col.ctypes.data,
                      ctypes.byref(rounds), ctypes.byref(conflicts))
    if k < 0:
        raise RuntimeError("omp_rsoc failed: %d" % k)
    return {"colors": col[:n], "K": int(k), "rounds": int(rounds.value), "conflicts": int(conflicts.value),
            "threads": th}


def colour_count(colors) -> int:
    """K = max + 1 (0 for no vertices)."""
    return int(colors.max()) + 1 if len(colors) else 0
