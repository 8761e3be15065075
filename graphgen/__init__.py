"""Seeded synthetic graph generators (inputs only; no colouring arithmetic).

Every generator returns symmetric CSR int32 arrays ``(row_ptr, col_idx)`` as
numpy arrays (``n = len(row_ptr) - 1``), with no self-loops and no duplicate
entries.  The heavy generators run in C (``graphgen.c``); tiny textbook graphs
(paths, cycles, cliques, ...) are built here in numpy for the tests.

The workloads stand in for the paper's test graphs (Section 4): simplicial
2D/3D meshes and R-MAT graphs with shuffled vertex ids.  The paper's own
matrices are not available.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32)
_lock = threading.Lock()
_lib = None

# tags used by the C side for the buffers it asks for
_TAGS = {0: "row_ptr", 1: "col_idx", 2: "vtx_off", 3: "nnz_off", 4: "perm"}


def build(force: bool = True) -> str:
    """Compile ``libgraphgen.so`` with gcc (OpenMP, strict FP for bit-identical output)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            lib = ctypes.CDLL(_LIB)
            i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
            lib.gg_tri_grid.argtypes = [i64, i64, i32, u64, _ALLOC_FN]
            lib.gg_lattice26.argtypes = [i64, i32, u64, _ALLOC_FN]
            lib.gg_rmat.argtypes = [i32, i64, f64, f64, f64, u64, i32, u64, ctypes.POINTER(i64), _ALLOC_FN]
            lib.gg_rgg.argtypes = [i64, f64, u64, _ALLOC_FN]
            lib.gg_batch.argtypes = [i64, u64, f64, f64, f64, ctypes.c_void_p, _ALLOC_FN]
            lib.gg_permutation.argtypes = [i64, u64, ctypes.c_void_p]
            lib.gg_splitmix64.argtypes = [u64]
            lib.gg_splitmix64.restype = u64
            for f in (lib.gg_tri_grid, lib.gg_lattice26, lib.gg_rmat, lib.gg_rgg, lib.gg_batch,
                      lib.gg_permutation):
                f.restype = i32
            _lib = lib
    return _lib


class _Arena:
    """Allocation callback handed to C: each request becomes a numpy array."""

    def __init__(self):
        self.arrays = {}
        self.cb = _ALLOC_FN(self._alloc)

    def _alloc(self, tag, count, elem):
        dt = {4: np.int32, 8: np.int64}[elem]
        base = np.empty(max(int(count), 1), dtype=dt)
        self.arrays[_TAGS[tag]] = base[: int(count)]
        return base.ctypes.data


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("graphgen.%s failed (code %d)" % (what, rc))


def splitmix64(x: int) -> int:
    return int(_load().gg_splitmix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def permutation(n: int, seed: int) -> np.ndarray:
    """Seeded Fisher-Yates permutation; ``perm[old] = new``."""
    out = np.empty(max(n, 1), dtype=np.int32)
    _check(_load().gg_permutation(n, seed, out.ctypes.data), "permutation")
    return out[:n]


def tri_grid(W: int, H: int | None = None, permute_seed: int | None = None):
    """W x H vertex grid with id r*W+c, edges right, down and the '\\' diagonal."""
    H = W if H is None else H
    ar = _Arena()
    _check(_load().gg_tri_grid(W, H, int(permute_seed is not None), permute_seed or 0, ar.cb), "tri_grid")
    return ar.arrays["row_ptr"], ar.arrays["col_idx"]


def lattice26(S: int, permute_seed: int | None = None):
    """S^3 lattice, id (z*S+y)*S+x, joined to all 26 stencil neighbours.

    A jittered lattice connected by the 26-neighbour stencil has the same
    adjacency whatever the jitter, so no point coordinates are generated."""
    ar = _Arena()
    _check(_load().gg_lattice26(S, int(permute_seed is not None), permute_seed or 0, ar.cb), "lattice26")
    return ar.arrays["row_ptr"], ar.arrays["col_idx"]


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1505, shuffle_seed: int | None = None, return_info: bool = False):
    """R-MAT graph, 2^scale vertices, edge_factor * 2^scale draws, symmetrised,
    self-loops and duplicates removed; ids shuffled when ``shuffle_seed`` is given."""
    ar = _Arena()
    dropped = ctypes.c_int64(0)
    _check(_load().gg_rmat(scale, edge_factor, a, b, c, seed, int(shuffle_seed is not None),
                           shuffle_seed or 0, ctypes.byref(dropped), ar.cb), "rmat")
    if return_info:
        return ar.arrays["row_ptr"], ar.arrays["col_idx"], {"self_loops_dropped": int(dropped.value),
                                                            "perm": ar.arrays.get("perm")}
    return ar.arrays["row_ptr"], ar.arrays["col_idx"]


def rgg(n: int, radius: float | None = None, mean_degree: float = 12.0, seed: int = 1505):
    """Random geometric graph: n uniform points in [0,1)^2, edge iff distance < radius
    (default radius sqrt(mean_degree / (pi n)))."""
    if radius is None:
        radius = float(np.sqrt(mean_degree / (np.pi * max(n, 1))))
    ar = _Arena()
    _check(_load().gg_rgg(n, radius, seed, ar.cb), "rgg")
    return ar.arrays["row_ptr"], ar.arrays["col_idx"]


def batch(G: int, seed: int = 1505, nmin: float = 1e3, nmax: float = 1e6, mean_degree: float = 12.0):
    """G independent graphs (triangulated grids or RGGs, sizes log-uniform in
    [nmin, nmax]) as a concatenated CSR with int64 offset tables.

    Returns dict(vtx_off, nnz_off, row_ptr_cat, col_idx_cat, kinds); graph g's
    local row_ptr (n_g + 1 entries) starts at row_ptr_cat[vtx_off[g] + g]."""
    ar = _Arena()
    kinds = np.zeros(max(G, 1), dtype=np.int32)
    _check(_load().gg_batch(G, seed, nmin, nmax, mean_degree, kinds.ctypes.data, ar.cb), "batch")
    return {"vtx_off": ar.arrays["vtx_off"], "nnz_off": ar.arrays["nnz_off"],
            "row_ptr_cat": ar.arrays["row_ptr"], "col_idx_cat": ar.arrays["col_idx"], "kinds": kinds[:G]}


def batch_member(b: dict, g: int):
    """Local CSR (row_ptr, col_idx) of graph g of a batch from :func:`batch`."""
    vo, no = b["vtx_off"], b["nnz_off"]
    n = int(vo[g + 1] - vo[g])
    s = int(vo[g]) + g
    return b["row_ptr_cat"][s: s + n + 1], b["col_idx_cat"][int(no[g]): int(no[g + 1])]


def concat(graphs):
    """Concatenate local CSR graphs into the batch layout used by :func:`batch`."""
    ns = [len(rp) - 1 for rp, _ in graphs]
    nnzs = [len(ci) for _, ci in graphs]
    vtx_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    nnz_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    vtx_off[1:] = np.cumsum(ns)
    nnz_off[1:] = np.cumsum(nnzs)
    row_ptr_cat = np.concatenate([np.asarray(rp, dtype=np.int32) for rp, _ in graphs]) if graphs else \
        np.zeros(0, np.int32)
    col_idx_cat = np.concatenate([np.asarray(ci, dtype=np.int32) for _, ci in graphs]) if graphs else \
        np.zeros(0, np.int32)
    return {"vtx_off": vtx_off, "nnz_off": nnz_off, "row_ptr_cat": row_ptr_cat, "col_idx_cat": col_idx_cat}


# ------------------------------------------------------- small textbook graphs

def from_edges(n: int, edges) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric CSR from an undirected edge list (duplicates and self-loops dropped)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if len(e):
        e = e[e[:, 0] != e[:, 1]]
        both = np.concatenate([e, e[:, ::-1]])
        both = np.unique(both, axis=0)
    else:
        both = np.zeros((0, 2), np.int64)
    deg = np.bincount(both[:, 0], minlength=n) if len(both) else np.zeros(n, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(deg)
    col_idx = both[:, 1].astype(np.int32)  # np.unique sorts by (src, dst)
    return row_ptr, col_idx


def path(n):
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def cycle(n):
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)] if n >= 3 else [])


def complete(n):
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def star(leaves, centre_first=True):
    """Star with ``leaves`` leaves; the centre is vertex 0 (or the last id)."""
    n = leaves + 1
    c = 0 if centre_first else n - 1
    return from_edges(n, [(c, v) for v in range(n) if v != c])


def grid4(W, H):
    """4-neighbour W x H grid, id r*W+c."""
    e = [(r * W + c, r * W + c + 1) for r in range(H) for c in range(W - 1)]
    e += [(r * W + c, (r + 1) * W + c) for r in range(H - 1) for c in range(W)]
    return from_edges(W * H, e)


def complete_bipartite(m, k):
    """K_{m,k}: side A = ids 0..m-1, side B = ids m..m+k-1."""
    return from_edges(m + k, [(i, m + j) for i in range(m) for j in range(k)])


def random_gnp(n, p, seed):
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(len(iu[0])) < p
    return from_edges(n, zip(iu[0][keep], iu[1][keep]))


def relabel(row_ptr, col_idx, perm):
    """Relabel vertex v as perm[v] (rows re-sorted)."""
    n = len(row_ptr) - 1
    perm = np.asarray(perm, dtype=np.int64)
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    return from_edges(n, zip(perm[src], perm[np.asarray(col_idx, dtype=np.int64)]))
