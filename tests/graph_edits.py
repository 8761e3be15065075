"""Edits of a symmetric CSR graph for the recolouring tests (seeded, CPU)."""
import numpy as np


def _edges(rp, ci):
    src = np.repeat(np.arange(len(rp) - 1, dtype=np.int64), np.diff(rp))
    keep = src < ci
    return np.stack([src[keep], ci[keep].astype(np.int64)], axis=1)


def csr_from_edges(n, e):
    a = np.concatenate([e[:, 0], e[:, 1]])
    b = np.concatenate([e[:, 1], e[:, 0]])
    order = np.lexsort((b, a))
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum(np.bincount(a, minlength=n))
    return rp, b[order].astype(np.int32)


def edit(rp, ci, seed, add=50, delete=50, new=5):
    """The graph after random edits: `delete` edges removed, `new` vertices
    appended (each joined to two old ones), `add` edges inserted.  Returns the
    edited CSR and the touched vertices (endpoints of inserted edges)."""
    rng = np.random.default_rng(seed)
    n = len(rp) - 1
    e = _edges(rp, ci)
    if delete and len(e):
        e = np.delete(e, rng.choice(len(e), size=min(delete, len(e)), replace=False), axis=0)
    n2 = n + new
    ins = [(int(v), int(u)) for v in range(n, n2) for u in rng.integers(0, n, size=2)]
    ins += [(int(a), int(b)) for a, b in rng.integers(0, n2, size=(add, 2)) if a != b]
    ins = np.array(sorted({(min(a, b), max(a, b)) for a, b in ins}), np.int64).reshape(-1, 2)
    key = lambda x: x[:, 0] * n2 + x[:, 1]
    ins = ins[~np.isin(key(ins), key(e))]
    rp2, ci2 = csr_from_edges(n2, np.concatenate([e, ins]))
    return rp2, ci2, np.unique(ins.ravel()).astype(np.int32)
