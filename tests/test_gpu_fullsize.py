"""Parity at the benchmark's full sizes: the 200^3 26-stencil lattice with
permuted ids (8 M vertices, 103 M edges) and R-MAT scale 22 with shuffled ids
(4.2 M vertices, 64 M edges).

Deterministic mode (Section 3, Algorithm 3 read round-synchronously, lower id
keeps) must equal the oracle's schedule: every colour, K, the recolouring
rounds, the conflicts and |L| of every round.  The oracle's results come
from tests/golden/fullsize_rsync.json, written by make_fullsize_golden.py
from oracle/ alone (a digest of the colour array, the counts, |L| per round,
and a digest of the input graph, checked first); on the lattice the oracle
also runs here (about a minute) and the colours are compared element by
element.  The optimistic mode must be valid with 0 <= c(v) <= deg(v) and is
held to its colour-count target against sequential First-Fit (Section 2.1,
Algorithm 1): within one colour on the power-law graph, within two on the
scrambled lattice.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = json.load(open(os.path.join(HERE, "golden", "fullsize_rsync.json")))
CONFIGS = {
    "lattice26_200_perm": (lambda: gg.lattice26(200, permute_seed=1505), 2, True),
    "rmat22_shuffled": (lambda: gg.rmat(22, 16, 0.57, 0.19, 0.19, seed=1505, shuffle_seed=1506), 1, False),
}


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("cfg", sorted(CONFIGS))
def test_full_size(lib, ctx, cfg):
    import torch
    gen, allow, live = CONFIGS[cfg]
    g = GOLDEN[cfg]
    print("case", cfg, "generating", flush=True)
    rp, ci = gen()
    assert sha(rp) == g["row_ptr_sha256"] and sha(ci) == g["col_idx_sha256"], "input graph differs from the golden's"
    n = len(rp) - 1
    d = torch.device("cuda:0")
    d_rp, d_ci = torch.from_numpy(rp).to(d), torch.from_numpy(ci).to(d)
    d_col = torch.full((n,), -5, dtype=torch.int32, device=d)
    print("case", cfg, "deterministic on the GPU", flush=True)
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("deterministic", "lower"),
                                  per_round_cap=4096)
    got = d_col.cpu().numpy()
    want = g["rsync_lower"]
    assert k == want["K"] and st["rounds"] == want["rounds"] and st["conflicts"] == want["conflicts"]
    assert [int(x) for x in st["L_sizes"]] == want["L_sizes"]
    assert sha(got) == want["colors_sha256"]
    if live:
        print("case", cfg, "oracle", flush=True)
        r = oracle.rsync(rp, ci, tie="lower")
        assert np.array_equal(got, r["colors"]) and r["K"] == k and r["rounds"] == st["rounds"]
    print("case", cfg, "optimistic on the GPU", flush=True)
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("optimistic", "lower"))
    got = d_col.cpu().numpy()
    assert oracle.check(rp, ci, got) == 0 and k == got.max() + 1
    kseq = g["seq_ff_K"]
    assert k <= kseq + allow, "optimistic %d colours, sequential First-Fit %d" % (k, kseq)
