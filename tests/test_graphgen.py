"""Input generators: exact sizes, symmetry, no self-loops or duplicates, seed reproducibility."""
import hashlib

import numpy as np
import pytest

import graphgen as gg


def _sym_simple(rp, ci):
    n = len(rp) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    ci = ci.astype(np.int64)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == len(ci)
    assert len(ci) == 0 or (ci.min() >= 0 and ci.max() < n)
    assert not np.any(src == ci), "self-loop"
    key = src * n + ci
    assert len(np.unique(key)) == len(key), "duplicate"
    rkey = ci * n + src
    assert np.array_equal(np.sort(key), np.sort(rkey)), "asymmetric"


@pytest.mark.parametrize("W,H", [(1, 1), (2, 3), (100, 100), (7, 19)])
def test_tri_grid_size(W, H):
    rp, ci = gg.tri_grid(W, H)
    assert len(rp) - 1 == W * H
    assert len(ci) == 2 * (3 * W * H - 2 * W - 2 * H + 1)
    _sym_simple(rp, ci)
    assert np.diff(rp).max() <= 6


def test_tri_grid_permuted_is_relabelling():
    rp, ci = gg.tri_grid(20, 15)
    rp2, ci2 = gg.tri_grid(20, 15, permute_seed=7)
    perm = gg.permutation(300, 7)
    r3, c3 = gg.relabel(rp, ci, perm)
    assert np.array_equal(rp2, r3) and np.array_equal(ci2, c3)
    assert sorted(perm) == list(range(300))


@pytest.mark.parametrize("S", [1, 2, 5, 12])
def test_lattice26_size(S):
    rp, ci = gg.lattice26(S)
    E = 3 * (S - 1) * S * S + 6 * (S - 1) ** 2 * S + 4 * (S - 1) ** 3
    assert len(rp) - 1 == S ** 3 and len(ci) == 2 * E
    _sym_simple(rp, ci)
    if S >= 3:
        assert np.diff(rp).max() == 26


def test_lattice26_full_size_formula():
    S = 200
    E = 3 * (S - 1) * S * S + 6 * (S - 1) ** 2 * S + 4 * (S - 1) ** 3
    assert E == 102_923_596


def test_rmat_simple_and_reproducible():
    rp, ci, info = gg.rmat(12, 16, seed=3, shuffle_seed=4, return_info=True)
    _sym_simple(rp, ci)
    rp2, ci2 = gg.rmat(12, 16, seed=3, shuffle_seed=4)
    assert hashlib.sha1(ci.tobytes()).digest() == hashlib.sha1(ci2.tobytes()).digest()
    assert np.array_equal(rp, rp2)
    assert info["self_loops_dropped"] > 0
    d = np.diff(rp)
    assert d.max() > 20 * d.mean()  # skewed degrees
    # shuffling relabels the unshuffled graph
    rp0, ci0 = gg.rmat(12, 16, seed=3)
    r3, c3 = gg.relabel(rp0, ci0, info["perm"])
    assert np.array_equal(r3, rp) and np.array_equal(c3, ci)


def test_rgg_and_batch():
    rp, ci = gg.rgg(3000, mean_degree=12, seed=5)
    _sym_simple(rp, ci)
    assert 9 < len(ci) / 3000 < 13
    b = gg.batch(24, seed=9, nmin=100, nmax=5000)
    assert len(b["vtx_off"]) == 25 and b["vtx_off"][-1] + 24 == len(b["row_ptr_cat"])
    assert b["nnz_off"][-1] == len(b["col_idx_cat"])
    for g in range(24):
        rp, ci = gg.batch_member(b, g)
        _sym_simple(rp, ci)
    b2 = gg.batch(24, seed=9, nmin=100, nmax=5000)
    assert np.array_equal(b["col_idx_cat"], b2["col_idx_cat"])
    assert set(b["kinds"]) == {0, 1}
