"""Workgroup append queues under pressure, on graphs of about 10^4 vertices.

Binning, the sweeps, the worklist rounds and the list set-up of a recolouring
append into per-workgroup queues in LDS and flush them to the global lists
when they fill.  With the default launch shapes a graph of this size gives
every workgroup one short walk, so no queue fills before the walk ends.  The
launch-shape options below shrink those grids to one workgroup (`grid_bin`,
`grid_thread`, `grid_list`), so that each queue fills and flushes many times
in the middle of its walk; the results must still equal the oracle element by
element (Section 3, Algorithm 3: every recoloured vertex joins L, every vertex
of a degree range joins its bin), and the library's own count checks
(RSOC_EINTERNAL) must stay silent.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.graph_edits import edit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _dev(rp, ci, fill=-5):
    import torch
    d = torch.device("cuda:0")
    n = len(rp) - 1
    return (torch.from_numpy(np.ascontiguousarray(rp)).to(d),
            torch.from_numpy(np.ascontiguousarray(ci) if len(ci) else np.zeros(1, np.int32)).to(d),
            torch.full((max(n, 1),), fill, dtype=torch.int32, device=d), n)


GRAPHS = {
    "tri_grid_100": lambda: gg.tri_grid(100),
    "tri_grid_100_perm": lambda: gg.tri_grid(100, permute_seed=1505),
    "rgg_10k": lambda: gg.rgg(10000, seed=21),
    "rmat_13": lambda: gg.rmat(13, 8, seed=22, shuffle_seed=23),
    "gnp_10k": lambda: gg.random_gnp(10000, 0.0025, 24),
}
_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


# one workgroup per launch where queues are used: the thread-bin queue of the
# sweeps and worklist rounds (default bins), and the hub queues of binning
# (small bin thresholds put most rows into the wavefront and workgroup bins)
SHAPES = {
    "one_wg": {"grid_bin": 1, "grid_thread": 1, "grid_list": 1},
    "one_wg_hubs": {"grid_bin": 1, "grid_thread": 1, "grid_list": 1, "grid_wave": 1, "t_thread": 3, "t_wave": 8},
    "two_wg_runs8": {"grid_bin": 2, "grid_thread": 2, "grid_list": 2, "chunk": 8},
}


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_deterministic_flushes_match_oracle(lib, ctx, name, tie, shape):
    rp, ci = graph(name)
    print("case", name, tie, shape, flush=True)
    want = oracle.rsync(rp, ci, tie=tie)
    d_rp, d_ci, d_col, n = _dev(rp, ci)
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("deterministic", tie, **SHAPES[shape]),
                                  per_round_cap=n + 2)
    assert np.array_equal(d_col.cpu().numpy()[:n], want["colors"])
    assert k == want["K"] and st["rounds"] == want["rounds"] and st["conflicts"] == want["conflicts"]
    assert list(st["L_sizes"]) == list(want["L_sizes"])
    # the bins hold every row of their degree range once
    deg = np.diff(rp)
    o = SHAPES[shape]
    tt, tw = o.get("t_thread", 32), o.get("t_wave", 2048)
    assert st["bin_counts"] == [int((deg <= tt).sum()), int(((deg > tt) & (deg <= tw)).sum()), int((deg > tw).sum())]


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_two_phase_flushes_match_oracle(lib, ctx, name, shape):
    rp, ci = graph(name)
    print("case", name, shape, flush=True)
    want = oracle.cat(rp, ci)
    d_rp, d_ci, d_col, n = _dev(rp, ci)
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("two_phase", **SHAPES[shape]),
                                  per_round_cap=n + 2)
    assert np.array_equal(d_col.cpu().numpy()[:n], want["colors"])
    assert list(st["L_sizes"]) == list(want["L_sizes"])


@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_optimistic_flushes_valid(lib, ctx, name, tie, shape):
    rp, ci = graph(name)
    print("case", name, tie, shape, flush=True)
    d_rp, d_ci, d_col, n = _dev(rp, ci)
    for full in (0, 1):
        k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col,
                                      lib.make_options("optimistic", tie, full_sweep=full, **SHAPES[shape]))
        got = d_col.cpu().numpy()[:n]
        assert oracle.check(rp, ci, got) == 0, full
        assert k == oracle.colour_count(got) and st["colors_distinct"] == len(np.unique(got))


@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("name", ["tri_grid_100_perm", "rgg_10k"])
def test_recolour_list_setup_flushes(lib, ctx, name, tie):
    """Every vertex of the edited graph touched: the recolouring's list set-up
    appends all of them through one workgroup's three queues."""
    import torch
    rp, ci = graph(name)
    prev = oracle.seq_ff(rp, ci)[0]
    rp2, ci2, _ = edit(rp, ci, seed=31, add=300, delete=300, new=20)
    n2 = len(rp2) - 1
    prev2 = np.full(n2, -1, np.int32)
    prev2[:len(prev)] = prev
    touched = np.arange(n2, dtype=np.int32)
    want = oracle.recolor(rp2, ci2, prev2, touched, tie=tie)
    for shape in ({"grid_bin": 1, "grid_list": 1}, {"grid_bin": 1, "grid_list": 1, "t_thread": 3, "t_wave": 8}):
        d_rp, d_ci, _, n = _dev(rp2, ci2)
        d_col = torch.from_numpy(prev2.copy()).to(d_rp.device)
        d_t = torch.from_numpy(touched).to(d_rp.device)
        k, st = lib.rsoc_recolor_device(ctx, d_rp, d_ci, n, d_col, d_t,
                                        lib.make_options("deterministic", tie, **shape), per_round_cap=n + 2)
        assert np.array_equal(d_col.cpu().numpy(), want["colors"]), shape
        assert k == want["K"] and list(st["L_sizes"]) == list(want["L_sizes"])


@pytest.mark.parametrize("mode", ["deterministic", "two_phase"])
def test_batch_flushes_match_oracle(lib, ctx, mode):
    graphs = [graph("tri_grid_100"), graph("rgg_10k"), gg.path(3000), graph("rmat_13")]
    b = gg.concat(graphs)
    import torch
    d = torch.device("cuda:0")
    rp = torch.from_numpy(b["row_ptr_cat"]).to(d)
    ci = torch.from_numpy(b["col_idx_cat"]).to(d)
    fn = oracle.rsync if mode == "deterministic" else oracle.cat
    wants = [fn(grp, gci) for grp, gci in graphs]
    for shape in ({"grid_bin": 1, "grid_thread": 1, "grid_list": 1},
                  {"grid_bin": 1, "grid_thread": 1, "grid_list": 1, "t_thread": 3, "t_wave": 8}):
        col = torch.full((int(b["vtx_off"][-1]),), -5, dtype=torch.int32, device=d)
        counts, kmax, st = lib.rsoc_color_batch(ctx, b["vtx_off"], b["nnz_off"], rp, ci, col,
                                                lib.make_options(mode, **shape))
        got = col.cpu().numpy()
        for g, want in enumerate(wants):
            lo, hi = int(b["vtx_off"][g]), int(b["vtx_off"][g + 1])
            assert np.array_equal(got[lo:hi], want["colors"]), (shape, g)
            assert counts[g] == want["K"]


def test_pool_flushes_match_oracle(lib, ctx):
    """Pool admission bins (and, for recolouring slots, lists) with one
    workgroup per slot; deterministic slots equal the oracle."""
    import torch
    names = ["tri_grid_100_perm", "rgg_10k", "rmat_13"]
    pool = lib.Pool(ctx, 0, 16)
    live = {}
    for name in names:
        for shape in ({"grid_bin": 1}, {"grid_bin": 1, "t_thread": 3, "t_wave": 8}):
            rp, ci = graph(name)
            d_rp, d_ci, d_col, n = _dev(rp, ci)
            slot = pool.admit(d_rp, d_ci, n, d_col, lib.make_options("deterministic", **shape))
            live[slot] = ("colour", name, d_rp, d_ci, d_col, None)
    rp, ci = graph("rgg_10k")
    prev = oracle.seq_ff(rp, ci)[0]
    rp2, ci2, _ = edit(rp, ci, seed=41, add=200, delete=200, new=10)
    n2 = len(rp2) - 1
    prev2 = np.full(n2, -1, np.int32)
    prev2[:len(prev)] = prev
    touched = np.arange(n2, dtype=np.int32)
    d_rp, d_ci, _, _ = _dev(rp2, ci2)
    d_col = torch.from_numpy(prev2.copy()).to(d_rp.device)
    d_t = torch.from_numpy(touched).to(d_rp.device)
    slot = pool.admit_recolor(d_rp, d_ci, n2, d_col, d_t, lib.make_options("deterministic", grid_bin=1))
    live[slot] = ("recolour", None, d_rp, d_ci, d_col, d_t)
    steps = 0
    while live:
        for s in pool.step():
            kind, name, _, _, d_col, _ = live.pop(s)
            k, st = pool.result(s)
            got = d_col.cpu().numpy()
            if kind == "colour":
                want = oracle.rsync(*graph(name))
            else:
                want = oracle.recolor(rp2, ci2, prev2, touched)
            assert np.array_equal(got[:len(want["colors"])], want["colors"]) and k == want["K"], (kind, name)
        steps += 1
        assert steps < 20000
    pool.close()
