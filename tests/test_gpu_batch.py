"""Batched colouring on the GPU: every graph of a batch must come out exactly as
the oracle colours it alone (round-synchronous modes: element by element;
optimistic mode: valid with 0 <= c(v) <= deg(v)), and exactly as a separate
single-graph call colours it."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _mixed_batch():
    graphs = [gg.path(7), gg.cycle(5), (np.zeros(1, np.int32), np.zeros(0, np.int32)), gg.complete(40),
              gg.star(300), gg.tri_grid(30, 17), gg.tri_grid(25, 25, permute_seed=3), gg.rmat(9, 8, seed=4, shuffle_seed=5),
              (np.zeros(4, np.int32), np.zeros(0, np.int32)), gg.rgg(2500, seed=6), gg.complete_bipartite(20, 70)]
    b = gg.batch(20, seed=77, nmin=50, nmax=4000)
    graphs += [gg.batch_member(b, g) for g in range(20)]
    return graphs


GRAPHS = _mixed_batch()
BATCH = gg.concat(GRAPHS)
# "default" sends the graphs of at most 2048 vertices to the workgroup-resident
# path (one workgroup per graph, every round inside it); the launch splits of
# the fused launches run with that path off, and "small64" divides the batch
SPLITS = {"default": {}, "allbins": {"t_thread": 3, "t_wave": 8, "small_cutoff": -1},
          "runs1": {"chunk": 1, "grid_thread": 7, "grid_list": 2, "small_cutoff": -1},
          "runs8": {"chunk": 8, "grid_thread": 3, "small_cutoff": -1}, "small64": {"small_cutoff": 64},
          # optimistic round 0's task bands: one per XCD; 128 bands over a grid
          # of 5 workgroups (most bands start with no workgroup of their own)
          "bands1": {"bands": 1, "small_cutoff": -1}, "bands16": {"bands": 16, "grid_thread": 5, "small_cutoff": -1}}


def _n_small(opts):
    cut = {-1: 0, 0: 2048}.get(opts.get("small_cutoff", 0), opts.get("small_cutoff", 0))
    return sum(1 for rp, _ in GRAPHS if 0 < len(rp) - 1 <= cut)


def _upload(lib, b):
    import torch
    d = torch.device("cuda:0")
    rp = torch.from_numpy(b["row_ptr_cat"]).to(d)
    ci = torch.from_numpy(b["col_idx_cat"] if len(b["col_idx_cat"]) else np.zeros(1, np.int32)).to(d)
    col = torch.full((max(int(b["vtx_off"][-1]), 1),), -5, dtype=torch.int32, device=d)
    return rp, ci, col


def _member_colours(col, b, g):
    return col[int(b["vtx_off"][g]): int(b["vtx_off"][g + 1])]


@pytest.mark.parametrize("split", sorted(SPLITS))
@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("mode", ["deterministic", "two_phase"])
def test_batch_round_synchronous_matches_oracle(lib, ctx, mode, tie, split):
    rp, ci, col = _upload(lib, BATCH)
    counts, kmax, st = lib.rsoc_color_batch(ctx, BATCH["vtx_off"], BATCH["nnz_off"], rp, ci, col,
                                            lib.make_options(mode, tie, **SPLITS[split]), per_round_cap=4096)
    got = col.cpu().numpy()
    fn = oracle.rsync if mode == "deterministic" else oracle.cat
    L_total = np.zeros(4096, np.int64)
    conflicts = rounds = 0
    for g, (grp, gci) in enumerate(GRAPHS):
        want = fn(grp, gci, tie=tie)
        assert np.array_equal(_member_colours(got, BATCH, g), want["colors"]), (mode, tie, g)
        assert counts[g] == want["K"], g
        L_total[:len(want["L_sizes"])] += want["L_sizes"]
        conflicts += want["conflicts"]
        rounds = max(rounds, want["rounds"])
    assert kmax == max(counts)
    assert st["small_graphs"] == (_n_small(SPLITS[split]) if mode == "deterministic" else 0)
    # the per-round |L| of the batch is the graphs' summed round by round,
    # whichever path coloured them
    if mode == "deterministic":
        assert st["rounds"] == rounds and st["conflicts"] == conflicts
        assert np.array_equal(st["L_sizes"], L_total[:rounds])


@pytest.mark.parametrize("split", sorted(SPLITS))
@pytest.mark.parametrize("full_sweep", [0, 1])
@pytest.mark.parametrize("tie", ["lower", "higher"])
def test_batch_optimistic_valid(lib, ctx, tie, full_sweep, split):
    rp, ci, col = _upload(lib, BATCH)
    counts, kmax, st = lib.rsoc_color_batch(ctx, BATCH["vtx_off"], BATCH["nnz_off"], rp, ci, col,
                                            lib.make_options("optimistic", tie, full_sweep=full_sweep,
                                                             **SPLITS[split]))
    got = col.cpu().numpy()
    for g, (grp, gci) in enumerate(GRAPHS):
        c = _member_colours(got, BATCH, g)
        assert oracle.check(grp, gci, c) == 0, g
        assert counts[g] == oracle.colour_count(c)
    assert st["small_graphs"] == _n_small(SPLITS[split])
    # the run length: the option's, or 0 when each graph's is chosen on the device
    assert st["chunk"] == SPLITS[split].get("chunk", 0)
    if not full_sweep:
        # round 1 inspects every vertex of U^0 (its thread-bin part walked from
        # round 0's per-task masks), and U^0 only holds vertices of the fused
        # launches' graphs
        n_fused = sum(len(grp) - 1 for grp, _ in GRAPHS) - sum(
            len(grp) - 1 for grp, _ in GRAPHS if 0 < len(grp) - 1 <= {-1: 0, 0: 2048}.get(
                SPLITS[split].get("small_cutoff", 0), SPLITS[split].get("small_cutoff", 0)))
        assert 0 <= st["worklist0"] <= n_fused
        if st["worklist0"]:
            assert st["inspected"] >= st["worklist0"]


def test_batch_equals_single_calls(lib, ctx):
    """Deterministic: each graph's colours in the batch equal a separate call's."""
    import torch
    rp, ci, col = _upload(lib, BATCH)
    lib.rsoc_color_batch(ctx, BATCH["vtx_off"], BATCH["nnz_off"], rp, ci, col, lib.make_options("deterministic"))
    got = col.cpu().numpy()
    d = torch.device("cuda:0")
    for g, (grp, gci) in enumerate(GRAPHS):
        n = len(grp) - 1
        if n == 0:
            continue
        d_rp = torch.from_numpy(grp).to(d)
        d_ci = torch.from_numpy(gci if len(gci) else np.zeros(1, np.int32)).to(d)
        d_col = torch.empty(n, dtype=torch.int32, device=d)
        lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("deterministic"))
        assert np.array_equal(d_col.cpu().numpy(), _member_colours(got, BATCH, g)), g


def test_batch_validation_and_empty(lib, ctx):
    import torch
    d = torch.device("cuda:0")
    z = torch.zeros(1, dtype=torch.int32, device=d)
    counts, k, st = lib.rsoc_color_batch(ctx, np.zeros(1, np.int64), np.zeros(1, np.int64), z, z, z)
    assert k == 0 and len(counts) == 0
    b = gg.concat([gg.cycle(5), gg.path(4)])
    bad = b["col_idx_cat"].copy()
    bad[2] = 9  # out of range for graph 0
    rp = torch.from_numpy(b["row_ptr_cat"]).to(d)
    ci = torch.from_numpy(bad).to(d)
    col = torch.empty(9, dtype=torch.int32, device=d)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_batch(ctx, b["vtx_off"], b["nnz_off"], rp, ci, col, lib.make_options(validate=1))
    assert e.value.code == lib.RSOC_ECSR


@pytest.mark.parametrize("cutoff", [0, 64, -1])
def test_batch_pass_bound(lib, ctx, cutoff):
    """A pass bound below what a path needs (n - 1 rounds, round-synchronous)
    ends the batch with RSOC_ENOCONV on either path."""
    b = gg.concat([gg.path(300), gg.cycle(6)])
    rp, ci, col = _upload(lib, b)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_batch(ctx, b["vtx_off"], b["nnz_off"], rp, ci, col,
                             lib.make_options("deterministic", max_rounds=5, small_cutoff=cutoff))
    assert e.value.code == lib.RSOC_ENOCONV


def test_batch_small_graphs_only_and_option_checked(lib, ctx):
    """A batch of small graphs only (no fused launch at all), optimistic and
    round-synchronous; cutoffs beyond 2048 and band counts outside 1..16 are
    refused."""
    graphs = [gg.complete(12), gg.star(50), gg.tri_grid(20, 9, permute_seed=2), gg.rmat(8, 8, seed=3, shuffle_seed=4)]
    b = gg.concat(graphs)
    rp, ci, col = _upload(lib, b)
    for mode in ("optimistic", "deterministic"):
        counts, kmax, st = lib.rsoc_color_batch(ctx, b["vtx_off"], b["nnz_off"], rp, ci, col, lib.make_options(mode))
        assert st["small_graphs"] == len(graphs)
        got = col.cpu().numpy()
        for g, (grp, gci) in enumerate(graphs):
            c = _member_colours(got, b, g)
            if mode == "deterministic":
                assert np.array_equal(c, oracle.rsync(grp, gci)["colors"]), g
            else:
                assert oracle.check(grp, gci, c) == 0 and counts[g] == oracle.colour_count(c), g
    for bad in ({"small_cutoff": 2049}, {"bands": 17}, {"bands": -1}):
        with pytest.raises(lib.RsocError) as e:
            lib.rsoc_color_batch(ctx, b["vtx_off"], b["nnz_off"], rp, ci, col, lib.make_options(**bad))
        assert e.value.code == lib.RSOC_EINVAL, bad
