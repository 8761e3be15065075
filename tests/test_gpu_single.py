"""Single-graph parity on the GPU: the HIP path (through the C ABI) against the
CPU oracle on the same seeded inputs.

Deterministic mode must equal the oracle's round-synchronous Algorithm 3
element by element (colours, recolouring rounds, |L| per round); two-phase
mode must equal the oracle's round-synchronous Algorithm 2; optimistic mode
(live reads, any interleaving) must give a valid colouring with
0 <= c(v) <= deg(v), and its colour count is reported against sequential
First-Fit.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def _dev(lib, rp, ci):
    import torch
    d = torch.device("cuda:0")
    n = len(rp) - 1
    return (torch.from_numpy(np.ascontiguousarray(rp)).to(d), torch.from_numpy(np.ascontiguousarray(ci)).to(d),
            torch.full((max(n, 1),), -5, dtype=torch.int32, device=d), n)


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _small_cases():
    cases = {
        "P2": gg.path(2), "P5": gg.path(5), "P300": gg.path(300), "C4": gg.cycle(4), "C5": gg.cycle(5),
        "C6": gg.cycle(6), "K5": gg.complete(5), "K70": gg.complete(70), "star": gg.star(200),
        "grid4": gg.grid4(23, 17), "tri_grid": gg.tri_grid(37, 29), "tri_grid_perm": gg.tri_grid(37, 29, permute_seed=5),
        "isolated": (np.zeros(8, np.int32), np.zeros(0, np.int32)), "single": (np.zeros(2, np.int32), np.zeros(0, np.int32)),
        "rmat10": gg.rmat(10, 8, seed=2, shuffle_seed=3), "rgg": gg.rgg(3000, seed=4),
        "kbip": gg.complete_bipartite(40, 90),
        # thread-bin rows whose neighbours are all coloured at the same instant:
        # round 0 keeps more than three (K30) and full 32-position masks (K33)
        "K30": gg.complete(30), "K33": gg.complete(33), "gnp_dense": gg.random_gnp(64, 0.45, 9),
    }
    rng = np.random.default_rng(1505)
    for i in range(6):
        n = int(rng.integers(2, 400))
        cases["gnp%d" % i] = gg.random_gnp(n, float(rng.uniform(0.005, 0.2)), int(rng.integers(1 << 30)))
    return cases


CASES = _small_cases()
# degree-bin thresholds small enough to route small graphs through every bin
BIN_SPLITS = {"default": {}, "allbins": {"t_thread": 3, "t_wave": 8}, "wave_only": {"t_thread": 1, "t_wave": 100000},
              "block_only": {"t_thread": 1, "t_wave": 1}, "runs1": {"chunk": 1, "grid_thread": 3, "grid_list": 3},
              "runs8": {"chunk": 8, "grid_thread": 5, "grid_list": 1}, "runs2": {"chunk": 2, "t_thread": 16},
              # optimistic ordered pass over small worklists: off, and at a
              # threshold of 4 with every degree bin in use
              "notail": {"tail": -1}, "tail4": {"tail": 4, "t_thread": 3, "t_wave": 8},
              # one workgroup per binning, sweep and worklist launch: its LDS
              # queues fill and flush in the middle of their walks
              "flush": {"grid_bin": 1, "grid_thread": 1, "grid_list": 1, "grid_wave": 1, "t_thread": 3, "t_wave": 8}}


@pytest.mark.parametrize("split", sorted(BIN_SPLITS))
@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_deterministic_matches_oracle(lib, ctx, name, tie, split):
    rp, ci = CASES[name]
    print("case", name, tie, split, flush=True)
    want = oracle.rsync(rp, ci, tie=tie)
    d_rp, d_ci, d_col, n = _dev(lib, rp, ci)
    o = lib.make_options("deterministic", tie, **BIN_SPLITS[split])
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, o, per_round_cap=n + 2)
    got = d_col.cpu().numpy()[:n]
    assert np.array_equal(got, want["colors"])
    assert k == want["K"]
    assert st["colors_distinct"] == len(np.unique(want["colors"]))
    assert st["rounds"] == want["rounds"] and st["conflicts"] == want["conflicts"]
    # round 1 sweeps V; every later pass inspects the list the pass before recoloured
    assert st["inspected"] == n + want["conflicts"]
    assert list(st["L_sizes"]) == list(want["L_sizes"])
    # |U| per pass: V, then what each round recoloured (U <- L), for every pass run
    assert st["passes"] == want["rounds"] + 1
    assert list(st["U_sizes"]) == [n] + list(want["L_sizes"])


@pytest.mark.parametrize("split", sorted(BIN_SPLITS))
@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_two_phase_matches_oracle(lib, ctx, name, tie, split):
    rp, ci = CASES[name]
    want = oracle.cat(rp, ci, tie=tie)
    d_rp, d_ci, d_col, n = _dev(lib, rp, ci)
    o = lib.make_options("two_phase", tie, **BIN_SPLITS[split])
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, o, per_round_cap=n + 2)
    got = d_col.cpu().numpy()[:n]
    assert np.array_equal(got, want["colors"])
    assert k == want["K"] and st["rounds"] == want["rounds"]
    assert list(st["L_sizes"]) == list(want["L_sizes"])


@pytest.mark.parametrize("full_sweep", [0, 1])
@pytest.mark.parametrize("split", sorted(BIN_SPLITS))
@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_optimistic_valid(lib, ctx, name, tie, split, full_sweep):
    rp, ci = CASES[name]
    d_rp, d_ci, d_col, n = _dev(lib, rp, ci)
    o = lib.make_options("optimistic", tie, full_sweep=full_sweep, **BIN_SPLITS[split])
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, o, per_round_cap=n + 2)
    got = d_col.cpu().numpy()[:n]
    assert oracle.check(rp, ci, got) == 0
    # |U| per pass: U^0, then what each round recoloured (no pass at all when
    # round 0 left nothing to inspect)
    U = list(st["U_sizes"])
    assert len(U) == st["passes"] and U[1:] == list(st["L_sizes"])[:max(len(U) - 1, 0)]
    if U:
        assert U[0] == st["worklist0"]
    assert k == oracle.colour_count(got)
    assert st["colors_distinct"] == len(np.unique(got))
    deg = np.diff(rp)
    assert k <= (deg.max() + 1 if n else 0)
    # the method's termination bound: |L| strictly shrinks, so at most n recolouring rounds
    assert st["rounds"] <= max(n, 0)


@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("name", ["K300", "rmat12", "hubcore"])
def test_ordered_tail_pass(lib, ctx, name, tie):
    """Mutually adjacent hubs: with the ordered pass over small worklists the
    colouring stays valid and the rounds stop growing with the core's size."""
    if name == "K300":
        rp, ci = gg.complete(300)
    elif name == "rmat12":
        rp, ci = gg.rmat(12, 16, seed=7, shuffle_seed=8)
    else:  # a 200-clique whose members also hold 40 leaves each
        edges = [(i, j) for i in range(200) for j in range(i + 1, 200)]
        edges += [(i, 200 + 40 * i + k) for i in range(200) for k in range(40)]
        rp, ci = gg.from_edges(200 + 200 * 40, np.array(edges, dtype=np.int64))
    d_rp, d_ci, d_col, n = _dev(lib, rp, ci)
    for tail in (0, -1):
        k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("optimistic", tie, tail=tail),
                                      per_round_cap=4096)
        got = d_col.cpu().numpy()[:n]
        assert oracle.check(rp, ci, got) == 0, tail
        assert k == oracle.colour_count(got) and k <= np.diff(rp).max() + 1
        # colours of 255 and more are counted through per-colour flags
        assert st["colors_distinct"] == len(np.unique(got))
        if name == "K300":
            assert k == 300
        if tail == 0:
            # round 1, one replay of 4 rounds, the ordered pass, the round that checks it
            assert st["rounds"] <= 7, st["L_sizes"]


def test_host_pointer_entry_points(lib, ctx):
    rp, ci = gg.tri_grid(50, 31, permute_seed=11)
    want = oracle.rsync(rp, ci)
    col, k, st = lib.rsoc_color_ex(ctx, rp, ci, options=lib.make_options("deterministic", validate=3))
    assert np.array_equal(col, want["colors"]) and k == want["K"]
    col, k = lib.rsoc_color(rp, ci)
    assert oracle.check(rp, ci, col) == 0 and k == oracle.colour_count(col)


def test_max_rounds_guard(lib, ctx):
    """P5 needs 4 recolouring passes plus a final empty one; a bound of 1 pass must
    stop with RSOC_ENOCONV and leave the state after that pass (the oracle's)."""
    rp, ci = gg.path(5)
    for m in (1, 2, 4):
        want = oracle.rsync(rp, ci, max_rounds=m, raise_on_noconv=False)
        assert want["status"] == oracle.ENOCONV
        d_rp, d_ci, d_col, n = _dev(lib, rp, ci)
        k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("deterministic", max_rounds=m),
                                      allow_noconv=True)
        assert k == lib.RSOC_ENOCONV
        assert np.array_equal(d_col.cpu().numpy()[:n], want["colors"])
    d_rp, d_ci, d_col, n = _dev(lib, rp, ci)
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("deterministic", max_rounds=5))
    assert k == 2


def test_device_validation_errors(lib, ctx):
    import torch
    rp, ci = gg.cycle(6)
    bad = ci.copy()
    bad[3] = 17  # out of range
    d_rp, d_ci, d_col, n = _dev(lib, rp, bad)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options(validate=1))
    assert e.value.code == lib.RSOC_ECSR
    loop = ci.copy()
    loop[0] = 0  # vertex 0 lists itself
    d_rp, d_ci, d_col, n = _dev(lib, rp, loop)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options(validate=1))
    assert e.value.code == lib.RSOC_ESELFLOOP
    # without validation a self-loop is ignored, exactly as in the oracle
    want = oracle.rsync(rp, loop)
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("deterministic"))
    assert np.array_equal(d_col.cpu().numpy()[:n], want["colors"])
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["optimistic", "deterministic", "two_phase"])
def test_unvalidated_input_checks(lib, ctx, mode):
    """Without validation the rounds are enqueued behind binning before the
    host sees its checks: bad row_ptr ends and edges without col_idx must
    still come back as RSOC_ECSR / RSOC_EINVAL (the sweeps return at once on
    them), and the context must colour the next graph normally."""
    rp, ci = gg.cycle(9)
    bad = rp.copy()
    bad[0] = 1
    d_rp, d_ci, d_col, n = _dev(lib, bad, ci)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options(mode))
    assert e.value.code == lib.RSOC_ECSR
    d_rp, d_ci, d_col, n = _dev(lib, rp, ci)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_device(ctx, d_rp, None, n, d_col, lib.make_options(mode))
    assert e.value.code == lib.RSOC_EINVAL
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options(mode))
    got = d_col.cpu().numpy()[:n]
    if mode == "optimistic":
        assert oracle.check(rp, ci, got) == 0 and k == oracle.colour_count(got)
    else:
        want = oracle.rsync(rp, ci) if mode == "deterministic" else oracle.cat(rp, ci)
        assert np.array_equal(got, want["colors"]) and k == want["K"]


def test_empty_graph(lib, ctx):
    import torch
    d = torch.device("cuda:0")
    z = torch.zeros(1, dtype=torch.int32, device=d)
    k, st = lib.rsoc_color_device(ctx, z, z, 0, z)
    assert k == 0


def test_config1_full(lib, ctx):
    """100 x 100 triangulated grid, natural and permuted ids, both tie rules."""
    for seed in (None, 1505):
        rp, ci = gg.tri_grid(100, permute_seed=seed)
        for tie in ("lower", "higher"):
            want = oracle.rsync(rp, ci, tie=tie)
            d_rp, d_ci, d_col, n = _dev(lib, rp, ci)
            k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("deterministic", tie),
                                          per_round_cap=1024)
            assert np.array_equal(d_col.cpu().numpy(), want["colors"]) and st["rounds"] == want["rounds"]
            assert list(st["L_sizes"]) == list(want["L_sizes"])
            k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("optimistic", tie))
            assert oracle.check(rp, ci, d_col.cpu().numpy()) == 0


@pytest.mark.parametrize("split", ["default", "allbins", "wave_only", "block_only", "runs1"])
@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_two_phase_live_valid(lib, ctx, name, tie, split):
    """Algorithm 2 with live reads (the paper's "C" as it runs beside
    Algorithm 3): any valid colouring with 0 <= c(v) <= deg(v) is correct; the
    one-sided test still lets the lowest vertex of U leave it in every round,
    so at most n rounds; every round recolours all of U, so its |L| is the
    next round's |U|."""
    rp, ci = CASES[name]
    d_rp, d_ci, d_col, n = _dev(lib, rp, ci)
    o = lib.make_options("two_phase_live", tie, **BIN_SPLITS[split])
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, o, per_round_cap=n + 2)
    got = d_col.cpu().numpy()[:n]
    assert oracle.check(rp, ci, got) == 0
    assert k == oracle.colour_count(got) and st["colors_distinct"] == len(np.unique(got))
    deg = np.diff(rp)
    assert k <= (deg.max() + 1 if n else 0)
    assert st["rounds"] <= max(n, 1)


def test_two_phase_live_single_graph_only(lib, ctx):
    """The live two-phase mode is refused where only Algorithm 3 runs (the
    pool, the recolouring) and by the batch."""
    import torch
    rp, ci = gg.tri_grid(20, 20)
    d_rp, d_ci, d_col, n = _dev(lib, rp, ci)
    o = lib.make_options("two_phase_live")
    b = gg.concat([(rp, ci)])
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_batch(ctx, b["vtx_off"], b["nnz_off"], d_rp, d_ci, d_col, o)
    assert e.value.code == lib.RSOC_EINVAL
    pool = lib.Pool(ctx, 0, 4)
    with pytest.raises(lib.RsocError) as e:
        pool.admit(d_rp, d_ci, n, d_col, o)
    assert e.value.code == lib.RSOC_EINVAL
    pool.close()
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_recolor_device(ctx, d_rp, d_ci, n, d_col, torch.zeros(1, dtype=torch.int32, device=d_col.device), o)
    assert e.value.code == lib.RSOC_EINVAL
