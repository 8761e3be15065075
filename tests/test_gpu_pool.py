"""Continuous-batching pool on the GPU: graphs admitted at different times and
coloured by shared fused rounds must come out as they do alone (round-
synchronous mode: identical to the oracle; optimistic: valid)."""
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


def _dev(rp, ci):
    import torch
    d = torch.device("cuda:0")
    n = len(rp) - 1
    return (torch.from_numpy(np.ascontiguousarray(rp)).to(d),
            torch.from_numpy(np.ascontiguousarray(ci) if len(ci) else np.zeros(1, np.int32)).to(d),
            torch.full((max(n, 1),), -5, dtype=torch.int32, device=d), n)


GRAPHS = [gg.path(9), gg.cycle(7), gg.complete(30), gg.star(500), gg.tri_grid(40, 23), gg.tri_grid(31, 31, permute_seed=8),
          gg.rmat(11, 8, seed=9, shuffle_seed=10), gg.rgg(4000, seed=11), (np.zeros(1, np.int32), np.zeros(0, np.int32)),
          gg.complete_bipartite(33, 65), gg.grid4(50, 20),
          # colours of 255 and more: the distinct count goes through per-colour flags
          gg.complete(300)]
MODES = [("deterministic", "lower"), ("optimistic", "lower"), ("deterministic", "higher"), ("optimistic", "higher")]


def _check(lib, g, mode, tie, col, k, st=None):
    rp, ci = GRAPHS[g]
    n = len(rp) - 1
    got = col.cpu().numpy()[:n]
    if st is not None:
        assert st["colors_distinct"] == len(np.unique(got)), (g, mode, tie)
    if mode == "deterministic":
        want = oracle.rsync(rp, ci, tie=tie)
        assert np.array_equal(got, want["colors"]) and k == want["K"], (g, mode, tie)
    else:
        assert oracle.check(rp, ci, got) == 0 and k == oracle.colour_count(got), (g, mode, tie)


@pytest.mark.parametrize("split", [{}, {"t_thread": 3, "t_wave": 8}])
def test_pool_staggered_admission(lib, ctx, split):
    pool = lib.Pool(ctx, 0, 64)
    pending = [(g, MODES[(g + i) % 4]) for i in range(2) for g in range(len(GRAPHS))]
    live = {}
    done = 0
    steps = 0
    while pending or live:
        # admit two new graphs per step while older ones are mid-way
        for _ in range(2):
            if pending:
                g, (mode, tie) = pending.pop(0)
                d_rp, d_ci, d_col, n = _dev(*GRAPHS[g])
                slot = pool.admit(d_rp, d_ci, n, d_col, lib.make_options(mode, tie, **split))
                live[slot] = (g, mode, tie, d_rp, d_ci, d_col)
        for slot in pool.step():
            g, mode, tie, d_rp, d_ci, d_col = live.pop(slot)
            k, st = pool.result(slot)
            _check(lib, g, mode, tie, d_col, k, st)
            done += 1
        steps += 1
        assert steps < 5000
    assert done == 2 * len(GRAPHS) and pool.live() == 0 and pool.reserved_bytes() == 0
    pool.close()


def test_pool_budget_and_slots(lib, ctx):
    rp, ci = gg.tri_grid(64, 64)
    n = len(rp) - 1
    from paper_1505_04086_amd import serve
    per = serve.slot_scratch_bytes(n, False)  # optimistic slot scratch, as the serving layer accounts it
    pool = lib.Pool(ctx, per + per // 2, 8)
    a = _dev(rp, ci)
    b = _dev(rp, ci)
    s0 = pool.admit(a[0], a[1], n, a[2])
    assert pool.reserved_bytes() == per
    assert pool.try_admit(b[0], b[1], n, b[2]) == lib.RSOC_EBUDGET  # does not fit next to the first
    fin = []
    while not fin:
        fin = pool.step()
    assert fin == [s0]
    k, st = pool.result(s0)
    _check_valid = oracle.check(rp, ci, a[2].cpu().numpy())
    assert _check_valid == 0
    assert pool.reserved_bytes() == 0
    s1 = pool.admit(b[0], b[1], n, b[2])  # fits once the first is released
    while not pool.step():
        pass
    pool.result(s1)
    with pytest.raises(lib.RsocError) as e:
        pool.result(s1)
    assert e.value.code == lib.RSOC_ENOTFOUND
    pool.close()
    small = lib.Pool(ctx, 0, 2)
    p, q, r = _dev(*gg.path(5)), _dev(*gg.path(5)), _dev(*gg.path(5))
    small.admit(p[0], p[1], 5, p[2])
    small.admit(q[0], q[1], 5, q[2])
    assert small.try_admit(r[0], r[1], 5, r[2]) == lib.RSOC_EBUDGET  # slot table full
    small.close()


def test_pool_max_rounds_guard(lib, ctx):
    pool = lib.Pool(ctx, 0, 4)
    d = _dev(*gg.path(6))
    slot = pool.admit(d[0], d[1], 6, d[2], lib.make_options("deterministic", max_rounds=2))
    while not pool.step():
        pass
    with pytest.raises(lib.RsocError) as e:
        pool.result(slot)
    assert e.value.code == lib.RSOC_ENOCONV
    want = oracle.rsync(*gg.path(6), max_rounds=2, raise_on_noconv=False)
    assert np.array_equal(d[2].cpu().numpy()[:6], want["colors"])
    pool.close()


def test_pool_admission_errors_arrive_with_the_result(lib, ctx):
    """Admission waits on nothing: bad row_ptr ends and edges without col_idx
    finish their slot at the next step and come back from rsoc_pool_result,
    next to a good graph admitted beside them."""
    import torch
    pool = lib.Pool(ctx, 0, 8)
    good = _dev(*gg.cycle(9))
    rp, ci = gg.cycle(7)
    bad_rp = rp.copy()
    bad_rp[0] = 1
    bad = _dev(bad_rp, ci)
    d = torch.device("cuda:0")
    nocol = (torch.from_numpy(rp).to(d), None, torch.empty(7, dtype=torch.int32, device=d))
    slots = {"good": pool.admit(good[0], good[1], 9, good[2]), "bad": pool.admit(bad[0], bad[1], 7, bad[2]),
             "nocol": pool.admit(nocol[0], nocol[1], 7, nocol[2])}
    done = set()
    while len(done) < 3:
        done |= set(pool.step())
    assert done == set(slots.values())
    for name, code in (("bad", lib.RSOC_ECSR), ("nocol", lib.RSOC_EINVAL)):
        with pytest.raises(lib.RsocError) as e:
            pool.result(slots[name])
        assert e.value.code == code
    k, st = pool.result(slots["good"])
    assert oracle.check(*gg.cycle(9), good[2].cpu().numpy()[:9]) == 0 and k == 3
    assert pool.live() == 0 and pool.reserved_bytes() == 0
    pool.close()


def test_pool_recolour_requests(lib, ctx):
    """Recolouring requests (previous colouring + touched vertices) admitted
    beside ordinary colourings into the same fused rounds: deterministic ones
    equal the oracle's recolouring, optimistic ones are valid; an empty U^0
    leaves the colouring as it was; a touched id out of range comes back as
    RSOC_EINVAL."""
    import torch
    from tests.graph_edits import edit
    d = torch.device("cuda:0")
    jobs = []
    graphs = [G for G in GRAPHS if len(G[0]) > 1]
    for g, (mode, tie) in enumerate(MODES * 2):
        rp, ci = graphs[(g * 3) % len(graphs)]
        n = len(rp) - 1
        prev, _ = oracle.seq_ff(rp, ci)
        rp2, ci2, touched = edit(rp, ci, seed=g, add=20, delete=20, new=3)
        prev2 = np.concatenate([prev, np.full(len(rp2) - 1 - n, -1, np.int32)])
        jobs.append(("recolor", mode, tie, rp2, ci2, prev2, touched))
        jobs.append(("colour", mode, tie, rp, ci, None, None))
    rp, ci = gg.cycle(9)
    prev, _ = oracle.seq_ff(rp, ci)
    jobs.append(("recolor", "deterministic", "lower", rp, ci, prev, np.zeros(0, np.int32)))  # nothing to do
    pool = lib.Pool(ctx, 0, 64)
    live, done, tensors = {}, {}, {}  # slot -> job index (slot ids are reused once released); job index -> result

    def collect(slots):
        for f in slots:
            done[live.pop(f)] = pool.result(f)

    for j, (kind, mode, tie, rp, ci, prev, touched) in enumerate(jobs):
        n = len(rp) - 1
        d_rp, d_ci = torch.from_numpy(rp).to(d), torch.from_numpy(ci).to(d)
        opts = lib.make_options(mode, tie)
        if kind == "recolor":
            d_col = torch.from_numpy(prev).to(d)
            d_t = torch.from_numpy(touched).to(d) if len(touched) else None
            slot = pool.admit_recolor(d_rp, d_ci, n, d_col, d_t, opts)
        else:
            d_col = torch.empty(n, dtype=torch.int32, device=d)
            d_t = None
            slot = pool.admit(d_rp, d_ci, n, d_col, opts)
        live[slot] = j
        tensors[j] = (d_rp, d_ci, d_col, d_t)
        collect(pool.step())  # staggered: older slots are mid-way when newer ones arrive
    steps = 0
    while len(done) < len(jobs):
        collect(pool.step())
        steps += 1
        assert steps < 5000
    for j, (kind, mode, tie, rp, ci, prev, touched) in enumerate(jobs):
        k, st = done[j]
        got = tensors[j][2].cpu().numpy()
        slot = j
        if kind == "recolor" and mode == "deterministic":
            want = oracle.recolor(rp, ci, prev, touched, tie=tie)
            assert np.array_equal(got, want["colors"]) and k == want["K"], (slot, tie)
        elif kind == "colour" and mode == "deterministic":
            want = oracle.rsync(rp, ci, tie=tie)
            assert np.array_equal(got, want["colors"]) and k == want["K"], (slot, tie)
        else:
            assert oracle.check(rp, ci, got) == 0 and k == oracle.colour_count(got), (slot, kind, mode)
    assert pool.live() == 0
    # a touched id outside [0, n)
    rp, ci = gg.path(5)
    d_col = torch.zeros(5, dtype=torch.int32, device=d)
    slot = pool.admit_recolor(torch.from_numpy(rp).to(d), torch.from_numpy(ci).to(d), 5, d_col,
                              torch.tensor([7], dtype=torch.int32, device=d))
    while slot not in pool.step():
        pass
    with pytest.raises(lib.RsocError) as e:
        pool.result(slot)
    assert e.value.code == lib.RSOC_EINVAL
    pool.close()


def test_pool_split_step(lib, ctx):
    """rsoc_pool_step_launch / rsoc_pool_step_finish: graphs admitted (and
    earlier results taken) while a launched round runs join a later round;
    every result is as with rsoc_pool_step.  A second launch, a plain step
    while one is in flight, and a finish without a launch are refused."""
    pool = lib.Pool(ctx, 0, 64)
    pending = [(g, MODES[(g + i) % 4]) for i in range(2) for g in range(len(GRAPHS))]
    live, ready = {}, []
    done = steps = 0
    with pytest.raises(lib.RsocError) as e:
        pool.step_finish()
    assert e.value.code == lib.RSOC_EINVAL
    while pending or live:
        pool.step_launch()
        if steps == 0:
            for bad in (pool.step_launch, pool.step):
                with pytest.raises(lib.RsocError) as e:
                    bad()
                assert e.value.code == lib.RSOC_EINVAL
        # results of the previous round, then new graphs, while this round runs
        for slot in ready:
            g, mode, tie, d_rp, d_ci, d_col = live.pop(slot)
            k, st = pool.result(slot)
            _check(lib, g, mode, tie, d_col, k, st)
            done += 1
        for _ in range(3):
            if pending:
                g, (mode, tie) = pending.pop(0)
                d_rp, d_ci, d_col, n = _dev(*GRAPHS[g])
                slot = pool.admit(d_rp, d_ci, n, d_col, lib.make_options(mode, tie))
                live[slot] = (g, mode, tie, d_rp, d_ci, d_col)
        ready = pool.step_finish()
        steps += 1
        assert steps < 5000
    assert done == 2 * len(GRAPHS) and pool.live() == 0 and pool.reserved_bytes() == 0
    pool.close()


def test_pool_many_slots_one_step(lib, ctx):
    """Many slots of very different sizes in the same rounds (the device deals
    each table over its buckets): every result as alone."""
    import torch
    pool = lib.Pool(ctx, 0, 300)
    live = {}
    rng = np.random.default_rng(5)
    for i in range(260):
        g = int(rng.integers(len(GRAPHS)))
        mode, tie = MODES[i % 4]
        d_rp, d_ci, d_col, n = _dev(*GRAPHS[g])
        live[pool.admit(d_rp, d_ci, n, d_col, lib.make_options(mode, tie))] = (g, mode, tie, d_rp, d_ci, d_col)
    torch.cuda.synchronize()
    done = steps = 0
    while live:
        for slot in pool.step():
            g, mode, tie, d_rp, d_ci, d_col = live.pop(slot)
            k, st = pool.result(slot)
            _check(lib, g, mode, tie, d_col, k, st)
            done += 1
        steps += 1
        assert steps < 5000
    assert done == 260 and pool.live() == 0
    pool.close()


@pytest.mark.parametrize("mode", ["deterministic", "optimistic"])
def test_pool_one_large_slot(lib, ctx, mode):
    """One large graph alone in the pool: every workgroup takes many tasks of
    the same slot, so its append buffers carry over from task to task and fill
    up several times (flushed when full, when the slot changes and at the end
    of the launch).  Deterministic: equal to the oracle; optimistic: valid."""
    import torch
    rp, ci = gg.lattice26(128, permute_seed=17)  # 2.1 M vertices: about four tasks per workgroup
    n = len(rp) - 1
    d = torch.device("cuda:0")
    d_rp, d_ci = torch.from_numpy(rp).to(d), torch.from_numpy(ci).to(d)
    d_col = torch.full((n,), -5, dtype=torch.int32, device=d)
    pool = lib.Pool(ctx, 0, 8)
    slot = pool.admit(d_rp, d_ci, n, d_col, lib.make_options(mode))
    steps = 0
    while True:
        fin = pool.step()
        steps += 1
        assert steps < 1000
        if slot in fin:
            break
    k, st = pool.result(slot)
    got = d_col.cpu().numpy()
    if mode == "deterministic":
        want = oracle.rsync(rp, ci)
        assert np.array_equal(got, want["colors"]) and k == want["K"]
        assert st["rounds"] == want["rounds"] and st["conflicts"] == want["conflicts"]
    else:
        assert oracle.check(rp, ci, got) == 0 and k == oracle.colour_count(got)
    assert st["colors_distinct"] == len(np.unique(got))
    pool.close()


def test_pool_more_spans_than_lds_holds(lib, ctx):
    """2100 slots in the same rounds: a task table's spans (one per slot)
    exceed what the dealing kernel stages in LDS (2048), so it reads them from
    memory; every result as alone."""
    import torch
    small = [gg.path(9), gg.cycle(7), gg.complete(6), gg.star(20), gg.tri_grid(5, 4)]
    pool = lib.Pool(ctx, 0, 2200)
    live = {}
    d = torch.device("cuda:0")
    dev = [(torch.from_numpy(rp).to(d), torch.from_numpy(ci).to(d)) for rp, ci in small]
    for i in range(2100):
        g = i % len(small)
        mode, tie = MODES[i % 4]
        n = len(small[g][0]) - 1
        col = torch.full((n,), -5, dtype=torch.int32, device=d)
        live[pool.admit(dev[g][0], dev[g][1], n, col, lib.make_options(mode, tie))] = (g, mode, tie, col)
    torch.cuda.synchronize()
    steps = 0
    while live:
        for slot in pool.step(cap=4096):
            g, mode, tie, col = live.pop(slot)
            k, st = pool.result(slot)
            rp, ci = small[g]
            got = col.cpu().numpy()
            if mode == "deterministic":
                assert np.array_equal(got, oracle.rsync(rp, ci, tie=tie)["colors"]), g
            else:
                assert oracle.check(rp, ci, got) == 0, g
        steps += 1
        assert steps < 1000
    pool.close()
