"""The request loop on the GPU: each request's result is the same alone (one
call per request) and in the mix (continuous batching under a tight HBM
budget, staggered arrivals).

Tolerance: round-synchronous (deterministic) requests must be identical to
the oracle both ways; optimistic requests must be valid colourings with
0 <= c(v) <= deg(v) both ways, and their colour counts may differ by at most
max(2, 10%) between the two runs (speculation order differs)."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def _graphs():
    gs = [gg.tri_grid(120, 90), gg.lattice26(18, permute_seed=3), gg.rmat(12, 16, seed=4, shuffle_seed=5),
          gg.tri_grid(40, 40, permute_seed=6), gg.rgg(20000, seed=7), gg.lattice26(25, permute_seed=8),
          gg.rmat(13, 16, seed=9, shuffle_seed=10), gg.path(1000), gg.complete(60),
          (np.zeros(1, np.int32), np.zeros(0, np.int32))]
    return gs


GRAPHS = _graphs()


def test_alone_equals_mix(lib):
    import torch
    from paper_1505_04086_amd import serve
    ctx = lib.Context(0)
    det = lib.make_options("deterministic")
    opt = lib.make_options("optimistic")
    reqs_spec = [(i, det if i % 2 == 0 else opt) for i in range(len(GRAPHS))] * 2

    def make(arrivals):
        return [serve.Request(k, torch.from_numpy(GRAPHS[g][0]).pin_memory(), torch.from_numpy(GRAPHS[g][1]).pin_memory(),
                              float(arrivals[k]), options=o) for k, (g, o) in enumerate(reqs_spec)]

    alone = serve.PlainServer(ctx).run(make(np.zeros(len(reqs_spec))))
    # budget for roughly three of the larger graphs at a time: admission must wait for releases
    largest = max(serve.csr_bytes(len(rp) - 1, len(ci)) for rp, ci in GRAPHS)
    # every request through the pool (no single-graph runs on an idle server)
    sv = serve.Server(ctx, hbm_budget=int(3 * largest / 0.65), scratch_share=0.35, max_slots=8,
                      solo_when_idle=False)
    arrivals = np.cumsum(np.full(len(reqs_spec), 0.0005))
    mix = sv.run(make(arrivals))
    sv.close()
    assert len(mix) == len(alone) == len(reqs_spec)
    by_id = {r.rid: r for r in mix}
    for a in alone:
        m = by_id[a.rid]
        g, o = reqs_spec[a.rid]
        rp, ci = GRAPHS[g]
        if o.mode == lib.RSOC_MODE_DETERMINISTIC:
            want = oracle.rsync(rp, ci)
            assert np.array_equal(a.colors, want["colors"]) and np.array_equal(m.colors, want["colors"]), a.rid
            assert a.k == m.k == want["K"]
        else:
            assert oracle.check(rp, ci, a.colors) == 0 and oracle.check(rp, ci, m.colors) == 0, a.rid
            assert abs(a.k - m.k) <= max(2, 0.1 * a.k), (a.k, m.k)
        assert m.latency >= 0
    assert sv.ledger.used == 0
    # device-resident requests (CSR already in HBM, colours left on the device)
    dev = torch.device("cuda:0")
    res = [(torch.from_numpy(rp).to(dev), torch.from_numpy(ci if len(ci) else np.zeros(1, np.int32)).to(dev))
           for rp, ci in GRAPHS]
    sv = serve.Server(ctx, hbm_budget=int(3 * largest / 0.65), scratch_share=0.35, max_slots=8)
    mix2 = sv.run([serve.Request(k, res[g][0], res[g][1], float(arrivals[k]), options=o)
                   for k, (g, o) in enumerate(reqs_spec)])
    sv.close()
    for m in mix2:
        g, o = reqs_spec[m.rid]
        rp, ci = GRAPHS[g]
        got = m.colors.cpu().numpy()
        if o.mode == lib.RSOC_MODE_DETERMINISTIC:
            assert np.array_equal(got, oracle.rsync(rp, ci)["colors"]), m.rid
        else:
            assert oracle.check(rp, ci, got) == 0, m.rid
    ctx.close()


def test_recolour_requests_served(lib):
    """Recolouring requests (colouring from before the edits + touched
    vertices) served beside colouring requests, in the mix and alone:
    deterministic ones equal the oracle's recolouring, optimistic ones are
    valid."""
    from paper_1505_04086_amd import serve
    from tests.graph_edits import edit
    ctx = lib.Context(0)
    specs = []
    for i, (rp, ci) in enumerate(GRAPHS[:7]):
        n = len(rp) - 1
        prev, _ = oracle.seq_ff(rp, ci)
        rp2, ci2, touched = edit(rp, ci, seed=100 + i, add=200, delete=100, new=10)
        prev2 = np.concatenate([prev, np.full(len(rp2) - 1 - n, -1, np.int32)])
        mode = "deterministic" if i % 2 == 0 else "optimistic"
        specs.append((rp2, ci2, prev2, touched, mode))
        specs.append((rp, ci, None, None, mode))

    def make():
        return [serve.Request(k, rp, ci, 0.0002 * k, options=lib.make_options(mode), prev_colors=prev,
                              touched=touched) for k, (rp, ci, prev, touched, mode) in enumerate(specs)]

    largest = max(serve.csr_bytes(len(s[0]) - 1, len(s[1])) for s in specs)
    sv = serve.Server(ctx, hbm_budget=int(3 * largest / 0.65), scratch_share=0.35, max_slots=8,
                      solo_when_idle=False)
    mix = sv.run(make())
    assert sv.solo == 0
    sv.close()
    alone = serve.PlainServer(ctx).run(make())
    for out in (mix, alone):
        assert len(out) == len(specs)
        for r in out:
            rp, ci, prev, touched, mode = specs[r.rid]
            if mode == "deterministic":
                want = oracle.recolor(rp, ci, prev, touched) if prev is not None else oracle.rsync(rp, ci)
                assert np.array_equal(r.colors, want["colors"]) and r.k == want["K"], r.rid
            else:
                assert oracle.check(rp, ci, r.colors) == 0 and r.k == oracle.colour_count(r.colors), r.rid
    assert sv.ledger.used == 0
    ctx.close()


def test_idle_server_runs_lone_requests_directly(lib):
    """Requests spaced far apart each find the server idle and are coloured
    with the single-graph entry point (host and device-resident CSR,
    colourings and recolourings); the results are those of the plain path:
    deterministic ones equal the oracle's, optimistic ones are valid."""
    import torch
    from paper_1505_04086_amd import serve
    from tests.graph_edits import edit
    ctx = lib.Context(0)
    dev = torch.device("cuda:0")
    specs = []
    for i, (rp, ci) in enumerate(GRAPHS[:6]):
        mode = "deterministic" if i % 2 == 0 else "optimistic"
        specs.append((rp, ci, None, None, mode, i % 3 == 1))
        if i < 3:
            n = len(rp) - 1
            prev, _ = oracle.seq_ff(rp, ci)
            rp2, ci2, touched = edit(rp, ci, seed=200 + i, add=100, delete=50, new=5)
            prev2 = np.concatenate([prev, np.full(len(rp2) - 1 - n, -1, np.int32)])
            specs.append((rp2, ci2, prev2, touched, mode, False))

    def make(rp, ci, resident):
        if resident:
            return torch.from_numpy(rp).to(dev), torch.from_numpy(ci if len(ci) else np.zeros(1, np.int32)).to(dev)
        return rp, ci

    def requests(gap):
        reqs = []
        for k, (rp, ci, prev, touched, mode, resident) in enumerate(specs):
            a, b = make(rp, ci, resident)
            reqs.append(serve.Request(k, a, b, gap * k, options=lib.make_options(mode), prev_colors=prev,
                                      touched=touched))
        return reqs

    serve.PlainServer(ctx).run(requests(0.0))  # first-use set-up of the context, outside the spaced run
    sv = serve.Server(ctx, hbm_budget=1 << 30, max_slots=8)
    out = sv.run(requests(0.1))
    sv.close()
    assert len(out) == len(specs) and sv.ledger.used == 0
    assert sv.solo == len(specs), "every request should have found the server idle"
    for r in out:
        rp, ci, prev, touched, mode, resident = specs[r.rid]
        got = r.colors.cpu().numpy() if resident else r.colors
        if mode == "deterministic":
            want = oracle.recolor(rp, ci, prev, touched) if prev is not None else oracle.rsync(rp, ci)
            assert np.array_equal(got, want["colors"]) and r.k == want["K"], r.rid
        else:
            assert oracle.check(rp, ci, got) == 0 and r.k == oracle.colour_count(got), r.rid
    ctx.close()
