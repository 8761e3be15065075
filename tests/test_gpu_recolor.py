"""Recolouring after topology edits on the GPU, through the C ABI: the
round-synchronous mode equals the oracle element by element (colours, K,
rounds, |L| per round); the optimistic mode gives a valid colouring within the
First-Fit bound."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.graph_edits import csr_from_edges as _csr, edit

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "recolor_worked_examples.json")


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _run(lib, ctx, rp, ci, prev, touched, mode, tie="lower", **kw):
    import torch
    d = torch.device("cuda:0")
    n = len(rp) - 1
    d_rp = torch.from_numpy(np.ascontiguousarray(rp)).to(d)
    d_ci = torch.from_numpy(np.ascontiguousarray(ci) if len(ci) else np.zeros(1, np.int32)).to(d)
    d_col = torch.from_numpy(np.ascontiguousarray(prev, dtype=np.int32)).to(d)
    d_t = torch.from_numpy(np.ascontiguousarray(touched, dtype=np.int32)).to(d) if len(touched) else None
    k, st = lib.rsoc_recolor_device(ctx, d_rp, d_ci, n, d_col, d_t, lib.make_options(mode, tie, **kw),
                                    per_round_cap=4096)
    return k, st, d_col.cpu().numpy()


def _check(lib, ctx, rp, ci, prev, touched, mode, tie, **kw):
    k, st, got = _run(lib, ctx, rp, ci, prev, touched, mode, tie, **kw)
    if mode == "deterministic":
        want = oracle.recolor(rp, ci, prev, touched, tie=tie)
        assert np.array_equal(got, want["colors"]) and k == want["K"]
        assert st["rounds"] == want["rounds"] and list(st["L_sizes"]) == list(want["L_sizes"])
    else:
        assert oracle.check(rp, ci, got) == 0 and k == oracle.colour_count(got)
    assert st["colors_distinct"] == len(np.unique(got))
    return st


SPLITS = {"default": {}, "allbins": {"t_thread": 3, "t_wave": 8}, "wave_only": {"t_thread": 1, "t_wave": 100000},
          "grid1": {"grid_list": 1}}


@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("mode", ["deterministic", "optimistic"])
def test_recolor_worked_examples(lib, ctx, mode, tie):
    g = json.load(open(GOLDEN))
    for case in g["cases"]:
        e = np.array(case["edges"], np.int64)
        rp, ci = _csr(case["n"], np.sort(e, axis=1))
        k, st, got = _run(lib, ctx, rp, ci, case["prev"], case["touched"], mode, tie)
        if mode == "deterministic":
            w = case["lower_keeps" if tie == "lower" else "higher_keeps"]
            assert got.tolist() == w["colors"] and st["rounds"] == w["rounds"], case["name"]
        else:
            assert oracle.check(rp, ci, got) == 0


GRAPHS = {"tri_grid": lambda: gg.tri_grid(60, 45, permute_seed=2), "rmat": lambda: gg.rmat(12, 8, seed=5, shuffle_seed=6),
          "rgg": lambda: gg.rgg(5000, seed=7), "star": lambda: gg.star(3000), "k40": lambda: gg.complete(40)}


@pytest.mark.parametrize("split", sorted(SPLITS))
@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("mode", ["deterministic", "optimistic"])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_recolor_after_edits(lib, ctx, name, mode, tie, split):
    rp, ci = GRAPHS[name]()
    n = len(rp) - 1
    prev, _ = oracle.seq_ff(rp, ci)
    rp2, ci2, touched = edit(rp, ci, seed=n + len(ci))
    prev2 = np.concatenate([prev, np.full(len(rp2) - 1 - n, -1, np.int32)])
    _check(lib, ctx, rp2, ci2, prev2, touched, mode, tie, **SPLITS[split])


@pytest.mark.parametrize("mode", ["deterministic", "optimistic"])
def test_recolor_special_starts(lib, ctx, mode):
    """No colours at all (everyone recoloured), all colours 0 with every vertex
    touched (the round-synchronous schedule itself), and a valid colouring
    with nothing touched (left alone)."""
    rp, ci = gg.tri_grid(40, 30, permute_seed=4)
    n = len(rp) - 1
    _check(lib, ctx, rp, ci, np.full(n, -1, np.int32), [], mode, "lower")
    _check(lib, ctx, rp, ci, np.zeros(n, np.int32), np.arange(n), mode, "lower")
    prev, _ = oracle.seq_ff(rp, ci)
    k, st, got = _run(lib, ctx, rp, ci, prev, [], mode)
    assert np.array_equal(got, prev) and st["rounds"] == 0 and st["worklist0"] == 0


def test_recolor_large_lattice(lib, ctx):
    """10^6-vertex permuted lattice coloured by the library, 2000 edges
    inserted and deleted, 100 new vertices: deterministic equals the oracle,
    optimistic is valid."""
    import torch
    rp, ci = gg.lattice26(100, permute_seed=11)
    n = len(rp) - 1
    d = torch.device("cuda:0")
    d_col = torch.empty(n, dtype=torch.int32, device=d)
    lib.rsoc_color_device(ctx, torch.from_numpy(rp).to(d), torch.from_numpy(ci).to(d), n, d_col)
    prev = d_col.cpu().numpy()
    rp2, ci2, touched = edit(rp, ci, seed=12, add=2000, delete=2000, new=100)
    prev2 = np.concatenate([prev, np.full(len(rp2) - 1 - n, -1, np.int32)])
    for mode in ("deterministic", "optimistic"):
        st = _check(lib, ctx, rp2, ci2, prev2, touched, mode, "lower")
        assert st["worklist0"] <= len(touched) + 100 + 4000


def _spider(leaves, tie):
    """A hub joined to `leaves` leaves; the hub loses every tie (highest id
    under lower-keeps, id 0 under higher-keeps)."""
    n = leaves + 1
    hub = n - 1 if tie == "lower" else 0
    others = np.array([v for v in range(n) if v != hub], np.int64)
    e = np.stack([np.full(leaves, hub, np.int64), others], axis=1)
    rp, ci = gg.from_edges(n, e)
    return rp, ci, hub, others


@pytest.mark.parametrize("top", [1000, 5000])
@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("mode", ["deterministic", "optimistic"])
def test_recolor_hub_high_colour(lib, ctx, mode, tie, top):
    """A 5000-leaf hub (workgroup bin) whose leaves hold colours 0..top-1
    (cycling) and whose own colour clashes with a leaf it loses to: its
    First-Fit answer is top, beyond the wavefront window (4096 colours) and,
    for top = 5000, beyond every colour the byte shadow can hold."""
    rp, ci, hub, others = _spider(5000, tie)
    prev = np.zeros(len(rp) - 1, np.int32)
    prev[others] = np.arange(len(others)) % top
    prev[hub] = 0
    print("case", mode, tie, top, flush=True)
    st = _check(lib, ctx, rp, ci, prev, [hub], mode, tie)
    assert st["rounds"] >= 1


def test_recolor_errors(lib, ctx):
    import torch
    rp, ci = gg.cycle(8)
    d = torch.device("cuda:0")
    d_rp, d_ci = torch.from_numpy(rp).to(d), torch.from_numpy(ci).to(d)
    col = torch.zeros(8, dtype=torch.int32, device=d)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_recolor_device(ctx, d_rp, d_ci, 8, col, torch.tensor([1, 9], dtype=torch.int32, device=d))
    assert e.value.code == lib.RSOC_EINVAL
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_recolor_device(ctx, d_rp, d_ci, 8, col, None, lib.make_options("two_phase"))
    assert e.value.code == lib.RSOC_EINVAL
    bad = rp.copy()
    bad[0] = 1
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_recolor_device(ctx, torch.from_numpy(bad).to(d), d_ci, 8, col, None)
    assert e.value.code == lib.RSOC_ECSR
    k, st = lib.rsoc_recolor_device(ctx, d_rp, d_ci, 8, col, torch.arange(8, dtype=torch.int32, device=d),
                                    lib.make_options("deterministic"))
    want = oracle.recolor(rp, ci, np.zeros(8, np.int32), np.arange(8))
    assert np.array_equal(col.cpu().numpy(), want["colors"]) and k == want["K"]
