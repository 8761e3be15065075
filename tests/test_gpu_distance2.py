"""Distance-2 colouring on the GPU (G^2 built on the device, then the same
rounds), through the C ABI: round-synchronous mode equals the oracle's
Algorithm 3 on its own G^2 element by element; optimistic mode gives a valid
colouring of G^2 (no two vertices within distance 2 share a colour)."""
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


GRAPHS = {"path": lambda: gg.path(50), "cycle": lambda: gg.cycle(31), "star": lambda: gg.star(100),
          "tri_grid": lambda: gg.tri_grid(40, 30, permute_seed=3), "grid4": lambda: gg.grid4(33, 20),
          "lattice": lambda: gg.lattice26(10, permute_seed=4), "rmat": lambda: gg.rmat(7, 4, seed=5, shuffle_seed=6),
          "gnp": lambda: gg.random_gnp(300, 0.05, 7), "k20": lambda: gg.complete(20),
          "hub_over_1024": lambda: gg.star(1500)}
SPLITS = {"default": {}, "allbins": {"t_thread": 3, "t_wave": 8}}


@pytest.mark.parametrize("split", sorted(SPLITS))
@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_distance2_deterministic_matches_oracle(lib, ctx, name, tie, split):
    rp, ci = GRAPHS[name]()
    d_rp, d_ci, d_col, n = _dev(rp, ci)
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col,
                                  lib.make_options("deterministic", tie, distance=2, **SPLITS[split]),
                                  per_round_cap=4096)
    want = oracle.rsync_d2(rp, ci, tie=tie)
    got = d_col.cpu().numpy()[:n]
    assert np.array_equal(got, want["colors"]) and k == want["K"]
    assert st["rounds"] == want["rounds"] and list(st["L_sizes"]) == list(want["L_sizes"])


@pytest.mark.parametrize("full_sweep", [0, 1])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_distance2_optimistic_valid(lib, ctx, name, full_sweep):
    rp, ci = GRAPHS[name]()
    d_rp, d_ci, d_col, n = _dev(rp, ci)
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col,
                                  lib.make_options("optimistic", distance=2, full_sweep=full_sweep))
    got = d_col.cpu().numpy()[:n]
    rp2, ci2 = oracle.square(rp, ci)
    assert oracle.check(rp2.astype(np.int32), ci2, got) == 0 and k == oracle.colour_count(got)


def test_distance2_larger_meshes(lib, ctx):
    """A 60^3 permuted lattice (2-hop walks of 702 entries) and a 300 x 300
    grid: deterministic equals the oracle, optimistic is valid."""
    for rp, ci in (gg.lattice26(60, permute_seed=8), gg.tri_grid(300, 300, permute_seed=9)):
        d_rp, d_ci, d_col, n = _dev(rp, ci)
        k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("deterministic", distance=2))
        want = oracle.rsync_d2(rp, ci)
        assert np.array_equal(d_col.cpu().numpy()[:n], want["colors"]) and k == want["K"]
        k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("optimistic", distance=2))
        rp2, ci2 = oracle.square(rp, ci)
        assert oracle.check(rp2.astype(np.int32), ci2, d_col.cpu().numpy()[:n]) == 0


def test_distance2_host_entry_and_errors(lib, ctx):
    rp, ci = gg.tri_grid(20, 15, permute_seed=1)
    n = len(rp) - 1
    col, k, st = lib.rsoc_color_ex(ctx, rp, ci, n, options=lib.make_options("deterministic", distance=2))
    want = oracle.rsync_d2(rp, ci)
    assert np.array_equal(col, want["colors"]) and k == want["K"]
    # a 2-hop walk over the limit (a leaf of a 9000-leaf star sees every leaf)
    d_rp, d_ci, d_col, n = _dev(*gg.star(9000))
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options(distance=2))
    assert e.value.code == lib.RSOC_EINVAL
    # validation looks at G itself
    rp, ci = gg.cycle(6)
    loop = ci.copy()
    loop[0] = 0
    d_rp, d_ci, d_col, n = _dev(rp, loop)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options(distance=2, validate=1))
    assert e.value.code == lib.RSOC_ESELFLOOP
    bad = rp.copy()
    bad[0] = 1
    d_rp, d_ci, d_col, n = _dev(bad, ci)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options(distance=2))
    assert e.value.code == lib.RSOC_ECSR
    # the context colours distance 1 normally afterwards
    d_rp, d_ci, d_col, n = _dev(rp, ci)
    k, st = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, lib.make_options("deterministic"))
    assert np.array_equal(d_col.cpu().numpy()[:n], oracle.rsync(rp, ci)["colors"])
