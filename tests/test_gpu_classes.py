"""Colour classes on the GPU against the oracle (bit-exact: the classes and the
order inside each class are unique), through the C ABI."""
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


def _classes(lib, ctx, colors, K):
    import torch
    d = torch.device("cuda:0")
    n = len(colors)
    d_c = torch.from_numpy(np.ascontiguousarray(colors, dtype=np.int32)).to(d)
    d_ptr = torch.full((K + 1,), -3, dtype=torch.int32, device=d)
    d_vtx = torch.full((max(n, 1),), -3, dtype=torch.int32, device=d)
    lib.rsoc_color_classes(ctx, d_c if n else None, n, K, d_ptr, d_vtx[:n] if n else None)
    return d_ptr.cpu().numpy(), d_vtx.cpu().numpy()[:n]


# sizes around the 64-id rows and 1024-id sub-tiles; K beyond one window of
# 2048 colours runs several passes
@pytest.mark.parametrize("n,K", [(0, 0), (0, 5), (1, 1), (63, 2), (64, 3), (65, 3), (1023, 19), (1024, 19),
                                 (1025, 19), (5000, 2048), (5000, 2049), (70000, 5000), (300001, 19),
                                 (100000, 1), (4096, 100000)])
def test_classes_random_colours(lib, ctx, n, K):
    rng = np.random.default_rng(n * 7 + K)
    c = rng.integers(0, max(K, 1), size=n).astype(np.int32)
    ptr, vtx = _classes(lib, ctx, c, K)
    want_ptr, want_vtx = oracle.classes(c, K)
    assert np.array_equal(ptr, want_ptr) and np.array_equal(vtx, want_vtx)


@pytest.mark.parametrize("name", ["tri_grid", "rmat", "lattice"])
def test_classes_of_colourings(lib, ctx, name):
    """Classes of the library's own colourings: identical to the oracle's and
    independent sets of the graph."""
    import torch
    rp, ci = {"tri_grid": lambda: gg.tri_grid(300, 200, permute_seed=5),
              "rmat": lambda: gg.rmat(14, 16, seed=3, shuffle_seed=4),
              "lattice": lambda: gg.lattice26(100, permute_seed=9)}[name]()
    d = torch.device("cuda:0")
    n = len(rp) - 1
    d_rp, d_ci = torch.from_numpy(rp).to(d), torch.from_numpy(ci).to(d)
    d_col = torch.empty(n, dtype=torch.int32, device=d)
    K, _ = lib.rsoc_color_device(ctx, d_rp, d_ci, n, d_col)
    col = d_col.cpu().numpy()
    assert oracle.check(rp, ci, col) == 0
    ptr, vtx = _classes(lib, ctx, col, K)
    want_ptr, want_vtx = oracle.classes(col, K)
    assert np.array_equal(ptr, want_ptr) and np.array_equal(vtx, want_vtx)
    # each class is independent: no edge joins two members of one class
    cls = np.empty(n, np.int64)
    for k in range(K):
        cls[vtx[ptr[k]:ptr[k + 1]]] = k
    src = np.repeat(np.arange(n), np.diff(rp))
    assert not np.any((cls[src] == cls[ci]) & (src != ci))


def test_classes_errors(lib, ctx):
    import torch
    d = torch.device("cuda:0")
    c = torch.tensor([0, 1, 3, 1], dtype=torch.int32, device=d)
    ptr = torch.empty(4, dtype=torch.int32, device=d)
    vtx = torch.empty(4, dtype=torch.int32, device=d)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_classes(ctx, c, 4, 3, ptr, vtx)  # colour 3 outside [0, 3)
    assert e.value.code == lib.RSOC_EINVAL
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_classes(ctx, c, 4, 0, ptr, vtx)
    assert e.value.code == lib.RSOC_EINVAL
    # the context still works afterwards
    lib.rsoc_color_classes(ctx, c, 4, 4, torch.empty(5, dtype=torch.int32, device=d), vtx)
    assert vtx.cpu().tolist() == [0, 1, 3, 2]
