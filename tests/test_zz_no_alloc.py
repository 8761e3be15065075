"""rsoc_color_classes_noalloc (no context, fixed per-GPU scratch, no
allocation) against rsoc_color_classes, element by element, through the C ABI.

Calls follow each other on one GPU, so each one reuses the scratch the
previous call left behind: a larger input first, then smaller ones, must each
equal the context entry point (and the oracle's classes)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _run(lib, fn, colors, K, ctx=None):
    import torch
    d = torch.device("cuda:0")
    n = len(colors)
    d_c = torch.from_numpy(np.ascontiguousarray(colors, dtype=np.int32)).to(d)
    d_ptr = torch.full((K + 1,), -3, dtype=torch.int32, device=d)
    d_vtx = torch.full((max(n, 1),), -3, dtype=torch.int32, device=d)
    if ctx is None:
        fn(d_c if n else None, n, K, d_ptr, d_vtx[:n] if n else None)
    else:
        fn(ctx, d_c if n else None, n, K, d_ptr, d_vtx[:n] if n else None)
    return d_ptr.cpu().numpy(), d_vtx.cpu().numpy()[:n]


# (n, K) in call order: a count table over several passes (3 M ids, 1000
# colours: at most 357 colours per pass in the fixed table), then smaller inputs
SEQUENCES = [
    [(3_000_000, 1000), (70_000, 5000)],
    [(300_001, 19), (1025, 3)],
    [(5000, 2049), (0, 4)],
]


@pytest.mark.parametrize("seq", SEQUENCES, ids=lambda s: "_".join("%dx%d" % c for c in s))
def test_noalloc_matches_context_entry_point(lib, seq):
    ctx = lib.Context(0)
    try:
        for i, (n, K) in enumerate(seq):
            print("call", i, "n", n, "K", K, flush=True)
            rng = np.random.default_rng(1000 * i + n + K)
            c = rng.integers(0, K, size=n).astype(np.int32)
            got_ptr, got_vtx = _run(lib, lib.rsoc_color_classes_noalloc, c, K)
            ref_ptr, ref_vtx = _run(lib, lib.rsoc_color_classes, c, K, ctx)
            assert np.array_equal(got_ptr, ref_ptr) and np.array_equal(got_vtx, ref_vtx)
            if n <= 300_001:
                want_ptr, want_vtx = oracle.classes(c, K)
                assert np.array_equal(got_ptr, want_ptr) and np.array_equal(got_vtx, want_vtx)
    finally:
        ctx.close()


def test_noalloc_errors(lib):
    import torch
    d = torch.device("cuda:0")
    buf = torch.zeros(8, dtype=torch.int32, device=d)
    # more vertices than the fixed count table covers: refused on the host, nothing launched
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_classes_noalloc(buf, (1 << 30) + 1, 4, buf, buf)
    assert e.value.code == lib.RSOC_ESCRATCH
    # a colour outside [0, K), found on the device, as for the context entry point
    c = torch.tensor([0, 1, 7, 2], dtype=torch.int32, device=d)
    with pytest.raises(lib.RsocError) as e:
        lib.rsoc_color_classes_noalloc(c, 4, 3, buf, buf[:4])
    assert e.value.code == lib.RSOC_EINVAL
    # and the next call is unaffected by that one's error flag
    ptr = torch.full((4,), -3, dtype=torch.int32, device=d)
    vtx = torch.full((4,), -3, dtype=torch.int32, device=d)
    c = torch.tensor([2, 0, 2, 1], dtype=torch.int32, device=d)
    lib.rsoc_color_classes_noalloc(c, 4, 3, ptr, vtx)
    assert ptr.cpu().tolist() == [0, 1, 2, 4] and vtx.cpu().tolist() == [1, 3, 0, 2]
