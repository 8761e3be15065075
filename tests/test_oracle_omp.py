"""The OpenMP run of Algorithm 3 (oracle/omp_rsoc.c), the CPU baseline the
benchmark times on the host's cores.  With one thread, round 0 is Algorithm 1
in natural order and nothing is left to recolour, so the result must equal
sequential First-Fit element by element (Section 4 runs Algorithm 3 from one
thread up); with several threads any valid colouring within the First-Fit
bound is a correct result."""
import numpy as np
import pytest

import graphgen as gg
import oracle

GRAPHS = {
    "path": lambda: gg.path(50),
    "cycle5": lambda: gg.cycle(5),
    "K9": lambda: gg.complete(9),
    "star": lambda: gg.star(100),
    "tri_grid_perm": lambda: gg.tri_grid(120, 90, permute_seed=5),
    "rmat13": lambda: gg.rmat(13, 16, seed=3, shuffle_seed=4),
    "lattice30": lambda: gg.lattice26(30, permute_seed=2),
    "rgg": lambda: gg.rgg(5000, seed=7),
    "empty": lambda: (np.zeros(6, np.int32), np.zeros(0, np.int32)),
}


@pytest.mark.parametrize("tie", ["lower", "higher"])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_one_thread_is_sequential_first_fit(name, tie):
    rp, ci = GRAPHS[name]()
    want, k = oracle.seq_ff(rp, ci)
    got = oracle.omp_rsoc(rp, ci, tie=tie, threads=1)
    assert np.array_equal(got["colors"], want) and got["K"] == k
    assert got["rounds"] == 0 and got["conflicts"] == 0


@pytest.mark.parametrize("threads", [2, 4, 8])
@pytest.mark.parametrize("name", ["tri_grid_perm", "rmat13", "lattice30", "K9", "star"])
def test_threads_give_valid_colourings(name, threads):
    rp, ci = GRAPHS[name]()
    for tie in ("lower", "higher"):
        got = oracle.omp_rsoc(rp, ci, tie=tie, threads=threads)
        assert oracle.check(rp, ci, got["colors"]) == 0
        assert got["K"] <= int(np.diff(rp).max()) + 1
