"""Pins for the CPU oracle: facts fixed by the paper or by mathematics, checked
against the oracle without using the oracle to produce the expectation.

Each pin takes an oracle object ``O`` (the default build, or a deliberately
broken copy in the mutation tests) and raises AssertionError on a mismatch.

Sources of the expected values:
* closed forms derived by hand (paths, cycles, grids, cliques, stars,
  complete bipartite graphs) for Algorithm 1 (Section 2.1) and for the
  round-synchronous Algorithm 3 (Section 3);
* worked examples derived round by round (tests/golden/);
* the paper's Figure 7 graph (Section 5);
* networkx's greedy colouring, an independent First-Fit implementation;
* brute-force chromatic numbers on graphs of at most 10 vertices;
* the Delta+1 bound (Section 2.1) and c(v) <= deg(v);
* reversal symmetry between the two tie rules and strict shrinking of |L|
  (every round at least the extreme-id recoloured vertex settles).
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _deg(rp):
    return np.diff(np.asarray(rp))


def _valid(rp, ci, c):
    rp = np.asarray(rp)
    ci = np.asarray(ci)
    src = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    keep = src != ci
    return not np.any(c[src[keep]] == c[ci[keep]])


def chromatic_number(n, edges):
    """Brute force: smallest k admitting a proper colouring (backtracking)."""
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    if n == 0:
        return 0
    order = sorted(range(n), key=lambda v: -len(adj[v]))
    for k in range(1, n + 1):
        col = {}

        def bt(i):
            if i == n:
                return True
            v = order[i]
            used = {col[u] for u in adj[v] if u in col}
            for c in range(k):
                if c not in used:
                    col[v] = c
                    if bt(i + 1):
                        return True
                    del col[v]
            return False

        if bt(0):
            return k
    return n


def _edges_of(rp, ci):
    rp = np.asarray(rp)
    out = []
    for v in range(len(rp) - 1):
        for u in ci[rp[v]:rp[v + 1]]:
            if u > v:
                out.append((v, int(u)))
    return out


def _small_graphs(count, seed, nmax=10):
    rng = np.random.default_rng(seed)
    for i in range(count):
        n = int(rng.integers(1, nmax + 1))
        p = float(rng.uniform(0.1, 0.9))
        yield gg.random_gnp(n, p, int(rng.integers(1 << 30)))


# ------------------------------------------------------------ Algorithm 1

def pin_seq_closed_forms(O):
    for n in (1, 2, 3, 7, 100):
        c, K = O.seq_ff(*gg.path(n))
        assert list(c) == [v % 2 for v in range(n)], ("path", n)
    for n in (4, 6, 50):
        c, K = O.seq_ff(*gg.cycle(n))
        assert list(c) == [v % 2 for v in range(n)] and K == 2, ("even cycle", n)
    for n in (3, 5, 51):
        c, K = O.seq_ff(*gg.cycle(n))
        assert list(c) == [v % 2 for v in range(n - 1)] + [2] and K == 3, ("odd cycle", n)
    for W, H in ((1, 1), (5, 4), (17, 9)):
        c, K = O.seq_ff(*gg.grid4(W, H))
        want = [(r + q) % 2 for r in range(H) for q in range(W)]
        assert list(c) == want, ("grid4", W, H)
    for n in (1, 2, 6, 20):
        c, K = O.seq_ff(*gg.complete(n))
        assert list(c) == list(range(n)) and K == n, ("K_n", n)
    c, K = O.seq_ff(*gg.star(7, centre_first=True))
    assert list(c) == [0] + [1] * 7
    c, K = O.seq_ff(*gg.star(7, centre_first=False))
    assert list(c) == [0] * 7 + [1]
    c, K = O.seq_ff(*gg.complete_bipartite(4, 4))
    assert list(c) == [0] * 4 + [1] * 4 and K == 2


def pin_seq_golden_tri_grid(O):
    g = _load("seq_ff_tri_grid_6x3.json")
    rp, ci = gg.tri_grid(g["W"], g["H"])
    c, K = O.seq_ff(rp, ci)
    assert np.array_equal(c.reshape(g["H"], g["W"]), np.array(g["colors_by_row"]))
    assert K == g["K"]


def pin_seq_networkx(O):
    import networkx as nx

    def check(rp, ci):
        G = nx.Graph()
        n = len(rp) - 1
        G.add_nodes_from(range(n))
        G.add_edges_from(_edges_of(rp, ci))
        want = nx.greedy_color(G, strategy=lambda g, colors: sorted(g.nodes()))
        c, K = O.seq_ff(rp, ci)
        assert [want[v] for v in range(n)] == list(c)

    for rp, ci in _small_graphs(60, 7, nmax=40):
        check(rp, ci)
    check(*gg.tri_grid(12, 9, permute_seed=3))
    check(*gg.rmat(8, 8, seed=11, shuffle_seed=5))


def pin_seq_bounds_and_bruteforce(O):
    for rp, ci in _small_graphs(80, 11, nmax=10):
        n = len(rp) - 1
        c, K = O.seq_ff(rp, ci)
        d = _deg(rp)
        assert _valid(rp, ci, c)
        assert np.all(c <= d) and np.all(c >= 0)
        assert K <= (d.max() if n else 0) + 1
        assert chromatic_number(n, _edges_of(rp, ci)) <= K


def pin_seq_some_order_is_optimal(O):
    """For <= 7 vertices some visiting order makes First-Fit optimal."""
    for rp, ci in _small_graphs(12, 13, nmax=7):
        n = len(rp) - 1
        chi = chromatic_number(n, _edges_of(rp, ci))
        best = n + 1
        for perm in itertools.permutations(range(n)):
            r2, c2 = gg.relabel(rp, ci, perm)
            best = min(best, O.seq_ff(r2, c2)[1])
        assert best == chi


# ------------------------------------------------------------ Algorithm 3

def _res(r):
    return list(r["colors"]), r["rounds"], list(r["L_sizes"])


def pin_rsync_fig7(O):
    g = _load("fig7_two_vertex.json")
    rp, ci = gg.from_edges(g["n"], g["edges"])
    for tie, key in (("lower", "lower_keeps"), ("higher", "higher_keeps")):
        r = O.rsync(rp, ci, tie=tie)
        assert _res(r) == (g[key]["colors"], g[key]["rounds"], g[key]["L_sizes"]), tie
    # without the id test the two endpoints flip together until the guard trips
    for passes, state in g["no_id_test"]["state_after_pass"].items():
        r = O.rsync(rp, ci, tie="none", max_rounds=int(passes), raise_on_noconv=False)
        assert r["status"] == -7 and list(r["colors"]) == state, passes


def pin_rsync_worked_examples(O):
    for case in _load("rsync_worked_examples.json")["cases"]:
        rp, ci = gg.from_edges(case["n"], case["edges"])
        for tie, key in (("lower", "lower_keeps"), ("higher", "higher_keeps")):
            if key not in case:
                continue
            r = O.rsync(rp, ci, tie=tie)
            want = case[key]
            assert _res(r) == (want["colors"], want["rounds"], want["L_sizes"]), (case["name"], tie)


def pin_rsync_closed_forms(O):
    for n in (2, 3, 10, 257):
        r = O.rsync(*gg.path(n), tie="lower")
        assert list(r["colors"]) == [v % 2 for v in range(n)]
        assert r["rounds"] == n - 1 and list(r["L_sizes"]) == [n - k for k in range(1, n)]
        assert r["conflicts"] == n * (n - 1) // 2
    for n in (2, 9, 40):
        r = O.rsync(*gg.complete(n), tie="lower")
        assert list(r["colors"]) == list(range(n)) and r["rounds"] == n - 1
        r = O.rsync(*gg.complete(n), tie="higher")
        assert list(r["colors"]) == list(range(n - 1, -1, -1))
    # empty graph, isolated vertices: colour 0, nothing to recolour
    r = O.rsync(np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert r["K"] == 0 and r["rounds"] == 0
    r = O.rsync(np.zeros(6, np.int32), np.zeros(0, np.int32))
    assert list(r["colors"]) == [0] * 5 and r["K"] == 1 and r["rounds"] == 0


def pin_rsync_first_round(O):
    """Round 0 leaves every vertex at colour 0, so round 1 moves exactly the vertices
    that have a neighbour they lose to, each to mex{0} = 1."""
    for rp, ci in list(_small_graphs(30, 17, nmax=30)) + [gg.tri_grid(9, 7, permute_seed=2)]:
        n = len(rp) - 1
        src = np.repeat(np.arange(n), np.diff(rp))
        for tie in ("lower", "higher"):
            lose = (ci < src) if tie == "lower" else (ci > src)
            has = np.zeros(n, bool)
            has[src[lose]] = True
            r = O.rsync(rp, ci, tie=tie, max_rounds=1, raise_on_noconv=False)
            assert list(r["colors"]) == list(has.astype(np.int32)), tie
            if has.any():
                assert r["status"] == -7 and list(r["L_sizes"]) == [int(has.sum())]


def pin_rsync_invariants(O):
    graphs = list(_small_graphs(60, 19, nmax=40))
    graphs += [gg.tri_grid(15, 11), gg.tri_grid(15, 11, permute_seed=9), gg.rmat(9, 8, seed=3, shuffle_seed=4)]
    for rp, ci in graphs:
        n = len(rp) - 1
        d = _deg(rp)
        for tie in ("lower", "higher"):
            r = O.rsync(rp, ci, tie=tie)
            c = r["colors"]
            assert _valid(rp, ci, c) and np.all(c >= 0) and np.all(c <= d)
            assert r["K"] <= (d.max() if n else 0) + 1
            L = list(r["L_sizes"])
            assert all(a > b for a, b in zip(L, L[1:])), L
            assert r["rounds"] <= max(n - 1, 0)
            assert r["conflicts"] == sum(L)


def pin_rsync_reversal(O):
    """higher-keeps on G equals lower-keeps on G relabelled by v -> n-1-v, read back."""
    graphs = list(_small_graphs(60, 23, nmax=30)) + [gg.tri_grid(13, 8), gg.rmat(8, 8, seed=5, shuffle_seed=6)]
    for rp, ci in graphs:
        n = len(rp) - 1
        rev = np.arange(n - 1, -1, -1)
        r2, c2 = gg.relabel(rp, ci, rev)
        hi = O.rsync(rp, ci, tie="higher")
        lo = O.rsync(r2, c2, tie="lower")
        assert np.array_equal(hi["colors"], lo["colors"][rev])
        assert list(hi["L_sizes"]) == list(lo["L_sizes"])


# ------------------------------------------------------------ Algorithm 2

def pin_cat_examples(O):
    rp, ci = gg.from_edges(2, [(0, 1)])
    r = O.cat(rp, ci, tie="lower")
    assert list(r["colors"]) == [0, 1] and r["rounds"] == 2 and list(r["L_sizes"]) == [1, 0]
    rp, ci = gg.cycle(4)
    r = O.cat(rp, ci, tie="lower")
    assert list(r["colors"]) == [0, 1, 0, 2] and r["rounds"] == 3 and list(r["L_sizes"]) == [3, 2, 0]
    for rp, ci in _small_graphs(40, 29, nmax=30):
        d = _deg(rp)
        for tie in ("lower", "higher"):
            r = O.cat(rp, ci, tie=tie)
            assert _valid(rp, ci, r["colors"]) and np.all(r["colors"] <= d)


# ------------------------------------------------------------ checker

def pin_check(O):
    rp, ci = gg.cycle(5)
    assert O.check(rp, ci, np.array([0, 1, 0, 1, 2], np.int32)) == 0
    assert O.check(rp, ci, np.array([0, 1, 0, 1, 0], np.int32)) > 0   # edge 4-0
    assert O.check(rp, ci, np.array([0, 1, 0, 1, 3], np.int32)) > 0   # 3 > deg 2
    assert O.check(rp, ci, np.array([0, 1, 0, 1, -1], np.int32)) > 0


# ------------------------------------------------------------ colour classes

def pin_classes_golden(O):
    g = _load("colour_classes_example.json")
    c = np.array(g["colors"], np.int32)
    for key, K in (("K3", 3), ("K5", 5)):
        ptr, vtx = O.classes(c, K)
        assert ptr.tolist() == g[key]["ptr"] and vtx.tolist() == g[key]["vtx"], key


def pin_classes_library(O):
    """Class k = the vertices of colour k in ascending id is exactly a stable
    sort of the ids by colour; the starts are the running sums of a bincount."""
    rng = np.random.default_rng(1505)
    for n, K in ((1, 1), (2, 1), (17, 3), (1000, 7), (4096, 300), (5000, 5000)):
        c = rng.integers(0, K, size=n).astype(np.int32)
        ptr, vtx = O.classes(c, K)
        assert np.array_equal(vtx, np.argsort(c, kind="stable").astype(np.int32))
        want = np.concatenate([[0], np.cumsum(np.bincount(c, minlength=K))])
        assert np.array_equal(ptr, want.astype(np.int32))
    ptr, vtx = O.classes(np.zeros(0, np.int32), 4)
    assert ptr.tolist() == [0, 0, 0, 0, 0] and len(vtx) == 0


def pin_classes_independent_sets(O):
    """On valid colourings every class is an independent set and the classes
    partition V."""
    for rp, ci in _small_graphs(40, seed=77, nmax=40):
        n = len(rp) - 1
        c, K = O.seq_ff(rp, ci)
        ptr, vtx = O.classes(c, K)
        assert ptr[0] == 0 and ptr[-1] == n and sorted(vtx.tolist()) == list(range(n))
        for k in range(K):
            members = vtx[ptr[k]:ptr[k + 1]]
            assert np.all(np.diff(members) > 0) and np.all(c[members] == k)
            s = set(members.tolist())
            for v in members:
                assert not any(int(u) in s for u in ci[rp[v]:rp[v + 1]] if u != v)


def pin_classes_range(O):
    for bad in ([0, 3, 1], [0, -1, 1]):
        try:
            O.classes(np.array(bad, np.int32), 3)
        except ValueError:
            continue
        raise AssertionError("colour outside [0, K) accepted: %s" % bad)


# ------------------------------------------------------------ recolouring after edits

def _csr_from_edges(n, edges):
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum([len(x) for x in adj])
    ci = np.array([u for x in adj for u in sorted(x)], np.int32)
    return rp, ci


def pin_recolor_worked_examples(O):
    g = _load("recolor_worked_examples.json")
    for case in g["cases"]:
        rp, ci = _csr_from_edges(case["n"], case["edges"])
        for tie, key in (("lower", "lower_keeps"), ("higher", "higher_keeps")):
            r = O.recolor(rp, ci, np.array(case["prev"], np.int32), case["touched"], tie=tie)
            w = case[key]
            assert r["colors"].tolist() == w["colors"] and r["rounds"] == w["rounds"], (case["name"], tie)
            assert r["L_sizes"].tolist() == w["L_sizes"], (case["name"], tie)


def pin_recolor_reduces_to_rsync(O):
    """From all colours 0 with every vertex touched, the recolouring is the
    round-synchronous schedule itself (its round 0 is that state)."""
    graphs = list(_small_graphs(30, seed=91, nmax=12)) + [gg.cycle(6), gg.complete(5), gg.path(7)]
    for rp, ci in graphs:
        n = len(rp) - 1
        for tie in ("lower", "higher"):
            want = O.rsync(rp, ci, tie=tie)
            r = O.recolor(rp, ci, np.zeros(n, np.int32), np.arange(n), tie=tie)
            assert np.array_equal(r["colors"], want["colors"]) and r["rounds"] == want["rounds"]
            assert np.array_equal(r["L_sizes"], want["L_sizes"])


def pin_recolor_from_uncoloured(O):
    """From no colours at all, the first pass gives everyone colour 0 (every
    vertex is defective and sees no coloured neighbour); the rest is the
    round-synchronous schedule."""
    for rp, ci in _small_graphs(30, seed=92, nmax=12):
        n = len(rp) - 1
        want = O.rsync(rp, ci)
        r = O.recolor(rp, ci, np.full(n, -1, np.int32), [])
        assert np.array_equal(r["colors"], want["colors"]) and r["rounds"] == want["rounds"] + 1
        assert r["L_sizes"].tolist() == [n] + want["L_sizes"].tolist()


def pin_recolor_edits(O):
    """Random edge insertions into validly coloured graphs: the result is a
    valid colouring within the First-Fit bound, only recoloured vertices
    change, and a valid colouring with nothing touched is left alone."""
    rng = np.random.default_rng(93)
    for rp, ci in _small_graphs(40, seed=94, nmax=30):
        n = len(rp) - 1
        prev, _ = O.seq_ff(rp, ci)
        same = O.recolor(rp, ci, prev, [])
        assert np.array_equal(same["colors"], prev) and same["rounds"] == 0
        edges = {(int(a), int(b)) for a in range(n) for b in ci[rp[a]:rp[a + 1]] if a < b}
        add = [(int(a), int(b)) for a, b in rng.integers(0, n, size=(3, 2)) if a != b]
        edges |= {(min(a, b), max(a, b)) for a, b in add}
        rp2, ci2 = _csr_from_edges(n, sorted(edges))
        touched = [x for e in add for x in e]
        for tie in ("lower", "higher"):
            r = O.recolor(rp2, ci2, prev, touched, tie=tie)
            assert _valid(rp2, ci2, r["colors"]) and np.all(r["colors"] <= np.diff(rp2))
            assert int(np.sum(r["colors"] != prev)) <= r["conflicts"]


def pin_recolor_range(O):
    rp, ci = gg.path(4)
    try:
        O.recolor(rp, ci, np.zeros(4, np.int32), [4])
    except ValueError:
        return
    raise AssertionError("touched id outside [0, n) accepted")


# ------------------------------------------------------------ distance-2 (the square G^2)

def _within2(rp, ci, v):
    """Vertices at distance 1 or 2 from v, by breadth-first search."""
    seen = {v: 0}
    frontier = [v]
    for depth in (1, 2):
        nxt = []
        for x in frontier:
            for u in ci[rp[x]:rp[x + 1]]:
                u = int(u)
                if u not in seen:
                    seen[u] = depth
                    nxt.append(u)
        frontier = nxt
    return sorted(u for u in seen if u != v)


def pin_square_bruteforce(O):
    for rp, ci in list(_small_graphs(40, seed=95, nmax=25)) + [gg.star(7), gg.grid4(5, 4), gg.tri_grid(6, 5)]:
        rp2, ci2 = O.square(rp, ci)
        for v in range(len(rp) - 1):
            assert ci2[rp2[v]:rp2[v + 1]].tolist() == _within2(rp, ci, v), v


def pin_square_closed_forms(O):
    n = 9
    rp, ci = gg.path(n)
    rp2, ci2 = O.square(rp, ci)
    for v in range(n):
        assert ci2[rp2[v]:rp2[v + 1]].tolist() == [u for u in range(v - 2, v + 3) if 0 <= u < n and u != v]
    rp, ci = gg.cycle(n)
    rp2, ci2 = O.square(rp, ci)
    for v in range(n):
        assert ci2[rp2[v]:rp2[v + 1]].tolist() == sorted((v + d) % n for d in (-2, -1, 1, 2))
    rp, ci = gg.star(5)  # centre 0 and 5 leaves: G^2 is K6
    rp2, ci2 = O.square(rp, ci)
    assert np.diff(rp2).tolist() == [5] * 6
    # distance-2 First-Fit in id order: a path gets v mod 3, a star's leaves all differ
    c, K = O.seq_ff(*[np.asarray(x, np.int32) for x in O.square(*gg.path(10))])
    assert c.tolist() == [v % 3 for v in range(10)] and K == 3
    c, K = O.seq_ff(*[np.asarray(x, np.int32) for x in O.square(*gg.star(5))])
    assert c.tolist() == list(range(6)) and K == 6


def pin_square_colouring_valid(O):
    """A colouring of G^2 separates every pair within distance 2 in G."""
    for rp, ci in _small_graphs(20, seed=96, nmax=30):
        rp2, ci2 = O.square(rp, ci)
        for tie in ("lower", "higher"):
            c = O.rsync(rp2.astype(np.int32), ci2, tie=tie)["colors"]
            for v in range(len(rp) - 1):
                assert all(c[u] != c[v] for u in _within2(rp, ci, v))


ALL_PINS = [pin_seq_closed_forms, pin_seq_golden_tri_grid, pin_seq_networkx, pin_seq_bounds_and_bruteforce,
            pin_seq_some_order_is_optimal, pin_rsync_fig7, pin_rsync_worked_examples, pin_rsync_closed_forms,
            pin_rsync_first_round, pin_rsync_invariants, pin_rsync_reversal, pin_cat_examples, pin_check,
            pin_classes_golden, pin_classes_library, pin_classes_independent_sets, pin_classes_range,
            pin_recolor_worked_examples, pin_recolor_reduces_to_rsync, pin_recolor_from_uncoloured,
            pin_recolor_edits, pin_recolor_range, pin_square_bruteforce, pin_square_closed_forms,
            pin_square_colouring_valid]
