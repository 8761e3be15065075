#!/usr/bin/env python3
"""Benchmark: speculative First-Fit colouring throughput on one MI355X.

A step is one full colouring (round 0, the detect-and-recolour rounds until
the worklist is empty, and the colour count) of one synthetic graph that is
already resident in HBM, through the C ABI.  The metric is undirected edges
coloured per second (GE/s); the colours used are reported beside sequential
First-Fit's.

Workloads (--workload):
  mesh3d  (default) 200^3 lattice, 26-neighbour stencil, ids permuted by seed
          (8,000,000 vertices, 102,923,596 edges)
  rmat    R-MAT scale 22, edge factor 16, a,b,c = .57,.19,.19, symmetrised,
          self-loops and duplicates dropped, ids shuffled
  mesh2d  100 x 100 triangulated grid, natural ids
  batched 4096 grids / random geometric graphs, 1e3..1e6 vertices, one batch
  served  Poisson request stream through the continuous-batching pool

The JSON line also carries the dominant kernel's roofline (algorithmic bytes
per launch over its HIP-event duration, against 8 TB/s HBM) and the CPU
oracle timed on this host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak


# sources the round kernels and their launch shapes are built from, for the
# single-graph workloads and for the batch (the figures in
# profiles/traffic.json stay valid while the code in these is unchanged)
SINGLE_KERNEL_SOURCES = ("device_common.hpp", "vertex_ops.hpp", "single_kernels.hpp", "single.hpp", "host_common.hpp",
                         "hub_kernels.hpp")
ROUND_KERNEL_SOURCES = SINGLE_KERNEL_SOURCES + ("batch_kernels.hpp", "batch.hpp")


def _code_only(text: bytes) -> bytes:
    """C++ source without its comments and blank lines (what the compiler
    sees): a comment edit does not invalidate counters taken on the code."""
    out, i, n = bytearray(), 0, len(text)
    while i < n:
        if text.startswith(b"//", i):
            j = text.find(b"\n", i)
            i = n if j < 0 else j
        elif text.startswith(b"/*", i):
            j = text.find(b"*/", i + 2)
            i = n if j < 0 else j + 2
        elif text[i:i + 1] == b'"':  # string literal, copied whole
            j = i + 1
            while j < n and text[j:j + 1] != b'"':
                j += 2 if text[j:j + 1] == b"\\" else 1
            out += text[i:j + 1]
            i = j + 1
        else:
            out += text[i:i + 1]
            i += 1
    return b"\n".join(ln.rstrip() for ln in bytes(out).splitlines() if ln.strip())


def kernel_source_hash(workload: str = "mesh3d") -> str:
    """Hash of the code (comments and blank lines left out) the workload's
    round kernels are built from."""
    h = hashlib.sha1()
    d = os.path.join(ROOT, "paper_1505_04086_amd", "csrc")
    for f in (ROUND_KERNEL_SOURCES if workload == "batched" else SINGLE_KERNEL_SOURCES):
        h.update(_code_only(open(os.path.join(d, f), "rb").read()))
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel: str, options=None):
    """HBM traffic per launch measured with rocprofv3 counters, if it was taken
    for the current kernel sources (and, where recorded, the same launch
    options), else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except Exception:
        return None
    if rec.get("source_hashes", {}).get(workload) != kernel_source_hash(workload):
        return None
    ent = rec.get("workloads", {}).get(workload, {}).get(kernel)
    # one entry, or a list of entries taken with different launch options
    for e in (ent if isinstance(ent, list) else [ent]):
        if e is not None and e.get("options", options or {}) == (options or {}):
            return e.get("bytes_per_launch")
    return None


def make_graph(workload: str, seed: int, sample: bool = False):
    """The workload's graph; sample=True gives a smaller graph of the same
    kind (the bounded sample of a CPU baseline that would take minutes on the
    full graph)."""
    import graphgen as gg
    if workload == "mesh3d":
        S = 100 if sample else 200
        rp, ci = gg.lattice26(S, permute_seed=seed)
        desc = "lattice26 %d^3, ids permuted (seed %d)" % (S, seed)
    elif workload == "rmat":
        sc = 20 if sample else 22
        rp, ci = gg.rmat(sc, 16, 0.57, 0.19, 0.19, seed=seed, shuffle_seed=seed + 1)
        desc = "rmat scale %d ef 16 (.57,.19,.19,.05), symmetrised, ids shuffled (seed %d)" % (sc, seed)
    elif workload == "mesh2d":
        rp, ci = gg.tri_grid(100)
        desc = "triangulated grid 100x100, natural ids"
    else:
        raise ValueError(workload)
    return rp, ci, desc


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(rp, ci, budget_s: float = 12.0, workload: str = "mesh3d", seed: int = 1505, legs: bool = True):
    """CPU baselines on this host, all from oracle/ (never tuned for this):
    sequential First-Fit (Algorithm 1) on one core, repeated on the full graph
    until about budget_s seconds; the round-synchronous Algorithm 3 schedule on
    one core on a bounded sample of the workload; Algorithm 3 with OpenMP
    (live reads, as the paper runs it) on every core this process may use, in
    a child process started with OMP_PROC_BIND=close, on the full graph.
    Returns (baseline dict, sequential First-Fit colour count)."""
    import oracle
    E = len(ci) // 2
    reps, t_total = 0, 0.0
    while t_total < budget_s and reps < 50:
        t0 = time.perf_counter()
        _, kseq = oracle.seq_ff(rp, ci)
        t_total += time.perf_counter() - t0
        reps += 1
    out = {"value": E * reps / t_total / 1e9, "unit": "GE/s", "cores": 1, "kind": "oracle",
           "sample": "oracle sequential First-Fit (Algorithm 1) on the full graph, %d run(s), %.1f s" % (reps, t_total),
           "host_cores": host_cores()}
    if not legs:
        return out, kseq
    # round-synchronous schedule on one core, on a smaller graph of the same kind
    srp, sci, sdesc = make_graph(workload, seed, sample=True)
    t0 = time.perf_counter()
    r = oracle.rsync(srp, sci, tie="lower")
    ts = time.perf_counter() - t0
    out["rsync_1core"] = {"value": len(sci) // 2 / ts / 1e9, "unit": "GE/s", "cores": 1, "kind": "oracle",
                          "sample": "oracle round-synchronous Algorithm 3 on %s, one run, %.1f s" % (sdesc, ts),
                          "colors": r["K"], "rounds": r["rounds"], "conflicts": r["conflicts"]}
    # OpenMP Algorithm 3 on all cores (a child process: the OpenMP runtime
    # reads OMP_PROC_BIND when it starts)
    env = dict(os.environ, OMP_PROC_BIND="close", OMP_PLACES="cores")
    env.setdefault("OMP_NUM_THREADS", str(host_cores()))
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-omp-leg", "--workload", workload, "--seed", str(seed),
           "--cpu-budget", str(max(2.0, budget_s / 2))]
    res = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    if res.returncode == 0:
        out["omp_rsoc"] = json.loads(res.stdout.strip().splitlines()[-1])
    else:
        out["omp_rsoc"] = {"error": (res.stderr or "")[-400:]}
    return out, kseq


def cpu_omp_leg(args):
    """Child process of cpu_baseline: Algorithm 3 with OpenMP on the full
    workload graph, repeated until about args.cpu_budget seconds."""
    import oracle
    rp, ci, desc = make_graph(args.workload, args.seed)
    E = len(ci) // 2
    reps, t_total, r = 0, 0.0, None
    while t_total < args.cpu_budget and reps < 50:
        t0 = time.perf_counter()
        r = oracle.omp_rsoc(rp, ci, tie="lower")
        t_total += time.perf_counter() - t0
        reps += 1
    valid = oracle.check(rp, ci, r["colors"]) == 0
    print(json.dumps({"value": E * reps / t_total / 1e9, "unit": "GE/s", "cores": r["threads"], "kind": "oracle",
                      "sample": "Algorithm 3 with OpenMP (oracle/omp_rsoc.c, live reads) on %s, %d run(s), %.1f s, "
                                "OMP_PROC_BIND=%s" % (desc, reps, t_total, os.environ.get("OMP_PROC_BIND")),
                      "colors": r["K"], "rounds": r["rounds"], "conflicts": r["conflicts"], "valid": valid}))


def colouring_valid(rp, ci, col) -> bool:
    """Sanity check of a colouring the benchmark produced: every colour in
    [0, degree] and no edge joining equal colours (numpy, rows in slices)."""
    import numpy as np
    n = len(rp) - 1
    col = np.asarray(col)
    deg = np.diff(rp)
    if n == 0:
        return True
    if col.min() < 0 or np.any(col > deg):
        return False
    step = 1 << 22
    for v0 in range(0, n, step):
        v1 = min(n, v0 + step)
        src = np.repeat(np.arange(v0, v1, dtype=np.int32), deg[v0:v1])
        dst = ci[rp[v0]:rp[v1]]
        if np.any((col[src] == col[dst]) & (src != dst)):
            return False
    return True


def bench_distance2(args, rsoc, ctx, d_rp, d_ci, n, E, stream):
    import numpy as np
    import torch
    d_col = torch.empty(n, dtype=torch.int32, device=torch.device("cuda:0"))
    opts = rsoc.make_options(args.mode, "lower", distance=2)
    try:
        rsoc.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, opts, stream=stream)
    except rsoc.RsocError as e:  # 2-hop walks over the limit (hubs): not supported
        return {"supported": False, "status": e.code}
    reps = max(2, args.steps // 5)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k, st = rsoc.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, opts, stream=stream)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    # sampled check: every sampled vertex and its neighbours (pairwise within
    # distance 2) carry distinct colours
    col = d_col.cpu().numpy()
    rp, ci = d_rp.cpu().numpy(), d_ci.cpu().numpy()
    rng = np.random.default_rng(args.seed + 11)
    for w in rng.integers(0, n, size=min(n, 100000)):
        c = col[np.append(ci[rp[w]:rp[w + 1]], w)]
        if len(np.unique(c)) != len(c):
            raise SystemExit("bench: distance-2 colouring invalid around vertex %d" % w)
    return {"supported": True, "ms": t * 1e3, "GEps_of_G": E / t / 1e9, "colors": k, "rounds": st["rounds"],
            "max_degree_G2": st["max_degree"], "colouring_ms_device": st["ms"],
            "check": "100000 sampled vertices: each with its neighbours all distinct"}


def insert_edges(rp, ci, add):
    """CSR with the edges `add` (pairs, no duplicates of existing edges, no
    self-loops) inserted at the ends of their rows."""
    import numpy as np
    n = len(rp) - 1
    a = np.concatenate([add[:, 0], add[:, 1]])
    b = np.concatenate([add[:, 1], add[:, 0]])
    extra = np.bincount(a, minlength=n)
    rp2 = np.zeros(n + 1, np.int64)
    rp2[1:] = np.cumsum(np.diff(rp) + extra)
    ci2 = np.empty(int(rp2[-1]), np.int32)
    shift = np.concatenate([[0], np.cumsum(extra)[:-1]])  # inserted entries in rows before each row
    row = np.repeat(np.arange(n, dtype=np.int32), np.diff(rp))
    ci2[np.arange(len(ci), dtype=np.int64) + shift[row]] = ci
    order = np.argsort(a, kind="stable")
    a, b = a[order], b[order]
    first = np.searchsorted(a, a)  # rank of each inserted entry inside its row
    ci2[rp2[a + 1] - extra[a] + (np.arange(len(a)) - first)] = b
    return rp2.astype(np.int32), ci2


def bench_recolor(args, rsoc, ctx, rp, ci, col, stream, full_s, edits=10000):
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    n = len(rp) - 1
    rng = np.random.default_rng(args.seed + 7)
    pairs = rng.integers(0, n, size=(edits * 2, 2))
    pairs = np.unique(np.sort(pairs[pairs[:, 0] != pairs[:, 1]], axis=1), axis=0)
    # drop pairs that are edges already (a row is at most a few dozen entries here)
    present = np.array([p[1] in ci[rp[p[0]]:rp[p[0] + 1]] for p in pairs], bool)
    add = pairs[~present][:edits]
    rp2, ci2 = insert_edges(rp, ci, add)
    touched = np.unique(add.ravel()).astype(np.int32)
    d_rp, d_ci = torch.from_numpy(rp2).to(dev), torch.from_numpy(ci2).to(dev)
    d_t = torch.from_numpy(touched).to(dev)
    d_prev = torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).to(dev)
    d_col = torch.empty_like(d_prev)
    opts = rsoc.make_options(args.mode, "lower")
    d_col.copy_(d_prev)
    rsoc.rsoc_recolor_device(ctx, d_rp, d_ci, n, d_col, d_t, opts, stream=stream)
    reps = max(3, args.steps // 2)
    times = []
    for _ in range(reps):
        d_col.copy_(d_prev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k, st = rsoc.rsoc_recolor_device(ctx, d_rp, d_ci, n, d_col, d_t, opts, stream=stream)
        times.append(time.perf_counter() - t0)
    got = d_col.cpu().numpy()
    if not colouring_valid(rp2, ci2, got):
        raise SystemExit("bench: invalid colouring after recolouring")
    t = float(np.median(times))
    return {"inserted_edges": int(len(add)), "touched": int(len(touched)), "worklist0": st["worklist0"],
            "recoloured": st["conflicts"], "rounds": st["rounds"], "colors": k, "ms": t * 1e3,
            "full_colouring_ms": full_s * 1e3, "speedup_vs_full": full_s / t,
            "changed": int(np.sum(got != col))}


def bench_single(args):
    import numpy as np
    import torch

    import paper_1505_04086_amd as rsoc

    dev = torch.device("cuda:0")
    t = time.perf_counter()
    rp, ci, desc = make_graph(args.workload, args.seed)
    n = len(rp) - 1
    E = len(ci) // 2
    gen_s = time.perf_counter() - t
    print("[bench] %s: n=%d |E|=%d (generated in %.1f s)" % (desc, n, E, gen_s), file=sys.stderr, flush=True)
    d_rp = torch.from_numpy(rp).to(dev)
    d_ci = torch.from_numpy(ci).to(dev)
    d_col = torch.empty(n, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    ctx = rsoc.Context(0)
    stream = torch.cuda.current_stream()
    opts = rsoc.make_options(args.mode, "lower", timing=1)

    def step():
        return rsoc.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, opts, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        k, st = step()
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    print("[bench] %d steps in %.3f s" % (args.steps, elapsed), file=sys.stderr, flush=True)
    col = d_col.cpu().numpy()
    valid = colouring_valid(rp, ci, col)
    if not valid:
        raise SystemExit("bench: invalid colouring produced")

    ms_dev = float(np.median([s["ms"] for s in stats]))
    # dominant kernel: the larger of the two full-graph launches (round 0 / round 1)
    r0 = float(np.mean([s["ms_round0"] for s in stats]))
    r1 = float(np.mean([s["ms_round1"] for s in stats]))
    st = stats[-1]
    if r1 >= r0 or args.mode != "optimistic":
        kname, kms, kbytes = "round1_detect_recolour", r1, st["bytes_round1"]
        kbytes_lib = kbytes
    else:
        kname, kms = "round0_first_fit", r0
        # round-0 bytes as the method defines the round: row_ptr, every
        # adjacency entry and the colour it names, one colour write per vertex
        kbytes = 4 * (n + 1) + 8 * len(ci) + 4 * n
        # the library's own count of what its pruned round 0 must move (each
        # edge's colour read from one end only, plus the bins and U^0)
        kbytes_lib = st["bytes_round0"]
    achieved = kbytes / (kms * 1e-3) / 1e9
    traffic = load_traffic(args.workload, kname)

    out = {
        "metric": "edges colored/s (GE/s) + colors used",
        "value": E * args.steps / elapsed / 1e9,
        "unit": "GE/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "edges": E, "nnz": len(ci), "mode": args.mode, "tie": "lower",
                   "max_degree": st["max_degree"]},
        "colors": st["colors"],
        "colors_distinct": st["colors_distinct"],
        "chunk": st["chunk"],
        "rounds": st["rounds"],
        "conflicts": st["conflicts"],
        "worklist0": st["worklist0"],
        "device_ms_median": ms_dev,
        "device_GEps": E / (ms_dev * 1e-3) / 1e9,
        "alg_bytes_per_step": st["alg_bytes"],
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel_ms": kms, "alg_bytes_per_launch": kbytes,
                     "library_bytes_per_launch": kbytes_lib,
                     "frac_library_bytes": kbytes_lib / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        # the launch after round 0 (the masked first worklist round by default),
        # with the library's count of the bytes it must move
        "round1": {"kernel_ms": r1, "alg_bytes_per_launch": st["bytes_round1"],
                   "traffic": load_traffic(args.workload, "round1_detect_recolour")},
    }
    if not args.no_extras:
        # colour classes of the colouring just made (its independent sets, one per
        # colour, ids ascending): read colours, write ids and class starts
        K = st["colors"]
        d_ptr = torch.empty(K + 1, dtype=torch.int32, device=dev)
        d_vtx = torch.empty(n, dtype=torch.int32, device=dev)
        rsoc.rsoc_color_classes(ctx, d_col, n, K, d_ptr, d_vtx, stream=stream)
        torch.cuda.synchronize()
        reps = max(3, args.steps // 2)
        tc = time.perf_counter()
        for _ in range(reps):
            rsoc.rsoc_color_classes(ctx, d_col, n, K, d_ptr, d_vtx, stream=stream)
        torch.cuda.synchronize()
        tc = (time.perf_counter() - tc) / reps
        ptr, vtx = d_ptr.cpu().numpy(), d_vtx.cpu().numpy()
        if not (ptr[0] == 0 and ptr[-1] == n and np.all(np.diff(ptr) >= 0)
                and np.all(col[vtx] == np.repeat(np.arange(K), np.diff(ptr)))):
            raise SystemExit("bench: colour classes inconsistent with the colouring")
        cls_bytes = 8 * n + 4 * (K + 1)
        out["color_classes"] = {"ms": tc * 1e3, "classes": K, "alg_bytes": cls_bytes,
                                "GBps": cls_bytes / tc / 1e9, "frac_hbm": cls_bytes / tc / 1e9 / HBM_PEAK_GBS}
        # distance-2 colouring of the same graph (G^2 built on the device, then
        # the same rounds); timed end to end, the build of G^2 included
        # (an extra that fails is recorded with its error beside the headline
        # figures, which are already measured)
        try:
            out["distance2"] = bench_distance2(args, rsoc, ctx, d_rp, d_ci, n, E, stream)
        except rsoc.RsocError as e:
            out["distance2"] = {"error": str(e)}
            print("[bench] distance-2 colouring failed: %s" % e, file=sys.stderr, flush=True)
        # recolouring after topology edits: random edges inserted (both endpoints
        # touched), starting from the colouring just made
        try:
            out["recolor_after_edits"] = bench_recolor(args, rsoc, ctx, rp, ci, col, stream, elapsed / args.steps)
        except rsoc.RsocError as e:
            out["recolor_after_edits"] = {"error": str(e)}
            print("[bench] recolouring after edits failed: %s" % e, file=sys.stderr, flush=True)
        if args.mode == "optimistic":
            # the literal reading (round 0 over all neighbours, round 1 over all of V)
            o3 = rsoc.make_options("optimistic", "lower", timing=1, full_sweep=1)
            rsoc.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, o3, stream=stream)
            torch.cuda.synchronize()
            tf = time.perf_counter()
            reps = max(1, args.steps // 4)
            for _ in range(reps):
                kf, sf = rsoc.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, o3, stream=stream)
            torch.cuda.synchronize()
            tf = (time.perf_counter() - tf) / reps
            out["full_sweep"] = {"GEps": E / tf / 1e9, "colors": kf, "rounds": sf["rounds"], "conflicts": sf["conflicts"],
                                 "ms_round0": sf["ms_round0"], "ms_round1": sf["ms_round1"]}
            if not colouring_valid(rp, ci, d_col.cpu().numpy()):
                raise SystemExit("bench: invalid colouring produced (full sweep)")
    if (args.det_too or not args.no_extras) and args.mode == "optimistic":
        # the paper's comparison (Section 4, Table 1): Algorithm 3 (R) and its
        # predecessor Algorithm 2 (C) on the same graph, round-synchronously
        # and with live reads -- recolouring rounds ("iterations"), conflicts,
        # colours
        comp = {}
        for name in ("deterministic", "two_phase", "two_phase_live"):
            o2 = rsoc.make_options(name, "lower", timing=0)
            rsoc.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, o2, stream=stream)
            torch.cuda.synchronize()
            reps = 3
            td = time.perf_counter()
            for _ in range(reps):
                kd, sd = rsoc.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, o2, stream=stream)
            torch.cuda.synchronize()
            td = (time.perf_counter() - td) / reps
            if not colouring_valid(rp, ci, d_col.cpu().numpy()):
                raise SystemExit("bench: invalid colouring produced (%s)" % name)
            comp[name] = {"GEps": E / td / 1e9, "ms": td * 1e3, "colors": kd, "rounds": sd["rounds"],
                          "passes": sd["passes"], "conflicts": sd["conflicts"], "device_ms": sd["ms"]}
        out["deterministic"] = comp["deterministic"]
        out["two_phase"] = comp["two_phase"]
        # with live reads, beside Algorithm 3's literal flow (full_sweep) and
        # its default flow: the paper's own comparison
        out["two_phase_live"] = comp["two_phase_live"]
    if not args.no_cpu:
        cb, kseq = cpu_baseline(rp, ci, args.cpu_budget, args.workload, args.seed)
        out["cpu_baseline"] = cb
        out["colors_seq_first_fit"] = kseq
    ctx.close()
    return out


def bench_rmat_extra(args):
    """The power-law workload beside the headline: R-MAT scale 22 (ids
    shuffled), optimistic mode, throughput and colours against sequential
    First-Fit (timed once on one core: the CPU leg of this workload), with
    the hub-first round 0 (default) and without it."""
    import numpy as np
    import torch

    import oracle
    import paper_1505_04086_amd as rsoc

    dev = torch.device("cuda:0")
    rp, ci, desc = make_graph("rmat", args.seed)
    n, E = len(rp) - 1, len(ci) // 2
    d_rp, d_ci = torch.from_numpy(rp).to(dev), torch.from_numpy(ci).to(dev)
    d_col = torch.empty(n, dtype=torch.int32, device=dev)
    ctx = rsoc.Context(0)
    stream = torch.cuda.current_stream()
    res = {"workload": desc, "n": n, "edges": E}
    for name, hf in (("hub_first", 0), ("hub_first_off", -1)):
        opts = rsoc.make_options("optimistic", "lower", hub_first=hf)
        for _ in range(2):
            rsoc.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, opts, stream=stream)
        torch.cuda.synchronize()
        reps, ks, sts = 5, [], []
        t0 = time.perf_counter()
        for _ in range(reps):
            k, st = rsoc.rsoc_color_device(ctx, d_rp, d_ci, n, d_col, opts, stream=stream)
            ks.append(k)
            sts.append(st)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        if not colouring_valid(rp, ci, d_col.cpu().numpy()):
            raise SystemExit("bench: invalid R-MAT colouring (%s)" % name)
        res[name] = {"GEps": E / el / 1e9, "ms": el * 1e3, "colors": ks, "colors_distinct": sts[-1]["colors_distinct"],
                     "rounds": sts[-1]["rounds"], "conflicts": sts[-1]["conflicts"],
                     "device_ms_median": float(np.median([x["ms"] for x in sts]))}
    t0 = time.perf_counter()
    _, kseq = oracle.seq_ff(rp, ci)
    ts = time.perf_counter() - t0
    res["colors_seq_first_fit"] = kseq
    res["cpu_baseline"] = {"value": E / ts / 1e9, "unit": "GE/s", "cores": 1, "kind": "oracle",
                           "sample": "oracle sequential First-Fit on the full graph, one run, %.1f s" % ts}
    res["colors_within_seq_plus_1"] = max(res["hub_first"]["colors"]) <= kseq + 1
    ctx.close()
    return res


def _pinned(a):
    import torch
    return torch.from_numpy(a).pin_memory()


def bench_batched(args):
    """Config: many independent grids / random geometric graphs in one batch;
    batched fused launches vs one call per graph on the same device-resident data."""
    import numpy as np
    import torch

    import graphgen as gg
    import paper_1505_04086_amd as rsoc

    dev = torch.device("cuda:0")
    t = time.perf_counter()
    b = gg.batch(args.batch_graphs, seed=args.seed, nmin=1e3, nmax=1e6, mean_degree=12.0)
    G = args.batch_graphs
    vo, no = b["vtx_off"], b["nnz_off"]
    E = int(no[-1]) // 2
    print("[bench] batch of %d graphs: %d vertices, %d edges (generated in %.1f s)"
          % (G, int(vo[-1]), E, time.perf_counter() - t), file=sys.stderr, flush=True)
    d_rp = torch.from_numpy(b["row_ptr_cat"]).to(dev)
    d_ci = torch.from_numpy(b["col_idx_cat"]).to(dev)
    d_col = torch.empty(int(vo[-1]), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    ctx = rsoc.Context(0)
    stream = torch.cuda.current_stream()
    tune_info = None
    tune_key = "batch-grids-rgg-1e3-1e6-deg12-%s" % args.mode
    if args.tune:
        from paper_1505_04086_amd import tune
        cached = tune.lookup(tune_key)
        if cached is not None:
            args.tuned = cached
            tune_info = {"options": cached, "from_cache": tune.tune_file()}
    if args.tune and tune_info is None:
        # autotune on a smaller batch drawn from the same distribution (another
        # seed); the result goes to the tuning cache, which later runs read
        from paper_1505_04086_amd import tune
        tb = gg.batch(args.tune_graphs, seed=args.seed + 1, nmin=1e3, nmax=1e6, mean_degree=12.0)
        t_rp = torch.from_numpy(tb["row_ptr_cat"]).to(dev)
        t_ci = torch.from_numpy(tb["col_idx_cat"]).to(dev)
        t_col = torch.empty(int(tb["vtx_off"][-1]), dtype=torch.int32, device=dev)
        tt = time.perf_counter()
        # grid_thread is left at its default: the batched sweeps claim their
        # tasks, so a grid beyond the resident workgroups only waits, and the
        # 256-graph sample is too small to rank grids for the full batch
        space = {k: tune.SPACE[k] for k in ("chunk", "t_thread", "lookahead", "rounds_per_sync", "small_cutoff")}
        best, best_t, trials = tune.coordinate_descent(
            lambda o: tune._timer(lambda: rsoc.rsoc_color_batch(ctx, tb["vtx_off"], tb["nnz_off"], t_rp, t_ci, t_col,
                                                                rsoc.make_options(args.mode, **o)), 3),
            space=space, sweeps=1)
        tune.save(tune_key, best, best_t * 1e3)
        args.tuned = tune.lookup(tune_key)
        tune_info = {"graphs": args.tune_graphs, "seconds": time.perf_counter() - tt, "trials": len(trials),
                     "best_ms": best_t * 1e3, "default_ms": trials[0][1] * 1e3, "options": args.tuned,
                     "cache": tune.tune_file()}
        print("[bench] tuned %s" % json.dumps(tune_info), file=sys.stderr, flush=True)
        del t_rp, t_ci, t_col
    opts = rsoc.make_options(args.mode, "lower", timing=1, **(args.tuned or {}))
    for _ in range(args.warmup):
        rsoc.rsoc_color_batch(ctx, vo, no, d_rp, d_ci, d_col, opts, stream=stream)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counts, kmax, st = rsoc.rsoc_color_batch(ctx, vo, no, d_rp, d_ci, d_col, opts, stream=stream)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    col = d_col.cpu().numpy()
    # validity of every 16th graph (host check; all of them would take longer than the run)
    bad = 0
    for g in range(0, G, 16):
        rp, ci = gg.batch_member(b, g)
        bad += not colouring_valid(rp, ci, col[int(vo[g]):int(vo[g + 1])])
    if bad:
        raise SystemExit("bench: %d invalid graphs in the batch" % bad)
    # plain form: one rsoc_color_device call per graph, same device-resident data
    plain_opts = rsoc.make_options(args.mode, "lower")
    rp_off = vo + np.arange(G + 1)

    def plain_pass():
        for g in range(G):
            n = int(vo[g + 1] - vo[g])
            rsoc.rsoc_color_device(ctx, d_rp[int(rp_off[g]):int(rp_off[g]) + n + 1], d_ci[int(no[g]):int(no[g + 1])],
                                   n, d_col[int(vo[g]):int(vo[g + 1])], plain_opts, stream=stream)

    plain_pass()
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for _ in range(args.plain_reps):
        plain_pass()
    torch.cuda.synchronize()
    tp = (time.perf_counter() - tp) / args.plain_reps
    st = stats[-1]
    kms = float(np.mean([x["ms_round0"] for x in stats]))
    # the launch options in effect (the run length as the library chose it
    # when the options leave it open), which the counters are keyed by
    launch = dict(args.tuned or {}, chunk=st["chunk"])
    kbytes = st["bytes_round0"]
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
    value = E * args.steps / elapsed / 1e9
    out = {
        "metric": "edges colored/s (GE/s) + colors used; batched vs plain",
        "value": value, "unit": "GE/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "batch of %d triangulated grids / random geometric graphs, 1e3..1e6 vertices "
                               "log-uniform, mean degree 12 (seed %d)" % (G, args.seed),
                   "graphs": G, "vertices": int(vo[-1]), "edges": E, "nnz": int(no[-1]), "mode": args.mode,
                   "tuned": args.tuned or {}},
        "colors_max": int(kmax), "rounds": st["rounds"], "conflicts": st["conflicts"], "chunk": st["chunk"],
        "autotune": tune_info,
        "plain": {"GEps": E / tp / 1e9, "ms_per_pass": tp * 1e3, "calls_per_pass": G},
        "batched_over_plain": value / (E / tp / 1e9),
        "roofline": {"bound": "hbm", "kernel": "batched_round0_first_fit", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None if achieved is None else achieved / HBM_PEAK_GBS,
                     "traffic": load_traffic("batched", "batched_round0_first_fit", launch), "kernel_ms": kms,
                     "alg_bytes_per_launch": kbytes},
    }
    ctx.close()
    return out


def make_requests(N: int, seed: int):
    """Served workload: sizes log-uniform in [1e4, 4e6] vertices; 35% 2D
    triangulated grids (natural ids), 35% 3D 26-stencil lattices (ids
    permuted), 30% R-MAT scale 14..20, edge factor 16 (ids shuffled)."""
    import concurrent.futures as cf

    import numpy as np

    import graphgen as gg
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(N):
        u = rng.random()
        n = float(np.exp(rng.uniform(np.log(1e4), np.log(4e6))))
        if u < 0.35:
            specs.append(("mesh2d", max(2, int(round(np.sqrt(n)))), i))
        elif u < 0.70:
            specs.append(("mesh3d", max(2, int(round(n ** (1 / 3)))), i))
        else:
            specs.append(("rmat", int(rng.integers(14, 21)), i))

    def gen(sp):
        kind, p, i = sp
        if kind == "mesh2d":
            return gg.tri_grid(p)
        if kind == "mesh3d":
            return gg.lattice26(p, permute_seed=seed * 1000 + i)
        return gg.rmat(p, 16, seed=seed * 1000 + i, shuffle_seed=seed * 1000 + i + 7)

    graphs = []
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(8) as ex:
        for k in range(0, len(specs), 100):
            graphs.extend(ex.map(gen, specs[k:k + 100]))
            print("[bench] generated %d of %d requests (%.0f s)" % (len(graphs), len(specs), time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    return specs, graphs


def _lat_ms(lat):
    import numpy as np
    lat = np.asarray(lat)
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3)}


def bench_served(args):
    import numpy as np
    import torch

    import paper_1505_04086_amd as rsoc
    from paper_1505_04086_amd import serve

    t = time.perf_counter()
    specs, graphs = make_requests(args.requests, args.seed)
    E_tot = sum(len(ci) // 2 for _, ci in graphs)
    V_tot = sum(len(rp) - 1 for rp, _ in graphs)
    dev = torch.device("cuda:0")
    # the timed runs start with every request's CSR resident in HBM; the
    # PCIe-inclusive variant (host arrays copied in, colours copied out) is
    # measured once at saturation beside it
    resident = [(torch.from_numpy(rp).to(dev), torch.from_numpy(ci if len(ci) else np.zeros(1, np.int32)).to(dev))
                for rp, ci in graphs]
    torch.cuda.synchronize()
    print("[bench] %d requests: %d vertices, %d edges (generated in %.1f s)"
          % (len(graphs), V_tot, E_tot, time.perf_counter() - t), file=sys.stderr, flush=True)
    ctx = rsoc.Context(0)
    opts = rsoc.make_options(args.mode, "lower")
    src = {"resident": resident}

    def reqs(arrivals, kind="resident"):
        data = src[kind]
        return [serve.Request(i, data[i][0], data[i][1], float(arrivals[i]), options=opts)
                for i in range(len(graphs))]

    zero = np.zeros(len(graphs))
    # warm both paths (graph capture, allocator)
    serve.PlainServer(ctx, opts).run(reqs(zero)[:4])
    sv = serve.Server(ctx, args.hbm_budget, options=opts)
    sv.run(reqs(zero)[:4])
    sv.close()

    def run_plain(arr):
        t0 = time.monotonic()
        out = serve.PlainServer(ctx, opts).run(reqs(arr), clock0=t0)
        return out, max(r.done for r in out) - t0

    def run_served(arr):
        s = serve.Server(ctx, args.hbm_budget, options=opts)
        t0 = time.monotonic()
        out = s.run(reqs(arr), clock0=t0)
        steps = s.steps
        s.close()
        return out, max(r.done for r in out) - t0, steps

    plain_out, plain_span = run_plain(zero)
    served_out, served_span, served_steps = run_served(zero)
    print("[bench] saturation: plain %.3f s, served %.3f s (%d steps)" % (plain_span, served_span, served_steps),
          file=sys.stderr, flush=True)
    for r in served_out:
        rp, ci = graphs[r.rid]
        if r.k < 0 or (r.rid % 4 == 0 and not colouring_valid(rp, ci, r.colors.cpu().numpy())):
            raise SystemExit("bench: invalid served colouring for request %d" % r.rid)
    served_out = [dict(rid=r.rid, latency=r.latency, k=r.k) for r in served_out]  # drop result tensors
    # PCIe-inclusive variant at saturation (pinned host arrays)
    src["host"] = [(_pinned(rp), _pinned(ci)) for rp, ci in graphs]
    t0 = time.monotonic()
    h_plain = serve.PlainServer(ctx, opts).run(reqs(zero, "host"), clock0=t0)
    h_plain_span = max(r.done for r in h_plain) - t0
    hs = serve.Server(ctx, args.hbm_budget, options=opts)
    t0 = time.monotonic()
    h_served = hs.run(reqs(zero, "host"), clock0=t0)
    h_served_span = max(r.done for r in h_served) - t0
    hs.close()
    del src["host"], h_plain, h_served
    cap_rps = len(graphs) / plain_span
    rates = {}
    rng = np.random.default_rng(args.seed + 99)
    for f in args.rate_factors:
        lam = f * cap_rps
        arr = np.cumsum(rng.exponential(1.0 / lam, size=len(graphs)))
        arr -= arr[0]
        po, pspan = run_plain(arr)
        so, sspan, _ = run_served(arr)
        rates["%.2gx" % f] = {"rate_rps": lam, "plain": dict(serve.latency_summary(po), GEps=E_tot / pspan / 1e9),
                              "served": dict(serve.latency_summary(so), GEps=E_tot / sspan / 1e9)}
        print("[bench] rate %.2gx: %s" % (f, json.dumps(rates["%.2gx" % f])), file=sys.stderr, flush=True)
    value = E_tot / served_span / 1e9
    plain_ge = E_tot / plain_span / 1e9
    out = {
        "metric": "edges colored/s (GE/s) + colors used; served vs plain, p50/p99 latency",
        "value": value, "unit": "GE/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": served_span * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "%d requests, sizes 1e4..4e6 log-uniform; 35%% 2D grids, 35%% 3D lattices, 30%% R-MAT "
                               "scale 14..20 (seed %d)" % (len(graphs), args.seed),
                   "requests": len(graphs), "vertices": V_tot, "edges": E_tot, "mode": args.mode,
                   "hbm_budget": args.hbm_budget},
        "saturation": {"served_GEps": value, "plain_GEps": plain_ge, "served_over_plain": value / plain_ge,
                       "served_steps": served_steps,
                       "served_latency": _lat_ms([r["latency"] for r in served_out]),
                       "plain_latency": serve.latency_summary(plain_out)},
        "pcie_inclusive_saturation": {"served_GEps": E_tot / h_served_span / 1e9,
                                      "plain_GEps": E_tot / h_plain_span / 1e9,
                                      "served_over_plain": h_plain_span / h_served_span},
        "poisson": rates,
        "colors_max": int(max(r["k"] for r in served_out)),
    }
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mesh3d", choices=["mesh3d", "rmat", "mesh2d", "batched", "served"])
    ap.add_argument("--mode", default="optimistic", choices=["optimistic", "deterministic", "two_phase"])
    ap.add_argument("--seed", type=int, default=1505)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the colouring (no colour classes, recolouring, distance-2 or literal-flow runs)")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--det-too", action="store_true", help="also time deterministic mode once")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--plain-reps", type=int, default=1)
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--hbm-budget", type=int, default=16 << 30)
    ap.add_argument("--rate-factors", type=float, nargs="*", default=[0.5, 1.0, 2.0, 4.0])
    ap.add_argument("--tune", action="store_true", help="autotune launch options first (batched workload)")
    ap.add_argument("--tune-graphs", type=int, default=256)
    ap.add_argument("--options", default=None,
                    help="batched workload: launch options as JSON (e.g. '{\"chunk\": 4}') instead of tuning")
    ap.add_argument("--cpu-omp-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--gather-probe", action="store_true",
                    help="only time random 4-byte gathers from a 4 MB table (the access pattern of round 0's "
                         "colour reads, without the rest of the round)")
    args = ap.parse_args()
    args.tuned = json.loads(args.options) if args.options else None
    if args.cpu_omp_leg:
        cpu_omp_leg(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only (--gpus 1); multi-GPU runs are not supported",
              file=sys.stderr)
        sys.exit(2)
    if args.gather_probe:
        # 2^27 random indices into a 2^20-entry int32 table (4 MB, the size of
        # the 8 M-vertex lattice's nibble shadow), gathered with torch.take:
        # besides the gathers it streams the indices in and the values out
        import torch
        g = torch.Generator(device="cuda:0")
        g.manual_seed(args.seed)
        table = torch.arange(1 << 20, dtype=torch.int32, device="cuda:0")
        idx = torch.randint(0, 1 << 20, (1 << 27,), dtype=torch.int64, device="cuda:0", generator=g)
        out = torch.take(table, idx)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            out = torch.take(table, idx)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        ok = bool((out[:1000] == idx[:1000].to(torch.int32)).all())
        print(json.dumps({"gather_probe": {"gathers": 1 << 27, "table_bytes": 4 << 20, "ms": dt * 1e3,
                                           "G_gathers_per_s": (1 << 27) / dt / 1e9,
                                           "stream_bytes": (1 << 27) * (8 + 4), "checked": ok}}), flush=True)
        return
    if args.copy_probe:
        import torch
        x = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 4, "launches": 3}), flush=True)
        return
    if args.workload == "batched":
        out = bench_batched(args)
    elif args.workload == "served":
        out = bench_served(args)
    else:
        out = bench_single(args)
        if args.workload == "mesh3d" and not args.no_extras:
            default_extras(args, out)
    print(json.dumps(out), flush=True)


def _free_device():
    import gc

    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _guarded(name, fn, *a):
    """Runs one extra of the default benchmark; an extra that fails is
    recorded with its error beside the headline figures, which are already
    measured."""
    t0 = time.perf_counter()
    try:
        r = fn(*a)
    except Exception as e:  # noqa: BLE001 -- reported in the JSON line
        print("[bench] %s failed: %r" % (name, e), file=sys.stderr, flush=True)
        r = {"error": repr(e)}
    _free_device()
    r["wall_s"] = time.perf_counter() - t0
    print("[bench] %s done in %.1f s" % (name, r["wall_s"]), file=sys.stderr, flush=True)
    return r


def default_extras(args, out):
    """The rest of the metric beside the headline line: the power-law graph
    (colours against sequential First-Fit), the batched form (4096 graphs,
    autotuned on a 256-graph sample, against one call per graph) and the
    served form (1000 Poisson requests at 0.5, 1, 2 and 4 times the plain
    form's capacity plus saturation, against one call per request, p50/p99)."""
    import copy
    _free_device()
    out["rmat_scale22"] = _guarded("rmat", bench_rmat_extra, args)
    a = copy.copy(args)
    a.steps, a.warmup, a.tune, a.tuned = 3, 1, True, None
    b = _guarded("batched", bench_batched, a)
    out["batched"] = b
    a = copy.copy(args)
    s = _guarded("served", bench_served, a)
    out["served"] = s
    out["batched_over_plain"] = b.get("batched_over_plain")
    out["served_over_plain"] = s.get("saturation", {}).get("served_over_plain")
    lat = {}
    for key, rec in s.get("poisson", {}).items():
        lat[key] = {side: {q: rec[side].get(q) for q in ("p50_ms", "p99_ms")} for side in ("plain", "served")}
    if "saturation" in s:
        lat["saturation"] = {"plain": {q: s["saturation"]["plain_latency"].get(q) for q in ("p50_ms", "p99_ms")},
                             "served": {q: s["saturation"]["served_latency"].get(q) for q in ("p50_ms", "p99_ms")}}
    out["latency_ms"] = lat
    out["tuned_options"] = (b.get("autotune") or {}).get("options")


if __name__ == "__main__":
    main()
