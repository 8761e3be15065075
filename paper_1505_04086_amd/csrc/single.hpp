// single.hpp -- host driver of the single-graph path (rsoc_color_device and friends).
//
// Binning, the argument completion (k_args) and the sweeps are enqueued
// without the host waiting in between: the sweeps read the bin sizes on the
// device, and the host takes them (for the worklist launch shapes) from a
// copy that lands while round 0 runs.  Validation, when asked for, is the one
// step the host waits for before any round.
// Round 0 and round 1 are launched directly (both cover all of V, except in
// the default optimistic flow, where round 1 is the masked pass over U^0);
// the later rounds only touch the worklist and are launched as a captured HIP graph of
// `rounds_per_sync` rounds, after which the host reads the worklist size (one
// 64-byte copy) and either stops or replays the graph.  ROCm 7.2 has no
// conditional graph nodes, so every kernel of a captured round first reads the
// device-side worklist size and returns at once when it is zero.
#pragma once

#include <map>
#include <vector>
#include <tuple>

#include "host_common.hpp"
#include "hub_kernels.hpp"
#include "single_kernels.hpp"
#include "tail_kernels.hpp"

struct rsoc_ctx {
    int device = 0;
    hipStream_t own = nullptr;    // stream for host-pointer calls
    hipStream_t cap = nullptr;    // capture stream
    rsoc::DevBuf wl0, wl1, hubW, hubB, pend, flags, col8, col4, aux;
    rsoc::DevBuf mark, tail;      // ordered pass over a small worklist (tail_kernels.hpp)
    rsoc::DevBuf hubs;            // hub-first round 0: sorted hubs, their lists (hub_kernels.hpp)
    rsoc::DevBuf cls_h, cls_p, cls_st;  // colour classes (classes.hpp)
    rsoc::DevBuf sq_t, sq_rp, sq_ci, sq_misc, sq_big;  // G^2 for distance-2 colouring (square.hpp)
    rsoc::DevBuf args, state;     // SingleArgs, SingleState (fixed addresses: graphs point at them)
    rsoc::HostPinned host;        // pinned staging for small copies
    rsoc::HostPinned b_tasks_host;  // a batch's task table on its way to the device
    rsoc::DevBuf drp, dci, dcol;  // device copies for host-pointer calls
    std::map<std::tuple<int, int, int, int, int, int, int>, hipGraphExec_t> graphs;
    hipEvent_t ev[8] = {};
    // batched path scratch (batch.hpp)
    rsoc::DevBuf b_desc, b_wl0, b_wl1, b_pend, b_u0mask, b_gchunk, b_state, b_hub, b_kmax, b_tasks, b_args, b_col8, b_small;
    int32_t *b_colp = nullptr;
};

namespace rsoc {

struct HostStaging {
    SingleArgs args;
    SingleState head;  // only the header part is ever copied
    int32_t L1;        // |L| of the first recolouring round
    int32_t rp_ends[2];
    int32_t cls_err;   // colour classes: a colour was outside [0, K)
    unsigned long long sq_total;  // distance 2: entries of G^2 ...
    int32_t sq_err;               // ... a 2-hop walk over the limit
    int32_t sq_pad, sq_verr;      // validation of G
};

inline int32_t ctx_init(rsoc_ctx *c, int device) {
    c->device = device;
    RSOC_HIP(hipSetDevice(device));
    RSOC_HIP(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
    RSOC_HIP(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    RSOC_TRY(c->args.reserve(sizeof(SingleArgs)));
    RSOC_TRY(c->state.reserve(sizeof(SingleState)));
    RSOC_TRY(c->host.reserve(sizeof(HostStaging) + 4096));
    RSOC_TRY(c->b_args.reserve(1024));  // holds a BatchArgs (fixed address: captured graphs use it)
    RSOC_TRY(c->b_state.reserve(sizeof(SingleState)));
    for (auto &e : c->ev) RSOC_HIP(hipEventCreate(&e));
    return RSOC_OK;
}

inline void ctx_free(rsoc_ctx *c) {
    (void)hipSetDevice(c->device);
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (rsoc::DevBuf *b : {&c->col8, &c->col4, &c->aux, &c->mark, &c->tail, &c->hubs, &c->cls_h, &c->cls_p, &c->cls_st,
                            &c->sq_t, &c->sq_rp, &c->sq_ci, &c->sq_misc, &c->sq_big, &c->wl0, &c->wl1, &c->hubW, &c->hubB, &c->pend, &c->flags, &c->args, &c->state, &c->drp,
                            &c->dci, &c->dcol, &c->b_desc, &c->b_wl0, &c->b_wl1, &c->b_pend, &c->b_u0mask, &c->b_gchunk,
                            &c->b_state, &c->b_hub, &c->b_kmax, &c->b_tasks, &c->b_args, &c->b_col8, &c->b_small})
        b->release();
    c->host.release();
    c->b_tasks_host.release();
    if (c->own) (void)hipStreamDestroy(c->own);
    if (c->cap) (void)hipStreamDestroy(c->cap);
}

// Launches one worklist round (no sweep) for the given mode.
template <int MODE, int TIE>
inline void launch_list_round(rsoc_ctx *c, hipStream_t s, int parity, int gB, int gW, int gT) {
    const SingleArgs *A = c->args.as<SingleArgs>();
    SingleState *S = c->state.as<SingleState>();
    const int grid = gB + gW + gT;
    if (two_phase_mode(MODE)) {
        k_round<kAssign, MODE, TIE, false><<<grid, kBlock, 0, s>>>(A, S, parity, gB, gW, gT);
        if (MODE == kTwoPhase) k_scatter<false, true><<<gT, kBlock, 0, s>>>(A, S, parity);
        k_round<kDetect, MODE, TIE, false><<<grid, kBlock, 0, s>>>(A, S, parity, gB, gW, gT);
    } else {
        k_round<kRecolor, MODE, TIE, false><<<grid, kBlock, 0, s>>>(A, S, parity, gB, gW, gT);
        if (MODE == kDeterministic) k_scatter<false, false><<<gT, kBlock, 0, s>>>(A, S, parity);
    }
    k_round_end<MODE, false><<<1, 64, 0, s>>>(A, S);
}

template <int MODE, int TIE>
inline void launch_list_rounds(rsoc_ctx *c, hipStream_t s, int K, int gB, int gW, int gT) {
    for (int r = 0; r < K; ++r) launch_list_round<MODE, TIE>(c, s, r & 1, gB, gW, gT);
}

inline void launch_list_rounds_dyn(rsoc_ctx *c, hipStream_t s, int mode, int tie, int K, int gB, int gW, int gT) {
    if (mode == kOptimistic)
        tie ? launch_list_rounds<kOptimistic, kHigherKeeps>(c, s, K, gB, gW, gT)
            : launch_list_rounds<kOptimistic, kLowerKeeps>(c, s, K, gB, gW, gT);
    else if (mode == kDeterministic)
        tie ? launch_list_rounds<kDeterministic, kHigherKeeps>(c, s, K, gB, gW, gT)
            : launch_list_rounds<kDeterministic, kLowerKeeps>(c, s, K, gB, gW, gT);
    else if (mode == kTwoPhase)
        tie ? launch_list_rounds<kTwoPhase, kHigherKeeps>(c, s, K, gB, gW, gT)
            : launch_list_rounds<kTwoPhase, kLowerKeeps>(c, s, K, gB, gW, gT);
    else
        tie ? launch_list_rounds<kTwoPhaseLive, kHigherKeeps>(c, s, K, gB, gW, gT)
            : launch_list_rounds<kTwoPhaseLive, kLowerKeeps>(c, s, K, gB, gW, gT);
}

// Captured graph of K worklist rounds followed by the colour statistics and
// the copy of the state header to the host, cached per (mode, tie, K, grid
// split, statistics grid).  Everything the kernels need beyond their launch
// shapes is read on the device (arguments block, state), so one graph serves
// every input with these shapes.
inline int32_t get_round_graph(rsoc_ctx *c, int mode, int tie, int K, int gB, int gW, int gT, int gstat,
                               hipGraphExec_t *out) {
    auto key = std::make_tuple(mode, tie, K, gB, gW, gT, gstat);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) { *out = it->second; return RSOC_OK; }
    hipGraph_t g = nullptr;
    HostStaging *h = c->host.as<HostStaging>();
    RSOC_HIP(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    launch_list_rounds_dyn(c, c->cap, mode, tie, K, gB, gW, gT);
    k_colour_stats<<<gstat, kBlock, 0, c->cap>>>(c->args.as<SingleArgs>(), c->state.as<SingleState>());
    k_head_out<<<1, kHeadBlock, 0, c->cap>>>(c->args.as<SingleArgs>(), c->state.as<SingleState>(), &h->head, &h->L1);
    hipError_t le = hipGetLastError();
    hipError_t ee = hipStreamEndCapture(c->cap, &g);
    if (le != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(le, "capture launch", __FILE__, __LINE__); }
    if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture", __FILE__, __LINE__);
    hipGraphExec_t ex = nullptr;
    hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate", __FILE__, __LINE__);
    c->graphs[key] = ex;
    *out = ex;
    return RSOC_OK;
}

// Rounds 0 and 1 up to the first worklist round.  gB/gW/gT split the sweep
// grid: the sweeps read the bin sizes on the device, so gB and gW may exceed
// what the bins need (the surplus workgroups find nothing to do).  Returns
// true when the first worklist round (the masked one, launch_masked_round1)
// is still to be enqueued; the next round reads worklist buffer 0.
template <int MODE, int TIE>
inline bool launch_sweep_rounds(rsoc_ctx *c, hipStream_t s, int32_t *col, int n, int gB, int gW, int gT, bool timing,
                                bool full_sweep) {
    const SingleArgs *A = c->args.as<SingleArgs>();
    SingleState *S = c->state.as<SingleState>();
    const int grid = gB + gW + gT;
    const int fill_grid = std::min(div_up(n, kBlock), 4096);  // two-phase scatter
    hipEvent_t *ev = c->ev;
    // Sweep rounds read no worklist and append into buffer 0 (parity 1); the
    // colours were filled for round 0 by k_args (round-synchronous modes: that
    // fill is round 0, every vertex colour 0).  With timing, ev[2..3] and
    // ev[4..5] bracket round 0 and round 1.
    if (MODE == kOptimistic) {
        if (!full_sweep) {
            // round 0: tentative First-Fit of all of V with live reads over
            // the neighbours each vertex loses to, collecting the only
            // vertices that can end the round defective as U^0 (into buffer
            // 1, with what each read uncoloured)
            launch_ev(k_round<kAssign, kOptimistic, TIE, true, 1>, grid, kBlock, s, timing ? ev[2] : nullptr,
                      timing ? ev[3] : nullptr, A, S, 0, gB, gW, gT);
            k_round_end<MODE, true, true><<<1, 64, 0, s>>>(A, S);
            return true;
        }
        // round 0 over all neighbours
        launch_ev(k_round<kAssign, kOptimistic, TIE, true, 0>, grid, kBlock, s, timing ? ev[2] : nullptr,
                  timing ? ev[3] : nullptr, A, S, 1, gB, gW, gT);
    }
    if (two_phase_mode(MODE)) {
        // Algorithm 2, first round: tentative colouring of V (published by
        // the scatter, or in place with live reads), detect
        if (MODE == kTwoPhaseLive && timing) (void)hipEventRecord(c->ev[2], s);
        k_round<kAssign, MODE, TIE, true><<<grid, kBlock, 0, s>>>(A, S, 1, gB, gW, gT);
        if (MODE == kTwoPhase) k_scatter<true, false><<<fill_grid, kBlock, 0, s>>>(A, S, 1);
        else if (timing) (void)hipEventRecord(c->ev[3], s);
        if (timing) (void)hipEventRecord(c->ev[4], s);
        k_round<kDetect, MODE, TIE, true><<<grid, kBlock, 0, s>>>(A, S, 1, gB, gW, gT);
        if (timing) (void)hipEventRecord(c->ev[5], s);
    } else {
        if (timing) (void)hipEventRecord(c->ev[4], s);
        // round 1: detect-and-recolour over U^0 = V
        k_round<kRecolor, MODE, TIE, true><<<grid, kBlock, 0, s>>>(A, S, 1, gB, gW, gT);
        if (timing) (void)hipEventRecord(c->ev[5], s);
        if (MODE == kDeterministic) k_scatter<false, false><<<std::max(1, gT), kBlock, 0, s>>>(A, S, 1);
    }
    k_round_end<MODE, true><<<1, 64, 0, s>>>(A, S);
    return false;
}

// Round 1 of the default optimistic flow: detect-and-recolour over U^0,
// testing only the kept neighbours of thread-bin entries; appends to buffer 0.
template <int TIE>
inline void launch_masked_round1(rsoc_ctx *c, hipStream_t s, int gBl, int gWl, int gTl, bool timing) {
    const SingleArgs *A = c->args.as<SingleArgs>();
    SingleState *S = c->state.as<SingleState>();
    launch_ev(k_round<kRecolor, kOptimistic, TIE, false, 2>, gBl + gWl + gTl, kBlock, s, timing ? c->ev[4] : nullptr,
              timing ? c->ev[5] : nullptr, A, S, 1, gBl, gWl, gTl);
    k_round_end<kOptimistic, false><<<1, 64, 0, s>>>(A, S);
}

inline bool launch_sweep_dyn(rsoc_ctx *c, hipStream_t s, int mode, int tie, int32_t *col, int n, int gB, int gW,
                             int gT, bool timing, bool full) {
#define RSOC_SWEEP(M, T) launch_sweep_rounds<M, T>(c, s, col, n, gB, gW, gT, timing, full)
    if (mode == kOptimistic)
        return tie ? RSOC_SWEEP(kOptimistic, kHigherKeeps) : RSOC_SWEEP(kOptimistic, kLowerKeeps);
    if (mode == kDeterministic)
        return tie ? RSOC_SWEEP(kDeterministic, kHigherKeeps) : RSOC_SWEEP(kDeterministic, kLowerKeeps);
    if (mode == kTwoPhase)
        return tie ? RSOC_SWEEP(kTwoPhase, kHigherKeeps) : RSOC_SWEEP(kTwoPhase, kLowerKeeps);
    return tie ? RSOC_SWEEP(kTwoPhaseLive, kHigherKeeps) : RSOC_SWEEP(kTwoPhaseLive, kLowerKeeps);
#undef RSOC_SWEEP
}

inline int32_t ensure_single_scratch(rsoc_ctx *c, int64_t n, bool need_aux, hipStream_t s) {
    const size_t b = sizeof(int32_t) * (size_t)(n + 2);
    RSOC_TRY(c->wl0.reserve(b));
    RSOC_TRY(c->wl1.reserve(b));
    RSOC_TRY(c->hubW.reserve(b));
    RSOC_TRY(c->hubB.reserve(b));
    RSOC_TRY(c->pend.reserve(b));
    const size_t had = c->flags.bytes;
    RSOC_TRY(c->flags.reserve(b));
    // colour flags stay zero between calls (k_head_out clears what it counts)
    if (c->flags.bytes != had) RSOC_HIP(hipMemsetAsync(c->flags.p, 0, c->flags.bytes, s));
    RSOC_TRY(c->col8.reserve((size_t)n + 64));
    RSOC_TRY(c->col4.reserve(sizeof(uint32_t) * (size_t)(n / 8 + 2)));
    if (need_aux) RSOC_TRY(c->aux.reserve(sizeof(int4) * (size_t)(n + 2)));
    return RSOC_OK;
}

// mark[] is zero between calls (k_tail_unmark restores what k_tail_mark set).
inline int32_t ensure_tail_scratch(rsoc_ctx *c, int64_t n, hipStream_t s) {
    const size_t had = c->mark.bytes;
    RSOC_TRY(c->mark.reserve(sizeof(int32_t) * (size_t)(n + 2)));
    if (c->mark.bytes != had) RSOC_HIP(hipMemsetAsync(c->mark.p, 0, c->mark.bytes, s));
    RSOC_TRY(c->tail.reserve(tail_bytes()));
    return RSOC_OK;
}

// One optimistic round over the current worklist (m entries, buffer 0) as an
// ordered pass; its recoloured vertices become the next worklist.
template <int TIE>
inline void launch_tail(rsoc_ctx *c, hipStream_t s, int m) {
    const SingleArgs *A = c->args.as<SingleArgs>();
    SingleState *S = c->state.as<SingleState>();
    const TailBuf t = tail_layout(c->tail.p);
    int32_t *mark = c->mark.as<int32_t>();
    const int g = div_up(m, kBlock);
    k_tail_mark<<<g, kBlock, 0, s>>>(A, S, t, mark, m);
    k_tail_prep<TIE><<<m, kBlock, 0, s>>>(A, t, mark);
    k_tail_seq<TIE, true><<<1, kBlock, 0, s>>>(A, S, t, m);
    k_tail_unmark<<<g, kBlock, 0, s>>>(t, mark, m);
    k_round_end<kOptimistic, false><<<1, 64, 0, s>>>(A, S);
}

inline int32_t status_from_err(int32_t err) {
    if (err & 1) return RSOC_ECSR;
    if (err & 2) return RSOC_ESELFLOOP;
    return RSOC_OK;
}

// Algorithmic bytes of the colouring (what the method itself must move,
// counted whether served by cache or HBM):
//   round 0, optimistic, literal (full_sweep): row_ptr 4(n+1) + col_idx 4 nnz
//     + neighbour colours 4 nnz + colour writes 4n + hub lists 4(nW+nB);
//   round 0, optimistic, default: the same but neighbour colours only for the
//     neighbours a vertex loses to (4 nnz/2 on a symmetric graph without
//     self-loops) plus 8 |U^0| for collecting U^0 with its position masks
//     (read back, 4 |U^0|, by round 1);
//   round 0, round-synchronous: the colour fill 4n;
//   round 1 as a sweep: row_ptr 4(n+1) + own colour 4n + 8 nnz + hub lists,
//     plus per recoloured vertex 8 (colour write + append), or 20 when staged
//     (stage write, append, then list read, stage read, colour write);
//   round 1 over U^0 (default optimistic flow): the masks 4 |U^0| plus the
//     worklist-round cost below of its own inspections;
//   worklist rounds: per inspected vertex 16 (list entry, row_ptr pair, own
//     colour) + 8 per adjacency entry read (the masked round 1 reads only the
//     masked entries of a vertex it keeps) + the per-recoloured cost above.
inline void alg_bytes(int mode, bool full_sweep, int64_t n, int64_t nnz, int64_t nW, int64_t nB, int64_t u0,
                      int64_t L1, int64_t conflicts, uint64_t inspected, uint64_t deg_sum, uint64_t inspected1,
                      uint64_t deg_sum1, int64_t &b0, int64_t &b1, int64_t &total) {
    const int64_t per_rec = (mode == kOptimistic) ? 8 : 20;
    if (two_phase_mode(mode)) {
        b0 = 4 * n;
        b1 = (4 * (n + 1) + 8 * nnz + 4 * n + 4 * (nW + nB)) + 12 * n + (4 * (n + 1) + 4 * n + 8 * nnz + 4 * (nW + nB)) +
             4 * L1;
        total = b0 + b1 + 44 * (int64_t)inspected + 16 * (int64_t)deg_sum + 4 * (conflicts - L1);
        return;
    }
    if (mode == kOptimistic && !full_sweep) {
        b0 = 4 * (n + 1) + 4 * nnz + 4 * (nnz / 2) + 4 * n + 4 * (nW + nB) + 8 * u0;
        b1 = 4 * u0 + 16 * (int64_t)inspected1 + 8 * (int64_t)deg_sum1 + per_rec * L1;
        total = b0 + 4 * u0 + 16 * (int64_t)inspected + 8 * (int64_t)deg_sum + per_rec * conflicts;
        return;
    }
    b0 = (mode == kOptimistic) ? 4 * (n + 1) + 8 * nnz + 4 * n + 4 * (nW + nB) : 4 * n;
    b1 = 4 * (n + 1) + 4 * n + 8 * nnz + 4 * (nW + nB) + per_rec * L1;
    total = b0 + b1 + 16 * (int64_t)inspected + 8 * (int64_t)deg_sum + per_rec * (conflicts - L1);
}

// The single-graph driver.  All pointers are device pointers.  nt >= 0: a
// recolouring after topology edits instead of a colouring: col holds the
// colouring before the edits, touched[0, nt) the vertices the edits touched;
// the rounds start from that state with U^0 = the touched vertices plus those
// without a valid First-Fit colour (no round 0; Algorithm 3's rounds as in a
// colouring).
inline int32_t run_single(rsoc_ctx *c, const int32_t *rp, const int32_t *ci, int32_t n, int32_t *col,
                          const Options &o, rsoc_stats *st, hipStream_t s, const int32_t *touched = nullptr,
                          int32_t nt = -1) {
    const bool inc = nt >= 0;
    HostStaging *h = c->host.as<HostStaging>();
    SingleState *S = c->state.as<SingleState>();
    if (st) {
        int32_t *keep = st->per_round_L, *keepU = st->per_round_U;
        int32_t cap = st->per_round_cap;
        memset(st, 0, sizeof(*st));
        st->per_round_L = keep;
        st->per_round_U = keepU;
        st->per_round_cap = cap;
    }
    if (n == 0) return 0;
    RSOC_TRY(ensure_single_scratch(c, n, o.mode == kOptimistic && !o.full_sweep && !inc, s));

    SingleArgs &a = h->args;
    a.rp = rp;
    a.ci = ci;
    a.col = col;
    a.col8 = c->col8.as<uint8_t>();
    a.col4 = c->col4.as<uint32_t>();
    a.pend = c->pend.as<int32_t>();
    a.aux = c->aux.as<int4>();
    a.wl[0] = c->wl0.as<int32_t>();
    a.wl[1] = c->wl1.as<int32_t>();
    a.hubW = c->hubW.as<int32_t>();
    a.hubB = c->hubB.as<int32_t>();
    a.n = n;
    a.t_thread = o.t_thread;
    a.t_wave = o.t_wave;
    a.max_rounds = o.max_rounds;
    a.offW = a.offB = 0;  // k_args sets them once the bins are known
    int gTs = std::min(div_up(n, kStep), o.grid_thread);
    if (gTs >= kXcds) gTs -= gTs % kXcds;
    const int64_t look = o.lookahead == -1 ? 0 : (o.lookahead > 0 ? o.lookahead : (int64_t)gTs * kStep);
    a.look = (int)std::min<int64_t>(look, INT32_MAX);
    a.look_auto = o.lookahead == 0 ? 1 : 0;
    a.chunk = inc ? 1 : o.chunk;  // 0: k_args picks it from the locality sample
    a.flags = c->flags.as<int32_t>();
    // hub-first round 0: optimistic default flow only (the round-synchronous
    // modes fix their result; the literal flow keeps the paper's round 0)
    const bool hub_first = o.hub_first != 0 && o.mode == kOptimistic && !o.full_sweep && !inc;
    a.hub_t = hub_first ? o.hub_first : 0;
    a.hubC = a.hubS = a.hub_cpre = nullptr;
    a.hub_bits = nullptr;
    if (hub_first) {
        const size_t had = c->hubs.bytes;
        RSOC_TRY(c->hubs.reserve(kHubBytes));
        // the hub bit sets are zero between calls (k_hub_ff clears what it reads)
        if (c->hubs.bytes != had) RSOC_HIP(hipMemsetAsync(c->hubs.p, 0, c->hubs.bytes, s));
        int32_t *hb = c->hubs.as<int32_t>();
        a.hubC = hb;
        a.hubS = hb + kHubCap;
        a.hub_cpre = hb + 2 * kHubCap;
        a.hub_bits = reinterpret_cast<uint32_t *>(hb + kHubTablesInts);
    }
    k_setup<<<1, kBlock, 0, s>>>(c->args.as<SingleArgs>(), a, S, (int)(kStateHeader / 4), 1);
    // binning: each workgroup ends with one global atomic per non-empty hub
    // queue, so fewer, longer-running workgroups (power-law graphs fill the
    // queues of nearly every workgroup)
    const int vgrid = std::min(div_up(n, kBlock), o.grid_bin ? o.grid_bin : 1024);
    // binning (reads row_ptr only: also checks its ends and publishes nnz),
    // with the id-locality sample in extra workgroups unless the CSR is to be
    // validated first (the sample reads rows)
    const bool validate = (o.validate & RSOC_CHECK_CSR) != 0;
    const int ns = (o.chunk == 0 && ci && !inc) ? std::min(n, 16384) : 0;
    const int gloc = div_up(ns, kBlock);
    k_bin<<<vgrid + (validate ? 0 : gloc), kBlock, 0, s>>>(c->args.as<SingleArgs>(), S, validate ? 0 : gloc, ns);
    RSOC_LAUNCH_CHECK();
    if (validate) {
        RSOC_HIP(hipMemcpyAsync(&h->head, S, kStateHeader, hipMemcpyDeviceToHost, s));
        RSOC_HIP(hipStreamSynchronize(s));
        if (h->head.err & 1) return RSOC_ECSR;
        if (h->head.nnz > 0 && !ci) return RSOC_EINVAL;
        k_validate<<<vgrid, kBlock, 0, s>>>(rp, ci, n, &S->err);
        if (gloc) k_bin<<<gloc, kBlock, 0, s>>>(c->args.as<SingleArgs>(), S, gloc, ns);
        RSOC_LAUNCH_CHECK();
        RSOC_HIP(hipMemcpyAsync(&h->head, S, kStateHeader, hipMemcpyDeviceToHost, s));
        RSOC_HIP(hipStreamSynchronize(s));
        RSOC_TRY(status_from_err(h->head.err));
    }
    // The bin sizes come back to the host (k_args writes the state header into
    // the pinned staging) while round 0 runs: the sweeps read them on the
    // device, and their hub sections are sized for the most the bins could
    // need unless validation already brought the sizes.
    // ... and it fills the colours for round 0; its start is the start of the
    // colouring (ev[0]); with timing, ev[2..3] bracket it in the round-
    // synchronous modes, where that fill is round 0
    const bool opt = o.mode == kOptimistic;
    const bool timing = o.timing != 0 && !inc;
    bool masked = false;
    if (!inc) {
        if (timing && !opt) RSOC_HIP(hipEventRecord(c->ev[2], s));
        launch_ev(k_args, std::min(div_up(n, kBlock), 4096), kBlock, s, c->ev[0], c->ev[6], c->args.as<SingleArgs>(),
                  S, &h->head, col, c->col8.as<uint8_t>(), (int64_t)n, o.mode == kDeterministic ? 0 : -1,
                  opt ? c->col4.as<uint32_t>() : (uint32_t *)nullptr, (int64_t)(opt ? n / 8 + 1 : 0));
        RSOC_LAUNCH_CHECK();
        if (timing && !opt) RSOC_HIP(hipEventRecord(c->ev[3], s));
        if (hub_first) {
            const SingleArgs *A = c->args.as<SingleArgs>();
            k_hub_sort<<<1, kHubSortBlock, 0, s>>>(A, S);
            if (o.tie) {
                k_hub_lists<kHigherKeeps><<<kHubListGrid, kBlock, 0, s>>>(A, S);
                k_hub_ff<kHigherKeeps><<<1, kHubFfBlock, 0, s>>>(A, S);
            } else {
                k_hub_lists<kLowerKeeps><<<kHubListGrid, kBlock, 0, s>>>(A, S);
                k_hub_ff<kLowerKeeps><<<1, kHubFfBlock, 0, s>>>(A, S);
            }
            RSOC_LAUNCH_CHECK();
        }
        const int gB = validate ? std::min(h->head.nB, 1024) : std::min(n, 1024);
        const int gW = std::min(div_up(validate ? h->head.nW : n, kWavesPerBlock), o.grid_wave);
        masked = launch_sweep_dyn(c, s, o.mode, o.tie, col, n, gB, gW, gTs, timing, o.full_sweep != 0);
        RSOC_LAUNCH_CHECK();
    } else {
        // the colours stay (no fill); shadows and U^0 come from them and the
        // touched list (pend serves as the mark array: the staged colours of
        // the round-synchronous mode are written before they are read)
        launch_ev(k_args, 1, kBlock, s, c->ev[0], c->ev[6], c->args.as<SingleArgs>(), S, &h->head, (int32_t *)nullptr,
                  (uint8_t *)nullptr, (int64_t)0, 0, (uint32_t *)nullptr, (int64_t)0);
        const int g = std::min(div_up(n, kBlock), 4096);
        int32_t *mark = c->pend.as<int32_t>();
        const SingleArgs *A = c->args.as<SingleArgs>();
        if (opt) k_inc_shadow<true><<<g, kBlock, 0, s>>>(A, mark);
        else k_inc_shadow<false><<<g, kBlock, 0, s>>>(A, mark);
        if (nt > 0) k_inc_touch<<<std::min(div_up(nt, kBlock), 1024), kBlock, 0, s>>>(A, S, touched, nt, mark);
        k_inc_list<<<o.grid_bin ? std::min(g, o.grid_bin) : g, kBlock, 0, s>>>(A, S, mark);
        if (opt) k_round_end<kOptimistic, true, true><<<1, 64, 0, s>>>(A, S);
        else k_round_end<kDeterministic, true, true><<<1, 64, 0, s>>>(A, S);
        RSOC_LAUNCH_CHECK();
    }
    RSOC_HIP(hipEventSynchronize(c->ev[6]));
    if (h->head.err & kErrNoRun) {
        // the sweeps return at once on such input; let them drain
        RSOC_HIP(hipStreamSynchronize(s));
        return (h->head.err & 1) ? RSOC_ECSR : RSOC_EINVAL;
    }
    const int64_t nnz = h->head.nnz;
    const int nW = h->head.nW, nB = h->head.nB, maxdeg = h->head.maxdeg;
    const int nT = n - nW - nB;
    const int chunk = h->head.chunk;
    const int gBl = std::min(nB, 256);  // more concurrent hubs only add hub conflicts
    const int gWl = std::min(div_up(nW, kWavesPerBlock), o.grid_wave);
    const int gTl = std::max(1, std::min(div_up(nT, kStep), o.grid_list));
    if (masked) {
        o.tie ? launch_masked_round1<kHigherKeeps>(c, s, gBl, gWl, gTl, timing)
              : launch_masked_round1<kLowerKeeps>(c, s, gBl, gWl, gTl, timing);
        RSOC_LAUNCH_CHECK();
    }
    hipGraphExec_t gexec = nullptr;
    // colour count (K = max + 1) and distinct colours: the statistics close
    // every replay, so the one host check per replay also brings them; they
    // count once the worklist is empty
    // four 16-byte loads in flight per lane; few workgroups, so that their
    // merges into the shared statistics words stay few
    const int gstat = std::min(div_up(n, 16 * 4 * kBlock), 512);
    RSOC_TRY(get_round_graph(c, o.mode, o.tie, o.rounds_per_sync, gBl, gWl, gTl, gstat, &gexec));

    int32_t status = RSOC_OK;
    const int tail_max = o.tail == -1 ? 0 : (o.tail == 0 ? kTailMax : std::min(o.tail, kTailMax));
    for (;;) {
        RSOC_HIP(hipGraphLaunch(gexec, s));
        RSOC_HIP(hipEventRecord(c->ev[1], s));
        RSOC_HIP(hipStreamSynchronize(s));
        const int left = h->head.cnt_in[0] + h->head.cnt_in[1] + h->head.cnt_in[2];
        if (left == 0) break;
        if (h->head.passes >= o.max_rounds) { status = RSOC_ENOCONV; break; }
        // the ordered pass pays off where the list has stopped shrinking
        // quickly (mutually adjacent hubs), not where a round or two more
        // would empty it
        if (o.mode == kOptimistic && left <= tail_max && 2 * (int64_t)h->head.lastL >= h->head.prevL) {
            RSOC_TRY(ensure_tail_scratch(c, n, s));
            o.tie ? launch_tail<kHigherKeeps>(c, s, left) : launch_tail<kLowerKeeps>(c, s, left);
            RSOC_LAUNCH_CHECK();
        }
    }
    if (st && (st->per_round_L || st->per_round_U) && st->per_round_cap > 0) {
        // |L| of round i+1 is the device history; |U| of pass i+1 is U^0 for
        // the first pass and the previous round's |L| after it (U <- L)
        const int cnt = std::min(std::min(std::max(h->head.rounds, h->head.passes), st->per_round_cap), kHistCap);
        std::vector<int32_t> hist((size_t)std::max(cnt, 1), 0);
        if (cnt > 0) {
            RSOC_HIP(hipMemcpyAsync(hist.data(), S->hist, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, s));
            RSOC_HIP(hipStreamSynchronize(s));
        }
        if (st->per_round_L)
            for (int i = 0; i < std::min(h->head.rounds, cnt); ++i) st->per_round_L[i] = hist[i];
        if (st->per_round_U) {
            const bool sweep1u = !inc && !(o.mode == kOptimistic && !o.full_sweep);
            const int np = std::min(h->head.passes, st->per_round_cap);
            for (int i = 0; i < np; ++i)
                st->per_round_U[i] = i == 0 ? (sweep1u ? n : h->head.u0) : (i - 1 < cnt ? hist[i - 1] : 0);
        }
    }
    if (h->head.err & (4 | kErrListCount)) return RSOC_EINTERNAL;  // never expected
    if (h->head.err & 16) return RSOC_EINVAL;  // a touched id outside [0, n)
    if (st) {
        st->rounds = h->head.rounds;
        st->passes = h->head.passes;
        st->colors = h->head.kmax;
        int distinct = h->head.distinct;
        for (uint32_t w : h->head.cbits) distinct += __builtin_popcount(w);
        st->colors_distinct = distinct;
        st->conflicts = h->head.conflicts;
        const bool sweep1 = !inc && !(o.mode == kOptimistic && !o.full_sweep);
        st->inspected = (int64_t)h->head.inspected + (sweep1 ? n : 0);
        st->max_degree = maxdeg;
        st->bin_counts[0] = nT;
        st->bin_counts[1] = nW;
        st->bin_counts[2] = nB;
        float ms = 0;
        RSOC_HIP(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        st->ms = ms;
        if (timing) {
            float m0 = 0, m1 = 0;
            RSOC_HIP(hipEventElapsedTime(&m0, c->ev[2], c->ev[3]));
            RSOC_HIP(hipEventElapsedTime(&m1, c->ev[4], c->ev[5]));
            st->ms_round0 = m0;
            st->ms_round1 = m1;
        }
        int64_t b0, b1, tot;
        const int64_t l1 = h->head.rounds > 0 ? h->L1 : 0;
        if (inc) {
            // set-up: colours read, shadows written, row_ptr for degrees, marks
            // written and read, touched ids, U^0 appended; then the rounds
            b0 = 4 * n + n + (opt ? 4 * (n / 8 + 1) : 0) + 4 * (n + 1) + 8 * (int64_t)n + 4 * (int64_t)nt +
                 4 * (int64_t)h->head.u0;
            b1 = 0;
            tot = b0 + 16 * (int64_t)h->head.inspected + 8 * (int64_t)h->head.deg_sum +
                  (opt ? 8 : 20) * h->head.conflicts;
        } else {
            alg_bytes(o.mode, o.full_sweep != 0, n, nnz, nW, nB, h->head.u0, l1, h->head.conflicts,
                      h->head.inspected, h->head.deg_sum, h->head.inspected1, h->head.deg_sum1, b0, b1, tot);
        }
        st->bytes_round0 = b0;
        st->worklist0 = sweep1 ? n : h->head.u0;
        st->chunk = chunk;
        st->bytes_round1 = b1;
        st->alg_bytes = tot;
    }
    if (status < 0) return status;
    return h->head.kmax;
}

}  // namespace rsoc
