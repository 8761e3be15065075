// batch.hpp -- host driver of rsoc_color_batch: G independent graphs coloured
// by one sequence of fused launches (round 0, then captured worklist rounds),
// with the same round structure as the single-graph driver.
#pragma once

#include <cmath>
#include <vector>

#include "batch_kernels.hpp"
#include "single.hpp"

namespace rsoc {

template <int MODE, int TIE>
inline void launch_blist_round(rsoc_ctx *c, hipStream_t s, int parity, int gB, int gW, int gT) {
    const BatchArgs *A = c->b_args.as<BatchArgs>();
    SingleState *S = c->b_state.as<SingleState>();
    const int grid = gB + gW + gT;
    if (MODE == kTwoPhase) {
        k_bround<kAssign, kTwoPhase, TIE, false><<<grid, kBlock, 0, s>>>(A, S, parity, gB, gW, gT);
        k_bscatter<false, true><<<gT, kBlock, 0, s>>>(A, S, parity);
        k_bround<kDetect, kTwoPhase, TIE, false><<<grid, kBlock, 0, s>>>(A, S, parity, gB, gW, gT);
    } else {
        k_bround<kRecolor, MODE, TIE, false><<<grid, kBlock, 0, s>>>(A, S, parity, gB, gW, gT);
        if (MODE == kDeterministic) k_bscatter<false, false><<<gT, kBlock, 0, s>>>(A, S, parity);
    }
    k_bround_end<MODE, false><<<1, 64, 0, s>>>(A, S);
}

inline void launch_blist_rounds_dyn(rsoc_ctx *c, hipStream_t s, int mode, int tie, int K, int gB, int gW, int gT) {
    for (int r = 0; r < K; ++r) {
        const int p = r & 1;
        if (mode == kOptimistic)
            tie ? launch_blist_round<kOptimistic, kHigherKeeps>(c, s, p, gB, gW, gT)
                : launch_blist_round<kOptimistic, kLowerKeeps>(c, s, p, gB, gW, gT);
        else if (mode == kDeterministic)
            tie ? launch_blist_round<kDeterministic, kHigherKeeps>(c, s, p, gB, gW, gT)
                : launch_blist_round<kDeterministic, kLowerKeeps>(c, s, p, gB, gW, gT);
        else
            tie ? launch_blist_round<kTwoPhase, kHigherKeeps>(c, s, p, gB, gW, gT)
                : launch_blist_round<kTwoPhase, kLowerKeeps>(c, s, p, gB, gW, gT);
    }
}

inline int32_t get_batch_graph(rsoc_ctx *c, int mode, int tie, int K, int gB, int gW, int gT, hipGraphExec_t *out) {
    auto key = std::make_tuple(100 + mode, tie, K, gB, gW, gT, 0);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) { *out = it->second; return RSOC_OK; }
    hipGraph_t g = nullptr;
    RSOC_HIP(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    launch_blist_rounds_dyn(c, c->cap, mode, tie, K, gB, gW, gT);
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

// gB/gW/gT: the sweep's grid; gBl/gWl/gTl: the list rounds' grid.
template <int MODE, int TIE>
inline void launch_bsweep(rsoc_ctx *c, hipStream_t s, int64_t nV, int gB, int gW, int gT, bool full_sweep,
                          bool timing, int gBl, int gWl, int gTl) {
    const BatchArgs *A = c->b_args.as<BatchArgs>();
    SingleState *S = c->b_state.as<SingleState>();
    const int grid = gB + gW + gT;
    const int fill_grid = (int)std::min<int64_t>(div_up(nV, kBlock), 8192);
    int32_t *col = c->b_colp;
    uint8_t *col8 = c->b_col8.as<uint8_t>();
    if (MODE == kDeterministic) {
        k_fill<<<fill_grid, kBlock, 0, s>>>(col, col8, nV, 0);
    } else {
        k_fill<<<fill_grid, kBlock, 0, s>>>(col, col8, nV, -1);
        if (MODE == kOptimistic) {
            if (timing) (void)hipEventRecord(c->ev[2], s);
            if (!full_sweep) {
                k_bround<kAssign, kOptimistic, TIE, true, 1><<<grid, kBlock, 0, s>>>(A, S, 1, gB, gW, gT);
                if (timing) (void)hipEventRecord(c->ev[3], s);
                k_bround_end<MODE, true, true><<<1, 64, 0, s>>>(A, S);
                // round 1 over U^0, its thread-bin part walked task by task from
                // round 0's masks with the sweep's grid, then one list round at
                // parity 1, so that the captured rounds find their list at parity 0
                k_bround<kRecolor, kOptimistic, TIE, false, 2><<<gBl + gWl + gT, kBlock, 0, s>>>(A, S, 0, gBl, gWl,
                                                                                             gT);
                k_bround_end<MODE, false><<<1, 64, 0, s>>>(A, S);
                launch_blist_round<kOptimistic, TIE>(c, s, 1, gBl, gWl, gTl);
                return;
            }
            k_bround<kAssign, kOptimistic, TIE, true, 0><<<grid, kBlock, 0, s>>>(A, S, 1, gB, gW, gT);
            if (timing) (void)hipEventRecord(c->ev[3], s);
        }
    }
    if (MODE == kTwoPhase) {
        k_bround<kAssign, kTwoPhase, TIE, true><<<grid, kBlock, 0, s>>>(A, S, 1, gB, gW, gT);
        k_bscatter<true, false><<<fill_grid, kBlock, 0, s>>>(A, S, 1);
        k_bround<kDetect, kTwoPhase, TIE, true><<<grid, kBlock, 0, s>>>(A, S, 1, gB, gW, gT);
    } else {
        k_bround<kRecolor, MODE, TIE, true><<<grid, kBlock, 0, s>>>(A, S, 1, gB, gW, gT);
        if (MODE == kDeterministic) k_bscatter<false, false><<<std::max(1, gT), kBlock, 0, s>>>(A, S, 1);
    }
    k_bround_end<MODE, true><<<1, 64, 0, s>>>(A, S);
}

inline void launch_bsweep_dyn(rsoc_ctx *c, hipStream_t s, int mode, int tie, int64_t nV, int gB, int gW, int gT,
                              bool full, bool timing, int gBl, int gWl, int gTl) {
    if (mode == kOptimistic)
        tie ? launch_bsweep<kOptimistic, kHigherKeeps>(c, s, nV, gB, gW, gT, full, timing, gBl, gWl, gTl)
            : launch_bsweep<kOptimistic, kLowerKeeps>(c, s, nV, gB, gW, gT, full, timing, gBl, gWl, gTl);
    else if (mode == kDeterministic)
        tie ? launch_bsweep<kDeterministic, kHigherKeeps>(c, s, nV, gB, gW, gT, full, timing, gBl, gWl, gTl)
            : launch_bsweep<kDeterministic, kLowerKeeps>(c, s, nV, gB, gW, gT, full, timing, gBl, gWl, gTl);
    else
        tie ? launch_bsweep<kTwoPhase, kHigherKeeps>(c, s, nV, gB, gW, gT, full, timing, gBl, gWl, gTl)
            : launch_bsweep<kTwoPhase, kLowerKeeps>(c, s, nV, gB, gW, gT, full, timing, gBl, gWl, gTl);
}

struct BatchHost {
    BatchArgs args;
    SingleState head;
};
static_assert(sizeof(BatchArgs) <= 1024, "b_args holds one BatchArgs");
static_assert(sizeof(BatchHost) <= sizeof(HostStaging) + 4096, "pinned staging holds one BatchHost");

inline int32_t run_batch(rsoc_ctx *c, int32_t G, const int64_t *vtx_off, const int64_t *nnz_off, const int32_t *rp,
                         const int32_t *ci, int32_t *col, int32_t *counts_out, const Options &o, rsoc_stats *st,
                         hipStream_t s) {
    if (st) {
        int32_t *keep = st->per_round_L, *keepU = st->per_round_U;
        int32_t cap = st->per_round_cap;
        memset(st, 0, sizeof(*st));
        st->per_round_L = keep;
        st->per_round_U = keepU;
        st->per_round_cap = cap;
    }
    if (vtx_off[0] != 0 || nnz_off[0] != 0) return RSOC_ECSR;
    for (int g = 0; g < G; ++g) {
        if (vtx_off[g + 1] < vtx_off[g] || nnz_off[g + 1] < nnz_off[g]) return RSOC_ECSR;
        if (vtx_off[g + 1] - vtx_off[g] > INT32_MAX - 1 || nnz_off[g + 1] - nnz_off[g] > INT32_MAX) return RSOC_EINVAL;
    }
    const int64_t nV = vtx_off[G];
    if (nV >= INT32_MAX) return RSOC_EINVAL;
    if (G == 0 || nV == 0) {
        for (int g = 0; g < G; ++g)
            if (counts_out) counts_out[g] = 0;
        return 0;
    }
    // graphs of at most small_cutoff vertices are coloured by one workgroup
    // each (k_bsmall); the others by the fused launches
    const bool small_ok = o.small_cutoff > 0 && o.mode != kTwoPhase;
    auto is_small = [&](int g) {
        const int64_t n = vtx_off[g + 1] - vtx_off[g];
        return small_ok && n > 0 && n <= o.small_cutoff;
    };
    std::vector<int32_t> small;
    // sweep tasks: (graph, first vertex) chunks of kTaskLen vertices, in graph
    // order; the fused launches' graphs first, then the small graphs' (which
    // only validation and the colour count walk).  Written straight into
    // pinned memory, so that the upload is one DMA.
    int64_t nVL = 0, nt_large = 0, nt_small = 0;
    for (int g = 0; g < G; ++g) {
        const int64_t k = (vtx_off[g + 1] - vtx_off[g] + kTaskLen - 1) / kTaskLen;
        if (is_small(g)) {
            small.push_back(g);
            nt_small += k;
        } else {
            nVL += vtx_off[g + 1] - vtx_off[g];
            nt_large += k;
        }
    }
    if (nt_large + nt_small > INT32_MAX) return RSOC_EINVAL;
    const int ntasks = (int)nt_large;
    const int ntasks_all = (int)(nt_large + nt_small);
    RSOC_TRY(c->b_tasks_host.reserve(sizeof(int64_t) * (size_t)std::max(ntasks_all, 1)));
    int64_t *const tasks = c->b_tasks_host.as<int64_t>();
    {
        int64_t wl = 0, ws = nt_large;
        for (int g = 0; g < G; ++g) {
            int64_t &w = is_small(g) ? ws : wl;
            for (int64_t st0 = 0; st0 < vtx_off[g + 1] - vtx_off[g]; st0 += kTaskLen)
                tasks[w++] = ((int64_t)g << 32) | (uint32_t)st0;
        }
    }
    const int nsmall = (int)small.size();
    constexpr int kSmallStatInts = kSmallStatHist + kSmallMax + 2;
    RSOC_TRY(c->b_desc.reserve(sizeof(int64_t) * 2 * (size_t)(G + 1)));
    RSOC_TRY(c->b_tasks.reserve(sizeof(int64_t) * (size_t)std::max(ntasks_all, 1)));
    RSOC_TRY(c->b_col8.reserve((size_t)nV + 64));
    if (o.mode != kOptimistic) RSOC_TRY(c->b_pend.reserve(sizeof(int32_t) * (size_t)nV));
    else {
        // optimistic mode stages no colours: the staging buffer holds, for
        // U^0's lane-group entries, the row positions round 0 read uncoloured
        RSOC_TRY(c->b_u0mask.reserve(sizeof(uint32_t) * kTaskWords * (size_t)std::max(ntasks, 1)));
        RSOC_TRY(c->b_pend.reserve(sizeof(uint32_t) * (size_t)nV));
    }
    RSOC_TRY(c->b_wl0.reserve(sizeof(int64_t) * (size_t)(nV + 1)));
    RSOC_TRY(c->b_wl1.reserve(sizeof(int64_t) * (size_t)(nV + 1)));
    RSOC_TRY(c->b_hub.reserve(sizeof(int64_t) * (size_t)(nV + 1)));
    RSOC_TRY(c->b_kmax.reserve(sizeof(int32_t) * (size_t)G));
    RSOC_TRY(c->b_small.reserve(sizeof(int32_t) * (size_t)(kSmallStatInts + nsmall)));
    int32_t *d_small_stat = c->b_small.as<int32_t>();
    int32_t *d_small = d_small_stat + kSmallStatInts;
    int64_t *d_voff = c->b_desc.as<int64_t>();
    int64_t *d_noff = d_voff + (G + 1);
    RSOC_HIP(hipMemcpyAsync(d_voff, vtx_off, sizeof(int64_t) * (size_t)(G + 1), hipMemcpyHostToDevice, s));
    RSOC_HIP(hipMemcpyAsync(d_noff, nnz_off, sizeof(int64_t) * (size_t)(G + 1), hipMemcpyHostToDevice, s));
    RSOC_HIP(hipMemcpyAsync(c->b_tasks.p, tasks, sizeof(int64_t) * (size_t)ntasks_all, hipMemcpyHostToDevice,
                            s));
    if (nsmall)
        RSOC_HIP(hipMemcpyAsync(d_small, small.data(), sizeof(int32_t) * (size_t)nsmall, hipMemcpyHostToDevice, s));
    RSOC_HIP(hipMemsetAsync(d_small_stat, 0, sizeof(int32_t) * kSmallStatInts, s));
    c->b_colp = col;

    BatchHost *h = c->host.as<BatchHost>();
    BatchArgs &a = h->args;
    a.voff = d_voff;
    a.noff = d_noff;
    a.rp = rp;
    a.ci = ci;
    a.col = col;
    a.col8 = c->b_col8.as<uint8_t>();
    a.pend = c->b_pend.as<int32_t>();
    a.wl[0] = c->b_wl0.as<int64_t>();
    a.wl[1] = c->b_wl1.as<int64_t>();
    a.hub = c->b_hub.as<int64_t>();
    a.tasks = c->b_tasks.as<int64_t>();
    a.u0mask = c->b_u0mask.as<uint32_t>();
    a.u0pos = o.mode == kOptimistic ? c->b_pend.as<uint32_t>() : nullptr;
    a.kg = c->b_kmax.as<int32_t>();
    a.nV = nV;
    a.hub_cap = nV + 1;
    a.offW = a.offB = 0;
    a.G = G;
    a.ntasks = ntasks;
    a.ntasks_all = ntasks_all;
    a.small = d_small;
    a.small_stat = d_small_stat;
    a.nsmall = nsmall;
    a.t_thread = o.t_thread;
    a.t_wave = o.t_wave;
    a.max_rounds = o.max_rounds;
    a.look = 0;
    a.chunk = 1;
    // run length: the option's for every graph, else each sweep task takes
    // its graph's, chosen on the device (k_bchunk), and the worklist rounds
    // walk their lists in runs of kChunk: a list keeps the order in which a
    // grid's vertices were appended, and neighbouring groups taking
    // consecutive entries would recolour adjacent vertices at the same
    // instant (25 rounds instead of 7 on the 4096-graph batch)
    if (o.chunk == 0) {
        RSOC_TRY(c->b_gchunk.reserve((size_t)std::max(G, 1)));
        a.gchunk = c->b_gchunk.as<uint8_t>();
    } else {
        a.gchunk = nullptr;
    }
    // round 0's bands (claim_task): ranges of the fused launches' tasks of
    // about equal work, a task's work taken as its vertices times one plus
    // its graph's mean degree (a graph's tasks then weigh n_g + nnz_g in all);
    // band x starts at the first task with at least x/nbands of the work
    // before it
    a.nbands = kXcds * o.bands;
    {
        double total = 0;
        for (int g = 0; g < G; ++g)
            if (!is_small(g)) total += (double)(vtx_off[g + 1] - vtx_off[g] + nnz_off[g + 1] - nnz_off[g]);
        int x = 1;
        double before = 0;  // work of the graphs before g
        int64_t t0 = 0;     // their tasks
        a.band[0] = 0;
        for (int g = 0; g < G && x < a.nbands; ++g) {
            if (is_small(g)) continue;
            const int64_t n = vtx_off[g + 1] - vtx_off[g];
            const int64_t k = (n + kTaskLen - 1) / kTaskLen;
            const double gw = (double)(n + nnz_off[g + 1] - nnz_off[g]);
            const double per_task = n > 0 ? kTaskLen * gw / (double)n : 0.0;
            for (; x < a.nbands && total * x / a.nbands <= before + gw; ++x) {
                const double need = total * x / a.nbands - before;
                int64_t j = per_task > 0 ? (int64_t)std::ceil(need / per_task) : 0;
                a.band[x] = (int)(t0 + std::min(std::max<int64_t>(j, 0), k));
            }
            before += gw;
            t0 += k;
        }
        for (; x <= a.nbands; ++x) a.band[x] = ntasks;
    }
    SingleState *S = c->b_state.as<SingleState>();
    RSOC_HIP(hipMemcpyAsync(c->b_args.p, &a, sizeof(a), hipMemcpyHostToDevice, s));
    RSOC_HIP(hipMemsetAsync(S, 0, kStateHeader, s));
    RSOC_HIP(hipMemsetAsync(c->b_kmax.p, 0, sizeof(int32_t) * (size_t)G, s));
    const int tgrid = std::min(ntasks, o.grid_bin ? o.grid_bin : 8192);
    const int tgrid_all = std::max(1, std::min(ntasks_all, o.grid_bin ? o.grid_bin : 8192));
    if (o.validate & RSOC_CHECK_CSR) {
        k_bvalidate<<<tgrid_all, kBlock, 0, s>>>(c->b_args.as<BatchArgs>(), &S->err);
        RSOC_LAUNCH_CHECK();
    }
    if (ntasks > 0) k_bbin<<<tgrid, kBlock, 0, s>>>(c->b_args.as<BatchArgs>(), S);
    if (o.chunk == 0 && ntasks > 0) k_bchunk<<<div_up(G, kWavesPerBlock), kBlock, 0, s>>>(c->b_args.as<BatchArgs>());
    RSOC_LAUNCH_CHECK();
    RSOC_HIP(hipMemcpyAsync(&h->head, S, kStateHeader, hipMemcpyDeviceToHost, s));
    RSOC_HIP(hipStreamSynchronize(s));
    RSOC_TRY(status_from_err(h->head.err));
    const int nW = h->head.nW, nB = h->head.nB;
    const int64_t nT = nVL - nW - nB;
    const bool timing = o.timing && o.mode == kOptimistic;
    int32_t status = RSOC_OK;
    RSOC_HIP(hipEventRecord(c->ev[0], s));
    if (ntasks > 0) {
        a.offW = nT;
        a.offB = nT + nW;
        const int gB = std::min(nB, 1024);
        const int gW = std::min(div_up(nW, kWavesPerBlock), o.grid_wave);
        // the optimistic default flow's sweeps claim their tasks (claim_task):
        // a grid beyond the resident workgroups costs nothing there
        const bool claims = o.mode == kOptimistic && !o.full_sweep;
        const int gTs = std::max(1, std::min(ntasks, (claims && !o.grid_thread_given) ? 4096 : o.grid_thread));
        const int64_t look = o.lookahead == -1 ? 0 : (o.lookahead > 0 ? o.lookahead : 2ll * gTs * kStep);
        a.look = (int)std::min<int64_t>(look, INT32_MAX);
        a.chunk = o.chunk ? o.chunk : kChunk;
        RSOC_HIP(hipMemcpyAsync(c->b_args.p, &a, sizeof(a), hipMemcpyHostToDevice, s));
        const int gBl = std::min(nB, 256);
        const int gWl = std::min(div_up(nW, kWavesPerBlock), o.grid_wave);
        const int gTl = (int)std::max<int64_t>(1, std::min<int64_t>(div_up(nT, kStep), o.grid_list));
        hipGraphExec_t gexec = nullptr;
        RSOC_TRY(get_batch_graph(c, o.mode, o.tie, o.rounds_per_sync, gBl, gWl, gTl, &gexec));
        launch_bsweep_dyn(c, s, o.mode, o.tie, nV, gB, gW, gTs, o.full_sweep != 0, timing, gBl, gWl, gTl);
        RSOC_LAUNCH_CHECK();
        for (;;) {
            RSOC_HIP(hipGraphLaunch(gexec, s));
            RSOC_HIP(hipMemcpyAsync(&h->head, S, kStateHeader, hipMemcpyDeviceToHost, s));
            RSOC_HIP(hipStreamSynchronize(s));
            const int left = h->head.cnt_in[0] + h->head.cnt_in[1] + h->head.cnt_in[2];
            if (left == 0) break;
            if (h->head.passes >= o.max_rounds) { status = RSOC_ENOCONV; break; }
        }
    }
    // the small graphs, one workgroup each, after the fused launches (whose
    // colour fill covers the whole batch)
    if (nsmall > 0) {
        const int sgrid = std::min(nsmall, 8192);
        const BatchArgs *A = c->b_args.as<BatchArgs>();
        if (o.mode == kOptimistic)
            o.tie ? k_bsmall<kOptimistic, kHigherKeeps><<<sgrid, kBlock, 0, s>>>(A)
                  : k_bsmall<kOptimistic, kLowerKeeps><<<sgrid, kBlock, 0, s>>>(A);
        else
            o.tie ? k_bsmall<kDeterministic, kHigherKeeps><<<sgrid, kBlock, 0, s>>>(A)
                  : k_bsmall<kDeterministic, kLowerKeeps><<<sgrid, kBlock, 0, s>>>(A);
        RSOC_LAUNCH_CHECK();
    }
    RSOC_HIP(hipEventRecord(c->ev[1], s));
    k_bcount<<<tgrid_all, kBlock, 0, s>>>(c->b_args.as<BatchArgs>(), &S->err);
    RSOC_LAUNCH_CHECK();
    RSOC_HIP(hipMemcpyAsync(&h->head, S, kStateHeader, hipMemcpyDeviceToHost, s));
    std::vector<int32_t> kg((size_t)G);
    RSOC_HIP(hipMemcpyAsync(kg.data(), c->b_kmax.p, sizeof(int32_t) * (size_t)G, hipMemcpyDeviceToHost, s));
    const bool want_hist = st && st->per_round_L && st->per_round_cap > 0;
    std::vector<int32_t> sstat((size_t)kSmallStatInts, 0);
    if (nsmall > 0)
        RSOC_HIP(hipMemcpyAsync(sstat.data(), d_small_stat,
                                sizeof(int32_t) * (size_t)(want_hist ? kSmallStatInts : kSmallStatHist),
                                hipMemcpyDeviceToHost, s));
    RSOC_HIP(hipStreamSynchronize(s));
    if (sstat[2]) status = RSOC_ENOCONV;
    int64_t small_conf = 0;
    memcpy(&small_conf, &sstat[4], sizeof(small_conf));
    const int rounds_all = std::max(ntasks > 0 ? h->head.rounds : 0, sstat[1]);
    if (want_hist) {
        const int cnt = std::min(std::min(rounds_all, st->per_round_cap), kHistCap);
        const int cf = std::min(ntasks > 0 ? h->head.rounds : 0, cnt);
        if (cf > 0)
            RSOC_HIP(hipMemcpyAsync(st->per_round_L, S->hist, sizeof(int32_t) * cf, hipMemcpyDeviceToHost, s));
        RSOC_HIP(hipStreamSynchronize(s));
        for (int r = cf; r < cnt; ++r) st->per_round_L[r] = 0;
        for (int r = 0; r < cnt && r < kSmallMax + 2; ++r) st->per_round_L[r] += sstat[kSmallStatHist + r];
    }
    if (h->head.err & (4 | kErrListCount)) return RSOC_EINTERNAL;  // never expected
    int32_t kmax = 0;
    for (int g = 0; g < G; ++g) {
        if (counts_out) counts_out[g] = kg[g];
        kmax = std::max(kmax, kg[g]);
    }
    if (st) {
        st->rounds = rounds_all;
        st->passes = std::max(ntasks > 0 ? h->head.passes : 0, sstat[0]);
        st->colors = kmax;
        st->colors_distinct = -1;
        st->conflicts = (ntasks > 0 ? h->head.conflicts : 0) + small_conf;
        st->inspected = (int64_t)h->head.inspected;
        st->max_degree = h->head.maxdeg;
        st->bin_counts[0] = (int32_t)nT;
        st->bin_counts[1] = nW;
        st->bin_counts[2] = nB;
        st->worklist0 = h->head.u0;
        st->chunk = a.gchunk ? 0 : a.chunk;
        st->small_graphs = nsmall;
        float ms = 0;
        RSOC_HIP(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        st->ms = ms;
        const int64_t nnzT = nnz_off[G];
        if (timing && ntasks > 0) {
            float m0 = 0;
            RSOC_HIP(hipEventElapsedTime(&m0, c->ev[2], c->ev[3]));
            st->ms_round0 = m0;
        }
        // round 0 (optimistic): task table 8/task, row_ptr 4(n+G), col_idx 4 nnz,
        // colours of the neighbours a vertex loses to (4 nnz/2), colour
        // writes 4n, hub lists 8(nW+nB), U^0: a 64-byte mask per task, 4 per
        // lane-group entry (its row positions read uncoloured) and 8 per listed
        // entry of the wavefront and workgroup bins (the fused launches' graphs)
        if (o.mode == kOptimistic && ntasks > 0) {
            int64_t nnzL = 0;
            int GL = 0;
            for (int g = 0; g < G; ++g)
                if (!is_small(g)) nnzL += nnz_off[g + 1] - nnz_off[g], ++GL;
            st->bytes_round0 = 8 * (int64_t)ntasks + 4 * (nVL + GL) + 4 * nnzL +
                               (o.full_sweep ? 4 * nnzL : 4 * (nnzL / 2)) + 4 * nVL + 8 * (int64_t)(nW + nB) +
                               (o.full_sweep ? 0
                                             : 8 * (int64_t)h->head.u0_listed + 4 * kTaskWords * (int64_t)ntasks +
                                                   4 * (int64_t)(h->head.u0 - h->head.u0_listed));
        }
        (void)nnzT;
    }
    if (status < 0) return status;
    return kmax;
}

}  // namespace rsoc

extern "C" int32_t rsoc_color_batch(rsoc_ctx *ctx, int32_t G, const int64_t *vtx_off, const int64_t *nnz_off,
                                    const int32_t *d_row_ptr_cat, const int32_t *d_col_idx_cat, int32_t *d_colors_cat,
                                    int32_t *counts_out, const rsoc_options *opts, rsoc_stats *stats,
                                    void *hip_stream) {
    using namespace rsoc;
    if (!ctx || G < 0 || (G > 0 && (!vtx_off || !nnz_off))) return RSOC_EINVAL;
    if (G > 0 && vtx_off[G] > 0 && (!d_row_ptr_cat || !d_colors_cat)) return RSOC_EINVAL;
    if (G > 0 && nnz_off[G] > 0 && !d_col_idx_cat) return RSOC_EINVAL;
    Options o;
    RSOC_TRY(resolve_options(opts, G > 0 ? vtx_off[G] : 0, o));
    if (o.distance == 2) return RSOC_EINVAL;  // distance 2: single-graph entry points only
    if (o.mode == kTwoPhaseLive) return RSOC_EINVAL;  // single-graph entry points only
    RSOC_HIP(hipSetDevice(ctx->device));
    return run_batch(ctx, G, vtx_off, nnz_off, d_row_ptr_cat, d_col_idx_cat, d_colors_cat, counts_out, o, stats,
                     (hipStream_t)hip_stream);
}
