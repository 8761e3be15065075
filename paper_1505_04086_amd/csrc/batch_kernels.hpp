// batch_kernels.hpp -- kernels of the batched path: many independent graphs
// coloured by the same fused launches.
//
// The batch is a concatenation of G local-id CSR graphs with int64 offset
// tables.  A round of Algorithm 3 (Section 3) over the whole batch is one
// launch: round-0 and sweep rounds walk a task table of (graph, first vertex)
// chunks; worklist rounds walk packed (graph << 32 | local id) entries.  Every
// vertex only ever meets neighbours of its own graph and ties are decided on
// local ids, so each graph is coloured exactly as a separate call colours it
// (bit-identically in the round-synchronous modes).
#pragma once

#include "single_kernels.hpp"

namespace rsoc {

constexpr int kTaskLen = kStep;  // vertices per sweep task (one workgroup step)
constexpr int kTaskWords = kTaskLen / 32;  // 32-bit words of a task's U^0 mask

struct BatchArgs {
    const int64_t *voff;  // [G+1] vertex offsets of the graphs
    const int64_t *noff;  // [G+1] adjacency offsets of the graphs
    const int32_t *rp;    // concatenated local row_ptr arrays (graph g at voff[g] + g)
    const int32_t *ci;    // concatenated local column ids (graph g at noff[g])
    int32_t *col;         // concatenated colours (graph g at voff[g])
    uint8_t *col8;        // byte shadow of col
    int32_t *pend;        // staged colours (round-synchronous modes)
    int64_t *wl[2];       // packed worklists; bin segments start at 0, offW, offB
    int64_t *hub;         // static hub lists: wavefront bin from the front, workgroup bin from the back
    const int64_t *tasks; // packed (graph << 32 | first local vertex) sweep tasks
    int32_t *kg;          // [G] per-graph max colour + 1
    int64_t nV;           // total vertices (< 2^31)
    int64_t hub_cap;      // entries of hub
    int64_t offW, offB;   // worklist segment offsets
    int32_t G, ntasks;
    int32_t t_thread, t_wave, max_rounds, look;
    int32_t chunk;        // run of consecutive ids one lane group walks
    int32_t ntasks_all;   // tasks of every graph (the first ntasks are the fused launches' graphs)
    const int32_t *small; // graphs coloured by one workgroup each (k_bsmall)
    int32_t *small_stat;  // their statistics: see k_bsmall
    int32_t nsmall;
    uint32_t *u0mask;            // optimistic round 0: per task, bit l = its l-th vertex is in U^0 (thread bin)
    uint32_t *u0pos;             // [nV] for those vertices: the row positions of the neighbours round 0 read
                                 // uncoloured (group_vertices' unc)
    uint8_t *gchunk;             // [G] run length of each graph's sweeps, when the option leaves it open (else null)
    int32_t nbands;              // optimistic round 0: sweep bands, kXcds per band index of an XCD
    int32_t band[kMaxBands + 1]; // band b is tasks [band[b], band[b+1]) (about equal work)
};

__device__ __forceinline__ int64_t pack_item(int g, int v) { return ((int64_t)g << 32) | (uint32_t)v; }
__device__ __forceinline__ int item_graph(int64_t x) { return (int)(x >> 32); }
__device__ __forceinline__ int item_vertex(int64_t x) { return (int)(uint32_t)x; }

// Base pointers of one graph of the batch.
struct GraphView {
    const RSOC_GLOBAL int32_t *rp;
    const RSOC_GLOBAL int32_t *ci;
    const RSOC_GLOBAL int32_t *col;
    const RSOC_GLOBAL uint8_t *col8;
    int64_t voff;
    int n;
};

__device__ __forceinline__ GraphView graph_view(const BatchArgs &a, int g) {
    GraphView w;
    const int64_t vo = a.voff[g];
    w.voff = vo;
    w.n = (int)(a.voff[g + 1] - vo);
    w.rp = gro(a.rp + vo + g);
    w.ci = gro(a.ci + a.noff[g]);
    w.col = gro(a.col + vo);
    w.col8 = gro(a.col8 + vo);
    return w;
}

__device__ __forceinline__ void wave_append64(bool take, int64_t x, int *counter, int64_t *list, bool from_back,
                                              int64_t cap) {
    uint64_t m = ballot(take);
    if (m == 0) return;
    int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    if (take) {
        const int64_t pos = base + lanes_below(m);
        list[from_back ? cap - 1 - pos : pos] = x;
    }
}

// The batch's optimistic rounds 0 and 1 sweep their tasks in nbands =
// kXcds * B bands of about equal work, B of them per XCD, the XCD's bands one
// contiguous part of the batch: each band is handed out in order from its own
// counter, so the tasks in flight on one XCD form B narrow ranges of its part
// (a few graphs) and those graphs' colours stay in the XCD's L2 while the
// ranges cross them.  A workgroup starts on a band of its own XCD (hardware
// deals consecutive workgroups round-robin over the XCDs) and, once that band
// is exhausted, helps the following ones, so every task is claimed exactly
// once whatever the grid and however unequal the bands turn out.
__device__ __forceinline__ int home_band(const BatchArgs &a, int bid) {
    const int per = a.nbands / kXcds;
    return (bid % kXcds) * per + (bid / kXcds) % per;
}
// Returns the next task, or -1 when every band is exhausted; *k counts the
// bands this workgroup has finished with (start at 0).  Thread 0 only.
__device__ __forceinline__ int claim_task(const BatchArgs &a, SingleState *S, int home, int *k) {
    while (*k < a.nbands) {
        const int x = (home + *k) % a.nbands;
        const int lo = a.band[x], hi = a.band[x + 1];
        if (lo < hi) {
            const int i = atomicAdd(&S->next_task[x], 1);
            if (i < hi - lo) return lo + i;
        }
        ++*k;
    }
    return -1;
}

// --------------------------------------------------------------- binning --
// Appends x for every lane with `take` to the wavefront's LDS buffer buf
// (*bn entries, at most kWave); when the ballot would overflow it, the buffer
// first goes to the static hub list (one global atomic per flush).  Called by
// the whole wavefront in lockstep.
__device__ __forceinline__ void wave_hub_flush(int64_t *buf, int *bn, int *counter, int64_t *hub, bool from_back,
                                               int64_t cap) {
    const int cnt = *bn;
    if (cnt == 0) return;
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, cnt);
    base = __shfl(base, 0);
    if (lane_id() < cnt) {
        const int64_t pos = (int64_t)base + lane_id();
        hub[from_back ? cap - 1 - pos : pos] = buf[lane_id()];
    }
    wave_lds_sync();
    if (lane_id() == 0) *bn = 0;
    wave_lds_sync();
}
__device__ __forceinline__ void wave_hub_push(bool take, int64_t x, int64_t *buf, int *bn, int *counter, int64_t *hub,
                                              bool from_back, int64_t cap) {
    const uint64_t m = ballot(take);
    if (m == 0) return;
    if (*bn + __popcll(m) > kWave) wave_hub_flush(buf, bn, counter, hub, from_back, cap);
    if (take) buf[*bn + lanes_below(m)] = x;
    wave_lds_sync();
    if (lane_id() == 0) *bn += __popcll(m);
    wave_lds_sync();
}

// Degree bins of the fused launches' graphs: one wavefront per task (no
// workgroup barrier), rows above t_wave to the workgroup hub list (from the
// back of `hub`), rows above t_thread to the wavefront list (from the front);
// the lane-group bin needs no list (the sweeps walk the tasks).
__global__ __launch_bounds__(kBlock) void k_bbin(const BatchArgs *__restrict__ A, SingleState *S) {
    __shared__ int64_t qW[kWavesPerBlock][kWave], qB[kWavesPerBlock][kWave];
    __shared__ int nqW[kWavesPerBlock], nqB[kWavesPerBlock];
    const BatchArgs a = *A;
    const int wv = threadIdx.x / kWave;
    const int nwv = (int)gridDim.x * kWavesPerBlock;
    if (lane_id() == 0) nqW[wv] = nqB[wv] = 0;
    wave_lds_sync();
    int md = 0;
    for (int t = (int)blockIdx.x * kWavesPerBlock + wv; t < a.ntasks; t += nwv) {
        const int64_t task = a.tasks[t];
        const int g = item_graph(task), start = item_vertex(task);
        const GraphView w = graph_view(a, g);
        const int end = min(w.n, start + kTaskLen);
        // every row_ptr pair of the task in flight at once, then the appends
        constexpr int kPer = kTaskLen / kWave;
        int d[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int v = start + k * kWave + lane_id();
            d[k] = v < end ? w.rp[v + 1] - w.rp[v] : -1;
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int v = start + k * kWave + lane_id();
            md = max(md, d[k]);
            wave_hub_push(d[k] > a.t_wave, pack_item(g, v), qB[wv], &nqB[wv], &S->nB, a.hub, true, a.hub_cap);
            wave_hub_push(d[k] > a.t_thread && d[k] <= a.t_wave, pack_item(g, v), qW[wv], &nqW[wv], &S->nW, a.hub,
                          false, a.hub_cap);
        }
    }
    wave_hub_flush(qB[wv], &nqB[wv], &S->nB, a.hub, true, a.hub_cap);
    wave_hub_flush(qW[wv], &nqW[wv], &S->nW, a.hub, false, a.hub_cap);
    md = wave_max_i32(md);
    if (lane_id() == 0 && md > __hip_atomic_load(&S->maxdeg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&S->maxdeg, md);
}

// Run length per graph (the option chunk = 0): one wavefront per graph reads
// up to 64 rows spread over the graph and picks kChunk when at least 2 % of
// their entries join ids less than kChunk apart (a grid in natural order),
// else 1 (random ids, where runs only spread a wavefront's rows and writes
// over more cache lines).
__global__ __launch_bounds__(kBlock) void k_bchunk(const BatchArgs *__restrict__ A) {
    const BatchArgs a = *A;
    const int g = (int)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
    if (g >= a.G) return;
    const GraphView w = graph_view(a, g);
    uint64_t near = 0, sampled = 0;
    const int ns = min(w.n, kWave);
    if (lane_id() < ns) locality_row(w.rp, w.ci, (int)((int64_t)lane_id() * w.n / ns), w.rp[w.n], near, sampled);
    near = wave_sum_u64(near);
    sampled = wave_sum_u64(sampled);
    if (lane_id() == 0) a.gchunk[g] = (uint8_t)pick_chunk(0, near, sampled);
}

__global__ __launch_bounds__(kBlock) void k_bvalidate(const BatchArgs *__restrict__ A, int32_t *err) {
    const BatchArgs a = *A;
    int flags = 0;
    for (int t = blockIdx.x; t < a.ntasks_all; t += gridDim.x) {
        const int64_t task = a.tasks[t];
        const int g = item_graph(task), start = item_vertex(task);
        const GraphView w = graph_view(a, g);
        const int end = min(w.n, start + kTaskLen);
        const int64_t nnz = a.noff[g + 1] - a.noff[g];
        if (start == 0 && threadIdx.x == 0 && w.rp[0] != 0) flags |= 1;
        for (int v = start + threadIdx.x; v < end; v += kBlock) {
            const int b = w.rp[v], e = w.rp[v + 1];
            if (b > e || b < 0 || (int64_t)e > nnz) { flags |= 1; continue; }
            for (int j = b; j < e; ++j) {
                const int u = w.ci[j];
                if ((unsigned)u >= (unsigned)w.n) flags |= 1;
                else if (u == v) flags |= 2;
            }
        }
    }
    if (ballot(flags != 0)) {
        int f = flags;
        for (int off = 32; off > 0; off >>= 1) f |= __shfl_xor(f, off);
        if (lane_id() == 0) atomicOr(err, f);
    }
}

// Appends packed items into the workgroup's LDS queue / flushes it.
__device__ __forceinline__ void queue_push64(bool take, int64_t x, int64_t *q, int *qn) {
    const uint64_t m = ballot(take);
    if (m == 0) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(qn, __popcll(m));
    base = __shfl(base, leader);
    if (take) q[base + lanes_below(m)] = x;
}

// cnt: the queue size every wavefront agreed on (see queue_flush_n).
__device__ __forceinline__ void queue_flush64_n(int cnt, int64_t *q, int *qn, int *qbase, int *counter, int64_t *out) {
    if (cnt == 0) return;
    if (threadIdx.x == 0) {
        *qbase = atomicAdd(counter, cnt);
        *qn = 0;
    }
    __syncthreads();
    const int base = *qbase;
    for (int i = threadIdx.x; i < cnt; i += kBlock) out[base + i] = q[i];
    __syncthreads();
}
__device__ __forceinline__ void queue_flush64(int64_t *q, int *qn, int *qbase, int *counter, int64_t *out) {
    queue_flush64_n(queue_size(qn), q, qn, qbase, counter, out);
}

// ----------------------------------------------------------------- round --
// Same contract as k_round (PHASE, MODE, TIE, SWEEP, ROUND0), over the batch.
// Batched round 1, lane groups: the vertices of `list` (n entries, ids of the
// task's graph tw) recoloured kGroup lanes each -- PH = kAssign gives a vertex
// known to be defective First-Fit over all its neighbours, PH = kRecolor
// detects first -- written in place and appended to the next list.  Called by
// the whole workgroup (n is the same for every thread).
template <int PH, int TIE>
__device__ __forceinline__ void task_recolour(const int *list, int n, const GraphView &tw, int tg, int look,
                                              RSOC_GLOBAL int32_t *wcol, RSOC_GLOBAL uint8_t *wcol8, int64_t *q,
                                              int *qn, int *qbase, int *counter, int64_t *out, uint64_t &degs) {
    const int gi = threadIdx.x / kGroup;
    const bool leader = (threadIdx.x & (kGroup - 1)) == 0;
    for (int base = 0; base < n; base += kSub) {
        int v[kNV], b[kNV], e[kNV], cv[kNV], nc[kNV];
        bool act[kNV];
        uint32_t unc[kNV] = {};
        const RSOC_GLOBAL int32_t *cis[kNV];
        const RSOC_GLOBAL uint8_t *c8s[kNV];
#pragma unroll
        for (int i = 0; i < kNV; ++i) {
            const int idx = base + i * kGpb + gi;
            v[i] = idx < n ? list[idx] : -1;
            b[i] = e[i] = 0;
            cis[i] = tw.ci;
            c8s[i] = tw.col8;
            if (v[i] >= 0) {
                b[i] = tw.rp[v[i]];
                e[i] = tw.rp[v[i] + 1];
            }
            cv[i] = (PH != kAssign && v[i] >= 0) ? (int)tw.col8[v[i]] : 255;
        }
        group_vertices<PH, TIE, kGroup, kGroupSlots, false, kNV>(v, b, e, cis, c8s, cv, look, nc, act, unc);
#pragma unroll
        for (int i = 0; i < kNV; ++i) {
            if (v[i] < 0) act[i] = false;
            if (leader && v[i] >= 0) {
                degs += (uint64_t)(e[i] - b[i]);
                if (act[i]) {
                    wcol[tw.voff + v[i]] = nc[i];
                    wcol8[tw.voff + v[i]] = (uint8_t)nc[i];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kNV; ++i) queue_push64(act[i] && leader, pack_item(tg, v[i]), q, qn);
        const int cq = queue_size(qn);
        if (cq > kQueueCap - kSub) queue_flush64_n(cq, q, qn, qbase, counter, out);
    }
}

template <int PHASE, int MODE, int TIE, bool SWEEP, int ROUND0 = 0>
__global__ __launch_bounds__(kBlock) void k_bround(const BatchArgs *__restrict__ A, SingleState *S, int parity,
                                                   int gB, int gW, int gT) {
    __shared__ uint32_t lds[kLdsWords];
    __shared__ int64_t q[kQueueCap];
    __shared__ int sh_min, qn, qbase, sh_step, tcount;
    __shared__ unsigned long long sh_acc[2];
    __shared__ int64_t wbuf[kWavesPerBlock][kWaveBuf];
    __shared__ int wbn[kWavesPerBlock];
    const BatchArgs a = *A;
    if (!SWEEP && S->passes >= a.max_rounds) return;
    // Optimistic round 0 records the thread-bin part of U^0 as one bit mask
    // per task (kMaskU0) and round 1 walks those masks (kTaskList), claiming
    // the tasks band by band as round 0 did: it then meets each graph in the
    // same narrow ranges, on the same XCD, with the colours it reads in L2
    // (a packed list in append order would send each XCD's round 1 to every
    // graph of every band at once).
    constexpr bool kMaskU0 = PHASE == kAssign && ROUND0 == 1;
    constexpr bool kTaskList = PHASE == kRecolor && ROUND0 == 2 && !SWEEP && MODE == kOptimistic;
    __shared__ uint32_t tmask[kMaskU0 ? kTaskWords : 1];
    __shared__ int16_t tpos[kTaskList ? kTaskLen : 1];
    __shared__ int tdef[kTaskList ? kTaskLen : 1], tover[kTaskList ? kTaskLen : 1];
    __shared__ int ndef, nover;
    const int cT = SWEEP ? a.ntasks : S->cnt_in[kBinThread];
    const int cW = SWEEP ? S->nW : S->cnt_in[kBinWave];
    const int cB = SWEEP ? S->nB : S->cnt_in[kBinBlock];
    int64_t *const in = parity ? a.wl[1] : a.wl[0];
    int64_t *const out = parity ? a.wl[0] : a.wl[1];
    constexpr bool kFlagAppend = PHASE == kAssign && ROUND0 == 1;
    constexpr bool kWinOnly = kFlagAppend;
    constexpr bool kAppend = PHASE != kAssign || kFlagAppend;
    constexpr bool kWrite = PHASE != kDetect;
    constexpr bool kAcct = PHASE != kAssign && !SWEEP;
    constexpr bool kQueueT = kAppend && !kMaskU0;  // thread-bin appends go through the LDS queue
    RSOC_GLOBAL int32_t *wcolg = grw((MODE == kOptimistic) ? a.col : a.pend);
    RSOC_GLOBAL uint8_t *wcol8g = grw(a.col8);
    uint64_t items = 0, degs = 0, flagged = 0;
    const int bid = blockIdx.x;
    if (bid < gB) {
        if (threadIdx.x == 0) qn = 0;
        __syncthreads();
        for (int i = bid; i < cB; i += gB) {
            const int64_t it = SWEEP ? a.hub[a.hub_cap - 1 - i] : in[a.offB + i];
            const int g = item_graph(it), v = item_vertex(it);
            const GraphView w = graph_view(a, g);
            const int b = w.rp[v], e = w.rp[v + 1];
            int nc = 0;
            bool unc = false;
            const bool act = block_vertex<PHASE, TIE, kWinOnly>(v, b, e, w.ci, w.col, w.col8, lds, &sh_min, a.look, nc, unc);
            const bool take = (kFlagAppend ? unc : act) && kAppend;
            if (threadIdx.x == 0) {
                items += 1;
                degs += (uint64_t)(e - b);
                if (act && kWrite) {
                    wcolg[w.voff + v] = nc;
                    if (MODE == kOptimistic) wcol8g[w.voff + v] = shadow_of(nc);
                }
                if (take) q[qn++] = it;
            }
            const int cq = queue_size(&qn);
            if (cq == kQueueCap) queue_flush64_n(cq, q, &qn, &qbase, &S->cnt_out[kBinBlock], out + a.offB);
        }
        if (kAppend) queue_flush64(q, &qn, &qbase, &S->cnt_out[kBinBlock], out + a.offB);
    } else if (bid < gB + gW) {
        const int wv = threadIdx.x / kWave;
        const int wi = (bid - gB) * kWavesPerBlock + wv;
        const int nw = gW * kWavesPerBlock;
        uint32_t *bm = lds + wv * kWaveWindowWords;
        if (lane_id() == 0) wbn[wv] = 0;
        wave_lds_sync();
        for (int i = wi; i < cW; i += nw) {
            const int64_t it = SWEEP ? a.hub[i] : in[a.offW + i];
            const int g = item_graph(it), v = item_vertex(it);
            const GraphView w = graph_view(a, g);
            const int b = w.rp[v], e = w.rp[v + 1];
            int nc = 0;
            bool unc = false;
            const bool act = wave_vertex<PHASE, TIE, kWinOnly>(v, b, e, w.ci, w.col, w.col8, bm, a.look, nc, unc);
            if (lane_id() == 0) {
                items += 1;
                degs += (uint64_t)(e - b);
                if (act && kWrite) {
                    wcolg[w.voff + v] = nc;
                    if (MODE == kOptimistic) wcol8g[w.voff + v] = shadow_of(nc);
                }
            }
            if (kAppend) wave_buf_push<int64_t>((kFlagAppend ? unc : act), it, wbuf[wv], &wbn[wv],
                                                &S->cnt_out[kBinWave], out + a.offW);
        }
        if (kAppend) wave_buf_flush<int64_t>(wbuf[wv], &wbn[wv], &S->cnt_out[kBinWave], out + a.offW);
    } else {
        const int tb = bid - gB - gW;
        const int gi = threadIdx.x / kGroup;
        const bool leader = (threadIdx.x & (kGroup - 1)) == 0;
        if (kQueueT) {
            if (threadIdx.x == 0) qn = 0;
            __syncthreads();
        }
        if (kMaskU0 && threadIdx.x < kTaskWords) tmask[threadIdx.x] = 0;
        // SWEEP: one task (a chunk of one graph) per workgroup step;
        // worklist rounds: kStep packed items per step.
        // Optimistic round 0 claims its tasks band by band (claim_task).  A
        // fixed stride over the task table instead lets workgroups drift apart
        // over a long sweep: the tasks in flight then span many graphs at once,
        // whose colour gathers (random ids in a geometric graph) evict one
        // another from L2, and the rounds read several times the bytes.
        constexpr bool kClaim = (SWEEP && ROUND0 == 1) || kTaskList;
        const int64_t nsteps = SWEEP       ? (int64_t)a.ntasks
                               : kTaskList ? (cT > 0 ? (int64_t)a.ntasks : 0)
                                           : ((int64_t)cT + kStep - 1) / kStep;
        int64_t step = tb;
        int bands_done = 0;
        if (kClaim) {
            if (threadIdx.x == 0) sh_step = claim_task(a, S, home_band(a, bid), &bands_done);
            __syncthreads();
            step = sh_step < 0 ? nsteps : sh_step;
        }
        while (step < nsteps) {
            // the next task is claimed when this one starts (the claim's round
            // trip overlaps this task's loads)
            int next = 0;
            if (kClaim && threadIdx.x == 0) next = claim_task(a, S, home_band(a, bid), &bands_done);
            int tg = 0, tstart = 0, tlen = 0, tcur = 0;
            GraphView tw = {};
            if (SWEEP || kTaskList) {
                tcur = ((kFlagAppend || kTaskList) && TIE == kHigherKeeps) ? (int)(nsteps - 1 - step) : (int)step;
                const int64_t task = a.tasks[tcur];
                tg = item_graph(task);
                tstart = item_vertex(task);
                tw = graph_view(a, tg);
                tlen = min(kTaskLen, tw.n - tstart);
            }
            const int tchunk = (SWEEP && a.gchunk) ? (int)a.gchunk[tg] : a.chunk;
            if (kTaskList) {
                // the task's U^0 positions, compacted in LDS by the first wavefront
                if (threadIdx.x < kWave) {
                    const uint32_t m = threadIdx.x < kTaskWords
                                           ? gro(a.u0mask)[(int64_t)tcur * kTaskWords + threadIdx.x] : 0u;
                    int incl = __popc(m);
#pragma unroll
                    for (int d = 1; d < kTaskWords; d <<= 1) {
                        const int o = __shfl_up(incl, d);
                        if (lane_id() >= d) incl += o;
                    }
                    int k = incl - __popc(m);
                    for (uint32_t mm = m; mm; mm &= mm - 1) tpos[k++] = (int16_t)(threadIdx.x * 32 + __builtin_ctz(mm));
                    if (threadIdx.x == kTaskWords - 1) tcount = incl;
                    if (threadIdx.x == 0) ndef = nover = 0;
                }
                __syncthreads();
                const int cnt = tcount;
                // one thread per vertex of U^0: only the neighbours round 0 read
                // uncoloured (at most three, at the row positions it recorded)
                // can hold its colour; a defective vertex, and one with more
                // than three such neighbours, goes to the lane groups below (as
                // the single-graph masked round)
                for (int idx = threadIdx.x; idx < cnt; idx += kBlock) {
                    const int li = tpos[idx];
                    const int v = TIE == kHigherKeeps ? tstart + tlen - 1 - li : tstart + li;
                    const uint32_t pm = gro(a.u0pos)[tw.voff + v];
                    const int cv = tw.col8[v];
                    const bool over = __popc(pm) > 3;
                    int4 x = make_int4(-1, -1, -1, (int)pm);
                    if (!over) {
                        const int b = tw.rp[v];
                        uint32_t mm = pm;
                        if (mm) { x.x = tw.ci[b + __builtin_ctz(mm)]; mm &= mm - 1; }
                        if (mm) { x.y = tw.ci[b + __builtin_ctz(mm)]; mm &= mm - 1; }
                        if (mm) x.z = tw.ci[b + __builtin_ctz(mm)];
                    }
                    const bool def = !over && lane_detect_kept<false>(v, x, cv, tw.col8, nullptr);
                    items += 1;
                    degs += (uint64_t)__popc(pm);
                    if (def) tdef[atomicAdd(&ndef, 1)] = v;
                    if (over) tover[atomicAdd(&nover, 1)] = v;
                }
                __syncthreads();
                task_recolour<kAssign, TIE>(tdef, ndef, tw, tg, a.look, wcolg, wcol8g, q, &qn, &qbase,
                                            &S->cnt_out[kBinThread], out, degs);
                task_recolour<kRecolor, TIE>(tover, nover, tw, tg, a.look, wcolg, wcol8g, q, &qn, &qbase,
                                             &S->cnt_out[kBinThread], out, degs);
            }
            for (int r = 0; r < (kTaskList ? 0 : kChunk); ++r) {
                int v[kNV], b[kNV], e[kNV], cv[kNV], nc[kNV], gg[kNV];
                bool act[kNV];
                uint32_t unc[kNV] = {};
                const RSOC_GLOBAL int32_t *cis[kNV];
                const RSOC_GLOBAL uint8_t *c8s[kNV];
                int64_t vo[kNV];
#pragma unroll
                for (int i = 0; i < kNV; ++i) {
                    v[i] = -1;
                    b[i] = e[i] = 0;
                    gg[i] = 0;
                    const int li = step_offset(r, i, gi, tchunk);
                    if (SWEEP) {
                        if (li < tlen) v[i] = (kFlagAppend && TIE == kHigherKeeps) ? tstart + tlen - 1 - li : tstart + li;
                        gg[i] = tg;
                        cis[i] = tw.ci;
                        c8s[i] = tw.col8;
                        vo[i] = tw.voff;
                        if (v[i] >= 0) {
                            b[i] = tw.rp[v[i]];
                            e[i] = tw.rp[v[i] + 1];
                        }
                    } else {
                        const int64_t idx = step * kStep + li;
                        cis[i] = gro(a.ci);
                        c8s[i] = gro(a.col8);
                        vo[i] = 0;
                        if (idx < cT) {
                            const int64_t it = in[idx];
                            gg[i] = item_graph(it);
                            v[i] = item_vertex(it);
                            const GraphView w = graph_view(a, gg[i]);
                            cis[i] = w.ci;
                            c8s[i] = w.col8;
                            vo[i] = w.voff;
                            b[i] = w.rp[v[i]];
                            e[i] = w.rp[v[i] + 1];
                        }
                    }
                    if (SWEEP && v[i] >= 0 && e[i] - b[i] > a.t_thread) e[i] = b[i] = 0, v[i] = -1;
                    cv[i] = (PHASE != kAssign && v[i] >= 0) ? (int)c8s[i][v[i]] : 255;
                }
                group_vertices<PHASE, TIE, kGroup, kGroupSlots, kWinOnly, kNV>(v, b, e, cis, c8s, cv, a.look, nc,
                                                                               act, unc);
#pragma unroll
                for (int i = 0; i < kNV; ++i) {
                    if (v[i] < 0) {
                        act[i] = false;
                        unc[i] = 0;
                    }
                    if (leader && v[i] >= 0) {
                        items += 1;
                        degs += (uint64_t)(e[i] - b[i]);
                        if (act[i] && kWrite) {
                            wcolg[vo[i] + v[i]] = nc[i];
                            if (MODE == kOptimistic) wcol8g[vo[i] + v[i]] = (uint8_t)nc[i];
                        }
                    }
                }
                if (kMaskU0) {
#pragma unroll
                    for (int i = 0; i < kNV; ++i)
                        if (leader && unc[i] != 0) {
                            const int li = step_offset(r, i, gi, tchunk);
                            atomicOr(&tmask[li >> 5], 1u << (li & 31));
                            a.u0pos[vo[i] + v[i]] = unc[i];
                            flagged += 1;
                        }
                }
                if (kQueueT) {
#pragma unroll
                    for (int i = 0; i < kNV; ++i)
                        queue_push64((kFlagAppend ? unc[i] != 0 : act[i]) && leader, pack_item(gg[i], v[i]), q, &qn);
                    const int cq = queue_size(&qn);
                    if (cq > kQueueCap - kSub) queue_flush64_n(cq, q, &qn, &qbase, &S->cnt_out[kBinThread], out);
                }
            }
            if (kClaim) {
                __syncthreads();  // every thread has read sh_step (and set its flags in tmask)
                if (threadIdx.x == 0) sh_step = next;
                if (kMaskU0 && threadIdx.x < kTaskWords) {
                    a.u0mask[(int64_t)tcur * kTaskWords + threadIdx.x] = tmask[threadIdx.x];
                    tmask[threadIdx.x] = 0;  // cleared before the barrier that opens the next task
                }
                __syncthreads();
                step = sh_step < 0 ? nsteps : sh_step;
            } else {
                step += gT;
            }
        }
        if (kQueueT) queue_flush64(q, &qn, &qbase, &S->cnt_out[kBinThread], out);
    }
    if (kMaskU0) {
        // |U^0|'s thread-bin part (the masks hold the entries themselves)
        flagged = wave_sum_u64(flagged);
        if (lane_id() == 0 && flagged) atomicAdd(&S->cnt_out[kBinThread], (int)flagged);
    }
    if (kAcct) {
        if (threadIdx.x == 0) { sh_acc[0] = 0; sh_acc[1] = 0; }
        __syncthreads();
        items = wave_sum_u64(items);
        degs = wave_sum_u64(degs);
        if (lane_id() == 0 && items) {
            atomicAdd(&sh_acc[0], (unsigned long long)items);
            atomicAdd(&sh_acc[1], (unsigned long long)degs);
        }
        __syncthreads();
        if (threadIdx.x == 0 && sh_acc[0]) {
            atomicAdd((unsigned long long *)&S->inspected, sh_acc[0]);
            atomicAdd((unsigned long long *)&S->deg_sum, sh_acc[1]);
        }
    }
}

// --------------------------------------------------------------- scatter --
template <bool SWEEP, bool USE_IN>
__global__ __launch_bounds__(kBlock) void k_bscatter(const BatchArgs *__restrict__ A, SingleState *S, int parity) {
    const BatchArgs a = *A;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    RSOC_GLOBAL int32_t *col = grw(a.col);
    RSOC_GLOBAL uint8_t *col8 = grw(a.col8);
    const RSOC_GLOBAL int32_t *pend = gro(a.pend);
    if (SWEEP) {
        for (int64_t x = t0; x < a.nV; x += stride) {
            const int c = pend[x];
            col[x] = c;
            col8[x] = shadow_of(c);
        }
        return;
    }
    if (S->passes >= a.max_rounds) return;
    const bool use_wl1 = USE_IN ? (parity != 0) : (parity == 0);
    const int64_t *lst = use_wl1 ? a.wl[1] : a.wl[0];
    const int32_t *cnt = USE_IN ? S->cnt_in : S->cnt_out;
    for (int bin = 0; bin < 3; ++bin) {
        const int c = cnt[bin];
        const int64_t off = bin == 0 ? 0 : (bin == 1 ? a.offW : a.offB);
        for (int64_t i = t0; i < c; i += stride) {
            const int64_t it = lst[off + i];
            const int64_t x = a.voff[item_graph(it)] + item_vertex(it);
            const int cc = pend[x];
            col[x] = cc;
            col8[x] = shadow_of(cc);
        }
    }
}

template <int MODE, bool SWEEP, bool PUBLISH_ONLY = false>
__global__ void k_bround_end(const BatchArgs *__restrict__ A, SingleState *S) {
    if (threadIdx.x != 0) return;
    if (PUBLISH_ONLY) {
        S->u0 = S->cnt_out[0] + S->cnt_out[1] + S->cnt_out[2];
        S->u0_listed = S->cnt_out[1] + S->cnt_out[2];
        for (int x = 0; x < kMaxBands; ++x) S->next_task[x] = 0;  // round 1 claims the tasks again
        for (int b = 0; b < 3; ++b) {
            S->cnt_in[b] = S->cnt_out[b];
            S->cnt_out[b] = 0;
        }
        return;
    }
    if (!SWEEP && S->passes >= A->max_rounds) return;
    const int in_total = SWEEP ? (int)A->nV : (S->cnt_in[0] + S->cnt_in[1] + S->cnt_in[2]);
    const int out_total = S->cnt_out[0] + S->cnt_out[1] + S->cnt_out[2];
    if (in_total > 0) {
        S->passes += 1;
        if (MODE == kTwoPhase || out_total > 0) {
            if (S->rounds < kHistCap) S->hist[S->rounds] = out_total;
            S->rounds += 1;
            S->conflicts += out_total;
        }
    }
    for (int b = 0; b < 3; ++b) {
        S->cnt_in[b] = S->cnt_out[b];
        S->cnt_out[b] = 0;
    }
}

// Per-graph colour count: kg[g] = max colour + 1; flags colours outside [0, n_g).
__global__ __launch_bounds__(kBlock) void k_bcount(const BatchArgs *__restrict__ A, int32_t *err) {
    // one wavefront per task, no workgroup barrier
    const BatchArgs a = *A;
    const int nwv = (int)gridDim.x * kWavesPerBlock;
    for (int t = (int)blockIdx.x * kWavesPerBlock + (int)threadIdx.x / kWave; t < a.ntasks_all; t += nwv) {
        const int64_t task = a.tasks[t];
        const int g = item_graph(task), start = item_vertex(task);
        const GraphView w = graph_view(a, g);
        const int end = min(w.n, start + kTaskLen);
        // the task's colours, all loads in flight at once
        constexpr int kPer = kTaskLen / kWave;
        int c[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int v = start + k * kWave + lane_id();
            c[k] = v < end ? w.col[v] : -1;
        }
        int m = -1;
        bool bad = false;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const bool in = start + k * kWave + lane_id() < end;
            bad |= in && (c[k] < 0 || c[k] >= w.n);
            m = max(m, c[k]);
        }
        if (ballot(bad) && lane_id() == 0) atomicOr(err, 4);
        m = wave_max_i32(m);
        if (lane_id() == 0 && m + 1 > __hip_atomic_load(&a.kg[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&a.kg[g], m + 1);
    }
}

// ------------------------------------------------------ small graphs --
// Graphs of at most kSmallMaxVertices vertices, one workgroup each: all of
// Algorithm 3 (Section 3) inside the workgroup, with __syncthreads() as the
// round barrier and the colours, staged colours and worklists in LDS; one
// thread per vertex (v = t, t + 256, ...).  MODE kDeterministic is the
// round-synchronous reading (round 0 colours every vertex 0, U^0 = V; a round
// tests and recolours from the colours of the previous barrier and publishes
// the staged colours after it), so each graph comes out as the oracle's
// schedule colours it.  MODE kOptimistic reads the colours as they stand:
// round 0 gives every vertex the smallest colour absent among its neighbours
// coloured at that moment, then rounds over U^0 = V detect (a neighbour the
// vertex loses to holds its colour) and recolour in place.  Row bounds are
// clamped into the graph's own adjacency and neighbour ids outside [0, n)
// are skipped, so unchecked input cannot reach outside it.
// small_stat: [0] most passes, [1] most recolouring rounds, [2] 1 if a graph
// hit max_rounds, [4..5] conflicts (64-bit), from [8] |L| per round summed
// over the graphs.
constexpr int kSmallMax = kSmallMaxVertices;
constexpr int kSmallStatHist = 8;

// smallest colour absent among v's neighbours whose colours are >= 0 (colours
// below 64 at a time: a colour is at most the degree, so the windows end)
__device__ __forceinline__ int small_first_fit(int v, int b, int e, const RSOC_GLOBAL int32_t *ci, int n,
                                               const volatile int *c) {
    for (int base = 0;; base += 64) {
        uint64_t used = 0;
        for (int j = b; j < e; ++j) {
            const int u = ci[j];
            if ((unsigned)u >= (unsigned)n || u == v) continue;
            const int x = c[u] - base;
            if (x >= 0 && x < 64) used |= 1ull << x;
        }
        if (~used) return base + __builtin_ctzll(~used);
    }
}

template <int MODE, int TIE>
__global__ __launch_bounds__(kBlock) void k_bsmall(const BatchArgs *__restrict__ A) {
    __shared__ int c[kSmallMax];
    __shared__ int p[MODE == kDeterministic ? kSmallMax : 1];
    __shared__ int lst[2][kSmallMax];
    __shared__ int nU, nL;
    const BatchArgs a = *A;
    const int t = threadIdx.x;
    int32_t *stat = a.small_stat;
    volatile int *cv = c;
    for (int k = blockIdx.x; k < a.nsmall; k += gridDim.x) {
        const int g = a.small[k];
        const GraphView w = graph_view(a, g);
        const int n = min(w.n, kSmallMax);
        const int nnz = (int)(a.noff[g + 1] - a.noff[g]);
        auto row = [&](int v, int &b, int &e) {
            b = min(max(w.rp[v], 0), nnz);
            e = min(max(w.rp[v + 1], b), nnz);
        };
        for (int v = t; v < n; v += kBlock) {
            c[v] = MODE == kDeterministic ? 0 : -1;
            lst[0][v] = v;
        }
        if (t == 0) {
            nU = n;
            nL = 0;
        }
        __syncthreads();
        if (MODE == kOptimistic) {
            for (int v = t; v < n; v += kBlock) {
                int b, e;
                row(v, b, e);
                cv[v] = small_first_fit(v, b, e, w.ci, n, cv);
            }
            __syncthreads();
        }
        int passes = 0, rounds = 0, par = 0;
        int64_t conf = 0;
        for (;;) {
            const int m = nU;
            if (m == 0) break;
            if (passes >= a.max_rounds) {
                if (t == 0) atomicOr(stat + 2, 1);
                break;
            }
            const int *U = lst[par];
            int *L = lst[par ^ 1];
            for (int i = t; i < m; i += kBlock) {
                const int v = U[i];
                int b, e;
                row(v, b, e);
                const int mine = cv[v];
                bool def = false;
                for (int j = b; j < e && !def; ++j) {
                    const int u = w.ci[j];
                    if ((unsigned)u >= (unsigned)n || u == v) continue;
                    def = loses<TIE>(v, u) && cv[u] == mine;
                }
                if (!def) continue;
                const int nc = small_first_fit(v, b, e, w.ci, n, cv);
                if (MODE == kDeterministic) p[v] = nc;
                else cv[v] = nc;
                L[atomicAdd(&nL, 1)] = v;
            }
            __syncthreads();
            const int l = nL;
            if (MODE == kDeterministic)
                for (int i = t; i < l; i += kBlock) c[L[i]] = p[L[i]];
            __syncthreads();
            ++passes;
            if (l) {
                ++rounds;
                conf += l;
                if (t == 0 && rounds <= kSmallMax + 1) atomicAdd(stat + kSmallStatHist + rounds - 1, l);
            }
            if (t == 0) {
                nU = l;
                nL = 0;
            }
            par ^= 1;
            __syncthreads();
        }
        int32_t *out = a.col + w.voff;
        for (int v = t; v < n; v += kBlock) out[v] = c[v];
        if (t == 0) {
            atomicMax(stat + 0, passes);
            atomicMax(stat + 1, rounds);
            atomicAdd(reinterpret_cast<unsigned long long *>(stat + 4), (unsigned long long)conf);
        }
        __syncthreads();  // the LDS arrays are the next graph's
    }
}

}  // namespace rsoc
