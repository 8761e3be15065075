// pool_kernels.hpp -- kernels of the continuous-batching pool.
//
// A pool slot is one admitted graph with its own worklists.  One pool step is
// one fused launch over a task table whose tasks belong to different slots
// and different rounds: a slot admitted since the last step runs its round 0
// (optimistic) or round 1 (round-synchronous) in the same launch in which
// older slots run a later worklist round.  Mode and tie rule are per slot.
#pragma once

#include "hub_kernels.hpp"
#include "single_kernels.hpp"

namespace rsoc {

enum PoolPhase : int { kSlotFree = 0, kSlotNew = 1, kSlotRunning = 2, kSlotDone = 3 };
// kRecolorMasked: the thread-bin part of an optimistic slot's first worklist
// round, whose entries carry what round 0 kept for them (see k_round's ROUND0)
enum PoolTaskKind : int { kAssignSweep = 0, kRecolorSweep = 1, kRecolorList = 2, kRecolorMasked = 3 };
constexpr int kPoolAuxCap = 256;     // round-0 queue length when entries carry their kept neighbours
constexpr int kPoolMaskedBuf = 512;  // per-wavefront append buffer of the masked round
constexpr int kPoolTaskT = kStep;  // thread-bin items per task (one workgroup step)
constexpr int kPoolTaskW = 32;   // wavefront-bin items per task
constexpr int kPoolTaskB = 2;    // workgroup-bin items per task

struct PoolSlot {
    const int32_t *rp, *ci;
    int32_t *col;
    uint8_t *col8;
    uint32_t *col4;     // 4-bit shadow read and published by round 0 (optimistic slots)
    int4 *aux;          // round 0's kept neighbours of U^0's thread-bin entries (optimistic slots)
    int32_t *pend;
    int32_t *wl[2];
    int32_t *hubW, *hubB;
    int64_t nnz;
    int64_t conflicts;
    int32_t n, mode, tie, max_rounds, t_thread, t_wave, look, parity;
    int32_t offW, offB;
    int32_t cnt_in[4], cnt_out[4];
    int32_t nW, nB, maxdeg, passes, rounds, kmax, err, phase, u0, status;
    int32_t chunk, masked;  // masked: the next round is the first worklist round after round 0
    const int32_t *touched;  // recolouring after edits: the touched vertices (nt of them)
    int32_t nt, recolor;     // recolor: the slot starts from the colouring in col
    uint64_t near, sampled;  // id locality sample (admission)
    uint32_t cbits[8];       // colours below 255 in use (k_pcount, once the slot is done)
    int32_t distinct;        // distinct colours of 255 and more (k_pdistinct)
    // hub-first round 0 (hub_kernels.hpp): hub_opt is the option (0 off, -1
    // automatic threshold, else the threshold); nH hubs were coloured at
    // admission, those above hub_t (written together by k_hub_ff)
    int32_t hub_opt, nH, hub_t;
};

// Hub-first pass of an optimistic slot at admission, with the single-graph
// kernels and a SingleArgs / SingleState of the admission stream's own (the
// admissions on one stream run one after another): k_phub_collect fills them
// from the slot and collects the hubs, k_hub_lists and k_hub_ff colour them,
// and k_hub_ff's last act copies their number and threshold into the slot
// and clears the counts for the stream's next admission (they start zeroed).
__global__ __launch_bounds__(kBlock) void k_phub_collect(PoolSlot *slots, int slot, SingleArgs *A, SingleState *S,
                                                         int32_t *hub_tables) {
    const PoolSlot *sp = slots + slot;
    SingleArgs a = {};
    a.rp = sp->rp;
    a.ci = sp->ci;
    a.col = sp->col;
    a.col8 = sp->col8;
    a.col4 = sp->col4;
    a.hubW = sp->hubW;
    a.hubB = sp->hubB;
    a.n = sp->n;
    a.t_thread = sp->t_thread;
    a.t_wave = sp->t_wave;
    a.hub_t = sp->hub_opt;
    a.hubC = hub_tables;
    a.hubS = hub_tables + kHubCap;
    a.hub_cpre = hub_tables + 2 * kHubCap;
    a.hub_bits = reinterpret_cast<uint32_t *>(hub_tables + kHubTablesInts);
    a.pend = sp->wl[1];  // the hubs' position map (free until the slot's first round appends there)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *A = a;
        S->nW = sp->nW;
        S->nB = sp->nB;
        S->maxdeg = sp->maxdeg;
        S->err = sp->status < 0 ? kErrNoRun : 0;
    }
    if (sp->status < 0 || a.hub_t == 0) return;
    // hub_collect with the slot's own sizes (S's are written by block 0 in
    // this same launch)
    const int maxdeg = sp->maxdeg;
    const int T = hub_threshold(a, maxdeg);
    if (blockIdx.x == 0 && threadIdx.x == 0) S->hub_t = T;
    if (maxdeg <= T) return;
    const int nW = sp->nW, nB = sp->nB;
    const int from = T >= a.t_wave ? nW : 0;
    const RSOC_GLOBAL int32_t *rp = gro(a.rp);
    for (int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nW + nB;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int v = i < nW ? a.hubW[i] : a.hubB[i - nW];
        const bool hub = rp[v + 1] - rp[v] > T;
        const uint64_t m = ballot(hub);
        int at = 0;
        const int lead = m ? __ffsll((unsigned long long)m) - 1 : 0;
        if (m && lane_id() == lead) at = atomicAdd(&S->nHc, __popcll(m));
        at = __shfl(at, lead) + lanes_below(m);
        if (hub && at < kHubCap) a.hubC[at] = v;
    }
}

static_assert(offsetof(PoolSlot, hub_t) == offsetof(PoolSlot, nH) + sizeof(int32_t),
              "k_hub_ff writes nH and hub_t as two adjacent words");

struct PoolTask {
    int32_t slot, kind, begin, end;
};

// Task tables are dealt on the device.  A step's table of one (kind, tie
// rule) and bin is described by one PoolDeal and its spans, one per slot in
// the step: the slot's item count in that bin and its number of tasks
// (ceil(items / per)).  Task r of a slot with T tasks goes to bucket
// floor(r * kDealBuckets / T); the table lists the buckets in order, within a
// bucket the slots in span order, within a slot its tasks in order.  The
// workgroups take the table in order, so every graph advances through its
// ids at the same relative pace and has about the same small fraction of
// them in flight at any time, as a single-graph sweep does; dealt slot by
// slot, a graph would have all its vertices coloured in the same instant
// (each reading its neighbours uncoloured: most would end round 0
// defective), and the last graphs of the table would get the whole grid to
// themselves.
struct PoolSpan {
    int32_t slot, items, ntask;
};
struct PoolDeal {
    int32_t span0, nspan, per, kind, at, ntask;  // at: the table's first entry in the task array
};
constexpr int kDealBuckets = 4096;
constexpr int kDealBlock = 1024;

// first task of bucket b among T: ceil(b * T / kDealBuckets)
__device__ __forceinline__ int deal_first(int64_t T, int b) {
    return (int)((T * b + kDealBuckets - 1) / kDealBuckets);
}

__device__ __forceinline__ int wave_incl_scan(int x) {
    const int ln = lane_id();
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (ln >= off) x += y;
    }
    return x;
}

// grid (tables, kDealSplit): every workgroup of a table computes the bucket
// sizes and their exclusive scan in LDS, then its wavefronts write the tasks
// of its share of the buckets, one bucket per wavefront at a time.  The spans
// are staged in LDS (up to kDealLdsSpans; beyond that they are read from
// global memory, in order).
constexpr int kDealSplit = 8;
constexpr int kDealLdsSpans = 2048;

__global__ __launch_bounds__(kDealBlock) void k_pdeal(const PoolDeal *__restrict__ deals,
                                                      const PoolSpan *__restrict__ spans,
                                                      PoolTask *__restrict__ tasks) {
    constexpr int kPer = kDealBuckets / kDealBlock;
    constexpr int kWaves = kDealBlock / kWave;
    __shared__ int first[kDealBuckets];
    __shared__ int wsum[kWaves];
    __shared__ PoolSpan lsp[kDealLdsSpans];
    const PoolDeal d = deals[blockIdx.x];
    const bool in_lds = d.nspan <= kDealLdsSpans;
    for (int k = threadIdx.x; in_lds && k < d.nspan; k += kDealBlock) lsp[k] = spans[d.span0 + k];
    __syncthreads();
    const PoolSpan *sp = in_lds ? lsp : spans + d.span0;
    const int b0 = threadIdx.x * kPer;
    int c[kPer] = {};
    for (int k = 0; k < d.nspan; ++k) {
        const int64_t T = sp[k].ntask;
        int lo = deal_first(T, b0);
        for (int j = 0; j < kPer; ++j) {
            const int hi = deal_first(T, b0 + j + 1);
            c[j] += hi - lo;
            lo = hi;
        }
    }
    int mine = 0;
    for (int j = 0; j < kPer; ++j) mine += c[j];
    const int wv = threadIdx.x / kWave, ln = lane_id();
    const int incl = wave_incl_scan(mine);
    if (ln == kWave - 1) wsum[wv] = incl;
    __syncthreads();
    if (wv == 0) {
        const int w = wave_incl_scan(ln < kWaves ? wsum[ln] : 0);
        if (ln < kWaves) wsum[ln] = w;
    }
    __syncthreads();
    int base = incl - mine + (wv > 0 ? wsum[wv - 1] : 0);
    for (int j = 0; j < kPer; ++j) {
        first[b0 + j] = base;
        base += c[j];
    }
    __syncthreads();
    PoolTask *out = tasks + d.at;
    constexpr int kShare = kDealBuckets / kDealSplit;
    const int bend = (blockIdx.y + 1) * kShare;
    for (int b = blockIdx.y * kShare + wv; b < bend; b += kWaves) {
        int run = first[b];
        for (int k0 = 0; k0 < d.nspan; k0 += kWave) {
            const int k = k0 + ln;
            int lo = 0, cnt = 0, slot = 0, items = 0;
            if (k < d.nspan) {
                const PoolSpan e = sp[k];
                slot = e.slot;
                items = e.items;
                lo = deal_first(e.ntask, b);
                cnt = deal_first(e.ntask, b + 1) - lo;
            }
            const int x = wave_incl_scan(cnt);
            PoolTask *o = out + run + x - cnt;
            for (int j = 0; j < cnt; ++j) {
                const int64_t beg = (int64_t)(lo + j) * d.per;
                o[j] = {slot, d.kind, (int)beg, (int)min<int64_t>(items, beg + d.per)};
            }
            run += __shfl(x, kWave - 1);
        }
    }
}

// Admission: fills the colours (round 0 of the round-synchronous mode), bins
// by degree, samples id locality, and checks the ends of row_ptr (status
// RSOC_ECSR when row_ptr[0] != 0 or row_ptr[n] < 0, RSOC_EINVAL when edges
// come without col_idx); nnz = row_ptr[n] is recorded for the host.
__global__ __launch_bounds__(kBlock) void k_pinit(PoolSlot *slots, int slot) {
    __shared__ int sh[kWavesPerBlock];
    __shared__ int qW[kQueueCap], qB[kQueueCap];
    __shared__ int nqW, nqB, qbase;
    if (threadIdx.x == 0) nqW = nqB = 0;
    __syncthreads();
    PoolSlot *sp = slots + slot;
    const RSOC_GLOBAL int32_t *rp = gro(sp->rp);
    const int n = sp->n;
    const int fillc = sp->mode == kOptimistic ? -1 : 0;
    const RSOC_GLOBAL int32_t *ci = gro(sp->ci);
    const int64_t nnz = rp[n];
    const bool rows_ok = rp[0] == 0 && nnz >= 0 && (nnz == 0 || sp->ci != nullptr);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sp->nnz = nnz;
        if (!rows_ok) sp->status = (rp[0] != 0 || nnz < 0) ? -2 /* RSOC_ECSR */ : -1 /* RSOC_EINVAL */;
    }
    int md = 0;
    uint64_t near = 0, sampled = 0;
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
        const int v = (int)(base + threadIdx.x);
        int d = -1;
        if (v < n) {
            d = rp[v + 1] - rp[v];
            if (sp->recolor) {
                // recolouring: colours stay; byte shadow from them; mark in
                // wl[1] (free until the first round appends there) every
                // vertex without a valid First-Fit colour
                const int c = sp->col[v];
                sp->col8[v] = shadow_of(c);
                sp->wl[1][v] = (c < 0 || c > d) ? 1 : 0;
            } else {
                sp->col[v] = fillc;
                sp->col8[v] = shadow_of(fillc);
                if (sp->col4 && (v & 7) == 0) sp->col4[v >> 3] = ~0u;  // every nibble 15: nothing published yet
                if ((v & 255) == 0 && rows_ok) locality_row(rp, ci, v, nnz, near, sampled);  // id-locality sample
            }
        }
        md = max(md, d);
        queue_push(d > sp->t_wave, v, qB, &nqB);
        queue_push(d > sp->t_thread && d <= sp->t_wave, v, qW, &nqW);
        int cB, cW;
        queue_sizes(&nqB, &nqW, cB, cW);
        if (cB > kQueueCap - kBlock) queue_flush_n(cB, qB, &nqB, &qbase, &sp->nB, sp->hubB);
        if (cW > kQueueCap - kBlock) queue_flush_n(cW, qW, &nqW, &qbase, &sp->nW, sp->hubW);
    }
    queue_flush(qB, &nqB, &qbase, &sp->nB, sp->hubB);
    queue_flush(qW, &nqW, &qbase, &sp->nW, sp->hubW);
    near = wave_sum_u64(near);
    sampled = wave_sum_u64(sampled);
    if (lane_id() == 0 && sampled) {
        atomicAdd((unsigned long long *)&sp->near, (unsigned long long)near);
        atomicAdd((unsigned long long *)&sp->sampled, (unsigned long long)sampled);
    }
    md = block_max(md, sh);
    if (threadIdx.x == 0) atomicMax(&sp->maxdeg, md);
}

// Recolouring slots, after k_pinit: the touched vertices are marked too (an
// id outside [0, n) gives status RSOC_EINVAL) ...
__global__ __launch_bounds__(kBlock) void k_ptouch(PoolSlot *slots, int slot) {
    PoolSlot *sp = slots + slot;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < sp->nt; i += (int64_t)gridDim.x * kBlock) {
        const int t = sp->touched[i];
        if (t < 0 || t >= sp->n) bad = true;
        else sp->wl[1][t] = 1;
    }
    if (ballot(bad) && lane_id() == 0) atomicMin(&sp->status, -1);  // RSOC_EINVAL
}

// ... and the marked vertices become the first worklist, by degree bin, in
// wl[0] (parity 0), counted straight into cnt_in.
__global__ __launch_bounds__(kBlock) void k_plist(PoolSlot *slots, int slot) {
    __shared__ int qT[kQueueCap], qW[kQueueCap], qB[kQueueCap];
    __shared__ int nqT, nqW, nqB, qbase;
    PoolSlot *sp = slots + slot;
    const RSOC_GLOBAL int32_t *rp = gro(sp->rp);
    const int n = sp->n;
    const int offW = n - sp->nW - sp->nB, offB = n - sp->nB;
    const int32_t *mark = sp->wl[1];
    int32_t *const out = sp->wl[0];
    if (threadIdx.x == 0) nqT = nqW = nqB = 0;
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
        const int v = (int)(base + threadIdx.x);
        const bool m = v < n && mark[v] != 0;
        const int d = m ? rp[v + 1] - rp[v] : 0;
        queue_push(m && d > sp->t_wave, v, qB, &nqB);
        queue_push(m && d > sp->t_thread && d <= sp->t_wave, v, qW, &nqW);
        queue_push(m && d <= sp->t_thread, v, qT, &nqT);
        int cB, cW, cT;
        queue_sizes(&nqB, &nqW, &nqT, cB, cW, cT);
        if (cB > kQueueCap - kBlock) queue_flush_n(cB, qB, &nqB, &qbase, &sp->cnt_in[kBinBlock], out + offB);
        if (cW > kQueueCap - kBlock) queue_flush_n(cW, qW, &nqW, &qbase, &sp->cnt_in[kBinWave], out + offW);
        if (cT > kQueueCap - kBlock) queue_flush_n(cT, qT, &nqT, &qbase, &sp->cnt_in[kBinThread], out);
    }
    queue_flush(qB, &nqB, &qbase, &sp->cnt_in[kBinBlock], out + offB);
    queue_flush(qW, &nqW, &qbase, &sp->cnt_in[kBinWave], out + offW);
    queue_flush(qT, &nqT, &qbase, &sp->cnt_in[kBinThread], out);
}

template <int TIE, int KIND>
__device__ __forceinline__ void pool_thread_task(PoolSlot *sp, const PoolSlot &s, const PoolTask &tk, int *q, int *qn,
                                                 int *qbase, int4 *qa, bool flush) {
    constexpr int PHASE = KIND == kAssignSweep ? kAssign : kRecolor;
    constexpr bool SWEEP = KIND != kRecolorList;
    constexpr bool kWinOnly = KIND == kAssignSweep;
    // round 0 (optimistic slots only) reads and publishes the 4-bit shadow;
    // later rounds read the byte shadow, so no nibble is ever read stale
    constexpr bool kNib = KIND == kAssignSweep;
    const RSOC_GLOBAL int32_t *rp = gro(s.rp);
    const RSOC_GLOBAL int32_t *ci = gro(s.ci);
    const RSOC_GLOBAL uint8_t *c8 = gro(s.col8);
    RSOC_GLOBAL uint32_t *c4 = grw(s.col4);
    const bool opt = s.mode == kOptimistic;
    RSOC_GLOBAL int32_t *wcol = grw(opt ? s.col : s.pend);
    RSOC_GLOBAL uint8_t *wcol8 = grw(s.col8);
    const int32_t *in = s.parity ? s.wl[1] : s.wl[0];
    int32_t *out = s.parity ? s.wl[0] : s.wl[1];
    const int gi = threadIdx.x / kGroup;
    const bool leader = (threadIdx.x & (kGroup - 1)) == 0;
    for (int base = tk.begin; base < tk.end; base += kStep) {
        for (int r = 0; r < kChunk; ++r) {
            int v[kNV], b[kNV], e[kNV], cv[kNV], nc[kNV];
            bool act[kNV];
            uint32_t unc[kNV] = {};
            int keep[kNV][4];
#pragma unroll
            for (int i = 0; i < kNV; ++i) {
                const int idx = base + step_offset(r, i, gi, s.chunk);
                v[i] = -1;
                b[i] = e[i] = 0;
                if (idx < tk.end) {
                    if (SWEEP) v[i] = (KIND == kAssignSweep && TIE == kHigherKeeps) ? s.n - 1 - idx : idx;
                    else v[i] = in[idx];
                    b[i] = rp[v[i]];
                    e[i] = rp[v[i] + 1];
                    if (SWEEP && e[i] - b[i] > s.t_thread) e[i] = b[i] = 0, v[i] = -1;
                }
                cv[i] = (PHASE != kAssign && v[i] >= 0) ? (int)c8[v[i]] : 255;
            }
            const RSOC_GLOBAL int32_t *cis[kNV];
            const RSOC_GLOBAL uint8_t *c8s[kNV];
            const RSOC_GLOBAL uint32_t *c4s[kNV];
#pragma unroll
            for (int i = 0; i < kNV; ++i) cis[i] = ci, c8s[i] = c8, c4s[i] = c4;
            // after a hub-first pass round 0 reads all neighbours (hub colours)
            const int look = (KIND == kAssignSweep && s.nH) ? INT_MAX : s.look;
            group_vertices<PHASE, TIE, kGroup, kGroupSlots, kWinOnly, kNV, kNib>(v, b, e, cis, c8s, cv, look, nc,
                                                                                 act, unc, c4s, kNib ? keep : nullptr,
                                                                                 KIND == kAssignSweep && s.nH > 0);
#pragma unroll
            for (int i = 0; i < kNV; ++i) {
                if (v[i] < 0) {
                    act[i] = false;
                    unc[i] = 0;
                }
                if (leader && act[i]) {
                    wcol[v[i]] = nc[i];
                    if (opt) wcol8[v[i]] = (uint8_t)nc[i];
                }
            }
            if (kNib) {
                int ids[kNV];
#pragma unroll
                for (int i = 0; i < kNV; ++i) {
                    const int idx = base + step_offset(r, i, gi, s.chunk);
                    ids[i] = idx < tk.end ? (TIE == kHigherKeeps ? s.n - 1 - idx : idx) : -1;
                }
                publish_nibbles<kNV>(ids, v, nc, c4, leader);
            }
#pragma unroll
            for (int i = 0; i < kNV; ++i)
                queue_push<int4>((KIND == kAssignSweep ? unc[i] != 0 : act[i]) && leader, v[i], q, qn,
                                 kNib ? qa : nullptr,
                                 kNib ? make_int4(keep[i][0], keep[i][1], keep[i][2], keep[i][3]) : int4{});
            const int cq = queue_size(qn);
            if (cq > (kNib ? kPoolAuxCap : kQueueCap) - kSub)
                queue_flush_n<int4>(cq, q, qn, qbase, &sp->cnt_out[kBinThread], out, kNib ? qa : nullptr, s.aux);
        }
    }
    if (flush) queue_flush<int4>(q, qn, qbase, &sp->cnt_out[kBinThread], out, kNib ? qa : nullptr, s.aux);
}

// The first worklist round after round 0, thread-bin entries: one lane per
// entry tests only the neighbours round 0 kept for it (lane_detect_kept);
// defective entries, and entries that kept more than three, go to the lane
// groups (wave_recolour_selected); appends gather in the wavefront's buffer.
template <int TIE>
__device__ __forceinline__ void pool_masked_task(PoolSlot *sp, const PoolSlot &s, const PoolTask &tk, int *ms,
                                                 int *mb, int *mbn, bool flush) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const int32_t *in = s.parity ? s.wl[1] : s.wl[0];
    int32_t *out = s.parity ? s.wl[0] : s.wl[1];
    const RSOC_GLOBAL int32_t *rp = gro(s.rp);
    const RSOC_GLOBAL int32_t *ci = gro(s.ci);
    const RSOC_GLOBAL uint8_t *c8 = gro(s.col8);
    const RSOC_GLOBAL v4i *ax = (const RSOC_GLOBAL v4i *)s.aux;
    RSOC_GLOBAL int32_t *wcol = grw(s.col);
    RSOC_GLOBAL uint8_t *wcol8 = grw(s.col8);
    const int wv = threadIdx.x / kWave;
    uint64_t degs = 0, apps = 0;
    for (int base = tk.begin + wv * kWave; base < tk.end; base += kWavesPerBlock * kWave) {
        const int idx = base + lane_id();
        int v = -1, cv = 255;
        int4 x = {0, 0, 0, 0};
        if (idx < tk.end) {
            v = in[idx];
            const v4i y = ax[idx];
            x = make_int4(y.x, y.y, y.z, y.w);
            cv = c8[v];
        }
        const bool over = v >= 0 && __popc((uint32_t)x.w) > 3;
        const bool def = v >= 0 && !over && lane_detect_kept<false>(v, x, cv, c8, nullptr);
        wave_recolour_selected<kAssign, TIE, false>(ballot(def), v, ms, mb, mbn, rp, ci, c8, nullptr, wcol, wcol8,
                                                    nullptr, s.look, degs, apps);
        const uint64_t om = ballot(over);
        if (om)
            wave_recolour_selected<kRecolor, TIE, false>(om, v, ms, mb, mbn, rp, ci, c8, nullptr, wcol, wcol8,
                                                         nullptr, s.look, degs, apps);
        if (*mbn >= kPoolMaskedBuf - kWave) wave_buf_flush(mb, mbn, &sp->cnt_out[kBinThread], out);
    }
    if (flush) wave_buf_flush(mb, mbn, &sp->cnt_out[kBinThread], out);
}

template <int TIE, int KIND>
__device__ __forceinline__ void pool_wave_task(PoolSlot *sp, const PoolSlot &s, const PoolTask &tk, uint32_t *lds,
                                               int *wbuf, int *wbn, bool flush) {
    constexpr int PHASE = KIND == kAssignSweep ? kAssign : kRecolor;
    constexpr bool kWinOnly = KIND == kAssignSweep;
    const int wv = threadIdx.x / kWave;
    uint32_t *bm = lds + wv * kWaveWindowWords;
    const bool opt = s.mode == kOptimistic;
    const int32_t *in = (KIND == kRecolorList) ? (s.parity ? s.wl[1] : s.wl[0]) + s.offW : s.hubW;
    int32_t *out = (s.parity ? s.wl[0] : s.wl[1]) + s.offW;
    const bool hubs = KIND == kAssignSweep && s.nH > 0;  // hub-first: hubs done, all neighbours read
    for (int i = tk.begin + wv; i < tk.end; i += kWavesPerBlock) {
        const int v = in[i];
        const int b = s.rp[v], e = s.rp[v + 1];
        if (hubs && e - b > s.hub_t) continue;  // a hub (wavefront-uniform)
        int nc = 0;
        bool unc = false;
        const bool act = wave_vertex<PHASE, TIE, kWinOnly>(v, b, e, gro(s.ci), gro(s.col), gro(s.col8), bm,
                                                           hubs ? INT_MAX : s.look, nc, unc, hubs, gro(s.col4));
        if (lane_id() == 0 && act) {
            (opt ? s.col : s.pend)[v] = nc;
            if (opt) s.col8[v] = shadow_of(nc);
            if (KIND == kAssignSweep) publish_nibble(grw(s.col4), v, nc);
        }
        wave_buf_push(KIND == kAssignSweep ? unc : act, v, wbuf, wbn, &sp->cnt_out[kBinWave], out);
    }
    if (flush) wave_buf_flush(wbuf, wbn, &sp->cnt_out[kBinWave], out);
}

template <int TIE, int KIND>
__device__ __forceinline__ void pool_block_task(PoolSlot *sp, const PoolSlot &s, const PoolTask &tk, uint32_t *lds,
                                                int *sh_min) {
    constexpr int PHASE = KIND == kAssignSweep ? kAssign : kRecolor;
    constexpr bool kWinOnly = KIND == kAssignSweep;
    const bool opt = s.mode == kOptimistic;
    const int32_t *in = (KIND == kRecolorList) ? (s.parity ? s.wl[1] : s.wl[0]) + s.offB : s.hubB;
    int32_t *out = (s.parity ? s.wl[0] : s.wl[1]) + s.offB;
    const bool hubs = KIND == kAssignSweep && s.nH > 0;  // hub-first: hubs done, all neighbours read
    for (int i = tk.begin; i < tk.end; ++i) {
        const int v = in[i];
        const int b = s.rp[v], e = s.rp[v + 1];
        if (hubs && e - b > s.hub_t) continue;  // a hub (workgroup-uniform)
        int nc = 0;
        bool unc = false;
        const bool act = block_vertex<PHASE, TIE, kWinOnly>(v, b, e, gro(s.ci), gro(s.col), gro(s.col8), lds, sh_min,
                                                            hubs ? INT_MAX : s.look, nc, unc, hubs, gro(s.col4));
        if (threadIdx.x == 0) {
            if (act) {
                (opt ? s.col : s.pend)[v] = nc;
                if (opt) s.col8[v] = shadow_of(nc);
                if (KIND == kAssignSweep) publish_nibble(grw(s.col4), v, nc);
            }
            if (KIND == kAssignSweep ? unc : act) out[atomicAdd(&sp->cnt_out[kBinBlock], 1)] = v;
        }
    }
}

// One fused pool round for the tasks of one kind and tie rule (one launch per
// pair present in the step, so that each gets the registers of its own code
// and not those of the largest).  Blocks [0,gT) take thread-bin tasks,
// [gT,gT+gW) wavefront-bin tasks, the rest workgroup-bin tasks (grid-stride
// over each).  kRecolorMasked has thread-bin tasks only.
template <int KIND, int TIE>
__global__ __launch_bounds__(kBlock) void k_pstep(PoolSlot *slots, const PoolTask *__restrict__ tasks, int ntB,
                                                  int ntW, int ntT, int gB, int gW, int gT) {
    constexpr bool kMasked = KIND == kRecolorMasked;
    constexpr bool kAux = KIND == kAssignSweep;
    __shared__ uint32_t lds[kMasked ? 1 : kLdsWords];
    __shared__ int q[kMasked ? 1 : kQueueCap];
    __shared__ int sh_min, qn, qbase;
    __shared__ int wbuf[kWavesPerBlock][kMasked ? 1 : kWaveBuf];
    __shared__ int wbn[kWavesPerBlock];
    __shared__ int4 qa[kAux ? kPoolAuxCap : 1];
    __shared__ int mstage[kWavesPerBlock][kMasked ? kWave : 1];
    __shared__ int mbuf[kWavesPerBlock][kMasked ? kPoolMaskedBuf : 1];
    const int bid = blockIdx.x;
    if (threadIdx.x == 0) qn = 0;
    if (threadIdx.x < kWavesPerBlock) wbn[threadIdx.x] = 0;
    __syncthreads();
    // thread-bin workgroups come first in the grid, so they are dispatched
    // first: the order in which round 0 walks the ids must not wait behind
    // the hubs
    const int sec = bid < gT ? 0 : (bid < gT + gW ? 1 : 2);
    int first, count, stride, self;
    if (sec == 0) { first = ntB + ntW; count = ntT; stride = gT; self = bid; }
    else if (sec == 1) { first = ntB; count = ntW; stride = gW; self = bid - gT; }
    else { first = 0; count = ntB; stride = gB; self = bid - gT - gW; }
    const int wv = threadIdx.x / kWave;
    for (int t = self; t < count; t += stride) {
        const PoolTask tk = tasks[first + t];
        PoolSlot *sp = slots + tk.slot;
        const PoolSlot s = *sp;
        // what a task appends stays in the LDS buffers while the workgroup's
        // next task belongs to the same slot (same lists, same counter): one
        // global atomic per buffer-full, not per task -- with one or two
        // large slots every flush hits the same counter, and 1024 workgroups'
        // per-task atomics on it serialised the round
        const bool flush = t + stride >= count || tasks[first + t + stride].slot != tk.slot;
        if (kMasked) pool_masked_task<TIE>(sp, s, tk, mstage[wv], mbuf[wv], &wbn[wv], flush);
        else if (sec == 2) pool_block_task<TIE, KIND>(sp, s, tk, lds, &sh_min);
        else if (sec == 1) pool_wave_task<TIE, KIND>(sp, s, tk, lds, wbuf[wv], &wbn[wv], flush);
        else pool_thread_task<TIE, KIND>(sp, s, tk, q, &qn, &qbase, qa, flush);
    }
}

// Round-synchronous slots publish their staged colours (col = pend for L).
__global__ __launch_bounds__(kBlock) void k_pscatter(PoolSlot *slots, const int32_t *__restrict__ active, int nact) {
    for (int k = blockIdx.y; k < nact; k += gridDim.y) {
        PoolSlot *sp = slots + active[k];
        if (sp->mode == kOptimistic) continue;
        const int32_t *lst = sp->wl[sp->parity ^ 1];
        for (int bin = 0; bin < 3; ++bin) {
            const int c = sp->cnt_out[bin];
            const int off = bin == 0 ? 0 : (bin == 1 ? sp->offW : sp->offB);
            for (int i = blockIdx.x * kBlock + threadIdx.x; i < c; i += gridDim.x * kBlock) {
                const int v = lst[off + i];
                const int cc = sp->pend[v];
                sp->col[v] = cc;
                sp->col8[v] = shadow_of(cc);
            }
        }
    }
}

// Per-slot round end: counts the pass, publishes the appended list, flips the
// worklist parity, and marks the slot done when its worklist is empty (or
// the pass bound is reached).
__global__ void k_pround_end(PoolSlot *slots, const int32_t *__restrict__ active, int nact) {
    for (int k = threadIdx.x; k < nact; k += blockDim.x) {
        PoolSlot *sp = slots + active[k];
        const int out_total = sp->cnt_out[0] + sp->cnt_out[1] + sp->cnt_out[2];
        const bool round0 = sp->phase == kSlotNew && sp->mode == kOptimistic;
        sp->masked = round0 ? 1 : 0;
        if (round0) {
            sp->u0 = out_total;
        } else {
            sp->passes += 1;
            if (out_total > 0) {
                sp->rounds += 1;
                sp->conflicts += out_total;
            }
        }
        for (int b = 0; b < 3; ++b) {
            sp->cnt_in[b] = sp->cnt_out[b];
            sp->cnt_out[b] = 0;
        }
        sp->parity ^= 1;
        sp->phase = kSlotRunning;
        if (out_total == 0) {
            sp->phase = kSlotDone;
        } else if (!round0 && sp->passes >= sp->max_rounds) {
            sp->phase = kSlotDone;
            sp->status = -7;  // RSOC_ENOCONV
        }
    }
}

// Last act of a slot's set-up: the fields the rounds need that follow from
// what the set-up found (bin offsets, the chunk from the locality sample,
// |U^0| of a recolouring), or the end of a slot whose input was rejected.
// The download that follows gives the host its final state.
__global__ void k_pready(PoolSlot *slots, int slot) {
    PoolSlot *sp = slots + slot;
    if (sp->status < 0) {
        sp->phase = kSlotDone;  // bad row_ptr ends, missing col_idx, touched id out of range
        return;
    }
    sp->offW = sp->n - sp->nW - sp->nB;
    sp->offB = sp->n - sp->nB;
    sp->chunk = pick_chunk(sp->chunk, sp->near, sp->sampled);
    // an empty U^0 still takes one (empty) step, which ends the slot and
    // counts its colours
    if (sp->recolor) sp->u0 = sp->cnt_in[0] + sp->cnt_in[1] + sp->cnt_in[2];
}

// Colour statistics of the slots that finished in this step, enqueued right
// after the step's round (grid.y walks the step's active slots; the others
// leave at once): K (kmax), the colours below 255 in use (cbits), and a flag
// per colour of 255 and more in the slot's first worklist buffer (free once
// the slot is done; k_pflags_clear zeroed the flags up to its max degree,
// which bounds every colour), which k_pdistinct counts.
__device__ __forceinline__ bool wide_colours(const PoolSlot *sp) { return sp->maxdeg >= 255 && sp->n > 255; }

__global__ __launch_bounds__(kBlock) void k_pcount(PoolSlot *slots, const int32_t *__restrict__ active, int nact) {
    __shared__ int sh[kWavesPerBlock];
    __shared__ uint32_t bits[8];
    for (int k = blockIdx.y; k < nact; k += gridDim.y) {
        PoolSlot *sp = slots + active[k];
        if (sp->phase != kSlotDone) continue;  // uniform over the workgroup
        const int n = sp->n;
        if ((int64_t)blockIdx.x * kBlock >= n) continue;
        __syncthreads();
        if (threadIdx.x < 8) bits[threadIdx.x] = 0;
        __syncthreads();
        int32_t *flags = sp->wl[0];
        const int32_t *col = sp->col;
        int m = -1;
        bool bad = false;
        for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
            const int c = col[v];
            bad |= (c < 0 || c >= n);
            m = max(m, c);
            if (c >= 0 && c < 255) lds_or(&bits[c >> 5], 1u << (c & 31));
            else if (c >= 255 && c < n) flags[c] = 1;
        }
        if (ballot(bad) && lane_id() == 0) atomicOr(&sp->err, 4);
        m = block_max(m, sh);
        if (threadIdx.x == 0) atomicMax(&sp->kmax, m + 1);
        if (threadIdx.x < 8 && bits[threadIdx.x]) atomicOr(&sp->cbits[threadIdx.x], bits[threadIdx.x]);
    }
}

// Zeroes the flags k_pcount sets: colours 255 .. min(max degree, n - 1).
__global__ __launch_bounds__(kBlock) void k_pflags_clear(PoolSlot *slots, const int32_t *__restrict__ active,
                                                         int nact) {
    for (int k = blockIdx.y; k < nact; k += gridDim.y) {
        PoolSlot *sp = slots + active[k];
        if (sp->phase != kSlotDone || !wide_colours(sp)) continue;
        const int hi = min(sp->maxdeg, sp->n - 1);
        for (int c = 255 + blockIdx.x * kBlock + threadIdx.x; c <= hi; c += gridDim.x * kBlock) sp->wl[0][c] = 0;
    }
}

// Counts the flags of colours 255 .. kmax - 1 into sp->distinct (one
// workgroup per slot).
__global__ __launch_bounds__(kBlock) void k_pdistinct(PoolSlot *slots, const int32_t *__restrict__ active, int nact) {
    __shared__ int sh[kWavesPerBlock];
    for (int k = blockIdx.y; k < nact; k += gridDim.y) {
        PoolSlot *sp = slots + active[k];
        if (sp->phase != kSlotDone || !wide_colours(sp)) continue;
        const int hi = min(sp->kmax, sp->n);
        int cnt = 0;
        for (int c = 255 + (int)threadIdx.x; c < hi; c += kBlock) cnt += sp->wl[0][c];
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        __syncthreads();
        if (lane_id() == 0) sh[threadIdx.x / kWave] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < kWavesPerBlock; ++w) t += sh[w];
            sp->distinct = t;
        }
    }
}

}  // namespace rsoc
