// single_kernels.hpp -- kernels of the single-graph colouring path.
//
// One round of Algorithm 3 (Section 3) is one launch of k_round: its
// workgroups are split into three sections, one per degree bin (workgroup-,
// wavefront- and thread-per-vertex), so a round is a single launch whatever
// the degree mix.  The kernel boundary after it is the round's barrier.
// Vertices recoloured in the round are appended, per bin, to the next round's
// worklist (wavefront-aggregated atomics).  k_round_end then publishes the
// list sizes and keeps the round statistics, so the host only needs to look
// at the worklist size every few rounds.
#pragma once

#include "vertex_ops.hpp"

namespace rsoc {

// Device-resident arguments of one single-graph colouring.  Captured HIP graphs
// take a pointer to this block, so one captured round loop serves any input.
struct SingleArgs {
    const int32_t *rp;   // row_ptr[n+1]
    const int32_t *ci;   // col_idx[nnz]
    int32_t *col;        // colours[n]
    int32_t *pend;       // staged colours (round-synchronous modes), indexed by vertex
    int32_t *wl[2];      // worklist buffers; bin segments start at 0, offW, offB
    int32_t *hubW;       // static list of wavefront-bin vertices
    int32_t *hubB;       // static list of workgroup-bin vertices
    int32_t n;
    int32_t t_thread;
    int32_t t_wave;
    int32_t max_rounds;  // bound on inspection passes
    int32_t offW, offB;  // segment offsets inside wl buffers
};

// Device-side round state.
struct SingleState {
    int32_t cnt_in[4];    // size of each bin of the current worklist
    int32_t cnt_out[4];   // appends so far into the next worklist
    int32_t nW, nB;       // static bin sizes (binning)
    int32_t maxdeg;
    int32_t passes;       // inspection passes executed (rounds >= 1)
    int32_t rounds;       // passes that recoloured somebody
    int32_t kmax;         // max colour + 1
    int32_t distinct;
    int32_t err;          // bit 0 bad CSR, bit 1 self-loop, bit 2 colour out of range
    int64_t conflicts;    // sum of |L|
    uint64_t inspected;   // vertices inspected by worklist rounds
    uint64_t deg_sum;     // their degree sum
    int32_t pad[2];
    int32_t hist[kHistCap];  // |L| of recolouring round i+1
};

// ------------------------------------------------------------------ fill --
__global__ void k_fill(int32_t *p, int64_t n, int32_t value) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ------------------------------------------------------------- validate --
// Flags malformed rows (decreasing offsets, offsets past nnz, column ids out
// of range) and self-loops.
__global__ void k_validate(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, int32_t n, int64_t nnz,
                           int32_t *err) {
    int flags = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int b = rp[v], e = rp[v + 1];
        if (b > e || b < 0 || (int64_t)e > nnz) { flags |= 1; continue; }
        for (int j = b; j < e; ++j) {
            const int u = ci[j];
            if ((unsigned)u >= (unsigned)n) flags |= 1;
            else if (u == (int)v) flags |= 2;
        }
    }
    if (flags) atomicOr(err, flags);
}

// ------------------------------------------------------------------ bin --
// Splits V by degree: deg <= t_thread stays implicit (thread bin); larger rows
// go to the static wavefront / workgroup lists.  Also finds the max degree.
__global__ __launch_bounds__(kBlock) void k_bin(const SingleArgs *__restrict__ A, SingleState *S) {
    const SingleArgs a = *A;
    int md = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < a.n; base += stride) {
        const int v = (int)(base + threadIdx.x);
        int d = -1;
        if (v < a.n) d = a.rp[v + 1] - a.rp[v];
        md = max(md, d);
        wave_append(d > a.t_wave, v, &S->nB, a.hubB);
        wave_append(d > a.t_thread && d <= a.t_wave, v, &S->nW, a.hubW);
    }
    md = wave_max_i32(md);
    if (lane_id() == 0) atomicMax(&S->maxdeg, md);
}

// ---------------------------------------------------------------- round --
// PHASE: kAssign (First-Fit), kRecolor (detect + First-Fit), kDetect.
// MODE: kOptimistic writes colours in place (live reads); otherwise new
//       colours are staged in pend[] and published by k_scatter.
// SWEEP: the round covers all of V (rounds 0 and 1): the thread bin walks
//        vertex ids directly, the other bins read the static lists; otherwise
//        the round reads worklist buffer `parity` and appends to parity^1.
// Sections: blocks [0,gB) workgroup bin, [gB,gB+gW) wavefront bin, rest thread bin.
template <int PHASE, int MODE, int TIE, bool SWEEP>
__global__ __launch_bounds__(kBlock) void k_round(const SingleArgs *__restrict__ A, SingleState *S, int parity,
                                                  int gB, int gW, int gT) {
    __shared__ uint32_t lds[kLdsWords];
    __shared__ int sh_min;
    __shared__ unsigned long long sh_acc[2];
    const SingleArgs a = *A;
    if (!SWEEP && S->passes >= a.max_rounds) return;  // guard: the round may not run
    const int cT = SWEEP ? a.n : S->cnt_in[kBinThread];
    const int cW = SWEEP ? S->nW : S->cnt_in[kBinWave];
    const int cB = SWEEP ? S->nB : S->cnt_in[kBinBlock];
    const int32_t *inT = a.wl[parity];
    const int32_t *inW = SWEEP ? a.hubW : a.wl[parity] + a.offW;
    const int32_t *inB = SWEEP ? a.hubB : a.wl[parity] + a.offB;
    int32_t *out = a.wl[parity ^ 1];
    int32_t *wcol = (MODE == kOptimistic) ? a.col : a.pend;
    const int32_t *rcol = a.col;
    constexpr bool kAppend = PHASE != kAssign;
    constexpr bool kWrite = PHASE != kDetect;
    constexpr bool kAcct = PHASE != kAssign && !SWEEP;  // worklist rounds count their inspections
    uint64_t items = 0, degs = 0;
    const int bid = blockIdx.x;
    if (bid < gB) {
        for (int i = bid; i < cB; i += gB) {
            const int v = inB[i];
            const int b = a.rp[v], e = a.rp[v + 1];
            int nc = 0;
            const bool act = block_vertex<PHASE, TIE>(v, b, e, a.ci, rcol, lds, &sh_min, nc);
            if (threadIdx.x == 0) {
                items += 1;
                degs += (uint64_t)(e - b);
                if (act && kWrite) wcol[v] = nc;
                if (act && kAppend) out[a.offB + atomicAdd(&S->cnt_out[kBinBlock], 1)] = v;
            }
        }
    } else if (bid < gB + gW) {
        const int wv = threadIdx.x / kWave;
        const int w = (bid - gB) * kWavesPerBlock + wv;
        const int nw = gW * kWavesPerBlock;
        uint32_t *bm = lds + wv * kWaveWindowWords;
        for (int i = w; i < cW; i += nw) {
            const int v = inW[i];
            const int b = a.rp[v], e = a.rp[v + 1];
            int nc = 0;
            const bool act = wave_vertex<PHASE, TIE>(v, b, e, a.ci, rcol, bm, nc);
            if (lane_id() == 0) {
                items += 1;
                degs += (uint64_t)(e - b);
                if (act && kWrite) wcol[v] = nc;
                if (act && kAppend) out[a.offW + atomicAdd(&S->cnt_out[kBinWave], 1)] = v;
            }
        }
    } else {
        int tb = bid - gB - gW;
        if (SWEEP) tb = xcd_contiguous(tb, gT);
        const int64_t stride = (int64_t)gT * kBlock;
        for (int64_t base = (int64_t)tb * kBlock; base < cT; base += stride) {
            const int i = (int)(base + threadIdx.x);
            bool act = false;
            int v = 0, nc = 0;
            if (i < cT) {
                v = SWEEP ? i : inT[i];
                const int b = a.rp[v], e = a.rp[v + 1];
                if (!SWEEP || e - b <= a.t_thread) {
                    act = thread_vertex<PHASE, TIE>(v, b, e, a.ci, rcol, nc);
                    items += 1;
                    degs += (uint64_t)(e - b);
                }
            }
            if (act && kWrite) wcol[v] = nc;
            if (kAppend) wave_append(act, v, &S->cnt_out[kBinThread], out);
        }
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

// -------------------------------------------------------------- scatter --
// Publishes staged colours: col[v] = pend[v] for every v of the chosen list
// (USE_IN: the current worklist buffer `parity` with cnt_in; otherwise the
// list just appended into buffer parity^1 with cnt_out; SWEEP: all of V).
template <bool SWEEP, bool USE_IN>
__global__ __launch_bounds__(kBlock) void k_scatter(const SingleArgs *__restrict__ A, SingleState *S, int parity) {
    const SingleArgs a = *A;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (SWEEP) {
        for (int64_t v = t0; v < a.n; v += stride) a.col[v] = a.pend[v];
        return;
    }
    if (S->passes >= a.max_rounds) return;
    const int32_t *lst = a.wl[USE_IN ? parity : (parity ^ 1)];
    const int32_t *cnt = USE_IN ? S->cnt_in : S->cnt_out;
    const int off[3] = {0, a.offW, a.offB};
    for (int bin = 0; bin < 3; ++bin) {
        const int c = cnt[bin];
        for (int64_t i = t0; i < c; i += stride) {
            const int v = lst[off[bin] + i];
            a.col[v] = a.pend[v];
        }
    }
}

// ------------------------------------------------------------ round end --
// Runs after a round (single thread): counts the pass, records |L|, makes the
// appended list the next worklist and clears the append counters.
template <int MODE, bool SWEEP>
__global__ void k_round_end(const SingleArgs *__restrict__ A, SingleState *S) {
    if (threadIdx.x != 0) return;
    if (!SWEEP && S->passes >= A->max_rounds) return;  // the guarded round did nothing
    const int in_total = SWEEP ? A->n : (S->cnt_in[0] + S->cnt_in[1] + S->cnt_in[2]);
    const int out_total = S->cnt_out[0] + S->cnt_out[1] + S->cnt_out[2];
    if (in_total > 0) {
        S->passes += 1;
        if (MODE == kTwoPhase) {
            if (S->rounds < kHistCap) S->hist[S->rounds] = out_total;
            S->rounds += 1;
            S->conflicts += out_total;
        } else if (out_total > 0) {
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

// --------------------------------------------------------- colour stats --
// K = max colour + 1; marks used colours (flags[0..maxdeg]) for the distinct
// count; flags an error if any colour is outside [0, maxdeg].
__global__ __launch_bounds__(kBlock) void k_colour_stats(const int32_t *__restrict__ col, int64_t n, int32_t maxdeg,
                                                         int32_t *flags, int32_t *kmax, int32_t *err) {
    int m = -1;
    bool bad = false;
    for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        const int c = col[v];
        if (c < 0 || c > maxdeg) { bad = true; continue; }
        m = max(m, c);
        flags[c] = 1;
    }
    m = wave_max_i32(m);
    if (lane_id() == 0) atomicMax(kmax, m + 1);
    if (ballot(bad) && lane_id() == 0) atomicOr(err, 4);
}

__global__ __launch_bounds__(kBlock) void k_count_flags(const int32_t *__restrict__ flags, int64_t len, int32_t *out) {
    int s = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < len; i += (int64_t)gridDim.x * kBlock) s += flags[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane_id() == 0 && s) atomicAdd(out, s);
}

}  // namespace rsoc
