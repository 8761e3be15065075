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
    uint8_t *col8;       // byte shadow of the colours: min(colour, 255), 255 when uncoloured
    uint32_t *col4;      // 4-bit shadow (8 per word): 0..13, 14 = 14 or more, 15 = consult col8 (optimistic mode)
    int32_t *pend;       // staged colours (round-synchronous modes), indexed by vertex
    int4 *aux;           // optimistic mode: what round 0 kept for U^0's thread-bin entries (parallel
                         // to that part of the list): up to three neighbour ids, position mask
    int32_t *wl[2];      // worklist buffers; bin segments start at 0, offW, offB
    int32_t *hubW;       // static list of wavefront-bin vertices
    int32_t *hubB;       // static list of workgroup-bin vertices
    int32_t n;
    int32_t t_thread;
    int32_t t_wave;
    int32_t max_rounds;  // bound on inspection passes
    int32_t offW, offB;  // segment offsets inside wl buffers
    int32_t look;        // round-0 lookahead (ids within `look` of v are read even when v wins against them)
    int32_t chunk;       // run of consecutive ids one lane group walks (1, 2, 4 or 8)
    int32_t look_auto;   // look is the default: k_args sets it to 0 once chunk turns out 1
    int32_t *flags;      // flags[c] for colours c >= 255 in use (zero between calls)
    // hub-first round 0 (optimistic, default flow; hub_kernels.hpp): hub_t is
    // the degree above which a vertex is a hub (0: off; -1: chosen from the
    // max degree, see hub_threshold); hubC the hubs as binning's lists give
    // them, hubS the same sorted by id; hub_bits per hub (by its position in
    // tie order) the bit set of the positions of the hubs it loses to
    int32_t hub_t;
    int32_t *hubC, *hubS, *hub_cpre;
    uint32_t *hub_bits;
};

// Hub-first round 0: at most kHubCap hubs (else the pass is skipped); the
// automatic threshold is max(t_thread, kHubMinDeg, max degree / kHubDiv).
constexpr int kHubCap = 4096;
constexpr int kHubMinDeg = 32;
constexpr int kHubDiv = 32;

__device__ __forceinline__ int hub_threshold(const SingleArgs &a, int maxdeg) {
    return a.hub_t > 0 ? a.hub_t : max(max(a.t_thread, kHubMinDeg), maxdeg / kHubDiv);
}

constexpr int kAccSlots = 16;   // cache lines the inspection counts are spread over
constexpr int kAccStride = 16;  // 64-bit words per line (128 bytes)
// Words of each acc line: what the worklist rounds inspected, and the
// independent counts that check the list sizes (bit 5 of err): entries a
// round decided to append (counted where the decision is taken, not by the
// queues), and the rows binning found in the wavefront / workgroup ranges.
enum AccWord : int { kAccItems = 0, kAccDegs = 1, kAccAppended = 2, kAccBinW = 3, kAccBinB = 4 };
constexpr int kErrListCount = 32;
constexpr int kErrNoRun = 1 | 8;  // err bits that keep the sweeps from running (bad row_ptr ends, no col_idx)

// Device-side round state.
struct SingleState {
    int32_t cnt_in[4];    // size of each bin of the current worklist
    int32_t cnt_out[4];   // appends so far into the next worklist
    int32_t nW, nB;       // static bin sizes (binning)
    int32_t maxdeg;
    int32_t passes;       // inspection passes executed (rounds >= 1)
    int32_t rounds;       // passes that recoloured somebody
    int32_t err;          // bit 0 bad CSR, bit 1 self-loop, bit 2 colour out of range, bit 3 edges without
                          // col_idx, bit 4 a touched id out of range (recolouring), bit 5 a list size
                          // that differs from the independent count of its entries
    int32_t nnz;          // row_ptr[n] (read by k_bin)
    int32_t lastL, prevL; // |L| of the last two rounds that inspected anything
    // colour statistics (k_colour_stats; cleared before each computation)
    int32_t kmax;         // max colour + 1
    int32_t distinct;     // distinct colours >= 255
    uint32_t cbits[8];    // set of colours < 255 used
    int64_t conflicts;    // sum of |L|
    uint64_t inspected;   // vertices inspected by worklist rounds
    uint64_t deg_sum;     // their degree sum
    int32_t u0;           // |U^0| when round 0 collects it (optimistic, default flow)
    int32_t chunk;        // run length of the sweeps (k_args)
    uint64_t inspected1, deg_sum1;  // inspected / deg_sum as they stood after the first worklist round
    uint64_t near, sampled;  // id locality sample: row entries with |u - v| < kChunk, entries sampled
    int32_t nH;           // hubs coloured before round 0 (0: none, or the hub-first pass is off)
    int32_t nHc;          // vertices above the hub threshold (k_args; the pass is off above kHubCap)
    int32_t hub_t;        // the hub threshold in use (k_args)
    int32_t next_task[kMaxBands];  // tasks handed out so far per band (batched optimistic rounds 0 and 1)
    int32_t u0_listed;    // batched: the part of |U^0| kept as list entries (wavefront and workgroup bins)
    int32_t hist[kHistCap];  // |L| of recolouring round i+1
    // worklist rounds' inspection counts (inspected, degree sum), spread over
    // kAccSlots cache lines so that a round's workgroups do not all add to one
    // line; k_round_end folds them into inspected / deg_sum
    alignas(128) unsigned long long acc[kAccSlots * kAccStride];
};

// the part of SingleState the host reads after a round (everything but hist)
constexpr size_t kStateHeader = offsetof(SingleState, hist);
static_assert(kStateHeader % 4 == 0, "header copied as 32-bit words");

// Closes a round graph (one workgroup): counts the flags k_colour_stats set
// for colours 255 .. min(max degree, n - 1, kmax - 1) into S->distinct and clears them,
// then copies the state header (and |L| of the first recolouring round) into
// the host's pinned staging, from the device, so that no copy command follows
// the rounds: the host reads it once the stream is synchronised.
constexpr int kHeadBlock = 1024;
__global__ __launch_bounds__(kHeadBlock) void k_head_out(const SingleArgs *__restrict__ A, SingleState *S,
                                                         SingleState *dst, int32_t *l1) {
    __shared__ int sh[kHeadBlock / kWave];
    // flags are set only for colours 255 .. kmax - 1 (k_colour_stats raised
    // kmax past every colour it flagged)
    const int64_t len = (int64_t)min(min(S->maxdeg, A->n - 1) + 1, S->kmax) - 255;
    if (len > 0) {
        int32_t *const flags = A->flags + 255;
        int cnt = 0;
        constexpr int kIn = 8;  // loads in flight per lane
        for (int64_t i0 = threadIdx.x; i0 < len; i0 += (int64_t)kIn * kHeadBlock) {
            int f[kIn];
#pragma unroll
            for (int k = 0; k < kIn; ++k) {
                const int64_t i = i0 + (int64_t)k * kHeadBlock;
                f[k] = i < len ? flags[i] : 0;
            }
#pragma unroll
            for (int k = 0; k < kIn; ++k) {
                cnt += f[k];
                if (f[k]) flags[i0 + (int64_t)k * kHeadBlock] = 0;
            }
        }
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        if (lane_id() == 0) sh[threadIdx.x / kWave] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < kHeadBlock / kWave; ++w) t += sh[w];
            S->distinct += t;
        }
        __syncthreads();
    }
    const int32_t *src = reinterpret_cast<const int32_t *>(S);
    int32_t *d = reinterpret_cast<int32_t *>(dst);
    for (int i = threadIdx.x; i < (int)(kStateHeader / 4); i += kHeadBlock) d[i] = src[i];
    if (threadIdx.x == 0) *l1 = S->hist[0];
}

__device__ __forceinline__ uint8_t shadow_of(int c) { return (uint8_t)((unsigned)c < 255u ? c : 255); }

// Round 0 of the optimistic mode: v's nibble is 15 (nothing written since the
// fill) and becomes min(c, 14) with one atomic AND, so that the colour is
// visible to the 4-bit gathers as soon as it is chosen (hub bins; the lane
// groups combine the nibbles of one word first).
__device__ __forceinline__ void publish_nibble(RSOC_GLOBAL uint32_t *col4, int v, int c) {
    const int sh = (v & 7) << 2;
    atomicAnd((uint32_t *)&col4[v >> 3], ~(0xfu << sh) | ((uint32_t)min(c, 14) << sh));
}

// ------------------------------------------------------------------ fill --
// p[0, n) = value, its byte shadow p8 (if given) and, if given, the 4-bit
// shadow words p4[0, n4) = all ones (every nibble 15).
__device__ __forceinline__ void fill_colours(int32_t *p, uint8_t *p8, int64_t n, int32_t value, uint32_t *p4,
                                             int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        p[i] = value;
        if (p8) p8[i] = shadow_of(value);
    }
    if (p4)
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += stride) p4[i] = ~0u;
}
__global__ void k_fill(int32_t *p, uint8_t *p8, int64_t n, int32_t value, uint32_t *p4 = nullptr, int64_t n4 = 0) {
    fill_colours(p, p8, n, value, p4, n4);
}

// ----------------------------------------------------------------- setup --
// Writes the colouring's device-resident arguments (passed by value) and,
// when clear is set, zeroes the round-state header (everything before hist):
// one small launch instead of a copy and a fill.
__global__ void k_setup(SingleArgs *A, SingleArgs a, SingleState *S, int header_words, int clear) {
    if (threadIdx.x == 0) *A = a;
    if (clear) {
        int32_t *w = reinterpret_cast<int32_t *>(S);
        for (int i = threadIdx.x; i < header_words; i += blockDim.x) w[i] = 0;
        for (int i = threadIdx.x; i < kAccSlots * kAccStride; i += blockDim.x) S->acc[i] = 0;
    }
}

// ------------------------------------------------------------- validate --
// Flags malformed rows (decreasing offsets, offsets past nnz, column ids out
// of range) and self-loops.
__global__ void k_validate(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, int32_t n, int32_t *err) {
    const int64_t nnz = rp[n];
    int flags = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int b = rp[v], e = rp[v + 1];
        if (b > e || b < 0 || (int64_t)e > nnz || nnz < 0 || rp[0] != 0) { flags |= 1; continue; }
        for (int j = b; j < e; ++j) {
            const int u = ci[j];
            if ((unsigned)u >= (unsigned)n) flags |= 1;
            else if (u == (int)v) flags |= 2;
        }
    }
    if (ballot(flags != 0)) {
        // one atomic per wavefront with a finding
        int f = flags;
        for (int off = 32; off > 0; off >>= 1) f |= __shfl_xor(f, off);
        if (lane_id() == 0) atomicOr(err, f);
    }
}

// Workgroup max of an int; the result is valid in thread 0.
__device__ __forceinline__ int block_max(int x, int *sh) {
    x = wave_max_i32(x);
    if (lane_id() == 0) sh[threadIdx.x / kWave] = x;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < kWavesPerBlock; ++w) x = max(x, sh[w]);
    return x;
}

// ------------------------------------------------------------------ bin --
// Splits V by degree: deg <= t_thread stays implicit (thread bin); larger rows
// go to the static wavefront / workgroup lists.  Also finds the max degree,
// publishes nnz = row_ptr[n] and checks the ends of row_ptr (row_ptr[0] = 0,
// row_ptr[n] >= 0; err bit 0 otherwise).  The first `gloc` workgroups take the
// id-locality sample instead (ns rows), so that its dependent loads start
// first and overlap the binning.
template <class T = int>
__device__ __forceinline__ void queue_push(bool take, int v, int *q, int *qn, T *qx = nullptr, T x = T());
template <class T = int>
__device__ __forceinline__ void queue_flush(int *q, int *qn, int *qbase, int *counter, int32_t *out,
                                            const T *qx = nullptr, T *outx = nullptr);
template <class T = int>
__device__ __forceinline__ void queue_flush_n(int cnt, int *q, int *qn, int *qbase, int *counter, int32_t *out,
                                              const T *qx = nullptr, T *outx = nullptr);

__device__ __forceinline__ void locality_row(const RSOC_GLOBAL int32_t *rp, const RSOC_GLOBAL int32_t *ci, int v,
                                             int64_t nnz, uint64_t &near, uint64_t &sampled);

__global__ __launch_bounds__(kBlock) void k_bin(const SingleArgs *__restrict__ A, SingleState *S, int gloc, int ns) {
    __shared__ int sh[kWavesPerBlock];
    __shared__ int qW[kQueueCap], qB[kQueueCap];
    __shared__ int nqW, nqB, qbase;
    const SingleArgs a = *A;
    const RSOC_GLOBAL int32_t *rp = gro(a.rp);
    if ((int)blockIdx.x < gloc) {
        uint64_t near = 0, sampled = 0;
        const int k = (int)blockIdx.x * kBlock + threadIdx.x;
        if (k < ns) locality_row(rp, gro(a.ci), (int)((int64_t)k * a.n / ns), rp[a.n], near, sampled);
        near = wave_sum_u64(near);
        sampled = wave_sum_u64(sampled);
        if (lane_id() == 0 && sampled) {
            atomicAdd((unsigned long long *)&S->near, (unsigned long long)near);
            atomicAdd((unsigned long long *)&S->sampled, (unsigned long long)sampled);
        }
        return;
    }
    const int bb = (int)blockIdx.x - gloc, nbb = (int)gridDim.x - gloc;
    if (bb == 0 && threadIdx.x == 0) {
        const int r0 = rp[0], rn = rp[a.n];
        S->nnz = rn;
        if (r0 != 0 || rn < 0) atomicOr(&S->err, 1);
    }
    int md = 0;
    uint64_t rowsW = 0, rowsB = 0;  // independent count of the rows each hub list must receive
    if (threadIdx.x == 0) nqW = nqB = 0;
    __syncthreads();
    const int64_t stride = (int64_t)nbb * kBlock;
    for (int64_t base = (int64_t)bb * kBlock; base < a.n; base += stride) {
        const int v = (int)(base + threadIdx.x);
        int d = -1;
        if (v < a.n) d = rp[v + 1] - rp[v];
        md = max(md, d);
        rowsB += d > a.t_wave;
        rowsW += d > a.t_thread && d <= a.t_wave;
        // workgroup queues: one global atomic per flush, not per wavefront
        queue_push(d > a.t_wave, v, qB, &nqB);
        queue_push(d > a.t_thread && d <= a.t_wave, v, qW, &nqW);
        int cB, cW;
        queue_sizes(&nqB, &nqW, cB, cW);
        if (cB > kQueueCap - kBlock) queue_flush_n(cB, qB, &nqB, &qbase, &S->nB, a.hubB);
        if (cW > kQueueCap - kBlock) queue_flush_n(cW, qW, &nqW, &qbase, &S->nW, a.hubW);
    }
    queue_flush(qB, &nqB, &qbase, &S->nB, a.hubB);
    queue_flush(qW, &nqW, &qbase, &S->nW, a.hubW);
    rowsW = wave_sum_u64(rowsW);
    rowsB = wave_sum_u64(rowsB);
    if (lane_id() == 0 && (rowsW | rowsB)) {
        unsigned long long *slot = S->acc + (blockIdx.x % kAccSlots) * kAccStride;
        if (rowsW) atomicAdd(&slot[kAccBinW], (unsigned long long)rowsW);
        if (rowsB) atomicAdd(&slot[kAccBinB], (unsigned long long)rowsB);
    }
    md = block_max(md, sh);
    // most workgroups find nothing larger than what is already published
    if (threadIdx.x == 0 && md > __hip_atomic_load(&S->maxdeg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&S->maxdeg, md);
}

// Folds the acc words w of all lines into one total and clears them.
__device__ __forceinline__ unsigned long long acc_take(SingleState *S, int w) {
    unsigned long long t = 0;
    for (int k = 0; k < kAccSlots; ++k) {
        unsigned long long *slot = S->acc + k * kAccStride;
        t += slot[w];
        slot[w] = 0;
    }
    return t;
}

// Hub-first round 0 (hub_kernels.hpp), called by a whole grid once binning is
// done: every vertex above the hub threshold joins hubC (only the wavefront
// and workgroup bins can hold one: the threshold is at least t_thread);
// S->nHc counts them, also past kHubCap; S->hub_t = the threshold.
__device__ __forceinline__ void hub_collect(const SingleArgs *A, SingleState *S) {
    if (A->hub_t == 0 || (S->err & kErrNoRun)) return;
    const int maxdeg = S->maxdeg;
    const int T = hub_threshold(*A, maxdeg);
    if (blockIdx.x == 0 && threadIdx.x == 0) S->hub_t = T;
    if (maxdeg <= T) return;
    const int nW = S->nW, nB = S->nB;
    const int from = T >= A->t_wave ? nW : 0;  // rows above t_wave are all in the workgroup bin
    const RSOC_GLOBAL int32_t *rp = gro(A->rp);
    for (int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nW + nB;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int v = i < nW ? A->hubW[i] : A->hubB[i - nW];
        const bool hub = rp[v + 1] - rp[v] > T;
        const uint64_t m = ballot(hub);
        int slot = 0;
        const int lead = m ? __ffsll((unsigned long long)m) - 1 : 0;
        if (m && lane_id() == lead) slot = atomicAdd(&S->nHc, __popcll(m));
        slot = __shfl(slot, lead) + lanes_below(m);
        if (hub && slot < kHubCap) A->hubC[slot] = v;
    }
}

// Completes the arguments once binning is done, on the device, so that the
// rounds can be enqueued behind binning without the host waiting for it: the
// worklists' bin segments, the run length (option 0: from the locality
// sample), and bit 3 of err when there are edges but no col_idx.  The sweeps
// do not run while err has bit 0 (row_ptr ends, from k_bin) or bit 3 set.
// Workgroup 0 does that and then sends the header to the host's staging (dst)
// as k_head_out does; the whole grid meanwhile fills the colours for round 0
// (value, its byte shadow, and all-ones 4-bit shadow words p4[0, n4) if
// given), as k_fill would.
__global__ void k_args(SingleArgs *A, SingleState *S, SingleState *dst, int32_t *col, uint8_t *col8, int64_t n,
                       int32_t value, uint32_t *col4, int64_t n4) {
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            const int nv = A->n;
            A->offW = nv - S->nW - S->nB;
            A->offB = nv - S->nB;
            A->chunk = pick_chunk(A->chunk, S->near, S->sampled);
            S->chunk = A->chunk;
            // ids without locality: a neighbour v wins against is seldom
            // coloured before v (the sweep's band is gT * kSub ids wide), so by
            // default round 0 reads none of them
            if (A->look_auto && A->chunk == 1) A->look = 0;
            if (A->ci == nullptr && S->nnz > 0) S->err |= 8;
            // the hub lists hold exactly the rows binning counted in their ranges
            const unsigned long long rw = acc_take(S, kAccBinW), rb = acc_take(S, kAccBinB);
            if (rw != (unsigned long long)S->nW || rb != (unsigned long long)S->nB) S->err |= kErrListCount;
        }
        __syncthreads();
        const int32_t *src = reinterpret_cast<const int32_t *>(S);
        int32_t *d = reinterpret_cast<int32_t *>(dst);
        for (int i = threadIdx.x; i < (int)(kStateHeader / 4); i += blockDim.x) d[i] = src[i];
    }
    hub_collect(A, S);
    fill_colours(col, col8, n, value, col4, n4);
}

// Id-locality sample: rows of `ns` vertices spread evenly over [0, n) (rows
// longer than the thread bin, or not inside [0, nnz), skipped); counts
// entries joining ids less than kChunk apart.  One vertex per thread, its row
// read eight entries at a time.
__device__ __forceinline__ void locality_row(const RSOC_GLOBAL int32_t *rp, const RSOC_GLOBAL int32_t *ci, int v,
                                             int64_t nnz, uint64_t &near, uint64_t &sampled) {
    const int b = rp[v], e = rp[v + 1];
    if (b < 0 || e < b || (int64_t)e > nnz || e - b > kThreadBinMax) return;
    for (int j0 = b; j0 < e; j0 += 8) {
        int u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = (j0 + k < e) ? ci[j0 + k] : INT_MIN / 2;
#pragma unroll
        for (int k = 0; k < 8; ++k) near += (uint64_t)(abs(u[k] - v) < kChunk);
    }
    sampled += (uint64_t)(e - b);
}

// Per-wavefront append buffer in LDS (wavefront-bin vertices are appended one
// at a time by lane 0; one global atomic per kWaveBuf entries).
constexpr int kWaveBuf = 64;
constexpr int kMaskedBuf = 512;  // flushed when fewer than a wavefront's worth of slots are left
constexpr int kAuxCap = 1024;    // round-0 queue length when U^0 entries carry their kept neighbours

template <class T>
__device__ __forceinline__ void wave_buf_flush(T *buf, int *bn, int *counter, T *out) {
    wave_lds_sync();
    const int cnt = *bn;
    if (cnt == 0) return;
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, cnt);
    base = __shfl(base, 0);
    for (int i = lane_id(); i < cnt; i += kWave) out[base + i] = buf[i];
    wave_lds_sync();
    if (lane_id() == 0) *bn = 0;
    wave_lds_sync();
}

// Lane 0 pushes x when take; the whole wavefront calls this (flushes when full).
template <class T>
__device__ __forceinline__ void wave_buf_push(bool take, T x, T *buf, int *bn, int *counter, T *out) {
    if (lane_id() == 0 && take) buf[(*bn)++] = x;
    wave_lds_sync();
    if (*bn == kWaveBuf) wave_buf_flush(buf, bn, counter, out);
}

// Appends v for every lane with `take` into the workgroup's LDS queue (and,
// when qx is given, x beside it).  Called by every thread of the workgroup in
// lockstep (the loop is workgroup-uniform).
template <class T>
__device__ __forceinline__ void queue_push(bool take, int v, int *q, int *qn, T *qx, T x) {
    const uint64_t m = ballot(take);
    if (m == 0) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(qn, __popcll(m));
    base = __shfl(base, leader);
    if (take) {
        q[base + lanes_below(m)] = v;
        if (qx) qx[base + lanes_below(m)] = x;
    }
}

// Moves the queue's cnt entries to the global list (one global atomic per
// flush); the side entries qx, when given, go to the same positions of outx.
// cnt is the queue size every wavefront agreed on (queue_size), so the whole
// workgroup takes the same path; the counter is reset before the first
// barrier (every wavefront has read it already and none appends until the
// flush returns), and the last barrier frees the queue and qbase again.
template <class T>
__device__ __forceinline__ void queue_flush_n(int cnt, int *q, int *qn, int *qbase, int *counter, int32_t *out,
                                              const T *qx, T *outx) {
    if (cnt == 0) return;
    if (threadIdx.x == 0) {
        *qbase = atomicAdd(counter, cnt);
        *qn = 0;
    }
    __syncthreads();
    const int base = *qbase;
    for (int i = threadIdx.x; i < cnt; i += kBlock) {
        out[base + i] = q[i];
        if (qx) outx[base + i] = qx[i];
    }
    __syncthreads();
}

template <class T>
__device__ __forceinline__ void queue_flush(int *q, int *qn, int *qbase, int *counter, int32_t *out, const T *qx,
                                            T *outx) {
    queue_flush_n<T>(queue_size(qn), q, qn, qbase, counter, out, qx, outx);
}

// Masked round: the entries of this wavefront selected by sel (bit = lane,
// vertex v of that lane) are staged in the wavefront's LDS slots ms and
// handled kGroup lanes each: PH = kAssign gives a vertex known to be defective
// First-Fit over all neighbours; PH = kRecolor detects first.  Recoloured
// vertices are written (colour, byte shadow, nibble invalidated) and added to
// the wavefront's append buffer mb (*mbn entries).
template <int PH, int TIE, bool NIB>
__device__ __forceinline__ void wave_recolour_selected(uint64_t sel, int v, int *ms, int *mb, int *mbn,
                                                       const RSOC_GLOBAL int32_t *rp, const RSOC_GLOBAL int32_t *ci,
                                                       const RSOC_GLOBAL uint8_t *col8,
                                                       const RSOC_GLOBAL uint32_t *col4, RSOC_GLOBAL int32_t *wcol,
                                                       RSOC_GLOBAL uint8_t *wcol8, RSOC_GLOBAL uint32_t *wcol4,
                                                       int look, uint64_t &degs, uint64_t &napp) {
    if (sel & (1ull << lane_id())) ms[lanes_below(sel)] = v;
    wave_lds_sync();
    const int nd = __popcll(sel);
    const int gi = lane_id() / kGroup;
    const bool leader = (lane_id() & (kGroup - 1)) == 0;
    for (int d0 = 0; d0 < nd; d0 += kWave / kGroup) {
        int gv[1] = {-1}, gb[1] = {0}, ge[1] = {0}, gcv[1] = {255}, gnc[1] = {0};
        bool gact[1];
        uint32_t gunc[1] = {};
        int x = 0;
        const int k = lane_id() & (kGroup - 1);
        if (d0 + gi < nd) {
            gv[0] = ms[d0 + gi];
            if (k < 2) x = rp[gv[0] + k];
            else if (PH != kAssign && k == 2) x = col8[gv[0]];
        }
        const int g0 = lane_id() & ~(kGroup - 1);
        gb[0] = __shfl(x, g0);
        ge[0] = __shfl(x, g0 + 1);
        if (PH != kAssign) gcv[0] = __shfl(x, g0 + 2);
        if (gv[0] < 0) gb[0] = ge[0] = 0, gcv[0] = 255;
        const RSOC_GLOBAL int32_t *gci[1] = {ci};
        const RSOC_GLOBAL uint8_t *gc8[1] = {col8};
        const RSOC_GLOBAL uint32_t *gc4[1] = {col4};
        group_vertices<PH, TIE, kGroup, kGroupSlots, false, 1, NIB>(gv, gb, ge, gci, gc8, gcv, look, gnc, gact, gunc,
                                                                   gc4);
        const bool w = leader && gv[0] >= 0 && gact[0];
        if (leader && gv[0] >= 0) degs += (uint64_t)(ge[0] - gb[0]);
        if (w) {
            wcol[gv[0]] = gnc[0];
            wcol8[gv[0]] = (uint8_t)gnc[0];
            // a recoloured vertex's nibble becomes 15: readers then use col8
            if (NIB) atomicOr((uint32_t *)&wcol4[gv[0] >> 3], 0xfu << ((gv[0] & 7) << 2));
        }
        const uint64_t am = ballot(w);
        if (lane_id() == 0) napp += (uint64_t)__popcll(am);
        if (w) mb[*mbn + lanes_below(am)] = gv[0];
        wave_lds_sync();
        if (lane_id() == 0) *mbn += __popcll(am);
        wave_lds_sync();
    }
}

// Round 0 of the optimistic mode, lane groups: publishes into the 4-bit
// shadow the colours this sub-step chose.  ids[i] is the vertex id slot i of
// this lane's group covers (-1 past the end; v[i] is -1 when that vertex
// belongs to another bin and was not coloured here).  The ids of a
// wavefront's 8 groups are monotone in the group index, so the groups sharing
// a 32-bit word are contiguous: a segmented OR-scan over them gathers the
// bits to clear and the last group of each word issues one atomic AND (the
// nibbles start at 15 and each is set once).
template <int NV>
__device__ __forceinline__ void publish_nibbles(const int (&ids)[NV], const int (&v)[NV], const int (&nc)[NV],
                                                RSOC_GLOBAL uint32_t *col4, bool leader) {
    const int g = lane_id() / kGroup;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int key = ids[i] >= 0 ? (ids[i] >> 3) : -1 - g;
        uint32_t clr = v[i] >= 0 ? (0xfu ^ (uint32_t)min(nc[i], 14)) << ((v[i] & 7) << 2) : 0u;
#pragma unroll
        for (int d = 1; d < kWave / kGroup; d <<= 1) {
            const uint32_t oc = __shfl_up(clr, d * kGroup);
            const int ok = __shfl_up(key, d * kGroup);
            if (g >= d && ok == key) clr |= oc;
        }
        const int nk = __shfl_down(key, kGroup);
        const bool last = g == kWave / kGroup - 1 || nk != key;
        if (leader && last && clr) atomicAnd((uint32_t *)&col4[key], ~clr);
    }
}

// ---------------------------------------------------------------- round --
// PHASE: kAssign (First-Fit), kRecolor (detect + First-Fit), kDetect.
// MODE: kOptimistic writes colours in place (live reads); otherwise new
//       colours are staged in pend[] and published by k_scatter.
// SWEEP: the round covers all of V (rounds 0 and 1): the thread bin walks
//        vertex ids directly, the other bins read the static lists; otherwise
//        the round reads worklist buffer `parity` and appends to parity^1.
// Sections: blocks [0,gB) workgroup bin, [gB,gB+gW) wavefront bin, then gT
// thread bin (kGroup lanes per vertex).
// ROUND0 (kAssign only): 0 = First-Fit over all neighbours, no appends;
// 1 = First-Fit over the neighbours v loses to, sweeping in the order that
// visits them first, and v is appended to the next worklist iff one of them
// was still uncoloured when read (only such v can end round 0 defective); a
// thread-bin v also stores which neighbours those were (aux).
// ROUND0 = 2 (kRecolor, optimistic, worklist): the round right after that:
// thread-bin entries take one lane each and only test the stored positions
// (lane_detect_kept); the defective ones are then recoloured by lane groups.
template <int PHASE, int MODE, int TIE, bool SWEEP, int ROUND0 = 0>
__global__ __launch_bounds__(kBlock) void k_round(const SingleArgs *__restrict__ A, SingleState *S, int parity,
                                                  int gB_, int gW_, int gT) {
    __shared__ uint32_t lds[kLdsWords];
    constexpr bool kFlagAppend = PHASE == kAssign && ROUND0 == 1;
    constexpr bool kMasked = PHASE == kRecolor && ROUND0 == 2 && !SWEEP && MODE == kOptimistic;
    __shared__ int q[kQueueCap];
    __shared__ int4 qa[kFlagAppend ? kAuxCap : 1];
    __shared__ int sh_min, qn, qbase;
    __shared__ unsigned long long sh_acc[3];
    __shared__ int wbuf[kWavesPerBlock][kWaveBuf];
    __shared__ int wbn[kWavesPerBlock];
    // masked round: per-wavefront defective staging and append buffer
    __shared__ int mstage[kMasked ? kWavesPerBlock : 1][kMasked ? kWave : 1];
    __shared__ int mbuf[kMasked ? kWavesPerBlock : 1][kMasked ? kMaskedBuf : 1];
    __shared__ int mbn[kWavesPerBlock];
    const SingleArgs a = *A;
    if (!SWEEP && S->passes >= a.max_rounds) return;  // guard: the round may not run
    if (SWEEP && (S->err & kErrNoRun)) return;        // the input failed its checks
    // hub-first round 0 (hub_kernels.hpp): the hubs already hold their
    // colours; every other vertex reads all of its neighbours, those it wins
    // against through the 4-bit shadow first (a hub's nibble is its colour,
    // or 14 for 14 and more, settled exactly), so that none takes a hub's
    // colour
    const int nHub = kFlagAppend ? S->nH : 0;
    const int hubT = nHub ? S->hub_t : INT_MAX;
    const int look = nHub ? INT_MAX : a.look;
    const int cT = SWEEP ? a.n : S->cnt_in[kBinThread];
    const int cW = SWEEP ? S->nW : S->cnt_in[kBinWave];
    const int cB = SWEEP ? S->nB : S->cnt_in[kBinBlock];
    int32_t *const in = parity ? a.wl[1] : a.wl[0];
    int32_t *const out = parity ? a.wl[0] : a.wl[1];
    const RSOC_GLOBAL int32_t *inT = gro(in);
    const RSOC_GLOBAL int32_t *inW = gro(SWEEP ? a.hubW : in + a.offW);
    const RSOC_GLOBAL int32_t *inB = gro(SWEEP ? a.hubB : in + a.offB);
    const RSOC_GLOBAL int32_t *rp = gro(a.rp);
    const RSOC_GLOBAL int32_t *ci = gro(a.ci);
    const RSOC_GLOBAL int32_t *rcol = gro(a.col);
    const RSOC_GLOBAL uint8_t *rcol8 = gro(a.col8);
    RSOC_GLOBAL int32_t *wcol = grw(live_mode(MODE) ? a.col : a.pend);
    RSOC_GLOBAL uint8_t *wcol8 = grw(a.col8);
    // The 4-bit shadow is kept in optimistic mode (colours change in place):
    // round 0 publishes each colour into it as soon as it is chosen
    // (publish_nibble); a recoloured vertex's nibble becomes 15.
    constexpr bool kNib = MODE == kOptimistic;
    constexpr bool kPublish = kNib && PHASE == kAssign;
    // a round 0 over all neighbours (ROUND0 = 0) gathers from the byte
    // shadow: half its neighbours are still uncoloured, and each of those
    // would cost a nibble read and then a byte read
    constexpr bool kNibRead = kNib && (PHASE != kAssign || kFlagAppend);
    const RSOC_GLOBAL uint32_t *rcol4 = gro(a.col4);
    RSOC_GLOBAL uint32_t *wcol4 = grw(a.col4);
    constexpr bool kWinOnly = kFlagAppend;
    constexpr bool kAppend = PHASE != kAssign || kFlagAppend;
    constexpr bool kWrite = PHASE != kDetect;
    constexpr bool kAcct = PHASE != kAssign && !SWEEP;  // worklist rounds count their inspections
    uint64_t items = 0, degs = 0;
    uint64_t apps = 0;  // entries this thread decided to append (the list-size check)
    // A sweep's hub sections may be launched larger than its bins need (the
    // host enqueues it before it knows the bin sizes): the workgroups the bins
    // need keep the front of the grid and the surplus, at its end, leaves.
    const int gB = SWEEP ? min(gB_, cB) : gB_;
    const int gW = SWEEP ? min(gW_, (cW + kWavesPerBlock - 1) / kWavesPerBlock) : gW_;
    const int bid = blockIdx.x;
    if (bid >= gB + gW + gT) return;
    if (bid < gB) {
        if (threadIdx.x == 0) qn = 0;
        __syncthreads();
        for (int i = bid; i < cB; i += gB) {
            const int v = inB[i];
            const int b = rp[v], e = rp[v + 1];
            if (nHub && e - b > hubT) continue;  // a hub: coloured before this round (workgroup-uniform)
            int nc = 0;
            bool unc = false;
            const bool act = block_vertex<PHASE, TIE, kWinOnly>(v, b, e, ci, rcol, rcol8, lds, &sh_min, look, nc, unc,
                                                                nHub > 0, rcol4);
            const bool take = (kFlagAppend ? unc : act) && kAppend;
            if (threadIdx.x == 0) {
                items += 1;
                degs += (uint64_t)(e - b);
                if (act && kWrite) {
                    wcol[v] = nc;
                    if (live_mode(MODE)) wcol8[v] = shadow_of(nc);
                    if (kPublish) publish_nibble(wcol4, v, nc);
                    else if (kNib) atomicOr((uint32_t *)&wcol4[v >> 3], 0xfu << ((v & 7) << 2));
                }
                if (take) {
                    q[qn++] = v;
                    apps += 1;
                }
            }
            const int cq = queue_size(&qn);
            if (cq == kQueueCap) queue_flush_n(cq, q, &qn, &qbase, &S->cnt_out[kBinBlock], out + a.offB);
        }
        if (kAppend) queue_flush(q, &qn, &qbase, &S->cnt_out[kBinBlock], out + a.offB);
    } else if (bid < gB + gW) {
        const int wv = threadIdx.x / kWave;
        const int w = (bid - gB) * kWavesPerBlock + wv;
        const int nw = gW * kWavesPerBlock;
        uint32_t *bm = lds + wv * kWaveWindowWords;
        if (lane_id() == 0) wbn[wv] = 0;
        wave_lds_sync();
        for (int i = w; i < cW; i += nw) {
            const int v = inW[i];
            const int b = rp[v], e = rp[v + 1];
            if (nHub && e - b > hubT) continue;  // a hub (wavefront-uniform)
            int nc = 0;
            bool unc = false;
            const bool act =
                wave_vertex<PHASE, TIE, kWinOnly>(v, b, e, ci, rcol, rcol8, bm, look, nc, unc, nHub > 0, rcol4);
            if (lane_id() == 0) {
                items += 1;
                degs += (uint64_t)(e - b);
                if (act && kWrite) {
                    wcol[v] = nc;
                    if (live_mode(MODE)) wcol8[v] = shadow_of(nc);
                    if (kPublish) publish_nibble(wcol4, v, nc);
                    else if (kNib) atomicOr((uint32_t *)&wcol4[v >> 3], 0xfu << ((v & 7) << 2));
                }
            }
            if (kAppend && lane_id() == 0 && (kFlagAppend ? unc : act)) apps += 1;
            if (kAppend) wave_buf_push((kFlagAppend ? unc : act), v, wbuf[wv], &wbn[wv], &S->cnt_out[kBinWave],
                                       out + a.offW);
        }
        if (kAppend) wave_buf_flush(wbuf[wv], &wbn[wv], &S->cnt_out[kBinWave], out + a.offW);
    } else if (kMasked) {
        // one lane per list entry; wavefronts run independently (no workgroup
        // barrier): defective vertices are staged in the wavefront's LDS slots
        // and recoloured kGroup lanes each, appends gather in its LDS buffer
        const int wv = threadIdx.x / kWave;
        const int nwv = gT * kWavesPerBlock;
        int *ms = mstage[wv];
        int *mb = mbuf[wv];
        if (lane_id() == 0) mbn[wv] = 0;
        wave_lds_sync();
        typedef int v4i __attribute__((ext_vector_type(4)));
        const RSOC_GLOBAL v4i *ax = (const RSOC_GLOBAL v4i *)a.aux;
        for (int64_t base = (int64_t)((bid - gB - gW) * kWavesPerBlock + wv) * kWave; base < cT;
             base += (int64_t)nwv * kWave) {
            const int64_t idx = base + lane_id();
            int v = -1, cv = 255;
            int4 x = {0, 0, 0, 0};
            if (idx < cT) {
                v = inT[idx];
                const v4i y = ax[idx];
                x = make_int4(y.x, y.y, y.z, y.w);
                cv = rcol8[v];
            }
            // up to three kept neighbours: tested here; more: the lane groups
            // run the full detection for that vertex
            const bool over = v >= 0 && __popc((uint32_t)x.w) > 3;
            const bool def = v >= 0 && !over && lane_detect_kept<kNib>(v, x, cv, rcol8, rcol4);
            if (v >= 0) {
                items += 1;
                degs += (uint64_t)__popc((uint32_t)x.w);
            }
            wave_recolour_selected<kAssign, TIE, kNib>(ballot(def), v, ms, mb, &mbn[wv], rp, ci, rcol8, rcol4, wcol,
                                                       wcol8, wcol4, a.look, degs, apps);
            const uint64_t om = ballot(over);
            if (om)
                wave_recolour_selected<kRecolor, TIE, kNib>(om, v, ms, mb, &mbn[wv], rp, ci, rcol8, rcol4, wcol,
                                                            wcol8, wcol4, a.look, degs, apps);
            if (mbn[wv] >= kMaskedBuf - kWave) wave_buf_flush(mb, &mbn[wv], &S->cnt_out[kBinThread], out);
        }
        // what the wavefronts still hold leaves in one workgroup-wide flush
        // (one global atomic per workgroup instead of one per wavefront)
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < kWavesPerBlock; ++w) tot += mbn[w];
            qbase = tot ? atomicAdd(&S->cnt_out[kBinThread], tot) : 0;
        }
        __syncthreads();
        int off = qbase;
        for (int w = 0; w < wv; ++w) off += mbn[w];
        for (int i = lane_id(); i < mbn[wv]; i += kWave) out[off + i] = mb[i];
    } else {
        int tb = bid - gB - gW;
        // worklist-free sweeps that need no particular order keep each XCD on
        // one id range (neighbouring ids share its L2); round 0 sweeps in order
        if (SWEEP && PHASE != kAssign) tb = xcd_contiguous(tb, gT);
        const int gi = threadIdx.x / kGroup;
        const bool leader = (threadIdx.x & (kGroup - 1)) == 0;
        if (kAppend) {
            if (threadIdx.x == 0) qn = 0;
            __syncthreads();
        }
        // A sweep over ids with locality (chunk c > 1) gives each workgroup
        // step kStep ids, walked as runs of c in order.  Over ids without
        // locality (c = 1) a step is one sub-step of kSub ids: the grid then
        // sweeps a band of gT * kSub ids at a time, not gT * kStep, so a
        // vertex finds far fewer of the lower ids it reads still uncoloured
        // (round 0 collects fewer vertices into U^0).  A worklist has no
        // order to keep and is often short after round 1, so there a step is
        // kSub entries too: the list spreads over the whole grid instead of a
        // few workgroups walking kChunk dependent sub-steps each.
        const int c = SWEEP ? a.chunk : 1;
        const int kRuns = c > 1 ? kChunk : 1;
        const int kUnit = c > 1 ? kStep : kSub;
        const int64_t stride = (int64_t)gT * kUnit;
        for (int64_t base = (int64_t)tb * kUnit; base < cT; base += stride) {
            for (int r = 0; r < kRuns; ++r) {
                int v[kNV], b[kNV], e[kNV], cv[kNV], nc[kNV];
                bool act[kNV];
                uint32_t unc[kNV] = {};
                int keep[kNV][4];
                // per-vertex scalars are loaded by one lane of the group each
                // and shuffled to the others: the texture addresser's work
                // grows with the lanes a load has active, not with its lines
                const int k = threadIdx.x & (kGroup - 1);
                const int g0 = lane_id() & ~(kGroup - 1);
#pragma unroll
                for (int i = 0; i < kNV; ++i) {
                    const int64_t idx = base + step_offset(r, i, gi, c);
                    v[i] = -1;
                    if (idx < cT) {
                        if (SWEEP) {
                            v[i] = (kFlagAppend && TIE == kHigherKeeps) ? (int)(cT - 1 - idx) : (int)idx;
                        } else {
                            int x = 0;
                            if (k == 0) x = inT[idx];
                            v[i] = __shfl(x, g0);
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < kNV; ++i) {
                    int x = 0;
                    if (v[i] >= 0) {
                        if (k < 2) x = rp[v[i] + k];
                        else if (PHASE != kAssign && k == 2) x = rcol8[v[i]];
                    }
                    b[i] = __shfl(x, g0);
                    e[i] = __shfl(x, g0 + 1);
                    cv[i] = (PHASE != kAssign && v[i] >= 0) ? __shfl(x, g0 + 2) : 255;
                    if (v[i] < 0) b[i] = e[i] = 0;
                    if (SWEEP && e[i] - b[i] > a.t_thread) e[i] = b[i] = 0, v[i] = -1;  // another bin's vertex
                }
                const RSOC_GLOBAL int32_t *cis[kNV];
                const RSOC_GLOBAL uint8_t *c8s[kNV];
                const RSOC_GLOBAL uint32_t *c4s[kNV];
#pragma unroll
                for (int i = 0; i < kNV; ++i) cis[i] = ci, c8s[i] = rcol8, c4s[i] = rcol4;
                group_vertices<PHASE, TIE, kGroup, kGroupSlots, kWinOnly, kNV, kNibRead>(v, b, e, cis, c8s, cv, look, nc,
                                                                                     act, unc, c4s,
                                                                                     kFlagAppend ? keep : nullptr,
                                                                                     nHub > 0);
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
                            wcol[v[i]] = nc[i];
                            if (live_mode(MODE)) wcol8[v[i]] = (uint8_t)nc[i];
                            // a recoloured vertex's nibble becomes 15: readers then use col8
                            // (round 0 publishes nibbles below, one atomic per word)
                            if (kNib && !kPublish) atomicOr((uint32_t *)&wcol4[v[i] >> 3], 0xfu << ((v[i] & 7) << 2));
                        }
                    }
                }
                if (kPublish) {
                    int ids[kNV];
#pragma unroll
                    for (int i = 0; i < kNV; ++i) {
                        const int64_t idx = base + step_offset(r, i, gi, c);
                        ids[i] = idx < cT ? ((kFlagAppend && TIE == kHigherKeeps) ? (int)(cT - 1 - idx) : (int)idx) : -1;
                    }
                    publish_nibbles<kNV>(ids, v, nc, wcol4, leader);
                }
                if (kAppend) {
#pragma unroll
                    for (int i = 0; i < kNV; ++i) apps += ((kFlagAppend ? unc[i] != 0 : act[i]) && leader) ? 1 : 0;
#pragma unroll
                    for (int i = 0; i < kNV; ++i)
                        queue_push<int4>((kFlagAppend ? unc[i] != 0 : act[i]) && leader, v[i], q, &qn,
                                         kFlagAppend ? qa : nullptr,
                                         kFlagAppend ? make_int4(keep[i][0], keep[i][1], keep[i][2], keep[i][3])
                                                     : int4{});
                    const int cq = queue_size(&qn);
                    if (cq > (kFlagAppend ? kAuxCap : kQueueCap) - kSub)
                        queue_flush_n<int4>(cq, q, &qn, &qbase, &S->cnt_out[kBinThread], out,
                                            kFlagAppend ? qa : nullptr, a.aux);
                }
            }
        }
        if (kAppend)
            queue_flush<int4>(q, &qn, &qbase, &S->cnt_out[kBinThread], out, kFlagAppend ? qa : nullptr, a.aux);
    }
    if (kAcct || kAppend) {
        if (threadIdx.x < 3) sh_acc[threadIdx.x] = 0;
        __syncthreads();
        items = wave_sum_u64(items);
        degs = wave_sum_u64(degs);
        apps = wave_sum_u64(apps);
        if (lane_id() == 0 && kAcct && items) {
            atomicAdd(&sh_acc[0], (unsigned long long)items);
            atomicAdd(&sh_acc[1], (unsigned long long)degs);
        }
        if (lane_id() == 0 && apps) atomicAdd(&sh_acc[2], (unsigned long long)apps);
        __syncthreads();
        unsigned long long *slot = S->acc + (blockIdx.x % kAccSlots) * kAccStride;
        if (threadIdx.x == 0 && sh_acc[0]) {
            atomicAdd(&slot[kAccItems], sh_acc[0]);
            atomicAdd(&slot[kAccDegs], sh_acc[1]);
        }
        if (threadIdx.x == 0 && sh_acc[2]) atomicAdd(&slot[kAccAppended], sh_acc[2]);
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
    RSOC_GLOBAL int32_t *col = grw(a.col);
    RSOC_GLOBAL uint8_t *col8 = grw(a.col8);
    const RSOC_GLOBAL int32_t *pend = gro(a.pend);
    if (SWEEP) {
        for (int64_t v = t0; v < a.n; v += stride) {
            const int c = pend[v];
            col[v] = c;
            col8[v] = shadow_of(c);
        }
        return;
    }
    if (S->passes >= a.max_rounds) return;
    const bool use_wl1 = USE_IN ? (parity != 0) : (parity == 0);
    const RSOC_GLOBAL int32_t *lst = gro(use_wl1 ? a.wl[1] : a.wl[0]);
    const int32_t *cnt = USE_IN ? S->cnt_in : S->cnt_out;
    for (int bin = 0; bin < 3; ++bin) {
        const int c = cnt[bin];
        const int off = bin == 0 ? 0 : (bin == 1 ? a.offW : a.offB);
        for (int64_t i = t0; i < c; i += stride) {
            const int v = lst[off + i];
            const int cc = pend[v];
            col[v] = cc;
            col8[v] = shadow_of(cc);
        }
    }
}

// ------------------------------------------------ recolouring after edits --
// Set-up of a recolouring that starts from a given colouring (col[], the
// colouring before the edits; negative = no colour): the byte shadow and, in
// the optimistic mode (NIB), the 4-bit shadow follow col, and mark[v] = 1 for
// every vertex without a valid First-Fit colour (negative, or above its
// degree), else 0.
template <bool NIB>
__global__ __launch_bounds__(kBlock) void k_inc_shadow(const SingleArgs *__restrict__ A, int32_t *mark) {
    const SingleArgs a = *A;
    const RSOC_GLOBAL int32_t *col = gro(a.col);
    const RSOC_GLOBAL int32_t *rp = gro(a.rp);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int64_t v = t0; v < a.n; v += stride) {
        const int c = col[v];
        a.col8[v] = shadow_of(c);
        mark[v] = (c < 0 || c > rp[v + 1] - rp[v]) ? 1 : 0;
    }
    if (NIB)
        for (int64_t w = t0; w < (int64_t)a.n / 8 + 1; w += stride) {
            uint32_t word = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int64_t v = w * 8 + k;
                const int c = v < a.n ? col[v] : -1;
                word |= (c < 0 ? 15u : (uint32_t)min(c, 14)) << (4 * k);
            }
            a.col4[w] = word;
        }
}

// Marks the touched vertices; an id outside [0, n) sets err bit 4 and is
// skipped.
__global__ __launch_bounds__(kBlock) void k_inc_touch(const SingleArgs *__restrict__ A, SingleState *S,
                                                      const int32_t *__restrict__ touched, int64_t nt, int32_t *mark) {
    const int n = A->n;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nt; i += (int64_t)gridDim.x * kBlock) {
        const int t = touched[i];
        if (t < 0 || t >= n) bad = true;
        else mark[t] = 1;
    }
    if (ballot(bad) && lane_id() == 0) atomicOr(&S->err, 16);
}

// U^0 of the recolouring: the marked vertices, appended by degree bin into
// worklist buffer 0 (k_round_end then publishes them as the current list).
__global__ __launch_bounds__(kBlock) void k_inc_list(const SingleArgs *__restrict__ A, SingleState *S,
                                                     const int32_t *__restrict__ mark) {
    __shared__ int qT[kQueueCap], qW[kQueueCap], qB[kQueueCap];
    __shared__ int nqT, nqW, nqB, qbase;
    const SingleArgs a = *A;
    const RSOC_GLOBAL int32_t *rp = gro(a.rp);
    int32_t *const out = a.wl[0];
    uint64_t apps = 0;
    if (threadIdx.x == 0) nqT = nqW = nqB = 0;
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < a.n; base += (int64_t)gridDim.x * kBlock) {
        const int v = (int)(base + threadIdx.x);
        const bool m = v < a.n && mark[v] != 0;
        const int d = m ? rp[v + 1] - rp[v] : 0;
        apps += m ? 1 : 0;
        queue_push(m && d > a.t_wave, v, qB, &nqB);
        queue_push(m && d > a.t_thread && d <= a.t_wave, v, qW, &nqW);
        queue_push(m && d <= a.t_thread, v, qT, &nqT);
        int cB, cW, cT;
        queue_sizes(&nqB, &nqW, &nqT, cB, cW, cT);
        if (cB > kQueueCap - kBlock) queue_flush_n(cB, qB, &nqB, &qbase, &S->cnt_out[kBinBlock], out + a.offB);
        if (cW > kQueueCap - kBlock) queue_flush_n(cW, qW, &nqW, &qbase, &S->cnt_out[kBinWave], out + a.offW);
        if (cT > kQueueCap - kBlock) queue_flush_n(cT, qT, &nqT, &qbase, &S->cnt_out[kBinThread], out);
    }
    queue_flush(qB, &nqB, &qbase, &S->cnt_out[kBinBlock], out + a.offB);
    queue_flush(qW, &nqW, &qbase, &S->cnt_out[kBinWave], out + a.offW);
    queue_flush(qT, &nqT, &qbase, &S->cnt_out[kBinThread], out);
    apps = wave_sum_u64(apps);
    if (lane_id() == 0 && apps)
        atomicAdd(&S->acc[(blockIdx.x % kAccSlots) * kAccStride + kAccAppended], (unsigned long long)apps);
}

// ------------------------------------------------------------ round end --
// Runs after a round (single thread): counts the pass, records |L|, makes the
// appended list the next worklist and clears the append counters.
// PUBLISH_ONLY: after round 0 (no pass to count): only publish the appended list.
template <int MODE, bool SWEEP, bool PUBLISH_ONLY = false>
__global__ void k_round_end(const SingleArgs *__restrict__ A, SingleState *S) {
    // the colour statistics that follow the rounds start from zero
    if (threadIdx.x < 8) S->cbits[threadIdx.x] = 0;
    if (threadIdx.x != 0) return;
    S->kmax = 0;
    S->distinct = 0;
    // the appended list holds exactly the entries the round decided to append
    if (acc_take(S, kAccAppended) != (unsigned long long)(S->cnt_out[0] + S->cnt_out[1] + S->cnt_out[2]))
        S->err |= kErrListCount;
    if (PUBLISH_ONLY) {
        S->u0 = S->cnt_out[0] + S->cnt_out[1] + S->cnt_out[2];
        for (int b = 0; b < 3; ++b) {
            S->cnt_in[b] = S->cnt_out[b];
            S->cnt_out[b] = 0;
        }
        return;
    }
    if (!SWEEP && S->passes >= A->max_rounds) return;  // the guarded round did nothing
    S->inspected += acc_take(S, kAccItems);
    S->deg_sum += acc_take(S, kAccDegs);
    const int in_total = SWEEP ? A->n : (S->cnt_in[0] + S->cnt_in[1] + S->cnt_in[2]);
    const int out_total = S->cnt_out[0] + S->cnt_out[1] + S->cnt_out[2];
    if (in_total > 0) {
        S->prevL = S->lastL;
        S->lastL = out_total;
        S->passes += 1;
        if (S->passes == 1) {
            S->inspected1 = S->inspected;
            S->deg_sum1 = S->deg_sum;
        }
        if (two_phase_mode(MODE)) {
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
// K = max colour + 1 and the set of colours used, read from the byte shadow
// (16 vertices per lane and load, four loads at a time); only a vertex whose shadow is 255
// (colour 255 or more, or none) reads its full colour.  Colours below 64 are
// gathered in a register mask, 64..254 in the workgroup's LDS set, both then
// OR-ed into S->cbits; colours >= 255 mark flags[c] (counted, and cleared, by
// k_head_out).  A colour outside [0, maxdeg] sets err bit 2.
// Everything is read on the device (arguments block, max degree), so the
// kernel can close a captured round graph; every colour is at most
// min(max degree, n - 1), a First-Fit value over at most that many neighbours.
__global__ __launch_bounds__(kBlock) void k_colour_stats(const SingleArgs *__restrict__ A, SingleState *S) {
    __shared__ uint32_t bits[8];
    __shared__ int sh[kWavesPerBlock];
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    const int64_t n = A->n;
    const int32_t maxdeg = min(S->maxdeg, A->n - 1);
    int32_t *const flags = A->flags;
    const RSOC_GLOBAL v4u *c16 = (const RSOC_GLOBAL v4u *)A->col8;  // 16 bytes per entry (col8 holds n + 64 bytes)
    const RSOC_GLOBAL int32_t *col = gro(A->col);
    if (threadIdx.x < 8) bits[threadIdx.x] = 0;
    __syncthreads();
    int m = -1;
    bool bad = false;
    uint64_t low = 0;
    const int64_t n16 = (n + 15) / 16;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    // four 16-byte loads in flight per lane before any is examined
    constexpr int kIn = 4;
    for (int64_t t0 = blockIdx.x * (int64_t)kBlock + threadIdx.x; t0 < n16; t0 += kIn * stride) {
        v4u w[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) {
            const int64_t t = t0 + k * stride;
            if (t < n16) w[k] = c16[t];
        }
#pragma unroll
        for (int k = 0; k < kIn; ++k) {
            const int64_t t = t0 + k * stride;
            if (t >= n16) break;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int64_t v = t * 16 + j;
                if (v >= n) break;
                int c = (int)((w[k][j >> 2] >> ((j & 3) * 8)) & 255u);
                if (c == 255) {
                    c = col[v];
                    if (c < 0 || c > maxdeg) { bad = true; continue; }
                    if (c >= 255) {
                        if (flags[c] == 0) flags[c] = 1;  // racy but idempotent
                        m = max(m, c);
                        continue;
                    }
                }
                if (c > maxdeg) { bad = true; continue; }
                m = max(m, c);
                if (c < 64) low |= 1ull << c;
                else lds_or(&bits[c >> 5], 1u << (c & 31));
            }
        }
    }
    if (ballot(bad) && lane_id() == 0) atomicOr(&S->err, 4);
    for (int off = 32; off > 0; off >>= 1) low |= __shfl_xor(low, off);
    if (lane_id() == 0 && low) {
        lds_or(&bits[0], (uint32_t)low);
        lds_or(&bits[1], (uint32_t)(low >> 32));
    }
    m = block_max(m, sh);
    __syncthreads();
    if (threadIdx.x < 8 && bits[threadIdx.x] &&
        (bits[threadIdx.x] & ~__hip_atomic_load(&S->cbits[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
        atomicOr(&S->cbits[threadIdx.x], bits[threadIdx.x]);
    if (threadIdx.x == 0 && m + 1 > __hip_atomic_load(&S->kmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&S->kmax, m + 1);
}

}  // namespace rsoc
