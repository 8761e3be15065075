// hub_kernels.hpp -- hub-first round 0 of the optimistic mode.
//
// Round 0 of Algorithm 3 (Section 3) colours every vertex once, in parallel,
// each from the colours its neighbours hold at that moment; the optimistic
// mode may interleave those First-Fit steps in any order.  On power-law
// graphs the order matters for the colour count: a hub coloured while its
// neighbours are still uncoloured gets a small colour, collides, and is then
// recoloured against all of its (by then coloured) neighbours, whose colours
// were chosen without regard to it -- hundreds of colours beyond sequential
// First-Fit on R-MAT graphs.  Sequential First-Fit (Section 2.1, Algorithm 1)
// avoids that because a hub's later neighbours see its colour.
//
// This interleaving therefore runs the hubs' First-Fit steps first, one hub
// after another in tie order (ascending id when the lower id keeps its
// colour), each over the hubs coloured before it -- the only coloured
// neighbours at that point -- so the hubs end up with the sequential
// First-Fit colouring of the subgraph they induce, without a conflict among
// them.  Round 0 then colours every other vertex reading all of its
// neighbours (not only the ones it loses to), so none takes a hub's colour,
// and no hub ever needs recolouring: later rounds recolour against all
// neighbours, hubs included.
//
// k_args (after binning) collects the hubs: the vertices above the threshold
// (by default max(32, max degree / 32)), at most kHubCap, else the pass is
// skipped.  Two launches follow: k_hub_lists sorts them by id and builds, for
// each hub, the bit set of the hubs it loses to, by position in tie order
// (one workgroup per hub, a binary search of the sorted hub ids in LDS for
// each neighbour); k_hub_ff walks the hubs in tie order in one workgroup with
// their colours and a block of bit sets in LDS, two barriers per hub, and
// writes the colours (and both shadows) once the walk is done.
#pragma once

#include "single_kernels.hpp"

namespace rsoc {

constexpr int kHubWords = kHubCap / 32;  // words of a hub's bit set of the hubs it loses to, at most
constexpr int kHubFfBlock = 512;
constexpr int kHubBufWords = 4096;       // LDS words for a block of consecutive hubs' bit sets
constexpr int kHubListGrid = 1024;

// Scratch of the hub tables (ctx buffer `hubs`): hubC, hubS (kHubCap each)
// and the chunk prefix (kHubCap + 1, padded), then one bit set of
// W = ceil(nH / 32) words per hub, in tie order.
constexpr size_t kHubTablesInts = 3 * kHubCap + 64;
constexpr size_t kHubTablesBytes = sizeof(int32_t) * kHubTablesInts;
constexpr size_t kHubBytes = kHubTablesBytes + sizeof(uint32_t) * (size_t)kHubCap * kHubWords;

// Sorts ids[0, m) ascending in LDS (bitonic, padded to a power of two with
// INT_MAX; ids must hold that many entries).  Every thread of the workgroup
// calls it.
__device__ __forceinline__ void lds_sort_ids(int *ids, int m) {
    int P = 1;
    while (P < m) P <<= 1;
    for (int i = m + (int)threadIdx.x; i < P; i += blockDim.x) ids[i] = INT_MAX;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const int x = ids[i], y = ids[l];
                    if ((x > y) == ((i & k) == 0)) {
                        ids[i] = y;
                        ids[l] = x;
                    }
                }
            }
            __syncthreads();
        }
}

// Position of hub id u among the sorted ids[0, m), or -1.
__device__ __forceinline__ int hub_find(const int *ids, int m, int u) {
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ids[mid] < u) lo = mid + 1;
        else hi = mid;
    }
    return (lo < m && ids[lo] == u) ? lo : -1;
}

// The hubs sorted by id (hubS) and their number (S->nH, which turns the pass
// on), each hub's sorted position in pos[] (the context's staging array,
// unused by the optimistic mode; only the hubs' entries are written), and the
// scanned numbers of kHubChunk-entry chunks of their rows (hub_cpre: chunk k
// of all the hubs' rows is chunk k - cpre[p] of the hub at sorted position
// p, cpre[p] <= k < cpre[p + 1]).  One workgroup.
constexpr int kHubChunk = 4096;
constexpr int kHubSortBlock = 1024;
__global__ __launch_bounds__(kHubSortBlock) void k_hub_sort(const SingleArgs *__restrict__ A, SingleState *S) {
    __shared__ int ids[kHubCap];
    __shared__ int part[kHubSortBlock];
    const int nH = S->nHc;
    if (nH == 0 || nH > kHubCap) return;
    const SingleArgs a = *A;
    const int t = threadIdx.x;
    for (int i = t; i < nH; i += kHubSortBlock) ids[i] = a.hubC[i];
    lds_sort_ids(ids, nH);
    const RSOC_GLOBAL int32_t *rp = gro(a.rp);
    constexpr int kPer = kHubCap / kHubSortBlock;
    int cnt[kPer], sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int i = t * kPer + k;
        cnt[k] = 0;
        if (i < nH) {
            const int h = ids[i];
            a.hubS[i] = h;
            a.pend[h] = i;
            cnt[k] = (rp[h + 1] - rp[h] + kHubChunk - 1) / kHubChunk;
        }
        sum += cnt[k];
    }
    // exclusive scan of the per-thread sums (wavefronts, then across them)
    int incl = sum;
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(incl, off);
        if (lane_id() >= off) incl += y;
    }
    if (lane_id() == kWave - 1) part[t / kWave] = incl;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < t / kWave; ++w) base += part[w];
    int run = base + incl - sum;
    if (t == 0) a.hub_cpre[0] = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        run += cnt[k];
        a.hub_cpre[t * kPer + k + 1] = run;
    }
    if (t == 0) S->nH = nH;
}

// The bit set of the hubs each hub loses to, by position in tie order, at
// hub_bits + i * W (W = ceil(nH / 32) words) for the hub at tie-order
// position i.  The hubs' rows are cut into chunks of kHubChunk entries, taken
// by the workgroups in turn: a chunk's neighbours that are hubs the row's hub
// loses to are marked in an LDS bit set (duplicate entries collapse), whose
// non-zero words are then ORed into the global bit set (the words are zero
// on entry: k_hub_ff clears what it reads).  A neighbour u is recognised as
// the hub at sorted position q by pos[u] == q and hubS[q] == u: pos holds
// anything at all outside the hubs' entries, and the second test rejects it.
template <int TIE>
__global__ __launch_bounds__(kBlock) void k_hub_lists(const SingleArgs *__restrict__ A, SingleState *S) {
    __shared__ int ids[kHubCap];
    __shared__ int cpre[kHubCap + 1];
    __shared__ uint32_t mark[kHubWords];
    const int nH = S->nH;
    if (nH == 0) return;
    const SingleArgs a = *A;
    const int t = threadIdx.x;
    const int ntask = a.hub_cpre[nH];
    if ((int)blockIdx.x >= ntask) return;
    for (int i = t; i < nH; i += kBlock) ids[i] = a.hubS[i];
    for (int i = t; i <= nH; i += kBlock) cpre[i] = a.hub_cpre[i];
    __syncthreads();
    const RSOC_GLOBAL int32_t *rp = gro(a.rp);
    const RSOC_GLOBAL int32_t *ci = gro(a.ci);
    const RSOC_GLOBAL int32_t *pos = gro(a.pend);
    const int W = (nH + 31) / 32;
    constexpr int U = kHubChunk / kBlock;  // entries per thread and chunk
    for (int task = blockIdx.x; task < ntask; task += gridDim.x) {
        int lo = 0, hi = nH;  // the last p with cpre[p] <= task
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cpre[mid] <= task) lo = mid;
            else hi = mid;
        }
        const int p = lo;
        const int h = ids[p];
        const int b = rp[h] + (task - cpre[p]) * kHubChunk, e = min(rp[h + 1], b + kHubChunk);
        for (int w = t; w < W; w += kBlock) mark[w] = 0;
        __syncthreads();
        int u[U], q[U];
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const int j = b + s * kBlock + t;
            u[s] = j < e ? __builtin_nontemporal_load(ci + j) : h;
        }
#pragma unroll
        for (int s = 0; s < U; ++s) q[s] = (u[s] != h && loses<TIE>(h, u[s])) ? pos[u[s]] : -1;
#pragma unroll
        for (int s = 0; s < U; ++s) {
            if ((unsigned)q[s] >= (unsigned)nH || ids[q[s]] != u[s]) continue;
            const int k = TIE == kLowerKeeps ? q[s] : nH - 1 - q[s];
            lds_or(&mark[k >> 5], 1u << (k & 31));
        }
        __syncthreads();
        const int i = TIE == kLowerKeeps ? p : nH - 1 - p;
        uint32_t *out = a.hub_bits + (size_t)i * W;
        for (int w = t; w < W; w += kBlock)
            if (mark[w]) atomicOr(&out[w], mark[w]);
        __syncthreads();  // mark is reused by the next chunk
    }
}

// The walk over the hubs in tie order (one workgroup), then the colours out.
// The bit sets of a block of consecutive hubs are copied into LDS at once (one
// memory round trip per block); a hub then costs LDS work and two barriers.
// Each thread keeps the colours of its 8 hub positions in registers (set as
// the walk settles them), and the smallest-colour search reads only colours
// up to one above the largest given so far.
// Its forbidden colours (those of the hubs it loses to; each thread takes 8
// bits of one word of its bit set) are marked in an LDS array by writing the
// hub's stamp (position + 1) at each colour -- plain writes, so the many
// threads that mark the same colour of a dense core need no atomics and
// nothing is ever cleared; the smallest unmarked colour is then found per
// wavefront (a ballot over 8 colours per lane) and across the wavefronts.
// The inner step has no branches: a thread reads its 8 colours whatever its
// bits, and the write of an unset bit goes to a spare word of its own (1.6
// times faster than the branching form on R-MAT scale 22).  Measured and not
// kept: one wavefront walking alone without barriers (its LDS reads then wait
// on one another), one barrier per hub (the marks of hub k + 1 made while hub
// k's colour is found), reading the next hub's colours ahead, one barrier per
// hub with two mark arrays alternating and every wavefront finding the
// smallest colour by itself (R-MAT scale 22: 1.23 ms against 1.0 ms; 1.43 ms
// with the wavefronts that hold no bit-set word skipping the search): each
// slower.
constexpr int kHubFfWaves = kHubFfBlock / kWave;
constexpr int kHubColPerThread = kHubCap / kHubFfBlock;  // colours each thread examines (8)
// done (pool admissions only, else null): receives the hub count and
// threshold, and S's counts go back to zero for the next use of S.
template <int TIE>
__global__ __launch_bounds__(kHubFfBlock) void k_hub_ff(const SingleArgs *__restrict__ A, SingleState *S,
                                                        int32_t *done = nullptr) {
    __shared__ uint16_t hc[kHubCap];
    __shared__ uint32_t bits[kHubBufWords];
    __shared__ int mark[kHubCap + kWave];     // mark[c] == i + 1: colour c is forbidden for hub i
                                              // (the last kWave words take the writes of unset bits)
    __shared__ int wmin[2][kHubFfWaves];      // per-wavefront smallest unmarked colour, by step parity
    const int nH = S->nH;
    if (done && threadIdx.x == 0) {
        done[0] = nH;
        done[1] = S->hub_t;
    }
    if (nH == 0) {
        if (done && threadIdx.x == 0) S->nHc = S->hub_t = 0;
        return;
    }
    const SingleArgs a = *A;
    const int t = threadIdx.x;
    const int W = (nH + 31) / 32;
    const int B = kHubBufWords / W;  // hubs per block (at least 32)
    for (int c = t; c < kHubCap + kWave; c += kHubFfBlock) mark[c] = 0;
    const RSOC_GLOBAL uint32_t *gb = gro(a.hub_bits);
    const int word = t >> 2, sub = (t & 3) * 8;  // this thread's 8 bits of a bit set
    const int wv = t / kWave;
    // the colours of this thread's 8 hub positions, kept in registers as the
    // walk settles them (a position's bit is set only for hubs after it)
    int own[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) own[b] = 0;
    int maxc = -1;                               // largest colour given so far
    for (int i0 = 0; i0 < nH; i0 += B) {
        const int nb = min(B, nH - i0);
        constexpr int kLoads = kHubBufWords / kHubFfBlock;
        uint32_t r[kLoads];
#pragma unroll
        for (int k = 0; k < kLoads; ++k) {
            const int w = k * kHubFfBlock + t;
            r[k] = w < nb * W ? gb[(size_t)i0 * W + w] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kLoads; ++k) bits[k * kHubFfBlock + t] = r[k];
        // the words go back to zero for the next call's k_hub_lists
#pragma unroll
        for (int k = 0; k < kLoads; ++k) {
            const int w = k * kHubFfBlock + t;
            if (w < nb * W && r[k]) a.hub_bits[(size_t)i0 * W + w] = 0u;
        }
        __syncthreads();
        for (int h = 0; h < nb; ++h) {
            const int i = i0 + h;
            const int stamp = i + 1;
            // branch-free: the 8 colours are read whatever the bits, and an
            // unset bit's write goes to the lane's own spare word
            if (word < W) {
                const uint32_t byte = (bits[h * W + word] >> sub) & 0xffu;
#pragma unroll
                for (int b = 0; b < 8; ++b) mark[((byte >> b) & 1u) ? own[b] : kHubCap + lane_id()] = stamp;
            }
            __syncthreads();
            // the smallest colour not marked for hub i: hub i loses to at most
            // i hubs and every colour given so far is at most maxc, so it is at
            // most min(i, maxc + 1); thread t looks at colours 8t .. 8t + 7
            const int c0 = t * kHubColPerThread;
            int first = INT_MAX;
            if (c0 <= min(i, maxc + 1)) {
                int m8[kHubColPerThread];
#pragma unroll
                for (int k = 0; k < kHubColPerThread; ++k) m8[k] = mark[c0 + k];
#pragma unroll
                for (int k = kHubColPerThread - 1; k >= 0; --k) first = m8[k] != stamp ? c0 + k : first;
            }
            // the lowest lane with an unmarked colour holds the wavefront's smallest
            const uint64_t found = ballot(first != INT_MAX);
            const int lf = __shfl(first, found ? __ffsll((unsigned long long)found) - 1 : 0);
            if (lane_id() == 0) wmin[i & 1][wv] = found ? lf : INT_MAX;
            __syncthreads();
            int cc = INT_MAX;
#pragma unroll
            for (int w = 0; w < kHubFfWaves; ++w) cc = min(cc, wmin[i & 1][w]);
            if (t == 0) hc[i] = (uint16_t)cc;
            maxc = max(maxc, cc);
#pragma unroll
            for (int b = 0; b < 8; ++b) own[b] = (word * 32 + sub + b == i) ? cc : own[b];
        }
        // the last hub's barriers also end every read of `bits` of this block
    }
    __syncthreads();
    RSOC_GLOBAL int32_t *col = grw(a.col);
    RSOC_GLOBAL uint8_t *col8 = grw(a.col8);
    RSOC_GLOBAL uint32_t *col4 = grw(a.col4);
    for (int i = t; i < nH; i += kHubFfBlock) {
        const int h = a.hubS[TIE == kLowerKeeps ? i : nH - 1 - i];
        const int c = hc[i];
        col[h] = c;
        col8[h] = shadow_of(c);
        publish_nibble(col4, h, c);
    }
    if (done && t == 0) S->nH = S->nHc = S->hub_t = 0;
}

}  // namespace rsoc
