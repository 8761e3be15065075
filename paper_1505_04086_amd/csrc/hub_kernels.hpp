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
// each hub, the list of hubs it loses to, as positions in tie order (one
// workgroup per hub, a binary search of the sorted hub ids in LDS for each
// neighbour); k_hub_ff walks the hubs in tie
// order in one workgroup with their colours in LDS, two barriers per hub,
// the lists of the next hubs loaded while the current one is settled, and
// writes the colours (and both shadows) once the walk is done.
#pragma once

#include "single_kernels.hpp"

namespace rsoc {

constexpr int64_t kHubEntCap = (int64_t)kHubCap * (kHubCap - 1) / 2;  // list entries, at most
constexpr int kHubFfBlock = 512;
constexpr int kHubFfSlots = kHubCap / kHubFfBlock;  // list entries per thread: any list fits
constexpr int kHubListGrid = 1024;

// Scratch of the hub lists and tables (ctx buffer `hubs`): hubC, hubS,
// hub_ls, hub_ll (kHubCap each), then the list entries.
constexpr size_t kHubTablesBytes = sizeof(int32_t) * 4 * kHubCap;
constexpr size_t kHubBytes = kHubTablesBytes + sizeof(uint16_t) * (size_t)kHubEntCap;

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

// For each hub (grid-stride), the hubs it loses to, as positions in tie
// order, marked in an LDS bit set (duplicate row entries collapse) and
// written out in ascending order: hub_ls[i] / hub_ll[i] = start and length of
// the list of the hub at tie-order position i.
// Every workgroup first sorts the hubs by id itself (the same order in each;
// at most kHubCap ids, a few microseconds), workgroup 0 publishes the sorted
// list and their number (S->nH, which turns the pass on).
template <int TIE>
__global__ __launch_bounds__(kBlock) void k_hub_lists(const SingleArgs *__restrict__ A, SingleState *S) {
    __shared__ int ids[kHubCap];
    __shared__ uint32_t mark[kHubCap / 32];
    __shared__ int wsum[kHubCap / 32];
    __shared__ int base;
    const int nH = S->nHc;
    if (nH == 0 || nH > kHubCap || (int)blockIdx.x >= nH) return;
    const SingleArgs a = *A;
    const int t = threadIdx.x;
    for (int i = t; i < nH; i += kBlock) ids[i] = a.hubC[i];
    lds_sort_ids(ids, nH);
    if (blockIdx.x == 0) {
        for (int i = t; i < nH; i += kBlock) a.hubS[i] = ids[i];
        if (t == 0) S->nH = nH;
    }
    const RSOC_GLOBAL int32_t *rp = gro(a.rp);
    const RSOC_GLOBAL int32_t *ci = gro(a.ci);
    constexpr int kW = kHubCap / 32;
    constexpr int U = 4;
    for (int p = blockIdx.x; p < nH; p += gridDim.x) {
        for (int w = t; w < kW; w += kBlock) mark[w] = 0;
        __syncthreads();
        const int h = ids[p];
        const int b = rp[h], e = rp[h + 1];
        for (int j0 = b; j0 < e; j0 += kBlock * U) {
            int u[U];
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const int j = j0 + s * kBlock + t;
                u[s] = j < e ? __builtin_nontemporal_load(ci + j) : h;
            }
#pragma unroll
            for (int s = 0; s < U; ++s) {
                if (u[s] == h || !loses<TIE>(h, u[s])) continue;
                const int q = hub_find(ids, nH, u[s]);
                if (q < 0) continue;
                const int k = TIE == kLowerKeeps ? q : nH - 1 - q;
                lds_or(&mark[k >> 5], 1u << (k & 31));
            }
        }
        __syncthreads();
        // exclusive scan of the per-word counts (one wavefront, lane t holding
        // words 2t and 2t + 1 of the kW = 128)
        static_assert(kW == 2 * kWave, "two mark words per lane");
        if (t < kWave) {
            const int c0 = __popc(mark[2 * t]), c1 = __popc(mark[2 * t + 1]);
            int incl = c0 + c1;
            for (int off = 1; off < kWave; off <<= 1) {
                const int y = __shfl_up(incl, off);
                if (lane_id() >= off) incl += y;
            }
            wsum[2 * t] = incl - c0 - c1;
            wsum[2 * t + 1] = incl - c1;
            if (t == kWave - 1) base = incl ? atomicAdd(&S->hub_ecnt, incl) : 0;
            if (t == kWave - 1) {
                const int i = TIE == kLowerKeeps ? p : nH - 1 - p;
                a.hub_ls[i] = base;
                a.hub_ll[i] = incl;
            }
        }
        __syncthreads();
        RSOC_GLOBAL uint16_t *le = grw(a.hub_le) + base;
        for (int w = t; w < kW; w += kBlock) {
            uint32_t m = mark[w];
            int o = wsum[w];
            while (m) {
                le[o++] = (uint16_t)(w * 32 + __builtin_ctz(m));
                m &= m - 1;
            }
        }
        __syncthreads();  // mark, wsum and base are reused by the next hub
    }
}

// Loads the list of the hub at tie-order position i (-1 past its end).
__device__ __forceinline__ void hub_load_list(const RSOC_GLOBAL uint16_t *le, const int *ls, const int *ll, int i,
                                              int nH, int (&r)[kHubFfSlots]) {
    const int len = i < nH ? ll[i] : 0;
    const int st = i < nH ? ls[i] : 0;
#pragma unroll
    for (int s = 0; s < kHubFfSlots; ++s) {
        const int k = s * kHubFfBlock + (int)threadIdx.x;
        r[s] = k < len ? (int)le[st + k] : -1;
    }
}

// One hub of the walk: its First-Fit colour over the hubs of its list r,
// then r is refilled with the list of the hub four positions on.
__device__ __forceinline__ void hub_ff_step(int i, int nH, int (&r)[kHubFfSlots], int &prev, uint16_t *hc,
                                            uint32_t *bm, int *mx, const RSOC_GLOBAL uint16_t *le, const int *ls,
                                            const int *ll) {
    const int t = threadIdx.x;
#pragma unroll
    for (int s = 0; s < kHubFfSlots; ++s) {
        const int j = r[s];
        if (j >= 0) {
            // hub i - 1 was settled in the previous step: its colour is in
            // every thread's register, not yet behind a barrier in LDS
            const int c = (j == i - 1) ? prev : (int)hc[j];
            lds_or(&bm[c >> 5], 1u << (c & 31));
        }
    }
    hub_load_list(le, ls, ll, i + 4, nH, r);
    __syncthreads();
    // every set bit is a colour of an earlier hub (below i), and the list has
    // at most i entries, so the smallest clear bit lies in words 0 .. i/32;
    // each of those words is examined and cleared by its own thread
    if (t <= (i >> 5)) {
        const uint32_t w = bm[t];
        if (w != 0xffffffffu) atomicMin(&mx[i & 1], t * 32 + __builtin_ctz(~w));
        bm[t] = 0;
    }
    if (t == 0) mx[(i + 1) & 1] = INT_MAX;  // read by every thread before this step's first barrier
    __syncthreads();
    const int c = mx[i & 1];
    if (t == 0) hc[i] = (uint16_t)c;
    prev = c;
}

// The walk over the hubs in tie order (one workgroup), then the colours out.
template <int TIE>
__global__ __launch_bounds__(kHubFfBlock) void k_hub_ff(const SingleArgs *__restrict__ A, SingleState *S) {
    __shared__ uint16_t hc[kHubCap];
    __shared__ int ls[kHubCap], ll[kHubCap];
    __shared__ uint32_t bm[kHubCap / 32];
    __shared__ int mx[2];
    const int nH = S->nH;
    if (nH == 0) return;
    const SingleArgs a = *A;
    const int t = threadIdx.x;
    for (int i = t; i < nH; i += kHubFfBlock) {
        ls[i] = a.hub_ls[i];
        ll[i] = a.hub_ll[i];
    }
    for (int w = t; w < kHubCap / 32; w += kHubFfBlock) bm[w] = 0;
    if (t == 0) mx[0] = INT_MAX;
    __syncthreads();
    const RSOC_GLOBAL uint16_t *le = gro(a.hub_le);
    int r0[kHubFfSlots], r1[kHubFfSlots], r2[kHubFfSlots], r3[kHubFfSlots];
    hub_load_list(le, ls, ll, 0, nH, r0);
    hub_load_list(le, ls, ll, 1, nH, r1);
    hub_load_list(le, ls, ll, 2, nH, r2);
    hub_load_list(le, ls, ll, 3, nH, r3);
    int prev = -1;
    for (int i = 0; i < nH; i += 4) {
        hub_ff_step(i, nH, r0, prev, hc, bm, mx, le, ls, ll);
        if (i + 1 < nH) hub_ff_step(i + 1, nH, r1, prev, hc, bm, mx, le, ls, ll);
        if (i + 2 < nH) hub_ff_step(i + 2, nH, r2, prev, hc, bm, mx, le, ls, ll);
        if (i + 3 < nH) hub_ff_step(i + 3, nH, r3, prev, hc, bm, mx, le, ls, ll);
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
}

}  // namespace rsoc
