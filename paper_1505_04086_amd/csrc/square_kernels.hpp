// square_kernels.hpp -- the square G^2 of a graph, for distance-2 colouring
// (Section 6: d-distance colouring is the colouring of the power graph G^d;
// u and w are adjacent in G^2 iff they are within distance 2 in G).  Built
// once on the device; the distance-1 rounds then colour it unchanged.
//
// Row v of G^2 is N(v) together with N(u) for every u in N(v), without v and
// without repeats.  One wavefront per vertex walks that multiset (T(v) =
// deg(v) + sum of deg(u) entries) flattened: 64 neighbours u at a time, their
// row lengths scanned across the lanes, then 64 entries of the concatenated
// rows per step (four steps' loads in flight together), each lane finding its
// row by a binary search over the 64 offsets held by the lanes (shuffles).
// Repeats are dropped by an open-addressing hash set in the wavefront's LDS
// (at least twice T slots).  Two passes use the same walk: the
// first counts the distinct entries of each row, the second (after an
// exclusive scan of the counts) writes them, in hash-table order.
#pragma once

#include "device_common.hpp"

namespace rsoc {

constexpr int kSqSmallT = 1024;   // T(v) up to this: 2048-slot table, four wavefronts per workgroup
constexpr int kSqBigT = 8192;     // up to this: 16384-slot table, one wavefront per workgroup
constexpr int kSqSmallTab = 2 * kSqSmallT;
constexpr int kSqBigTab = 2 * kSqBigT;

// T(v) = deg(v) + sum over u in N(v) of deg(u), capped just above kSqBigT
// (counting stops there); err bit 0 when some T(v) exceeds kSqBigT.  Eight
// lanes per vertex gather the neighbours' degrees side by side.  Vertices with
// T(v) > kSqSmallT (few: near hubs) are listed in big[], *nbig of them.
__global__ __launch_bounds__(kBlock) void k_sq_size(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                    int32_t n, int32_t *T, int32_t *err, int32_t *big,
                                                    int32_t *nbig) {
    constexpr int G = 8;
    const int k = threadIdx.x & (G - 1);
    bool over = false;
    const int64_t ng = (int64_t)gridDim.x * (kBlock / G);
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G; v < n; v += ng) {
        const int b = rp[v], e = rp[v + 1];
        int64_t t = 0;
        for (int j = b + k; j < e && t <= kSqBigT; j += G) {
            const int u = ci[j];
            t += rp[u + 1] - rp[u];
        }
#pragma unroll
        for (int o = 1; o < G; o <<= 1) t += __shfl_xor(t, o);
        t += e - b;
        if (k == 0) {
            over |= t > kSqBigT;
            T[v] = (int32_t)min<int64_t>(t, kSqBigT + 1);
            if (t > kSqSmallT && t <= kSqBigT) big[atomicAdd(nbig, 1)] = (int32_t)v;
        }
    }
    if (ballot(over) && lane_id() == 0) atomicOr(err, 1);
}

__device__ __forceinline__ uint32_t sq_hash(int x) { return (uint32_t)x * 2654435761u; }

// Inserts x into the wavefront's table (size a power of two); true when x
// was not there yet.  Lanes insert concurrently: a plain read settles the
// common case (x already there, most 2-hop entries being repeats); an empty
// slot is claimed with an LDS compare-and-swap.
__device__ __forceinline__ bool sq_insert(int32_t *tab, int mask, int shift, int x) {
    uint32_t h = sq_hash(x) >> shift;
    for (;;) {
        const int cur = tab[h];
        if (cur == x) return false;
        if (cur == -1) {
            const int prev = atomicCAS(&tab[h], -1, x);
            if (prev == -1) return true;
            if (prev == x) return false;
        }
        h = (h + 1) & mask;
    }
}

// One wavefront per vertex with lo < T(v) <= hi, WPB wavefronts per
// workgroup, TAB table slots per wavefront.  FILL = false: cnt[v] = distinct
// entries of row v of G^2; FILL = true: writes them at out[start[v] ...).
template <int WPB, int TAB, bool FILL>
__global__ __launch_bounds__(WPB *kWave) void k_sq_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                       int32_t n, const int32_t *__restrict__ T, int lo, int hi,
                                                       const int32_t *list, const int32_t *nlist, int32_t *cnt,
                                                       const int32_t *__restrict__ start, int32_t *out) {
    __shared__ int32_t tabs[WPB][TAB];
    const int wv = threadIdx.x / kWave, lane = lane_id();
    int32_t *tab = tabs[wv];
    const RSOC_GLOBAL int32_t *rpg = gro(rp);
    const RSOC_GLOBAL int32_t *cig = gro(ci);
    const int64_t nw = (int64_t)gridDim.x * WPB;
    // all vertices, or the listed ones
    const int64_t items = list ? *nlist : n;
    for (int64_t v0 = (int64_t)blockIdx.x * WPB + wv; v0 < items; v0 += nw) {
        const int v = list ? list[v0] : (int)v0;
        const int t = T[v];
        if (t <= lo || t > hi) continue;  // the same for every lane of the wavefront
        // table of at least 2T slots (a power of two, at most TAB): at most
        // half full, so every probe sequence ends
        int size = kWave;
        while (size < 2 * t && size < TAB) size <<= 1;
        const int mask = size - 1;
        const int shift = 32 - __builtin_ctz((unsigned)size);
        for (int i = lane; i < size; i += kWave) tab[i] = -1;
        wave_lds_sync();
        int fresh = 0;
        const int b = rpg[v], e = rpg[v + 1];
        for (int j0 = b; j0 < e; j0 += kWave) {
            // 64 neighbours: each lane's u, its row start and length, and the
            // exclusive scan of the lengths across the lanes
            const int j = j0 + lane;
            const int u = j < e ? cig[j] : -1;
            const int rb = u >= 0 ? rpg[u] : 0;
            const int len = u >= 0 ? rpg[u + 1] - rb : 0;
            if (u >= 0 && u != v) fresh += sq_insert(tab, mask, shift, u);
            int incl = len;
            for (int o = 1; o < kWave; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            const int excl = incl - len;
            const int total = __shfl(incl, kWave - 1);
            constexpr int kIn = 4;  // steps of 64 entries whose loads are in flight together
            for (int t0 = 0; t0 < total; t0 += kIn * kWave) {
                int w[kIn];
#pragma unroll
                for (int r = 0; r < kIn; ++r) {
                    const int q = t0 + r * kWave + lane;
                    // the neighbour whose row holds entry q of the
                    // concatenation: the last lane k with excl(k) <= q (every
                    // lane takes part in the shuffles)
                    int k = 0;
#pragma unroll
                    for (int step = kWave / 2; step > 0; step >>= 1) {
                        const int cand = __shfl(excl, k + step);
                        if (cand <= q) k += step;
                    }
                    const int rbk = __shfl(rb, k), ek = __shfl(excl, k);
                    w[r] = q < total ? cig[rbk + (q - ek)] : v;
                }
#pragma unroll
                for (int r = 0; r < kIn; ++r)
                    if (w[r] != v) fresh += sq_insert(tab, mask, shift, w[r]);
            }
        }
        wave_lds_sync();
        if (!FILL) {
            for (int o = 32; o > 0; o >>= 1) fresh += __shfl_xor(fresh, o);
            if (lane == 0) cnt[v] = fresh;
        } else {
            int at = start[v];
            RSOC_GLOBAL int32_t *og = grw(out);
            for (int i0 = 0; i0 < size; i0 += kWave) {
                const int x = tab[i0 + lane];
                const uint64_t m = ballot(x >= 0);
                if (x >= 0) og[at + __popcll(m & ((1ull << lane) - 1))] = x;
                at += __popcll(m);
            }
        }
        wave_lds_sync();  // the table is cleared for the next vertex
    }
}

// Sum of the row counts, 64-bit (one atomic per workgroup).
__global__ __launch_bounds__(kBlock) void k_sq_total(const int32_t *__restrict__ cnt, int32_t n,
                                                     unsigned long long *total) {
    __shared__ unsigned long long sh[kWavesPerBlock];
    unsigned long long s = 0;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
        s += (unsigned long long)cnt[v];
    s = wave_sum_u64(s);
    if (lane_id() == 0) sh[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) t += sh[w];
        if (t) atomicAdd(total, t);
    }
}

// row_ptr of G^2 from the scanned counts: rp2[n] = the total.
__global__ void k_sq_tail(int32_t *rp2, int32_t n, const unsigned long long *total) {
    if (threadIdx.x == 0) rp2[n] = (int32_t)*total;
}

}  // namespace rsoc
