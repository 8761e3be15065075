// tail_kernels.hpp -- the optimistic mode's round once the worklist is small.
//
// On graphs whose hubs form a dense core (power-law graphs) the last
// defective vertices are mostly mutual neighbours.  Recoloured at the same
// time, they read one another's old colours, take the same smallest free
// colour, and each round settles only one or two of them.  Once the worklist
// L holds at most kTailMax vertices, one round is therefore run as an ordered
// pass: each entry of L is detected and, if defective, recoloured after the
// entries before it and sees their new colours.  That is one of the interleavings the
// optimistic round (Algorithm 3, Section 3) allows -- detection, then
// First-Fit over the colours as they stand -- so the round is unchanged in
// kind; it only cannot create a conflict inside L.  The recoloured vertices
// form the next worklist as usual, and the next round checks them.
//
//   k_tail_mark    numbers L: tv[i] = i-th entry, mark[v] = i + 1.
//   k_tail_prep    one workgroup per entry, all in parallel: splits the row.
//                  Neighbours in L are recorded by position (their colours may
//                  change during the pass); the colours of the others cannot,
//                  so they give the fixed part of the detection and, as at most
//                  dL neighbours are in L, the first dL + 1 colours they leave
//                  free, among which First-Fit's answer lies.
//   k_tail_seq     one workgroup walks L in the order the prep workgroups
//                  stored their lists, with the current colours of L in LDS.
//   k_tail_unmark  clears mark.
#pragma once

#include "single_kernels.hpp"

namespace rsoc {

constexpr int kTailMax = 1024;  // largest worklist given an ordered pass
constexpr int kTailData = kTailMax * (2 * kTailMax + 1);  // ints of packed per-entry lists

// Scratch of the ordered pass (one allocation, carved by tail_layout).  The
// prep workgroups claim walk slots and data offsets together (one 64-bit
// atomic), so the walk's order is the slots' and its lists lie contiguously
// in that order.
struct TailBuf {
    int32_t *tv;                // [kTailMax] entries of L (list order; a neighbour's "position")
    int4 *slot;                 // [kTailMax] per walk slot: {entry, dL, fixed-part defect, degree}
    int32_t *soff;              // [kTailMax] per walk slot: offset of its lists in data
    unsigned long long *alloc;  // (slots << 32) | ints claimed
    int32_t *data;              // [kTailData] per slot: dL positions, then dL + 1 free colours
};

inline size_t tail_bytes() {
    return sizeof(int32_t) * kTailMax + sizeof(int4) * kTailMax + sizeof(int32_t) * kTailMax + 256 +
           sizeof(int32_t) * (size_t)kTailData;
}

__host__ __device__ inline TailBuf tail_layout(void *base) {
    char *p = static_cast<char *>(base);
    TailBuf t;
    t.tv = reinterpret_cast<int32_t *>(p);
    p += sizeof(int32_t) * kTailMax;
    t.slot = reinterpret_cast<int4 *>(p);
    p += sizeof(int4) * kTailMax;
    t.soff = reinterpret_cast<int32_t *>(p);
    p += sizeof(int32_t) * kTailMax;
    t.alloc = reinterpret_cast<unsigned long long *>(p);
    p += 256;
    t.data = reinterpret_cast<int32_t *>(p);
    return t;
}

// The current worklist is buffer 0 (an even number of rounds has run since
// round 1 appended into it); its bins are concatenated in the order thread,
// wavefront, workgroup.
__global__ void k_tail_mark(const SingleArgs *__restrict__ A, const SingleState *__restrict__ S, TailBuf t,
                            int32_t *mark, int m) {
    const SingleArgs a = *A;
    const int c0 = S->cnt_in[kBinThread], c1 = S->cnt_in[kBinWave];
    if (blockIdx.x == 0 && threadIdx.x == 0) *t.alloc = 0ull;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const int pos = i < c0 ? i : (i < c0 + c1 ? a.offW + (i - c0) : a.offB + (i - c0 - c1));
        const int v = a.wl[0][pos];
        t.tv[i] = v;
        mark[v] = i + 1;
    }
}

template <int TIE>
__global__ __launch_bounds__(kBlock) void k_tail_prep(const SingleArgs *__restrict__ A, TailBuf t,
                                                      const int32_t *__restrict__ mark) {
    __shared__ uint32_t bm[kBlockWindowWords];
    __shared__ int nbrL[kTailMax], freL[kTailMax + 1];
    __shared__ int sh_dl, sh_got, sh_off;
    const SingleArgs a = *A;
    const RSOC_GLOBAL int32_t *rp = gro(a.rp);
    const RSOC_GLOBAL int32_t *ci = gro(a.ci);
    const RSOC_GLOBAL int32_t *col = gro(a.col);
    const int i = blockIdx.x;
    const int v = t.tv[i];
    const int b = rp[v], e = rp[v + 1];
    const int cv = col[v];
    if (threadIdx.x == 0) sh_dl = sh_got = 0;
    bool sdef = false;
    for (int base = 0;; base += kBlockWindowBits) {
        for (int w = threadIdx.x; w < kBlockWindowWords; w += kBlock) bm[w] = 0u;
        __syncthreads();
        // U entries per thread in flight; mark and colour are read together
        constexpr int U = 8;
        for (int j0 = b; j0 < e; j0 += kBlock * U) {
            int u[U], p[U], c[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int j = j0 + q * kBlock + (int)threadIdx.x;
                u[q] = j < e ? ci[j] : v;
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                p[q] = u[q] != v ? mark[u[q]] : 0;
                c[q] = u[q] != v ? col[u[q]] : -1;
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (u[q] == v) continue;
                if (p[q]) {
                    if (base == 0) {
                        const int k = atomicAdd(&sh_dl, 1);  // > m - 1 only with repeated row entries
                        if (k < kTailMax) nbrL[k] = p[q] - 1;
                    }
                    continue;
                }
                if (base == 0 && c[q] == cv && loses<TIE>(v, u[q])) sdef = true;
                if (c[q] >= base && c[q] < base + kBlockWindowBits)
                    lds_or(&bm[(c[q] - base) >> 5], 1u << ((c[q] - base) & 31));
            }
        }
        sdef = __syncthreads_or(sdef);
        // the free colours of this window, in order, until dL + 1 are known (a
        // neighbour in L missing from the list -- repeated row entries -- can
        // only cost a conflict that the next round finds)
        if (threadIdx.x == 0) {
            if (base == 0) sh_dl = min(sh_dl, kTailMax);
            const int need = sh_dl + 1;
            int got = sh_got;
            for (int w = 0; w < kBlockWindowWords && got < need; ++w) {
                uint32_t f = ~bm[w];
                while (f && got < need) {
                    freL[got++] = base + 32 * w + __builtin_ctz(f);
                    f &= f - 1;
                }
            }
            sh_got = got;
        }
        __syncthreads();
        if (sh_got >= sh_dl + 1) break;
    }
    const int dL = sh_dl;
    if (threadIdx.x == 0) {
        const unsigned long long got =
            atomicAdd(t.alloc, (1ull << 32) | (unsigned long long)(2 * dL + 1));
        const int slot = (int)(got >> 32), off = (int)(got & 0xffffffffull);
        t.slot[slot] = make_int4(i, dL, sdef ? 1 : 0, e - b);
        t.soff[slot] = off;
        sh_off = off;
    }
    __syncthreads();
    int32_t *out = t.data + sh_off;
    for (int k = threadIdx.x; k < dL; k += kBlock) out[k] = nbrL[k];
    for (int k = threadIdx.x; k <= dL; k += kBlock) out[dL + k] = freL[k];
}

// The walk itself runs from LDS only.  The slots' lists are staged chunk by
// chunk (at most kStage ints each) with flat loads of the packed data, the
// next chunk's loads issued before the current chunk is walked; the
// workgroup's threads are spread over each entry's lists (two workgroup
// barriers per slot, three when its vertex is recoloured).
constexpr int kStage = 8192;
constexpr int kSeen = 4096;  // colour range (above an entry's first free colour) stamped in LDS
constexpr int kStageQ = kStage / kBlock;

template <int TIE, bool NIB>
__global__ __launch_bounds__(kBlock) void k_tail_seq(const SingleArgs *__restrict__ A, SingleState *S, TailBuf t,
                                                     int m) {
    __shared__ int colL[kTailMax], tvL[kTailMax];
    __shared__ int4 slotL[kTailMax];
    __shared__ int offL[kTailMax];
    __shared__ int cb[kTailMax + 1];
    __shared__ int buf[2][kStage];
    __shared__ int seen[kSeen];
    __shared__ uint32_t used[(kTailMax + 1 + 31) / 32];
    __shared__ int degL[kTailMax];
    __shared__ unsigned char recl[kTailMax];
    __shared__ int cnt[3];
    __shared__ int sh_nc, sh_j;
    const SingleArgs a = *A;
    RSOC_GLOBAL int32_t *col = grw(a.col);
    RSOC_GLOBAL uint8_t *col8 = grw(a.col8);
    RSOC_GLOBAL uint32_t *col4 = grw(a.col4);
    const RSOC_GLOBAL int32_t *data = gro(t.data);
    const int tid = threadIdx.x, lane = lane_id();
    {
        constexpr int Q = kTailMax / kBlock;
        int v[Q], c[Q], o[Q];
        int4 sl[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = tid + q * kBlock;
            v[q] = i < m ? t.tv[i] : 0;
            sl[q] = i < m ? t.slot[i] : make_int4(0, 0, 0, 0);
            o[q] = i < m ? t.soff[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) c[q] = tid + q * kBlock < m ? col[v[q]] : 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = tid + q * kBlock;
            if (i < m) {
                tvL[i] = v[q];
                colL[i] = c[q];
                slotL[i] = sl[q];
                offL[i] = o[q];
                recl[i] = 0;
            }
        }
    }
    __syncthreads();
    for (int s = tid; s < m; s += kBlock) degL[slotL[s].x] = slotL[s].w;
    if (tid < 3) cnt[tid] = S->cnt_out[tid];
    for (int w = tid; w < kSeen; w += kBlock) seen[w] = 0;
    if (tid == 0) sh_j = INT_MAX;
    __syncthreads();
    // chunks of consecutive slots whose lists fit kStage ints
    if (tid == 0) {
        int nc = 0, s = 0;
        cb[0] = 0;
        while (s < m) {
            const int base = offL[s];
            while (s < m && offL[s] + 2 * slotL[s].y + 1 - base <= kStage) ++s;
            cb[++nc] = s;
        }
        sh_nc = nc;
    }
    __syncthreads();
    const int nchunks = sh_nc;
    auto chunk_base = [&](int ch) { return offL[cb[ch]]; };
    auto chunk_len = [&](int ch) {
        const int last = cb[ch + 1] - 1;
        return offL[last] + 2 * slotL[last].y + 1 - offL[cb[ch]];
    };
    int x[kStageQ];
    {
        const int b0 = chunk_base(0), l0 = chunk_len(0);
#pragma unroll
        for (int q = 0; q < kStageQ; ++q) {
            const int k = q * kBlock + tid;
            x[q] = k < l0 ? data[b0 + k] : 0;
        }
#pragma unroll
        for (int q = 0; q < kStageQ; ++q) buf[0][q * kBlock + tid] = x[q];
    }
    __syncthreads();
    for (int ch = 0; ch < nchunks; ++ch) {
        const bool more = ch + 1 < nchunks;
        if (more) {
            const int bn = chunk_base(ch + 1), ln = chunk_len(ch + 1);
#pragma unroll
            for (int q = 0; q < kStageQ; ++q) {
                const int k = q * kBlock + tid;
                x[q] = k < ln ? data[bn + k] : 0;
            }
        }
        const int *B = buf[ch & 1];
        const int base = chunk_base(ch);
        for (int s = cb[ch]; s < cb[ch + 1]; ++s) {
            const int4 mt = slotL[s];
            const int i = mt.x, dL = mt.y, v = tvL[i], cv = colL[i];
            const int *pos = B + (offL[s] - base);
            const int *F = pos + dL;
            const int F0 = F[0];
            const bool narrow = F[dL] - F0 < kSeen;
            // one pass over the neighbours in L: detection, and their colours
            // stamped s + 1 in seen (relative to F[0]; stamps of earlier slots
            // are simply other values)
            bool c = false;
            for (int k0 = 0; k0 < dL; k0 += 4 * kBlock) {
                int p[4], cc[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = k0 + q * kBlock + tid;
                    p[q] = k < dL ? pos[k] : -1;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) cc[q] = p[q] >= 0 ? colL[p[q]] : -1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (p[q] < 0) continue;
                    c |= cc[q] == cv && loses<TIE>(v, tvL[p[q]]);
                    const int d = cc[q] - F0;
                    if (narrow && d >= 0 && d < kSeen) seen[d] = s + 1;
                }
            }
            if (!__syncthreads_or(c) && !mt.z) continue;
            // First-Fit: the first of F[0, dL] that no neighbour in L holds
            // now (at most dL of the dL + 1 can be held)
            int j = INT_MAX;
            if (narrow) {
                for (int k = tid; k <= dL; k += kBlock)
                    if (seen[F[k] - F0] != s + 1) j = min(j, k);
            } else {
                // free colours spread wider than seen: bits past dL are set so
                // that they are never chosen, then a binary search per
                // neighbour marks the held ones
                const int nw = (dL + 1 + 31) / 32;
                for (int w = tid; w < nw; w += kBlock) {
                    const int lo = 32 * w;
                    used[w] = (dL + 1 - lo >= 32) ? 0u : ~((1u << (dL + 1 - lo)) - 1u);
                }
                __syncthreads();
                for (int k = tid; k < dL; k += kBlock) {
                    const int cc = colL[pos[k]];
                    int lo = 0, hi = dL + 1;  // lower bound of cc in the sorted F[0, dL]
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (F[mid] < cc) lo = mid + 1;
                        else hi = mid;
                    }
                    if (lo <= dL && F[lo] == cc) lds_or(&used[lo >> 5], 1u << (lo & 31));
                }
                __syncthreads();
                for (int w = tid; w < nw; w += kBlock)
                    if (used[w] != ~0u) j = min(j, 32 * w + __builtin_ctz(~used[w]));
            }
            for (int off = 32; off > 0; off >>= 1) j = min(j, __shfl_xor(j, off));
            if (lane == 0 && j != INT_MAX) atomicMin(&sh_j, j);
            __syncthreads();
            // the new colour stays in LDS until the walk ends: no global
            // store is in flight when the next barrier's fence waits
            if (tid == 0) {
                colL[i] = F[min(sh_j, dL)];  // sh_j <= dL always: dL + 1 candidates, at most dL held
                recl[i] = 1;
                sh_j = INT_MAX;
            }
            __syncthreads();
        }
        if (more) {
#pragma unroll
            for (int q = 0; q < kStageQ; ++q) buf[(ch + 1) & 1][q * kBlock + tid] = x[q];
        }
        __syncthreads();
    }
    // publish the recoloured vertices and append them to the next worklist
    for (int i = tid; i < m; i += kBlock) {
        if (!recl[i]) continue;
        const int v = tvL[i], nc = colL[i], deg = degL[i];
        col[v] = nc;
        col8[v] = shadow_of(nc);
        if (NIB) atomicOr((uint32_t *)&col4[v >> 3], 0xfu << ((v & 7) << 2));
        const int bin = deg <= a.t_thread ? kBinThread : (deg <= a.t_wave ? kBinWave : kBinBlock);
        const int off = bin == kBinThread ? 0 : (bin == kBinWave ? a.offW : a.offB);
        a.wl[0][off + atomicAdd(&cnt[bin], 1)] = v;
    }
    __syncthreads();
    if (tid < 3) S->cnt_out[tid] = cnt[tid];
    if (tid == 0) {
        S->inspected += (uint64_t)m;
        unsigned long long rec = 0;
        for (int i = 0; i < m; ++i) rec += recl[i];
        S->acc[kAccAppended] += rec;
    }
}

__global__ void k_tail_unmark(TailBuf t, int32_t *mark, int m) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) mark[t.tv[i]] = 0;
}

}  // namespace rsoc
