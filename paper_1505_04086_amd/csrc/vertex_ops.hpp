// vertex_ops.hpp -- the per-vertex work of a colouring round, in three shapes
// chosen by degree: one thread, one wavefront, or one workgroup per vertex.
//
// Every shape computes, for vertex v with row [b, e) of col_idx:
//   * detection (Algorithm 3's test, Section 3): does a neighbour u != v that
//     v loses to (by the tie rule) hold v's colour?
//   * First-Fit (Algorithm 1, Section 2.1): the smallest colour absent among
//     all neighbours u != v.  Colours < 0 (uncoloured) are ignored.  Since v
//     has at most e-b neighbours, the answer is at most e-b, so a window of
//     colours [base, base+W) with W > e-b always contains it.
// Phase kAssign computes First-Fit only; kRecolor detects and, if defective,
// computes First-Fit; kDetect only detects.
#pragma once

#include <limits.h>

#include "device_common.hpp"

namespace rsoc {

// ---------------------------------------------------------------- thread --
// Rows of at most 63 neighbours: the forbidden set of colours 0..63 is one
// 64-bit register mask and the answer is its lowest clear bit.
template <int PHASE, int TIE>
__device__ __forceinline__ bool thread_vertex(int v, int b, int e, const int32_t *__restrict__ ci,
                                              const int32_t *col, int &newc) {
    const int cv = (PHASE == kAssign) ? -1 : col[v];
    uint64_t mask = 0;
    bool conflict = false;
    for (int j = b; j < e; ++j) {
        const int u = __builtin_nontemporal_load(ci + j);
        if (u == v) continue;
        const int cu = col[u];
        if (PHASE != kAssign) conflict |= (cu == cv) && loses<TIE>(v, u);
        if (PHASE != kDetect) mask |= ((unsigned)cu < 64u) ? (1ull << cu) : 0ull;
    }
    newc = (int)__builtin_ctzll(~mask);
    return PHASE == kAssign ? true : conflict;
}

// -------------------------------------------------------------- wavefront --
// One wavefront per vertex: lanes stride the row (coalesced), the conflict
// flag is a ballot, and the forbidden colours go into a per-wavefront LDS
// bitmap window of kWaveWindowBits bits, scanned for its first clear bit with
// ballots.  Returns the same value in every lane; newc valid in every lane.
template <int PHASE, int TIE>
__device__ __forceinline__ bool wave_vertex(int v, int b, int e, const int32_t *__restrict__ ci, const int32_t *col,
                                            uint32_t *bm, int &newc) {
    const int lane = lane_id();
    if (PHASE != kAssign) {
        const int cv = col[v];
        bool any = false;
        for (int j0 = b; j0 < e; j0 += kWave) {
            const int j = j0 + lane;
            bool c = false;
            if (j < e) {
                const int u = ci[j];
                c = (u != v) && loses<TIE>(v, u) && (col[u] == cv);
            }
            if (ballot(c)) { any = true; break; }
        }
        if (!any) return false;
        if (PHASE == kDetect) return true;
    }
    for (int base = 0;; base += kWaveWindowBits) {
        for (int w = lane; w < kWaveWindowWords; w += kWave) bm[w] = 0u;
        wave_lds_sync();
        for (int j = b + lane; j < e; j += kWave) {
            const int u = ci[j];
            if (u == v) continue;
            const int rel = col[u] - base;
            if ((unsigned)rel < (unsigned)kWaveWindowBits) lds_or(&bm[rel >> 5], 1u << (rel & 31));
        }
        wave_lds_sync();
        for (int w0 = 0; w0 < kWaveWindowWords; w0 += kWave) {
            const uint32_t word = bm[w0 + lane];
            const uint64_t m = ballot(word != 0xffffffffu);
            if (m) {
                const int l = __ffsll((unsigned long long)m) - 1;
                const uint32_t wl = __shfl(word, l);
                newc = base + (w0 + l) * 32 + __builtin_ctz(~wl);
                wave_lds_sync();
                return true;
            }
        }
        wave_lds_sync();
    }
}

// -------------------------------------------------------------- workgroup --
// One workgroup per vertex (hubs): threads stride the row, the conflict flag
// is a workgroup OR, forbidden colours go into an LDS bitmap window of
// kBlockWindowBits bits; the first clear word is found with an LDS atomicMin.
// Must be called by the whole workgroup; newc valid in every thread.
template <int PHASE, int TIE>
__device__ __forceinline__ bool block_vertex(int v, int b, int e, const int32_t *__restrict__ ci, const int32_t *col,
                                             uint32_t *bm, int *sh_min, int &newc) {
    const int t = threadIdx.x;
    if (PHASE != kAssign) {
        const int cv = col[v];
        int any = 0;
        for (int j0 = b; j0 < e; j0 += kBlock * 8) {
            bool c = false;
            const int j1 = min(e, j0 + kBlock * 8);
            for (int j = j0 + t; j < j1; j += kBlock) {
                const int u = ci[j];
                c |= (u != v) && loses<TIE>(v, u) && (col[u] == cv);
            }
            any = __syncthreads_or(c);
            if (any) break;
        }
        if (!any) return false;
        if (PHASE == kDetect) return true;
    }
    for (int base = 0;; base += kBlockWindowBits) {
        for (int w = t; w < kBlockWindowWords; w += kBlock) bm[w] = 0u;
        if (t == 0) *sh_min = INT_MAX;
        __syncthreads();
        for (int j = b + t; j < e; j += kBlock) {
            const int u = ci[j];
            if (u == v) continue;
            const int rel = col[u] - base;
            if ((unsigned)rel < (unsigned)kBlockWindowBits) lds_or(&bm[rel >> 5], 1u << (rel & 31));
        }
        __syncthreads();
        for (int w = t; w < kBlockWindowWords; w += kBlock)
            if (bm[w] != 0xffffffffu) { atomicMin(sh_min, w); break; }
        __syncthreads();
        const int w = *sh_min;
        if (w != INT_MAX) {
            newc = base + w * 32 + __builtin_ctz(~bm[w]);
            __syncthreads();
            return true;
        }
        __syncthreads();
    }
}

}  // namespace rsoc
