// classes_kernels.hpp -- colour classes: the independent sets a colouring
// defines, one per colour (the use of colouring Section 1 describes: the
// vertices of one class can be processed concurrently).  Class k lists the
// vertices of colour k in ascending id.
//
// A stable counting sort by colour, MI355X-shaped:
//   * each wavefront owns a sub-tile of kClsSub consecutive ids, walked as 16
//     rows of 64 (one coalesced 256-byte load per row);
//   * counting: one LDS add per lane and row;
//   * placing: inside a row, the lanes of each colour are found as a bit set
//     in LDS (a lane's rank among them is a popcount), and the lowest lane of
//     each colour advances that colour's LDS counter for all of them, so the
//     order within a class is the id order;
//   * the per-(colour, sub-tile) counts are laid out colour-major and scanned
//     exclusively: entry (c, s) becomes the position of sub-tile s's first
//     vertex of colour c;
//   * colours are handled in windows of at most kClsWin (the per-wavefront LDS
//     counters), one pass per window.
#pragma once

#include "device_common.hpp"

namespace rsoc {

constexpr int kClsSub = 1024;                             // ids per wavefront sub-tile
constexpr int kClsRows = kClsSub / kWave;                 // rows of 64 ids per sub-tile
constexpr int kClsWin = 512;                              // colours per pass
constexpr int kClsChunk = 4096;                           // scan: entries per workgroup (16 per lane)
constexpr int kClsTopMax = 16384;                         // scan: chunk sums one workgroup scans
constexpr int64_t kClsHMax = (int64_t)kClsChunk * kClsTopMax;  // entries of one pass's count table

// base: number of vertices with a colour below the current window (the
// classes before it); err bit 0: a colour outside [0, K).
struct ClsState {
    int64_t base;
    int32_t err;
    int32_t pad;
};

__global__ void k_cls_init(ClsState *st) {
    if (threadIdx.x == 0) {
        st->base = 0;
        st->err = 0;
    }
}

// Per-sub-tile counts of the colours in [c0, c0 + W): H[(c - c0) * nsub + s].
// CHECK: also flags colours outside [0, K) (first pass).
template <bool CHECK>
__global__ __launch_bounds__(kBlock) void k_cls_count(const int32_t *__restrict__ colors, int64_t n, int32_t K,
                                                      int32_t c0, int32_t W, int64_t nsub, int32_t *H,
                                                      ClsState *st) {
    __shared__ int32_t cnt[kWavesPerBlock][kClsWin];
    const int wv = threadIdx.x / kWave, lane = lane_id();
    const int64_t sub = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    if (sub >= nsub) return;  // whole wavefronts leave; nothing below waits on the workgroup
    int32_t *ct = cnt[wv];
    for (int i = lane; i < W; i += kWave) ct[i] = 0;
    wave_lds_sync();
    const RSOC_GLOBAL int32_t *cg = gro(colors);
    // all rows' loads in flight before the first is examined
    int cr[kClsRows];
#pragma unroll
    for (int r = 0; r < kClsRows; ++r) {
        const int64_t v = sub * kClsSub + (int64_t)r * kWave + lane;
        cr[r] = v < n ? cg[v] : -1;
    }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < kClsRows; ++r) {
        const int64_t v = sub * kClsSub + (int64_t)r * kWave + lane;
        const int c = cr[r];
        if (CHECK && v < n && (c < 0 || c >= K)) bad = true;
        const bool in = v < n && c >= c0 && c < c0 + W;
        if (in) atomicAdd(&ct[c - c0], 1);  // equal colours of a row are serialised by the LDS
    }
    wave_lds_sync();
    for (int i = lane; i < W; i += kWave) H[(int64_t)i * nsub + sub] = ct[i];
    if (CHECK && ballot(bad) && lane == 0) atomicOr(&st->err, 1);
}

// Exclusive scan of H[0, len) in place, in three steps: chunk sums, a scan of
// the sums (plus the classes before the window, st->base, which then advances
// by the window's total), and each chunk's own scan from its offset.
__global__ __launch_bounds__(kBlock) void k_cls_scan_reduce(const int32_t *__restrict__ H, int64_t len,
                                                            int32_t *P) {
    __shared__ int sh[kWavesPerBlock];
    const int64_t b0 = (int64_t)blockIdx.x * kClsChunk;
    int s = 0;
    for (int j = 0; j < kClsChunk / kBlock; ++j) {
        const int64_t i = b0 + (int64_t)j * kBlock + threadIdx.x;
        if (i < len) s += H[i];
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane_id() == 0) sh[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) t += sh[w];
        P[blockIdx.x] = t;
    }
}

constexpr int kClsTopBlock = 1024;
__global__ __launch_bounds__(kClsTopBlock) void k_cls_scan_top(int32_t *P, int m, ClsState *st) {
    constexpr int kPer = kClsTopMax / kClsTopBlock;  // consecutive sums per lane
    __shared__ int sh[kClsTopBlock / kWave];
    const int t = threadIdx.x;
    int x[kPer];
    int s = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = t * kPer + j;
        x[j] = i < m ? P[i] : 0;
        s += x[j];
    }
    // exclusive scan of the lanes' sums: within the wavefront, then across
    int incl = s;
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(incl, off);
        if (lane_id() >= off) incl += y;
    }
    if (lane_id() == kWave - 1) sh[t / kWave] = incl;
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < t / kWave; ++w) wbase += sh[w];
    int total = 0;
    for (int w = 0; w < kClsTopBlock / kWave; ++w) total += sh[w];
    const int64_t base = st->base;
    int run = (int)base + wbase + incl - s;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = t * kPer + j;
        if (i < m) P[i] = run;
        run += x[j];
    }
    __syncthreads();  // every lane has read st->base
    if (t == 0) st->base = base + total;
}

__global__ __launch_bounds__(kBlock) void k_cls_scan_down(int32_t *H, int64_t len, const int32_t *__restrict__ P) {
    constexpr int kPer = kClsChunk / kBlock;  // consecutive entries per lane
    __shared__ int sh[kWavesPerBlock];
    const int t = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kClsChunk + (int64_t)t * kPer;
    int x[kPer];
    int s = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        x[j] = b0 + j < len ? H[b0 + j] : 0;
        s += x[j];
    }
    int incl = s;
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(incl, off);
        if (lane_id() >= off) incl += y;
    }
    if (lane_id() == kWave - 1) sh[t / kWave] = incl;
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < t / kWave; ++w) wbase += sh[w];
    int run = P[blockIdx.x] + wbase + incl - s;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        if (b0 + j < len) H[b0 + j] = run;
        run += x[j];
    }
}

// Class starts of the window: ptr[c0 + i] = position of sub-tile 0's first
// vertex of colour c0 + i; the last window also writes ptr[K] (= n when every
// colour was in range).
__global__ void k_cls_ptr(const int32_t *__restrict__ H, int64_t nsub, int32_t c0, int32_t W, int32_t K,
                          int32_t *ptr, const ClsState *st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < W) ptr[c0 + i] = H[(int64_t)i * nsub];
    if (i == 0 && c0 + W == K) ptr[K] = (int32_t)st->base;
}

// Places the vertices of colours [c0, c0 + W): a lane of colour c in a row
// goes after the earlier ones of its sub-tile (the wavefront's LDS counter,
// started from the scanned table) and the lanes below it of the same colour.
// The lanes of each colour in a row are found through an LDS bit set per
// colour: every lane sets its bit, then reads its colour's set back.
__global__ __launch_bounds__(kBlock) void k_cls_scatter(const int32_t *__restrict__ colors, int64_t n, int32_t c0,
                                                        int32_t W, int64_t nsub, const int32_t *__restrict__ H,
                                                        int32_t *vtx) {
    __shared__ int32_t cnt[kWavesPerBlock][kClsWin];
    __shared__ uint32_t bits[kWavesPerBlock][kClsWin][2];
    const int wv = threadIdx.x / kWave, lane = lane_id();
    const int64_t sub = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    if (sub >= nsub) return;
    int32_t *ct = cnt[wv];
    uint32_t(*bs)[2] = bits[wv];
    for (int i = lane; i < W; i += kWave) {
        ct[i] = H[(int64_t)i * nsub + sub];
        bs[i][0] = bs[i][1] = 0;
    }
    wave_lds_sync();
    const RSOC_GLOBAL int32_t *cg = gro(colors);
    RSOC_GLOBAL int32_t *out = grw(vtx);
    int cr[kClsRows];
#pragma unroll
    for (int r = 0; r < kClsRows; ++r) {
        const int64_t v = sub * kClsSub + (int64_t)r * kWave + lane;
        cr[r] = v < n ? cg[v] : -1;
    }
    const int half = lane >> 5;
    const uint32_t bit = 1u << (lane & 31);
    for (int r = 0; r < kClsRows; ++r) {
        const int64_t v = sub * kClsSub + (int64_t)r * kWave + lane;
        const int c = cr[r];
        const bool in = v < n && c >= c0 && c < c0 + W;
        const int k = in ? c - c0 : 0;
        if (in) atomicOr(&bs[k][half], bit);
        wave_lds_sync();
        uint64_t mine = 0;
        if (in) mine = (uint64_t)bs[k][0] | ((uint64_t)bs[k][1] << 32);
        const int lead = in ? __ffsll((unsigned long long)mine) - 1 : lane;
        // each colour's lowest lane advances its counter by the colour's lanes
        // and clears the set for the next row (LDS operations of a wavefront
        // take effect in order)
        int old = 0;
        if (in && lead == lane) {
            old = atomicAdd(&ct[k], __popcll(mine));
            bs[k][0] = bs[k][1] = 0;
        }
        wave_lds_sync();
        const int base = __shfl(old, lead);
        if (in) out[base + __popcll(mine & ((1ull << lane) - 1))] = (int32_t)v;
    }
}

}  // namespace rsoc
