// device_common.hpp -- wavefront helpers and constants shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsoc {

// Global-memory (address space 1) views of plain pointers: loads through them
// compile to global_load_* instead of flat loads (pointers read from device
// memory would otherwise stay generic).
#define RSOC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const RSOC_GLOBAL T *gro(const T *p) { return (const RSOC_GLOBAL T *)p; }
template <class T>
__device__ __forceinline__ RSOC_GLOBAL T *grw(T *p) { return (RSOC_GLOBAL T *)p; }

constexpr int kWave = 64;                 // CDNA wavefront width
constexpr int kBlock = 256;               // threads per workgroup for every round kernel
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kWaveWindowBits = 4096;     // forbidden-colour window of a wavefront (512 B of LDS)
constexpr int kWaveWindowWords = kWaveWindowBits / 32;
constexpr int kBlockWindowBits = 32768;   // forbidden-colour window of a workgroup (4 KB of LDS)
constexpr int kBlockWindowWords = kBlockWindowBits / 32;
constexpr int kLdsWords = (kBlockWindowWords > kWavesPerBlock * kWaveWindowWords) ? kBlockWindowWords
                                                                                  : kWavesPerBlock * kWaveWindowWords;
constexpr int kHistCap = 1 << 16;         // per-round |L| history kept on the device
constexpr int kXcds = 8;                  // MI355X: 8 accelerator complex dies, 32 CUs each
constexpr int kMaxBandsPerXcd = 16;      // sweep bands per XCD of a batch's optimistic round 0
constexpr int kMaxBands = kXcds * kMaxBandsPerXcd;
constexpr int kGroup = 8;                 // lanes per vertex in the thread bin
constexpr int kGroupSlots = 4;            // row entries each lane holds: thread-bin degree <= 32
constexpr int kThreadBinMax = kGroup * kGroupSlots;
constexpr int kQueueCap = 1024;           // per-workgroup append queue (LDS) of the thread bin
// Thread-bin walk: each lane group takes kNV runs of kChunk consecutive
// vertex ids and walks them one id at a time (both runs side by side), so
// ids that are adjacent in a natural-order mesh are coloured one after the
// other by the same lanes, as a CPU thread walks its block of ids.
constexpr int kNV = 2;                              // vertices per lane group per sub-step
constexpr int kGpb = kBlock / kGroup;               // lane groups per workgroup
constexpr int kChunk = 8;                           // consecutive ids per run
constexpr int kSub = kNV * kGpb;                    // vertices per sub-step
constexpr int kStep = kSub * kChunk;                // vertices per workgroup step

// Run length of consecutive ids per lane group: the option when given, else
// kChunk when at least 2% of sampled row entries join ids less than kChunk
// apart (a natural-order mesh: walking runs keeps those neighbours out of the
// same instant), else 1 (scrambled ids: neighbouring groups stream
// neighbouring rows).
__host__ __device__ inline int pick_chunk(int option, uint64_t near, uint64_t sampled) {
    if (option) return option;
    return (sampled > 0 && near * 50 >= sampled) ? kChunk : 1;
}

// Position inside a workgroup step of sub-step r (0..kChunk-1), run i, lane
// group gi, when each group walks runs of c consecutive ids (c a power of two
// dividing kChunk; c = 1 puts consecutive ids in neighbouring groups, which
// streams rows best when ids carry no locality).
__host__ __device__ constexpr int step_offset(int r, int i, int gi, int c) {
    return (r / c) * (kSub * c) + (i * kGpb + gi) * c + (r % c);
}

enum Phase : int { kAssign = 0, kRecolor = 1, kDetect = 2 };
enum Mode : int { kOptimistic = 0, kDeterministic = 1, kTwoPhase = 2, kTwoPhaseLive = 3 };
// modes that write colours in place and read them live
__host__ __device__ constexpr bool live_mode(int m) { return m == kOptimistic || m == kTwoPhaseLive; }
__host__ __device__ constexpr bool two_phase_mode(int m) { return m == kTwoPhase || m == kTwoPhaseLive; }
enum Tie : int { kLowerKeeps = 0, kHigherKeeps = 1 };
enum Bin : int { kBinThread = 0, kBinWave = 1, kBinBlock = 2 };

// v is defective against neighbour u with the same colour iff it loses the tie.
template <int TIE>
__device__ __forceinline__ bool loses(int v, int u) {
    return TIE == kLowerKeeps ? (u < v) : (u > v);
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

// number of set bits of m below this lane
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// OR of a predicate over the G-lane group this lane belongs to (G divides 64).
template <int G>
__device__ __forceinline__ bool group_any(bool p) {
    const uint64_t m = ballot(p);
    const int g0 = lane_id() & ~(G - 1);
    return ((m >> g0) & ((G == 64) ? ~0ull : ((1ull << G) - 1))) != 0;
}

// OR of a 32-bit value over the G-lane group (butterfly).
template <int G>
__device__ __forceinline__ uint32_t group_or32(uint32_t x) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) x |= __shfl_xor(x, off);
    return x;
}

// OR of a 64-bit value over the G-lane group (butterfly).
template <int G>
__device__ __forceinline__ uint64_t group_or64(uint64_t x) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)x, off), hi = __shfl_xor((uint32_t)(x >> 32), off);
        x |= ((uint64_t)hi << 32) | lo;
    }
    return x;
}

// Orders this wavefront's LDS accesses across lanes (a compiler barrier; the
// hardware executes one wavefront's LDS instructions in order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void lds_or(uint32_t *p, uint32_t bits) {
    __hip_atomic_fetch_or(p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Appends `v` for every lane with `take` set: one global atomic per wavefront,
// positions from the lane prefix count.
__device__ __forceinline__ void wave_append(bool take, int v, int *counter, int *list) {
    uint64_t m = ballot(take);
    if (m == 0) return;
    int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    if (take) list[base + lanes_below(m)] = v;
}

// Sizes of a workgroup's LDS append queues as every wavefront sees them; the
// whole workgroup calls this between its appends and any flush decision.  A
// wavefront goes on to its next append (an LDS atomic on the same counter) as
// soon as it has read the counter, so a count read after a single barrier can
// differ between wavefronts: a slower one may already see the next step's
// appends, decide to flush alone, and its flush barriers then pair with the
// other wavefronts' loop barriers (entries lost, duplicated, or written past
// the queue).  The first barrier ends the appends in flight; the second holds
// every wavefront until all have read the same values.
__device__ __forceinline__ int queue_size(const int *qn) {
    __syncthreads();
    const int c = *(const volatile int *)qn;
    __syncthreads();
    return c;
}
__device__ __forceinline__ void queue_sizes(const int *qa, const int *qb, int &ca, int &cb) {
    __syncthreads();
    ca = *(const volatile int *)qa;
    cb = *(const volatile int *)qb;
    __syncthreads();
}
__device__ __forceinline__ void queue_sizes(const int *qa, const int *qb, const int *qc, int &ca, int &cb, int &cc) {
    __syncthreads();
    ca = *(const volatile int *)qa;
    cb = *(const volatile int *)qb;
    cc = *(const volatile int *)qc;
    __syncthreads();
}

// Wavefront sum of a 64-bit value (result valid in every lane).
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ int wave_max_i32(int x) {
    for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off));
    return x;
}

// Block index remapped so that each XCD works on one contiguous range of the
// section: hardware dispatches consecutive workgroups round-robin over XCDs,
// so blocks b, b+8, b+16, ... share an L2.  Only a bijection when nblocks is
// a multiple of kXcds; otherwise returns b unchanged.
__device__ __forceinline__ int xcd_contiguous(int b, int nblocks) {
    if (nblocks % kXcds) return b;
    int per = nblocks / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

}  // namespace rsoc
