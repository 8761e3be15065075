// host_common.hpp -- error plumbing and small host utilities for the C ABI.
#pragma once

#include <hip/hip_ext.h>
#include <algorithm>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "device_common.hpp"
#include "rsoc.h"

namespace rsoc {

// Text of the last HIP error on this host thread (rsoc_last_error).
inline char *last_error_buf() {
    static thread_local char buf[256] = {0};
    return buf;
}

inline int32_t hip_fail(hipError_t e, const char *what, const char *file, int line) {
    snprintf(last_error_buf(), 256, "%s: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    return (e == hipErrorOutOfMemory) ? RSOC_ENOMEM : RSOC_EHIP;
}

#define RSOC_HIP(call)                                                          \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) return ::rsoc::hip_fail(e_, #call, __FILE__, __LINE__); \
    } while (0)

#define RSOC_TRY(expr)                      \
    do {                                    \
        int32_t r_ = (expr);                \
        if (r_ < 0) return r_;              \
    } while (0)

#define RSOC_LAUNCH_CHECK() RSOC_HIP(hipGetLastError())

// Launches kernel f on `grid` workgroups of `block` lanes.  Events given
// (either may be null) record the kernel's own start and end: they are part
// of its dispatch, so no marker command waits between it and its neighbours
// on the stream.
template <typename... P, typename... Args>
inline void launch_ev(void (*f)(P...), int grid, int block, hipStream_t s, hipEvent_t start, hipEvent_t stop,
                      Args... args) {
    hipExtLaunchKernelGGL(f, dim3(grid), dim3(block), 0, s, start, stop, 0, args...);
}

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

inline int round_up_to(int x, int m) { return ((x + m - 1) / m) * m; }

// Device buffer that only grows.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    int32_t reserve(size_t want) {
        if (want <= bytes) return RSOC_OK;
        if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
        size_t b = want < 256 ? 256 : want;
        RSOC_HIP(hipMalloc(&p, b));
        bytes = b;
        return RSOC_OK;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

struct HostPinned {
    void *p = nullptr;
    size_t bytes = 0;
    int32_t reserve(size_t want) {
        if (want <= bytes) return RSOC_OK;
        if (p) { (void)hipHostFree(p); p = nullptr; bytes = 0; }
        size_t b = want < 256 ? 256 : want;
        RSOC_HIP(hipHostMalloc(&p, b, hipHostMallocDefault));
        bytes = b;
        return RSOC_OK;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

// Largest graph of a batch coloured by one workgroup (colours and worklists in
// LDS; the option small_cutoff).
constexpr int kSmallMaxVertices = 2048;
// Sweep bands per XCD of a batch's optimistic round 0 (the option bands;
// at most kMaxBandsPerXcd).
constexpr int kDefaultBandsPerXcd = 4;

struct Options {
    int mode, tie, max_rounds, validate, t_thread, t_wave, grid_thread, grid_wave, rounds_per_sync,
        timing, full_sweep, lookahead, chunk, grid_list, tail, distance, grid_bin, hub_first, small_cutoff, bands;
    bool grid_thread_given;  // grid_thread came from the caller (not the default)
};

inline int32_t resolve_options(const rsoc_options *o, int64_t n, Options &r) {
    rsoc_options d;
    memset(&d, 0, sizeof(d));
    if (o) d = *o;
    r.mode = d.mode;
    r.tie = d.tie;
    if (r.mode < RSOC_MODE_OPTIMISTIC || r.mode > RSOC_MODE_TWO_PHASE_LIVE) return RSOC_EINVAL;
    if (r.tie != RSOC_TIE_LOWER_KEEPS && r.tie != RSOC_TIE_HIGHER_KEEPS) return RSOC_EINVAL;
    if (d.max_rounds < 0 || d.t_thread < 0 || d.t_thread > 32 || d.t_wave < 0 || d.grid_thread < 0 ||
        d.grid_wave < 0 || d.rounds_per_sync < 0 || d.validate < 0 || d.validate > 3 || d.grid_list < 0)
        return RSOC_EINVAL;
    if (d.reserved || d.grid_bin < 0) return RSOC_EINVAL;
    if (d.bands < 0 || d.bands > kMaxBandsPerXcd) return RSOC_EINVAL;
    r.bands = d.bands ? d.bands : kDefaultBandsPerXcd;
    if (d.small_cutoff < -1 || d.small_cutoff > kSmallMaxVertices) return RSOC_EINVAL;
    if (d.hub_first < -1) return RSOC_EINVAL;
    r.grid_bin = d.grid_bin;  // 0: each launch site's own default
    if (d.distance < 0 || d.distance > 2) return RSOC_EINVAL;
    r.distance = d.distance == 2 ? 2 : 1;
    if (d.tail < -1) return RSOC_EINVAL;
    r.tail = d.tail;  // 0: library default; clamped to the largest allowed where used
    if (d.chunk != 0 && d.chunk != 1 && d.chunk != 2 && d.chunk != 4 && d.chunk != 8) return RSOC_EINVAL;
    r.chunk = d.chunk;
    if (d.lookahead < -1) return RSOC_EINVAL;
    r.lookahead = d.lookahead;
    if (d.full_sweep < 0 || d.full_sweep > 1) return RSOC_EINVAL;
    r.full_sweep = d.full_sweep;
    r.max_rounds = d.max_rounds ? d.max_rounds : (int)((n + 1 < INT32_MAX) ? n + 1 : INT32_MAX);
    r.validate = d.validate;
    r.t_thread = d.t_thread ? d.t_thread : 32;
    r.t_wave = d.t_wave ? d.t_wave : 2048;
    if (r.t_wave < r.t_thread) r.t_wave = r.t_thread;
    r.grid_thread = d.grid_thread ? d.grid_thread : 1024;
    r.grid_thread_given = d.grid_thread != 0;
    r.grid_wave = d.grid_wave ? d.grid_wave : 2048;
    r.grid_list = d.grid_list ? d.grid_list : 1024;
    r.rounds_per_sync = d.rounds_per_sync ? d.rounds_per_sync : 4;
    if (r.rounds_per_sync & 1) r.rounds_per_sync += 1;  // worklist buffers alternate: keep it even
    r.timing = d.timing;
    // hub threshold: 0 = off, -1 = automatic (from the max degree, on the
    // device), else the degree given, never below the lane-group bin's limit,
    // so that hubs are wavefront- or workgroup-bin vertices
    r.hub_first = d.hub_first == -1 ? 0 : (d.hub_first == 0 ? -1 : std::max(d.hub_first, r.t_thread));
    r.small_cutoff = d.small_cutoff == -1 ? 0 : (d.small_cutoff == 0 ? kSmallMaxVertices : d.small_cutoff);
    return RSOC_OK;
}

}  // namespace rsoc
