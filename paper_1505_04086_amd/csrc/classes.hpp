// classes.hpp -- host drivers of rsoc_color_classes and
// rsoc_color_classes_noalloc (kernels: classes_kernels.hpp).
#pragma once

#include <mutex>

#include "classes_kernels.hpp"
#include "single.hpp"

namespace rsoc {

// Colours per pass: the per-wavefront LDS counters hold kClsWin, and one
// pass's count table (colours x sub-tiles) must fit in hcap entries.
inline int64_t cls_window(int32_t K, int64_t nsub, int64_t hcap) {
    return std::max<int64_t>(1, std::min<int64_t>({(int64_t)K, kClsWin, hcap / nsub}));
}

// Enqueues the whole extraction for n > 0: H must hold cls_window(...) * nsub
// entries, P one per kClsChunk of them, st one ClsState.  Each pass rewrites
// every entry of H and P it reads, and k_cls_init clears st, so the scratch
// needs no clearing between calls.  The error flag is left in st->err.
inline int32_t enqueue_classes(const int32_t *colors, int32_t n, int32_t K, int32_t *ptr, int32_t *vtx, hipStream_t s,
                               int32_t *H, int32_t *P, ClsState *st, int64_t hcap) {
    k_cls_init<<<1, 64, 0, s>>>(st);
    const int64_t nsub = (n + kClsSub - 1) / kClsSub;
    const int64_t W = cls_window(K, nsub, hcap);
    const int gsub = (int)((nsub + kWavesPerBlock - 1) / kWavesPerBlock);
    for (int64_t c0 = 0; c0 < K; c0 += W) {
        const int32_t w = (int32_t)std::min<int64_t>(W, K - c0);
        const int64_t lw = (int64_t)w * nsub;
        const int mw = (int)((lw + kClsChunk - 1) / kClsChunk);
        if (c0 == 0)
            k_cls_count<true><<<gsub, kBlock, 0, s>>>(colors, n, K, (int32_t)c0, w, nsub, H, st);
        else
            k_cls_count<false><<<gsub, kBlock, 0, s>>>(colors, n, K, (int32_t)c0, w, nsub, H, st);
        k_cls_scan_reduce<<<mw, kBlock, 0, s>>>(H, lw, P);
        k_cls_scan_top<<<1, kClsTopBlock, 0, s>>>(P, mw, st);
        k_cls_scan_down<<<mw, kBlock, 0, s>>>(H, lw, P);
        k_cls_ptr<<<div_up(w, kBlock), kBlock, 0, s>>>(H, nsub, (int32_t)c0, w, K, ptr, st);
        k_cls_scatter<<<gsub, kBlock, 0, s>>>(colors, n, (int32_t)c0, w, nsub, H, vtx);
        RSOC_LAUNCH_CHECK();
    }
    return RSOC_OK;
}

// n == 0: K + 1 empty classes.
inline int32_t empty_classes(int32_t K, int32_t *ptr, hipStream_t s) {
    k_fill<<<div_up((int64_t)K + 1, kBlock), kBlock, 0, s>>>(ptr, nullptr, (int64_t)K + 1, 0);
    RSOC_LAUNCH_CHECK();
    RSOC_HIP(hipStreamSynchronize(s));
    return RSOC_OK;
}

inline int32_t run_classes(rsoc_ctx *c, const int32_t *colors, int32_t n, int32_t K, int32_t *ptr, int32_t *vtx,
                           hipStream_t s) {
    HostStaging *h = c->host.as<HostStaging>();
    if (n == 0) return empty_classes(K, ptr, s);
    const int64_t nsub = (n + kClsSub - 1) / kClsSub;
    const int64_t len = cls_window(K, nsub, kClsHMax) * nsub;
    RSOC_TRY(c->cls_st.reserve(sizeof(ClsState)));
    RSOC_TRY(c->cls_h.reserve(sizeof(int32_t) * (size_t)len));
    RSOC_TRY(c->cls_p.reserve(sizeof(int32_t) * (size_t)((len + kClsChunk - 1) / kClsChunk)));
    RSOC_TRY(enqueue_classes(colors, n, K, ptr, vtx, s, c->cls_h.as<int32_t>(), c->cls_p.as<int32_t>(),
                             c->cls_st.as<ClsState>(), kClsHMax));
    ClsState *st = c->cls_st.as<ClsState>();
    RSOC_HIP(hipMemcpyAsync(&h->cls_err, &st->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RSOC_HIP(hipStreamSynchronize(s));
    return h->cls_err ? RSOC_EINVAL : RSOC_OK;
}

// ---------------------------------------------------------------------------
// The variant that allocates nothing.  Its scratch (the class state, the scan
// sums and one pass's count table) is one fixed device array per GPU, held
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: the device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is ever
// handed to kernels.  Every call on a GPU shares its array, so calls that
// overlap on one GPU (other streams, other host threads) race.
constexpr int64_t kNaHCap = (int64_t)1 << 20;                  // count-table entries (4 MiB)
constexpr int64_t kNaPCap = kNaHCap / kClsChunk;                // scan sums (256)
constexpr size_t kNaOffP = 256;                                 // after the ClsState
constexpr size_t kNaOffH = kNaOffP + sizeof(int32_t) * kNaPCap;  // 256-byte aligned
constexpr size_t kNaScratchBytes = kNaOffH + sizeof(int32_t) * kNaHCap;
constexpr int64_t kNaMaxN = kNaHCap * kClsSub;                  // 2^30 vertices: one colour per pass at most
constexpr int kNaMaxDevices = 64;
static_assert(sizeof(ClsState) <= kNaOffP && kNaOffH % 256 == 0, "scratch layout");
static_assert(kNaPCap <= kClsTopMax, "one scan workgroup takes every pass's sums");

static __device__ __align__(256) unsigned char scratch[kNaScratchBytes];

// Device address of `scratch` on the current device, looked up on the first
// call there (once per device, under a lock).
inline int32_t noalloc_scratch(unsigned char **out) {
    static std::mutex mu;
    static unsigned char *addr[kNaMaxDevices] = {};
    int dev = -1;
    RSOC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return RSOC_EINVAL;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        RSOC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return RSOC_EHIP;
        addr[dev] = static_cast<unsigned char *>(p);
    }
    *out = addr[dev];
    return RSOC_OK;
}

inline int32_t run_classes_noalloc(const int32_t *colors, int32_t n, int32_t K, int32_t *ptr, int32_t *vtx,
                                   hipStream_t s) {
    if ((int64_t)n > kNaMaxN) return RSOC_ESCRATCH;
    unsigned char *base = nullptr;
    RSOC_TRY(noalloc_scratch(&base));
    if (n == 0) return empty_classes(K, ptr, s);
    ClsState *st = reinterpret_cast<ClsState *>(base);
    RSOC_TRY(enqueue_classes(colors, n, K, ptr, vtx, s, reinterpret_cast<int32_t *>(base + kNaOffH),
                             reinterpret_cast<int32_t *>(base + kNaOffP), st, kNaHCap));
    int32_t err = 0;  // pageable host word: the copy below is synchronous for it
    RSOC_HIP(hipMemcpyAsync(&err, &st->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RSOC_HIP(hipStreamSynchronize(s));
    return err ? RSOC_EINVAL : RSOC_OK;
}

}  // namespace rsoc
