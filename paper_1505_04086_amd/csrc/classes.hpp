// classes.hpp -- host driver of rsoc_color_classes (classes_kernels.hpp).
#pragma once

#include "classes_kernels.hpp"
#include "single.hpp"

namespace rsoc {

inline int32_t run_classes(rsoc_ctx *c, const int32_t *colors, int32_t n, int32_t K, int32_t *ptr, int32_t *vtx,
                           hipStream_t s) {
    HostStaging *h = c->host.as<HostStaging>();
    if (n == 0) {  // K + 1 empty classes
        k_fill<<<div_up((int64_t)K + 1, kBlock), kBlock, 0, s>>>(ptr, nullptr, (int64_t)K + 1, 0);
        RSOC_LAUNCH_CHECK();
        RSOC_HIP(hipStreamSynchronize(s));
        return RSOC_OK;
    }
    RSOC_TRY(c->cls_st.reserve(sizeof(ClsState)));
    ClsState *st = c->cls_st.as<ClsState>();
    k_cls_init<<<1, 64, 0, s>>>(st);
    const int64_t nsub = (n + kClsSub - 1) / kClsSub;
    // colours per pass: the LDS counters, and a count table the scan can take
    const int64_t W = std::max<int64_t>(1, std::min<int64_t>({(int64_t)K, kClsWin, kClsHMax / nsub}));
    const int64_t len = W * nsub;
    const int64_t m = (len + kClsChunk - 1) / kClsChunk;
    RSOC_TRY(c->cls_h.reserve(sizeof(int32_t) * (size_t)std::max<int64_t>(len, 1)));
    RSOC_TRY(c->cls_p.reserve(sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1)));
    int32_t *H = c->cls_h.as<int32_t>();
    int32_t *P = c->cls_p.as<int32_t>();
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
    RSOC_HIP(hipMemcpyAsync(&h->cls_err, &st->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RSOC_HIP(hipStreamSynchronize(s));
    return h->cls_err ? RSOC_EINVAL : RSOC_OK;
}

}  // namespace rsoc
