// square.hpp -- host driver of the distance-2 colouring: G^2 is built on the
// device (square_kernels.hpp) and coloured by run_single unchanged.
#pragma once

#include "classes_kernels.hpp"
#include "single.hpp"
#include "square_kernels.hpp"

namespace rsoc {

// Builds G^2 of the device CSR (rp, ci, n) into the context's scratch; on
// success *rp2 / *ci2 point at it.
inline int32_t build_square(rsoc_ctx *c, const int32_t *rp, const int32_t *ci, int32_t n, hipStream_t s,
                            const int32_t **rp2, const int32_t **ci2) {
    HostStaging *h = c->host.as<HostStaging>();
    if ((n + kClsChunk - 1) / kClsChunk > kClsTopMax) return RSOC_EINVAL;  // the row-start scan's reach
    RSOC_TRY(c->sq_t.reserve(sizeof(int32_t) * (size_t)(n + 1)));
    RSOC_TRY(c->sq_rp.reserve(sizeof(int32_t) * (size_t)(n + 1)));
    RSOC_TRY(c->sq_misc.reserve(256));
    RSOC_TRY(c->cls_st.reserve(sizeof(ClsState)));
    RSOC_TRY(c->cls_p.reserve(sizeof(int32_t) * (size_t)kClsTopMax));
    int32_t *T = c->sq_t.as<int32_t>();
    int32_t *R = c->sq_rp.as<int32_t>();
    unsigned long long *total = c->sq_misc.as<unsigned long long>();
    int32_t *err = reinterpret_cast<int32_t *>(total + 1);
    int32_t *nbig = err + 1;
    RSOC_TRY(c->sq_big.reserve(sizeof(int32_t) * (size_t)(n + 1)));
    int32_t *big = c->sq_big.as<int32_t>();
    RSOC_HIP(hipMemsetAsync(c->sq_misc.p, 0, 16, s));
    const int g = std::min(div_up(n, kBlock), 4096);
    k_sq_size<<<std::min(div_up(n, kBlock / 8), 8192), kBlock, 0, s>>>(rp, ci, n, T, err, big, nbig);
    // a walk over the limit ends it here, before the expensive passes
    RSOC_LAUNCH_CHECK();
    RSOC_HIP(hipMemcpyAsync(&h->sq_total, c->sq_misc.p, 16, hipMemcpyDeviceToHost, s));
    RSOC_HIP(hipStreamSynchronize(s));
    if (h->sq_err) return RSOC_EINVAL;
    // count pass: rows with T <= kSqSmallT four wavefronts a workgroup, the
    // listed rest one wavefront each with a larger table
    k_sq_rows<4, kSqSmallTab, false><<<std::min(div_up(n, 4), 65536), 4 * kWave, 0, s>>>(
        rp, ci, n, T, -1, kSqSmallT, nullptr, nullptr, R, nullptr, nullptr);
    k_sq_rows<1, kSqBigTab, false><<<std::min(n, 2048), kWave, 0, s>>>(rp, ci, n, T, kSqSmallT, kSqBigT, big, nbig, R,
                                                                         nullptr, nullptr);
    k_sq_total<<<g, kBlock, 0, s>>>(R, n, total);
    RSOC_LAUNCH_CHECK();
    RSOC_HIP(hipMemcpyAsync(&h->sq_total, c->sq_misc.p, 16, hipMemcpyDeviceToHost, s));
    RSOC_HIP(hipStreamSynchronize(s));
    if (h->sq_err || h->sq_total > (unsigned long long)INT32_MAX) return RSOC_EINVAL;
    // row starts: exclusive scan of the counts in place, then the total
    const int64_t len = n;
    const int m = (int)((len + kClsChunk - 1) / kClsChunk);
    ClsState *st = c->cls_st.as<ClsState>();
    k_cls_init<<<1, 64, 0, s>>>(st);
    k_cls_scan_reduce<<<m, kBlock, 0, s>>>(R, len, c->cls_p.as<int32_t>());
    k_cls_scan_top<<<1, kClsTopBlock, 0, s>>>(c->cls_p.as<int32_t>(), m, st);
    k_cls_scan_down<<<m, kBlock, 0, s>>>(R, len, c->cls_p.as<int32_t>());
    k_sq_tail<<<1, 64, 0, s>>>(R, n, total);
    RSOC_TRY(c->sq_ci.reserve(sizeof(int32_t) * (size_t)std::max<unsigned long long>(h->sq_total, 1)));
    int32_t *C = c->sq_ci.as<int32_t>();
    k_sq_rows<4, kSqSmallTab, true><<<std::min(div_up(n, 4), 65536), 4 * kWave, 0, s>>>(
        rp, ci, n, T, -1, kSqSmallT, nullptr, nullptr, nullptr, R, C);
    k_sq_rows<1, kSqBigTab, true><<<std::min(n, 2048), kWave, 0, s>>>(rp, ci, n, T, kSqSmallT, kSqBigT, big, nbig,
                                                                        nullptr, R, C);
    RSOC_LAUNCH_CHECK();
    *rp2 = R;
    *ci2 = C;
    return RSOC_OK;
}

// Colouring of G (distance 1) or of G^2 (distance 2).  For distance 2 the
// ends of row_ptr are checked (and, when asked for, all of G is validated)
// before anything reads the rows.
inline int32_t run_colouring(rsoc_ctx *c, const int32_t *rp, const int32_t *ci, int32_t n, int32_t *col,
                             const Options &o, rsoc_stats *st, hipStream_t s) {
    if (o.distance != 2 || n == 0) return run_single(c, rp, ci, n, col, o, st, s);
    HostStaging *h = c->host.as<HostStaging>();
    RSOC_HIP(hipMemcpyAsync(&h->rp_ends[0], rp, 4, hipMemcpyDeviceToHost, s));
    RSOC_HIP(hipMemcpyAsync(&h->rp_ends[1], rp + n, 4, hipMemcpyDeviceToHost, s));
    RSOC_HIP(hipStreamSynchronize(s));
    if (h->rp_ends[0] != 0 || h->rp_ends[1] < 0) return RSOC_ECSR;
    if (h->rp_ends[1] > 0 && !ci) return RSOC_EINVAL;
    if (o.validate & RSOC_CHECK_CSR) {
        RSOC_TRY(c->sq_misc.reserve(256));
        int32_t *verr = reinterpret_cast<int32_t *>(c->sq_misc.as<char>() + 16);
        RSOC_HIP(hipMemsetAsync(verr, 0, 4, s));
        k_validate<<<std::min(div_up(n, kBlock), 4096), kBlock, 0, s>>>(rp, ci, n, verr);
        RSOC_LAUNCH_CHECK();
        RSOC_HIP(hipMemcpyAsync(&h->sq_verr, verr, 4, hipMemcpyDeviceToHost, s));
        RSOC_HIP(hipStreamSynchronize(s));
        RSOC_TRY(status_from_err(h->sq_verr));
    }
    const int32_t *rp2 = nullptr, *ci2 = nullptr;
    RSOC_TRY(build_square(c, rp, ci, n, s, &rp2, &ci2));
    Options o2 = o;
    o2.validate = 0;
    return run_single(c, rp2, ci2, n, col, o2, st, s);
}

}  // namespace rsoc
