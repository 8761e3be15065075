// batch.hpp -- batched colouring of many graphs (placeholder until the fused path lands).
#pragma once
#include "single.hpp"

extern "C" int32_t rsoc_color_batch(rsoc_ctx *ctx, int32_t G, const int64_t *vtx_off, const int64_t *nnz_off,
                                    const int32_t *d_row_ptr_cat, const int32_t *d_col_idx_cat, int32_t *d_colors_cat,
                                    int32_t *counts_out, const rsoc_options *opts, rsoc_stats *stats, void *hip_stream) {
    (void)ctx; (void)G; (void)vtx_off; (void)nnz_off; (void)d_row_ptr_cat; (void)d_col_idx_cat; (void)d_colors_cat;
    (void)counts_out; (void)opts; (void)stats; (void)hip_stream;
    return RSOC_EINVAL;
}
