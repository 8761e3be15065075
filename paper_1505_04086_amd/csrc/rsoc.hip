// rsoc.hip -- librsoc: the C ABI (include/rsoc.h) over the gfx950 kernels.
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "host_common.hpp"
#include "single.hpp"
#include "batch.hpp"
#include "pool.hpp"
#include "classes.hpp"
#include "square.hpp"

using namespace rsoc;

extern "C" {

void rsoc_default_options(rsoc_options *opts) {
    if (!opts) return;
    memset(opts, 0, sizeof(*opts));
    opts->mode = RSOC_MODE_OPTIMISTIC;
    opts->tie = RSOC_TIE_LOWER_KEEPS;
}

const char *rsoc_strerror(int32_t status) {
    switch (status) {
        case RSOC_OK: return "ok";
        case RSOC_EINVAL: return "invalid argument";
        case RSOC_ECSR: return "malformed CSR (row_ptr[0] != 0, decreasing row_ptr or column id out of range)";
        case RSOC_ESELFLOOP: return "self-loop in the graph";
        case RSOC_EASYM: return "asymmetric adjacency (an edge stored in one direction only)";
        case RSOC_ENOMEM: return "out of memory";
        case RSOC_EHIP: return "HIP runtime error";
        case RSOC_ENOCONV: return "worklist not empty after max_rounds passes";
        case RSOC_EBUDGET: return "pool admission refused (HBM budget or slot table full)";
        case RSOC_ENOTFOUND: return "unknown or unfinished pool slot";
        case RSOC_EINTERNAL: return "internal consistency check failed (a colour outside [0, degree] or a list size "
                                    "that differs from its independent count): a library defect";
        case RSOC_ESCRATCH: return "input larger than the fixed scratch of the no-allocation entry point allows";
        default: return status >= 0 ? "ok" : "unknown error";
    }
}

const char *rsoc_last_error(void) { return last_error_buf(); }

int32_t rsoc_check_csr(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t flags) {
    if (n < 0 || !row_ptr || (flags & ~3)) return RSOC_EINVAL;
    if (row_ptr[0] != 0) return RSOC_ECSR;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return RSOC_ECSR;
    const int64_t nnz = row_ptr[n];
    if (nnz > 0 && !col_idx) return RSOC_EINVAL;
    for (int32_t v = 0; v < n; ++v)
        for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
            const int32_t u = col_idx[j];
            if (u < 0 || u >= n) return RSOC_ECSR;
            if (u == v) return RSOC_ESELFLOOP;
        }
    if (flags & RSOC_CHECK_SYMMETRY) {
        // transpose by counting, then compare each row with its transposed row as multisets
        std::vector<int64_t> tp((size_t)n + 1, 0);
        for (int64_t j = 0; j < nnz; ++j) tp[(size_t)col_idx[j] + 1]++;
        for (int32_t v = 0; v < n; ++v) tp[v + 1] += tp[v];
        std::vector<int32_t> tc((size_t)nnz);
        std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
        for (int32_t v = 0; v < n; ++v)
            for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) tc[(size_t)fill[col_idx[j]]++] = v;
        std::vector<int32_t> row;
        for (int32_t v = 0; v < n; ++v) {
            if (tp[v + 1] - tp[v] != row_ptr[v + 1] - row_ptr[v]) return RSOC_EASYM;
            row.assign(col_idx + row_ptr[v], col_idx + row_ptr[v + 1]);
            std::sort(row.begin(), row.end());
            std::sort(tc.begin() + tp[v], tc.begin() + tp[v + 1]);
            if (!std::equal(row.begin(), row.end(), tc.begin() + tp[v])) return RSOC_EASYM;
        }
    }
    return RSOC_OK;
}

int32_t rsoc_ctx_create(rsoc_ctx **out, int32_t device) {
    if (!out) return RSOC_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return RSOC_EINVAL;
    rsoc_ctx *c = new (std::nothrow) rsoc_ctx();
    if (!c) return RSOC_ENOMEM;
    int32_t r = ctx_init(c, device);
    if (r < 0) {
        ctx_free(c);
        delete c;
        return r;
    }
    *out = c;
    return RSOC_OK;
}

void rsoc_ctx_destroy(rsoc_ctx *ctx) {
    if (!ctx) return;
    ctx_free(ctx);
    delete ctx;
}

int32_t rsoc_color_device(rsoc_ctx *ctx, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t n,
                          int32_t *d_colors_out, const rsoc_options *opts, rsoc_stats *stats, void *hip_stream) {
    if (!ctx || n < 0 || (n > 0 && (!d_row_ptr || !d_colors_out))) return RSOC_EINVAL;
    Options o;
    RSOC_TRY(resolve_options(opts, n, o));
    RSOC_HIP(hipSetDevice(ctx->device));
    return run_colouring(ctx, d_row_ptr, d_col_idx, n, d_colors_out, o, stats, (hipStream_t)hip_stream);
}

int32_t rsoc_color_ex(rsoc_ctx *ctx, const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t *colors_out,
                      const rsoc_options *opts, rsoc_stats *stats) {
    if (!ctx || n < 0 || (n > 0 && (!row_ptr || !colors_out))) return RSOC_EINVAL;
    Options o;
    RSOC_TRY(resolve_options(opts, n, o));
    if (n == 0) {
        if (stats) {
            int32_t *keep = stats->per_round_L, *keepU = stats->per_round_U;
            int32_t cap = stats->per_round_cap;
            memset(stats, 0, sizeof(*stats));
            stats->per_round_L = keep;
            stats->per_round_U = keepU;
            stats->per_round_cap = cap;
        }
        return 0;
    }
    if (o.validate) RSOC_TRY(rsoc_check_csr(row_ptr, col_idx, n, o.validate));
    else if (row_ptr[0] != 0 || row_ptr[n] < 0) return RSOC_ECSR;
    const int64_t nnz = row_ptr[n];
    if (nnz > 0 && !col_idx) return RSOC_EINVAL;
    RSOC_HIP(hipSetDevice(ctx->device));
    RSOC_TRY(ctx->drp.reserve(sizeof(int32_t) * (size_t)(n + 1)));
    RSOC_TRY(ctx->dci.reserve(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
    RSOC_TRY(ctx->dcol.reserve(sizeof(int32_t) * (size_t)n));
    hipStream_t s = ctx->own;
    RSOC_HIP(hipMemcpyAsync(ctx->drp.p, row_ptr, sizeof(int32_t) * (size_t)(n + 1), hipMemcpyHostToDevice, s));
    if (nnz > 0)
        RSOC_HIP(hipMemcpyAsync(ctx->dci.p, col_idx, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, s));
    o.validate = 0;  // already checked on the host
    int32_t k = run_colouring(ctx, ctx->drp.as<int32_t>(), ctx->dci.as<int32_t>(), n, ctx->dcol.as<int32_t>(), o, stats,
                              s);
    if (k < 0 && k != RSOC_ENOCONV) return k;
    RSOC_HIP(hipMemcpyAsync(colors_out, ctx->dcol.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
    RSOC_HIP(hipStreamSynchronize(s));
    return k;
}

int32_t rsoc_recolor_device(rsoc_ctx *ctx, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t n,
                            int32_t *d_colors_inout, const int32_t *d_touched, int32_t n_touched,
                            const rsoc_options *opts, rsoc_stats *stats, void *hip_stream) {
    if (!ctx || n < 0 || n_touched < 0 || (n > 0 && (!d_row_ptr || !d_colors_inout)) || (n_touched > 0 && !d_touched))
        return RSOC_EINVAL;
    Options o;
    RSOC_TRY(resolve_options(opts, n, o));
    if (two_phase_mode(o.mode)) return RSOC_EINVAL;  // Algorithm 2 recolours all of U: no incremental reading
    if (o.distance == 2) return RSOC_EINVAL;
    RSOC_HIP(hipSetDevice(ctx->device));
    return run_single(ctx, d_row_ptr, d_col_idx, n, d_colors_inout, o, stats, (hipStream_t)hip_stream, d_touched,
                      n_touched);
}

int32_t rsoc_color_classes(rsoc_ctx *ctx, const int32_t *d_colors, int32_t n, int32_t K, int32_t *d_class_ptr,
                           int32_t *d_class_vtx, void *hip_stream) {
    if (!ctx || n < 0 || K < 0 || (n > 0 && K < 1) || !d_class_ptr || (n > 0 && (!d_colors || !d_class_vtx)))
        return RSOC_EINVAL;
    RSOC_HIP(hipSetDevice(ctx->device));
    return run_classes(ctx, d_colors, n, K, d_class_ptr, d_class_vtx, (hipStream_t)hip_stream);
}

int32_t rsoc_color_classes_noalloc(const int32_t *d_colors, int32_t n, int32_t K, int32_t *d_class_ptr,
                                   int32_t *d_class_vtx, void *hip_stream) {
    if (n < 0 || K < 0 || (n > 0 && K < 1) || !d_class_ptr || (n > 0 && (!d_colors || !d_class_vtx)))
        return RSOC_EINVAL;
    return run_classes_noalloc(d_colors, n, K, d_class_ptr, d_class_vtx, (hipStream_t)hip_stream);
}

static std::mutex g_default_mu;
static rsoc_ctx *g_default_ctx = nullptr;

int32_t rsoc_color(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t *colors_out) {
    std::lock_guard<std::mutex> lk(g_default_mu);
    if (!g_default_ctx) RSOC_TRY(rsoc_ctx_create(&g_default_ctx, 0));
    rsoc_options o;
    rsoc_default_options(&o);
    o.validate = RSOC_CHECK_CSR;
    return rsoc_color_ex(g_default_ctx, row_ptr, col_idx, n, colors_out, &o, nullptr);
}

}  // extern "C"
