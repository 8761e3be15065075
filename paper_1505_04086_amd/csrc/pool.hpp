// pool.hpp -- continuous batching (placeholder until the pool lands).
#pragma once
#include "single.hpp"

struct rsoc_pool { int dummy; };

extern "C" {
int32_t rsoc_pool_create(rsoc_ctx *, int64_t, int32_t, rsoc_pool **out) { if (out) *out = nullptr; return RSOC_EINVAL; }
void rsoc_pool_destroy(rsoc_pool *) {}
int32_t rsoc_pool_admit(rsoc_pool *, const int32_t *, const int32_t *, int32_t, int32_t *, const rsoc_options *) { return RSOC_EINVAL; }
int32_t rsoc_pool_step(rsoc_pool *, void *, int32_t *, int32_t) { return RSOC_EINVAL; }
int32_t rsoc_pool_live(const rsoc_pool *) { return 0; }
int64_t rsoc_pool_reserved_bytes(const rsoc_pool *) { return 0; }
int32_t rsoc_pool_result(rsoc_pool *, int32_t, rsoc_stats *) { return RSOC_ENOTFOUND; }
}
