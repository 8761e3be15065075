// pool.hpp -- continuous batching: graphs are admitted into slots while others
// are being coloured; every rsoc_pool_step is one fused round over all live
// slots.  Slot scratch (worklists, hub lists, colour shadow, staging) comes
// from an arena sized by the HBM budget; admission is refused with
// RSOC_EBUDGET when it does not fit.
//
// The host waits on the device once per step, never per request:
// admission only enqueues the slot's set-up (k_pinit, and the hub-first pass
// of an optimistic slot) on one of kAdmitStreams admission streams, in turn,
// and records the slot's own event; a step takes in the new slots whose
// set-up has completed (one look at their downloaded state) and leaves the
// others for a later step, so a long set-up (the hub walk of a large
// power-law graph is one workgroup's sequential work) neither holds up the
// rounds of the slots already running nor the set-up of the next requests,
// which proceed on the other streams.  A step enqueues, behind its round,
// the colour counts of the slots the round finishes (kernels that skip the
// others) and one download of the slot table; taking a result then needs no
// device work at all.  The step is split in two (rsoc_pool_step_launch,
// rsoc_pool_step_finish) so that a caller can admit the next graphs while
// the round runs.  Releases go on the context's own stream and record
// p->ev, which admissions and steps wait for before touching the slot table.
#pragma once

#include <map>
#include <vector>

#include "pool_kernels.hpp"
#include "single.hpp"

struct rsoc_pool {
    rsoc_ctx *ctx = nullptr;
    int64_t budget = 0;    // 0: unlimited (per-slot hipMalloc)
    int64_t reserved = 0;  // scratch bytes held by admitted slots
    int max_slots = 0;
    rsoc::DevBuf slots_dev, tasks_dev, active_dev, arena;
    rsoc::HostPinned mirror, active_host;
    std::map<int64_t, int64_t> free_blocks;  // arena offset -> size
    struct Alloc {
        int64_t off = -1, bytes = 0;
        void *own = nullptr;  // per-slot allocation when the pool has no arena
    };
    std::vector<Alloc> allocs;
    std::vector<char> reported;  // finished slot already returned by a step
    std::vector<char> pending;   // admitted, set-up enqueued, host fields not yet final
    hipEvent_t ev = nullptr;     // recorded after release work on the context's stream
    rsoc::HostPinned stage;      // step download of all slots (copied into the mirror for active ones)
    // admission streams, each with the workspace of the hub-first pass it runs
    // (hub_kernels.hpp; admissions on one stream run one after another)
    static constexpr int kAdmitStreams = 8;
    hipStream_t astream[kAdmitStreams] = {};
    rsoc::DevBuf hub_args[kAdmitStreams], hub_state[kAdmitStreams], hubs[kAdmitStreams];
    int next_astream = 0;
    std::vector<hipEvent_t> slot_ev;  // recorded after a slot's set-up
    // task-table descriptors of a step (PoolDeal[24], then the spans)
    rsoc::DevBuf deal_dev;
    rsoc::HostPinned deal_host;
    // a step launched by rsoc_pool_step_launch and not yet finished: its
    // stream and its number of active slots (listed in active_host)
    bool inflight = false;
    hipStream_t inflight_s = nullptr;
    int inflight_nact = 0;
};

namespace rsoc {

constexpr int64_t kPoolAlign = 256;

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// two worklists, two hub lists, the byte shadow, then the 4-bit shadow and
// round 0's kept neighbours (optimistic) or the staged colours
// (round-synchronous)
inline int64_t pool_slot_bytes(int64_t n, int mode) {
    const int64_t l = align_up(4 * (n + 1), kPoolAlign);
    return 4 * l + align_up(n + 64, kPoolAlign) +
           (mode == kOptimistic ? align_up(4 * (n / 8 + 2), kPoolAlign) + align_up(16 * (n + 2), kPoolAlign) : l);
}

inline int64_t arena_alloc(rsoc_pool *p, int64_t bytes) {
    for (auto it = p->free_blocks.begin(); it != p->free_blocks.end(); ++it) {
        if (it->second >= bytes) {
            const int64_t off = it->first, sz = it->second;
            p->free_blocks.erase(it);
            if (sz > bytes) p->free_blocks[off + bytes] = sz - bytes;
            return off;
        }
    }
    return -1;
}

inline void arena_free(rsoc_pool *p, int64_t off, int64_t bytes) {
    auto it = p->free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != p->free_blocks.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        p->free_blocks.erase(nx);
    }
    if (it != p->free_blocks.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            p->free_blocks.erase(it);
        }
    }
}

inline PoolSlot *pool_mirror(rsoc_pool *p) { return p->mirror.as<PoolSlot>(); }

inline int32_t pool_upload_slot(rsoc_pool *p, int slot, hipStream_t s) {
    RSOC_HIP(hipMemcpyAsync(p->slots_dev.as<PoolSlot>() + slot, pool_mirror(p) + slot, sizeof(PoolSlot),
                            hipMemcpyHostToDevice, s));
    return RSOC_OK;
}

inline int32_t pool_download_slot(rsoc_pool *p, int slot, hipStream_t s) {
    RSOC_HIP(hipMemcpyAsync(pool_mirror(p) + slot, p->slots_dev.as<PoolSlot>() + slot, sizeof(PoolSlot),
                            hipMemcpyDeviceToHost, s));
    return RSOC_OK;
}

inline void pool_release(rsoc_pool *p, int slot) {
    rsoc_pool::Alloc &a = p->allocs[slot];
    if (a.own) (void)hipFree(a.own);
    if (a.off >= 0) arena_free(p, a.off, a.bytes);
    p->reserved -= a.bytes;
    a = rsoc_pool::Alloc();
    PoolSlot &m = pool_mirror(p)[slot];
    memset(&m, 0, sizeof(m));
    m.phase = kSlotFree;
}

}  // namespace rsoc

extern "C" {

int32_t rsoc_pool_create(rsoc_ctx *ctx, int64_t hbm_budget_bytes, int32_t max_slots, rsoc_pool **out) {
    using namespace rsoc;
    if (!out) return RSOC_EINVAL;
    *out = nullptr;
    if (!ctx || hbm_budget_bytes < 0 || max_slots <= 0 || max_slots > 65536) return RSOC_EINVAL;
    RSOC_HIP(hipSetDevice(ctx->device));
    rsoc_pool *p = new (std::nothrow) rsoc_pool();
    if (!p) return RSOC_ENOMEM;
    p->ctx = ctx;
    p->budget = hbm_budget_bytes;
    p->max_slots = max_slots;
    p->allocs.resize((size_t)max_slots);
    p->reported.assign((size_t)max_slots, 0);
    p->pending.assign((size_t)max_slots, 0);
    int32_t r = RSOC_OK;
    p->slot_ev.assign((size_t)max_slots, nullptr);
    bool ok = hipEventCreateWithFlags(&p->ev, hipEventDisableTiming) == hipSuccess;
    if (!ok) p->ev = nullptr;
    for (auto &e : p->slot_ev)
        if (ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) e = nullptr, ok = false;
    for (auto &st : p->astream)
        if (ok && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr, ok = false;
    if (!ok) {
        rsoc_pool_destroy(p);
        return RSOC_EHIP;
    }
    if ((r = p->slots_dev.reserve(sizeof(PoolSlot) * (size_t)max_slots)) < 0 ||
        (r = p->mirror.reserve(sizeof(PoolSlot) * (size_t)max_slots)) < 0 ||
        (r = p->stage.reserve(sizeof(PoolSlot) * (size_t)max_slots)) < 0 ||
        (r = p->active_dev.reserve(sizeof(int32_t) * (size_t)max_slots)) < 0 ||
        (r = p->active_host.reserve(sizeof(int32_t) * (size_t)max_slots)) < 0 ||
        (hbm_budget_bytes > 0 && (r = p->arena.reserve((size_t)hbm_budget_bytes)) < 0)) {
        rsoc_pool_destroy(p);
        return r;
    }
    memset(p->mirror.p, 0, sizeof(PoolSlot) * (size_t)max_slots);
    if (hbm_budget_bytes > 0) p->free_blocks[0] = hbm_budget_bytes;
    hipError_t e = hipMemcpy(p->slots_dev.p, p->mirror.p, sizeof(PoolSlot) * (size_t)max_slots, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        rsoc_pool_destroy(p);
        return hip_fail(e, "hipMemcpy", __FILE__, __LINE__);
    }
    *out = p;
    return RSOC_OK;
}

void rsoc_pool_destroy(rsoc_pool *p) {
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    for (auto &a : p->allocs)
        if (a.own) (void)hipFree(a.own);
    if (p->ev) (void)hipStreamSynchronize(p->ctx->own);
    for (auto &st : p->astream)
        if (st) (void)hipStreamSynchronize(st);
    if (p->inflight && p->inflight_nact > 0) (void)hipStreamSynchronize(p->inflight_s);
    for (rsoc::DevBuf *b : {&p->slots_dev, &p->tasks_dev, &p->active_dev, &p->deal_dev, &p->arena}) b->release();
    for (int k = 0; k < rsoc_pool::kAdmitStreams; ++k) {
        p->hub_args[k].release();
        p->hub_state[k].release();
        p->hubs[k].release();
    }
    for (rsoc::HostPinned *b : {&p->mirror, &p->deal_host, &p->active_host, &p->stage}) b->release();
    if (p->ev) (void)hipEventDestroy(p->ev);
    for (auto &e : p->slot_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &st : p->astream)
        if (st) (void)hipStreamDestroy(st);
    delete p;
}

namespace rsoc {

// Admission of a colouring (recolor = false) or of a recolouring after edits
// (col holds the colouring before the edits, touched[0, nt) the touched
// vertices): the slot starts with its round 0, or straight with worklist
// rounds over U^0.
inline int32_t pool_admit(rsoc_pool *p, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t n,
                          int32_t *d_colors_out, const rsoc_options *opts, bool recolor, const int32_t *d_touched,
                          int32_t nt) {
    if (!p || n < 0 || (n > 0 && (!d_row_ptr || !d_colors_out)) || nt < 0 || (nt > 0 && !d_touched))
        return RSOC_EINVAL;
    Options o;
    RSOC_TRY(resolve_options(opts, n, o));
    if (two_phase_mode(o.mode)) return RSOC_EINVAL;  // the pool runs Algorithm 3 only
    if (o.distance == 2) return RSOC_EINVAL;                // distance 2: single-graph entry points only
    rsoc_ctx *c = p->ctx;
    RSOC_HIP(hipSetDevice(c->device));
    int slot = -1;
    for (int i = 0; i < p->max_slots; ++i)
        if (pool_mirror(p)[i].phase == kSlotFree) { slot = i; break; }
    if (slot < 0) return RSOC_EBUDGET;
    const int64_t bytes = pool_slot_bytes(n, o.mode);
    rsoc_pool::Alloc al;
    al.bytes = bytes;
    char *base = nullptr;
    if (p->budget > 0) {
        if (p->reserved + bytes > p->budget) return RSOC_EBUDGET;
        al.off = arena_alloc(p, bytes);
        if (al.off < 0) return RSOC_EBUDGET;  // fragmented: wait for releases
        base = p->arena.as<char>() + al.off;
    } else {
        hipError_t e = hipMalloc(&al.own, (size_t)bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc", __FILE__, __LINE__);
        base = static_cast<char *>(al.own);
    }
    p->allocs[slot] = al;
    p->reserved += bytes;
    // the slot's set-up runs on the next admission stream, after the release
    // work on the context's stream (the slot table entry it overwrites)
    const int as = p->next_astream;
    p->next_astream = (p->next_astream + 1) % rsoc_pool::kAdmitStreams;
    hipStream_t s = p->astream[as];
    if (hipStreamWaitEvent(s, p->ev, 0) != hipSuccess) {
        pool_release(p, slot);
        return RSOC_EHIP;
    }
    int32_t r = RSOC_OK;
    const int64_t l = align_up(4 * (int64_t)(n + 1), kPoolAlign);
    PoolSlot &m = pool_mirror(p)[slot];
    memset(&m, 0, sizeof(m));
    m.rp = d_row_ptr;
    m.ci = d_col_idx;
    m.col = d_colors_out;
    m.wl[0] = reinterpret_cast<int32_t *>(base);
    m.wl[1] = reinterpret_cast<int32_t *>(base + l);
    m.hubW = reinterpret_cast<int32_t *>(base + 2 * l);
    m.hubB = reinterpret_cast<int32_t *>(base + 3 * l);
    m.col8 = reinterpret_cast<uint8_t *>(base + 4 * l);
    char *tail = base + 4 * l + align_up(n + 64, kPoolAlign);
    m.pend = o.mode == kOptimistic ? nullptr : reinterpret_cast<int32_t *>(tail);
    m.col4 = o.mode == kOptimistic ? reinterpret_cast<uint32_t *>(tail) : nullptr;
    m.aux = o.mode == kOptimistic ? reinterpret_cast<int4 *>(tail + align_up(4 * (n / 8 + 2), kPoolAlign)) : nullptr;
    m.n = n;
    m.mode = o.mode;
    m.tie = o.tie;
    m.max_rounds = o.max_rounds;
    m.t_thread = o.t_thread;
    m.t_wave = o.t_wave;
    m.look = o.lookahead == -1 ? 0 : (o.lookahead > 0 ? o.lookahead : (1 << 20));
    m.phase = n > 0 ? (recolor ? kSlotRunning : kSlotNew) : kSlotDone;  // nothing to colour: done at once
    m.chunk = recolor ? 1 : o.chunk;  // 0: chosen from the locality sample when the set-up is seen
    m.recolor = recolor ? 1 : 0;
    m.touched = d_touched;
    m.nt = recolor ? nt : 0;
    m.hub_opt = (o.mode == kOptimistic && !recolor) ? o.hub_first : 0;
    if (m.hub_opt != 0 && n > 0) {
        const size_t had = p->hubs[as].bytes;
        if ((r = p->hub_args[as].reserve(sizeof(SingleArgs))) < 0 ||
            (r = p->hub_state[as].reserve(sizeof(SingleState))) < 0 || (r = p->hubs[as].reserve(kHubBytes)) < 0) {
            pool_release(p, slot);
            return r;
        }
        // the hub bit sets and the state's counts are zero between admissions
        // (k_hub_ff clears what it reads and resets the counts)
        if (p->hubs[as].bytes != had &&
            (hipMemsetAsync(p->hubs[as].p, 0, p->hubs[as].bytes, s) != hipSuccess ||
             hipMemsetAsync(p->hub_state[as].p, 0, p->hub_state[as].bytes, s) != hipSuccess)) {
            pool_release(p, slot);
            return RSOC_EHIP;
        }
    }
    p->reported[slot] = 0;
    if ((r = pool_upload_slot(p, slot, s)) < 0) { pool_release(p, slot); return r; }
    if (n > 0) {
        const int gbin = std::min(div_up(n, kBlock), o.grid_bin ? o.grid_bin : 1024);
        k_pinit<<<gbin, kBlock, 0, s>>>(p->slots_dev.as<PoolSlot>(), slot);
        if (m.hub_opt != 0) {
            SingleArgs *A = p->hub_args[as].as<SingleArgs>();
            SingleState *S = p->hub_state[as].as<SingleState>();
            PoolSlot *sd = p->slots_dev.as<PoolSlot>();
            int32_t *done = &sd[slot].nH;  // nH, hub_t: adjacent fields of the slot
            k_phub_collect<<<gbin, kBlock, 0, s>>>(sd, slot, A, S, p->hubs[as].as<int32_t>());
            k_hub_sort<<<1, kHubSortBlock, 0, s>>>(A, S);
            if (o.tie) {
                k_hub_lists<kHigherKeeps><<<kHubListGrid, kBlock, 0, s>>>(A, S);
                k_hub_ff<kHigherKeeps><<<1, kHubFfBlock, 0, s>>>(A, S, done);
            } else {
                k_hub_lists<kLowerKeeps><<<kHubListGrid, kBlock, 0, s>>>(A, S);
                k_hub_ff<kLowerKeeps><<<1, kHubFfBlock, 0, s>>>(A, S, done);
            }
        }
        if (recolor) {
            if (nt > 0) k_ptouch<<<std::min(div_up(nt, kBlock), 256), kBlock, 0, s>>>(p->slots_dev.as<PoolSlot>(), slot);
            k_plist<<<gbin, kBlock, 0, s>>>(p->slots_dev.as<PoolSlot>(), slot);
        }
        k_pready<<<1, 1, 0, s>>>(p->slots_dev.as<PoolSlot>(), slot);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { pool_release(p, slot); return hip_fail(e, "k_pinit", __FILE__, __LINE__); }
        if ((r = pool_download_slot(p, slot, s)) < 0) { pool_release(p, slot); return r; }
    }
    // the slot is taken in by the first step that finds this event complete
    p->pending[slot] = 1;
    RSOC_HIP(hipEventRecord(p->slot_ev[slot], s));
    return slot;
}

}  // namespace rsoc

int32_t rsoc_pool_admit(rsoc_pool *p, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t n,
                        int32_t *d_colors_out, const rsoc_options *opts) {
    return rsoc::pool_admit(p, d_row_ptr, d_col_idx, n, d_colors_out, opts, false, nullptr, 0);
}

int32_t rsoc_pool_admit_recolor(rsoc_pool *p, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t n,
                                int32_t *d_colors_inout, const int32_t *d_touched, int32_t n_touched,
                                const rsoc_options *opts) {
    return rsoc::pool_admit(p, d_row_ptr, d_col_idx, n, d_colors_inout, opts, true, d_touched, n_touched);
}

int32_t rsoc_pool_step_launch(rsoc_pool *p, void *hip_stream) {
    using namespace rsoc;
    if (!p || p->inflight) return RSOC_EINVAL;
    rsoc_ctx *c = p->ctx;
    RSOC_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    PoolSlot *m = pool_mirror(p);
    // release work on the context's stream comes first
    RSOC_HIP(hipStreamWaitEvent(s, p->ev, 0));
    // new slots whose set-up has completed (their state downloaded) join this
    // step; when no slot is running, the step waits for the earliest pending one
    bool any_running = false;
    int first_pending = -1;
    for (int i = 0; i < p->max_slots; ++i) {
        if (p->pending[i]) {
            if (first_pending < 0) first_pending = i;
        } else if (m[i].phase == kSlotNew || m[i].phase == kSlotRunning) {
            any_running = true;
        }
    }
    if (first_pending >= 0) {
        if (!any_running) RSOC_HIP(hipEventSynchronize(p->slot_ev[first_pending]));
        for (int i = 0; i < p->max_slots; ++i) {
            if (!p->pending[i]) continue;
            const hipError_t q = hipEventQuery(p->slot_ev[i]);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return hip_fail(q, "hipEventQuery", __FILE__, __LINE__);
            // the set-up finished the slot's state on the device (k_pready)
            // and downloaded it: the mirror entry is final
            p->pending[i] = 0;
        }
    }
    // Spans of the task tables, one table per (kind, tie rule) and bin; a
    // slot's thread-bin items may belong to another kind than its other bins
    // (the masked first worklist round).  Tables are laid out by (kind, tie
    // rule), each with its workgroup-bin tasks, then wavefront-bin, then
    // thread-bin; k_pdeal fills them on the device.
    constexpr int kKinds = 8;  // kind * 2 + tie
    constexpr int kPer[3] = {kPoolTaskB, kPoolTaskW, kPoolTaskT};
    std::vector<PoolSpan> spans[kKinds][3];
    int nact = 0, maxn = 0;
    int32_t *act = p->active_host.as<int32_t>();
    for (int i = 0; i < p->max_slots; ++i) {
        const PoolSlot &sl = m[i];
        if (p->pending[i]) continue;  // set-up still running (its mirror entry may be mid-download)
        if (sl.phase != kSlotNew && sl.phase != kSlotRunning) continue;
        int kind, cnt[3];  // workgroup, wavefront, thread bin
        if (sl.phase == kSlotNew) {
            kind = sl.mode == kOptimistic ? kAssignSweep : kRecolorSweep;
            cnt[2] = sl.n;  // the sweep skips the other bins' vertices
            cnt[1] = sl.nW;
            cnt[0] = sl.nB;
        } else {
            kind = kRecolorList;
            cnt[2] = sl.cnt_in[0];
            cnt[1] = sl.cnt_in[1];
            cnt[0] = sl.cnt_in[2];
        }
        // the thread bin's part of the first worklist round after round 0
        const int kindT = (sl.phase == kSlotRunning && sl.masked) ? kRecolorMasked : kind;
        for (int bin = 0; bin < 3; ++bin) {
            if (cnt[bin] <= 0) continue;
            const int k = (bin == 2 ? kindT : kind) * 2 + sl.tie;
            spans[k][bin].push_back({i, cnt[bin], (int)((cnt[bin] + (int64_t)kPer[bin] - 1) / kPer[bin])});
        }
        act[nact++] = i;
        maxn = std::max(maxn, sl.n);
    }
    p->inflight_nact = nact;
    p->inflight_s = s;
    if (nact == 0) {
        p->inflight = true;
        return RSOC_OK;
    }
    int ndeal = 0, nspan = 0;
    int64_t ntask = 0;
    int tstart[kKinds], tcount[kKinds][3];
    PoolDeal deals[kKinds * 3];
    for (int k = 0; k < kKinds; ++k) {
        tstart[k] = (int)ntask;
        for (int bin = 0; bin < 3; ++bin) {
            int64_t t = 0;
            for (const PoolSpan &e : spans[k][bin]) t += e.ntask;
            tcount[k][bin] = (int)t;
            if (t) deals[ndeal++] = {nspan, (int)spans[k][bin].size(), kPer[bin], k / 2, (int)ntask, (int)t};
            nspan += (int)spans[k][bin].size();
            ntask += t;
        }
    }
    if (ntask > INT32_MAX) return RSOC_EINVAL;  // more tasks than a table indexes (not reachable below 2^31 vertices)
    const size_t deal_bytes = sizeof(PoolDeal) * kKinds * 3;
    RSOC_TRY(p->tasks_dev.reserve(sizeof(PoolTask) * (size_t)std::max<int64_t>(ntask, 1)));
    RSOC_TRY(p->deal_host.reserve(deal_bytes + sizeof(PoolSpan) * (size_t)nspan));
    RSOC_TRY(p->deal_dev.reserve(deal_bytes + sizeof(PoolSpan) * (size_t)nspan));
    char *dh = p->deal_host.as<char>();
    memcpy(dh, deals, sizeof(PoolDeal) * ndeal);
    PoolSpan *sh = reinterpret_cast<PoolSpan *>(dh + deal_bytes);
    for (int k = 0; k < kKinds; ++k)
        for (int bin = 0; bin < 3; ++bin) sh = std::copy(spans[k][bin].begin(), spans[k][bin].end(), sh);
    RSOC_HIP(hipMemcpyAsync(p->deal_dev.p, dh, deal_bytes + sizeof(PoolSpan) * (size_t)nspan, hipMemcpyHostToDevice,
                            s));
    RSOC_HIP(hipMemcpyAsync(p->active_dev.p, act, sizeof(int32_t) * nact, hipMemcpyHostToDevice, s));
    PoolTask *tasks = p->tasks_dev.as<PoolTask>();
    k_pdeal<<<dim3(ndeal, kDealSplit), kDealBlock, 0, s>>>(p->deal_dev.as<PoolDeal>(),
                                         reinterpret_cast<const PoolSpan *>(p->deal_dev.as<char>() + deal_bytes),
                                         tasks);
    // one launch per (kind, tie rule) present; a slot's tasks are all of one
    // kind but the masked round's wavefront/workgroup-bin ones, whose launch
    // comes first (the launches run in stream order; each hub recoloured
    // first reads the thread-bin colours as they stand, so the masked test of
    // those vertices stays sound)
    PoolSlot *sd = p->slots_dev.as<PoolSlot>();
    for (int k = 0; k < kKinds; ++k) {
        const int nb = tcount[k][0], nw = tcount[k][1], nt = tcount[k][2];
        const int gB = std::min(nb, 256);
        const int gW = std::min(nw, 2048);
        // no more thread-bin workgroups than fit on the device at once: the
        // grid-stride walk would otherwise leave the tasks of the ones that
        // wait to the end, out of id order, and round 0 would read many more
        // neighbours uncoloured
        const int gT = std::min(nt, 1024);
        if (gB + gW + gT == 0) continue;
        PoolTask *tk = tasks + tstart[k];
#define RSOC_PSTEP(KD, T) k_pstep<KD, T><<<gB + gW + gT, kBlock, 0, s>>>(sd, tk, nb, nw, nt, gB, gW, gT)
        switch (k) {
            case 0: RSOC_PSTEP(kAssignSweep, kLowerKeeps); break;
            case 1: RSOC_PSTEP(kAssignSweep, kHigherKeeps); break;
            case 2: RSOC_PSTEP(kRecolorSweep, kLowerKeeps); break;
            case 3: RSOC_PSTEP(kRecolorSweep, kHigherKeeps); break;
            case 4: RSOC_PSTEP(kRecolorList, kLowerKeeps); break;
            case 5: RSOC_PSTEP(kRecolorList, kHigherKeeps); break;
            case 6: RSOC_PSTEP(kRecolorMasked, kLowerKeeps); break;
            default: RSOC_PSTEP(kRecolorMasked, kHigherKeeps); break;
        }
#undef RSOC_PSTEP
    }
    const int32_t *ad = p->active_dev.as<int32_t>();
    bool any_staged = false;
    for (int k = 0; k < nact; ++k) any_staged |= m[act[k]].mode != kOptimistic;
    if (any_staged) k_pscatter<<<dim3(64, std::min(nact, 64)), kBlock, 0, s>>>(sd, ad, nact);
    k_pround_end<<<1, 256, 0, s>>>(sd, ad, nact);
    // colour counts of the slots this round finished (the kernels skip the
    // others), then one download of the slot table
    const int gy = std::min(nact, 1024);
    k_pflags_clear<<<dim3(16, gy), kBlock, 0, s>>>(sd, ad, nact);
    k_pcount<<<dim3(std::max(1, std::min(div_up(maxn, kBlock), 128)), gy), kBlock, 0, s>>>(sd, ad, nact);
    k_pdistinct<<<dim3(1, gy), kBlock, 0, s>>>(sd, ad, nact);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) return hip_fail(le, "k_pstep", __FILE__, __LINE__);
    RSOC_HIP(hipMemcpyAsync(p->stage.p, sd, sizeof(PoolSlot) * (size_t)p->max_slots, hipMemcpyDeviceToHost, s));
    p->inflight = true;
    return RSOC_OK;
}

int32_t rsoc_pool_step_finish(rsoc_pool *p, int32_t *finished_slots, int32_t cap) {
    using namespace rsoc;
    if (!p || !p->inflight || cap < 0 || (cap > 0 && !finished_slots)) return RSOC_EINVAL;
    RSOC_HIP(hipSetDevice(p->ctx->device));
    p->inflight = false;
    PoolSlot *m = pool_mirror(p);
    if (p->inflight_nact > 0) {
        RSOC_HIP(hipStreamSynchronize(p->inflight_s));
        // only the slots of this step changed on the device
        const PoolSlot *st = p->stage.as<PoolSlot>();
        const int32_t *act = p->active_host.as<int32_t>();
        for (int k = 0; k < p->inflight_nact; ++k) m[act[k]] = st[act[k]];
    }
    // report finished slots (including ones a previous step could not fit in `cap`)
    int nfin = 0;
    for (int i = 0; i < p->max_slots && nfin < cap; ++i) {
        if (m[i].phase == kSlotDone && !p->reported[i] && !p->pending[i]) {
            p->reported[i] = 1;
            finished_slots[nfin++] = i;
        }
    }
    return nfin;
}

int32_t rsoc_pool_step(rsoc_pool *p, void *hip_stream, int32_t *finished_slots, int32_t cap) {
    if (!p || p->inflight || cap < 0 || (cap > 0 && !finished_slots)) return RSOC_EINVAL;
    RSOC_TRY(rsoc_pool_step_launch(p, hip_stream));
    return rsoc_pool_step_finish(p, finished_slots, cap);
}

int32_t rsoc_pool_live(const rsoc_pool *p) {
    if (!p) return RSOC_EINVAL;
    const rsoc::PoolSlot *m = p->mirror.as<rsoc::PoolSlot>();
    int live = 0;
    for (int i = 0; i < p->max_slots; ++i) live += p->pending[i] || m[i].phase != rsoc::kSlotFree;
    return live;
}

int64_t rsoc_pool_reserved_bytes(const rsoc_pool *p) { return p ? p->reserved : RSOC_EINVAL; }

int32_t rsoc_pool_result(rsoc_pool *p, int32_t slot, rsoc_stats *stats) {
    using namespace rsoc;
    if (!p || slot < 0 || slot >= p->max_slots) return RSOC_ENOTFOUND;
    PoolSlot &m = pool_mirror(p)[slot];
    if (m.phase != kSlotDone || p->pending[slot]) return RSOC_ENOTFOUND;
    rsoc_ctx *c = p->ctx;
    RSOC_HIP(hipSetDevice(c->device));
    if (stats) {
        int32_t *keep = stats->per_round_L, *keepU = stats->per_round_U;
        int32_t cap = stats->per_round_cap;
        memset(stats, 0, sizeof(*stats));
        stats->per_round_L = keep;
        stats->per_round_U = keepU;
        stats->per_round_cap = cap;
        stats->rounds = m.rounds;
        stats->passes = m.passes;
        stats->colors = m.kmax;
        int distinct = m.distinct;
        for (uint32_t w : m.cbits) distinct += __builtin_popcount(w);
        stats->colors_distinct = m.status < 0 ? 0 : distinct;
        stats->conflicts = m.conflicts;
        stats->max_degree = m.maxdeg;
        stats->bin_counts[0] = m.n - m.nW - m.nB;
        stats->bin_counts[1] = m.nW;
        stats->bin_counts[2] = m.nB;
        stats->worklist0 = m.mode == kOptimistic ? m.u0 : m.n;
        stats->chunk = m.chunk;
    }
    const int32_t k = (m.err & 4) ? RSOC_EINTERNAL : (m.status < 0 ? m.status : m.kmax);
    // the freed slot's device copy is refreshed before the next step reads it
    hipStream_t s = c->own;
    pool_release(p, slot);
    RSOC_TRY(pool_upload_slot(p, slot, s));
    RSOC_HIP(hipEventRecord(p->ev, s));
    return k;
}

}  // extern "C"
