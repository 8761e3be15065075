/*
 * rsoc.h -- C ABI of librsoc: speculative First-Fit graph colouring on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Rokos, Gorman, Kelly, "A Fast and Scalable Graph Coloring Algorithm
 * for Multi-core and Many-core Architectures" (arXiv 1505.04086), Section 3,
 * Algorithm 3 ("RSOC"): a tentative First-Fit round over every vertex, then
 * rounds that each inspect the vertices recoloured in the previous round,
 * recolour the ones that still share a colour with a neighbour they lose to,
 * and collect them for the next round, with one barrier per round, until a
 * round recolours nobody.  The First-Fit step gives a vertex the smallest
 * colour absent among its neighbours (Section 2.1, Algorithm 1).
 *
 * Problem statement (Section 2.1): input an undirected graph G(V,E), output a
 * colour c(v) per vertex such that adjacent vertices differ, plus the number
 * of colours.
 *
 * Conventions shared by every entry point:
 *  - Graph: symmetric CSR, int32.  row_ptr has n+1 entries, row_ptr[0] == 0,
 *    non-decreasing, row_ptr[n] = nnz <= 2^31-1; col_idx has nnz entries in
 *    [0, n).  Both directions of every edge must be present.  Duplicate
 *    entries are harmless.  Self-loops are rejected when validation is on;
 *    otherwise they are ignored.  Rows need not be sorted.
 *  - Colours: int32, 0-based (the paper's palette {1..d+1} shifted down by
 *    one).  Every colour satisfies 0 <= c(v) <= deg(v), hence at most
 *    max-degree + 1 colours (Section 2.1).
 *  - Return value: >= 0 on success (the colour count K = max colour + 1, 0
 *    for n == 0, or the documented value), < 0 an rsoc_status code.
 *  - Ownership: the caller owns every buffer it passes in; the library never
 *    frees or retains caller memory (except pool slots, see below).  A context
 *    owns its device scratch, grows it on demand and frees it at destroy.
 *  - Threading: one host thread at a time per context / pool.  No C++
 *    exception crosses this ABI.
 *  - Streams: entry points taking `hip_stream` (a hipStream_t; NULL = the
 *    default stream) enqueue their kernels there and synchronise it before
 *    returning.
 */
#ifndef RSOC_H
#define RSOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSOC_OK = 0,
    RSOC_EINVAL = -1,     /* null pointer, n < 0, bad option value */
    RSOC_ECSR = -2,       /* row_ptr[0] != 0, decreasing row_ptr, col_idx out of range */
    RSOC_ESELFLOOP = -3,  /* a self-loop, with validation on */
    RSOC_EASYM = -4,      /* an edge stored in one direction only (RSOC_CHECK_SYMMETRY) */
    RSOC_ENOMEM = -5,     /* device or host allocation failed */
    RSOC_EHIP = -6,       /* a HIP runtime error (see rsoc_last_error) */
    RSOC_ENOCONV = -7,    /* the worklist was still non-empty after max_rounds passes */
    RSOC_EBUDGET = -8,    /* pool admission refused: HBM budget or slot table full */
    RSOC_ENOTFOUND = -9,  /* unknown or unfinished pool slot */
    RSOC_EINTERNAL = -10, /* an internal consistency check failed on the device: a colour outside
                             [0, degree], or a worklist / hub list whose size differs from an independent
                             count of the entries it must hold.  Never expected: it signals a defect of the
                             library, not of the input; the colours are then unspecified. */
    RSOC_ESCRATCH = -11   /* the input needs more scratch than the fixed array of a no-allocation entry
                             point holds (see rsoc_color_classes_noalloc); nothing was launched */
} rsoc_status;

typedef enum {
    /* The paper's Algorithm 3 as written: reads see whatever neighbour colours
     * are in memory (live), writes go straight to the colour array.  Any valid
     * colouring is a correct result; it may differ from run to run. */
    RSOC_MODE_OPTIMISTIC = 0,
    /* Algorithm 3 read round-synchronously: every read of a round sees the
     * colours of the previous barrier and every write of the round lands at
     * the next barrier.  Round 0 therefore gives every vertex colour 0.  The
     * result is unique and bit-reproducible. */
    RSOC_MODE_DETERMINISTIC = 1,
    /* Algorithm 2 (Section 2.2, the predecessor scheme): per round a tentative
     * First-Fit over U, a barrier, conflict detection over U into L, a barrier,
     * U <- L.  Round-synchronous reads, so the result is unique. */
    RSOC_MODE_TWO_PHASE = 2,
    /* Algorithm 2 as the paper runs it beside Algorithm 3 (Section 4): the
     * same two phases per round, with live reads and writes straight to the
     * colour array, as RSOC_MODE_OPTIMISTIC does for Algorithm 3; the first
     * round colours all of V, reading every neighbour.  Any valid colouring
     * is a correct result.  rsoc_color_ex / rsoc_color_device only (the
     * batch, the pool and the recolouring return RSOC_EINVAL). */
    RSOC_MODE_TWO_PHASE_LIVE = 3
} rsoc_mode;

typedef enum {
    RSOC_TIE_LOWER_KEEPS = 0,  /* on a conflict the lower vertex id keeps its colour */
    RSOC_TIE_HIGHER_KEEPS = 1  /* the paper's test: V_i is defective if a neighbour V_j > V_i shares its colour */
} rsoc_tie;

enum { RSOC_CHECK_CSR = 1, RSOC_CHECK_SYMMETRY = 2 };

typedef struct {
    int32_t mode;        /* rsoc_mode (default RSOC_MODE_OPTIMISTIC) */
    int32_t tie;         /* rsoc_tie (default RSOC_TIE_LOWER_KEEPS) */
    int32_t max_rounds;  /* bound on inspection passes (rounds >= 1); 0 => n + 1, which no input reaches */
    int32_t validate;    /* bitmask of RSOC_CHECK_*; symmetry is checked only for host-pointer calls */
    /* tuning; 0 selects the library default (or the tuned value) */
    int32_t t_thread;    /* max degree coloured by a group of 8 lanes (<= 32; default 32) */
    int32_t t_wave;      /* max degree coloured by one wavefront; larger rows use a workgroup (default 2048) */
    int32_t grid_thread; /* workgroups given to the thread bin per round launch (default 1024; 4096 for
                          * rsoc_color_batch's optimistic rounds 0 and 1, whose workgroups claim tasks
                          * from counters, so that extra ones only wait) */
    int32_t grid_wave;   /* workgroups given to the wavefront bin (default 2048) */
    int32_t rounds_per_sync; /* rounds enqueued (as one HIP graph) per host check of the worklist (default 4, even) */
    /* rsoc_color_batch: graphs of at most this many vertices (at most 2048;
     * 0 = library default 2048, -1 = none) are coloured by one workgroup each,
     * every round inside it with the workgroup barrier as the round barrier and
     * the colours in LDS, beside the fused launches that take the larger graphs
     * (optimistic and round-synchronous modes; two-phase graphs always take the
     * fused launches).  Round-synchronous results are unchanged (the same
     * schedule); optimistic graphs so coloured run Algorithm 3 as written:
     * round 0 over all neighbours as they stand, round 1 over all of V.
     * Ignored by the other entry points. */
    int32_t small_cutoff;
    int32_t timing;      /* 1: record per-kernel HIP events (fills the ms_* fields of rsoc_stats) */
    /* Optimistic mode only.  0 (default): round 0 gives each vertex the smallest
     * colour absent among the neighbours it loses a tie to (the ones sequential
     * First-Fit in tie order would have coloured first) and collects the
     * vertices that read one of those still uncoloured; round 1 inspects only
     * them, since no other vertex can be defective after round 0.  1: the literal
     * reading: round 0 reads all neighbours and round 1 inspects all of V. */
    int32_t full_sweep;
    /* Optimistic default flow: round 0 also reads neighbours it wins against
     * whose id is within this distance (the sweep may have coloured them
     * already).  0 = library default: none where the ids carry no locality
     * (run length 1), else the ids all workgroups cover in one step; for
     * batches twice that.  -1 = none. */
    int32_t lookahead;
    /* Run of consecutive vertex ids one 8-lane group colours one after the
     * other in sweeps (1, 2, 4 or 8).  0 = chosen per graph from a sample of
     * its rows: 8 when ids carry locality (natural-order meshes, where
     * neighbours coloured at the same instant would conflict), else 1. */
    int32_t chunk;
    /* Workgroups given to the thread bin of worklist rounds (rounds >= 1 over
     * a list; default 1024).  Those rounds are latency-bound chains of
     * dependent loads (list entry, row, neighbour colours), so they want more
     * workgroups in flight than the sweeps. */
    int32_t grid_list;
    /* Optimistic mode: once the worklist holds at most this many vertices
     * (0 = library default 1024, the most allowed; -1 = never) and its last
     * round shrank it by less than half, one round is run as an ordered pass
     * over it -- each vertex detected and recoloured after the ones before
     * it, seeing their new colours -- so that mutually adjacent hubs stop
     * taking the same colour round after round. */
    int32_t tail;
    /* 1 (or 0): colour G; 2: distance-2 colouring, i.e. colour G^2, in which
     * vertices within distance 2 in G are adjacent (Section 6).  G^2 is built
     * on the device (about 4 bytes per entry of G^2, kept by the context) and
     * coloured by the same rounds; statistics (max_degree, bins, bytes)
     * refer to G^2.  Single-graph entry points only (rsoc_color_device,
     * rsoc_color_ex, rsoc_color); needs every 2-hop walk deg(v) + the degrees
     * of v's neighbours <= 8192, n <= 2^26 and G^2 below 2^31 entries, else
     * RSOC_EINVAL. */
    int32_t distance;
    /* Workgroups of the launches that bin the vertices by degree and build
     * list-shaped inputs (a recolouring's first worklist): 0 = library
     * default (1024 for a single graph and a pool slot, up to 8192 for a
     * batch).  Each such workgroup walks its share of the ids and appends to
     * queues in LDS (one per workgroup; one per wavefront in a batch); a small
     * value makes every queue fill and flush many times, which tests use to
     * reach those flushes on small graphs. */
    int32_t grid_bin;
    /* Optimistic mode, default round-0 flow, single-graph entry points: the
     * vertices of degree above this threshold ("hubs"; 0 = library default,
     * max(32, t_thread, max degree / 32); -1 = off; a value below t_thread
     * counts as t_thread) are coloured first, one after another in tie
     * order, each with the smallest colour absent among the hubs coloured
     * before it; round 0 then colours every other vertex reading all of its
     * neighbours, so that none takes a hub's colour and no hub is ever
     * recoloured.  Without it, hubs are coloured at the start of round 0
     * while their neighbours are still uncoloured, and recoloured later
     * against all of them, which on power-law graphs costs hundreds of
     * colours beyond sequential First-Fit.  Skipped (round 0 as without it)
     * when more than 4096 vertices exceed the threshold. */
    int32_t hub_first;
    /* rsoc_color_batch, optimistic round 0: sweep bands per XCD (1 .. 16; 0 =
     * library default).  The fused launches' tasks are cut into 8 x bands
     * ranges of about equal work; each is handed out in order from its own
     * counter, each XCD's workgroups start on its own ranges, and a workgroup
     * whose range is exhausted helps the next ones.  More bands spread the
     * vertices coloured at one instant over more graphs (fewer neighbours
     * read before they are coloured, a shorter round-1 list); fewer keep
     * fewer graphs' colours in each XCD's L2.  Ignored by the other entry
     * points and modes. */
    int32_t bands;
    int32_t reserved; /* must be zero */
} rsoc_options;

typedef struct {
    int32_t rounds;          /* recolouring rounds R: rounds >= 1 that recoloured at least one vertex */
    int32_t passes;          /* inspection passes executed (R, plus the final pass that finds nothing) */
    int32_t colors;          /* K = max colour + 1 */
    int32_t colors_distinct; /* number of distinct colours used (gaps are possible in parallel modes) */
    int64_t conflicts;       /* sum over rounds of |L| (vertices recoloured after round 0) */
    int64_t inspected;       /* vertices inspected in rounds >= 1 */
    int64_t alg_bytes;       /* algorithmic bytes moved by the colouring (model: see the library docs) */
    double ms;               /* device time from the first round-0 kernel to convergence */
    double ms_round0;        /* (timing) duration of the round-0 launch */
    double ms_round1;        /* (timing) duration of the round-1 launch */
    int64_t bytes_round0;    /* algorithmic bytes of the round-0 launch */
    int64_t bytes_round1;    /* algorithmic bytes of the round-1 launch */
    int32_t max_degree;
    int32_t bin_counts[3];   /* vertices per degree bin: thread, wavefront, workgroup */
    int32_t *per_round_L;    /* optional caller array: per_round_L[i] = |L| of recolouring round i+1 */
    int32_t per_round_cap;   /* its length */
    int32_t worklist0;       /* |U^0|: vertices round 1 inspects */
    int32_t chunk;           /* run length used by the sweeps (rsoc_color_batch: 0 when chosen per graph) */
    int32_t small_graphs;    /* rsoc_color_batch: graphs coloured by one workgroup each (small_cutoff) */
    int32_t *per_round_U;    /* optional caller array of per_round_cap entries: per_round_U[i] = |U| of
                                inspection pass i+1 (U^0, then the previous round's L), for the passes run */
} rsoc_stats;

typedef struct rsoc_ctx rsoc_ctx;
typedef struct rsoc_pool rsoc_pool;

/* Fills *opts with the defaults (optimistic mode, lower id keeps). */
void rsoc_default_options(rsoc_options *opts);

/*
 * The problem statement as one call (Section 2.1; Algorithm 3 of Section 3):
 * host arrays in, host colours out, default options, on device 0.  Returns K.
 * Validates the CSR structure and rejects self-loops.
 */
int32_t rsoc_color(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t *colors_out);

/* Creates a context on HIP device `device`.  Returns RSOC_OK or an error. */
int32_t rsoc_ctx_create(rsoc_ctx **out, int32_t device);
void rsoc_ctx_destroy(rsoc_ctx *ctx);

/*
 * Host-pointer colouring with options and statistics (stats may be NULL).
 * Copies the CSR to the device, colours it, copies colours_out back.
 * Returns K.
 */
int32_t rsoc_color_ex(rsoc_ctx *ctx, const int32_t *row_ptr, const int32_t *col_idx, int32_t n,
                      int32_t *colors_out, const rsoc_options *opts, rsoc_stats *stats);

/*
 * Device-pointer colouring (Algorithm 3 on a device-resident graph).
 * d_row_ptr[n+1], d_col_idx[nnz], d_colors_out[n] are device pointers owned
 * by the caller; the kernels run on `hip_stream`, which is synchronised before
 * returning.  d_colors_out is overwritten.  Returns K.
 */
int32_t rsoc_color_device(rsoc_ctx *ctx, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t n,
                          int32_t *d_colors_out, const rsoc_options *opts, rsoc_stats *stats, void *hip_stream);

/*
 * Batched colouring of G independent graphs in one sequence of fused launches.
 * Layout (all device pointers except the offset tables):
 *   vtx_off[G+1], nnz_off[G+1]: host int64 prefix sums of n_g and nnz_g;
 *   d_row_ptr_cat: graph g's local row_ptr (n_g+1 entries, starting at 0)
 *                  begins at element vtx_off[g] + g;
 *   d_col_idx_cat: graph g's local column ids begin at element nnz_off[g];
 *   d_colors_cat:  graph g's colours begin at element vtx_off[g].
 * Each graph is coloured exactly as a separate call would colour it (in
 * deterministic mode bit-identically).  counts_out[g] (host, may be NULL)
 * receives K_g.  Returns max_g K_g.  Sum of n_g must stay below 2^31.
 */
int32_t rsoc_color_batch(rsoc_ctx *ctx, int32_t G, const int64_t *vtx_off, const int64_t *nnz_off,
                         const int32_t *d_row_ptr_cat, const int32_t *d_col_idx_cat, int32_t *d_colors_cat,
                         int32_t *counts_out, const rsoc_options *opts, rsoc_stats *stats, void *hip_stream);

/*
 * Continuous batching.  A pool accepts graphs (already on the device) while
 * others are being coloured; each rsoc_pool_step runs one fused round over all
 * live slots (newly admitted slots run their round 0 in the same launch in
 * which older ones run a later round) and reports the slots that finished.
 * hbm_budget_bytes bounds the device scratch the pool's slots may hold
 * (worklists and staging: about 16 bytes per vertex); 0 means unlimited.
 */
int32_t rsoc_pool_create(rsoc_ctx *ctx, int64_t hbm_budget_bytes, int32_t max_slots, rsoc_pool **out);
void rsoc_pool_destroy(rsoc_pool *pool);
/* Admits a graph: reserves a slot and its scratch and enqueues the slot's
 * set-up on the context's stream (no wait on the device; the next
 * rsoc_pool_step orders itself after it).  The device pointers must stay valid
 * until rsoc_pool_result.  Returns a slot id >= 0, or RSOC_EBUDGET if its
 * scratch does not fit now.  Wrong row_ptr ends (row_ptr[0] != 0 or
 * row_ptr[n] < 0, RSOC_ECSR) and edges without col_idx (RSOC_EINVAL) finish the
 * slot at the next step with that status, returned by rsoc_pool_result. */
int32_t rsoc_pool_admit(rsoc_pool *pool, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t n,
                        int32_t *d_colors_out, const rsoc_options *opts);
/* Admits a recolouring after topology edits (as rsoc_recolor_device: the
 * colouring before the edits in d_colors_inout, negative = none, the touched
 * vertices in d_touched[n_touched], which may repeat ids): the slot starts
 * with Algorithm 3's worklist rounds over U^0 = the touched vertices plus
 * those without a valid First-Fit colour, in the same fused rounds as the
 * other slots.  d_touched must stay valid until the next rsoc_pool_step
 * returns, the other pointers until rsoc_pool_result.  Modes as for
 * rsoc_recolor_device.  Returns a slot id, RSOC_EBUDGET or RSOC_EINVAL; a
 * touched id outside [0, n) finishes the slot with RSOC_EINVAL (returned by
 * rsoc_pool_result). */
int32_t rsoc_pool_admit_recolor(rsoc_pool *pool, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t n,
                                int32_t *d_colors_inout, const int32_t *d_touched, int32_t n_touched,
                                const rsoc_options *opts);
/* One fused round over all live slots on hip_stream (synchronised).  Writes up
 * to `cap` finished slot ids to finished_slots.  Returns the number finished
 * (they stay reserved until rsoc_pool_result), or RSOC_EINVAL while a step
 * launched by rsoc_pool_step_launch is not finished. */
int32_t rsoc_pool_step(rsoc_pool *pool, void *hip_stream, int32_t *finished_slots, int32_t cap);
/* rsoc_pool_step in two halves, for a caller that overlaps host work with the
 * round (Section 3: one barrier per round is the method's synchronisation;
 * here the host's wait for it is deferred).  rsoc_pool_step_launch enqueues
 * the round on hip_stream and returns without waiting for it (it may wait for
 * a pending admission's set-up when no slot is running).  Until
 * rsoc_pool_step_finish, the pool accepts rsoc_pool_admit,
 * rsoc_pool_admit_recolor, rsoc_pool_result (of slots reported by earlier
 * steps), rsoc_pool_live and rsoc_pool_reserved_bytes; another launch or
 * rsoc_pool_step returns RSOC_EINVAL.  Slots admitted meanwhile join a later
 * step.  rsoc_pool_step_finish waits for the launched round and reports
 * finished slots as rsoc_pool_step does; without a launched step it returns
 * RSOC_EINVAL.  Both return RSOC_EHIP on a HIP failure. */
int32_t rsoc_pool_step_launch(rsoc_pool *pool, void *hip_stream);
int32_t rsoc_pool_step_finish(rsoc_pool *pool, int32_t *finished_slots, int32_t cap);
/* Number of admitted slots that are not yet released. */
int32_t rsoc_pool_live(const rsoc_pool *pool);
/* Scratch bytes currently reserved by admitted slots. */
int64_t rsoc_pool_reserved_bytes(const rsoc_pool *pool);
/* Statistics of a finished slot (stats may be NULL); releases the slot and
 * its budget.  Returns K, the slot's error status, or RSOC_ENOTFOUND when the
 * slot is not a finished one.  Enqueues no device work that it waits for. */
int32_t rsoc_pool_result(rsoc_pool *pool, int32_t slot, rsoc_stats *stats);

/*
 * Recolouring after topology edits (Section 1: graphs whose topology changes
 * between colourings, as in morph kernels and mesh adaptivity, are recoloured
 * in every iteration).  Device pointers as for rsoc_color_device, on the
 * edited graph.  d_colors_inout[n] holds the colouring from before the edits
 * (negative: no colour yet, e.g. a new vertex) and receives the result.
 * d_touched[n_touched] (device, may repeat ids) lists the vertices the edits
 * touched: both endpoints of every inserted edge (deletions create no
 * conflict).  Algorithm 3's rounds then run from that state, with
 * U^0 = the touched vertices plus every vertex whose colour is negative or
 * above its degree, such a vertex counting as defective; no round 0.  Modes
 * RSOC_MODE_OPTIMISTIC (any valid colouring) and RSOC_MODE_DETERMINISTIC
 * (round-synchronous: identical to the reference schedule); two-phase is
 * RSOC_EINVAL.  Options and statistics as for rsoc_color_device (worklist0 =
 * |U^0|; ms_round0/ms_round1 are not measured).  Synchronises hip_stream.
 * Returns K, or RSOC_EINVAL (also for a touched id outside [0, n), found on
 * the device), RSOC_ECSR, RSOC_ENOCONV, RSOC_EHIP.
 */
int32_t rsoc_recolor_device(rsoc_ctx *ctx, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t n,
                            int32_t *d_colors_inout, const int32_t *d_touched, int32_t n_touched,
                            const rsoc_options *opts, rsoc_stats *stats, void *hip_stream);

/*
 * Colour classes (Section 1: a colouring splits the vertices into independent
 * sets, one per colour, whose members can be processed concurrently).
 * d_colors[n]: device int32 colours in [0, K) (K = the count rsoc_color_*
 * returns, or any larger palette size).  Outputs, device and caller-owned:
 * d_class_ptr[K+1] and d_class_vtx[n]; class k is
 * d_class_vtx[d_class_ptr[k] .. d_class_ptr[k+1]), in ascending vertex id
 * (unused colours give empty classes).  Runs on hip_stream and synchronises
 * it; its scratch (4 bytes per colour and 1024 vertices, at most 2 bytes per
 * vertex) is the context's.
 * Returns RSOC_OK, or RSOC_EINVAL for null pointers, n < 0, K < 0, K = 0 with
 * n > 0, or a colour outside [0, K) (found on the device; the outputs are then
 * unspecified).
 */
int32_t rsoc_color_classes(rsoc_ctx *ctx, const int32_t *d_colors, int32_t n, int32_t K, int32_t *d_class_ptr,
                           int32_t *d_class_vtx, void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the colour
 * classes of rsoc_color_classes, with identical arguments and results, but
 * without a context and without any allocation.  Its scratch is one fixed
 * device array of 4,195,584 bytes per GPU (a count table of 2^20 entries, the
 * scan sums and the state), created with the library and held until the
 * process ends.  It runs on the current HIP device (hipSetDevice), on
 * hip_stream, which must belong to that device and is synchronised before
 * returning.  Every call on one GPU uses that GPU's array: calls that overlap
 * on one GPU (other streams or host threads) race and must not be issued.
 * Each call re-initialises what it reads, so consecutive calls need nothing
 * cleared.  Returns RSOC_OK, RSOC_EINVAL as rsoc_color_classes, or
 * RSOC_ESCRATCH when n > 2^30 (the count table must hold one colour's counts
 * for every 1024 vertices); nothing is launched then.
 */
int32_t rsoc_color_classes_noalloc(const int32_t *d_colors, int32_t n, int32_t K, int32_t *d_class_ptr,
                                   int32_t *d_class_vtx, void *hip_stream);

/* Host-side CSR check (flags: RSOC_CHECK_*).  Returns RSOC_OK or the first error found. */
int32_t rsoc_check_csr(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t flags);

/* Static string for a status code. */
const char *rsoc_strerror(int32_t status);

/* Text of the last HIP error seen on this host thread ("" if none). */
const char *rsoc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RSOC_H */
