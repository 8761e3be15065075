/*
 * omp_rsoc.c -- Algorithm 3 (Section 3, "RSOC") on the host's cores with
 * OpenMP: the paper's own setting (multi-core CPUs, one barrier per round).
 * TEST INFRASTRUCTURE ONLY: the benchmark times it as a CPU baseline and the
 * tests pin it; nothing in the GPU library calls it, and it shares no code
 * with the GPU library or with oracle.c.
 *
 * Paper: Rokos, Gorman, Kelly, "A Fast and Scalable Graph Coloring Algorithm
 * for Multi-core and Many-core Architectures" (arXiv 1505.04086).
 *
 * What it computes, in the paper's order:
 *  - round 0: every vertex, in a parallel loop, takes the smallest colour
 *    absent among its neighbours that are coloured when it reads them (live
 *    reads: another thread may be colouring a neighbour at the same moment;
 *    an uncoloured neighbour is -1 and is ignored);
 *  - U^0 = V; then, while U is not empty, a parallel loop over U: a vertex
 *    with a neighbour it loses to (the tie rule) holding its colour takes the
 *    smallest colour absent among all of its neighbours, read live, and joins
 *    the recoloured list L (each thread fills its own part of L, and the parts
 *    are joined after the loop's barrier); U <- L.
 * Colours are read and written with relaxed atomic operations (the live reads
 * of the optimistic scheme, without data races in the C sense).
 *
 * With one thread, round 0 visits the vertices in natural order, so it is
 * Algorithm 1 (Section 2.1) and round 1 finds nothing to recolour: the result
 * equals sequential First-Fit.
 *
 * Returns K = max colour + 1 (0 for n = 0), or -1 bad argument, -5 out of
 * memory, -7 when max_rounds passes did not empty the worklist.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int32_t ld(const int32_t *p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
static void st(int32_t *p, int32_t x) { __atomic_store_n(p, x, __ATOMIC_RELAXED); }

/* Smallest colour absent among v's neighbours (self-loops skipped; only
 * colours <= deg(v) can block it).  mark[] belongs to the calling thread and
 * holds stamps: colour c is taken iff mark[c] == stamp. */
static int32_t first_fit(int32_t v, const int32_t *rp, const int32_t *ci, int32_t *col, int32_t *mark,
                         int32_t stamp) {
    const int32_t b = rp[v], e = rp[v + 1], d = e - b;
    for (int32_t k = b; k < e; ++k) {
        const int32_t u = ci[k];
        if (u == v) continue;
        const int32_t c = ld(&col[u]);
        if (c >= 0 && c <= d) mark[c] = stamp;
    }
    int32_t m = 0;
    while (mark[m] == stamp) ++m;
    return m;
}

int32_t omp_rsoc(int32_t n, const int32_t *rp, const int32_t *ci, int32_t tie, int32_t threads, int32_t max_rounds,
                 int32_t *col, int32_t *rounds_out, int64_t *conflicts_out) {
    if (n < 0 || (n > 0 && (!rp || !col)) || (tie != 0 && tie != 1) || threads < 1) return -1;
    if (rounds_out) *rounds_out = 0;
    if (conflicts_out) *conflicts_out = 0;
    if (n == 0) return 0;
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; ++v)
        if (rp[v + 1] - rp[v] > maxd) maxd = rp[v + 1] - rp[v];
    int32_t *U = malloc(sizeof(int32_t) * (size_t)n);
    int32_t *L = malloc(sizeof(int32_t) * (size_t)n);
    int32_t *marks = malloc(sizeof(int32_t) * (size_t)threads * (size_t)(maxd + 2));
    int64_t *part = malloc(sizeof(int64_t) * (size_t)(threads + 1));
    if (!U || !L || !marks || !part) {
        free(U), free(L), free(marks), free(part);
        return -5;
    }
    for (int64_t i = 0; i < (int64_t)threads * (maxd + 2); ++i) marks[i] = -1;
    for (int32_t v = 0; v < n; ++v) col[v] = -1;
    int32_t m = n, rounds = 0, passes = 0, status = 0;
    int64_t conflicts = 0;
#pragma omp parallel num_threads(threads)
    {
        const int tid = omp_get_thread_num();
        const int nt = omp_get_num_threads();
        int32_t *mark = marks + (size_t)tid * (size_t)(maxd + 2);
        int32_t stamp = 0;
        /* round 0 */
#pragma omp for schedule(static)
        for (int32_t v = 0; v < n; ++v) st(&col[v], first_fit(v, rp, ci, col, mark, stamp++));
#pragma omp for schedule(static)
        for (int32_t v = 0; v < n; ++v) U[v] = v;
        /* rounds over the worklist; the loop condition is read after a barrier */
        for (;;) {
#pragma omp barrier
            if (m == 0 || status) break;
            /* this thread's share of U (contiguous, as a static schedule), its
             * recoloured vertices collected in order at the front of it */
            const int64_t lo = (int64_t)m * tid / nt, hi = (int64_t)m * (tid + 1) / nt;
            int64_t cnt = 0;
            for (int64_t i = lo; i < hi; ++i) {
                const int32_t v = U[i];
                const int32_t cv = ld(&col[v]);
                int defective = 0;
                for (int32_t k = rp[v]; k < rp[v + 1] && !defective; ++k) {
                    const int32_t u = ci[k];
                    if (u == v) continue;
                    const int loses = tie == 0 ? (u < v) : (u > v);
                    if (loses && ld(&col[u]) == cv) defective = 1;
                }
                if (defective) {
                    st(&col[v], first_fit(v, rp, ci, col, mark, stamp++));
                    L[lo + cnt++] = v;
                }
            }
            part[tid] = cnt;
#pragma omp barrier
#pragma omp single
            {
                int64_t tot = 0;
                for (int t = 0; t < nt; ++t) tot += part[t];
                ++passes;
                if (tot) ++rounds;
                conflicts += tot;
                /* L's parts, joined: U <- L */
                int64_t o = 0;
                for (int t = 0; t < nt; ++t) {
                    const int64_t plo = (int64_t)m * t / nt;
                    memcpy(U + o, L + plo, sizeof(int32_t) * (size_t)part[t]);
                    o += part[t];
                }
                m = (int32_t)tot;
                if (m && max_rounds > 0 && passes >= max_rounds) status = -7;
            }
        }
    }
    int32_t K = 0;
    for (int32_t v = 0; v < n; ++v)
        if (col[v] + 1 > K) K = col[v] + 1;
    free(U), free(L), free(marks), free(part);
    if (rounds_out) *rounds_out = rounds;
    if (conflicts_out) *conflicts_out = conflicts;
    return status ? status : K;
}
