/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for speculative
 * First-Fit colouring and the colour classes a colouring defines.  TEST INFRASTRUCTURE ONLY: only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may call it.  It shares no
 * code, header or helper with the GPU library.
 *
 * Paper: Rokos, Gorman, Kelly, "A Fast and Scalable Graph Coloring Algorithm
 * for Multi-core and Many-core Architectures" (arXiv 1505.04086).
 *
 * Conventions (readings of the paper, restated):
 *  - colours are 0-based; the paper's palette {1..d+1} (Section 2.1) maps to
 *    {0..d};
 *  - the "number of colours" returned is K = max colour + 1 (0 for n = 0);
 *  - self-loops (u == v) are skipped wherever a row is scanned;
 *  - the graph is undirected and given as symmetric CSR; duplicates are
 *    harmless;
 *  - tie rule: TIE_LOWER_KEEPS marks v defective when a LOWER-id neighbour
 *    shares its colour (the lower id keeps its colour); TIE_HIGHER_KEEPS is
 *    the paper's own test (Algorithms 2 and 3 mark V_i when a neighbour
 *    V_j > V_i has the same colour, so the higher id keeps its colour);
 *    TIE_NONE drops the id test (both endpoints recolour), which is the
 *    scheme of the livelock example in Section 5 / Figure 7 and exists only
 *    to exercise the max_rounds guard.
 *
 * All routines return >= 0 on success and a negative code on error:
 *   -1 bad argument, -5 out of memory, -7 max_rounds reached before the
 *   worklist emptied.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { TIE_LOWER_KEEPS = 0, TIE_HIGHER_KEEPS = 1, TIE_NONE = 2 };
enum { ORC_EINVAL = -1, ORC_ENOMEM = -5, ORC_ENOCONV = -7 };

/* Smallest colour k >= 0 not in { col[u] : u in adj(v), u != v, col[u] >= 0 }.
 * `seen` is a zeroed scratch array of at least deg(v)+1 bytes; it is left
 * zeroed on return.  Only colours <= deg(v) can block the answer, because
 * deg(v) neighbours can occupy at most deg(v) of the values 0..deg(v). */
static int32_t smallest_free_colour(int32_t v, const int32_t *row_ptr, const int32_t *col_idx,
                                    const int32_t *col, unsigned char *seen) {
    int32_t b = row_ptr[v], e = row_ptr[v + 1];
    int32_t d = e - b;
    for (int32_t k = b; k < e; ++k) {
        int32_t u = col_idx[k];
        if (u == v) continue;
        int32_t cu = col[u];
        if (cu >= 0 && cu <= d) seen[cu] = 1;
    }
    int32_t m = 0;
    while (seen[m]) ++m;
    for (int32_t k = b; k < e; ++k) {
        int32_t u = col_idx[k];
        int32_t cu = col[u];
        if (cu >= 0 && cu <= d) seen[cu] = 0;
    }
    return m;
}

static int32_t max_degree(int32_t n, const int32_t *row_ptr) {
    int32_t d = 0;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] - row_ptr[v] > d) d = row_ptr[v + 1] - row_ptr[v];
    return d;
}

static int32_t colour_count(int32_t n, const int32_t *col) {
    int32_t k = 0;
    for (int32_t v = 0; v < n; ++v)
        if (col[v] + 1 > k) k = col[v] + 1;
    return k;
}

/*
 * Sequential First-Fit (Section 2.1, Algorithm 1).  Vertices are visited in
 * natural id order; each takes the smallest colour not held by an already
 * coloured neighbour.  Returns K.
 */
int32_t orc_seq_ff(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t *colors) {
    if (n < 0 || (n > 0 && (!row_ptr || !colors))) return ORC_EINVAL;
    unsigned char *seen = (unsigned char *)calloc((size_t)max_degree(n, row_ptr) + 2, 1);
    if (!seen) return ORC_ENOMEM;
    for (int32_t v = 0; v < n; ++v) colors[v] = -1; /* nobody coloured yet */
    for (int32_t v = 0; v < n; ++v) colors[v] = smallest_free_colour(v, row_ptr, col_idx, colors, seen);
    free(seen);
    return colour_count(n, colors);
}

/* Does v lose a tie against neighbour u under the given rule? */
static int loses(int32_t v, int32_t u, int32_t tie) {
    if (tie == TIE_LOWER_KEEPS) return u < v;
    if (tie == TIE_HIGHER_KEEPS) return u > v;
    return 1; /* TIE_NONE */
}

/*
 * Reduced-synchronisation optimistic colouring (Section 3, Algorithm 3) under
 * a deterministic round-synchronous reading: every read in a round sees the
 * colours as they stood at the preceding barrier (a snapshot), and all writes
 * of the round become visible together at the next barrier.
 *
 * Round 0 is the tentative First-Fit over all vertices.  In a snapshot in
 * which no vertex is coloured yet, every vertex sees no coloured neighbour and
 * takes colour 0.  U^0 is then all of V.  Each later round inspects U^{i-1}:
 * a vertex that (still) shares its colour with a neighbour it loses to is
 * recoloured with the smallest colour absent among all its neighbours and
 * joins L; U^i is L.  The loop ends when a round recolours nobody.
 *
 * Outputs: colors[n]; *rounds_out = number of rounds that recoloured at least
 * one vertex (R); *conflicts_out = sum of |L| over those rounds; L_sizes[i]
 * (if non-NULL, up to L_cap entries) = |L| of recolouring round i+1.
 * max_rounds bounds the number of inspection passes (rounds i >= 1, the last
 * of which finds nothing to recolour); <= 0 means n + 1, enough for any graph
 * because |L| shrinks by at least one per round.  Returns K, or ORC_ENOCONV
 * when the worklist is still non-empty after max_rounds passes (colors then
 * holds the state reached).
 */
int32_t orc_rsync(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t tie, int32_t max_rounds,
                  int32_t *colors, int32_t *rounds_out, int64_t *conflicts_out, int32_t *L_sizes,
                  int32_t L_cap) {
    if (n < 0 || (n > 0 && (!row_ptr || !colors)) || tie < 0 || tie > 2) return ORC_EINVAL;
    if (max_rounds <= 0) max_rounds = n + 1;
    int32_t *snap = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *U = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    unsigned char *seen = (unsigned char *)calloc((size_t)max_degree(n, row_ptr) + 2, 1);
    if (!snap || !U || !L || !seen) { free(snap); free(U); free(L); free(seen); return ORC_ENOMEM; }

    /* round 0 against the all-uncoloured snapshot: everyone takes colour 0 */
    for (int32_t v = 0; v < n; ++v) colors[v] = 0;
    int32_t nU = n;
    for (int32_t v = 0; v < n; ++v) U[v] = v; /* U^0 <- V */

    int32_t rounds = 0, passes = 0;
    int64_t conflicts = 0;
    int32_t rc = 0;
    while (nU > 0) {
        if (passes == max_rounds) { rc = ORC_ENOCONV; break; } /* the guard */
        passes++;
        memcpy(snap, colors, sizeof(int32_t) * (size_t)n); /* state at the barrier */
        int32_t nL = 0;
        for (int32_t k = 0; k < nU; ++k) {
            int32_t v = U[k];
            int defective = 0;
            for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
                int32_t u = col_idx[j];
                if (u != v && loses(v, u, tie) && snap[u] == snap[v]) { defective = 1; break; }
            }
            if (defective) {
                colors[v] = smallest_free_colour(v, row_ptr, col_idx, snap, seen);
                L[nL++] = v;
            }
        }
        if (nL == 0) break;
        if (L_sizes && rounds < L_cap) L_sizes[rounds] = nL;
        rounds++;
        conflicts += nL;
        int32_t *t = U; U = L; L = t; /* U^i <- L */
        nU = nL;
    }
    if (rounds_out) *rounds_out = rounds;
    if (conflicts_out) *conflicts_out = conflicts;
    free(snap); free(U); free(L); free(seen);
    return rc < 0 ? rc : colour_count(n, colors);
}

/*
 * The predecessor scheme of Catalyurek et al. (Section 2.2, Algorithm 2) under
 * the same snapshot reading: each round first gives every vertex of U the
 * smallest colour absent among its neighbours in the snapshot (Phase 1), a
 * barrier publishes the new colours, then every vertex of U that shares its
 * colour with a neighbour it loses to joins L (Phase 2), and U <- L.
 * Uncoloured vertices (before their first Phase 1) hold -1 and are ignored.
 * Outputs as for orc_rsync; here every round with non-empty U counts, and
 * *rounds_out is the number of Phase-1 passes.
 */
int32_t orc_cat(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t tie, int32_t max_rounds,
                int32_t *colors, int32_t *rounds_out, int64_t *conflicts_out, int32_t *L_sizes, int32_t L_cap) {
    if (n < 0 || (n > 0 && (!row_ptr || !colors)) || tie < 0 || tie > 1) return ORC_EINVAL;
    if (max_rounds <= 0) max_rounds = n + 1;
    int32_t *snap = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *U = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    unsigned char *seen = (unsigned char *)calloc((size_t)max_degree(n, row_ptr) + 2, 1);
    if (!snap || !U || !L || !seen) { free(snap); free(U); free(L); free(seen); return ORC_ENOMEM; }
    for (int32_t v = 0; v < n; ++v) { colors[v] = -1; U[v] = v; }
    int32_t nU = n, rounds = 0, rc = 0;
    int64_t conflicts = 0;
    while (nU > 0) {
        if (rounds >= max_rounds) { rc = ORC_ENOCONV; break; }
        /* Phase 1: tentative colouring of U from the snapshot */
        memcpy(snap, colors, sizeof(int32_t) * (size_t)n);
        for (int32_t k = 0; k < nU; ++k)
            colors[U[k]] = smallest_free_colour(U[k], row_ptr, col_idx, snap, seen);
        rounds++;
        /* barrier; Phase 2: conflict detection on the published colours */
        int32_t nL = 0;
        for (int32_t k = 0; k < nU; ++k) {
            int32_t v = U[k];
            for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
                int32_t u = col_idx[j];
                if (u != v && loses(v, u, tie) && colors[u] == colors[v]) { L[nL++] = v; break; }
            }
        }
        if (L_sizes && rounds - 1 < L_cap) L_sizes[rounds - 1] = nL;
        conflicts += nL;
        int32_t *t = U; U = L; L = t;
        nU = nL;
    }
    if (rounds_out) *rounds_out = rounds;
    if (conflicts_out) *conflicts_out = conflicts;
    free(snap); free(U); free(L); free(seen);
    return rc < 0 ? rc : colour_count(n, colors);
}

/*
 * Checker: counts edges (v,u), u != v, whose endpoints share a colour (each
 * undirected edge counted once per direction stored), and vertices whose
 * colour is negative or above their degree.  Returns the sum (0 = valid, and
 * every colour within the First-Fit bound c(v) <= deg(v) of Section 2.1).
 */
int64_t orc_check(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *colors) {
    if (n < 0 || (n > 0 && (!row_ptr || !colors))) return ORC_EINVAL;
    int64_t bad = 0;
    for (int32_t v = 0; v < n; ++v) {
        int32_t d = row_ptr[v + 1] - row_ptr[v];
        if (colors[v] < 0 || colors[v] > d) ++bad;
        for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
            int32_t u = col_idx[j];
            if (u != v && colors[u] == colors[v]) ++bad;
        }
    }
    return bad;
}

/*
 * Colour classes.  A colouring splits V into independent sets, one per
 * colour, whose vertices can be processed concurrently (the use of colouring
 * the introduction describes, Section 1).  Class k holds the vertices of
 * colour k in ascending id: class_vtx[ptr[k] .. ptr[k+1]).  Written as the
 * counting sort it is: count each colour, prefix sums give each class's
 * start, then one pass over the vertices in id order places each one.
 * Returns 0, or ORC_EINVAL when a colour lies outside [0, K).
 */
int32_t orc_classes(int32_t n, const int32_t *colors, int32_t K, int32_t *ptr, int32_t *vtx) {
    if (n < 0 || K < 0 || !ptr || (n > 0 && (!colors || !vtx))) return ORC_EINVAL;
    for (int32_t v = 0; v < n; ++v)
        if (colors[v] < 0 || colors[v] >= K) return ORC_EINVAL;
    for (int32_t k = 0; k <= K; ++k) ptr[k] = 0;
    for (int32_t v = 0; v < n; ++v) ptr[colors[v] + 1] += 1;  /* size of each class */
    for (int32_t k = 0; k < K; ++k) ptr[k + 1] += ptr[k];     /* start of each class */
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
    if (!next) return ORC_ENOMEM;
    for (int32_t k = 0; k < K; ++k) next[k] = ptr[k];
    for (int32_t v = 0; v < n; ++v) vtx[next[colors[v]]++] = v;  /* ascending id within a class */
    free(next);
    return 0;
}

/*
 * Recolouring after topology edits.  The introduction (Section 1) names
 * applications that change the graph between colourings (morph kernels, mesh
 * adaptivity) and so recolour in every iteration.  Reading: Algorithm 3 under
 * the snapshot reading of orc_rsync, started from the colouring the graph had
 * before the edits instead of from round 0, with
 *   U^0 = the touched vertices (the endpoints of inserted edges; an edge
 *         deletion cannot create a conflict) together with every vertex whose
 *         colour is negative (no colour yet, e.g. a new vertex) or above its
 *         degree (outside the First-Fit bound c(v) <= deg(v) of Section 2.1,
 *         possible after deletions),
 * and a vertex of U^{i-1} counted defective when its colour is such a one or
 * when it shares its colour with a neighbour it loses to.  Defective vertices
 * take the smallest colour absent among their neighbours' snapshot colours
 * (negative ones ignored) and form L; U^i <- L.  colors[] is read as the
 * previous colouring and written with the result; touched[0, nt) may repeat
 * ids.  Outputs and return value as for orc_rsync (ORC_EINVAL also for a
 * touched id outside [0, n)).
 */
int32_t orc_recolor(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t tie, int32_t max_rounds,
                    int32_t *colors, const int32_t *touched, int32_t nt, int32_t *rounds_out,
                    int64_t *conflicts_out, int32_t *L_sizes, int32_t L_cap) {
    if (n < 0 || nt < 0 || (n > 0 && (!row_ptr || !colors)) || (nt > 0 && !touched) || tie < 0 || tie > 1)
        return ORC_EINVAL;
    for (int32_t k = 0; k < nt; ++k)
        if (touched[k] < 0 || touched[k] >= n) return ORC_EINVAL;
    if (max_rounds <= 0) max_rounds = n + 1;
    int32_t *snap = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *U = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    unsigned char *in_u0 = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    unsigned char *seen = (unsigned char *)calloc((size_t)max_degree(n, row_ptr) + 2, 1);
    if (!snap || !U || !L || !in_u0 || !seen) {
        free(snap); free(U); free(L); free(in_u0); free(seen);
        return ORC_ENOMEM;
    }
    /* U^0: touched vertices and those without a valid First-Fit colour */
    for (int32_t k = 0; k < nt; ++k) in_u0[touched[k]] = 1;
    int32_t nU = 0;
    for (int32_t v = 0; v < n; ++v) {
        const int32_t d = row_ptr[v + 1] - row_ptr[v];
        if (in_u0[v] || colors[v] < 0 || colors[v] > d) U[nU++] = v;
    }
    int32_t rounds = 0, passes = 0;
    int64_t conflicts = 0;
    int32_t rc = 0;
    while (nU > 0) {
        if (passes == max_rounds) { rc = ORC_ENOCONV; break; }
        passes++;
        memcpy(snap, colors, sizeof(int32_t) * (size_t)n);
        int32_t nL = 0;
        for (int32_t k = 0; k < nU; ++k) {
            int32_t v = U[k];
            const int32_t d = row_ptr[v + 1] - row_ptr[v];
            int defective = snap[v] < 0 || snap[v] > d;
            for (int32_t j = row_ptr[v]; j < row_ptr[v + 1] && !defective; ++j) {
                int32_t u = col_idx[j];
                if (u != v && loses(v, u, tie) && snap[u] == snap[v]) defective = 1;
            }
            if (defective) {
                colors[v] = smallest_free_colour(v, row_ptr, col_idx, snap, seen);
                L[nL++] = v;
            }
        }
        if (nL == 0) break;
        if (L_sizes && rounds < L_cap) L_sizes[rounds] = nL;
        rounds++;
        conflicts += nL;
        int32_t *t = U; U = L; L = t;
        nU = nL;
    }
    if (rounds_out) *rounds_out = rounds;
    if (conflicts_out) *conflicts_out = conflicts;
    free(snap); free(U); free(L); free(in_u0); free(seen);
    return rc < 0 ? rc : colour_count(n, colors);
}

/*
 * The square G^2 of a graph (Section 6 names d-distance colouring, i.e. the
 * colouring of the d-th power graph G^d, as the extension the method suits:
 * u and w are adjacent in G^2 iff they are within distance 2 in G).  Row v of
 * G^2 lists, in ascending order and once each, every vertex other than v that
 * is a neighbour of v or a neighbour of one of v's neighbours.  Two passes
 * over the same loop: the first counts into out_rp (out_rp[n] = nnz of G^2),
 * the second (out_ci non-NULL, out_cap entries) writes.  `mark` is the
 * last-visited stamp of each vertex.  Returns nnz(G^2), ORC_EINVAL, or
 * ORC_ENOMEM (also when out_cap is too small).
 */
int64_t orc_square(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int64_t *out_rp, int32_t *out_ci,
                   int64_t out_cap) {
    if (n < 0 || (n > 0 && (!row_ptr || !out_rp))) return ORC_EINVAL;
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *row = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!mark || !row) { free(mark); free(row); return ORC_ENOMEM; }
    for (int32_t v = 0; v < n; ++v) mark[v] = -1;
    out_rp[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        int32_t len = 0;
        mark[v] = v; /* v itself is never listed */
        for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
            const int32_t u = col_idx[j];
            if (mark[u] != v) { mark[u] = v; row[len++] = u; }
            for (int32_t k = row_ptr[u]; k < row_ptr[u + 1]; ++k) {
                const int32_t w = col_idx[k];
                if (mark[w] != v) { mark[w] = v; row[len++] = w; }
            }
        }
        out_rp[v + 1] = out_rp[v] + len;
        if (out_ci) {
            if (out_rp[v + 1] > out_cap) { free(mark); free(row); return ORC_ENOMEM; }
            /* ascending order: insertion sort of the (short) row */
            for (int32_t a = 1; a < len; ++a) {
                const int32_t x = row[a];
                int32_t b = a - 1;
                while (b >= 0 && row[b] > x) { row[b + 1] = row[b]; --b; }
                row[b + 1] = x;
            }
            memcpy(out_ci + out_rp[v], row, sizeof(int32_t) * (size_t)len);
        }
    }
    free(mark); free(row);
    return out_rp[n];
}
