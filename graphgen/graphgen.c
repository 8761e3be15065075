/*
 * graphgen.c -- seeded synthetic graph generators (inputs only).
 *
 * This module produces undirected graphs in symmetric CSR int32 form for the
 * colouring library and for the CPU oracle.  It holds none of the colouring
 * method's arithmetic: it only builds adjacency structure.
 *
 * Workloads mirror the shapes the paper evaluates (Section 4): simplicial
 * 2D/3D meshes and R-MAT power-law graphs whose vertex ids are randomly
 * shuffled.  The paper's own matrices are not available, so these are
 * synthetic stand-ins:
 *   - tri_grid   : W x H vertex grid, every cell split by the "\" diagonal
 *                  (a triangulated 2D mesh);
 *   - lattice26  : S^3 lattice, every vertex joined to its 26 stencil
 *                  neighbours (a tetrahedral-mesh-like 3D graph);
 *   - rmat       : R-MAT (Chakrabarti et al.) with quadrant probabilities
 *                  a, b, c, d, self-loops and duplicates dropped, symmetrised;
 *   - rgg        : random geometric graph in the unit square;
 *   - batch      : many independent grids / RGGs concatenated with int64
 *                  offset tables.
 *
 * Random numbers: splitmix64 for seeding and xoshiro256** for streams
 * (Blackman & Vigna's published generators), doubles from the top 53 bits.
 * No libc random functions are used, so the bytes produced are identical
 * across compilers and platforms (build with -ffp-contract=off).
 *
 * Memory: every output array is obtained from a caller-supplied allocation
 * callback, so the Python side owns the buffers.  Temporary buffers are
 * malloc'd and freed here.  Every function returns 0 on success and a
 * negative value on allocation failure or bad arguments.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef void *(*gg_alloc_fn)(int32_t tag, int64_t count, int32_t elem_size);

enum { GG_TAG_ROW_PTR = 0, GG_TAG_COL_IDX = 1, GG_TAG_VTX_OFF = 2, GG_TAG_NNZ_OFF = 3, GG_TAG_PERM = 4 };

/* ---------------------------------------------------------------- RNG --- */

static uint64_t splitmix64_next(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gg_splitmix64(uint64_t x) { return splitmix64_next(&x); }

typedef struct { uint64_t s[4]; } xoshiro;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static void xo_seed(xoshiro *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64_next(&x);
}

static inline uint64_t xo_next(xoshiro *r) {
    uint64_t *s = r->s;
    const uint64_t result = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

static inline double xo_double(xoshiro *r) { return (double)(xo_next(r) >> 11) * 0x1.0p-53; }

/* Unbiased integer in [0, m) by rejection. */
static inline uint64_t xo_below(xoshiro *r, uint64_t m) {
    uint64_t lim = UINT64_MAX - (UINT64_MAX % m);
    uint64_t x;
    do { x = xo_next(r); } while (x >= lim);
    return x % m;
}

/* ------------------------------------------------------------ helpers --- */

static void sort_i32(int32_t *a, int64_t len);

static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

static void sort_i32(int32_t *a, int64_t len) {
    if (len < 32) {
        for (int64_t i = 1; i < len; ++i) {
            int32_t v = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
            a[j + 1] = v;
        }
    } else {
        qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/* Fisher-Yates: perm[old] = new id. */
static void fisher_yates(int32_t *perm, int64_t n, uint64_t seed) {
    xoshiro r;
    xo_seed(&r, seed);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)xo_below(&r, (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

int32_t gg_permutation(int64_t n, uint64_t seed, int32_t *perm_out) {
    if (n < 0 || (n > 0 && !perm_out)) return -1;
    fisher_yates(perm_out, n, seed);
    return 0;
}

/* Relabel a CSR graph: vertex v becomes perm[v]; rows are re-sorted. */
static int relabel_into(int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *perm,
                        int32_t *rp_out, int32_t *ci_out) {
    int32_t *deg_new = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!deg_new) return -2;
    for (int64_t v = 0; v < n; ++v) deg_new[perm[v]] = rp[v + 1] - rp[v];
    rp_out[0] = 0;
    for (int64_t v = 0; v < n; ++v) rp_out[v + 1] = rp_out[v] + deg_new[v];
    free(deg_new);
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
        int32_t nv = perm[v];
        int32_t dst = rp_out[nv];
        int32_t d = rp[v + 1] - rp[v];
        for (int32_t k = 0; k < d; ++k) ci_out[dst + k] = perm[ci[rp[v] + k]];
        sort_i32(ci_out + dst, d);
    }
    return 0;
}

/* Finish: optionally permute ids, then hand buffers to the caller. */
static int finish_csr(int64_t n, int32_t *rp, int32_t *ci, int64_t nnz, int permute, uint64_t perm_seed,
                      gg_alloc_fn alloc) {
    int32_t *rp_out = (int32_t *)alloc(GG_TAG_ROW_PTR, n + 1, 4);
    int32_t *ci_out = (int32_t *)alloc(GG_TAG_COL_IDX, nnz, 4);
    if (!rp_out || (nnz > 0 && !ci_out)) return -2;
    if (!permute) {
        memcpy(rp_out, rp, sizeof(int32_t) * (size_t)(n + 1));
        if (nnz) memcpy(ci_out, ci, sizeof(int32_t) * (size_t)nnz);
        return 0;
    }
    int32_t *perm = (int32_t *)alloc(GG_TAG_PERM, n, 4);
    if (!perm && n > 0) return -2;
    fisher_yates(perm, n, perm_seed);
    return relabel_into(n, rp, ci, perm, rp_out, ci_out);
}

/* ----------------------------------------------------- triangulated grid --- */

static int64_t tri_grid_fill(int64_t W, int64_t H, int32_t *rp, int32_t *ci) {
    /* vertex (r, c) has id r*W + c; edges to (r,c+1), (r+1,c), (r+1,c+1) */
    int64_t pos = 0;
    if (rp) rp[0] = 0;
    for (int64_t r = 0; r < H; ++r) {
        for (int64_t c = 0; c < W; ++c) {
            int64_t v = r * W + c;
            /* ascending neighbour ids: (-1,-1), (-1,0), (0,-1), (0,+1), (+1,0), (+1,+1) */
            if (r > 0 && c > 0) { if (ci) ci[pos] = (int32_t)(v - W - 1); ++pos; }
            if (r > 0) { if (ci) ci[pos] = (int32_t)(v - W); ++pos; }
            if (c > 0) { if (ci) ci[pos] = (int32_t)(v - 1); ++pos; }
            if (c + 1 < W) { if (ci) ci[pos] = (int32_t)(v + 1); ++pos; }
            if (r + 1 < H) { if (ci) ci[pos] = (int32_t)(v + W); ++pos; }
            if (r + 1 < H && c + 1 < W) { if (ci) ci[pos] = (int32_t)(v + W + 1); ++pos; }
            if (rp) rp[v + 1] = (int32_t)pos;
        }
    }
    return pos;
}

int32_t gg_tri_grid(int64_t W, int64_t H, int32_t permute, uint64_t perm_seed, gg_alloc_fn alloc) {
    if (W < 0 || H < 0 || W * H > INT32_MAX) return -1;
    int64_t n = W * H;
    int64_t nnz = tri_grid_fill(W, H, NULL, NULL);
    if (nnz > INT32_MAX) return -1;
    if (!permute) {
        int32_t *rp = (int32_t *)alloc(GG_TAG_ROW_PTR, n + 1, 4);
        int32_t *ci = (int32_t *)alloc(GG_TAG_COL_IDX, nnz, 4);
        if (!rp || (nnz && !ci)) return -2;
        tri_grid_fill(W, H, rp, ci);
        return 0;
    }
    int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!rp || !ci) { free(rp); free(ci); return -2; }
    tri_grid_fill(W, H, rp, ci);
    int rc = finish_csr(n, rp, ci, nnz, 1, perm_seed, alloc);
    free(rp); free(ci);
    return rc;
}

/* ---------------------------------------------------- 26-stencil lattice --- */

int32_t gg_lattice26(int64_t S, int32_t permute, uint64_t perm_seed, gg_alloc_fn alloc) {
    if (S < 0 || S * S * S > INT32_MAX) return -1;
    int64_t n = S * S * S;
    int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!rp) return -2;
    /* degree of (x,y,z) = (cx*cy*cz) - 1 where c* = number of in-range offsets in that axis */
    rp[0] = 0;
    for (int64_t z = 0; z < S; ++z)
        for (int64_t y = 0; y < S; ++y)
            for (int64_t x = 0; x < S; ++x) {
                int64_t cx = 1 + (x > 0) + (x + 1 < S), cy = 1 + (y > 0) + (y + 1 < S), cz = 1 + (z > 0) + (z + 1 < S);
                int64_t v = (z * S + y) * S + x;
                rp[v + 1] = rp[v] + (int32_t)(cx * cy * cz - 1);
            }
    int64_t nnz = rp[n];
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!ci) { free(rp); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < S; ++z)
        for (int64_t y = 0; y < S; ++y)
            for (int64_t x = 0; x < S; ++x) {
                int64_t v = (z * S + y) * S + x;
                int64_t pos = rp[v];
                /* dz, dy, dx ascending gives ascending neighbour ids */
                for (int dz = -1; dz <= 1; ++dz) {
                    int64_t zz = z + dz;
                    if (zz < 0 || zz >= S) continue;
                    for (int dy = -1; dy <= 1; ++dy) {
                        int64_t yy = y + dy;
                        if (yy < 0 || yy >= S) continue;
                        for (int dx = -1; dx <= 1; ++dx) {
                            int64_t xx = x + dx;
                            if (xx < 0 || xx >= S) continue;
                            if (!dx && !dy && !dz) continue;
                            ci[pos++] = (int32_t)((zz * S + yy) * S + xx);
                        }
                    }
                }
            }
    int rc = finish_csr(n, rp, ci, nnz, permute, perm_seed, alloc);
    free(rp); free(ci);
    return rc;
}

/* ----------------------------------------------------------------- R-MAT --- */

/*
 * Generates ef * 2^scale directed draws; each draw picks one quadrant per
 * level with probabilities (a, b, c, 1-a-b-c): a = (row bit 0, col bit 0),
 * b = (0, 1), c = (1, 0), d = (1, 1).  Self-loops are dropped, every edge is
 * stored in both directions and duplicates are removed.  With `shuffle`, ids
 * are relabelled by a seeded Fisher-Yates permutation before the CSR is built.
 * `dropped_self` (optional) receives the number of self-loop draws dropped.
 */
int32_t gg_rmat(int32_t scale, int64_t edge_factor, double a, double b, double c, uint64_t seed,
                int32_t shuffle, uint64_t perm_seed, int64_t *dropped_self, gg_alloc_fn alloc) {
    if (scale < 0 || scale > 30 || edge_factor < 0) return -1;
    int64_t n = (int64_t)1 << scale;
    int64_t m = edge_factor * n;
    double ab = a + b, abc = a + b + c;
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t *dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!src || !dst) { free(src); free(dst); return -2; }
    /* deterministic in the number of threads: edge blocks have their own streams */
    const int64_t BLK = 1 << 16;
    int64_t nblk = (m + BLK - 1) / BLK;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t blk = 0; blk < nblk; ++blk) {
        xoshiro r;
        xo_seed(&r, gg_splitmix64(seed ^ (0x5851F42D4C957F2Dull * (uint64_t)(blk + 1))));
        int64_t e0 = blk * BLK, e1 = e0 + BLK < m ? e0 + BLK : m;
        for (int64_t e = e0; e < e1; ++e) {
            uint32_t s = 0, t = 0;
            for (int32_t l = 0; l < scale; ++l) {
                double u = xo_double(&r);
                uint32_t rb, cb;
                if (u < a) { rb = 0; cb = 0; }
                else if (u < ab) { rb = 0; cb = 1; }
                else if (u < abc) { rb = 1; cb = 0; }
                else { rb = 1; cb = 1; }
                s = (s << 1) | rb;
                t = (t << 1) | cb;
            }
            src[e] = (int32_t)s;
            dst[e] = (int32_t)t;
        }
    }
    int32_t *perm = NULL;
    if (shuffle) {
        perm = (int32_t *)alloc(GG_TAG_PERM, n, 4);
        if (!perm) { free(src); free(dst); return -2; }
        fisher_yates(perm, n, perm_seed);
    }
    /* count both directions, skipping self-loops */
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!deg) { free(src); free(dst); return -2; }
    int64_t selfl = 0;
    for (int64_t e = 0; e < m; ++e) {
        int32_t s = src[e], t = dst[e];
        if (s == t) { ++selfl; continue; }
        if (perm) { s = perm[s]; t = perm[t]; src[e] = s; dst[e] = t; }
        deg[s]++; deg[t]++;
    }
    if (dropped_self) *dropped_self = selfl;
    int64_t tot = 0;
    for (int64_t v = 0; v < n; ++v) { int64_t d = deg[v]; deg[v] = tot; tot += d; }
    deg[n] = tot;
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!adj || !fill) { free(src); free(dst); free(deg); free(adj); free(fill); return -2; }
    memcpy(fill, deg, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < m; ++e) {
        int32_t s = src[e], t = dst[e];
        if (s == t) continue;
        adj[fill[s]++] = t;
        adj[fill[t]++] = s;
    }
    free(src); free(dst); free(fill);
    /* sort rows and drop duplicates in place; record new degrees */
    int32_t *ndeg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!ndeg) { free(deg); free(adj); return -2; }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; ++v) {
        int32_t *row = adj + deg[v];
        int64_t d = deg[v + 1] - deg[v];
        sort_i32(row, d);
        int64_t k = 0;
        for (int64_t j = 0; j < d; ++j)
            if (k == 0 || row[j] != row[k - 1]) row[k++] = row[j];
        ndeg[v] = (int32_t)k;
    }
    int64_t nnz = 0;
    for (int64_t v = 0; v < n; ++v) nnz += ndeg[v];
    if (nnz > INT32_MAX) { free(deg); free(adj); free(ndeg); return -1; }
    int32_t *rp = (int32_t *)alloc(GG_TAG_ROW_PTR, n + 1, 4);
    int32_t *ci = (int32_t *)alloc(GG_TAG_COL_IDX, nnz, 4);
    if (!rp || (nnz && !ci)) { free(deg); free(adj); free(ndeg); return -2; }
    rp[0] = 0;
    for (int64_t v = 0; v < n; ++v) rp[v + 1] = rp[v] + ndeg[v];
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) memcpy(ci + rp[v], adj + deg[v], sizeof(int32_t) * (size_t)ndeg[v]);
    free(deg); free(adj); free(ndeg);
    return 0;
}

/* ------------------------------------------------ random geometric graph --- */

typedef struct {
    int64_t n, G;
    double r2;
    double *x, *y;
    int32_t *cell_start; /* G*G + 1 */
    int32_t *cell_pts;   /* n, point ids grouped by cell, ascending within a cell */
} rgg_state;

static int rgg_build(rgg_state *st, int64_t n, double radius, uint64_t seed) {
    memset(st, 0, sizeof(*st));
    st->n = n;
    st->r2 = radius * radius;
    int64_t G = radius > 0 ? (int64_t)floor(1.0 / radius) : 1;
    if (G < 1) G = 1;
    if (G > 65536) G = 65536;
    st->G = G;
    st->x = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    st->y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    st->cell_start = (int32_t *)calloc((size_t)(G * G + 1), sizeof(int32_t));
    st->cell_pts = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!st->x || !st->y || !st->cell_start || !st->cell_pts || !cell_of) { free(cell_of); return -2; }
    xoshiro r;
    xo_seed(&r, seed);
    for (int64_t i = 0; i < n; ++i) {
        st->x[i] = xo_double(&r);
        st->y[i] = xo_double(&r);
        int64_t cx = (int64_t)(st->x[i] * (double)G), cy = (int64_t)(st->y[i] * (double)G);
        if (cx >= G) cx = G - 1;
        if (cy >= G) cy = G - 1;
        cell_of[i] = (int32_t)(cy * G + cx);
        st->cell_start[cell_of[i] + 1]++;
    }
    for (int64_t c = 0; c < G * G; ++c) st->cell_start[c + 1] += st->cell_start[c];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(G * G));
    if (!fill) { free(cell_of); return -2; }
    memcpy(fill, st->cell_start, sizeof(int32_t) * (size_t)(G * G));
    for (int64_t i = 0; i < n; ++i) st->cell_pts[fill[cell_of[i]]++] = (int32_t)i;
    free(fill);
    free(cell_of);
    return 0;
}

static void rgg_free(rgg_state *st) {
    free(st->x); free(st->y); free(st->cell_start); free(st->cell_pts);
}

/* Neighbours of point i (ids != i, squared distance < r^2); writes up to
 * all of them into out (if non-NULL) and returns the count.  Output is sorted. */
static int64_t rgg_neighbours(const rgg_state *st, int64_t i, int32_t *out) {
    int64_t G = st->G;
    int64_t cx = (int64_t)(st->x[i] * (double)G), cy = (int64_t)(st->y[i] * (double)G);
    if (cx >= G) cx = G - 1;
    if (cy >= G) cy = G - 1;
    int64_t cnt = 0;
    for (int64_t yy = cy - 1; yy <= cy + 1; ++yy) {
        if (yy < 0 || yy >= G) continue;
        for (int64_t xx = cx - 1; xx <= cx + 1; ++xx) {
            if (xx < 0 || xx >= G) continue;
            int64_t c = yy * G + xx;
            for (int32_t k = st->cell_start[c]; k < st->cell_start[c + 1]; ++k) {
                int32_t j = st->cell_pts[k];
                if (j == i) continue;
                double dx = st->x[i] - st->x[j], dy = st->y[i] - st->y[j];
                double d2 = dx * dx + dy * dy;
                if (d2 < st->r2) {
                    if (out) out[cnt] = j;
                    ++cnt;
                }
            }
        }
    }
    if (out) sort_i32(out, cnt);
    return cnt;
}

/* Count pass + fill pass into caller buffers (rp has n+1 slots). */
static int64_t rgg_count(const rgg_state *st) {
    int64_t tot = 0;
    for (int64_t i = 0; i < st->n; ++i) tot += rgg_neighbours(st, i, NULL);
    return tot;
}

static void rgg_fill(const rgg_state *st, int32_t *rp, int32_t *ci) {
    rp[0] = 0;
    for (int64_t i = 0; i < st->n; ++i) {
        int64_t d = rgg_neighbours(st, i, ci + rp[i]);
        rp[i + 1] = rp[i] + (int32_t)d;
    }
}

int32_t gg_rgg(int64_t n, double radius, uint64_t seed, gg_alloc_fn alloc) {
    if (n < 0 || n > INT32_MAX || !(radius >= 0)) return -1;
    rgg_state st;
    if (rgg_build(&st, n, radius, seed)) { rgg_free(&st); return -2; }
    int64_t nnz = rgg_count(&st);
    if (nnz > INT32_MAX) { rgg_free(&st); return -1; }
    int32_t *rp = (int32_t *)alloc(GG_TAG_ROW_PTR, n + 1, 4);
    int32_t *ci = (int32_t *)alloc(GG_TAG_COL_IDX, nnz, 4);
    if (!rp || (nnz && !ci)) { rgg_free(&st); return -2; }
    rgg_fill(&st, rp, ci);
    rgg_free(&st);
    return 0;
}

/* ------------------------------------------------------------- batches --- */

/*
 * Batch of G independent graphs.  Graph g draws from its own stream seeded by
 * splitmix64(base_seed * 2^32 + g): first n_g = round(exp(U[ln nmin, ln nmax])),
 * then a Bernoulli(1/2) type: a W x W triangulated grid with W = round(sqrt(n_g))
 * (max(W,1)), or an RGG of n_g points with radius sqrt(mean_deg / (pi n_g)).
 * Outputs:
 *   vtx_off[G+1] int64, nnz_off[G+1] int64   (prefix sums of n_g and nnz_g)
 *   row_ptr_cat  int32[vtx_off[G] + G]        (graph g's n_g+1 local entries
 *                                              start at vtx_off[g] + g)
 *   col_idx_cat  int32[nnz_off[G]]            (local ids)
 * kinds_out (optional, host int32[G]): 0 = grid, 1 = rgg.
 */
typedef struct { int64_t n, nnz; int32_t kind, W; double radius; uint64_t pseed; } batch_item;

static void batch_plan(int64_t g, uint64_t base_seed, double nmin, double nmax, double mean_deg, batch_item *it) {
    xoshiro r;
    xo_seed(&r, gg_splitmix64(base_seed * 4294967296ull + (uint64_t)g));
    double u = xo_double(&r);
    double ln = log(nmin) + u * (log(nmax) - log(nmin));
    int64_t ng = (int64_t)llround(exp(ln));
    if (ng < 1) ng = 1;
    double k = xo_double(&r);
    it->pseed = xo_next(&r);
    if (k < 0.5) {
        int64_t W = (int64_t)llround(sqrt((double)ng));
        if (W < 1) W = 1;
        it->kind = 0; it->W = (int32_t)W; it->n = W * W; it->radius = 0;
        it->nnz = 2 * (3 * W * W - 2 * W - 2 * W + 1);
        if (W == 1) it->nnz = 0;
    } else {
        it->kind = 1; it->W = 0; it->n = ng;
        it->radius = sqrt(mean_deg / (M_PI * (double)ng));
        it->nnz = -1;
    }
}

int32_t gg_batch(int64_t G, uint64_t base_seed, double nmin, double nmax, double mean_deg,
                 int32_t *kinds_out, gg_alloc_fn alloc) {
    if (G < 0 || !(nmin >= 1) || !(nmax >= nmin)) return -1;
    batch_item *items = (batch_item *)malloc(sizeof(batch_item) * (size_t)(G > 0 ? G : 1));
    if (!items) return -2;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < G; ++g) {
        batch_plan(g, base_seed, nmin, nmax, mean_deg, &items[g]);
        if (items[g].kind == 1) {
            rgg_state st;
            if (rgg_build(&st, items[g].n, items[g].radius, items[g].pseed)) {
#pragma omp atomic write
                err = 1;
            } else {
                items[g].nnz = rgg_count(&st);
            }
            rgg_free(&st);
        }
    }
    if (err) { free(items); return -2; }
    int64_t *vo = (int64_t *)alloc(GG_TAG_VTX_OFF, G + 1, 8);
    int64_t *no = (int64_t *)alloc(GG_TAG_NNZ_OFF, G + 1, 8);
    if (!vo || !no) { free(items); return -2; }
    vo[0] = 0; no[0] = 0;
    for (int64_t g = 0; g < G; ++g) {
        vo[g + 1] = vo[g] + items[g].n;
        no[g + 1] = no[g] + items[g].nnz;
        if (kinds_out) kinds_out[g] = items[g].kind;
    }
    int32_t *rp = (int32_t *)alloc(GG_TAG_ROW_PTR, vo[G] + G, 4);
    int32_t *ci = (int32_t *)alloc(GG_TAG_COL_IDX, no[G], 4);
    if (!rp || (no[G] && !ci)) { free(items); return -2; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < G; ++g) {
        int32_t *grp = rp + vo[g] + g;
        int32_t *gci = ci + no[g];
        if (items[g].kind == 0) {
            tri_grid_fill(items[g].W, items[g].W, grp, gci);
        } else {
            rgg_state st;
            if (rgg_build(&st, items[g].n, items[g].radius, items[g].pseed)) {
#pragma omp atomic write
                err = 1;
            } else {
                rgg_fill(&st, grp, gci);
            }
            rgg_free(&st);
        }
    }
    free(items);
    return err ? -2 : 0;
}
