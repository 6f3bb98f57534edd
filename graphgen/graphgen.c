/*
 * graphgen.c -- seeded synthetic graph generators (GNM, RMAT, 2D grid, 2D and 3D
 * RGG, random hyperbolic graphs).
 *
 * This module produces input edge lists only.  It holds none of the minimum
 * spanning forest arithmetic: both the GPU library and the CPU oracle consume
 * the arrays it writes, so a parity check never depends on how an input was
 * drawn.  Every random number comes from one counter-based generator:
 *
 *   mix(z)        the SplitMix64 output function (Steele, Lea & Flood,
 *                 "Fast splittable pseudorandom number generators", OOPSLA 2014)
 *   base(s, tag)  = mix(mix(s) ^ tag)           one independent stream per use
 *   draw(b, k)    = mix(b + (k + 1) * GAMMA)    the k-th value of stream b
 *
 * so any value can be recomputed from (seed, tag, k) alone, in any order and
 * on any number of threads.  graphgen/ref.py restates the same definitions in
 * numpy; the tests require both to agree bit for bit.
 *
 * Families follow the paper's experimental section (Instances and
 * Methodology): GNM (Erdos-Renyi with a fixed edge count), RMAT with the
 * Graph500 default probabilities, 2D grids, 2D and 3D random geometric graphs
 * and random hyperbolic graphs (threshold model).
 * Output format: undirected edges, each listed once, as SoA arrays
 * int32 u[m], int32 v[m], uint32 w[m]; the edge id is the array index.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define GAMMA 0x9E3779B97F4A7C15ULL
#define GG_PI 3.14159265358979323846   /* the double nearest pi */

enum { TAG_GNM = 1, TAG_RMAT = 2, TAG_PERM = 3, TAG_RMAT_W = 4, TAG_GRID_KEEP = 5,
       TAG_GRID_W = 6, TAG_RGG = 7, TAG_BATCH = 8, TAG_RGG3 = 9, TAG_RGG3_W = 10, TAG_RHG = 11,
       TAG_RHG_W = 12 };

static inline uint64_t mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t base(uint64_t seed, uint64_t tag) { return mix(mix(seed) ^ tag); }
static inline uint64_t draw(uint64_t b, uint64_t k) { return mix(b + (k + 1) * GAMMA); }

/* floor(r * n / 2^64) for n < 2^32, via two 32x32 products (exactly what ref.py does). */
static inline uint64_t below(uint64_t r, uint64_t n) {
    uint64_t hi = r >> 32, lo = r & 0xffffffffULL;
    return (hi * n + ((lo * n) >> 32)) >> 32;
}

/* ------------------------------------------------------------------ threads */

typedef void (*range_fn)(void* ctx, int64_t lo, int64_t hi);
typedef struct { range_fn fn; void* ctx; int64_t lo, hi; } job_t;

static void* run_job(void* p) {
    job_t* j = (job_t*)p;
    if (j->lo < j->hi) j->fn(j->ctx, j->lo, j->hi);
    return NULL;
}

int gg_threads(void) {
    const char* s = getenv("GRAPHGEN_THREADS");
    int t = s ? atoi(s) : (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (t < 1) t = 1;
    if (t > 64) t = 64;
    return t;
}

static void parallel_for(int64_t n, range_fn fn, void* ctx) {
    int t = gg_threads();
    if (n < 65536 || t == 1) { if (n > 0) fn(ctx, 0, n); return; }
    pthread_t th[64];
    job_t jobs[64];
    int64_t chunk = (n + t - 1) / t;
    for (int i = 0; i < t; ++i) {
        jobs[i].fn = fn; jobs[i].ctx = ctx;
        jobs[i].lo = i * chunk < n ? i * chunk : n;
        jobs[i].hi = (i + 1) * chunk < n ? (i + 1) * chunk : n;
        pthread_create(&th[i], NULL, run_job, &jobs[i]);
    }
    for (int i = 0; i < t; ++i) pthread_join(th[i], NULL);
}

/* --------------------------------------------------------------------- GNM */
/* Edge i: u uniform on [0,n); v uniform on [0,n) minus {u}, as
 * v = (u + 1 + U[0,n-1)) mod n; w uniform on [wlo, whi].  Draws 3i, 3i+1, 3i+2. */

typedef struct { int64_t n; uint32_t wlo, whi; uint64_t b; int32_t *u, *v; uint32_t* w; } gnm_ctx;

static void gnm_range(void* p, int64_t lo, int64_t hi) {
    gnm_ctx* c = (gnm_ctx*)p;
    uint64_t span = (uint64_t)c->whi - c->wlo + 1;
    for (int64_t i = lo; i < hi; ++i) {
        uint64_t a = below(draw(c->b, 3 * (uint64_t)i), (uint64_t)c->n);
        uint64_t d = below(draw(c->b, 3 * (uint64_t)i + 1), (uint64_t)c->n - 1);
        c->u[i] = (int32_t)a;
        c->v[i] = (int32_t)((a + 1 + d) % (uint64_t)c->n);
        c->w[i] = c->wlo + (uint32_t)below(draw(c->b, 3 * (uint64_t)i + 2), span);
    }
}

int gg_gnm(int64_t n, int64_t m, uint32_t wlo, uint32_t whi, uint64_t seed,
           int32_t* u, int32_t* v, uint32_t* w) {
    if (n < 2 || n > 0x7fffffffLL || m < 0 || wlo > whi) return -1;
    gnm_ctx c = { n, wlo, whi, base(seed, TAG_GNM), u, v, w };
    parallel_for(m, gnm_range, &c);
    return 0;
}

/* -------------------------------------------------------------------- RMAT */
/* Per level l (most significant bit first) one 32-bit draw x picks the
 * quadrant: x < ta -> (0,0), x < tab -> (0,1), x < tabc -> (1,0), else (1,1),
 * with ta = floor(a 2^32), tab = floor((a+b) 2^32), tabc = floor((a+b+c) 2^32).
 * Level l uses the high (l even) or low (l odd) half of 64-bit draw l/2 of edge
 * i, i.e. draw index i*ceil(scale/2) + l/2.  The weight is draw i of its own
 * stream.  Vertex ids are then mapped through a seeded 4-round balanced
 * Feistel bijection on [0, 2^scale) (cycle walking when scale is odd). */

typedef struct {
    int scale, h, permute;
    uint32_t ta, tab, tabc, wlo, whi;
    uint64_t b, bw, keys[4];
    int32_t *u, *v; uint32_t* w;
} rmat_ctx;

static inline uint64_t feistel(const rmat_ctx* c, uint64_t x) {
    uint64_t mask = (1ULL << c->h) - 1, lim = 1ULL << c->scale;
    do {
        uint64_t L = x >> c->h, R = x & mask;
        for (int k = 0; k < 4; ++k) {
            uint64_t F = mix(R ^ c->keys[k]) & mask;
            uint64_t nL = R, nR = L ^ F;
            L = nL; R = nR;
        }
        x = (L << c->h) | R;
    } while (x >= lim);
    return x;
}

static void rmat_range(void* p, int64_t lo, int64_t hi) {
    rmat_ctx* c = (rmat_ctx*)p;
    uint64_t per = (uint64_t)(c->scale + 1) / 2;
    uint64_t span = (uint64_t)c->whi - c->wlo + 1;
    for (int64_t i = lo; i < hi; ++i) {
        uint64_t a = 0, b = 0, r = 0;
        for (int l = 0; l < c->scale; ++l) {
            if ((l & 1) == 0) r = draw(c->b, (uint64_t)i * per + (uint64_t)(l >> 1));
            uint32_t x = (l & 1) ? (uint32_t)(r & 0xffffffffULL) : (uint32_t)(r >> 32);
            uint64_t ub, vb;
            if (x < c->ta) { ub = 0; vb = 0; }
            else if (x < c->tab) { ub = 0; vb = 1; }
            else if (x < c->tabc) { ub = 1; vb = 0; }
            else { ub = 1; vb = 1; }
            a = (a << 1) | ub;
            b = (b << 1) | vb;
        }
        if (c->permute) { a = feistel(c, a); b = feistel(c, b); }
        c->u[i] = (int32_t)a;
        c->v[i] = (int32_t)b;
        c->w[i] = c->wlo + (uint32_t)below(draw(c->bw, (uint64_t)i), span);
    }
}

int gg_rmat(int scale, int64_t m, double a, double b, double c, uint32_t wlo, uint32_t whi,
            int permute, uint64_t seed, int32_t* u, int32_t* v, uint32_t* w) {
    if (scale < 1 || scale > 31 || m < 0 || wlo > whi) return -1;
    if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
    rmat_ctx x;
    memset(&x, 0, sizeof x);
    x.scale = scale;
    x.h = (scale + 1) / 2;
    x.permute = permute;
    x.ta = (uint32_t)floor(a * 4294967296.0);
    x.tab = (uint32_t)floor((a + b) * 4294967296.0);
    x.tabc = (uint32_t)fmin(floor((a + b + c) * 4294967296.0), 4294967295.0);
    x.wlo = wlo; x.whi = whi;
    x.b = base(seed, TAG_RMAT);
    x.bw = base(seed, TAG_RMAT_W);
    uint64_t bp = base(seed, TAG_PERM);
    for (int k = 0; k < 4; ++k) x.keys[k] = draw(bp, (uint64_t)k);
    x.u = u; x.v = v; x.w = w;
    parallel_for(m, rmat_range, &x);
    return 0;
}

/* Exposed so that tests can check the bijection directly. */
int gg_rmat_permute(int scale, uint64_t seed, const int64_t* in, int64_t k, int64_t* out) {
    rmat_ctx x;
    memset(&x, 0, sizeof x);
    x.scale = scale; x.h = (scale + 1) / 2;
    uint64_t bp = base(seed, TAG_PERM);
    for (int j = 0; j < 4; ++j) x.keys[j] = draw(bp, (uint64_t)j);
    for (int64_t i = 0; i < k; ++i) out[i] = (int64_t)feistel(&x, (uint64_t)in[i]);
    return 0;
}

/* -------------------------------------------------------------------- grid */
/* rows x cols lattice, vertex id = i*cols + j.  Candidates are enumerated per
 * vertex in id order, right neighbour first, then the one below; candidate c
 * is kept iff the high half of draw c is below floor(keep 2^32).  The edge id
 * is the rank among kept candidates.  wmode 0: w = wlo for every edge;
 * wmode 1: w uniform on [wlo, whi] from draw c of the weight stream. */

typedef struct { int32_t *u, *v; uint32_t* w; int64_t m; } edge_buf;

typedef struct {
    int64_t rows, cols; uint32_t thr; int wmode; uint32_t wlo, whi;
    uint64_t bk, bw; int64_t* row_count; int64_t* row_start; edge_buf* out;
} grid_ctx;

static inline int64_t grid_cand0(const grid_ctx* g, int64_t i) { return i * (2 * g->cols - 1); }

static void grid_count_range(void* p, int64_t lo, int64_t hi) {
    grid_ctx* g = (grid_ctx*)p;
    for (int64_t i = lo; i < hi; ++i) {
        int64_t c = grid_cand0(g, i), cnt = 0;
        for (int64_t j = 0; j < g->cols; ++j) {
            if (j + 1 < g->cols) { cnt += (draw(g->bk, (uint64_t)c) >> 32) < g->thr; ++c; }
            if (i + 1 < g->rows) { cnt += (draw(g->bk, (uint64_t)c) >> 32) < g->thr; ++c; }
        }
        g->row_count[i] = cnt;
    }
}

static void grid_fill_range(void* p, int64_t lo, int64_t hi) {
    grid_ctx* g = (grid_ctx*)p;
    uint64_t span = (uint64_t)g->whi - g->wlo + 1;
    for (int64_t i = lo; i < hi; ++i) {
        int64_t c = grid_cand0(g, i), e = g->row_start[i];
        for (int64_t j = 0; j < g->cols; ++j) {
            int64_t x = i * g->cols + j;
            for (int dir = 0; dir < 2; ++dir) {
                int ok = dir == 0 ? (j + 1 < g->cols) : (i + 1 < g->rows);
                if (!ok) continue;
                if ((draw(g->bk, (uint64_t)c) >> 32) < g->thr) {
                    g->out->u[e] = (int32_t)x;
                    g->out->v[e] = (int32_t)(dir == 0 ? x + 1 : x + g->cols);
                    g->out->w[e] = g->wmode == 0 ? g->wlo
                                 : g->wlo + (uint32_t)below(draw(g->bw, (uint64_t)c), span);
                    ++e;
                }
                ++c;
            }
        }
    }
}

static void* grid_build(int64_t rows, int64_t cols, double keep, int wmode, uint32_t wlo,
                        uint32_t whi, uint64_t seed, int64_t* m_out) {
    if (rows < 1 || cols < 1 || rows * cols > 0x7fffffffLL || keep < 0 || keep > 1 || wlo > whi)
        return NULL;
    grid_ctx g;
    memset(&g, 0, sizeof g);
    g.rows = rows; g.cols = cols;
    g.thr = keep >= 1.0 ? 0xffffffffU : (uint32_t)floor(keep * 4294967296.0);
    g.wmode = wmode; g.wlo = wlo; g.whi = whi;
    g.bk = base(seed, TAG_GRID_KEEP);
    g.bw = base(seed, TAG_GRID_W);
    g.row_count = (int64_t*)calloc((size_t)rows, sizeof(int64_t));
    g.row_start = (int64_t*)calloc((size_t)rows + 1, sizeof(int64_t));
    parallel_for(rows, grid_count_range, &g);
    for (int64_t i = 0; i < rows; ++i) g.row_start[i + 1] = g.row_start[i] + g.row_count[i];
    int64_t m = g.row_start[rows];
    edge_buf* out = (edge_buf*)calloc(1, sizeof(edge_buf));
    out->m = m;
    out->u = (int32_t*)malloc((size_t)(m ? m : 1) * 4);
    out->v = (int32_t*)malloc((size_t)(m ? m : 1) * 4);
    out->w = (uint32_t*)malloc((size_t)(m ? m : 1) * 4);
    g.out = out;
    parallel_for(rows, grid_fill_range, &g);
    free(g.row_count);
    free(g.row_start);
    *m_out = m;
    return out;
}

/* --------------------------------------------------------------------- RGG */
/* n points uniform in [0,1)^2 (x from draw 2t, y from draw 2t+1, 53-bit
 * mantissa), bucketed into a G x G cell grid, G = floor(1/r) so a cell side is
 * at least r.  Vertex ids follow cell-major order (cell index cy*G + cx, then
 * draw order).  Edge {i,j} iff squared distance < r^2; edges are listed in
 * lexicographic (i, j) order with i < j, w = llround(wscale * distance). */

typedef struct {
    int64_t n, G; double r, r2, wscale;
    double *x, *y; int64_t* cell_start; int64_t* cnt; int64_t* start; edge_buf* out;
} rgg_ctx;

static inline int64_t rgg_cell_of(const rgg_ctx* g, double x, double y) {
    int64_t cx = (int64_t)(x * (double)g->G), cy = (int64_t)(y * (double)g->G);
    if (cx >= g->G) cx = g->G - 1;
    if (cy >= g->G) cy = g->G - 1;
    return cy * g->G + cx;
}

static void rgg_scan_vertex(rgg_ctx* g, int64_t i, int fill) {
    double xi = g->x[i], yi = g->y[i];
    int64_t ci = rgg_cell_of(g, xi, yi), cx = ci % g->G, cy = ci / g->G, k = 0;
    int64_t e = fill ? g->start[i] : 0;
    for (int64_t dy = -1; dy <= 1; ++dy) {
        int64_t yy = cy + dy;
        if (yy < 0 || yy >= g->G) continue;
        for (int64_t dx = -1; dx <= 1; ++dx) {
            int64_t xx = cx + dx;
            if (xx < 0 || xx >= g->G) continue;
            int64_t c = yy * g->G + xx;
            for (int64_t j = g->cell_start[c]; j < g->cell_start[c + 1]; ++j) {
                if (j <= i) continue;
                double ddx = g->x[j] - xi, ddy = g->y[j] - yi, d2 = ddx * ddx + ddy * ddy;
                if (d2 < g->r2) {
                    if (fill) {
                        g->out->u[e] = (int32_t)i;
                        g->out->v[e] = (int32_t)j;
                        g->out->w[e] = (uint32_t)llround(g->wscale * sqrt(d2));
                        ++e;
                    } else {
                        ++k;
                    }
                }
            }
        }
    }
    if (!fill) g->cnt[i] = k;
}

static void rgg_count_range(void* p, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) rgg_scan_vertex((rgg_ctx*)p, i, 0);
}
static void rgg_fill_range(void* p, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) rgg_scan_vertex((rgg_ctx*)p, i, 1);
}

typedef struct { uint64_t b; double *x, *y; } pts_ctx;
static void pts_range(void* p, int64_t lo, int64_t hi) {
    pts_ctx* c = (pts_ctx*)p;
    for (int64_t t = lo; t < hi; ++t) {
        c->x[t] = (double)(draw(c->b, 2 * (uint64_t)t) >> 11) * 0x1.0p-53;
        c->y[t] = (double)(draw(c->b, 2 * (uint64_t)t + 1) >> 11) * 0x1.0p-53;
    }
}

static void* rgg_build(int64_t n, double r, double wscale, uint64_t seed, int64_t* m_out) {
    if (n < 1 || n > 0x7fffffffLL || !(r > 0) || r > 1) return NULL;
    rgg_ctx g;
    memset(&g, 0, sizeof g);
    g.n = n; g.r = r; g.r2 = r * r; g.wscale = wscale;
    g.G = (int64_t)floor(1.0 / r);
    if (g.G < 1) g.G = 1;
    if (g.G > 1 << 20) g.G = 1 << 20;
    double* px = (double*)malloc((size_t)n * 8);
    double* py = (double*)malloc((size_t)n * 8);
    pts_ctx pc = { base(seed, TAG_RGG), px, py };
    parallel_for(n, pts_range, &pc);
    int64_t ncell = g.G * g.G;
    g.cell_start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t* cellof = (int64_t*)malloc((size_t)n * 8);
    for (int64_t t = 0; t < n; ++t) {
        cellof[t] = rgg_cell_of(&g, px[t], py[t]);
        g.cell_start[cellof[t] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) g.cell_start[c + 1] += g.cell_start[c];
    int64_t* fillp = (int64_t*)malloc((size_t)ncell * 8);
    memcpy(fillp, g.cell_start, (size_t)ncell * 8);
    g.x = (double*)malloc((size_t)n * 8);
    g.y = (double*)malloc((size_t)n * 8);
    for (int64_t t = 0; t < n; ++t) {          /* stable counting sort by cell */
        int64_t id = fillp[cellof[t]]++;
        g.x[id] = px[t];
        g.y[id] = py[t];
    }
    free(fillp); free(cellof); free(px); free(py);
    g.cnt = (int64_t*)malloc((size_t)n * 8);
    g.start = (int64_t*)malloc((size_t)(n + 1) * 8);
    parallel_for(n, rgg_count_range, &g);
    g.start[0] = 0;
    for (int64_t i = 0; i < n; ++i) g.start[i + 1] = g.start[i] + g.cnt[i];
    int64_t m = g.start[n];
    edge_buf* out = (edge_buf*)calloc(1, sizeof(edge_buf));
    out->m = m;
    out->u = (int32_t*)malloc((size_t)(m ? m : 1) * 4);
    out->v = (int32_t*)malloc((size_t)(m ? m : 1) * 4);
    out->w = (uint32_t*)malloc((size_t)(m ? m : 1) * 4);
    g.out = out;
    parallel_for(n, rgg_fill_range, &g);
    free(g.x); free(g.y); free(g.cnt); free(g.start); free(g.cell_start);
    *m_out = m;
    return out;
}

/* ------------------------------------------------------------------ 3D RGG */
/* n points uniform in [0,1)^3 (x, y, z from draws 3t, 3t+1, 3t+2, 53-bit
 * mantissa), bucketed into a G^3 cell grid, G = floor(1/r).  Vertex ids follow
 * cell-major order (cell (cz*G + cy)*G + cx, then draw order).  Edge {i,j} iff
 * squared distance < r^2, listed in lexicographic (i, j) order with i < j;
 * w uniform on [wlo, whi] from draw e (the edge's id) of the weight stream. */

typedef struct {
    int64_t n, G; double r2; uint32_t wlo, whi; uint64_t bw;
    double *x, *y, *z; int64_t* cell_start; int64_t* cnt; int64_t* start; edge_buf* out;
} rgg3_ctx;

static inline int64_t rgg3_axis(const rgg3_ctx* g, double a) {
    int64_t c = (int64_t)(a * (double)g->G);
    return c >= g->G ? g->G - 1 : c;
}

static void rgg3_scan_vertex(rgg3_ctx* g, int64_t i, int fill) {
    const double xi = g->x[i], yi = g->y[i], zi = g->z[i];
    const int64_t cx = rgg3_axis(g, xi), cy = rgg3_axis(g, yi), cz = rgg3_axis(g, zi);
    const int64_t G = g->G;
    int64_t e = fill ? g->start[i] : 0, k = 0;
    for (int64_t dz = -1; dz <= 1; ++dz) {
        const int64_t zz = cz + dz;
        if (zz < 0 || zz >= G) continue;
        for (int64_t dy = -1; dy <= 1; ++dy) {
            const int64_t yy = cy + dy;
            if (yy < 0 || yy >= G) continue;
            for (int64_t dx = -1; dx <= 1; ++dx) {
                const int64_t xx = cx + dx;
                if (xx < 0 || xx >= G) continue;
                const int64_t c = (zz * G + yy) * G + xx;
                for (int64_t j = g->cell_start[c]; j < g->cell_start[c + 1]; ++j) {
                    if (j <= i) continue;
                    const double ddx = g->x[j] - xi, ddy = g->y[j] - yi, ddz = g->z[j] - zi;
                    const double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
                    if (d2 < g->r2) {
                        if (fill) {
                            g->out->u[e] = (int32_t)i;
                            g->out->v[e] = (int32_t)j;
                            ++e;
                        } else {
                            ++k;
                        }
                    }
                }
            }
        }
    }
    if (!fill) g->cnt[i] = k;
}

/* The candidates of vertex i come cell by cell, so its row is sorted by j
 * after the scan; weights are drawn per edge id. */
static int cmp_i32(const void* a, const void* b) {
    const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static void rgg3_count_range(void* p, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) rgg3_scan_vertex((rgg3_ctx*)p, i, 0);
}
static void rgg3_fill_range(void* p, int64_t lo, int64_t hi) {
    rgg3_ctx* g = (rgg3_ctx*)p;
    for (int64_t i = lo; i < hi; ++i) {
        rgg3_scan_vertex(g, i, 1);
        const int64_t a = g->start[i], b = g->start[i + 1];
        qsort(g->out->v + a, (size_t)(b - a), 4, cmp_i32);
        for (int64_t e = a; e < b; ++e)
            g->out->w[e] = g->wlo + (uint32_t)below(draw(g->bw, (uint64_t)e),
                                                    (uint64_t)g->whi - g->wlo + 1);
    }
}

typedef struct { uint64_t b; double *x, *y, *z; } pts3_ctx;
static void pts3_range(void* p, int64_t lo, int64_t hi) {
    pts3_ctx* c = (pts3_ctx*)p;
    for (int64_t t = lo; t < hi; ++t) {
        c->x[t] = (double)(draw(c->b, 3 * (uint64_t)t) >> 11) * 0x1.0p-53;
        c->y[t] = (double)(draw(c->b, 3 * (uint64_t)t + 1) >> 11) * 0x1.0p-53;
        c->z[t] = (double)(draw(c->b, 3 * (uint64_t)t + 2) >> 11) * 0x1.0p-53;
    }
}

static void* rgg3_build(int64_t n, double r, uint32_t wlo, uint32_t whi, uint64_t seed,
                        int64_t* m_out) {
    if (n < 1 || n > 0x7fffffffLL || !(r > 0) || r > 1 || wlo > whi) return NULL;
    rgg3_ctx g;
    memset(&g, 0, sizeof g);
    g.n = n; g.r2 = r * r; g.wlo = wlo; g.whi = whi;
    g.bw = base(seed, TAG_RGG3_W);
    g.G = (int64_t)floor(1.0 / r);
    if (g.G < 1) g.G = 1;
    if (g.G > 1 << 10) g.G = 1 << 10;
    double* px = (double*)malloc((size_t)n * 8);
    double* py = (double*)malloc((size_t)n * 8);
    double* pz = (double*)malloc((size_t)n * 8);
    pts3_ctx pc = { base(seed, TAG_RGG3), px, py, pz };
    parallel_for(n, pts3_range, &pc);
    const int64_t ncell = g.G * g.G * g.G;
    g.cell_start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t* cellof = (int64_t*)malloc((size_t)n * 8);
    for (int64_t t = 0; t < n; ++t) {
        cellof[t] = (rgg3_axis(&g, pz[t]) * g.G + rgg3_axis(&g, py[t])) * g.G +
                    rgg3_axis(&g, px[t]);
        g.cell_start[cellof[t] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) g.cell_start[c + 1] += g.cell_start[c];
    int64_t* fillp = (int64_t*)malloc((size_t)ncell * 8);
    memcpy(fillp, g.cell_start, (size_t)ncell * 8);
    g.x = (double*)malloc((size_t)n * 8);
    g.y = (double*)malloc((size_t)n * 8);
    g.z = (double*)malloc((size_t)n * 8);
    for (int64_t t = 0; t < n; ++t) {          /* stable counting sort by cell */
        const int64_t id = fillp[cellof[t]]++;
        g.x[id] = px[t];
        g.y[id] = py[t];
        g.z[id] = pz[t];
    }
    free(fillp); free(cellof); free(px); free(py); free(pz);
    g.cnt = (int64_t*)malloc((size_t)n * 8);
    g.start = (int64_t*)malloc((size_t)(n + 1) * 8);
    parallel_for(n, rgg3_count_range, &g);
    g.start[0] = 0;
    for (int64_t i = 0; i < n; ++i) g.start[i + 1] = g.start[i] + g.cnt[i];
    const int64_t m = g.start[n];
    edge_buf* out = (edge_buf*)calloc(1, sizeof(edge_buf));
    out->m = m;
    out->u = (int32_t*)malloc((size_t)(m ? m : 1) * 4);
    out->v = (int32_t*)malloc((size_t)(m ? m : 1) * 4);
    out->w = (uint32_t*)malloc((size_t)(m ? m : 1) * 4);
    g.out = out;
    parallel_for(n, rgg3_fill_range, &g);
    free(g.x); free(g.y); free(g.z); free(g.cnt); free(g.start); free(g.cell_start);
    *m_out = m;
    return out;
}

/* --------------------------------------------------------------------- RHG */
/* Random hyperbolic graph, threshold model (Krioukov et al., Phys. Rev. E 82,
 * 2010): n points in a hyperbolic disk of radius R; angle 2 pi U, radius with
 * density alpha sinh(alpha r) / (cosh(alpha R) - 1), alpha = (gamma - 1) / 2,
 * which gives a power-law degree distribution of exponent gamma; two points
 * are adjacent iff their hyperbolic distance is below R.  Here gamma = 3
 * (alpha = 1), as in the paper's experiments, and R = 2 ln(8 n / (pi k)) for an
 * expected average degree k (the model's large-n approximation for alpha = 1).
 *
 * With alpha = 1 the inverse-CDF radius has cosh(r) = 1 + U (cosh R - 1), so
 * per point A = cosh r = 1 + U (cosh R - 1) and B = sinh r = sqrt(A^2 - 1)
 * need no transcendental beyond cosh R; the angle phi = U' in turns gives
 * C = cos(2 pi phi), S = sin(2 pi phi).  The adjacency test is plain
 * arithmetic in a fixed order,
 *     A_p A_q - B_p B_q (C_p C_q + S_p S_q) < cosh R,
 * (the hyperbolic law of cosines), so the edge set depends only on these
 * per-point values.  U from draw 2t, U' from draw 2t + 1 (53-bit mantissa).
 * Vertex ids follow angular order (by phi, then draw index), which gives the
 * graph the locality of the paper's angular partition.  Edges are listed in
 * lexicographic (i, j) order with i < j; w uniform on [wlo, whi] from draw e of
 * the weight stream.
 *
 * Search: points split into radial bands of unit width, each band sorted by
 * angle; for point p and a band whose smallest radius is b, every neighbour
 * in the band lies within the angle t with cos t = (A_p cosh b - cosh R) /
 * (B_p sinh b) (the widest angle is reached at the band's inner radius), and
 * the window is widened by 1e-9 radians so that rounding can never drop a
 * neighbour: the exact test above decides every candidate. */

typedef struct {
    int64_t n, nb; double coshR, R; uint32_t wlo, whi; uint64_t bw;
    double *A, *B, *C, *S, *phi;      /* per vertex id (angular order) */
    int64_t* band_start;              /* [nb + 1] into band_ids */
    int32_t* band_ids;                /* vertex ids of each band, by angle */
    double* band_phi;                 /* their angles */
    double* band_cosh;                /* cosh, sinh of each band's inner radius */
    double* band_sinh;
    int64_t* cnt; int64_t* start; edge_buf* out;
} rhg_ctx;

/* First index in [lo, hi) of a sorted array with value >= x. */
static int64_t lower_idx(const double* a, int64_t lo, int64_t hi, double x) {
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* The adjacency test of p and q, evaluated in this order everywhere. */
static inline int rhg_adjacent(const rhg_ctx* g, int64_t p, int64_t q) {
    return g->A[p] * g->A[q] - g->B[p] * g->B[q] * (g->C[p] * g->C[q] + g->S[p] * g->S[q]) <
           g->coshR;
}

typedef struct { int32_t* v; int64_t k, cap; } nbr_buf;

static void nbr_push(nbr_buf* b, int32_t j) {
    if (b->k == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 256;
        b->v = (int32_t*)realloc(b->v, (size_t)b->cap * 4);
    }
    b->v[b->k++] = j;
}

/* Neighbours j > i of vertex i, unsorted. */
static void rhg_neighbours(const rhg_ctx* g, int64_t i, nbr_buf* out) {
    out->k = 0;
    const double Ai = g->A[i], Bi = g->B[i], pi_ = g->phi[i];
    for (int64_t b = 0; b < g->nb; ++b) {
        const int64_t lo = g->band_start[b], hi = g->band_start[b + 1];
        if (lo == hi) continue;
        double half;                      /* window half-width in turns */
        const double den = Bi * g->band_sinh[b];
        const double c = den > 0 ? (Ai * g->band_cosh[b] - g->coshR) / den : -2.0;
        if (c <= -1.0) half = 0.5;
        else if (c >= 1.0) half = 1e-9;
        else half = acos(c) / (2.0 * GG_PI) + 1e-9;
        if (half >= 0.5) {
            for (int64_t t = lo; t < hi; ++t) {
                const int32_t j = g->band_ids[t];
                if (j <= i) continue;
                if (rhg_adjacent(g, i, j)) nbr_push(out, j);
            }
            continue;
        }
        /* angular window [pi_ - half, pi_ + half] on the circle of unit length */
        double a0 = pi_ - half, a1 = pi_ + half;
        for (int part = 0; part < 2; ++part) {
            double x0 = a0, x1 = a1;
            if (part == 0) {              /* the part inside [0, 1) */
                if (x0 < 0) x0 = 0;
                if (x1 > 1) x1 = 1;
            } else {                      /* the wrapped part, if any */
                if (a0 < 0) { x0 = a0 + 1; x1 = 1; }
                else if (a1 > 1) { x0 = 0; x1 = a1 - 1; }
                else break;
            }
            const int64_t t0 = lower_idx(g->band_phi, lo, hi, x0);
            for (int64_t t = t0; t < hi && g->band_phi[t] <= x1; ++t) {
                const int32_t j = g->band_ids[t];
                if (j <= i) continue;
                if (rhg_adjacent(g, i, j)) nbr_push(out, j);
            }
        }
    }
}

typedef struct { rhg_ctx* g; int fill; } rhg_job;

static void rhg_range(void* p, int64_t lo, int64_t hi) {
    rhg_job* jb = (rhg_job*)p;
    rhg_ctx* g = jb->g;
    nbr_buf buf = { NULL, 0, 0 };
    for (int64_t i = lo; i < hi; ++i) {
        rhg_neighbours(g, i, &buf);
        if (!jb->fill) { g->cnt[i] = buf.k; continue; }
        qsort(buf.v, (size_t)buf.k, 4, cmp_i32);
        const int64_t e0 = g->start[i];
        for (int64_t k = 0; k < buf.k; ++k) {
            const int64_t e = e0 + k;
            g->out->u[e] = (int32_t)i;
            g->out->v[e] = buf.v[k];
            g->out->w[e] = g->wlo + (uint32_t)below(draw(g->bw, (uint64_t)e),
                                                    (uint64_t)g->whi - g->wlo + 1);
        }
    }
    free(buf.v);
}

typedef struct { uint64_t b; double coshR; double *A, *phi; } rhg_pts_ctx;
static void rhg_pts_range(void* p, int64_t lo, int64_t hi) {
    rhg_pts_ctx* c = (rhg_pts_ctx*)p;
    for (int64_t t = lo; t < hi; ++t) {
        const double u = (double)(draw(c->b, 2 * (uint64_t)t) >> 11) * 0x1.0p-53;
        c->A[t] = 1.0 + u * (c->coshR - 1.0);
        c->phi[t] = (double)(draw(c->b, 2 * (uint64_t)t + 1) >> 11) * 0x1.0p-53;
    }
}

typedef struct { double phi; int64_t t; } ang_key;
static int cmp_ang(const void* a, const void* b) {
    const ang_key* x = (const ang_key*)a;
    const ang_key* y = (const ang_key*)b;
    if (x->phi != y->phi) return x->phi < y->phi ? -1 : 1;
    return (x->t > y->t) - (x->t < y->t);
}

static void* rhg_build(int64_t n, double avg_deg, uint32_t wlo, uint32_t whi, uint64_t seed,
                       int64_t* m_out) {
    if (n < 2 || n > 0x7fffffffLL || !(avg_deg > 0) || wlo > whi) return NULL;
    rhg_ctx g;
    memset(&g, 0, sizeof g);
    g.n = n; g.wlo = wlo; g.whi = whi;
    g.R = 2.0 * log(8.0 * (double)n / (GG_PI * avg_deg));
    if (!(g.R > 0)) return NULL;
    g.coshR = cosh(g.R);
    g.bw = base(seed, TAG_RHG_W);
    double* A0 = (double*)malloc((size_t)n * 8);
    double* phi0 = (double*)malloc((size_t)n * 8);
    rhg_pts_ctx pc = { base(seed, TAG_RHG), g.coshR, A0, phi0 };
    parallel_for(n, rhg_pts_range, &pc);
    ang_key* order = (ang_key*)malloc((size_t)n * sizeof(ang_key));
    for (int64_t t = 0; t < n; ++t) { order[t].phi = phi0[t]; order[t].t = t; }
    qsort(order, (size_t)n, sizeof(ang_key), cmp_ang);
    g.A = (double*)malloc((size_t)n * 8);
    g.B = (double*)malloc((size_t)n * 8);
    g.C = (double*)malloc((size_t)n * 8);
    g.S = (double*)malloc((size_t)n * 8);
    g.phi = (double*)malloc((size_t)n * 8);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t t = order[i].t;
        g.A[i] = A0[t];
        g.B[i] = sqrt(A0[t] * A0[t] - 1.0);
        g.phi[i] = phi0[t];
        g.C[i] = cos(2.0 * GG_PI * phi0[t]);
        g.S[i] = sin(2.0 * GG_PI * phi0[t]);
    }
    free(order); free(A0); free(phi0);
    /* radial bands of unit width; band of a vertex from r = acosh(A) (only the
     * search uses it: a band's inner radius bounds the window) */
    g.nb = (int64_t)ceil(g.R);
    if (g.nb < 1) g.nb = 1;
    g.band_start = (int64_t*)calloc((size_t)g.nb + 1, sizeof(int64_t));
    int32_t* bandof = (int32_t*)malloc((size_t)n * 4);
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = (int64_t)floor(acosh(g.A[i]));
        if (b >= g.nb) b = g.nb - 1;
        if (b < 0) b = 0;
        bandof[i] = (int32_t)b;
        g.band_start[b + 1]++;
    }
    for (int64_t b = 0; b < g.nb; ++b) g.band_start[b + 1] += g.band_start[b];
    g.band_ids = (int32_t*)malloc((size_t)n * 4);
    g.band_phi = (double*)malloc((size_t)n * 8);
    int64_t* fillp = (int64_t*)malloc((size_t)g.nb * 8);
    memcpy(fillp, g.band_start, (size_t)g.nb * 8);
    for (int64_t i = 0; i < n; ++i) {      /* ids ascending = angle ascending */
        const int64_t pos = fillp[bandof[i]]++;
        g.band_ids[pos] = (int32_t)i;
        g.band_phi[pos] = g.phi[i];
    }
    free(fillp); free(bandof);
    g.band_cosh = (double*)malloc((size_t)g.nb * 8);
    g.band_sinh = (double*)malloc((size_t)g.nb * 8);
    for (int64_t b = 0; b < g.nb; ++b) {
        /* a slightly smaller inner radius only widens the window */
        const double rb = b > 0 ? (double)b - 1e-9 : 0.0;
        g.band_cosh[b] = cosh(rb);
        g.band_sinh[b] = sinh(rb);
    }
    g.cnt = (int64_t*)malloc((size_t)n * 8);
    g.start = (int64_t*)malloc((size_t)(n + 1) * 8);
    rhg_job jc = { &g, 0 };
    parallel_for(n, rhg_range, &jc);
    g.start[0] = 0;
    for (int64_t i = 0; i < n; ++i) g.start[i + 1] = g.start[i] + g.cnt[i];
    const int64_t m = g.start[n];
    edge_buf* out = (edge_buf*)calloc(1, sizeof(edge_buf));
    out->m = m;
    out->u = (int32_t*)malloc((size_t)(m ? m : 1) * 4);
    out->v = (int32_t*)malloc((size_t)(m ? m : 1) * 4);
    out->w = (uint32_t*)malloc((size_t)(m ? m : 1) * 4);
    g.out = out;
    rhg_job jf = { &g, 1 };
    parallel_for(n, rhg_range, &jf);
    free(g.A); free(g.B); free(g.C); free(g.S); free(g.phi); free(g.band_start);
    free(g.band_ids); free(g.band_phi); free(g.band_cosh); free(g.band_sinh);
    free(g.cnt); free(g.start);
    *m_out = m;
    return out;
}

/* ----------------------------------------------- variable-size result handles */

void* gg_grid_build(int64_t rows, int64_t cols, double keep, int wmode, uint32_t wlo,
                    uint32_t whi, uint64_t seed, int64_t* m_out) {
    return grid_build(rows, cols, keep, wmode, wlo, whi, seed, m_out);
}

void* gg_rgg2d_build(int64_t n, double r, double wscale, uint64_t seed, int64_t* m_out) {
    return rgg_build(n, r, wscale, seed, m_out);
}

void* gg_rgg3d_build(int64_t n, double r, uint32_t wlo, uint32_t whi, uint64_t seed,
                     int64_t* m_out) {
    return rgg3_build(n, r, wlo, whi, seed, m_out);
}

void* gg_rhg_build(int64_t n, double avg_deg, uint32_t wlo, uint32_t whi, uint64_t seed,
                   int64_t* m_out) {
    return rhg_build(n, avg_deg, wlo, whi, seed, m_out);
}

/* Copies a built edge list into caller arrays of length m and releases it. */
int gg_take(void* h, int32_t* u, int32_t* v, uint32_t* w) {
    edge_buf* b = (edge_buf*)h;
    if (!b) return -1;
    memcpy(u, b->u, (size_t)b->m * 4);
    memcpy(v, b->v, (size_t)b->m * 4);
    memcpy(w, b->w, (size_t)b->m * 4);
    free(b->u); free(b->v); free(b->w); free(b);
    return 0;
}

/* ------------------------------------------------------------------ batches */
/* Many independent GNM graphs.  Graph g: n_g = round(2^(lo + (hi - lo) U)),
 * U uniform on [0, 1) from the 53-bit draw 2g of the batch stream; average
 * degree d_g = dlo + (dhi - dlo) U' from draw 2g + 1; m_g = round(n_g d_g / 2).
 * Its edges are gg_gnm(n_g, m_g, wlo, whi, seed_g) with seed_g = draw 2G + g.
 * Vertex ids are local to the graph, in [0, n_g). */
int gg_batch_plan(int64_t G, double lo, double hi, double dlo, double dhi, uint64_t seed,
                  int64_t* n_out, int64_t* m_out) {
    if (G < 0 || lo < 1 || hi < lo || dlo < 0 || dhi < dlo) return -1;
    uint64_t b = base(seed, TAG_BATCH);
    for (int64_t g = 0; g < G; ++g) {
        double u1 = (double)(draw(b, 2 * (uint64_t)g) >> 11) * 0x1.0p-53;
        double u2 = (double)(draw(b, 2 * (uint64_t)g + 1) >> 11) * 0x1.0p-53;
        int64_t n = (int64_t)llround(pow(2.0, lo + (hi - lo) * u1));
        if (n < 2) n = 2;
        double d = dlo + (dhi - dlo) * u2;
        n_out[g] = n;
        m_out[g] = (int64_t)llround((double)n * d / 2.0);
    }
    return 0;
}

typedef struct {
    const int64_t *n, *m, *eoff; int64_t G, first; uint32_t wlo, whi; uint64_t b;
    int32_t *u, *v; uint32_t* w;
} batch_ctx;

static void batch_range(void* p, int64_t lo, int64_t hi) {
    batch_ctx* c = (batch_ctx*)p;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t g = c->first + i;
        gnm_ctx gc = { c->n[g], c->wlo, c->whi,
                       base(draw(c->b, 2 * (uint64_t)c->G + (uint64_t)g), TAG_GNM),
                       c->u + c->eoff[i], c->v + c->eoff[i], c->w + c->eoff[i] };
        gnm_range(&gc, 0, c->m[g]);
    }
}

/* Fills graphs [first, first + count) of a G-graph batch planned by
 * gg_batch_plan (n, m of the whole batch); graph first + i is written at
 * offset eoff[i] of u, v, w. */
int gg_batch_fill(int64_t G, int64_t first, int64_t count, const int64_t* n, const int64_t* m,
                  const int64_t* eoff, uint32_t wlo, uint32_t whi, uint64_t seed, int32_t* u,
                  int32_t* v, uint32_t* w) {
    if (G < 0 || first < 0 || count < 0 || first + count > G || wlo > whi) return -1;
    batch_ctx c = { n, m, eoff, G, first, wlo, whi, base(seed, TAG_BATCH), u, v, w };
    int t = gg_threads();
    if (count < 2 * t) { batch_range(&c, 0, count); return 0; }
    pthread_t th[64];
    job_t jobs[64];
    int64_t chunk = (count + t - 1) / t;
    for (int i = 0; i < t; ++i) {
        jobs[i].fn = batch_range; jobs[i].ctx = &c;
        jobs[i].lo = i * chunk < count ? i * chunk : count;
        jobs[i].hi = (i + 1) * chunk < count ? (i + 1) * chunk : count;
        pthread_create(&th[i], NULL, run_job, &jobs[i]);
    }
    for (int i = 0; i < t; ++i) pthread_join(th[i], NULL);
    return 0;
}

/* Raw stream access for the bit-exactness tests of ref.py. */
uint64_t gg_draw(uint64_t seed, uint64_t tag, uint64_t k) { return draw(base(seed, tag), k); }
