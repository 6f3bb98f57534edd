/*
 * oracle/kruskal.c -- CPU oracle for the minimum spanning forest (TEST
 * INFRASTRUCTURE ONLY).
 *
 * Plain, single-threaded, deliberately unoptimised code that states what the
 * GPU library must compute.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load it.  It shares no source, header, table or helper
 * with the GPU library.
 *
 * Problem (paper Sec. II-B): for an undirected weighted multigraph output a
 * minimum spanning tree of every connected component (a minimum spanning
 * forest, MSF).  Ties between equal weights are broken consistently so the
 * MSF is unique (Sec. II-C): here edge e precedes edge f iff
 * (w_e, e) < (w_f, f) lexicographically, i.e. iff key(e) < key(f) with
 * key(e) = w_e * 2^32 + e.  Under this strict order
 *
 *     e is in the MSF  <=>  u_e != v_e and u_e, v_e are not connected by
 *                           edges that precede e.
 *
 * Kruskal's algorithm decides exactly this predicate edge by edge in key
 * order with a union-find structure, which is why it is the oracle here.
 * Vertices are 0-based ids in [0, n); edge e is (u[e], v[e], w[e]).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_EINVAL = -1, OR_ERANGE = -2, OR_ENOMEM = -3 };

/* ---------------------------------------------------------- input rules */
/* n in [0, 2^31-1], m in [0, 2^32-1], n = 0 forces m = 0, ids in [0, n). */
static int validate(const int32_t* u, const int32_t* v, int64_t m, int64_t n) {
    if (n < 0 || n > 0x7fffffffLL || m < 0 || m > 0xffffffffLL) return OR_EINVAL;
    if (n == 0 && m != 0) return OR_EINVAL;
    if (m > 0 && (!u || !v)) return OR_EINVAL;
    for (int64_t e = 0; e < m; ++e)
        if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n) return OR_ERANGE;
    return OR_OK;
}

/* ------------------------------------------------------------- sorting */
/* Ascending LSD radix sort of 64-bit keys, 16 bits per pass.  A textbook
 * counting sort per digit; passes whose digit is constant are skipped. */
static int sort_keys(uint64_t* a, int64_t k) {
    uint64_t* tmp = (uint64_t*)malloc((size_t)(k ? k : 1) * sizeof(uint64_t));
    int64_t* cnt = (int64_t*)malloc(65536 * sizeof(int64_t));
    if (!tmp || !cnt) { free(tmp); free(cnt); return OR_ENOMEM; }
    for (int shift = 0; shift < 64; shift += 16) {
        memset(cnt, 0, 65536 * sizeof(int64_t));
        for (int64_t i = 0; i < k; ++i) cnt[(a[i] >> shift) & 0xffff]++;
        int constant = 0;
        for (int d = 0; d < 65536; ++d) if (cnt[d] == k) constant = 1;
        if (constant) continue;
        int64_t sum = 0;
        for (int d = 0; d < 65536; ++d) { int64_t c = cnt[d]; cnt[d] = sum; sum += c; }
        for (int64_t i = 0; i < k; ++i) tmp[cnt[(a[i] >> shift) & 0xffff]++] = a[i];
        memcpy(a, tmp, (size_t)k * sizeof(uint64_t));
    }
    free(tmp);
    free(cnt);
    return OR_OK;
}

/* ---------------------------------------------------------- union-find */
/* Disjoint sets with path halving and union by size. */
typedef struct { int32_t* parent; int32_t* size; } dsu_t;

static int dsu_init(dsu_t* d, int64_t n) {
    d->parent = (int32_t*)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
    d->size = (int32_t*)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
    if (!d->parent || !d->size) { free(d->parent); free(d->size); return OR_ENOMEM; }
    for (int64_t x = 0; x < n; ++x) { d->parent[x] = (int32_t)x; d->size[x] = 1; }
    return OR_OK;
}
static void dsu_free(dsu_t* d) { free(d->parent); free(d->size); }
static int32_t dsu_find(dsu_t* d, int32_t x) {
    while (d->parent[x] != x) {
        d->parent[x] = d->parent[d->parent[x]];
        x = d->parent[x];
    }
    return x;
}
/* Returns 1 if a and b were in different sets (and merges them), else 0. */
static int dsu_union(dsu_t* d, int32_t a, int32_t b) {
    a = dsu_find(d, a);
    b = dsu_find(d, b);
    if (a == b) return 0;
    if (d->size[a] < d->size[b]) { int32_t t = a; a = b; b = t; }
    d->parent[b] = a;
    d->size[a] += d->size[b];
    return 1;
}

/* ------------------------------------------------------------- Kruskal */
/* mask[e] = 1 iff e is in the (w, e)-ordered MSF; *total = sum of their
 * weights; *count = number of MSF edges (= n minus the number of connected
 * components, isolated vertices included). */
int oracle_msf_kruskal(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m,
                       int64_t n, uint8_t* mask, uint64_t* total, int64_t* count) {
    int st = validate(u, v, m, n);
    if (st != OR_OK) return st;
    if (m > 0 && (!w || !mask)) return OR_EINVAL;
    if (m > 0) memset(mask, 0, (size_t)m);
    *total = 0;
    *count = 0;
    /* keys of every non-self-loop edge; self-loops never join two sets */
    uint64_t* keys = (uint64_t*)malloc((size_t)(m ? m : 1) * sizeof(uint64_t));
    if (!keys) return OR_ENOMEM;
    int64_t k = 0;
    for (int64_t e = 0; e < m; ++e)
        if (u[e] != v[e]) keys[k++] = ((uint64_t)w[e] << 32) | (uint64_t)e;
    if ((st = sort_keys(keys, k)) != OR_OK) { free(keys); return st; }
    dsu_t d;
    if ((st = dsu_init(&d, n)) != OR_OK) { free(keys); return st; }
    for (int64_t i = 0; i < k; ++i) {
        int64_t e = (int64_t)(keys[i] & 0xffffffffULL);
        if (dsu_union(&d, u[e], v[e])) {
            mask[e] = 1;
            *total += w[e];
            *count += 1;
        }
    }
    dsu_free(&d);
    free(keys);
    return OR_OK;
}

/* Number of connected components of (V, E), isolated vertices included. */
int64_t oracle_components(const int32_t* u, const int32_t* v, int64_t m, int64_t n) {
    if (validate(u, v, m, n) != OR_OK) return -1;
    dsu_t d;
    if (dsu_init(&d, n) != OR_OK) return -1;
    int64_t c = n;
    for (int64_t e = 0; e < m; ++e) c -= dsu_union(&d, u[e], v[e]);
    dsu_free(&d);
    return c;
}

/* Sorting step exposed so the tests can compare it with a library sort. */
int oracle_sort_u64(uint64_t* a, int64_t k) { return sort_keys(a, k); }
