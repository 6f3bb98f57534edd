/*
 * oracle/check.c -- independent certificate check of a candidate minimum
 * spanning forest (TEST INFRASTRUCTURE ONLY; shares no code with the GPU
 * library or with kruskal.c).
 *
 * A set F of edges is THE minimum spanning forest under the strict order
 * key(e) = w_e * 2^32 + e (paper Sec. II-B/II-C, ties broken consistently) iff
 *   (1) F has no self-loop and no cycle,
 *   (2) |F| = n - c, c = number of connected components of the whole graph,
 *       so F spans every component, and
 *   (3) cycle property: every other non-self-loop edge e is heavier than
 *       every F edge on the F-path between its endpoints (otherwise swapping
 *       would give a lighter forest).
 * (1)+(2) make F a spanning forest: an acyclic F with n - c edges has
 * exactly c trees, none crossing a component, hence one per component, so
 * the two ends of every edge lie in one F-tree.  (3) is the optimality
 * certificate, and it makes F unique because the order is strict.  Path
 * maxima come from binary lifting on F rooted by BFS, so the check costs
 * O((n + m) log n).
 *
 * Return value: 0 = valid MSF, 1 = self-loop in F, 2 = cycle in F,
 * 3 = |F| != n - c, 5 = cycle property violated, <0 = bad input / out of
 * memory.  (Code 4 is not used: an edge joining two F-trees cannot remain
 * once (1) and (2) hold.)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int64_t find_root(int64_t* p, int64_t x) {
    int64_t r = x;
    while (p[r] != r) r = p[r];
    while (p[x] != r) { int64_t nx = p[x]; p[x] = r; x = nx; }
    return r;
}

int oracle_msf_check(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m,
                     int64_t n, const uint8_t* mask, uint64_t* total_out, int64_t* count_out) {
    if (n < 0 || m < 0 || m > 0xffffffffLL || (n == 0 && m)) return -1;
    for (int64_t e = 0; e < m; ++e)
        if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n) return -1;
    int rc = 0;
    int64_t* comp = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    int64_t* tree = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!comp || !tree) { free(comp); free(tree); return -2; }
    for (int64_t x = 0; x < n; ++x) { comp[x] = x; tree[x] = x; }

    /* (1) no self-loop, no cycle; also the forest's total and size */
    uint64_t total = 0;
    int64_t fcount = 0;
    for (int64_t e = 0; e < m && !rc; ++e) {
        if (!mask[e]) continue;
        if (u[e] == v[e]) { rc = 1; break; }
        int64_t a = find_root(tree, u[e]), b = find_root(tree, v[e]);
        if (a == b) { rc = 2; break; }
        tree[a] = b;
        total += w[e];
        fcount++;
    }
    /* (2) |F| = n - c */
    int64_t c = n;
    for (int64_t e = 0; e < m && !rc; ++e) {
        int64_t a = find_root(comp, u[e]), b = find_root(comp, v[e]);
        if (a != b) { comp[a] = b; --c; }
    }
    if (!rc && fcount != n - c) rc = 3;
    free(comp);
    if (total_out) *total_out = total;
    if (count_out) *count_out = fcount;
    if (rc) { free(tree); return rc; }

    /* (3) cycle property via binary lifting over F */
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) if (mask[e]) { deg[u[e] + 1]++; deg[v[e] + 1]++; }
    for (int64_t x = 0; x < n; ++x) deg[x + 1] += deg[x];
    int64_t* adj = (int64_t*)malloc((size_t)(2 * fcount + 1) * sizeof(int64_t));
    int64_t* fill = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    memcpy(fill, deg, (size_t)n * sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e)
        if (mask[e]) { adj[fill[u[e]]++] = e; adj[fill[v[e]]++] = e; }
    free(fill);
    int32_t* depth = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t* par = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    uint64_t* pkey = (uint64_t*)malloc((size_t)(n + 1) * sizeof(uint64_t));
    int64_t* queue = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    for (int64_t x = 0; x < n; ++x) depth[x] = -1;
    int32_t maxdepth = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (depth[s] >= 0) continue;
        depth[s] = 0; par[s] = (int32_t)s; pkey[s] = 0;
        int64_t qh = 0, qt = 0;
        queue[qt++] = s;
        while (qh < qt) {
            int64_t x = queue[qh++];
            for (int64_t i = deg[x]; i < deg[x + 1]; ++i) {
                int64_t e = adj[i];
                int64_t y = u[e] == x ? v[e] : u[e];
                if (depth[y] >= 0) continue;
                depth[y] = depth[x] + 1;
                if (depth[y] > maxdepth) maxdepth = depth[y];
                par[y] = (int32_t)x;
                pkey[y] = ((uint64_t)w[e] << 32) | (uint64_t)e;
                queue[qt++] = y;
            }
        }
    }
    free(queue); free(adj); free(deg);
    int L = 1;
    while ((1LL << L) <= maxdepth) ++L;
    int32_t** up = (int32_t**)malloc((size_t)L * sizeof(int32_t*));
    uint64_t** mx = (uint64_t**)malloc((size_t)L * sizeof(uint64_t*));
    up[0] = par; mx[0] = pkey;
    for (int k = 1; k < L; ++k) {
        up[k] = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
        mx[k] = (uint64_t*)malloc((size_t)(n + 1) * sizeof(uint64_t));
        for (int64_t x = 0; x < n; ++x) {
            int32_t mid = up[k - 1][x];
            up[k][x] = up[k - 1][mid];
            mx[k][x] = mx[k - 1][x] > mx[k - 1][mid] ? mx[k - 1][x] : mx[k - 1][mid];
        }
    }
    for (int64_t e = 0; e < m && !rc; ++e) {
        if (mask[e] || u[e] == v[e]) continue;
        int64_t a = u[e], b = v[e];
        uint64_t best = 0;
        if (depth[a] < depth[b]) { int64_t t = a; a = b; b = t; }
        int32_t diff = depth[a] - depth[b];
        for (int k = 0; k < L; ++k)
            if (diff >> k & 1) { if (mx[k][a] > best) best = mx[k][a]; a = up[k][a]; }
        if (a != b) {
            for (int k = L - 1; k >= 0; --k) {
                if (up[k][a] != up[k][b]) {
                    if (mx[k][a] > best) best = mx[k][a];
                    if (mx[k][b] > best) best = mx[k][b];
                    a = up[k][a]; b = up[k][b];
                }
            }
            if (mx[0][a] > best) best = mx[0][a];
            if (mx[0][b] > best) best = mx[0][b];
        }
        uint64_t ke = ((uint64_t)w[e] << 32) | (uint64_t)e;
        if (!(best < ke)) rc = 5;
    }
    for (int k = 1; k < L; ++k) { free(up[k]); free(mx[k]); }
    free(up); free(mx); free(par); free(pkey); free(depth); free(tree);
    return rc;
}
