/*
 * ORACLE -- test infrastructure only.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may call it; the library never does.
 *
 * Plain, single-threaded CPU computation of the k-hop neighborhood count that
 * the paper benchmarks (Section III: "k-hop neighborhood count", k = 1, 2, 3, 6):
 *
 *     count(G, s, k) = | { v : 1 <= dist_G(s, v) <= k } |
 *
 * where dist_G is the unweighted shortest-path length in the graph G built
 * from raw edge tuples.  Readings of points the paper leaves open:
 *   - "within k": distances 1..k are counted, the seed itself never is;
 *   - self-loops and duplicate tuples carry no adjacency (they are dropped);
 *   - an undirected graph has each tuple in both directions, a directed graph
 *     is followed along out-edges;
 *   - k = 0 gives 0.
 * The paper computes a hop as a sparse matrix-vector product over the boolean
 * semiring masked by the complement of the visited set (Section II); after l
 * such products the visited set is exactly { v : dist(s, v) <= l }, so the
 * count is the plain breadth-first-search count computed here.
 *
 * Also returned: the traversed-edge credit TE = sum over the vertices at
 * distance 0..k-1 of their out-degree (distinct neighbors, self excluded),
 * which is what a top-down search must inspect; benchmarks divide it by time.
 *
 * A filtered form (oracle_khop_filtered) restricts the search to the vertices
 * an `allowed` array marks: a vertex other than the seed is reached only if
 * it is allowed, so paths run through allowed vertices only (the seed itself
 * is always the start).  Restricting the relation types is a filter on the
 * tuples before the adjacency is built, so it needs nothing here.
 *
 * The adjacency is built here from the tuples with its own counting sort and
 * duplicate marking; nothing is shared with the GPU library.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n;
    int64_t nnz;
    int64_t *off; /* n + 1 row offsets */
    int32_t *adj; /* distinct out-neighbors of each vertex, self excluded */
} oracle_graph;

void oracle_free(oracle_graph *g) {
    if (!g) return;
    free(g->off);
    free(g->adj);
    free(g);
}

/* Returns 0 on success, -1 on invalid arguments, -2 on allocation failure. */
int oracle_build(const int32_t *src, const int32_t *dst, int64_t m, int64_t n, int directed,
                 oracle_graph **out) {
    if (!out || n < 1 || m < 0 || (m > 0 && (!src || !dst))) return -1;
    for (int64_t e = 0; e < m; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -2;
    /* 1. count arcs per tail vertex (self-loops dropped) */
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] == dst[e]) continue;
        cnt[src[e]] += 1;
        if (!directed) cnt[dst[e]] += 1;
    }
    /* 2. exclusive prefix sum -> provisional row starts */
    int64_t *start = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!start) { free(cnt); return -2; }
    start[0] = 0;
    for (int64_t v = 0; v < n; ++v) start[v + 1] = start[v] + cnt[v];
    int64_t arcs = start[n];
    int32_t *tmp = (int32_t *)malloc((size_t)(arcs > 0 ? arcs : 1) * sizeof(int32_t));
    if (!tmp) { free(cnt); free(start); return -2; }
    /* 3. scatter arcs into their rows */
    for (int64_t v = 0; v < n; ++v) cnt[v] = start[v];
    for (int64_t e = 0; e < m; ++e) {
        int32_t u = src[e], v = dst[e];
        if (u == v) continue;
        tmp[cnt[u]++] = v;
        if (!directed) tmp[cnt[v]++] = u;
    }
    /* 4. keep the first occurrence of each neighbor per row (mark[v] = row that last saw v) */
    int64_t *mark = cnt; /* reuse: n + 1 entries */
    for (int64_t v = 0; v < n; ++v) mark[v] = -1;
    oracle_graph *g = (oracle_graph *)calloc(1, sizeof(oracle_graph));
    if (!g) { free(cnt); free(start); free(tmp); return -2; }
    g->n = n;
    g->off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!g->off) { free(cnt); free(start); free(tmp); free(g); return -2; }
    int64_t w = 0;
    g->off[0] = 0;
    for (int64_t u = 0; u < n; ++u) {
        for (int64_t i = start[u]; i < start[u + 1]; ++i) {
            int32_t v = tmp[i];
            if (mark[v] != u) {
                mark[v] = u;
                tmp[w++] = v; /* w <= i: compaction in place */
            }
        }
        g->off[u + 1] = w;
    }
    free(cnt);
    free(start);
    g->nnz = w;
    g->adj = (int32_t *)realloc(tmp, (size_t)(w > 0 ? w : 1) * sizeof(int32_t));
    if (!g->adj) { g->adj = tmp; }
    *out = g;
    return 0;
}

int64_t oracle_num_vertices(const oracle_graph *g) { return g ? g->n : -1; }
int64_t oracle_num_arcs(const oracle_graph *g) { return g ? g->nnz : -1; }

/* Out-degree (distinct neighbors, self excluded) of every vertex into deg[n]. */
int oracle_degrees(const oracle_graph *g, int64_t *deg) {
    if (!g || !deg) return -1;
    for (int64_t v = 0; v < g->n; ++v) deg[v] = g->off[v + 1] - g->off[v];
    return 0;
}

/*
 * Breadth-first search from s, expanding levels 0 .. k-1.
 * level_counts (may be NULL) receives k entries: level_counts[l-1] is the
 * number of vertices at distance exactly l.  *te (may be NULL) receives the
 * traversed-edge credit.  dist_out (may be NULL) receives n entries: the
 * distance of each vertex if it is at most k, else -1.
 * Returns the count, or -1 on invalid arguments / -2 on allocation failure.
 */
int64_t oracle_khop(const oracle_graph *g, int32_t s, int32_t k, int64_t *level_counts, int64_t *te,
                    int32_t *dist_out) {
    if (!g || s < 0 || s >= g->n || k < 0) return -1;
    const int64_t n = g->n;
    int32_t *dist = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!dist || !queue) { free(dist); free(queue); return -2; }
    for (int64_t v = 0; v < n; ++v) dist[v] = -1;
    if (level_counts)
        for (int32_t l = 0; l < k; ++l) level_counts[l] = 0;
    int64_t head = 0, tail = 0, count = 0, edges = 0;
    dist[s] = 0;
    queue[tail++] = s;
    while (head < tail) {
        int32_t u = queue[head++];
        if (dist[u] >= k) continue; /* vertices at distance k are not expanded */
        edges += g->off[u + 1] - g->off[u];
        for (int64_t i = g->off[u]; i < g->off[u + 1]; ++i) {
            int32_t v = g->adj[i];
            if (dist[v] < 0) {
                dist[v] = dist[u] + 1;
                queue[tail++] = v;
                count += 1;
                if (level_counts) level_counts[dist[v] - 1] += 1;
            }
        }
    }
    if (te) *te = edges;
    if (dist_out)
        for (int64_t v = 0; v < n; ++v) dist_out[v] = dist[v];
    free(dist);
    free(queue);
    return count;
}

/*
 * Breadth-first search from s over levels 0 .. k-1 that enters only vertices
 * with allowed[v] != 0 (allowed has n entries; the seed is exempt).  Returns
 * the number of vertices found at distance 1..k; *te (may be NULL) receives
 * the out-degree sum of the vertices expanded (distance 0..k-1).  -1 on
 * invalid arguments, -2 on allocation failure.
 */
int64_t oracle_khop_filtered(const oracle_graph *g, int32_t s, int32_t k, const uint8_t *allowed, int64_t *te) {
    if (!g || !allowed || s < 0 || s >= g->n || k < 0) return -1;
    const int64_t n = g->n;
    int32_t *dist = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!dist || !queue) { free(dist); free(queue); return -2; }
    for (int64_t v = 0; v < n; ++v) dist[v] = -1;
    int64_t head = 0, tail = 0, count = 0, edges = 0;
    dist[s] = 0;
    queue[tail++] = s;
    while (head < tail) {
        int32_t u = queue[head++];
        if (dist[u] >= k) continue;
        edges += g->off[u + 1] - g->off[u];
        for (int64_t i = g->off[u]; i < g->off[u + 1]; ++i) {
            int32_t v = g->adj[i];
            if (dist[v] < 0 && allowed[v]) {
                dist[v] = dist[u] + 1;
                queue[tail++] = v;
                count += 1;
            }
        }
    }
    if (te) *te = edges;
    free(dist);
    free(queue);
    return count;
}

/* Many seeds at one k: counts[i] (and te[i] when te is not NULL) for seeds[i]. */
int oracle_khop_many(const oracle_graph *g, const int32_t *seeds, int64_t num_seeds, int32_t k,
                     int64_t *counts, int64_t *te) {
    if (!g || num_seeds < 0 || (num_seeds > 0 && (!seeds || !counts))) return -1;
    for (int64_t i = 0; i < num_seeds; ++i) {
        int64_t t = 0;
        int64_t c = oracle_khop(g, seeds[i], k, NULL, &t, NULL);
        if (c < 0) return (int)c;
        counts[i] = c;
        if (te) te[i] = t;
    }
    return 0;
}
