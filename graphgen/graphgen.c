/*
 * Seeded synthetic graph inputs for the k-hop neighborhood count.
 *
 * This module only produces inputs: raw edge tuples (self-loops and duplicate
 * tuples are left in, exactly as a generator emits them) and seed draws.  It
 * holds none of the traversal arithmetic; the library under test and the
 * oracle each build their own adjacency from these tuples.
 *
 * Randomness is counter based: value i of stream `tag` under seed `seed` is
 * SplitMix64's output function applied to key + (i+1)*gamma (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), with
 * key itself a SplitMix64 mix of (seed, tag).  Every edge is a pure function of
 * its index, so the output is identical at any thread count.
 *
 * Graph shapes follow the paper's benchmark datasets (Section III): a
 * Graph500-style R-MAT graph and a Twitter-like directed power-law graph.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t tag) {
    return mix64(mix64(seed) ^ (tag * GAMMA + 0x632be59bd9b4e019ULL));
}

static inline uint64_t ctr_u64(uint64_t key, uint64_t i) {
    return mix64(key + (i + 1) * GAMMA);
}

/* uniform double in [0, 1) from the top 53 bits */
static inline double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* uniform integer in [0, bound) by multiply-shift (Lemire 2019) */
static inline uint64_t below(uint64_t r, uint64_t bound) {
    return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

uint64_t gg_u64(uint64_t seed, uint64_t tag, uint64_t i) { return ctr_u64(stream_key(seed, tag), i); }

/* Fisher-Yates permutation of [0, n) driven by stream `tag`. */
int gg_permutation(int64_t n, uint64_t seed, uint64_t tag, int32_t *perm) {
    if (n < 0 || (n > 0 && !perm)) return -1;
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    uint64_t key = stream_key(seed, tag);
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)below(ctr_u64(key, (uint64_t)i), (uint64_t)i + 1);
        int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
    return 0;
}

enum { TAG_RMAT_EDGES = 1, TAG_RMAT_RELABEL = 2, TAG_CL_EDGES = 3, TAG_CL_PERM_OUT = 4,
       TAG_CL_PERM_IN = 5, TAG_SEEDS = 6 };

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) as used by the Graph500 generator:
 * `scale` recursive quadrant choices per tuple with probabilities a, b, c and
 * d = 1 - a - b - c, no noise, followed (when `relabel` is set) by a seeded
 * random relabelling of the 2^scale vertices.  Writes m = edge_factor * 2^scale tuples.
 */
int gg_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed,
            int relabel, int32_t *src, int32_t *dst) {
    if (scale < 1 || scale > 30 || edge_factor < 1 || !src || !dst) return -1;
    if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
    const int64_t n = (int64_t)1 << scale;
    const int64_t m = edge_factor * n;
    /* quadrant thresholds on a 32-bit uniform */
    const double two32 = 4294967296.0;
    const uint64_t ta = (uint64_t)(a * two32);
    const uint64_t tb = (uint64_t)((a + b) * two32);
    const uint64_t tc = (uint64_t)((a + b + c) * two32);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!perm) return -2;
    if (relabel) gg_permutation(n, seed, TAG_RMAT_RELABEL, perm);
    else for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    const uint64_t key = stream_key(seed, TAG_RMAT_EDGES);
    const int draws = (scale + 1) / 2; /* two 32-bit quadrant choices per 64-bit draw */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        uint64_t u = 0, v = 0;
        int lvl = 0;
        for (int d = 0; d < draws; ++d) {
            uint64_t r = ctr_u64(key, (uint64_t)e * (uint64_t)draws + (uint64_t)d);
            for (int h = 0; h < 2 && lvl < scale; ++h, ++lvl) {
                uint64_t x = (r >> (32 * h)) & 0xffffffffULL;
                uint64_t rb = 0, cb = 0;
                if (x < ta) { rb = 0; cb = 0; }
                else if (x < tb) { rb = 0; cb = 1; }
                else if (x < tc) { rb = 1; cb = 0; }
                else { rb = 1; cb = 1; }
                u = (u << 1) | rb;
                v = (v << 1) | cb;
            }
        }
        src[e] = perm[u];
        dst[e] = perm[v];
    }
    free(perm);
    return 0;
}

/*
 * Directed Chung-Lu power-law graph standing in for the paper's Twitter graph:
 * vertex rank i carries weight proportional to 1/(i + x); out- and in-ranks are
 * assigned by two independent seeded permutations.  Each tuple draws its
 * source and its target independently from the continuous density 1/(t + x)
 * on [0, n) by inverse transform, t = x * (exp(u * ln((n + x)/x)) - 1), and
 * takes rank floor(t).  This gives a degree distribution with exponent 2 and
 * an expected maximum degree of about m * ln(1 + 1/x) / ln((n + x)/x).
 */
int gg_chung_lu(int64_t n, int64_t m, double x, uint64_t seed, int32_t *src, int32_t *dst) {
    if (n < 1 || n > 2147483647LL || m < 0 || x <= 0 || (m > 0 && (!src || !dst))) return -1;
    int32_t *po = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!po || !pi) { free(po); free(pi); return -2; }
    gg_permutation(n, seed, TAG_CL_PERM_OUT, po);
    gg_permutation(n, seed, TAG_CL_PERM_IN, pi);
    const double L = log(((double)n + x) / x);
    const uint64_t key = stream_key(seed, TAG_CL_EDGES);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        double u1 = u01(ctr_u64(key, 2 * (uint64_t)e));
        double u2 = u01(ctr_u64(key, 2 * (uint64_t)e + 1));
        int64_t i = (int64_t)floor(x * expm1(u1 * L));
        int64_t j = (int64_t)floor(x * expm1(u2 * L));
        if (i < 0) i = 0;
        if (i >= n) i = n - 1;
        if (j < 0) j = 0;
        if (j >= n) j = n - 1;
        src[e] = po[i];
        dst[e] = pi[j];
    }
    free(po);
    free(pi);
    return 0;
}

/*
 * Seeds drawn uniformly without replacement from the vertices that touch at
 * least one tuple whose endpoints differ (in either role).  Writes `count`
 * seeds (fewer if fewer candidates exist) and returns how many were written,
 * or a negative value on error.  `candidates_out`, if not NULL, receives the
 * number of candidate vertices.
 */
int64_t gg_draw_seeds(const int32_t *src, const int32_t *dst, int64_t m, int64_t n, int64_t count,
                      uint64_t seed, uint64_t stream, int32_t *out, int64_t *candidates_out) {
    if (n < 1 || m < 0 || count < 0 || (m > 0 && (!src || !dst)) || (count > 0 && !out)) return -1;
    uint8_t *mark = (uint8_t *)calloc((size_t)n, 1);
    if (!mark) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        int32_t u = src[e], v = dst[e];
        if (u != v && u >= 0 && u < n && v >= 0 && v < n) {
            mark[u] = 1;
            mark[v] = 1;
        }
    }
    int64_t nc = 0;
    for (int64_t v = 0; v < n; ++v) nc += mark[v];
    if (candidates_out) *candidates_out = nc;
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    if (!cand) { free(mark); return -2; }
    int64_t p = 0;
    for (int64_t v = 0; v < n; ++v)
        if (mark[v]) cand[p++] = (int32_t)v;
    free(mark);
    int64_t take = count < nc ? count : nc;
    uint64_t key = stream_key(seed, TAG_SEEDS + 16 * stream);
    for (int64_t i = 0; i < take; ++i) { /* partial Fisher-Yates from the front */
        int64_t j = i + (int64_t)below(ctr_u64(key, (uint64_t)i), (uint64_t)(nc - i));
        int32_t t = cand[i];
        cand[i] = cand[j];
        cand[j] = t;
        out[i] = cand[i];
    }
    free(cand);
    return take;
}
