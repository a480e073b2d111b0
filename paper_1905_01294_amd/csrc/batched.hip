// Batched multi-source k-hop count on gfx950.
//
// Up to 64*W seeds share one traversal (W = 1..16): each vertex carries W 64-bit words
// of seed bits (vertex-major, word w of vertex v at v*W + w).  A hop is then
// the boolean product of the paper's Section II with a dense bit matrix in
// place of the frontier vector,
//     N[v] = (OR over in-neighbors u of F[u]) AND NOT V[v] AND active_l,
// where active_l keeps the seeds whose own k is at least l (mixed k in one
// batch), followed by V |= N, F <- N.
//   hop 1     top-down from the seeds: a block per seed ORs its bit into the
//             out-neighbors' F and V words (atomicOr).  No mask is needed:
//             before hop 1 seed j's bit is set only at seed j, which has no
//             self-loop, so every bit pushed is new;
//   hop >= 2  bottom-up: a group of G lanes (one per active word) per vertex
//             scans the in-neighbors G at a time against a frontier bitmap
//             (one bit per vertex, L2-resident) and gathers the words F[u] of
//             the hits only, stopping as soon as every still-needed bit of
//             the vertex is found; vertices above the heavy threshold are
//             split into edge chunks of a whole wave each;
//   count     per seed column: each 64x64 bit block of V (64 vertices, one
//             word) is transposed across the wave with six butterfly
//             exchanges, so lane j's popcount is column j's count.
// Seeds arrive sorted by k (largest first), so at hop l only the leading
// words still hold active seeds and the lane groups shrink with them.
#include <algorithm>

#include "khop_impl.h"
#include "wave.h"

namespace khop {

using namespace dev;

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// Frontier bitmaps of one hop (bit v: some word of F[v] may be nonzero; a
// superset only costs gathers) and 64-lane counts of their set bits.  A hop
// reads `cur`, sets bits of `next` and clears `clear`, the bitmap of the hop
// after it.
struct FrontierBits {
    const uint64_t *cur;
    uint64_t *next;
    uint64_t *clear;
    const int64_t *cnt_cur;
    int64_t *cnt_next;
    int64_t *cnt_clear;
};
constexpr int kCntLanes = 64;
// A frontier holding more than n / kDenseDiv vertices is dense: a hop over
// one-word rows then skips the bitmap test, since most in-edges would hit.
constexpr int kDenseDiv = 16;

// Sets bit v of a frontier bitmap; returns whether this call set it.  The
// plain read skips most repeats on hubs.
__device__ __forceinline__ bool fb_set(uint64_t *fb, int32_t v) {
    const uint64_t bit = 1ull << (v & 63);
    if (fb[v >> 6] & bit) return false;
    const uint64_t old = atomicOr((unsigned long long *)&fb[v >> 6], (unsigned long long)bit);
    return !(old & bit);
}

// Adds a wave's count of newly set frontier bits (one lane calls).
__device__ __forceinline__ void fb_count(int64_t *cnt, int64_t v) {
    if (v) atomicAdd((unsigned long long *)&cnt[(blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) & (kCntLanes - 1)],
                     (unsigned long long)v);
}

// Whether the frontier counted in cnt is dense (wave-uniform).
__device__ __forceinline__ bool fb_dense(const int64_t *cnt, int64_t n) {
    return wave_sum(cnt[lane_id() & (kCntLanes - 1)]) * kDenseDiv > n;
}

// Top-down frontier of a batched hop: every vertex the hop found is appended
// as its chunks of out-edges (at least one chunk, empty for out-degree 0),
// with its out-degree added to a 64-lane sum.
constexpr int kChunk = 256;
struct ChunkQueue {
    uint64_t *rec;  // (vertex << 32) | chunk index
    int64_t *len;   // records appended
    int64_t *mf;    // out-degree sum of the appended vertices, 64 lanes
};
enum { HOP_PUSH = 0, HOP_PULL = 1 };

// Appends the chunks of v for the lanes with app set; one atomic per wave.
// Every lane of the wave must call it.
__device__ __forceinline__ void cq_append(const ChunkQueue &q, bool app, int32_t v, int64_t deg) {
    const int lane = lane_id();
    const int64_t nch = app ? std::max<int64_t>(1, (deg + kChunk - 1) / kChunk) : 0;
    const int64_t ex = wave_exclusive_sum(nch);
    const int64_t tot = shfl64(ex + nch, kWave - 1);
    if (!tot) return;  // wave-uniform
    int64_t base = 0;
    if (lane == 0) base = (int64_t)atomicAdd((unsigned long long *)q.len, (unsigned long long)tot);
    base = shfl64(base, 0);
    for (int64_t c = 0; c < nch; ++c) q.rec[base + ex + c] = ((uint64_t)(uint32_t)v << 32) | (uint64_t)c;
    const int64_t dsum = wave_sum(app ? deg : 0);
    if (lane == 0 && dsum)
        atomicAdd((unsigned long long *)&q.mf[(blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) & (kCntLanes - 1)],
                  (unsigned long long)dsum);
}

__global__ void __launch_bounds__(kBlock) batch_zero_kernel(uint64_t *a, uint64_t *b, uint64_t *c, int64_t words,
                                                           uint64_t *fb, int64_t fb_words, int64_t *fc, int64_t *acc,
                                                           int64_t nacc, int32_t *flags, int32_t *mode, int nflags,
                                                           int64_t *cq_len, int64_t *cq_mf) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < words; i += stride) {
        a[i] = 0;
        b[i] = 0;
        c[i] = 0;
    }
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < nflags; i += kBlock) mode[i] = HOP_PUSH;
        for (int i = threadIdx.x; i < 3 * kCntLanes; i += kBlock) cq_mf[i] = 0;
        if (threadIdx.x < 3) cq_len[threadIdx.x] = 0;
    }
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < fb_words; i += stride) fb[i] = 0;
    if (blockIdx.x == 0) {
        for (int64_t i = threadIdx.x; i < nacc; i += kBlock) acc[i] = 0;
        for (int i = threadIdx.x; i < nflags; i += kBlock) flags[i] = 0;
        for (int i = threadIdx.x; i < 3 * kCntLanes; i += kBlock) fc[i] = 0;
    }
}

// V gets bit j at seed j.
__global__ void __launch_bounds__(kBlock) batch_seed_kernel(uint64_t *V, const int32_t *seeds, const int32_t *perm,
                                                           int nslots, int W) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= nslots) return;
    const int32_t s = seeds[perm[j]];
    const int64_t at = (int64_t)s * W + (j >> 6);
    atomicOr((unsigned long long *)&V[at], 1ull << (j & 63));
}


// Hop 1: one block per seed slot with k >= 1 ORs its bit into F and V of each
// out-neighbor and marks the neighbor in the frontier bitmap.  A seed's row is
// split into kSeedParts spans of whole 256-edge rounds, each a work item of
// its own, so that a hub seed does not hold up the launch.
constexpr int kSeedParts = 8;
__global__ void __launch_bounds__(kBlock) batch_push_seeds_kernel(const int64_t *__restrict__ rowptr,
                                                                 const int32_t *__restrict__ colidx,
                                                                 const int32_t *seeds, const int32_t *perm,
                                                                 const int32_t *ks_sorted, int nslots, int W,
                                                                 uint64_t *F, uint64_t *V, uint64_t *fb,
                                                                 int64_t *fb_cnt, ChunkQueue q, int32_t *flag,
                                                                 const uint64_t *__restrict__ vmask) {
    int64_t fresh = 0;
    for (int64_t t = blockIdx.x; t < (int64_t)nslots * kSeedParts; t += gridDim.x) {
        const int j = (int)(t / kSeedParts), part = (int)(t % kSeedParts);
        if (ks_sorted[j] < 1) continue;
        const int32_t s = seeds[perm[j]];
        const int64_t rb = rowptr[s], re = rowptr[s + 1];
        const int64_t span = ((re - rb + kSeedParts - 1) / kSeedParts + kBlock - 1) / kBlock * kBlock;
        const int64_t b = rb + part * span, e = std::min(re, b + span);
        if (b >= e) continue;  // block-uniform
        const unsigned long long bit = 1ull << (j & 63);
        const int w = j >> 6;
        if (part == 0 && threadIdx.x == 0) atomicOr(flag, 1);
        for (int64_t x0 = b; x0 < e; x0 += kBlock) {  // block-uniform: every lane reaches the append
            const int64_t x = x0 + threadIdx.x;
            bool app = false;
            int32_t v = 0;
            int64_t deg = 0;
            if (x < e) v = colidx[x];
            // every neighbor is new, unless a vertex mask leaves it out (it is never entered)
            if (x < e && (!vmask || ((vmask[v >> 6] >> (v & 63)) & 1ull))) {
                atomicOr((unsigned long long *)&F[(int64_t)v * W + w], bit);
                atomicOr((unsigned long long *)&V[(int64_t)v * W + w], bit);
                app = fb_set(fb, v);
                if (app) deg = rowptr[v + 1] - rowptr[v];
            }
            fresh += app;
            cq_append(q, app, v, deg);
        }
    }
    fresh = wave_sum(fresh);
    if (lane_id() == 0) fb_count(fb_cnt, fresh);
}

// One-hop queries take no bit: a wave per seed tests the seed's row against
// the visited set a one-hop search starts from (the seed and, under a vertex
// mask, the vertices outside it) and counts the neighbors that pass.  A row
// holds no duplicate, so each neighbor counts once, as its bit would in the
// bit-column count.
__global__ void __launch_bounds__(kBlock) batch_row_count_kernel(const int64_t *__restrict__ rowptr,
                                                                const int32_t *__restrict__ colidx,
                                                                const int32_t *seeds, const int32_t *perm, int nq,
                                                                const uint64_t *__restrict__ vmask, int64_t *out,
                                                                int64_t *units) {
    const int lane = lane_id();
    const int q = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (q >= nq) return;  // wave-uniform
    const int32_t i = perm[q];
    const int32_t s = seeds[i];
    const int64_t b = rowptr[s], e = rowptr[s + 1];
    int64_t c = 0;
    for (int64_t x0 = b; x0 < e; x0 += kWave) {
        const int64_t x = x0 + lane;
        bool fresh = false;
        if (x < e) {
            const int32_t v = colidx[x];
            fresh = v != s && (!vmask || ((vmask[v >> 6] >> (v & 63)) & 1ull));
        }
        c += __popcll(ballot(fresh));
    }
    if (lane == 0) {
        out[i] = c;
        if (units) unit_add(units, 0, e - b);
    }
}

// Bits of the groups of G lanes that have any bit of m: bit g for group g.
template <int G>
__device__ __forceinline__ uint64_t group_any(uint64_t m) {
    if constexpr (G == 1) {
        return m;
    } else {
        constexpr uint64_t gm = (1ull << G) - 1;
        uint64_t r = 0;
#pragma unroll
        for (int g = 0; g < kWave / G; ++g)
            if ((m >> (g * G)) & gm) r |= 1ull << g;
        return r;
    }
}

// A 64-bit zero that loads of lanes with nothing to read point at, so that a
// group of loads can be issued unconditionally, all in flight at once, with
// no branch (and no wait) between them.
__device__ uint64_t kZeroWords[8] = {0, 0, 0, 0, 0, 0, 0, 0};

// The frontier word of vertex u that lane word wi gathers, or 0 when take is
// false (the load then reads the shared zero word).  With one-word rows whose
// active seeds all sit in the low 16 or 32 bits, the bottom-up kernels read a
// narrow copy Fs instead (FS = 16 or 32, else 0): a hit then costs 2 or 4
// bytes of a line shared by 64 or 32 vertices, and the copy (4 or 8 MB for two
// million vertices) stays far more in L2 than F does.
template <int FS>
__device__ __forceinline__ uint64_t frontier_word(const uint64_t *__restrict__ F, const void *__restrict__ Fs,
                                                  int64_t u, int W, int wi, bool take) {
    if constexpr (FS == 16) {
        return *(take ? (const uint16_t *)Fs + u : (const uint16_t *)kZeroWords);
    } else if constexpr (FS == 32) {
        return *(take ? (const uint32_t *)Fs + u : (const uint32_t *)kZeroWords);
    } else {
        return *(take ? F + u * W + wi : kZeroWords);
    }
}

__device__ uint64_t kOnesWords[8] = {~0ull, ~0ull, ~0ull, ~0ull, ~0ull, ~0ull, ~0ull, ~0ull};

constexpr int kPullR = 4;  // in-edges per lane per step of the bottom-up kernels (loads in flight)

// Builds that narrow copy of a one-word frontier (bits = 16 or 32); it exits
// at once when the hop went top-down or the frontier is empty.
__global__ void __launch_bounds__(kBlock) batch_frontier_copy_kernel(const uint64_t *__restrict__ F, int64_t n,
                                                                    void *Fs, int bits, const int32_t *mode_l,
                                                                    const int32_t *prev_flag) {
    if (*prev_flag == 0) return;
    if (mode_l && *mode_l == HOP_PUSH) return;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
        const uint64_t x = F[v];
        if (bits == 16) ((uint16_t *)Fs)[v] = (uint16_t)x;
        else ((uint32_t *)Fs)[v] = (uint32_t)x;
    }
}

// The bitmap tests of a step's kPullR in-edges: all loads first, then the
// bits, so that no branch separates the loads and all are in flight at once.
__device__ __forceinline__ void test_bits(const uint64_t *__restrict__ bm, const int32_t (&u)[kPullR], bool all,
                                          bool (&hit)[kPullR]) {
    uint64_t w[kPullR];
#pragma unroll
    for (int r = 0; r < kPullR; ++r) {
        const uint32_t uu = u[r] >= 0 ? (uint32_t)u[r] : 0u;
        w[r] = *(all ? kOnesWords : bm + (uu >> 6));
    }
#pragma unroll
    for (int r = 0; r < kPullR; ++r) hit[r] = u[r] >= 0 && ((w[r] >> ((uint32_t)u[r] & 63u)) & 1ull);
}

// The LDS row of a wave between the bitmap tests and the gathers of a step.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// Hop >= 2, light vertices: G lanes per vertex (lane word = lane % G).  Each
// step every lane of a group loads kPullR consecutive in-edges of the vertex
// with one 16-byte load (the group covers kPullR * G consecutive ones) and
// tests them against the frontier bitmap Fbc; the group's hits are packed
// into its part of the wave's LDS row, and each lane gathers its word of F[u]
// for four hits at a time (of the narrow copy Fs when FS is 16 or 32; with
// one lane per vertex a lane gathers its own hits, with no LDS).  Every load of a step is unconditional
// (lanes with nothing to load read a valid dummy address), so the step keeps
// kPullR loads in flight per lane instead of one.  The group stops once every
// lane holds all of its needed bits.  Vertices with a new bit are marked in
// Fbn; Fbz (the bitmap of the hop after this one) is cleared on the way.
// With `order` (ascending in-degree) the groups take the vertices in that
// order, so the groups of a wave scan lists of one length and finish
// together; without it, in id order, so that a wave's rows are contiguous and
// its vertices share one frontier bitmap word (one-word rows: the scattered
// row accesses and per-vertex bitmap claims of the sorted order cost more than
// the uneven scans).  Registers are capped for eight waves per SIMD: its
// latency is hidden by waves in flight (at seven the 1024-seed batches ran 2%
// slower).
template <int G, int FS = 0>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8)))
batch_pull_kernel(const int32_t *__restrict__ order, const int64_t *__restrict__ in_rowptr,
                  const int32_t *__restrict__ in_colidx, uint64_t *__restrict__ V, const uint64_t *__restrict__ F,
                  const void *__restrict__ Fs, uint64_t *__restrict__ Fn, int64_t n, int W, int wact,
                  const uint64_t *__restrict__ act, int heavy, int64_t first, FrontierBits fb,
                  const int32_t *mode_l, const int32_t *prev_flag, int32_t *flag, int64_t *units) {
    if (*prev_flag == 0) return;  // empty frontier: nothing left to find
    if (mode_l && *mode_l == HOP_PUSH) return;  // this hop went top-down
    {
        const int64_t nw = (n + kWave - 1) / kWave;
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nw; i += (int64_t)gridDim.x * kBlock)
            fb.clear[i] = 0;
        if (blockIdx.x == 0 && threadIdx.x < kCntLanes) fb.cnt_clear[threadIdx.x] = 0;
    }
    const uint64_t *__restrict__ Fbc = fb.cur;
    // skipping the bitmap test pays only with one-word rows: a wider row costs
    // far more to gather than the test
    const bool dense = wact == 1 && fb_dense(fb.cnt_cur, n);
    constexpr int VPW = kWave / G;       // vertices per wave
    constexpr int SLOTS = kPullR * G;    // hits a group can hold per step
    __shared__ int32_t s_hit[kWavesPerBlock][kPullR * kWave];
    __shared__ int32_t s_junk[kWavesPerBlock][kWave];
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    const int grp = lane / G;
    const int wi = lane % G;
    const uint64_t grp_bits = ((G == 64) ? ~0ull : ((1ull << G) - 1)) << (grp * G);
    const uint64_t below = lane == 0 ? 0ull : ((~0ull) >> (kWave - lane));  // lanes below this one
    const uint64_t actw = wi < wact ? act[wi] : 0ull;
    int32_t *const hits = &s_hit[wv][grp * SLOTS];
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    bool any = false;
    int64_t examined = 0, scanned = 0, gathered = 0, fresh = 0;
    for (int64_t wvi = (int64_t)blockIdx.x * kWavesPerBlock + wv; first + wvi * VPW < n; wvi += nwaves) {
        const int64_t idx = first + wvi * VPW + grp;
        const int64_t v = idx >= n ? n : order ? order[idx] : idx;
        const bool valid = v < n && wi < wact;
        const int64_t at = v * W + wi;
        uint64_t need = 0;
        int64_t b = 0, e = 0;
        if (valid) need = ~V[at] & actw;
        // the group works on v only if some lane still needs a bit
        const bool grp_need = (ballot(need != 0) & grp_bits) != 0;
        if (grp_need && v < n) {
            b = in_rowptr[v];
            e = in_rowptr[v + 1];
            if (e - b > heavy) e = b;  // the heavy kernel takes it
        }
        uint64_t acc = 0;
        bool active = grp_need && (e > b);
        if (active) scanned += (wi == 0);
        int64_t x0 = b;
        while (ballot(active)) {
            // the step's in-edge loads, all issued before any is used: the
            // indices first (some group of the wave is active, so the graph
            // has arcs and index 0 exists), then the loads, then the selects
            // lane wi takes in-edges x0 + 4 wi .. x0 + 4 wi + 3 of the group's
            // 4 G, in one 16-byte load
            const int64_t base = x0 + (int64_t)kPullR * wi;
            const int64_t left = active ? e - base : 0;  // of them, those before the vertex's end
            static_assert(kPullR == 4, "one 16-byte load per lane and step");
            const i32x4_u q = load4(in_colidx, left > 0 ? base : 0);
            int32_t u[kPullR];
#pragma unroll
            for (int r = 0; r < kPullR; ++r) u[r] = r < left ? q[r] : -1;
            bool hit[kPullR];
            test_bits(Fbc, u, dense, hit);
            // a lane whose word already holds every needed bit gathers nothing
            // (it reads the zero word instead)
            const bool lane_open = (acc & need) != need;
            if constexpr (G == 1) {
                // a lane is its own group: it gathers its own hits, four in flight
                uint64_t f[kPullR];
                int nh = 0;
#pragma unroll
                for (int r = 0; r < kPullR; ++r) {
                    const bool take = hit[r] && lane_open;
                    f[r] = frontier_word<FS>(F, Fs, take ? u[r] : 0, W, wi, take);
                    nh += hit[r];
                }
                acc |= (f[0] | f[1]) | (f[2] | f[3]);
                gathered += nh;
            } else {
                // pack the group's hits into its LDS slots (misses write to
                // the lane's junk slot: no branch)
                int nh = 0;
#pragma unroll
                for (int r = 0; r < kPullR; ++r) {
                    const uint64_t hm = ballot(hit[r]) & grp_bits;
                    *(hit[r] ? &hits[nh + __popcll(hm & below)] : &s_junk[wv][lane]) = u[r];
                    nh += __popcll(hm);
                }
                wave_lds_sync();
                // four gathers in flight per lane
                for (int j0 = 0; ballot(j0 < nh); j0 += 4) {
                    uint64_t f[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const bool take = j0 + q < nh && lane_open;
                        const int32_t hu = hits[take ? j0 + q : 0];  // an index inside the group's slots either way
                        f[q] = frontier_word<FS>(F, Fs, take ? hu : 0, W, wi, take);
                    }
                    acc |= (f[0] | f[1]) | (f[2] | f[3]);
                }
                if (wi == 0) gathered += nh;
                wave_lds_sync();  // the slots are rewritten next step only after every lane has read them
            }
            if (active) {
                if (wi == 0) examined += std::min<int64_t>((int64_t)SLOTS, e - x0);
                x0 += SLOTS;
                if (x0 >= e) active = false;
            }
            // the group stops once every lane holds all of its needed bits
            const bool ok = (acc & need) == need;
            if ((ballot(!ok) & grp_bits) == 0) active = false;
        }
        uint64_t nx = 0;
        if (valid && grp_need) {
            nx = acc & need;
            Fn[at] = nx;
            if (nx) {
                V[at] |= nx;
                any = true;
            }
        } else if (valid) {
            Fn[at] = 0;
        }
        const uint64_t gm = group_any<G>(ballot(nx != 0));
        if (order) {
            // one bitmap claim per vertex with a new bit (the lane of its word 0)
            if (wi == 0 && ((gm >> grp) & 1ull) && fb_set(fb.next, (int32_t)v)) ++fresh;
        } else if (gm && lane == 0) {
            const int64_t v0 = wvi * VPW;  // (id order: first is 0) VPW divides 64: the wave's vertices share one bitmap word
            const uint64_t old = atomicOr((unsigned long long *)&fb.next[v0 >> 6], (unsigned long long)(gm << (v0 & 63)));
            fresh += __popcll(gm << (v0 & 63) & ~old);
        }
    }
    fresh = wave_sum(fresh);  // counted by the lanes of word 0, or by lane 0
    if (lane == 0) fb_count(fb.cnt_next, fresh);
    if (ballot(any) && lane == 0) atomicOr(flag, 1);
    if (units) {
        const int64_t ex = wave_sum(examined), sc = wave_sum(scanned), ga = wave_sum(gathered);
        if (lane == 0) {
            unit_add(units, 1, ex);
            unit_add(units, 2, sc);
            unit_add(units, 3, ga);
        }
    }
}

template <int G>
__device__ __forceinline__ uint64_t subgroup_or(uint64_t v) {
#pragma unroll
    for (int off = G; off < kWave; off <<= 1) v |= (uint64_t)__shfl_xor((long long)v, off, kWave);
    return v;
}

// Hop >= 2, heavy vertices: one wave per edge chunk of a heavy vertex.  The
// wave loads 64 in-edges per round, four rounds at a time, tests them against
// the frontier bitmap, packs the hits of the four rounds in LDS and gathers
// their words with 64/G streams of G lanes, four hits per stream at a time;
// every load is unconditional, so a lane keeps four in flight.  The chunk's
// findings are ORed into the vertex's next-frontier and visited words
// atomically (the light kernel left zeros).  FS as in the light kernel.
template <int G, int FS = 0>
__global__ void __launch_bounds__(kBlock) batch_pull_heavy_kernel(
    const int32_t *__restrict__ in_colidx, uint64_t *V, const uint64_t *__restrict__ F, const void *__restrict__ Fs,
    uint64_t *Fn, int W, int wact,
    const uint64_t *__restrict__ act, const int32_t *__restrict__ hvert, const int64_t *__restrict__ hbegin,
    const int64_t *__restrict__ hend, int64_t n_items, int64_t n, FrontierBits fb, const int32_t *mode_l,
    const int32_t *prev_flag, int32_t *flag, int64_t *units) {
    if (*prev_flag == 0) return;
    if (mode_l && *mode_l == HOP_PUSH) return;  // this hop went top-down
    const uint64_t *__restrict__ Fbc = fb.cur;
    // skipping the bitmap test pays only with one-word rows: a wider row costs
    // far more to gather than the test
    const bool dense = wact == 1 && fb_dense(fb.cnt_cur, n);
    constexpr int S = kWave / G;  // gather streams
    __shared__ int32_t s_hit[kWavesPerBlock][kPullR * kWave];
    __shared__ int32_t s_junk[kWavesPerBlock][kWave];
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    const int wi = lane % G;
    const int sg = lane / G;
    const uint64_t actw = wi < wact ? act[wi] : 0ull;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    bool any = false;
    int64_t examined = 0, gathered = 0, fresh = 0;
    for (int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + wv; i < n_items; i += nwaves) {
        // the chunk's record in one round trip, then its vertex's visited word
        const int64_t v = hvert[i], b = hbegin[i], e = hend[i];  // e > b
        const int64_t at = v * W + wi;
        uint64_t need = 0;
        if (wi < wact) need = ~__hip_atomic_load(&V[at], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & actw;
        if (!ballot(need != 0)) continue;
        uint64_t acc = 0, full = 0;
        for (int64_t x0 = b; x0 < e; x0 += kPullR * kWave) {
            int32_t u[kPullR];
#pragma unroll
            for (int r = 0; r < kPullR; ++r) {
                const int64_t x = x0 + r * kWave + lane;
                const int32_t uu = in_colidx[x < e ? x : b];
                u[r] = x < e ? uu : -1;
            }
            bool hit[kPullR];
            test_bits(Fbc, u, dense, hit);
            // words that hold every needed bit (over all lanes, as of the last
            // round) are not gathered again
            const bool lane_open = (full & need) != need;
            int nh = 0;
            if constexpr (G == 1) {
                // one-word rows: every lane gathers its own hits, four in flight
                uint64_t f[kPullR];
#pragma unroll
                for (int r = 0; r < kPullR; ++r) {
                    const bool take = hit[r] && lane_open;
                    f[r] = frontier_word<FS>(F, Fs, take ? u[r] : 0, W, wi, take);
                    nh += __popcll(ballot(hit[r]));
                }
                acc |= (f[0] | f[1]) | (f[2] | f[3]);
            } else {
                // pack the hits of the four rounds, in order, into the wave's
                // LDS row (misses write to the lane's junk slot: no branch)
#pragma unroll
                for (int r = 0; r < kPullR; ++r) {
                    const uint64_t hm = ballot(hit[r]);
                    *(hit[r] ? &s_hit[wv][nh + mask_rank(hm)] : &s_junk[wv][lane]) = u[r];
                    nh += __popcll(hm);
                }
                wave_lds_sync();
                // stream sg takes hits sg, sg + S, ...: four of its hits in flight at a time
                for (int j0 = sg; j0 < nh; j0 += 4 * S) {
                    uint64_t f[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int j = j0 + q * S;
                        const bool take = j < nh && lane_open;
                        const int32_t hu = s_hit[wv][take ? j : 0];  // an index inside the wave's row either way
                        f[q] = frontier_word<FS>(F, Fs, take ? hu : 0, W, wi, take);
                    }
                    acc |= (f[0] | f[1]) | (f[2] | f[3]);
                }
                wave_lds_sync();  // the row is rewritten next round only after every lane has read it
            }
            gathered += nh;
            examined += std::min<int64_t>(kPullR * kWave, e - x0);
            full = subgroup_or<G>(acc);
            if (!ballot((full & need) != need)) break;
        }
        acc = subgroup_or<G>(acc);
        const uint64_t nx = (sg == 0 && wi < wact) ? (acc & need) : 0ull;
        if (nx) {
            atomicOr((unsigned long long *)&Fn[at], (unsigned long long)nx);
            atomicOr((unsigned long long *)&V[at], (unsigned long long)nx);
            any = true;
        }
        if (ballot(nx != 0) && lane == 0) fresh += fb_set(fb.next, (int32_t)v);
    }
    if (lane == 0) fb_count(fb.cnt_next, fresh);
    if (ballot(any) && lane == 0) atomicOr(flag, 1);
    if (units && lane == 0) {
        unit_add(units, 1, examined);
        unit_add(units, 3, gathered);
    }
}

// Hop >= 2, top-down: one wave per chunk of the previous hop's queue, a group
// of G lanes (one per active word) per out-edge, so a round covers 64/G
// edges.  A word's candidate bits F[u] & active & NOT V[v] are claimed with
// atomicOr on V (the old value keeps each bit exactly-once) and ORed into N;
// a vertex gaining any bit is appended (its bitmap bit makes that once).
// Every block first takes the direction: top-down while the frontier's
// out-edges stay at most nnz / push_div, and with `sticky` never again once a
// hop has gone bottom-up.  Block 0 records it for the hop's other kernels and
// resets the queue the next hop appends to (qreset; read and written by no
// other kernel of this hop).
//
// N is not cleared between hops: a bit it still holds from an earlier hop
// sits on a vertex its seed had already reached, whose neighbors the seed has
// reached by now too, so the bit can never claim anything.
template <int G>
__global__ void __launch_bounds__(kBlock) batch_push_kernel(
    const int64_t *__restrict__ rowptr, const int32_t *__restrict__ colidx, uint64_t *V,
    const uint64_t *__restrict__ F, uint64_t *N, int64_t n, int64_t nnz, int W, int wact,
    const uint64_t *__restrict__ act, int push_div, ChunkQueue qin, ChunkQueue qout, ChunkQueue qreset,
    FrontierBits fb, const int32_t *mode_prev, int32_t *mode_l, const int32_t *prev_flag, int32_t *flag,
    int64_t *units) {
    if (*prev_flag == 0) return;
    const int lane = lane_id();
    const int64_t mf = wave_sum(qin.mf[lane & (kCntLanes - 1)]);
    const bool pull = (mode_prev && *mode_prev == HOP_PULL) || mf * (int64_t)push_div > nnz;
    if (blockIdx.x == 0 && threadIdx.x < kCntLanes) {
        if (threadIdx.x == 0) *mode_l = pull ? HOP_PULL : HOP_PUSH;
        qreset.mf[threadIdx.x] = 0;
        if (threadIdx.x == 0) *qreset.len = 0;
    }
    if (pull) return;
    {
        const int64_t nw = (n + kWave - 1) / kWave;
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nw; i += (int64_t)gridDim.x * kBlock)
            fb.clear[i] = 0;
        if (blockIdx.x == 0 && threadIdx.x < kCntLanes) fb.cnt_clear[threadIdx.x] = 0;
    }
    constexpr int EPR = kWave / G;  // out-edges per round, one per group
    const int grp = lane / G;
    const int wi = lane % G;
    const uint64_t grp_bits = ((G == 64) ? ~0ull : ((1ull << G) - 1)) << (grp * G);
    const uint64_t actw = wi < wact ? act[wi] : 0ull;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t nrec = *qin.len;
    bool any = false;
    int64_t fresh = 0, edges = 0;
    for (int64_t c = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; c < nrec; c += nwaves) {
        const uint64_t rec = qin.rec[c];
        const int32_t u = (int32_t)(rec >> 32);
        const int64_t rb = rowptr[u], re = rowptr[u + 1];
        const int64_t b = rb + (int64_t)(rec & 0xffffffffull) * kChunk, e = std::min<int64_t>(b + kChunk, re);
        const uint64_t fu = wi < wact ? (F[(int64_t)u * W + wi] & actw) : 0ull;
        if (!ballot(fu != 0)) continue;  // wave-uniform: the source holds no active bit
        edges += e - b;
        for (int64_t x0 = b; x0 < e; x0 += EPR) {
            const int64_t x = x0 + grp;
            const bool ve = x < e;
            const int32_t v = ve ? colidx[x] : 0;
            uint64_t newb = 0;
            if (ve && fu) {
                const int64_t at = (int64_t)v * W + wi;
                const uint64_t cand = fu & ~V[at];
                if (cand) {
                    const uint64_t old = atomicOr((unsigned long long *)&V[at], (unsigned long long)cand);
                    newb = cand & ~old;
                    if (newb) atomicOr((unsigned long long *)&N[at], (unsigned long long)newb);
                }
            }
            const bool gnew = (ballot(newb != 0) & grp_bits) != 0;
            bool app = false;
            int64_t deg = 0;
            if (gnew && wi == 0 && fb_set(fb.next, v)) {
                app = true;
                deg = rowptr[v + 1] - rowptr[v];
            }
            any |= gnew;
            fresh += app;
            cq_append(qout, app, v, deg);
        }
    }
    fresh = wave_sum(fresh);
    if (lane == 0) fb_count(fb.cnt_next, fresh);
    if (ballot(any) && lane == 0) atomicOr(flag, 1);
    // 4 B per out-edge and 8 B per active word of its head's visited row
    if (units && lane == 0) unit_add(units, 1, edges);
}

// One butterfly stage of a 64x64 bit transpose held one row per lane: the
// block of columns with bit s clear in the rows with bit s set trades places
// with the block of columns with bit s set in the rows with bit s clear.
__device__ __forceinline__ uint64_t transpose_stage(uint64_t x, int s, uint64_t lo) {
    const uint64_t y = (uint64_t)__shfl_xor((long long)x, s, kWave);
    return (lane_id() & s) ? ((x & ~lo) | ((y & ~lo) >> s)) : ((x & lo) | ((y & lo) << s));
}

// Lane i holds row i on entry; lane j holds column j (bit i = row i's bit j) on return.
__device__ __forceinline__ uint64_t transpose64(uint64_t x) {
    x = transpose_stage(x, 32, 0x00000000FFFFFFFFull);
    x = transpose_stage(x, 16, 0x0000FFFF0000FFFFull);
    x = transpose_stage(x, 8, 0x00FF00FF00FF00FFull);
    x = transpose_stage(x, 4, 0x0F0F0F0F0F0F0F0Full);
    x = transpose_stage(x, 2, 0x3333333333333333ull);
    x = transpose_stage(x, 1, 0x5555555555555555ull);
    return x;
}

// counts_acc[w*64 + bit] += number of vertices whose word w has that bit, for
// words w0 .. w0 + nwords - 1 (at most 16) of rows W words long.  A wave takes
// 64 vertices at a time and all the words asked for: lane i loads vertex i's
// words (one row, so the words after the first come from lines already in
// cache), and for each word the wave's 64 values are transposed and popcounted.
// With a vertex mask (vmask, one bit per vertex) only the vertices in it are counted.
constexpr int kCountMaxWords = 16;
__global__ void __launch_bounds__(kBlock) batch_count_kernel(const uint64_t *__restrict__ V, int64_t n, int W, int w0,
                                                            int nwords, const uint64_t *__restrict__ vmask,
                                                            int64_t *counts_acc) {
    const int lane = lane_id();
    __shared__ int64_t s_acc[kWavesPerBlock][kWave];
    int64_t acc[kCountMaxWords];
#pragma unroll
    for (int j = 0; j < kCountMaxWords; ++j) acc[j] = 0;
    const int64_t nchunks = (n + kWave - 1) / kWave;
    for (int64_t c = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; c < nchunks;
         c += (int64_t)gridDim.x * kWavesPerBlock) {
        const int64_t v = c * kWave + lane;
        const bool in = v < n && (!vmask || ((vmask[c] >> lane) & 1ull));
        const uint64_t *row = V + (in ? v : 0) * W + w0;
        uint64_t x[kCountMaxWords];
#pragma unroll
        for (int j = 0; j < kCountMaxWords; ++j) x[j] = j < nwords ? row[j] : 0ull;  // (vertex 0's row when out)
#pragma unroll
        for (int j = 0; j < kCountMaxWords; ++j) x[j] = in ? x[j] : 0ull;
#pragma unroll
        for (int j = 0; j < kCountMaxWords; ++j)
            if (j < nwords && ballot(x[j] != 0)) acc[j] += __popcll(transpose64(x[j]));
    }
#pragma unroll
    for (int j = 0; j < kCountMaxWords; ++j) {
        if (j >= nwords) break;
        s_acc[threadIdx.x / kWave][lane] = acc[j];
        __syncthreads();
        if (threadIdx.x < kWave) {
            int64_t t = 0;
            for (int i = 0; i < kWavesPerBlock; ++i) t += s_acc[i][threadIdx.x];
            if (t) atomicAdd((unsigned long long *)&counts_acc[(w0 + j) * kWave + threadIdx.x], (unsigned long long)t);
        }
        __syncthreads();
    }
}

// Repacks rows of W words to their first Wn words: Vn[v*Wn + w] = V[v*W + w],
// likewise F.  The destination does not overlap the sources.
__global__ void __launch_bounds__(kBlock) batch_narrow_kernel(const uint64_t *__restrict__ V,
                                                             const uint64_t *__restrict__ F, int64_t n, int W, int Wn,
                                                             uint64_t *__restrict__ Vn, uint64_t *__restrict__ Fn) {
    const int64_t total = n * Wn;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const int64_t v = i / Wn, w = i - v * Wn;
        Vn[i] = V[v * W + w];
        Fn[i] = F[v * W + w];
    }
}

// A slot's count less its seed, which the count includes unless a vertex mask left the seed out.
__global__ void batch_output_kernel(const int64_t *counts_acc, const int32_t *perm, int nslots,
                                    const int32_t *seeds, const uint64_t *vmask, int64_t *out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nslots) return;
    const int32_t s = seeds[perm[j]];
    const int64_t self = (!vmask || ((vmask[s >> 6] >> (s & 63)) & 1ull)) ? 1 : 0;
    out[perm[j]] = counts_acc[j] - self;
}

// With a vertex mask: every seed starts with the vertices outside the mask
// visited (all bits of their rows set), so no hop enters them.
__global__ void __launch_bounds__(kBlock) batch_mask_kernel(uint64_t *V, int64_t n, int W,
                                                           const uint64_t *__restrict__ vmask) {
    const int64_t total = n * W;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const int64_t v = i / W;
        if (!((vmask[v >> 6] >> (v & 63)) & 1ull)) V[i] = ~0ull;
    }
}

__global__ void __launch_bounds__(kBlock) fill_zero_u64(uint64_t *a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) a[i] = 0;
}

}  // namespace

struct BatchCtx {
    khop_graph *g = nullptr;
    int W = 0;  // words per vertex (1..16)
    uint64_t *V = nullptr, *F = nullptr, *N = nullptr;
    void *Fs = nullptr;        // narrow copy of a one-word frontier (n uint16 or uint32)
    uint64_t *Fb = nullptr;    // three frontier bitmaps of nw words each (hop l uses slot l % 3)
    int64_t *Fc = nullptr;     // their set-bit counts, 64 lanes each
    int64_t *acc = nullptr;    // 64 * W counters
    uint64_t *act = nullptr;   // kActRows * W active masks, one row per distinct set of active seeds
    int32_t *flags = nullptr;  // kRing frontier-nonempty flags, level l at l % kRing
    int32_t *mode = nullptr;   // kRing hop directions (HOP_PUSH / HOP_PULL), level l at l % kRing
    uint64_t *cq_rec[3] = {};  // top-down chunk queues by hop % 3
    int64_t *cq_len = nullptr; // their lengths
    int64_t *cq_mf = nullptr;  // their out-degree sums, 64 lanes each
    int32_t *perm = nullptr;   // slot -> caller index
    int32_t *ks = nullptr;     // k per slot (sorted)
    void *arena = nullptr;
    // pinned staging of the per-batch tables, reusable once stage_ev has fired
    uint64_t *h_act = nullptr;
    int32_t *h_perm = nullptr;
    int32_t *h_ks = nullptr;
    void *h_arena = nullptr;
    hipEvent_t stage_ev = nullptr;
    // Per-level records live in a ring: a hop reads its own level's and the
    // level before's, and the run clears ring slots ahead of the levels that
    // reuse them, so traversals of any depth fit.
    static constexpr int kRing = 4096;
    int act_rows = 0;          // 64 * W + 1: seeds sorted by k make the active sets a chain of prefixes
};

// The layout of a batch context's device arena: its total bytes, and when
// base is not null, every device pointer of c set into it.
static size_t batch_layout(int64_t n, int64_t nnz, int words, BatchCtx *c, char *base) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t bits = al((size_t)n * words * 8);
    const int act_rows = 64 * words + 1;
    size_t off = 0;
    const size_t oV = off;
    off += bits;
    const size_t oF = off;
    off += bits;
    const size_t oN = off;
    off += bits;
    const size_t oFb = off;
    off += al(3 * (size_t)((n + 63) / 64) * 8);
    const size_t oFs = off;
    off += al((size_t)n * 4);
    const size_t oFc = off;
    off += al(3 * kCntLanes * 8);
    const size_t oacc = off;
    off += al(64 * (size_t)words * 8);
    const size_t oact = off;
    off += al((size_t)act_rows * words * 8);
    const size_t oflags = off;
    off += al(BatchCtx::kRing * 4);
    const size_t omode = off;
    off += al(BatchCtx::kRing * 4);
    const int64_t cq_cap = n + nnz / kChunk + kWave;
    size_t ocq[3];
    for (int i = 0; i < 3; ++i) {
        ocq[i] = off;
        off += al((size_t)cq_cap * 8);
    }
    const size_t ocql = off;
    off += al(3 * 8);
    const size_t ocqm = off;
    off += al(3 * kCntLanes * 8);
    const size_t operm = off;
    off += al(64 * (size_t)words * 4);
    const size_t oks = off;
    off += al(64 * (size_t)words * 4);
    if (!base) return off;
    c->arena = base;
    c->act_rows = act_rows;
    c->V = (uint64_t *)(base + oV);
    c->F = (uint64_t *)(base + oF);
    c->N = (uint64_t *)(base + oN);
    c->Fb = (uint64_t *)(base + oFb);
    c->Fs = (void *)(base + oFs);
    c->Fc = (int64_t *)(base + oFc);
    c->acc = (int64_t *)(base + oacc);
    c->act = (uint64_t *)(base + oact);
    c->flags = (int32_t *)(base + oflags);
    c->mode = (int32_t *)(base + omode);
    for (int i = 0; i < 3; ++i) c->cq_rec[i] = (uint64_t *)(base + ocq[i]);
    c->cq_len = (int64_t *)(base + ocql);
    c->cq_mf = (int64_t *)(base + ocqm);
    c->perm = (int32_t *)(base + operm);
    c->ks = (int32_t *)(base + oks);
    return off;
}

size_t batch_ctx_bytes(int64_t n, int64_t nnz, int words) { return batch_layout(n, nnz, words, nullptr, nullptr); }

BatchCtx *batch_ctx_create(khop_graph *g, int words) {
    BatchCtx *c = new BatchCtx();
    c->g = g;
    c->W = words;
    const size_t bytes = batch_layout(g->n, g->nnz, words, c, nullptr);
    void *arena = nullptr;
    if (hipMalloc(&arena, bytes) != hipSuccess) {
        delete c;
        (void)hipGetLastError();
        fail(KHOP_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes for a batch context failed");
    }
    batch_layout(g->n, g->nnz, words, c, (char *)arena);
    const size_t hbytes = (size_t)c->act_rows * words * 8 + 2 * 64 * (size_t)words * 4;
    if (hipHostMalloc(&c->h_arena, hbytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(c->arena);
        delete c;
        fail(KHOP_ENOMEM, "pinned host allocation for a batch context failed");
    }
    c->h_act = (uint64_t *)c->h_arena;
    c->h_perm = (int32_t *)(c->h_act + (size_t)c->act_rows * words);
    c->h_ks = c->h_perm + 64 * words;
    KHOP_HIP(hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming));
    KHOP_HIP(hipEventRecord(c->stage_ev, nullptr));
    return c;
}

void batch_ctx_destroy(BatchCtx *c) {
    if (!c) return;
    if (c->stage_ev) {
        (void)hipEventSynchronize(c->stage_ev);
        (void)hipEventDestroy(c->stage_ev);
    }
    if (c->h_arena) (void)hipHostFree(c->h_arena);
    if (c->arena) (void)hipFree(c->arena);
    delete c;
}

int batch_ctx_words(const BatchCtx *c) { return c->W; }

// The per-level records one hop of a batch run uses: the active seeds' bits
// of the level, and the ring slots of the level's and the previous level's
// direction and frontier-nonempty flag.
struct LevelCtl {
    const uint64_t *act;
    const int32_t *mode_prev;
    int32_t *mode_l;
    const int32_t *flag_prev;
    int32_t *flag_l;
};

static int ring_slot(int64_t L) { return (int)(L % BatchCtx::kRing); }

static LevelCtl level_ctl(BatchCtx *c, int64_t L, const uint64_t *act) {
    return LevelCtl{act, c->mode + ring_slot(L - 1), c->mode + ring_slot(L), c->flags + ring_slot(L - 1),
                    c->flags + ring_slot(L)};
}

static FrontierBits frontier_bits(BatchCtx *c, int64_t n, int64_t L) {
    const int64_t nw = (n + 63) / 64;
    const int a = (int)((L - 1) % 3), b = (int)(L % 3), z = (int)((L + 1) % 3);
    return FrontierBits{c->Fb + a * nw, c->Fb + b * nw, c->Fb + z * nw,
                        c->Fc + a * kCntLanes, c->Fc + b * kCntLanes, c->Fc + z * kCntLanes};
}

template <int G>
static void launch_pull(khop_graph *g, BatchCtx *c, const HeavyTable &ht, int grid_per_cu, int64_t L,
                        const LevelCtl &lc, int wact, int Wr, hipStream_t st, uint64_t *V, uint64_t *F, uint64_t *Fn,
                        int fs_bits) {
    const int64_t n = g->n, nw = (n + 63) / 64;
    // rows of two or more words: the vertices by in-degree (one-word rows: in
    // id order), past those with no in-edge, whose rows only ever hold zeros
    // (F and N start zero, and no hop can find such a vertex)
    int64_t first = 0;
    const int32_t *order = G >= 2 ? in_degree_order(g, &first) : nullptr;
    const int64_t waves_needed = (n - first + (kWave / G) - 1) / (kWave / G);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((waves_needed + kWavesPerBlock - 1) / kWavesPerBlock,
                                                                 (int64_t)g->cu_count * grid_per_cu));
    const FrontierBits fb = frontier_bits(c, n, L);
    {
        ProfScope ps(g, KK_BATCH_PULL, st);
        auto k = fs_bits == 16 ? batch_pull_kernel<G, 16> : fs_bits == 32 ? batch_pull_kernel<G, 32>
                                                                           : batch_pull_kernel<G, 0>;
        hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, st, order, g->d_in_rowptr, g->d_in_colidx, V, F,
                           (const void *)c->Fs, Fn, n, Wr, wact, lc.act, ht.threshold, first, fb, lc.mode_l,
                           lc.flag_prev, lc.flag_l, ps.units());
        // bytes: V read and write-back and Fn write per active word of the vertices taken, the frontier bitmap once,
        // 4 per examined in-edge, 16 per scanned vertex, 8 per gathered word (fs_bits / 8 from the narrow copy)
        const double gw = fs_bits ? fs_bits / 8.0 : 8.0 * wact;
        ps.end(3.0 * 8.0 * (double)(n - first) * wact + 2.0 * 8.0 * nw, 0, 4.0, 16.0, gw);
    }
    if (ht.n > 0) {
        const int hgrid = (int)std::max<int64_t>(
            1, std::min<int64_t>((ht.n + kWavesPerBlock - 1) / kWavesPerBlock, (int64_t)g->cu_count * 8));
        ProfScope ps(g, KK_BATCH_PULL_HEAVY, st);
        auto k = fs_bits == 16 ? batch_pull_heavy_kernel<G, 16> : fs_bits == 32 ? batch_pull_heavy_kernel<G, 32>
                                                                                 : batch_pull_heavy_kernel<G, 0>;
        hipLaunchKernelGGL(k, dim3(hgrid), dim3(kBlock), 0, st, g->d_in_colidx, V, F, (const void *)c->Fs, Fn, Wr,
                           wact, lc.act, ht.d_vert, ht.d_begin, ht.d_end, ht.n, n, fb, lc.mode_l, lc.flag_prev,
                           lc.flag_l, ps.units());
        ps.end(16.0 * (double)ht.n, 0, 4.0, 0, fs_bits ? fs_bits / 8.0 : 8.0 * wact);
    }
}

static ChunkQueue chunk_queue(BatchCtx *c, int slot) {
    return ChunkQueue{c->cq_rec[slot], c->cq_len + slot, c->cq_mf + slot * kCntLanes};
}

// Hop L's top-down kernel, which also takes the hop's direction (it exits at
// once when the hop goes bottom-up).
template <int G>
static void launch_push(khop_graph *g, BatchCtx *c, int push_div, int64_t L, const LevelCtl &lc, int wact, int Wr,
                        hipStream_t st, uint64_t *V, uint64_t *F, uint64_t *Fn) {
    const int64_t n = g->n;
    const FrontierBits fb = frontier_bits(c, n, L);
    const int a = (int)((L - 1) % 3), b = (int)(L % 3), z = (int)((L + 1) % 3);
    {
        ProfScope ps(g, KK_BATCH_PUSH, st);
        hipLaunchKernelGGL((batch_push_kernel<G>), dim3(g->cu_count * 8), dim3(kBlock), 0, st, g->d_rowptr,
                           g->d_colidx, V, F, Fn, n, g->nnz, Wr, wact, lc.act, push_div, chunk_queue(c, a),
                           chunk_queue(c, b), chunk_queue(c, z), fb, lc.mode_prev, lc.mode_l, lc.flag_prev,
                           lc.flag_l, ps.units());
        // bytes: 4 per out-edge + 8 per active word of its head's visited and next rows
        ps.end(0, 0, 4.0 + 16.0 * wact);
    }
}

__global__ void clear_ring_kernel(int32_t *flags, int32_t *mode, int start, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        const int at = (start + i) % BatchCtx::kRing;
        flags[at] = 0;
        mode[at] = HOP_PUSH;
    }
}

void batch_run(khop_graph *g, BatchCtx *c, const int32_t *d_seeds, const int32_t *h_perm,
               const int32_t *h_ks_sorted, int64_t num_seeds, int64_t *d_counts, hipStream_t st,
               const uint64_t *d_vmask) {
    const Params P = params_of(g);
    // A level whose rows take G lanes per vertex chunks the in-edges of
    // vertices above G/2 times the one-lane threshold: a lane group scans 4 G
    // in-edges per step, and wide rows take their vertices by degree, so
    // their scans are even without chunking
    auto heavy_for = [&](int G) { return batch_heavy_table(g, P.batch_heavy * std::max(1, G / 2)); };
    // Slots come sorted by k, largest first, with the one-hop queries last:
    // those are answered from their seeds' rows and take no bit, so the rows
    // of the bitsets are W words wide for the other nslots slots.
    int nslots = (int)num_seeds;
    while (nslots > 0 && h_ks_sorted[nslots - 1] == 1) --nslots;
    const int W = std::max(1, (nslots + 63) / 64);
    const int Wc = c->W;  // the stride of the active-mask table
    const int64_t n = g->n;
    int64_t kmax = 0;
    for (int j = 0; j < nslots; ++j) kmax = std::max<int64_t>(kmax, h_ks_sorted[j]);
    // no search goes deeper than n - 1 hops: a hop past that finds nothing
    const int64_t levels = std::min<int64_t>(kmax, n);
    // The seeds active at level l are those with k >= l: a prefix of the
    // slots.  One row of the table per distinct k (largest first): row r
    // holds the slots with k >= dk[r], and level l uses the last row whose
    // dk is still >= l.
    std::vector<int64_t> dk;
    std::vector<int> dcnt;
    for (int j = 0; j < nslots; ++j) {
        if (h_ks_sorted[j] < 1) break;  // k = 0 slots (after every k >= 2) are never active
        if (dk.empty() || h_ks_sorted[j] != dk.back()) dk.push_back(h_ks_sorted[j]);
        if (j + 1 == nslots || h_ks_sorted[j + 1] != h_ks_sorted[j]) dcnt.push_back(j + 1);
    }
    const int rows = (int)dk.size();
    // the staging buffer may still feed the previous batch's copies
    KHOP_HIP(hipEventSynchronize(c->stage_ev));
    uint64_t *act = c->h_act;
    std::fill(act, act + (size_t)std::max(rows, 1) * Wc, 0ull);
    for (int r = 0; r < rows; ++r)
        for (int j = 0; j < dcnt[r]; ++j) act[(size_t)r * Wc + (j >> 6)] |= 1ull << (j & 63);
    std::copy(h_perm, h_perm + num_seeds, c->h_perm);
    std::copy(h_ks_sorted, h_ks_sorted + num_seeds, c->h_ks);
    if (rows > 0) KHOP_HIP(hipMemcpyAsync(c->act, act, (size_t)rows * Wc * 8, hipMemcpyHostToDevice, st));
    KHOP_HIP(hipMemcpyAsync(c->perm, c->h_perm, (size_t)num_seeds * 4, hipMemcpyHostToDevice, st));
    KHOP_HIP(hipMemcpyAsync(c->ks, c->h_ks, (size_t)num_seeds * 4, hipMemcpyHostToDevice, st));
    KHOP_HIP(hipEventRecord(c->stage_ev, st));
    if (num_seeds > nslots) {
        const int nq = (int)num_seeds - nslots;
        ProfScope ps(g, KK_BATCH_PUSH, st);
        hipLaunchKernelGGL(batch_row_count_kernel, dim3((nq + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0,
                           st, g->d_rowptr, g->d_colidx, d_seeds, c->perm + nslots, nq, d_vmask, d_counts,
                           ps.units());
        // bytes: the seed's row pointers, 4 per out-edge
        ps.end(16.0 * nq, 4.0);
        KHOP_HIP(hipGetLastError());
    }
    if (nslots == 0) return;
    const int zgrid = (int)std::min<int64_t>(((int64_t)n * W + kBlock - 1) / kBlock, (int64_t)g->cu_count * 8);
    {
        ProfScope ps(g, KK_BATCH_INIT, st);
        hipLaunchKernelGGL(batch_zero_kernel, dim3(std::max(zgrid, 1)), dim3(kBlock), 0, st, c->V, c->F, c->N,
                           (int64_t)n * W, c->Fb, 3 * ((n + 63) / 64), c->Fc, c->acc, (int64_t)64 * W, c->flags,
                           c->mode, BatchCtx::kRing, c->cq_len, c->cq_mf);
        ps.end(3.0 * 8.0 * n * W + 3.0 * 8.0 * ((n + 63) / 64));
    }
    if (d_vmask)
        hipLaunchKernelGGL(batch_mask_kernel, dim3(std::max(zgrid, 1)), dim3(kBlock), 0, st, c->V, n, W, d_vmask);
    hipLaunchKernelGGL(batch_seed_kernel, dim3((nslots + kBlock - 1) / kBlock), dim3(kBlock), 0, st, c->V, d_seeds,
                       c->perm, nslots, W);
    uint64_t *F = c->F, *Nb = c->N;
    if (levels >= 1) {
        ProfScope ps(g, KK_BATCH_PUSH, st);
        hipLaunchKernelGGL(batch_push_seeds_kernel, dim3(std::min(nslots * kSeedParts, 4096)), dim3(kBlock), 0, st,
                           g->d_rowptr, g->d_colidx, d_seeds, c->perm, c->ks, nslots, W, F, c->V,
                           c->Fb + (int64_t)((n + 63) / 64), c->Fc + kCntLanes, chunk_queue(c, 1),
                           c->flags + ring_slot(1), d_vmask);
        ps.end(0);
    }
    // Rows are Wr words long.  Seeds are sorted by k, so the active words of a
    // level are a prefix; once they fit in half a row, the words behind them
    // (finished seeds) are counted and the rows are repacked to the active
    // width, which every later level then reads and writes.
    uint64_t *V = c->V;
    int Wr = W;
    auto count_words = [&](int w0, int nwords) {
        ProfScope ps(g, KK_BATCH_COUNT, st);
        const int cgx = (int)std::max<int64_t>(1, std::min<int64_t>((n + 64 * kWavesPerBlock - 1) / (64 * kWavesPerBlock),
                                                                     (int64_t)g->cu_count * 8));
        for (int w = w0; w < w0 + nwords; w += kCountMaxWords)
            hipLaunchKernelGGL(batch_count_kernel, dim3(cgx), dim3(kBlock), 0, st, V, n, Wr, w,
                               std::min(kCountMaxWords, w0 + nwords - w), d_vmask, c->acc);
        ps.end(8.0 * n * nwords);
    };
    int r = rows - 1;  // the table row of the current level
    constexpr int kHalf = BatchCtx::kRing / 2;
    for (int64_t L = 2; L <= levels; ++L) {
        while (r >= 0 && dk[r] < L) --r;
        if (r < 0) break;
        const int wa = (dcnt[r] + 63) / 64;
        if (L % kHalf == 0) {
            // ring slots of levels L + 1 .. L + kHalf last served levels a whole ring earlier
            hipLaunchKernelGGL(clear_ring_kernel, dim3(1), dim3(256), 0, st, c->flags, c->mode, ring_slot(L + 1),
                               kHalf);
        }
        if (2 * wa <= Wr) {
            count_words(wa, Wr - wa);
            // V and F move into the spare buffer (both fit: 2 * wa <= Wr); the old V becomes the next frontier's buffer
            uint64_t *Vn = Nb, *Fnew = Nb + (int64_t)n * wa;
            {
                ProfScope ps(g, KK_BATCH_INIT, st);
                const int ng = (int)std::min<int64_t>(((int64_t)n * wa + kBlock - 1) / kBlock, (int64_t)g->cu_count * 8);
                hipLaunchKernelGGL(batch_narrow_kernel, dim3(std::max(ng, 1)), dim3(kBlock), 0, st, V, F, n, Wr, wa,
                                   Vn, Fnew);
                ps.end(2.0 * 8.0 * n * wa * 2);
            }
            // the next frontier's buffer starts clear (a top-down hop only ORs into it)
            hipLaunchKernelGGL(fill_zero_u64, dim3(std::max((int)std::min<int64_t>(((int64_t)n * wa + kBlock - 1) / kBlock,
                                                                              (int64_t)g->cu_count * 8), 1)),
                               dim3(kBlock), 0, st, V, (int64_t)n * wa);
            Nb = V;
            V = Vn;
            F = Fnew;
            Wr = wa;
        }
        const LevelCtl lc = level_ctl(c, L, c->act + (size_t)r * Wc);
        int G = 1;
        while (G < wa) G <<= 1;
        switch (G) {
            case 1: {
                launch_push<1>(g, c, P.batch_push_div, L, lc, wa, Wr, st, V, F, Nb);
                // one-word rows whose active seeds fit in 16 or 32 bits are gathered from a narrow copy
                int fs_bits = 0;
                if (Wr == 1) {
                    const int top = dcnt[r] - 1;
                    fs_bits = top < 16 ? 16 : top < 32 ? 32 : 0;
                }
                if (fs_bits) {
                    ProfScope ps(g, KK_BATCH_INIT, st);
                    const int cg = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock,
                                                                               (int64_t)g->cu_count * 8));
                    hipLaunchKernelGGL(batch_frontier_copy_kernel, dim3(cg), dim3(kBlock), 0, st, F, n, c->Fs, fs_bits,
                                       lc.mode_l, lc.flag_prev);
                    ps.end(8.0 * n + n * fs_bits / 8.0);
                }
                launch_pull<1>(g, c, heavy_for(1), P.batch_grid, L, lc, wa, Wr, st, V, F, Nb, fs_bits);
                break;
            }
            case 2:
                launch_push<2>(g, c, P.batch_push_div, L, lc, wa, Wr, st, V, F, Nb);
                launch_pull<2>(g, c, heavy_for(2), P.batch_grid, L, lc, wa, Wr, st, V, F, Nb, 0);
                break;
            case 4:
                launch_push<4>(g, c, P.batch_push_div, L, lc, wa, Wr, st, V, F, Nb);
                launch_pull<4>(g, c, heavy_for(4), P.batch_grid, L, lc, wa, Wr, st, V, F, Nb, 0);
                break;
            case 8:
                launch_push<8>(g, c, P.batch_push_div, L, lc, wa, Wr, st, V, F, Nb);
                launch_pull<8>(g, c, heavy_for(8), P.batch_grid, L, lc, wa, Wr, st, V, F, Nb, 0);
                break;
            default:
                launch_push<16>(g, c, P.batch_push_div, L, lc, wa, Wr, st, V, F, Nb);
                launch_pull<16>(g, c, heavy_for(16), P.batch_grid, L, lc, wa, Wr, st, V, F, Nb, 0);
                break;
        }
        std::swap(F, Nb);
        if ((L % 8) == 0 && L < levels) {
            // long traversals: stop once the frontier is empty
            int32_t flag = 1;
            KHOP_HIP(hipMemcpyAsync(&flag, c->flags + ring_slot(L), 4, hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipStreamSynchronize(st));
            if (!flag) break;
        }
    }
    count_words(0, Wr);
    hipLaunchKernelGGL(batch_output_kernel, dim3((nslots + 255) / 256), dim3(256), 0, st, c->acc, c->perm, nslots,
                       d_seeds, d_vmask, d_counts);
    KHOP_HIP(hipGetLastError());
}

}  // namespace khop
