// Plain single-query k-hop count on gfx950.
//
// One hop is the masked boolean product of the paper's Section II: the next
// frontier is (A^T f) AND NOT visited over the (OR, AND) semiring.  Each hop
// runs as three launches, with every cross-block hand-off at a kernel boundary
// (no intra-kernel fences, which on a multi-XCD part would write back L2):
//   expand  top-down (push): edge-balanced sweep over the frontier queue that
//           marks unvisited heads in a byte map (same-value races, no
//           atomics); or bottom-up (pull): each unvisited vertex scans its
//           in-neighbors against the frontier bitmap and stops at the first
//           hit; one wave per 64-vertex word writes the next-frontier word
//           straight from a ballot (single writer).  Vertices above the heavy
//           threshold are split into edge chunks that many waves scan.
//   count   per block of words: after a push, ballot(mark AND NOT visited)
//           gives each next-frontier word and visited |= word; then the
//           block's level popcount, queue length and frontier degree sums go
//           to a per-block slot and, by one atomic per field, to the block's
//           superblock total.
//   finish  every block adds up the superblock totals (identical in every
//           block, so the direction choice needs no broadcast) and its own
//           prefix; block 0 advances the level state; when the next hop is a
//           push each block writes its part of the ascending frontier queue
//           and the exclusive prefix of the queue's out-degrees (LDS prefix
//           sums, no atomics).
// The level state is double buffered by level parity so that blocks of a
// finish launch never read what block 0 of the same launch writes.  No hop
// needs a host round trip; the host only enqueues.
#include <algorithm>
#include <cmath>

#include "khop_impl.h"
#include "wave.h"

namespace khop {

using namespace dev;

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPart = 4;  // per-block partials: cnt, qcnt, mf, din
enum { DIR_PUSH = KHOP_DIR_PUSH, DIR_PULL = KHOP_DIR_PULL };

struct LevelState {
    int64_t count;  // vertices at distance 1..level
    int64_t te;     // out-degree sum of levels 0..min(level, k-1)
    int64_t nf;     // frontier size (vertices at distance == level)
    int64_t qlen;   // frontier vertices with out-degree > 0 (queue length)
    int64_t mf;     // out-degree sum of the frontier
    int64_t mu;     // in-degree sum of unvisited vertices
    int32_t dir;    // direction of the next expansion
    int32_t done;   // the count is final and written out
};

struct PlainCtl {
    LevelState st[2];  // state after level l lives in st[l & 1]
    int64_t *out_count;
    int64_t *out_te;
    int32_t k, dir_mode, alpha, beta;
};

struct Graph {
    const int64_t *__restrict__ rowptr;
    const int32_t *__restrict__ colidx;
    const int64_t *__restrict__ in_rowptr;
    const int32_t *__restrict__ in_colidx;
    int64_t n;
    int64_t nw;  // 64-vertex words
    int directed;
    int heavy;   // bottom-up: in-degree above which the chunk kernel takes a vertex
};

struct State {
    uint64_t *V;     // visited bitmap
    uint64_t *F0;    // frontier bitmaps, double buffered by level parity
    uint64_t *F1;
    uint8_t *nextb;  // top-down mark bytes, all zero between hops
    int32_t *q;      // frontier queue
    int64_t *qoff;   // exclusive prefix of queue out-degrees, qoff[qlen] = mf
    int64_t *part;   // per-block partials (nblk * kPart)
    int64_t *sup;    // superblock totals, 2 * nsup * kPart (level parity)
    int wpb;         // words per block of the count / finish kernels
    int nblk;        // blocks of the count / finish kernels
    int sb;          // blocks per superblock
    int nsup;        // superblocks
};

struct HeavyChunks {
    const int32_t *vert;   // vertex of each chunk
    const int64_t *begin;  // first in-edge of each chunk
    const int64_t *end;    // one past its last in-edge
    int64_t n;
};

__device__ __forceinline__ uint64_t *frontier(const State &s, int completed_levels) {
    return (completed_levels & 1) ? s.F1 : s.F0;
}

__device__ int64_t block_sum(int64_t v) {
    __shared__ int64_t s_v[kWavesPerBlock];
    v = wave_sum(v);
    if (lane_id() == 0) s_v[threadIdx.x / kWave] = v;
    __syncthreads();
    int64_t t = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) t += s_v[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ void unit_add(int64_t *units, int i, int64_t v) {
    if (units && v) atomicAdd((unsigned long long *)&units[i], (unsigned long long)v);
}

// ------------------------------------------------------------------ init

__global__ void __launch_bounds__(kBlock) plain_init_kernel(PlainCtl *ctl, Graph g, State s, const int32_t *seeds,
                                                           int64_t qi, int k, int dir_mode, int alpha, int beta,
                                                           int64_t nnz_in, int64_t *out_count, int64_t *out_te,
                                                           int64_t *units) {
    const int32_t seed = seeds[qi];
    const bool valid = seed >= 0 && (int64_t)seed < g.n;
    const int64_t sw = valid ? (seed >> 6) : -1;
    const uint64_t sbit = valid ? (1ull << (seed & 63)) : 0;
    for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < g.nw; w += (int64_t)gridDim.x * kBlock) {
        const uint64_t x = (w == sw) ? sbit : 0ull;
        s.V[w] = x;
        s.F0[w] = x;
    }
    if (blockIdx.x == 0) {
        // superblock totals of level 1 start at zero
        int64_t *sup1 = s.sup + (int64_t)s.nsup * kPart;
        for (int i = threadIdx.x; i < s.nsup * kPart; i += kBlock) sup1[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->out_count = out_count + qi;
        ctl->out_te = out_te ? out_te + qi : nullptr;
        ctl->dir_mode = dir_mode;
        ctl->alpha = alpha;
        ctl->beta = beta;
        ctl->k = k;
        LevelState &st = ctl->st[0];
        st.count = 0;
        // the other parity slot is read at hop 2; it must not keep the previous query's state
        ctl->st[1].done = (!valid || k == 0) ? 1 : 0;
        if (!valid) {
            st.done = 1;
            out_count[qi] = -1;
            if (out_te) out_te[qi] = -1;
            return;
        }
        const int64_t od = g.rowptr[seed + 1] - g.rowptr[seed];
        const int64_t id = g.in_rowptr[seed + 1] - g.in_rowptr[seed];
        s.qoff[0] = 0;
        if (od > 0) {
            s.q[0] = seed;
            s.qoff[1] = od;
        }
        st.qlen = od > 0 ? 1 : 0;
        st.nf = 1;
        st.mf = od;
        st.mu = nnz_in - id;
        st.te = k >= 1 ? od : 0;
        st.dir = dir_mode == DIR_PULL ? DIR_PULL : DIR_PUSH;
        st.done = (k == 0) ? 1 : 0;
        if (k == 0) {
            out_count[qi] = 0;
            if (out_te) out_te[qi] = 0;
        }
        if (units) units[0] = 2 * 8 * g.nw;
    }
}

// ------------------------------------------------------------------ top-down

// Edge-balanced sweep: wave w owns edges [E*w/W, E*(w+1)/W) of the frontier's
// concatenated adjacency lists.  Within a 64-edge window the owning queue
// entry of each lane is base - 1 + (number of list starts at or before it).
__device__ void push_expand(const LevelState &st, const Graph &g, const State &s, int64_t *units) {
    const int lane = lane_id();
    const int64_t qlen = st.qlen;
    const int64_t E = st.mf;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t e0 = E * wid / nwaves, e1 = E * (wid + 1) / nwaves;
    if (units && wid == 0 && lane == 0) unit_add(units, 0, 4 * E + 20 * qlen);
    if (e0 >= e1) return;
    __shared__ uint64_t s_mask[kWavesPerBlock];
    uint64_t *smask = &s_mask[threadIdx.x / kWave];
    const int32_t *__restrict__ q = s.q;
    const int64_t *__restrict__ qoff = s.qoff;

    // base = #{ j < qlen : qoff[j] < e0 } by a 64-way search
    int64_t lo = 0, hi = qlen;
    while (hi - lo > kWave) {
        const int64_t step = (hi - lo + kWave - 1) / kWave;
        const int64_t p = lo + (int64_t)lane * step;
        const bool less = p < hi && qoff[p] < e0;
        const int t = __popcll(ballot(less));
        const int64_t nlo = t ? lo + (int64_t)(t - 1) * step + 1 : lo;
        hi = std::min(hi, lo + (int64_t)t * step);
        lo = nlo;
    }
    {
        const int64_t p = lo + lane;
        const bool less = p < hi && qoff[p] < e0;
        lo += __popcll(ballot(less));
    }
    int64_t base = lo;
    int64_t carry_beg = 0, carry_off = 0;
    if (base > 0) {
        carry_beg = g.rowptr[q[base - 1]];
        carry_off = qoff[base - 1];
    }
    const uint64_t *__restrict__ V = s.V;
    uint8_t *__restrict__ nextb = s.nextb;
    for (int64_t b = e0; b < e1; b += kWave) {
        const int64_t j = base + lane;
        bool inwin = false;
        int64_t offj = 0, begj = 0;
        if (j < qlen) {
            offj = qoff[j];
            inwin = offj < b + kWave;
        }
        if (inwin) begj = g.rowptr[q[j]];
        if (lane == 0) *smask = 0;
        __builtin_amdgcn_wave_barrier();
        if (inwin) atomicOr((unsigned long long *)smask, 1ull << (offj - b));
        __builtin_amdgcn_wave_barrier();
        const uint64_t starts = *smask;
        const int ns = __popcll(ballot(inwin));
        const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1);
        const int c = __popcll(starts & le);
        const int src = c > 0 ? c - 1 : 0;
        const int64_t sb = shfl64(begj, src), so = shfl64(offj, src);
        const int64_t e = b + lane;
        if (e < e1) {
            const int64_t beg = c ? sb : carry_beg;
            const int64_t off = c ? so : carry_off;
            const int32_t v = g.colidx[beg + (e - off)];
            if (!test_bit(V, v)) nextb[v] = 1;
        }
        if (ns > 0) {
            carry_beg = shfl64(begj, ns - 1);
            carry_off = shfl64(offj, ns - 1);
        }
        base += ns;
        __builtin_amdgcn_wave_barrier();
    }
}

// ------------------------------------------------------------------ bottom-up

// Each wave takes 64-vertex words in turn.  Unvisited vertices of in-degree up
// to `light` scan alone (4 in-edges per round); heavier ones up to g.heavy are
// scanned by the whole wave, 256 in-edges per round; heavier still are left
// for the chunk kernel.
__device__ void pull_expand(int L, const Graph &g, const State &s, int light, int64_t *units) {
    const int lane = lane_id();
    const uint64_t *__restrict__ Fc = frontier(s, L - 1);
    uint64_t *__restrict__ Fn = frontier(s, L);
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    int64_t c_pe = 0, c_pv = 0;
    for (int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; w < g.nw; w += nwaves) {
        const uint64_t vis = s.V[w];
        const int64_t v = w * kWave + lane;
        const bool unv = v < g.n && !((vis >> lane) & 1ull);
        uint64_t found_mask = 0;
        if (ballot(unv)) {
            int64_t b = 0, e = 0;
            if (unv) {
                b = g.in_rowptr[v];
                e = g.in_rowptr[v + 1];
            }
            const int64_t d = e - b;
            bool found = false;
            int64_t examined = 0;
            if (unv && d <= light) {
                int64_t x = b;
                for (; x + 4 <= e; x += 4) {
                    const int32_t u0 = g.in_colidx[x], u1 = g.in_colidx[x + 1];
                    const int32_t u2 = g.in_colidx[x + 2], u3 = g.in_colidx[x + 3];
                    const bool h0 = test_bit(Fc, u0), h1 = test_bit(Fc, u1);
                    const bool h2 = test_bit(Fc, u2), h3 = test_bit(Fc, u3);
                    if (h0 | h1 | h2 | h3) {
                        examined += h0 ? 1 : h1 ? 2 : h2 ? 3 : 4;
                        found = true;
                        break;
                    }
                    examined += 4;
                }
                if (!found) {
                    for (; x < e; ++x) {
                        ++examined;
                        if (test_bit(Fc, g.in_colidx[x])) {
                            found = true;
                            break;
                        }
                    }
                }
            }
            uint64_t medium = ballot(unv && d > light && d <= g.heavy);
            while (medium) {
                const int h = __builtin_ctzll(medium);
                medium &= medium - 1;
                const int64_t hb = shfl64(b, h), he = shfl64(e, h);
                bool hit = false;
                int64_t scanned = 0;
                for (int64_t x0 = hb; x0 < he; x0 += 4 * kWave) {
                    bool any = false;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t x = x0 + r * kWave + lane;
                        if (x < he) any |= test_bit(Fc, g.in_colidx[x]);
                    }
                    scanned += std::min<int64_t>(4 * kWave, he - x0);
                    if (ballot(any)) {
                        hit = true;
                        break;
                    }
                }
                if (lane == h) {
                    found = hit;
                    examined = scanned;
                }
            }
            found_mask = ballot(found);
            if (units) {
                c_pe += wave_sum(examined);
                c_pv += __popcll(ballot(unv && d <= g.heavy));
            }
        }
        if (lane == 0) {
            Fn[w] = found_mask;
            if (found_mask) s.V[w] = vis | found_mask;
        }
    }
    if (units && lane == 0) {
        // 4 B per examined in-edge, 16 B of row pointers per scanned vertex
        unit_add(units, 0, 4 * c_pe + 16 * c_pv);
        if (blockIdx.x == 0 && threadIdx.x == 0) unit_add(units, 0, 2 * ((g.n + 7) / 8));
    }
}

__global__ void __launch_bounds__(kBlock) plain_expand_kernel(const PlainCtl *ctl, int L, Graph g, State s, int light,
                                                             int64_t *units) {
    const LevelState &st = ctl->st[(L - 1) & 1];
    if (st.done) return;
    if (st.dir == DIR_PUSH) {
        push_expand(st, g, s, units);
    } else {
        pull_expand(L, g, s, light, units);
    }
}

// Bottom-up chunks of heavy vertices: a wave scans one chunk of in-edges of a
// still-unvisited vertex; a hit sets its frontier and visited bits atomically.
__global__ void __launch_bounds__(kBlock) plain_pull_heavy_kernel(const PlainCtl *ctl, int L, Graph g, State s,
                                                                 HeavyChunks hc, int64_t *units) {
    const LevelState &st = ctl->st[(L - 1) & 1];
    if (st.done || st.dir != DIR_PULL) return;
    const int lane = lane_id();
    const uint64_t *__restrict__ Fc = frontier(s, L - 1);
    uint64_t *Fn = frontier(s, L);
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    int64_t examined = 0;
    for (int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; i < hc.n; i += nwaves) {
        const int32_t v = hc.vert[i];
        const uint64_t bit = 1ull << (v & 63);
        // visited before this hop, or already found by another chunk
        if (__hip_atomic_load(&s.V[v >> 6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit) continue;
        const int64_t b = hc.begin[i], e = hc.end[i];
        bool hit = false;
        for (int64_t x0 = b; x0 < e; x0 += 4 * kWave) {
            bool any = false;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t x = x0 + r * kWave + lane;
                if (x < e) any |= test_bit(Fc, g.in_colidx[x]);
            }
            examined += std::min<int64_t>(4 * kWave, e - x0);
            if (ballot(any)) {
                hit = true;
                break;
            }
        }
        if (hit && lane == 0) {
            atomicOr((unsigned long long *)&Fn[v >> 6], (unsigned long long)bit);
            atomicOr((unsigned long long *)&s.V[v >> 6], (unsigned long long)bit);
        }
    }
    if (units && lane == 0) unit_add(units, 0, 4 * examined);
}

// ------------------------------------------------------------------ count

__global__ void __launch_bounds__(kBlock) plain_count_kernel(const PlainCtl *ctl, int L, Graph g, State s,
                                                            int64_t *units) {
    const LevelState &st = ctl->st[(L - 1) & 1];
    if (st.done) return;
    const bool pushed = st.dir == DIR_PUSH;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    uint64_t *__restrict__ Fn = frontier(s, L);
    const int64_t w0 = (int64_t)blockIdx.x * s.wpb;
    const int64_t w1 = std::min<int64_t>(w0 + s.wpb, g.nw);
    int64_t c_cnt = 0, c_q = 0, c_mf = 0, c_din = 0;
    for (int64_t w = w0 + wv; w < w1; w += kWavesPerBlock) {
        const int64_t v = w * kWave + lane;
        uint64_t m;
        if (pushed) {
            const uint8_t nb = v < g.n ? s.nextb[v] : 0;
            const uint64_t vis = s.V[w];
            m = ballot(nb && !((vis >> lane) & 1ull));
            if (nb) s.nextb[v] = 0;
            if (lane == 0) {
                Fn[w] = m;
                if (m) s.V[w] = vis | m;
            }
        } else {
            m = Fn[w];
        }
        if (m) {
            const bool fresh = (m >> lane) & 1ull;
            int64_t od = 0, din = 0;
            if (fresh) {
                od = g.rowptr[v + 1] - g.rowptr[v];
                din = g.directed ? g.in_rowptr[v + 1] - g.in_rowptr[v] : od;
            }
            c_cnt += __popcll(m);
            c_q += __popcll(ballot(fresh && od > 0));
            c_mf += wave_sum(od);
            c_din += wave_sum(din);
        }
    }
    const bool l0 = lane == 0;
    const int64_t t_cnt = block_sum(l0 ? c_cnt : 0), t_q = block_sum(l0 ? c_q : 0);
    const int64_t t_mf = block_sum(l0 ? c_mf : 0), t_din = block_sum(l0 ? c_din : 0);
    if (threadIdx.x < kPart) {
        const int64_t val = threadIdx.x == 0 ? t_cnt : threadIdx.x == 1 ? t_q : threadIdx.x == 2 ? t_mf : t_din;
        s.part[(int64_t)blockIdx.x * kPart + threadIdx.x] = val;
        int64_t *sup = s.sup + ((int64_t)(L & 1) * s.nsup + blockIdx.x / s.sb) * kPart;
        if (val) atomicAdd((unsigned long long *)&sup[threadIdx.x], (unsigned long long)val);
    }
    if (units && threadIdx.x == 0) {
        if (blockIdx.x == 0) unit_add(units, 0, pushed ? g.n + 2 * ((g.n + 7) / 8) : (g.n + 7) / 8);
        unit_add(units, 0, 16 * t_cnt);
    }
}

// ------------------------------------------------------------------ finish

__global__ void __launch_bounds__(kBlock) plain_finish_kernel(PlainCtl *ctl, int L, Graph g, State s,
                                                             int64_t *units) {
    const LevelState &st = ctl->st[(L - 1) & 1];
    if (st.done) return;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    const int64_t *sup = s.sup + (int64_t)(L & 1) * s.nsup * kPart;
    // level totals and this block's exclusive queue / degree offsets
    const int my_sup = blockIdx.x / s.sb;
    int64_t t_cnt = 0, t_q = 0, t_mf = 0, t_din = 0, o_q = 0, o_mf = 0;
    for (int i = threadIdx.x; i < s.nsup; i += kBlock) {
        const int64_t *p = sup + (int64_t)i * kPart;
        t_cnt += p[0];
        t_q += p[1];
        t_mf += p[2];
        t_din += p[3];
        if (i < my_sup) {
            o_q += p[1];
            o_mf += p[2];
        }
    }
    for (int b = my_sup * s.sb + threadIdx.x; b < blockIdx.x; b += kBlock) {
        o_q += s.part[(int64_t)b * kPart + 1];
        o_mf += s.part[(int64_t)b * kPart + 2];
    }
    t_cnt = block_sum(t_cnt);
    t_q = block_sum(t_q);
    t_mf = block_sum(t_mf);
    t_din = block_sum(t_din);
    o_q = block_sum(o_q);
    o_mf = block_sum(o_mf);
    // next state (every block computes the same)
    const int64_t mu = st.mu - t_din;
    const int done = (t_cnt == 0) || (L >= ctl->k);
    int dir = st.dir;
    if (ctl->dir_mode == DIR_PUSH) {
        dir = DIR_PUSH;
    } else if (ctl->dir_mode == DIR_PULL) {
        dir = DIR_PULL;
    } else if (dir == DIR_PUSH) {
        if (t_mf * (int64_t)ctl->alpha > mu) dir = DIR_PULL;
    } else {
        if (t_cnt * (int64_t)ctl->beta < g.n) dir = DIR_PUSH;
    }
    if (blockIdx.x == 0) {
        int64_t *nsup = s.sup + (int64_t)((L + 1) & 1) * s.nsup * kPart;
        if (!done)
            for (int i = threadIdx.x; i < s.nsup * kPart; i += kBlock) nsup[i] = 0;
        if (threadIdx.x == 0) {
            LevelState &nx = ctl->st[L & 1];
            nx.count = st.count + t_cnt;
            nx.te = st.te + (L < ctl->k ? t_mf : 0);
            nx.nf = t_cnt;
            nx.qlen = t_q;
            nx.mf = t_mf;
            nx.mu = mu;
            nx.dir = dir;
            nx.done = done;
            if (done) {
                // later hops read either parity slot; both must say done
                ctl->st[(L + 1) & 1].done = 1;
                *ctl->out_count = nx.count;
                if (ctl->out_te) *ctl->out_te = nx.te;
            } else if (dir == DIR_PUSH) {
                s.qoff[t_q] = t_mf;
            }
            if (units && !done && dir == DIR_PUSH) unit_add(units, 0, (g.n + 7) / 8 + 28 * t_q);
        }
    }
    if (done || dir != DIR_PUSH) return;
    // ascending queue: each wave takes a contiguous quarter of the block's words
    const uint64_t *__restrict__ Fn = frontier(s, L);
    const int64_t w0 = (int64_t)blockIdx.x * s.wpb;
    const int per = (s.wpb + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t a0 = std::min<int64_t>(w0 + (int64_t)wv * per, g.nw);
    const int64_t a1 = std::min<int64_t>(std::min<int64_t>(a0 + per, w0 + s.wpb), g.nw);
    __shared__ int64_t s_q[kWavesPerBlock], s_d[kWavesPerBlock];
    int64_t tq = 0, td = 0;
    for (int64_t w = a0; w < a1; ++w) {
        const uint64_t m = Fn[w];
        if (!m) continue;
        const int64_t v = w * kWave + lane;
        int64_t od = 0;
        if ((m >> lane) & 1ull) od = g.rowptr[v + 1] - g.rowptr[v];
        tq += __popcll(ballot(od > 0));
        td += wave_sum(od);
    }
    if (lane == 0) {
        s_q[wv] = tq;
        s_d[wv] = td;
    }
    __syncthreads();
    int64_t qpos = o_q, dpos = o_mf;
    for (int i = 0; i < wv; ++i) {
        qpos += s_q[i];
        dpos += s_d[i];
    }
    for (int64_t w = a0; w < a1; ++w) {
        const uint64_t m = Fn[w];
        if (!m) continue;
        const int64_t v = w * kWave + lane;
        int64_t od = 0;
        if ((m >> lane) & 1ull) od = g.rowptr[v + 1] - g.rowptr[v];
        const uint64_t qm = ballot(od > 0);
        const int64_t dx = wave_exclusive_sum(od);
        if (od > 0) {
            const int64_t at = qpos + mask_rank(qm);
            s.q[at] = (int32_t)v;
            s.qoff[at] = dpos + dx;
        }
        qpos += __popcll(qm);
        dpos += wave_sum(od);
    }
}

__global__ void fill_kernel(int64_t *a, int64_t *b, int64_t n, int64_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a[i] = value;
        if (b) b[i] = value;
    }
}

}  // namespace

struct PlainCtx {
    khop_graph *g = nullptr;
    PlainCtl *ctl = nullptr;
    State s{};
    int expand_grid = 1;
    void *arena = nullptr;
};

PlainCtx *plain_ctx_create(khop_graph *g) {
    PlainCtx *c = new PlainCtx();
    c->g = g;
    const int64_t n = g->n, nw = (n + 63) / 64;
    // word ranges for count / finish: at most about 4096 blocks
    int wpb = (int)std::max<int64_t>(16, (nw + 4095) / 4096);
    wpb = (wpb + 3) & ~3;
    const int nblk = (int)((nw + wpb - 1) / wpb);
    const int sb = std::max(8, (int)std::ceil(std::sqrt((double)nblk)));
    const int nsup = (nblk + sb - 1) / sb;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_ctl = off;
    off += al(sizeof(PlainCtl));
    const size_t o_V = off;
    off += al(nw * 8);
    const size_t o_F0 = off;
    off += al(nw * 8);
    const size_t o_F1 = off;
    off += al(nw * 8);
    const size_t o_nb = off;
    off += al(n);
    const size_t o_q = off;
    off += al(n * 4);
    const size_t o_qoff = off;
    off += al((n + 1) * 8);
    const size_t o_part = off;
    off += al((size_t)nblk * kPart * 8);
    const size_t o_sup = off;
    off += al((size_t)2 * nsup * kPart * 8);
    hipError_t e = hipMalloc(&c->arena, off);
    if (e != hipSuccess) {
        delete c;
        (void)hipGetLastError();
        fail(KHOP_ENOMEM, "device allocation of " + std::to_string(off) + " bytes for a query context failed");
    }
    char *base = (char *)c->arena;
    c->ctl = (PlainCtl *)(base + o_ctl);
    c->s.V = (uint64_t *)(base + o_V);
    c->s.F0 = (uint64_t *)(base + o_F0);
    c->s.F1 = (uint64_t *)(base + o_F1);
    c->s.nextb = (uint8_t *)(base + o_nb);
    c->s.q = (int32_t *)(base + o_q);
    c->s.qoff = (int64_t *)(base + o_qoff);
    c->s.part = (int64_t *)(base + o_part);
    c->s.sup = (int64_t *)(base + o_sup);
    c->s.wpb = wpb;
    c->s.nblk = nblk;
    c->s.sb = sb;
    c->s.nsup = nsup;
    c->expand_grid = (int)std::max<int64_t>(1, std::min<int64_t>((nw + 15) / 16, (int64_t)g->cu_count * 8));
    KHOP_HIP(hipMemset(c->arena, 0, off));
    KHOP_HIP(hipDeviceSynchronize());
    return c;
}

void plain_ctx_destroy(PlainCtx *c) {
    if (!c) return;
    if (c->arena) (void)hipFree(c->arena);
    delete c;
}

void plain_fill_zero_outputs(int64_t *d_counts, int64_t *d_te, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, st, d_counts, d_te, n, (int64_t)0);
    KHOP_HIP(hipGetLastError());
}

void plain_run(khop_graph *g, PlainCtx *c, const int32_t *d_seeds, int64_t num_seeds, int32_t k, int64_t *d_counts,
               int64_t *d_te, hipStream_t st) {
    if (num_seeds <= 0) return;
    if (k == 0) {
        plain_fill_zero_outputs(d_counts, d_te, num_seeds, st);
        return;
    }
    const Params &P = g->params;
    const HeavyTable &ht = plain_heavy_table(g);
    Graph gr{g->d_rowptr, g->d_colidx, g->d_in_rowptr, g->d_in_colidx, g->n, (g->n + 63) / 64, g->directed,
             ht.threshold};
    HeavyChunks hc{ht.d_vert, ht.d_begin, ht.d_end, ht.n};
    const int nblk = c->s.nblk;
    const int init_grid = (int)std::max<int64_t>(1, std::min<int64_t>((gr.nw + kBlock - 1) / kBlock, 256));
    const int heavy_grid =
        (int)std::max<int64_t>(1, std::min<int64_t>((ht.n + kWavesPerBlock - 1) / kWavesPerBlock, g->cu_count * 8));
    const int64_t nnz_in = g->nnz;
    for (int64_t i = 0; i < num_seeds; ++i) {
        {
            ProfScope ps(g, KK_PLAIN_INIT, st);
            hipLaunchKernelGGL(plain_init_kernel, dim3(init_grid), dim3(kBlock), 0, st, c->ctl, gr, c->s, d_seeds, i,
                               (int)k, P.dir_mode, P.alpha, P.beta, nnz_in, d_counts, d_te, ps.units());
            ps.end(0, 1);
        }
        for (int L = 1; L <= k; ++L) {
            {
                ProfScope ps(g, KK_PLAIN_EXPAND, st);
                hipLaunchKernelGGL(plain_expand_kernel, dim3(c->expand_grid), dim3(kBlock), 0, st, c->ctl, L, gr,
                                   c->s, P.pull_light, ps.units());
                ps.end(0, 1);
            }
            if (ht.n > 0 && P.dir_mode != KHOP_DIR_PUSH) {
                ProfScope ps(g, KK_PLAIN_PULL_HEAVY, st);
                hipLaunchKernelGGL(plain_pull_heavy_kernel, dim3(heavy_grid), dim3(kBlock), 0, st, c->ctl, L, gr,
                                   c->s, hc, ps.units());
                ps.end(0, 1);
            }
            {
                ProfScope ps(g, KK_PLAIN_COMPACT, st);
                hipLaunchKernelGGL(plain_count_kernel, dim3(nblk), dim3(kBlock), 0, st, c->ctl, L, gr, c->s,
                                   ps.units());
                ps.end(0, 1);
            }
            {
                ProfScope ps(g, KK_PLAIN_QUEUE, st);
                hipLaunchKernelGGL(plain_finish_kernel, dim3(nblk), dim3(kBlock), 0, st, c->ctl, L, gr, c->s,
                                   ps.units());
                ps.end(0, 1);
            }
        }
    }
    KHOP_HIP(hipGetLastError());
}

}  // namespace khop
