// Plain single-query k-hop count on gfx950.
//
// One hop is the masked boolean product of the paper's Section II: the next
// frontier is (A^T f) AND NOT visited over the (OR, AND) semiring.  Each hop
// runs as
//   expand   top-down (push): edge-balanced sweep over the frontier queue,
//            marking unvisited heads in a byte map (benign same-value races,
//            no atomics); or bottom-up (pull): every unvisited vertex scans
//            its in-neighbors against the frontier bitmap and stops at the
//            first hit, one wave per 64-vertex word writing the next-frontier
//            word straight from a ballot (single writer, no atomics);
//   compact  after a push: ballot(next byte AND NOT visited) per 64-vertex
//            word -> next-frontier word, visited |= word, level popcount;
//   queue    when the next hop is a push: the ascending frontier queue and
//            the exclusive prefix of its out-degrees, from per-block counts
//            and LDS prefix sums (two passes, no atomics).
// The last block to finish an expand/compact launch (one ticket atomic per
// block) reduces the per-block partials, adds the level popcount to the count,
// and picks the next direction (Beamer-style thresholds on frontier and
// unvisited edge counts), so no hop needs a host round trip.
#include <algorithm>

#include "khop_impl.h"
#include "wave.h"

namespace khop {

using namespace dev;

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPart = 6;  // per-block partials: cnt, qcnt, mf, din, pull edges, pull vertices
enum { DIR_PUSH = KHOP_DIR_PUSH, DIR_PULL = KHOP_DIR_PULL };

struct PlainCtl {
    int64_t count;  // vertices at distance 1..level
    int64_t te;     // out-degree sum of levels 0..min(level, k-1)
    int64_t nf;     // frontier size (vertices at distance == level)
    int64_t qlen;   // frontier vertices with out-degree > 0 (queue length)
    int64_t mf;     // out-degree sum of the frontier
    int64_t mu;     // in-degree sum of unvisited vertices
    int64_t *out_count;
    int64_t *out_te;
    int32_t dir;    // direction of the next expansion
    int32_t level;  // completed levels
    int32_t done;   // the count is final and written out
    int32_t k;
    int32_t dir_mode, alpha, beta, pad0;
    uint32_t ticket;
    uint32_t pad1;
};

struct Graph {
    const int64_t *__restrict__ rowptr;
    const int32_t *__restrict__ colidx;
    const int64_t *__restrict__ in_rowptr;
    const int32_t *__restrict__ in_colidx;
    int64_t n;
    int64_t nw;  // 64-vertex words
    int directed;
};

struct State {
    uint64_t *V;      // visited bitmap
    uint64_t *F0;     // frontier bitmaps, double buffered by level parity
    uint64_t *F1;
    uint8_t *nextb;   // top-down mark bytes, all zero between hops
    int32_t *q;       // frontier queue
    int64_t *qoff;    // exclusive prefix of queue out-degrees, qoff[qlen] = mf
    int64_t *part;    // per-block partials
    int64_t *boff;    // per-block queue / degree offsets
    int wpb;          // words per block
    int nblk;         // blocks of the word-range kernels
};

__device__ __forceinline__ uint64_t *frontier(const State &s, int completed_levels) {
    return (completed_levels & 1) ? s.F1 : s.F0;
}

__device__ __forceinline__ int64_t ld_relaxed(const int64_t *p) {
    return __hip_atomic_load(const_cast<int64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide exclusive scan of two values; totals returned through t0/t1.
__device__ void block_scan2(int64_t a, int64_t b, int64_t &ea, int64_t &eb, int64_t &t0, int64_t &t1) {
    __shared__ int64_t s_a[kWavesPerBlock], s_b[kWavesPerBlock];
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    int64_t xa = wave_exclusive_sum(a), xb = wave_exclusive_sum(b);
    if (lane == kWave - 1) {
        s_a[wv] = xa + a;
        s_b[wv] = xb + b;
    }
    __syncthreads();
    int64_t pa = 0, pb = 0, ta = 0, tb = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
        if (i < wv) {
            pa += s_a[i];
            pb += s_b[i];
        }
        ta += s_a[i];
        tb += s_b[i];
    }
    __syncthreads();
    ea = xa + pa;
    eb = xb + pb;
    t0 = ta;
    t1 = tb;
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

// One ticket per block; true in every thread of the last block to arrive.
__device__ bool arrive_last(PlainCtl *ctl, int nblk) {
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = __hip_atomic_fetch_add(&ctl->ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (t == (uint32_t)nblk - 1);
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last != 0;
}

// Executed by the last block: reduce partials, prefix the queue offsets, advance the level.
__device__ void finalize_level(PlainCtl *ctl, int L, const State &s, const Graph &g, int64_t *units) {
    int64_t run_q = 0, run_d = 0, tot_c = 0, tot_i = 0, tot_pe = 0, tot_pv = 0;
    for (int base = 0; base < s.nblk; base += kBlock) {
        const int b = base + threadIdx.x;
        int64_t c = 0, qc = 0, md = 0, di = 0, pe = 0, pv = 0;
        if (b < s.nblk) {
            const int64_t *p = s.part + (int64_t)b * kPart;
            c = ld_relaxed(p + 0);
            qc = ld_relaxed(p + 1);
            md = ld_relaxed(p + 2);
            di = ld_relaxed(p + 3);
            pe = ld_relaxed(p + 4);
            pv = ld_relaxed(p + 5);
        }
        int64_t eq, ed, tq, td;
        block_scan2(qc, md, eq, ed, tq, td);
        if (b < s.nblk) {
            s.boff[2 * (int64_t)b] = run_q + eq;
            s.boff[2 * (int64_t)b + 1] = run_d + ed;
        }
        run_q += tq;
        run_d += td;
        tot_c += block_sum(c);
        tot_i += block_sum(di);
        tot_pe += block_sum(pe);
        tot_pv += block_sum(pv);
    }
    if (threadIdx.x == 0) {
        const int64_t cnt = tot_c;
        ctl->count += cnt;
        ctl->level = L;
        ctl->nf = cnt;
        ctl->qlen = run_q;
        ctl->mf = run_d;
        ctl->mu -= tot_i;
        s.qoff[run_q] = run_d;
        if (L < ctl->k) ctl->te += run_d;
        const int done = (cnt == 0) || (L >= ctl->k);
        int dir = ctl->dir;
        if (ctl->dir_mode == DIR_PUSH) {
            dir = DIR_PUSH;
        } else if (ctl->dir_mode == DIR_PULL) {
            dir = DIR_PULL;
        } else if (dir == DIR_PUSH) {
            if (run_d * (int64_t)ctl->alpha > ctl->mu) dir = DIR_PULL;
        } else {
            if (cnt * (int64_t)ctl->beta < g.n) dir = DIR_PUSH;
        }
        ctl->dir = dir;
        ctl->done = done;
        if (done) {
            *ctl->out_count = ctl->count;
            if (ctl->out_te) *ctl->out_te = ctl->te;
        }
        ctl->ticket = 0;
        if (units) {
            // bottom-up hop: 4 B per examined in-edge, 16 B row pointers per scanned
            // vertex, visited read + frontier write of n/8 B each
            units[0] = 4 * tot_pe + 16 * tot_pv + 2 * ((g.n + 7) / 8);
            units[1] = tot_pe;
            units[2] = tot_pv;
        }
    }
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
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->out_count = out_count + qi;
        ctl->out_te = out_te ? out_te + qi : nullptr;
        ctl->ticket = 0;
        ctl->dir_mode = dir_mode;
        ctl->alpha = alpha;
        ctl->beta = beta;
        ctl->k = k;
        ctl->level = 0;
        ctl->count = 0;
        if (!valid) {
            ctl->done = 1;
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
        ctl->qlen = od > 0 ? 1 : 0;
        ctl->nf = 1;
        ctl->mf = od;
        ctl->mu = nnz_in - id;
        ctl->te = k >= 1 ? od : 0;
        ctl->dir = dir_mode == DIR_PULL ? DIR_PULL : DIR_PUSH;
        ctl->done = (k == 0) ? 1 : 0;
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
__device__ void push_expand(const PlainCtl *ctl, const Graph &g, const State &s) {
    const int lane = lane_id();
    const int64_t qlen = ctl->qlen;
    const int64_t E = ctl->mf;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t e0 = E * wid / nwaves, e1 = E * (wid + 1) / nwaves;
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

__device__ void pull_expand(PlainCtl *ctl, int L, const Graph &g, const State &s, int light, int64_t *units) {
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    const uint64_t *__restrict__ Fc = frontier(s, L - 1);
    uint64_t *__restrict__ Fn = frontier(s, L);
    const int64_t w0 = (int64_t)blockIdx.x * s.wpb;
    const int64_t w1 = std::min<int64_t>(w0 + s.wpb, g.nw);
    int64_t c_cnt = 0, c_q = 0, c_mf = 0, c_din = 0, c_pe = 0, c_pv = 0;  // lane-0 totals
    for (int64_t w = w0 + wv; w < w1; w += kWavesPerBlock) {
        const uint64_t vis = s.V[w];
        const int64_t v = w * kWave + lane;
        const bool unv = v < g.n && !((vis >> lane) & 1ull);
        uint64_t found_mask = 0;
        int64_t b = 0, e = 0;
        if (ballot(unv)) {
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
            uint64_t heavy = ballot(unv && d > light);
            while (heavy) {
                const int h = __builtin_ctzll(heavy);
                heavy &= heavy - 1;
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
            c_pe += wave_sum(examined);
            c_pv += __popcll(ballot(unv));
        }
        if (lane == 0) {
            Fn[w] = found_mask;
            if (found_mask) s.V[w] = vis | found_mask;
        }
        if (found_mask) {
            const bool f = (found_mask >> lane) & 1ull;
            int64_t od = 0, din = 0;
            if (f) {
                din = e - b;
                od = g.directed ? g.rowptr[v + 1] - g.rowptr[v] : din;
            }
            c_cnt += __popcll(found_mask);
            c_q += __popcll(ballot(f && od > 0));
            c_mf += wave_sum(od);
            c_din += wave_sum(din);
        }
    }
    // block partials (lane values are wave-uniform; count each wave once)
    const bool l0 = lane == 0;
    const int64_t t_cnt = block_sum(l0 ? c_cnt : 0), t_q = block_sum(l0 ? c_q : 0);
    const int64_t t_mf = block_sum(l0 ? c_mf : 0), t_din = block_sum(l0 ? c_din : 0);
    const int64_t t_pe = block_sum(l0 ? c_pe : 0), t_pv = block_sum(l0 ? c_pv : 0);
    if (threadIdx.x == 0) {
        int64_t *p = s.part + (int64_t)blockIdx.x * kPart;
        p[0] = t_cnt;
        p[1] = t_q;
        p[2] = t_mf;
        p[3] = t_din;
        p[4] = t_pe;
        p[5] = t_pv;
    }
    if (arrive_last(ctl, s.nblk)) finalize_level(ctl, L, s, g, units);
}

__global__ void __launch_bounds__(kBlock) plain_expand_kernel(PlainCtl *ctl, int L, Graph g, State s, int light,
                                                             int64_t *units) {
    const int done = ctl->done, level = ctl->level, dir = ctl->dir;
    if (done || level != L - 1) {
        if (units && blockIdx.x == 0 && threadIdx.x == 0) units[0] = 0;
        return;
    }
    if (dir == DIR_PUSH) {
        if (units && blockIdx.x == 0 && threadIdx.x == 0) {
            // top-down hop: 4 B per frontier edge, 16 B row pointers + 4 B queue entry per frontier vertex
            units[0] = 4 * ctl->mf + 20 * ctl->qlen;
            units[1] = ctl->mf;
            units[2] = ctl->qlen;
        }
        push_expand(ctl, g, s);
    } else {
        pull_expand(ctl, L, g, s, light, units);
    }
}

// ------------------------------------------------------------------ compaction

__global__ void __launch_bounds__(kBlock) plain_compact_kernel(PlainCtl *ctl, int L, Graph g, State s,
                                                              int64_t *units) {
    const int done = ctl->done, level = ctl->level;
    if (done || level != L - 1) {  // a bottom-up hop already compacted
        if (units && blockIdx.x == 0 && threadIdx.x == 0) units[0] = 0;
        return;
    }
    if (units && blockIdx.x == 0 && threadIdx.x == 0) units[0] = g.n + (g.n + 7) / 8;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    uint64_t *__restrict__ Fn = frontier(s, L);
    const int64_t w0 = (int64_t)blockIdx.x * s.wpb;
    const int64_t w1 = std::min<int64_t>(w0 + s.wpb, g.nw);
    int64_t c_cnt = 0, c_q = 0, c_mf = 0, c_din = 0;
    for (int64_t w = w0 + wv; w < w1; w += kWavesPerBlock) {
        const int64_t v = w * kWave + lane;
        const uint8_t nb = v < g.n ? s.nextb[v] : 0;
        const uint64_t vis = s.V[w];
        const bool fresh = nb && !((vis >> lane) & 1ull);
        const uint64_t m = ballot(fresh);
        if (nb) s.nextb[v] = 0;
        if (lane == 0) {
            Fn[w] = m;
            if (m) s.V[w] = vis | m;
        }
        if (m) {
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
    if (threadIdx.x == 0) {
        int64_t *p = s.part + (int64_t)blockIdx.x * kPart;
        p[0] = t_cnt;
        p[1] = t_q;
        p[2] = t_mf;
        p[3] = t_din;
        p[4] = 0;
        p[5] = 0;
    }
    if (arrive_last(ctl, s.nblk)) finalize_level(ctl, L, s, g, nullptr);
}

// ------------------------------------------------------------------ queue

// Ascending frontier queue + out-degree prefix: each wave takes a contiguous
// quarter of the block's words; pass A totals, LDS exchange, pass B writes.
__global__ void __launch_bounds__(kBlock) plain_queue_kernel(PlainCtl *ctl, int L, Graph g, State s,
                                                            int64_t *units) {
    const int done = ctl->done, level = ctl->level, dir = ctl->dir;
    if (done || level != L || dir != DIR_PUSH) {
        if (units && blockIdx.x == 0 && threadIdx.x == 0) units[0] = 0;
        return;
    }
    if (units && blockIdx.x == 0 && threadIdx.x == 0) units[0] = (g.n + 7) / 8 + 12 * ctl->qlen + 16 * ctl->nf;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
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
    int64_t qpos = s.boff[2 * (int64_t)blockIdx.x], dpos = s.boff[2 * (int64_t)blockIdx.x + 1];
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
    void *arena = nullptr;
};

PlainCtx *plain_ctx_create(khop_graph *g) {
    PlainCtx *c = new PlainCtx();
    c->g = g;
    const int64_t n = g->n, nw = (n + 63) / 64;
    const int wpb = g->params.words_per_block;
    const int nblk = (int)((nw + wpb - 1) / wpb);
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
    const size_t o_boff = off;
    off += al((size_t)nblk * 2 * 8);
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
    c->s.boff = (int64_t *)(base + o_boff);
    c->s.wpb = wpb;
    c->s.nblk = nblk;
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
    Graph gr{g->d_rowptr, g->d_colidx, g->d_in_rowptr, g->d_in_colidx, g->n, (g->n + 63) / 64, g->directed};
    const Params &P = g->params;
    const int nblk = c->s.nblk;
    const int init_grid = (int)std::max<int64_t>(1, std::min<int64_t>((gr.nw + kBlock - 1) / kBlock, 1024));
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
                hipLaunchKernelGGL(plain_expand_kernel, dim3(nblk), dim3(kBlock), 0, st, c->ctl, L, gr, c->s,
                                   P.pull_light, ps.units());
                ps.end(0, 1);
            }
            {
                ProfScope ps(g, KK_PLAIN_COMPACT, st);
                hipLaunchKernelGGL(plain_compact_kernel, dim3(nblk), dim3(kBlock), 0, st, c->ctl, L, gr, c->s,
                                   ps.units());
                ps.end(0, 1);
            }
            if (L < k) {
                ProfScope ps(g, KK_PLAIN_QUEUE, st);
                hipLaunchKernelGGL(plain_queue_kernel, dim3(nblk), dim3(kBlock), 0, st, c->ctl, L, gr, c->s,
                                   ps.units());
                ps.end(0, 1);
            }
        }
    }
    KHOP_HIP(hipGetLastError());
}

}  // namespace khop
