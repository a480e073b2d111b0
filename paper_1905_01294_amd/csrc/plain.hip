// Plain single-query k-hop count on gfx950.
//
// One hop is the masked boolean product of the paper's Section II: the next
// frontier is (A^T f) AND NOT visited over the (OR, AND) semiring.  A query is
// one hop per launch; a hop 2..k-1 is followed by a compaction kernel
// (which exits at once unless the hop marked bytes).  All of the seed's
// neighbors are new (a row has no duplicate and no self-loop), so hop 1
// needs no claims unless the seed has more than 64 neighbors per region (it
// queues them 64 to a region), and as a last hop it counts them straight
// from the seed's row (with no vertex mask, a one-hop query is a single
// launch that reads its seed's degree).  A later last hop only counts:
// bottom-up it counts its finds, top-down it marks bytes that a later launch
// counts.  So no last hop needs a compaction.
// Consecutive queries are pipelined.  A step launch runs the last hop of
// query i-1 and hop 1 of query i side by side on separate blocks, and on a
// third set of blocks counts the byte marks an earlier query's last hop left,
// writes that query's predecessor's count and sets up query i+1 (its
// control record, and its bitmaps reset).  So a query needs no launch of its
// own for set-up, and one of k >= 2 hops costs k-1 launches plus
// compactions.
// Bitmaps and region counters rotate over three states, control records over
// five slots and queues over two sets.  Every cross-block hand-off happens at
// a kernel boundary (intra-kernel release fences would write back L2 on this
// multi-XCD part).
//
// The frontier queue is split into regions of consecutive vertices; region r
// owns queue slots [r*RC, (r+1)*RC) and one packed 64-bit counter
// (count << 33 | out-degree sum), so that appending a batch reserves its slots
// and its out-degree offsets with one atomic, and appends spread over many
// addresses instead of serialising on one.
//
// Hop kernel, all blocks:
//   1. read the previous hop's region counters, prefix their degree sums in
//      LDS, and pick the direction with Beamer-style thresholds on the totals
//      (every block computes the same choice);
//   2. top-down (push): an edge-balanced sweep over the regions' queues.  With
//      few frontier edges each unvisited head is claimed by an atomicOr on its
//      visited word (the old value makes the discovery exactly-once) and
//      appended at once; with many, heads are only marked in a byte map (no
//      atomics) and the compaction kernel turns the marks into frontier words
//      with ballots;
//      bottom-up (pull): one wave per 64-vertex word, each unvisited vertex
//      tests its probe in-neighbor (largest out-degree), then scans its other
//      in-neighbors against the frontier bitmap and stops at the first hit;
//      the ballot of hits is the word's new frontier bits.
//      In-edges of vertices above the heavy threshold are split into chunks
//      that any wave may scan.
// Block 0 keeps the running count and traversed-edge sum.  Within a query,
// hop records, region counters and frontier bitmaps rotate over three slots
// (hop l writes slot l, reads slot l-1 and clears slot l+1), queues over two.
#include <algorithm>

#include "khop_impl.h"
#include "plain_plan.h"
#include "wave.h"

namespace khop {

using namespace dev;

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxRegions = 256;  // regions of a hop: four per lane of the one wave that prefixes them
constexpr int kSumBits = 33;         // packed (count << 33) | sum
constexpr uint64_t kSumMask = (1ull << kSumBits) - 1;
constexpr int kTail = 256;           // lanes of a query's last-hop counter
enum { DIR_PUSH = KHOP_DIR_PUSH, DIR_PULL = KHOP_DIR_PULL };
enum { MODE_PULL = 0, MODE_PUSH_ATOMIC = 1, MODE_PUSH_BYTES = 2, MODE_IDLE = 3 };

struct RegRec {
    uint64_t qpack;  // (queued vertices << 33) | their out-degree sum
    uint64_t fpack;  // (discovered vertices << 33) | their in-degree sum
};

struct HopHdr {
    int64_t mu_before;  // in-degree sum of the vertices unvisited before this hop
    int32_t dir;        // direction this hop used
    int32_t mode;       // MODE_*
};

struct PlainCtl {
    HopHdr hdr[3];      // hop l's header in hdr[l % 3]; hdr[0] describes the seed
    int64_t count_acc;  // vertices discovered at hops 1..l-1 (kept by block 0 of hop l)
    int64_t te_acc;     // out-degree sum of the frontiers of hops 0..l-1
    int64_t *out_count;
    int64_t *out_te;
    int64_t push_atomic_max;  // frontier edges up to which a push claims heads atomically
    int32_t k, dir_mode, alpha, beta;
    int32_t valid;
    int32_t last_bytes;  // the last hop left byte marks (counted by a later step launch)
    int32_t reached;     // largest level found non-empty so far (the seed's is 0)
    int32_t more;        // breadth-first search: the level the last probe read is non-empty
    int64_t *level_out;  // breadth-first search: size of each level 1..level_cap (else null)
    int64_t level_cap;
    int64_t seed_beg;    // the seed's first out-edge, its out- and in-degree (hop 1 reads them)
    int64_t seed_od;
    int64_t seed_id;
    int64_t tail[kTail];  // discoveries of the last hop, spread over many addresses
};

struct Graph {
    const int64_t *__restrict__ rowptr;
    const int32_t *__restrict__ colidx;
    const int64_t *__restrict__ in_rowptr;
    const int32_t *__restrict__ in_colidx;
    int64_t n;
    int64_t nw;  // 64-vertex words
    int directed;
    int heavy;   // bottom-up: in-degree above which the chunk table takes a vertex
    // per vertex: the first entry of its in-row (largest out-degree), -1 with
    // none.  (Last: placed among the fields above it, it changed the step
    // kernel's scalar register allocation, and a step launch took 0.3 to
    // 0.5 µs longer.)
    const int32_t *__restrict__ probe;
};

// What one query runs on: the bitmaps, byte map and region counters of one
// of the three states, and the queues of one of the two sets.  (A step
// launch counts the marks an earlier query left while the query whose last
// hop it runs may mark its own: the byte maps must differ.)
struct State {
    uint64_t *V;       // visited bitmap
    uint64_t *F[3];    // frontier bitmaps by hop % 3
    uint8_t *nextb;    // top-down marks (byte mode), all zero between hops
    uint8_t *nsum;     // one byte per 64-vertex word: some mark of the word may be set
    int32_t *dist;     // breadth-first search: distance of each vertex, set when it is found (else null)
    const uint64_t *vmask;  // vertices the search may enter, one bit each (null: all); the others start visited
    int64_t *qb[2];    // region queues by hop parity, nreg * rc slots: the row begin of each queued vertex
    int64_t *qoff[2];  // out-degree prefix within each region's queue
    RegRec *regs;      // 3 * nreg region counters
    // One byte per block of 64 words (4096 vertices): some visited or frontier
    // bit of the block may be set beyond the query's start (its seed; under a
    // vertex mask, the vertices outside it).  A query's set-up rewrites only
    // the flagged blocks and the seed's.  Null: every set-up rewrites every word.
    uint8_t *dirty;
    int nreg;          // regions
    int rw;            // words per region
    int64_t rc;        // slots per region (rw * 64)
};

struct HeavyChunks {
    const int32_t *vert;   // vertex of each chunk
    const int64_t *begin;  // first in-edge of each chunk
    const int64_t *end;    // one past its last in-edge
    int64_t n;
};

// The blocks of a launch that run one piece of its work: a launch may split
// its grid between a hop of one query and hop 1 of the next, and each piece
// sees only its own block index and block count.
struct Part {
    int64_t bid;  // block index within the piece
    int64_t nb;   // blocks of the piece
};


__device__ __forceinline__ int64_t pk_count(uint64_t p) { return (int64_t)(p >> kSumBits); }
__device__ __forceinline__ int64_t pk_sum(uint64_t p) { return (int64_t)(p & kSumMask); }
__device__ __forceinline__ uint64_t pk(int64_t count, int64_t sum) {
    return ((uint64_t)count << kSumBits) + (uint64_t)sum;
}

// Appends one discovered vertex v, whose out-edges start at beg (a single lane).
__device__ __forceinline__ void append_one(const State &s, RegRec *regs, int L, int32_t v, int64_t beg, int64_t od,
                                           int64_t id) {
    const int r = (int)(((int64_t)v >> 6) / s.rw);
    if (od > 0) {
        const uint64_t old = atomicAdd((unsigned long long *)&regs[r].qpack, (unsigned long long)pk(1, od));
        const int64_t at = (int64_t)r * s.rc + pk_count(old);
        s.qb[L & 1][at] = beg;
        s.qoff[L & 1][at] = pk_sum(old);
    }
    atomicAdd((unsigned long long *)&regs[r].fpack, (unsigned long long)pk(1, id));
}

// Per-wave LDS buffer of discoveries in one region, flushed with one
// returning atomic per region instead of one per word.
constexpr int kBufCap = 512;
struct WaveBuf {
    int64_t *v;    // LDS, cap row begins of the buffered vertices
    int32_t *d;    // their out-degrees
    int cap;       // entries the buffer holds (at least 64)
    int cnt;       // buffered entries (wave-uniform)
    int reg;       // region of the buffered entries, -1 if none
    int64_t nf;    // discovered in that region (all, wave-uniform)
    int64_t din;   // their in-degree sum
};

__device__ void wb_flush(WaveBuf &b, const State &s, RegRec *regs, int L) {
    if (b.reg < 0 || (b.cnt == 0 && b.nf == 0)) return;
    const int lane = lane_id();
    int64_t dsum = 0;
    for (int i = lane; i < b.cnt; i += kWave) dsum += b.d[i];
    dsum = wave_sum(dsum);
    uint64_t old = 0;
    if (lane == 0) {
        if (b.cnt) old = atomicAdd((unsigned long long *)&regs[b.reg].qpack, (unsigned long long)pk(b.cnt, dsum));
        if (b.nf) atomicAdd((unsigned long long *)&regs[b.reg].fpack, (unsigned long long)pk(b.nf, b.din));
    }
    old = (uint64_t)shfl64((int64_t)old, 0);
    const int64_t base = (int64_t)b.reg * s.rc + pk_count(old);
    int64_t dpos = pk_sum(old);
    for (int i0 = 0; i0 < b.cnt; i0 += kWave) {
        const int i = i0 + lane;
        const int64_t d = i < b.cnt ? b.d[i] : 0;
        const int64_t dx = wave_exclusive_sum(d);
        if (i < b.cnt) {
            s.qb[L & 1][base + i] = b.v[i];
            s.qoff[L & 1][base + i] = dpos + dx;
        }
        dpos += wave_sum(d);
    }
    b.cnt = 0;
    b.nf = 0;
    b.din = 0;
    __builtin_amdgcn_wave_barrier();
}

// Buffers the lanes of word w that have `found`, with their row begins (wave-uniform call).
__device__ __forceinline__ void wb_word(WaveBuf &b, const State &s, RegRec *regs, int L, int64_t w, bool found,
                                       int64_t beg, int64_t od, int64_t id) {
    const uint64_t fm = ballot(found);
    if (!fm) return;
    const int r = (int)(w / s.rw);
    const bool qd = found && od > 0;
    const uint64_t qm = ballot(qd);
    const int nq = __popcll(qm);
    if (r != b.reg || b.cnt + nq > b.cap) {
        wb_flush(b, s, regs, L);
        b.reg = r;
    }
    if (qd) {
        const int at = b.cnt + mask_rank(qm);
        b.v[at] = beg;
        b.d[at] = (int32_t)od;
    }
    b.cnt += nq;
    b.nf += __popcll(fm);
    b.din += wave_sum(found ? id : 0);
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------------ query set-up and close

// Lanes whose byte of x is nonzero, one bit per byte (16 bytes).
__device__ __forceinline__ uint32_t nonzero_bytes(uint4 x) {
    auto f = [](uint32_t w) -> uint32_t {
        const uint32_t y = (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;
        return ((y >> 7) & 1u) | ((y >> 14) & 2u) | ((y >> 21) & 4u) | ((y >> 28) & 8u);
    };
    return f(x.x) | (f(x.y) << 4) | (f(x.z) << 8) | (f(x.w) << 12);
}

// Marks head v in the byte map and, with `summary`, its word in the summary
// (plain stores).
__device__ __forceinline__ void mark(const State &s, int32_t v, bool summary) {
    s.nextb[v] = 1;
    if (summary) s.nsum[v >> 6] = 1;
}

// A last hop's marks are counted by a later launch that reads, on a graph of
// up to this many 64-vertex words (a byte map of up to 4 MB), the whole byte
// map: one sequential read costs less than a summary store beside every
// scattered mark.  On larger graphs the marks keep a summary, and only the
// flagged words are read.  (The marks of an inner hop always keep one: the
// compaction after the hop reads them.)
constexpr int64_t kMarkSummaryWords = 65536;
__device__ __forceinline__ bool last_marks_summary(const Graph &g) { return g.nw > kMarkSummaryWords; }

// The byte marks a byte-mode last hop left on the 64 vertices of word w that
// were unvisited (visited word vis); the marks and the word's summary byte
// are cleared, and `had` says whether there were any.  The byte map is padded
// to whole words.
__device__ __forceinline__ int64_t close_marks_word(const State &s, int64_t w, uint64_t vis, bool &had) {
    uint4 *mb = (uint4 *)(s.nextb + w * kWave);
    uint64_t m = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) m |= (uint64_t)nonzero_bytes(mb[j]) << (16 * j);
    had = m != 0;
    if (!m) return 0;
    s.nsum[w] = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) mb[j] = make_uint4(0, 0, 0, 0);
    return __popcll(m & ~vis);
}

// Adds a wave's share of a finished query's last-hop discoveries.
__device__ __forceinline__ void add_tail(PlainCtl *ctl, int64_t wid, int64_t v) {
    if (v) atomicAdd((unsigned long long *)&ctl->tail[wid & (kTail - 1)], (unsigned long long)v);
}

// Writes the count and traversed edges of a finished query (one wave).  Every
// field is read first, so the loads overlap.
__device__ void finalize(PlainCtl *ctl) {
    const int lane = lane_id();
    const int32_t valid = ctl->valid;
    const int64_t cacc = ctl->count_acc, teacc = ctl->te_acc;
    int64_t *const oc = ctl->out_count, *const ot = ctl->out_te;
    int64_t t = 0;
#pragma unroll
    for (int i = 0; i < kTail / kWave; ++i) t += ctl->tail[i * kWave + lane];
#pragma unroll
    for (int i = 0; i < kTail / kWave; ++i) ctl->tail[i * kWave + lane] = 0;
    t = wave_sum(t);
    if (lane == 0 && valid) {
        *oc = cacc + t;
        if (ot) *ot = teacc;
    }
}

// One block: the control record of query qi (seed `seed`) and the region
// counters of its hops 0 and 1 (hop 0 holds the seed).  Its bitmap words are
// reset by the caller's grid.
__device__ void setup_query(PlainCtl *ctl, const Graph &g, const State &s, int32_t seed, int64_t qi, int k,
                            int dir_mode, int alpha, int beta, int64_t push_atomic_max, int64_t nnz_in,
                            int64_t *out_count, int64_t *out_te, int64_t *units) {
    const bool valid = seed >= 0 && (int64_t)seed < g.n;
    for (int i = threadIdx.x; i < 2 * s.nreg; i += kBlock) {
        s.regs[i].qpack = 0;
        s.regs[i].fpack = 0;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    ctl->out_count = out_count + qi;
    ctl->out_te = out_te ? out_te + qi : nullptr;
    ctl->dir_mode = dir_mode;
    ctl->alpha = alpha;
    ctl->beta = beta;
    ctl->k = k;
    ctl->valid = valid;
    ctl->last_bytes = 0;
    ctl->reached = 0;
    ctl->more = 1;
    ctl->level_out = nullptr;
    ctl->level_cap = 0;
    ctl->push_atomic_max = push_atomic_max;
    ctl->count_acc = 0;
    ctl->te_acc = 0;
    ctl->seed_od = 0;
    if (!valid) {
        out_count[qi] = -1;
        if (out_te) out_te[qi] = -1;
        return;
    }
    const int64_t beg = g.rowptr[seed];
    const int64_t od = g.rowptr[seed + 1] - beg;
    const int64_t id = g.in_rowptr[seed + 1] - g.in_rowptr[seed];
    ctl->seed_beg = beg;
    ctl->seed_od = od;
    ctl->seed_id = id;
    const int64_t sw = seed >> 6;
    const int r = (int)(sw / s.rw);
    // hop 0's counters describe the seed; no queue entry is needed, since a
    // top-down hop 1 reads the seed's row from this record
    if (od > 0) s.regs[r].qpack = pk(1, od);
    s.regs[r].fpack = pk(1, id);
    ctl->hdr[0].mu_before = nnz_in;
    ctl->hdr[0].dir = dir_mode == DIR_PULL ? DIR_PULL : DIR_PUSH;
    ctl->hdr[0].mode = MODE_IDLE;
}

// Word w of a query's visited and frontier bitmaps at its start: the seed's
// bit only (sw = -1: no seed).  With a vertex mask, the vertices outside it
// start visited, so that the mask of every masked product (NOT visited)
// excludes them too and the search never enters them (bits past the last
// vertex stay clear).
__device__ __forceinline__ void reset_word(const State &s, const Graph &g, int64_t w, int64_t sw, uint64_t sbit) {
    const uint64_t x = (w == sw) ? sbit : 0ull;
    uint64_t v = x;
    if (s.vmask) {
        const uint64_t valid = (w == g.nw - 1 && (g.n & 63)) ? ((1ull << (g.n & 63)) - 1) : ~0ull;
        v |= ~s.vmask[w] & valid;
    }
    s.V[w] = v;
    s.F[0][w] = x;
    s.F[1][w] = 0;
}

// Flags the block of word w: a visited or frontier bit of it is being set.
__device__ __forceinline__ void mark_dirty(const State &s, int64_t w) {
    if (s.dirty) s.dirty[w >> 6] = 1;
}

// The block flag after a set-up that reset word w (every lane of the wave,
// whose 64 words are the block; the lane of its first word writes): set for
// the seed's block and, under a vertex mask, for every block.
__device__ __forceinline__ void reset_dirty(const State &s, int64_t w, int64_t sw) {
    if (s.dirty && (w & 63) == 0) s.dirty[w >> 6] = (s.vmask || (sw >= 0 && (w >> 6) == (sw >> 6))) ? 1 : 0;
}

// Set-up of the first query of a run (later queries are set up by the hop 1
// of the query before them).
__global__ void __launch_bounds__(kBlock) plain_init_kernel(PlainCtl *ctl, Graph g, State s, const int32_t *seeds,
                                                           int64_t qi, int k, int dir_mode, int alpha, int beta,
                                                           int64_t push_atomic_max, int64_t nnz_in,
                                                           int64_t *out_count, int64_t *out_te, int64_t *units) {
    const int32_t seed = seeds[qi];
    const bool valid = seed >= 0 && (int64_t)seed < g.n;
    const int64_t sw = valid ? (seed >> 6) : -1;
    const uint64_t sbit = valid ? (1ull << (seed & 63)) : 0;
    for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < g.nw; w += (int64_t)gridDim.x * kBlock) {
        reset_word(s, g, w, sw, sbit);
        reset_dirty(s, w, sw);
    }
    if (blockIdx.x == 0) {
        setup_query(ctl, g, s, seed, qi, k, dir_mode, alpha, beta, push_atomic_max, nnz_in, out_count, out_te,
                    units);
        if (threadIdx.x == 0) unit_add(units, 0, 3 * 8 * g.nw);  // every word of V, F[0] and F[1]
    }
}

// End of a run: the last query's byte marks (if its last hop left any), and
// the count of the query before it.
__global__ void __launch_bounds__(kBlock) plain_close_kernel(PlainCtl *ctl_last, PlainCtl *ctl_before,
                                                            int fin_before, Graph g, State s_last, int64_t *units) {
    if (ctl_last->last_bytes) {
        const bool summary = last_marks_summary(g);
        int64_t fresh = 0, flagged = 0;
        for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < g.nw; w += (int64_t)gridDim.x * kBlock)
            if (!summary || s_last.nsum[w]) {
                bool had;
                fresh += close_marks_word(s_last, w, s_last.V[w], had);
                flagged += had;
            }
        fresh = wave_sum(fresh);
        flagged = wave_sum(flagged);
        if (lane_id() == 0) add_tail(ctl_last, (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave, fresh);
        // the summary bytes (or the whole byte map), then the marks cleared and visited word of each flagged word
        if (lane_id() == 0) unit_add(units, 0, 72 * flagged);
        if (blockIdx.x == 0 && threadIdx.x == 0) unit_add(units, 0, summary ? g.nw : 64 * g.nw);
    }
    if (blockIdx.x == 0 && threadIdx.x < kWave && fin_before) finalize(ctl_before);
}

// A one-hop query with no vertex mask, as one launch of its own: its visited
// set is the seed alone, which a row (no self-loop, no duplicate) does not
// hold, so every out-neighbor is new and the count is the out-degree (which
// is also the edges it traverses).  An invalid seed gets -1.
__global__ void __launch_bounds__(kWave) plain_degree_kernel(const int32_t *seeds, int64_t i,
                                                            const int64_t *__restrict__ rowptr, int64_t n,
                                                            int64_t *counts, int64_t *te) {
    if (threadIdx.x != 0) return;
    const int32_t seed = seeds[i];
    const bool valid = seed >= 0 && (int64_t)seed < n;
    const int64_t d = valid ? rowptr[seed + 1] - rowptr[seed] : -1;
    counts[i] = d;
    if (te) te[i] = d;
}

// Writes the last query's count (wave 0) and, when given, the count of the
// one before it (wave 1).
__global__ void __launch_bounds__(2 * kWave) plain_final_kernel(PlainCtl *ctl, PlainCtl *ctl_before) {
    if (threadIdx.x < kWave) finalize(ctl);
    else if (ctl_before) finalize(ctl_before);
}

// ------------------------------------------------------------------ top-down

// Edge-balanced sweep: wave w owns edges [E*w/W, E*(w+1)/W) of the frontier's
// concatenated adjacency lists, region after region.  Within a 64-edge window
// of one region's queue, the owning entry of each lane is base - 1 + (number
// of list starts at or before it).
// With `last` set (the query's final hop) discoveries are only counted into
// *found: no frontier word, queue entry or degree is needed afterwards.
// Claims head v, seen unvisited, with an atomicOr on its visited word (the
// old value makes the discovery exactly-once) and appends it.
__device__ __forceinline__ void push_claim(int L, const Graph &g, const State &s, RegRec *cur, uint64_t *Fn,
                                           int32_t v) {
    const uint64_t bit = 1ull << (v & 63);
    const uint64_t old = atomicOr((unsigned long long *)&s.V[v >> 6], (unsigned long long)bit);
    if (old & bit) return;
    atomicOr((unsigned long long *)&Fn[v >> 6], (unsigned long long)bit);
    mark_dirty(s, v >> 6);
    if (s.dist) s.dist[v] = L;
    const int64_t vb = g.rowptr[v];
    const int64_t od = g.rowptr[v + 1] - vb;
    const int64_t id = g.directed ? g.in_rowptr[v + 1] - g.in_rowptr[v] : od;
    append_one(s, cur, L, v, vb, od, id);
}

constexpr int kWin = 4;  // windows of 64 frontier edges in flight per wave

// A top-down hop: in byte mode each frontier edge's head gets a byte mark
// (the visited test happens when the marks are turned into frontier words or
// counted; `summary` flags its word too), else heads seen unvisited are
// claimed.
__device__ void push_hop(int L, int mode, bool summary, int64_t E, const int64_t *epre, const int32_t *qcnt,
                         const Graph &g, const State &s, RegRec *cur, uint64_t *smask, int64_t *ent,
                         int64_t *units, const Part &pt) {
    const int lane = lane_id();
    const int64_t nwaves = pt.nb * kWavesPerBlock;
    const int64_t wid = pt.bid * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t e0 = E * wid / nwaves, e1 = E * (wid + 1) / nwaves;
    if (e0 >= e1) return;
    uint64_t *Fn = s.F[L % 3];
    // first region whose edges reach past e0
    int r = 0;
    {
        int lo = 0, hi = s.nreg - 1;  // largest r with epre[r] <= e0
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (epre[mid] <= e0) lo = mid;
            else hi = mid - 1;
        }
        r = lo;
    }
    int64_t starts_seen = 0;  // queue entries whose lists start in this wave's range
    for (; r < s.nreg && epre[r] < e1; ++r) {
        const int64_t rb = epre[r], re = epre[r + 1];
        const int64_t a0 = std::max(e0, rb) - rb, a1 = std::min(e1, re) - rb;  // local edge range
        if (a0 >= a1) continue;
        const int64_t qlen = qcnt[r];
        const int64_t *__restrict__ qb = s.qb[(L - 1) & 1] + (int64_t)r * s.rc;
        const int64_t *__restrict__ qoff = s.qoff[(L - 1) & 1] + (int64_t)r * s.rc;
        const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1);
        if (qlen <= kWave) {
            // short queue: lane j holds entry j, so every window finds its
            // entries with ballots and shuffles; kWin windows at a time, their
            // column-index and visited loads issued together
            const bool has = lane < qlen;
            const int64_t offl = has ? qoff[lane] : INT64_MAX;
            const int64_t begl = has ? qb[lane] : 0;
            for (int64_t b0 = a0; b0 < a1; b0 += kWin * kWave) {
                int64_t at[kWin];
#pragma unroll
                for (int r = 0; r < kWin; ++r) {
                    const int64_t b = b0 + (int64_t)r * kWave;
                    at[r] = -1;
                    if (b >= a1) continue;  // uniform
                    const int base = __popcll(ballot(offl < b));  // entries starting before the window
                    const bool inwin = offl >= b && offl < b + kWave;
                    if (lane == 0) smask[r] = 0;
                    __builtin_amdgcn_wave_barrier();
                    if (inwin) atomicOr((unsigned long long *)&smask[r], 1ull << (offl - b));
                    __builtin_amdgcn_wave_barrier();
                    const int owner = base + __popcll(smask[r] & le) - 1;  // entry of edge b + lane
                    const int64_t ob = shfl64(begl, owner), oo = shfl64(offl, owner);
                    const int64_t e = b + lane;
                    if (e < a1) at[r] = ob + (e - oo);
                    starts_seen += __popcll(ballot(inwin));
                }
                int32_t v[kWin];
#pragma unroll
                for (int r = 0; r < kWin; ++r) v[r] = at[r] >= 0 ? g.colidx[at[r]] : -1;
                if (mode == MODE_PUSH_BYTES) {
#pragma unroll
                    for (int r = 0; r < kWin; ++r)
                        if (v[r] >= 0) mark(s, v[r], summary);
                } else {
                    uint64_t vw[kWin];
#pragma unroll
                    for (int r = 0; r < kWin; ++r) vw[r] = v[r] >= 0 ? s.V[v[r] >> 6] : ~0ull;
#pragma unroll
                    for (int r = 0; r < kWin; ++r)
                        if (!((vw[r] >> (v[r] & 63)) & 1ull)) push_claim(L, g, s, cur, Fn, v[r]);
                }
                __builtin_amdgcn_wave_barrier();
            }
            continue;
        }
        // base = #{ j < qlen : qoff[j] < a0 } by a 64-way search
        int64_t lo = 0, hi = qlen;
        while (hi - lo > kWave) {
            const int64_t step = (hi - lo + kWave - 1) / kWave;
            const int64_t p = lo + (int64_t)lane * step;
            const bool less = p < hi && qoff[p] < a0;
            const int t = __popcll(ballot(less));
            const int64_t nlo = t ? lo + (int64_t)(t - 1) * step + 1 : lo;
            hi = std::min(hi, lo + (int64_t)t * step);
            lo = nlo;
        }
        {
            const int64_t p = lo + lane;
            const bool less = p < hi && qoff[p] < a0;
            lo += __popcll(ballot(less));
        }
        int64_t base = lo;
        int64_t carry_beg = 0, carry_off = 0;  // the entry whose list holds the edge before the window
        if (base > 0) {
            carry_beg = qb[base - 1];
            carry_off = qoff[base - 1];
        }
        // kWin windows of 64 edges at a time.  Their lists start at most
        // kWin * 64 times, so entries base .. base + kWin*64 - 1 (staged in
        // LDS: row begins in ent[0..255], offsets in ent[256..511]) own every
        // edge of them; bit i of smask[r] marks a list starting at edge
        // b + 64r + i.  The column-index loads of all the windows are then
        // issued together.
        int64_t *const eb = ent, *const eo = ent + kWin * kWave;
        for (int64_t b = a0; b < a1; b += kWin * kWave) {
#pragma unroll
            for (int i = 0; i < kWin; ++i) {
                const int64_t j = base + lane + (int64_t)i * kWave;
                eo[lane + i * kWave] = j < qlen ? qoff[j] : INT64_MAX;
                eb[lane + i * kWave] = j < qlen ? qb[j] : 0;
            }
            if (lane < kWin) smask[lane] = 0;
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int i = 0; i < kWin; ++i) {
                const int64_t o = eo[lane + i * kWave] - b;  // >= 0: the entries start at or after b
                if (o < kWin * kWave) atomicOr((unsigned long long *)&smask[o >> 6], 1ull << (o & 63));
            }
            __builtin_amdgcn_wave_barrier();
            int64_t at[kWin];
            int before = 0;  // staged entries starting before window r
#pragma unroll
            for (int r = 0; r < kWin; ++r) {
                const uint64_t sm = smask[r];
                const int c = __popcll(sm & le);
                const int idx = before + c - 1;  // staged entry of edge b + 64r + lane, -1: the carry
                const int64_t ob = idx >= 0 ? eb[idx] : carry_beg, oo = idx >= 0 ? eo[idx] : carry_off;
                const int64_t br = b + (int64_t)r * kWave, e = br + lane;
                at[r] = e < a1 ? ob + (e - oo) : -1;
                if (br < a1) {
                    before += __popcll(sm);
                    // lists starting in this wave's range (a1 may cut the window)
                    starts_seen += __popcll(a1 - br >= kWave ? sm : sm & ((1ull << (a1 - br)) - 1));
                }
            }
            int32_t v[kWin];
#pragma unroll
            for (int r = 0; r < kWin; ++r) v[r] = at[r] >= 0 ? g.colidx[at[r]] : -1;
            if (mode == MODE_PUSH_BYTES) {
#pragma unroll
                for (int r = 0; r < kWin; ++r)
                    if (v[r] >= 0) mark(s, v[r], summary);
            } else {
                uint64_t vw[kWin];
#pragma unroll
                for (int r = 0; r < kWin; ++r) vw[r] = v[r] >= 0 ? s.V[v[r] >> 6] : ~0ull;
#pragma unroll
                for (int r = 0; r < kWin; ++r)
                    if (!((vw[r] >> (v[r] & 63)) & 1ull)) push_claim(L, g, s, cur, Fn, v[r]);
            }
            if (before > 0) {
                carry_beg = eb[before - 1];
                carry_off = eo[before - 1];
            }
            base += before;
            __builtin_amdgcn_wave_barrier();
        }
    }
    // 4 B per frontier edge, 20 B (row pointer, queue entry, offset) per frontier vertex
    if (units && lane == 0) unit_add(units, 0, 4 * (e1 - e0) + 20 * starts_seen);
}

// ------------------------------------------------------------------ bottom-up

// Whether any of the in-edges x, x + 64, x + 128, x + 192 below end comes
// from the frontier Fc.  The four index loads, then the four bitmap loads,
// are made unconditionally (an edge past end reads edge safe, a valid index
// whose result is dropped), so that no branch separates them and all four
// are in flight at once.
__device__ __forceinline__ bool any_hit4(const uint64_t *__restrict__ Fc, const int32_t *__restrict__ colidx,
                                         int64_t x, int64_t end, int64_t safe) {
    int32_t u[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) u[r] = colidx[x + r * kWave < end ? x + r * kWave : safe];
    uint64_t w[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) w[r] = Fc[(uint32_t)u[r] >> 6];
    bool any = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) any |= x + r * kWave < end && ((w[r] >> ((uint32_t)u[r] & 63u)) & 1ull);
    return any;
}

// Each wave takes its run of 64-vertex words kPullWords at a time.  Every
// unvisited vertex of in-degree up to g.heavy scans its first `light`
// in-edges alone, four per round (one 16-byte load of the round's indices,
// whose entries past the scan are ignored, then its four bitmap loads, in
// flight at once, whatever the degree; the rounds of a lane's vertices in the
// words taken together are issued together); those with more edges and no hit
// yet have the rest scanned by the whole wave, 256 in-edges per round; heavier
// vertices come from the chunk table after the words.  One word at a time:
// two raise the hop and step kernels' registers past what five waves per SIMD
// allow, and a step launch's blocks then no longer fit the device at once.
constexpr int kPullWords = 1;
__device__ void pull_hop(int L, bool last, const Graph &g, const State &s, int light, const HeavyChunks &hc,
                         RegRec *cur, WaveBuf &wb, int64_t *found_out, int64_t *units, const Part &pt) {
    const int lane = lane_id();
    light = std::min(light, g.heavy);  // the chunk table alone takes vertices above g.heavy
    const uint64_t *__restrict__ Fc = s.F[(L - 1) % 3];
    const int32_t *__restrict__ icol = g.in_colidx;
    uint64_t *Fn = s.F[L % 3];
    const int64_t nwaves = pt.nb * kWavesPerBlock;
    const int64_t wid = pt.bid * kWavesPerBlock + threadIdx.x / kWave;
    int64_t c_pe = 0, c_pv = 0;
    // a contiguous run of words per wave keeps its discoveries in one or two regions
    const int64_t wpw = (g.nw + nwaves - 1) / nwaves;
    const int64_t wb0 = std::min(wid * wpw, g.nw), wb1 = std::min(wb0 + wpw, g.nw);
    for (int64_t w0 = wb0; w0 < wb1; w0 += kPullWords) {
        uint64_t vis[kPullWords];
        bool unv[kPullWords];
        int32_t pr[kPullWords];
#pragma unroll
        for (int i = 0; i < kPullWords; ++i) {
            // the visited word and the probe in-neighbors in one round trip; a
            // vertex with no in-edge (probe -1) is never found bottom-up
            const int64_t w = w0 + i, v = w * kWave + lane;
            const bool inr = w < wb1 && v < g.n;
            vis[i] = w < wb1 ? s.V[w] : ~0ull;
            pr[i] = inr ? g.probe[v] : -1;
            unv[i] = inr && !((vis[i] >> lane) & 1ull) && pr[i] >= 0;
        }
        bool anyu = false;
#pragma unroll
        for (int i = 0; i < kPullWords; ++i) anyu |= unv[i];
        if (!ballot(anyu)) continue;
        // the row pointers, and beside them the probe's frontier word
        int64_t b[kPullWords], e[kPullWords];
        uint64_t pw[kPullWords];
#pragma unroll
        for (int i = 0; i < kPullWords; ++i) {
            const int64_t v = (w0 + i) * kWave + lane;
            b[i] = unv[i] ? g.in_rowptr[v] : 0;
            e[i] = unv[i] ? g.in_rowptr[v + 1] : 0;
            pw[i] = Fc[unv[i] ? (uint32_t)pr[i] >> 6 : 0u];
        }
        // a vertex whose probe is in the frontier is found without reading an
        // in-edge; every other unvisited vertex first scans up to `light`
        // in-edges alone, after the probe (the first in-edge of its row): on a
        // wide frontier most find a hit there, whatever their degree
        bool found[kPullWords], act[kPullWords];
        int64_t examined[kPullWords], x[kPullWords], le[kPullWords];
#pragma unroll
        for (int i = 0; i < kPullWords; ++i) {
            const int64_t d = e[i] - b[i];
            found[i] = unv[i] && d <= g.heavy && ((pw[i] >> ((uint32_t)pr[i] & 63u)) & 1ull);
            examined[i] = 0;
            x[i] = b[i] + 1;
            le[i] = b[i] + std::min<int64_t>(d, light);
            act[i] = unv[i] && !found[i] && d <= g.heavy && x[i] < le[i];
        }
        bool going = false;
#pragma unroll
        for (int i = 0; i < kPullWords; ++i) going |= act[i];
        while (going) {
            // the round's four in-edges in one 16-byte load (those past the
            // scan are ignored below)
            int32_t u[kPullWords][4];
#pragma unroll
            for (int i = 0; i < kPullWords; ++i) {
                const i32x4_u q = load4(icol, act[i] ? x[i] : 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) u[i][r] = q[r];
            }
            uint64_t fw[kPullWords][4];
#pragma unroll
            for (int i = 0; i < kPullWords; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) fw[i][r] = Fc[(uint32_t)u[i][r] >> 6];
            going = false;
#pragma unroll
            for (int i = 0; i < kPullWords; ++i) {
                if (!act[i]) continue;
                int pos = 4;  // first hit of the round
#pragma unroll
                for (int r = 3; r >= 0; --r)
                    if (x[i] + r < le[i] && ((fw[i][r] >> ((uint32_t)u[i][r] & 63u)) & 1ull)) pos = r;
                if (pos < 4) {
                    examined[i] += pos + 1;
                    found[i] = true;
                    act[i] = false;
                } else {
                    examined[i] += std::min<int64_t>(4, le[i] - x[i]);
                    x[i] += 4;
                    act[i] = x[i] < le[i];
                }
                going |= act[i];
            }
        }
#pragma unroll
        for (int i = 0; i < kPullWords; ++i) {
            const int64_t w = w0 + i;
            if (w >= wb1) break;  // uniform
            const int64_t v = w * kWave + lane, d = e[i] - b[i];
            // the rest of the in-edges of vertices with no hit yet: the whole wave, 256 per round
            uint64_t medium = ballot(unv[i] && !found[i] && d > light && d <= g.heavy);
            while (medium) {
                const int h = __builtin_ctzll(medium);
                medium &= medium - 1;
                const int64_t hb = shfl64(b[i], h) + light, he = shfl64(e[i], h);
                bool hit = false;
                int64_t scanned = 0;
                for (int64_t x0 = hb; x0 < he; x0 += 4 * kWave) {
                    const bool any = any_hit4(Fc, icol, x0 + lane, he, hb);
                    scanned += std::min<int64_t>(4 * kWave, he - x0);
                    if (ballot(any)) {
                        hit = true;
                        break;
                    }
                }
                if (lane == h) {
                    found[i] = hit;
                    examined[i] += scanned;
                }
            }
            const uint64_t fm = ballot(found[i]);
            if (last) {
                // final hop: only the count matters (chunk vertices are counted below)
                if (lane == 0) *found_out += __popcll(fm);
            } else {
                if (fm && lane == 0) {
                    // chunk waves may set heavy bits of the same words concurrently
                    atomicOr((unsigned long long *)&s.V[w], (unsigned long long)fm);
                    atomicOr((unsigned long long *)&Fn[w], (unsigned long long)fm);
                    mark_dirty(s, w);
                }
                if (found[i] && s.dist) s.dist[v] = L;
                int64_t od = 0, vb = b[i];  // undirected: the in-row is the out-row
                if (found[i] && g.directed) {
                    vb = g.rowptr[v];
                    od = g.rowptr[v + 1] - vb;
                } else if (found[i]) {
                    od = d;
                }
                wb_word(wb, s, cur, L, w, found[i], vb, od, d);
            }
            if (units) {
                c_pe += wave_sum(examined[i]);
                c_pv += __popcll(ballot(unv[i] && d <= g.heavy));
            }
        }
    }
    wb_flush(wb, s, cur, L);
    // edge chunks of heavy vertices
    int64_t h_ex = 0;
    for (int64_t i = wid; i < hc.n; i += nwaves) {
        const int32_t v = hc.vert[i];
        const uint64_t bit = 1ull << (v & 63);
        // visited before this hop, or already found by another chunk
        if (__hip_atomic_load(&s.V[v >> 6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit) continue;
        const int64_t b = hc.begin[i], e = hc.end[i];
        bool hit = false;
        for (int64_t x0 = b; x0 < e; x0 += 4 * kWave) {
            const bool any = any_hit4(Fc, g.in_colidx, x0 + lane, e, b);
            h_ex += std::min<int64_t>(4 * kWave, e - x0);
            if (ballot(any)) {
                hit = true;
                break;
            }
        }
        if (hit && lane == 0) {
            const uint64_t old = atomicOr((unsigned long long *)&s.V[v >> 6], (unsigned long long)bit);
            mark_dirty(s, v >> 6);
            if (!(old & bit)) {
                if (last) {
                    *found_out += 1;
                } else {
                    atomicOr((unsigned long long *)&Fn[v >> 6], (unsigned long long)bit);
                    if (s.dist) s.dist[v] = L;
                    const int64_t vb = g.rowptr[v];
                    const int64_t od = g.rowptr[v + 1] - vb;
                    const int64_t id = g.in_rowptr[v + 1] - g.in_rowptr[v];
                    append_one(s, cur, L, v, vb, od, id);
                }
            }
        }
    }
    if (units && lane == 0) {
        // 4 B per examined in-edge, 16 B of row pointers and the 4-byte probe per scanned vertex
        unit_add(units, 0, 4 * (c_pe + h_ex) + 20 * c_pv);
        if (wid == 0) unit_add(units, 0, 2 * ((g.n + 7) / 8));
    }
}

// Top-down hop 1 of a seed with at most 64 * nreg neighbors, not the query's
// last hop.  Every neighbor is new (the visited set holds only the seed, and
// a row has no duplicates and no self-loop), so no claim is needed: the
// visited and frontier bits are set with atomics whose old value is not read,
// and the wave that takes neighbors 64c..64c+63 appends them to region c's
// queue with a wave prefix of their out-degrees and plain stores of the
// region's counters (the queue's regions need not match the vertices' ids;
// full regions of at most 64 entries keep hop 2's sweep on its short path).
__device__ void hop1_push_free(const Graph &g, const State &s, int64_t beg, int64_t E, int64_t *units,
                               const Part &pt) {
    const int lane = lane_id();
    const int64_t nwaves = pt.nb * kWavesPerBlock;
    RegRec *cur = s.regs + s.nreg;  // hop 1's slot
    for (int64_t c = pt.bid * kWavesPerBlock + threadIdx.x / kWave; c * kWave < E; c += nwaves) {
        const int64_t e = c * kWave + lane;
        int64_t vb = 0, od = 0, id = 0;
        bool take = e < E;
        int32_t v = 0;
        if (take) {
            v = g.colidx[beg + e];
            take = !s.vmask || ((s.vmask[v >> 6] >> (v & 63)) & 1ull);  // outside the vertex mask: never entered
        }
        if (take) {
            vb = g.rowptr[v];
            od = g.rowptr[v + 1] - vb;
            id = g.directed ? g.in_rowptr[v + 1] - g.in_rowptr[v] : od;
            const uint64_t bit = 1ull << (v & 63);
            __hip_atomic_fetch_or(&s.V[v >> 6], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_or(&s.F[1][v >> 6], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            mark_dirty(s, v >> 6);
            if (s.dist) s.dist[v] = 1;
        }
        const uint64_t qm = ballot(od > 0);
        const int64_t off = wave_exclusive_sum(od);  // lists with no edges add nothing
        const int64_t at = c * s.rc + mask_rank(qm);
        if (od > 0) {
            s.qb[1][at] = vb;
            s.qoff[1][at] = off;
        }
        const int64_t esum = wave_sum(od), isum = wave_sum(id);
        const int64_t nf = __popcll(ballot(take));
        if (lane == 0) {
            cur[c].qpack = pk(__popcll(qm), esum);
            cur[c].fpack = pk(nf, isum);
            // 4 B per out-edge of the seed, 20 B (row pointers, queue entry, offset) per neighbor taken
            if (units) unit_add(units, 0, 4 * std::min<int64_t>(kWave, E - c * kWave) + 20 * nf);
        }
    }
}

// Top-down hop 1 of a hub seed, not the query's last hop: the seed alone is
// the frontier, so its out-edges are read straight from its adjacency list
// (64 per wave) with no region prefix or queue search.  Heads are claimed
// with atomicOr on their visited words (their row pointers are loaded beside
// the claim) and appended to the regions of their ids.
__device__ void hop1_push(const Graph &g, const State &s, int64_t beg, int64_t E, int64_t *units, const Part &pt) {
    const int lane = lane_id();
    const int64_t nwaves = pt.nb * kWavesPerBlock;
    const int64_t wid = pt.bid * kWavesPerBlock + threadIdx.x / kWave;
    RegRec *cur = s.regs + s.nreg;  // hop 1's slot
    uint64_t *Fn = s.F[1];
    int64_t edges = 0;
    for (int64_t e0 = wid * kWave; e0 < E; e0 += nwaves * kWave) {
        const int64_t e = e0 + lane;
        if (e < E) {
            const int32_t v = g.colidx[beg + e];
            const uint64_t bit = 1ull << (v & 63);
            const uint64_t old = atomicOr((unsigned long long *)&s.V[v >> 6], (unsigned long long)bit);
            const int64_t vb = g.rowptr[v];
            const int64_t od = g.rowptr[v + 1] - vb;
            const int64_t id = g.directed ? g.in_rowptr[v + 1] - g.in_rowptr[v] : od;
            if (!(old & bit)) {
                atomicOr((unsigned long long *)&Fn[v >> 6], (unsigned long long)bit);
                mark_dirty(s, v >> 6);
                if (s.dist) s.dist[v] = 1;
                append_one(s, cur, 1, v, vb, od, id);
            }
        }
        edges += std::min<int64_t>(kWave, E - e0);
    }
    // 4 B per out-edge of the seed
    if (units && lane == 0 && edges) unit_add(units, 0, 4 * edges);
}

// Top-down hop 1 as the query's last hop: the seed's row is tested against
// the visited bitmap (the seed and, under a vertex mask, the vertices outside
// it) and the new heads are counted.  A row holds no duplicate, so each head
// is counted once with no claim, and nothing is left for a later count.
// Without a vertex mask the visited set is the seed alone, which its row (no
// self-loop) does not hold: the count is the seed's out-degree, and the row
// is not read.
__device__ void hop1_last(PlainCtl *ctl, const Graph &g, const State &s, int64_t beg, int64_t E, int64_t *units,
                          const Part &pt) {
    const int lane = lane_id();
    const int64_t nwaves = pt.nb * kWavesPerBlock;
    const int64_t wid = pt.bid * kWavesPerBlock + threadIdx.x / kWave;
    if (!s.vmask) {
        if (wid == 0 && lane == 0) add_tail(ctl, 0, E);
        return;
    }
    int64_t found = 0, edges = 0;
    for (int64_t e0 = wid * kWave; e0 < E; e0 += nwaves * kWave) {
        const int64_t e = e0 + lane;
        bool fresh = false;
        if (e < E) {
            const int32_t v = g.colidx[beg + e];
            fresh = !((s.V[v >> 6] >> (v & 63)) & 1ull);
        }
        found += __popcll(ballot(fresh));
        edges += std::min<int64_t>(kWave, E - e0);
    }
    if (lane == 0) {
        add_tail(ctl, wid, found);
        // 4 B per out-edge of the seed and 8 B of its head's visited word
        if (units && edges) unit_add(units, 0, 12 * edges);
    }
}

// One hop of query ctl on its state s.  No validity test: an invalid seed
// leaves every region counter at zero, so each of its hops sees an empty
// frontier.  The control words are read up front, beside the region
// counters, so their loads overlap.
__device__ void hop_body(PlainCtl *ctl, int L, const Graph &g, const State &s, int light, const HeavyChunks &hc,
                         int64_t *units, const Part &pt) {
    const int t = threadIdx.x, lane = lane_id(), wv = t / kWave;
    const int64_t wid = pt.bid * kWavesPerBlock + wv;
    // wave 0 loads the previous hop's region counters (four per lane) first, so
    // that their loads are in flight with the control words'
    constexpr int kRpl = kMaxRegions / kWave;  // regions per lane
    RegRec rr[kRpl];
    if (wv == 0) {
        const RegRec *prev = s.regs + (int64_t)((L - 1) % 3) * s.nreg;
#pragma unroll
        for (int j = 0; j < kRpl; ++j) {
            const int r = lane * kRpl + j;
            rr[j] = r < s.nreg ? prev[r] : RegRec{0, 0};
        }
    }
    const int32_t k = ctl->k, dir_mode = ctl->dir_mode, alpha = ctl->alpha, beta = ctl->beta;
    const int64_t push_atomic_max = ctl->push_atomic_max;
    const HopHdr hp = ctl->hdr[(L - 1) % 3];
    const bool last = L >= k;  // the final hop only counts
    if (L + 1 < k) {
        // the slots hop l+1 writes start clear (a last hop only counts: it
        // writes no frontier word or region counter)
        RegRec *nx = s.regs + (int64_t)((L + 1) % 3) * s.nreg;
        for (int64_t i = pt.bid * kBlock + t; i < s.nreg; i += pt.nb * kBlock) {
            nx[i].qpack = 0;
            nx[i].fpack = 0;
        }
        uint64_t *Fz = s.F[(L + 1) % 3];
        for (int64_t w = pt.bid * kBlock + t; w < g.nw; w += pt.nb * kBlock) Fz[w] = 0;
    }
    if (L == 1) {
        // the same direction test as below, on the seed's degrees; when it
        // says bottom-up the general path below runs a pull
        const int64_t E = ctl->seed_od, beg = ctl->seed_beg;
        const int64_t mu = hp.mu_before - ctl->seed_id;
        const bool push = ctl->valid && (dir_mode == DIR_PUSH ||
                                         (dir_mode != DIR_PULL && (hp.dir == DIR_PUSH ? E * (int64_t)alpha <= mu
                                                                                       : (int64_t)beta < g.n)));
        if (push) {
            if (pt.bid == 0 && t == 0) {
                ctl->hdr[1].mu_before = mu;
                ctl->hdr[1].dir = DIR_PUSH;
                ctl->hdr[1].mode = MODE_PUSH_ATOMIC;
                ctl->te_acc += E;
                if (units) unit_add(units, 0, 24);
            }
            // (one region of rc >= 64 slots per 64 neighbors)
            if (last)
                hop1_last(ctl, g, s, beg, E, units, pt);
            else if (E <= (int64_t)kWave * s.nreg)
                hop1_push_free(g, s, beg, E, units, pt);
            else
                hop1_push(g, s, beg, E, units, pt);
            return;
        }
    }
    __shared__ int64_t s_epre[kMaxRegions + 1];
    __shared__ int32_t s_qcnt[kMaxRegions];
    __shared__ int64_t s_tot[3];
    __shared__ uint64_t s_mask[kWavesPerBlock][kWin];
    // wave 0 prefixes the region counters' degree sums and totals them; one
    // barrier publishes the result
    if (wv == 0) {
        int64_t q[kRpl], lq = 0, lf = 0, ld = 0;
#pragma unroll
        for (int j = 0; j < kRpl; ++j) {
            const int r = lane * kRpl + j;
            q[j] = pk_sum(rr[j].qpack);
            s_qcnt[r] = (int32_t)pk_count(rr[j].qpack);
            lf += pk_count(rr[j].fpack);
            ld += pk_sum(rr[j].fpack);
            lq += q[j];
        }
        int64_t pre = wave_exclusive_sum(lq);
#pragma unroll
        for (int j = 0; j < kRpl; ++j) {
            const int r = lane * kRpl + j;
            if (r <= s.nreg) s_epre[r] = pre;  // entry nreg gets the total
            pre += q[j];
        }
        const int64_t E = wave_sum(lq), nf = wave_sum(lf), din = wave_sum(ld);
        if (lane == 0) {
            s_tot[0] = E;
            s_tot[1] = nf;
            s_tot[2] = din;
            if (s.nreg == kMaxRegions) s_epre[kMaxRegions] = E;
        }
    }
    __syncthreads();
    const int64_t E = s_tot[0], nf = s_tot[1], din = s_tot[2];
    const int64_t mu = hp.mu_before - din;
    int dir = hp.dir;
    if (L == 1) {
        dir = DIR_PULL;  // the same test on the seed's degrees chose bottom-up above
    } else if (dir_mode == DIR_PUSH) {
        dir = DIR_PUSH;
    } else if (dir_mode == DIR_PULL) {
        dir = DIR_PULL;
    } else if (dir == DIR_PUSH) {
        if (E * (int64_t)alpha > mu) dir = DIR_PULL;
    } else {
        if (nf * (int64_t)beta < g.n) dir = DIR_PUSH;
    }
    // a top-down last hop only marks bytes (they are counted when the next
    // query starts); earlier hops claim heads atomically up to push_atomic_max
    // frontier edges
    const int mode = nf == 0 ? MODE_IDLE
                     : dir == DIR_PULL ? MODE_PULL
                     : (!last && E <= push_atomic_max ? MODE_PUSH_ATOMIC : MODE_PUSH_BYTES);
    if (pt.bid == 0 && t == 0) {
        ctl->hdr[L % 3].mu_before = mu;
        ctl->hdr[L % 3].dir = dir;
        ctl->hdr[L % 3].mode = mode;
        if (last) ctl->last_bytes = mode == MODE_PUSH_BYTES;
        if (L >= 2) ctl->count_acc += nf;
        if (nf > 0) ctl->reached = L - 1;
        if (L >= 2 && L - 1 <= ctl->level_cap) ctl->level_out[L - 2] = nf;
        ctl->te_acc += E;
        if (units) unit_add(units, 0, 16 * s.nreg);
    }
    if (mode == MODE_PULL && pt.bid == 0 && t == 0) unit_add(units, 1, 1);  // the launch's role, for profiling
    if (mode == MODE_IDLE) return;  // empty frontier: nothing left to find
    RegRec *cur = s.regs + (int64_t)(L % 3) * s.nreg;
    int64_t found = 0;  // final bottom-up hop: discoveries of this wave
    // a bottom-up hop's discovery buffers, or a top-down hop's staged queue entries
    __shared__ int64_t s_bv[kWavesPerBlock][kBufCap];
    static_assert(kBufCap >= 2 * kWin * kWave, "staged queue entries fit the buffer");
    if (mode == MODE_PULL) {
        __shared__ int32_t s_bd[kWavesPerBlock][kBufCap];
        WaveBuf wb{s_bv[wv], s_bd[wv], kBufCap, 0, -1, 0, 0};
        pull_hop(L, last, g, s, light, hc, cur, wb, &found, units, pt);
        found = shfl64(found, 0);
    } else {
        push_hop(L, mode, !last || last_marks_summary(g), E, s_epre, s_qcnt, g, s, cur, s_mask[wv], s_bv[wv], units,
                 pt);
    }
    if (last && lane == 0) add_tail(ctl, wid, found);
}

// The work of a step launch besides its hops: the byte marks that a finished
// query's last hop left are counted, the count of the query before it is
// written, and the next query is set up (its record, and its state's bitmaps
// reset).  The marks' state may be the one reset: each word is counted before
// it is reset, by the same thread.
struct StepBook {
    PlainCtl *ctl_marks;  // the query whose marks are counted (null: none)
    PlainCtl *ctl_fin;    // the query whose count is written (null: none)
    PlainCtl *ctl_setup;  // the record set up for query qn (never ctl_fin's slot)
    int64_t qn;           // next query, -1 if none
    const int32_t *seeds;
    int64_t *out_count;
    int64_t *out_te;
    int64_t push_atomic_max;
    int64_t nnz_in;
    int32_t k, dir_mode, alpha, beta;
};

// The states of a step launch's two hop pieces, in one argument: the kernel
// indexes it by piece, so that the hop's code is inlined once (two call sites
// doubled the kernel's code and its spilled scalar registers, and a step took
// about 0.2 µs longer).
struct HopStates {
    State s[2];  // the last hop's query, the hop-1 query
};

// One step of the query pipeline, three pieces of work in one launch, each on
// blocks of its own: the last hop (hop k) of the previous query (nb_last
// blocks, ctl_last on state hs.s[0]), hop 1 of the current query (nb_h1
// blocks, ctl_h1 on state hs.s[1]), and the bookkeeping of bk on the remaining blocks
// (marks of state sm, reset of state sr).  The pieces share no memory but the
// profiling counters, so the second query's hop 1 overlaps the first's last
// hop.  Every hand-off between them happens at the launch boundary.
__global__ void __launch_bounds__(kBlock) plain_step_kernel(PlainCtl *ctl_last, int64_t nb_last, PlainCtl *ctl_h1,
                                                           int64_t nb_h1, HopStates hs, StepBook bk, State sm,
                                                           State sr, Graph g, int light, HeavyChunks hc,
                                                           int64_t *units) {
    const int64_t b = blockIdx.x;
    if (b < nb_last + nb_h1) {
        const int r = b < nb_last ? 0 : 1;
        hop_body(r == 0 ? ctl_last : ctl_h1, r == 0 ? bk.k : 1, g, hs.s[r], light, hc, units,
                 r == 0 ? Part{b, nb_last} : Part{b - nb_last, nb_h1});
        return;
    }
    // the bookkeeping blocks: the word sweep, then one block that writes the
    // finished count and one that sets up the next query (their control
    // slots differ, and neither touches what the sweep reads or writes)
    const int64_t nbk = (int64_t)gridDim.x - nb_last - nb_h1, bb = b - nb_last - nb_h1;
    const int t = threadIdx.x;
    if (bb == nbk - 2) {
        if (bk.ctl_fin && t < kWave) finalize(bk.ctl_fin);
        return;
    }
    const int32_t nseed = bk.qn >= 0 ? bk.seeds[bk.qn] : -1;
    if (bb == nbk - 1) {
        if (bk.qn >= 0)
            setup_query(bk.ctl_setup, g, sr, nseed, bk.qn, bk.k, bk.dir_mode, bk.alpha, bk.beta, bk.push_atomic_max,
                        bk.nnz_in, bk.out_count, bk.out_te, units);
        return;
    }
    const Part pt{bb, nbk - 2};
    const bool marks = bk.ctl_marks && bk.ctl_marks->last_bytes;  // not written in this launch
    const bool nvalid = nseed >= 0 && (int64_t)nseed < g.n;
    const int64_t nsw = nvalid ? (nseed >> 6) : -1;
    const uint64_t nsbit = nvalid ? (1ull << (nseed & 63)) : 0;
    int64_t fresh = 0, flagged = 0, rewritten = 0;
    const bool summary = last_marks_summary(g);
    // each wave takes whole 64-word blocks (kBlock is a multiple of 64)
    for (int64_t w = pt.bid * kBlock + t; w < g.nw; w += pt.nb * kBlock) {
        if (marks && (!summary || sm.nsum[w])) {
            bool had;
            fresh += close_marks_word(sm, w, sm.V[w], had);
            flagged += had;
        }
        if (bk.qn >= 0) {
            // only the blocks the state's last query set bits in, and the new seed's
            const bool stale = !sr.dirty || sr.vmask || sr.dirty[w >> 6] || (nsw >= 0 && (w >> 6) == (nsw >> 6));
            if (stale) {
                reset_word(sr, g, w, nsw, nsbit);
                ++rewritten;
            }
            reset_dirty(sr, w, nsw);
        }
    }
    if (units && bk.qn >= 0) {
        // 24 B per rewritten word of V, F[0] and F[1]; the block flags once
        rewritten = wave_sum(rewritten);
        if (lane_id() == 0) unit_add(units, 0, 24 * rewritten);
        if (pt.bid == 0 && t == 0 && sr.dirty) unit_add(units, 0, (g.nw + 63) / 64);
    }
    if (marks) {
        fresh = wave_sum(fresh);
        flagged = wave_sum(flagged);
        if (lane_id() == 0) add_tail(bk.ctl_marks, pt.bid * kWavesPerBlock + t / kWave, fresh);
        // the summary bytes, then the marks and visited word of each flagged word
        if (lane_id() == 0) unit_add(units, 0, 72 * flagged);
        if (pt.bid == 0 && t == 0) unit_add(units, 0, summary ? g.nw : 64 * g.nw);
    }
}

__global__ void __launch_bounds__(kBlock) plain_hop_kernel(PlainCtl *ctl, int L, Graph g, State s, int light,
                                                          HeavyChunks hc, int64_t *units) {
    hop_body(ctl, L, g, s, light, hc, units, Part{(int64_t)blockIdx.x, (int64_t)gridDim.x});
}

// After a byte-mode push: ballot(mark AND NOT visited) per 64-vertex word is
// the word's new frontier bits; visited |= them, marks cleared, and the word's
// discoveries appended to its region's queue.  Each wave takes a contiguous
// run of words: their summary bytes in one load (one word per lane), then the
// marked words four at a time, whose marks and visited words are loaded
// together, then the row pointers of all their new vertices together.  The
// grid is what the device holds at once (its small discovery buffers let
// eight blocks share a compute unit), so every wave works from the start.
constexpr int kCompactBuf = 256;
__global__ void __launch_bounds__(kBlock) plain_compact_kernel(const PlainCtl *ctl, int L, Graph g, State s,
                                                              int64_t *units) {
    if (!ctl->valid || ctl->hdr[L % 3].mode != MODE_PUSH_BYTES) return;
    const int lane = lane_id();
    uint64_t *Fn = s.F[L % 3];
    RegRec *cur = s.regs + (int64_t)(L % 3) * s.nreg;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t wid = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (units && wid == 0 && lane == 0) unit_add(units, 0, g.nw);  // the summary bytes
    __shared__ int64_t s_bv[kWavesPerBlock][kCompactBuf];
    __shared__ int32_t s_bd[kWavesPerBlock][kCompactBuf];
    const int wv = threadIdx.x / kWave;
    WaveBuf wb{s_bv[wv], s_bd[wv], kCompactBuf, 0, -1, 0, 0};
    const int64_t wpw = (g.nw + nwaves - 1) / nwaves;
    const int64_t wb0 = std::min(wid * wpw, g.nw), wb1 = std::min(wb0 + wpw, g.nw);
    int64_t found_total = 0;
    for (int64_t c0 = wb0; c0 < wb1; c0 += kWave) {
        const int64_t wl = c0 + lane;
        const bool flagged = wl < wb1 && s.nsum[wl];
        uint64_t pend = ballot(flagged);
        if (flagged) s.nsum[wl] = 0;
        // the word's marks, visited and frontier words
        if (lane == 0 && pend) unit_add(units, 0, 80 * (int64_t)__popcll(pend));
        while (pend) {
            int64_t w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                w[i] = pend ? c0 + __builtin_ctzll(pend) : -1;
                pend &= pend - 1;
            }
            uint8_t nb[4];
            uint64_t vis[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t v = w[i] * kWave + lane;
                nb[i] = (w[i] >= 0 && v < g.n) ? s.nextb[v] : 0;
                vis[i] = w[i] >= 0 ? s.V[w[i]] : ~0ull;
            }
            bool fresh[4];
            int64_t vb[4], od[4], id[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t v = w[i] * kWave + lane;
                fresh[i] = nb[i] && !((vis[i] >> lane) & 1ull);
                vb[i] = 0;
                od[i] = 0;
                id[i] = 0;
                if (fresh[i]) {
                    vb[i] = g.rowptr[v];
                    od[i] = g.rowptr[v + 1];
                    id[i] = g.directed ? g.in_rowptr[v + 1] - g.in_rowptr[v] : 0;
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (w[i] < 0) break;  // uniform
                const int64_t v = w[i] * kWave + lane;
                const uint64_t m = ballot(fresh[i]);
                if (nb[i]) s.nextb[v] = 0;
                if (fresh[i] && s.dist) s.dist[v] = L;
                if (lane == 0 && m) {
                    s.V[w[i]] = vis[i] | m;
                    Fn[w[i]] = m;
                    mark_dirty(s, w[i]);
                }
                const int64_t d = od[i] - vb[i];
                wb_word(wb, s, cur, L, w[i], fresh[i], vb[i], d, g.directed ? id[i] : d);
                found_total += __popcll(m);
            }
        }
    }
    wb_flush(wb, s, cur, L);
    if (lane == 0) unit_add(units, 0, 16 * found_total);
}

// ------------------------------------------------------------------ breadth-first search to the end

// The hop kernels above, with no hop marked last, are a level-synchronous
// breadth-first search; with s.dist set, every vertex found at hop l gets
// distance l, written once by the wave or lane whose claim (atomicOr on its
// visited word, or the ballot of a word's fresh bits) found it.

// Set-up: the distance vector when there is one (0 at the seed, -1
// elsewhere), the level sizes when asked for (zero), the visited and frontier
// bitmaps, and the control record with no last hop.
__global__ void __launch_bounds__(kBlock) plain_bfs_init_kernel(PlainCtl *ctl, Graph g, State s, int32_t seed,
                                                               int64_t *levels, int64_t level_cap, int dir_mode,
                                                               int alpha, int beta, int64_t push_atomic_max,
                                                               int64_t nnz_in, int64_t *units) {
    const int64_t sw = seed >> 6;
    const uint64_t sbit = 1ull << (seed & 63);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int64_t w = t0; w < g.nw; w += stride) {
        reset_word(s, g, w, sw, sbit);
        reset_dirty(s, w, sw);
    }
    if (s.dist)
        for (int64_t v = t0; v < g.n; v += stride) s.dist[v] = v == seed ? 0 : -1;
    if (levels)
        for (int64_t l = t0; l < level_cap; l += stride) levels[l] = 0;
    if (blockIdx.x == 0) {
        setup_query(ctl, g, s, seed, 0, INT32_MAX, dir_mode, alpha, beta, push_atomic_max, nnz_in, nullptr, nullptr,
                    units);
        if (threadIdx.x == 0) {
            ctl->level_out = levels;
            ctl->level_cap = levels ? level_cap : 0;
            if (units && s.dist) unit_add(units, 0, 4 * g.n);
            unit_add(units, 0, 3 * 8 * g.nw);  // every word of V, F[0] and F[1]
        }
    }
}

// After hop L (one wave): whether level L is non-empty (ctl->more), the
// largest non-empty level (ctl->reached), and into the outputs given, the
// count of levels 1..L, that level, and the out-degree sum of levels 0..L-1
// (the traversed edges of a search of depth L).  Level L's region counters
// stay intact until hop L+2 clears them.  A query with an invalid seed
// already holds -1 in its outputs and is left alone.
__global__ void __launch_bounds__(kWave) plain_bfs_probe_kernel(PlainCtl *ctl, State s, int L, int64_t *out_count,
                                                               int32_t *out_depth, int64_t *out_te) {
    const int lane = lane_id();
    const RegRec *lv = s.regs + (int64_t)(L % 3) * s.nreg;
    int64_t nf = 0;
    for (int r = lane; r < s.nreg; r += kWave) nf += pk_count(lv[r].fpack);
    nf = wave_sum(nf);
    if (lane != 0) return;
    if (L == 0) nf = 0;  // level 0 is the seed, never counted
    const int32_t depth = nf > 0 ? L : ctl->reached;
    ctl->reached = depth;
    ctl->more = nf > 0;
    if (L >= 1 && L <= ctl->level_cap) ctl->level_out[L - 1] = nf;
    if (!ctl->valid) return;
    if (out_count) *out_count = ctl->count_acc + nf;
    if (out_depth) *out_depth = depth;
    if (out_te) *out_te = ctl->te_acc;
}

// ------------------------------------------------------------------ the neighborhood as vertex ids

// After a search with no last hop, the visited bitmap is {v : dist <= depth};
// without the seed's bit it is the k-hop neighborhood.  Three launches turn it
// into ascending vertex ids: per-block popcounts of kBlock words, one block
// scanning those into offsets, and a write in which each wave takes 64 words,
// one at a time, and its lanes store the word's ids side by side.
__device__ __forceinline__ uint64_t set_word(const uint64_t *V, int64_t w, int32_t seed) {
    const uint64_t m = V[w];
    return w == (seed >> 6) ? m & ~(1ull << (seed & 63)) : m;
}

__device__ __forceinline__ int64_t block_exclusive_sum(int64_t v, int64_t *lds_waves, int64_t *total) {
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    const int64_t x = wave_exclusive_sum(v);
    if (lane == kWave - 1) lds_waves[wv] = x + v;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
        const int64_t t = lds_waves[i];
        if (i < wv) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + x;
}

__global__ void __launch_bounds__(kBlock) plain_set_count_kernel(const uint64_t *V, int64_t nw, int32_t seed,
                                                                int64_t *partial) {
    __shared__ int64_t s_w[kWavesPerBlock];
    const int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t pc = w < nw ? __popcll(set_word(V, w, seed)) : 0;
    int64_t total = 0;
    block_exclusive_sum(pc, s_w, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// One block: exclusive prefix of the nb block counts in place, the total to *count.
__global__ void __launch_bounds__(kBlock) plain_set_scan_kernel(int64_t *partial, int64_t nb, int64_t *count) {
    __shared__ int64_t s_w[kWavesPerBlock];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < nb ? partial[b] : 0;
        int64_t total = 0;
        const int64_t x = block_exclusive_sum(v, s_w, &total);
        if (b < nb) partial[b] = carry + x;
        carry += total;
    }
    if (threadIdx.x == 0 && count) *count = carry;
}

__global__ void __launch_bounds__(kBlock) plain_set_write_kernel(const uint64_t *V, int64_t nw, int32_t seed,
                                                                const int64_t *offsets, int32_t *ids, int64_t cap,
                                                                int64_t *units) {
    __shared__ int64_t s_w[kWavesPerBlock];
    const int lane = lane_id();
    const int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t m = w < nw ? set_word(V, w, seed) : 0;
    int64_t total = 0;
    const int64_t pos = offsets[blockIdx.x] + block_exclusive_sum(__popcll(m), s_w, &total);
    const int64_t w0 = w - lane;  // the wave's first word
    for (int j = 0; j < kWave; ++j) {
        const uint64_t mj = (uint64_t)shfl64((int64_t)m, j);
        const int64_t pj = shfl64(pos, j);
        if (!mj || pj >= cap) continue;  // wave-uniform
        if ((mj >> lane) & 1ull) {
            const int64_t at = pj + __popcll(mj & ((1ull << lane) - 1));
            if (at < cap) ids[at] = (int32_t)((w0 + j) * kWave + lane);
        }
    }
    if (units) {
        // 4 B per id written
        const int64_t written = wave_sum(std::min<int64_t>(pos + __popcll(m), cap) - std::min(pos, cap));
        if (lane == 0) unit_add(units, 0, 4 * written);
    }
}

__global__ void fill_kernel(int64_t *a, int64_t *b, int64_t n, int64_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a[i] = value;
        if (b) b[i] = value;
    }
}

}  // namespace

// Bitmap states, control slots and queue sets rotate over consecutive
// queries as plain_plan.h lays out: a step launch works on the last hop of
// query q-1 and hop 1 of query q, counts the marks of an earlier query and
// resets the state of query q+1.  Queues are needed only by the two queries
// with hops in flight, so two sets suffice.
constexpr int kStates = kPlanStates;
constexpr int kSlots = kPlanSlots;
static_assert(kPlanQueueSets == 2, "queue sets rotate by query parity");

struct PlainCtx {
    khop_graph *g = nullptr;
    PlainCtl *ctl = nullptr;  // kSlots control slots
    State s[kStates]{};       // bitmaps, byte maps and region counters of each state
    int64_t *qb[2][2]{};      // queue sets by query parity, each by hop parity
    int64_t *qoff[2][2]{};
    int init_grid = 1;
    int64_t *set_partial = nullptr;  // block counts, then offsets, of the neighborhood-set kernels
    int64_t set_blocks = 0;
    void *arena = nullptr;
    int32_t *h_flags = nullptr;  // pinned: a deep query's reached level and frontier-nonempty flag
    // A context in the no-allocation scratch: its runs are not profiled (that
    // creates events) and take the chunk table the graph already has instead
    // of building one for a changed threshold.
    bool fixed = false;
    // Launch sequences captured as HIP graphs, replayed when a run repeats
    // one (same pointers, sizes and settings; the inputs' contents may differ).
    struct Captured {
        const int32_t *seeds = nullptr;
        int64_t num = 0;
        int32_t k = 0;
        int64_t *counts = nullptr, *te = nullptr;
        const uint64_t *vmask = nullptr;
        Params P{};
        const int32_t *hvert = nullptr;
        int heavy = -1;
        hipGraphExec_t exec = nullptr;  // null: seen once, not captured yet
        bool failed = false;            // capture did not succeed: always launch directly
        uint64_t used = 0;
    };
    std::vector<Captured> captured;
    uint64_t clock = 0;
    bool graphs = true;                 // replay repeated runs from captured graphs
    hipStream_t cap_stream = nullptr;   // the stream runs are captured on
};

namespace {

// The state query q runs on: bitmaps of state q % 3, queues of set q % 2.
State query_state(const PlainCtx *c, int64_t q, const uint64_t *vmask, int32_t *dist) {
    State x = c->s[q % kStates];
    for (int i = 0; i < 2; ++i) {
        x.qb[i] = c->qb[q & 1][i];
        x.qoff[i] = c->qoff[q & 1][i];
    }
    x.vmask = vmask;
    x.dist = dist;
    return x;
}

PlainCtl *query_slot(const PlainCtx *c, int64_t q) { return c->ctl + q % kSlots; }

// Blocks of the hop and compaction launches: plain_grid per compute unit,
// and no more than the bitmap has 8 (hop) or 16 (compaction) words per block.
struct Grids {
    int hop, compact;
};
Grids grids(const khop_graph *g, const Params &P) {
    const int64_t nw = (g->n + 63) / 64, cap = (int64_t)g->cu_count * P.plain_grid;
    // compaction: eight words per wave, up to eight blocks per compute unit
    return Grids{(int)std::max<int64_t>(1, std::min<int64_t>((nw + 7) / 8, cap)),
                 (int)std::max<int64_t>(1, std::min<int64_t>((nw + 31) / 32, (int64_t)g->cu_count * 8))};
}

}  // namespace

// The layout of a query context in one device allocation: the total bytes,
// and when base is not null, every pointer of c set into it.
static size_t plain_layout(const khop_graph *g, PlainCtx *c, char *base) {
    const int64_t n = g->n, nw = (n + 63) / 64;
    const int nreg = (int)std::min<int64_t>(kMaxRegions, nw);
    const int rw = (int)((nw + nreg - 1) / nreg);
    const int64_t rc = (int64_t)rw * kWave;
    const int64_t slots = (int64_t)nreg * rc;  // >= n
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_ctl = off;
    off += al(kSlots * sizeof(PlainCtl));
    size_t o_V[kStates], o_F[kStates][3], o_regs[kStates], o_nb[kStates], o_ns[kStates], o_dirty[kStates];
    for (int p = 0; p < kStates; ++p) {
        o_nb[p] = off;
        off += al(nw * 64);  // the byte map, padded to whole words
        o_ns[p] = off;
        off += al(nw);
        o_dirty[p] = off;
        off += al((nw + 63) / 64);
        o_V[p] = off;
        off += al(nw * 8);
        for (int i = 0; i < 3; ++i) {
            o_F[p][i] = off;
            off += al(nw * 8);
        }
        o_regs[p] = off;
        off += al((size_t)3 * nreg * sizeof(RegRec));
    }
    const int64_t set_blocks = (nw + kBlock - 1) / kBlock;
    const size_t o_part = off;
    off += al((size_t)set_blocks * 8);
    size_t o_q[2][2], o_qoff[2][2];
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i) {
            o_q[j][i] = off;
            off += al(slots * 8);
            o_qoff[j][i] = off;
            off += al(slots * 8);
        }
    if (!base) return off;
    c->g = const_cast<khop_graph *>(g);
    c->arena = base;
    c->ctl = (PlainCtl *)(base + o_ctl);
    c->set_partial = (int64_t *)(base + o_part);
    c->set_blocks = set_blocks;
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i) {
            c->qb[j][i] = (int64_t *)(base + o_q[j][i]);
            c->qoff[j][i] = (int64_t *)(base + o_qoff[j][i]);
        }
    for (int p = 0; p < kStates; ++p) {
        State &st = c->s[p];
        st.V = (uint64_t *)(base + o_V[p]);
        for (int i = 0; i < 3; ++i) st.F[i] = (uint64_t *)(base + o_F[p][i]);
        st.regs = (RegRec *)(base + o_regs[p]);
        st.nextb = (uint8_t *)(base + o_nb[p]);
        st.nsum = (uint8_t *)(base + o_ns[p]);
        st.dirty = (uint8_t *)(base + o_dirty[p]);
        st.nreg = nreg;
        st.rw = rw;
        st.rc = rc;
    }
    c->init_grid = (int)std::max<int64_t>(1, std::min<int64_t>((nw + kBlock - 1) / kBlock, 512));
    return off;
}

PlainCtx *plain_ctx_create(khop_graph *g) {
    PlainCtx *c = new PlainCtx();
    const size_t bytes = plain_layout(g, c, nullptr);
    void *arena = nullptr;
    if (hipMalloc(&arena, bytes) != hipSuccess) {
        delete c;
        (void)hipGetLastError();
        fail(KHOP_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes for a query context failed");
    }
    plain_layout(g, c, (char *)arena);
    if (hipHostMalloc((void **)&c->h_flags, 2 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(arena);
        delete c;
        fail(KHOP_ENOMEM, "pinned host allocation for a query context failed");
    }
    KHOP_HIP(hipMemset(arena, 0, bytes));
    KHOP_HIP(hipDeviceSynchronize());
    return c;
}

void plain_ctx_set_graphs(PlainCtx *c, bool on) { c->graphs = on; }

void plain_ctx_destroy(PlainCtx *c) {
    if (!c) return;
    for (auto &e : c->captured)
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->arena) (void)hipFree(c->arena);
    if (c->h_flags) (void)hipHostFree(c->h_flags);
    delete c;
}

void plain_fill_zero_outputs(int64_t *d_counts, int64_t *d_te, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, st, d_counts, d_te, n, (int64_t)0);
    KHOP_HIP(hipGetLastError());
}

// Hops a query of the pipelined path may have.  A deeper k (a request to
// count everything within reach, in effect) runs its queries one at a time as
// searches with no last hop, launched in groups, with a host check between
// groups that ends the query once its frontier is empty: past its seed's
// eccentricity every further hop would find nothing.
constexpr int kDeepHops = 32;

static void plain_deep(khop_graph *g, PlainCtx *c, const Params &P, const Graph &gr, const HeavyChunks &hc,
                       const Grids &gd, const int32_t *d_seeds, int64_t num_seeds, int64_t k, int64_t *d_counts,
                       int64_t *d_te, hipStream_t st, const uint64_t *d_vmask) {
    const int64_t pam = (int64_t)P.push_atomic_max;
    const int hop1_grid = P.dir_mode == KHOP_DIR_PULL ? gd.hop : std::max(c->init_grid, g->cu_count / 4);
    const State s = query_state(c, 0, d_vmask, nullptr);
    PlainCtl *ctl = query_slot(c, 0);
    for (int64_t i = 0; i < num_seeds; ++i) {
        {
            ProfScope ps(g, KK_PLAIN_INIT, st);
            hipLaunchKernelGGL(plain_init_kernel, dim3(c->init_grid), dim3(kBlock), 0, st, ctl, gr, s, d_seeds, i,
                               (int)INT32_MAX, P.dir_mode, P.alpha, P.beta, pam, g->nnz, d_counts, d_te, ps.units());
            ps.end(0, 1);
        }
        int64_t H = 0;  // hops launched
        int64_t group = std::max(2, g->bfs_hops_hint.load(std::memory_order_relaxed));
        while (H < k) {
            const int64_t upto = std::min(k, H + group);
            for (int64_t L = H + 1; L <= upto; ++L) {
                ProfScope ps(g, L == 1 ? KK_PLAIN_STEP : KK_PLAIN_HOP_PUSH, st);
                if (L == 1) {
                    const StepBook bk{nullptr, nullptr, nullptr, -1, nullptr, nullptr, nullptr, pam, g->nnz,
                                      INT32_MAX, (int32_t)P.dir_mode, (int32_t)P.alpha, (int32_t)P.beta};
                    hipLaunchKernelGGL(plain_step_kernel, dim3(hop1_grid), dim3(kBlock), 0, st, (PlainCtl *)nullptr,
                                       (int64_t)0, ctl, (int64_t)hop1_grid, HopStates{{State{}, s}}, bk, State{},
                                       State{}, gr, P.pull_light, hc, ps.units());
                    ps.end(0, 1);
                    continue;
                }
                hipLaunchKernelGGL(plain_hop_kernel, dim3(gd.hop), dim3(kBlock), 0, st, ctl, (int)L, gr, s,
                                   P.pull_light, hc, ps.units());
                ps.end_split(0, 1, KK_PLAIN_HOP_PULL, 1);
                ProfScope pc(g, KK_PLAIN_COMPACT, st);
                hipLaunchKernelGGL(plain_compact_kernel, dim3(gd.compact), dim3(kBlock), 0, st, ctl, (int)L, gr, s,
                                   pc.units());
                pc.end(0, 1);
            }
            H = upto;
            if (H >= k) break;
            hipLaunchKernelGGL(plain_bfs_probe_kernel, dim3(1), dim3(kWave), 0, st, ctl, s, (int)H,
                               (int64_t *)nullptr, (int32_t *)nullptr, (int64_t *)nullptr);
            // reached and more are adjacent in the control record
            KHOP_HIP(hipMemcpyAsync(c->h_flags, &ctl->reached, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipStreamSynchronize(st));
            if (!c->h_flags[1]) {
                if (c->h_flags[0] > 0) g->bfs_hops_hint.store(c->h_flags[0] + 1, std::memory_order_relaxed);
                break;
            }
            group = std::min<int64_t>(2 * group, 1024);
        }
        // the count of levels 1..H and the out-degree sum of levels 0..H-1: the
        // query's answer, since any level past H is empty (or H = k)
        hipLaunchKernelGGL(plain_bfs_probe_kernel, dim3(1), dim3(kWave), 0, st, ctl, s, (int)H, d_counts + i,
                           (int32_t *)nullptr, d_te ? d_te + i : (int64_t *)nullptr);
    }
    KHOP_HIP(hipGetLastError());
}

// The launches of a run of queries (k >= 1) with the settings P and chunk table ht.
static void plain_launch(khop_graph *g, PlainCtx *c, const Params &P, const HeavyTable &ht, khop_graph *pg,
                         const int32_t *d_seeds, int64_t num_seeds, int32_t k, int64_t *d_counts, int64_t *d_te,
                         hipStream_t st, const uint64_t *d_vmask) {
    const Grids gd = grids(g, P);
    Graph gr{g->d_rowptr, g->d_colidx, g->d_in_rowptr, g->d_in_colidx, g->n, (g->n + 63) / 64, g->directed,
             ht.threshold, g->d_probe};
    HeavyChunks hc{ht.d_vert, ht.d_begin, ht.d_end, ht.n};
    if (k > kDeepHops) {
        // no search goes deeper than n - 1 hops: a larger k counts the same
        plain_deep(g, c, P, gr, hc, gd, d_seeds, num_seeds, std::min<int64_t>(k, g->n), d_counts, d_te, st, d_vmask);
        return;
    }
    if (k == 1 && !d_vmask && P.dir_mode == KHOP_DIR_AUTO) {
        // one-hop queries, each one launch that reads its seed's degree (a
        // forced direction runs the hop itself)
        for (int64_t i = 0; i < num_seeds; ++i) {
            ProfScope ps(pg, KK_PLAIN_DEGREE, st);
            hipLaunchKernelGGL(plain_degree_kernel, dim3(1), dim3(kWave), 0, st, d_seeds, i, g->d_rowptr, g->n,
                               d_counts, d_te);
            ps.end(4.0 + 16.0 + 8.0 * (d_te ? 2 : 1));
        }
        KHOP_HIP(hipGetLastError());
        return;
    }
    if (!P.plain_pipeline && num_seeds > 1) {
        // one query at a time: each a pipeline of one query, its own launch sequence
        for (int64_t i = 0; i < num_seeds; ++i)
            plain_launch(g, c, P, ht, pg, d_seeds + i, 1, k, d_counts + i, d_te ? d_te + i : nullptr, st, d_vmask);
        return;
    }
    const int64_t nnz_in = g->nnz;
    const int64_t pam = (int64_t)P.push_atomic_max;
    // hop 1 starts from the seed alone (top-down unless forced): the set-up
    // grid suffices
    const int h1_grid = P.dir_mode == KHOP_DIR_PULL ? gd.hop : std::max(c->init_grid, g->cu_count / 4);
    auto state = [&](int64_t q) { return query_state(c, q, d_vmask, nullptr); };
    auto slot = [&](int64_t q) { return query_slot(c, q); };
    {
        ProfScope ps(pg, KK_PLAIN_INIT, st);
        hipLaunchKernelGGL(plain_init_kernel, dim3(c->init_grid), dim3(kBlock), 0, st, slot(0), gr, state(0),
                           d_seeds, (int64_t)0, (int)k, P.dir_mode, P.alpha, P.beta, pam, nnz_in, d_counts, d_te,
                           ps.units());
        ps.end(0, 1);
    }
    // Step j runs the last hop of query j-1 (when k >= 2) beside hop 1 of
    // query j; hops 2..k-1 of query j follow it (plain_plan.h).
    const int64_t m = num_seeds;
    const int64_t nsteps = plain_plan_steps(k, m);
    for (int64_t j = 0; j < nsteps; ++j) {
        const PlainStep ps_j = plain_plan_step(k, m, j);
        const int64_t qm = ps_j.marks, qn = ps_j.setup;
        const StepBook bk{qm >= 0 ? slot(qm) : nullptr, ps_j.fin >= 0 ? slot(ps_j.fin) : nullptr,
                          qn >= 0 ? slot(qn) : nullptr, qn, d_seeds, d_counts, d_te, pam, nnz_in, (int32_t)k,
                          (int32_t)P.dir_mode, (int32_t)P.alpha, (int32_t)P.beta};
        // a k = 2 query's last hop expands only its seed's neighbors' rows:
        // two blocks per compute unit carry it with less per-block work
        // (dispatch, region prefix) than the hop grid
        const int64_t last_grid = k == 2 ? std::min<int64_t>(gd.hop, 2 * (int64_t)g->cu_count) : gd.hop;
        const int64_t nb_last = ps_j.last >= 0 ? last_grid : 0, nb_h1 = ps_j.h1 >= 0 ? h1_grid : 0;
        // the word sweep's blocks, then the count's and the set-up's
        const int64_t nb_book = (qm >= 0 || qn >= 0) ? c->init_grid + 2 : 0;
        {
            ProfScope ps(pg, KK_PLAIN_STEP, st);
            hipLaunchKernelGGL(plain_step_kernel, dim3((unsigned)(nb_last + nb_h1 + nb_book)), dim3(kBlock), 0, st,
                               ps_j.last >= 0 ? slot(ps_j.last) : nullptr, nb_last,
                               ps_j.h1 >= 0 ? slot(ps_j.h1) : nullptr, nb_h1,
                               HopStates{{ps_j.last >= 0 ? state(ps_j.last) : State{},
                                          ps_j.h1 >= 0 ? state(ps_j.h1) : State{}}},
                               bk, qm >= 0 ? state(qm) : State{}, qn >= 0 ? state(qn) : State{}, gr,
                               P.pull_light, hc, ps.units());
            ps.end(0, 1);
        }
        if (ps_j.h1 < 0) continue;
        PlainCtl *cq = slot(ps_j.h1);
        const State sq = state(ps_j.h1);
        for (int L = 2; L < k; ++L) {
            {
                ProfScope ps(pg, KK_PLAIN_HOP_PUSH, st);
                hipLaunchKernelGGL(plain_hop_kernel, dim3(gd.hop), dim3(kBlock), 0, st, cq, L, gr, sq,
                                   P.pull_light, hc, ps.units());
                ps.end_split(0, 1, KK_PLAIN_HOP_PULL, 1);
            }
            ProfScope ps(pg, KK_PLAIN_COMPACT, st);
            hipLaunchKernelGGL(plain_compact_kernel, dim3(gd.compact), dim3(kBlock), 0, st, cq, L, gr, sq,
                               ps.units());
            ps.end(0, 1);
        }
    }
    // the last query's marks and the count of the one before it, then the last
    // count.  A run of k = 1 leaves no marks (its only hop counts as it goes),
    // so its last two counts are both written by the final launch.
    const PlainStep cl = plain_plan_close(m);
    if (k >= 2) {
        ProfScope ps(pg, KK_PLAIN_INIT, st);
        hipLaunchKernelGGL(plain_close_kernel, dim3(c->init_grid), dim3(kBlock), 0, st, slot(cl.marks),
                           cl.fin >= 0 ? slot(cl.fin) : nullptr, (int)(cl.fin >= 0), gr, state(cl.marks),
                           ps.units());
        ps.end(0, 1);
    }
    hipLaunchKernelGGL(plain_final_kernel, dim3(1), dim3(2 * kWave), 0, st, slot(m - 1),
                       k < 2 && cl.fin >= 0 ? slot(cl.fin) : nullptr);
    KHOP_HIP(hipGetLastError());
}

// Whether two settings give the same launches.
static bool same_params(const Params &a, const Params &b) {
    return a.dir_mode == b.dir_mode && a.alpha == b.alpha && a.beta == b.beta && a.pull_light == b.pull_light &&
           a.pull_heavy == b.pull_heavy && a.push_atomic_max == b.push_atomic_max && a.plain_grid == b.plain_grid &&
           a.plain_pipeline == b.plain_pipeline;
}

void plain_run(khop_graph *g, PlainCtx *c, const int32_t *d_seeds, int64_t num_seeds, int32_t k, int64_t *d_counts,
               int64_t *d_te, hipStream_t st, const uint64_t *d_vmask) {
    if (num_seeds <= 0) return;
    if (k == 0) {
        plain_fill_zero_outputs(d_counts, d_te, num_seeds, st);
        return;
    }
    const Params P = params_of(g);
    const HeavyTable ht = c->fixed ? plain_heavy_table_current(g) : plain_heavy_table(g, P.pull_heavy);
    khop_graph *const pg = c->fixed ? nullptr : g;  // profiled launches (none for a fixed context)
    // With the graph option, a run that repeats an earlier one (the same
    // pointers, sizes and settings) replays the launch sequence captured the
    // second time it was seen, as one HIP graph: the host's work per launch
    // is what bounds a k = 1 query, but a graph launch costs more than that
    // saves unless the run is long.  Profiled runs (their launches are
    // bracketed by events), runs on the no-allocation scratch and deep runs
    // (host checks between hop groups) always launch directly.
    const bool capturable = c->graphs && P.plain_graphs && !c->fixed && k <= kDeepHops && !g->prof.on;
    if (!capturable) {
        plain_launch(g, c, P, ht, pg, d_seeds, num_seeds, k, d_counts, d_te, st, d_vmask);
        return;
    }
    constexpr size_t kMaxCaptured = 8, kMaxSeen = 64;
    PlainCtx::Captured *e = nullptr;
    for (auto &x : c->captured)
        if (x.seeds == d_seeds && x.num == num_seeds && x.k == k && x.counts == d_counts && x.te == d_te &&
            x.vmask == d_vmask && x.hvert == ht.d_vert && x.heavy == ht.threshold && same_params(x.P, P)) {
            e = &x;
            break;
        }
    if (!e) {
        // first sight: launch directly and remember the run (a full list
        // forgets its oldest run that holds no graph)
        if (c->captured.size() >= kMaxSeen) {
            auto old = c->captured.end();
            for (auto it = c->captured.begin(); it != c->captured.end(); ++it)
                if (!it->exec && (old == c->captured.end() || it->used < old->used)) old = it;
            if (old != c->captured.end()) c->captured.erase(old);
        }
        if (c->captured.size() < kMaxSeen) {
            PlainCtx::Captured n;
            n.seeds = d_seeds;
            n.num = num_seeds;
            n.k = k;
            n.counts = d_counts;
            n.te = d_te;
            n.vmask = d_vmask;
            n.P = P;
            n.hvert = ht.d_vert;
            n.heavy = ht.threshold;
            n.used = ++c->clock;
            c->captured.push_back(n);
        }
        plain_launch(g, c, P, ht, pg, d_seeds, num_seeds, k, d_counts, d_te, st, d_vmask);
        return;
    }
    e->used = ++c->clock;
    if (!e->exec && !e->failed) {
        size_t held = 0;
        for (const auto &x : c->captured) held += x.exec != nullptr;
        if (held >= kMaxCaptured) {
            e->failed = true;  // the context holds its share of graphs: this run launches directly
        } else {
            if (!c->cap_stream) KHOP_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            hipError_t err = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
            if (err == hipSuccess) {
                try {
                    plain_launch(g, c, P, ht, nullptr, d_seeds, num_seeds, k, d_counts, d_te, c->cap_stream,
                                 d_vmask);
                } catch (...) {
                    err = hipErrorUnknown;
                }
                const hipError_t end = hipStreamEndCapture(c->cap_stream, &graph);
                if (err == hipSuccess) err = end;
            }
            if (err == hipSuccess) err = hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (err != hipSuccess) {
                (void)hipGetLastError();
                e->exec = nullptr;
                e->failed = true;
            }
        }
    }
    if (!e->exec) {
        plain_launch(g, c, P, ht, pg, d_seeds, num_seeds, k, d_counts, d_te, st, d_vmask);
        return;
    }
    KHOP_HIP(hipGraphLaunch(e->exec, st));
}

void plain_bfs(khop_graph *g, PlainCtx *c, int32_t seed, int32_t max_depth, int32_t *d_dist, int64_t *d_count,
               int32_t *d_depth, int64_t *d_levels, int64_t level_cap, int32_t *h_flags, hipStream_t st) {
    const Params P = params_of(g);
    const HeavyTable ht = plain_heavy_table(g, P.pull_heavy);
    const Grids gd = grids(g, P);
    Graph gr{g->d_rowptr, g->d_colidx, g->d_in_rowptr, g->d_in_colidx, g->n, (g->n + 63) / 64, g->directed,
             ht.threshold, g->d_probe};
    HeavyChunks hc{ht.d_vert, ht.d_begin, ht.d_end, ht.n};
    const int64_t pam = (int64_t)P.push_atomic_max;
    const int hop1_grid = P.dir_mode == KHOP_DIR_PULL ? gd.hop : std::max(c->init_grid, g->cu_count / 4);
    const State s = query_state(c, 0, nullptr, d_dist);
    PlainCtl *ctl = query_slot(c, 0);
    {
        ProfScope ps(g, KK_PLAIN_INIT, st);
        hipLaunchKernelGGL(plain_bfs_init_kernel, dim3(c->init_grid), dim3(kBlock), 0, st, ctl, gr, s, seed, d_levels,
                           d_levels ? level_cap : (int64_t)0, P.dir_mode, P.alpha, P.beta, pam, g->nnz, ps.units());
        ps.end(0, 1);
    }
    const int64_t limit = max_depth < 0 ? INT32_MAX : max_depth;
    int64_t H = 0;  // hops launched
    // hops per group between host checks: one more than the last search's depth
    int64_t group = std::max(2, g->bfs_hops_hint.load(std::memory_order_relaxed));
    while (H < limit) {
        const int64_t upto = h_flags ? std::min(limit, H + group) : limit;
        for (int64_t L = H + 1; L <= upto; ++L) {
            ProfScope ps(g, L == 1 ? KK_PLAIN_STEP : KK_PLAIN_HOP_PUSH, st);
            if (L == 1) {
                // hop 1 alone: the set-up above replaces the pipeline's other work
                const StepBook bk{nullptr, nullptr, nullptr, -1, nullptr, nullptr, nullptr, pam, g->nnz, INT32_MAX,
                                  (int32_t)P.dir_mode, (int32_t)P.alpha, (int32_t)P.beta};
                hipLaunchKernelGGL(plain_step_kernel, dim3(hop1_grid), dim3(kBlock), 0, st, (PlainCtl *)nullptr,
                                   (int64_t)0, ctl, (int64_t)hop1_grid, HopStates{{State{}, s}}, bk, State{},
                                   State{}, gr, P.pull_light, hc, ps.units());
                ps.end(0, 1);
                continue;
            }
            hipLaunchKernelGGL(plain_hop_kernel, dim3(gd.hop), dim3(kBlock), 0, st, ctl, (int)L, gr, s,
                               P.pull_light, hc, ps.units());
            ps.end_split(0, 1, KK_PLAIN_HOP_PULL, 1);
            ProfScope pc(g, KK_PLAIN_COMPACT, st);
            hipLaunchKernelGGL(plain_compact_kernel, dim3(gd.compact), dim3(kBlock), 0, st, ctl, (int)L, gr, s,
                               pc.units());
            pc.end(0, 1);
        }
        H = upto;
        if (!h_flags || H >= limit) break;
        hipLaunchKernelGGL(plain_bfs_probe_kernel, dim3(1), dim3(kWave), 0, st, ctl, s, (int)H, (int64_t *)nullptr,
                           (int32_t *)nullptr, (int64_t *)nullptr);
        // reached and more are adjacent in the control record
        KHOP_HIP(hipMemcpyAsync(h_flags, &ctl->reached, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        KHOP_HIP(hipStreamSynchronize(st));
        if (!h_flags[1]) {
            // a search of depth D ends after D + 1 hops (the last finds nothing)
            g->bfs_hops_hint.store(h_flags[0] + 1, std::memory_order_relaxed);
            break;
        }
        group = std::min<int64_t>(2 * group, 1024);
    }
    hipLaunchKernelGGL(plain_bfs_probe_kernel, dim3(1), dim3(kWave), 0, st, ctl, s, (int)H, d_count, d_depth,
                       (int64_t *)nullptr);
    KHOP_HIP(hipGetLastError());
}

void plain_set(khop_graph *g, PlainCtx *c, int32_t seed, int32_t *d_ids, int64_t capacity, int64_t *d_count,
               hipStream_t st) {
    const int64_t nw = (g->n + 63) / 64;
    const int64_t nb = c->set_blocks;
    const uint64_t *V = c->s[0].V;
    ProfScope ps(g, KK_PLAIN_SET, st);
    hipLaunchKernelGGL(plain_set_count_kernel, dim3((unsigned)nb), dim3(kBlock), 0, st, V, nw, seed, c->set_partial);
    hipLaunchKernelGGL(plain_set_scan_kernel, dim3(1), dim3(kBlock), 0, st, c->set_partial, nb, d_count);
    const bool write = capacity > 0 && d_ids;
    if (write)
        hipLaunchKernelGGL(plain_set_write_kernel, dim3((unsigned)nb), dim3(kBlock), 0, st, V, nw, seed,
                           (const int64_t *)c->set_partial, d_ids, capacity, ps.units());
    // the visited bitmap read once per pass, the block counts written, scanned and read
    ps.end((double)(write ? 2 : 1) * 8.0 * (double)nw + (write ? 4.0 : 2.0) * 8.0 * (double)nb, 1);
    KHOP_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ the no-allocation entry point

// Scratch for one query context per device, for callers that cannot
// allocate: 160 MiB holds the context of a graph of up to about 2.4 million
// vertices (69 bytes per vertex plus fixed parts).  Each device holds its own
// copy from the library's load until the process ends.  In host code the
// array's name is not a device address: its address on each device comes from
// hipGetSymbolAddress, made once per device with that device current.
constexpr size_t kScratchBytes = (size_t)160 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<char *> g_scratch_ptr;  // by device

char *scratch_on(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
    if (!g_scratch_ptr[(size_t)device]) {
        void *p = nullptr;
        KHOP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(KHOP_EDEVICE, "hipGetSymbolAddress returned no address for the query scratch");
        g_scratch_ptr[(size_t)device] = (char *)p;
    }
    return g_scratch_ptr[(size_t)device];
}

// Byte ranges to zero, each 8-byte aligned and padded to a multiple of 8.
struct ZeroRanges {
    uint64_t *p[8];
    int64_t words[8];
    int n;
};

__global__ void __launch_bounds__(kBlock) zero_ranges_kernel(ZeroRanges z) {
    for (int r = 0; r < z.n; ++r)
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < z.words[r]; i += (int64_t)gridDim.x * kBlock)
            z.p[r][i] = 0;
}

}  // namespace

size_t plain_noalloc_capacity() { return kScratchBytes; }
int plain_noalloc_max_k() { return kDeepHops; }

void plain_run_noalloc(khop_graph *g, const int32_t *d_seeds, int64_t num_seeds, int32_t k, int64_t *d_counts,
                       int64_t *d_te, hipStream_t st) {
    if (k > kDeepHops)
        fail(KHOP_ERANGE, "k = " + std::to_string(k) + " is deeper than the " + std::to_string(kDeepHops) +
                              " hops the no-allocation path runs (deeper queries need host-checked hop groups)");
    PlainCtx c;
    const size_t bytes = plain_layout(g, &c, nullptr);
    if (bytes > kScratchBytes)
        fail(KHOP_ERANGE, "a query context for " + std::to_string(g->n) + " vertices needs " + std::to_string(bytes) +
                              " bytes, more than the " + std::to_string(kScratchBytes) + "-byte no-allocation scratch");
    if (plain_heavy_table_current(g).threshold < 0) fail(KHOP_EINTERNAL, "the graph has no bottom-up chunk table");
    if (num_seeds <= 0) return;
    plain_layout(g, &c, scratch_on(g->device));
    c.fixed = true;
    // the scratch's bitmaps hold whatever an earlier call left: no block
    // flags, so that every set-up rewrites every word
    for (int p = 0; p < kStates; ++p) c.s[p].dirty = nullptr;
    // an earlier call (perhaps on another graph) left the scratch in any
    // state: the byte marks, their summaries and the control records, which
    // the path expects zero between queries, start clear
    const int64_t nw = (g->n + 63) / 64;
    ZeroRanges z{};
    for (int p = 0; p < kStates; ++p) {
        z.p[z.n] = (uint64_t *)c.s[p].nextb;
        z.words[z.n++] = nw * 8;  // nw * 64 bytes
        z.p[z.n] = (uint64_t *)c.s[p].nsum;
        z.words[z.n++] = (nw + 7) / 8;  // inside the 256-byte padding of the summary
    }
    z.p[z.n] = (uint64_t *)c.ctl;
    z.words[z.n++] = (int64_t)(kSlots * sizeof(PlainCtl) + 7) / 8;
    const int zgrid = (int)std::max<int64_t>(1, std::min<int64_t>((nw * 8 + kBlock - 1) / kBlock, 1024));
    hipLaunchKernelGGL(zero_ranges_kernel, dim3(zgrid), dim3(kBlock), 0, st, z);
    KHOP_HIP(hipGetLastError());
    plain_run(g, &c, d_seeds, num_seeds, k, d_counts, d_te, st, nullptr);
}

}  // namespace khop
