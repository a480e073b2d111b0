// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "khop.h"

namespace khop {

// Thrown inside the library, mapped to a status at the C boundary.
struct Error {
    int status;
    std::string msg;
};

[[noreturn]] void fail(int status, const std::string &msg);
void set_last_error(const std::string &msg);  // khop_last_error() of the calling thread
[[noreturn]] void hip_fail(hipError_t e, const char *what, const char *file, int line);

#define KHOP_HIP(call)                                                  \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) ::khop::hip_fail(e_, #call, __FILE__, __LINE__); \
    } while (0)

// Host-side CSR produced by the graph builder.
struct HostCSR {
    int64_t n = 0;
    std::vector<int64_t> rowptr;  // n + 1
    std::vector<int32_t> colidx;  // rowptr[n]
};

// Arcs a[i] -> b[i] (plus b[i] -> a[i] when `both`), self-loops and duplicates
// dropped, neighbors ascending.
HostCSR build_csr(const int32_t *a, const int32_t *b, int64_t m, int64_t n, bool both);
uint64_t csr_hash(const HostCSR &c);
int host_threads();

// Zero entries past the end of each device column array: kernels read four
// consecutive column indices with one 16-byte load from any index.
constexpr int64_t kColidxPad = 4;

// Tunable engine parameters (per graph).
struct Params {
    int dir_mode = KHOP_DIR_AUTO;
    int alpha = 14;        // push -> pull when mf * alpha > mu
    int beta = 24;         // pull -> push when nf * beta < n
    int pull_light = 32;   // plain bottom-up: lane-serial scan up to this degree
    int pull_heavy = 4096; // plain bottom-up: 256-edge chunks above this in-degree
    int push_atomic_max = 65536;  // plain top-down: claim heads atomically up to this many frontier edges
    int batch_seeds = 1024;    // batched: seeds per launch (64 * words)
    int batch_heavy = 256;     // batched bottom-up: chunked above this in-degree (one lane per vertex; G lanes: G/2 times it)
    int batch_push_div = 64;   // batched: top-down level when frontier arcs * div < total arcs
    int plain_grid = 4;        // plain hop and compaction kernels: blocks per compute unit
    int batch_grid = 16;       // batched bottom-up kernel: blocks per compute unit
    int plain_pipeline = 1;    // plain path: consecutive queries overlap by one launch (0: one at a time)
    int plain_graphs = 0;      // plain path: repeated runs replay captured HIP graphs
};

struct PlainCtx;
struct BatchCtx;

// Edge chunks of the vertices whose in-degree exceeds a threshold, so that a
// bottom-up scan of a hub is shared by many waves.
struct HeavyTable {
    int threshold = -1;
    int64_t chunk = 0;
    int32_t *d_vert = nullptr;
    int64_t *d_begin = nullptr;
    int64_t *d_end = nullptr;
    int64_t n = 0;
};

// A pooled context remembers the stream and completion event of its last use.
struct CtxUse {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
};

enum KernelKind {
    KK_PLAIN_INIT = 0,
    KK_PLAIN_STEP,      // a step launch of the plain pipeline: a query's hop 1 beside the last hop of the one before
    KK_PLAIN_HOP_PUSH,  // a hop 2..k-1 (or of a search) that went top-down, or found an empty frontier
    KK_PLAIN_HOP_PULL,  // a hop 2..k-1 (or of a search) that went bottom-up
    KK_PLAIN_COMPACT,
    KK_BATCH_INIT,
    KK_BATCH_PUSH,
    KK_BATCH_PULL,
    KK_BATCH_PULL_HEAVY,
    KK_BATCH_COUNT,
    KK_PLAIN_SET,     // the three kernels that list one neighborhood as ids, timed together
    KK_PLAIN_DEGREE,  // a one-hop query with no vertex mask: one launch that reads its seed's degree
    KK_EMPTY_LAUNCH,  // an empty kernel timed the same way: the event bracket's own cost
    KK_COUNT_KINDS
};
extern const char *const kKernelNames[KK_COUNT_KINDS];

// Per-kernel profiling with HIP events.  Each profiled launch may also own a
// slot of 4 device counter fields (64 int64 lanes each, summed on the host)
// that the kernel fills with the sizes its traffic depends on (edges examined,
// frontier size, ...).
struct Profiler {
    bool on = false;
    int64_t *d_units = nullptr;  // cap * 4 * 64
    int64_t cap = 0;
    int64_t next_slot = 0;
    struct Pending {
        int kind;
        hipEvent_t e0, e1;
        double fixed_bytes;
        int64_t slot;
        double w[4];
        int alt_kind;   // counted under this kind instead when counter field alt_field is nonzero (-1: never)
        int alt_field;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> events;
    int64_t launches[KK_COUNT_KINDS] = {};
    double ms[KK_COUNT_KINDS] = {};
    double bytes[KK_COUNT_KINDS] = {};
};

// Brackets one kernel launch with HIP events when profiling is on.
class ProfScope {
   public:
    ProfScope(khop_graph *g, int kind, hipStream_t st);
    // Device counter slot for the kernel (-1 when not profiling).
    int64_t *units() const { return units_; }
    // bytes = fixed + sum_i w[i] * units[i]
    void end(double fixed_bytes, double w0 = 0, double w1 = 0, double w2 = 0, double w3 = 0);
    // As end(fixed_bytes, w0), but the launch counts under alt_kind when the
    // kernel set counter field alt_field (a role it chose on the device).
    void end_split(double fixed_bytes, double w0, int alt_kind, int alt_field);

   private:
    khop_graph *g_;
    int kind_;
    hipStream_t st_;
    hipEvent_t e0_ = nullptr;
    int64_t slot_ = -1;
    int64_t *units_ = nullptr;
};

void prof_collect(khop_graph *g);  // caller holds g->prof_mu
void prof_delay(hipStream_t st);
void prof_empty(hipStream_t st);    // prof.hip

}  // namespace khop

struct khop_graph {
    int device = 0;
    int64_t n = 0;
    int64_t nnz = 0;  // stored arcs (out)
    int directed = 0;
    int64_t *d_rowptr = nullptr;
    int32_t *d_colidx = nullptr;
    int64_t *d_in_rowptr = nullptr;  // == d_rowptr when undirected
    int32_t *d_in_colidx = nullptr;
    // Per vertex, the in-neighbor of largest out-degree (ties: the lowest id),
    // which graph load puts first in the vertex's in-row; -1 for a vertex with
    // no in-edge.  The plain bottom-up hop tests it before reading the row.
    int32_t *d_probe = nullptr;
    khop::HeavyTable plain_heavy;    // chunks for the plain bottom-up hop
    std::vector<khop::HeavyTable> batch_heavy;  // chunks for the batched bottom-up hops, one table per threshold
    int32_t *d_in_order = nullptr;   // vertices by ascending in-degree (ties by id), built on first use
    int64_t in_order_zero = 0;       // how many of them have no in-edge (they come first)
    std::vector<khop::HeavyTable> heavy_retired;  // replaced tables, freed with the graph
    std::mutex heavy_mu;             // guards the tables above
    std::vector<int64_t> h_outdeg;   // host copy of out-degrees
    std::vector<int64_t> h_indeg;
    uint64_t hash = 0;
    khop::Params params;             // read through params_of(), written through params_set()
    std::mutex params_mu;
    hipStream_t stream = nullptr;    // stream of the host-pointer entry points
    std::mutex mu;                   // guards the context pools, heavy list and profiler
    std::vector<khop::PlainCtx *> plain_free;
    std::vector<khop::BatchCtx *> batch_free;
    std::mutex prof_mu;
    khop::Profiler prof;
    int cu_count = 256;
    std::atomic<int> bfs_hops_hint{8};  // hops the last unlimited breadth-first search took
};

namespace khop {

// plain.hip
PlainCtx *plain_ctx_create(khop_graph *g);
void plain_ctx_destroy(PlainCtx *c);
// Whether the context replays repeated runs from captured HIP graphs (on by default).
void plain_ctx_set_graphs(PlainCtx *c, bool on);
// d_vmask (may be null): one bit per vertex, the vertices the searches may enter (the seeds are exempt).
void plain_run(khop_graph *g, PlainCtx *c, const int32_t *d_seeds, int64_t num_seeds, int32_t k,
               int64_t *d_counts, int64_t *d_te, hipStream_t st, const uint64_t *d_vmask = nullptr);
void plain_fill_zero_outputs(int64_t *d_counts, int64_t *d_te, int64_t n, hipStream_t st);
// plain_run on a query context laid out in the library's static device
// scratch: allocates nothing.  Throws KHOP_ERANGE when the graph's context
// does not fit the scratch or k exceeds the pipelined path's depth.
void plain_run_noalloc(khop_graph *g, const int32_t *d_seeds, int64_t num_seeds, int32_t k, int64_t *d_counts,
                       int64_t *d_te, hipStream_t st);
size_t plain_noalloc_capacity();  // bytes of that scratch
int plain_noalloc_max_k();
// Breadth-first search from one (valid) seed, up to max_depth hops (< 0: no
// limit), on the context's first state.  Distances go to d_dist[n] and the
// size of each level 1..level_cap to d_levels when those are not null; the
// count of levels 1..max_depth and the largest non-empty level go to d_count /
// d_depth when not null.  h_flags (pinned, two int32) lets the host check
// between groups of hops whether the frontier is empty; without it exactly
// max_depth hops are enqueued (max_depth >= 0 then).
void plain_bfs(khop_graph *g, PlainCtx *c, int32_t seed, int32_t max_depth, int32_t *d_dist, int64_t *d_count,
               int32_t *d_depth, int64_t *d_levels, int64_t level_cap, int32_t *h_flags, hipStream_t st);
// After plain_bfs on the same context and stream: the searched neighborhood
// (visited vertices but the seed) as ascending ids, the first `capacity` of
// them into d_ids, and their number into *d_count (device pointers).
void plain_set(khop_graph *g, PlainCtx *c, int32_t seed, int32_t *d_ids, int64_t capacity, int64_t *d_count,
               hipStream_t st);

// abi.cpp: batched launches of a seed set (seeds on the device, ks on the host), pooled contexts
void run_batched(khop_graph *g, const int32_t *d_seeds, const int32_t *h_ks, int64_t num, int64_t *d_counts,
                 hipStream_t st, const uint64_t *d_vmask = nullptr);

// batched.hip
BatchCtx *batch_ctx_create(khop_graph *g, int words);
// Device bytes of a batch context of `words` 64-seed words for a graph of n vertices and nnz arcs.
size_t batch_ctx_bytes(int64_t n, int64_t nnz, int words);
void batch_ctx_destroy(BatchCtx *c);
int batch_ctx_words(const BatchCtx *c);
// Runs one batch of at most 64 * words seeds.  Slot j is seed d_seeds[h_perm[j]]
// at depth h_ks_sorted[j] (non-increasing in j); its count goes to d_counts[h_perm[j]].
// d_vmask (may be null): one bit per vertex, the vertices the searches may enter (the seeds are exempt).
void batch_run(khop_graph *g, BatchCtx *c, const int32_t *d_seeds, const int32_t *h_perm,
               const int32_t *h_ks_sorted, int64_t num_seeds, int64_t *d_counts, hipStream_t st,
               const uint64_t *d_vmask = nullptr);

// heavy.cpp: the chunk table for a threshold, (re)built when the threshold
// changes.  The copy returned stays valid until graph_free.
HeavyTable plain_heavy_table(khop_graph *g, int threshold);
HeavyTable batch_heavy_table(khop_graph *g, int threshold);
// The plain table as it stands, never rebuilt (graph_load_csr builds one for the default threshold).
HeavyTable plain_heavy_table_current(khop_graph *g);
void heavy_tables_free(khop_graph *g);
// The graph's vertices sorted by in-degree, ascending, ties by id (device
// array of n ids, built on first use, freed with the tables); *zero (when not
// null) gets the number of them with no in-edge, which come first.
const int32_t *in_degree_order(khop_graph *g, int64_t *zero = nullptr);
// A consistent copy of the graph's options, and their replacement (options
// change between calls; a call runs on the copy it took when it started).
Params params_of(khop_graph *g);
void params_set(khop_graph *g, const Params &p);

// tune.cpp: hash of the library's sources, fixed at build time
const char *source_hash();

}  // namespace khop
