/*
 * khop.h -- C ABI of libkhop.so, an MI355X (gfx950) engine for the k-hop
 * neighborhood count benchmarked in RedisGraph (Cailliau et al.,
 * arXiv:1905.01294, Section III: "k-hop neighborhood count", k = 1, 2, 3, 6).
 *
 * The count of a seed s at depth k is |{ v : 1 <= dist(s, v) <= k }|, the
 * number of vertices at hop distance 1..k.  As in the paper's Section II, one
 * hop is a sparse matrix-vector product of the adjacency matrix with the
 * frontier over the boolean (OR, AND) semiring, masked by the complement of
 * the visited set; after l products the visited set is { v : dist(s, v) <= l }.
 *
 * Conventions for every entry point:
 *   - the return value is a status: KHOP_OK (0) or a negative KHOP_E* code;
 *   - on error, output arguments are left untouched and khop_last_error()
 *     returns a message (thread local, valid until the thread's next call);
 *   - no C++ exception crosses this boundary;
 *   - input arrays are borrowed for the duration of the call only; output
 *     arrays are owned by the caller;
 *   - argument validation happens before any device work, so invalid calls
 *     fail the same way with or without a GPU;
 *   - a HIP runtime failure maps to KHOP_EDEVICE, a failed device allocation
 *     to KHOP_ENOMEM.
 */
#ifndef KHOP_H
#define KHOP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct khop_graph khop_graph;   /* opaque; immutable once loaded */
typedef struct khop_server khop_server; /* opaque */

enum khop_status {
    KHOP_OK = 0,
    KHOP_EINVAL = -1,     /* NULL pointer with a nonzero length, bad id, k < 0, bad option */
    KHOP_ERANGE = -2,     /* a size the engine's index types cannot hold */
    KHOP_ENOMEM = -3,     /* host or device allocation failed */
    KHOP_EDEVICE = -4,    /* no usable gfx950 device, or a HIP runtime error */
    KHOP_EBUSY = -5,      /* the server's request queue is full */
    KHOP_ETIMEDOUT = -6,  /* a served request passed its deadline before it ran */
    KHOP_EINTERNAL = -7   /* unexpected internal failure */
};

/* flags for graph_load_csr */
enum { KHOP_UNDIRECTED = 0, KHOP_DIRECTED = 1 };

/*
 * Build the device graph from raw edge tuples (src[i], dst[i]), i < num_edges,
 * over vertices [0, num_vertices).  The adjacency matrix of the paper's
 * storage model (Section II: graphs kept as sparse adjacency matrices in a
 * compressed representation) is built as CSR with int64 row pointers and
 * int32 column indices, neighbors ascending:
 *   - self-loops and duplicate tuples are dropped;
 *   - KHOP_UNDIRECTED stores every tuple in both directions;
 *   - KHOP_DIRECTED follows tuples from src to dst and also keeps the
 *     transpose (in-edges) for bottom-up expansion.
 * src/dst are host pointers (int32, length num_edges).  Errors: NULL with
 * num_edges > 0, num_vertices <= 0, an endpoint outside [0, num_vertices) or
 * unknown flags -> KHOP_EINVAL (the whole load is rejected);
 * num_vertices > INT32_MAX or more than 2^62 arcs -> KHOP_ERANGE.  On success
 * *out owns the graph until graph_free.
 */
int graph_load_csr(const int32_t *src, const int32_t *dst, int64_t num_edges, int64_t num_vertices,
                   uint32_t flags, khop_graph **out);

/*
 * Typed form of graph_load_csr: tuple i carries a relation type rel[i] in
 * [0, 64), and only the tuples whose type has its bit set in rel_mask are
 * kept.  The graph is the union of the selected relations' adjacency
 * matrices (a traversal over several relation types follows any of them), so
 * every count, search and server entry point traverses only those
 * relations: the typed form of a query plan's traversal, whose plans the
 * paper turns into sparse-matrix operations (Section II).  rel is a host array of num_edges bytes.  Errors as
 * graph_load_csr, plus KHOP_EINVAL for rel NULL with num_edges > 0 or a type
 * of 64 or more; endpoints are checked on the kept tuples only.
 */
int graph_load_csr_typed(const int32_t *src, const int32_t *dst, const uint8_t *rel, int64_t num_edges,
                         int64_t num_vertices, uint32_t flags, uint64_t rel_mask, khop_graph **out);

/* Release a graph and its device memory.  NULL is accepted (KHOP_OK). */
int graph_free(khop_graph *g);

/* Sizes of a loaded graph: vertices, stored arcs (after cleanup) and directedness. */
int graph_info(const khop_graph *g, int64_t *num_vertices, int64_t *num_arcs, int32_t *directed);

/* Out-degree of every vertex (stored arcs, self-loops and duplicates dropped) into deg[num_vertices] (host). */
int graph_degrees(const khop_graph *g, int64_t *deg);

/*
 * Plain single-query path (the paper's protocol in Section III: seeds run one
 * after another, each answered by its own count).  For each seeds[i] in order,
 * one launch sequence computes counts[i] = |{ v : 1 <= dist(seeds[i], v) <= k }|
 * and, when traversed_edges is not NULL, traversed_edges[i] = the sum of the
 * out-degrees of the vertices at distance 0..k-1 (the edges a top-down search
 * inspects; the numerator of TEPS).  Host pointers, length num_seeds.  Each
 * query is complete (count copied to the host) before the next starts.
 * Errors: a seed outside [0, n) or k < 0 -> KHOP_EINVAL.  k == 0 gives 0.
 * num_seeds == 0 is a no-op.  Duplicate seeds give identical answers.
 */
int khop_count(khop_graph *g, const int32_t *seeds, int64_t num_seeds, int32_t k, int64_t *counts,
               int64_t *traversed_edges);

/*
 * Same computation with device-resident arrays, enqueued on `hip_stream`
 * (a hipStream_t; NULL means the null stream) without host synchronisation:
 * d_seeds (int32), d_counts and d_traversed_edges (int64, may be NULL) are
 * device pointers of length num_seeds.  Seeds are validated on the device:
 * a seed outside [0, n) yields count -1 and traversed edges -1 for that query.
 * The caller synchronises the stream before reading the outputs.  The seeds
 * are answered in order, and consecutive queries overlap by one launch (the
 * last hop of one runs beside hop 1 of the next) unless the option
 * KHOP_OPT_PLAIN_PIPELINE is 0.  With k = 1 and no forced direction each
 * query is one launch that reads its seed's out-degree: a row holds no
 * self-loop or duplicate, so that is its one-hop count (and its traversed
 * edges).  With k > 32 the queries run one at a time
 * as searches whose hops are launched in groups, and the call waits on the
 * stream between groups to learn whether the frontier has emptied (a query
 * never runs more hops than its search has levels, so any k is cheap).
 */
int khop_count_dev(khop_graph *g, const int32_t *d_seeds, int64_t num_seeds, int32_t k, int64_t *d_counts,
                   int64_t *d_traversed_edges, void *hip_stream);

/*
 * khop_count_dev for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and outputs, with the query context placed in a static
 * device scratch array of the library (160 MiB per device, held from the
 * library's load until the process ends), so the call makes no hipMalloc,
 * hipFree or other allocation, and waits on nothing.  Limits: the graph's
 * query context must fit the scratch (about 69 bytes per vertex: up to about
 * 2.4 million vertices) and k must be at most 32; otherwise KHOP_ERANGE with
 * nothing enqueued.  Other errors as khop_count_dev.  Every call on one GPU
 * shares that GPU's scratch, which keeps the last call's contents (each call
 * clears what must start at zero): calls that overlap on one GPU, from two
 * streams or two threads, race and must not be made.  Options are read as in
 * khop_count_dev, but a changed bottom-up chunk threshold
 * (KHOP_OPT_PULL_HEAVY) does not rebuild the chunk table here; the table the
 * graph already has is used, which changes no count.  Not profiled.
 */
int khop_count_dev_noalloc(khop_graph *g, const int32_t *d_seeds, int64_t num_seeds, int32_t k, int64_t *d_counts,
                           int64_t *d_traversed_edges, void *hip_stream);

/*
 * Label-filtered count: the k-hop count of each seed in the subgraph of the
 * vertices whose bit is set in label_bits (bit v % 64 of word v / 64; the
 * seed itself is always the start, labeled or not), i.e. counts[i] =
 * |{ v labeled : 1 <= dist'(seeds[i], v) <= k }| where dist' only follows
 * paths through labeled vertices.  This is the vertex-label mask of a typed
 * query plan applied inside each masked product: the vertices outside the
 * mask start visited, so NOT visited excludes them.  traversed_edges (may be
 * NULL) as in khop_count, over the vertices the filtered search expands.
 * Host pointers: label_bits has ceil(n / 64) words (bits past n ignored),
 * seeds/counts num_seeds entries.  All seeds are enqueued as one pipelined
 * sequence (as khop_count_dev), then one synchronisation.  Errors as khop_count,
 * plus label_bits NULL -> KHOP_EINVAL.
 */
int khop_count_labeled(khop_graph *g, const int32_t *seeds, int64_t num_seeds, int32_t k, const uint64_t *label_bits,
                       int64_t *counts, int64_t *traversed_edges);

/* Device-pointer form of khop_count_labeled (d_label_bits on the device), as khop_count_dev. */
int khop_count_labeled_dev(khop_graph *g, const int32_t *d_seeds, int64_t num_seeds, int32_t k,
                           const uint64_t *d_label_bits, int64_t *d_counts, int64_t *d_traversed_edges,
                           void *hip_stream);

/*
 * Batched multi-source path: seeds travel together as per-vertex 64-bit seed
 * bitsets, so each hop becomes a boolean sparse matrix - dense bit-matrix
 * product (OR-accumulate), masked by the complement of each seed's visited
 * bits.  counts[i] is the k-hop count of seeds[i] at depth ks[i] (mixed k in
 * one call).  Seeds with k = 1 take no bit: their counts come from their own
 * rows, beside the bitset launches.  Host pointers of length num_seeds.
 * Errors as khop_count.
 */
int khop_count_batched(khop_graph *g, const int32_t *seeds, const int32_t *ks, int64_t num_seeds,
                       int64_t *counts);

/* Device-pointer form of khop_count_batched, enqueued on hip_stream without host synchronisation. */
int khop_count_batched_dev(khop_graph *g, const int32_t *d_seeds, const int32_t *d_ks, int64_t num_seeds,
                           int64_t *d_counts, void *hip_stream);

/*
 * Batched form of khop_count_labeled: counts[i] is the label-filtered k-hop
 * count of seeds[i] at depth ks[i].  Every seed's visited bits start set on
 * the vertices outside label_bits, so no hop enters them, and the per-seed
 * count skips them.  Host pointers (label_bits ceil(n / 64) words).  Errors
 * as khop_count_batched, plus label_bits NULL -> KHOP_EINVAL.
 */
int khop_count_batched_labeled(khop_graph *g, const int32_t *seeds, const int32_t *ks, int64_t num_seeds,
                               const uint64_t *label_bits, int64_t *counts);

/*
 * Breadth-first distances from one seed: the level-synchronous search behind
 * the k-hop count (Section III; each level one masked product of Section II)
 * run to the end, on the kernels of khop_count plus one store per discovered
 * vertex.  dist[v] = the hop distance from seed to v when it is at most
 * max_depth, else -1; dist[seed] = 0.  max_depth < 0 means no limit.
 * *count (may be NULL) = the vertices at distance 1..max_depth (the k-hop
 * count at k = max_depth, or the size of the seed's reach minus one);
 * *depth (may be NULL) = the largest distance found.  dist is a host array of
 * num_vertices int32, written only on success.  Hops are launched in groups
 * and the host checks between groups whether the frontier has emptied, so a
 * search costs about depth + 1 hop launches whatever max_depth is.
 * Errors: seed outside [0, n) or dist NULL -> KHOP_EINVAL; KHOP_ENOMEM when
 * the device distance buffer cannot be allocated.
 */
int khop_bfs(khop_graph *g, int32_t seed, int32_t max_depth, int32_t *dist, int64_t *count, int32_t *depth);

/*
 * Device-pointer form of khop_bfs on hip_stream: d_dist (int32, num_vertices
 * entries), d_count (one int64, may be NULL) and d_depth (one int32, may be
 * NULL) are device pointers, written in stream order.  With max_depth >= 0
 * exactly max_depth hops are enqueued and the host never waits (hops after
 * the frontier empties exit at once).  With max_depth < 0 the call waits on
 * the stream between groups of hops to learn whether the frontier has
 * emptied, and returns once the last hop is enqueued; the caller still
 * synchronises before reading the outputs.  Errors as khop_bfs (the seed is
 * checked on the host).
 */
int khop_bfs_dev(khop_graph *g, int32_t seed, int32_t max_depth, int32_t *d_dist, int64_t *d_count,
                 int32_t *d_depth, void *hip_stream);

/*
 * Exactly-l counts: level_counts[l-1] = |{ v : dist(seed, v) = l }| for
 * l = 1..k, from one search of depth k (the sizes of the frontiers the masked
 * products of Section II produce; their sum is the k-hop count).  Host array
 * of k int64.  Errors: seed outside [0, n), k < 0, or level_counts NULL with
 * k > 0 -> KHOP_EINVAL.  k == 0 writes nothing.
 */
int khop_levels(khop_graph *g, int32_t seed, int32_t k, int64_t *level_counts);

/* Device-pointer form of khop_levels on hip_stream (k hops enqueued, no host wait). */
int khop_levels_dev(khop_graph *g, int32_t seed, int32_t k, int64_t *d_level_counts, void *hip_stream);

/*
 * The k-hop neighborhood itself, { v : 1 <= dist(seed, v) <= k }, as
 * ascending vertex ids (the result set a graph query returns; large result
 * sets are among the costs the paper's Section IV names;
 * k < 0: everything the seed reaches).  The first min(count, capacity) ids go
 * to ids (host, capacity int32), and *count receives the full size, so a
 * caller with too small a buffer learns the size it needs.  Errors: seed
 * outside [0, n), capacity < 0, ids NULL with capacity > 0, or count NULL ->
 * KHOP_EINVAL.
 */
int khop_neighborhood(khop_graph *g, int32_t seed, int32_t k, int32_t *ids, int64_t capacity, int64_t *count);

/*
 * Device-pointer form of khop_neighborhood on hip_stream: d_ids (capacity
 * int32) and d_count (one int64) are device pointers written in stream order.
 * With k >= 0 the host never waits; with k < 0 it waits between groups of
 * hops as khop_bfs_dev does.
 */
int khop_neighborhood_dev(khop_graph *g, int32_t seed, int32_t k, int32_t *d_ids, int64_t capacity,
                          int64_t *d_count, void *hip_stream);

/* Engine options (per graph). */
enum khop_option {
    KHOP_OPT_DIRECTION = 1,     /* KHOP_DIR_AUTO (default), KHOP_DIR_PUSH or KHOP_DIR_PULL */
    KHOP_OPT_ALPHA = 2,         /* push -> pull when frontier edges * alpha > unvisited edges */
    KHOP_OPT_BETA = 3,          /* pull -> push when frontier vertices * beta < n */
    KHOP_OPT_PULL_LIGHT = 4,    /* bottom-up: degree up to which one lane scans a vertex alone */
    KHOP_OPT_BATCH_SEEDS = 5,   /* seeds per batched launch: 64, 128, 256, 512 or 1024 */
    KHOP_OPT_BATCH_HEAVY = 6,   /* batched bottom-up: in-degree above which a vertex's in-edges are split into
                                   1024-edge chunks, a wave each (levels whose rows take G > 2 lanes per
                                   vertex: G/2 times it) */
    KHOP_OPT_BATCH_PUSH = 7,    /* batched: frontier-degree fraction (1/x of arcs) under which a level goes top-down */
    KHOP_OPT_PULL_HEAVY = 8,    /* bottom-up: in-degree above which a vertex's in-edges are split into chunks */
    KHOP_OPT_PUSH_ATOMIC = 9,   /* top-down: frontier edges up to which heads are claimed atomically
                                   (else byte marks) */
    KHOP_OPT_PLAIN_GRID = 10,   /* plain hop and compaction launches: blocks per compute unit (1..64) */
    KHOP_OPT_BATCH_GRID = 11,   /* batched bottom-up launches: blocks per compute unit (1..64) */
    KHOP_OPT_PLAIN_PIPELINE = 12, /* 1 (default): consecutive plain queries overlap by one launch;
                                    0: each query runs its own launch sequence, start to count, before the
                                    next starts (the paper's strictly sequential protocol) */
    KHOP_OPT_PLAIN_GRAPHS = 13  /* 0 (default): every plain run launches its kernels directly; 1: a run
                                   repeated with the same device pointers, sizes and settings replays its
                                   launch sequence, captured as a HIP graph the second time it is seen (it
                                   can pay for long runs of shallow queries, whose launches are short; a
                                   graph launch's own cost outweighs it for short runs) */
};
enum { KHOP_DIR_AUTO = 0, KHOP_DIR_PUSH = 1, KHOP_DIR_PULL = 2 };

int khop_set_option(khop_graph *g, int32_t option, int64_t value);
int khop_get_option(const khop_graph *g, int32_t option, int64_t *value);

/*
 * Autotuner: times candidate settings on the resident graph with seeds drawn
 * from its non-isolated vertices, keeps the fastest, and leaves the graph's
 * options set to it: for the plain path the direction thresholds, the
 * bottom-up lane and chunk thresholds, the atomic top-down limit and the
 * hop kernels' blocks per compute unit; for the batched path the seeds per
 * launch with the heavy-vertex threshold, the top-down/bottom-up switch and
 * the bottom-up kernels' blocks per compute unit.  seeds_per_launch > 0
 * restricts the batched search to that batch size.  Results are cached per
 * (library sources, device, graph content hash) in memory and in the file
 * named by $KHOP_TUNE_CACHE (default ~/.cache/khop/tune.txt), so settings
 * tuned for other kernels are never reused.  A forced direction option is
 * left as it is.
 */
int khop_autotune(khop_graph *g, int32_t seeds_per_launch);

/* Seconds the last khop_autotune call in this process spent searching; 0 when
 * its settings came from the cache (or no call has run). */
double khop_autotune_seconds(void);

/* Per-kernel timing of the engine, measured with HIP events on the stream each kernel runs on. */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;          /* summed event-to-event time of the launches */
    double algorithmic_bytes; /* summed bytes the launches must move, from the per-unit traffic model */
} khop_kernel_stat;

/* enable != 0 starts collecting (and clears previous statistics); 0 stops.
 * Enabling also times 16 empty launches bracketed the same way, reported
 * under the name "empty_launch": the events' own share of each launch. */
int khop_profile(khop_graph *g, int32_t enable);
/* Copy up to max entries of the statistics collected so far; *n_out receives the count. */
int khop_profile_read(khop_graph *g, khop_kernel_stat *out, int32_t max, int32_t *n_out);

/* ------------------------------------------------------------ serving */

typedef struct {
    uint64_t ticket;
    int32_t status;       /* KHOP_OK or KHOP_ETIMEDOUT */
    int32_t graph_id;
    int32_t seed;
    int32_t k;
    int64_t count;
    int64_t t_submit_ns;  /* CLOCK_MONOTONIC at submission */
    int64_t t_admit_ns;   /* when its seed bit entered a running batch, or its single-query group started */
    int64_t t_done_ns;    /* when its count reached the host */
    int32_t path;         /* KHOP_PATH_BATCH or KHOP_PATH_SINGLE: what answered it */
    int32_t reserved;     /* 0 */
} khop_result;
enum { KHOP_PATH_BATCH = 0, KHOP_PATH_SINGLE = 1 };

/*
 * A continuous-batching server for k-hop queries (the throughput-oriented
 * serving model of the paper's Section II, where a pool of workers answers
 * concurrent queries).  Graphs stay resident.  Each graph has two batch
 * lanes, one for queries with k <= 2 and one for deeper ones (short queries
 * never wait behind deep traversals), and each lane has two run slots with a
 * HIP stream each.  A free slot takes the requests waiting in its lane (FIFO,
 * up to 64 per word of its batch context) as one batched launch sequence:
 * the computation of khop_count_batched, seeds as bit columns of one bitset
 * product per hop.  Requests that arrive while a lane's slots are busy join
 * its next launch as soon as a slot frees, so launches of a lane, of all
 * lanes and of all graphs overlap on the device and the batch size follows
 * the load.  Each graph also has a single-query lane on a stream of its own
 * that answers queries one at a time through the plain path (the paper's one
 * query per worker), in groups of one k.  A single query costs more device
 * time than its share of a batch, so that lane takes arrivals only while the
 * device time it would need stays low (decayed sums over about 5 ms of the
 * arrivals' measured single-query costs: cheap queries, up to 0.05 ms, while
 * theirs stays under half the device; dearer ones while all arrivals' stays
 * under the whole, with hysteresis) and it would still answer before the
 * batch lane (its backlog against the lane's measured launch time and the
 * wait for a free slot).  So queries get the single-query latency at low
 * load and the batches' throughput at high load; khop_result.path says which
 * answered, and khop_server_set_option can force one path.
 * mem_budget_bytes bounds the device memory of the batch contexts the slots
 * hold (khop_server_batch_bytes gives one context's size; a slot takes the
 * widest context, up to max_batch_seeds / 64 words, that the budget left
 * allows, and gives it back when it has been idle for 2 s or another lane
 * waits for memory); requests wait while no context fits, and time out at
 * their deadline.  max_batch_seeds (64..1024, a multiple of 64) bounds the
 * queries of one launch.
 */
int khop_server_create(int64_t mem_budget_bytes, int32_t max_batch_seeds, khop_server **out);
/*
 * Register a loaded graph (borrowed; it must outlive the server).  Its
 * single-query lane's query context (about 69 bytes per vertex: bitmaps,
 * byte marks and frontier queues) and the lanes' small staging buffers are
 * allocated here, outside mem_budget_bytes.
 */
int khop_server_add_graph(khop_server *s, khop_graph *g, int32_t *graph_id);

/* Device bytes of one batch context of `words` 64-query words (1..16) for graph g: what a run slot
 * of the server charges to its memory budget.  Errors: NULL arguments or words out of range -> KHOP_EINVAL. */
int khop_server_batch_bytes(const khop_graph *g, int32_t words, int64_t *bytes);

/* Counters of one lane of a server, since it was created. */
typedef struct {
    int32_t graph_id;
    int32_t lane;      /* KHOP_LANE_SHORT (batches of k <= 2), KHOP_LANE_DEEP (k > 2) or KHOP_LANE_SINGLE */
    int64_t launches;  /* batched launches (single-query lane: launch sequences) completed */
    int64_t queries;   /* queries they answered */
    double busy_ms;    /* their summed time from enqueue to completion (launches may overlap) */
    double max_ms;     /* the longest */
    int32_t words;     /* 64-query words of the widest batch context the lane holds now (0: none) */
    int32_t queued;    /* requests waiting in the lane */
} khop_server_stat;
enum { KHOP_LANE_SHORT = 0, KHOP_LANE_DEEP = 1, KHOP_LANE_SINGLE = 2 };
/* Copy up to max lane counters (two batch lanes per graph, then one single-query lane per graph)
 * into out (host); *n_out receives how many were written. */
int khop_server_stats(khop_server *s, khop_server_stat *out, int32_t max, int32_t *n_out);

/* Server options. */
enum khop_server_option {
    KHOP_SERVER_ROUTE = 1 /* KHOP_ROUTE_AUTO (default), KHOP_ROUTE_BATCH or KHOP_ROUTE_PLAIN */
};
enum { KHOP_ROUTE_AUTO = 0, KHOP_ROUTE_BATCH = 1, KHOP_ROUTE_PLAIN = 2 };
/* Set a server option.  It applies to requests the scheduler has not routed yet (in practice, those
 * submitted after the call).  Unknown option or value -> KHOP_EINVAL. */
int khop_server_set_option(khop_server *s, int32_t option, int64_t value);
/* Queue one query; deadline_ns is an absolute CLOCK_MONOTONIC time, 0 = none. */
int khop_server_submit(khop_server *s, int32_t graph_id, int32_t seed, int32_t k, int64_t deadline_ns,
                       uint64_t *ticket);
/* Move up to max finished results into out (host array); *n_out receives how many. */
int khop_server_poll(khop_server *s, khop_result *out, int64_t max, int64_t *n_out);
/* Block until every submitted request has a result (or timeout_ms passes; then KHOP_ETIMEDOUT). */
int khop_server_drain(khop_server *s, int64_t timeout_ms);
/* Stop the scheduler; unfinished requests are dropped.  NULL is accepted. */
int khop_server_destroy(khop_server *s);

/* Message of the calling thread's last failed call ("" if none). */
const char *khop_last_error(void);

/* Library version string. */
const char *khop_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KHOP_H */
