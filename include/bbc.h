/*
 * bbc.h -- balanced-butterfly counting on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libbbc.so.  Plain pointers and sizes only.
 *
 * The operation (Das, Abidi, Shingane, Kiran, "Balanced Butterfly Counting in
 * Bipartite-Network", Section 2): G = (U, V, E) is a signed bipartite graph,
 * E a set of pairs (u, v) in U x V, each labelled + or -.  A butterfly is a
 * 4-cycle u1-v1-u2-v2 (u1 != u2 in U, v1 != v2 in V, all four edges in E;
 * Definition 1); it is balanced when it holds an even number of negative edges
 * (Definition 2).  bbc_count returns the number of balanced butterflies (the
 * problem statement of Section 2), together with the number of unbalanced ones
 * and the number W of wedges the bucket method enumerates: wedges (u, v, w)
 * whose start u has a higher priority than the middle v and the end w, the
 * priority being (degree, id) with ids 0..|U|-1 for U and |U|..|U|+|V|-1 for V
 * (Definition 4, Algorithm 2).  All results are exact integers.
 *
 * Errors: every call returns a bbc_status.  On any status other than BBC_OK
 * nothing is written to the caller's output buffers, and bbc_last_error()
 * gives a one-line description.  After BBC_ERR_DEVICE the context must be
 * destroyed.
 *
 * Threading: a context is not thread safe; distinct contexts may be used from
 * distinct threads at once.
 */
#ifndef BBC_H
#define BBC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bbc_status {
    BBC_PENDING = 1,              /* bbc_server_poll only: the job has not finished yet */
    BBC_OK = 0,
    BBC_ERR_INVALID_ARG = -1,     /* negative size, NULL pointer with n_edges > 0, bad flag */
    BBC_ERR_VERTEX_RANGE = -2,    /* an edge names u >= n_u, v >= n_v or a negative id */
    BBC_ERR_BAD_SIGN = -3,        /* an edge sign other than +1 or -1 */
    BBC_ERR_DUPLICATE_EDGE = -4,  /* the same (u, v) pair twice, whatever the signs */
    BBC_ERR_TOO_LARGE = -5,       /* n_u + n_v >= 2^30 or n_edges >= 2^31 - 1024 */
    BBC_ERR_OVERFLOW = -6,        /* a count does not fit in int64_t */
    BBC_ERR_OUT_OF_MEMORY = -7,   /* device workspace could not be allocated or exceeds
                                     the BBC_MAX_DEVICE_BYTES budget */
    BBC_ERR_DEVICE = -8,          /* a HIP runtime call failed; the context is unusable */
    BBC_ERR_NOT_IMPLEMENTED = -9, /* a requested feature is not built */
    BBC_ERR_INTERNAL = -10        /* an internal capacity was exceeded (see bbc_last_error) */
} bbc_status;

typedef struct bbc_context bbc_context; /* opaque: device, stream, workspace arena */

typedef struct bbc_result {
    int64_t balanced;   /* balanced butterflies (even number of negative edges) */
    int64_t unbalanced; /* butterflies with an odd number of negative edges */
    int64_t wedges;     /* W: wedges kept by the vertex-priority filter */
} bbc_result;

/* flags for bbc_count */
enum {
    BBC_INPUT_ON_DEVICE = 1u,  /* edge_u/edge_v/edge_sign are device pointers on the
                                  context's device, ordered on its stream */
    BBC_OUTPUT_ON_DEVICE = 2u, /* with BBC_PER_VERTEX: per_vertex is a device pointer
                                  on the context's device */
    BBC_PER_VERTEX = 4u        /* also fill per_vertex (see bbc_count) */
};

/*
 * Create a context on HIP device `device`.  `hip_stream` is a hipStream_t the
 * library launches all work on (borrowed, not destroyed by bbc_destroy); NULL
 * makes the library create and own a stream.  *out receives the context.
 * Returns BBC_ERR_INVALID_ARG for out == NULL, BBC_ERR_DEVICE if the device or
 * stream cannot be used.
 */
bbc_status bbc_create(int device, void* hip_stream, bbc_context** out);

/* Release the context's workspace and stream (if owned).  NULL is a no-op. */
void bbc_destroy(bbc_context* ctx);

/*
 * Count the balanced butterflies of the signed bipartite graph with vertex
 * sets U = {0..n_u-1}, V = {0..n_v-1} and edges i = 0..n_edges-1 given by
 * (edge_u[i], edge_v[i]) with sign edge_sign[i] in {+1, -1}.
 *
 * Inputs (int32 ids, int8 signs, all length n_edges) are host pointers, or
 * device pointers when flags has BBC_INPUT_ON_DEVICE; they are only read, and
 * only for the duration of the call.  The edge order is arbitrary.
 * `out` (host) receives the counts.  With BBC_PER_VERTEX, `per_vertex` (host,
 * n_u + n_v entries, U first then V) receives for every vertex the number of
 * balanced butterflies that contain it (Section 5.1); otherwise it may be NULL.
 * With BBC_OUTPUT_ON_DEVICE as well, `per_vertex` is a device buffer of that
 * size on the context's device (written on the device, never copied to the
 * host); the flag without BBC_PER_VERTEX is INVALID_ARG.  Either buffer is
 * written only when the call returns BBC_OK.
 *
 * The call is synchronous: it returns when the counts are on the host.
 * An empty graph, or one with fewer than two vertices on a side, gives zeros.
 */
bbc_status bbc_count(bbc_context* ctx, int32_t n_u, int32_t n_v, int64_t n_edges,
                     const int32_t* edge_u, const int32_t* edge_v, const int8_t* edge_sign,
                     uint32_t flags, bbc_result* out, int64_t* per_vertex);

/*
 * bbc_count without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and errors as bbc_count, with
 * these limits:
 *  - flags must hold BBC_INPUT_ON_DEVICE (device edge arrays), and
 *    BBC_PER_VERTEX needs BBC_OUTPUT_ON_DEVICE (a caller's device buffer);
 *    anything else is BBC_ERR_INVALID_ARG;
 *  - the whole workspace comes from one static device array of
 *    BBC_NOALLOC_SCRATCH_BYTES per device, which the library holds from its
 *    first use on that device until the process ends; a graph whose workspace
 *    does not fit gets BBC_ERR_TOO_LARGE (bbc_workspace_bytes estimates it;
 *    about 4 million edges fit), with the outputs untouched;
 *  - the call makes no hipMalloc / hipFree / hipHostMalloc and no host heap
 *    allocation; HIP-graph replay (BBC_PARAM_GRAPHS) is not used for it.
 * Every allocation-free call on one device uses the same array, whatever the
 * context: calls that overlap in time on one device race and give wrong
 * results, so they must be serialised by the caller.  The array keeps the
 * last call's contents; the call clears whatever it needs.
 */
#define BBC_NOALLOC_SCRATCH_BYTES (256ull << 20)
bbc_status bbc_count_noalloc(bbc_context* ctx, int32_t n_u, int32_t n_v, int64_t n_edges,
                             const int32_t* edge_u, const int32_t* edge_v,
                             const int8_t* edge_sign, uint32_t flags, bbc_result* out,
                             int64_t* per_vertex);

/*
 * Count many independent graphs in one call (the batched workload).
 *
 * Graph g has vertex sets {0..n_u[g]-1} and {0..n_v[g]-1} and the edges
 * i = edge_offset[g] .. edge_offset[g+1]-1 of the concatenated arrays
 * edge_u / edge_v / edge_sign (ids local to the graph, layout as in
 * bbc_count).  edge_offset has n_graphs + 1 non-decreasing entries.  The size
 * arrays and edge_offset are host memory; the edge arrays are host memory, or
 * device memory with BBC_INPUT_ON_DEVICE.  Only BBC_INPUT_ON_DEVICE is
 * accepted in flags.
 *
 * Every butterfly lies inside one graph, and the method counts it once at its
 * vertex of highest priority (Theorem 1), so the batch is counted as one
 * disjoint union: one relabel and CSR build over all graphs, one planner pass
 * and one persistent wedge-kernel launch whose work items are drawn from all
 * graphs, with totals kept per graph.  The priority inside each graph is the
 * same as in bbc_count, so out[g] equals what bbc_count returns for graph g
 * alone, W included.  Graphs with more than 16384 vertices on a side are
 * counted one at a time inside the call.
 *
 * Outputs (host, n_graphs entries each): status[g] is the bbc_status graph g
 * would get from bbc_count (VERTEX_RANGE, BAD_SIGN, DUPLICATE_EDGE,
 * TOO_LARGE, INVALID_ARG for a negative size, OVERFLOW, OUT_OF_MEMORY);
 * out[g] holds its counts when status[g] == BBC_OK and zeros otherwise.  An
 * invalid graph does not disturb the others.
 *
 * The call returns BBC_OK when every graph got a status, or a call-level error
 * (INVALID_ARG for NULL arrays / decreasing offsets / unknown flags,
 * OUT_OF_MEMORY, DEVICE, INTERNAL) with the outputs unspecified.
 * bbc_last_phase_ms and bbc_last_stats then describe the whole call (sums
 * over its internal passes).
 */
bbc_status bbc_count_batch(bbc_context* ctx, int32_t n_graphs, const int32_t* n_u,
                           const int32_t* n_v, const int64_t* edge_offset, const int32_t* edge_u,
                           const int32_t* edge_v, const int8_t* edge_sign, uint32_t flags,
                           bbc_result* out, int32_t* status);

/*
 * Device workspace a bbc_count of this size may hold at once (bytes; an
 * estimate that errs high), or -1 for sizes bbc_count rejects.
 */
int64_t bbc_workspace_bytes(int32_t n_u, int32_t n_v, int64_t n_edges);

/*
 * Counting service with continuous batching.
 *
 * A server owns worker threads, each with its own context (workspace and HIP
 * stream of default priority) on one device.  Jobs (signed bipartite graphs,
 * host arrays copied at submission) are accepted at any time:
 *   - jobs with at most small_side vertices on each side wait for the
 *     batching worker, which, whenever it is free, takes all waiting small
 *     jobs (up to max_batch_graphs) and counts them with one bbc_count_batch
 *     call; jobs arriving meanwhile form the next batch;
 *   - larger jobs go to large_workers workers running bbc_count
 *     concurrently on their own streams, overlapping on the device with the
 *     batches.
 * Admission by device memory: each worker reserves what its workspace really
 * holds (its arenas stay allocated between jobs), and while it runs jobs the
 * larger of that and their footprint (input plus bbc_workspace_bytes), with
 * its workspace capped at that grant; a worker starts jobs only while the
 * reservations stay within memory_budget.  A job whose workspace turns out
 * larger than its estimate is queued again with the larger footprint; idle
 * workers release their workspace while a job waits for memory; a job larger
 * than the whole budget finishes with BBC_ERR_OUT_OF_MEMORY.  Device memory
 * held by the workers' workspaces therefore stays within memory_budget.
 * Results are exact and do not depend on what else runs.
 *
 * bbc_server_create: cfg may be NULL for defaults (device 0, 2 large workers,
 * budget 90% of the device memory free at creation, small_side 16384,
 * max_batch_graphs 65536; a zero field takes its default).  INVALID_ARG for
 * out of range fields, DEVICE if the device cannot be used.
 * bbc_server_submit: *ticket identifies the job.  INVALID_ARG for bad sizes or
 * NULL arrays, TOO_LARGE as for bbc_count.  Input errors of the graph itself
 * (ids, signs, duplicates) are reported as the job's status.
 * bbc_server_poll: waits up to wait_ms (0: no wait, < 0: until done); returns
 * BBC_PENDING if the job is still queued or running, or BBC_OK with *out,
 * *job_status (the bbc_status of the count) and *latency_ms (submission to
 * completion; may be NULL) filled in, after which the ticket is released.
 * INVALID_ARG for an unknown ticket.
 * bbc_server_stats: up to 12 values: [0] jobs submitted, [1] completed,
 * [2] batches run, [3] jobs counted in batches, [4] largest batch, [5] peak
 * reserved bytes, [6] peak jobs running at once, [7] memory budget, [8] jobs
 * waiting now, [9] bytes reserved now, [10] workspace releases, [11] jobs
 * queued again after outgrowing their estimate.
 * bbc_server_destroy: finishes every submitted job, then releases the server
 * (results not polled are dropped).  NULL is a no-op.
 * One server may be used from several threads at once.
 */
typedef struct bbc_server bbc_server;
typedef struct bbc_server_config {
    int32_t device;
    int32_t large_workers;    /* 0..16 */
    int64_t memory_budget;    /* bytes */
    int32_t small_side;       /* 0..16384 */
    int32_t max_batch_graphs;
} bbc_server_config;
bbc_status bbc_server_create(const bbc_server_config* cfg, bbc_server** out);
bbc_status bbc_server_submit(bbc_server* srv, int32_t n_u, int32_t n_v, int64_t n_edges,
                             const int32_t* edge_u, const int32_t* edge_v,
                             const int8_t* edge_sign, uint64_t* ticket);
bbc_status bbc_server_poll(bbc_server* srv, uint64_t ticket, int32_t wait_ms, bbc_result* out,
                           int32_t* job_status, double* latency_ms);
bbc_status bbc_server_stats(bbc_server* srv, int64_t* stats, int n);
void bbc_server_destroy(bbc_server* srv);

/*
 * Autotuner: pick the work-split tunables for a workload by measurement.
 * The input is laid out as for bbc_count_batch (n_graphs = 1 tunes
 * bbc_count on that graph).  Starting from the context's current settings,
 * a coordinate search tries, in this order, record-chunk floors {16K, 64K,
 * 256K, 1M, 4M} wedges; hash targets {1024, 2048, 4096, 8192} and probe
 * limits {32, 256, 2048} (only when some graph has more than 16384 vertices
 * on a side, the only graphs whose starts are cut into end-vertex tiles);
 * light cuts {512, 1024, 2048}; grab divisors {8, 16, 32}; and, for a batch,
 * union sizes {2^24, 2^26, 2^28, 2^30} edges.  Each setting is timed as the
 * best of `repeats` whole calls (1..100) and a value is kept only for a gain
 * above 3%.  Every call must give the same counts and statuses as the first
 * one (else BBC_ERR_INTERNAL, and the settings are restored).  On success the
 * best settings stay on the context; chosen[0..5] (may be NULL; 6 entries)
 * receives {chunk wedges, hash target, probe limit, light cut, grab divisor,
 * union edges} and *best_ms (may be NULL) the best call time in milliseconds
 * (host clock).
 */
bbc_status bbc_autotune(bbc_context* ctx, int32_t n_graphs, const int32_t* n_u,
                        const int32_t* n_v, const int64_t* edge_offset, const int32_t* edge_u,
                        const int32_t* edge_v, const int8_t* edge_sign, uint32_t flags,
                        int32_t repeats, int64_t* chosen, double* best_ms);

/* Static description of a status code (never NULL). */
const char* bbc_status_string(bbc_status status);

/* Detail of the context's last failure ("" if none; never NULL for a valid ctx). */
const char* bbc_last_error(const bbc_context* ctx);

/* Library version: major * 10000 + minor * 100 + patch. */
int bbc_version(void);

/*
 * Phase timing of the context's last bbc_count, measured with HIP events on the
 * context's stream when timing is enabled (bbc_set_timing(ctx, 1)).
 * phase: 0 = whole device pipeline (first kernel to last),
 *        1 = preprocessing (validation, degrees, priority relabel, CSR build),
 *        2 = wedge enumeration and bucket counting (the wedge kernel alone),
 *        3 = planning (work estimate and work-item construction),
 *        4 = the part of planning that buckets the wedges through short
 *            middle rows of split starts by piece (k_short_wedges; 0 when the
 *            pipeline runs as captured HIP graphs).
 * *ms receives milliseconds.  BBC_ERR_INVALID_ARG for an unknown phase or when
 * timing was off during the last call.
 */
bbc_status bbc_set_timing(bbc_context* ctx, int enabled);
bbc_status bbc_last_phase_ms(const bbc_context* ctx, int phase, double* ms);

/*
 * Work statistics of the last successful bbc_count (for throughput and
 * roofline accounting): stats[0] = number of vertices with at least one
 * edge, [1] = edges, [2] = W, [3] = middle records (oriented edges used as
 * u->v with v below u), [4] = work items run by the wedge kernel,
 * [5] = hashed work pieces whose on-chip table overflowed and that were
 * redone in smaller parts, [6] = start vertices with at least one wedge,
 * [7] = heavy work items (one piece of one start each), [8], [9], [10],
 * [11], [12] = pieces of starts cut into end-vertex tiles: one dense tile
 * (32-bit counters), two dense tiles with 16-bit counters, a hashed run of
 * tiles, four dense tiles with 8-bit counters, eight dense tiles with 4-bit
 * counters; [13] = starts counted by one wavefront alone (small end ranges).
 * `n` is the capacity of `stats`; up to 14 values are written.
 */
bbc_status bbc_last_stats(const bbc_context* ctx, int64_t* stats, int n);

/*
 * Tunable work-split thresholds of a context.  They change how the work is
 * cut into pieces, never the result: every setting in range counts exactly.
 *   BBC_PARAM_HASH_TARGET  expected wedges per hashed run of end-vertex tiles
 *                          of a heavy start (Section 5.2's per-start buckets,
 *                          split along the end-vertex axis); tiles expected to
 *                          hold more get dense counters.  Default 4096, range
 *                          [64, 1048576].
 *   BBC_PARAM_PROBE_LIMIT  hash probes a heavy start's hashed piece tries
 *                          before it gives up; the piece is then redone in
 *                          halves (or densely).  Default 256, range [1, 8192].
 *   BBC_PARAM_CHUNK_WEDGES least wedges per record chunk when a start with a
 *                          small end-vertex range is split over several
 *                          workgroups (partial counts merged exactly by
 *                          C(a+b,2) = C(a,2) + C(b,2) + ab); the chunk is also
 *                          at least W / 2048.  Default 65536, range
 *                          [1024, 2^40].
 *   BBC_PARAM_GRAPHS       1: run the pipeline's two device segments (input
 *                          checks to work totals; work items to results) as
 *                          HIP graphs, captured when a segment's sizes,
 *                          buffers and settings are new and replayed while
 *                          they repeat (e.g. the same batch shape again).
 *                          Results are identical either way.  With timing
 *                          on, phase 1 is then the first segment and phase 2
 *                          the second.  Default 0.
 *   BBC_PARAM_GRAPH_CAPTURES, BBC_PARAM_GRAPH_REPLAYS  (bbc_get_param only)
 *                          segments captured and replayed so far.
 *   BBC_PARAM_LIGHT_MAX    most wedges of a "light" start: light starts share
 *                          work items, each with its own region of one on-chip
 *                          hash table; heavier ones are work items of their
 *                          own.  Default 2048, range [16, 2048].
 *   BBC_PARAM_GRAB_DIV     a work item's records are taken by the waves of its
 *                          workgroup in grabs of about 1/GRAB_DIV of them (light
 *                          items and starts that are not cut along the end
 *                          vertices; capped at 64 records).  Default 16, range
 *                          [4, 64].
 *   BBC_PARAM_UNION_EDGES  bbc_count_batch counts consecutive small graphs
 *                          as one union graph of at most this many edges
 *                          (smaller unions: more passes, but each pass's work
 *                          arrays fit the on-package cache).  Default 2^30,
 *                          range [2^16, 2^30].
 *   BBC_PARAM_WAVE_SHARE   a start whose end vertices fit one wavefront's
 *                          counters (and with at most 65536 wedges) is counted
 *                          by that wavefront alone when its cost, W_u + 8 k_u
 *                          (wedges plus 8 per middle), is at most W /
 *                          WAVE_SHARE of the count's W wedges (but at least
 *                          4096 and at most 32768), so that no wavefront
 *                          keeps counting long after the others; 0 lifts
 *                          this bound.  Default 2048, range [0, 2^20].
 * bbc_set_param returns BBC_ERR_INVALID_ARG for a NULL context, an unknown
 * parameter or a value out of range (the setting is then unchanged);
 * bbc_get_param writes the current value to *value.
 */
enum {
    BBC_PARAM_HASH_TARGET = 1,
    BBC_PARAM_PROBE_LIMIT = 2,
    BBC_PARAM_CHUNK_WEDGES = 3,
    BBC_PARAM_GRAPHS = 4,         /* 0 / 1 */
    BBC_PARAM_GRAPH_CAPTURES = 5, /* read only */
    BBC_PARAM_GRAPH_REPLAYS = 6,  /* read only */
    BBC_PARAM_LIGHT_MAX = 7,
    BBC_PARAM_GRAB_DIV = 8,
    BBC_PARAM_UNION_EDGES = 9,
    BBC_PARAM_WAVE_SHARE = 10
};
bbc_status bbc_set_param(bbc_context* ctx, int param, int64_t value);
bbc_status bbc_get_param(const bbc_context* ctx, int param, int64_t* value);

#ifdef __cplusplus
}
#endif

#endif /* BBC_H */
