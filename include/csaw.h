/*
 * csaw.h -- C-ABI of libcsaw, an MI355X (gfx950) implementation of the hot
 * path of C-SAW (Pandey et al., "C-SAW: A Framework for Graph Sampling and
 * Random Walk on GPUs", SC20, arXiv 2009.09103): bias-based neighbor
 * selection for graph sampling and random walks.
 *
 * The method (paper Sections II-B, III and IV):
 *   - a candidate pool is the adjacency list N(v) of a frontier vertex
 *     (GatherNeighbors, fig:api(b));
 *   - every candidate carries a bias (EdgeBias, Eq. edgebias);
 *   - a candidate is selected with probability proportional to its bias
 *     (Theorem 1) by inverse transform sampling over the prefix sum of the
 *     biases (Section II-B, Eq. equ:tp);
 *   - sampling selects NeighborSize distinct candidates (without
 *     replacement); a draw that hits an already selected candidate is
 *     re-drawn (Section IV-B), and after a fixed number of rounds the
 *     remaining slots draw directly from the prefix with the selected
 *     candidates removed (updated sampling, fig:brs(b), through the inverse
 *     map of Theorem 2, Eq. eq:brs_random);
 *   - Update keeps vertices an instance already visited out of its frontier;
 *     random walks select one candidate per step.
 *
 * Arithmetic is exact: uint32 biases, uint64 prefix sums, a 64-bit draw
 * mapped onto [0, W) by r = floor(u * W / 2^64); no floating point. Random
 * numbers come from Philox4x32-10 (Salmon et al., SC'11) keyed by the call's
 * rng_seed (low 32 bits first) with one counter per draw:
 *   sampling: (instance id mod 2^32, layer, vertex, slot | round << 16),
 *             round 0..CSAW_ROUNDS-1, and round 0xFFFF for the direct draw;
 *   walks:    (walker id mod 2^32, step, vertex, 0).
 * Results therefore depend only on (graph, bias, seeds, fanouts or length,
 * rng_seed, instance / walker ids): not on batching, launch shape, stream or
 * order.
 *
 * Conventions for every entry point:
 *   - Every call returns a csaw_status. No exception crosses the ABI.
 *     csaw_last_error() gives a human-readable message for the calling
 *     thread's last failure.
 *   - "DEVICE" pointers are device memory of the graph's device (for
 *     example a torch tensor's data_ptr()); "HOST" pointers are ordinary host
 *     memory. The caller owns every buffer it passes; the library never
 *     keeps a caller pointer after the call returns.
 *   - stream is a hipStream_t (NULL = the legacy default stream). Work is
 *     enqueued on it; csaw_sample and csaw_walk return after the stream has
 *     finished the call's work, so outputs are ready on return.
 *   - Vertex ids are int32 in [0, n), n < 2^31.
 */
#ifndef CSAW_H
#define CSAW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CSAW_OK = 0,
    CSAW_ERR_INVALID_ARG = 1,    /* bad argument; nothing was written        */
    CSAW_ERR_OUT_OF_MEMORY = 2,  /* device allocation failed, or an output
                                    capacity was too small (counts are still
                                    reported)                                */
    CSAW_ERR_DEVICE = 3,         /* a HIP call failed                         */
    CSAW_ERR_BUSY = 4,           /* server queue full                         */
    CSAW_ERR_NOT_READY = 5,      /* server result not finished yet            */
    CSAW_ERR_UNSUPPORTED = 6,    /* valid but outside this build's limits     */
    CSAW_ERR_CANCELLED = 7       /* server request cancelled before it ran    */
} csaw_status;

/* EdgeBias kinds (Eq. edgebias, Section III-C; Table tbl:samplespace).
 *   UNIFORM          b = 1: unbiased neighbor sampling, DeepWalk.
 *   EDGE_WEIGHT      b = edge_weight[e] given at csaw_graph_create.
 *   NEIGHBOR_DEGREE  b = out-degree of the neighbor: biased neighbor
 *                    sampling and biased DeepWalk (Section II-A).
 *   NODE2VEC         walks only: b = w_return if the neighbor is the previous
 *                    vertex, w_common if it is adjacent to the previous
 *                    vertex, w_outward otherwise (node2vec's second-order
 *                    bias, Section II-A); the first step is unbiased.
 *                    Requires sorted adjacency lists.                      */
typedef enum {
    CSAW_BIAS_UNIFORM = 0,
    CSAW_BIAS_EDGE_WEIGHT = 1,
    CSAW_BIAS_NEIGHBOR_DEGREE = 2,
    CSAW_BIAS_NODE2VEC = 3,
    /* walks only: the Metropolis-Hastings random walk (Section II-A). A
     * uniform neighbor u of v is proposed (counter word 3 = 0) and accepted
     * iff x * deg(u) < deg(v) * 2^32, x in [0, 2^32) drawn with counter
     * (walker id, step, v, 4); a rejected proposal is a step that stays at v.
     * The uniform distribution over vertices is stationary. */
    CSAW_BIAS_METROPOLIS_HASTINGS = 4
} csaw_bias_kind;

/* Fanout value meaning "every neighbor with a positive bias" (snowball). */
#define CSAW_FANOUT_ALL (-1)
/* Largest fanout that is drawn (a fanout >= the number of positive-bias
 * neighbors takes all of them and has no limit). */
#define CSAW_MAX_FANOUT 64
/* Repeated-sampling rounds before the direct draw: the default and the
 * largest value of csaw_sample_args.rounds. */
#define CSAW_ROUNDS 8
/* csaw_sample_args.rounds value for no rounds at all: every slot takes the
 * direct draw from the updated prefix (Theorem 2's inverse) in slot order. */
#define CSAW_DIRECT_ONLY (-1)
/* Most layers per sampling call. */
#define CSAW_MAX_LAYERS 16

typedef struct csaw_graph_s* csaw_graph;
typedef void* csaw_stream; /* hipStream_t */

/* ------------------------------------------------------------------ graph */

/* Upload a CSR graph to the current device; it stays resident in HBM until
 * csaw_graph_destroy (the paper's in-memory setting, Section IV).
 *   num_vertices  n, 0 <= n < 2^31
 *   num_edges     m, 0 <= m < 2^40
 *   rowptr        HOST int64[n+1], rowptr[0] = 0, non-decreasing, rowptr[n] = m
 *   col           HOST int32[m], ids in [0, n); N(v) = col[rowptr[v] .. rowptr[v+1])
 *   edge_weight   HOST uint32[m] or NULL (needed by CSAW_BIAS_EDGE_WEIGHT)
 *   flags         must be 0
 *   stream        used for the uploads; the call synchronises it
 *   out           receives the handle
 * Errors: INVALID_ARG for any violated bound above (checked on the host in
 * O(n + m)); OUT_OF_MEMORY if the device allocations fail. Whether every
 * adjacency list is sorted is recorded; NODE2VEC walks need it. On the
 * device the row offsets are 32-bit words when m < 2^32 and 64-bit
 * otherwise. */
csaw_status csaw_graph_create(int64_t num_vertices, int64_t num_edges, const int64_t* rowptr,
                              const int32_t* col, const uint32_t* edge_weight, uint32_t flags,
                              csaw_stream stream, csaw_graph* out);

/* Free the graph and its device memory. No call on it may be running. */
csaw_status csaw_graph_destroy(csaw_graph g);

/* HOST outputs (each nullable): n, m, largest out-degree, 1 if every
 * adjacency list is sorted. */
csaw_status csaw_graph_info(csaw_graph g, int64_t* num_vertices, int64_t* num_edges,
                            int64_t* max_degree, int32_t* sorted);

/* --------------------------------------------------------------- sampling */

/* Neighbor sampling (fig:api(b) with FrontierSize = all): for every instance
 * i, F_0 = the distinct seeds of i, which are also its visited set; layer l
 * selects fanout(i, l) neighbors of every v in F_l (increasing v) and emits
 * one edge (v, neighbor) per selection; F_{l+1} is the set of selected
 * neighbors that i has not visited, which then become visited (Update,
 * Eq. update). Edges to visited vertices are still emitted. An instance stops
 * at its first zero fanout.
 *
 * Selection at v with biases b over N(v), W = sum b, P = #{b > 0}:
 * W = 0 selects nothing; fanout = CSAW_FANOUT_ALL or fanout >= P selects
 * every positive-bias neighbor in list order; otherwise fanout distinct
 * neighbors drawn as described at the top of this file. */
typedef struct {
    int32_t num_instances;        /* >= 0                                        */
    const int64_t* seed_offsets;  /* HOST int64[num_instances+1], non-decreasing,
                                     seed_offsets[0] = 0                          */
    const int32_t* seeds;         /* DEVICE int32[seed_offsets[num_instances]],
                                     ids in [0, n); duplicates are merged          */
    uint64_t instance_base;       /* instance i has id instance_base + i          */
    int32_t num_layers;           /* 0 .. CSAW_MAX_LAYERS                         */
    const int32_t* fanouts;       /* HOST: int32[num_layers] shared by all
                                     instances if fanout_stride == 0, else row i
                                     at fanouts + i*fanout_stride; values
                                     CSAW_FANOUT_ALL, 0 (stop) or 1..65535;
                                     values above CSAW_MAX_FANOUT are UNSUPPORTED
                                     when they would need a draw                  */
    int32_t fanout_stride;        /* 0, or >= num_layers                          */
    int32_t bias_kind;            /* UNIFORM, EDGE_WEIGHT or NEIGHBOR_DEGREE, used when
                                     bias_kinds is NULL                           */
    const int32_t* bias_kinds;    /* HOST int32[num_instances] or NULL            */
    uint64_t rng_seed;            /* Philox key, used when rng_seeds is NULL      */
    const uint64_t* instance_ids; /* HOST uint64[num_instances] or NULL: instance
                                     i has this id instead of instance_base + i   */
    const uint64_t* rng_seeds;    /* HOST uint64[num_instances] or NULL: a Philox
                                     key per instance, so that instances from
                                     unrelated requests share one call            */
    int32_t rounds;               /* repeated-sampling rounds before the direct
                                     draws (Section IV-B): 0 = CSAW_ROUNDS (the
                                     default), 1..CSAW_ROUNDS, or CSAW_DIRECT_ONLY.
                                     Every value samples the same law; the edges
                                     differ (other draws are used)                */
    uint32_t burn_threshold;      /* forest fire sampling (Section II-A): 0 = off;
                                     else each frontier vertex v takes
                                     NeighborSize = min(G, fanout) (64 for a
                                     fanout of -1), G geometric with
                                     P(G >= j) = (burn_threshold / 2^32)^j, from
                                     Philox trials with counter (instance id,
                                     layer, v, 0xFFFE << 16 | j / 4), word j mod 4:
                                     trial j burns iff the word < burn_threshold   */
} csaw_sample_args;

typedef struct {
    int32_t* src;             /* DEVICE int32[edge_capacity]                       */
    int32_t* dst;             /* DEVICE int32[edge_capacity]                       */
    int64_t edge_capacity;
    int64_t* offsets;         /* DEVICE int64[num_layers*num_instances+1] or NULL:
                                 offsets[l*num_instances + i] is the first edge of
                                 (layer l, instance i); the last entry is the total */
    int64_t num_edges;        /* written: total number of edges                    */
} csaw_sample_out;

/* Output order: by layer, then instance, then source vertex (increasing),
 * then slot. Errors: INVALID_ARG (bad argument, or a seed outside [0, n),
 * detected on the device: outputs are then unspecified); OUT_OF_MEMORY if
 * edge_capacity < the total (num_edges still receives the total; edges that
 * fit are written); UNSUPPORTED for a drawn fanout above CSAW_MAX_FANOUT. */
csaw_status csaw_sample(csaw_graph g, const csaw_sample_args* args, csaw_sample_out* out,
                        csaw_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): csaw_sample
 * with the same arguments, outputs and errors, whose device scratch (frontier
 * arrays, tables, control block, instance bitmaps) is one array of
 * CSAW_NOALLOC_SCRATCH_BYTES per device, held by the library until the
 * process ends. It calls no hipMalloc, hipFree, hipHostMalloc or allocator
 * callback (host-side bookkeeping uses ordinary heap memory), captures no
 * launch sequence and runs every kernel on `stream`. Calls on one device are
 * serialised by the library (the array keeps the last call's contents; each
 * call clears what must start at zero), so overlapping calls wait for each
 * other rather than race.
 * Errors, beyond those of csaw_sample: OUT_OF_MEMORY (before any device work)
 * when the call's scratch -- sized from the seed counts, fanouts and n like
 * csaw_sample_bound -- exceeds CSAW_NOALLOC_SCRATCH_BYTES; NOT_READY if a
 * NEIGHBOR_DEGREE instance needs the graph's degree tables before any
 * csaw_sample or csaw_walk call has built them (building them allocates). */
#define CSAW_NOALLOC_SCRATCH_BYTES (128ll << 20)
csaw_status csaw_sample_noalloc(csaw_graph g, const csaw_sample_args* args, csaw_sample_out* out,
                                csaw_stream stream);

/* Upper bound of the number of edges csaw_sample can emit for these
 * arguments (capacity planning; host-only, seeds are not read).
 * HOST out: max_edges. */
csaw_status csaw_sample_bound(csaw_graph g, const csaw_sample_args* args, int64_t* max_edges);

/* Work assignment of the sampling kernel by degree bucket (the frontier
 * queue of Section III-A, with sub-wave groups for small lists). A frontier
 * entry whose work -- the candidates of a take-all list or of a weighted
 * draw, the slots of an unbiased draw -- is at most bound16 is served by 16
 * lanes, four entries to a wavefront; at most bound32, by 32 lanes; the
 * others by a whole wavefront (or the long-list path). 0 turns a bucket off.
 * Results never depend on these bounds (the draws are keyed by their
 * counters and taken in slot order either way); only the speed does.
 * The setting belongs to the graph and applies to later calls. */
typedef struct {
    int32_t bound16;              /* [0, 16], default 16                          */
    int32_t bound32;              /* [0, 32], default 32                          */
} csaw_tuning;

/* INVALID_ARG if a bound is outside its range. A call already running keeps
 * the setting it started with; calls from several threads may see either
 * setting, with the same results. */
csaw_status csaw_set_tuning(csaw_graph g, const csaw_tuning* tuning);
/* HOST out: tuning. */
csaw_status csaw_get_tuning(csaw_graph g, csaw_tuning* tuning);

/* Autotuner: runs csaw_sample(g, args, out, stream) under each candidate
 * setting (warm-up call, then `reps` timed calls; reps in [1, 100]), keeps
 * the fastest median on the graph and writes it to *chosen (HOST, nullable).
 * Other calls on the same graph while it runs use whichever candidate is
 * current; their results are unchanged.
 * The outputs are those of csaw_sample, identical under every setting. An
 * error of any call is returned as is (the graph keeps its previous setting). */
csaw_status csaw_autotune_sample(csaw_graph g, const csaw_sample_args* args, csaw_sample_out* out, int32_t reps,
                                 csaw_stream stream, csaw_tuning* chosen);

/* ------------------------------------------------------------------ walks */

/* Random walks (Section II-A: DeepWalk, biased DeepWalk, node2vec,
 * multi-independent walks). Walker w (id walker_base + w) starts at
 * starts[w]; at each step from v the biases of N(v) are evaluated; if v has no
 * neighbor or W = 0 the walk stops, otherwise one neighbor is drawn (with
 * replacement) and the walker moves there. */
typedef struct {
    int32_t bias_kind;            /* csaw_bias_kind                               */
    uint32_t w_return;            /* NODE2VEC weights (uint32)                    */
    uint32_t w_common;
    uint32_t w_outward;
    int64_t num_walkers;          /* >= 0                                         */
    const int32_t* starts;        /* DEVICE int32[num_walkers], ids in [0, n)     */
    uint64_t walker_base;         /* walker w has id walker_base + w              */
    int32_t length;               /* number of steps, >= 0                        */
    uint64_t rng_seed;            /* Philox key                                   */
    const uint64_t* walker_ids;   /* DEVICE uint64[num_walkers] or NULL: walker w
                                     has this id instead of walker_base + w (an
                                     exact subset of a larger run)                */
    uint32_t restart_threshold;   /* random walk with restart / with jump
                                     (Section II-A): each step first draws x in
                                     [0, 2^32) (counter (walker id, step, v, 2));
                                     x < restart_threshold moves the walker back to
                                     its start, x < restart_threshold +
                                     jump_threshold to a vertex drawn in [0, n)
                                     (counter (walker id, step, v, 3)); such a move
                                     is a step and forgets the previous vertex.
                                     Both 0: plain walks. Their sum is at most 2^32 */
    uint32_t jump_threshold;
} csaw_walk_args;

/* paths: DEVICE int32[num_walkers * (length+1)], walker-major; path[0] is
 * the start, entries after a stop are -1.
 * total_steps: HOST int64 or NULL, receives the number of steps taken by all
 * walkers (sampled edges).
 * Errors: INVALID_ARG (bad argument, unsorted lists for NODE2VEC, NODE2VEC
 * on a graph where some edge (u, x) has no reverse edge (x, u) -- checked on
 * the device by the graph's first NODE2VEC walk, then remembered -- missing
 * edge weights, or a start outside [0, n) detected on the device). */
csaw_status csaw_walk(csaw_graph g, const csaw_walk_args* args, int32_t* paths,
                      int64_t* total_steps, csaw_stream stream);

/* Walk guide (weighted first-order walks, EDGE_WEIGHT and NEIGHBOR_DEGREE;
 * the inverse transform selection of Section II-B, Eq. equ:tp, served in
 * a constant expected number of loads). On a weight
 * array's first walk the graph builds, once: the exact inclusive prefix of
 * every edge in its list (8 bytes per edge), and per list of total W and
 * degree d a table of K <= 2 d equal buckets of width 2^s over [0, W), each
 * holding the first position whose interval reaches its start, with that
 * position's prefix and neighbor (16 bytes per bucket, 2 m + n entries),
 * and per vertex its list and W (16 bytes, when m < 2^32). A step's draw r
 * then lies between the positions of buckets r >> s and (r >> s) + 1, and
 * m = #{i : S_(i+1) <= r} follows from the two buckets or a few exact
 * prefixes: the same pick as a search of the whole prefix. About 48 bytes
 * per edge per weight array (51 GB for 2^30 edges); with the guide off (or
 * not yet built in a caller memory call) walks take the chunk tables with
 * one wavefront per walker, with the same paths. Sampling calls draw from
 * the long lists (more than 512 edges) of a weight array through its guide
 * when it is built and on (a walk or a server builds it), else through the
 * chunk tables: the same edges either way.
 * enable: 1 (default) or 0. A walk already running keeps its route. INVALID_ARG
 * otherwise. Turning the guide off does not free built tables. */
csaw_status csaw_set_walk_guides(csaw_graph g, int32_t enable);
/* HOST out: enable. */
csaw_status csaw_get_walk_guides(csaw_graph g, int32_t* enable);

/* ------------------------------------------- multi-dimensional random walk */

/* Multi-dimensional random walk, a.k.a. frontier sampling (Section II-A;
 * the VertexBias select site of fig:api(b); example fig:layer_example).
 * Instance i (id instance_base + i) keeps a pool of
 * P_i = pool_offsets[i+1] - pool_offsets[i] vertices (the FrontierPool),
 * initially pool[pool_offsets[i] .. pool_offsets[i+1]). At step
 * s = 0 .. budget-1 one pool vertex v is selected with probability
 * deg(v) / (total pool degree) (VertexBias = out-degree, Philox counter
 * (instance id, s, 0xFFFFFFFF, 0) over the degree prefix in pool order),
 * one neighbor u of v uniformly (counter (instance id, s, v, 1)), the edge
 * (v, u) is sampled and u replaces v in the pool (Update). An instance whose
 * pool has total degree 0 ends. */
#define CSAW_MAX_POOL 2048

typedef struct {
    int32_t num_instances;        /* >= 0                                         */
    const int64_t* pool_offsets;  /* HOST int64[num_instances+1], non-decreasing,
                                     pool_offsets[0] = 0, every pool of at most
                                     CSAW_MAX_POOL vertices                       */
    const int32_t* pool;          /* DEVICE int32[pool_offsets[num_instances]],
                                     ids in [0, n)                                */
    uint64_t instance_base;       /* instance i has id instance_base + i          */
    int64_t budget;               /* edges sampled per instance, >= 0             */
    uint64_t rng_seed;            /* Philox key                                   */
} csaw_mdrw_args;

/* src, dst: DEVICE int32[num_instances * budget], instance-major in step
 * order; entries after an instance has ended are -1.
 * steps: DEVICE int64[num_instances] or NULL: edges sampled per instance.
 * total_edges: HOST int64 or NULL: edges sampled by all instances.
 * Errors: INVALID_ARG (bad argument, or a pool vertex outside [0, n)
 * detected on the device: outputs are then unspecified); UNSUPPORTED for a
 * pool larger than CSAW_MAX_POOL. */
csaw_status csaw_mdrw(csaw_graph g, const csaw_mdrw_args* args, int32_t* src, int32_t* dst, int64_t* steps,
                      int64_t* total_edges, csaw_stream stream);

/* ---------------------------------------------------------- layer sampling */

/* Layer sampling (Section II-A: a constant number of neighbors selected for
 * the whole frontier in each round). Instance i (id instance_base + i)
 * starts from its seeds F_0 (sorted, distinct, at most CSAW_MAX_POOL) and
 * visits them. Layer l: the lists N(v) of v in F_l, concatenated in
 * increasing v, form one candidate list with the call's EdgeBias;
 * min(fanouts[l], P) distinct candidates are selected from it as from one
 * adjacency list (every positive one when the fanout reaches P), with
 * counter (instance id, layer, 0xFFFFFFFF, slot | round << 16); slot j is
 * the edge (owner, neighbor). F_{l+1} = the picked neighbors not visited
 * (sorted, distinct), which are then visited. */
typedef struct {
    int32_t num_instances;        /* >= 0                                         */
    const int64_t* seed_offsets;  /* HOST int64[num_instances+1], non-decreasing,
                                     seed_offsets[0] = 0                           */
    const int32_t* seeds;         /* DEVICE int32: each instance's seeds sorted
                                     and distinct, ids in [0, n)                   */
    uint64_t instance_base;
    int32_t num_layers;           /* 0 .. CSAW_MAX_LAYERS                          */
    const int32_t* fanouts;       /* HOST int32[num_layers], each 1..64            */
    int32_t bias_kind;            /* UNIFORM, EDGE_WEIGHT or NEIGHBOR_DEGREE       */
    uint64_t rng_seed;
    int32_t rounds;               /* as csaw_sample_args.rounds                    */
} csaw_layer_args;

/* DEVICE outputs: src/dst int32[num_instances][num_layers][K] with K = the
 * largest fanout, slot order, -1 past the count; counts
 * int32[num_instances][num_layers]. Errors: INVALID_ARG (bad argument, or
 * seeds out of range, unsorted or repeated, detected on the device: outputs
 * are then unspecified); UNSUPPORTED for more than CSAW_MAX_POOL seeds in an
 * instance. */
csaw_status csaw_layer_sample(csaw_graph g, const csaw_layer_args* args, int32_t* src, int32_t* dst,
                              int32_t* counts, csaw_stream stream);

/* ---------------------------------------------------------- out of memory */

/* A graph larger than device memory (Section V, out-of-memory sampling):
 * the adjacency and edge weights stay in pinned host memory, split into
 * num_partitions vertex ranges of about m / num_partitions edges each; the
 * row offsets and per-vertex tables are resident. At most max_resident
 * partitions are on the device at once (one slot each, sized for the largest
 * partition). csaw_sample_streamed loads, for every layer, the partitions
 * that hold frontier vertices with edges to sample, busiest first (most
 * edges), those already resident before the others, each load overlapping
 * the previous partition's selection on a second stream; the selection of a
 * partition's frontier vertices runs while it is resident. Results are
 * bit-identical to csaw_sample on the same graph.
 *   arguments as csaw_graph_create, plus
 *   num_partitions  1..64
 *   max_resident    1..num_partitions
 * Errors: INVALID_ARG (bad CSR or counts), OUT_OF_MEMORY (device slots or
 * pinned host copies). The graph's degree bias tables are built here, one
 * partition at a time. */
typedef struct csaw_pgraph_s* csaw_pgraph;
csaw_status csaw_pgraph_create(int64_t num_vertices, int64_t num_edges, const int64_t* rowptr, const int32_t* col,
                               const uint32_t* edge_weight, int32_t num_partitions, int32_t max_resident,
                               csaw_stream stream, csaw_pgraph* out);
csaw_status csaw_pgraph_destroy(csaw_pgraph g);

typedef struct {
    int64_t partition_loads;      /* partitions loaded into a device slot       */
    int64_t bytes_loaded;         /* host-to-device bytes of those loads        */
} csaw_stream_stats;

/* csaw_sample on a partitioned graph: same arguments, outputs and errors;
 * stats (HOST, nullable) receives the call's partition loads. One call runs
 * at a time per graph (others wait). */
csaw_status csaw_sample_streamed(csaw_pgraph g, const csaw_sample_args* args, csaw_sample_out* out,
                                 csaw_stream stream, csaw_stream_stats* stats);

/* ------------------------------------------------------- device scratch */

/* Device scratch of the calls (each graph's workspaces: per-call frontier and
 * edge-count arrays, instance bitmaps) comes from alloc_fn (bytes, user),
 * which returns a device pointer or NULL (the call then fails with
 * OUT_OF_MEMORY); a buffer is returned with the free_fn that was set when it
 * was allocated, once no work uses it (at a workspace's growth or at
 * csaw_graph_destroy), so a pair must stay valid until every graph that used
 * it is destroyed. Both NULL (the default): hipMalloc / hipFree. The graph's
 * own arrays (CSR, weights, tables) always use hipMalloc. Process-wide; it
 * applies from the next allocation. INVALID_ARG if only one of the two is
 * NULL. */
typedef void* (*csaw_alloc_fn)(size_t bytes, void* user);
typedef void (*csaw_free_fn)(void* ptr, void* user);
csaw_status csaw_set_allocator(csaw_alloc_fn alloc_fn, csaw_free_fn free_fn, void* user);

/* ---------------------------------------------------------------- serving */

/* A request server over one resident graph (the batched multi-instance
 * setting of Section V taken to a request stream): requests -- one sampling
 * instance or one batch of walkers each -- are submitted from any thread with
 * host inputs. Executor threads, each with its own stream and one block of
 * device memory allocated when the server is created, take the request at the
 * head of the queue and, if it is a sampling request, every waiting sampling
 * request whose addition keeps the batch's exact device need (seeds, edge
 * outputs, offsets, frontiers, instance bitmaps) within the block, into one
 * multi-instance csaw_sample-equivalent call (continuous batching); a walk
 * request takes every waiting walk request of the same bias kind and node2vec
 * weights whose paths and tables still fit the block into one launch, each
 * walker keyed by its own request's rng_seed, id and length. Requests that
 * arrive while others run are
 * admitted as executors and memory free up, and their work overlaps on the
 * device. Serving allocates no device memory: the server holds exactly the
 * blocks it allocated at creation. A request's result is bit-identical to
 * running it alone: its draws are keyed by its own id and rng_seed. If a batch
 * fails, its requests are run again one by one, so that only a faulty request
 * reports an error. */
typedef struct csaw_server_s* csaw_server;

typedef struct {
    int64_t memory_budget_bytes;  /* device memory the server allocates at creation,
                                     split evenly among its executors (0: 32 GiB) */
    int32_t max_batch;            /* most sampling requests per call (0: 512)        */
    int32_t queue_capacity;       /* most waiting requests before BUSY (0: 65536)    */
    int32_t num_streams;          /* executor threads/streams, 1..16 (0: 2)          */
    int64_t max_batch_walkers;    /* most walkers per walk call; a single larger
                                     request still runs alone (0: 262144)          */
    int64_t result_pool_bytes;    /* pinned host memory allocated at creation for
                                     result arrays: walk paths are copied from the
                                     device straight into them, the rest without
                                     page faults; arrays that do not fit come from
                                     the heap, through staging (0: none)          */
} csaw_server_config;

typedef enum { CSAW_REQUEST_SAMPLE = 0, CSAW_REQUEST_WALK = 1 } csaw_request_kind;

typedef struct {
    int32_t kind;                 /* csaw_request_kind                             */
    uint64_t id;                  /* sampling: instance id; walks: id of walker 0  */
    uint64_t rng_seed;            /* Philox key                                    */
    int32_t bias_kind;            /* csaw_bias_kind                                */
    /* sampling */
    const int32_t* seeds;         /* HOST int32[num_seeds], copied at submit       */
    int64_t num_seeds;
    const int32_t* fanouts;       /* HOST int32[num_layers], copied at submit      */
    int32_t num_layers;
    /* walks */
    const int32_t* starts;        /* HOST int32[num_walkers], copied at submit     */
    int64_t num_walkers;
    int32_t length;
    uint32_t w_return, w_common, w_outward;
} csaw_request;

typedef struct {
    csaw_status status;           /* outcome of this request                       */
    int32_t kind;
    /* sampling: edges in (layer, source, slot) order; layer l is
       [layer_offsets[l], layer_offsets[l+1]) */
    int64_t num_edges;
    int32_t* src;
    int32_t* dst;
    int32_t num_layers;
    int64_t* layer_offsets;
    /* walks: int32[num_walkers * (length+1)], -1 after a stop */
    int32_t* paths;
    int64_t num_walkers;
    int32_t length;
    int64_t steps;                /* sampled edges of a walk request               */
    /* latency, microseconds from submit */
    double queued_us;             /* until its batch started                       */
    double total_us;              /* until its result was in host memory           */
    int32_t batch_requests;       /* requests served by the same call (1: alone)   */
} csaw_result;

/* Errors: INVALID_ARG (bad config); OUT_OF_MEMORY if the executors' device
 * blocks or pinned staging buffers cannot be allocated. Builds the graph's
 * degree (and edge-weight) tables first, so that no request does. The server
 * keeps g; g must outlive it. */
csaw_status csaw_server_create(csaw_graph g, const csaw_server_config* cfg, csaw_server* out);
/* Validates and copies the request (INVALID_ARG: bad ids, bias kind, sizes;
 * OUT_OF_MEMORY: the request alone needs more device memory than one
 * executor's block; BUSY: queue full). HOST out: ticket, used to fetch the
 * result. */
csaw_status csaw_server_submit(csaw_server s, const csaw_request* req, uint64_t* ticket);
/* NOT_READY until the request is done; then hands over *result (the caller
 * frees it with csaw_result_free). INVALID_ARG for an unknown ticket. */
csaw_status csaw_server_poll(csaw_server s, uint64_t ticket, csaw_result** result);
/* As poll, but waits up to timeout_us (< 0: no limit). */
csaw_status csaw_server_wait(csaw_server s, uint64_t ticket, int64_t timeout_us, csaw_result** result);
void csaw_result_free(csaw_result* r);
/* Withdraws a request that has not started: its result (fetched with poll or
 * wait as usual) then has status CANCELLED. BUSY if it is already running or
 * done; INVALID_ARG for an unknown ticket. */
csaw_status csaw_server_cancel(csaw_server s, uint64_t ticket);
/* HOST outputs (each nullable): device bytes and pinned host bytes the server
 * holds (fixed from creation to destruction); the result pool
 * (result_pool_bytes) is held on top, until the server and the last result
 * using it are freed. */
csaw_status csaw_server_memory(csaw_server s, int64_t* device_bytes, int64_t* pinned_host_bytes);
/* Finishes every submitted request, stops the executors and frees the
 * server. Results not fetched are freed. */
csaw_status csaw_server_destroy(csaw_server s);

/* --------------------------------------------------------------- profiling */

/* When enabled, the library brackets each kernel launch with HIP events on
 * the stream the kernel runs on, so that kernel time can be read without an
 * external profiler. Process-wide; off by default. */
csaw_status csaw_profile_enable(int32_t on);
csaw_status csaw_profile_reset(void);
/* Sum of event-measured durations (ms) and launch count of the kernels whose
 * name starts with `prefix` since the last reset. Synchronises the events.
 * HOST outputs. */
csaw_status csaw_profile_read(const char* prefix, double* total_ms, int64_t* launches);

/* ------------------------------------------------------------------- misc */

/* Message of the calling thread's last failed call ("" if none). The string
 * stays valid until the thread's next call into the library. */
const char* csaw_last_error(void);

/* Library version string (static storage). */
const char* csaw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CSAW_H */
