/*
 * csaw_oracle.c -- CPU ORACLE for C-SAW's bias-based vertex selection
 * (Pandey, Li, Hoisie, Li, Liu: "C-SAW: A Framework for Graph Sampling and
 * Random Walk on GPUs", SC20, arXiv 2009.09103).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the definition that the GPU
 * library is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product path never does. It
 * shares no code, header, table or constant generator with the GPU library:
 * every constant below is restated here from its published source.
 *
 * Plain, slow and obviously correct on purpose: linear scans instead of
 * binary searches, a byte-marker array instead of a bitmap, one sequential
 * loop per definition. OpenMP only runs independent work on separate
 * threads -- instances, walkers, or the vertices of one frontier (whose
 * selections use their own counters) -- and every result is identical to a
 * serial run.
 *
 * What is computed (each function cites the passage it follows):
 *   - Theorem 1 (Section II-B): a candidate is drawn with probability
 *     proportional to its bias b_k.
 *   - Inverse transform sampling over the exclusive prefix sum S of the
 *     biases (Section II-B, Eq. equ:tp, worked example of fig:example(b)),
 *     in exact integers: no normalisation by the total, r drawn in [0, W).
 *   - Sampling without replacement (Section II-A, traversal-based sampling)
 *     by repeated sampling (Section IV-B, "naive solutions", fig:brs(a)) for
 *     a fixed number of rounds, then the inverse map of Theorem 2
 *     (Eq. eq:brs_random) generalised to any number of pre-selected
 *     candidates, in integers, which draws directly from the updated CTPS
 *     (fig:brs(b)).
 *   - The generic sampling loop of fig:api(b): GatherNeighbors, EdgeBias,
 *     Select(NeighborSize), Update (visited filter), Sampled append.
 *   - Random walks (Section II-A): first-order biased walks, node2vec and
 *     the Metropolis-Hastings walk.
 *
 * Parity status of each function is listed in its comment ("pinned by").
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------
 * Bias kinds (EdgeBias, Eq. edgebias, Section III-C).
 *   UNIFORM          b = 1 (unbiased neighbor sampling, DeepWalk)
 *   EDGE_WEIGHT      b = caller-supplied uint32 weight of the edge
 *   NEIGHBOR_DEGREE  b = out-degree of the neighbor (biased DeepWalk and
 *                    biased neighbor sampling use the degree as the bias,
 *                    Section II-A and fig:example(a))
 *   NODE2VEC         b = w_return if x is the previous vertex, w_common if x
 *                    is adjacent to the previous vertex, else w_outward
 *                    (node2vec's distance-based bias, Section II-A); the
 *                    first step of a walk has no previous vertex and is
 *                    unbiased.
 * ------------------------------------------------------------------------- */
enum { ORC_UNIFORM = 0, ORC_EDGE_WEIGHT = 1, ORC_NEIGHBOR_DEGREE = 2, ORC_NODE2VEC = 3, ORC_METROPOLIS = 4 };

/* Round index reserved for the exact conditional draw. */
#define ORC_FALLBACK_ROUND 0xFFFFu
#define ORC_BURN_ROUND 0xFFFEu      /* counter word 3 of the forest fire trials */
#define ORC_BURN_CAP_ALL 64         /* burning cap of a fanout of -1 */

/* ---------------------------------------------------------------------------
 * Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As
 * Easy as 1, 2, 3", SC'11. Ten rounds of the 4x32 Philox S-box with
 * multipliers 0xD2511F53 and 0xCD9E8D57 and Weyl key increments 0x9E3779B9
 * and 0xBB67AE85 (the golden ratio and sqrt(3)-1 in 32-bit fixed point).
 * The paper itself uses cuRAND (Section VI); any counter-based generator
 * serves, and this one keeps every draw a pure function of its counter.
 * Pinned by: agreement with an independent implementation (PyTorch's
 * at::philox_engine) over many keys and counters; bit balance; chi-square.
 * ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t key_in[2], const uint32_t ctr_in[4], uint32_t out[4])
{
    uint32_t k0 = key_in[0], k1 = key_in[1];
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* r = floor(u * W / 2^64): maps a uniform 64-bit word onto [0, W) with
 * every value receiving floor(2^64/W) or ceil(2^64/W) preimages. This is
 * the integer stand-in for "generate r in (0,1) and search the CTPS"
 * (Section II-B) -- searching floor(r*W) in S is searching r in F = S/W.
 * Pinned by: exact 128-bit reference arithmetic in Python on random and
 * extreme operands; closed form for powers of two. */
uint64_t orc_range(uint64_t u, uint64_t W)
{
    unsigned __int128 p = (unsigned __int128)u * (unsigned __int128)W;
    return (uint64_t)(p >> 64);
}

/* One draw: key = rng_seed split in 32-bit halves (low half first),
 * counter = (c0, c1, c2, c3); u = x0 + 2^32 x1. */
uint64_t orc_draw(uint64_t rng_seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t W)
{
    uint32_t key[2] = {(uint32_t)rng_seed, (uint32_t)(rng_seed >> 32)};
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t x[4];
    orc_philox4x32_10(key, ctr, x);
    uint64_t u = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    return orc_range(u, W);
}

/* Exclusive prefix sum of the biases, S[0] = 0, S[i+1] = S[i] + b_i,
 * S[d] = W (Section II-B; the printed example S = {0,3,9,11,13,15} for
 * b = (3,6,2,2,2) fixes the exclusive convention). uint64 cannot overflow:
 * d < 2^31 and b < 2^32. */
static void prefix(const uint32_t* b, int64_t d, uint64_t* S)
{
    S[0] = 0;
    for (int64_t i = 0; i < d; ++i) S[i + 1] = S[i] + (uint64_t)b[i];
}

void orc_prefix(const uint32_t* b, int64_t d, uint64_t* S) { prefix(b, d, S); }

/* Inverse transform search, by definition: the selected candidate is the
 * one whose region [S_i, S_{i+1}) contains r, i.e. the largest i in [0, d)
 * with S_i <= r (Section II-B, fig:example(b)). A zero bias owns an empty
 * region and is never returned. Linear scan: the oracle does not need the
 * binary search the paper uses for speed.
 * Pinned by: exhaustive preimage counts (#{r : m(r) = i} = b_i) and the
 * paper's worked example (r = 0.5 selects v7). */
int64_t orc_its(const uint64_t* S, int64_t d, uint64_t r)
{
    int64_t m = 0;
    for (int64_t i = 0; i < d; ++i)
        if (S[i] <= r) m = i;
    return m;
}

/* Inverse map of Theorem 2 (Eq. eq:brs_random) generalised to a set A of
 * pre-selected candidates and written in integers. r is a draw in
 * [0, W - sum_{s in A} b_s), i.e. a position in the updated CTPS that omits
 * A (fig:brs(b)). Walking A in increasing position, every pre-selected
 * region that starts at or before the running r is stepped over by adding
 * its width; the result is the position in the original CTPS that updated
 * sampling would select (for one pre-selected vertex this is exactly
 * F = F'/lambda + delta when k > s and F = F'/lambda when k < s).
 * acc_sorted lists A in increasing position.
 * Pinned by: brute force against inverse transform search over an
 * explicitly rebuilt list without A, for every r, on many random lists;
 * the paper's example (v7 pre-selected, r = 0.58 -> v10). */
uint64_t orc_skip_map(const uint64_t* S, const uint32_t* b, const int64_t* acc_sorted,
                      int32_t na, uint64_t r)
{
    for (int32_t t = 0; t < na; ++t) {
        int64_t s = acc_sorted[t];
        if (S[s] <= r) r += (uint64_t)b[s];
    }
    return r;
}

/*
 * Select up to k distinct candidates out of d with biases b (the Select
 * step of the generic loop of fig:api(b), for one frontier vertex).
 *
 *   W = sum b, P = #{i : b_i > 0}.
 *   W == 0            -> nothing is selected.
 *   k >= P (or k < 0) -> every positive-bias candidate, in list order
 *                        (NeighborSize at least the pool: snowball case).
 *   otherwise         -> k slots j = 0..k-1:
 *     rounds a = 0..rounds-1: every slot that is still open, in increasing
 *       j, draws r with counter (c0, c1, c2, j | a << 16) and takes
 *       m = its(r); the slot keeps m unless m is already held by a slot
 *       (from an earlier round, or a lower slot of this round) -- the
 *       repeated sampling of fig:brs(a) with collisions settled in slot
 *       order;
 *     then every slot still open, in increasing j, draws r in
 *       [0, W - sum_{held} b) with counter (c0, c1, c2, j | 0xFFFF << 16),
 *       maps it through orc_skip_map and takes m = its(r): a direct draw
 *       from the updated CTPS (fig:brs(b)).
 *   Both steps give the next new candidate with probability proportional to
 *   its bias among the ones not yet held, so the held set follows the
 *   updated-sampling law regardless of how many rounds ran.
 *
 * pos_out receives min(k, P) positions in slot order. Returns that count.
 * *n_fallback (nullable) receives the number of slots that needed the
 * direct draw, *n_draws (nullable) the number of draws of either kind (the
 * attempts of the selection; counting only, no effect on the result).
 * Pinned by: chi-square of set frequencies against the exact successive-
 * sampling probabilities (enumerated), for rounds = 0 and rounds = 8,
 * including a skewed case that always reaches the direct draw; invariants
 * (distinct, positive bias, exactly min(k, P)); weight-scale invariance.
 */
int32_t orc_select(const uint32_t* b, int64_t d, int64_t k, int32_t rounds,
                   uint64_t rng_seed, uint32_t c0, uint32_t c1, uint32_t c2,
                   int64_t* pos_out, int32_t* n_fallback, int64_t* n_draws)
{
    if (n_fallback) *n_fallback = 0;
    if (n_draws) *n_draws = 0;
    if (d <= 0) return 0;
    uint64_t* S = (uint64_t*)malloc((size_t)(d + 1) * sizeof(uint64_t));
    prefix(b, d, S);
    const uint64_t W = S[d];
    int64_t P = 0;
    for (int64_t i = 0; i < d; ++i) P += (b[i] > 0);
    if (W == 0) { free(S); return 0; }
    if (k < 0 || k >= P) {
        int32_t c = 0;
        for (int64_t i = 0; i < d; ++i)
            if (b[i] > 0) pos_out[c++] = i;
        free(S);
        return c;
    }
    int64_t* held = pos_out; /* held[j] = position of slot j, -1 while open */
    for (int64_t j = 0; j < k; ++j) held[j] = -1;

    for (int32_t a = 0; a < rounds; ++a) {
        int open = 0;
        for (int64_t j = 0; j < k; ++j) {
            if (held[j] >= 0) continue;
            uint64_t r = orc_draw(rng_seed, c0, c1, c2, (uint32_t)j | ((uint32_t)a << 16), W);
            if (n_draws) ++*n_draws;
            int64_t m = orc_its(S, d, r);
            int taken = 0;
            for (int64_t q = 0; q < k; ++q)
                if (held[q] == m) { taken = 1; break; }
            if (!taken) held[j] = m;
            else open = 1;
        }
        if (!open) break;
    }

    int64_t* acc = (int64_t*)malloc((size_t)k * sizeof(int64_t));
    for (int64_t j = 0; j < k; ++j) {
        if (held[j] >= 0) continue;
        /* held set in increasing position, and the mass it removes */
        int32_t na = 0;
        uint64_t removed = 0;
        for (int64_t q = 0; q < k; ++q)
            if (held[q] >= 0) { acc[na++] = held[q]; removed += b[held[q]]; }
        for (int32_t x = 1; x < na; ++x) {           /* insertion sort */
            int64_t v = acc[x];
            int32_t y = x - 1;
            while (y >= 0 && acc[y] > v) { acc[y + 1] = acc[y]; --y; }
            acc[y + 1] = v;
        }
        uint64_t r = orc_draw(rng_seed, c0, c1, c2, (uint32_t)j | (ORC_FALLBACK_ROUND << 16), W - removed);
        r = orc_skip_map(S, b, acc, na, r);
        held[j] = orc_its(S, d, r);
        if (n_fallback) ++*n_fallback;
        if (n_draws) ++*n_draws;
    }
    free(acc);
    free(S);
    return (int32_t)k;
}

/*
 * Forest fire NeighborSize (Section II-A names forest fire sampling as
 * neighbor sampling with a variable number of neighbors per vertex set by a
 * burning probability; the rule is Leskovec and Faloutsos, KDD'06): a vertex
 * burns G neighbors, G geometric with P(G >= j) = p^j, p = burn / 2^32,
 * capped at cap. Trial j = 0, 1, ... succeeds iff word (j mod 4) of the
 * Philox block with counter (c0, c1, c2, 0xFFFE << 16 | j / 4) is below
 * burn; G is the number of successes before the first failure, or cap.
 * Pinned by: the capped geometric law (chi-square over many vertices), the
 * counter layout replayed with the independent Philox, and the two ends
 * (burn = 2^32 - 1 burns cap neighbors, burn = 0 none).
 */
int32_t orc_burn_count(uint64_t rng_seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t burn, int32_t cap)
{
    uint32_t key[2] = {(uint32_t)rng_seed, (uint32_t)(rng_seed >> 32)};
    int32_t g = 0;
    for (uint32_t blk = 0; g < cap; ++blk) {
        uint32_t ctr[4] = {c0, c1, c2, (ORC_BURN_ROUND << 16) | blk};
        uint32_t x[4];
        orc_philox4x32_10(key, ctr, x);
        for (int w = 0; w < 4 && g < cap; ++w) {
            if (x[w] >= burn) return g;
            ++g;
        }
    }
    return g;
}

/* ---------------------------------------------------------------------------
 * Graph helpers. CSR: rowptr int64[n+1], col int32[m]; adjacency lists are
 * sorted. GatherNeighbors (fig:api(b)) of v is col[rowptr[v] ..
 * rowptr[v+1]).
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    const int64_t* rowptr;
    const int32_t* col;
    const uint32_t* ew;   /* nullable */
} orc_graph;

static inline int64_t deg(const orc_graph* g, int64_t v) { return g->rowptr[v + 1] - g->rowptr[v]; }

/* EdgeBias for the static kinds over the list of v (Eq. edgebias). */
static int edge_bias_static(const orc_graph* g, int32_t kind, int64_t v, uint32_t* b)
{
    int64_t beg = g->rowptr[v], d = deg(g, v);
    for (int64_t i = 0; i < d; ++i) {
        int64_t e = beg + i;
        switch (kind) {
        case ORC_UNIFORM: b[i] = 1; break;
        case ORC_EDGE_WEIGHT:
            if (!g->ew) return -1;
            b[i] = g->ew[e];
            break;
        case ORC_NEIGHBOR_DEGREE: b[i] = (uint32_t)deg(g, g->col[e]); break;
        default: return -1;
        }
    }
    return 0;
}

/* Algorithmic byte model (what the method has to move; the GPU data layout
 * is int64 row offsets, int32 ids, uint32 weights):
 *   per expanded frontier vertex: 8 (frontier entry: vertex + instance)
 *     + 16 (row-offset pair) + 4*deg if the bias reads a weight array
 *     + 4*s (neighbor ids at the s picks) + 8*s (the s output edges);
 *   per walk step: 16 (row offsets) + 4*deg (weights, or for node2vec the
 *     neighbor list) + 4*deg(prev) (node2vec: the previous list) + 4
 *     (neighbor id at the pick; node2vec reads the whole list anyway) + 4
 *     (path entry). */
static double select_bytes(int32_t kind, int64_t d, int64_t s)
{
    double bytes = 8.0 + 16.0 + 12.0 * (double)s;
    if (kind == ORC_EDGE_WEIGHT || kind == ORC_NEIGHBOR_DEGREE) bytes += 4.0 * (double)d;
    return bytes;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* growable int32 vector */
typedef struct { int32_t* p; int64_t n, cap; } ivec;
static int iv_push(ivec* v, int32_t x)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 64;
        int32_t* q = (int32_t*)realloc(v->p, (size_t)nc * sizeof(int32_t));
        if (!q) return -1;
        v->p = q; v->cap = nc;
    }
    v->p[v->n++] = x;
    return 0;
}

/*
 * Neighbor sampling for a batch of instances: the loop of fig:api(b) with
 * FrontierSize = all, EdgeBias of a static kind, NeighborSize = fanout of
 * the layer, and Update = "not visited by this instance before" (the
 * sampling-without-replacement filter, Section II-A and Section III-C).
 *
 * Instance i (global id inst_id = instance_ids ? instance_ids[i] :
 * instance_base + i) starts from the distinct seeds
 * seeds[seed_off[i] .. seed_off[i+1]), which form F_0 and the visited set.
 * Layer l = 0..L_i-1 (L_i = layers before the first zero fanout) selects,
 * for every v in F_l in increasing id, orc_select(b(v), fanout, counter
 * (inst_id mod 2^32, l, v, slot|round)) and emits (v, neighbor) per pick;
 * F_{l+1} = distinct picked neighbors not yet visited, then they are
 * marked visited. Edges to visited vertices are still emitted.
 * Fanout -1 selects every positive-bias neighbor. With burn != 0 (forest
 * fire), vertex v's NeighborSize is orc_burn_count(rng_seed, inst_id, l, v,
 * burn, cap) with cap = the fanout (ORC_BURN_CAP_ALL for -1).
 *
 * Output, in order (layer, instance, src, slot): src/dst[cap];
 * offsets[l*ni + i] is the first edge of (layer l, instance i) and
 * offsets[L*ni] the total. Returns 0, 1 on invalid input, 2 if cap is too
 * small (*num_edges still receives the total).
 * stats (nullable, double[5]): algorithmic bytes, number of expanded
 * vertices, number of direct (fallback) draws, sum of degrees expanded,
 * number of draws of either kind.
 */
/* Per-thread scratch and statistics of the vertex expansions. */
typedef struct {
    uint32_t* b; int64_t bcap;
    int64_t* pos; int64_t poscap;
    double bytes, expanded, fb, deg, draws;
} vscratch;

/* One frontier vertex v of instance inst_id at layer l with fanout k0:
 * NeighborSize (the fanout, or the forest fire count capped by it), biases,
 * orc_select with counter (inst_id mod 2^32, l, v, .), and its edges appended
 * to (os, od) in slot order. Returns 0, or 1 if a bias cannot be evaluated. */
static int expand_vertex(const orc_graph* g, int32_t kind, uint64_t rng_seed, uint64_t inst_id, int32_t l,
                         int64_t k0, uint32_t burn, int32_t rounds, int32_t v, vscratch* w, ivec* os, ivec* od)
{
    int64_t k = k0;
    if (burn)
        k = orc_burn_count(rng_seed, (uint32_t)inst_id, (uint32_t)l, (uint32_t)v, burn,
                           k < 0 ? ORC_BURN_CAP_ALL : (int32_t)k);
    int64_t d = deg(g, v), beg = g->rowptr[v];
    if (d > w->bcap) {
        w->bcap = d; w->b = (uint32_t*)realloc(w->b, (size_t)w->bcap * sizeof(uint32_t));
    }
    if (d > w->poscap) {
        w->poscap = d; w->pos = (int64_t*)realloc(w->pos, (size_t)w->poscap * sizeof(int64_t));
    }
    if (d > 0 && edge_bias_static(g, kind, v, w->b) != 0) return 1;
    int32_t nfb = 0;
    int64_t ndr = 0;
    int32_t s = orc_select(w->b, d, k, rounds, rng_seed, (uint32_t)inst_id, (uint32_t)l, (uint32_t)v, w->pos,
                           &nfb, &ndr);
    for (int32_t j = 0; j < s; ++j) {
        iv_push(os, v);
        iv_push(od, g->col[beg + w->pos[j]]);
    }
    w->bytes += select_bytes(kind, d, s);
    w->expanded += 1;
    w->fb += nfb;
    w->draws += (double)ndr;
    w->deg += (double)d;
    return 0;
}

/* Every layer of instance i into es/ed[l*ni + i]. visited is an all-zero
 * byte array of n entries, left all-zero. With inner_threads > 1 the
 * vertices of each layer are split into that many contiguous ranges, one per
 * thread, and the ranges' edges are appended in range order: the same edges
 * in the same order as one thread. */
static int sample_instance(const orc_graph* g, int32_t ni, int32_t i, const int64_t* seed_off, const int32_t* seeds,
                           uint64_t inst_id, int32_t kind, const int32_t* fo, int32_t L, uint64_t rng_seed,
                           int32_t rounds, uint32_t burn, unsigned char* visited, ivec* es, ivec* ed,
                           int inner_threads, vscratch* w)
{
    int failed = 0;
    int32_t Li = 0;
    while (Li < L && fo[Li] != 0) ++Li;
    ivec all = {0}, cur = {0}, nxt = {0};
    /* F_0: distinct seeds, ascending */
    for (int64_t s = seed_off[i]; s < seed_off[i + 1]; ++s) {
        int32_t v = seeds[s];
        if (!visited[v]) { visited[v] = 1; iv_push(&cur, v); iv_push(&all, v); }
    }
    qsort(cur.p, (size_t)cur.n, sizeof(int32_t), cmp_i32);
    for (int32_t l = 0; l < Li; ++l) {
        ivec* os = &es[(int64_t)l * ni + i];
        ivec* od = &ed[(int64_t)l * ni + i];
        if (inner_threads <= 1) {
            for (int64_t f = 0; f < cur.n && !failed; ++f)
                failed = expand_vertex(g, kind, rng_seed, inst_id, l, fo[l], burn, rounds, cur.p[f], w, os, od);
        } else {
            int T = inner_threads;
            ivec* ts = (ivec*)calloc((size_t)T, sizeof(ivec));
            ivec* td = (ivec*)calloc((size_t)T, sizeof(ivec));
            vscratch* tw = (vscratch*)calloc((size_t)T, sizeof(vscratch));
            int tfail = 0;
            #pragma omp parallel num_threads(T) reduction(| : tfail)
            {
#ifdef _OPENMP
                int t = omp_get_thread_num(), nt = omp_get_num_threads();
#else
                int t = 0, nt = 1;
#endif
                int64_t lo = cur.n * t / nt, hi = cur.n * (t + 1) / nt;
                for (int64_t f = lo; f < hi && !tfail; ++f)
                    tfail |= expand_vertex(g, kind, rng_seed, inst_id, l, fo[l], burn, rounds, cur.p[f], &tw[t],
                                           &ts[t], &td[t]);
            }
            failed |= tfail;
            for (int t = 0; t < T; ++t) {
                for (int64_t q = 0; q < ts[t].n; ++q) { iv_push(os, ts[t].p[q]); iv_push(od, td[t].p[q]); }
                w->bytes += tw[t].bytes; w->expanded += tw[t].expanded; w->fb += tw[t].fb;
                w->deg += tw[t].deg; w->draws += tw[t].draws;
                free(ts[t].p); free(td[t].p); free(tw[t].b); free(tw[t].pos);
            }
            free(ts); free(td); free(tw);
        }
        if (failed) break;
        if (l + 1 < Li) {
            /* Update: next frontier = picked neighbors not visited */
            nxt.n = 0;
            for (int64_t e = 0; e < od->n; ++e) {
                int32_t x = od->p[e];
                if (!visited[x]) { visited[x] = 1; iv_push(&nxt, x); iv_push(&all, x); }
            }
            qsort(nxt.p, (size_t)nxt.n, sizeof(int32_t), cmp_i32);
            ivec t = cur; cur = nxt; nxt = t;
        }
    }
    for (int64_t q = 0; q < all.n; ++q) visited[all.p[q]] = 0;
    free(all.p); free(cur.p); free(nxt.p);
    return failed;
}

int32_t orc_sample(int64_t n, const int64_t* rowptr, const int32_t* col, const uint32_t* ew,
                   int32_t ni, const int64_t* seed_off, const int32_t* seeds,
                   uint64_t instance_base, const uint64_t* instance_ids,
                   int32_t L, const int32_t* fanouts, int32_t fanout_stride,
                   const int32_t* bias_kinds, int32_t bias_kind,
                   uint64_t rng_seed, int32_t rounds, uint32_t burn,
                   int64_t cap, int32_t* src, int32_t* dst, int64_t* offsets,
                   int64_t* num_edges, double* stats, int32_t nthreads)
{
    orc_graph g = {n, rowptr, col, ew};
    if (ni < 0 || L < 0 || n < 0 || rounds < 0 || rounds >= (int32_t)ORC_BURN_ROUND) return 1;
    for (int32_t i = 0; i < ni; ++i) {
        int32_t kind = bias_kinds ? bias_kinds[i] : bias_kind;
        if (kind != ORC_UNIFORM && kind != ORC_EDGE_WEIGHT && kind != ORC_NEIGHBOR_DEGREE) return 1;
        if (kind == ORC_EDGE_WEIGHT && !ew) return 1;
        if (seed_off[i + 1] < seed_off[i]) return 1;
        for (int64_t s = seed_off[i]; s < seed_off[i + 1]; ++s)
            if (seeds[s] < 0 || seeds[s] >= n) return 1;
        for (int32_t l = 0; l < L; ++l) {
            int32_t f = fanouts[(fanout_stride ? (int64_t)i * fanout_stride : 0) + l];
            if (f < -1 || f > 0xFFFF) return 1;   /* slot index has 16 bits */
        }
    }
    /* per (instance, layer) edge lists */
    ivec* es = (ivec*)calloc((size_t)ni * (size_t)(L > 0 ? L : 1), sizeof(ivec));
    ivec* ed = (ivec*)calloc((size_t)ni * (size_t)(L > 0 ? L : 1), sizeof(ivec));
    double tot_bytes = 0, tot_expanded = 0, tot_fb = 0, tot_deg = 0, tot_draws = 0;
    int failed = 0;
#ifdef _OPENMP
    int T = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    int T = 1;
#endif
    if (ni >= T || T <= 1) {
        /* independent instances on separate threads */
        #pragma omp parallel num_threads(T) reduction(+ : tot_bytes, tot_expanded, tot_fb, tot_deg, tot_draws)
        {
            unsigned char* visited = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
            vscratch w = {0};
            #pragma omp for schedule(dynamic, 1)
            for (int32_t i = 0; i < ni; ++i) {
                uint64_t inst_id = instance_ids ? instance_ids[i] : instance_base + (uint64_t)i;
                int32_t kind = bias_kinds ? bias_kinds[i] : bias_kind;
                const int32_t* fo = fanouts + (fanout_stride ? (int64_t)i * fanout_stride : 0);
                if (sample_instance(&g, ni, i, seed_off, seeds, inst_id, kind, fo, L, rng_seed, rounds, burn,
                                    visited, es, ed, 1, &w)) {
                    #pragma omp atomic write
                    failed = 1;
                }
            }
            tot_bytes += w.bytes; tot_expanded += w.expanded; tot_fb += w.fb; tot_deg += w.deg;
            tot_draws += w.draws;
            free(visited); free(w.b); free(w.pos);
        }
    } else {
        /* fewer instances than threads: one instance at a time, each layer's
         * frontier split over the threads */
        unsigned char* visited = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
        vscratch w = {0};
        for (int32_t i = 0; i < ni && !failed; ++i) {
            uint64_t inst_id = instance_ids ? instance_ids[i] : instance_base + (uint64_t)i;
            int32_t kind = bias_kinds ? bias_kinds[i] : bias_kind;
            const int32_t* fo = fanouts + (fanout_stride ? (int64_t)i * fanout_stride : 0);
            failed = sample_instance(&g, ni, i, seed_off, seeds, inst_id, kind, fo, L, rng_seed, rounds, burn,
                                     visited, es, ed, T, &w);
        }
        tot_bytes = w.bytes; tot_expanded = w.expanded; tot_fb = w.fb; tot_deg = w.deg; tot_draws = w.draws;
        free(visited); free(w.b); free(w.pos);
    }
    if (failed) {
        for (int64_t q = 0; q < (int64_t)ni * L; ++q) { free(es[q].p); free(ed[q].p); }
        free(es); free(ed);
        return 1;
    }
    int64_t total = 0;
    for (int32_t l = 0; l < L; ++l)
        for (int32_t i = 0; i < ni; ++i) {
            if (offsets) offsets[(int64_t)l * ni + i] = total;
            total += es[(int64_t)l * ni + i].n;
        }
    if (offsets) offsets[(int64_t)L * ni] = total;
    if (num_edges) *num_edges = total;
    int rc = 0;
    if (total > cap) rc = 2;
    else {
        int64_t w = 0;
        for (int32_t l = 0; l < L; ++l)
            for (int32_t i = 0; i < ni; ++i) {
                ivec* os = &es[(int64_t)l * ni + i];
                ivec* od = &ed[(int64_t)l * ni + i];
                if (os->n) {
                    memcpy(src + w, os->p, (size_t)os->n * sizeof(int32_t));
                    memcpy(dst + w, od->p, (size_t)od->n * sizeof(int32_t));
                }
                w += os->n;
            }
    }
    for (int64_t q = 0; q < (int64_t)ni * L; ++q) { free(es[q].p); free(ed[q].p); }
    free(es); free(ed);
    if (stats) {
        stats[0] = tot_bytes; stats[1] = tot_expanded; stats[2] = tot_fb; stats[3] = tot_deg;
        stats[4] = tot_draws;
    }
    return rc;
}

/*
 * Random walks (Section II-A): walker w (global id wid = walker_ids ?
 * walker_ids[w] : walker_base + w) starts at starts[w] and takes up to
 * `length` steps. At step s from vertex v (previous vertex t, none at s=0)
 * the biases of N(v) are evaluated, W = sum; if v has no neighbor or W = 0
 * the walk stops and the rest of its path is -1. Otherwise one candidate is
 * drawn with replacement (round 0, slot 0): counter (wid mod 2^32, s, v, 0),
 * r in [0, W), m = its(r), and the walk moves to col[rowptr[v] + m].
 * NODE2VEC tests membership of x in N(t) with a marker array.
 * Restart and jump (Section II-A, random walk with restart / with jump, as
 * Update rules): when restart_threshold or jump_threshold is non-zero, every
 * step first draws x in [0, 2^32) with counter (wid, s, v, 2); x <
 * restart_threshold moves the walker back to its start, otherwise x <
 * restart_threshold + jump_threshold moves it to the vertex drawn in [0, n)
 * with counter (wid, s, v, 3); either move is a step and forgets the
 * previous vertex (the next node2vec step is unbiased). Otherwise the step is
 * the one above, including the stop at a dead end.
 * METROPOLIS (Section II-A names the Metropolis-Hastings random walk among
 * the unbiased walks; the rule is the standard one that makes the uniform
 * distribution over vertices stationary): the drawn neighbor u is a uniform
 * proposal, accepted iff x * deg(u) < deg(v) * 2^32 for x in [0, 2^32) drawn
 * with counter (wid, s, v, 4), i.e. with probability min(1, deg(v)/deg(u));
 * a rejected proposal is a step that stays at v.
 *
 * paths: int32[nw * (length+1)], walker-major. steps (nullable): int64[nw],
 * number of steps taken. stats (nullable, double[2]): algorithmic bytes,
 * total steps. Returns 0, or 1 on invalid input.
 */
int32_t orc_walk(int64_t n, const int64_t* rowptr, const int32_t* col, const uint32_t* ew,
                 int32_t bias_kind, uint32_t w_return, uint32_t w_common, uint32_t w_outward,
                 int64_t nw, const int32_t* starts, uint64_t walker_base, const uint64_t* walker_ids,
                 int32_t length, uint64_t rng_seed, uint32_t restart_threshold, uint32_t jump_threshold,
                 int32_t* paths, int64_t* steps, double* stats, int32_t nthreads)
{
    orc_graph g = {n, rowptr, col, ew};
    if (length < 0 || nw < 0) return 1;
    if ((uint64_t)restart_threshold + (uint64_t)jump_threshold > ((uint64_t)1 << 32)) return 1;
    if (jump_threshold && n == 0) return 1;
    if (bias_kind < ORC_UNIFORM || bias_kind > ORC_METROPOLIS) return 1;
    if (bias_kind == ORC_EDGE_WEIGHT && !ew) return 1;
    for (int64_t w = 0; w < nw; ++w)
        if (starts[w] < 0 || starts[w] >= n) return 1;
    double tot_bytes = 0, tot_steps = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel reduction(+ : tot_bytes, tot_steps)
    {
        unsigned char* mark = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
        uint32_t* b = NULL; int64_t bcap = 0;
        uint64_t* S = NULL; int64_t scap = 0;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t w = 0; w < nw; ++w) {
            uint64_t wid = walker_ids ? walker_ids[w] : walker_base + (uint64_t)w;
            int32_t* path = paths + w * (int64_t)(length + 1);
            int64_t v = starts[w], t = -1;
            path[0] = (int32_t)v;
            int32_t s = 0;
            for (; s < length; ++s) {
                if (restart_threshold | jump_threshold) {
                    const uint64_t x = orc_draw(rng_seed, (uint32_t)wid, (uint32_t)s, (uint32_t)v, 2u,
                                                (uint64_t)1 << 32);
                    int64_t to = -1;
                    if (x < restart_threshold) to = starts[w];
                    else if (x < (uint64_t)restart_threshold + jump_threshold)
                        to = (int64_t)orc_draw(rng_seed, (uint32_t)wid, (uint32_t)s, (uint32_t)v, 3u, (uint64_t)n);
                    if (to >= 0) {
                        path[s + 1] = (int32_t)to;
                        t = -1;
                        v = to;
                        tot_bytes += 8.0;
                        continue;
                    }
                }
                int64_t d = deg(&g, v), beg = rowptr[v];
                if (d == 0) break;
                if (d > bcap) { bcap = d; b = (uint32_t*)realloc(b, (size_t)bcap * sizeof(uint32_t)); }
                if (d + 1 > scap) { scap = d + 1; S = (uint64_t*)realloc(S, (size_t)scap * sizeof(uint64_t)); }
                double bytes = 16.0 + 4.0;
                if (bias_kind == ORC_NODE2VEC) {
                    if (t < 0) {
                        for (int64_t i = 0; i < d; ++i) b[i] = 1;
                    } else {
                        for (int64_t e = rowptr[t]; e < rowptr[t + 1]; ++e) mark[col[e]] = 1;
                        for (int64_t i = 0; i < d; ++i) {
                            int32_t x = col[beg + i];
                            b[i] = (x == t) ? w_return : (mark[x] ? w_common : w_outward);
                        }
                        for (int64_t e = rowptr[t]; e < rowptr[t + 1]; ++e) mark[col[e]] = 0;
                        bytes += 4.0 * (double)deg(&g, t);
                    }
                    bytes += 4.0 * (double)d;
                } else if (bias_kind == ORC_METROPOLIS) {
                    for (int64_t i = 0; i < d; ++i) b[i] = 1;   /* uniform proposal */
                    bytes += 4.0 + 16.0;
                } else {
                    edge_bias_static(&g, bias_kind, v, b);
                    if (bias_kind == ORC_UNIFORM) bytes += 4.0;
                    else bytes += 4.0 * (double)d + 4.0;
                }
                prefix(b, d, S);
                if (S[d] == 0) break;
                uint64_t r = orc_draw(rng_seed, (uint32_t)wid, (uint32_t)s, (uint32_t)v, 0u, S[d]);
                int64_t m = orc_its(S, d, r);
                int64_t u = col[beg + m];
                if (bias_kind == ORC_METROPOLIS) {
                    /* accept u with probability min(1, deg(v) / deg(u)):
                     * x / 2^32 < d / deg(u), compared exactly in integers;
                     * a rejected proposal is a step that stays at v */
                    const uint64_t x = orc_draw(rng_seed, (uint32_t)wid, (uint32_t)s, (uint32_t)v, 4u,
                                                (uint64_t)1 << 32);
                    if (x * (uint64_t)deg(&g, u) >= ((uint64_t)d << 32)) u = v;
                }
                path[s + 1] = (int32_t)u;
                t = v;
                v = u;
                tot_bytes += bytes;
            }
            if (steps) steps[w] = s;
            tot_steps += s;
            for (int32_t q = s + 1; q <= length; ++q) path[q] = -1;
        }
        free(mark); free(b); free(S);
    }
    if (stats) { stats[0] = tot_bytes; stats[1] = tot_steps; }
    return 0;
}

/*
 * Layer sampling (Section II-A: unlike neighbor and forest fire sampling,
 * which select neighbors per frontier vertex, layer sampling selects a
 * constant number of neighbors for the whole frontier in each round).
 * Instance i (id iid = instance_base + i): F_0 = its seeds (sorted, distinct:
 * checked), visited = F_0. Layer l = 0..L-1 with k = fanouts[l]:
 *   pool = the lists N(v) of v in F_l, concatenated in increasing v (list
 *   order inside); b = EdgeBias of each pool position (Eq. edgebias);
 *   Select: orc_select(b, |pool|, k, rounds, counter (iid, l, 0xFFFFFFFF,
 *   slot | round << 16)) -- k distinct positions, or every positive one
 *   when k >= P;
 *   Sampled: slot j is the edge (owner of position j, neighbor at it);
 *   Update: F_{l+1} = distinct picked neighbors not visited, increasing;
 *   visited gains them.
 * Output: src/dst[(i * L + l) * K + j] for slot j (-1 past the count),
 * counts[i * L + l] (K = the largest fanout). Returns 0, or 1 on invalid
 * input (unsorted or repeated seeds, a fanout outside [1, 64]).
 */
int32_t orc_layer_sample(int64_t n, const int64_t* rowptr, const int32_t* col, const uint32_t* ew,
                         int32_t ni, const int64_t* seed_off, const int32_t* seeds, uint64_t instance_base,
                         int32_t L, const int32_t* fanouts, int32_t bias_kind, uint64_t rng_seed, int32_t rounds,
                         int32_t* src, int32_t* dst, int32_t* counts)
{
    orc_graph g = {n, rowptr, col, ew};
    if (ni < 0 || L < 0 || rounds < 0 || rounds >= (int32_t)ORC_BURN_ROUND) return 1;
    if (bias_kind != ORC_UNIFORM && bias_kind != ORC_EDGE_WEIGHT && bias_kind != ORC_NEIGHBOR_DEGREE) return 1;
    if (bias_kind == ORC_EDGE_WEIGHT && !ew) return 1;
    int32_t K = 0;
    for (int32_t l = 0; l < L; ++l) {
        if (fanouts[l] < 1 || fanouts[l] > 64) return 1;
        if (fanouts[l] > K) K = fanouts[l];
    }
    for (int32_t i = 0; i < ni; ++i) {
        if (seed_off[i + 1] < seed_off[i]) return 1;
        for (int64_t s = seed_off[i]; s < seed_off[i + 1]; ++s) {
            if (seeds[s] < 0 || seeds[s] >= n) return 1;
            if (s > seed_off[i] && seeds[s] <= seeds[s - 1]) return 1;
        }
    }
    for (int64_t q = 0; q < (int64_t)ni * L * K; ++q) src[q] = dst[q] = -1;
    unsigned char* visited = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int32_t i = 0; i < ni; ++i) {
        const uint64_t iid = instance_base + (uint64_t)i;
        ivec cur = {0}, nxt = {0}, all = {0};
        for (int64_t s = seed_off[i]; s < seed_off[i + 1]; ++s) {
            iv_push(&cur, seeds[s]);
            iv_push(&all, seeds[s]);
            visited[seeds[s]] = 1;
        }
        for (int32_t l = 0; l < L; ++l) {
            int64_t D = 0;
            for (int64_t f = 0; f < cur.n; ++f) D += deg(&g, cur.p[f]);
            uint32_t* b = (uint32_t*)malloc((size_t)(D > 0 ? D : 1) * sizeof(uint32_t));
            int32_t* own = (int32_t*)malloc((size_t)(D > 0 ? D : 1) * sizeof(int32_t));
            int32_t* nb = (int32_t*)malloc((size_t)(D > 0 ? D : 1) * sizeof(int32_t));
            int64_t at = 0;
            for (int64_t f = 0; f < cur.n; ++f) {
                const int32_t v = cur.p[f];
                edge_bias_static(&g, bias_kind, v, b + at);
                for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e, ++at) {
                    own[at] = v;
                    nb[at] = col[e];
                }
            }
            int64_t* pos = (int64_t*)malloc((size_t)(D > 0 ? D : 1) * sizeof(int64_t));
            const int32_t c = orc_select(b, D, fanouts[l], rounds, rng_seed, (uint32_t)iid, (uint32_t)l,
                                         0xFFFFFFFFu, pos, NULL, NULL);
            counts[(int64_t)i * L + l] = c;
            nxt.n = 0;
            for (int32_t j = 0; j < c; ++j) {
                const int64_t o = ((int64_t)i * L + l) * K + j;
                src[o] = own[pos[j]];
                dst[o] = nb[pos[j]];
                if (!visited[nb[pos[j]]]) {
                    visited[nb[pos[j]]] = 1;
                    iv_push(&nxt, nb[pos[j]]);
                    iv_push(&all, nb[pos[j]]);
                }
            }
            qsort(nxt.p, (size_t)nxt.n, sizeof(int32_t), cmp_i32);
            ivec t = cur; cur = nxt; nxt = t;
            free(b); free(own); free(nb); free(pos);
        }
        for (int64_t q = 0; q < all.n; ++q) visited[all.p[q]] = 0;
        free(cur.p); free(nxt.p); free(all.p);
    }
    free(visited);
    return 0;
}

/*
 * Multi-dimensional random walk, a.k.a. frontier sampling (Section II-A; the
 * VertexBias select site of fig:api(b); worked example fig:layer_example).
 * Instance i (id iid = instance_base + i) keeps a pool of
 * P_i = pool_off[i+1] - pool_off[i] vertices, initially
 * pool[pool_off[i] .. pool_off[i+1]). Step s = 0 .. budget-1:
 *   VertexBias: b_j = out-degree of pool vertex j, W = sum b_j; W = 0 ends
 *   the instance.
 *   Select one frontier vertex: r = draw(iid, s, 0xFFFFFFFF, 0) in [0, W),
 *   j = its(prefix of b in pool order, r), v = pool[j].
 *   EdgeBias 1, NeighborSize 1: m = draw(iid, s, v, 1) in [0, deg v),
 *   u = col[rowptr[v] + m].
 *   Sampled: edge s of the instance is (v, u).
 *   Update: pool[j] = u.
 * Output: src/dst[i * budget + s], -1 once the instance has ended;
 * steps[i] (nullable) = edges sampled. Returns 0, or 1 on invalid input.
 */
int32_t orc_mdrw(int64_t n, const int64_t* rowptr, const int32_t* col, int32_t ni,
                 const int64_t* pool_off, const int32_t* pool, uint64_t instance_base,
                 int64_t budget, uint64_t rng_seed, int32_t* src, int32_t* dst, int64_t* steps)
{
    if (ni < 0 || budget < 0) return 1;
    for (int32_t i = 0; i < ni; ++i) {
        if (pool_off[i + 1] < pool_off[i]) return 1;
        for (int64_t j = pool_off[i]; j < pool_off[i + 1]; ++j)
            if (pool[j] < 0 || pool[j] >= n) return 1;
    }
    for (int32_t i = 0; i < ni; ++i) {
        const uint64_t iid = instance_base + (uint64_t)i;
        const int64_t P = pool_off[i + 1] - pool_off[i];
        int32_t* fp = (int32_t*)malloc((size_t)(P > 0 ? P : 1) * sizeof(int32_t));
        uint32_t* b = (uint32_t*)malloc((size_t)(P > 0 ? P : 1) * sizeof(uint32_t));
        uint64_t* S = (uint64_t*)malloc((size_t)(P + 1) * sizeof(uint64_t));
        memcpy(fp, pool + pool_off[i], (size_t)P * sizeof(int32_t));
        int64_t s = 0;
        for (; s < budget; ++s) {
            for (int64_t j = 0; j < P; ++j) b[j] = (uint32_t)(rowptr[fp[j] + 1] - rowptr[fp[j]]);
            prefix(b, P, S);
            if (S[P] == 0) break;
            const uint64_t r = orc_draw(rng_seed, (uint32_t)iid, (uint32_t)s, 0xFFFFFFFFu, 0u, S[P]);
            const int64_t j = orc_its(S, P, r);
            const int32_t v = fp[j];
            const int64_t d = rowptr[v + 1] - rowptr[v];
            const uint64_t m = orc_draw(rng_seed, (uint32_t)iid, (uint32_t)s, (uint32_t)v, 1u, (uint64_t)d);
            const int32_t u = col[rowptr[v] + (int64_t)m];
            src[(int64_t)i * budget + s] = v;
            dst[(int64_t)i * budget + s] = u;
            fp[j] = u;
        }
        if (steps) steps[i] = s;
        for (int64_t q = s; q < budget; ++q) {
            src[(int64_t)i * budget + q] = -1;
            dst[(int64_t)i * budget + q] = -1;
        }
        free(fp); free(b); free(S);
    }
    return 0;
}

/* Number of OpenMP threads a parallel region would use (for reporting). */
int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
