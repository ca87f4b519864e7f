/*
 * Seeded synthetic input generator: R-MAT graphs in CSR form.
 *
 * This file produces INPUTS only. It contains none of the sampling method's
 * arithmetic (no bias, prefix sum, draw or selection); both the CPU oracle
 * and the GPU library consume its output as plain arrays.
 *
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): each edge descends `scale`
 * levels of the adjacency matrix, picking one of four quadrants with
 * probabilities (a, b, c, 1-a-b-c) at every level. The graphs stand in for
 * the power-law social/web graphs of the paper's evaluation (Table of
 * datasets, Section VI).
 *
 * Determinism: the quadrant choice of edge e at level l is a pure function of
 * (gen_seed, e, l) through the SplitMix64 finaliser (Steele, Lea, Flood,
 * OOPSLA 2014), so the edge list does not depend on the thread count. Vertex
 * ids are relabelled by a seeded Fisher-Yates permutation so that degree is
 * not correlated with id. Self-loops and duplicate edges are dropped and each
 * adjacency list is sorted ascending.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static void sort_i32(int32_t* a, int64_t n)
{
    if (n < 32) {
        for (int64_t i = 1; i < n; ++i) {
            int32_t x = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
            a[j + 1] = x;
        }
    } else {
        qsort(a, (size_t)n, sizeof(int32_t), cmp_i32);
    }
}

/* Pass 1 of graph construction: count edges so the caller can size buffers.
 * Returns the number of directed edge slots before dedup (num_edges, doubled
 * when symmetrize != 0). */
int64_t rmat_raw_slots(int64_t num_edges, int symmetrize)
{
    return symmetrize ? 2 * num_edges : num_edges;
}

/*
 * Build the CSR of an R-MAT graph with n = 2^scale vertices.
 *
 *   rowptr  out, int64[n+1]
 *   col     out, int32[cap_col]; cap_col >= rmat_raw_slots(...)
 *   returns the number of kept directed edges m (rowptr[n]), or -1 on
 *   allocation failure, -2 if cap_col is too small.
 */
int64_t rmat_build_csr(int32_t scale, int64_t num_edges, double a, double b, double c,
                       uint64_t gen_seed, int symmetrize, int64_t* rowptr,
                       int32_t* col, int64_t cap_col, int nthreads)
{
    if (scale < 1 || scale > 30) return -3;
    const int64_t n = (int64_t)1 << scale;
    const int64_t slots = rmat_raw_slots(num_edges, symmetrize);
    if (cap_col < slots) return -2;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* quadrant thresholds on a 16-bit uniform */
    const uint32_t ta = (uint32_t)(a * 65536.0 + 0.5);
    const uint32_t tb = (uint32_t)((a + b) * 65536.0 + 0.5);
    const uint32_t tc = (uint32_t)((a + b + c) * 65536.0 + 0.5);

    /* seeded relabelling permutation (sequential Fisher-Yates) */
    int32_t* perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    uint32_t* src = (uint32_t*)malloc((size_t)slots * sizeof(uint32_t));
    int64_t* cursor = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!perm || !src || !cursor) { free(perm); free(src); free(cursor); return -1; }
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    {
        uint64_t st = mix64(gen_seed ^ 0x5851f42d4c957f2dull);
        for (int64_t i = n - 1; i > 0; --i) {
            st = mix64(st);
            int64_t j = (int64_t)(st % (uint64_t)(i + 1));
            int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
    }

    /* edge draws: dst goes to col[] temporarily, src to src[] */
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < num_edges; ++e) {
        uint32_t s = 0, d = 0;
        uint64_t h = 0;
        for (int32_t l = 0; l < scale; ++l) {
            if ((l & 3) == 0) h = mix64(gen_seed * 0x2545f4914f6cdd1dull ^ mix64((uint64_t)e * 8u + (uint64_t)(l >> 2)));
            uint32_t q = (uint32_t)(h & 0xffffu);
            h >>= 16;
            uint32_t sb, db;
            if (q < ta)      { sb = 0; db = 0; }
            else if (q < tb) { sb = 0; db = 1; }
            else if (q < tc) { sb = 1; db = 0; }
            else             { sb = 1; db = 1; }
            s = (s << 1) | sb;
            d = (d << 1) | db;
        }
        s = (uint32_t)perm[s];
        d = (uint32_t)perm[d];
        src[e] = s;
        col[e] = (int32_t)d;
        if (symmetrize) {
            src[num_edges + e] = d;
            col[num_edges + e] = (int32_t)s;
        }
    }
    free(perm);

    /* degree count, then bucket dst ids by src into a scratch array */
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < slots; ++e)
        __atomic_fetch_add(&cursor[src[e] + 1], 1, __ATOMIC_RELAXED);
    for (int64_t v = 0; v < n; ++v) cursor[v + 1] += cursor[v];
    int32_t* tmp = (int32_t*)malloc((size_t)slots * sizeof(int32_t));
    if (!tmp) { free(src); free(cursor); return -1; }
    memcpy(rowptr, cursor, (size_t)(n + 1) * sizeof(int64_t)); /* raw starts */
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < slots; ++e) {
        int64_t p = __atomic_fetch_add(&cursor[src[e]], 1, __ATOMIC_RELAXED);
        tmp[p] = col[e];
    }
    free(src);

    /* sort, dedup and drop self-loops per row; cursor[v] = kept count */
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < n; ++v) {
        int64_t b0 = rowptr[v], e0 = rowptr[v + 1];
        sort_i32(tmp + b0, e0 - b0);
        int64_t w = b0;
        for (int64_t i = b0; i < e0; ++i) {
            int32_t x = tmp[i];
            if (x == (int32_t)v) continue;
            if (w > b0 && tmp[w - 1] == x) continue;
            tmp[w++] = x;
        }
        cursor[v] = w - b0;
    }
    /* compact into col with the final rowptr */
    int64_t* kept_start = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!kept_start) { free(tmp); free(cursor); return -1; }
    kept_start[0] = 0;
    for (int64_t v = 0; v < n; ++v) kept_start[v + 1] = kept_start[v] + cursor[v];
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < n; ++v)
        memcpy(col + kept_start[v], tmp + rowptr[v], (size_t)cursor[v] * sizeof(int32_t));
    memcpy(rowptr, kept_start, (size_t)(n + 1) * sizeof(int64_t));
    free(kept_start);
    free(tmp);
    free(cursor);
    return rowptr[n];
}

/* Out-degree of every destination, as uint32 edge weights: w[e] = deg(col[e]).
 * This is an input transformation (an edge-weight array handed to the
 * library as EDGE_WEIGHT), used by the served-stream workload. */
void rmat_dst_outdeg_weights(int64_t n, int64_t m, const int64_t* rowptr,
                             const int32_t* col, uint32_t* w, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    (void)n;
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        int32_t x = col[e];
        w[e] = (uint32_t)(rowptr[x + 1] - rowptr[x]);
    }
}
