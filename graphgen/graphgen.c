/*
 * Seeded synthetic graph inputs for the BFS path and for its oracle.
 *
 * This module only builds inputs: R-MAT graphs and 4-neighbour 2-D grids in
 * symmetric CSR form (int64 row offsets, int32 column indices), and seeded
 * root lists.  It holds none of the search's arithmetic, so both the CPU
 * oracle and the GPU library can take their inputs from it.
 *
 * Workload (the paper's benchmark graphs, Section 4): R-MAT edge lists with
 * 2^scale vertices and edgefactor * 2^scale generated edges, made undirected
 * by adding the opposite of every edge.  The paper used the Graph500 reference
 * generator, which is not reproduced here: this is an R-MAT generator written
 * from the R-MAT definition (Chakrabarti, Zhan & Faloutsos, 2004), recursive
 * quadrant choice with probabilities A, B, C, D = 1-A-B-C, one choice per bit
 * of the vertex ids.  No noise is added to the probabilities.  Vertex ids are
 * relabelled by a keyed pseudo-random permutation, self-loops are dropped,
 * duplicate edges are merged and every row is sorted ascending.
 *
 * Randomness is counter based: draw(key, i) = splitmix64(key + i), with
 * splitmix64 the finaliser published by Steele, Lea & Flood ("Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  Every draw is a pure
 * function of (seed, edge index, bit level), so passes can be recomputed
 * instead of stored and the result does not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t splitmix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t gg_splitmix64(uint64_t z) { return splitmix64(z); }

/* Domain-separated stream keys derived from the user seed. */
#define STREAM_EDGES 0x45444745ULL /* "EDGE" */
#define STREAM_PERM  0x5045524dULL /* "PERM" */
#define STREAM_ROOTS 0x524f4f54ULL /* "ROOT" */

static inline uint64_t stream_key(uint64_t seed, uint64_t stream)
{
    return splitmix64(splitmix64(seed) ^ (stream * 0xd1b54a32d192ed03ULL));
}

/* 4-round balanced Feistel network on 2*half bits, keyed. A bijection. */
static inline uint64_t feistel(uint64_t x, int half, uint64_t key)
{
    const uint64_t mask = (half >= 64) ? ~0ULL : ((1ULL << half) - 1);
    uint64_t L = x >> half, R = x & mask;
    for (int i = 0; i < 4; ++i) {
        uint64_t F = splitmix64(key + (uint64_t)i * 0x632be59bd9b4e019ULL + R) & mask;
        uint64_t nL = R;
        R = L ^ F;
        L = nL;
    }
    return (L << half) | R;
}

/* Keyed permutation of [0, 2^scale): Feistel on 2*ceil(scale/2) bits with
 * cycle walking, so it stays a bijection for odd scales. */
uint32_t gg_permute(uint32_t v, int scale, uint64_t key)
{
    const int half = (scale + 1) / 2;
    const uint64_t n = 1ULL << scale;
    uint64_t x = v;
    do {
        x = feistel(x, half, key);
    } while (x >= n);
    return (uint32_t)x;
}

static inline uint64_t prob_threshold(double p)
{
    if (p <= 0.0) return 0;
    if (p >= 1.0) return ~0ULL;
    return (uint64_t)ldexp(p, 64);
}

/* One R-MAT edge: at each of `scale` levels pick a quadrant of the adjacency
 * matrix, A = (top, left), B = (top, right), C = (bottom, left), D = rest. */
static inline void rmat_edge(uint64_t key, int scale, uint64_t e, uint64_t tA,
                             uint64_t tAB, uint64_t tABC, uint32_t *src,
                             uint32_t *dst)
{
    uint32_t s = 0, d = 0;
    for (int l = 0; l < scale; ++l) {
        const uint64_t r = splitmix64(key + ((e << 6) | (uint64_t)l));
        const uint32_t row = r >= tAB;
        const uint32_t colb = (r >= tA && r < tAB) || (r >= tABC);
        s = (s << 1) | row;
        d = (d << 1) | colb;
    }
    *src = s;
    *dst = d;
}

/* Raw generated edge list (before symmetrisation), for tests and tools. */
void gg_rmat_edges(int scale, int64_t n_edges, double A, double B, double C,
                   uint64_t seed, int relabel, uint32_t *src, uint32_t *dst)
{
    const uint64_t tA = prob_threshold(A), tAB = prob_threshold(A + B);
    const uint64_t tABC = prob_threshold(A + B + C);
    const uint64_t ekey = stream_key(seed, STREAM_EDGES);
    const uint64_t pkey = stream_key(seed, STREAM_PERM);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_edges; ++e) {
        uint32_t s, d;
        rmat_edge(ekey, scale, (uint64_t)e, tA, tAB, tABC, &s, &d);
        if (relabel) {
            s = gg_permute(s, scale, pkey);
            d = gg_permute(d, scale, pkey);
        }
        src[e] = s;
        dst[e] = d;
    }
}

/* ---------------------------------------------------------------------- */
/* Row sorting helpers (per-row neighbour lists are sorted ascending).     */

static void insertion_sort_u32(uint32_t *a, int64_t n)
{
    for (int64_t i = 1; i < n; ++i) {
        uint32_t x = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > x) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = x;
    }
}

/* LSD radix sort, 8 bits per pass, using tmp of the same length. */
static void radix_sort_u32(uint32_t *a, uint32_t *tmp, int64_t n, int bits)
{
    uint32_t *src = a, *dst = tmp;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        int64_t cnt[257];
        memset(cnt, 0, sizeof(cnt));
        for (int64_t i = 0; i < n; ++i) cnt[((src[i] >> shift) & 255u) + 1]++;
        for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
        for (int64_t i = 0; i < n; ++i) dst[cnt[(src[i] >> shift) & 255u]++] = src[i];
        uint32_t *t = src;
        src = dst;
        dst = t;
        passes++;
    }
    if (passes & 1) memcpy(a, src, (size_t)n * sizeof(uint32_t));
}

static void sort_row(uint32_t *a, uint32_t *tmp, int64_t n, int bits)
{
    if (n <= 48) insertion_sort_u32(a, n);
    else radix_sort_u32(a, tmp, n, bits);
}

/* ---------------------------------------------------------------------- */

/*
 * Symmetric CSR of an R-MAT graph.
 *
 * off must hold 2^scale + 1 int64; col must hold at least
 * 2 * edgefactor * 2^scale int32 (the bound before merging duplicates).
 * Returns the number of directed entries written (nnz), or -1 on allocation
 * failure / bad arguments.
 */
int64_t gg_rmat_csr(int scale, int edgefactor, double A, double B, double C,
                    uint64_t seed, int relabel, int64_t *off, int32_t *col)
{
    if (scale < 1 || scale > 30 || edgefactor < 1) return -1;
    const int64_t V = (int64_t)1 << scale;
    const int64_t M = (int64_t)edgefactor * V;
    const uint64_t tA = prob_threshold(A), tAB = prob_threshold(A + B);
    const uint64_t tABC = prob_threshold(A + B + C);
    const uint64_t ekey = stream_key(seed, STREAM_EDGES);
    const uint64_t pkey = stream_key(seed, STREAM_PERM);

    /* Bucket rows by their high bits so each bucket can be sorted alone. */
    int bbits = scale < 12 ? scale : 12;
    const int64_t NB = (int64_t)1 << bbits;
    const int rbits = scale - bbits; /* row bits inside a bucket */

    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    int64_t *hist = (int64_t *)calloc((size_t)nthreads * (size_t)NB, sizeof(int64_t));
    if (!hist) return -1;

    /* Pass 1: count directed entries per bucket, per thread. */
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int64_t *h = hist + (int64_t)tid * NB;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < M; ++e) {
            uint32_t s, d;
            rmat_edge(ekey, scale, (uint64_t)e, tA, tAB, tABC, &s, &d);
            if (relabel) {
                s = gg_permute(s, scale, pkey);
                d = gg_permute(d, scale, pkey);
            }
            if (s == d) continue;
            h[s >> rbits]++;
            h[d >> rbits]++;
        }
    }
    /* Bucket-major, thread-minor exclusive offsets. */
    int64_t *bstart = (int64_t *)malloc((size_t)(NB + 1) * sizeof(int64_t));
    if (!bstart) {
        free(hist);
        return -1;
    }
    int64_t total = 0;
    for (int64_t b = 0; b < NB; ++b) {
        bstart[b] = total;
        for (int t = 0; t < nthreads; ++t) {
            int64_t c = hist[(int64_t)t * NB + b];
            hist[(int64_t)t * NB + b] = total;
            total += c;
        }
    }
    bstart[NB] = total;

    /* Packed entries: (row within bucket) << 32 | neighbour. */
    uint64_t *ent = (uint64_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(uint64_t));
    if (!ent) {
        free(hist);
        free(bstart);
        return -1;
    }
    /* Pass 2: regenerate and scatter (same static schedule as pass 1). */
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int64_t *h = hist + (int64_t)tid * NB;
        const uint64_t rmask = (rbits >= 32) ? 0xffffffffULL : ((1ULL << rbits) - 1);
#pragma omp for schedule(static)
        for (int64_t e = 0; e < M; ++e) {
            uint32_t s, d;
            rmat_edge(ekey, scale, (uint64_t)e, tA, tAB, tABC, &s, &d);
            if (relabel) {
                s = gg_permute(s, scale, pkey);
                d = gg_permute(d, scale, pkey);
            }
            if (s == d) continue;
            ent[h[s >> rbits]++] = ((uint64_t)(s & rmask) << 32) | d;
            ent[h[d >> rbits]++] = ((uint64_t)(d & rmask) << 32) | s;
        }
    }
    free(hist);

    /* Pass 3: per bucket, counting-sort by row, sort + merge each row.
     * Unique neighbours are written back at the bucket's start as uint32,
     * and per-row unique counts go to off[row + 1]. */
    const int64_t RB = (int64_t)1 << rbits; /* rows per bucket */
    off[0] = 0;
#pragma omp parallel
    {
        int64_t *rcount = (int64_t *)malloc((size_t)(RB + 1) * sizeof(int64_t));
        uint32_t *rowbuf = NULL;
        uint32_t *tmp = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t b = 0; b < NB; ++b) {
            const int64_t lo = bstart[b], n = bstart[b + 1] - lo;
            if (n > cap) {
                free(rowbuf);
                free(tmp);
                cap = n;
                rowbuf = (uint32_t *)malloc((size_t)cap * sizeof(uint32_t));
                tmp = (uint32_t *)malloc((size_t)cap * sizeof(uint32_t));
            }
            memset(rcount, 0, (size_t)(RB + 1) * sizeof(int64_t));
            for (int64_t i = 0; i < n; ++i) rcount[(ent[lo + i] >> 32) + 1]++;
            for (int64_t r = 0; r < RB; ++r) rcount[r + 1] += rcount[r];
            for (int64_t i = 0; i < n; ++i) {
                uint64_t x = ent[lo + i];
                rowbuf[rcount[x >> 32]++] = (uint32_t)x;
            }
            /* rcount[r] now holds the end of row r; row r starts at rcount[r-1]. */
            uint32_t *outp = (uint32_t *)(ent + lo); /* reuse bucket storage */
            int64_t w = 0, start = 0;
            for (int64_t r = 0; r < RB; ++r) {
                const int64_t end = rcount[r];
                uint32_t *row = rowbuf + start;
                const int64_t len = end - start;
                sort_row(row, tmp, len, scale);
                int64_t u = 0;
                for (int64_t i = 0; i < len; ++i) {
                    if (i == 0 || row[i] != row[i - 1]) {
                        outp[w + u] = row[i];
                        u++;
                    }
                }
                off[b * RB + r + 1] = u;
                w += u;
                start = end;
            }
        }
        free(rcount);
        free(rowbuf);
        free(tmp);
    }
    /* Row offsets: inclusive scan of counts (serial; V + 1 entries). */
    for (int64_t v = 0; v < V; ++v) off[v + 1] += off[v];
    const int64_t nnz = off[V];
    /* Copy merged rows into col (buckets are in row order). */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < NB; ++b) {
        const uint32_t *src = (const uint32_t *)(ent + bstart[b]);
        const int64_t o = off[b * RB];
        const int64_t n = off[(b + 1) * RB] - o;
        memcpy(col + o, src, (size_t)n * sizeof(int32_t));
    }
    free(ent);
    free(bstart);
    return nnz;
}

/*
 * 4-neighbour 2-D grid of w x h vertices, id = row * w + column, rows sorted
 * (up, left, right, down). off: w*h+1 int64; col: 2*(2*w*h - w - h) int32.
 */
int64_t gg_grid_csr(int32_t w, int32_t h, int64_t *off, int32_t *col)
{
    if (w < 1 || h < 1) return -1;
    const int64_t V = (int64_t)w * h;
    off[0] = 0;
    for (int64_t v = 0; v < V; ++v) {
        const int32_t r = (int32_t)(v / w), c = (int32_t)(v % w);
        int deg = (r > 0) + (c > 0) + (c < w - 1) + (r < h - 1);
        off[v + 1] = off[v] + deg;
    }
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < V; ++v) {
        const int32_t r = (int32_t)(v / w), c = (int32_t)(v % w);
        int64_t o = off[v];
        if (r > 0) col[o++] = (int32_t)(v - w);
        if (c > 0) col[o++] = (int32_t)(v - 1);
        if (c < w - 1) col[o++] = (int32_t)(v + 1);
        if (r < h - 1) col[o++] = (int32_t)(v + w);
    }
    return off[V];
}

/*
 * n distinct roots drawn uniformly among vertices with degree > 0, in draw
 * order. Returns the number written (< n only if fewer such vertices exist).
 */
int32_t gg_pick_roots(int32_t V, const int64_t *off, int32_t n, uint64_t seed,
                      int32_t *out)
{
    const uint64_t key = stream_key(seed, STREAM_ROOTS);
    int64_t nonzero = 0;
    for (int64_t v = 0; v < V; ++v) nonzero += off[v + 1] > off[v];
    if (nonzero < n) n = (int32_t)nonzero;
    int32_t got = 0;
    for (uint64_t i = 0; got < n; ++i) {
        const uint64_t r = splitmix64(key + i);
        /* Lemire's multiply-high range reduction. */
        const int32_t v = (int32_t)(((unsigned __int128)r * (uint64_t)V) >> 64);
        if (off[v + 1] == off[v]) continue;
        int dup = 0;
        for (int32_t j = 0; j < got; ++j) dup |= out[j] == v;
        if (!dup) out[got++] = v;
    }
    return got;
}
