/*
 * Host-side memory and undefined-behaviour check of the two C libraries the
 * tests load (the seeded graph generator and the CPU oracle): built with
 * AddressSanitizer and UBSan by tests/test_sanitizers.py and run on small
 * graphs, including the edge cases (one vertex, isolated vertices, a root
 * with no edges, directed input, duplicates and self-loops).
 * Exit status 0 means every call returned the expected value and the
 * sanitizers reported nothing.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t gg_rmat_csr(int scale, int edgefactor, double A, double B, double C,
                    uint64_t seed, int relabel, int64_t *off, int32_t *col);
int64_t gg_grid_csr(int32_t w, int32_t h, int64_t *off, int32_t *col);
int32_t gg_pick_roots(int32_t V, const int64_t *off, int32_t n, uint64_t seed, int32_t *out);
int32_t oracle_bfs(int32_t V, const int64_t *off, const int32_t *col, int32_t root,
                   int32_t *level, int32_t *parent, int64_t *frontier_sizes,
                   int64_t *edges_scanned);
int32_t oracle_components(int32_t V, const int64_t *off, const int32_t *col, int32_t *comp);
int32_t oracle_validate(int32_t V, const int64_t *off, const int32_t *col, int32_t root,
                        const int32_t *level, const int32_t *parent, int32_t directed,
                        int32_t rows_sorted, const int32_t *comp, int32_t *bad_vertex);

static int failures = 0;
#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            failures++;                                                \
        }                                                              \
    } while (0)

/* every root of the graph: search, validate with and without labels */
static void all_roots(int32_t V, const int64_t *off, const int32_t *col, int directed,
                      int32_t max_roots)
{
    int32_t *lv = malloc(sizeof(int32_t) * V), *pa = malloc(sizeof(int32_t) * V);
    int32_t *comp = malloc(sizeof(int32_t) * V);
    int64_t *fs = malloc(sizeof(int64_t) * (V + 1));
    CHECK(oracle_components(V, off, col, comp) == 0);
    for (int32_t r = 0; r < V && r < max_roots; ++r) {
        int64_t scanned = -1;
        int32_t n = oracle_bfs(V, off, col, r, lv, pa, fs, &scanned);
        CHECK(n >= 1 && n <= V);
        int64_t tot = 0;
        for (int32_t i = 0; i < n; ++i) tot += fs[i];
        int64_t reached = 0, deg = 0;
        for (int32_t v = 0; v < V; ++v)
            if (lv[v] >= 0) {
                reached++;
                deg += off[v + 1] - off[v];
            }
        CHECK(tot == reached && deg == scanned);
        int32_t bad = -2;
        CHECK(oracle_validate(V, off, col, r, lv, pa, directed, 1, NULL, &bad) == 0);
        if (!directed) CHECK(oracle_validate(V, off, col, r, lv, pa, 0, 0, comp, &bad) == 0);
    }
    /* nullable outputs and bad arguments */
    CHECK(oracle_bfs(V, off, col, 0, lv, pa, NULL, NULL) >= 1);
    CHECK(oracle_bfs(V, off, col, V, lv, pa, fs, NULL) == -1);
    CHECK(oracle_bfs(V, off, col, -1, lv, pa, fs, NULL) == -1);
    CHECK(oracle_validate(V, off, col, V, lv, pa, directed, 1, NULL, NULL) == -1);
    free(lv);
    free(pa);
    free(comp);
    free(fs);
}

int main(void)
{
#ifdef SANITIZER_SELF_TEST
    /* a planted heap overflow: the sanitizer must stop the run here */
    {
        int32_t *a = malloc(sizeof(int32_t) * 4);
        volatile int32_t i = 4;
        a[i] = 1;
        free(a);
    }
#endif
    /* R-MAT scale 10, then its roots */
    {
        const int scale = 10, ef = 16;
        const int32_t V = 1 << scale;
        int64_t *off = malloc(sizeof(int64_t) * (V + 1));
        int32_t *col = malloc(sizeof(int32_t) * 2 * ef * V);
        int64_t nnz = gg_rmat_csr(scale, ef, 0.57, 0.19, 0.19, 1010, 1, off, col);
        CHECK(nnz > 0 && off[V] == nnz);
        int32_t roots[8];
        CHECK(gg_pick_roots(V, off, 8, 2010, roots) == 8);
        all_roots(V, off, col, 0, 64);
        CHECK(gg_rmat_csr(0, ef, 0.57, 0.19, 0.19, 1, 1, off, col) == -1);
        free(off);
        free(col);
    }
    /* grids, including one vertex and one row */
    {
        const int32_t dims[3][2] = {{7, 5}, {1, 1}, {9, 1}};
        for (int i = 0; i < 3; ++i) {
            const int32_t w = dims[i][0], h = dims[i][1], V = w * h;
            int64_t *off = malloc(sizeof(int64_t) * (V + 1));
            int32_t *col = malloc(sizeof(int32_t) * (2 * (2 * V - w - h) + 1));
            CHECK(gg_grid_csr(w, h, off, col) == 2 * (2 * (int64_t)V - w - h));
            all_roots(V, off, col, 0, V);
            free(off);
            free(col);
        }
    }
    /* directed 5-cycle 0->1->2->3->4->0 plus an isolated vertex 5,
     * a self-loop on 2 and a duplicated edge 0->1 */
    {
        const int64_t off[7] = {0, 2, 3, 5, 6, 7, 7};
        const int32_t col[7] = {1, 1, 2, 2, 3, 4, 0};
        all_roots(6, off, col, 1, 6);
        int32_t roots[6];
        CHECK(gg_pick_roots(6, off, 6, 3, roots) == 5); /* vertex 5 has no edges */
    }
    if (failures) fprintf(stderr, "%d checks failed\n", failures);
    return failures ? 1 : 0;
}
