/*
 * CPU oracle for the level-synchronous BFS (TEST INFRASTRUCTURE ONLY).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  The GPU library never links or calls it, and it
 * includes nothing from the GPU library.
 *
 * What is computed.  For a CSR graph and a root r the search of the paper
 * (Algorithms 1 and 2, any processor grid) outputs
 *   level[v]  = the hop distance from r to v along out-edges (the number of
 *               edges of a shortest path), -1 when v is not reachable;
 *   parent[v] = r for v = r, -1 for unreachable v, otherwise some u with
 *               (u, v) an edge and level[u] = level[v] - 1.
 * level[] has exactly one correct value, so the oracle computes it from its
 * definition with the textbook first-in first-out traversal: vertices leave
 * the queue in non-decreasing distance order, and a vertex's distance is
 * fixed when it is first seen, at one more than the distance of the vertex
 * being scanned.  parent[] is one valid choice (the vertex that first saw
 * it); the paper's atomic claim may pick another, so parents elsewhere are
 * checked with the validator below, never compared.
 *
 * The validator checks a (level, parent) pair against the graph without
 * running a search: it is the tree check of the benchmark's validation
 * (Section 3.2 states results are validated; the invariants are the
 * standard BFS-tree properties):
 *   V1 level[r] = 0 and parent[r] = r;
 *   V2 every reached v != r has parent[v] = u with (u, v) an edge;
 *   V3 ... and level[u] = level[v] - 1;
 *   V4 every edge (u, v): undirected graphs: both ends reached with
 *      |level[u] - level[v]| <= 1, or both unreached; directed graphs:
 *      u reached implies v reached and level[v] <= level[u] + 1;
 *   V5 (undirected, optional) the reached set is exactly r's connected
 *      component as labelled by a caller-supplied comp[] (union-find below,
 *      an algorithm independent of BFS).  V2 + V3 connect every reached
 *      vertex to r and V4 closes the reached set under adjacency, so V5
 *      cannot fail first: it is a cross-check of the others, not a
 *      separate invariant;
 *   V6 unreached vertices have level -1 and parent -1, and no level is
 *      below -1.
 * V1 + V2/V3 + V4 together force level[] to equal the hop distance.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

/* Hop distances from root by a first-in first-out traversal.
 * frontier_sizes (nullable, capacity V + 1) receives the number of vertices
 * at each distance, 0 first.  Returns the number of distinct distances
 * (the search's level count), or -1 on bad arguments / no memory.
 * *edges_scanned receives the sum of out-degrees of reached vertices. */
int32_t oracle_bfs(int32_t V, const int64_t *off, const int32_t *col,
                   int32_t root, int32_t *level, int32_t *parent,
                   int64_t *frontier_sizes, int64_t *edges_scanned)
{
    if (V <= 0 || root < 0 || root >= V || !off || !level || !parent) return -1;
    int32_t *fifo = (int32_t *)malloc((size_t)V * sizeof(int32_t));
    if (!fifo) return -1;
    memset(level, 0xff, (size_t)V * sizeof(int32_t));   /* all -1 */
    memset(parent, 0xff, (size_t)V * sizeof(int32_t));
    level[root] = 0;
    parent[root] = root;
    int64_t head = 0, tail = 0, degsum = 0;
    fifo[tail++] = root;
    while (head < tail) {
        const int32_t x = fifo[head++];
        const int32_t dx = level[x];
        const int64_t a = off[x], b = off[x + 1];
        degsum += b - a;
        for (int64_t e = a; e < b; ++e) {
            const int32_t y = col[e];
            if (level[y] < 0) {
                level[y] = dx + 1;
                parent[y] = x;
                fifo[tail++] = y;
            }
        }
    }
    /* the queue holds every reached vertex once, in distance order */
    const int32_t depth = level[fifo[tail - 1]];
    if (frontier_sizes) {
        for (int32_t d = 0; d <= depth; ++d) frontier_sizes[d] = 0;
        for (int64_t i = 0; i < tail; ++i) frontier_sizes[level[fifo[i]]]++;
    }
    if (edges_scanned) *edges_scanned = degsum;
    free(fifo);
    return depth + 1;
}

/* Union-find with path halving and union by size. */
static int32_t uf_find(int32_t *p, int32_t x)
{
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

/* comp[v] = smallest vertex id of v's connected component (undirected view
 * of the edge list).  Returns 0, or -1 on no memory. */
int32_t oracle_components(int32_t V, const int64_t *off, const int32_t *col,
                          int32_t *comp)
{
    int32_t *p = (int32_t *)malloc((size_t)V * sizeof(int32_t));
    int32_t *sz = (int32_t *)malloc((size_t)V * sizeof(int32_t));
    if (!p || !sz) {
        free(p);
        free(sz);
        return -1;
    }
    for (int32_t v = 0; v < V; ++v) {
        p[v] = v;
        sz[v] = 1;
    }
    for (int32_t u = 0; u < V; ++u) {
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            int32_t a = uf_find(p, u), b = uf_find(p, col[e]);
            if (a == b) continue;
            if (sz[a] < sz[b]) {
                int32_t t = a;
                a = b;
                b = t;
            }
            p[b] = a;
            sz[a] += sz[b];
        }
    }
    /* label each component by its smallest member */
    for (int32_t v = 0; v < V; ++v) sz[v] = INT32_MAX;
    for (int32_t v = 0; v < V; ++v) {
        int32_t r = uf_find(p, v);
        if (v < sz[r]) sz[r] = v;
    }
    for (int32_t v = 0; v < V; ++v) comp[v] = sz[uf_find(p, v)];
    free(p);
    free(sz);
    return 0;
}

/* Binary search for x in the sorted row of u; linear scan if unsorted. */
static int has_edge(const int64_t *off, const int32_t *col, int32_t u, int32_t x,
                    int sorted)
{
    int64_t lo = off[u], hi = off[u + 1];
    if (!sorted) {
        for (int64_t e = lo; e < hi; ++e)
            if (col[e] == x) return 1;
        return 0;
    }
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < off[u + 1] && col[lo] == x;
}

/*
 * Validate a BFS result.  Returns 0 when every invariant holds, otherwise the
 * number (1..6) of the first failing invariant, with *bad_vertex set to an
 * offending vertex.  directed = 0 assumes a symmetric graph.  rows_sorted
 * allows binary search for edge membership.  comp (nullable, undirected
 * only) enables V5 against those component labels.  -1 on bad args.
 */
int32_t oracle_validate(int32_t V, const int64_t *off, const int32_t *col,
                        int32_t root, const int32_t *level,
                        const int32_t *parent, int32_t directed,
                        int32_t rows_sorted, const int32_t *comp,
                        int32_t *bad_vertex)
{
    int32_t dummy;
    if (!bad_vertex) bad_vertex = &dummy;
    *bad_vertex = -1;
    if (V <= 0 || root < 0 || root >= V) return -1;
    /* V1 */
    if (level[root] != 0 || parent[root] != root) {
        *bad_vertex = root;
        return 1;
    }
    /* V6 */
    for (int32_t v = 0; v < V; ++v) {
        if (level[v] < -1 || ((level[v] == -1) != (parent[v] == -1))) {
            *bad_vertex = v;
            return 6;
        }
    }
    /* V2, V3 */
    for (int32_t v = 0; v < V; ++v) {
        if (v == root || level[v] < 0) continue;
        const int32_t u = parent[v];
        if (u < 0 || u >= V) {
            *bad_vertex = v;
            return 2;
        }
        /* edge (u, v): in a symmetric graph look in v's row (same answer) */
        int ok = directed ? has_edge(off, col, u, v, rows_sorted)
                          : has_edge(off, col, v, u, rows_sorted);
        if (!ok) {
            *bad_vertex = v;
            return 2;
        }
        if (level[u] != level[v] - 1) {
            *bad_vertex = v;
            return 3;
        }
    }
    /* V4 */
    for (int32_t u = 0; u < V; ++u) {
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            const int32_t v = col[e];
            const int32_t lu = level[u], lv = level[v];
            if (directed) {
                if (lu >= 0 && (lv < 0 || lv > lu + 1)) {
                    *bad_vertex = v;
                    return 4;
                }
            } else {
                if ((lu < 0) != (lv < 0)) {
                    *bad_vertex = lu < 0 ? u : v;
                    return 4;
                }
                if (lu >= 0 && (lu - lv > 1 || lv - lu > 1)) {
                    *bad_vertex = v;
                    return 4;
                }
            }
        }
    }
    /* V5 */
    if (!directed && comp) {
        const int32_t rc = comp[root];
        for (int32_t v = 0; v < V; ++v) {
            if ((comp[v] == rc) != (level[v] >= 0)) {
                *bad_vertex = v;
                return 5;
            }
        }
    }
    return 0;
}
