/*
 * CPU oracle for the level-synchronous BFS (TEST INFRASTRUCTURE ONLY).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  The GPU library never links or calls it, and it
 * includes nothing from the GPU library.
 *
 * What is computed.  For a CSR graph and a root r:
 *   level[v]  = number of edges on a shortest path from r to v, or -1 when v
 *               is not reachable (level[r] = 0);
 *   parent[v] = r for v = r, -1 for unreachable v, otherwise the vertex u
 *               through which v was first discovered (an in-neighbour of v
 *               with level[u] = level[v] - 1).
 * This is the output of the paper's search (Algorithm 1 with a single
 * processor, R = C = 1; initialisation as in Algorithm 2): level, pred and
 * the visited bitmap start at -1, -1, 0; the root gets level 0, pred = itself
 * and its visited bit; the current level counter starts at 1; each round
 * scans the edge list of every frontier vertex, and every neighbour whose
 * visited bit is clear is marked visited, given the scanning vertex as
 * predecessor and the current level, and joins the next frontier; the search
 * stops when the next frontier is empty.  Levels are unique; predecessors are
 * one valid choice among several (first discoverer in frontier order, rows
 * scanned in stored order).
 *
 * The validator checks a (level, parent) pair against the graph without
 * running a search: it is the tree check described with the benchmark's
 * validation (Section 3.2 states results are validated; the invariants are
 * the standard BFS-tree properties):
 *   V1 level[r] = 0 and parent[r] = r;
 *   V2 every reached v != r has parent[v] = u with (u, v) an edge;
 *   V3 ... and level[u] = level[v] - 1;
 *   V4 every edge (u, v): undirected graphs: both ends reached with
 *      |level[u] - level[v]| <= 1, or both unreached; directed graphs:
 *      u reached implies v reached and level[v] <= level[u] + 1;
 *   V5 (undirected) the reached set is exactly r's connected component,
 *      computed by union-find, an algorithm independent of BFS;
 *   V6 unreached vertices have level -1 and parent -1, and no level is
 *      below -1.
 * V1 + V2/V3 + V4 together force level[] to equal the hop distance.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

/* Serial BFS.  frontier_sizes (nullable, capacity V + 1) receives the size
 * of each level's frontier, level 0 first.  Returns the number of levels
 * (number of non-empty frontiers), or -1 on bad arguments / no memory.
 * *edges_scanned receives the sum of out-degrees of reached vertices. */
int32_t oracle_bfs(int32_t V, const int64_t *off, const int32_t *col,
                   int32_t root, int32_t *level, int32_t *pred,
                   int64_t *frontier_sizes, int64_t *edges_scanned)
{
    if (V <= 0 || root < 0 || root >= V || !off || !level || !pred) return -1;
    uint8_t *bmap = (uint8_t *)calloc((size_t)V, 1);
    int32_t *front = (int32_t *)malloc((size_t)V * sizeof(int32_t));
    int32_t *next = (int32_t *)malloc((size_t)V * sizeof(int32_t));
    if (!bmap || !front || !next) {
        free(bmap);
        free(front);
        free(next);
        return -1;
    }
    for (int32_t v = 0; v < V; ++v) {
        level[v] = -1;
        pred[v] = -1;
    }
    int64_t nfront = 0, scanned = 0;
    level[root] = 0;
    pred[root] = root;
    bmap[root] = 1;
    front[nfront++] = root;
    int32_t nlevels = 0;
    int32_t lvl = 1;
    while (1) {
        if (frontier_sizes) frontier_sizes[nlevels] = nfront;
        nlevels++;
        int64_t nnext = 0;
        for (int64_t i = 0; i < nfront; ++i) {
            const int32_t u = front[i];
            scanned += off[u + 1] - off[u];
            for (int64_t e = off[u]; e < off[u + 1]; ++e) {
                const int32_t v = col[e];
                if (bmap[v] == 0) {
                    bmap[v] = 1;
                    pred[v] = u;
                    level[v] = lvl;
                    next[nnext++] = v;
                }
            }
        }
        if (nnext == 0) break;
        int32_t *t = front;
        front = next;
        next = t;
        nfront = nnext;
        lvl++;
    }
    if (edges_scanned) *edges_scanned = scanned;
    free(bmap);
    free(front);
    free(next);
    return nlevels;
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
 * allows binary search for edge membership.  -1 on no memory / bad args.
 */
int32_t oracle_validate(int32_t V, const int64_t *off, const int32_t *col,
                        int32_t root, const int32_t *level,
                        const int32_t *parent, int32_t directed,
                        int32_t rows_sorted, int32_t *bad_vertex)
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
    if (!directed) {
        int32_t *comp = (int32_t *)malloc((size_t)V * sizeof(int32_t));
        if (!comp) return -1;
        if (oracle_components(V, off, col, comp) != 0) {
            free(comp);
            return -1;
        }
        const int32_t rc = comp[root];
        for (int32_t v = 0; v < V; ++v) {
            if ((comp[v] == rc) != (level[v] >= 0)) {
                *bad_vertex = v;
                free(comp);
                return 5;
            }
        }
        free(comp);
    }
    return 0;
}
