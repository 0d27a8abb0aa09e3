// Edge -> thread mapping of one tile of frontier edges (device code).
//
// The frontier entries Q[0..qlen) have an exclusive cumulative degree array
// cumul; frontier edge e belongs to entry k = max{l : cumul[l] <= e} and is
// the (e - cumul[k])-th neighbour of that entry's row (Section 3.4: the
// mapping formula, read with the exclusive scan, and Algorithm 3).
//
// A workgroup owns the tile of TILE = 256 * EPT consecutive edges
// [e0, e0 + TILE).  tile_k[t] is the entry holding edge t * TILE, so the
// entries overlapping tile t are tile_k[t] .. tile_k[t + 1].  They are staged
// in LDS; each thread binary-searches the staged cumulative degrees once for
// its first slot and then advances linearly over EPT consecutive slots
// (Section 3.4.1), recording slot -> entry in LDS.  Edges are then read with
// a slot stride of 256 so a wave's 64 column loads are contiguous.
#pragma once

#include "bfs_internal.h"

namespace bfsmi {

// Staging holds up to CAP + 1 frontier entries per tile.  A tile that
// overlaps more entries (frontier vertices of degree < 2 on average) uses
// the global search path instead, so LDS stays small and occupancy high.
template <int EPT>
struct TileLds {
    static constexpr int TILE = kWG * EPT;
    static constexpr int CAP = TILE / 2;
    int32_t cum[CAP + 1];
    int32_t uid[CAP + 1];     // id reported for the entry (parent value)
    int64_t base[CAP + 1];    // row start minus cumulative degree
    uint16_t map[TILE];
};

// Fills, for j < EPT, the edge slot threadIdx.x + j * 256 of tile `tile`:
// ok[j] (slot is a real edge), uid[j] (the entry's id, mapped through
// uid_map when it is not null), col_val[j] (the neighbour read from col) and
// eidx[j] (the global edge index).  Every thread of the workgroup must call
// it (it contains barriers); the caller must barrier before reusing L.
template <int EPT>
__device__ __forceinline__ void map_tile(TileLds<EPT>& L, int32_t tile, int64_t r,
                                         const int32_t* __restrict__ Q,
                                         const int64_t* __restrict__ cumul,
                                         const int32_t* __restrict__ tile_k,
                                         const int64_t* __restrict__ off,
                                         const int32_t* __restrict__ col,
                                         const int32_t* __restrict__ uid_map,
                                         int32_t uid[EPT], int32_t col_val[EPT], bool ok[EPT],
                                         int64_t eidx[EPT])
{
    constexpr int TILE = TileLds<EPT>::TILE;
    const int64_t e0 = (int64_t)tile * TILE;
    const int64_t rem = r - e0;
    const int32_t n_e = rem < TILE ? (int32_t)rem : TILE;
    const int32_t k_lo = tile_k[tile];
    const int32_t k_hi = tile_k[tile + 1];
    const int32_t n_k = k_hi - k_lo + 1;

    if (n_k <= TileLds<EPT>::CAP + 1) {
        for (int32_t i = threadIdx.x; i < n_k; i += kWG) {
            const int32_t k = k_lo + i;
            const int32_t x = Q[k];
            const int64_t c = cumul[k];
            const int64_t rel = c - e0;
            L.cum[i] = rel > 0 ? (int32_t)rel : 0;
            L.uid[i] = uid_map ? uid_map[x] : x;
            L.base[i] = off[x] - c;
        }
        __syncthreads();
        const int32_t s0 = threadIdx.x * EPT;
        if (s0 < n_e) {
            int32_t lo = 0, hi = n_k - 1;  // L.cum[0] == 0 <= s0
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (L.cum[mid] <= s0) lo = mid;
                else hi = mid - 1;
            }
            int32_t i = lo;
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const int32_t sl = s0 + j;
                if (sl < n_e) {
                    while (i + 1 < n_k && L.cum[i + 1] <= sl) ++i;
                    L.map[sl] = (uint16_t)i;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int32_t sl = threadIdx.x + j * kWG;
            ok[j] = sl < n_e;
            uid[j] = 0;
            col_val[j] = 0;
            eidx[j] = e0 + sl;
            if (ok[j]) {
                const int32_t i = L.map[sl];
                uid[j] = L.uid[i];
                col_val[j] = __builtin_nontemporal_load(col + (L.base[i] + e0 + sl));
            }
        }
    } else {
        // More entries than the staging holds (low-degree or zero-degree
        // entries): search the global cumulative array for each edge.
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int32_t sl = threadIdx.x + j * kWG;
            ok[j] = sl < n_e;
            uid[j] = 0;
            col_val[j] = 0;
            eidx[j] = e0 + sl;
            if (ok[j]) {
                const int64_t e = e0 + sl;
                int32_t lo = k_lo, hi = k_hi;
                while (lo < hi) {
                    const int32_t mid = lo + ((hi - lo + 1) >> 1);
                    if (cumul[mid] <= e) lo = mid;
                    else hi = mid - 1;
                }
                const int32_t x = Q[lo];
                uid[j] = uid_map ? uid_map[x] : x;
                col_val[j] = col[off[x] + (e - cumul[lo])];
            }
        }
    }
}

}  // namespace bfsmi
