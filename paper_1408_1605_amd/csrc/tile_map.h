// Edge -> thread mapping of one tile of frontier edges (device code).
//
// The frontier entries k = 0..qlen-1 have an exclusive cumulative degree
// array cumul; frontier edge e belongs to entry k = max{l : cumul[l] <= e}
// and is the (e - cumul[k])-th neighbour of that entry's row (Section 3.4:
// the mapping formula, read with the exclusive scan, and Algorithm 3).  The
// degree scan also stores, per entry, its row start (rowstart[k]) and the id
// reported as parent (uid[k]), so mapping a tile needs no dependent gathers.
//
// A workgroup owns the tile of TILE = 256 * EPT consecutive edges
// [e0, e0 + TILE).  tile_k[t] is the entry holding edge t * TILE, so the
// entries overlapping tile t are tile_k[t] .. tile_k[t + 1].  They are staged
// in LDS; each thread binary-searches the staged cumulative degrees once for
// its first slot and then advances linearly over EPT consecutive slots
// (Section 3.4.1), recording slot -> entry in LDS.  Edges are then read with
// a slot stride of 256 so a wave's 64 column loads are contiguous.
//
// A tile's staging entries are fetched into registers one tile ahead
// (fetch_stage), so their latency overlaps the previous tile's probes.
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
    static constexpr int PER = (CAP + 1 + kWG - 1) / kWG;  // entries per thread
    int32_t cum[CAP + 1];
    int32_t uid[CAP + 1];     // id reported for the entry (parent value)
    int64_t base[CAP + 1];    // row start minus cumulative degree
    uint16_t map[TILE];
};

template <int EPT>
struct StageRegs {
    int32_t tile, k_lo, k_hi;
    int64_t cum[TileLds<EPT>::PER];
    int64_t rs[TileLds<EPT>::PER];
    int32_t uid[TileLds<EPT>::PER];
};

// Issue the loads of tile `tile`'s staging entries (tile >= ntiles: a
// harmless in-range load, marked invalid).  The loads are unconditional,
// with indices clamped into [k_lo, k_hi], so the compiler can count them
// and wait for earlier loads without waiting for these.
template <int EPT>
__device__ __forceinline__ StageRegs<EPT> fetch_stage(int32_t tile, int32_t ntiles,
                                                      const int64_t* __restrict__ cumul,
                                                      const int64_t* __restrict__ rowstart,
                                                      const int32_t* __restrict__ uidv,
                                                      const int32_t* __restrict__ tile_k)
{
    StageRegs<EPT> R;
    const bool valid = tile < ntiles;
    R.tile = valid ? tile : -1;
    const int32_t t = valid ? tile : 0;
    R.k_lo = valid ? tile_k[t] : 0;
    R.k_hi = valid ? tile_k[t + 1] : 0;
#pragma unroll
    for (int m = 0; m < TileLds<EPT>::PER; ++m) {
        int32_t k = R.k_lo + (int32_t)threadIdx.x + m * kWG;
        k = k < R.k_hi ? k : R.k_hi;
        R.cum[m] = cumul[k];
        R.rs[m] = rowstart[k];
        R.uid[m] = uidv[k];
    }
    return R;
}

// Map tile R.tile and load its column values: for j < EPT, slot
// threadIdx.x + j * 256 gives ok[j] (a real edge), uid[j] (the entry's
// reported id), col_val[j] (the neighbour) and eidx[j] (the edge index).
// Every thread of the workgroup must call it (it contains barriers); the
// caller must barrier before the next call reuses L.
template <int EPT>
__device__ __forceinline__ void map_tile(TileLds<EPT>& L, const StageRegs<EPT>& R, int64_t r,
                                         const int64_t* __restrict__ cumul,
                                         const int64_t* __restrict__ rowstart,
                                         const int32_t* __restrict__ uidv,
                                         const int32_t* __restrict__ col,
                                         int32_t uid[EPT], int32_t col_val[EPT], bool ok[EPT],
                                         int64_t eidx[EPT])
{
    constexpr int TILE = TileLds<EPT>::TILE;
    const int64_t e0 = (int64_t)R.tile * TILE;
    const int64_t rem = r - e0;
    const int32_t n_e = rem < TILE ? (int32_t)rem : TILE;
    const int32_t k_lo = R.k_lo, k_hi = R.k_hi;
    const int32_t n_k = k_hi - k_lo + 1;

    if (n_k <= TileLds<EPT>::CAP + 1) {
#pragma unroll
        for (int m = 0; m < TileLds<EPT>::PER; ++m) {
            const int32_t i = threadIdx.x + m * kWG;
            if (i < n_k) {
                const int64_t rel = R.cum[m] - e0;
                L.cum[i] = rel > 0 ? (int32_t)rel : 0;
                L.uid[i] = R.uid[m];
                L.base[i] = R.rs[m] - R.cum[m];
            }
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
        // unconditional loads: slots past the tile's last edge re-read it
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int32_t sl0 = threadIdx.x + j * kWG;
            ok[j] = sl0 < n_e;
            const int32_t sl = ok[j] ? sl0 : n_e - 1;
            eidx[j] = e0 + sl0;
            const int32_t i = L.map[sl];
            uid[j] = L.uid[i];
            col_val[j] = __builtin_nontemporal_load(col + (L.base[i] + e0 + sl));
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
                uid[j] = uidv[lo];
                col_val[j] = col[rowstart[lo] + (e - cumul[lo])];
            }
        }
    }
}

}  // namespace bfsmi
