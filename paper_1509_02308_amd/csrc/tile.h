// tile.h -- set-partitioned replay of materialised traces (standard cache
// models): descriptors and launchers shared by tile_kernels.hip and the
// host scheduler in capi.hip.
#pragma once

#include "common.h"

namespace pc {

// Accesses per tile: one wave reads a tile, sorts its accesses to the lanes
// that own their sets, and the lanes replay them.
constexpr uint32_t kTile = 1024;
constexpr uint32_t kTileJ = kTile / kWave;
// State rows (dwords per lane) of the largest row class.
constexpr uint32_t kTileMaxRows = 512;

// One (pair, part) of a materialised replay.  A pair whose sets do not fit
// one wave's LDS is split into P = 2^lp parts; part p owns the sets s with
// s mod P == p and replays only their accesses.
struct TileItem {
    uint64_t start;       // first index of the trace in idx
    uint64_t len;         // accesses
    uint64_t base;        // byte address of element 0
    uint64_t count_from;  // first access counted in misses_steady
    uint64_t bitoff;      // word offset of the pair's hit bits
    uint32_t model;
    uint32_t trace_id;    // RANDOM counter word
    uint32_t out;         // pair index (counter slot)
    uint32_t part;        // part | lp << 16
};

struct TileArgs {
    const TileItem* items;
    uint32_t n_items;
    uint32_t persistent;     // 1: waves pull items from *queue; 0: block b runs item b
    uint32_t* queue;
    const DevModel* models;
    const int32_t* idx;
    uint64_t* misses;        // 2 per pair (parts of a split pair add into zeroed counters)
    uint32_t* bits;          // or NULL
    uint32_t rows;           // state dwords per lane of this launch's row class
    const volatile uint32_t* abort_flag;
    uint32_t* status;        // bit 0: aborted, bit 1: negative index seen
};

// Layout of one (pair, part) in a wave.  The part's T_p sets are spread over
// G = min(64, largest power of two <= T_p) lane groups of W = 64 / G lanes:
// set u of the part belongs to group (u + u / G) mod G, in slot u / G of that
// group; lane r of a group holds ways r, r + W, r + 2W, ... of each of its
// sets (kw = ceil(a / W) of them).  Per set and lane: LRU kw 8-byte (tag,
// last-use stamp) entries; the others kw tags, then (used by the group's
// first lane) FIFO one insertion pointer or tree-PLRU ceil((a-1)/32)
// node-bit words.
struct TileLayout {
    uint32_t lg;      // log2 G
    uint32_t lw;      // log2 W
    uint32_t kw;      // ways per lane per set
    uint32_t rs;      // dword rows per set and lane
    uint32_t slots;   // sets per group (rounded up)
};
__host__ __device__ inline TileLayout tile_layout(int pol, uint32_t a, uint32_t sets, uint32_t lp, uint32_t part) {
    TileLayout L;
    const uint32_t tp = (sets - part + (1u << lp) - 1) >> lp;
    L.lg = 0;
    while (L.lg < 6 && (2u << L.lg) <= tp) ++L.lg;
    L.lw = 6 - L.lg;
    L.kw = (a + (1u << L.lw) - 1) >> L.lw;
    const uint32_t meta = pol == PCHASE_FIFO ? 1u : pol == PCHASE_PLRU ? (a + 30) / 32 : 0u;
    L.rs = pol == PCHASE_LRU ? 2 * L.kw : L.kw + meta;
    L.slots = (tp + (1u << L.lg) - 1) >> L.lg;
    return L;
}
// Way classes of the kernels: per-lane ways read per unrolled chunk 1, 2,
// 4, 8, 16.
constexpr int kTileWayClasses = 5;
__host__ __device__ inline int tile_way_class(uint32_t kw) {
    return kw <= 1 ? 0 : kw <= 2 ? 1 : kw <= 4 ? 2 : kw <= 8 ? 3 : 4;
}
size_t tile_lds_bytes(uint32_t rows);
hipError_t launch_tile(int pol, int wcls, const TileArgs& a, uint32_t blocks, hipStream_t s);
hipError_t tile_occupancy(int pol, int wcls, uint32_t rows, int* blocks_per_cu);
hipError_t tile_prepare_lds();

}  // namespace pc
