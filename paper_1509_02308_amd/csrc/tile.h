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

// Per-set rows: a tags, then the policy's state: LRU a last-use stamps,
// FIFO one insertion pointer, tree-PLRU ceil((a-1)/32) node-bit words.
__host__ __device__ inline uint32_t tile_meta_rows(int pol, uint32_t a) {
    return pol == PCHASE_LRU ? a : pol == PCHASE_FIFO ? 1u : pol == PCHASE_PLRU ? (a + 30) / 32 : 0u;
}
size_t tile_lds_bytes(uint32_t rows);
hipError_t launch_tile(int pol, const TileArgs& a, uint32_t blocks, hipStream_t s);
hipError_t tile_occupancy(int pol, uint32_t rows, int* blocks_per_cu);
hipError_t tile_prepare_lds();

}  // namespace pc
