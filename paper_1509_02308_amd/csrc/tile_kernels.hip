// tile_kernels.hip -- set-partitioned replay of materialised index traces
// through standard set-associative models (Mei & Chu, Section 4.1,
// Assumptions 1-3, with the non-LRU policies of Sections 4.5-4.6).
//
// The hit or miss of an access depends only on the earlier accesses of its
// own set (the set of address x is (x >> unit) mod T, and a set's a ways are
// touched by nothing else).  So a pair is replayed by one wave whose 64
// lanes own disjoint groups of sets, each lane holding the state of its sets
// in an LDS column (row r of lane l at dword 64 r + l: no two lanes share a
// bank), and replaying only the accesses of its own sets, in trace order.
//
// The trace streams through in tiles of kTile accesses, read coalesced (lane
// l takes accesses 64 j + l of the tile).  Per tile:
//   1. every access gets its line and set; an access to the same line as the
//      access just before it in the trace is a hit that changes no policy's
//      state (the way is already the most recently used one, FIFO and random
//      replacement ignore hits, and the tree-PLRU path bits already point
//      away from it), so its hit bit is set at once;
//   2. the remaining accesses ("heads") are counting-sorted by owner lane,
//      stably: a bucket histogram, its prefix over the lanes, then the
//      position of each head = its bucket's cursor + the number of lower
//      lanes with a head for the same bucket in the same row (ballots);
//   3. each lane replays its bucket in order against its LDS state;
//   4. the tile's hit bits go out as whole words.
// A pair whose state does not fit one wave's LDS is split into P = 2^lp
// parts (part p owns sets s with s mod P == p); the parts read the whole
// trace each, keep only their own sets' accesses and merge their outputs.
#include "sweep_lane.h"
#include "tile.h"

namespace pc {

struct TileLds {
    uint32_t* state;    // rows x 64
    uint32_t* line;     // kTile: line of each sorted head
    uint32_t* info;     // kTile: tile offset | (first row of its set) << 10
    uint32_t* tbits;    // kTile / 32: hit bits of the tile
    uint32_t* bcnt;     // 64: heads per owner lane
    uint32_t* cursor;   // 64: next free slot of each owner's bucket
};

size_t tile_lds_bytes(uint32_t rows) {
    return ((size_t)rows * kWave + 2 * kTile + kTile / 32 + 2 * kWave) * 4;
}

// Replays one head against the lane's column `col` (row r at col[64 r]);
// the set's rows start at rowb.  k is the access index within the pair.
template <int POL>
__device__ __forceinline__ bool tile_access(uint32_t* col, uint32_t rowb, uint32_t line, uint32_t a,
                                            uint64_t k, const DevModel& m, uint32_t trace_id) {
    uint32_t* tg = col + (size_t)rowb * kWave;
    if constexpr (POL == PCHASE_LRU) {
        // one pass: the hit way, and the way with the oldest last-use stamp
        // (empty ways have stamp 0 and fill lowest index first; used ways
        // have stamp k + 1 >= 1, distinct)
        uint32_t* st = tg + (size_t)a * kWave;
        uint32_t hw = kInvalidTag, vw = 0, vs = 0xFFFFFFFFu;
        for (uint32_t w = 0; w < a; ++w) {
            const uint32_t t = tg[(size_t)w * kWave], s = st[(size_t)w * kWave];
            if (t == line) hw = w;
            if (s < vs) {
                vs = s;
                vw = w;
            }
        }
        const uint32_t stamp = (uint32_t)k + 1u;
        if (hw != kInvalidTag) {
            st[(size_t)hw * kWave] = stamp;
            return true;
        }
        tg[(size_t)vw * kWave] = line;
        st[(size_t)vw * kWave] = stamp;
        return false;
    } else {
        uint32_t hw = kInvalidTag, fi = kInvalidTag;
        for (uint32_t w = 0; w < a; ++w) {
            const uint32_t t = tg[(size_t)w * kWave];
            if (t == line) hw = w;
            if (t == kInvalidTag && fi == kInvalidTag) fi = w;
        }
        const bool hit = hw != kInvalidTag;
        uint32_t* meta = tg + (size_t)a * kWave;
        if constexpr (POL == PCHASE_FIFO) {
            // ways fill in index order, so the insertion pointer is also the
            // lowest empty way until the set is full
            if (!hit) {
                const uint32_t x = meta[0];
                tg[(size_t)x * kWave] = line;
                meta[0] = x + 1 == a ? 0u : x + 1;
            }
        } else if constexpr (POL == PCHASE_PLRU) {
            const uint32_t nw = (a + 30) / 32;
            PlruBits b;
            uint32_t wd[4] = {0, 0, 0, 0};
            for (uint32_t i = 0; i < nw; ++i) wd[i] = meta[(size_t)i * kWave];
            b.lo = (uint64_t)wd[0] | ((uint64_t)wd[1] << 32);
            b.hi = (uint64_t)wd[2] | ((uint64_t)wd[3] << 32);
            const uint32_t x = hit ? hw : fi != kInvalidTag ? fi : b.victim(m.log2_ways, a);
            b.touch(x, m.log2_ways);
            wd[0] = (uint32_t)b.lo;
            wd[1] = (uint32_t)(b.lo >> 32);
            wd[2] = (uint32_t)b.hi;
            wd[3] = (uint32_t)(b.hi >> 32);
            for (uint32_t i = 0; i < nw; ++i) meta[(size_t)i * kWave] = wd[i];
            if (!hit) tg[(size_t)x * kWave] = line;
        } else {  // RANDOM: Philox4x32-10(key = seed, counter = (k_lo, k_hi, trace, 0)).x mod a
            if (!hit) {
                const uint32_t x = fi != kInvalidTag
                                       ? fi
                                       : philox_x((uint32_t)k, (uint32_t)(k >> 32), trace_id, 0u, m.seed_lo, m.seed_hi) % a;
                tg[(size_t)x * kWave] = line;
            }
        }
        return hit;
    }
}

template <int POL>
__device__ void tile_item(const TileArgs& args, const TileItem& it, const TileLds& L, int lane) {
    const DevModel m = args.models[it.model];
    const uint32_t a = m.ways, T = m.sets;
    const uint32_t lp = it.part >> 16, part = it.part & 0xFFFFu, P = 1u << lp;
    const uint32_t RS = a + tile_meta_rows(POL, a);
    const UDiv32 tdiv = make_udiv32(T);
    uint32_t* col = L.state + lane;

    // cold state for this lane's sets: set u = lane + 64 j of the part holds
    // rows [j RS, (j+1) RS)
    const uint32_t t_part = (T - part + P - 1) >> lp;
    const uint32_t slots = (t_part + kWave - 1) / kWave;
    for (uint32_t j = 0; j < slots; ++j)
        for (uint32_t q = 0; q < RS; ++q) col[(size_t)(j * RS + q) * kWave] = q < a ? kInvalidTag : 0u;

    const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t mt = 0, ms = 0;
    bool bad = false;
    uint32_t carry = kInvalidTag;   // line of the access before the tile
    const int32_t* tr = args.idx + it.start;
    for (uint64_t k0 = 0; k0 < it.len; k0 += kTile) {
        L.bcnt[lane] = 0;
        __syncthreads();
        // --- 1. lines, sets, heads; bucket counts
        uint32_t ln[kTileJ], mt_[kTileJ];   // line; head-of-own-set flag | owner | first row
        uint32_t prev_last = carry;
#pragma unroll
        for (uint32_t j = 0; j < kTileJ; ++j) {
            const uint64_t k = k0 + j * kWave + lane;
            const bool valid = k < it.len;
            int32_t v = valid ? tr[k] : 0;
            if (v < 0) {
                bad = true;
                v = 0;
            }
            const uint64_t addr = it.base + ((uint64_t)(uint32_t)v << 2);
            const uint32_t line = valid ? (uint32_t)(addr >> m.line_shift) : kInvalidTag;
            const uint32_t unit = (uint32_t)(addr >> m.unit_shift);
            const uint32_t set = unit - tdiv.div(unit) * T;
            uint32_t prev = __shfl_up(line, 1, kWave);
            if (lane == 0) prev = prev_last;
            prev_last = __shfl(line, kWave - 1, kWave);
            const bool own = valid && (set & (P - 1)) == part;
            const bool head = own && line != prev;
            const uint32_t u = set >> lp;
            const uint32_t owner = u & (kWave - 1);
            ln[j] = line;
            mt_[j] = (head ? 0x80000000u : 0u) | (owner << 24) | ((u >> 6) * RS);
            // repeats of the previous line: hits with no state change
            const uint64_t rep = __ballot(own && !head);
            if (lane == 0) {
                L.tbits[2 * j] = (uint32_t)rep;
                L.tbits[2 * j + 1] = (uint32_t)(rep >> 32);
            }
            if (head) atomicAdd(&L.bcnt[owner], 1u);
        }
        carry = prev_last;
        __syncthreads();
        // --- 2. stable counting sort of the heads by owner lane
        const uint32_t cnt = L.bcnt[lane];
        uint32_t incl = cnt;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += t;
        }
        const uint32_t first = incl - cnt;
        L.cursor[lane] = first;
        __syncthreads();
#pragma unroll
        for (uint32_t j = 0; j < kTileJ; ++j) {
            const bool head = (mt_[j] >> 31) != 0;
            const uint32_t owner = (mt_[j] >> 24) & 63u;
            uint64_t peers = __ballot(head);
#pragma unroll
            for (int b = 0; b < 6; ++b) {
                const uint64_t bb = __ballot(head && ((owner >> b) & 1u));
                peers &= ((owner >> b) & 1u) ? bb : ~bb;
            }
            uint32_t pos = 0;
            if (head) pos = L.cursor[owner] + (uint32_t)__popcll(peers & lt_mask);
            __syncthreads();
            if (head) {
                L.line[pos] = ln[j];
                L.info[pos] = (j * kWave + lane) | ((mt_[j] & 0x00FFFFFFu) << 10);
                if ((peers & lt_mask) == 0) L.cursor[owner] += (uint32_t)__popcll(peers);
            }
            __syncthreads();
        }
        // --- 3. every lane replays its own heads in trace order
        for (uint32_t e = first; e < incl; ++e) {
            const uint32_t line = L.line[e], info = L.info[e];
            const uint32_t kl = info & (kTile - 1);
            const uint64_t k = k0 + kl;
            if (tile_access<POL>(col, info >> 10, line, a, k, m, it.trace_id)) {
                atomicOr(&L.tbits[kl >> 5], 1u << (kl & 31));
            } else {
                ++mt;
                ms += k >= it.count_from ? 1u : 0u;
            }
        }
        __syncthreads();
        // --- 4. hit bits of the tile
        if (args.bits) {
            const uint64_t rem = it.len - k0;
            const uint32_t words = rem >= kTile ? kTile / 32 : (uint32_t)((rem + 31) / 32);
            uint32_t* out = args.bits + it.bitoff + (k0 >> 5);
            if (lane < (int)words) {
                const uint32_t w = L.tbits[lane];
                if (P > 1) {
                    if (w) atomicOr(out + lane, w);
                } else {
                    out[lane] = w;
                }
            }
        }
    }
    // counts of the pair (or part)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mt += __shfl_xor(mt, o, kWave);
        ms += __shfl_xor(ms, o, kWave);
    }
    if (__ballot(bad) != 0 && lane == 0) atomicOr(args.status, 2u);
    if (lane == 0) {
        uint64_t* c = args.misses + 2ull * it.out;
        if (P > 1) {
            atomicAdd(reinterpret_cast<unsigned long long*>(c), (unsigned long long)mt);
            atomicAdd(reinterpret_cast<unsigned long long*>(c + 1), (unsigned long long)ms);
        } else {
            c[0] = mt;
            c[1] = ms;
        }
    }
}

template <int POL>
__global__ void __launch_bounds__(64) tile_kernel(TileArgs args) {
    extern __shared__ uint32_t lds[];
    const int lane = threadIdx.x;
    TileLds L;
    L.state = lds;
    L.line = lds + (size_t)args.rows * kWave;
    L.info = L.line + kTile;
    L.tbits = L.info + kTile;
    L.bcnt = L.tbits + kTile / 32;
    L.cursor = L.bcnt + kWave;
    if (!args.persistent) {
        if (blockIdx.x < args.n_items) tile_item<POL>(args, args.items[blockIdx.x], L, lane);
        return;
    }
    for (uint32_t iter = 0;; ++iter) {
        uint32_t t = 0;
        if (lane == 0) {
            t = atomicAdd(args.queue, 1u);
            // the host flag is polled on the first pull and every 8th after it
            if ((iter & 7) == 0 && args.abort_flag != nullptr && *args.abort_flag != 0) {
                atomicOr(args.status, 1u);
                t = args.n_items;
            }
        }
        t = __shfl(t, 0, kWave);
        if (t >= args.n_items) break;
        tile_item<POL>(args, args.items[t], L, lane);
    }
}

using TileFn = void (*)(TileArgs);

static TileFn tile_fn(int pol) {
    switch (pol) {
        case PCHASE_LRU: return tile_kernel<PCHASE_LRU>;
        case PCHASE_FIFO: return tile_kernel<PCHASE_FIFO>;
        case PCHASE_PLRU: return tile_kernel<PCHASE_PLRU>;
        default: return tile_kernel<PCHASE_RANDOM>;
    }
}

hipError_t launch_tile(int pol, const TileArgs& a, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL(tile_fn(pol), dim3(blocks), dim3(kWave), tile_lds_bytes(a.rows), s, a);
    return hipGetLastError();
}

hipError_t tile_occupancy(int pol, uint32_t rows, int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)tile_fn(pol), kWave,
                                                        tile_lds_bytes(rows));
}

hipError_t tile_prepare_lds() {
    for (int pol = 0; pol < 4; ++pol) {
        hipError_t e = hipFuncSetAttribute((const void*)tile_fn(pol), hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)tile_lds_bytes(kTileMaxRows));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pc
