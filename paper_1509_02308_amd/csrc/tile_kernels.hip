// tile_kernels.hip -- set-partitioned replay of materialised index traces
// through standard set-associative models (Mei & Chu, Section 4.1,
// Assumptions 1-3, with the non-LRU policies of Sections 4.5-4.6).
//
// The hit or miss of an access depends only on the earlier accesses of its
// own set (the set of address x is (x >> unit) mod T, and a set's a ways are
// touched by nothing else).  So a pair is replayed by one wave whose lane
// groups own disjoint sets (TileLayout: G groups of W lanes, the ways of a
// set spread over the W lanes of its group), each lane holding its part of
// the state in an LDS column (row r of lane l at dword 64 r + l: no two lanes
// share a bank), and each group replaying only the accesses of its own
// sets, in trace order.
//
// The trace streams through in tiles of kTile accesses, read coalesced (lane
// l takes accesses 64 j + l of the tile), the next tile's loads in flight
// while this one is replayed.  Per tile:
//   1. every access gets its line and set; an access to the same line as the
//      access just before it in the trace is a hit that changes no policy's
//      state (the way is already the most recently used one, FIFO and random
//      replacement ignore hits, and the tree-PLRU path bits already point
//      away from it), so its hit bit is set at once;
//   2. the remaining accesses ("heads") are counting-sorted by owning group,
//      stably: a bucket histogram, its prefix over the groups, then the
//      position of each head = its bucket's cursor + the number of lower
//      lanes with a head for the same bucket in the same row (ballots);
//   3. each group replays its bucket in order: every lane scans its ways of
//      the set, and the group combines (hit by ballot, victim by a
//      reduction over its lanes);
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
    uint32_t* bcnt;     // 64: heads per group
    uint32_t* cursor;   // 64: next free slot of each group's bucket
};

size_t tile_lds_bytes(uint32_t rows) {
    return ((size_t)rows * kWave + 2 * kTile + kTile / 32 + 2 * kWave) * 4;
}

// The block is one wave: the LDS operations of a wave take effect in program
// order, so a compiler-level fence is all that separates the phases.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Minimum over the W = 2^lw lanes of the caller's aligned lane group.
__device__ __forceinline__ uint64_t group_min(uint64_t v, uint32_t lw) {
    for (uint32_t o = 1; o < (1u << lw); o <<= 1) {
        const uint64_t t = __shfl_xor(v, o, kWave);
        v = t < v ? t : v;
    }
    return v;
}

constexpr uint64_t kNone64 = ~0ull;

// Replays one head: the group's W lanes (lane r holds ways r + W i, i < kw,
// in its column `col` from row rowb on) decide hit or miss together and
// update the state.  k is the access index within the pair.  Returns hit.
// The per-lane ways are read in unrolled chunks of A (clamped to the lane's
// last way, whose repeats change no result), so a chunk's loads are in
// flight together and the scan has no branches.
template <int POL, int A>
__device__ __forceinline__ bool tile_access(uint32_t* col, uint32_t rowb, uint32_t line, uint32_t a,
                                            const TileLayout& ly, uint32_t r, uint32_t gbase, uint64_t gmask,
                                            uint64_t k, const DevModel& m, uint32_t trace_id) {
    const uint32_t W = 1u << ly.lw, kw = ly.kw;
    // local way i of this lane is way i*W + r: the lane holds nloc of them
    const uint32_t nloc = r < a ? (a - r + W - 1) >> ly.lw : 0u;
    if constexpr (POL == PCHASE_LRU) {
        // one pass: the hit way, and the lowest (stamp, way) key: empty ways
        // have stamp 0 (so the lowest-numbered empty way wins), used ways
        // stamp k + 1 >= 1, all distinct
        const uint32_t lane = threadIdx.x & (kWave - 1);
        uint2* e = reinterpret_cast<uint2*>(col - lane) + (size_t)(rowb / 2) * kWave + lane;
        uint32_t hi = kInvalidTag;
        uint64_t key = kNone64;
        if (nloc) {
            for (uint32_t i0 = 0; i0 < kw; i0 += A) {
                uint2 v[A];
#pragma unroll
                for (int i = 0; i < A; ++i) v[i] = e[(size_t)min(i0 + i, nloc - 1) * kWave];
#pragma unroll
                for (int i = 0; i < A; ++i) {
                    const uint32_t li = min(i0 + i, nloc - 1);
                    hi = v[i].x == line ? li : hi;
                    const uint64_t kk = ((uint64_t)v[i].y << 32) | (li * W + r);
                    key = kk < key ? kk : key;
                }
            }
        }
        const uint32_t stamp = (uint32_t)k + 1u;
        const bool hit = (__ballot(hi != kInvalidTag) & gmask) != 0;
        if (hit) {
            if (hi != kInvalidTag) e[(size_t)hi * kWave].y = stamp;
            return true;
        }
        const uint32_t x = (uint32_t)group_min(key, ly.lw);
        if ((x & (W - 1)) == r) e[(size_t)(x >> ly.lw) * kWave] = make_uint2(line, stamp);
        return false;
    } else {
        uint32_t* tg = col + (size_t)rowb * kWave;
        uint32_t hi = kInvalidTag, fi = kInvalidTag;
        if (nloc) {
            for (uint32_t i0 = 0; i0 < kw; i0 += A) {
                uint32_t v[A];
#pragma unroll
                for (int i = 0; i < A; ++i) v[i] = tg[(size_t)min(i0 + i, nloc - 1) * kWave];
#pragma unroll
                for (int i = 0; i < A; ++i) {
                    const uint32_t li = min(i0 + i, nloc - 1);
                    hi = v[i] == line ? li : hi;
                    fi = (v[i] == kInvalidTag && fi == kInvalidTag) ? li : fi;
                }
            }
        }
        const uint64_t hm = __ballot(hi != kInvalidTag) & gmask;
        const bool hit = hm != 0;
        uint32_t* meta = tg + (size_t)kw * kWave;   // used by the group's first lane
        if constexpr (POL == PCHASE_FIFO) {
            // ways fill in index order, so the insertion pointer is also the
            // lowest empty way until the set is full
            if (!hit) {
                uint32_t x = r == 0 ? meta[0] : 0u;
                x = __shfl(x, gbase, kWave);
                if ((x & (W - 1)) == r) tg[(size_t)(x >> ly.lw) * kWave] = line;
                if (r == 0) meta[0] = x + 1 == a ? 0u : x + 1;
            }
        } else {
            // lowest-numbered empty way of the set, if any
            uint32_t x = kInvalidTag;
            if (!hit) {
                const uint64_t f = group_min(fi == kInvalidTag ? kNone64 : (uint64_t)(fi * W + r), ly.lw);
                x = f == kNone64 ? kInvalidTag : (uint32_t)f;
            }
            if constexpr (POL == PCHASE_PLRU) {
                if (hit) {
                    const uint32_t hl = (uint32_t)__ffsll((unsigned long long)hm) - 1u;
                    x = __shfl(hi * W + r, (int)hl, kWave);
                }
                if (r == 0) {
                    const uint32_t nw = (a + 30) / 32;
                    PlruBits b;
                    uint32_t wd[4] = {0, 0, 0, 0};
                    for (uint32_t i = 0; i < nw; ++i) wd[i] = meta[(size_t)i * kWave];
                    b.lo = (uint64_t)wd[0] | ((uint64_t)wd[1] << 32);
                    b.hi = (uint64_t)wd[2] | ((uint64_t)wd[3] << 32);
                    if (x == kInvalidTag) x = b.victim(m.log2_ways, a);
                    b.touch(x, m.log2_ways);
                    wd[0] = (uint32_t)b.lo;
                    wd[1] = (uint32_t)(b.lo >> 32);
                    wd[2] = (uint32_t)b.hi;
                    wd[3] = (uint32_t)(b.hi >> 32);
                    for (uint32_t i = 0; i < nw; ++i) meta[(size_t)i * kWave] = wd[i];
                }
                if (!hit) {
                    x = __shfl(x, gbase, kWave);
                    if ((x & (W - 1)) == r) tg[(size_t)(x >> ly.lw) * kWave] = line;
                }
            } else {  // RANDOM: Philox4x32-10(key = seed, counter = (k_lo, k_hi, trace, 0)).x mod a
                if (!hit) {
                    if (x == kInvalidTag)
                        x = philox_x((uint32_t)k, (uint32_t)(k >> 32), trace_id, 0u, m.seed_lo, m.seed_hi) % a;
                    if ((x & (W - 1)) == r) tg[(size_t)(x >> ly.lw) * kWave] = line;
                }
            }
        }
        return hit;
    }
}

// `it` is taken by value and the arguments the tile loop needs are copied
// into registers first: the phase fences would otherwise make the compiler
// re-read them from memory, waiting on the prefetched trace loads each time.
template <int POL, int A>
__device__ __forceinline__ void tile_item(const TileArgs& args, const TileItem it, const TileLds& L, int lane) {
    const DevModel m = args.models[it.model];
    uint32_t* const bits_out = args.bits;
    uint64_t* const misses = args.misses;
    uint32_t* const status = args.status;
    const uint32_t a = m.ways, T = m.sets;
    const uint32_t lp = it.part >> 16, part = it.part & 0xFFFFu, P = 1u << lp;
    const TileLayout ly = tile_layout(POL, a, T, lp, part);
    const uint32_t G = 1u << ly.lg, W = 1u << ly.lw;
    const uint32_t grp = (uint32_t)lane >> ly.lw, r = (uint32_t)lane & (W - 1), gbase = grp << ly.lw;
    const uint64_t gmask = W == 64 ? ~0ull : (((1ull << W) - 1ull) << gbase);
    const UDiv32 tdiv = make_udiv32(T);
    uint32_t* col = L.state + lane;

    // cold state: every lane's rows of every slot of its group
    if constexpr (POL == PCHASE_LRU) {
        uint2* e = reinterpret_cast<uint2*>(L.state) + lane;
        for (uint32_t q = 0; q < ly.slots * ly.kw; ++q) e[(size_t)q * kWave] = make_uint2(kInvalidTag, 0u);
    } else {
        for (uint32_t j = 0; j < ly.slots; ++j)
            for (uint32_t q = 0; q < ly.rs; ++q) col[(size_t)(j * ly.rs + q) * kWave] = q < ly.kw ? kInvalidTag : 0u;
    }

    const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t mt = 0, ms = 0;
    bool bad = false;
    uint32_t carry = kInvalidTag;   // line of the access before the tile
    const int32_t* tr = args.idx + it.start;
    // the next tile's indices are loaded while this one is replayed; every
    // lane loads all kTileJ of its indices unconditionally (clamped to the
    // last access), so the loads go out together
    int32_t cur[kTileJ];
    auto load_tile = [&](uint64_t t0, int32_t (&dst)[kTileJ]) {
#pragma unroll
        for (uint32_t j = 0; j < kTileJ; ++j) {
            const uint64_t k = t0 + j * kWave + lane;
            dst[j] = tr[k < it.len ? k : it.len - 1];
        }
    };
    if (it.len) load_tile(0, cur);
    for (uint64_t k0 = 0; k0 < it.len; k0 += kTile) {
        // (unconditional: past the last tile it reloads the last access,
        // and the copy below keeps the loads where they are issued)
        int32_t nxt[kTileJ];
        load_tile(k0 + kTile, nxt);
        __builtin_amdgcn_sched_barrier(0);
        L.bcnt[lane] = 0;
        wave_sync();
        // --- 1. lines, sets, heads; bucket counts
        uint32_t ln[kTileJ], mt_[kTileJ];   // line; head-of-own-set flag | group | first row
        uint32_t prev_last = carry;
#pragma unroll
        for (uint32_t j = 0; j < kTileJ; ++j) {
            const uint64_t k = k0 + j * kWave + lane;
            const bool valid = k < it.len;
            int32_t v = valid ? cur[j] : 0;
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
            // set u of the part: group (u + u / G) mod G, slot u / G (the
            // rotation by the slot keeps strides that are multiples of the
            // line spread over the groups)
            const uint32_t u = set >> lp;
            const uint32_t owner = (u + (u >> ly.lg)) & (G - 1);
            ln[j] = line;
            mt_[j] = (head ? 0x80000000u : 0u) | (owner << 24) | ((u >> ly.lg) * ly.rs);
            // repeats of the previous line: hits with no state change
            const uint64_t rep = __ballot(own && !head);
            if (lane == 0) {
                L.tbits[2 * j] = (uint32_t)rep;
                L.tbits[2 * j + 1] = (uint32_t)(rep >> 32);
            }
            if (head) atomicAdd(&L.bcnt[owner], 1u);
        }
        carry = prev_last;
        wave_sync();
        // --- 2. stable counting sort of the heads by owning group
        const uint32_t cnt = L.bcnt[lane];
        uint32_t incl = cnt;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += t;
        }
        const uint32_t first = incl - cnt;
        L.cursor[lane] = first;
        wave_sync();
#pragma unroll
        for (uint32_t j = 0; j < kTileJ; ++j) {
            const bool head = (mt_[j] >> 31) != 0;
            const uint32_t owner = (mt_[j] >> 24) & 63u;
            uint64_t peers = __ballot(head);
            for (uint32_t b = 0; b < ly.lg; ++b) {
                const uint64_t bb = __ballot(head && ((owner >> b) & 1u));
                peers &= ((owner >> b) & 1u) ? bb : ~bb;
            }
            // one wave: its LDS operations take effect in program order, so
            // the cursors read here are those the previous row left
            if (head) {
                const uint32_t pos = L.cursor[owner] + (uint32_t)__popcll(peers & lt_mask);
                L.line[pos] = ln[j];
                L.info[pos] = (j * kWave + lane) | ((mt_[j] & 0x00FFFFFFu) << 10);
                if ((peers & lt_mask) == 0) L.cursor[owner] = pos + (uint32_t)__popcll(peers);
            }
        }
        wave_sync();
        // --- 3. every group replays its own heads in trace order
        const uint32_t g_first = __shfl(first, (int)grp, kWave), g_end = __shfl(incl, (int)grp, kWave);
        for (uint32_t e = g_first; e < g_end; ++e) {
            const uint32_t line = L.line[e], info = L.info[e];
            const uint32_t kl = info & (kTile - 1);
            const uint64_t k = k0 + kl;
            const bool hit = tile_access<POL, A>(col, info >> 10, line, a, ly, r, gbase, gmask, k, m, it.trace_id);
            if (r == 0) {
                if (hit) {
                    atomicOr(&L.tbits[kl >> 5], 1u << (kl & 31));
                } else {
                    ++mt;
                    ms += k >= it.count_from ? 1u : 0u;
                }
            }
        }
        wave_sync();
        // --- 4. hit bits of the tile
        if (bits_out) {
            const uint64_t rem = it.len - k0;
            const uint32_t words = rem >= kTile ? kTile / 32 : (uint32_t)((rem + 31) / 32);
            uint32_t* out = bits_out + it.bitoff + (k0 >> 5);
            if (lane < (int)words) {
                const uint32_t w = L.tbits[lane];
                if (P > 1) {
                    if (w) atomicOr(out + lane, w);
                } else {
                    out[lane] = w;
                }
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < kTileJ; ++j) cur[j] = nxt[j];
    }
    // counts of the pair (or part)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mt += __shfl_xor(mt, o, kWave);
        ms += __shfl_xor(ms, o, kWave);
    }
    if (__ballot(bad) != 0 && lane == 0) atomicOr(status, 2u);
    if (lane == 0) {
        uint64_t* c = misses + 2ull * it.out;
        if (P > 1) {
            atomicAdd(reinterpret_cast<unsigned long long*>(c), (unsigned long long)mt);
            atomicAdd(reinterpret_cast<unsigned long long*>(c + 1), (unsigned long long)ms);
        } else {
            c[0] = mt;
            c[1] = ms;
        }
    }
}

template <int POL, int A>
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
        if (blockIdx.x < args.n_items) tile_item<POL, A>(args, args.items[blockIdx.x], L, lane);
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
        tile_item<POL, A>(args, args.items[t], L, lane);
    }
}

using TileFn = void (*)(TileArgs);

template <int POL>
static TileFn tile_fn_a(int wcls) {
    switch (wcls) {
        case 0: return tile_kernel<POL, 1>;
        case 1: return tile_kernel<POL, 2>;
        case 2: return tile_kernel<POL, 4>;
        case 3: return tile_kernel<POL, 8>;
        default: return tile_kernel<POL, 16>;
    }
}

static TileFn tile_fn(int pol, int wcls) {
    switch (pol) {
        case PCHASE_LRU: return tile_fn_a<PCHASE_LRU>(wcls);
        case PCHASE_FIFO: return tile_fn_a<PCHASE_FIFO>(wcls);
        case PCHASE_PLRU: return tile_fn_a<PCHASE_PLRU>(wcls);
        default: return tile_fn_a<PCHASE_RANDOM>(wcls);
    }
}

hipError_t launch_tile(int pol, int wcls, const TileArgs& a, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL(tile_fn(pol, wcls), dim3(blocks), dim3(kWave), tile_lds_bytes(a.rows), s, a);
    return hipGetLastError();
}

hipError_t tile_occupancy(int pol, int wcls, uint32_t rows, int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)tile_fn(pol, wcls), kWave,
                                                        tile_lds_bytes(rows));
}

hipError_t tile_prepare_lds() {
    for (int pol = 0; pol < 4; ++pol)
        for (int wc = 0; wc < kTileWayClasses; ++wc) {
            hipError_t e = hipFuncSetAttribute((const void*)tile_fn(pol, wc),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)tile_lds_bytes(kTileMaxRows));
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace pc
