// stream_kernels.hip -- replay of materialised index traces (any access
// sequence, e.g. a recorded fine-grained P-chase) through set-associative
// cache models (Mei & Chu, Section 4.1, Assumptions 1-3, with the non-LRU
// policies of Sections 4.5-4.6).
//
// A group of W lanes (W = associativity rounded up to a power of two, at
// most 64) replays one (model, trace) pair: lane w holds way w (and way
// w+64 when a > 64) of whichever set the current access maps to, so a tag
// lookup is one compare per lane and a ballot.  Accesses are processed in
// trace order; the trace is streamed from HBM W indices at a time and
// broadcast through cross-lane shuffles.
//
// The cache state of a pair lives in a slab of device memory owned by its
// group: per set a 32-byte header (epoch, FIFO pointer, PLRU bits) that only
// the group's first lane reads and writes, and per way an 8-byte entry
// (tag, LRU rank) that only the owning lane reads and writes, so every
// memory dependence stays within one lane.  A set whose header epoch is not
// the current pair's is empty; its first access rewrites every entry.
// A group's slab serves pair after pair with different set counts, so a
// header slot may hold an old entry word (tag, rank) of an earlier pair; the
// header's epoch word carries all-ones in its high half, which no entry word
// (rank <= 0xFF) can, so such leftovers never pass for a current header.
#include "common.h"

namespace pc {

struct SetHeader {
    uint64_t epoch;  // kEpochTag | pair epoch
    uint64_t lo;     // PLRU node bits 0-63
    uint64_t hi;     // PLRU node bits 64-126
    uint64_t ptr;    // FIFO: next way to replace
};
constexpr uint64_t kEpochTag = 0xFFFFFFFF00000000ull;



__device__ __forceinline__ uint32_t plru_get(uint64_t lo, uint64_t hi, uint32_t n) {
    return n < 64 ? (uint32_t)(lo >> n) & 1u : (uint32_t)(hi >> (n - 64)) & 1u;
}
__device__ __forceinline__ void plru_put(uint64_t& lo, uint64_t& hi, uint32_t n, uint32_t v) {
    if (n < 64) lo = (lo & ~(1ull << n)) | ((uint64_t)v << n);
    else hi = (hi & ~(1ull << (n - 64))) | ((uint64_t)v << (n - 64));
}

// GEN: a generalised model (per-set ways, optional set table, weighted
// random replacement): the set's way count and entry base come from
// set_info, and m.ways is the widest set.
template <int POL, int W, bool GEN>
__device__ void stream_pair(const StreamArgs& args, const StreamPair& pr, uint32_t pair_index,
                            int gl, int gbase, uint8_t* slab) {
    const DevModel m = args.models[pr.model];
    const uint32_t amax = m.ways;
    const uint32_t T = m.sets;
    DevGeneral g{};
    if constexpr (GEN) g = args.gen[pr.model];
    const uint32_t epoch = args.epoch_base + pair_index + 1;
    SetHeader* hdr = reinterpret_cast<SetHeader*>(slab);
    const uint64_t gmask = (W == 64) ? ~0ull : (((1ull << (W & 63)) - 1ull) << gbase);
    const bool two = (W == 64) && (amax > 64);
    const bool own0_all = (uint32_t)gl < amax;
    const bool own1_all = two && (uint32_t)(gl + 64) < amax;

    uint64_t mt = 0, ms = 0;
    uint32_t* bits = args.bits ? args.bits + pr.bitoff : nullptr;
    bool bad = false;
    // a long pair, or one with a large state, may be split into parts by set
    // (set mod nparts == part, nparts a power of two), each part holding only
    // its own sets (slot set >> log2 nparts):
    // sets are independent, so each part replays its own sets exactly and
    // merges its hit bits and counts into zeroed outputs
    const uint32_t nparts = pr.pad >> 16, part = pr.pad & 0xFFFFu;
    const bool split = nparts > 1;
    // part p keeps its sets at set >> pshift; a generalised model's part
    // keeps the whole layout (its sets differ in size), skipping the others
    const uint32_t pshift = (split && !GEN) ? (uint32_t)(__ffs((int)nparts) - 1) : 0u;
    const uint32_t Tl = (split && !GEN) ? (T + nparts - 1) >> pshift : T;   // set slots of this pair or part
    uint2* ent = reinterpret_cast<uint2*>(slab + (size_t)Tl * sizeof(SetHeader));
    uint64_t cur_w = ~0ull;
    uint32_t word = 0;
    auto flush = [&]() {
        if (bits != nullptr && gl == 0 && cur_w != ~0ull) {
            if (split) {
                if (word) atomicOr(bits + cur_w, word);
            } else {
                bits[cur_w] = word;
            }
        }
    };
    auto put_bit = [&](uint64_t k, bool hit) {
        if ((k >> 5) != cur_w) {
            flush();
            cur_w = k >> 5;
            word = 0;
        }
        word |= (hit ? 1u : 0u) << (k & 31);
    };
    // line of the previous access of this part: a repeat is a hit that
    // leaves every policy's state as it is (the way is already the most
    // recent one, FIFO and random replacement change nothing on a hit, and
    // the PLRU path bits already point away from it), so it needs no state
    // access
    uint32_t last_line = kInvalidTag;

    // the trace is read V indices per lane per round (W * V per group), the
    // next round prefetched while this one is replayed, so that a narrow
    // group does not wait on one load per access
    constexpr int V = (W >= 64) ? 1 : 8;
    const uint64_t CH = (uint64_t)W * V;
    int32_t cur[V], nxt[V];
    auto load = [&](uint64_t c0, int32_t (&dst)[V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint64_t kk = c0 + (uint64_t)gl * V + v;
            dst[v] = kk < pr.len ? args.idx[pr.start + kk] : 0;
        }
    };
    load(0, cur);
    const UDiv32 tdiv = make_udiv32(T);

    for (uint64_t k0 = 0; k0 < pr.len; k0 += CH) {
        if (k0 + CH < pr.len) load(k0 + CH, nxt);
        const uint32_t nstep = (pr.len - k0 < CH) ? (uint32_t)(pr.len - k0) : (uint32_t)CH;
        for (uint32_t i = 0; i < nstep; ++i) {
            const uint64_t k = k0 + i;
            const uint32_t comp = i % V;
            int32_t mv = cur[0];
#pragma unroll
            for (int v = 1; v < V; ++v) mv = comp == (uint32_t)v ? cur[v] : mv;
            const int32_t j = __shfl(mv, gbase + (int)(i / V), kWave);
            bad |= j < 0;
            const uint64_t xa = pr.base + ((uint64_t)(uint32_t)(j < 0 ? 0 : j) << args.elem_shift);
            const uint32_t line = (uint32_t)(xa >> m.line_shift);
            if (line == last_line) {
                put_bit(k, true);
                continue;
            }
            const uint32_t ux = (uint32_t)(xa >> m.unit_shift);
            uint32_t set;
            if constexpr (GEN) {
                set = g.table_len ? args.set_table[g.table_off + ux % g.table_len] : ux - tdiv.div(ux) * T;
            } else {
                set = ux - tdiv.div(ux) * T;
            }
            if (split && (set & (nparts - 1)) != part) continue;
            last_line = line;

            // the set's entries and (first lane) header, loaded together
            const uint32_t lset = set >> pshift;
            uint32_t a = amax, log2a = m.log2_ways;
            uint64_t eb;
            bool own0 = own0_all, own1 = own1_all;
            if constexpr (GEN) {
                const uint2 si = args.set_info[g.set_off + set];
                a = si.x;
                eb = si.y;
                own0 = (uint32_t)gl < a;
                own1 = two && (uint32_t)(gl + 64) < a;
                log2a = 31u - (uint32_t)__clz((int)a);
            } else {
                eb = (uint64_t)lset * a;
            }
            uint2 e0 = make_uint2(kInvalidTag, 0xFFu), e1 = make_uint2(kInvalidTag, 0xFFu);
            uint2 r0 = e0, r1 = e1;
            if (own0) r0 = ent[eb + gl];
            if (own1) r1 = ent[eb + gl + 64];
            uint32_t h_ep = 0, h_ptr = 0;
            uint64_t h_lo = 0, h_hi = 0;
            if (gl == 0) {
                const SetHeader h = hdr[lset];
                h_ep = (h.epoch == (kEpochTag | epoch) && (uint32_t)(h.ptr >> 32) == ~epoch) ? epoch : 0u;
                h_ptr = (uint32_t)h.ptr;
                h_lo = h.lo;
                h_hi = h.hi;
            }
            h_ep = __shfl(h_ep, gbase, kWave);
            const bool fresh = h_ep != epoch;
            if (fresh) {
                h_ptr = 0;
                h_lo = 0;
                h_hi = 0;
            } else {
                h_ptr = __shfl(h_ptr, gbase, kWave);
                h_lo = __shfl(h_lo, gbase, kWave);
                h_hi = __shfl(h_hi, gbase, kWave);
                e0 = r0;
                e1 = r1;
            }
            const uint64_t hm0 = __ballot(own0 && e0.x == line) & gmask;
            const uint64_t hm1 = __ballot(own1 && e1.x == line) & gmask;
            const uint64_t vm0 = __ballot(own0 && e0.x != kInvalidTag) & gmask;
            const uint64_t vm1 = __ballot(own1 && e1.x != kInvalidTag) & gmask;
            const uint32_t nvalid = (uint32_t)(__popcll(vm0) + __popcll(vm1));
            const bool hit = (hm0 | hm1) != 0;
            uint32_t hw = 0;
            if (hm0) hw = (uint32_t)(__ffsll((long long)hm0) - 1 - gbase);
            else if (hm1) hw = (uint32_t)(__ffsll((long long)hm1) - 1 - gbase) + 64;

            uint32_t x;  // way used by this access
            bool hdr_dirty = fresh;
            if (POL == PCHASE_LRU) {
                uint32_t ax;
                if (hit) {
                    x = hw;
                    const uint32_t src = hw & 63u;
                    const uint32_t g0 = __shfl(e0.y, gbase + (int)src, kWave);
                    const uint32_t g1 = __shfl(e1.y, gbase + (int)src, kWave);
                    ax = hw < 64 ? g0 : g1;
                } else if (nvalid < a) {
                    x = nvalid;
                    ax = nvalid;
                } else {
                    const uint64_t o0 = __ballot(own0 && e0.y == a - 1) & gmask;
                    const uint64_t o1 = __ballot(own1 && e1.y == a - 1) & gmask;
                    x = o0 ? (uint32_t)(__ffsll((long long)o0) - 1 - gbase)
                           : (uint32_t)(__ffsll((long long)o1) - 1 - gbase) + 64;
                    ax = a - 1;
                }
                if (own0 && e0.y < ax) e0.y += 1;
                if (own1 && e1.y < ax) e1.y += 1;
            } else if (POL == PCHASE_FIFO) {
                x = hit ? hw : h_ptr;
                if (!hit) {
                    h_ptr = (h_ptr + 1 == a) ? 0 : h_ptr + 1;
                    hdr_dirty = true;
                }
            } else if (POL == PCHASE_PLRU) {
                if (hit) x = hw;
                else if (nvalid < a) x = nvalid;
                else {
                    uint32_t node = 0;
                    for (uint32_t d = 0; d < log2a; ++d) node = 2 * node + 1 + plru_get(h_lo, h_hi, node);
                    x = node - (a - 1);
                }
                uint32_t node = 0;
                for (uint32_t d = 0; d < log2a; ++d) {
                    const uint32_t dir = (x >> (log2a - 1 - d)) & 1u;
                    plru_put(h_lo, h_hi, node, dir ^ 1u);
                    node = 2 * node + 1 + dir;
                }
                hdr_dirty = true;
            } else if (POL == PCHASE_WRANDOM) {
                if (hit) x = hw;
                else if (nvalid < a) x = nvalid;
                else {
                    // lowest way whose cumulative weight exceeds u mod S: the
                    // weights are positive-sum and cumulative, so one lane of
                    // the set's a ways qualifies; the lowest is the victim
                    const uint32_t u = philox_x((uint32_t)k, (uint32_t)(k >> 32), pr.trace_id, 0u, m.seed_lo,
                                                m.seed_hi);
                    const uint32_t r = u % args.cum_w[g.cum_off + a - 1];
                    const uint32_t c0 = own0 ? args.cum_w[g.cum_off + gl] : 0u;
                    const uint32_t c1 = own1 ? args.cum_w[g.cum_off + gl + 64] : 0u;
                    const uint64_t q0 = __ballot(own0 && r < c0) & gmask;
                    const uint64_t q1 = __ballot(own1 && r < c1) & gmask;
                    x = q0 ? (uint32_t)(__ffsll((long long)q0) - 1 - gbase)
                           : (uint32_t)(__ffsll((long long)q1) - 1 - gbase) + 64;
                }
            } else {
                if (hit) x = hw;
                else if (nvalid < a) x = nvalid;
                else x = philox_x((uint32_t)k, (uint32_t)(k >> 32), pr.trace_id, 0u, m.seed_lo,
                                  m.seed_hi) % a;
            }
            bool dirty0 = fresh, dirty1 = fresh;
            if (POL == PCHASE_LRU) {
                dirty0 = dirty1 = true;
            }
            if ((uint32_t)gl == x) {
                e0.x = line;
                e0.y = 0;
                dirty0 = true;
            }
            if ((uint32_t)gl + 64 == x) {
                e1.x = line;
                e1.y = 0;
                dirty1 = true;
            }
            if (own0 && dirty0) ent[eb + gl] = e0;
            if (own1 && dirty1) ent[eb + gl + 64] = e1;
            if (gl == 0 && hdr_dirty) {
                SetHeader h;
                h.epoch = kEpochTag | epoch;
                h.lo = h_lo;
                h.hi = h_hi;
                h.ptr = (uint64_t)h_ptr | ((uint64_t)(~epoch) << 32);
                hdr[lset] = h;
            }

            if (!hit) {
                ++mt;
                ms += (k >= pr.count_from) ? 1u : 0u;
            }
            put_bit(k, hit);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) cur[v] = nxt[v];
    }
    flush();
    if (gl == 0) {
        if (split) {
            if (mt) atomicAdd((unsigned long long*)&args.misses[2 * (uint64_t)pr.out], (unsigned long long)mt);
            if (ms) atomicAdd((unsigned long long*)&args.misses[2 * (uint64_t)pr.out + 1], (unsigned long long)ms);
        } else {
            args.misses[2 * (uint64_t)pr.out] = mt;
            args.misses[2 * (uint64_t)pr.out + 1] = ms;
        }
        if (bad) atomicOr(args.status, 2u);
    }
}

template <int POL, int W, bool GEN>
__global__ void __launch_bounds__(256) stream_kernel(StreamArgs args) {
    constexpr int G = kWave / W;
    const int lane = threadIdx.x & (kWave - 1);
    const int gl = lane % W;
    const int gbase = lane - gl;
    const uint64_t group = ((uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * G +
                           (uint64_t)(lane / W);
    uint8_t* slab = args.slab + group * args.slab_bytes;
    for (uint32_t iter = 0;; ++iter) {
        uint32_t t = 0;
        if (gl == 0) {
            t = atomicAdd(args.queue, 1u);
            // the host flag is polled on the first pull and every 8th after it
            if ((iter & 7) == 0 && args.abort_flag != nullptr && *args.abort_flag != 0) {
                atomicOr(args.status, 1u);
                t = args.n_pairs;
            }
        }
        t = __shfl(t, gbase, kWave);
        if (t >= args.n_pairs) break;
        stream_pair<POL, W, GEN>(args, args.pairs[t], t, gl, gbase, slab);
    }
}

using StreamFn = void (*)(StreamArgs);

template <bool GEN>
static StreamFn pick_stream(int pol, int w) {
#define PC_W(P)                                        \
    switch (w) {                                       \
        case 1: return stream_kernel<P, 1, GEN>;       \
        case 2: return stream_kernel<P, 2, GEN>;       \
        case 4: return stream_kernel<P, 4, GEN>;       \
        case 8: return stream_kernel<P, 8, GEN>;       \
        case 16: return stream_kernel<P, 16, GEN>;     \
        case 32: return stream_kernel<P, 32, GEN>;     \
        default: return stream_kernel<P, 64, GEN>;     \
    }
    switch (pol) {
        case PCHASE_LRU: PC_W(PCHASE_LRU)
        case PCHASE_FIFO: PC_W(PCHASE_FIFO)
        case PCHASE_PLRU: PC_W(PCHASE_PLRU)
        case PCHASE_RANDOM: PC_W(PCHASE_RANDOM)
        default:
            if constexpr (GEN) {
                PC_W(PCHASE_WRANDOM)
            } else {
                return nullptr;   // weighted random exists for generalised models only
            }
    }
#undef PC_W
}

static StreamFn pick_stream_any(int pol, int w, bool gen) {
    return gen ? pick_stream<true>(pol, w) : pick_stream<false>(pol, w);
}

hipError_t launch_stream(int pol, int w, bool gen, const StreamArgs& args, uint32_t blocks, hipStream_t stream) {
    const StreamFn f = pick_stream_any(pol, w, gen);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(blocks), dim3(256), 0, stream, args);
    return hipGetLastError();
}

hipError_t stream_occupancy(int pol, int w, bool gen, int* blocks_per_cu) {
    const StreamFn f = pick_stream_any(pol, w, gen);
    if (!f) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)f, 256, 0);
}

}  // namespace pc
