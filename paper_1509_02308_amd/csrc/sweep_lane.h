// sweep_lane.h -- per-lane part of the probe replay: the state of one cache
// set and the enumeration of that set's accesses, in trace order, straight
// from the probe (N, s, j0, base, passes).
//
// Method (Mei & Chu, Section 4.1, Assumptions 1-3; Section 4.2): access k of
// a probe visits element (j0 + k*s) mod N (Listing 1 + Listing 2) and falls
// in set (address >> unit) mod T; only that set's a ways are involved, so
// the hit/miss decision of an access depends only on the earlier accesses of
// its own set.  Within one increasing sweep of the chase the accesses of a
// set are those inside units t, t+T, t+2T, ..., and the accesses inside one
// line are consecutive in the trace: only the first of such a run can miss,
// the others hit and leave every policy's state unchanged.
//
// Three ways to hold the a ways of a set:
//   RegSet   ways in registers, loops unrolled to the class bound (a <= 16);
//   MapSet   an LDS column per lane: a map from the line's index within the
//            set to its way, plus per way its line index and LRU links, so
//            every access costs O(1) LDS operations whatever a is (used
//            when the set's lines in the probe fit the map);
//   ScanSet  an LDS column per lane with tags and LRU ranks, scanned per
//            access (any a <= 128, any probe).
// LDS columns are laid out row-major over the 64 lanes of a wave (row r of
// lane l at dword r*64 + l), so lanes never share a bank.
#pragma once

#include "common.h"

namespace pc {

// ------------------------------------------------------------ PLRU tree --
// a-1 node bits in heap order (children of n: 2n+1 left, 2n+2 right; leaf of
// way w is a-1+w); a 0 bit sends the victim search left.
struct PlruBits {
    uint64_t lo = 0, hi = 0;
    __device__ __forceinline__ uint32_t get(uint32_t n) const {
        return n < 64 ? (uint32_t)(lo >> n) & 1u : (uint32_t)(hi >> (n - 64)) & 1u;
    }
    __device__ __forceinline__ void put(uint32_t n, uint32_t v) {
        if (n < 64) lo = (lo & ~(1ull << n)) | ((uint64_t)v << n);
        else hi = (hi & ~(1ull << (n - 64))) | ((uint64_t)v << (n - 64));
    }
    // a use of way x makes every node on its path point to the other child.
    // The node of level d on the path is 2^d - 1 + (x >> (depth - d)) (heap
    // order is level order) and the direction taken there is bit
    // depth-1-d of x, so all path bits follow from x without a chain; up to
    // depth MAXD <= 6 every node sits in `lo`.
    template <int MAXD>
    __device__ __forceinline__ void touch_upto(uint32_t x, uint32_t depth) {
        uint64_t mask = 0, val = 0;
#pragma unroll
        for (int d = 0; d < MAXD; ++d) {
            if (d < (int)depth) {
                const uint32_t node = (1u << d) - 1u + (x >> (depth - d));
                const uint32_t dir = (x >> (depth - 1 - d)) & 1u;
                mask |= 1ull << node;
                val |= (uint64_t)(dir ^ 1u) << node;
            }
        }
        lo = (lo & ~mask) | val;
    }
    template <int MAXD>
    __device__ __forceinline__ uint32_t victim_upto(uint32_t depth, uint32_t a) const {
        uint32_t node = 0;
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
            if (d < (int)depth) node = 2 * node + 1 + ((uint32_t)(lo >> node) & 1u);
        return node - (a - 1);
    }
    __device__ __forceinline__ void touch(uint32_t x, uint32_t depth) {
        if (depth <= 6) {
            touch_upto<6>(x, depth);
            return;
        }
        uint32_t node = 0;
        for (uint32_t d = 0; d < depth; ++d) {
            uint32_t dir = (x >> (depth - 1 - d)) & 1u;
            put(node, dir ^ 1u);
            node = 2 * node + 1 + dir;
        }
    }
    __device__ __forceinline__ uint32_t victim(uint32_t depth, uint32_t a) const {
        if (depth <= 6) return victim_upto<6>(depth, a);
        uint32_t node = 0;
        for (uint32_t d = 0; d < depth; ++d) node = 2 * node + 1 + get(node);
        return node - (a - 1);
    }
};

__device__ __forceinline__ uint32_t random_way(const DevModel& m, uint32_t k, uint32_t trace_id) {
    return philox_x(k, 0u, trace_id, 0u, m.seed_lo, m.seed_hi) % m.ways;
}

// ----------------------------------------------- set state in registers --
template <int A>
struct Log2Of {
    static constexpr int v = A <= 1 ? 0 : 1 + Log2Of<(A > 1 ? A / 2 : 1)>::v;
};
template <>
struct Log2Of<1> {
    static constexpr int v = 0;
};

template <int POL, int A>
struct RegSet {
    uint32_t tag[A];
    uint32_t stamp[A];  // LRU: trace index of the way's last use (distinct, so the minimum is the LRU way)
    uint32_t nvalid;    // ways fill in index order, so ways < nvalid are valid
    uint32_t ptr;       // FIFO: next way to replace
    PlruBits bits;

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int w = 0; w < A; ++w) {
            tag[w] = kInvalidTag;
            stamp[w] = 0;
        }
        nvalid = 0;
        ptr = 0;
        bits = PlruBits();
    }

    __device__ __forceinline__ bool access(uint32_t line, uint32_t, const DevModel& m, uint32_t k,
                                           uint32_t trace_id) {
        if constexpr (A == 1) {
            // one way: every policy keeps the last line (an empty way holds
            // kInvalidTag, above every line: addresses stay below 2^34 - 8)
            const bool hit = tag[0] == line;
            tag[0] = line;
            return hit;
        }
        const uint32_t a = m.ways;
        int hw = -1;
#pragma unroll
        for (int w = 0; w < A; ++w)
            if (w < (int)a && tag[w] == line) hw = w;
        const bool hit = hw >= 0;
        if constexpr (POL == PCHASE_LRU) {
            uint32_t x;
            if (hit) {
                x = (uint32_t)hw;
            } else if (nvalid < a) {
                x = nvalid++;
            } else {
                // all ways valid: the least recently used is the oldest stamp
                x = 0;
                uint32_t old = stamp[0];
#pragma unroll
                for (int w = 1; w < A; ++w)
                    if (w < (int)a && stamp[w] < old) {
                        old = stamp[w];
                        x = (uint32_t)w;
                    }
            }
#pragma unroll
            for (int w = 0; w < A; ++w)
                if ((uint32_t)w == x) {
                    stamp[w] = k;
                    tag[w] = line;
                }
        } else if constexpr (POL == PCHASE_FIFO) {
            if (!hit) {
                uint32_t x = ptr;
                ptr = (ptr + 1 == a) ? 0 : ptr + 1;
#pragma unroll
                for (int w = 0; w < A; ++w)
                    if ((uint32_t)w == x) tag[w] = line;
            }
        } else if constexpr (POL == PCHASE_PLRU) {
            constexpr int D = Log2Of<A>::v;
            uint32_t x;
            if (hit) x = (uint32_t)hw;
            else if (nvalid < a) x = nvalid++;
            else x = bits.victim_upto<D>(m.log2_ways, a);
            bits.touch_upto<D>(x, m.log2_ways);
            if (!hit) {
#pragma unroll
                for (int w = 0; w < A; ++w)
                    if ((uint32_t)w == x) tag[w] = line;
            }
        } else {  // RANDOM
            if (!hit) {
                uint32_t x;
                if (nvalid < a) x = nvalid++;
                else x = random_way(m, k, trace_id);
#pragma unroll
                for (int w = 0; w < A; ++w)
                    if ((uint32_t)w == x) tag[w] = line;
            }
        }
        return hit;
    }
};

// --------------------------------------- set state in an LDS column: map --
// Byte-addressed rows, so that no update needs a read-modify-write:
//   rows [0, mapw)            the map: byte q = way of the set's line with
//                             index q, 0xFF if absent;
//   LRU only, A4 = ceil(a/4) rows each: byte w = previous, then next, way of
//                             w in recency order;
//   then the line index q held by way w: one byte per way when the map has
//                             at most 256 entries, else a halfword.
// (LDS row r of this lane is dword r*64 of its column.)
__host__ __device__ inline bool map_q8(uint32_t map_rows) { return 4 * map_rows <= 256; }
__host__ __device__ inline uint32_t map_class_rows(uint32_t map_rows, uint32_t a, int policy) {
    const uint32_t links = policy == PCHASE_LRU ? 2 * ((a + 3) / 4) : 0;
    return map_rows + links + (map_q8(map_rows) ? (a + 3) / 4 : (a + 1) / 2);
}

template <int POL>
struct MapSet {
    static constexpr uint32_t kNil = 0xFFu;
    uint32_t* col;
    uint32_t mapw, prev_row, next_row, q_row;
    bool q8;
    uint32_t nvalid, ptr, head, tail;
    PlruBits bits;

    __device__ __forceinline__ uint8_t* byte_at(uint32_t r, uint32_t j) {
        return reinterpret_cast<uint8_t*>(col + (size_t)r * kWave) + j;
    }
    __device__ __forceinline__ uint32_t map_get(uint32_t q) { return *byte_at(q >> 2, q & 3); }
    __device__ __forceinline__ void map_put(uint32_t q, uint32_t w) { *byte_at(q >> 2, q & 3) = (uint8_t)w; }
    __device__ __forceinline__ uint32_t prev_of(uint32_t w) { return *byte_at(prev_row + (w >> 2), w & 3); }
    __device__ __forceinline__ uint32_t next_of(uint32_t w) { return *byte_at(next_row + (w >> 2), w & 3); }
    __device__ __forceinline__ void set_prev(uint32_t w, uint32_t p) { *byte_at(prev_row + (w >> 2), w & 3) = (uint8_t)p; }
    __device__ __forceinline__ void set_next(uint32_t w, uint32_t n) { *byte_at(next_row + (w >> 2), w & 3) = (uint8_t)n; }
    __device__ __forceinline__ uint32_t q_of(uint32_t w) {
        if (q8) return *byte_at(q_row + (w >> 2), w & 3);
        return *reinterpret_cast<uint16_t*>(byte_at(q_row + (w >> 1), 2 * (w & 1)));
    }
    __device__ __forceinline__ void set_q(uint32_t w, uint32_t q) {
        if (q8) *byte_at(q_row + (w >> 2), w & 3) = (uint8_t)q;
        else *reinterpret_cast<uint16_t*>(byte_at(q_row + (w >> 1), 2 * (w & 1))) = (uint16_t)q;
    }

    __device__ __forceinline__ void init(uint32_t* c, uint32_t map_rows, uint32_t a) {
        col = c;
        mapw = map_rows;
        q8 = map_q8(map_rows);
        prev_row = mapw;
        next_row = mapw + (a + 3) / 4;
        q_row = POL == PCHASE_LRU ? next_row + (a + 3) / 4 : mapw;
        for (uint32_t r = 0; r < mapw; ++r) col[(size_t)r * kWave] = 0xFFFFFFFFu;
        nvalid = 0;
        ptr = 0;
        head = tail = kNil;
        bits = PlruBits();
    }

    __device__ __forceinline__ void unlink(uint32_t x) {
        const uint32_t p = prev_of(x), n = next_of(x);
        if (p != kNil) set_next(p, n);
        else head = n;
        if (n != kNil) set_prev(n, p);
        else tail = p;
    }
    __device__ __forceinline__ void push_front(uint32_t x) {
        set_prev(x, kNil);
        set_next(x, head);
        if (head != kNil) set_prev(head, x);
        head = x;
        if (tail == kNil) tail = x;
    }

    __device__ __forceinline__ bool access(uint32_t, uint32_t q, const DevModel& m, uint32_t k,
                                           uint32_t trace_id) {
        const uint32_t a = m.ways;
        const uint32_t w = map_get(q);
        const bool hit = w != kNil;
        if constexpr (POL == PCHASE_LRU) {
            if (hit) {
                if (head != w) {
                    unlink(w);
                    push_front(w);
                }
                return true;
            }
            uint32_t x;
            if (nvalid < a) {
                x = nvalid++;
            } else {
                x = tail;
                map_put(q_of(x), kNil);
                unlink(x);
            }
            set_q(x, q);
            map_put(q, x);
            push_front(x);
            return false;
        } else {
            if constexpr (POL == PCHASE_PLRU) {
                if (hit) {
                    bits.touch(w, m.log2_ways);
                    return true;
                }
            } else {
                if (hit) return true;
            }
            uint32_t x;
            if constexpr (POL == PCHASE_FIFO) {
                x = ptr;
                ptr = (ptr + 1 == a) ? 0 : ptr + 1;
            } else if constexpr (POL == PCHASE_PLRU) {
                x = nvalid < a ? nvalid : bits.victim(m.log2_ways, a);
            } else {
                x = nvalid < a ? nvalid : random_way(m, k, trace_id);
            }
            if (nvalid < a) ++nvalid;
            else map_put(q_of(x), kNil);
            set_q(x, q);
            map_put(q, x);
            if constexpr (POL == PCHASE_PLRU) bits.touch(x, m.log2_ways);
            return false;
        }
    }
};

// -------------------------------------- set state in an LDS column: scan --
// Rows [0, a): tags; rows [a, a + ceil(a/4)): LRU ranks, four 8-bit ranks per
// dword (0xFF = empty way).
template <int POL>
struct ScanSet {
    uint32_t* col;
    uint32_t a;
    uint32_t nvalid, ptr;
    PlruBits bits;

    __device__ __forceinline__ uint32_t& tag(uint32_t w) { return col[(size_t)w * kWave]; }
    __device__ __forceinline__ uint32_t& rank_word(uint32_t w) { return col[(size_t)(a + (w >> 2)) * kWave]; }
    __device__ __forceinline__ uint32_t rank(uint32_t w) { return (rank_word(w) >> ((w & 3) * 8)) & 0xFFu; }
    __device__ __forceinline__ void set_rank(uint32_t w, uint32_t v) {
        uint32_t& d = rank_word(w);
        const uint32_t sh = (w & 3) * 8;
        d = (d & ~(0xFFu << sh)) | (v << sh);
    }

    __device__ __forceinline__ void init(uint32_t* c, uint32_t ways) {
        col = c;
        a = ways;
        nvalid = 0;
        ptr = 0;
        bits = PlruBits();
        for (uint32_t w = 0; w < a; ++w) tag(w) = kInvalidTag;
        if (POL == PCHASE_LRU)
            for (uint32_t w = 0; w < a; w += 4) rank_word(w) = 0xFFFFFFFFu;
    }

    __device__ __forceinline__ bool access(uint32_t line, uint32_t, const DevModel& m, uint32_t k,
                                           uint32_t trace_id) {
        uint32_t hw = kInvalidTag;
        for (uint32_t w = 0; w < a; ++w)
            if (tag(w) == line) hw = w;
        const bool hit = hw != kInvalidTag;
        uint32_t x;
        if constexpr (POL == PCHASE_LRU) {
            uint32_t ax;
            if (hit) {
                x = hw;
                ax = rank(hw);
            } else if (nvalid < a) {
                x = nvalid;
                ax = nvalid;
                ++nvalid;
            } else {
                ax = a - 1;
                x = 0;
                for (uint32_t w = 0; w < a; ++w)
                    if (rank(w) == a - 1) x = w;
            }
            // ranks below ax move up by one; way x becomes the most recent
            for (uint32_t w = 0; w < a; w += 4) {
                uint32_t d = rank_word(w), o = 0;
#pragma unroll
                for (uint32_t b = 0; b < 4; ++b) {
                    uint32_t g = (d >> (8 * b)) & 0xFFu;
                    if (w + b < a) {
                        if (g < ax) ++g;
                        if (w + b == x) g = 0;
                    }
                    o |= g << (8 * b);
                }
                rank_word(w) = o;
            }
            if (!hit) tag(x) = line;
        } else if constexpr (POL == PCHASE_FIFO) {
            if (!hit) {
                x = ptr;
                ptr = (ptr + 1 == a) ? 0 : ptr + 1;
                tag(x) = line;
            }
        } else if constexpr (POL == PCHASE_PLRU) {
            if (hit) x = hw;
            else if (nvalid < a) x = nvalid++;
            else x = bits.victim(m.log2_ways, a);
            bits.touch(x, m.log2_ways);
            if (!hit) tag(x) = line;
        } else {
            if (!hit) {
                x = nvalid < a ? nvalid++ : random_way(m, k, trace_id);
                tag(x) = line;
            }
        }
        return hit;
    }
};

// ------------------------------------------------- access enumeration ----
// One increasing sweep of a pass: elements r, r+se, ... (cnt of them) at
// byte addresses xf, xf+sb, ...; everything here is independent of the set,
// so a lane computes it once and walks each of its sets from it.
struct Sweep {
    uint64_t xf;     // address of the first access
    uint32_t cnt;    // accesses in the sweep
    uint32_t kin;    // index of the first access within the pass
    uint32_t uf, ul; // first and last unit touched (addresses < 2^34, units >= 4 bytes)
    uint32_t qf;     // floor(uf / T)
    uint32_t rem;    // uf mod T
    uint32_t unit_mode;  // 1: walk units (stride below T units), 0: walk accesses
    uint32_t fast;   // unit mode: offsets fit 32 bits, divide by the stride's multiplier
    // aligned (1): a unit is one line, the stride divides it and the sweep
    // starts on a stride boundary: every full unit holds R accesses and the
    // first access of unit uf + d is d*R - off0, no division needed.
    // strided (2): the stride is dd units: access i lies in unit uf + i dd,
    // so set rem + c (mod T) holds the accesses i = i0 + j R with R =
    // T / g, g = gcd(dd, T), when g divides c, and i0 = (c / g) off0 mod R,
    // off0 the inverse of dd / g modulo R.
    uint32_t aligned;
    uint32_t R;
    uint32_t off0;
};

// Inverse of x modulo n (gcd(x, n) = 1, n >= 1) by the extended Euclidean
// algorithm; 0 when n == 1.
__device__ __forceinline__ uint32_t inv_mod(uint32_t x, uint32_t n) {
    int64_t r0 = n, r1 = x % n, t0 = 0, t1 = 1;
    while (r1 != 0) {
        const int64_t q = r0 / r1;
        const int64_t r2 = r0 - q * r1, t2 = t0 - q * t1;
        r0 = r1;
        r1 = r2;
        t0 = t1;
        t1 = t2;
    }
    if (t0 < 0) t0 += n;
    return n == 1 ? 0u : (uint32_t)t0;
}

__device__ __forceinline__ uint32_t gcd_u32(uint32_t x, uint32_t y) {
    while (y) {
        const uint32_t t = x % y;
        x = y;
        y = t;
    }
    return x;
}

__device__ __forceinline__ void sweep_geo(Sweep& w, uint64_t xf, uint64_t sb, uint32_t cnt, uint32_t kin,
                                          const DevModel& m, const DevProbe& p) {
    const uint32_t us = m.unit_shift;
    const uint64_t U = 1ull << us;
    w.xf = xf;
    w.cnt = cnt;
    w.kin = kin;
    const uint64_t uf = xf >> us;
    w.uf = (uint32_t)uf;
    w.ul = (uint32_t)((xf + (uint64_t)(cnt - 1) * sb) >> us);
    w.qf = w.uf / m.sets;
    w.rem = w.uf - w.qf * m.sets;
    w.unit_mode = (sb > 0 && sb < U * m.sets) ? 1u : 0u;
    w.fast = (w.unit_mode && p.sb_fast && (uint64_t)(cnt - 1) * sb + U + sb < (1ull << 32)) ? 1u : 0u;
    w.aligned = 0;
    w.R = 0;
    w.off0 = 0;
    if (w.unit_mode && m.unit_shift == m.line_shift && sb <= U && (U % sb) == 0 && (xf % sb) == 0) {
        const uint64_t R = U / sb;
        if (cnt < (1u << 30) && R * m.sets < (1ull << 30)) {
            w.aligned = 1;
            w.R = (uint32_t)R;
            w.off0 = (uint32_t)((xf - (uf << us)) / sb);
        }
    } else if (sb > 0 && (sb & (U - 1)) == 0 && cnt > 1 && cnt < (1u << 30)) {
        const uint64_t dd = sb >> us;
        const uint32_t T = m.sets;
        const uint32_t dm = (uint32_t)(dd % T);
        const uint32_t g = gcd_u32(dm, T);   // gcd(0, T) = T
        const uint32_t P = T / g;
        if (dd < (1ull << 32)) {
            w.aligned = 2;
            w.R = P;
            w.off0 = inv_mod((uint32_t)((dd / g) % P), P);
        }
    }
}

// Calls visit(line, q, k0, r) for every run of r consecutive accesses
// k0 .. k0+r-1 of one sweep inside one line of set `set`, in trace order.
// q is the line's index among the set's lines of the probe:
// (floor(u/T) - floor(u_lo/T)) * R + (line mod R), with u the line's unit,
// u_lo the probe's lowest unit and R lines per unit.
template <class Visit>
__device__ __forceinline__ void sweep_walk(const Sweep& w, uint32_t kpass, uint64_t sb, const DevModel& m,
                                           const DevProbe& p, uint32_t set, uint32_t qlo, Visit& visit) {
    const uint32_t T = m.sets;
    const uint32_t us = m.unit_shift, ls = m.line_shift;
    const uint32_t rsh = us - ls;
    const uint64_t U = 1ull << us;
    const uint64_t xf = w.xf;
    const uint32_t cnt = w.cnt, kstart = kpass + w.kin;
    if (w.aligned == 2) {
        // strided: only this set's accesses i0, i0 + P, ...; the unit grows
        // by P dd = T (dd / g), so its quotient by T grows by dd / g, and
        // the line by P (sb >> ls) (the stride is a multiple of the line)
        const uint32_t c = set >= w.rem ? set - w.rem : set + T - w.rem;
        const uint32_t P = w.R, g = T / P;
        if (c % g) return;
        const uint32_t i0 = (uint32_t)(((uint64_t)(c / g) * w.off0) % P);
        if (i0 >= cnt) return;
        const uint32_t n = (cnt - 1 - i0) / P + 1;
        const uint64_t dd = sb >> us, lb = sb >> ls;
        const uint32_t sdg = (uint32_t)(dd / g);
        uint32_t Q = w.qf + (uint32_t)(((uint64_t)w.rem + (uint64_t)i0 * dd) / T) - qlo;
        uint32_t line = (uint32_t)((xf >> ls) + (uint64_t)i0 * lb);
        const uint32_t lstep = (uint32_t)((uint64_t)P * lb);   // wraps only past the last access
        uint32_t k = kstart + i0;
        for (uint32_t j = 0; j < n; ++j, line += lstep, Q += sdg, k += P)
            visit(line, (Q << rsh) + (line & ((1u << rsh) - 1)), k, 1);
        return;
    }
    if (w.aligned) {
        // unit u = uf + d starts at access d*R - off0; units advance by T
        const uint32_t d = set >= w.rem ? set - w.rem : set + T - w.rem;
        uint32_t u = w.uf + d;
        uint32_t Q = w.qf + (set < w.rem ? 1u : 0u) - qlo;
        const int32_t R = (int32_t)w.R;
        const int32_t step = (int32_t)(T * w.R);
        const int32_t last = (int32_t)cnt - 1;
        for (int32_t ilo_raw = (int32_t)(d * w.R) - (int32_t)w.off0; ilo_raw <= last;
             ilo_raw += step, u += T, ++Q) {
            const int32_t ilo = ilo_raw < 0 ? 0 : ilo_raw;
            const int32_t ihi = ilo_raw + R - 1 < last ? ilo_raw + R - 1 : last;
            visit(u, Q, kstart + (uint32_t)ilo, (uint32_t)(ihi - ilo + 1));
        }
        return;
    }
    if (w.unit_mode) {
        // the first unit of this set at or after uf, and its quotient by T;
        // counted iterations, since u + T may pass 2^32 after the last unit
        const uint64_t u0 = (uint64_t)w.uf + (set >= w.rem ? set - w.rem : set + T - w.rem);
        if (u0 > w.ul) return;
        const uint32_t n_units = (uint32_t)(w.ul - u0) / T + 1;
        uint32_t u = (uint32_t)u0;
        uint32_t Q = w.qf + (set < w.rem ? 1u : 0u) - qlo;
        for (uint32_t it = 0; it < n_units; ++it, u += T, ++Q) {
            const uint64_t lo = (uint64_t)u << us;
            uint32_t ilo, ihi;
            if (w.fast) {
                ilo = lo <= xf ? 0 : p.sb_div.div((uint32_t)(lo - xf + sb - 1));
                ihi = p.sb_div.div((uint32_t)(lo + U - 1 - xf));
            } else {
                ilo = lo <= xf ? 0 : (uint32_t)udiv64(lo - xf + sb - 1, sb);
                const uint64_t h = udiv64(lo + U - 1 - xf, sb);
                ihi = h > cnt - 1 ? cnt - 1 : (uint32_t)h;
            }
            if (ihi > cnt - 1) ihi = cnt - 1;
            if (ilo > ihi) continue;
            if (rsh == 0) {
                visit(u, Q, kstart + ilo, ihi - ilo + 1);
            } else {
                uint32_t i = ilo;
                while (i <= ihi) {
                    const uint32_t line = (uint32_t)((xf + (uint64_t)i * sb) >> ls);
                    const uint64_t lend = (uint64_t)(line + 1) << ls;
                    uint64_t inext = udiv64(lend - xf + sb - 1, sb);
                    if (inext > (uint64_t)ihi + 1) inext = (uint64_t)ihi + 1;
                    visit(line, (Q << rsh) + (line & ((1u << rsh) - 1)), kstart + i, (uint32_t)inext - i);
                    i = (uint32_t)inext;
                }
            }
        }
    } else {
        // stride of at least T units (or a single access): walk the
        // accesses, tracking the set and the unit's quotient by T
        // incrementally (the unit advances by d or d+1 per access)
        uint64_t x = xf;
        uint32_t u = w.uf;
        uint32_t st = w.rem;
        uint32_t Q = w.qf - qlo;
        const uint64_t d0 = sb >> us;
        const uint64_t dq0 = udiv64(d0, T), dq1 = udiv64(d0 + 1, T);
        const uint32_t dm0 = (uint32_t)(d0 - dq0 * T), dm1 = (uint32_t)(d0 + 1 - dq1 * T);
        for (uint32_t i = 0; i < cnt; ++i) {
            if (st == set) {
                const uint32_t line = (uint32_t)(x >> ls);
                visit(line, (Q << rsh) + (line & ((1u << rsh) - 1)), kstart + i, 1);
            }
            if (i + 1 == cnt) break;
            const uint64_t xn = x + sb;
            const uint32_t un = (uint32_t)(xn >> us);
            const bool one = ((uint64_t)(un - u) == d0);
            st += one ? dm0 : dm1;
            Q += (uint32_t)(one ? dq0 : dq1);
            if (st >= T) {
                st -= T;
                ++Q;
            }
            x = xn;
            u = un;
        }
    }
}

// Sweeps of one pass, in order: calls f(sweep) for each.
template <class F>
__device__ __forceinline__ void pass_sweeps(const DevProbe& p, const DevModel& m, F& f) {
    const uint32_t es = p.elem_shift;
    const uint64_t sb = (uint64_t)p.se << es;
    Sweep w;
    if (p.se == 0) {  // s is a multiple of N: the chase stays on j0
        sweep_geo(w, p.base + ((uint64_t)p.j0 << es), 0, 1, 0, m, p);
        f(w);
        return;
    }
    uint32_t r = p.j0, kpos = 0;
    while (kpos < p.L) {
        // one increasing sweep: r, r+se, ... < ne
        uint32_t cnt = (uint32_t)(((uint64_t)p.ne - r + p.se - 1) / p.se);
        if (cnt > p.L - kpos) cnt = p.L - kpos;
        sweep_geo(w, p.base + ((uint64_t)r << es), sb, cnt, kpos, m, p);
        f(w);
        kpos += cnt;
        r = (uint32_t)((uint64_t)r + (uint64_t)cnt * p.se - p.ne);
    }
}

__device__ __forceinline__ uint32_t probe_qlo(const DevProbe& p, const DevModel& m) {
    return (uint32_t)(p.base >> m.unit_shift) / m.sets;
}

// All runs of set `set` over the whole probe (every pass), in trace order.
template <class Visit>
__device__ __forceinline__ void probe_runs(const DevProbe& p, const DevModel& m, uint32_t set, Visit& visit) {
    const uint64_t sb = (uint64_t)p.se << p.elem_shift;
    const uint32_t qlo = probe_qlo(p, m);
    for (uint32_t pass = 0; pass < p.passes; ++pass) {
        const uint32_t kpass = pass * p.L;
        auto f = [&](const Sweep& w) { sweep_walk(w, kpass, sb, m, p, set, qlo, visit); };
        pass_sweeps(p, m, f);
    }
}

// Sweeps of one pass precomputed for a lane that replays many sets of the
// same probe; probes with more than kCachedSweeps sweeps per pass fall back
// to probe_runs.
// Field-wise select of two sweeps held in registers (a select of their
// addresses would force both into scratch memory).
__device__ __forceinline__ Sweep pick_sweep(bool first, const Sweep& a, const Sweep& b) {
    Sweep w;
    w.xf = first ? a.xf : b.xf;
    w.cnt = first ? a.cnt : b.cnt;
    w.kin = first ? a.kin : b.kin;
    w.uf = first ? a.uf : b.uf;
    w.ul = first ? a.ul : b.ul;
    w.qf = first ? a.qf : b.qf;
    w.rem = first ? a.rem : b.rem;
    w.unit_mode = first ? a.unit_mode : b.unit_mode;
    w.fast = first ? a.fast : b.fast;
    w.aligned = first ? a.aligned : b.aligned;
    w.R = first ? a.R : b.R;
    w.off0 = first ? a.off0 : b.off0;
    return w;
}

// The two sweeps are named members, not an array: a runtime index into a
// per-lane array would place it in scratch memory.
constexpr int kCachedSweeps = 2;
struct SweepCache {
    Sweep w0, w1;
    uint32_t n;   // sweeps per pass, or kCachedSweeps + 1 if they do not fit
    uint32_t qlo;
    uint64_t sb;
};

__device__ __forceinline__ void sweep_cache(SweepCache& c, const DevProbe& p, const DevModel& m) {
    c.n = 0;
    c.qlo = probe_qlo(p, m);
    c.sb = (uint64_t)p.se << p.elem_shift;
    c.w0 = Sweep{};
    c.w1 = Sweep{};
    // unconditional field-wise updates: a store whose destination depends
    // on the branch taken would keep the cache in scratch memory
    auto f = [&](const Sweep& w) {
        c.w0 = pick_sweep(c.n == 0, w, c.w0);
        c.w1 = pick_sweep(c.n == 1, w, c.w1);
        ++c.n;
    };
    pass_sweeps(p, m, f);
}

template <class Visit>
__device__ __forceinline__ void cached_runs(const SweepCache& c, const DevProbe& p, const DevModel& m, uint32_t set,
                                            Visit& visit) {
    if (c.n > kCachedSweeps) {
        probe_runs(p, m, set, visit);
        return;
    }
    for (uint32_t pass = 0; pass < p.passes; ++pass) {
        const uint32_t kpass = pass * p.L;
        for (uint32_t i = 0; i < c.n; ++i) {
            const Sweep w = pick_sweep(i != 0, c.w1, c.w0);
            sweep_walk(w, kpass, c.sb, m, p, set, c.qlo, visit);
        }
    }
}

// Capacity a MapSet needs for probe p under model m: number of distinct line
// indices q any set can see.
inline uint64_t map_entries(const DevProbe& p, const DevModel& m) {
    const uint64_t xlo = p.base, xhi = p.base + ((uint64_t)(p.ne - 1) << p.elem_shift);
    const uint64_t ulo = xlo >> m.unit_shift, uhi = xhi >> m.unit_shift;
    const uint64_t qspan = uhi / m.sets - ulo / m.sets + 1;
    return qspan << (m.unit_shift - m.line_shift);
}

}  // namespace pc
