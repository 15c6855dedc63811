/*
 * oracle.c -- plain, slow, obviously-correct CPU reference of the P-chase
 * cache-model replay.  TEST INFRASTRUCTURE ONLY: loaded by the tests, the
 * smoke check and the benchmark's CPU-baseline leg, never by the product
 * path.  Shares nothing with the HIP implementation.
 *
 * Data structures are chosen for readability, not speed: every set keeps
 * its ways as arrays of (valid, tag, stamp), LRU and FIFO pick the victim by
 * the smallest time stamp, tree-PLRU keeps its a-1 node bits as bytes.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11, Section 3: the Philox round is two
 * 32x32->64 multiplications whose high halves are xored with the other two
 * counter words and the round key; the key is bumped by the golden-ratio
 * and sqrt(3)-1 Weyl constants between rounds; ten rounds).               */
/* ---------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ---------------------------------------------------------------------- */
/* Trace generation: Listing 1 fills A[i] = (i + stride) mod size, Listing 2
 * follows j = A[j].  Starting from j0 the k-th visited index is therefore
 * (j0 + k*stride) mod size, and one pass is the cycle of that map through
 * j0, of length size / gcd(size, stride mod size).                        */
/* ---------------------------------------------------------------------- */
static uint64_t gcd_u64(uint64_t x, uint64_t y)
{
    while (y != 0) {
        uint64_t t = x % y;
        x = y;
        y = t;
    }
    return x;
}

static int probe_ok(const orc_probe *p)
{
    if (p->elem == 0) return 0;
    if (p->n_bytes == 0 || p->n_bytes % p->elem != 0) return 0;
    if (p->s_bytes % p->elem != 0) return 0;
    uint64_t ne = p->n_bytes / p->elem;
    if (ne >= (1ull << 31)) return 0;
    if (p->j0 >= ne) return 0;
    if (p->passes == 0) return 0;
    return 1;
}

uint64_t orc_cycle_len(const orc_probe *p)
{
    if (!probe_ok(p)) return 0;
    uint64_t ne = p->n_bytes / p->elem;
    uint64_t se = (p->s_bytes / p->elem) % ne;
    return ne / gcd_u64(ne, se);
}

uint64_t orc_trace_len(const orc_probe *p)
{
    uint64_t L = orc_cycle_len(p);
    return L * (L ? p->passes : 0);
}

uint64_t orc_trace(const orc_probe *p, int32_t *out, uint64_t cap)
{
    uint64_t len = orc_trace_len(p);
    if (len == 0 || len > cap) return 0;
    uint64_t ne = p->n_bytes / p->elem;
    uint64_t se = p->s_bytes / p->elem;
    for (uint64_t k = 0; k < len; ++k) {
        /* 128-bit product: k*se can exceed 64 bits only in theory, keep it exact */
        unsigned __int128 v = (unsigned __int128)k * se + p->j0;
        out[k] = (int32_t)(uint64_t)(v % ne);
    }
    return len;
}

/* ---------------------------------------------------------------------- */
/* Non-uniform-stride trace (Section 5.2, Fig. 13(b)): the array is set up
 * so that the chase leaves each visited element by the stride of the
 * segment that element belongs to.  Walked literally: visit, then step by
 * the current segment's stride modulo the array size; every pass starts
 * again at j0 (the last element of a pass points back to the first).      */
/* ---------------------------------------------------------------------- */
uint64_t orc_trace_nu_len(const orc_nu_probe *p, const uint64_t *counts)
{
    if (p->elem == 0 || p->n_bytes == 0 || p->n_bytes % p->elem != 0) return 0;
    uint64_t ne = p->n_bytes / p->elem;
    if (ne >= (1ull << 31) || p->j0 >= ne || p->passes == 0 || p->n_segments == 0) return 0;
    uint64_t per_pass = 0;
    for (uint64_t i = 0; i < p->n_segments; ++i) {
        if (counts[i] == 0) return 0;
        per_pass += counts[i];
    }
    return per_pass * p->passes;
}

uint64_t orc_trace_nu(const orc_nu_probe *p, const uint64_t *s_bytes, const uint64_t *counts,
                      int32_t *out, uint64_t cap)
{
    uint64_t len = orc_trace_nu_len(p, counts);
    if (len == 0 || len > cap) return 0;
    for (uint64_t i = 0; i < p->n_segments; ++i)
        if (s_bytes[i] % p->elem != 0) return 0;
    uint64_t ne = p->n_bytes / p->elem;
    uint64_t k = 0;
    for (uint64_t pass = 0; pass < p->passes; ++pass) {
        uint64_t j = p->j0;
        for (uint64_t i = 0; i < p->n_segments; ++i) {
            uint64_t step = (s_bytes[i] / p->elem) % ne;
            for (uint64_t t = 0; t < counts[i]; ++t) {
                out[k++] = (int32_t)j;
                j = (j + step) % ne;
            }
        }
    }
    return len;
}

/* ---------------------------------------------------------------------- */
/* Model checks: Assumption 1 (T*a*b == C), a power-of-two line, a
 * power-of-two associativity for the binary PLRU tree, and a set unit no
 * smaller than a line.                                                     */
/* ---------------------------------------------------------------------- */
static int is_pow2(uint64_t x) { return x != 0 && (x & (x - 1)) == 0; }

int orc_model_check(const orc_model *m)
{
    if (m->ways == 0 || m->sets == 0 || m->line == 0) return -1;
    if (!is_pow2(m->line)) return -1;
    if (m->sets * m->ways * m->line != m->capacity) return -1;
    if (m->policy > ORC_RANDOM) return -1;
    if (m->policy == ORC_PLRU && !is_pow2(m->ways)) return -1;
    if (m->set_shift != 0) {
        if (m->set_shift >= 63) return -1;
        if ((1ull << m->set_shift) < m->line) return -1;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Replay (Section 4.1, Assumptions 1-3, generalised to the non-LRU
 * policies).  The cache starts empty; a miss fills the lowest-numbered
 * empty way of its set, and only when the set is full does the policy
 * choose a victim.                                                          */
/* ---------------------------------------------------------------------- */
typedef struct orc_cache {
    uint64_t T, a;
    uint8_t *valid;   /* [T][a] */
    uint64_t *tag;    /* [T][a] line number held by the way */
    uint64_t *stamp;  /* [T][a] LRU: time of last use; FIFO: time of fill */
    uint8_t *tree;    /* [T][a-1] PLRU node bits, heap order */
} orc_cache;

static int cache_init(orc_cache *c, uint64_t T, uint64_t a)
{
    c->T = T;
    c->a = a;
    c->valid = (uint8_t *)calloc(T * a, 1);
    c->tag = (uint64_t *)calloc(T * a, sizeof(uint64_t));
    c->stamp = (uint64_t *)calloc(T * a, sizeof(uint64_t));
    c->tree = (uint8_t *)calloc(T * (a > 1 ? a - 1 : 1), 1);
    return (c->valid && c->tag && c->stamp && c->tree) ? 0 : -1;
}

static void cache_free(orc_cache *c)
{
    free(c->valid);
    free(c->tag);
    free(c->stamp);
    free(c->tree);
}

/* tree-PLRU: node n has children 2n+1 (left) and 2n+2 (right); the leaf of
 * way w is node a-1+w.  A 0 bit sends the victim search left, a 1 bit
 * right; a use of way w turns every bit on its path to point away from w. */
static void plru_touch(uint8_t *bits, uint64_t a, uint64_t w)
{
    uint64_t node = a - 1 + w;
    while (node != 0) {
        uint64_t parent = (node - 1) / 2;
        int came_from_left = (node == 2 * parent + 1);
        bits[parent] = came_from_left ? 1 : 0;
        node = parent;
    }
}

static uint64_t plru_victim(const uint8_t *bits, uint64_t a)
{
    uint64_t node = 0;
    while (node < a - 1) node = 2 * node + 1 + (bits[node] ? 1 : 0);
    return node - (a - 1);
}

static uint64_t random_victim(const orc_model *m, uint64_t k, uint64_t trace_id)
{
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32),
                       (uint32_t)trace_id, (uint32_t)(trace_id >> 32)};
    uint32_t key[2] = {(uint32_t)m->seed, (uint32_t)(m->seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return (uint64_t)out[0] % m->ways;
}

int orc_replay(const orc_model *m, const int32_t *idx, uint64_t len,
               uint64_t base, uint64_t elem, uint64_t trace_id,
               uint64_t count_from, uint8_t *hits,
               uint64_t *misses_total, uint64_t *misses_steady)
{
    if (orc_model_check(m) != 0) return -1;
    if (elem == 0) return -1;
    orc_cache c;
    if (cache_init(&c, m->sets, m->ways) != 0) {
        cache_free(&c);
        return -3;
    }
    const uint64_t a = m->ways;
    uint64_t mt = 0, ms = 0;
    for (uint64_t k = 0; k < len; ++k) {
        if (idx[k] < 0) {
            cache_free(&c);
            return -1;
        }
        uint64_t addr = base + elem * (uint64_t)idx[k];
        uint64_t line = addr / m->line;
        uint64_t unit = m->set_shift ? (addr >> m->set_shift) : line;
        uint64_t set = unit % m->sets;
        uint8_t *valid = c.valid + set * a;
        uint64_t *tag = c.tag + set * a;
        uint64_t *stamp = c.stamp + set * a;
        uint8_t *tree = c.tree + set * (a > 1 ? a - 1 : 1);

        int64_t way = -1;
        for (uint64_t w = 0; w < a; ++w)
            if (valid[w] && tag[w] == line) way = (int64_t)w;

        int hit = (way >= 0);
        if (hit) {
            if (m->policy == ORC_LRU) stamp[way] = k;
            if (m->policy == ORC_PLRU && a > 1) plru_touch(tree, a, (uint64_t)way);
        } else {
            int64_t empty = -1;
            for (uint64_t w = 0; w < a && empty < 0; ++w)
                if (!valid[w]) empty = (int64_t)w;
            uint64_t v;
            if (empty >= 0) {
                v = (uint64_t)empty;
            } else if (m->policy == ORC_LRU || m->policy == ORC_FIFO) {
                v = 0;
                for (uint64_t w = 1; w < a; ++w)
                    if (stamp[w] < stamp[v]) v = w;
            } else if (m->policy == ORC_PLRU) {
                v = a > 1 ? plru_victim(tree, a) : 0;
            } else {
                v = random_victim(m, k, trace_id);
            }
            valid[v] = 1;
            tag[v] = line;
            stamp[v] = k;
            if (m->policy == ORC_PLRU && a > 1) plru_touch(tree, a, v);
            mt += 1;
            if (k >= count_from) ms += 1;
        }
        if (hits) hits[k] = (uint8_t)hit;
    }
    cache_free(&c);
    if (misses_total) *misses_total = mt;
    if (misses_steady) *misses_steady = ms;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Generalised cache: sets of their own associativity, a table mapping and
 * weighted random replacement.  Same fill rule (lowest empty way first) and
 * the same per-set LRU/FIFO stamps, PLRU trees and Philox draws as above,
 * each set sized by its own way count.                                      */
/* ---------------------------------------------------------------------- */
int orc_general_check(const orc_general *g)
{
    if (g->line == 0 || !is_pow2(g->line) || g->sets == 0 || g->ways == NULL) return -1;
    if (g->policy > ORC_WRANDOM) return -1;
    if (g->set_shift != 0 && (g->set_shift >= 63 || (1ull << g->set_shift) < g->line)) return -1;
    if (g->table_len != 0) {
        if (g->table == NULL) return -1;
        for (uint64_t i = 0; i < g->table_len; ++i)
            if (g->table[i] >= g->sets) return -1;
    }
    for (uint64_t t = 0; t < g->sets; ++t) {
        if (g->ways[t] == 0) return -1;
        if (g->policy == ORC_PLRU && !is_pow2(g->ways[t])) return -1;
        if (g->policy == ORC_WRANDOM) {
            if (g->weights == NULL) return -1;
            uint64_t sum = 0;
            for (uint64_t w = 0; w < g->ways[t]; ++w) sum += g->weights[w];
            if (sum == 0 || sum > 65536) return -1;
        }
    }
    return 0;
}

static uint64_t weighted_victim(const orc_general *g, uint64_t a, uint64_t k, uint64_t trace_id)
{
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32),
                       (uint32_t)trace_id, (uint32_t)(trace_id >> 32)};
    uint32_t key[2] = {(uint32_t)g->seed, (uint32_t)(g->seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    uint64_t sum = 0;
    for (uint64_t w = 0; w < a; ++w) sum += g->weights[w];
    uint64_t r = (uint64_t)out[0] % sum;
    uint64_t cum = 0;
    for (uint64_t w = 0; w < a; ++w) {
        cum += g->weights[w];
        if (r < cum) return w;
    }
    return a - 1;  /* not reached: r < sum */
}

int orc_replay_general(const orc_general *g, const int32_t *idx, uint64_t len,
                       uint64_t base, uint64_t elem, uint64_t trace_id,
                       uint64_t count_from, uint8_t *hits,
                       uint64_t *misses_total, uint64_t *misses_steady)
{
    if (orc_general_check(g) != 0 || elem == 0) return -1;
    /* each set's ways live at first[t] .. first[t] + ways[t] - 1 */
    uint64_t *first = (uint64_t *)calloc(g->sets + 1, sizeof(uint64_t));
    if (!first) return -3;
    for (uint64_t t = 0; t < g->sets; ++t) first[t + 1] = first[t] + g->ways[t];
    const uint64_t total = first[g->sets];
    uint8_t *valid = (uint8_t *)calloc(total, 1);
    uint64_t *tag = (uint64_t *)calloc(total, sizeof(uint64_t));
    uint64_t *stamp = (uint64_t *)calloc(total, sizeof(uint64_t));
    uint8_t *tree = (uint8_t *)calloc(total, 1);   /* a-1 node bits of a set at first[t] */
    if (!valid || !tag || !stamp || !tree) {
        free(first); free(valid); free(tag); free(stamp); free(tree);
        return -3;
    }
    uint64_t mt = 0, ms = 0;
    int rc = 0;
    for (uint64_t k = 0; k < len; ++k) {
        if (idx[k] < 0) { rc = -1; break; }
        uint64_t addr = base + elem * (uint64_t)idx[k];
        uint64_t line = addr / g->line;
        uint64_t unit = g->set_shift ? (addr >> g->set_shift) : line;
        uint64_t set = g->table_len ? g->table[unit % g->table_len] : unit % g->sets;
        uint64_t a = g->ways[set], o = first[set];
        int64_t way = -1;
        for (uint64_t w = 0; w < a; ++w)
            if (valid[o + w] && tag[o + w] == line) way = (int64_t)w;
        int hit = (way >= 0);
        if (hit) {
            if (g->policy == ORC_LRU) stamp[o + way] = k;
            if (g->policy == ORC_PLRU && a > 1) plru_touch(tree + o, a, (uint64_t)way);
        } else {
            int64_t empty = -1;
            for (uint64_t w = 0; w < a && empty < 0; ++w)
                if (!valid[o + w]) empty = (int64_t)w;
            uint64_t v;
            if (empty >= 0) {
                v = (uint64_t)empty;
            } else if (g->policy == ORC_LRU || g->policy == ORC_FIFO) {
                v = 0;
                for (uint64_t w = 1; w < a; ++w)
                    if (stamp[o + w] < stamp[o + v]) v = w;
            } else if (g->policy == ORC_PLRU) {
                v = a > 1 ? plru_victim(tree + o, a) : 0;
            } else if (g->policy == ORC_RANDOM) {
                uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32),
                                   (uint32_t)trace_id, (uint32_t)(trace_id >> 32)};
                uint32_t key[2] = {(uint32_t)g->seed, (uint32_t)(g->seed >> 32)};
                uint32_t out[4];
                orc_philox4x32_10(ctr, key, out);
                v = (uint64_t)out[0] % a;
            } else {
                v = weighted_victim(g, a, k, trace_id);
            }
            valid[o + v] = 1;
            tag[o + v] = line;
            stamp[o + v] = k;
            if (g->policy == ORC_PLRU && a > 1) plru_touch(tree + o, a, v);
            mt += 1;
            if (k >= count_from) ms += 1;
        }
        if (hits) hits[k] = (uint8_t)hit;
    }
    free(first); free(valid); free(tag); free(stamp); free(tree);
    if (rc) return rc;
    if (misses_total) *misses_total = mt;
    if (misses_steady) *misses_steady = ms;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Latency -> hit/miss.  The paper's average-latency model t = t0 + tm*r
 * separates accesses into a fast (hit) and a slow (miss) population; the
 * threshold is the lower end of the widest gap between distinct values.   */
/* ---------------------------------------------------------------------- */
void orc_classify(const uint32_t *lat, uint64_t n, uint32_t theta, uint8_t *hits)
{
    for (uint64_t i = 0; i < n; ++i) hits[i] = lat[i] <= theta ? 1 : 0;
}

static int cmp_u32(const void *x, const void *y)
{
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return a < b ? -1 : (a > b ? 1 : 0);
}

uint32_t orc_auto_threshold(const uint32_t *lat, uint64_t n)
{
    if (n == 0) return 0;
    uint32_t *v = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!v) return 0;
    memcpy(v, lat, n * sizeof(uint32_t));
    qsort(v, n, sizeof(uint32_t), cmp_u32);
    uint32_t best_lo = v[n - 1], best_gap = 0;
    for (uint64_t i = 1; i < n; ++i) {
        uint32_t gap = v[i] - v[i - 1];
        if (gap > best_gap) {  /* strict: the lowest of equal-width gaps wins */
            best_gap = gap;
            best_lo = v[i - 1];
        }
    }
    free(v);
    return best_lo;
}

/* ---------------------------------------------------------------------- */
/* Inference: the Fig. 6 procedure reads C, b, T/a and the policy off the
 * traces; here every candidate model is replayed against the observed
 * traces and scored by the number of mismatched hit/miss decisions.       */
/* ---------------------------------------------------------------------- */
int64_t orc_infer_general(const orc_general *cands, uint64_t n_cands,
                          const orc_probe *probes, uint64_t n_probes,
                          const uint8_t *obs_hits, const uint64_t *obs_off,
                          const uint64_t *count_from, uint64_t *m, uint64_t *n)
{
    uint64_t maxlen = 0;
    for (uint64_t p = 0; p < n_probes; ++p) {
        uint64_t len = orc_trace_len(&probes[p]);
        if (len == 0) return -2;
        if (len > maxlen) maxlen = len;
    }
    int32_t *tr = (int32_t *)malloc((maxlen ? maxlen : 1) * sizeof(int32_t));
    uint8_t *hit = (uint8_t *)malloc(maxlen ? maxlen : 1);
    if (!tr || !hit) {
        free(tr);
        free(hit);
        return -3;
    }
    /* Step (iv) of Section 4.2 with generalised candidates: each candidate
     * replays every observed probe; m counts the accesses, from count_from
     * on, whose hit or miss differs from the observation, n those compared */
    for (uint64_t c = 0; c < n_cands; ++c) {
        m[c] = 0;
        n[c] = 0;
        if (orc_general_check(&cands[c]) != 0) continue;
        for (uint64_t p = 0; p < n_probes; ++p) {
            uint64_t len = orc_trace(&probes[p], tr, maxlen);
            orc_replay_general(&cands[c], tr, len, probes[p].base, probes[p].elem, p,
                               count_from[p], hit, NULL, NULL);
            const uint8_t *ob = obs_hits + obs_off[p];
            for (uint64_t k = count_from[p]; k < len; ++k) {
                m[c] += (hit[k] != ob[k]);
                n[c] += 1;
            }
        }
    }
    free(tr);
    free(hit);

    int64_t best = -1;
    for (uint64_t c = 0; c < n_cands; ++c) {
        if (n[c] == 0) continue;
        if (best < 0) {
            best = (int64_t)c;
            continue;
        }
        unsigned __int128 lhs = (unsigned __int128)m[c] * n[best];
        unsigned __int128 rhs = (unsigned __int128)m[best] * n[c];
        if (lhs < rhs) best = (int64_t)c;
    }
    return best;
}

int orc_in_own_sweep(const orc_model *c, const orc_probe *p)
{
    uint64_t C = c->capacity, b = c->line, N = p->n_bytes, s = p->s_bytes;
    if (2 * N < C || N > 2 * C) return 0;
    if (N % b != 0) return 0;
    return (2 * s == b) || (s == b) || (s == 2 * b);
}

int64_t orc_infer(const orc_model *cands, uint64_t n_cands,
                  const orc_probe *probes, uint64_t n_probes,
                  const uint8_t *obs_hits, const uint64_t *obs_off,
                  const uint64_t *count_from, int probe_select,
                  uint64_t *m, uint64_t *n)
{
    uint64_t maxlen = 0;
    for (uint64_t p = 0; p < n_probes; ++p) {
        uint64_t len = orc_trace_len(&probes[p]);
        if (len == 0) return -2;
        if (len > maxlen) maxlen = len;
    }
    int32_t *tr = (int32_t *)malloc((maxlen ? maxlen : 1) * sizeof(int32_t));
    uint8_t *hit = (uint8_t *)malloc(maxlen ? maxlen : 1);
    if (!tr || !hit) {
        free(tr);
        free(hit);
        return -3;
    }
    for (uint64_t c = 0; c < n_cands; ++c) {
        m[c] = 0;
        n[c] = 0;
        if (orc_model_check(&cands[c]) != 0) continue;
        for (uint64_t p = 0; p < n_probes; ++p) {
            if (probe_select == 1 && !orc_in_own_sweep(&cands[c], &probes[p])) continue;
            uint64_t len = orc_trace(&probes[p], tr, maxlen);
            orc_replay(&cands[c], tr, len, probes[p].base, probes[p].elem, p,
                       count_from[p], hit, NULL, NULL);
            const uint8_t *ob = obs_hits + obs_off[p];
            for (uint64_t k = count_from[p]; k < len; ++k) {
                m[c] += (hit[k] != ob[k]);
                n[c] += 1;
            }
        }
    }
    free(tr);
    free(hit);

    int64_t best = -1;
    for (uint64_t c = 0; c < n_cands; ++c) {
        if (n[c] == 0) continue;
        if (best < 0) {
            best = (int64_t)c;
            continue;
        }
        unsigned __int128 lhs = (unsigned __int128)m[c] * n[best];
        unsigned __int128 rhs = (unsigned __int128)m[best] * n[c];
        if (lhs < rhs) best = (int64_t)c;
    }
    return best;
}
