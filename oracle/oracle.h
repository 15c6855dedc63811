/*
 * oracle.h -- plain, single-threaded CPU reference of the fine-grained
 * P-chase cache-model replay (Mei & Chu, "Dissecting GPU Memory Hierarchy
 * through Microbenchmarking").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the HIP implementation; its types are
 * declared here on their own on purpose.
 *
 * Every function follows one passage of the paper:
 *   - trace generation:   Listing 1 (array initialisation) + Listing 2 (chase);
 *                         the non-uniform-stride chase of Section 5.2
 *   - replay:             Section 4.1, Assumptions 1-3 (set-associative model,
 *                         set bits directly above the offset bits, LRU) and
 *                         the non-LRU policies the paper observes
 *                         (Section 4.5 Fermi L1, Section 4.6 L2)
 *   - classification:     Section 4.1, average-latency model t = t0 + tm*r
 *   - inference:          Section 4.2, the two-stage procedure of Fig. 6,
 *                         done as an exhaustive exact search
 *   - Philox4x32-10:      Salmon, Moraes, Dror, Shaw, "Parallel random
 *                         numbers: as easy as 1, 2, 3", SC'11 (the RANDOM
 *                         policy's victim draw)
 */
#ifndef PCHASE_ORACLE_H
#define PCHASE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* replacement policies (Assumption 3 and its negation) */
enum { ORC_LRU = 0, ORC_FIFO = 1, ORC_PLRU = 2, ORC_RANDOM = 3 };

typedef struct orc_model {
    uint64_t capacity;  /* C, bytes */
    uint64_t line;      /* b, bytes, power of two */
    uint64_t ways;      /* a */
    uint64_t sets;      /* T; Assumption 1: T*a*b == C */
    uint64_t policy;    /* ORC_* */
    uint64_t set_shift; /* 0: set = line mod T; else set = (addr >> set_shift) mod T */
    uint64_t seed;      /* RANDOM policy key */
} orc_model;

typedef struct orc_probe {
    uint64_t n_bytes;   /* N */
    uint64_t s_bytes;   /* s */
    uint64_t base;      /* byte address of array element 0 */
    uint64_t j0;        /* start index */
    uint64_t elem;      /* bytes per array element */
    uint64_t passes;    /* number of full cycles through the chase */
} orc_probe;

/* Philox4x32-10 block: out = philox(ctr, key) */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Trace of one probe: number of accesses (passes * cycle length), 0 on error. */
uint64_t orc_trace_len(const orc_probe *p);
/* Cycle length L of one pass. 0 on error. */
uint64_t orc_cycle_len(const orc_probe *p);
/* Writes the accessed element indices j_0 .. j_{len-1}; returns len or 0. */
uint64_t orc_trace(const orc_probe *p, int32_t *out, uint64_t cap);

/* Non-uniform-stride probe (Section 5.2, Fig. 13(b)): segment i has
 * counts[i] >= 1 accesses, each left by a step of s_bytes[i]; a pass walks
 * the segments in order from j0 and every pass starts again at j0. */
typedef struct orc_nu_probe {
    uint64_t n_bytes;
    uint64_t base;
    uint64_t j0;
    uint64_t elem;
    uint64_t passes;
    uint64_t n_segments;
} orc_nu_probe;

/* passes * (sum of counts), 0 on error. */
uint64_t orc_trace_nu_len(const orc_nu_probe *p, const uint64_t *counts);
/* Writes the visited element indices; returns the length or 0. */
uint64_t orc_trace_nu(const orc_nu_probe *p, const uint64_t *s_bytes, const uint64_t *counts,
                      int32_t *out, uint64_t cap);

/* 0 if the model is valid, negative otherwise. */
int orc_model_check(const orc_model *m);

/*
 * Replay one trace (element indices, byte address = base + elem*idx) through
 * one cold model.  hits (nullable) receives one byte per access (1 = hit).
 * Returns 0 or a negative error.
 */
int orc_replay(const orc_model *m, const int32_t *idx, uint64_t len,
               uint64_t base, uint64_t elem, uint64_t trace_id,
               uint64_t count_from, uint8_t *hits,
               uint64_t *misses_total, uint64_t *misses_steady);

/*
 * Generalised cache (the organisations the paper finds that break
 * Assumptions 1-2 or 3): per-set associativity (the L2 TLB of Sec. 4.4 and
 * Fig. 9: one set of 17 entries and six of 8), a table from the set unit to
 * the set (the texture-L1 and read-only-cache mappings of Sec. 4.3), and
 * weighted random replacement (the Fermi L1 of Sec. 4.5: way 2 replaced
 * with probability 1/2, the others 1/6).
 *   unit = set_shift ? addr >> set_shift : addr / line
 *   set  = table_len ? table[unit mod table_len] : unit mod sets
 * Set t has ways[t] ways.  ORC_WRANDOM draws u = Philox4x32-10(key = seed,
 * counter = (k_lo, k_hi, trace_lo, trace_hi)).x for access k and evicts the
 * lowest way w with (u mod S) < weights[0] + ... + weights[w], S being the
 * sum of the set's first ways[t] weights.
 */
enum { ORC_WRANDOM = 4 };

typedef struct orc_general {
    uint64_t line;            /* b, bytes, power of two */
    uint64_t sets;            /* T */
    const uint64_t *ways;     /* [T], each >= 1 */
    uint64_t policy;          /* ORC_LRU .. ORC_WRANDOM */
    uint64_t set_shift;
    uint64_t table_len;
    const uint64_t *table;    /* [table_len], entries < T */
    const uint64_t *weights;  /* ORC_WRANDOM: one per way of the widest set */
    uint64_t seed;
} orc_general;

/* 0 if valid, negative otherwise. */
int orc_general_check(const orc_general *g);
/* As orc_replay, for a generalised cache. */
int orc_replay_general(const orc_general *g, const int32_t *idx, uint64_t len,
                       uint64_t base, uint64_t elem, uint64_t trace_id,
                       uint64_t count_from, uint8_t *hits,
                       uint64_t *misses_total, uint64_t *misses_steady);

/* Latency -> hit bit: hit iff lat <= theta. */
void orc_classify(const uint32_t *lat, uint64_t n, uint32_t theta, uint8_t *hits);
/* Largest-gap threshold over the distinct latency values. */
uint32_t orc_auto_threshold(const uint32_t *lat, uint64_t n);

/*
 * Exhaustive inference.  obs_hits holds the observed hit bytes of every
 * probe back to back (probe p starts at obs_off[p]; its length is the
 * probe's trace length).  count_from[p] = first access compared.
 * probe_select: 0 = every probe for every candidate, 1 = each candidate's
 * own sweep (C/2 <= N <= 2C, N % b == 0, s in {b/2, b, 2b}).
 * Writes m[c], n[c]; returns the best index (exact rational argmin of m/n,
 * lowest index on ties, candidates with n == 0 skipped) or -1.
 */
int64_t orc_infer(const orc_model *cands, uint64_t n_cands,
                  const orc_probe *probes, uint64_t n_probes,
                  const uint8_t *obs_hits, const uint64_t *obs_off,
                  const uint64_t *count_from, int probe_select,
                  uint64_t *m, uint64_t *n);

/*
 * Exhaustive inference over generalised candidates (Sections 4.3-4.5):
 * every candidate replays every probe; otherwise as orc_infer.  Invalid
 * candidates get n = 0 and are skipped.
 */
int64_t orc_infer_general(const orc_general *cands, uint64_t n_cands,
                          const orc_probe *probes, uint64_t n_probes,
                          const uint8_t *obs_hits, const uint64_t *obs_off,
                          const uint64_t *count_from, uint64_t *m, uint64_t *n);

/* 1 if probe p belongs to candidate c's own sweep. */
int orc_in_own_sweep(const orc_model *c, const orc_probe *p);

#ifdef __cplusplus
}
#endif
#endif
