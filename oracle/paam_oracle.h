/*
 * CPU oracle of the PAAM worst-case response-time analysis.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, plain reference that the
 * GPU path is checked against.  Nothing on the product path may include,
 * link or call it; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.
 *
 * It follows Sec. IV-F of the paper (Admission Control): Eq. (1) (H*),
 * Lemma 1 / Eq. (2) (arrival bound mu), Lemma 2 / Eq. (3) (per-segment
 * handling time), Lemma 3 / Eq. (4) (per-chain handling time), the double
 * bound min(Eq. 3, Eq. 4), Lemma 4 / Eq. (5) (PiCAS) and Theorem 1 / Eq. (6),
 * plus the end-to-end sum over sub-chains that closes Sec. IV-F.  All times
 * are int64 nanoseconds; ORACLE_INF saturates every sum and product.
 */
#ifndef PAAM_ORACLE_H
#define PAAM_ORACLE_H
#include <stdint.h>

#define ORACLE_INF INT64_MAX

typedef struct {
  int64_t n_sets;
  const int64_t *set_chain_off, *set_exec_off, *set_accel_off; /* [n_sets+1] */
  const int64_t *chain_cb_off;  /* [n_chains+1] callbacks of a chain, in precedence order */
  const int64_t *cb_seg_off;    /* [n_callbacks+1] accelerator segments of a callback */
  const int64_t *T, *D;         /* [n_chains] period, constrained deadline */
  const int32_t *prio;          /* [n_chains] unique within a set, larger = higher */
  const uint8_t *spin;          /* [n_chains] 1 = busy-waits on accelerator requests */
  const int64_t *E;             /* [n_callbacks] CPU WCET */
  const int16_t *exec;          /* [n_callbacks] set-local executor */
  const int64_t *A;             /* [n_segments] accelerator segment WCET */
  const int16_t *accel;         /* [n_segments] set-local accelerator */
  const int16_t *exec_core;     /* [n_executors] */
  const int32_t *exec_prio;     /* [n_executors] OS process priority, larger = higher */
  const int16_t *accel_buckets; /* [n_accels] number of buckets n */
  const int64_t *accel_eps;     /* [n_accels] per-request server overhead epsilon */
  const int64_t *accel_kappa;   /* [n_accels] device preemption cost kappa */
  const int64_t *eps_hop;       /* [n_sets] communication cost between sub-chains */
} oracle_chainsets;

typedef struct {
  int32_t blocking;       /* 0: LP callback's accelerator handling counts as blocking; 1: E_j only */
  int32_t cap_mult;       /* an iterate above cap_mult * D of its chain is INF */
  int32_t util_permille;  /* E and A enter as floor(x * util_permille / 1000) */
  int32_t full;           /* 1: bound every chain; 0: stop at the first missed deadline */
  int32_t bound;          /* 0: min(Lemma 2, Lemma 3); 1: Lemma 2 only; 2: Lemma 3 only */
} oracle_opts;

/* Per-set outputs.  chain_R[c] is the end-to-end bound of set-local chain c
 * (ORACLE_INF past its cap).  When !full and the set misses a deadline the
 * chains not yet analysed hold -1.  *worst is the chain with the largest
 * R/D (ties: lowest index), reported when the set is schedulable or when
 * full; else -1 with *worst_R = ORACLE_INF.  *terms counts every mu*weight
 * product evaluated.  order: chain ids from highest to lowest priority, or
 * NULL to use the prio array.  Returns 0, or -1 on invalid input. */
int oracle_analyse_set(const oracle_chainsets *cs, int64_t set, const int32_t *order,
                       const oracle_opts *opt, int64_t *chain_R, int8_t *sched, int32_t *worst,
                       int64_t *worst_R, int64_t *terms);

/* Lemma 2 bound of every segment of a set (set-local order), for tests. */
int oracle_segment_H(const oracle_chainsets *cs, int64_t set, const int32_t *order,
                     const oracle_opts *opt, int64_t *seg_H);

/* Sets [lo, hi): chain_R indexed by global chain id, the rest by set id. */
int oracle_wcrt_range(const oracle_chainsets *cs, const oracle_opts *opt, int64_t lo, int64_t hi,
                      int64_t *chain_R, int8_t *sched, int32_t *worst, int64_t *worst_R,
                      int64_t *terms);

/* Candidate priority order k of a set: k = 0 is the input order; k >= 1 is
 * order k-1 with two positions swapped, drawn from SplitMix64. */
int oracle_candidate_order(const oracle_chainsets *cs, int64_t set, uint64_t seed, int64_t k,
                           int32_t *order);

/* Plain search over candidates 0..n_cand-1 of sets [lo, hi): found[s] is the
 * smallest k whose order meets every deadline, -1 if none; n_eval[s] counts
 * the analyses run (the search stops at the first feasible k). */
int oracle_search_range(const oracle_chainsets *cs, const oracle_opts *opt, int32_t n_cand,
                        uint64_t seed, int64_t lo, int64_t hi, int32_t *found, int32_t *n_eval,
                        int64_t *terms);

/* Worst-fit-decreasing binding of the accelerator segments of sets [lo, hi)
 * to units (Sec. IV-E, Managing Multiple Accelerators).  units[a] >= 1 is
 * the unit count of accelerator type a (global type index); the units of a
 * set are numbered type by type.  An item is one segment (group 0), or the
 * segments of one callback (1) or one chain (2) on one type.  Item size
 * floor(min(sum A, 2^36) * 2^26 / T) clamped at 2^36; largest first (ties:
 * higher chain priority, then earlier first segment); each to the
 * least-loaded unit of its type (ties: lowest unit).  unit[g] receives the
 * set-local unit of every segment g.  Returns 0, or -1 on bad input. */
int oracle_wfd_range(const oracle_chainsets *cs, const int16_t *units, int32_t group, int64_t lo,
                     int64_t hi, int16_t *unit);

/* Event-driven simulation of sets [lo, hi) (paam_des.c): n_scen scenarios
 * per set, releases in [0, horizon].  offsets and obs are laid out per set
 * as [n_scen][C] blocks starting at set_chain_off[set] * n_scen: the first
 * release of every chain in, and its largest observed end-to-end response
 * (-1: no job completed) out.  status[set * n_scen + s]: 0 done, 1 a chain
 * needed a third live job, 2 more than max_steps time advances. */
typedef struct {
  int32_t n_scen;
  int64_t horizon;
  int32_t exec_permille;  /* 1000: WCETs; else actual times drawn from [floor(W*p/1000), W] */
  uint64_t seed;
  int32_t util_permille;  /* E and A enter as floor(x * util_permille / 1000) */
  int64_t max_steps;
} oracle_des_opts;

int oracle_des_range(const oracle_chainsets *cs, const oracle_des_opts *o, const int64_t *offsets,
                     int64_t lo, int64_t hi, int64_t *obs, int8_t *status);

#endif
