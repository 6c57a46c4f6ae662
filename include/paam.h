/*
 * libpaam -- batched worst-case response-time analysis of ROS 2 processing
 * chains served by a priority-driven accelerator manager, on AMD gfx950.
 *
 * The analysis is the admission test of the paper's Sec. IV-F: Eq. (1)
 * (H* = H + delta*epsilon), Lemma 1 / Eq. (2) (arrival bound
 * mu(t) = ceil(t/T) + 1), Lemma 2 / Eq. (3) (per-segment handling time),
 * Lemma 3 / Eq. (4) (per-chain handling time), their minimum, Theorem 1 /
 * Eq. (6) (chain response time; Lemma 4 / Eq. (5) when a chain has no
 * segment) and the end-to-end sum over sub-chains that closes the section.
 * The problem statement follows Sec. II-C (callback and chain tuples,
 * executors, priorities) and Sec. IV-C (buckets).
 *
 * Conventions
 *  - Times are int64 nanoseconds.  PAAM_INF (INT64_MAX) marks a bound whose
 *    recurrence exceeded its cap (cap_mult * D of the chain).
 *  - Every device buffer is owned by the caller; the library never allocates
 *    device memory.  *_bytes() report the sizes to provide.
 *  - Calls that take a stream are asynchronous on it; outputs are valid after
 *    the stream synchronises.  The stream argument is a hipStream_t (NULL is
 *    the default stream).
 *  - A missed deadline is a result, never an error.
 *  - On failure a call returns a negative paam_status and
 *    paam_last_error() (thread-local) describes it.
 */
#ifndef PAAM_H
#define PAAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t paam_status;
#define PAAM_OK 0
#define PAAM_E_INVAL (-1) /* malformed input: null pointer, bad offsets/indices, D > T, ... */
#define PAAM_E_RANGE (-2) /* a value outside the exactly representable range (times >= 2^36) */
#define PAAM_E_NOMEM (-3) /* a caller buffer is smaller than its *_bytes() size */
#define PAAM_E_HIP (-4)   /* a HIP runtime call failed; the message names it */
#define PAAM_E_STATE (-5) /* no usable gfx950 device, or a handle in the wrong state */

#define PAAM_INF INT64_MAX

typedef void *paam_stream; /* a hipStream_t */

/* Host CSR description of n_sets independent chain sets (Sec. II-C).
 * Offsets are global and non-decreasing; per-set indices are set-local. */
typedef struct {
  int64_t n_sets;
  const int64_t *set_chain_off; /* [n_sets+1] chains of a set */
  const int64_t *set_exec_off;  /* [n_sets+1] executors of a set */
  const int64_t *set_accel_off; /* [n_sets+1] accelerators of a set */
  const int64_t *chain_cb_off;  /* [n_chains+1] callbacks of a chain, in precedence order */
  const int64_t *cb_seg_off;    /* [n_callbacks+1] accelerator segments of a callback (eta_i) */
  const int64_t *T;             /* [n_chains] period T_c > 0 */
  const int64_t *D;             /* [n_chains] constrained deadline, 0 < D_c <= T_c */
  const int32_t *prio;          /* [n_chains] chain priority, unique in a set, larger = higher */
  const uint8_t *spin;          /* [n_chains] 1: busy-waits during its requests; 0: suspends */
  const int64_t *E;             /* [n_callbacks] CPU WCET E_i */
  const int16_t *exec;          /* [n_callbacks] set-local executor of the callback */
  const int64_t *A;             /* [n_segments] accelerator segment WCET A_ij */
  const int16_t *accel;         /* [n_segments] set-local accelerator of the segment (r_ij) */
  const int16_t *exec_core;     /* [n_executors] CPU core of the executor */
  const int32_t *exec_prio;     /* [n_executors] OS process priority, unique per core */
  const int16_t *accel_buckets; /* [n_accels] number of buckets n >= 1 (Sec. IV-C) */
  const int64_t *accel_eps;     /* [n_accels] per-request server overhead epsilon */
  const int64_t *accel_kappa;   /* [n_accels] device preemption cost kappa */
  const int64_t *eps_hop;       /* [n_sets] communication cost between consecutive sub-chains */
  /* Several units of one accelerator type (Sec. IV-E, "Managing Multiple
   * Accelerators"): NULL, or [n_accels] units of each accelerator (1..8,
   * at most 8 units per set in all).  Then accel[] names a type, and every
   * segment is bound to one unit of its type at upload by worst-fit
   * decreasing (paam_assign_units); each unit is analysed as an accelerator
   * of its own with its type's buckets, epsilon and kappa. */
  const int16_t *accel_units;
  int32_t unit_group;           /* PAAM_UNITS_*: what the bin packing places as one item */
} paam_chainset_host;

#define PAAM_UNITS_SEGMENT 0  /* each accelerator segment on its own */
#define PAAM_UNITS_CALLBACK 1 /* a callback's segments on one type stay together */
#define PAAM_UNITS_CHAIN 2    /* a chain's segments on one type stay together */

typedef struct paam_chainset paam_chainset; /* opaque host handle of an uploaded batch */

/* Size of the device arena paam_chainset_upload needs for this batch. */
paam_status paam_chainset_bytes(const paam_chainset_host *h, size_t *arena_bytes);

/* Validates the batch, derives its priority-independent structure
 * (sub-chains = maximal runs of consecutive callbacks on one executor,
 * executors of the same core with higher process priority, reciprocals of the
 * periods, a longest-first work order) and copies it into the caller's device arena (>= arena_bytes, 256-B
 * aligned).  Blocks until the copy is done.  *out must be released with
 * paam_chainset_free; the arena must outlive it.  Limits per set: 1..4096
 * chains, 1..32 executors, 0..8 accelerators, 65535 sub-chains; every time
 * below 2^36 ns; and the analysis keeps per-set tables of
 * 8*(4C + 2*NA*C + 2*X*C + 2*NA) + 4*(2C + NA*C + 10X + 16) bytes in the
 * 160 KB of LDS of a compute unit (plus 8*X*C when X*C <= 512), so for
 * example at most 869 chains with 8 executors and one accelerator, or 2,154
 * chains with one executor (C chains, X executors, NA accelerators; with
 * accel_units, NA counts units).  With accel_units a set holds at most 2048
 * segments.  PAAM_E_RANGE otherwise, at upload (and from
 * paam_chainset_bytes). */
paam_status paam_chainset_upload(const paam_chainset_host *h, void *d_arena, size_t arena_bytes,
                                 paam_stream stream, paam_chainset **out);
void paam_chainset_free(paam_chainset *cs);

/* Binds every segment of a batch uploaded with accel_units to one unit of its
 * accelerator type (Sec. IV-E: at registration, by a bin-packing heuristic
 * such as worst-fit decreasing), on the device, in place; upload runs it
 * once, and it may run again (the result is the same).  Items: one segment,
 * or the segments of one callback or one chain on one type (unit_group).
 * Size of an item: its utilisation sum(A)/T in fixed point,
 * floor(min(sum(A), 2^36) * 2^26 / T) clamped at 2^36.  Items are placed
 * largest first (ties: higher chain priority, then lower first segment
 * index), each on the unit of its type with the least load so far (ties: the
 * lowest unit); a unit's load is the sum of its items' sizes.  The units of a
 * set are numbered type by type (the units of type 0 first).  Asynchronous
 * on the stream; PAAM_E_STATE if the batch has no accel_units. */
paam_status paam_assign_units(paam_chainset *cs, paam_stream stream);

/* Copies the analysed accelerator (set-local unit) of every segment,
 * [n_segments] int16, into a caller device buffer.  Without accel_units it
 * is the input accel[].  Asynchronous on the stream. */
paam_status paam_chainset_seg_units(const paam_chainset *cs, int16_t *d_unit, paam_stream stream);

/* Counts of an uploaded batch: n_sets, n_chains, n_callbacks, n_segments,
 * n_subchains, and the per-set maxima of chains, sub-chains, segments. */
paam_status paam_chainset_info(const paam_chainset *cs, int64_t info[8]);

#define PAAM_BLOCK_SAFE 0  /* blocking by an LP callback includes its accelerator handling */
#define PAAM_BLOCK_PAPER 1 /* blocking = max E_j of LP callbacks, as printed in Eq. (5)/(6) */
#define PAAM_BOUND_MIN 0   /* H = min(Lemma 2 summed over segments, Lemma 3) */
#define PAAM_BOUND_L2 1    /* Lemma 2 only */
#define PAAM_BOUND_L3 2    /* Lemma 3 only */

typedef struct {
  int32_t blocking;      /* PAAM_BLOCK_* */
  int32_t cap_mult;      /* >= 1: an iterate above cap_mult * D of its chain makes it PAAM_INF */
  int32_t util_permille; /* >= 0: every E and A enters as floor(x * util_permille / 1000) */
  int32_t full;          /* 1: every chain's bound; 0: verdict only, stop a set at its first miss */
  int32_t bound;         /* PAAM_BOUND_* */
  int32_t waves_per_cu;  /* persistent waves per compute unit; 0 = per size class, the
                            choice of paam_wcrt_autotune if it ran on the handle, else 8 */
} paam_wcrt_opts;

/* Workspace for paam_wcrt_batch (device, caller-owned, 256-B aligned). */
paam_status paam_wcrt_bytes(const paam_chainset *cs, const paam_wcrt_opts *o, size_t *ws_bytes);

/* Analyses every set of the batch (Sec. IV-F, Theorem 1 and the end-to-end
 * sum).  Outputs, all device pointers:
 *   set_sched [n_sets]   1 if every chain meets its deadline
 *   set_worst [n_sets]   set-local chain with the largest R/D (ties: lowest
 *                        index); -1 for an unschedulable set when !full
 *   set_worst_R [n_sets] that chain's bound; PAAM_INF when set_worst is -1
 *   chain_R [n_chains]   end-to-end bound of every chain (PAAM_INF past its
 *                        cap); required when full, ignored (may be NULL) if not */
paam_status paam_wcrt_batch(const paam_chainset *cs, const paam_wcrt_opts *o, int8_t *set_sched,
                            int32_t *set_worst, int64_t *set_worst_R, int64_t *chain_R, void *d_ws,
                            size_t ws_bytes, paam_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * analysis as paam_wcrt_batch, with the same outputs, but with no workspace
 * argument.  Its scratch is a static device array of 64 MiB per GPU, held
 * until the process ends; the call allocates nothing.  The number of
 * persistent waves is limited to what that scratch holds (results do not
 * depend on it).  PAAM_E_RANGE if one wave of some size class of the batch
 * needs more scratch than the array holds.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller. */
paam_status paam_wcrt_batch_noalloc(const paam_chainset *cs, const paam_wcrt_opts *o,
                                    int8_t *set_sched, int32_t *set_worst, int64_t *set_worst_R,
                                    int64_t *chain_R, paam_stream stream);

/* Schedule autotuner.  For each size class of the batch (sets grouped by
 * chain count: up to 16, 32, 64, ... chains; the analysis launches once per
 * class), times the class's launch with every pair of persistent waves per
 * compute unit from cand (n_cand values in 1..32) and evaluations of each
 * lane's recurrence per engine step (1, 2, 3): one untimed launch, then reps
 * timed ones with HIP events on the stream.  The fastest pair of each class
 * is stored in the handle (the only change a call makes to a handle: do not
 * run it concurrently with other calls on the same handle); o->waves_per_cu
 * is set to 0, which makes later calls use the stored per-class choices, and
 * *best_ms receives the sum of the classes' best times (one batch launch).
 * Outputs as for paam_wcrt_batch (overwritten); the workspace must hold
 * paam_wcrt_bytes for waves_per_cu = the largest candidate.  Query the
 * workspace size again after tuning.  Blocks until the timing has finished. */
paam_status paam_wcrt_autotune(paam_chainset *cs, paam_wcrt_opts *o, const int32_t *cand,
                               int32_t n_cand, int32_t reps, int8_t *set_sched,
                               int32_t *set_worst, int64_t *set_worst_R, int64_t *chain_R,
                               void *d_ws, size_t ws_bytes, paam_stream stream, float *best_ms);

/* The schedule of the batch's size classes: for class k < cap,
 * classes[4k .. 4k+3] = largest chain count, number of sets, waves per CU and
 * evaluations per engine step used when o->waves_per_cu is 0 (the
 * autotuner's choice, else 8 and 2).  *n_classes receives the class count. */
paam_status paam_wcrt_schedule(const paam_chainset *cs, int32_t *classes, int32_t cap,
                               int32_t *n_classes);

/* ---------------- priority-order search (candidate orders) ----------------
 * Candidate 0 of a set is its uploaded order (chains by decreasing prio).
 * Candidate k >= 1 is candidate k-1 with two positions swapped: with u1, u2
 * the outputs 2k-2 and 2k-1 of the SplitMix64 stream of the set (state
 * starting at mix(seed + G*(set+1)), advancing by G = 0x9E3779B97F4A7C15 per
 * output, mix = the SplitMix64 output function), positions i = u1 mod C and
 * j = (i + 1 + u2 mod (C-1)) mod C swap.  A candidate is feasible when the
 * analysis (verdict mode) finds every chain within its deadline, i.e. the
 * admission test of Sec. IV-F accepts the set under that priority
 * assignment (Sec. II-C: static, unique chain priorities). */
typedef struct {
  int32_t n_cand;        /* candidate orders per set, 1..65536 */
  int32_t guided;        /* 0: plain search in index order; 1: lowest score first */
  int32_t top_k;         /* guided: candidates analysed in score order, 1..n_cand */
  int32_t fallback;      /* guided: 1 = plain search over the rest when none of the top_k is feasible */
  uint64_t seed;         /* seed of the swap walk */
  const float *d_scores; /* guided: [n_sets*n_cand] device scores (predicted max R/D); else NULL */
  paam_wcrt_opts wcrt;   /* analysis options; full is ignored (verdict mode) */
} paam_search_opts;

/* Workspace for paam_priority_search (device, caller-owned, 256-B aligned). */
paam_status paam_search_bytes(const paam_chainset *cs, const paam_search_opts *o, size_t *ws_bytes);

/* Searches every set for a feasible candidate order.  Outputs (device):
 *   found [n_sets]      plain: the smallest feasible k; guided: the first
 *                       feasible candidate in score order among the top_k
 *                       (ties: lower k), then, with fallback, the smallest
 *                       feasible k among the others; -1 if none; -2 if the
 *                       analysis hit its iteration guard
 *   n_exact [n_sets]    exact analyses run for the set
 *   found_prio [n_chains] (may be NULL) the found order as priorities
 *                       (C - position, larger = higher); untouched for sets
 *                       with found < 0 */
paam_status paam_priority_search(const paam_chainset *cs, const paam_search_opts *o,
                                 int32_t *found, int32_t *n_exact, int32_t *found_prio, void *d_ws,
                                 size_t ws_bytes, paam_stream stream);

/* ---------------- candidate-ranking surrogate ----------------------------
 * A learned ranking of candidate orders sits on top of the analysis: the exact
 * analysis above stays the sole judge of schedulability; the network only
 * decides which candidates reach it first.  None of it is part of the paper's
 * method.  A "pair" names one candidate order of one set and the utilisation
 * scale to analyse it at: int64 triples (set, k, util_permille), k as in the
 * search above (0 = uploaded order, k >= 1 = k swaps along the set's walk,
 * with the seed given to the call). */
#define PAAM_FEATURES 48      /* features per chain */
#define PAAM_MLP_HIDDEN 256   /* hidden units of both hidden layers */
#define PAAM_MLP_PARAMS 78593 /* float32 master parameters */
#define PAAM_MLP_PACKED 82176 /* bfloat16 packed weights (uint16 values) */

/* Workspace for paam_candidate_wcrt on n_pairs pairs. */
paam_status paam_candidate_bytes(const paam_chainset *cs, const paam_wcrt_opts *o, int64_t n_pairs,
                                 size_t *ws_bytes);

/* Exact analysis of explicit candidate orders (Sec. IV-F, every chain's bound
 * at cap o->cap_mult * D; o->full and o->util_permille are ignored: each pair
 * carries its own scale).  Outputs per pair (device):
 *   sched [n]    1 if every chain meets its deadline, 0 if not, -1 on the guard
 *   worst_R [n]  bound of the chain with the largest R/D (ties: lowest index),
 *                PAAM_INF past its cap
 *   worst_D [n]  that chain's deadline
 *   ratio [n]    min(worst_R / worst_D, cap_mult) as float (cap_mult when INF);
 *                the training target of the ranking network
 * Pairs must name existing sets, 0 <= k < 2^31 and util_permille >= 0
 * (checked on the device; a bad pair yields sched = -2). */
paam_status paam_candidate_wcrt(const paam_chainset *cs, const paam_wcrt_opts *o, uint64_t seed,
                                const int64_t *d_pairs, int64_t n_pairs, int8_t *sched,
                                int64_t *worst_R, int64_t *worst_D, float *ratio, void *d_ws,
                                size_t ws_bytes, paam_stream stream);

/* Workspace for paam_features. */
paam_status paam_features_bytes(const paam_chainset *cs, int64_t n_pairs, size_t *ws_bytes);

/* Per-chain features of candidate orders, 48 per chain (bfloat16 bit
 * patterns).  Pair i owns rows [i*row_stride, i*row_stride + C_i) of feat
 * ([n_pairs*row_stride][48], row_stride >= the largest set of the batch);
 * count[i] = C_i.  Rows past C_i are left untouched.  Every feature is a ratio
 * of exact integers rounded once to double, then to float and to bfloat16
 * (round to nearest even); utilisation terms are floor(x * 2^16 / T).
 * PAAM_E_RANGE if a set's total demand reaches 2^40 ns at the largest scale. */
paam_status paam_features(const paam_chainset *cs, uint64_t seed, const int64_t *d_pairs,
                          int64_t n_pairs, int32_t row_stride, uint16_t *feat, int32_t *count,
                          void *d_ws, size_t ws_bytes, paam_stream stream);

/* The network: per chain row x (48), z1 = W1 x + b1, h1 = max(z1, 0); per
 * candidate p = mean of h1 over its rows, z2 = W2 p + b2, h2 = max(z2, 0),
 * y = w3 . h2 + b3 (the predicted largest R/D).  float32 master parameters,
 * layout W1 [256][48] | b1 [256] | W2 [256][256] | b2 [256] | w3 [256] | b3.
 * Products take bfloat16 operands (x, W1, W2, w3, p, h2, each rounded to
 * nearest even) and accumulate in float32, W1 x and W2 p on the matrix cores.
 * Packed weights (uint16 bfloat16 patterns): W1 [256][64] (columns 48..63
 * zero) | W2 [256][256] | w3 [256]. */
paam_status paam_mlp_pack(const float *d_params, uint16_t *d_packed, paam_stream stream);

/* Forward over n candidates whose features paam_features wrote (row_stride,
 * count as there).  out [n] = y.  act (may be NULL) receives what the
 * backward pass needs: n * 1024 bytes (p and h2 as bfloat16). */
paam_status paam_mlp_forward(const float *d_params, const uint16_t *d_packed,
                             const uint16_t *feat, const int32_t *count, int64_t n,
                             int32_t row_stride, float *out, void *act, paam_stream stream);

/* Workspace for paam_mlp_backward. */
paam_status paam_mlp_backward_bytes(int64_t n, size_t *ws_bytes);

/* Gradient of the mean squared error (1/n) sum (y - target)^2 with respect to
 * the master parameters (straight through the bfloat16 roundings), float32,
 * reduced in a fixed order (deterministic).  grad [78593]; loss [1]. */
paam_status paam_mlp_backward(const float *d_params, const uint16_t *d_packed,
                              const uint16_t *feat, const int32_t *count, int64_t n,
                              int32_t row_stride, const float *out, const float *target,
                              const void *act, float *grad, float *loss, void *d_ws,
                              size_t ws_bytes, paam_stream stream);

/* One Adam step (Kingma & Ba 2015, with bias correction; step counts from 1)
 * on the float32 master parameters and moments, then repacks the bfloat16
 * weights. */
paam_status paam_mlp_adam_step(float *d_params, uint16_t *d_packed, float *d_m, float *d_v,
                               const float *grad, float lr, float beta1, float beta2, float eps,
                               int64_t step, paam_stream stream);

/* Workspace for paam_score_candidates. */
paam_status paam_score_bytes(const paam_chainset *cs, const paam_search_opts *o, size_t *ws_bytes);

/* Scores every candidate of every set with the network: scores
 * [n_sets * n_cand] (set-major), the input of a guided search with the same
 * options.  Features and forward run in chunks inside the workspace. */
paam_status paam_score_candidates(const paam_chainset *cs, const paam_search_opts *o,
                                  const float *d_params, const uint16_t *d_packed, float *scores,
                                  void *d_ws, size_t ws_bytes, paam_stream stream);

/* Thread-local description of the last failure ("" if none). */
/* ---- Simulation (Sec. V-A: observed latencies against the bound) -------
 * An event-driven simulation of every set under the model the analysis
 * bounds (Sec. II-C, IV-C, IV-D, IV-F): chain c releases a job every T_c
 * from its offset; a job runs the chain's callbacks in order, the next one
 * ready on its executor when the previous completes (after eps_hop when the
 * executor changes); an idle executor starts its ready callback of the
 * highest chain priority (then the earliest release) and keeps it to the
 * end, also while its requests are served; a callback is a CPU piece, then
 * per segment epsilon of CPU time, the request (A + 2 kappa on the device)
 * and a CPU piece (E split equally, the first E mod (eta+1) pieces one
 * longer); a core runs its demanding executor of the highest process
 * priority (an executor demands while it has CPU work, or while its request
 * is served if its chain busy-waits); an accelerator serves its highest
 * bucket level holding a request, one request at a time per level, highest
 * chain priority first, then submission order, and a higher level preempts.
 * Within an instant: releases, hop arrivals, executors by index, then
 * accelerators by index, repeated until nothing changes; time then jumps to
 * the next event.  A chain keeps at most two live jobs.
 * Actual times: with exec_permille = 1000 every job runs its WCETs (after
 * util_permille scaling); else each callback job's E and each segment's A
 * is W - (r mod (W - floor(W * exec_permille / 1000) + 1)), r from
 * SplitMix64 keyed by (seed, set, scenario, chain, job, callback, item).
 * Limits: 32 chains, 16 executors, 8 segments per callback, 8 buckets per
 * accelerator, and 12 bytes per callback plus 9 per segment of a set within
 * 48 KB (its tables are staged in LDS) -- PAAM_E_RANGE otherwise. */
typedef struct {
  int32_t n_scen;        /* scenarios per set, 1..2^20 */
  int32_t exec_permille; /* 0..1000 */
  int64_t horizon;       /* releases and completions in [0, horizon] ns, horizon < 2^40 */
  uint64_t seed;
  int32_t util_permille; /* 0..10^6: E and A enter as floor(x * util_permille / 1000) */
  int32_t reserved;      /* 0 */
  int64_t max_steps;     /* >= 1: time advances per scenario before it stops with status 2 */
} paam_des_opts;

/* d_offsets, d_obs: device int64, per set a [n_scen][C] block starting at
 * element set_chain_off[set] * n_scen (n_chains * n_scen in all): the first
 * release of every chain (>= 0) in; its largest observed end-to-end response
 * (completion minus release over the jobs completed by the horizon; -1: none)
 * out.  d_status [n_sets * n_scen] int8: 0 done, 1 a release found two live
 * jobs of its chain (the scenario stops there), 2 max_steps reached.
 * Asynchronous on the stream; no workspace. */
paam_status paam_des_batch(const paam_chainset *cs, const paam_des_opts *o,
                           const int64_t *d_offsets, int64_t *d_obs, int8_t *d_status,
                           paam_stream stream);

const char *paam_last_error(void);

/* Library version string. */
const char *paam_version(void);

#ifdef __cplusplus
}
#endif
#endif
