// Internal device layout of an uploaded batch (libpaam only).
//
// Everything that does not depend on priorities or on the utilisation scale
// is derived once on the host at upload: sub-chains (maximal runs of
// consecutive callbacks of a chain on one executor, the sub-chains of the
// end-to-end sum in Sec. IV-F), the solving order of executors on each core,
// the reciprocals of the periods, and a longest-first work order.  The
// kernels derive the rest (A*, buckets, blocking, Lemma 2/3, Theorem 1) per
// launch, because it changes with the utilisation level and the candidate
// priority order.
#pragma once
#include <stdint.h>

#include "paam.h"

namespace paam {

struct double2_t {
  double x, y;
};

constexpr int kWave = 64;
constexpr int kMaxExec = 32;     // executors per set (hpp masks are 32-bit)
constexpr int kMaxAccel = 8;     // accelerators per set (accelerator masks are 8-bit)
constexpr int kMaxChains = 4096; // chains per set
constexpr int kMaxRuns = 65535;  // sub-chains per set
constexpr int64_t kTimeLimit = int64_t(1) << 36;  // every input time is below 2^36 ns

// Pointers into the caller's device arena.  Offsets are global (int64);
// indices stored per chain, callback, segment or sub-chain are set-local.
struct DevBatch {
  int64_t n_sets, n_chains, n_cbs, n_segs, n_runs;
  // sets
  const int64_t *set_chain_off, *set_cb_off, *set_seg_off, *set_run_off, *set_exec_off,
      *set_accel_off;          // [n_sets+1]
  const int64_t *eps_hop;      // [n_sets]
  const int64_t *work_order;   // [n_sets] sets by decreasing estimated cost
  // chains
  const int64_t *T, *D;        // [n_chains]
  const double *Kd;            // [n_chains] 2T - 1
  const double *rcp;           // [n_chains] 1/T rounded towards +inf
  const double *KRr;           // [2 n_chains] per set, by rank under the uploaded priorities:
                               // (2T - 1, 1/T rounded up) of the chain at that rank
  const int16_t *rank0;        // [n_chains] rank under the uploaded priorities, 0 = highest
  const int32_t *chain_nrun;   // [n_chains] sub-chains of the chain
  const uint8_t *spin;         // [n_chains]
  // callbacks
  const int64_t *E;            // [n_cbs]
  const int64_t *cb_seg_off;   // [n_cbs+1] global segment offsets
  const int8_t *cb_exec;       // [n_cbs] set-local executor of the callback
  const int32_t *chain_cb_lo;  // [n_chains] set-local first callback of the chain
  // segments
  const int64_t *A;            // [n_segs]
  const int16_t *seg_accel;    // [n_segs]
  const int16_t *seg_chain;    // [n_segs]
  const int32_t *seg_order;    // [n_segs] per set: set-local segment ids by rank of their chain
  // sub-chains per set, ordered by (executor has hpp executors above it,
  // rank of the chain under the uploaded priorities, position in the chain)
  const int16_t *run_chain;    // [n_runs] set-local chain
  const int16_t *run_exec;     // [n_runs]
  const int32_t *run_cb_lo, *run_cb_hi;  // [n_runs] set-local callback range
  // executors
  const uint32_t *hpx_mask;        // [n_exec] executors of the same core with higher process priority
  // accelerators
  const int32_t *buckets;          // [n_accels]
  const int64_t *aeps, *akappa;    // [n_accels]
  // units of accelerator types (Sec. IV-E); the accelerators above are then
  // the units, numbered type by type within a set
  const int16_t *seg_type;         // [n_segs] set-local input type of each segment
  const int16_t *type_units;       // [n_types] units of each type
  const int64_t *set_type_off;     // [n_sets+1] types of a set
  int32_t unit_group;              // PAAM_UNITS_*, or -1: no units (seg_accel is the input)
  // per-set maxima over the batch
  int32_t max_C, max_X, max_NA, max_runs, max_segs;
};

}  // namespace paam

namespace paam {
// Sets of one size class (chain count in (limit/2, limit], limit a power of two
// from 16 up): a contiguous range of the work order and the class's maxima.
// The analysis and the search launch once per class, so the LDS tables, the
// per-wave scratch and the occupancy follow the class rather than the
// batch's largest set.
struct SizeClass {
  int64_t begin, count;
  int32_t max_C, max_X, max_NA, max_runs, max_segs;
  // schedule of the analysis kernel chosen by paam_wcrt_autotune (0: not tuned)
  int32_t tuned_waves, tuned_micro;
};
constexpr int kMaxClasses = 12;
}  // namespace paam

struct paam_chainset {
  paam::DevBatch dev;
  size_t arena_bytes;
  int64_t n_exec, n_accel;
  int64_t max_tot;  // largest total demand of a set: sum of E, A + 2 kappa and epsilon
  int32_t max_cb_segs, max_buckets;  // largest eta of a callback, most buckets of an accelerator
  int32_t max_set_cbs;               // most callbacks in a set
  int n_classes;
  paam::SizeClass cls[paam::kMaxClasses];
};

namespace paam {

struct WcrtLaunch {
  DevBatch b;
  paam_wcrt_opts o;
  int8_t *set_sched;
  int32_t *set_worst;
  int64_t *set_worst_R;
  int64_t *chain_R;
  unsigned long long *counter;  // work queue head, zeroed before the launch
  unsigned char *scratch;       // per persistent wave
  size_t scratch_stride;        // bytes per wave
  size_t lds_bytes;
  int grid;
  int micro;                    // evaluations of each lane's recurrence per engine step
};

struct SearchLaunch {
  DevBatch b;
  paam_search_opts o;
  int32_t *found;               // [n_sets]
  int32_t *n_exact;             // [n_sets]
  int32_t *found_prio;          // [n_chains] or null
  unsigned long long *counter;
  unsigned char *scratch;
  size_t scratch_stride;        // bytes per wave: analysis scratch + search slot
  size_t analysis_stride;       // offset of the search slot in a wave's scratch
  size_t lds_bytes;
  int grid;
};

struct CandLaunch {
  DevBatch b;
  paam_wcrt_opts o;
  uint64_t seed;
  const int64_t *pairs;         // [n_pairs][3] set, k, util_permille
  int64_t n_pairs;
  int8_t *sched;
  int64_t *worst_R, *worst_D;
  float *ratio;                 // or null
  unsigned long long *counter;
  unsigned char *scratch;
  size_t scratch_stride;        // wave_search_bytes
  size_t analysis_stride;       // offset of the candidate slot in a wave's scratch
  size_t lds_bytes;
  int grid;
};

// Features of candidate orders: explicit (set, k, util) pairs, or (pairs ==
// null) every candidate of sets [set0, set0 + n_items / ceil(n_cand/64)) in
// runs of 64 consecutive candidates.
struct FeatLaunch {
  DevBatch b;
  uint64_t seed;
  const int64_t *pairs;
  int64_t n_items;
  int64_t set0;
  int32_t n_cand, util, row_stride;
  int32_t item;                 // consecutive candidates of a set per work item (range mode)
  // range mode, prefix-scan schedule: the order-independent tables of set
  // set0 + s at set_tables + s * set_table_stride, built by launch_feat_tables
  // for n_table_sets sets and shared by the set's items (null: each item
  // builds them in its wave's scratch)
  unsigned char *set_tables;
  size_t set_table_stride;
  int64_t n_table_sets;
  uint16_t *feat;
  int32_t *count;
  unsigned long long *counter;
  unsigned char *scratch;
  size_t scratch_stride;
  int grid;
};

struct FwdLaunch {
  const float *params;
  const uint16_t *packed;
  const uint16_t *feat;
  const int32_t *count;
  int64_t n;
  int32_t row_stride;
  float *out;
  void *act;
};

struct BwdLaunch {
  const float *params;
  const uint16_t *packed;
  const uint16_t *feat;
  const int32_t *count;
  int64_t n;
  int32_t row_stride;
  const float *out, *target;
  const void *act;
  float *partial;
  size_t part_stride;  // floats per chunk
};

// Binds every segment to a unit of its type (writes seg_accel in place).
int launch_units(const DevBatch &b, int n_cus, void *stream);
size_t units_lds_bytes(int64_t max_segs);
constexpr int kMaxUnitSegs = 2048;  // segments per set when types have units

// Event-driven simulation (paam_des.hip): one lane per scenario.
constexpr int kDesChains = 32;  // chains per set
constexpr int kDesExec = 16;    // executors per set
constexpr int kDesSegs = 8;     // segments per callback
constexpr int kDesLevels = 8;   // buckets per accelerator
struct DesLaunch {
  DevBatch b;
  paam_des_opts o;
  const int64_t *offsets;
  int64_t *obs;
  int8_t *status;
  int grid;
  int32_t max_cbs, max_segs;  // per set, over the batch (sizes of the LDS tables)
};
int launch_des(const DesLaunch &L, void *stream);
size_t des_lds_bytes(int64_t max_cbs, int64_t max_segs);
constexpr size_t kDesLdsMax = 48 * 1024;  // LDS tables of one set

size_t feat_wave_bytes(const DevBatch &b);
// Feature tables of up to this size per wave live in LDS (else in the wave's
// global scratch); the host sizes the grid for the LDS it takes.
constexpr size_t kFeatLdsMax = 40 * 1024;
bool feat_in_lds(const DevBatch &b);
// Candidates per work item of the scoring features: the LDS-table schedule
// builds a set's tables once per item, so longer items pay there; the
// prefix-scan schedule (global tables) is faster with shorter ones.
int feat_item(const DevBatch &b);
size_t backward_partial_stride();
int64_t backward_chunks(int64_t n);
int launch_features(const FeatLaunch &L, void *stream);
int launch_feat_tables(const FeatLaunch &L, int grid, void *stream);
int launch_pack(const float *params, uint16_t *packed, void *stream);
int launch_forward(const FwdLaunch &L, void *stream);
int launch_backward(const BwdLaunch &L, float *grad, float *loss, void *stream);
int launch_adam(float *P, uint16_t *Q, float *M, float *V, const float *G, float lr, float b1,
                float b2, float eps, int64_t step, void *stream);

// Scratch and LDS sizes for one wave analysing one set at a time.
size_t wave_scratch_bytes(const DevBatch &b);
size_t wave_lds_bytes(const DevBatch &b);
size_t wave_search_bytes(const DevBatch &b);
// The same for the analysis kernel of paam_wcrt_batch (no period table in
// LDS, blocking table in the wave's scratch).
size_t wcrt_scratch_bytes(const DevBatch &b);
size_t wcrt_lds_bytes(const DevBatch &b);

// The scratch of paam_wcrt_batch_noalloc: a static device array of this
// size per GPU (queue counter, then per-wave scratch), and its address on the
// current device (resolved once per device; returns a hipError_t as int).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
int noalloc_scratch(void **out);

// Launches (defined in paam_kernels.hip); return a hipError_t as int.
int launch_wcrt(const WcrtLaunch &L, void *stream);
int launch_search(const SearchLaunch &L, void *stream);
int launch_candidates(const CandLaunch &L, void *stream);

}  // namespace paam
