// HIP kernels of libpaam for gfx950: the batched response-time analysis of
// the paper's Sec. IV-F.
//
// Arithmetic.  Every time is an integer below 2^53 held in an fp64 register:
// sums and products of such integers are exact, and +inf stands for a bound
// past its cap.  The arrival bound of Lemma 1 / Eq. (2),
// mu(t) = ceil(t/T) + 1 = floor((t + 2T - 1) / T), is evaluated as
// floor((t + K) * rcp) with K = 2T - 1 and rcp = 1/T rounded towards +inf:
// for 0 <= x < 2^50 the product lies in [x/T, x/T + x*2^-52/T], which never
// reaches the next integer above x/T, so the floor is the exact quotient.
// That is four fp64 operations per interference term (add, mul, floor, fma),
// all full-rate on CDNA4, instead of an integer division.
//
// Schedule.  One wavefront per chain set, pulled from a work queue in
// decreasing estimated cost.  Lanes run over segments (Lemma 2), then over
// sub-chains (Theorem 1).  All sub-chains of a set iterate together: the
// per-executor interference weights (hp and hpp terms of Eq. 6) are built
// once and then updated by every change of an H* value, and each sweep
// re-evaluates, packed into full 64-lane chunks, only the sub-chains that
// have not converged or read a weight that changed.  Each iterate starts
// below the least fixed point and the
// system is monotone, so this chaotic iteration ends at the same least fixed
// point a sequential evaluation in dependency order reaches.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>

#include "paam_device.h"
#include "paam_internal.h"

namespace paam {
namespace {

__device__ __forceinline__ double mu_term(double t, double K, double rcp) {
  return __builtin_floor((t + K) * rcp);
}

__device__ __forceinline__ double scale_time(int64_t x, int32_t u) {
  return (double)(u == 1000 ? x : (x * (int64_t)u) / 1000);
}

__device__ __forceinline__ void atomic_max_nonneg(double *p, double v) {
  // non-negative doubles (and +inf) order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ int wave_any(bool p) { return __any(p); }

__device__ __forceinline__ int wave_max_int(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ int wave_min_int(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

// R_a / D_a > R_b / D_b for R, D < 2^53 (INF largest), exact in 128 bits.
__device__ __forceinline__ bool ratio_gt(double Ra, int64_t Da, double Rb, int64_t Db) {
  if (isinf(Ra)) return !isinf(Rb);
  if (isinf(Rb)) return false;
  unsigned __int128 l = (unsigned __int128)(uint64_t)Ra * (uint64_t)Db;
  unsigned __int128 r = (unsigned __int128)(uint64_t)Rb * (uint64_t)Da;
  return l > r;
}

// The blocking table ([X][C] doubles, used before the iteration only) sits
// in LDS for sets of up to 512 chain-executor pairs, else in the wave's
// global scratch, so that large sets keep more waves per CU.
__host__ __device__ inline bool sb_in_scratch(int Cm, int Xm) { return (size_t)Cm * Xm > 512; }

// LDS of one wave.  Tables by rank (0 = highest priority) with row stride C.
struct Lds {
  double2 *KR;                       // [C] (2T-1, 1/T up) of the chain at a rank
  double *Dd, *partial;              // [C] deadline, running end-to-end sum
  double *Ahat, *Bacc;               // [NA][C] A-hat; a user's largest A*, then its Bacc
  double *WP, *Pt;                   // [X][C] hp+hpp weight (rank above), hpp weight (below)
  double *SB;                        // [X][C] blocking candidates, then staging of the first build
                                     // (in the wave's global scratch for large tables)
  double *aek;                       // [NA][2] epsilon, kappa of each accelerator
  int32_t *rank;                     // [C] rank of a chain
  int32_t *nrs;                      // [C] sub-chains of the chain at a rank | busy-waits << 16
  int32_t *level;                    // [NA][C] bucket level of a user, -1 for a non-user
  int32_t *wmin, *pmax;              // [2][X] lowest rank whose WP changed, highest whose Pt
                                     // changed: as seen by this sweep, as recorded for the next
  int32_t *lpx;                      // [X] executors of the core with lower process priority
  int32_t *hpx;                      // [X] executors of the core with higher process priority
  int32_t *dmin, *dspin;             // [X] per step: lowest rank of a pending Lemma 3 sub-chain
                                     // on the executor, pending busy-waiting ones on it
  int32_t *dfirst, *dblk;            // [X] lowest rank of any Lemma 3 sub-chain on the executor;
                                     // a higher-priority executor of its core holds a busy-waiting one
  int32_t *misc;                     // [16]
};

struct Scratch {
  double *SB;                              // [max_X][max_C] when not in LDS
  double *segAs, *segH;                    // [max_segs]
  double *r, *hs, *cst, *L2, *A0, *eps;    // [max_runs]
  int32_t *info, *alist;                   // [max_runs] packed sub-chain word, active list
  double2 *qs;                             // [max_segs] Lemma 2 queue: (A*, g | packed rank, acc)
  double2 *qr;                             // [max_runs] Theorem 1 queue: (constant, s | packed word)
};

// with_kr: the (2T-1, 1/T) table is in LDS (candidate orders); sb_lds: the
// blocking table is in LDS.
__device__ Lds carve_lds(unsigned char *base, int Cm, int Xm, int NAm, bool with_kr, bool sb_lds) {
  Lds l;
  double *d = reinterpret_cast<double *>(base);
  l.KR = reinterpret_cast<double2 *>(d);
  if (with_kr) d += 2 * Cm;
  l.Dd = d; d += Cm;
  l.partial = d; d += Cm;
  l.Ahat = d; d += NAm * Cm;
  l.Bacc = d; d += NAm * Cm;
  l.WP = d; d += Xm * Cm;
  l.Pt = d; d += Xm * Cm;
  l.SB = nullptr;
  if (sb_lds) {
    l.SB = d;
    d += Xm * Cm;
  }
  l.aek = d;
  d += 2 * NAm;
  int32_t *i = reinterpret_cast<int32_t *>(d);
  l.rank = i; i += Cm;
  l.nrs = i; i += Cm;
  l.level = i; i += NAm * Cm;
  l.wmin = i; i += 2 * Xm;
  l.pmax = i; i += 2 * Xm;
  l.lpx = i; i += Xm;
  l.hpx = i; i += Xm;
  l.dmin = i; i += Xm;
  l.dspin = i; i += Xm;
  l.dfirst = i; i += Xm;
  l.dblk = i; i += Xm;
  l.misc = i;
  return l;
}

__device__ Scratch carve_scratch(unsigned char *base, int max_segs, int max_runs, int Cm, int Xm,
                              bool sb_scratch) {
  Scratch s;
  double *d = reinterpret_cast<double *>(base);
  s.SB = nullptr;
  if (sb_scratch) {
    s.SB = d;
    d += (size_t)Xm * Cm;
  }
  s.segAs = d; d += max_segs;
  s.segH = d; d += max_segs;
  s.r = d; d += max_runs;
  s.hs = d; d += max_runs;
  s.cst = d; d += max_runs;
  s.L2 = d; d += max_runs;
  s.A0 = d; d += max_runs;
  s.eps = d; d += max_runs;
  d = reinterpret_cast<double *>((reinterpret_cast<uintptr_t>(d) + 15) & ~(uintptr_t)15);
  s.qs = reinterpret_cast<double2 *>(d); d += 2 * (size_t)max_segs;
  s.qr = reinterpret_cast<double2 *>(d); d += 2 * (size_t)max_runs;
  int32_t *i = reinterpret_cast<int32_t *>(d);
  s.info = i; i += max_runs;
  s.alist = i;
  return s;
}

// Every recurrence is monotone from below and bounded by its cap, so it
// stops; the guard only makes termination unconditional.  A set that trips it
// reports set_sched = -1.
constexpr int kMaxIter = 1 << 20;


// Packed word of a sub-chain: rank of its chain in bits 0-11 (fewer than
// 4,096 chains per set), executor in bits 12-16, accelerator mask in bits
// 17-24, then flags.  The compaction of a sweep reads only this word.
constexpr int kRankMask = 0xfff;
constexpr int kExecShift = 12;
constexpr int kAccShift = 17;
constexpr int kNeedL3 = 1 << 25;  // H* follows Lemma 3 at the current window
constexpr int kHasP = 1 << 26;    // the executor has higher-priority executors on its core
constexpr int kConv = 1 << 27;    // last evaluation changed nothing
constexpr int kInf = 1 << 28;     // the bound is past the cap

// Analyses one set under the uploaded priorities and writes its outputs.
// Called by all 64 lanes of a wave.  Always inlined: the LDS tables reach it
// through plain pointers, and only inlined does the compiler see that they
// address LDS and emit LDS atomics (an outlined copy would apply flat
// atomics to them, which LDS does not take for fp64).
// kSbLds: the blocking table is in LDS (else in the wave's global scratch).
// try_early: in verdict mode, run the miss check at the segments' lower
// bounds before Lemma 2 (below); returns whether that check proved the miss.
template <bool kSbLds>
__device__ __forceinline__ bool analyse_set(const DevBatch &b, const paam_wcrt_opts &o,
                                            int64_t set, Lds &L, Scratch &S, int8_t *set_sched,
                                            int32_t *set_worst, int64_t *set_worst_R,
                                            int64_t *chain_R, bool try_early) {
  const int lane = threadIdx.x;
  const int64_t c0 = b.set_chain_off[set];
  const int C = (int)(b.set_chain_off[set + 1] - c0);
  const int64_t x0 = b.set_exec_off[set];
  const int X = (int)(b.set_exec_off[set + 1] - x0);
  const int64_t a0 = b.set_accel_off[set];
  const int NA = (int)(b.set_accel_off[set + 1] - a0);
  const int64_t cb0 = b.set_cb_off[set];
  const int64_t g0 = b.set_seg_off[set];
  const int nseg = (int)(b.set_seg_off[set + 1] - g0);
  const int64_t run0 = b.set_run_off[set];
  const int nrun = (int)(b.set_run_off[set + 1] - run0);
  const int32_t u = o.util_permille;
  const bool full = o.full != 0;
  const double hop = (double)b.eps_hop[set];
  const double capm = (double)o.cap_mult;  // cap of a chain = capm * D
  double *const SB = kSbLds ? L.SB : S.SB;

  // ---- chain tables in rank order (rank 0 = highest priority) ----
  for (int c = lane; c < C; c += kWave) {
    const int rho = b.rank0[c0 + c];
    L.rank[c] = rho;
    L.KR[rho] = make_double2(b.Kd[c0 + c], b.rcp[c0 + c]);
    const int64_t D = b.D[c0 + c];
    L.Dd[rho] = (double)D;
    L.nrs[rho] = b.chain_nrun[c0 + c] | (b.spin[c0 + c] ? 1 << 16 : 0);
    L.partial[rho] = 0.0;
  }
  for (int i = lane; i < NA * C; i += kWave) {
    L.Ahat[i] = 0.0;
    L.Bacc[i] = 0.0;
    L.level[i] = -1;
  }
  for (int i = lane; i < X * C; i += kWave) {
    L.WP[i] = 0.0;
    L.Pt[i] = 0.0;
    SB[i] = 0.0;
  }
  for (int e = lane; e < X; e += kWave) {
    uint32_t m = 0;
    for (int e2 = 0; e2 < X; ++e2)
      if ((b.hpx_mask[x0 + e2] >> e) & 1u) m |= 1u << e2;
    L.lpx[e] = (int32_t)m;
    L.wmin[X + e] = C;
    L.pmax[X + e] = -1;
  }
  if (lane == 0) L.misc[0] = 0;  // iteration guard tripped
  __syncthreads();

  // ---- segments: A* = A + 2 kappa; per chain and accelerator sum and max ----
  for (int g = lane; g < nseg; g += kWave) {
    const int a = b.seg_accel[g0 + g];
    const int rho = L.rank[b.seg_chain[g0 + g]];
    const double As = scale_time(b.A[g0 + g], u) + 2.0 * (double)b.akappa[a0 + a];
    S.segAs[g] = As;
    atomicAdd(&L.Ahat[a * C + rho], As);
    atomic_max_nonneg(&L.Bacc[a * C + rho], As);
    L.level[a * C + rho] = 0;  // a user
  }
  __syncthreads();

  // ---- buckets (Sec. IV-C): the users of an accelerator in priority order,
  //      user r of m in level floor(r*n/m); then, in place of a user's
  //      largest A*, the largest A* of a lower-priority user of its level, the
  //      blocking term of Eq. (3).  Levels never decrease down the order, so
  //      one pass from the lowest rank up keeps a running maximum. ----
  for (int a = 0; a < NA; ++a) {
    int32_t *lv = L.level + a * C;
    int m = 0;
    for (int rb = 0; rb < C; rb += kWave) {
      const int rho = rb + lane;
      m += (int)__popcll(__ballot(rho < C && lv[rho] >= 0));
    }
    const int64_t n = b.buckets[a0 + a];
    int r0 = 0;
    for (int rb = 0; rb < C; rb += kWave) {
      const int rho = rb + lane;
      const bool us = rho < C && lv[rho] >= 0;
      const unsigned long long bm = __ballot(us);
      if (us) lv[rho] = (int)(((int64_t)(r0 + (int)__popcll(bm & ((1ull << lane) - 1ull))) * n) / m);
      r0 += (int)__popcll(bm);
    }
  }
  __syncthreads();
  for (int a = lane; a < NA; a += kWave) {
    const int32_t *lv = L.level + a * C;
    double *bx = L.Bacc + a * C;
    int cur = -1;
    double mx = 0.0;
    for (int rho = C - 1; rho >= 0; --rho) {
      const int lev = lv[rho];
      if (lev < 0) continue;
      const double own = bx[rho];
      bx[rho] = lev == cur ? mx : 0.0;
      mx = lev == cur ? fmax(mx, own) : own;
      cur = lev;
    }
  }
  // highest-priority rank with a request of positive length on each
  // accelerator: a chain of lower rank sees HP accelerator interference
  for (int a = lane; a < NA; a += kWave) {
    int f = C;
    for (int h = 0; h < C; ++h)
      if (L.Ahat[a * C + h] > 0.0) { f = h; break; }
    L.misc[1 + a] = f;
  }
  __syncthreads();

  // Verdict mode: a first pass with every segment's handling time at its
  // lower bound A* + same-bucket blocking (the base of Lemma 2, below each of
  // its iterates) runs the miss check below before Lemma 2.  Every quantity
  // built from those times only grows with them, so the check stays a lower
  // bound; a candidate whose miss it proves skips Lemma 2 and the rest.
  // Otherwise the tables are cleared and the second pass runs with the
  // Lemma 2 times.
  const bool early = !full;
  bool missed = false, early_miss = false;
  for (int pass = early && try_early ? 0 : 1; pass < 2 && !missed; ++pass) {
    if (pass == 0) {
      for (int g = lane; g < nseg; g += kWave) {
        const int a = b.seg_accel[g0 + g];
        const int rho = L.rank[b.seg_chain[g0 + g]];
        S.segH[g] = S.segAs[g] + L.Bacc[a * C + rho];
      }
      __syncthreads();
    } else {
      if (early && try_early) {
        for (int i = lane; i < X * C; i += kWave) {
          L.WP[i] = 0.0;
          L.Pt[i] = 0.0;
          SB[i] = 0.0;
        }
        __syncthreads();
      }
      // ---- Lemma 2 / Eq. (3): per-segment handling time ----
      for (int gb = 0; gb < nseg; gb += kWave) {
        const int g = gb + lane;
        const bool valid = g < nseg;
        int rho = 0, a = 0;
        double base = 0.0, capv = 0.0;
        if (valid) {
          a = b.seg_accel[g0 + g];
          rho = L.rank[b.seg_chain[g0 + g]];
          base = S.segAs[g] + L.Bacc[a * C + rho];
          capv = L.Dd[rho] * capm;
        }
        const double *Ah = L.Ahat + a * C;
        double h = 0.0;
        bool done = !valid;
        for (int it = 0; wave_any(!done); ++it) {
          if (it >= kMaxIter) {
            if (!done) L.misc[0] = 1;
            break;
          }
          if (!done) {
            double n0 = base, n1 = 0.0;
            int k = 0;
            for (; k + 1 < rho; k += 2) {
              const double2 q0 = L.KR[k], q1 = L.KR[k + 1];
              n0 = fma(mu_term(h, q0.x, q0.y), Ah[k], n0);
              n1 = fma(mu_term(h, q1.x, q1.y), Ah[k + 1], n1);
            }
            if (k < rho) {
              const double2 q0 = L.KR[k];
              n0 = fma(mu_term(h, q0.x, q0.y), Ah[k], n0);
            }
            const double nxt = n0 + n1;
            if (nxt > capv) {
              h = INFINITY;
              done = true;
            } else if (nxt == h) {
              done = true;
            } else {
              h = nxt;
            }
          }
        }
        if (valid) S.segH[g] = h;
      }
      __syncthreads();
    }
    // ---- sub-chains: own demand, Lemma 2 sum, Lemma 3 constant, overheads,
    //      and each callback as a blocking candidate ----
    const bool safe = o.blocking == PAAM_BLOCK_SAFE;
    for (int s = lane; s < nrun; s += kWave) {
      const int64_t rr = run0 + s;
      const int c = b.run_chain[rr];
      const int e = b.run_exec[rr];
      const int rho = L.rank[c];
      double E = 0.0, L2 = 0.0, A0 = 0.0, eps = 0.0, bmax = 0.0;
      int delta = 0, accm = 0;
      for (int j = b.run_cb_lo[rr]; j < b.run_cb_hi[rr]; ++j) {
        const double Ej = scale_time(b.E[cb0 + j], u);
        E += Ej;
        double bj = Ej;
        for (int64_t gg = b.cb_seg_off[cb0 + j]; gg < b.cb_seg_off[cb0 + j + 1]; ++gg) {
          const int g = (int)(gg - g0);
          const int a = b.seg_accel[gg];
          const double Hg = S.segH[g];
          const double ea = (double)b.aeps[a0 + a];
          L2 += Hg;
          A0 += S.segAs[g] + L.Bacc[a * C + rho];
          eps += ea;
          if (safe) bj += Hg + ea;
          ++delta;
          accm |= 1 << a;
        }
        bmax = fmax(bmax, bj);
      }
      atomic_max_nonneg(&SB[e * C + rho], bmax);
      const bool needL3 =
          delta > 0 && (o.bound == PAAM_BOUND_L3 || (o.bound == PAAM_BOUND_MIN && delta >= 2));
      // H* of a sub-chain that does not need Lemma 3 during the iteration.  With
      // one segment, Lemma 3 is the recurrence of Lemma 2 and R >= H at the
      // fixed point, so H* = L2 + eps there; with no HP request of positive
      // length, Lemma 3 is the constant A0 <= L2 (also at an unbounded window).
      bool hp_acc = false;
      for (int a = 0; a < NA; ++a)
        if (((accm >> a) & 1) && L.misc[1 + a] < rho) hp_acc = true;
      double hs0 = delta == 0 ? 0.0 : (hp_acc || o.bound == PAAM_BOUND_L2 ? L2 : A0) + eps;
      if (needL3) hs0 = 0.0;  // a valid start below the fixed point
      // per chain and executor: E + H* (own executor's weight) in WP, and
      // E + spin() (H* if the chain busy-waits, else its epsilon sum) in Pt
      atomicAdd(&L.WP[e * C + rho], E + hs0);
      atomicAdd(&L.Pt[e * C + rho], E + ((L.nrs[rho] >> 16) ? hs0 : eps));
      S.r[s] = 0.0;
      // constant part of the recurrence: E, blocking (added below) and, when H*
      // does not follow Lemma 3 during the iteration, H* itself; only the
      // others keep H* as state
      S.hs[s] = hs0;
      S.cst[s] = E + (needL3 ? 0.0 : hs0);
      S.L2[s] = L2;
      S.A0[s] = A0;
      S.eps[s] = eps;
      S.info[s] = rho | (e << kExecShift) | (accm << kAccShift) | (needL3 ? kNeedL3 : 0) |
                  (b.hpx_mask[x0 + e] != 0 ? kHasP : 0);
    }
    __syncthreads();
    // suffix maximum of blocking candidates per executor, lowest priority up
    for (int e = lane; e < X; e += kWave) {
      double m = 0.0;
      for (int rho = C - 1; rho >= 0; --rho) {
        m = fmax(m, SB[e * C + rho]);
        SB[e * C + rho] = m;
      }
    }
    __syncthreads();
    // blocking by one callback of a lower priority chain on the executor
    for (int s = lane; s < nrun; s += kWave) {
      const int w = S.info[s];
      const int rho = w & kRankMask;
      const int e = (w >> kExecShift) & 31;
      S.cst[s] += rho + 1 < C ? SB[e * C + rho + 1] : 0.0;
    }
    __syncthreads();
    // interference weights at the starting H*: WP[e][h] = E + H* of h on e (hp
    // term of a lower-ranked chain) + hpp weight; Pt[e][h] = hpp weight alone,
    // the sum over the core's higher-priority executors e2 of E + spin() of h
    // on e2.  From here on every change of an H* is added to the weights it
    // enters, and the ranks it touches are recorded for the next sweep.
    for (int i = lane; i < X * C; i += kWave) {
      const int e = i / C, h = i - e * C;
      double p = 0.0;
      for (uint32_t m = b.hpx_mask[x0 + e]; m; m &= m - 1) p += L.Pt[(__ffs(m) - 1) * C + h];
      SB[i] = p;  // blocking candidates are dead
    }
    __syncthreads();
    for (int i = lane; i < X * C; i += kWave) {
      L.WP[i] += SB[i];
      L.Pt[i] = SB[i];
    }
    __syncthreads();

    // ---- verdict mode: the first iterate of every sub-chain (each interferer
    //      counted once, a Lemma 3 sub-chain without its H*) is a lower bound;
    //      a chain whose sum of them passes its deadline proves the miss.
    //      Each sub-chain's sum runs over the ranks, so the check costs about
    //      as much as a sweep: before Lemma 2 it pays for every set size, after
    //      it only for sets of up to 64 chains (for larger ones the partial
    //      sums of the first sweep find a miss as early) ----
    if (early && (pass == 0 || C <= kWave)) {
      for (int s = lane; s < nrun; s += kWave) {
        const int w = S.info[s];
        const int rho = w & kRankMask, e = (w >> kExecShift) & 31;
        const double *wp = L.WP + e * C, *pt = L.Pt + e * C;
        double lb = S.cst[s];
        for (int h = 0; h < rho; ++h) lb += wp[h];
        if (w & kHasP)
          for (int h = rho + 1; h < C; ++h) lb += pt[h];
        atomicAdd(&L.partial[rho], lb);
      }
      __syncthreads();
      bool miss = false;
      for (int rho = lane; rho < C; rho += kWave) {
        if (L.partial[rho] + (double)((L.nrs[rho] & 0xffff) - 1) * hop > L.Dd[rho]) miss = true;
        L.partial[rho] = 0.0;
      }
      missed = wave_any(miss);
      early_miss = missed && pass == 0;
      __syncthreads();
    }
  }

  // ---- Theorem 1 / Eq. (6): all sub-chains of the set together ----
  for (int sweep = 0; !missed; ++sweep) {
    if (sweep >= kMaxIter) {
      if (lane == 0) L.misc[0] = 1;
      break;
    }
    // the weight changes of the last sweep become this sweep's view
    for (int e = lane; e < X; e += kWave) {
      L.wmin[e] = L.wmin[X + e];
      L.pmax[e] = L.pmax[X + e];
      L.wmin[X + e] = C;
      L.pmax[X + e] = -1;
    }
    __syncthreads();

    // compact the sub-chains to evaluate: not converged, or a weight they
    // read changed (WP of a higher rank, Pt of a lower rank)
    int nact = 0;
    for (int sb = 0; sb < nrun; sb += kWave) {
      const int s = sb + lane;
      bool act = false;
      if (s < nrun) {
        const int w = S.info[s];
        const int rho = w & kRankMask, e = (w >> kExecShift) & 31;
        act = !(w & kInf) && (!(w & kConv) || rho > L.wmin[e] || rho < L.pmax[e]);
      }
      const unsigned long long m = __ballot(act);
      if (act) S.alist[nact + (int)__popcll(m & ((1ull << lane) - 1ull))] = s;
      nact += (int)__popcll(m);
    }
    if (nact == 0) break;
    __syncthreads();

    for (int ib = 0; ib < nact; ib += kWave) {
      const int i = ib + lane;
      const bool valid = i < nact;
      int s = 0, rho = 0, e = 0, inf1 = 0;
      double r = 0.0, hs_old = 0.0, cst = 0.0;
      if (valid) {
        // every per-sub-chain load the evaluation needs, issued together
        s = S.alist[i];
        inf1 = S.info[s];
        rho = inf1 & kRankMask;
        e = (inf1 >> kExecShift) & 31;
        r = S.r[s];
        if (inf1 & kNeedL3) hs_old = S.hs[s];
        cst = S.cst[s];
      }
      const bool hasP = (inf1 & kHasP) != 0;
      // the loop bound is the same on every lane: keep it in a scalar register
      const int hend = __builtin_amdgcn_readfirstlane(wave_max_int(valid ? (hasP ? C : rho) : 0));
      const bool needL3 = (inf1 & kNeedL3) != 0;
      const int accm = (inf1 >> kAccShift) & 0xff;
      const double *wp = L.WP + e * C;
      const double *pt = L.Pt + e * C;
      double I0 = 0.0, I1 = 0.0, l3 = 0.0;
      int h = 0;
      if (NA == 1) {
        // One accelerator: the Lemma 3 weight of h is Ahat[h] for a lane that
        // needs Lemma 3 and ranks below h, else 0.  The sub-chains of a chunk
        // are sorted by rank, so h splits into three ranges: below every
        // lane's rank (hp weight for all), between the smallest and largest
        // rank (per-lane selects), above every rank (hpp weight for all).
        const bool l3on = needL3 && (accm & 1) != 0;
        const double *ah = L.Ahat;
        const int rlo = __builtin_amdgcn_readfirstlane(wave_min_int(valid ? rho : C));
        const int rhi = __builtin_amdgcn_readfirstlane(wave_max_int(valid ? rho : -1));
        const int e_lo = rlo < hend ? rlo : hend;
        const int e_mid = rhi + 1 < hend ? rhi + 1 : hend;
        const bool anyl3 = wave_any(l3on);
        if (!anyl3) {
          // no lane of the chunk follows Lemma 3: hp weights only
#pragma unroll 2
          for (; h + 1 < e_lo; h += 2) {
            const double2 q0 = L.KR[h], q1 = L.KR[h + 1];
            I0 = fma(mu_term(r, q0.x, q0.y), wp[h], I0);
            I1 = fma(mu_term(r, q1.x, q1.y), wp[h + 1], I1);
          }
        } else {
#pragma unroll 2
          for (; h + 1 < e_lo; h += 2) {
            const double2 q0 = L.KR[h], q1 = L.KR[h + 1];
            const double m0 = mu_term(r, q0.x, q0.y);
            const double m1 = mu_term(r, q1.x, q1.y);
            const double av0 = ah[h], av1 = ah[h + 1];
            I0 = fma(m0, wp[h], I0);
            I1 = fma(m1, wp[h + 1], I1);
            l3 = fma(m0, l3on ? av0 : 0.0, l3);
            l3 = fma(m1, l3on ? av1 : 0.0, l3);
          }
        }
        if (h < e_lo) {
          const double2 q0 = L.KR[h];
          const double m0 = mu_term(r, q0.x, q0.y);
          const double av0 = ah[h];
          I0 = fma(m0, wp[h], I0);
          l3 = fma(m0, l3on ? av0 : 0.0, l3);
          ++h;
        }
        // one table read per term: the lane picks WP below its rank, Pt above
        if (!anyl3) {
          for (; h + 1 < e_mid; h += 2) {
            const double2 q0 = L.KR[h], q1 = L.KR[h + 1];
            double w0 = (h < rho ? wp : pt)[h];
            double w1 = (h + 1 < rho ? wp : pt)[h + 1];
            w0 = h == rho ? 0.0 : w0;
            w1 = h + 1 == rho ? 0.0 : w1;
            I0 = fma(mu_term(r, q0.x, q0.y), w0, I0);
            I1 = fma(mu_term(r, q1.x, q1.y), w1, I1);
          }
        }
        for (; h + 1 < e_mid; h += 2) {
          const double2 q0 = L.KR[h], q1 = L.KR[h + 1];
          const double m0 = mu_term(r, q0.x, q0.y);
          const double m1 = mu_term(r, q1.x, q1.y);
          double w0 = (h < rho ? wp : pt)[h];
          double w1 = (h + 1 < rho ? wp : pt)[h + 1];
          w0 = h == rho ? 0.0 : w0;
          w1 = h + 1 == rho ? 0.0 : w1;
          const double av0 = ah[h], av1 = ah[h + 1];  // h + 1 < hend <= C: in bounds
          I0 = fma(m0, w0, I0);
          I1 = fma(m1, w1, I1);
          l3 = fma(m0, (l3on && h < rho) ? av0 : 0.0, l3);
          l3 = fma(m1, (l3on && h + 1 < rho) ? av1 : 0.0, l3);
        }
        if (h < e_mid) {
          const double2 q0 = L.KR[h];
          const double m0 = mu_term(r, q0.x, q0.y);
          double w0 = (h < rho ? wp : pt)[h];
          w0 = h == rho ? 0.0 : w0;
          const double av0 = ah[h];
          I0 = fma(m0, w0, I0);
          l3 = fma(m0, (l3on && h < rho) ? av0 : 0.0, l3);
          ++h;
        }
#pragma unroll 2
        for (; h + 1 < hend; h += 2) {
          const double2 q0 = L.KR[h], q1 = L.KR[h + 1];
          const double m0 = mu_term(r, q0.x, q0.y);
          const double m1 = mu_term(r, q1.x, q1.y);
          I0 = fma(m0, pt[h], I0);
          I1 = fma(m1, pt[h + 1], I1);
        }
        if (h < hend) {
          const double2 q0 = L.KR[h];
          const double m0 = mu_term(r, q0.x, q0.y);
          I0 = fma(m0, pt[h], I0);
          ++h;
        }
      }
      for (; h + 1 < hend; h += 2) {
        const double2 q0 = L.KR[h], q1 = L.KR[h + 1];
        const double m0 = mu_term(r, q0.x, q0.y);
        const double m1 = mu_term(r, q1.x, q1.y);
        double w0 = h < rho ? wp[h] : pt[h];
        double w1 = h + 1 < rho ? wp[h + 1] : pt[h + 1];
        w0 = h == rho ? 0.0 : w0;
        w1 = h + 1 == rho ? 0.0 : w1;
        I0 = fma(m0, w0, I0);
        I1 = fma(m1, w1, I1);
        if (needL3 && h < rho) {
          double a0s = 0.0, a1s = 0.0;
          for (int a = 0; a < NA; ++a)
            if ((accm >> a) & 1) {
              a0s += L.Ahat[a * C + h];
              a1s += h + 1 < rho ? L.Ahat[a * C + h + 1] : 0.0;
            }
          l3 = fma(m0, a0s, l3);
          l3 = fma(m1, a1s, l3);
        }
      }
      if (h < hend) {
        const double2 q0 = L.KR[h];
        const double m0 = mu_term(r, q0.x, q0.y);
        double w0 = h < rho ? wp[h] : pt[h];
        w0 = h == rho ? 0.0 : w0;
        I0 = fma(m0, w0, I0);
        if (needL3 && h < rho) {
          double a0s = 0.0;
          for (int a = 0; a < NA; ++a)
            if ((accm >> a) & 1) a0s += L.Ahat[a * C + h];
          l3 = fma(m0, a0s, l3);
        }
      }
      if (valid) {
        double hsn = hs_old;
        if (needL3) {
          const double L3 = S.A0[s] + l3;
          hsn = (o.bound == PAAM_BOUND_L3 ? L3 : fmin(S.L2[s], L3)) + S.eps[s];
        }
        double rn = cst + hsn + (I0 + I1);
        if (rn > L.Dd[rho] * capm) {
          rn = INFINITY;
          if (needL3) {
            // Lemma 3 at an unbounded window: unbounded iff an HP request of
            // positive length can interfere (then l3 > 0 already)
            const double L3i = l3 > 0.0 ? INFINITY : S.A0[s];
            hsn = (o.bound == PAAM_BOUND_L3 ? L3i : fmin(S.L2[s], L3i)) + S.eps[s];
          }
        }
        if (hsn != hs_old) {
          // H* of the chain on e enters its hp weight on e and, for a
          // busy-waiting chain, the hp and hpp weights on the core's
          // lower-priority executors
          const double dh = hsn - hs_old;
          atomicAdd(&L.WP[e * C + rho], dh);
          atomicMin(&L.wmin[X + e], rho);
          if (L.nrs[rho] >> 16) {
            for (uint32_t m = (uint32_t)L.lpx[e]; m; m &= m - 1) {
              const int e2 = __ffs(m) - 1;
              atomicAdd(&L.WP[e2 * C + rho], dh);
              atomicAdd(&L.Pt[e2 * C + rho], dh);
              atomicMin(&L.wmin[X + e2], rho);
              atomicMax(&L.pmax[X + e2], rho);
            }
          }
        }
        if (rn != r) atomicAdd(&L.partial[rho], rn - r);
        S.info[s] = (inf1 & ~kConv) | (rn == r ? kConv : 0) | (isinf(rn) ? kInf : 0);
        S.r[s] = rn;
        if (needL3) S.hs[s] = hsn;
      }
      if (!full) {
        // verdict mode: a chain of this chunk whose partial end-to-end sum
        // (a lower bound) already exceeds its deadline proves the miss
        bool miss = false;
        if (valid) miss = L.partial[rho] + (double)((L.nrs[rho] & 0xffff) - 1) * hop > L.Dd[rho];
        if (wave_any(miss)) {
          missed = true;
          break;
        }
      }
    }
    __syncthreads();
    if (missed) break;
    if (!full) {
      // every iterate is a lower bound: a partial end-to-end sum above the
      // deadline proves the miss
      bool miss = false;
      for (int rho = lane; rho < C; rho += kWave)
        if (L.partial[rho] + (double)((L.nrs[rho] & 0xffff) - 1) * hop > L.Dd[rho]) miss = true;
      if (wave_any(miss)) {
        missed = true;
        break;
      }
    }
  }

  // ---- end-to-end bounds, verdict, worst chain ----
  bool ok = !missed;
  if (!missed) {
    bool late = false;
    for (int rho = lane; rho < C; rho += kWave) {
      double R = L.partial[rho] + (double)((L.nrs[rho] & 0xffff) - 1) * hop;
      if (R > L.Dd[rho] * capm) R = INFINITY;
      L.partial[rho] = R;
      if (R > L.Dd[rho]) late = true;
    }
    ok = !wave_any(late);
  }
  __syncthreads();
  if (!missed && full && chain_R) {
    for (int c = lane; c < C; c += kWave) {
      const double R = L.partial[L.rank[c]];
      chain_R[c0 + c] = isinf(R) ? PAAM_INF : (int64_t)R;
    }
  }
  // worst chain: the largest R/D (exact cross-multiplication), ties to the
  // lowest chain index; each lane scans its chains, then a wave reduction
  int32_t w = -1;
  double wRd = 0.0;
  int64_t wD = 1;
  if (!missed && (ok || full)) {
    for (int c = lane; c < C; c += kWave) {
      const double R = L.partial[L.rank[c]];
      const int64_t D = b.D[c0 + c];
      if (w < 0 || ratio_gt(R, D, wRd, wD)) {
        w = c;
        wRd = R;
        wD = D;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const int w2 = __shfl_xor(w, off);
      const double R2 = __shfl_xor(wRd, off);
      const int64_t D2 = __shfl_xor(wD, off);
      bool take = false;
      if (w2 >= 0) {
        if (w < 0 || ratio_gt(R2, D2, wRd, wD)) take = true;
        else if (!ratio_gt(wRd, wD, R2, D2) && w2 < w) take = true;
      }
      if (take) {
        w = w2;
        wRd = R2;
        wD = D2;
      }
    }
  }
  if (lane == 0) {
    const int64_t wR = (w < 0 || isinf(wRd)) ? PAAM_INF : (int64_t)wRd;
    set_sched[set] = L.misc[0] ? -1 : (ok ? 1 : 0);
    set_worst[set] = w;
    set_worst_R[set] = wR;
  }
  __syncthreads();
  return early_miss;
}

// ------------------------- queue-driven analysis ---------------------------
//
// Source of the (2T - 1, 1/T rounded up) pair of the chain at rank h.  Under
// the uploaded priorities it is the rank-ordered table built at upload, which
// no kernel writes: a read at a wave-uniform rank is a scalar load, so the
// inner loops read only the per-lane weights from LDS.  Under a candidate
// order it is the wave's LDS table.
struct KRConst {
  static constexpr bool kUploaded = true;
  const __attribute__((address_space(4))) double *p;  // (2T - 1, 1/T) pairs by rank
  __device__ __forceinline__ double2 operator()(int h) const {
    return make_double2(p[2 * h], p[2 * h + 1]);
  }
};
struct KRShared {
  static constexpr bool kUploaded = false;
  const double2 *p;
  __device__ __forceinline__ double2 operator()(int h) const { return p[h]; }
};

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long lanes_below() {
  return (1ull << threadIdx.x) - 1ull;
}

// Wave-wide integer max / min (DPP, no LDS traffic); every lane gets the result.
extern "C" __device__ int __ockl_wfred_max_i32(int);
extern "C" __device__ int __ockl_wfred_min_i32(int);
__device__ __forceinline__ int wave_umax(int v) { return uniform_int(__ockl_wfred_max_i32(v)); }
__device__ __forceinline__ int wave_umin(int v) { return uniform_int(__ockl_wfred_min_i32(v)); }

// The analysis runs in one-wave workgroups, whose LDS operations take effect
// in program order: within an engine step a compiler fence at wavefront scope
// orders them, without the drain of outstanding global loads and stores that
// a workgroup barrier implies.  Phase boundaries that hand data over through
// global scratch keep the workgroup barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Inclusive suffix maximum over the lanes of a wave (lane i: max of lanes >= i).
__device__ __forceinline__ unsigned long long wave_suffix_max_u64(unsigned long long v) {
  for (int d = 1; d < kWave; d <<= 1) {
    const unsigned long long w = __shfl_down(v, d);
    if (threadIdx.x + d < kWave && w > v) v = w;
  }
  return v;
}

// Keys of the same-bucket blocking scan: (kLevTop - level) above the A* bits.
// A* < 2^47 (times below 2^36 scaled by at most 1000, plus 2 kappa) and
// levels below 2^15 (buckets are int16).
constexpr int kKeyShift = 47;
constexpr int kLevTop = 1 << 15;
constexpr unsigned long long kKeyMask = (1ull << kKeyShift) - 1ull;

// Two 32-bit fields in the bits of a double (queue records).
__device__ __forceinline__ double pack2(int hi, int lo) { return __hiloint2double(hi, lo); }

// Analyses one set under the uploaded priorities (kr: KRConst) or a candidate
// order whose ranks are in b.rank0 and whose (2T-1, 1/T) table is in L.KR
// (kr: KRShared), and writes its outputs.  Called by all 64 lanes of a wave.
//
// Every recurrence of Sec. IV-F is solved by a lane that owns one item
// (a segment for Lemma 2, a sub-chain for Theorem 1) and takes the next item
// from a queue when its own is final, so all lanes stay busy while items
// remain.  Lemma 2 items are independent.  Sub-chains are coupled only
// through the H* of the sub-chains whose H* follows Lemma 3 during the
// iteration (two or more segments): every other H* is a constant.  Those are
// queued first, each after the ones it reads (executors by the number of
// higher-priority executors on their core, then rank), then the sub-chains
// that read none of them, then the rest.  A sub-chain's value is final when
// an evaluation leaves it unchanged and every Lemma 3 sub-chain it reads is
// final; until then it is re-evaluated with the current weights.  Every
// iterate stays below the least fixed point (the system is monotone and
// starts at 0), so the final values are the least fixed points.
template <class KR, bool kSbLds, bool kFull>
__device__ __forceinline__ void analyse_set_q(const DevBatch &b, const paam_wcrt_opts &o,
                                              int64_t set, KR kr, Lds &L, Scratch &S,
                                              int8_t *set_sched, int32_t *set_worst,
                                              int64_t *set_worst_R, int64_t *chain_R, int micro) {
  const int lane = threadIdx.x;
  const int64_t c0 = b.set_chain_off[set];
  const int C = (int)(b.set_chain_off[set + 1] - c0);
  const int64_t x0 = b.set_exec_off[set];
  const int X = (int)(b.set_exec_off[set + 1] - x0);
  const int64_t a0 = b.set_accel_off[set];
  const int NA = (int)(b.set_accel_off[set + 1] - a0);
  const int64_t cb0 = b.set_cb_off[set];
  const int64_t g0 = b.set_seg_off[set];
  const int nseg = (int)(b.set_seg_off[set + 1] - g0);
  const int64_t run0 = b.set_run_off[set];
  const int nrun = (int)(b.set_run_off[set + 1] - run0);
  const int32_t u = o.util_permille;
  constexpr bool full = kFull;  // the launch picks the instantiation by the option
  const double hop = (double)b.eps_hop[set];
  const double capm = (double)o.cap_mult;
  const bool uploaded = KR::kUploaded;
  double *const SB = kSbLds ? L.SB : S.SB;

  // ---- chain tables in rank order (rank 0 = highest priority) ----
  for (int c = lane; c < C; c += kWave) {
    const int rho = b.rank0[c0 + c];
    L.rank[c] = rho;
    if (!uploaded) L.KR[rho] = make_double2(b.Kd[c0 + c], b.rcp[c0 + c]);
    L.Dd[rho] = (double)b.D[c0 + c];
    L.nrs[rho] = b.chain_nrun[c0 + c] | (b.spin[c0 + c] ? 1 << 16 : 0);
    L.partial[rho] = 0.0;
  }
  for (int i = lane; i < NA * C; i += kWave) {
    L.Ahat[i] = 0.0;
    L.Bacc[i] = 0.0;
    L.level[i] = -1;
  }
  for (int i = lane; i < X * C; i += kWave) {
    L.WP[i] = 0.0;
    L.Pt[i] = 0.0;
    SB[i] = 0.0;
  }
  for (int e = lane; e < X; e += kWave) {
    uint32_t m = 0;
    for (int e2 = 0; e2 < X; ++e2)
      if ((b.hpx_mask[x0 + e2] >> e) & 1u) m |= 1u << e2;
    L.lpx[e] = (int32_t)m;
    L.hpx[e] = (int32_t)b.hpx_mask[x0 + e];
    L.dfirst[e] = C;
    L.dspin[e] = 0;
    L.dmin[e] = 0;
  }
  for (int a = lane; a < NA; a += kWave) {
    L.aek[2 * a] = (double)b.aeps[a0 + a];
    L.aek[2 * a + 1] = (double)b.akappa[a0 + a];
  }
  if (lane == 0) L.misc[0] = 0;  // iteration guard tripped
  __syncthreads();

  // ---- segments: A* = A + 2 kappa; per chain and accelerator sum and max;
  //      the Lemma 2 queue (under the uploaded priorities: decreasing rank) ----
  for (int pos = lane; pos < nseg; pos += kWave) {
    const int g = uploaded ? b.seg_order[g0 + (nseg - 1 - pos)] : pos;
    const int a = b.seg_accel[g0 + g];
    const int rho = L.rank[b.seg_chain[g0 + g]];
    const double As = scale_time(b.A[g0 + g], u) + 2.0 * L.aek[2 * a + 1];
    S.segAs[g] = As;
    S.qs[pos] = make_double2(As, pack2(g, rho | (a << kExecShift)));
    atomicAdd(&L.Ahat[a * C + rho], As);
    atomic_max_nonneg(&L.Bacc[a * C + rho], As);
    L.level[a * C + rho] = 0;  // a user
  }
  __syncthreads();

  // ---- buckets (Sec. IV-C) and the same-bucket blocking term of Eq. (3),
  //      as in the sweep analysis ----
  for (int a = 0; a < NA; ++a) {
    int32_t *lv = L.level + a * C;
    int m = 0;
    for (int rb = 0; rb < C; rb += kWave) {
      const int rho = rb + lane;
      m += (int)__popcll(__ballot(rho < C && lv[rho] >= 0));
    }
    const int64_t n = b.buckets[a0 + a];
    int r0 = 0;
    for (int rb = 0; rb < C; rb += kWave) {
      const int rho = rb + lane;
      const bool us = rho < C && lv[rho] >= 0;
      const unsigned long long bm = __ballot(us);
      if (us) lv[rho] = (int)(((int64_t)(r0 + (int)__popcll(bm & lanes_below())) * n) / m);
      r0 += (int)__popcll(bm);
    }
  }
  __syncthreads();
  // In place of a user's largest A*: the largest A* of a lower-priority user
  // of its level.  Levels never decrease down the order, so among the users
  // below a rank the ones of the smallest level come first; the exclusive
  // suffix maximum of (smallest level first, then A*) keys gives the term.
  for (int a = 0; a < NA; ++a) {
    const int32_t *lv = L.level + a * C;
    double *bx = L.Bacc + a * C;
    unsigned long long carry = 0ull;
    for (int rb = ((C - 1) / kWave) * kWave; rb >= 0; rb -= kWave) {
      const int rho = rb + lane;
      const int lev = rho < C ? lv[rho] : -1;
      const unsigned long long key =
          lev >= 0 ? ((unsigned long long)(kLevTop - lev) << kKeyShift) |
                         (unsigned long long)bx[rho]
                   : 0ull;
      const unsigned long long incl = wave_suffix_max_u64(key);
      unsigned long long excl = __shfl_down(incl, 1);
      if (lane == kWave - 1) excl = 0ull;
      excl = excl > carry ? excl : carry;
      if (lev >= 0)
        bx[rho] = (excl != 0ull && kLevTop - (int)(excl >> kKeyShift) == lev)
                      ? (double)(excl & kKeyMask)
                      : 0.0;
      const unsigned long long top = __shfl(incl, 0);
      carry = top > carry ? top : carry;
    }
  }
  // highest-priority rank with a request of positive length on each
  // accelerator: a chain of lower rank sees HP accelerator interference
  for (int a = 0; a < NA; ++a) {
    int f = C;
    for (int rb = 0; rb < C; rb += kWave) {
      const unsigned long long m = __ballot(rb + lane < C && L.Ahat[a * C + rb + lane] > 0.0);
      if (m) {
        f = rb + __ffsll((long long)m) - 1;
        break;
      }
    }
    if (lane == 0) L.misc[1 + a] = f;
  }
  __syncthreads();

  // Verdict mode: a first pass with every segment's handling time at its
  // lower bound A* + same-bucket blocking (below every Lemma 2 iterate) runs
  // the miss check below before Lemma 2; everything built from those times
  // only grows with them, so the check stays a lower bound, and a set whose
  // miss it proves skips Lemma 2 and the rest.  Otherwise the tables and the
  // Lemma 3 counters are cleared and the second pass runs with Lemma 2.
  bool missed = false;
  int maxlev = 0;  // most higher-priority executors of an executor on its core
  for (int pass = full ? 1 : 0; pass < 2 && !missed; ++pass) {
    if (pass == 0) {
      for (int g = lane; g < nseg; g += kWave) {
        const int a = b.seg_accel[g0 + g];
        const int rho = L.rank[b.seg_chain[g0 + g]];
        S.segH[g] = S.segAs[g] + L.Bacc[a * C + rho];
      }
      __syncthreads();
    } else {
      if (!full) {
        for (int i = lane; i < X * C; i += kWave) {
          L.WP[i] = 0.0;
          L.Pt[i] = 0.0;
          SB[i] = 0.0;
        }
        for (int e = lane; e < X; e += kWave) {
          L.dfirst[e] = C;
          L.dspin[e] = 0;
          L.dmin[e] = 0;
        }
        __syncthreads();
      }
      // ---- Lemma 2 / Eq. (3): one segment per lane, refilled from the queue
      //      (the next 64 queue records are loaded one step ahead); a step
      //      iterates every lane's recurrence up to `micro` times, sharing the
      //      step's refill and bookkeeping ----
      {
        int qnext = 0;
        bool have = false;
        int g = 0, rho = 0, a = 0;
        double hv = 0.0, base = 0.0, capv = 0.0;
        double2 win = make_double2(0.0, 0.0);
        if (lane < nseg) win = S.qs[lane];
        for (int step = 0;; ++step) {
          const unsigned long long need = __ballot(!have);
          const int k = (int)__popcll(need & lanes_below());
          const double wA = __shfl(win.x, k), wP = __shfl(win.y, k);
          if (!have && qnext + k < nseg) {
            const int pk = __double2loint(wP);
            g = __double2hiint(wP);
            rho = pk & kRankMask;
            a = pk >> kExecShift;
            base = wA + L.Bacc[a * C + rho];
            capv = L.Dd[rho] * capm;
            hv = 0.0;
            have = true;
          }
          qnext += (int)__popcll(need);
          if (!wave_any(have)) break;
          if (qnext + lane < nseg) win = S.qs[qnext + lane];
          if (step >= kMaxIter) {
            if (lane == 0) L.misc[0] = 1;
            break;
          }
          const int hend = wave_umax(have ? rho : 0);
          const int klo = min(wave_umin(have ? rho : C), hend);
          const double *ah = L.Ahat + a * C;
          bool done = false;
          for (int it = 0; it < micro; ++it) {
            double n0 = 0.0, n1 = 0.0;
            int k2 = 0;
    #pragma unroll 2
            for (; k2 + 1 < klo; k2 += 2) {
              const double2 q0 = kr(k2), q1 = kr(k2 + 1);
              n0 = fma(mu_term(hv, q0.x, q0.y), ah[k2], n0);
              n1 = fma(mu_term(hv, q1.x, q1.y), ah[k2 + 1], n1);
            }
            if (k2 < klo) {
              const double2 q0 = kr(k2);
              n0 = fma(mu_term(hv, q0.x, q0.y), ah[k2], n0);
              ++k2;
            }
            for (; k2 + 1 < hend; k2 += 2) {
              const double2 q0 = kr(k2), q1 = kr(k2 + 1);
              const double w0 = k2 < rho ? ah[k2] : 0.0;
              const double w1 = k2 + 1 < rho ? ah[k2 + 1] : 0.0;
              n0 = fma(mu_term(hv, q0.x, q0.y), w0, n0);
              n1 = fma(mu_term(hv, q1.x, q1.y), w1, n1);
            }
            if (k2 < hend) {
              const double2 q0 = kr(k2);
              const double w0 = k2 < rho ? ah[k2] : 0.0;
              n0 = fma(mu_term(hv, q0.x, q0.y), w0, n0);
            }
            if (have && !done) {
              const double nxt = base + (n0 + n1);
              if (nxt > capv) {
                hv = INFINITY;
                done = true;
              } else {
                done = nxt == hv;
                hv = nxt;
              }
            }
            if (!wave_any(have && !done)) break;
          }
          if (have && done) {
            S.segH[g] = hv;
            have = false;
          }
        }
      }
      __syncthreads();
    }
    // ---- sub-chains: own demand, Lemma 2 sum, Lemma 3 constant, overheads,
    //      and each callback as a blocking candidate ----
    const bool safe = o.blocking == PAAM_BLOCK_SAFE;
    for (int s = lane; s < nrun; s += kWave) {
      const int64_t rr = run0 + s;
      const int c = b.run_chain[rr];
      const int e = b.run_exec[rr];
      const int rho = L.rank[c];
      double E = 0.0, L2 = 0.0, A0 = 0.0, eps = 0.0, bmax = 0.0;
      int delta = 0, accm = 0;
      for (int j = b.run_cb_lo[rr]; j < b.run_cb_hi[rr]; ++j) {
        const double Ej = scale_time(b.E[cb0 + j], u);
        E += Ej;
        double bj = Ej;
        for (int64_t gg = b.cb_seg_off[cb0 + j]; gg < b.cb_seg_off[cb0 + j + 1]; ++gg) {
          const int g = (int)(gg - g0);
          const int a = b.seg_accel[gg];
          const double Hg = S.segH[g];
          const double ea = L.aek[2 * a];
          L2 += Hg;
          A0 += S.segAs[g] + L.Bacc[a * C + rho];
          eps += ea;
          if (safe) bj += Hg + ea;
          ++delta;
          accm |= 1 << a;
        }
        bmax = fmax(bmax, bj);
      }
      atomic_max_nonneg(&SB[e * C + rho], bmax);
      const bool needL3 =
          delta > 0 && (o.bound == PAAM_BOUND_L3 || (o.bound == PAAM_BOUND_MIN && delta >= 2));
      // H* of a sub-chain that does not need Lemma 3 during the iteration (one
      // segment: Lemma 3 is the recurrence of Lemma 2 and R >= H at the fixed
      // point, so H* = L2 + eps; no HP request of positive length: Lemma 3 is
      // the constant A0 <= L2, also at an unbounded window)
      bool hp_acc = false;
      for (int a = 0; a < NA; ++a)
        if (((accm >> a) & 1) && L.misc[1 + a] < rho) hp_acc = true;
      double hs0 = delta == 0 ? 0.0 : (hp_acc || o.bound == PAAM_BOUND_L2 ? L2 : A0) + eps;
      if (needL3) {
        hs0 = 0.0;  // a start below the fixed point
        atomicMin(&L.dfirst[e], rho);
        if (L.nrs[rho] >> 16) atomicAdd(&L.dspin[e], 1);
        atomicAdd(&L.dmin[__popc((uint32_t)L.hpx[e])], 1);  // per level, before the engine
      }
      atomicAdd(&L.WP[e * C + rho], E + hs0);
      atomicAdd(&L.Pt[e * C + rho], E + ((L.nrs[rho] >> 16) ? hs0 : eps));
      S.cst[s] = E + (needL3 ? 0.0 : hs0);
      if (needL3) {  // the Lemma 3 constants are read by these sub-chains only
        S.L2[s] = L2;
        S.A0[s] = A0;
        S.eps[s] = eps;
      }
      S.info[s] = rho | (e << kExecShift) | (accm << kAccShift) | (needL3 ? kNeedL3 : 0) |
                  (b.hpx_mask[x0 + e] != 0 ? kHasP : 0);
    }
    __syncthreads();
    // suffix maximum of blocking candidates per executor, lowest priority up
    // (non-negative doubles order like their bit patterns)
    for (int e = 0; e < X; ++e) {
      unsigned long long carry = 0ull;
      for (int rb = ((C - 1) / kWave) * kWave; rb >= 0; rb -= kWave) {
        const int rho = rb + lane;
        const unsigned long long v =
            rho < C ? (unsigned long long)__double_as_longlong(SB[e * C + rho]) : 0ull;
        unsigned long long incl = wave_suffix_max_u64(v);
        incl = incl > carry ? incl : carry;
        if (rho < C) SB[e * C + rho] = __longlong_as_double((long long)incl);
        carry = __shfl(incl, 0);
      }
    }
    for (int e = lane; e < X; e += kWave) {
      bool blk = false;
      for (uint32_t mm = (uint32_t)L.hpx[e]; mm; mm &= mm - 1)
        if (L.dspin[__ffs(mm) - 1] > 0) blk = true;
      L.dblk[e] = blk ? 1 : 0;
    }
    __syncthreads();
    for (int s = lane; s < nrun; s += kWave) {
      const int w = S.info[s];
      const int rho = w & kRankMask;
      const int e = (w >> kExecShift) & 31;
      S.cst[s] += rho + 1 < C ? SB[e * C + rho + 1] : 0.0;
    }
    __syncthreads();
    // hpp weights: Pt[e][h] becomes the sum over the core's higher-priority
    // executors e2 of E + spin() of h on e2 (so far Pt[e2][h]), and enters
    // WP[e][h].  Executors are rewritten by decreasing number of
    // higher-priority executors on their core, so every Pt[e2] read is still
    // the one accumulated above.
    maxlev = 0;
    for (int e = lane; e < X; e += kWave) maxlev = max(maxlev, __popc((uint32_t)L.hpx[e]));
    maxlev = wave_umax(maxlev);
    for (int lev = maxlev; lev >= 1; --lev) {
      for (int i = lane; i < X * C; i += kWave) {
        const int e = i / C, h = i - e * C;
        const uint32_t hm = (uint32_t)L.hpx[e];
        if (__popc(hm) != lev) continue;
        double p = 0.0;
        for (uint32_t m = hm; m; m &= m - 1) p += L.Pt[(__ffs(m) - 1) * C + h];
        L.WP[i] += p;
        L.Pt[i] = p;
      }
      wave_sync();
    }
    for (int i = lane; i < X * C; i += kWave)
      if (L.hpx[i / C] == 0) L.Pt[i] = 0.0;

    __syncthreads();

    // ---- verdict mode: the first iterate of every sub-chain (each interferer
    //      counted once, a Lemma 3 sub-chain without its H*) is a lower bound;
    //      a chain whose sum of them passes its deadline proves the miss ----
    if (!full) {
      for (int s = lane; s < nrun; s += kWave) {
        const int w = S.info[s];
        const int rho = w & kRankMask, e = (w >> kExecShift) & 31;
        const double *wp = L.WP + e * C, *pt = L.Pt + e * C;
        double lb = S.cst[s];
        for (int h = 0; h < rho; ++h) lb += wp[h];
        if (w & kHasP)
          for (int h = rho + 1; h < C; ++h) lb += pt[h];
        atomicAdd(&L.partial[rho], lb);
      }
      __syncthreads();
      bool miss = false;
      for (int rho = lane; rho < C; rho += kWave) {
        if (L.partial[rho] + (double)((L.nrs[rho] & 0xffff) - 1) * hop > L.Dd[rho]) miss = true;
        L.partial[rho] = 0.0;
      }
      missed = wave_any(miss);
      __syncthreads();
    }
  }

  // ---- the queue of sub-chains: the Lemma 3 sub-chains first, each after
  //      every one it reads (by the number of higher-priority executors on
  //      their core, then rank), then those that read none of them
  //      (increasing position), then the others (decreasing position, written
  //      from the back); records (constant part of the recurrence,
  //      s | packed word) ----
  int n3 = 0;
  for (int l = 0; l <= maxlev; ++l) n3 += L.dmin[l];
  if (!missed) {
    int nl3 = 0, nind = 0, ndep = 0;
    for (int sb = 0; sb < nrun; sb += kWave) {
      const int s = sb + lane;
      int w = 0, cat = -1;  // 0: Lemma 3; 1: reads none of them; 2: other
      double c = 0.0;
      if (s < nrun) {
        w = S.info[s];
        c = S.cst[s];
        const int e = (w >> kExecShift) & 31;
        if (w & kNeedL3) cat = 0;
        else cat = ((w & kRankMask) <= L.dfirst[e] && !L.dblk[e]) ? 1 : 2;
      }
      const double2 rec = make_double2(c, pack2(s, w));
      const unsigned long long m3 = __ballot(cat == 0);
      const unsigned long long mi = __ballot(cat == 1);
      const unsigned long long md = __ballot(cat == 2);
      if (cat == 0) {
        // unsorted, into the free Lemma 2 queue (a Lemma 3 sub-chain has a
        // segment of its own, so there are at most as many as segments)
        const int i = nl3 + (int)__popcll(m3 & lanes_below());
        S.qs[i] = rec;
        S.alist[i] = (__popc((uint32_t)L.hpx[(w >> kExecShift) & 31]) << 12) | (w & kRankMask);
      }
      if (cat == 1) S.qr[n3 + nind + (int)__popcll(mi & lanes_below())] = rec;
      if (cat == 2) S.qr[nrun - 1 - (ndep + (int)__popcll(md & lanes_below()))] = rec;
      nl3 += (int)__popcll(m3);
      nind += (int)__popcll(mi);
      ndep += (int)__popcll(md);
    }
    __syncthreads();
    // the Lemma 3 sub-chains in key order (ties by position): each one's
    // place is the number of keys before it
    for (int ib = 0; ib < n3; ib += kWave) {
      const int i = ib + lane;
      const int ki = i < n3 ? S.alist[i] : 0x7fffffff;
      int pos = 0;
      for (int jb = 0; jb < n3; jb += kWave) {
        const int kv = jb + lane < n3 ? S.alist[jb + lane] : 0x7fffffff;
        const int jn = min(kWave, n3 - jb);
        for (int jj = 0; jj < jn; ++jj) {
          const int kj = __builtin_amdgcn_readlane(kv, jj);
          pos += (kj < ki || (kj == ki && jb + jj < i)) ? 1 : 0;
        }
      }
      if (i < n3) S.qr[pos] = S.qs[i];
    }
  }
  __syncthreads();

  // ---- Theorem 1 / Eq. (6): one sub-chain per lane, refilled from the
  //      queue; the next 64 records are loaded one step ahead ----
  if (!missed) {
    int qnext = 0;
    bool have = false;
    int s = 0, rho = 0, e = 0, inf1 = 0, hpxm = 0;
    double r = 0.0, cst = 0.0, hs = 0.0, L2v = 0.0, A0v = 0.0, epsv = 0.0, capv = 0.0;
    double2 win = make_double2(0.0, 0.0);
    if (lane < nrun) win = S.qr[lane];
    for (int step = 0;; ++step) {
      const unsigned long long need = __ballot(!have);
      const int k = (int)__popcll(need & lanes_below());
      const double wc = __shfl(win.x, k), wP = __shfl(win.y, k);
      if (!have && qnext + k < nrun) {
        s = __double2hiint(wP);
        inf1 = __double2loint(wP);
        rho = inf1 & kRankMask;
        e = (inf1 >> kExecShift) & 31;
        cst = wc;
        if (inf1 & kNeedL3) {
          L2v = S.L2[s];
          A0v = S.A0[s];
          epsv = S.eps[s];
        }
        hpxm = L.hpx[e];
        capv = L.Dd[rho] * capm;
        r = 0.0;
        hs = 0.0;
        have = true;
      }
      const bool l3live = qnext < n3;  // a Lemma 3 sub-chain was queued before this refill
      qnext += (int)__popcll(need);
      if (!wave_any(have)) break;
      if (qnext + lane < nrun) win = S.qr[qnext + lane];
      if (step >= kMaxIter) {
        if (lane == 0) L.misc[0] = 1;
        break;
      }
      const bool needL3 = have && (inf1 & kNeedL3) != 0;
      // Lemma 3 sub-chains not yet final: lowest rank and busy-waiting count
      // per executor (none once every one of them has left the lanes)
      bool blocked = false;
      if (l3live || wave_any(needL3)) {
        for (int x = lane; x < X; x += kWave) {
          L.dmin[x] = C;
          L.dspin[x] = 0;
        }
        wave_sync();
        if (needL3) {
          atomicMin(&L.dmin[e], rho);
          if (L.nrs[rho] >> 16) atomicAdd(&L.dspin[e], 1);
        }
        wave_sync();
        blocked = L.dmin[e] < rho;
        for (uint32_t m = (uint32_t)hpxm; m; m &= m - 1)
          if (L.dspin[__ffs(m) - 1] > 0) blocked = true;
      }

      const bool hasP = (inf1 & kHasP) != 0;
      const int hend = wave_umax(have ? (hasP ? C : rho) : 0);
      const int accm = (inf1 >> kAccShift) & 0xff;
      const double *wp = L.WP + e * C;
      const double *pt = L.Pt + e * C;
      const double *ah = L.Ahat;
      const bool l3on = needL3 && (accm & 1) != 0;
      int e_lo = 0, e_mid = 0;
      bool anyl3 = false;
      if (NA == 1) {
        // The Lemma 3 weight of h is A-hat[h] for a lane that needs Lemma 3
        // and ranks below h, else 0.  h splits into three ranges: below every
        // lane's rank (hp weight for all), between the smallest and largest
        // rank (per-lane selects), above every rank (hpp weight for all).
        const int rlo = wave_umin(have ? rho : C);
        const int rhi = wave_umax(have ? rho : -1);
        e_lo = rlo < hend ? rlo : hend;
        e_mid = rhi + 1 < hend ? rhi + 1 : hend;
        anyl3 = wave_any(l3on);
      }
      // up to `micro` evaluations with this step's items and weights
      double rr = r, hh = hs;
      bool conv = false;
      for (int it = 0; it < micro; ++it) {
        double I0 = 0.0, I1 = 0.0, l3 = 0.0;
        int h = 0;
        if (NA == 1) {
          if (!anyl3) {
#pragma unroll 2
            for (; h + 1 < e_lo; h += 2) {
              const double2 q0 = kr(h), q1 = kr(h + 1);
              I0 = fma(mu_term(rr, q0.x, q0.y), wp[h], I0);
              I1 = fma(mu_term(rr, q1.x, q1.y), wp[h + 1], I1);
            }
          } else {
#pragma unroll 2
            for (; h + 1 < e_lo; h += 2) {
              const double2 q0 = kr(h), q1 = kr(h + 1);
              const double m0 = mu_term(rr, q0.x, q0.y);
              const double m1 = mu_term(rr, q1.x, q1.y);
              const double av0 = ah[h], av1 = ah[h + 1];
              I0 = fma(m0, wp[h], I0);
              I1 = fma(m1, wp[h + 1], I1);
              l3 = fma(m0, l3on ? av0 : 0.0, l3);
              l3 = fma(m1, l3on ? av1 : 0.0, l3);
            }
          }
          if (h < e_lo) {
            const double2 q0 = kr(h);
            const double m0 = mu_term(rr, q0.x, q0.y);
            const double av0 = ah[h];
            I0 = fma(m0, wp[h], I0);
            l3 = fma(m0, l3on ? av0 : 0.0, l3);
            ++h;
          }
          for (; h + 1 < e_mid; h += 2) {
            const double2 q0 = kr(h), q1 = kr(h + 1);
            const double m0 = mu_term(rr, q0.x, q0.y);
            const double m1 = mu_term(rr, q1.x, q1.y);
            double w0 = (h < rho ? wp : pt)[h];
            double w1 = (h + 1 < rho ? wp : pt)[h + 1];
            w0 = h == rho ? 0.0 : w0;
            w1 = h + 1 == rho ? 0.0 : w1;
            const double av0 = ah[h], av1 = ah[h + 1];
            I0 = fma(m0, w0, I0);
            I1 = fma(m1, w1, I1);
            l3 = fma(m0, (l3on && h < rho) ? av0 : 0.0, l3);
            l3 = fma(m1, (l3on && h + 1 < rho) ? av1 : 0.0, l3);
          }
          if (h < e_mid) {
            const double2 q0 = kr(h);
            const double m0 = mu_term(rr, q0.x, q0.y);
            double w0 = (h < rho ? wp : pt)[h];
            w0 = h == rho ? 0.0 : w0;
            const double av0 = ah[h];
            I0 = fma(m0, w0, I0);
            l3 = fma(m0, (l3on && h < rho) ? av0 : 0.0, l3);
            ++h;
          }
#pragma unroll 2
          for (; h + 1 < hend; h += 2) {
            const double2 q0 = kr(h), q1 = kr(h + 1);
            I0 = fma(mu_term(rr, q0.x, q0.y), pt[h], I0);
            I1 = fma(mu_term(rr, q1.x, q1.y), pt[h + 1], I1);
          }
          if (h < hend) {
            const double2 q0 = kr(h);
            I0 = fma(mu_term(rr, q0.x, q0.y), pt[h], I0);
            ++h;
          }
        }
        for (; h < hend; ++h) {
          const double2 q0 = kr(h);
          const double m0 = mu_term(rr, q0.x, q0.y);
          double w0 = h < rho ? wp[h] : pt[h];
          w0 = h == rho ? 0.0 : w0;
          I0 = fma(m0, w0, I0);
          if (needL3 && h < rho) {
            double a0s = 0.0;
            for (int a = 0; a < NA; ++a)
              if ((accm >> a) & 1) a0s += L.Ahat[a * C + h];
            l3 = fma(m0, a0s, l3);
          }
        }
        if (have && !isinf(rr)) {
          double hsn = hh;
          if (needL3) {
            const double L3 = A0v + l3;
            hsn = (o.bound == PAAM_BOUND_L3 ? L3 : fmin(L2v, L3)) + epsv;
          }
          double rn = cst + hsn + (I0 + I1);
          if (rn > capv) {
            rn = INFINITY;
            if (needL3) {
              // Lemma 3 at an unbounded window: unbounded iff an HP request of
              // positive length can interfere (then l3 > 0 already)
              const double L3i = l3 > 0.0 ? INFINITY : A0v;
              hsn = (o.bound == PAAM_BOUND_L3 ? L3i : fmin(L2v, L3i)) + epsv;
            }
          }
          conv = rn == rr;
          rr = rn;
          hh = hsn;
        }
        if (!wave_any(have && !conv && !isinf(rr))) break;
      }
      if (have) {
        if (hh != hs) {
          // H* of the chain on e enters its hp weight on e and, for a
          // busy-waiting chain, the hp and hpp weights on the core's
          // lower-priority executors
          const double dh = hh - hs;
          atomicAdd(&L.WP[e * C + rho], dh);
          if (L.nrs[rho] >> 16) {
            for (uint32_t m = (uint32_t)L.lpx[e]; m; m &= m - 1) {
              const int e2 = __ffs(m) - 1;
              atomicAdd(&L.WP[e2 * C + rho], dh);
              atomicAdd(&L.Pt[e2 * C + rho], dh);
            }
          }
        }
        if (rr != r) atomicAdd(&L.partial[rho], rr - r);
        const bool fin = isinf(rr) || (conv && !blocked);
        r = rr;
        hs = hh;
        if (fin) have = false;
      }
      wave_sync();
      if (!full) {
        // every iterate is a lower bound: a partial end-to-end sum above the
        // deadline proves the miss
        const bool miss = L.partial[rho] + (double)((L.nrs[rho] & 0xffff) - 1) * hop > L.Dd[rho];
        if (wave_any(miss)) {
          missed = true;
          break;
        }
      }
    }
  }

  // ---- end-to-end bounds, verdict, worst chain ----
  const bool guard = L.misc[0] != 0;
  bool ok = !missed;
  if (!missed) {
    bool late = false;
    for (int rho = lane; rho < C; rho += kWave) {
      double R = L.partial[rho] + (double)((L.nrs[rho] & 0xffff) - 1) * hop;
      if (R > L.Dd[rho] * capm || guard) R = INFINITY;
      L.partial[rho] = R;
      if (R > L.Dd[rho]) late = true;
    }
    ok = !wave_any(late);
  }
  __syncthreads();
  if (!missed && full && chain_R) {
    for (int c = lane; c < C; c += kWave) {
      const double R = L.partial[L.rank[c]];
      chain_R[c0 + c] = isinf(R) ? PAAM_INF : (int64_t)R;
    }
  }
  // worst chain: the largest R/D (exact cross-multiplication), ties to the
  // lowest chain index; each lane scans its chains, then a wave reduction
  int32_t w = -1;
  double wRd = 0.0;
  int64_t wD = 1;
  if (!missed && !guard && (ok || full)) {
    for (int c = lane; c < C; c += kWave) {
      const double R = L.partial[L.rank[c]];
      const int64_t D = b.D[c0 + c];
      if (w < 0 || ratio_gt(R, D, wRd, wD)) {
        w = c;
        wRd = R;
        wD = D;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const int w2 = __shfl_xor(w, off);
      const double R2 = __shfl_xor(wRd, off);
      const int64_t D2 = __shfl_xor(wD, off);
      bool take = false;
      if (w2 >= 0) {
        if (w < 0 || ratio_gt(R2, D2, wRd, wD)) take = true;
        else if (!ratio_gt(wRd, wD, R2, D2) && w2 < w) take = true;
      }
      if (take) {
        w = w2;
        wRd = R2;
        wD = D2;
      }
    }
  }
  if (lane == 0) {
    const int64_t wR = (w < 0 || isinf(wRd)) ? PAAM_INF : (int64_t)wRd;
    set_sched[set] = guard ? -1 : (ok ? 1 : 0);
    set_worst[set] = w;
    set_worst_R[set] = wR;
  }
  __syncthreads();
}

__global__ void reset_counter(unsigned long long *counter) { *counter = 0ull; }

// The analysis under the uploaded priorities: the (2T-1, 1/T) table is read
// from the arena, the blocking table lives in the wave's global scratch, so a
// wave needs only the LDS tables of the iteration.
// Instantiated per mode: every chain's bound (kFull) or the verdict alone,
// so each compiles without the other's code.
template <bool kFull>
__global__ __launch_bounds__(kWave, 5) void wcrt_kernel(WcrtLaunch L) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  Lds l = carve_lds(lds_raw, L.b.max_C, L.b.max_X, L.b.max_NA > 0 ? L.b.max_NA : 1, false, false);
  Scratch s = carve_scratch(L.scratch + (size_t)blockIdx.x * L.scratch_stride, L.b.max_segs,
                            L.b.max_runs, L.b.max_C, L.b.max_X, true);
  // lane 0 claims queue positions; the index is then held in scalar
  // registers, so every branch on it is uniform across the wave.  The next
  // position is claimed before the current set is analysed.
  unsigned long long inext = 0;
  if (threadIdx.x == 0) inext = atomicAdd(L.counter, 1ull);
  inext = uniform_u64(inext);
  for (;;) {
    const unsigned long long i = inext;
    if (i >= (unsigned long long)L.b.n_sets) break;
    unsigned long long in2 = 0;
    if (threadIdx.x == 0) in2 = atomicAdd(L.counter, 1ull);
    inext = uniform_u64(in2);
    const int64_t set = L.b.work_order[i];
    const int64_t c0 = L.b.set_chain_off[set];
    KRConst kr{(const __attribute__((address_space(4))) double *)(L.b.KRr + 2 * c0)};
    analyse_set_q<KRConst, false, kFull>(L.b, L.o, set, kr, l, s, L.set_sched, L.set_worst,
                                   L.set_worst_R, L.chain_R, L.micro);
  }
}

// ---------------------------- priority search ------------------------------

// Per-wave search state after the analysis scratch: the verdict slot, the
// candidate order (chain at each rank), the ranks of the chains, the selected
// candidates of a guided search and the walk's step buffer.
constexpr int kMaxTopK = 1024;

struct SearchSlot {
  int64_t *worst_R;  // [1]
  int32_t *worst;    // [1]
  int8_t *sched;     // [1]
  int32_t *order;    // [max_C]
  int16_t *rank;     // [max_C]
  int32_t *sel;      // [kMaxTopK]
  int32_t *buf;      // [64]
};

__host__ __device__ inline size_t slot_sel_offset(int Cm) {
  return (16 + 6 * (size_t)Cm + 15) & ~(size_t)15;
}

__device__ SearchSlot carve_slot(unsigned char *base, int Cm) {
  SearchSlot q;
  q.worst_R = reinterpret_cast<int64_t *>(base);
  q.worst = reinterpret_cast<int32_t *>(base + 8);
  q.sched = reinterpret_cast<int8_t *>(base + 12);
  q.order = reinterpret_cast<int32_t *>(base + 16);
  q.rank = reinterpret_cast<int16_t *>(base + 16 + 4 * (size_t)Cm);
  q.sel = reinterpret_cast<int32_t *>(base + slot_sel_offset(Cm));
  q.buf = q.sel + kMaxTopK;
  return q;
}

// The uploaded order of a set (candidate 0) into the slot.
__device__ void base_order(const DevBatch &b, int64_t c0, int C, SearchSlot &q) {
  for (int c = threadIdx.x; c < C; c += kWave) {
    const int r = b.rank0[c0 + c];
    q.order[r] = c;
    q.rank[c] = (int16_t)r;
  }
  __syncthreads();
}

// Score key: ascending score in IEEE total order (-0 before +0, every NaN
// last), ties to the lower candidate index.
__device__ __forceinline__ uint64_t score_key(float f, int k) {
  uint32_t u = __float_as_uint(f);
  if (isnan(f)) {
    u = 0xFFFFFFFFu;
  } else {
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  }
  return ((uint64_t)u << 32) | (uint32_t)k;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o);
    v = w < v ? w : v;
  }
  return v;
}

// Priority-order search.  Each candidate is analysed by analyse_set in verdict
// mode, reading the candidate's ranks through the batch's rank table.
// Plain: candidates 0, 1, ... in index order; the first feasible is the
// smallest feasible k.  Guided: the top_k candidates by score in score order,
// then (with fallback) the others in index order.
template <bool kSbLds>
__global__ __launch_bounds__(kWave) void search_kernel(SearchLaunch L) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  Lds l = carve_lds(lds_raw, L.b.max_C, L.b.max_X, L.b.max_NA > 0 ? L.b.max_NA : 1, true, kSbLds);
  unsigned char *wbase = L.scratch + (size_t)blockIdx.x * L.scratch_stride;
  Scratch s = carve_scratch(wbase, L.b.max_segs, L.b.max_runs, L.b.max_C, L.b.max_X, !kSbLds);
  SearchSlot q = carve_slot(wbase + L.analysis_stride, L.b.max_C);
  paam_wcrt_opts o = L.o.wcrt;
  o.full = 0;
  const int n_cand = L.o.n_cand;
  for (;;) {
    // lane 0 claims the next set; the index is then held in scalar registers,
    // so every branch on it is uniform across the wave
    unsigned long long i = 0;
    if (threadIdx.x == 0) i = atomicAdd(L.counter, 1ull);
    i = uniform_u64(i);
    if (i >= (unsigned long long)L.b.n_sets) break;
    const int64_t set = L.b.work_order[i];
    const int64_t c0 = L.b.set_chain_off[set];
    const int C = (int)(L.b.set_chain_off[set + 1] - c0);
    base_order(L.b, c0, C, q);
    // the analysis reads rank0[c0 + c]: point it at this wave's candidate ranks
    DevBatch bq = L.b;
    bq.rank0 = q.rank - c0;
    int found = -1, n_eval = 0;
    // the miss check before Lemma 2 is tried until it first fails on the set
    // (on sets whose candidates it does not reject, it is work on top)
    bool early = true;
    int64_t cur = 0;  // candidate the slot's order holds
    if (L.o.guided) {
      const float *sc = L.o.d_scores + set * (int64_t)n_cand;
      const int K = L.o.top_k < n_cand ? L.o.top_k : n_cand;
      // the K smallest keys, in increasing order; up to 1,024 candidates the
      // keys are read once into registers (16 per lane)
      uint64_t prev = 0;
      if (n_cand <= 16 * kWave) {
        uint64_t keys[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int k = threadIdx.x + kWave * j;
          keys[j] = k < n_cand ? score_key(sc[k], k) : ~0ull;
        }
        for (int t = 0; t < K; ++t) {
          uint64_t best = ~0ull;
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if ((t == 0 || keys[j] > prev) && keys[j] < best) best = keys[j];
          best = wave_min_u64(best);
          if (threadIdx.x == 0) q.sel[t] = (int32_t)(uint32_t)best;
          prev = best;
        }
      } else {
        for (int t = 0; t < K; ++t) {
          uint64_t best = ~0ull;
          for (int k = threadIdx.x; k < n_cand; k += kWave) {
            const uint64_t key = score_key(sc[k], k);
            if ((t == 0 || key > prev) && key < best) best = key;
          }
          best = wave_min_u64(best);
          if (threadIdx.x == 0) q.sel[t] = (int32_t)(uint32_t)best;
          prev = best;
        }
      }
      __syncthreads();
      for (int t = 0; t < K; ++t) {
        const int k = q.sel[t];
        if (k < cur) {
          base_order(L.b, c0, C, q);
          cur = 0;
        }
        walk_order(q.order, q.rank, C, L.o.seed, set, cur, k, q.buf);
        cur = k;
        if (!analyse_set<kSbLds>(bq, o, set, l, s, q.sched - set, q.worst - set, q.worst_R - set,
                                 nullptr, early))
          early = false;
        ++n_eval;
        int v = 0;
        if (threadIdx.x == 0) v = q.sched[0];  // written by lane 0 of analyse_set
        v = __shfl(v, 0);
        if (v != 0) {
          found = v > 0 ? k : -2;
          break;
        }
      }
      if (found == -1 && L.o.fallback) {
        for (int k = 0; k < n_cand; ++k) {
          bool in = false;
          for (int t = threadIdx.x; t < K; t += kWave) in |= q.sel[t] == k;
          if (__any(in)) continue;
          if (k < cur) {
            base_order(L.b, c0, C, q);
            cur = 0;
          }
          walk_order(q.order, q.rank, C, L.o.seed, set, cur, k, q.buf);
          cur = k;
          if (!analyse_set<kSbLds>(bq, o, set, l, s, q.sched - set, q.worst - set,
                                   q.worst_R - set, nullptr, early))
            early = false;
          ++n_eval;
          int v = 0;
          if (threadIdx.x == 0) v = q.sched[0];
          v = __shfl(v, 0);
          if (v != 0) {
            found = v > 0 ? k : -2;
            break;
          }
        }
      }
    } else {
      for (int k = 0; k < n_cand; ++k) {
        walk_order(q.order, q.rank, C, L.o.seed, set, cur, k, q.buf);
        cur = k;
        if (!analyse_set<kSbLds>(bq, o, set, l, s, q.sched - set, q.worst - set, q.worst_R - set,
                                 nullptr, early))
          early = false;
        ++n_eval;
        int v = 0;
        if (threadIdx.x == 0) v = q.sched[0];
        v = __shfl(v, 0);
        if (v != 0) {
          found = v > 0 ? k : -2;
          break;
        }
      }
    }
    if (threadIdx.x == 0) {
      L.found[set] = found;
      L.n_exact[set] = n_eval;
    }
    if (L.found_prio && found >= 0)
      for (int r = threadIdx.x; r < C; r += kWave) L.found_prio[c0 + q.order[r]] = C - r;
    __syncthreads();
  }
}

// Exact analysis of explicit (set, k, util_permille) candidates: every
// chain's bound at cap_mult * D, reduced to the worst chain and its ratio.
template <bool kSbLds>
__global__ __launch_bounds__(kWave) void candidate_kernel(CandLaunch L) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  Lds l = carve_lds(lds_raw, L.b.max_C, L.b.max_X, L.b.max_NA > 0 ? L.b.max_NA : 1, true, kSbLds);
  unsigned char *wbase = L.scratch + (size_t)blockIdx.x * L.scratch_stride;
  Scratch s = carve_scratch(wbase, L.b.max_segs, L.b.max_runs, L.b.max_C, L.b.max_X, !kSbLds);
  SearchSlot q = carve_slot(wbase + L.analysis_stride, L.b.max_C);
  // Grid-stride over the pairs: the item index derives from blockIdx only, so
  // it is wave-uniform by construction.  (With a lane-0 queue fetch, the path
  // that skips a malformed pair was split by the compiler into a loop that
  // lanes 1..63 never leave.)
  for (int64_t i = blockIdx.x; i < L.n_pairs; i += gridDim.x) {
    const int64_t set = L.pairs[3 * i], k = L.pairs[3 * i + 1], u = L.pairs[3 * i + 2];
    if (set < 0 || set >= L.b.n_sets || k < 0 || k > 0x7FFFFFFF || u < 0 || u > 0x7FFFFFFF) {
      if (threadIdx.x == 0) {
        L.sched[i] = -2;
        L.worst_R[i] = PAAM_INF;
        L.worst_D[i] = 0;
        if (L.ratio) L.ratio[i] = (float)L.o.cap_mult;
      }
      continue;
    }
    const int64_t c0 = L.b.set_chain_off[set];
    const int C = (int)(L.b.set_chain_off[set + 1] - c0);
    base_order(L.b, c0, C, q);
    walk_order(q.order, q.rank, C, L.seed, set, 0, k, q.buf);
    DevBatch bq = L.b;
    bq.rank0 = q.rank - c0;
    paam_wcrt_opts o = L.o;
    o.full = 1;
    o.util_permille = (int32_t)u;
    analyse_set<kSbLds>(bq, o, set, l, s, q.sched - set, q.worst - set, q.worst_R - set, nullptr,
                        false);
    if (threadIdx.x == 0) {
      const int w = q.worst[0];
      const int64_t wR = q.worst_R[0];
      const int64_t D = L.b.D[c0 + (w < 0 ? 0 : w)];
      L.sched[i] = q.sched[0];
      L.worst_R[i] = wR;
      L.worst_D[i] = D;
      if (L.ratio) {
        const double cap = (double)L.o.cap_mult;
        double r = wR == PAAM_INF ? cap : (double)wR / (double)D;
        L.ratio[i] = (float)(r < cap ? r : cap);
      }
    }
    __syncthreads();
  }
}

}  // namespace

static size_t scratch_bytes(const DevBatch &b, bool sb_scratch) {
  size_t n = (size_t)b.max_segs * 4 * sizeof(double) + (size_t)b.max_runs * 8 * sizeof(double) +
             (size_t)b.max_runs * 2 * sizeof(int32_t) + 16;
  if (sb_scratch) n += (size_t)b.max_X * b.max_C * sizeof(double);
  return (n + 255) & ~(size_t)255;
}

static size_t lds_bytes(const DevBatch &b, bool with_kr, bool sb_lds) {
  const size_t Cm = b.max_C, Xm = b.max_X, NAm = b.max_NA > 0 ? b.max_NA : 1;
  const size_t d = (with_kr ? 2 * Cm : 0) + 2 * Cm + 2 * NAm * Cm + 2 * Xm * Cm +
                   (sb_lds ? Xm * Cm : 0) + 2 * NAm;
  return 8 * d + 4 * (2 * Cm + NAm * Cm + 10 * Xm + 16);
}

size_t wave_scratch_bytes(const DevBatch &b) {
  return scratch_bytes(b, sb_in_scratch(b.max_C, b.max_X));
}

size_t wave_search_bytes(const DevBatch &b) {
  const size_t slot = slot_sel_offset(b.max_C) + 4 * (size_t)(kMaxTopK + 64);
  return wave_scratch_bytes(b) + ((slot + 255) & ~(size_t)255);
}

size_t wave_lds_bytes(const DevBatch &b) {
  return lds_bytes(b, true, !sb_in_scratch(b.max_C, b.max_X));
}

size_t wcrt_scratch_bytes(const DevBatch &b) { return scratch_bytes(b, true); }

size_t wcrt_lds_bytes(const DevBatch &b) { return lds_bytes(b, false, false); }

int launch_wcrt(const WcrtLaunch &L, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, st, L.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  if (L.b.n_sets == 0) return 0;
  if (L.o.full)
    hipLaunchKernelGGL(wcrt_kernel<true>, dim3(L.grid), dim3(kWave), L.lds_bytes, st, L);
  else
    hipLaunchKernelGGL(wcrt_kernel<false>, dim3(L.grid), dim3(kWave), L.lds_bytes, st, L);
  return (int)hipGetLastError();
}

int launch_candidates(const CandLaunch &L, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (L.n_pairs == 0) return 0;
  if (sb_in_scratch(L.b.max_C, L.b.max_X))
    hipLaunchKernelGGL(candidate_kernel<false>, dim3(L.grid), dim3(kWave), L.lds_bytes, st, L);
  else
    hipLaunchKernelGGL(candidate_kernel<true>, dim3(L.grid), dim3(kWave), L.lds_bytes, st, L);
  return (int)hipGetLastError();
}

int launch_search(const SearchLaunch &L, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, st, L.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  if (L.b.n_sets == 0) return 0;
  if (sb_in_scratch(L.b.max_C, L.b.max_X))
    hipLaunchKernelGGL(search_kernel<false>, dim3(L.grid), dim3(kWave), L.lds_bytes, st, L);
  else
    hipLaunchKernelGGL(search_kernel<true>, dim3(L.grid), dim3(kWave), L.lds_bytes, st, L);
  return (int)hipGetLastError();
}

namespace {
std::mutex g_scratch_mutex;
void *g_scratch_dev[kMaxDevices];  // address of `scratch` on each device
}  // namespace

}  // namespace paam

// Scratch of paam_wcrt_batch_noalloc, for callers that cannot allocate: every
// GPU the library runs on holds one copy until the process ends.  In host
// code this name is a host-side stand-in; kernels and copies use the device
// address that hipGetSymbolAddress returns on each device.
static __device__ __attribute__((aligned(256))) unsigned char scratch[paam::kNoAllocScratchBytes];

namespace paam {

int noalloc_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return 0;
}

}  // namespace paam
