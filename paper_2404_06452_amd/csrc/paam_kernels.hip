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
// decreasing estimated cost.  Lanes run over segments (Lemma 2), then over the
// sub-chains of one executor at a time (Theorem 1).  Executors of a core are
// solved from the highest process priority down, so the hpp weights of
// Theorem 1 are final when an executor starts; inside an executor all
// sub-chains iterate together (Jacobi) until no value changes.  Every
// iteration starts below the least fixed point and is monotone, so the
// result is the same least fixed point a sequential evaluation reaches.
#include <hip/hip_runtime.h>
#include <math.h>

#include "paam_internal.h"

namespace paam {
namespace {

__device__ __forceinline__ double mu_term(double t, double K, double rcp) {
  return __builtin_floor((t + K) * rcp);
}

__device__ __forceinline__ double scale_time(int64_t x, int32_t u) {
  return (double)(u == 1000 ? x : (x * (int64_t)u) / 1000);
}

__device__ __forceinline__ void lds_max(double *p, double v) {
  // non-negative doubles (and +inf) order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ int wave_any(bool p) { return __any(p); }

__device__ __forceinline__ int wave_min_int(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max_int(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
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

struct Lds {
  double *K, *rc, *cap, *Dd, *partial, *W, *Wn, *P, *Hs;  // [C] by rank
  double *Ahat, *amax, *Bacc;                             // [NA][C]
  double *Ece, *epsce, *SB, *Hfin;                        // [X][C]
  int32_t *perm, *rank, *nrun, *spinf;                    // [C]
  int32_t *level, *uses;                                  // [NA][C]
  int32_t *misc;                                          // [16]
};

struct Scratch {
  double *segAs, *segH;                          // [max_segs]
  double *r, *hs, *cst, *L2, *A0, *eps;          // [max_runs]
  int32_t *info0, *info1;                        // [max_runs]
};

__device__ Lds carve_lds(unsigned char *base, int Cm, int Xm, int NAm) {
  Lds l;
  double *d = reinterpret_cast<double *>(base);
  l.K = d; d += Cm;
  l.rc = d; d += Cm;
  l.cap = d; d += Cm;
  l.Dd = d; d += Cm;
  l.partial = d; d += Cm;
  l.W = d; d += Cm;
  l.Wn = d; d += Cm;
  l.P = d; d += Cm;
  l.Hs = d; d += Cm;
  l.Ahat = d; d += NAm * Cm;
  l.amax = d; d += NAm * Cm;
  l.Bacc = d; d += NAm * Cm;
  l.Ece = d; d += Xm * Cm;
  l.epsce = d; d += Xm * Cm;
  l.SB = d; d += Xm * Cm;
  l.Hfin = d; d += Xm * Cm;
  int32_t *i = reinterpret_cast<int32_t *>(d);
  l.perm = i; i += Cm;
  l.rank = i; i += Cm;
  l.nrun = i; i += Cm;
  l.spinf = i; i += Cm;
  l.level = i; i += NAm * Cm;
  l.uses = i; i += NAm * Cm;
  l.misc = i;
  return l;
}

__device__ Scratch carve_scratch(unsigned char *base, int max_segs, int max_runs) {
  Scratch s;
  double *d = reinterpret_cast<double *>(base);
  s.segAs = d; d += max_segs;
  s.segH = d; d += max_segs;
  s.r = d; d += max_runs;
  s.hs = d; d += max_runs;
  s.cst = d; d += max_runs;
  s.L2 = d; d += max_runs;
  s.A0 = d; d += max_runs;
  s.eps = d; d += max_runs;
  int32_t *i = reinterpret_cast<int32_t *>(d);
  s.info0 = i; i += max_runs;
  s.info1 = i;
  return s;
}

// Every recurrence is monotone from below and bounded by its cap, so it
// stops; the guard only makes termination unconditional.  A set that trips it
// reports set_sched = -1.
constexpr int kMaxIter = 1 << 20;

constexpr int kNeedL3 = 1 << 8;
constexpr int kConv = 1 << 9;
constexpr int kHasSeg = 1 << 10;

// Analyses set `set` under the priority order perm (chain ids, highest
// first) if given, else under the uploaded priorities.  Writes the outputs
// of that set.  Called by all 64 lanes of a wave.
__device__ void analyse_set(const DevBatch &b, const paam_wcrt_opts &o, int64_t set, Lds &L,
                            Scratch &S, int8_t *set_sched, int32_t *set_worst,
                            int64_t *set_worst_R, int64_t *chain_R) {
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

  // ---- chain tables in rank order (rank 0 = highest priority) ----
  for (int c = lane; c < C; c += kWave) {
    const int rho = b.rank0[c0 + c];
    L.perm[rho] = c;
    L.rank[c] = rho;
    L.K[rho] = b.Kd[c0 + c];
    L.rc[rho] = b.rcp[c0 + c];
    const int64_t D = b.D[c0 + c];
    L.Dd[rho] = (double)D;
    L.cap[rho] = (double)D * (double)o.cap_mult;
    L.nrun[rho] = b.chain_nrun[c0 + c];
    L.spinf[rho] = b.spin[c0 + c];
    L.partial[rho] = 0.0;
  }
  for (int i = lane; i < NA * C; i += kWave) {
    L.Ahat[i] = 0.0;
    L.amax[i] = 0.0;
    L.uses[i] = 0;
  }
  for (int i = lane; i < X * C; i += kWave) {
    L.Ece[i] = 0.0;
    L.epsce[i] = 0.0;
    L.SB[i] = 0.0;
    L.Hfin[i] = 0.0;
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
    lds_max(&L.amax[a * C + rho], As);
    L.uses[a * C + rho] = 1;
  }
  __syncthreads();

  // ---- buckets (Sec. IV-C): users of an accelerator by priority, rank r of m
  //      in level floor(r*n/m); then the LP same-bucket maximum of Eq. (3) ----
  for (int rho = lane; rho < C; rho += kWave) {
    for (int a = 0; a < NA; ++a) {
      int lev = -1;
      if (L.uses[a * C + rho]) {
        int r = 0, m = 0;
        for (int h = 0; h < C; ++h) {
          const int us = L.uses[a * C + h];
          m += us;
          r += (us && h < rho) ? 1 : 0;
        }
        lev = (int)(((int64_t)r * b.buckets[a0 + a]) / m);
      }
      L.level[a * C + rho] = lev;
    }
  }
  __syncthreads();
  for (int rho = lane; rho < C; rho += kWave) {
    for (int a = 0; a < NA; ++a) {
      double bm = 0.0;
      const int lev = L.level[a * C + rho];
      if (lev >= 0) {
        for (int h = rho + 1; h < C; ++h)
          if (L.level[a * C + h] == lev) bm = fmax(bm, L.amax[a * C + h]);
      }
      L.Bacc[a * C + rho] = bm;
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
      capv = L.cap[rho];
    }
    double h = 0.0;
    bool done = !valid;
    for (int it = 0; wave_any(!done); ++it) {
      if (it >= kMaxIter) {
        if (!done) L.misc[0] = 1;
        break;
      }
      if (!done) {
        double nxt = base;
        const double *Ah = L.Ahat + a * C;
        for (int k = 0; k < rho; ++k) nxt = fma(mu_term(h, L.K[k], L.rc[k]), Ah[k], nxt);
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

  // ---- sub-chains, pass A: own demand, Lemma 2 sum, Lemma 3 constant,
  //      overheads, and each callback as a blocking candidate ----
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
    lds_max(&L.SB[e * C + rho], bmax);
    atomicAdd(&L.Ece[e * C + rho], E);
    atomicAdd(&L.epsce[e * C + rho], eps);
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
    S.r[s] = 0.0;
    S.hs[s] = hs0;
    S.cst[s] = E;  // blocking added in pass B
    S.L2[s] = L2;
    S.A0[s] = A0;
    S.eps[s] = eps;
    S.info0[s] = rho | (e << 16);
    S.info1[s] = accm | (needL3 ? kNeedL3 : 0) | (delta > 0 ? kHasSeg : 0);
  }
  __syncthreads();
  // suffix maximum of blocking candidates per executor, lowest priority up
  for (int e = lane; e < X; e += kWave) {
    double m = 0.0;
    for (int rho = C - 1; rho >= 0; --rho) {
      m = fmax(m, L.SB[e * C + rho]);
      L.SB[e * C + rho] = m;
    }
  }
  __syncthreads();
  // pass B: blocking by one callback of a lower priority chain on the executor
  for (int s = lane; s < nrun; s += kWave) {
    const int rho = S.info0[s] & 0xffff;
    const int e = S.info0[s] >> 16;
    const double B = rho + 1 < C ? L.SB[e * C + rho + 1] : 0.0;
    S.cst[s] += B;
  }
  __syncthreads();

  // ---- Theorem 1 / Eq. (6), executor by executor ----
  bool missed = false;
  for (int xi = 0; xi < X && !missed; ++xi) {
    const int e = b.exec_seq[x0 + xi];
    const int ne = b.er_cnt[x0 + e];
    if (ne == 0) continue;
    const int32_t *runs = b.exec_runs + run0 + b.er_off[x0 + e];
    const uint32_t hpx = b.hpx_mask[x0 + e];
    const bool hasP = hpx != 0;
    // hpp weights: E + spin() summed over the higher executors of the core
    for (int rho = lane; rho < C; rho += kWave) {
      double p = 0.0;
      for (int e2 = 0; e2 < X; ++e2) {
        if (!((hpx >> e2) & 1u)) continue;
        const double sp = L.spinf[rho] ? L.Hfin[e2 * C + rho] : L.epsce[e2 * C + rho];
        p += L.Ece[e2 * C + rho] + sp;
      }
      L.P[rho] = p;
      L.W[rho] = -1.0;  // forces the first comparison to see a change
    }
    __syncthreads();
    // largest rank among the executor's sub-chains bounds the hp loop
    int maxrho = 0;
    for (int i = lane; i < ne; i += kWave) maxrho = max(maxrho, S.info0[runs[i]] & 0xffff);
    maxrho = wave_max_int(maxrho);

    for (int sweep = 0;; ++sweep) {
      if (sweep >= kMaxIter) {
        if (lane == 0) L.misc[0] = 1;
        break;
      }
      // W = E + H* of every chain on this executor at the current iterates
      for (int rho = lane; rho < C; rho += kWave) L.Hs[rho] = 0.0;
      __syncthreads();
      for (int i = lane; i < ne; i += kWave) {
        const int s = runs[i];
        atomicAdd(&L.Hs[S.info0[s] & 0xffff], S.hs[s]);
      }
      __syncthreads();
      int wchg = C;
      for (int rho = lane; rho < C; rho += kWave) {
        const double w = L.Ece[e * C + rho] + L.Hs[rho];
        if (w != L.W[rho]) wchg = min(wchg, rho);
        L.Wn[rho] = w;
      }
      wchg = wave_min_int(wchg);
      __syncthreads();
      for (int rho = lane; rho < C; rho += kWave) L.W[rho] = L.Wn[rho];
      __syncthreads();

      bool any_active = false;
      for (int ib = 0; ib < ne; ib += kWave) {
        const int i = ib + lane;
        int s = -1, rho = 0, inf1 = 0;
        double r = 0.0;
        bool active = false;
        if (i < ne) {
          s = runs[i];
          rho = S.info0[s] & 0xffff;
          inf1 = S.info1[s];
          r = S.r[s];
          active = !isinf(r) && (!(inf1 & kConv) || rho > wchg);
        }
        if (!wave_any(active)) continue;
        any_active = true;
        const bool needL3 = (inf1 & kNeedL3) != 0;
        const int accm = inf1 & 0xff;
        double I = 0.0, l3 = 0.0;
        const int hend = hasP ? C : maxrho;
        for (int h = 0; h < hend; ++h) {
          const double m = mu_term(r, L.K[h], L.rc[h]);
          if (h < rho) {
            I = fma(m, L.W[h], I);
            if (needL3) {
              double ah = 0.0;
              for (int a = 0; a < NA; ++a)
                if ((accm >> a) & 1) ah += L.Ahat[a * C + h];
              l3 = fma(m, ah, l3);
            }
          }
          if (hasP && h != rho) I = fma(m, L.P[h], I);
        }
        if (active) {
          double hsn = S.hs[s];
          if (needL3) {
            const double L3 = S.A0[s] + l3;
            hsn = (o.bound == PAAM_BOUND_L3 ? L3 : fmin(S.L2[s], L3)) + S.eps[s];
          }
          double rn = S.cst[s] + hsn + I;
          if (rn > L.cap[rho]) {
            rn = INFINITY;
            if (needL3) {
              // Lemma 3 at an unbounded window: unbounded iff an HP request
              // of positive length can interfere (then l3 > 0 already)
              const double L3i = l3 > 0.0 ? INFINITY : S.A0[s];
              hsn = (o.bound == PAAM_BOUND_L3 ? L3i : fmin(S.L2[s], L3i)) + S.eps[s];
            }
          }
          S.info1[s] = (inf1 & ~kConv) | (rn == r ? kConv : 0);
          S.r[s] = rn;
          S.hs[s] = hsn;
        }
      }
      __syncthreads();
      if (!any_active && wchg == C && sweep > 0) break;
    }

    // the executor is solved: H* per chain on it, partial end-to-end sums
    for (int rho = lane; rho < C; rho += kWave) L.Hfin[e * C + rho] = L.Hs[rho];
    for (int i = lane; i < ne; i += kWave) {
      const int s = runs[i];
      atomicAdd(&L.partial[S.info0[s] & 0xffff], S.r[s]);
    }
    __syncthreads();
    if (!full) {
      bool miss = false;
      for (int rho = lane; rho < C; rho += kWave) {
        const double lb = L.partial[rho] + (double)(L.nrun[rho] - 1) * hop;
        if (lb > L.Dd[rho]) miss = true;
      }
      missed = wave_any(miss);
    }
  }

  // ---- end-to-end bounds, verdict, worst chain ----
  bool ok = !missed;
  if (!missed) {
    bool late = false;
    for (int rho = lane; rho < C; rho += kWave) {
      double R = L.partial[rho] + (double)(L.nrun[rho] - 1) * hop;
      if (R > L.cap[rho]) R = INFINITY;
      L.partial[rho] = R;
      if (R > L.Dd[rho]) late = true;
      if (full && chain_R) chain_R[c0 + L.perm[rho]] = isinf(R) ? PAAM_INF : (int64_t)R;
    }
    ok = !wave_any(late);
  }
  __syncthreads();
  if (lane == 0) {
    int32_t w = -1;
    int64_t wR = PAAM_INF;
    if (!missed && (ok || full)) {
      for (int c = 0; c < C; ++c) {
        const int rho = L.rank[c];
        if (w < 0) {
          w = c;
          continue;
        }
        const int rw = L.rank[w];
        if (ratio_gt(L.partial[rho], b.D[c0 + c], L.partial[rw], b.D[c0 + w])) w = c;
      }
      const double R = L.partial[L.rank[w]];
      wR = isinf(R) ? PAAM_INF : (int64_t)R;
    }
    set_sched[set] = L.misc[0] ? -1 : (ok ? 1 : 0);
    set_worst[set] = w;
    set_worst_R[set] = wR;
  }
  __syncthreads();
}

__global__ void reset_counter(unsigned long long *counter) { *counter = 0ull; }

__global__ __launch_bounds__(kWave) void wcrt_kernel(WcrtLaunch L) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  Lds l = carve_lds(lds_raw, L.b.max_C, L.b.max_X, L.b.max_NA > 0 ? L.b.max_NA : 1);
  Scratch s = carve_scratch(L.scratch + (size_t)blockIdx.x * L.scratch_stride, L.b.max_segs,
                            L.b.max_runs);
  for (;;) {
    unsigned long long i = 0;
    if (threadIdx.x == 0) i = atomicAdd(L.counter, 1ull);
    i = __shfl(i, 0);
    if (i >= (unsigned long long)L.b.n_sets) break;
    const int64_t set = L.b.work_order[i];
    analyse_set(L.b, L.o, set, l, s, L.set_sched, L.set_worst, L.set_worst_R, L.chain_R);
  }
}

}  // namespace

size_t wave_scratch_bytes(const DevBatch &b) {
  size_t n = (size_t)b.max_segs * 2 * sizeof(double) + (size_t)b.max_runs * 6 * sizeof(double) +
             (size_t)b.max_runs * 2 * sizeof(int32_t);
  return (n + 255) & ~(size_t)255;
}

size_t wave_lds_bytes(const DevBatch &b) {
  const size_t Cm = b.max_C, Xm = b.max_X, NAm = b.max_NA > 0 ? b.max_NA : 1;
  return 8 * (9 * Cm + 3 * NAm * Cm + 4 * Xm * Cm) + 4 * (4 * Cm + 2 * NAm * Cm + 16);
}

int launch_wcrt(const WcrtLaunch &L, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, st, L.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  if (L.b.n_sets == 0) return 0;
  hipLaunchKernelGGL(wcrt_kernel, dim3(L.grid), dim3(kWave), L.lds_bytes, st, L);
  return (int)hipGetLastError();
}

}  // namespace paam
