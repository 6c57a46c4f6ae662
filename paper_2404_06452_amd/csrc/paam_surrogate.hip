// HIP kernels of the candidate-ranking surrogate for gfx950: per-chain
// features of candidate priority orders, the network's forward pass on the
// matrix cores (bfloat16 operands, float32 accumulation), its backward pass
// and Adam in float32.  The exact analysis stays the judge of schedulability;
// these kernels only rank candidates for it.
#include <hip/hip_runtime.h>
#include <math.h>

#include "paam_device.h"
#include "paam_internal.h"

namespace paam {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ features

// Both schedules take every chain's higher-priority totals from prefix sums
// and its lower-priority terms from suffix maxima and counts over the rank
// order (O(C (X + NA)) per candidate).  Sets of up to 64 chains: a wave takes
// up to kMaxGroup consecutive candidates at once (lane g*C + r holds the chain
// at rank r of candidate g) and scans within each candidate's lanes.  Larger
// sets: one candidate at a time over 64-rank chunks with running totals.
constexpr int kMaxGroup = 16;
constexpr int kScanC = 64;  // sets with more chains use the prefix-scan schedule
// candidates per scoring work item: LDS-table schedule, prefix-scan schedule
constexpr int kFeatItemLds = 128, kFeatItemScan = 8;
constexpr int kFwd = 9;     // numerators of a chain from the prefix-scan schedule's forward pass
// wave-uniform running totals of the prefix-scan schedule, in LDS: forward
// (4 per executor, 4 per accelerator) and backward (3 and 3)
constexpr int kScanCarry = 7 * (kMaxExec + kMaxAccel);

// Per-wave tables: a set's order-independent totals (built once per set), the
// walk state, the ranks and orders of a pass's candidates, and the forward
// numerators and inversion counts of the large-set schedule.
struct FeatTables {
  int64_t *Ec, *Acc, *epc, *Emax, *qsum, *qasum, *T, *D;  // [Cm]
  int64_t *Ece, *Acce, *epce, *bl, *bS, *q, *qa;          // [Cm][X]
  int64_t *car;                                            // [Cm][X] E + A* + eps per chain and executor
  int64_t *hppn, *hppq;                                    // [Cm] OS-preemption numerators of a chain
  int64_t *Ahat, *Amax, *qA;                               // [Cm][NA]
  int64_t *setv;                                           // [8] set-level sums
  int64_t *colw;                                           // [2][Xm] column totals of hpp weights
  int64_t *fwd;                                            // [Cm][kFwd] forward-pass numerators by rank
  int32_t *inv;                                            // [2][Cm] RM inversions above / below
  int32_t *S, *dl, *ncb, *mine, *uses, *spin;              // [Cm]
  uint32_t *tmpl;                                          // [Cm][13] order-independent feature words
  int32_t *runs;                                           // [Cm][X]
  int32_t *dca, *nra;                                      // [Cm][NA]
  int32_t *hpx;                                            // [Xm]
  int32_t *order, *buf;                                    // [Cm], [64]
  int32_t *ordg;                                           // [max(64, Cm)] chain at each rank, per candidate of a pass
  int16_t *rank;                                           // [Cm]
  int16_t *rankg;                                          // [max(64, Cm)]
};

__host__ __device__ inline size_t feat_table_bytes(int Cm, int Xm, int NAm) {
  const size_t C = Cm, CX = (size_t)Cm * Xm, CA = (size_t)Cm * NAm;
  const size_t G = Cm > 64 ? (size_t)Cm : 64;
  const size_t scan = Cm > kScanC ? (size_t)kFwd * C : 0;
  const size_t n64 = 10 * C + 8 * CX + 3 * CA + 8 + 2 * (size_t)Xm + scan;
  const size_t n32 = 6 * C + 13 * C + CX + 2 * CA + Xm + C + 64 + G + (Cm > kScanC ? 2 * C : 0);
  const size_t n16 = C + G;
  return ((8 * n64 + 4 * n32 + 2 * n16) + 15) & ~(size_t)15;
}

__device__ FeatTables carve_feat(unsigned char *base, int Cm, int Xm, int NAm) {
  FeatTables t;
  const size_t C = Cm, CX = (size_t)Cm * Xm, CA = (size_t)Cm * NAm;
  const size_t G = Cm > 64 ? (size_t)Cm : 64;
  int64_t *d = reinterpret_cast<int64_t *>(base);
  t.Ec = d; d += C;
  t.Acc = d; d += C;
  t.epc = d; d += C;
  t.Emax = d; d += C;
  t.qsum = d; d += C;
  t.qasum = d; d += C;
  t.T = d; d += C;
  t.D = d; d += C;
  t.Ece = d; d += CX;
  t.Acce = d; d += CX;
  t.epce = d; d += CX;
  t.bl = d; d += CX;
  t.bS = d; d += CX;
  t.q = d; d += CX;
  t.qa = d; d += CX;
  t.car = d; d += CX;
  t.hppn = d; d += C;
  t.hppq = d; d += C;
  t.Ahat = d; d += CA;
  t.Amax = d; d += CA;
  t.qA = d; d += CA;
  t.setv = d; d += 8;
  t.colw = d; d += 2 * (size_t)Xm;
  t.fwd = nullptr;
  if (Cm > kScanC) {
    t.fwd = d;
    d += (size_t)kFwd * C;
  }
  int32_t *i = reinterpret_cast<int32_t *>(d);
  t.S = i; i += C;
  t.dl = i; i += C;
  t.ncb = i; i += C;
  t.mine = i; i += C;
  t.uses = i; i += C;
  t.spin = i; i += C;
  t.tmpl = reinterpret_cast<uint32_t *>(i); i += 13 * C;
  t.runs = i; i += CX;
  t.dca = i; i += CA;
  t.nra = i; i += CA;
  t.hpx = i; i += Xm;
  t.order = i; i += C;
  t.buf = i; i += 64;
  t.ordg = i; i += G;
  t.inv = nullptr;
  if (Cm > kScanC) {
    t.inv = i;
    i += 2 * C;
  }
  int16_t *h = reinterpret_cast<int16_t *>(i);
  t.rank = h; h += C;
  t.rankg = h;
  return t;
}

__device__ __forceinline__ int64_t scale_E(int64_t x, int32_t u) {
  return u == 1000 ? x : (x * (int64_t)u) / 1000;
}

// (double)n / (double)m, 0 when m == 0.
__device__ __forceinline__ double fratio(int64_t n, int64_t m) {
  return m == 0 ? 0.0 : (double)n / (double)m;
}

constexpr int64_t kQ = 65536;  // fixed-point scale of utilisation terms

// hpp weight of chain h on executor e: E plus, for a busy-waiting chain, its
// accelerator handling, else only its request overheads
__device__ __forceinline__ int64_t hpp_w(const FeatTables &t, int h, int e, int X) {
  const int i = h * X + e;
  return t.Ece[i] + (t.spin[h] ? t.Acce[i] + t.epce[i] : t.epce[i]);
}
__device__ __forceinline__ int64_t hpp_q(const FeatTables &t, int h, int e, int X) {
  const int i = h * X + e;
  return t.q[i] + (t.spin[h] ? t.qa[i] : 0);
}

// Wave-wide total and minimum of int64 values (butterfly over the 64 lanes).
__device__ __forceinline__ int64_t wave_total_i64(int64_t v) {
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int64_t wave_min_i64(int64_t v) {
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t n = __shfl_xor(v, o);
    v = n < v ? n : v;
  }
  return v;
}

// Order-independent tables of a set at utilisation scale u.  Lane c owns the
// rows of chain c.  Ends synchronised.
__device__ void feat_build(const DevBatch &b, int64_t set, int32_t u, FeatTables &t) {
  const int64_t c0 = b.set_chain_off[set];
  const int C = (int)(b.set_chain_off[set + 1] - c0);
  const int64_t x0 = b.set_exec_off[set];
  const int X = (int)(b.set_exec_off[set + 1] - x0);
  const int64_t a0 = b.set_accel_off[set];
  const int NA = (int)(b.set_accel_off[set + 1] - a0);
  const int NAm = NA > 0 ? NA : 1;
  const int64_t cb0 = b.set_cb_off[set];
  for (int e = threadIdx.x; e < X; e += kWave) t.hpx[e] = (int32_t)b.hpx_mask[x0 + e];
  for (int c = threadIdx.x; c < C; c += kWave) {
    int64_t E = 0, Ac = 0, ep = 0, Emax = 0;
    int S = 0, dl = 0, ncb = 0;
    uint32_t mine = 0, uses = 0;
    for (int e = 0; e < X; ++e) {
      const int i = c * X + e;
      t.Ece[i] = t.Acce[i] = t.epce[i] = t.bl[i] = t.bS[i] = 0;
      t.runs[i] = 0;
    }
    for (int a = 0; a < NAm; ++a) {
      const int i = c * NAm + a;
      t.Ahat[i] = t.Amax[i] = 0;
      t.dca[i] = t.nra[i] = 0;
    }
    // the chain's callbacks in order; a sub-chain is a maximal run of
    // consecutive callbacks on one executor (every table entry is a sum, a
    // maximum or a union, so the order of the sub-chains does not matter)
    const int jlo = b.chain_cb_lo[c0 + c];
    const int jhi = c + 1 < C ? b.chain_cb_lo[c0 + c + 1] : (int)(b.set_cb_off[set + 1] - cb0);
    int prev_e = -1;
    uint32_t accs = 0;
    for (int j = jlo; j < jhi; ++j) {
      const int e = b.cb_exec[cb0 + j];
      const int ie = c * X + e;
      if (e != prev_e) {
        for (uint32_t m = accs; m; m &= m - 1) t.nra[c * NAm + (__ffs(m) - 1)] += 1;
        accs = 0;
        ++S;
        t.runs[ie] += 1;
        mine |= 1u << e;
        prev_e = e;
      }
      {
        const int64_t Ej = scale_E(b.E[cb0 + j], u);
        ++ncb;
        E += Ej;
        t.Ece[ie] += Ej;
        Emax = Ej > Emax ? Ej : Emax;
        t.bl[ie] = Ej > t.bl[ie] ? Ej : t.bl[ie];
        int64_t bj = Ej;
        for (int64_t g = b.cb_seg_off[cb0 + j]; g < b.cb_seg_off[cb0 + j + 1]; ++g) {
          const int a = b.seg_accel[g];
          const int64_t As = scale_E(b.A[g], u) + 2 * b.akappa[a0 + a];
          const int64_t ea = b.aeps[a0 + a];
          Ac += As;
          ep += ea;
          ++dl;
          t.Acce[ie] += As;
          t.epce[ie] += ea;
          const int ia = c * NAm + a;
          t.Ahat[ia] += As;
          t.dca[ia] += 1;
          t.Amax[ia] = As > t.Amax[ia] ? As : t.Amax[ia];
          bj += As + ea;
          accs |= 1u << a;
          uses |= 1u << a;
        }
        t.bS[ie] = bj > t.bS[ie] ? bj : t.bS[ie];
      }
    }
    for (uint32_t m = accs; m; m &= m - 1) t.nra[c * NAm + (__ffs(m) - 1)] += 1;
    const int64_t T = b.T[c0 + c];
    int64_t qs = 0, qas = 0;
    for (int e = 0; e < X; ++e) {
      const int i = c * X + e;
      t.q[i] = (t.Ece[i] * kQ) / T;
      t.qa[i] = ((t.Acce[i] + t.epce[i]) * kQ) / T;
      qs += t.q[i];
      qas += t.qa[i];
    }
    for (int a = 0; a < NAm; ++a) t.qA[c * NAm + a] = (t.Ahat[c * NAm + a] * kQ) / T;
    t.Ec[c] = E;
    t.Acc[c] = Ac;
    t.epc[c] = ep;
    t.Emax[c] = Emax;
    t.qsum[c] = qs;
    t.qasum[c] = qas;
    t.T[c] = T;
    t.D[c] = b.D[c0 + c];
    t.S[c] = S;
    t.dl[c] = dl;
    t.ncb[c] = ncb;
    t.mine[c] = (int32_t)mine;
    t.uses[c] = (int32_t)uses;
    t.spin[c] = b.spin[c0 + c];
  }
  __syncthreads();
  // column totals of the hpp weights per executor and the set-level sums:
  // lanes over chains, then wave totals (integer sums, so exact in any order)
  {
    int64_t sum_q = 0, sum_qA = 0, sum_dem = 0, Tmin = INT64_MAX, max_qe = 0, tot = 0;
    for (int h = threadIdx.x; h < C; h += kWave) {
      tot += t.Ec[h] + t.Acc[h] + t.epc[h];
      sum_q += t.qsum[h];
      for (int a = 0; a < NA; ++a) sum_qA += t.qA[h * NAm + a];
      sum_dem += t.Ec[h] + t.Acc[h];
      Tmin = t.T[h] < Tmin ? t.T[h] : Tmin;
    }
    tot = wave_total_i64(tot);
    sum_q = wave_total_i64(sum_q);
    sum_qA = wave_total_i64(sum_qA);
    sum_dem = wave_total_i64(sum_dem);
    Tmin = wave_min_i64(Tmin);
    for (int e = 0; e < X; ++e) {
      int64_t w = 0, q = 0, qe = 0;
      for (int h = threadIdx.x; h < C; h += kWave) {
        w += hpp_w(t, h, e, X);
        q += hpp_q(t, h, e, X);
        qe += t.q[h * X + e];
      }
      w = wave_total_i64(w);
      q = wave_total_i64(q);
      qe = wave_total_i64(qe);
      max_qe = qe > max_qe ? qe : max_qe;
      if (threadIdx.x == 0) {
        t.colw[e] = w;
        t.colw[X + e] = q;
      }
    }
    if (threadIdx.x == 0) {
      t.setv[0] = sum_q;
      t.setv[1] = sum_qA;
      t.setv[2] = sum_dem;
      t.setv[3] = Tmin;
      t.setv[4] = max_qe;
      t.setv[5] = tot;
    }
  }
  __syncthreads();
  // OS preemption by higher process-priority executors of the same core does
  // not depend on the chain order: per (chain, executor), the column totals
  // over those executors minus the chain's own entries, weighted by the
  // chain's sub-chains on the executor (numerator) or counted once where it
  // has any (utilisation)
  for (int c = threadIdx.x; c < C; c += kWave) {
    int64_t nsum = 0, qsum = 0;
    for (int e = 0; e < X; ++e) {
      const int i = c * X + e;
      t.car[i] = t.Ece[i] + t.Acce[i] + t.epce[i];
      const int64_t rce = t.runs[i];
      int64_t n = 0, q = 0;
      for (uint32_t m = (uint32_t)t.hpx[e]; m; m &= m - 1) {
        const int e2 = __ffs(m) - 1;
        n += 2 * (t.colw[e2] - hpp_w(t, c, e2, X));
        q += t.colw[X + e2] - hpp_q(t, c, e2, X);
      }
      nsum += rce * n;
      qsum += rce > 0 ? q : 0;
    }
    t.hppn[c] = nsum;
    t.hppq[c] = qsum;
  }
  __syncthreads();
}

// Feature f of a row assembled in registers: two bfloat16 per 32-bit word.
__device__ __forceinline__ void put_feat(uint32_t *w, int f, double v) {
  w[f >> 1] |= (uint32_t)bf16_rne((float)v) << (16 * (f & 1));
}

// Order-dependent numerators of one chain under one candidate.
struct FeatNums {
  int64_t n19, n20, q21, q22, n_carry, q24, n25, n_bp, n_bs, m28, n29, n_hpp, q_hpp;
  int64_t n_acc, q33, n_bacc, n36, f37;
  double f35;
};

// Words of a row (two bfloat16 each) that hold only order-independent
// features: 0-13 (words 0-6), 14 (low half of word 7), 38-43 (words 19-21),
// 44 (low half of word 22) and 47 (high half of word 23).  Built once per
// set into t.tmpl[c][13] = words 0-7 and 19-23.
constexpr int kTmplWords = 13;

__device__ void feat_template(const DevBatch &b, int64_t set, const FeatTables &t, int c) {
  const int C = (int)(b.set_chain_off[set + 1] - b.set_chain_off[set]);
  const int X = (int)(b.set_exec_off[set + 1] - b.set_exec_off[set]);
  const int NA = (int)(b.set_accel_off[set + 1] - b.set_accel_off[set]);
  const int64_t hop = b.eps_hop[set];
  const int64_t T = t.T[c], D = t.D[c];
  const int S = t.S[c];
  const int64_t own = t.Ec[c] + t.Acc[c] + t.epc[c] + (int64_t)(S - 1) * hop;
  uint32_t w[24];
#pragma unroll
  for (int i = 0; i < 24; ++i) w[i] = 0u;
  put_feat(w, 0, fratio(t.Ec[c], D));
  put_feat(w, 1, fratio(t.Acc[c], D));
  put_feat(w, 2, fratio(t.epc[c], D));
  put_feat(w, 3, fratio((int64_t)(S - 1) * hop, D));
  put_feat(w, 4, fratio(own, D));
  put_feat(w, 5, fratio(t.Emax[c], D));
  put_feat(w, 6, fratio(S, 16));
  put_feat(w, 7, fratio(t.dl[c], 16));
  put_feat(w, 8, fratio(t.ncb[c], 32));
  put_feat(w, 9, fratio(__popc((uint32_t)t.mine[c]), X));
  put_feat(w, 10, fratio(D, T));
  put_feat(w, 11, fratio(T, (int64_t)1 << 30));
  put_feat(w, 12, t.spin[c] ? 1.0 : 0.0);
  put_feat(w, 13, fratio(t.qsum[c], kQ));
  put_feat(w, 14, fratio(t.qasum[c], kQ));
  put_feat(w, 38, fratio(t.setv[0], (int64_t)X * kQ));
  put_feat(w, 39, fratio(t.setv[4], kQ));
  put_feat(w, 40, fratio(t.setv[1], kQ));
  put_feat(w, 41, fratio(C, 256));
  put_feat(w, 42, fratio(X, 8));
  put_feat(w, 43, fratio(NA, 8));
  put_feat(w, 44, fratio(t.setv[3], T));
  put_feat(w, 47, fratio(t.Ec[c] + t.Acc[c], t.setv[2]));
  uint32_t *o = t.tmpl + (size_t)c * kTmplWords;
#pragma unroll
  for (int i = 0; i < 8; ++i) o[i] = w[i];
#pragma unroll
  for (int i = 0; i < 5; ++i) o[8 + i] = w[19 + i];
}

// The 48 features of chain c of rank rho, written to row[0..47]: the
// order-independent words from t.tmpl, the others from the numerators.
// Feature k here is feature k of the documented list; each is
// (double)N / (double)M of exact integers.
__device__ void feat_write(const DevBatch &b, int64_t set, const FeatTables &t, int c, int rho,
                           const FeatNums &f, uint16_t *row) {
  const int C = (int)(b.set_chain_off[set + 1] - b.set_chain_off[set]);
  const int64_t hop = b.eps_hop[set];
  const int64_t D = t.D[c];
  const int S = t.S[c];
  const int64_t own = t.Ec[c] + t.Acc[c] + t.epc[c] + (int64_t)(S - 1) * hop;
  uint32_t w[24];
  const uint32_t *tw = t.tmpl + (size_t)c * kTmplWords;
#pragma unroll
  for (int i = 0; i < 8; ++i) w[i] = tw[i];
#pragma unroll
  for (int i = 8; i < 19; ++i) w[i] = 0u;
#pragma unroll
  for (int i = 0; i < 5; ++i) w[19 + i] = tw[8 + i];
  put_feat(w, 15, fratio(rho, C));
  put_feat(w, 16, fratio(C - 1 - rho, C));
  put_feat(w, 17, rho == 0 ? 1.0 : 0.0);
  put_feat(w, 18, rho == C - 1 ? 1.0 : 0.0);
  put_feat(w, 19, fratio(f.n19, C));
  put_feat(w, 20, fratio(f.n20, C));
  put_feat(w, 21, fratio(f.q21, kQ));
  put_feat(w, 22, fratio(f.q22, kQ));
  put_feat(w, 23, fratio(f.n_carry, D));
  put_feat(w, 24, fratio(f.q24, kQ));
  put_feat(w, 25, fratio(f.n25, C));
  put_feat(w, 26, fratio(f.n_bp, D));
  put_feat(w, 27, fratio(f.n_bs, D));
  put_feat(w, 28, fratio(f.m28, D));
  put_feat(w, 29, fratio(f.n29, C));
  put_feat(w, 30, fratio(f.n_hpp, D));
  put_feat(w, 31, fratio(f.q_hpp, kQ));
  put_feat(w, 32, fratio(f.n_acc, D));
  put_feat(w, 33, fratio(f.q33, kQ));
  put_feat(w, 34, fratio(f.n_bacc, D));
  put_feat(w, 35, f.f35);
  put_feat(w, 36, fratio(f.n36, C));
  put_feat(w, 37, f.f37 ? 1.0 : 0.0);
  const int64_t n_est = own + f.n_carry + f.n_bs + f.n_hpp + f.n_acc + f.n_bacc;
  const int64_t q_est = f.q21 + f.q22 + f.q_hpp + f.q33;
  put_feat(w, 45, fratio(n_est, D));
  put_feat(w, 46, fratio(n_est, D) + fratio(q_est, kQ));
  // the row (96 bytes, 16-byte aligned) in six 16-byte stores
  uint4 *dst = reinterpret_cast<uint4 *>(row);
#pragma unroll
  for (int i = 0; i < 6; ++i) dst[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
}

// Chains ranked above / below c that beat / trail it in period (RM inversions).
__device__ __forceinline__ void rm_inversions(const FeatTables &t, const int16_t *rk, int C, int c,
                                              int rho, FeatNums &f) {
  const int64_t T = t.T[c];
  int64_t n19 = 0, n20 = 0;
  for (int h = 0; h < C; ++h) {
    const int64_t Th = t.T[h];
    const int rh = rk[h];
    n19 += (rh < rho && Th > T) ? 1 : 0;
    n20 += (rh > rho && Th < T) ? 1 : 0;
  }
  f.n19 = n19;
  f.n20 = n20;
}

__device__ __forceinline__ void hpp_terms(const FeatTables &t, int c, int X, FeatNums &f) {
  f.n_hpp = t.hppn[c];
  f.q_hpp = t.hppq[c];
}

// ---- prefix-scan schedule (sets of more than kScanC chains)

// Wave-wide inclusive prefix sum and suffix maximum over 64 lanes.
__device__ __forceinline__ int64_t wave_incl_sum(int64_t v) {
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t n = __shfl_up(v, o);
    if ((int)threadIdx.x >= o) v += n;
  }
  return v;
}
__device__ __forceinline__ int64_t wave_incl_suffix_sum(int64_t v) {
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t n = __shfl_down(v, o);
    if ((int)threadIdx.x + o < kWave) v += n;
  }
  return v;
}
__device__ __forceinline__ int64_t wave_incl_suffix_max(int64_t v) {
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t n = __shfl_down(v, o);
    if ((int)threadIdx.x + o < kWave) v = n > v ? n : v;
  }
  return v;
}

// RM inversion counts of every chain (t.inv) under the order in t.rank:
// computed in full, or, when the order differs from the previous one by the
// single swap of positions pa and pb, updated.  A chain ranked strictly
// between the two positions trades the swapped chain above it for the other;
// chains outside keep both on the same side; the two swapped chains are
// counted again by the whole wave.  Ends synchronised.
__device__ void feat_inversions(const FeatTables &t, int C, int pa, int pb, bool incremental) {
  const int lane = threadIdx.x;
  if (!incremental) {
    for (int c = lane; c < C; c += kWave) {
      FeatNums f;
      rm_inversions(t, t.rank, C, c, t.rank[c], f);
      t.inv[c] = (int32_t)f.n19;
      t.inv[C + c] = (int32_t)f.n20;
    }
    __syncthreads();
    return;
  }
  const int lo = pa < pb ? pa : pb, hi = pa < pb ? pb : pa;
  const int up = t.order[lo], down = t.order[hi];  // moved up to lo / down to hi
  const int64_t Tu = t.T[up], Td = t.T[down];
  for (int c = lane; c < C; c += kWave) {
    const int r = t.rank[c];
    if (r > lo && r < hi) {
      const int64_t Tc = t.T[c];
      t.inv[c] += (Tu > Tc ? 1 : 0) - (Td > Tc ? 1 : 0);
      t.inv[C + c] += (Td < Tc ? 1 : 0) - (Tu < Tc ? 1 : 0);
    }
  }
  int32_t a19 = 0, a20 = 0, b19 = 0, b20 = 0;
  for (int h = lane; h < C; h += kWave) {
    const int rh = t.rank[h];
    const int64_t Th = t.T[h];
    a19 += (rh < lo && Th > Tu) ? 1 : 0;
    a20 += (rh > lo && Th < Tu) ? 1 : 0;
    b19 += (rh < hi && Th > Td) ? 1 : 0;
    b20 += (rh > hi && Th < Td) ? 1 : 0;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    a19 += __shfl_xor(a19, o);
    a20 += __shfl_xor(a20, o);
    b19 += __shfl_xor(b19, o);
    b20 += __shfl_xor(b20, o);
  }
  if (lane == 0) {
    t.inv[up] = a19;
    t.inv[C + up] = a20;
    t.inv[down] = b19;
    t.inv[C + down] = b20;
  }
  __syncthreads();
}

// Sets of up to 64 chains: the ng candidates of a pass at once, lane
// g*C + r holding the chain at rank r of candidate g (order in t.ordg, ranks
// in t.rankg).  The scans of the prefix-scan schedule run segmented within
// each candidate's C lanes and need no running totals: every chain's
// higher-priority totals come from prefix sums, its lower-priority terms from
// suffix maxima and counts, the same-bucket blocking term from a suffix
// maximum segmented by bucket level.  Candidate g's rows start at
// rows + g * row_stride * 48.
// A 64-bit value moved by a DPP row shift (16-lane rows; 0 where the source
// lies outside the row): row_shr:n (0x110 + n) takes lane i - n, row_shl:n
// (0x100 + n) lane i + n.
template <int Ctrl>
__device__ __forceinline__ int64_t dpp64(int64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, Ctrl, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), Ctrl, 0xf, 0xf, true);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ void feat_group_scan(const DevBatch &b, int64_t set, const FeatTables &t, int C,
                                int ng, uint16_t *rows, int row_stride) {
  const int lane = threadIdx.x;
  const int X = (int)(b.set_exec_off[set + 1] - b.set_exec_off[set]);
  const int64_t a0 = b.set_accel_off[set];
  const int NA = (int)(b.set_accel_off[set + 1] - a0);
  const int NAm = NA > 0 ? NA : 1;
  const int g = lane / C, r = lane - g * C;
  const bool ok = g < ng;
  const int c = ok ? t.ordg[g * C + r] : 0;
  const uint32_t uses = ok ? (uint32_t)t.uses[c] : 0u;
  // Sets of exactly 16 chains: every candidate of a pass is one 16-lane row,
  // so the scans below run on DPP row shifts instead of LDS-routed shuffles
  // (the sums and maxima take 0 from outside the row; every scanned value is
  // non-negative).
  const bool rowwise = C == 16;
  auto sum_up = [&](int64_t v) {
    if (rowwise) {
      v += dpp64<0x111>(v);
      v += dpp64<0x112>(v);
      v += dpp64<0x114>(v);
      v += dpp64<0x118>(v);
      return v;
    }
    for (int o = 1; o < C; o <<= 1) {
      const int64_t n = __shfl_up(v, o);
      if (r >= o) v += n;
    }
    return v;
  };
  auto sum_down = [&](int64_t v) {
    if (rowwise) {
      v += dpp64<0x101>(v);
      v += dpp64<0x102>(v);
      v += dpp64<0x104>(v);
      v += dpp64<0x108>(v);
      return v;
    }
    for (int o = 1; o < C; o <<= 1) {
      const int64_t n = __shfl_down(v, o);
      if (r + o < C) v += n;
    }
    return v;
  };
  auto max_down = [&](int64_t v) {
    if (rowwise) {
      int64_t n = dpp64<0x101>(v);
      v = n > v ? n : v;
      n = dpp64<0x102>(v);
      v = n > v ? n : v;
      n = dpp64<0x104>(v);
      v = n > v ? n : v;
      n = dpp64<0x108>(v);
      v = n > v ? n : v;
      return v;
    }
    for (int o = 1; o < C; o <<= 1) {
      const int64_t n = __shfl_down(v, o);
      if (r + o < C) v = n > v ? n : v;
    }
    return v;
  };
  // the value of the next rank of the same candidate, 0 past the last
  auto next = [&](int64_t v) {
    if (rowwise) return dpp64<0x101>(v);
    const int64_t n = __shfl_down(v, 1);
    return r + 1 < C ? n : (int64_t)0;
  };
  FeatNums f;
  int64_t q21 = 0, q22 = 0, q24 = 0, n_carry = 0, n_bp = 0, n_bs = 0, m28 = 0, n25 = 0, n29 = 0;
  for (int e = 0; e < X; ++e) {
    int64_t vq = 0, vqa = 0, vcar = 0, rce = 0, vbl = 0, vbs = 0;
    if (ok) {
      const int i = c * X + e;
      vq = t.q[i];
      vqa = t.qa[i];
      vcar = t.car[i];
      rce = t.runs[i];
      vbl = t.bl[i];
      vbs = t.bS[i];
    }
    const int64_t vh = rce > 0 ? 1 : 0;
    const int64_t sq = sum_up(vq) - vq, sqa = sum_up(vqa) - vqa;
    const int64_t scar = sum_up(vcar) - vcar, nhp = sum_up(vh) - vh;
    const int64_t mbl = next(max_down(vbl)), mbs = next(max_down(vbs)), nlp = next(sum_down(vh));
    n_carry += rce * 2 * scar;
    n_bp += rce * mbl;
    n_bs += rce * mbs;
    if (rce > 0) {
      q21 += sq;
      q22 += sqa;
      q24 = sq + sqa > q24 ? sq + sqa : q24;
      n25 += nhp;
      n29 += nlp;
      m28 = mbs > m28 ? mbs : m28;
    }
  }
  f.q21 = q21; f.q22 = q22; f.q24 = q24; f.n_carry = n_carry; f.n_bp = n_bp; f.n_bs = n_bs;
  f.m28 = m28; f.n25 = n25; f.n29 = n29;
  int64_t n_acc = 0, q33 = 0, n_bacc = 0, n36 = 0, f37 = 0;
  double f35 = 0.0;
  for (int a = 0; a < NA; ++a) {
    int64_t vA = 0, vqA = 0, vu = 0, vmax = 0;
    if (ok) {
      const int i = c * NAm + a;
      vA = t.Ahat[i];
      vqA = t.qA[i];
      vu = t.dca[i] > 0 ? 1 : 0;
      vmax = vu ? t.Amax[i] : 0;
    }
    const int64_t vp = vA > 0 ? 1 : 0;
    const int64_t iu = sum_up(vu);
    const int64_t hpA = sum_up(vA) - vA, pqA = sum_up(vqA) - vqA, uab = iu - vu;
    const int64_t pab = sum_up(vp) - vp;
    const int64_t mu_ = __shfl(iu, g * C + C - 1 < kWave ? g * C + C - 1 : kWave - 1);
    const int64_t m = mu_ > 0 ? mu_ : 1;  // users of the accelerator in this candidate's set
    const int64_t nb = b.buckets[a0 + a];
    const int64_t key = (uab * nb) / m;    // bucket level of rank r
    int64_t xv = vmax;
    if (rowwise) {
      // the same segmented maximum on DPP row shifts (r + o < 16 keeps the
      // comparison inside the candidate's row)
      int64_t nv = dpp64<0x101>(xv), nk = dpp64<0x101>(key);
      if (r + 1 < C && nk == key) xv = nv > xv ? nv : xv;
      nv = dpp64<0x102>(xv);
      nk = dpp64<0x102>(key);
      if (r + 2 < C && nk == key) xv = nv > xv ? nv : xv;
      nv = dpp64<0x104>(xv);
      nk = dpp64<0x104>(key);
      if (r + 4 < C && nk == key) xv = nv > xv ? nv : xv;
      nv = dpp64<0x108>(xv);
      nk = dpp64<0x108>(key);
      if (r + 8 < C && nk == key) xv = nv > xv ? nv : xv;
    } else {
      for (int o = 1; o < C; o <<= 1) {
        const int64_t nv = __shfl_down(xv, o);
        const int64_t nk = __shfl_down(key, o);
        if (r + o < C && nk == key) xv = nv > xv ? nv : xv;
      }
    }
    const int64_t nv1 = rowwise ? dpp64<0x101>(xv) : __shfl_down(xv, 1);
    const int64_t nk1 = rowwise ? dpp64<0x101>(key) : __shfl_down(key, 1);
    if ((uses >> a) & 1u) {
      n_acc += 2 * (int64_t)t.nra[c * NAm + a] * hpA;
      q33 += pqA;
      n36 += uab;
      f37 |= pab > 0 ? 1 : 0;
      n_bacc += (int64_t)t.dca[c * NAm + a] * ((r + 1 < C && nk1 == key) ? nv1 : 0);
      const double lvr = fratio(key, nb);
      f35 = lvr > f35 ? lvr : f35;
    }
  }
  f.n_acc = n_acc; f.q33 = q33; f.n_bacc = n_bacc; f.n36 = n36; f.f37 = f37; f.f35 = f35;
  if (ok) {
    rm_inversions(t, t.rankg + g * C, C, c, r, f);
    hpp_terms(t, c, X, f);
    feat_write(b, set, t, c, r, f, rows + ((size_t)g * row_stride + c) * 48);
  }
}

// Prefix-scan schedule for one candidate (order in t.order, inversion
// counts in t.inv): lane r of each 64-rank chunk holds the chain at rank r.
// A forward pass over the chunks (ranks ascending) turns wave-wide prefix
// sums into every chain's higher-priority totals per executor (q, q_acc,
// E + A* + eps, chains with a sub-chain) and per accelerator (A-hat, its
// utilisation, users, positive requests); a backward pass (ranks descending)
// turns suffix maxima and counts into the lower-priority terms, and the
// same-bucket blocking into a suffix maximum segmented by bucket level (the
// level of a rank, u * n / m with u the users ranked above it, never
// decreases down the order).  Running totals between chunks sit in carry
// (LDS); the forward numerators of a rank wait in t.fwd.  Row c of rows
// receives chain c's 48 features.  Ends synchronised.
__device__ void feat_candidate_scan(const DevBatch &b, int64_t set, const FeatTables &t,
                                    int64_t *carry, uint16_t *rows) {
  const int lane = threadIdx.x;
  const int C = (int)(b.set_chain_off[set + 1] - b.set_chain_off[set]);
  const int X = (int)(b.set_exec_off[set + 1] - b.set_exec_off[set]);
  const int64_t a0 = b.set_accel_off[set];
  const int NA = (int)(b.set_accel_off[set + 1] - a0);
  const int NAm = NA > 0 ? NA : 1;
  const int32_t *ord = t.order;
  int64_t *cf = carry;                 // forward: [X][4], then [NA][4]
  int64_t *cb = carry + 4 * (X + NA);  // backward: [X][3], then [NA][3]
  for (int k = lane; k < 4 * (X + NA); k += kWave) cf[k] = 0;
  for (int k = lane; k < 3 * (X + NA); k += kWave) cb[k] = (k >= 3 * X && (k - 3 * X) % 3 == 2) ? -1 : 0;
  __syncthreads();

  // ---- forward pass
  for (int rb = 0; rb < C; rb += kWave) {
    const int r = rb + lane;
    const bool ok = r < C;
    const int c = ok ? ord[r] : 0;
    const uint32_t uses = ok ? (uint32_t)t.uses[c] : 0u;
    int64_t n_carry = 0, q21 = 0, q22 = 0, q24 = 0, n25 = 0;
    for (int e = 0; e < X; ++e) {
      int64_t vq = 0, vqa = 0, vcar = 0, rce = 0;
      if (ok) {
        const int i = c * X + e;
        vq = t.q[i];
        vqa = t.qa[i];
        vcar = t.car[i];
        rce = t.runs[i];
      }
      const int64_t vh = rce > 0 ? 1 : 0;
      const int64_t *cy = cf + 4 * e;
      const int64_t iq = wave_incl_sum(vq), iqa = wave_incl_sum(vqa);
      const int64_t ic = wave_incl_sum(vcar), ih = wave_incl_sum(vh);
      const int64_t sq = cy[0] + iq - vq, sqa = cy[1] + iqa - vqa;
      const int64_t scar = cy[2] + ic - vcar, nhp = cy[3] + ih - vh;
      n_carry += rce * 2 * scar;
      if (rce > 0) {
        q21 += sq;
        q22 += sqa;
        q24 = sq + sqa > q24 ? sq + sqa : q24;
        n25 += nhp;
      }
      const int64_t tq = __shfl(iq, kWave - 1), tqa = __shfl(iqa, kWave - 1);
      const int64_t tc = __shfl(ic, kWave - 1), th = __shfl(ih, kWave - 1);
      __syncthreads();
      if (lane == 0) {
        cf[4 * e] += tq;
        cf[4 * e + 1] += tqa;
        cf[4 * e + 2] += tc;
        cf[4 * e + 3] += th;
      }
    }
    int64_t n_acc = 0, q33 = 0, n36 = 0, f37 = 0;
    for (int a = 0; a < NA; ++a) {
      int64_t vA = 0, vqA = 0, vu = 0;
      if (ok) {
        const int i = c * NAm + a;
        vA = t.Ahat[i];
        vqA = t.qA[i];
        vu = t.dca[i] > 0 ? 1 : 0;
      }
      const int64_t vp = vA > 0 ? 1 : 0;
      const int64_t *cy = cf + 4 * (X + a);
      const int64_t iA = wave_incl_sum(vA), iqA = wave_incl_sum(vqA);
      const int64_t iu = wave_incl_sum(vu), ip = wave_incl_sum(vp);
      if ((uses >> a) & 1u) {
        n_acc += 2 * (int64_t)t.nra[c * NAm + a] * (cy[0] + iA - vA);
        q33 += cy[1] + iqA - vqA;
        n36 += cy[2] + iu - vu;
        f37 |= (cy[3] + ip - vp) > 0 ? 1 : 0;
      }
      const int64_t tA = __shfl(iA, kWave - 1), tqA = __shfl(iqA, kWave - 1);
      const int64_t tu = __shfl(iu, kWave - 1), tp = __shfl(ip, kWave - 1);
      __syncthreads();
      if (lane == 0) {
        cf[4 * (X + a)] += tA;
        cf[4 * (X + a) + 1] += tqA;
        cf[4 * (X + a) + 2] += tu;
        cf[4 * (X + a) + 3] += tp;
      }
    }
    if (ok) {
      int64_t *w = t.fwd + (size_t)r * kFwd;
      w[0] = n_carry;
      w[1] = q21;
      w[2] = q22;
      w[3] = q24;
      w[4] = n25;
      w[5] = n_acc;
      w[6] = q33;
      w[7] = n36;
      w[8] = f37;
    }
    __syncthreads();
  }

  // ---- backward pass
  for (int rb = ((C - 1) / kWave) * kWave; rb >= 0; rb -= kWave) {
    const int r = rb + lane;
    const bool ok = r < C;
    const int c = ok ? ord[r] : 0;
    const uint32_t uses = ok ? (uint32_t)t.uses[c] : 0u;
    int64_t n_bp = 0, n_bs = 0, m28 = 0, n29 = 0;
    for (int e = 0; e < X; ++e) {
      int64_t vbl = 0, vbs = 0, rce = 0;
      if (ok) {
        const int i = c * X + e;
        vbl = t.bl[i];
        vbs = t.bS[i];
        rce = t.runs[i];
      }
      const int64_t vh = rce > 0 ? 1 : 0;
      const int64_t *cy = cb + 3 * e;
      int64_t xbl = wave_incl_suffix_max(vbl), xbs = wave_incl_suffix_max(vbs);
      xbl = cy[0] > xbl ? cy[0] : xbl;
      xbs = cy[1] > xbs ? cy[1] : xbs;
      const int64_t xh = wave_incl_suffix_sum(vh) + cy[2];
      // values of the ranks below r: the next lane's, or the carry for lane 63
      int64_t mbl = __shfl_down(xbl, 1), mbs = __shfl_down(xbs, 1), nlp = __shfl_down(xh, 1);
      if (lane == kWave - 1) {
        mbl = cy[0];
        mbs = cy[1];
        nlp = cy[2];
      }
      n_bp += rce * mbl;
      n_bs += rce * mbs;
      if (rce > 0) {
        n29 += nlp;
        m28 = mbs > m28 ? mbs : m28;
      }
      const int64_t nbl = __shfl(xbl, 0), nbs = __shfl(xbs, 0), nh = __shfl(xh, 0);
      __syncthreads();
      if (lane == 0) {
        cb[3 * e] = nbl;
        cb[3 * e + 1] = nbs;
        cb[3 * e + 2] = nh;
      }
    }
    int64_t n_bacc = 0;
    double f35 = 0.0;
    for (int a = 0; a < NA; ++a) {
      const int64_t m = cf[4 * (X + a) + 2];  // users of the accelerator
      if (m == 0) continue;                  // wave-uniform
      const int64_t nb = b.buckets[a0 + a];
      int64_t vu = 0, vA = 0;
      if (ok) {
        const int i = c * NAm + a;
        vu = t.dca[i] > 0 ? 1 : 0;
        vA = vu ? t.Amax[i] : 0;
      }
      const int64_t *cy = cb + 3 * (X + a);
      const int64_t su = wave_incl_suffix_sum(vu) + cy[0];  // users at rank r or below
      const int64_t key = ((m - su) * nb) / m;              // level of rank r
      int64_t xv = vA;
      for (int o = 1; o < kWave; o <<= 1) {
        const int64_t nv = __shfl_down(xv, o);
        const int64_t nk = __shfl_down(key, o);
        if (lane + o < kWave && nk == key) xv = nv > xv ? nv : xv;
      }
      if (key == cy[2]) xv = cy[1] > xv ? cy[1] : xv;
      int64_t nv = __shfl_down(xv, 1), nk = __shfl_down(key, 1);
      if (lane == kWave - 1) {
        nv = cy[1];
        nk = cy[2];
      }
      if ((uses >> a) & 1u) {
        n_bacc += (int64_t)t.dca[c * NAm + a] * (nk == key ? nv : 0);
        const double lvr = fratio(key, nb);
        f35 = lvr > f35 ? lvr : f35;
      }
      const int64_t ns = __shfl(su, 0), nxv = __shfl(xv, 0), nxk = __shfl(key, 0);
      __syncthreads();
      if (lane == 0) {
        cb[3 * (X + a)] = ns;
        cb[3 * (X + a) + 1] = nxv;
        cb[3 * (X + a) + 2] = nxk;
      }
    }
    if (ok) {
      const int64_t *w = t.fwd + (size_t)r * kFwd;
      FeatNums f;
      f.n19 = t.inv[c];
      f.n20 = t.inv[C + c];
      f.n_carry = w[0];
      f.q21 = w[1];
      f.q22 = w[2];
      f.q24 = w[3];
      f.n25 = w[4];
      f.n_acc = w[5];
      f.q33 = w[6];
      f.n36 = w[7];
      f.f37 = w[8];
      f.n_bp = n_bp;
      f.n_bs = n_bs;
      f.m28 = m28;
      f.n29 = n29;
      f.n_bacc = n_bacc;
      f.f35 = f35;
      hpp_terms(t, c, X, f);
      feat_write(b, set, t, c, r, f, rows + (size_t)c * 48);
    }
    __syncthreads();
  }
}

// Work item i: explicit pairs (one candidate each), or in range mode a run of
// up to 64 consecutive candidates of one set.  Tables in LDS (kLds) or in the
// wave's global scratch.
template <bool kLds>
__device__ __forceinline__ void features_body(FeatLaunch L) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  unsigned char *base = kLds ? lds_raw : L.scratch + (size_t)blockIdx.x * L.scratch_stride;
  const int NAmx = L.b.max_NA > 0 ? L.b.max_NA : 1;
  const FeatTables tw = carve_feat(base, L.b.max_C, L.b.max_X, NAmx);
  __shared__ int64_t scan_carry[kScanCarry];
  const int lane = threadIdx.x;
  // grid-stride: the item index is wave-uniform by construction
  for (int64_t i = blockIdx.x; i < L.n_items; i += gridDim.x) {
    FeatTables t = tw;
    int64_t set, k0, n_k, out0;
    int32_t u;
    if (L.pairs) {
      set = L.pairs[3 * i];
      k0 = L.pairs[3 * i + 1];
      const int64_t uu = L.pairs[3 * i + 2];
      n_k = 1;
      out0 = (int64_t)i;
      if (set < 0 || set >= L.b.n_sets || k0 < 0 || k0 > 0x7FFFFFFF || uu < 0 ||
          uu > 0x7FFFFFFF) {
        if (lane == 0) L.count[i] = -1;
        continue;
      }
      u = (int32_t)uu;
    } else {
      const int64_t per = (L.n_cand + L.item - 1) / L.item;
      set = L.set0 + (int64_t)i / per;
      k0 = ((int64_t)i % per) * L.item;
      n_k = L.n_cand - k0 < L.item ? L.n_cand - k0 : L.item;
      out0 = (set - L.set0) * L.n_cand + k0;
      u = L.util;
    }
    const int64_t c0 = L.b.set_chain_off[set];
    const int C = (int)(L.b.set_chain_off[set + 1] - c0);
    const bool shared = !kLds && !L.pairs && L.set_tables != nullptr;
    if (shared) {
      // the set's tables and row templates were built by feat_tables_kernel;
      // the walk state, ranks, inversion counts and forward numerators stay
      // in the wave's scratch
      t = carve_feat(L.set_tables + (size_t)(set - L.set0) * L.set_table_stride, L.b.max_C,
                     L.b.max_X, NAmx);
      t.order = tw.order;
      t.rank = tw.rank;
      t.buf = tw.buf;
      t.ordg = tw.ordg;
      t.rankg = tw.rankg;
      t.fwd = tw.fwd;
      t.inv = tw.inv;
    } else {
      feat_build(L.b, set, u, t);
    }
    if (t.setv[5] >= ((int64_t)1 << 40)) {
      // integer numerators could overflow: no features for this set
      for (int64_t k = lane; k < n_k; k += kWave) L.count[out0 + k] = -2;
      continue;
    }
    if (!shared)
      for (int c = lane; c < C; c += kWave) feat_template(L.b, set, t, c);
    for (int c = lane; c < C; c += kWave) {
      const int r = L.b.rank0[c0 + c];
      t.order[r] = c;
      t.rank[c] = (int16_t)r;
    }
    __syncthreads();
    int64_t cur = 0;
    if (!kLds && C > kScanC) {
      for (int64_t k = k0; k < k0 + n_k; ++k) {
        const bool step = k > k0 && k == cur + 1;
        walk_order(t.order, t.rank, C, L.seed, set, cur, k, t.buf);
        cur = k;
        const int32_t pq = step ? swap_positions(L.seed, set, k, C) : 0;
        feat_inversions(t, C, pq & 0xffff, pq >> 16, step);
        const int64_t o = out0 + (k - k0);
        feat_candidate_scan(L.b, set, t, scan_carry, L.feat + (size_t)o * L.row_stride * 48);
        if (lane == 0) L.count[o] = C;
      }
      continue;
    }
    int G = C <= 64 ? 64 / C : 1;
    G = G < kMaxGroup ? G : kMaxGroup;
    for (int64_t kb = k0; kb < k0 + n_k; kb += G) {
      const int ng = (int)(k0 + n_k - kb < G ? k0 + n_k - kb : G);
      // ranks of the pass's candidates: the walk to candidate kb, then one
      // swap per further candidate, applied by each lane to its own chain's
      // rank (the chains at the two swapped ranks trade ranks)
      walk_order(t.order, t.rank, C, L.seed, set, cur, kb, t.buf);
      if (C >= 2 && lane >= 1 && lane < ng) t.buf[lane] = swap_positions(L.seed, set, kb + lane, C);
      __syncthreads();
      for (int c = lane; c < C; c += kWave) {
        int r = t.rank[c];
        t.rankg[c] = (int16_t)r;
        for (int j = 1; j < ng; ++j) {
          if (C >= 2) {
            const int32_t pq = t.buf[j];
            const int pa = pq & 0xffff, pb = pq >> 16;
            r = r == pa ? pb : (r == pb ? pa : r);
          }
          t.rankg[j * C + c] = (int16_t)r;
        }
      }
      __syncthreads();
      for (int c = lane; c < C; c += kWave) {
        const int r = t.rankg[(ng - 1) * C + c];
        t.rank[c] = (int16_t)r;
        t.order[r] = c;
      }
      cur = kb + ng - 1;
      // chain at each rank of every candidate of the pass
      for (int idx = lane; idx < ng * C; idx += kWave) {
        const int g = idx / C, c = idx - g * C;
        t.ordg[g * C + t.rankg[g * C + c]] = c;
      }
      __syncthreads();
      feat_group_scan(L.b, set, t, C, ng, L.feat + (size_t)(out0 + (kb - k0)) * L.row_stride * 48,
                      L.row_stride);
      for (int g = lane; g < ng; g += kWave) L.count[out0 + (kb - k0) + g] = C;
      __syncthreads();
    }
  }
}

// The order-independent tables and row templates of sets set0 .. set0 +
// n_table_sets - 1, one wave per set, into the per-set buffers that the
// candidate items of the prefix-scan schedule then share (read only).
__global__ __launch_bounds__(kWave) void feat_tables_kernel(FeatLaunch L) {
  const int NAmx = L.b.max_NA > 0 ? L.b.max_NA : 1;
  for (int64_t s = blockIdx.x; s < L.n_table_sets; s += gridDim.x) {
    const int64_t set = L.set0 + s;
    FeatTables t =
        carve_feat(L.set_tables + (size_t)s * L.set_table_stride, L.b.max_C, L.b.max_X, NAmx);
    feat_build(L.b, set, L.util, t);
    if (t.setv[5] < ((int64_t)1 << 40)) {
      const int C = (int)(L.b.set_chain_off[set + 1] - L.b.set_chain_off[set]);
      for (int c = threadIdx.x; c < C; c += kWave) feat_template(L.b, set, t, c);
    }
    __syncthreads();
  }
}

// LDS tables (sets of up to 64 chains): four waves per SIMD.  Global tables:
// the register budget of three waves per SIMD, without spills.
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(4))) void features_kernel_lds(
    FeatLaunch L) {
  features_body<true>(L);
}
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3))) void features_kernel_glb(
    FeatLaunch L) {
  features_body<false>(L);
}

// ------------------------------------------------------------------ network

constexpr int NF = 48, NH = 256, KP = 64;
constexpr int OW1 = 0, OB1 = 12288, OW2 = 12544, OB2 = 78080, OW3 = 78336, OB3 = 78592;
constexpr int NPARAM = 78593;
constexpr int PW1 = 0, PW2 = NH * KP, PW3 = PW2 + NH * NH, NPACK = PW3 + NH;

// Packed bfloat16 copy of the weights (W1 padded to 64 columns).
__global__ void pack_kernel(const float *__restrict__ P, uint16_t *__restrict__ Q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPACK) return;
  float v = 0.0f;
  if (i < PW2) {
    const int j = i / KP, f = i % KP;
    v = f < NF ? P[OW1 + j * NF + f] : 0.0f;
  } else if (i < PW3) {
    v = P[OW2 + (i - PW2)];
  } else {
    v = P[OW3 + (i - PW3)];
  }
  Q[i] = bf16_rne(v);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
  const uint4 v = *reinterpret_cast<const uint4 *>(p);
  return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero8() {
  const uint4 v = make_uint4(0, 0, 0, 0);
  return __builtin_bit_cast(bf16x8, v);
}

// max(x, 0) for finite x in one instruction: the median of x, 0 and the
// largest finite float (fmaxf would add a NaN-quieting instruction).
__device__ __forceinline__ float relu(float x) {
  return __builtin_amdgcn_fmed3f(x, 0.0f, 3.4028234663852886e38f);
}

// The value held by the lane l ^ 32 (the other 32-lane half), by one
// v_permlane32_swap of the value with itself.
__device__ __forceinline__ float other_half(float v) {
  const int iv = __float_as_int(v);
  const auto r = __builtin_amdgcn_permlane32_swap(iv, iv, false, false);
  return __int_as_float((threadIdx.x & 32) ? r[0] : r[1]);
}

// Sum of a value over the four 16-lane groups of a wave (lanes l, l^16,
// l^32, l^48): ds_swizzle exchanges the two halves of each 32-lane half, and
// v_permlane32_swap exchanges the two 32-lane halves.
__device__ __forceinline__ float sum_lane_groups(float v) {
  v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
  const int iv = __float_as_int(v);
  const auto r = __builtin_amdgcn_permlane32_swap(iv, iv, false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}

// 8 features k0..k0+7 of a row (zero past the 48 features or past the rows);
// rows are 96 bytes apart, so 16-byte aligned when the buffer is.
__device__ __forceinline__ bf16x8 load_x8(const uint16_t *row, int k0, bool valid) {
  if (!valid || k0 >= NF) return zero8();
  return load8(row + k0);
}

// Forward pass, one workgroup of four waves per block of 64 candidates
// (grid-stride over blocks).  v_mfma_f32_16x16x32_bf16 lane layout: lane l
// holds A[l%16][8(l/16)..+7], B[8(l/16)..+7][l%16] and D[4(l/16)+j][l%16].
// Layer 1: wave w takes candidates 16w..16w+15 of the block, 16 rows at a
// time, with W1 staged in LDS; the ReLU outputs of the valid rows are summed
// per column into the pool.  Layer 2: the 64 pooled vectors (bfloat16, LDS)
// times W2^T, wave w taking output columns 64w..64w+63 for all 64
// candidates; layer 3 sums w3 * h2 per candidate across the waves in LDS.
constexpr int kFwdBlock = 64;
constexpr int kPqStride = NH + 8;  // padded row of the pooled tile (bank spread)

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void forward_kernel(FwdLaunch L) {
  __shared__ __attribute__((aligned(16))) uint16_t W1s[NH * KP];
  __shared__ __attribute__((aligned(16))) uint16_t Pq[kFwdBlock * kPqStride];
  __shared__ float ysum[4][kFwdBlock];
  __shared__ float b1s[NH];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int li = l & 15, lg = l >> 4;
  const uint16_t *W2 = L.packed + PW2, *w3 = L.packed + PW3;
  const float *b1 = L.params + OB1, *b2 = L.params + OB2;
  {
    const uint4 *src = reinterpret_cast<const uint4 *>(L.packed + PW1);
    uint4 *dst = reinterpret_cast<uint4 *>(W1s);
    for (int i = tid; i < NH * KP / 8; i += 256) dst[i] = src[i];
  }
  float bias1[16];
  for (int nt = 0; nt < 16; ++nt) bias1[nt] = b1[nt * 16 + li];
  for (int i = tid; i < NH; i += 256) b1s[i] = b1[i];
  const int64_t nblocks = (L.n + kFwdBlock - 1) / kFwdBlock;
  __syncthreads();
  for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int64_t base = blk * kFwdBlock;
    // ---- layer 1 and pooling: 16 candidates per wave.  The row counts of
    // the wave's candidates are read at once (one per lane), and the feature
    // tile after the current one is loaded before the current tile's MFMAs.
    int myrows = 0;
    if (l < 16 && base + w * 16 + l < L.n) myrows = L.count[base + w * 16 + l];
    myrows = myrows < 0 ? 0 : myrows;
    auto load_tile = [&](int m, int r0, bf16x8 &t0, bf16x8 &t1) {
      const int rows = __shfl(myrows, m);
      const uint16_t *X = L.feat + (size_t)(base + w * 16 + m) * L.row_stride * NF;
      const int r = r0 + li;
      const bool rv = r < rows;
      t0 = load_x8(X + (size_t)r * NF, 8 * lg, rv);
      t1 = load_x8(X + (size_t)r * NF, 32 + 8 * lg, rv);
    };
    // The MFMA accumulator starts at the bias, so a tile's outputs are the
    // pre-activations themselves.  Rows past a candidate's chains hold zero
    // features, so their pre-activation is exactly the bias: every row of a
    // tile is summed through the ReLU without a per-element mask, and
    // (rows in the tiles - chains) * ReLU(bias) is taken off once per column.
    // every candidate of the wave within one 16-row tile (sets of up to 16
    // chains): four candidates share each W1 fragment read from LDS
    if (!__any(l < 16 && myrows > 16)) {
      // the tiles of the next four candidates load during this group's work
      bf16x8 nx[4][2];
      for (int j = 0; j < 4; ++j) load_tile(j, 0, nx[j][0], nx[j][1]);
      for (int m0 = 0; m0 < 16; m0 += 4) {
        bf16x8 a[4][2];
        for (int j = 0; j < 4; ++j) {
          a[j][0] = nx[j][0];
          a[j][1] = nx[j][1];
        }
        if (m0 + 4 < 16)
          for (int j = 0; j < 4; ++j) load_tile(m0 + 4 + j, 0, nx[j][0], nx[j][1]);
        // lane group lg ends up with the sums of candidate m0 + lg
        const int rows = __shfl(myrows, m0 + lg);
        const float pad = (float)(16 - rows);
        const float inv = rows > 0 ? 1.0f / (float)rows : 0.0f;
        uint16_t *dst = Pq + (w * 16 + m0 + lg) * kPqStride + li;
#pragma unroll 2
        for (int nt = 0; nt < 16; ++nt) {
          const int n = nt * 16 + li;
          const bf16x8 bb0 = load8(W1s + n * KP + 8 * lg);
          const bf16x8 bb1 = load8(W1s + n * KP + 32 + 8 * lg);
          const float bias = b1s[nt * 16 + li];
          f32x4 acc[4];
          for (int j = 0; j < 4; ++j) {
            acc[j] = f32x4{bias, bias, bias, bias};
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j][0], bb0, acc[j], 0, 0, 0);
          }
          for (int j = 0; j < 4; ++j)
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j][1], bb1, acc[j], 0, 0, 0);
          float v[4];
          for (int j = 0; j < 4; ++j)
            v[j] = (relu(acc[j][0]) + relu(acc[j][1])) + (relu(acc[j][2]) + relu(acc[j][3]));
          // 4 x 4 transpose-and-add over the lane groups: first between lane
          // groups lg and lg ^ 1 (candidates of parity lg & 1 stay), then
          // between lg and lg ^ 2 (candidate lg stays)
          const bool odd = (lg & 1) != 0;
          const float s0 = odd ? v[0] : v[1], s1 = odd ? v[2] : v[3];
          const float r0 = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(s0), 0x401F));
          const float r1 = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(s1), 0x401F));
          const float x = (odd ? v[1] : v[0]) + r0;  // candidate lg & 1
          const float y = (odd ? v[3] : v[2]) + r1;  // candidate (lg & 1) + 2
          const bool up = (lg & 2) != 0;
          const float tot = (up ? y : x) + other_half(up ? x : y);
          dst[nt * 16] = bf16_rne((tot - pad * relu(bias)) * inv);
        }
      }
    } else {
      bf16x8 na0, na1;
      load_tile(0, 0, na0, na1);
      for (int m = 0; m < 16; ++m) {
        const int mb = w * 16 + m;
        const int rows = __shfl(myrows, m);
        float pool[16];
        for (int nt = 0; nt < 16; ++nt) pool[nt] = 0.0f;
        int tiles = 0;
        for (int r0 = 0;; r0 += 16) {
          const bf16x8 a0 = na0, a1 = na1;
          if (r0 + 16 < rows) {
            load_tile(m, r0 + 16, na0, na1);
          } else if (m + 1 < 16) {
            load_tile(m + 1, 0, na0, na1);
          }
          if (r0 < rows) {
            ++tiles;
#pragma unroll 4
            for (int nt = 0; nt < 16; ++nt) {
              const int n = nt * 16 + li;
              const bf16x8 bb0 = load8(W1s + n * KP + 8 * lg);
              const bf16x8 bb1 = load8(W1s + n * KP + 32 + 8 * lg);
              const float bias = bias1[nt];
              f32x4 acc = {bias, bias, bias, bias};
              acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bb0, acc, 0, 0, 0);
              acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bb1, acc, 0, 0, 0);
              pool[nt] += (relu(acc[0]) + relu(acc[1])) + (relu(acc[2]) + relu(acc[3]));
            }
          }
          if (r0 + 16 >= rows) break;
        }
        const float pad = (float)(16 * tiles - rows);
        const float inv = rows > 0 ? 1.0f / (float)rows : 0.0f;
        for (int nt = 0; nt < 16; ++nt) {
          const float sv = sum_lane_groups(pool[nt]);
          const float p = (sv - pad * relu(bias1[nt])) * inv;
          if (lg == 0) Pq[mb * kPqStride + nt * 16 + li] = bf16_rne(p);
        }
      }
    }
    // ---- layer 2 (64 x 256 x 256) and layer 3 partial sums.  Step k8 takes
    // k = 32 k8 .. 32 k8 + 31 for the wave's four column tiles: the four
    // pooled fragments (LDS) feed 16 MFMAs, and the W2 fragments (from L2) are
    // loaded two steps ahead, the first two before the barrier, so no MFMA
    // waits on a load issued just before it.  Every accumulator still sums k
    // in increasing order.
    auto load_w2 = [&](int k8, bf16x8 (&dst)[4]) {
      for (int q = 0; q < 4; ++q) {
        const int n = (w * 4 + q) * 16 + li;
        dst[q] = load8(W2 + (size_t)n * NH + 32 * k8 + 8 * lg);
      }
    };
    bf16x8 wb[3][4];
    load_w2(0, wb[0]);
    load_w2(1, wb[1]);
    __syncthreads();
    f32x4 acc2[4][4];
    for (int q = 0; q < 4; ++q)
      for (int mt = 0; mt < 4; ++mt) acc2[q][mt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k8 = 0; k8 < NH / 32; ++k8) {
      if (k8 + 2 < NH / 32) load_w2(k8 + 2, wb[(k8 + 2) % 3]);
      bf16x8 a[4];
      for (int mt = 0; mt < 4; ++mt) a[mt] = load8(Pq + (mt * 16 + li) * kPqStride + 32 * k8 + 8 * lg);
      for (int q = 0; q < 4; ++q)
        for (int mt = 0; mt < 4; ++mt)
          acc2[q][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], wb[k8 % 3][q], acc2[q][mt], 0, 0, 0);
    }
    float yp[4][4];
    for (int mt = 0; mt < 4; ++mt)
      for (int j = 0; j < 4; ++j) yp[mt][j] = 0.0f;
    for (int q = 0; q < 4; ++q) {
      const int n = (w * 4 + q) * 16 + li;
      const float bias = b2[n];
      const float wv = bf16_value(w3[n]);
      for (int mt = 0; mt < 4; ++mt) {
        for (int j = 0; j < 4; ++j) {
          const int mb = mt * 16 + 4 * lg + j;
          const float z = acc2[q][mt][j] + bias;
          const uint16_t hq = bf16_rne(z > 0.0f ? z : 0.0f);
          yp[mt][j] += wv * bf16_value(hq);
          if (L.act && base + mb < L.n)
            reinterpret_cast<uint16_t *>(L.act)[(size_t)(base + mb) * 512 + 256 + n] = hq;
        }
      }
    }
    // sum over the 16 lanes of a row group, then over the four waves
    for (int mt = 0; mt < 4; ++mt) {
      for (int j = 0; j < 4; ++j) {
        float sv = yp[mt][j];
        sv += __shfl_xor(sv, 1);
        sv += __shfl_xor(sv, 2);
        sv += __shfl_xor(sv, 4);
        sv += __shfl_xor(sv, 8);
        if (li == 0) ysum[w][mt * 16 + 4 * lg + j] = sv;
      }
    }
    if (L.act) {
      for (int i = tid; i < kFwdBlock * NH; i += 256) {
        const int mb = i / NH, k = i - mb * NH;
        if (base + mb < L.n)
          reinterpret_cast<uint16_t *>(L.act)[(size_t)(base + mb) * 512 + k] = Pq[mb * kPqStride + k];
      }
    }
    __syncthreads();
    if (tid < kFwdBlock && base + tid < L.n)
      L.out[base + tid] = ((ysum[0][tid] + ysum[1][tid]) + (ysum[2][tid] + ysum[3][tid])) +
                          L.params[OB3];
    __syncthreads();
  }
}

// Backward over a chunk of kBwdChunk candidates per workgroup of 256 threads
// (thread j = hidden unit j); writes this chunk's partial gradient.
constexpr int kBwdChunk = 16;
constexpr int kBwdRows = 64;  // feature rows staged in LDS at a time
constexpr int kBwdThreads = NH;

__global__ __launch_bounds__(kBwdThreads) void backward_kernel(BwdLaunch L) {
  __shared__ __attribute__((aligned(16))) float dz2[NH][kBwdChunk];  // [hidden unit][candidate]
  __shared__ float pq[kBwdChunk][NH];
  __shared__ float dp[kBwdChunk][NH];
  __shared__ __attribute__((aligned(16))) float xs[kBwdRows][NF];
  const int j = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * kBwdChunk;
  const int nc = (int)((L.n - c0) < kBwdChunk ? (L.n - c0) : kBwdChunk);
  float *part = L.partial + (size_t)blockIdx.x * L.part_stride;
  const uint16_t *W2 = L.packed + PW2, *W1 = L.packed + PW1;
  const float w3j = bf16_value(L.packed[PW3 + j]);
  const float inv_n = 1.0f / (float)L.n;
  float gw3 = 0.0f, gb2 = 0.0f, gb3 = 0.0f, lsum = 0.0f;
  for (int m = 0; m < nc; ++m) {
    const int64_t cand = c0 + m;
    const uint16_t *a = reinterpret_cast<const uint16_t *>(L.act) + (size_t)cand * 512;
    const float d = L.out[cand] - L.target[cand];
    const float dy = 2.0f * d * inv_n;
    const float h2 = bf16_value(a[256 + j]);
    const float g = h2 > 0.0f ? dy * w3j : 0.0f;
    dz2[j][m] = g;
    pq[m][j] = bf16_value(a[j]);
    gw3 += dy * h2;
    gb2 += g;
    if (j == 0) {
      gb3 += dy;
      lsum += d * d;
    }
  }
  for (int m = nc; m < kBwdChunk; ++m) dz2[j][m] = 0.0f;
  __syncthreads();
  // dW2[i][j] = sum_m dz2(m, i) * pq[m][j]: thread j owns column j, so the
  // stores of every row are coalesced across the threads
  {
    float pqj[kBwdChunk];
    for (int m = 0; m < kBwdChunk; ++m) pqj[m] = m < nc ? pq[m][j] : 0.0f;
    for (int i = 0; i < NH; ++i) {
      float s = 0.0f;
      for (int m = 0; m < nc; ++m) s += dz2[i][m] * pqj[m];
      part[OW2 + i * NH + j] = s;
    }
  }
  // dp[m][k = j] = sum_i dz2(m, i) * W2[i][j]: each W2 element is read once
  // and feeds the chunk's candidates (every sum still runs over i in order)
  {
    float acc[kBwdChunk];
    for (int m = 0; m < kBwdChunk; ++m) acc[m] = 0.0f;
    for (int i = 0; i < NH; ++i) {
      const float w = bf16_value(W2[(size_t)i * NH + j]);
      for (int m = 0; m < kBwdChunk; ++m) acc[m] += dz2[i][m] * w;
    }
    for (int m = 0; m < nc; ++m) dp[m][j] = acc[m];
  }
  __syncthreads();
  // layer 1: recompute z1 per row, dz1 = dp / rows where z1 > 0.  A
  // candidate's rows are staged in LDS kBwdRows at a time; four rows are
  // evaluated together (independent dot products), and their contributions
  // are added in row order; a row whose z1 is not positive adds zeros, which
  // leaves every sum's bits unchanged, so no lane branches.
  float gw1[NF];
  for (int f = 0; f < NF; ++f) gw1[f] = 0.0f;
  float gb1 = 0.0f;
  float w1[NF];
  for (int f = 0; f < NF; ++f) w1[f] = bf16_value(W1[(size_t)j * KP + f]);
  const float b1j = L.params[OB1 + j];
  auto add_row = [&](const float *x, float g) {
    gb1 += g;
    for (int f = 0; f < NF; ++f) gw1[f] += g * x[f];
  };
  for (int m = 0; m < nc; ++m) {
    const int64_t cand = c0 + m;
    const int rows = L.count[cand] > 0 ? L.count[cand] : 0;
    const float g = rows > 0 ? dp[m][j] / (float)rows : 0.0f;
    const uint16_t *X = L.feat + (size_t)cand * L.row_stride * NF;
    for (int r0 = 0; r0 < rows; r0 += kBwdRows) {
      const int nr = rows - r0 < kBwdRows ? rows - r0 : kBwdRows;
      __syncthreads();  // the previous tile is consumed
      for (int i = j; i < nr * NF; i += kBwdThreads)
        xs[i / NF][i % NF] = bf16_value(X[(size_t)r0 * NF + i]);
      __syncthreads();
      int r = 0;
      for (; r + 4 <= nr; r += 4) {
        float z0 = b1j, z1 = b1j, z2 = b1j, z3 = b1j;
        for (int f = 0; f < NF; ++f) {
          z0 += w1[f] * xs[r][f];
          z1 += w1[f] * xs[r + 1][f];
          z2 += w1[f] * xs[r + 2][f];
          z3 += w1[f] * xs[r + 3][f];
        }
        add_row(xs[r], z0 > 0.0f ? g : 0.0f);
        add_row(xs[r + 1], z1 > 0.0f ? g : 0.0f);
        add_row(xs[r + 2], z2 > 0.0f ? g : 0.0f);
        add_row(xs[r + 3], z3 > 0.0f ? g : 0.0f);
      }
      for (; r < nr; ++r) {
        float z = b1j;
        for (int f = 0; f < NF; ++f) z += w1[f] * xs[r][f];
        add_row(xs[r], z > 0.0f ? g : 0.0f);
      }
    }
  }
  for (int f = 0; f < NF; ++f) part[OW1 + j * NF + f] = gw1[f];
  part[OB1 + j] = gb1;
  part[OB2 + j] = gb2;
  part[OW3 + j] = gw3;
  if (j == 0) {
    part[OB3] = gb3;
    part[NPARAM] = lsum;
  }
}

// grad[i] = sum over chunks in order; loss = sum of squared errors / n.
__global__ void reduce_kernel(const float *__restrict__ partial, size_t stride, int chunks,
                              int64_t n, float *__restrict__ grad, float *__restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > NPARAM) return;
  float s = 0.0f;
  for (int c = 0; c < chunks; ++c) s += partial[(size_t)c * stride + i];
  if (i < NPARAM) {
    grad[i] = s;
  } else if (loss) {
    loss[0] = s / (float)n;
  }
}

__global__ void adam_kernel(float *__restrict__ P, uint16_t *__restrict__ Q, float *__restrict__ M,
                            float *__restrict__ V, const float *__restrict__ G, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const float g = G[i];
  const float m = b1 * M[i] + (1.0f - b1) * g;
  const float v = b2 * V[i] + (1.0f - b2) * g * g;
  M[i] = m;
  V[i] = v;
  const float mh = m / c1, vh = v / c2;
  const float p = P[i] - lr * mh / (sqrtf(vh) + eps);
  P[i] = p;
  // repack the weight this parameter feeds (biases have no packed copy)
  if (i < OB1) {
    Q[PW1 + (i / NF) * KP + (i % NF)] = bf16_rne(p);
  } else if (i >= OW2 && i < OB2) {
    Q[PW2 + (i - OW2)] = bf16_rne(p);
  } else if (i >= OW3 && i < OB3) {
    Q[PW3 + (i - OW3)] = bf16_rne(p);
  }
}

}  // namespace

size_t feat_wave_bytes(const DevBatch &b) {
  const int NAm = b.max_NA > 0 ? b.max_NA : 1;
  return (feat_table_bytes(b.max_C, b.max_X, NAm) + 255) & ~(size_t)255;
}

// Sets of more than kScanC chains take the prefix-scan schedule, which keeps
// its tables in global memory.
bool feat_in_lds(const DevBatch &b) {
  return b.max_C <= kScanC && feat_wave_bytes(b) <= kFeatLdsMax;
}

int feat_item(const DevBatch &b) { return feat_in_lds(b) ? kFeatItemLds : kFeatItemScan; }

int launch_feat_tables(const FeatLaunch &L, int grid, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (L.n_table_sets == 0) return 0;
  hipLaunchKernelGGL(feat_tables_kernel, dim3(grid), dim3(kWave), 0, st, L);
  return (int)hipGetLastError();
}

int launch_features(const FeatLaunch &L, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (L.n_items == 0) return 0;
  if (feat_in_lds(L.b)) {
    hipLaunchKernelGGL(features_kernel_lds, dim3(L.grid), dim3(kWave), feat_wave_bytes(L.b), st,
                       L);
  } else {
    hipLaunchKernelGGL(features_kernel_glb, dim3(L.grid), dim3(kWave), 0, st, L);
  }
  return (int)hipGetLastError();
}

int launch_pack(const float *params, uint16_t *packed, void *stream) {
  hipLaunchKernelGGL(pack_kernel, dim3((NPACK + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     params, packed);
  return (int)hipGetLastError();
}

int launch_forward(const FwdLaunch &L, void *stream) {
  if (L.n == 0) return 0;
  const int64_t blocks = (L.n + kFwdBlock - 1) / kFwdBlock;
  const int64_t grid = blocks < 4096 ? blocks : 4096;  // persistent: 16 workgroups per CU at most
  hipLaunchKernelGGL(forward_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, L);
  return (int)hipGetLastError();
}

size_t backward_partial_stride() { return ((size_t)NPARAM + 1 + 63) & ~(size_t)63; }
int64_t backward_chunks(int64_t n) { return (n + kBwdChunk - 1) / kBwdChunk; }

int launch_backward(const BwdLaunch &L, float *grad, float *loss, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (L.n == 0) return 0;
  const int64_t chunks = backward_chunks(L.n);
  hipLaunchKernelGGL(backward_kernel, dim3((unsigned)chunks), dim3(kBwdThreads), 0, st, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  hipLaunchKernelGGL(reduce_kernel, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, st,
                     (const float *)L.partial, L.part_stride, (int)chunks, L.n, grad, loss);
  return (int)hipGetLastError();
}

int launch_adam(float *P, uint16_t *Q, float *M, float *V, const float *G, float lr, float b1,
                float b2, float eps, int64_t step, void *stream) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, P,
                     Q, M, V, G, lr, b1, b2, eps, c1, c2);
  return (int)hipGetLastError();
}

}  // namespace paam
