// Host side of libpaam: validation of the problem statement (Sec. II-C),
// derivation of its priority-independent structure, packing of the device
// arena, and the C-ABI entry points declared in include/paam.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "paam_internal.h"

namespace {

thread_local std::string g_err;

paam_status fail(paam_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

paam_status hip_fail(hipError_t e, const char *what) {
  return fail(PAAM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// 1/T rounded towards +inf: the smallest double c with c*T >= 1.
double rcp_up(int64_t T) {
  double c = 1.0 / (double)T;
  if (std::fma(c, (double)T, -1.0) < 0.0) c = std::nextafter(c, INFINITY);
  return c;
}

int device_ok(std::string *why) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *why = std::string("no HIP device: ") + hipGetErrorString(e);
    return 0;
  }
  hipDeviceProp_t p;
  e = hipGetDeviceProperties(&p, dev);
  if (e != hipSuccess) {
    *why = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e);
    return 0;
  }
  if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) {
    *why = std::string("device is ") + p.gcnArchName + ", libpaam is built for gfx950";
    return 0;
  }
  return 1;
}

// Structure derived on the host.
struct Plan {
  int64_t n_sets = 0, n_chains = 0, n_cbs = 0, n_segs = 0, n_runs = 0, n_exec = 0, n_accel = 0;
  std::vector<int64_t> set_cb_off, set_seg_off, set_run_off;
  std::vector<int16_t> run_chain, run_exec;
  std::vector<int32_t> run_cb_lo, run_cb_hi, chain_nrun, seg_order;
  std::vector<int16_t> rank0, seg_chain;
  std::vector<int8_t> cb_exec;
  std::vector<int32_t> chain_cb_lo;
  std::vector<uint32_t> hpx_mask;
  std::vector<double> Kd, rcp, KRr;
  std::vector<int32_t> buckets;
  std::vector<int64_t> aeps, akappa;
  // analysed accelerators per set: the input accelerators, or their units
  std::vector<int64_t> set_accel_x;
  int64_t n_types = 0;
  int32_t unit_group = -1;
  int32_t max_cb_segs = 0, max_buckets = 0, max_set_cbs = 0;
  std::vector<int64_t> work_order;
  int32_t max_C = 0, max_X = 0, max_NA = 0, max_runs = 0, max_segs = 0;
  std::vector<paam::SizeClass> classes;
  int64_t max_tot = 0;
};

#define REQ(cond, ...)                                   \
  do {                                                   \
    if (!(cond)) return fail(PAAM_E_INVAL, __VA_ARGS__); \
  } while (0)
#define RNG(cond, ...)                                   \
  do {                                                   \
    if (!(cond)) return fail(PAAM_E_RANGE, __VA_ARGS__); \
  } while (0)

// Runs f(lo, hi) over [0, n) on a few threads; returns the status of the
// lowest failing range (and keeps its message), or PAAM_OK.
template <class F>
paam_status parallel_ranges(int64_t n, F f) {
  int nt = (int)std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()), 16);
  if (n < 4096) nt = 1;
  std::vector<paam_status> st(nt, PAAM_OK);
  std::vector<std::string> msg(nt);
  auto body = [&](int t) {
    const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
    st[t] = f(lo, hi);
    if (st[t] != PAAM_OK) msg[t] = g_err;
  };
  if (nt == 1) {
    body(0);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(body, t);
    for (auto &x : th) x.join();
  }
  for (int t = 0; t < nt; ++t)
    if (st[t] != PAAM_OK) {
      g_err = msg[t];
      return st[t];
    }
  return PAAM_OK;
}

// Validates one set and returns its sub-chain count in *nrun.
paam_status check_set(const paam_chainset_host *h, int64_t s, int *nrun, double *cost,
                      int64_t *tot) {
  using paam::kTimeLimit;
  const int64_t c0 = h->set_chain_off[s];
  const int C = (int)(h->set_chain_off[s + 1] - c0);
  const int64_t x0 = h->set_exec_off[s];
  const int X = (int)(h->set_exec_off[s + 1] - x0);
  const int NA = (int)(h->set_accel_off[s + 1] - h->set_accel_off[s]);
  for (int e = 0; e < X; ++e)
    for (int f = 0; f < e; ++f)
      REQ(!(h->exec_core[x0 + e] == h->exec_core[x0 + f] &&
            h->exec_prio[x0 + e] == h->exec_prio[x0 + f]),
          "set %lld: executors %d and %d share core and process priority", (long long)s, f, e);
  std::vector<int32_t> pr(C);
  for (int c = 0; c < C; ++c) pr[c] = h->prio[c0 + c];
  std::sort(pr.begin(), pr.end());
  for (int c = 1; c < C; ++c)
    REQ(pr[c] != pr[c - 1], "set %lld: duplicate chain priority", (long long)s);
  int runs = 0;
  const int64_t a0 = h->set_accel_off[s];
  int64_t total = 0;  // saturates at 2^62
  auto add = [&](int64_t v) { total = total > ((int64_t)1 << 62) - v ? (int64_t)1 << 62 : total + v; };
  for (int c = 0; c < C; ++c) {
    const int64_t T = h->T[c0 + c], D = h->D[c0 + c];
    REQ(T > 0 && D > 0 && D <= T, "chain %lld: need 0 < D <= T (T=%lld D=%lld)",
        (long long)(c0 + c), (long long)T, (long long)D);
    RNG(T < kTimeLimit, "chain %lld: period >= 2^36 ns", (long long)(c0 + c));
    int prev_e = -1;
    for (int64_t j = h->chain_cb_off[c0 + c]; j < h->chain_cb_off[c0 + c + 1]; ++j) {
      const int e = h->exec[j];
      REQ(e >= 0 && e < X, "callback %lld: executor %d out of range", (long long)j, e);
      REQ(h->E[j] >= 0, "callback %lld: negative E", (long long)j);
      RNG(h->E[j] < kTimeLimit, "callback %lld: E >= 2^36 ns", (long long)j);
      for (int64_t g = h->cb_seg_off[j]; g < h->cb_seg_off[j + 1]; ++g) {
        REQ(h->A[g] >= 0, "segment %lld: negative A", (long long)g);
        RNG(h->A[g] < kTimeLimit, "segment %lld: A >= 2^36 ns", (long long)g);
        REQ(h->accel[g] >= 0 && h->accel[g] < NA, "segment %lld: accelerator out of range",
            (long long)g);
        add(h->A[g] + 2 * h->accel_kappa[a0 + h->accel[g]] + h->accel_eps[a0 + h->accel[g]]);
      }
      add(h->E[j]);
      if (e != prev_e) ++runs;
      prev_e = e;
    }
  }
  RNG(runs <= paam::kMaxRuns, "set %lld: %d sub-chains (max %d)", (long long)s, runs,
      paam::kMaxRuns);
  RNG(h->eps_hop[s] >= 0 && h->eps_hop[s] < kTimeLimit, "set %lld: hop cost outside [0, 2^36)",
      (long long)s);
  const int64_t cb0 = h->chain_cb_off[c0], cb1 = h->chain_cb_off[c0 + C];
  const int64_t nseg = h->cb_seg_off[cb1] - h->cb_seg_off[cb0];
  RNG(nseg <= (int64_t)1 << 30 && cb1 - cb0 <= (int64_t)1 << 30, "set %lld too large",
      (long long)s);
  *nrun = runs;
  *cost = (double)runs * (double)(C + 4) + (double)nseg * (double)C;
  *tot = total;
  return PAAM_OK;
}

// Fills the derived arrays of one set (after validation).
void fill_set(const paam_chainset_host *h, int64_t s, Plan &P) {
  const int64_t c0 = h->set_chain_off[s];
  const int C = (int)(h->set_chain_off[s + 1] - c0);
  const int64_t x0 = h->set_exec_off[s];
  const int X = (int)(h->set_exec_off[s + 1] - x0);
  const int64_t cb0 = h->chain_cb_off[c0], cb1 = h->chain_cb_off[c0 + C];
  const int64_t g0 = h->cb_seg_off[cb0], g1 = h->cb_seg_off[cb1];
  P.set_cb_off[s] = cb0;
  P.set_seg_off[s] = g0;
  for (int e = 0; e < X; ++e) {
    uint32_t m = 0;
    for (int f = 0; f < X; ++f)
      if (f != e && h->exec_core[x0 + e] == h->exec_core[x0 + f] &&
          h->exec_prio[x0 + f] > h->exec_prio[x0 + e])
        m |= 1u << f;
    P.hpx_mask[x0 + e] = m;
  }
  std::vector<int> order(C);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return h->prio[c0 + a] > h->prio[c0 + b]; });
  for (int r = 0; r < C; ++r) {
    const int c = order[r];
    P.rank0[c0 + c] = (int16_t)r;
    P.KRr[2 * (c0 + r)] = P.Kd[c0 + c];
    P.KRr[2 * (c0 + r) + 1] = P.rcp[c0 + c];
  }
  // sub-chains in chain order, then sorted by (hpp above, rank, position)
  struct Run {
    int16_t chain, exec;
    int32_t lo, hi;
  };
  std::vector<Run> runs;
  for (int c = 0; c < C; ++c) {
    int prev_e = -1;
    for (int64_t j = h->chain_cb_off[c0 + c]; j < h->chain_cb_off[c0 + c + 1]; ++j) {
      const int e = h->exec[j];
      const int jl = (int)(j - cb0);
      if (e != prev_e) {
        runs.push_back(Run{(int16_t)c, (int16_t)e, jl, jl + 1});
        prev_e = e;
      } else {
        runs.back().hi = jl + 1;
      }
    }
    for (int64_t j = h->chain_cb_off[c0 + c]; j < h->chain_cb_off[c0 + c + 1]; ++j) {
      for (int64_t g = h->cb_seg_off[j]; g < h->cb_seg_off[j + 1]; ++g) P.seg_chain[g] = (int16_t)c;
      P.cb_exec[j] = (int8_t)h->exec[j];
    }
    P.chain_cb_lo[c0 + c] = (int32_t)(h->chain_cb_off[c0 + c] - cb0);
  }
  for (const Run &r : runs) P.chain_nrun[c0 + r.chain]++;
  std::stable_sort(runs.begin(), runs.end(), [&](const Run &a, const Run &b) {
    const bool pa = P.hpx_mask[x0 + a.exec] != 0, pb = P.hpx_mask[x0 + b.exec] != 0;
    if (pa != pb) return pa < pb;
    return P.rank0[c0 + a.chain] < P.rank0[c0 + b.chain];
  });
  const int64_t r0 = P.set_run_off[s];
  for (size_t i = 0; i < runs.size(); ++i) {
    P.run_chain[r0 + i] = runs[i].chain;
    P.run_exec[r0 + i] = runs[i].exec;
    P.run_cb_lo[r0 + i] = runs[i].lo;
    P.run_cb_hi[r0 + i] = runs[i].hi;
  }
  std::vector<int32_t> so((size_t)(g1 - g0));
  std::iota(so.begin(), so.end(), 0);
  std::stable_sort(so.begin(), so.end(), [&](int a, int b) {
    return P.rank0[c0 + P.seg_chain[g0 + a]] < P.rank0[c0 + P.seg_chain[g0 + b]];
  });
  std::copy(so.begin(), so.end(), P.seg_order.begin() + g0);
}

paam_status make_plan(const paam_chainset_host *h, Plan &P) {
  using paam::kTimeLimit;
  REQ(h, "null batch");
  REQ(h->n_sets >= 0, "n_sets < 0");
  REQ(h->set_chain_off && h->set_exec_off && h->set_accel_off && h->chain_cb_off &&
          h->cb_seg_off && h->T && h->D && h->prio && h->spin && h->E && h->exec &&
          h->exec_core && h->exec_prio && h->accel_buckets && h->accel_eps && h->accel_kappa &&
          h->eps_hop,
      "null array in batch");
  const int64_t S = h->n_sets;
  P.n_sets = S;
  REQ(h->set_chain_off[0] == 0 && h->set_exec_off[0] == 0 && h->set_accel_off[0] == 0,
      "set offsets must start at 0");
  for (int64_t s = 0; s < S; ++s) {
    const int64_t C = h->set_chain_off[s + 1] - h->set_chain_off[s];
    const int64_t X = h->set_exec_off[s + 1] - h->set_exec_off[s];
    const int64_t NA = h->set_accel_off[s + 1] - h->set_accel_off[s];
    REQ(C >= 1 && C <= paam::kMaxChains, "set %lld: %lld chains (1..%d)", (long long)s,
        (long long)C, paam::kMaxChains);
    REQ(X >= 1 && X <= paam::kMaxExec, "set %lld: %lld executors (1..%d)", (long long)s,
        (long long)X, paam::kMaxExec);
    REQ(NA >= 0 && NA <= paam::kMaxAccel, "set %lld: %lld accelerators (0..%d)", (long long)s,
        (long long)NA, paam::kMaxAccel);
  }
  const int64_t NC = h->set_chain_off[S], NX = h->set_exec_off[S], NAc = h->set_accel_off[S];
  P.n_chains = NC;
  P.n_exec = NX;
  P.n_accel = NAc;
  REQ(h->chain_cb_off[0] == 0, "chain_cb_off must start at 0");
  for (int64_t c = 0; c < NC; ++c)
    REQ(h->chain_cb_off[c + 1] > h->chain_cb_off[c], "chain %lld has no callback", (long long)c);
  const int64_t NJ = h->chain_cb_off[NC];
  P.n_cbs = NJ;
  REQ(h->cb_seg_off[0] == 0, "cb_seg_off must start at 0");
  for (int64_t j = 0; j < NJ; ++j) {
    REQ(h->cb_seg_off[j + 1] >= h->cb_seg_off[j], "cb_seg_off decreases at %lld", (long long)j);
    P.max_cb_segs = std::max<int32_t>(P.max_cb_segs, (int32_t)std::min<int64_t>(
                                                         h->cb_seg_off[j + 1] - h->cb_seg_off[j], 1 << 30));
  }
  const int64_t NG = h->cb_seg_off[NJ];
  P.n_segs = NG;
  REQ(NG == 0 || (h->A && h->accel), "segments present but A/accel null");
  for (int64_t a = 0; a < NAc; ++a) {
    REQ(h->accel_buckets[a] >= 1, "accelerator %lld: buckets < 1", (long long)a);
    REQ(h->accel_eps[a] >= 0 && h->accel_kappa[a] >= 0, "accelerator %lld: negative overhead",
        (long long)a);
    RNG(h->accel_eps[a] < kTimeLimit && h->accel_kappa[a] < kTimeLimit,
        "accelerator %lld: overhead >= 2^36 ns", (long long)a);
    P.max_buckets = std::max<int32_t>(P.max_buckets, h->accel_buckets[a]);
  }
  // units of accelerator types (Sec. IV-E): each unit is analysed as an
  // accelerator of its own with its type's buckets and overheads
  P.n_types = NAc;
  P.set_accel_x.assign(h->set_accel_off, h->set_accel_off + S + 1);
  if (h->accel_units) {
    REQ(h->unit_group >= PAAM_UNITS_SEGMENT && h->unit_group <= PAAM_UNITS_CHAIN,
        "unit_group %d is not a PAAM_UNITS_* value", h->unit_group);
    P.unit_group = h->unit_group;
    for (int64_t a = 0; a < NAc; ++a)
      REQ(h->accel_units[a] >= 1 && h->accel_units[a] <= paam::kMaxAccel,
          "accelerator %lld: %d units (1..%d)", (long long)a, (int)h->accel_units[a],
          paam::kMaxAccel);
    for (int64_t s = 0; s < S; ++s) {
      int64_t n = 0;
      for (int64_t a = h->set_accel_off[s]; a < h->set_accel_off[s + 1]; ++a)
        n += h->accel_units[a];
      RNG(n <= paam::kMaxAccel, "set %lld: %lld accelerator units (max %d)", (long long)s,
          (long long)n, paam::kMaxAccel);
      P.set_accel_x[s + 1] = P.set_accel_x[s] + n;
    }
  }
  for (int64_t a = 0; a < NAc; ++a)
    for (int u = 0; u < (h->accel_units ? h->accel_units[a] : 1); ++u) {
      P.buckets.push_back(h->accel_buckets[a]);
      P.aeps.push_back(h->accel_eps[a]);
      P.akappa.push_back(h->accel_kappa[a]);
    }
  P.n_accel = P.set_accel_x[S];

  // pass 1: validate every set, count its sub-chains
  std::vector<int> nrun(S);
  std::vector<double> cost(S);
  std::vector<int64_t> tot(S);
  paam_status st = parallel_ranges(S, [&](int64_t lo, int64_t hi) -> paam_status {
    for (int64_t s = lo; s < hi; ++s) {
      paam_status r = check_set(h, s, &nrun[s], &cost[s], &tot[s]);
      if (r != PAAM_OK) return r;
    }
    return PAAM_OK;
  });
  if (st != PAAM_OK) return st;
  P.set_cb_off.resize(S + 1);
  P.set_seg_off.resize(S + 1);
  P.set_run_off.assign(S + 1, 0);
  for (int64_t s = 0; s < S; ++s) {
    P.set_run_off[s + 1] = P.set_run_off[s] + nrun[s];
    const int64_t c0 = h->set_chain_off[s];
    const int C = (int)(h->set_chain_off[s + 1] - c0);
    const int64_t cb0 = h->chain_cb_off[c0], cb1 = h->chain_cb_off[c0 + C];
    P.max_C = std::max(P.max_C, C);
    P.max_X = std::max(P.max_X, (int32_t)(h->set_exec_off[s + 1] - h->set_exec_off[s]));
    P.max_NA = std::max(P.max_NA, (int32_t)(P.set_accel_x[s + 1] - P.set_accel_x[s]));
    P.max_runs = std::max(P.max_runs, nrun[s]);
    P.max_tot = std::max(P.max_tot, tot[s]);
    P.max_segs = std::max(P.max_segs, (int32_t)(h->cb_seg_off[cb1] - h->cb_seg_off[cb0]));
    P.max_set_cbs = std::max(P.max_set_cbs, (int32_t)(cb1 - cb0));
  }
  RNG(!h->accel_units || P.max_segs <= paam::kMaxUnitSegs,
      "a set has %d segments; with accelerator units at most %d", P.max_segs, paam::kMaxUnitSegs);
  P.n_runs = P.set_run_off[S];
  P.set_cb_off[S] = NJ;
  P.set_seg_off[S] = NG;

  // pass 2: derived arrays
  P.Kd.resize(NC);
  P.rcp.resize(NC);
  for (int64_t c = 0; c < NC; ++c) {
    P.Kd[c] = (double)(2 * h->T[c] - 1);
    P.rcp[c] = rcp_up(h->T[c]);
  }
  P.KRr.resize(2 * NC);
  P.rank0.resize(NC);
  P.chain_nrun.assign(NC, 0);
  P.seg_chain.resize(NG);
  P.seg_order.resize(NG);
  P.cb_exec.resize(NJ);
  P.chain_cb_lo.resize(NC);
  P.hpx_mask.assign(NX, 0u);
  P.run_chain.resize(P.n_runs);
  P.run_exec.resize(P.n_runs);
  P.run_cb_lo.resize(P.n_runs);
  P.run_cb_hi.resize(P.n_runs);
  parallel_ranges(S, [&](int64_t lo, int64_t hi) -> paam_status {
    for (int64_t s = lo; s < hi; ++s) fill_set(h, s, P);
    return PAAM_OK;
  });
  // work order: by size class (chain count up to 16, 32, 64, ...), then by
  // decreasing estimated cost within a class
  auto size_class = [&](int64_t s) {
    const int C = (int)(h->set_chain_off[s + 1] - h->set_chain_off[s]);
    int k = 0;
    while ((16 << k) < C) ++k;
    return k;
  };
  P.work_order.resize(S);
  std::iota(P.work_order.begin(), P.work_order.end(), 0);
  std::stable_sort(P.work_order.begin(), P.work_order.end(), [&](int64_t a, int64_t b) {
    const int ka = size_class(a), kb = size_class(b);
    if (ka != kb) return ka < kb;
    return cost[a] > cost[b];
  });
  for (int64_t i = 0; i < S; ++i) {
    const int64_t s = P.work_order[i];
    const int k = size_class(s);
    if (P.classes.empty() || size_class(P.work_order[P.classes.back().begin]) != k)
      P.classes.push_back(paam::SizeClass{i, 0, 0, 0, 0, 1, 1, 0, 0});
    paam::SizeClass &c = P.classes.back();
    const int64_t c0 = h->set_chain_off[s];
    const int C = (int)(h->set_chain_off[s + 1] - c0);
    const int64_t cb0 = h->chain_cb_off[c0], cb1 = h->chain_cb_off[c0 + C];
    c.count += 1;
    c.max_C = std::max(c.max_C, C);
    c.max_X = std::max(c.max_X, (int32_t)(h->set_exec_off[s + 1] - h->set_exec_off[s]));
    c.max_NA = std::max(c.max_NA, (int32_t)(P.set_accel_x[s + 1] - P.set_accel_x[s]));
    c.max_runs = std::max(c.max_runs, nrun[s]);
    c.max_segs = std::max(c.max_segs, (int32_t)(h->cb_seg_off[cb1] - h->cb_seg_off[cb0]));
  }
  // the per-wave LDS tables of each class (the search and candidate kernels,
  // whose layout is the larger) must fit the 160 KB of a compute unit
  for (const paam::SizeClass &c : P.classes) {
    paam::DevBatch b{};
    b.max_C = c.max_C;
    b.max_X = c.max_X;
    b.max_NA = c.max_NA;
    b.max_runs = c.max_runs;
    b.max_segs = c.max_segs;
    const size_t lds = std::max(paam::wave_lds_bytes(b), paam::wcrt_lds_bytes(b));
    RNG(lds <= 160 * 1024,
        "sets of %d chains, %d executors and %d accelerators need %zu bytes of LDS per wave "
        "(max 163840): fewer chains or executors per set",
        c.max_C, c.max_X, c.max_NA, lds);
  }
  return PAAM_OK;
}

// Arena layout: every array 256-B aligned, in a fixed order.
struct Arena {
  size_t off = 0;
  template <class T>
  size_t take(int64_t n) {
    size_t o = off;
    off += ((size_t)std::max<int64_t>(n, 1) * sizeof(T) + 255) & ~(size_t)255;
    return o;
  }
};

struct Offsets {
  size_t set_chain_off, set_cb_off, set_seg_off, set_run_off, set_exec_off, set_accel_off, eps_hop,
      work_order, T, D, Kd, rcp, KRr, rank0, chain_nrun, spin, E, cb_seg_off, cb_exec, chain_cb_lo,
      A, seg_accel,
      seg_chain, seg_order, run_chain, run_exec, run_cb_lo, run_cb_hi, hpx_mask, buckets, aeps,
      akappa, seg_type, type_units, set_type_off, total;
};

Offsets layout(const Plan &P) {
  Arena a;
  Offsets o;
  const int64_t S = P.n_sets;
  o.set_chain_off = a.take<int64_t>(S + 1);
  o.set_cb_off = a.take<int64_t>(S + 1);
  o.set_seg_off = a.take<int64_t>(S + 1);
  o.set_run_off = a.take<int64_t>(S + 1);
  o.set_exec_off = a.take<int64_t>(S + 1);
  o.set_accel_off = a.take<int64_t>(S + 1);
  o.eps_hop = a.take<int64_t>(S);
  o.work_order = a.take<int64_t>(S);
  o.T = a.take<int64_t>(P.n_chains);
  o.D = a.take<int64_t>(P.n_chains);
  o.Kd = a.take<double>(P.n_chains);
  o.rcp = a.take<double>(P.n_chains);
  o.KRr = a.take<double>(2 * P.n_chains);
  o.rank0 = a.take<int16_t>(P.n_chains);
  o.chain_nrun = a.take<int32_t>(P.n_chains);
  o.spin = a.take<uint8_t>(P.n_chains);
  o.E = a.take<int64_t>(P.n_cbs);
  o.cb_seg_off = a.take<int64_t>(P.n_cbs + 1);
  o.cb_exec = a.take<int8_t>(P.n_cbs);
  o.chain_cb_lo = a.take<int32_t>(P.n_chains);
  o.A = a.take<int64_t>(P.n_segs);
  o.seg_accel = a.take<int16_t>(P.n_segs);
  o.seg_chain = a.take<int16_t>(P.n_segs);
  o.seg_order = a.take<int32_t>(P.n_segs);
  o.run_chain = a.take<int16_t>(P.n_runs);
  o.run_exec = a.take<int16_t>(P.n_runs);
  o.run_cb_lo = a.take<int32_t>(P.n_runs);
  o.run_cb_hi = a.take<int32_t>(P.n_runs);
  o.hpx_mask = a.take<uint32_t>(P.n_exec);
  o.buckets = a.take<int32_t>(P.n_accel);
  o.aeps = a.take<int64_t>(P.n_accel);
  o.akappa = a.take<int64_t>(P.n_accel);
  const bool units = P.unit_group >= 0;
  o.seg_type = a.take<int16_t>(units ? P.n_segs : 0);
  o.type_units = a.take<int16_t>(units ? P.n_types : 0);
  o.set_type_off = a.take<int64_t>(units ? S + 1 : 0);
  o.total = a.off;
  return o;
}

template <class T>
void put(std::vector<unsigned char> &buf, size_t off, const T *src, int64_t n) {
  if (n > 0) std::memcpy(buf.data() + off, src, (size_t)n * sizeof(T));
}

int num_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
    return 256;
  return n;
}

}  // namespace

extern "C" {

const char *paam_last_error(void) { return g_err.c_str(); }

const char *paam_version(void) { return "libpaam 0.1 (gfx950)"; }

paam_status paam_chainset_bytes(const paam_chainset_host *h, size_t *arena_bytes) {
  if (!arena_bytes) return fail(PAAM_E_INVAL, "arena_bytes is null");
  Plan P;
  paam_status st = make_plan(h, P);
  if (st != PAAM_OK) return st;
  *arena_bytes = layout(P).total;
  return PAAM_OK;
}

paam_status paam_chainset_upload(const paam_chainset_host *h, void *d_arena, size_t arena_bytes,
                                 paam_stream stream, paam_chainset **out) {
  if (!out) return fail(PAAM_E_INVAL, "out is null");
  *out = nullptr;
  std::string why;
  if (!device_ok(&why)) return fail(PAAM_E_STATE, "%s", why.c_str());
  Plan P;
  paam_status st = make_plan(h, P);
  if (st != PAAM_OK) return st;
  const Offsets o = layout(P);
  if (!d_arena) return fail(PAAM_E_INVAL, "arena is null");
  if ((reinterpret_cast<uintptr_t>(d_arena) & 255) != 0)
    return fail(PAAM_E_INVAL, "arena is not 256-byte aligned");
  if (arena_bytes < o.total)
    return fail(PAAM_E_NOMEM, "arena of %zu bytes, need %zu", arena_bytes, o.total);
  const int64_t S = P.n_sets;
  std::vector<unsigned char> buf(o.total, 0);
  put(buf, o.set_chain_off, h->set_chain_off, S + 1);
  put(buf, o.set_cb_off, P.set_cb_off.data(), S + 1);
  put(buf, o.set_seg_off, P.set_seg_off.data(), S + 1);
  put(buf, o.set_run_off, P.set_run_off.data(), S + 1);
  put(buf, o.set_exec_off, h->set_exec_off, S + 1);
  put(buf, o.set_accel_off, P.set_accel_x.data(), S + 1);
  put(buf, o.eps_hop, h->eps_hop, S);
  put(buf, o.work_order, P.work_order.data(), S);
  put(buf, o.T, h->T, P.n_chains);
  put(buf, o.D, h->D, P.n_chains);
  put(buf, o.Kd, P.Kd.data(), P.n_chains);
  put(buf, o.rcp, P.rcp.data(), P.n_chains);
  put(buf, o.KRr, P.KRr.data(), 2 * P.n_chains);
  put(buf, o.rank0, P.rank0.data(), P.n_chains);
  put(buf, o.chain_nrun, P.chain_nrun.data(), P.n_chains);
  put(buf, o.spin, h->spin, P.n_chains);
  put(buf, o.E, h->E, P.n_cbs);
  put(buf, o.cb_seg_off, h->cb_seg_off, P.n_cbs + 1);
  put(buf, o.cb_exec, P.cb_exec.data(), P.n_cbs);
  put(buf, o.chain_cb_lo, P.chain_cb_lo.data(), P.n_chains);
  put(buf, o.A, h->A, P.n_segs);
  put(buf, o.seg_accel, h->accel, P.n_segs);
  put(buf, o.seg_chain, P.seg_chain.data(), P.n_segs);
  put(buf, o.seg_order, P.seg_order.data(), P.n_segs);
  put(buf, o.run_chain, P.run_chain.data(), P.n_runs);
  put(buf, o.run_exec, P.run_exec.data(), P.n_runs);
  put(buf, o.run_cb_lo, P.run_cb_lo.data(), P.n_runs);
  put(buf, o.run_cb_hi, P.run_cb_hi.data(), P.n_runs);
  put(buf, o.hpx_mask, P.hpx_mask.data(), P.n_exec);
  put(buf, o.buckets, P.buckets.data(), P.n_accel);
  put(buf, o.aeps, P.aeps.data(), P.n_accel);
  put(buf, o.akappa, P.akappa.data(), P.n_accel);
  if (P.unit_group >= 0) {
    put(buf, o.seg_type, h->accel, P.n_segs);
    put(buf, o.type_units, h->accel_units, P.n_types);
    put(buf, o.set_type_off, h->set_accel_off, S + 1);
  }

  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(d_arena, buf.data(), o.total, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(arena)");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(upload)");

  paam_chainset *cs = new (std::nothrow) paam_chainset();
  if (!cs) return fail(PAAM_E_NOMEM, "host allocation failed");
  unsigned char *base = static_cast<unsigned char *>(d_arena);
  paam::DevBatch &b = cs->dev;
  b.n_sets = S;
  b.n_chains = P.n_chains;
  b.n_cbs = P.n_cbs;
  b.n_segs = P.n_segs;
  b.n_runs = P.n_runs;
#define BIND(field, T) b.field = reinterpret_cast<const T *>(base + o.field)
  BIND(set_chain_off, int64_t);
  BIND(set_cb_off, int64_t);
  BIND(set_seg_off, int64_t);
  BIND(set_run_off, int64_t);
  BIND(set_exec_off, int64_t);
  BIND(set_accel_off, int64_t);
  BIND(eps_hop, int64_t);
  BIND(work_order, int64_t);
  BIND(T, int64_t);
  BIND(D, int64_t);
  BIND(Kd, double);
  BIND(rcp, double);
  BIND(KRr, double);
  BIND(rank0, int16_t);
  BIND(chain_nrun, int32_t);
  BIND(spin, uint8_t);
  BIND(E, int64_t);
  BIND(cb_seg_off, int64_t);
  BIND(cb_exec, int8_t);
  BIND(chain_cb_lo, int32_t);
  BIND(A, int64_t);
  BIND(seg_accel, int16_t);
  BIND(seg_chain, int16_t);
  BIND(seg_order, int32_t);
  BIND(run_chain, int16_t);
  BIND(run_exec, int16_t);
  BIND(run_cb_lo, int32_t);
  BIND(run_cb_hi, int32_t);
  BIND(hpx_mask, uint32_t);
  BIND(buckets, int32_t);
  BIND(aeps, int64_t);
  BIND(akappa, int64_t);
  BIND(seg_type, int16_t);
  BIND(type_units, int16_t);
  BIND(set_type_off, int64_t);
#undef BIND
  b.unit_group = P.unit_group;
  b.max_C = P.max_C;
  b.max_X = P.max_X;
  b.max_NA = P.max_NA;
  b.max_runs = std::max(P.max_runs, 1);
  b.max_segs = std::max(P.max_segs, 1);
  cs->arena_bytes = o.total;
  cs->n_exec = P.n_exec;
  cs->n_accel = P.n_accel;
  cs->max_tot = P.max_tot;
  cs->max_cb_segs = P.max_cb_segs;
  cs->max_set_cbs = P.max_set_cbs;
  cs->max_buckets = P.max_buckets;
  cs->n_classes = (int)P.classes.size();
  for (int k = 0; k < cs->n_classes; ++k) cs->cls[k] = P.classes[k];
  if (P.unit_group >= 0) {
    paam_status ust = paam_assign_units(cs, stream);
    if (ust == PAAM_OK) {
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) ust = hip_fail(e, "hipStreamSynchronize(units)");
    }
    if (ust != PAAM_OK) {
      delete cs;
      return ust;
    }
  }
  *out = cs;
  return PAAM_OK;
}

void paam_chainset_free(paam_chainset *cs) { delete cs; }

paam_status paam_des_batch(const paam_chainset *cs, const paam_des_opts *o,
                           const int64_t *d_offsets, int64_t *d_obs, int8_t *d_status,
                           paam_stream stream) {
  if (!cs || !o) return fail(PAAM_E_INVAL, "null argument");
  if (o->n_scen < 1 || o->n_scen > (1 << 20)) return fail(PAAM_E_INVAL, "n_scen outside 1..2^20");
  if (o->exec_permille < 0 || o->exec_permille > 1000)
    return fail(PAAM_E_INVAL, "exec_permille outside 0..1000");
  if (o->util_permille < 0 || o->util_permille > 1000000)
    return fail(PAAM_E_INVAL, "util_permille outside 0..10^6");
  if (o->horizon < 0 || o->horizon >= ((int64_t)1 << 40))
    return fail(PAAM_E_RANGE, "horizon outside [0, 2^40)");
  if (o->max_steps < 1 || o->reserved != 0) return fail(PAAM_E_INVAL, "max_steps < 1 or reserved != 0");
  const paam::DevBatch &b = cs->dev;
  if (b.max_C > paam::kDesChains || b.max_X > paam::kDesExec || cs->max_cb_segs > paam::kDesSegs ||
      cs->max_buckets > paam::kDesLevels)
    return fail(PAAM_E_RANGE,
                "simulation holds at most %d chains, %d executors, %d segments per callback and "
                "%d buckets per accelerator per set",
                paam::kDesChains, paam::kDesExec, paam::kDesSegs, paam::kDesLevels);
  if (paam::des_lds_bytes(cs->max_set_cbs, b.max_segs) > paam::kDesLdsMax)
    return fail(PAAM_E_RANGE,
                "simulation keeps a set's callbacks and segments in LDS: 12 bytes per callback plus "
                "9 per segment, at most %zu bytes", paam::kDesLdsMax);
  if (b.n_sets == 0) return PAAM_OK;
  if (!d_offsets || !d_obs || !d_status) return fail(PAAM_E_INVAL, "null device buffer");
  paam::DesLaunch L;
  L.max_cbs = std::max(cs->max_set_cbs, 1);
  L.max_segs = std::max(b.max_segs, 1);
  L.b = b;
  L.o = *o;
  L.offsets = d_offsets;
  L.obs = d_obs;
  L.status = d_status;
  const int64_t work = b.n_sets * ((o->n_scen + paam::kWave - 1) / paam::kWave);
  const int64_t want = (int64_t)num_cus() * 16;
  L.grid = (int)std::min<int64_t>(work, want);
  const int rc = paam::launch_des(L, stream);
  if (rc != (int)hipSuccess) return hip_fail((hipError_t)rc, "des_kernel launch");
  return PAAM_OK;
}

paam_status paam_assign_units(paam_chainset *cs, paam_stream stream) {
  if (!cs) return fail(PAAM_E_INVAL, "null batch");
  if (cs->dev.unit_group < 0) return fail(PAAM_E_STATE, "batch was uploaded without accel_units");
  const int rc = paam::launch_units(cs->dev, num_cus(), stream);
  if (rc != (int)hipSuccess) return hip_fail((hipError_t)rc, "units_kernel launch");
  return PAAM_OK;
}

paam_status paam_chainset_seg_units(const paam_chainset *cs, int16_t *d_unit, paam_stream stream) {
  if (!cs) return fail(PAAM_E_INVAL, "null batch");
  if (cs->dev.n_segs == 0) return PAAM_OK;
  if (!d_unit) return fail(PAAM_E_INVAL, "d_unit is null");
  hipError_t e = hipMemcpyAsync(d_unit, cs->dev.seg_accel, (size_t)cs->dev.n_segs * sizeof(int16_t),
                                hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(seg units)");
  return PAAM_OK;
}

paam_status paam_chainset_info(const paam_chainset *cs, int64_t info[8]) {
  if (!cs || !info) return fail(PAAM_E_INVAL, "null argument");
  info[0] = cs->dev.n_sets;
  info[1] = cs->dev.n_chains;
  info[2] = cs->dev.n_cbs;
  info[3] = cs->dev.n_segs;
  info[4] = cs->dev.n_runs;
  info[5] = cs->dev.max_C;
  info[6] = cs->dev.max_runs;
  info[7] = cs->dev.max_segs;
  return PAAM_OK;
}

static paam_status check_opts(const paam_wcrt_opts *o) {
  if (!o) return fail(PAAM_E_INVAL, "opts is null");
  if (o->blocking != PAAM_BLOCK_SAFE && o->blocking != PAAM_BLOCK_PAPER)
    return fail(PAAM_E_INVAL, "blocking must be PAAM_BLOCK_SAFE or PAAM_BLOCK_PAPER");
  if (o->cap_mult < 1 || o->cap_mult > 64) return fail(PAAM_E_INVAL, "cap_mult must be 1..64");
  if (o->util_permille < 0 || o->util_permille > 1000000)
    return fail(PAAM_E_INVAL, "util_permille must be 0..1000000");
  if (o->bound < PAAM_BOUND_MIN || o->bound > PAAM_BOUND_L3)
    return fail(PAAM_E_INVAL, "bound must be PAAM_BOUND_MIN, _L2 or _L3");
  if (o->waves_per_cu < 0 || o->waves_per_cu > 32)
    return fail(PAAM_E_INVAL, "waves_per_cu must be 0..32");
  return PAAM_OK;
}

// The batch restricted to one size class: its slice of the work order and
// its maxima (set indices stay global).
static paam::DevBatch class_view(const paam_chainset *cs, int k) {
  paam::DevBatch b = cs->dev;
  const paam::SizeClass &c = cs->cls[k];
  b.work_order = cs->dev.work_order + c.begin;
  b.n_sets = c.count;
  b.max_C = c.max_C;
  b.max_X = c.max_X;
  b.max_NA = c.max_NA;
  b.max_runs = std::max(c.max_runs, 1);
  b.max_segs = std::max(c.max_segs, 1);
  return b;
}

static int grid_n(int64_t n_sets, const paam_wcrt_opts *o) {
  int w = o->waves_per_cu > 0 ? o->waves_per_cu : 8;
  int64_t g = (int64_t)num_cus() * w;
  if (g > n_sets) g = n_sets;
  return (int)std::max<int64_t>(g, 1);
}

constexpr int kDefaultMicro = 2;

// Schedule of size class k: waves per CU (o->waves_per_cu if set, else the
// autotuner's choice for the class, else 8) and evaluations per engine step.
static void class_schedule(const paam_chainset *cs, int k, const paam_wcrt_opts *o, int *waves,
                           int *micro) {
  const paam::SizeClass &c = cs->cls[k];
  *waves = o->waves_per_cu > 0 ? o->waves_per_cu : (c.tuned_waves > 0 ? c.tuned_waves : 8);
  *micro = c.tuned_micro > 0 ? c.tuned_micro : kDefaultMicro;
}

static int class_grid(const paam_chainset *cs, int k, const paam_wcrt_opts *o) {
  int w = 0, m = 0;
  class_schedule(cs, k, o, &w, &m);
  paam_wcrt_opts t = *o;
  t.waves_per_cu = w;
  return grid_n(cs->cls[k].count, &t);
}

paam_status paam_wcrt_bytes(const paam_chainset *cs, const paam_wcrt_opts *o, size_t *ws_bytes) {
  if (!cs || !ws_bytes) return fail(PAAM_E_INVAL, "null argument");
  paam_status st = check_opts(o);
  if (st != PAAM_OK) return st;
  size_t need = 256;
  for (int k = 0; k < cs->n_classes; ++k) {
    const paam::DevBatch b = class_view(cs, k);
    need = std::max(need, 256 + (size_t)class_grid(cs, k, o) * paam::wcrt_scratch_bytes(b));
  }
  *ws_bytes = need;
  return PAAM_OK;
}

// Launches the analysis of size class k with the given schedule.
static paam_status launch_class(const paam_chainset *cs, int k, const paam_wcrt_opts *o,
                                int waves, int micro, int8_t *set_sched, int32_t *set_worst,
                                int64_t *set_worst_R, int64_t *chain_R, unsigned char *base,
                                int64_t max_grid, paam_stream stream) {
  paam::WcrtLaunch L;
  L.b = class_view(cs, k);
  L.o = *o;
  L.set_sched = set_sched;
  L.set_worst = set_worst;
  L.set_worst_R = set_worst_R;
  L.chain_R = o->full ? chain_R : nullptr;
  L.counter = reinterpret_cast<unsigned long long *>(base);  // zeroed by a kernel per launch
  L.scratch = base + 256;
  L.scratch_stride = paam::wcrt_scratch_bytes(L.b);
  L.lds_bytes = paam::wcrt_lds_bytes(L.b);
  paam_wcrt_opts t = *o;
  t.waves_per_cu = waves;
  L.grid = (int)std::min<int64_t>(grid_n(L.b.n_sets, &t), max_grid);
  L.micro = micro;
  int e = paam::launch_wcrt(L, stream);
  if (e != 0) return hip_fail((hipError_t)e, "wcrt launch");
  return PAAM_OK;
}

static paam_status check_batch_args(const paam_chainset *cs, const paam_wcrt_opts *o,
                                    int8_t *set_sched, int32_t *set_worst, int64_t *set_worst_R,
                                    int64_t *chain_R) {
  if (!cs) return fail(PAAM_E_INVAL, "chainset is null");
  paam_status st = check_opts(o);
  if (st != PAAM_OK) return st;
  if (!set_sched || !set_worst || !set_worst_R)
    return fail(PAAM_E_INVAL, "set outputs must not be null");
  if (o->full && !chain_R) return fail(PAAM_E_INVAL, "full mode needs chain_R");
  if (paam::wcrt_lds_bytes(cs->dev) > 160 * 1024)
    return fail(PAAM_E_RANGE, "sets need %zu bytes of LDS per wave (max 163840)",
                paam::wcrt_lds_bytes(cs->dev));
  return PAAM_OK;
}

paam_status paam_wcrt_batch(const paam_chainset *cs, const paam_wcrt_opts *o, int8_t *set_sched,
                            int32_t *set_worst, int64_t *set_worst_R, int64_t *chain_R, void *d_ws,
                            size_t ws_bytes, paam_stream stream) {
  paam_status st = check_batch_args(cs, o, set_sched, set_worst, set_worst_R, chain_R);
  if (st != PAAM_OK) return st;
  size_t need = 0;
  paam_wcrt_bytes(cs, o, &need);
  if (!d_ws || ws_bytes < need)
    return fail(PAAM_E_NOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0)
    return fail(PAAM_E_INVAL, "workspace is not 256-byte aligned");
  // one launch per size class, in stream order on the same workspace
  for (int k = 0; k < cs->n_classes; ++k) {
    int w = 0, m = 0;
    class_schedule(cs, k, o, &w, &m);
    st = launch_class(cs, k, o, w, m, set_sched, set_worst, set_worst_R, chain_R,
                      static_cast<unsigned char *>(d_ws), INT64_MAX, stream);
    if (st != PAAM_OK) return st;
  }
  return PAAM_OK;
}

paam_status paam_wcrt_batch_noalloc(const paam_chainset *cs, const paam_wcrt_opts *o,
                                    int8_t *set_sched, int32_t *set_worst, int64_t *set_worst_R,
                                    int64_t *chain_R, paam_stream stream) {
  paam_status st = check_batch_args(cs, o, set_sched, set_worst, set_worst_R, chain_R);
  if (st != PAAM_OK) return st;
  // every size class must fit at least one wave into the static scratch
  for (int k = 0; k < cs->n_classes; ++k) {
    const size_t per = paam::wcrt_scratch_bytes(class_view(cs, k));
    if (per > paam::kNoAllocScratchBytes - 256)
      return fail(PAAM_E_RANGE,
                  "sets of %d chains need %zu bytes of scratch per wave; the static scratch "
                  "holds %zu",
                  cs->cls[k].max_C, per, paam::kNoAllocScratchBytes - 256);
  }
  void *base = nullptr;
  const int he = paam::noalloc_scratch(&base);
  if (he != 0) return hip_fail((hipError_t)he, "hipGetSymbolAddress(scratch)");
  for (int k = 0; k < cs->n_classes; ++k) {
    int w = 0, m = 0;
    class_schedule(cs, k, o, &w, &m);
    const int64_t fit = (int64_t)((paam::kNoAllocScratchBytes - 256) /
                                  paam::wcrt_scratch_bytes(class_view(cs, k)));
    st = launch_class(cs, k, o, w, m, set_sched, set_worst, set_worst_R, chain_R,
                      static_cast<unsigned char *>(base), fit, stream);
    if (st != PAAM_OK) return st;
  }
  return PAAM_OK;
}

paam_status paam_wcrt_autotune(paam_chainset *cs, paam_wcrt_opts *o, const int32_t *cand,
                               int32_t n_cand, int32_t reps, int8_t *set_sched,
                               int32_t *set_worst, int64_t *set_worst_R, int64_t *chain_R,
                               void *d_ws, size_t ws_bytes, paam_stream stream, float *best_ms) {
  if (!cs || !o || !cand || !best_ms) return fail(PAAM_E_INVAL, "null argument");
  if (n_cand < 1 || n_cand > 64 || reps < 1 || reps > 100)
    return fail(PAAM_E_INVAL, "need 1 <= n_cand <= 64 and 1 <= reps <= 100");
  for (int i = 0; i < n_cand; ++i)
    if (cand[i] < 1 || cand[i] > 32) return fail(PAAM_E_INVAL, "candidate waves_per_cu outside 1..32");
  paam_status st = check_batch_args(cs, o, set_sched, set_worst, set_worst_R, chain_R);
  if (st != PAAM_OK) return st;
  // the workspace must hold the largest candidate's grid for every class
  int wmax = 0;
  for (int i = 0; i < n_cand; ++i) wmax = std::max(wmax, (int)cand[i]);
  paam_wcrt_opts tmax = *o;
  tmax.waves_per_cu = wmax;
  size_t need = 0;
  paam_wcrt_bytes(cs, &tmax, &need);
  if (!d_ws || ws_bytes < need)
    return fail(PAAM_E_NOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0)
    return fail(PAAM_E_INVAL, "workspace is not 256-byte aligned");
  hipStream_t sh = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(he, "hipEventCreate");
  }
  unsigned char *base = static_cast<unsigned char *>(d_ws);
  paam_status st_out = PAAM_OK;
  float total = 0.0f;
  // per size class: every (waves per CU, evaluations per step) pair, one
  // untimed launch then reps timed ones; the fastest is kept in the handle
  for (int k = 0; k < cs->n_classes && st_out == PAAM_OK; ++k) {
    float best = 0.0f;
    int bw = -1, bm = kDefaultMicro;
    for (int i = 0; i < n_cand && st_out == PAAM_OK; ++i)
      for (int m = 1; m <= 3 && st_out == PAAM_OK; ++m) {
        st_out = launch_class(cs, k, o, cand[i], m, set_sched, set_worst, set_worst_R, chain_R,
                              base, INT64_MAX, stream);
        if (st_out != PAAM_OK) break;
        he = hipEventRecord(e0, sh);
        for (int r = 0; r < reps && st_out == PAAM_OK && he == hipSuccess; ++r)
          st_out = launch_class(cs, k, o, cand[i], m, set_sched, set_worst, set_worst_R,
                                chain_R, base, INT64_MAX, stream);
        if (he == hipSuccess) he = hipEventRecord(e1, sh);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess && st_out == PAAM_OK) st_out = hip_fail(he, "autotune timing");
        if (st_out != PAAM_OK) break;
        ms /= (float)reps;
        if (bw < 0 || ms < best) {
          best = ms;
          bw = cand[i];
          bm = m;
        }
      }
    if (st_out == PAAM_OK) {
      cs->cls[k].tuned_waves = bw;
      cs->cls[k].tuned_micro = bm;
      total += best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st_out != PAAM_OK) return st_out;
  o->waves_per_cu = 0;  // use the per-class choices
  *best_ms = total;
  return PAAM_OK;
}

paam_status paam_wcrt_schedule(const paam_chainset *cs, int32_t *classes, int32_t cap,
                               int32_t *n_classes) {
  if (!cs || !n_classes || (cap > 0 && !classes)) return fail(PAAM_E_INVAL, "null argument");
  *n_classes = cs->n_classes;
  for (int k = 0; k < cs->n_classes && k < cap; ++k) {
    int w = 0, m = 0;
    paam_wcrt_opts o{};
    class_schedule(cs, k, &o, &w, &m);
    classes[4 * k] = cs->cls[k].max_C;
    classes[4 * k + 1] = (int32_t)std::min<int64_t>(cs->cls[k].count, INT32_MAX);
    classes[4 * k + 2] = w;
    classes[4 * k + 3] = m;
  }
  return PAAM_OK;
}

static paam_status check_search(const paam_chainset *cs, const paam_search_opts *o) {
  if (!cs || !o) return fail(PAAM_E_INVAL, "null argument");
  paam_status st = check_opts(&o->wcrt);
  if (st != PAAM_OK) return st;
  if (o->n_cand < 1 || o->n_cand > 65536) return fail(PAAM_E_INVAL, "n_cand must be 1..65536");
  if (o->guided != 0 && o->guided != 1) return fail(PAAM_E_INVAL, "guided must be 0 or 1");
  if (o->guided) {
    if (o->top_k < 1 || o->top_k > o->n_cand) return fail(PAAM_E_INVAL, "top_k must be 1..n_cand");
    if (!o->d_scores) return fail(PAAM_E_INVAL, "guided search needs d_scores");
    if (o->top_k > 1024) return fail(PAAM_E_INVAL, "top_k must be <= 1024");
  }
  return PAAM_OK;
}

paam_status paam_search_bytes(const paam_chainset *cs, const paam_search_opts *o, size_t *ws_bytes) {
  if (!ws_bytes) return fail(PAAM_E_INVAL, "null argument");
  paam_status st = check_search(cs, o);
  if (st != PAAM_OK) return st;
  size_t need = 256;
  for (int k = 0; k < cs->n_classes; ++k) {
    const paam::DevBatch b = class_view(cs, k);
    need = std::max(need, 256 + (size_t)grid_n(b.n_sets, &o->wcrt) * paam::wave_search_bytes(b));
  }
  *ws_bytes = need;
  return PAAM_OK;
}

paam_status paam_priority_search(const paam_chainset *cs, const paam_search_opts *o,
                                 int32_t *found, int32_t *n_exact, int32_t *found_prio, void *d_ws,
                                 size_t ws_bytes, paam_stream stream) {
  paam_status st = check_search(cs, o);
  if (st != PAAM_OK) return st;
  if (!found || !n_exact) return fail(PAAM_E_INVAL, "found and n_exact must not be null");
  size_t need = 0;
  paam_search_bytes(cs, o, &need);
  if (!d_ws || ws_bytes < need)
    return fail(PAAM_E_NOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0)
    return fail(PAAM_E_INVAL, "workspace is not 256-byte aligned");
  if (paam::wave_lds_bytes(cs->dev) > 160 * 1024)
    return fail(PAAM_E_RANGE, "sets need %zu bytes of LDS per wave (max 163840)",
                paam::wave_lds_bytes(cs->dev));
  for (int k = 0; k < cs->n_classes; ++k) {
    paam::SearchLaunch L;
    L.b = class_view(cs, k);
    L.o = *o;
    L.found = found;
    L.n_exact = n_exact;
    L.found_prio = found_prio;
    L.counter = static_cast<unsigned long long *>(d_ws);
    L.scratch = static_cast<unsigned char *>(d_ws) + 256;
    L.scratch_stride = paam::wave_search_bytes(L.b);
    L.analysis_stride = paam::wave_scratch_bytes(L.b);
    L.lds_bytes = paam::wave_lds_bytes(L.b);
    L.grid = grid_n(L.b.n_sets, &o->wcrt);
    int e = paam::launch_search(L, stream);
    if (e != 0) return hip_fail((hipError_t)e, "search launch");
  }
  return PAAM_OK;
}

// ------------------------------------------------------ surrogate entry points

static int grid_items(int64_t n_items, int waves_per_cu) {
  int64_t g = (int64_t)num_cus() * (waves_per_cu > 0 ? waves_per_cu : 8);
  if (g > n_items) g = n_items;
  return (int)std::max<int64_t>(g, 1);
}

// Features grid: as many waves per CU as the kernel's registers allow (the
// LDS-table kernel is built for four waves per SIMD, the global-table kernel
// for three), fewer when the LDS tables do not fit that many.
static int feat_grid(const paam_chainset *cs, int64_t n_items) {
  int w = 12;
  if (paam::feat_in_lds(cs->dev)) {
    const size_t per = paam::feat_wave_bytes(cs->dev);
    w = (int)std::min<size_t>(16, (160 * 1024) / std::max<size_t>(per, 1));
    w = std::max(w, 1);
  }
  return grid_items(n_items, w);
}

static bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

paam_status paam_candidate_bytes(const paam_chainset *cs, const paam_wcrt_opts *o, int64_t n_pairs,
                                 size_t *ws_bytes) {
  if (!cs || !ws_bytes) return fail(PAAM_E_INVAL, "null argument");
  paam_status st = check_opts(o);
  if (st != PAAM_OK) return st;
  if (n_pairs < 0) return fail(PAAM_E_INVAL, "n_pairs < 0");
  *ws_bytes = 256 + (size_t)grid_items(n_pairs, o->waves_per_cu) * paam::wave_search_bytes(cs->dev);
  return PAAM_OK;
}

paam_status paam_candidate_wcrt(const paam_chainset *cs, const paam_wcrt_opts *o, uint64_t seed,
                                const int64_t *d_pairs, int64_t n_pairs, int8_t *sched,
                                int64_t *worst_R, int64_t *worst_D, float *ratio, void *d_ws,
                                size_t ws_bytes, paam_stream stream) {
  size_t need = 0;
  paam_status st = paam_candidate_bytes(cs, o, n_pairs, &need);
  if (st != PAAM_OK) return st;
  if (n_pairs > 0 && (!d_pairs || !sched || !worst_R || !worst_D))
    return fail(PAAM_E_INVAL, "pairs and outputs must not be null");
  if (!d_ws || ws_bytes < need)
    return fail(PAAM_E_NOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  if (!aligned(d_ws, 256)) return fail(PAAM_E_INVAL, "workspace is not 256-byte aligned");
  paam::CandLaunch L;
  L.b = cs->dev;
  L.o = *o;
  L.seed = seed;
  L.pairs = d_pairs;
  L.n_pairs = n_pairs;
  L.sched = sched;
  L.worst_R = worst_R;
  L.worst_D = worst_D;
  L.ratio = ratio;
  L.counter = static_cast<unsigned long long *>(d_ws);
  L.scratch = static_cast<unsigned char *>(d_ws) + 256;
  L.scratch_stride = paam::wave_search_bytes(cs->dev);
  L.analysis_stride = paam::wave_scratch_bytes(cs->dev);
  L.lds_bytes = paam::wave_lds_bytes(cs->dev);
  L.grid = grid_items(n_pairs, o->waves_per_cu);
  if (L.lds_bytes > 160 * 1024)
    return fail(PAAM_E_RANGE, "sets need %zu bytes of LDS per wave (max 163840)", L.lds_bytes);
  int e = paam::launch_candidates(L, stream);
  if (e != 0) return hip_fail((hipError_t)e, "candidate launch");
  return PAAM_OK;
}

paam_status paam_features_bytes(const paam_chainset *cs, int64_t n_pairs, size_t *ws_bytes) {
  if (!cs || !ws_bytes) return fail(PAAM_E_INVAL, "null argument");
  if (n_pairs < 0) return fail(PAAM_E_INVAL, "n_pairs < 0");
  *ws_bytes = 256 + (size_t)feat_grid(cs, n_pairs) * paam::feat_wave_bytes(cs->dev);
  return PAAM_OK;
}

paam_status paam_features(const paam_chainset *cs, uint64_t seed, const int64_t *d_pairs,
                          int64_t n_pairs, int32_t row_stride, uint16_t *feat, int32_t *count,
                          void *d_ws, size_t ws_bytes, paam_stream stream) {
  size_t need = 0;
  paam_status st = paam_features_bytes(cs, n_pairs, &need);
  if (st != PAAM_OK) return st;
  if (row_stride < cs->dev.max_C)
    return fail(PAAM_E_INVAL, "row_stride %d below the largest set (%d chains)", row_stride,
                cs->dev.max_C);
  if (n_pairs > 0 && (!d_pairs || !feat || !count))
    return fail(PAAM_E_INVAL, "pairs and outputs must not be null");
  if (!aligned(feat, 16)) return fail(PAAM_E_INVAL, "feat is not 16-byte aligned");
  if (cs->max_tot >= ((int64_t)1 << 40))
    return fail(PAAM_E_RANGE, "a set's total demand reaches 2^40 ns");
  if (!d_ws || ws_bytes < need)
    return fail(PAAM_E_NOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  if (!aligned(d_ws, 256)) return fail(PAAM_E_INVAL, "workspace is not 256-byte aligned");
  paam::FeatLaunch L;
  L.b = cs->dev;
  L.seed = seed;
  L.pairs = d_pairs;
  L.n_items = n_pairs;
  L.set0 = 0;
  L.n_cand = 0;
  L.item = 1;
  L.set_tables = nullptr;
  L.set_table_stride = 0;
  L.n_table_sets = 0;
  L.util = 1000;
  L.row_stride = row_stride;
  L.feat = feat;
  L.count = count;
  L.counter = static_cast<unsigned long long *>(d_ws);
  L.scratch = static_cast<unsigned char *>(d_ws) + 256;
  L.scratch_stride = paam::feat_wave_bytes(cs->dev);
  L.grid = feat_grid(cs, n_pairs);
  int e = paam::launch_features(L, stream);
  if (e != 0) return hip_fail((hipError_t)e, "features launch");
  return PAAM_OK;
}

paam_status paam_mlp_pack(const float *d_params, uint16_t *d_packed, paam_stream stream) {
  if (!d_params || !d_packed) return fail(PAAM_E_INVAL, "null argument");
  int e = paam::launch_pack(d_params, d_packed, stream);
  if (e != 0) return hip_fail((hipError_t)e, "pack launch");
  return PAAM_OK;
}

paam_status paam_mlp_forward(const float *d_params, const uint16_t *d_packed,
                             const uint16_t *feat, const int32_t *count, int64_t n,
                             int32_t row_stride, float *out, void *act, paam_stream stream) {
  if (n < 0 || row_stride < 1) return fail(PAAM_E_INVAL, "n < 0 or row_stride < 1");
  if (n > 0 && (!d_params || !d_packed || !feat || !count || !out))
    return fail(PAAM_E_INVAL, "null argument");
  if (!aligned(feat, 16) || !aligned(d_packed, 16) || (act && !aligned(act, 16)))
    return fail(PAAM_E_INVAL, "feat, packed weights and act must be 16-byte aligned");
  if (n > ((int64_t)1 << 35)) return fail(PAAM_E_RANGE, "too many candidates");
  paam::FwdLaunch L{d_params, d_packed, feat, count, n, row_stride, out, act};
  int e = paam::launch_forward(L, stream);
  if (e != 0) return hip_fail((hipError_t)e, "forward launch");
  return PAAM_OK;
}

paam_status paam_mlp_backward_bytes(int64_t n, size_t *ws_bytes) {
  if (!ws_bytes || n < 0) return fail(PAAM_E_INVAL, "bad argument");
  *ws_bytes = 256 + (size_t)std::max<int64_t>(paam::backward_chunks(n), 1) *
                        paam::backward_partial_stride() * sizeof(float);
  return PAAM_OK;
}

paam_status paam_mlp_backward(const float *d_params, const uint16_t *d_packed,
                              const uint16_t *feat, const int32_t *count, int64_t n,
                              int32_t row_stride, const float *out, const float *target,
                              const void *act, float *grad, float *loss, void *d_ws,
                              size_t ws_bytes, paam_stream stream) {
  size_t need = 0;
  paam_status st = paam_mlp_backward_bytes(n, &need);
  if (st != PAAM_OK) return st;
  if (n < 1) return fail(PAAM_E_INVAL, "the loss needs n >= 1 candidates");
  if (row_stride < 1) return fail(PAAM_E_INVAL, "row_stride < 1");
  if (!d_params || !d_packed || !feat || !count || !out || !target || !act || !grad)
    return fail(PAAM_E_INVAL, "null argument");
  if (!d_ws || ws_bytes < need)
    return fail(PAAM_E_NOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  if (!aligned(d_ws, 256)) return fail(PAAM_E_INVAL, "workspace is not 256-byte aligned");
  if (paam::backward_chunks(n) > 0x7FFFFFFF) return fail(PAAM_E_RANGE, "too many candidates");
  paam::BwdLaunch L{d_params, d_packed, feat, count, n, row_stride, out, target, act,
                    reinterpret_cast<float *>(static_cast<unsigned char *>(d_ws) + 256),
                    paam::backward_partial_stride()};
  int e = paam::launch_backward(L, grad, loss, stream);
  if (e != 0) return hip_fail((hipError_t)e, "backward launch");
  return PAAM_OK;
}

paam_status paam_mlp_adam_step(float *d_params, uint16_t *d_packed, float *d_m, float *d_v,
                               const float *grad, float lr, float beta1, float beta2, float eps,
                               int64_t step, paam_stream stream) {
  if (!d_params || !d_packed || !d_m || !d_v || !grad) return fail(PAAM_E_INVAL, "null argument");
  if (step < 1) return fail(PAAM_E_INVAL, "step counts from 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr >= 0.0f))
    return fail(PAAM_E_INVAL, "need 0 <= beta < 1, eps > 0, lr >= 0");
  int e = paam::launch_adam(d_params, d_packed, d_m, d_v, grad, lr, beta1, beta2, eps, step, stream);
  if (e != 0) return hip_fail((hipError_t)e, "adam launch");
  return PAAM_OK;
}

// Sets scored per chunk: at most 2^24 feature rows (1.6 GB).  Larger chunks
// of 256-chain sets (more waves in flight) measured slower: their per-wave
// feature tables no longer stay in the caches.
static int64_t score_chunk_sets(const paam_chainset *cs, const paam_search_opts *o) {
  const int64_t per = (int64_t)o->n_cand * std::max(cs->dev.max_C, 1);
  int64_t n = ((int64_t)1 << 24) / per;
  n = std::max<int64_t>(n, 1);
  return std::min<int64_t>(n, std::max<int64_t>(cs->dev.n_sets, 1));
}

paam_status paam_score_bytes(const paam_chainset *cs, const paam_search_opts *o, size_t *ws_bytes) {
  if (!cs || !o || !ws_bytes) return fail(PAAM_E_INVAL, "null argument");
  if (o->n_cand < 1 || o->n_cand > 65536) return fail(PAAM_E_INVAL, "n_cand must be 1..65536");
  paam_status st = check_opts(&o->wcrt);
  if (st != PAAM_OK) return st;
  const int64_t S = score_chunk_sets(cs, o);
  const int64_t pairs = S * o->n_cand;
  const int item = paam::feat_item(cs->dev);
  const int64_t items = S * ((o->n_cand + item - 1) / item);
  const size_t feat = ((size_t)pairs * std::max(cs->dev.max_C, 1) * 48 * 2 + 255) & ~(size_t)255;
  const size_t cnt = ((size_t)pairs * 4 + 255) & ~(size_t)255;
  // prefix-scan schedule: one shared copy of each chunk set's tables
  const size_t tables = paam::feat_in_lds(cs->dev) ? 0 : (size_t)S * paam::feat_wave_bytes(cs->dev);
  *ws_bytes = 256 + feat + cnt + (size_t)feat_grid(cs, items) * paam::feat_wave_bytes(cs->dev) +
              tables;
  return PAAM_OK;
}

paam_status paam_score_candidates(const paam_chainset *cs, const paam_search_opts *o,
                                  const float *d_params, const uint16_t *d_packed, float *scores,
                                  void *d_ws, size_t ws_bytes, paam_stream stream) {
  size_t need = 0;
  paam_status st = paam_score_bytes(cs, o, &need);
  if (st != PAAM_OK) return st;
  if (!d_params || !d_packed || !scores) return fail(PAAM_E_INVAL, "null argument");
  if (!d_ws || ws_bytes < need)
    return fail(PAAM_E_NOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  if (!aligned(d_ws, 256) || !aligned(d_packed, 16))
    return fail(PAAM_E_INVAL, "workspace (256 B) or packed weights (16 B) misaligned");
  if (cs->max_tot >= ((int64_t)1 << 40) / std::max<int64_t>(1, (o->wcrt.util_permille + 999) / 1000))
    return fail(PAAM_E_RANGE, "a set's total demand reaches 2^40 ns");
  const int32_t Cm = std::max(cs->dev.max_C, 1);
  const int64_t S = score_chunk_sets(cs, o);
  const int item = paam::feat_item(cs->dev);
  const int64_t per = (o->n_cand + item - 1) / item;
  unsigned char *w = static_cast<unsigned char *>(d_ws);
  const size_t feat_b = ((size_t)S * o->n_cand * Cm * 48 * 2 + 255) & ~(size_t)255;
  const size_t cnt_b = ((size_t)S * o->n_cand * 4 + 255) & ~(size_t)255;
  uint16_t *feat = reinterpret_cast<uint16_t *>(w + 256);
  int32_t *count = reinterpret_cast<int32_t *>(w + 256 + feat_b);
  unsigned char *scr = w + 256 + feat_b + cnt_b;
  const bool shared = !paam::feat_in_lds(cs->dev);
  unsigned char *tables =
      scr + (size_t)feat_grid(cs, S * per) * paam::feat_wave_bytes(cs->dev);
  for (int64_t s0 = 0; s0 < cs->dev.n_sets; s0 += S) {
    const int64_t ns = std::min<int64_t>(S, cs->dev.n_sets - s0);
    paam::FeatLaunch F;
    F.b = cs->dev;
    F.seed = o->seed;
    F.pairs = nullptr;
    F.n_items = ns * per;
    F.set0 = s0;
    F.n_cand = o->n_cand;
    F.item = item;
    F.util = o->wcrt.util_permille;
    F.row_stride = Cm;
    F.set_tables = shared ? tables : nullptr;
    F.set_table_stride = paam::feat_wave_bytes(cs->dev);
    F.n_table_sets = shared ? ns : 0;
    F.feat = feat;
    F.count = count;
    F.counter = reinterpret_cast<unsigned long long *>(w);
    F.scratch = scr;
    F.scratch_stride = paam::feat_wave_bytes(cs->dev);
    F.grid = feat_grid(cs, F.n_items);
    if (shared) {
      int e = paam::launch_feat_tables(F, (int)std::min<int64_t>(ns, (int64_t)num_cus() * 8), stream);
      if (e != 0) return hip_fail((hipError_t)e, "feature tables launch");
    }
    int e = paam::launch_features(F, stream);
    if (e != 0) return hip_fail((hipError_t)e, "features launch");
    paam::FwdLaunch L{d_params, d_packed, feat, count, ns * o->n_cand, Cm,
                      scores + s0 * (int64_t)o->n_cand, nullptr};
    e = paam::launch_forward(L, stream);
    if (e != 0) return hip_fail((hipError_t)e, "forward launch");
  }
  return PAAM_OK;
}

}  // extern "C"
