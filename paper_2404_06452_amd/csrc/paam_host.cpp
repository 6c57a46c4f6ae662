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
  std::vector<int32_t> run_cb_lo, run_cb_hi, chain_nrun, exec_runs, er_off, er_cnt;
  std::vector<int16_t> rank0, seg_chain, exec_seq;
  std::vector<uint32_t> hpx_mask;
  std::vector<double> Kd, rcp;
  std::vector<int32_t> buckets;
  std::vector<int64_t> work_order;
  int32_t max_C = 0, max_X = 0, max_NA = 0, max_runs = 0, max_segs = 0, max_runs_exec = 0;
};

#define REQ(cond, ...)                                   \
  do {                                                   \
    if (!(cond)) return fail(PAAM_E_INVAL, __VA_ARGS__); \
  } while (0)
#define RNG(cond, ...)                                   \
  do {                                                   \
    if (!(cond)) return fail(PAAM_E_RANGE, __VA_ARGS__); \
  } while (0)

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
  for (int64_t j = 0; j < NJ; ++j)
    REQ(h->cb_seg_off[j + 1] >= h->cb_seg_off[j], "cb_seg_off decreases at %lld", (long long)j);
  const int64_t NG = h->cb_seg_off[NJ];
  P.n_segs = NG;
  REQ(NG == 0 || (h->A && h->accel), "segments present but A/accel null");

  // executors, accelerators
  P.hpx_mask.assign(NX, 0u);
  P.exec_seq.assign(NX, 0);
  for (int64_t s = 0; s < S; ++s) {
    const int64_t x0 = h->set_exec_off[s];
    const int X = (int)(h->set_exec_off[s + 1] - x0);
    for (int e = 0; e < X; ++e)
      for (int f = 0; f < X; ++f) {
        if (e == f || h->exec_core[x0 + e] != h->exec_core[x0 + f]) continue;
        REQ(h->exec_prio[x0 + e] != h->exec_prio[x0 + f],
            "set %lld: executors %d and %d share core and process priority", (long long)s, e, f);
        if (h->exec_prio[x0 + f] > h->exec_prio[x0 + e]) P.hpx_mask[x0 + e] |= 1u << f;
      }
    std::vector<int> seq(X);
    std::iota(seq.begin(), seq.end(), 0);
    std::stable_sort(seq.begin(), seq.end(), [&](int a, int b) {
      if (h->exec_core[x0 + a] != h->exec_core[x0 + b])
        return h->exec_core[x0 + a] < h->exec_core[x0 + b];
      return h->exec_prio[x0 + a] > h->exec_prio[x0 + b];
    });
    for (int i = 0; i < X; ++i) P.exec_seq[x0 + i] = (int16_t)seq[i];
  }
  P.buckets.resize(NAc);
  for (int64_t a = 0; a < NAc; ++a) {
    REQ(h->accel_buckets[a] >= 1, "accelerator %lld: buckets < 1", (long long)a);
    REQ(h->accel_eps[a] >= 0 && h->accel_kappa[a] >= 0, "accelerator %lld: negative overhead",
        (long long)a);
    RNG(h->accel_eps[a] < kTimeLimit && h->accel_kappa[a] < kTimeLimit,
        "accelerator %lld: overhead >= 2^36 ns", (long long)a);
    P.buckets[a] = h->accel_buckets[a];
  }

  // chains
  P.Kd.resize(NC);
  P.rcp.resize(NC);
  P.rank0.resize(NC);
  P.chain_nrun.assign(NC, 0);
  for (int64_t c = 0; c < NC; ++c) {
    const int64_t T = h->T[c], D = h->D[c];
    REQ(T > 0 && D > 0 && D <= T, "chain %lld: need 0 < D <= T (T=%lld D=%lld)", (long long)c,
        (long long)T, (long long)D);
    RNG(T < kTimeLimit, "chain %lld: period >= 2^36 ns", (long long)c);
    P.Kd[c] = (double)(2 * T - 1);
    P.rcp[c] = rcp_up(T);
  }

  // sets: ranks, sub-chains, grouping by executor, segments' chains
  P.set_cb_off.resize(S + 1);
  P.set_seg_off.resize(S + 1);
  P.set_run_off.resize(S + 1);
  P.seg_chain.resize(NG);
  P.er_off.assign(NX, 0);
  P.er_cnt.assign(NX, 0);
  std::vector<double> cost(S);
  for (int64_t s = 0; s < S; ++s) {
    const int64_t c0 = h->set_chain_off[s];
    const int C = (int)(h->set_chain_off[s + 1] - c0);
    const int64_t x0 = h->set_exec_off[s];
    const int X = (int)(h->set_exec_off[s + 1] - x0);
    const int NA = (int)(h->set_accel_off[s + 1] - h->set_accel_off[s]);
    const int64_t cb0 = h->chain_cb_off[c0], cb1 = h->chain_cb_off[c0 + C];
    const int64_t g0 = h->cb_seg_off[cb0], g1 = h->cb_seg_off[cb1];
    P.set_cb_off[s] = cb0;
    P.set_seg_off[s] = g0;
    P.set_run_off[s] = (int64_t)P.run_chain.size();
    RNG(g1 - g0 <= (int64_t)1 << 30 && cb1 - cb0 <= (int64_t)1 << 30, "set %lld too large",
        (long long)s);
    std::vector<int> order(C);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return h->prio[c0 + a] > h->prio[c0 + b]; });
    for (int r = 0; r < C; ++r) {
      if (r > 0)
        REQ(h->prio[c0 + order[r]] != h->prio[c0 + order[r - 1]],
            "set %lld: duplicate chain priority", (long long)s);
      P.rank0[c0 + order[r]] = (int16_t)r;
    }
    const size_t runs_begin = P.run_chain.size();
    for (int c = 0; c < C; ++c) {
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
          P.seg_chain[g] = (int16_t)c;
        }
        const int jl = (int)(j - cb0);
        if (e != prev_e) {
          P.run_chain.push_back((int16_t)c);
          P.run_exec.push_back((int16_t)e);
          P.run_cb_lo.push_back(jl);
          P.run_cb_hi.push_back(jl + 1);
          P.chain_nrun[c0 + c]++;
          prev_e = e;
        } else {
          P.run_cb_hi.back() = jl + 1;
        }
      }
    }
    const int nrun = (int)(P.run_chain.size() - runs_begin);
    RNG(nrun <= paam::kMaxRuns, "set %lld: %d sub-chains (max %d)", (long long)s, nrun,
        paam::kMaxRuns);
    // group sub-chains by executor
    std::vector<int> cnt(X, 0);
    for (int r = 0; r < nrun; ++r) cnt[P.run_exec[runs_begin + r]]++;
    int off = 0, mre = 0;
    for (int e = 0; e < X; ++e) {
      P.er_off[x0 + e] = off;
      P.er_cnt[x0 + e] = cnt[e];
      off += cnt[e];
      mre = std::max(mre, cnt[e]);
    }
    std::vector<int> pos(X);
    for (int e = 0; e < X; ++e) pos[e] = P.er_off[x0 + e];
    P.exec_runs.resize(runs_begin + nrun);
    for (int r = 0; r < nrun; ++r) P.exec_runs[runs_begin + pos[P.run_exec[runs_begin + r]]++] = r;
    P.max_C = std::max(P.max_C, C);
    P.max_X = std::max(P.max_X, X);
    P.max_NA = std::max(P.max_NA, NA);
    P.max_runs = std::max(P.max_runs, nrun);
    P.max_segs = std::max(P.max_segs, (int32_t)(g1 - g0));
    P.max_runs_exec = std::max(P.max_runs_exec, mre);
    cost[s] = (double)nrun * (double)(C + 4) + (double)(g1 - g0) * (double)C;
  }
  for (int64_t s = 0; s < S; ++s) RNG(h->eps_hop[s] >= 0 && h->eps_hop[s] < kTimeLimit,
                                      "set %lld: hop cost outside [0, 2^36)", (long long)s);
  P.set_cb_off[S] = NJ;
  P.set_seg_off[S] = NG;
  P.set_run_off[S] = (int64_t)P.run_chain.size();
  P.n_runs = (int64_t)P.run_chain.size();
  P.work_order.resize(S);
  std::iota(P.work_order.begin(), P.work_order.end(), 0);
  std::stable_sort(P.work_order.begin(), P.work_order.end(),
                   [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
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
      work_order, T, D, Kd, rcp, rank0, chain_nrun, spin, E, cb_seg_off, A, seg_accel, seg_chain,
      run_chain, run_exec, run_cb_lo, run_cb_hi, exec_runs, er_off, er_cnt, hpx_mask, exec_seq,
      buckets, aeps, akappa, total;
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
  o.rank0 = a.take<int16_t>(P.n_chains);
  o.chain_nrun = a.take<int32_t>(P.n_chains);
  o.spin = a.take<uint8_t>(P.n_chains);
  o.E = a.take<int64_t>(P.n_cbs);
  o.cb_seg_off = a.take<int64_t>(P.n_cbs + 1);
  o.A = a.take<int64_t>(P.n_segs);
  o.seg_accel = a.take<int16_t>(P.n_segs);
  o.seg_chain = a.take<int16_t>(P.n_segs);
  o.run_chain = a.take<int16_t>(P.n_runs);
  o.run_exec = a.take<int16_t>(P.n_runs);
  o.run_cb_lo = a.take<int32_t>(P.n_runs);
  o.run_cb_hi = a.take<int32_t>(P.n_runs);
  o.exec_runs = a.take<int32_t>(P.n_runs);
  o.er_off = a.take<int32_t>(P.n_exec);
  o.er_cnt = a.take<int32_t>(P.n_exec);
  o.hpx_mask = a.take<uint32_t>(P.n_exec);
  o.exec_seq = a.take<int16_t>(P.n_exec);
  o.buckets = a.take<int32_t>(P.n_accel);
  o.aeps = a.take<int64_t>(P.n_accel);
  o.akappa = a.take<int64_t>(P.n_accel);
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
  put(buf, o.set_accel_off, h->set_accel_off, S + 1);
  put(buf, o.eps_hop, h->eps_hop, S);
  put(buf, o.work_order, P.work_order.data(), S);
  put(buf, o.T, h->T, P.n_chains);
  put(buf, o.D, h->D, P.n_chains);
  put(buf, o.Kd, P.Kd.data(), P.n_chains);
  put(buf, o.rcp, P.rcp.data(), P.n_chains);
  put(buf, o.rank0, P.rank0.data(), P.n_chains);
  put(buf, o.chain_nrun, P.chain_nrun.data(), P.n_chains);
  put(buf, o.spin, h->spin, P.n_chains);
  put(buf, o.E, h->E, P.n_cbs);
  put(buf, o.cb_seg_off, h->cb_seg_off, P.n_cbs + 1);
  put(buf, o.A, h->A, P.n_segs);
  put(buf, o.seg_accel, h->accel, P.n_segs);
  put(buf, o.seg_chain, P.seg_chain.data(), P.n_segs);
  put(buf, o.run_chain, P.run_chain.data(), P.n_runs);
  put(buf, o.run_exec, P.run_exec.data(), P.n_runs);
  put(buf, o.run_cb_lo, P.run_cb_lo.data(), P.n_runs);
  put(buf, o.run_cb_hi, P.run_cb_hi.data(), P.n_runs);
  put(buf, o.exec_runs, P.exec_runs.data(), P.n_runs);
  put(buf, o.er_off, P.er_off.data(), P.n_exec);
  put(buf, o.er_cnt, P.er_cnt.data(), P.n_exec);
  put(buf, o.hpx_mask, P.hpx_mask.data(), P.n_exec);
  put(buf, o.exec_seq, P.exec_seq.data(), P.n_exec);
  put(buf, o.buckets, P.buckets.data(), P.n_accel);
  put(buf, o.aeps, h->accel_eps, P.n_accel);
  put(buf, o.akappa, h->accel_kappa, P.n_accel);

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
  BIND(rank0, int16_t);
  BIND(chain_nrun, int32_t);
  BIND(spin, uint8_t);
  BIND(E, int64_t);
  BIND(cb_seg_off, int64_t);
  BIND(A, int64_t);
  BIND(seg_accel, int16_t);
  BIND(seg_chain, int16_t);
  BIND(run_chain, int16_t);
  BIND(run_exec, int16_t);
  BIND(run_cb_lo, int32_t);
  BIND(run_cb_hi, int32_t);
  BIND(exec_runs, int32_t);
  BIND(er_off, int32_t);
  BIND(er_cnt, int32_t);
  BIND(hpx_mask, uint32_t);
  BIND(exec_seq, int16_t);
  BIND(buckets, int32_t);
  BIND(aeps, int64_t);
  BIND(akappa, int64_t);
#undef BIND
  b.max_C = P.max_C;
  b.max_X = P.max_X;
  b.max_NA = P.max_NA;
  b.max_runs = std::max(P.max_runs, 1);
  b.max_segs = std::max(P.max_segs, 1);
  b.max_runs_exec = P.max_runs_exec;
  cs->arena_bytes = o.total;
  cs->n_exec = P.n_exec;
  cs->n_accel = P.n_accel;
  *out = cs;
  return PAAM_OK;
}

void paam_chainset_free(paam_chainset *cs) { delete cs; }

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

static int grid_for(const paam_chainset *cs, const paam_wcrt_opts *o) {
  int w = o->waves_per_cu > 0 ? o->waves_per_cu : 8;
  int64_t g = (int64_t)num_cus() * w;
  if (g > cs->dev.n_sets) g = cs->dev.n_sets;
  return (int)std::max<int64_t>(g, 1);
}

paam_status paam_wcrt_bytes(const paam_chainset *cs, const paam_wcrt_opts *o, size_t *ws_bytes) {
  if (!cs || !ws_bytes) return fail(PAAM_E_INVAL, "null argument");
  paam_status st = check_opts(o);
  if (st != PAAM_OK) return st;
  *ws_bytes = 256 + (size_t)grid_for(cs, o) * paam::wave_scratch_bytes(cs->dev);
  return PAAM_OK;
}

paam_status paam_wcrt_batch(const paam_chainset *cs, const paam_wcrt_opts *o, int8_t *set_sched,
                            int32_t *set_worst, int64_t *set_worst_R, int64_t *chain_R, void *d_ws,
                            size_t ws_bytes, paam_stream stream) {
  if (!cs) return fail(PAAM_E_INVAL, "chainset is null");
  paam_status st = check_opts(o);
  if (st != PAAM_OK) return st;
  if (!set_sched || !set_worst || !set_worst_R)
    return fail(PAAM_E_INVAL, "set outputs must not be null");
  if (o->full && !chain_R) return fail(PAAM_E_INVAL, "full mode needs chain_R");
  size_t need = 0;
  paam_wcrt_bytes(cs, o, &need);
  if (!d_ws || ws_bytes < need)
    return fail(PAAM_E_NOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
  if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0)
    return fail(PAAM_E_INVAL, "workspace is not 256-byte aligned");
  paam::WcrtLaunch L;
  L.b = cs->dev;
  L.o = *o;
  L.set_sched = set_sched;
  L.set_worst = set_worst;
  L.set_worst_R = set_worst_R;
  L.chain_R = o->full ? chain_R : nullptr;
  L.counter = static_cast<unsigned long long *>(d_ws);
  L.scratch = static_cast<unsigned char *>(d_ws) + 256;
  L.scratch_stride = paam::wave_scratch_bytes(cs->dev);
  L.lds_bytes = paam::wave_lds_bytes(cs->dev);
  L.grid = grid_for(cs, o);
  if (L.lds_bytes > 160 * 1024)
    return fail(PAAM_E_RANGE, "sets need %zu bytes of LDS per wave (max 163840)", L.lds_bytes);
  int e = paam::launch_wcrt(L, stream);
  if (e != 0) return hip_fail((hipError_t)e, "wcrt launch");
  return PAAM_OK;
}

}  // extern "C"
