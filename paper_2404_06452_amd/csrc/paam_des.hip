// Event-driven simulation of chain sets under the PAAM model, one lane per
// (set, scenario): the observed end-to-end latencies that the analysis of
// Sec. IV-F must bound (the paper's Case Study 1, Sec. V-A, checks the same
// property on real hardware).
//
// A wave takes 64 scenarios of one set, so every lane reads the same set
// tables while it runs its own timeline; lanes never synchronise.  A lane's
// state (two job slots per chain, executors, the request being served on
// every bucket level) lives in private arrays, whose per-lane interleaving
// makes accesses to one slot index coalesce across the wave.
//
// The model (Sec. II-C, IV-C, IV-D, IV-F):
//  * releases every T from the chain's offset; callbacks in chain order; the
//    next callback is ready on its executor when the previous one completes,
//    after the hop cost when the executor changes;
//  * an idle executor starts its ready callback of the highest chain
//    priority (then the earliest release) and keeps it to the end, also while
//    its requests are served;
//  * a callback: CPU piece, then per segment epsilon of CPU, the request
//    (A + 2 kappa on the device), CPU piece; E split equally over the pieces;
//  * a core runs its demanding executor of the highest process priority
//    (CPU work left, or a request in service of a busy-waiting chain);
//  * an accelerator serves its highest bucket level holding a request; one
//    request at a time per level, highest chain priority first, then in
//    submission order; a higher level preempts a lower one.
// Within an instant the rules apply in a fixed order until nothing changes:
// releases, hop arrivals, executors by index (start, then advance past
// finished pieces or submit), accelerators by index (highest occupied level:
// start its next request, or finish the served one).  Time then jumps to the
// next event: a release, a hop arrival, the end of a running CPU piece, or
// the end of a served request.  All times are int64 nanoseconds.
#include <hip/hip_runtime.h>

#include "paam_internal.h"

namespace paam {
namespace {

constexpr int kSlots = 2 * kDesChains;
enum : int8_t { kFree = 0, kReady = 1, kHop = 2, kRun = 3 };

// SplitMix64 output function (Steele, Lea and Flood, 2014).
__device__ inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

struct Slot {
  int64_t release;
  int64_t left;    // remaining time of the current piece; -1 not started; -2 request submitted;
                   // the arrival time while the job travels between executors
  int64_t rleft;   // remaining service of the submitted request
  int32_t job, seq, cb;  // cb: set-local callback
  int8_t state, exec, pos, queued, ra, rl;
};

struct Sim {
  const DevBatch *b;
  const paam_des_opts *o;
  int64_t set, scen, c0, a0, x0, j0;
  int n_cb;
  int C, X, NA;
};

__device__ inline int64_t scaled(const Sim &s, int64_t x) { return x * s.o->util_permille / 1000; }

// Actual time of item `item` of callback `cbl` (index within its chain) of
// job `job` of chain c: the WCET W, or a draw from [floor(W p / 1000), W].
__device__ int64_t actual(const Sim &s, int c, int32_t job, int cbl, int item, int64_t W) {
  const int p = s.o->exec_permille;
  if (p >= 1000) return W;
  const int64_t lo = W * p / 1000;
  if (W <= lo) return W;
  uint64_t k = s.o->seed;
  k = sm_mix(k + kGamma * (uint64_t)(s.set + 1));
  k = sm_mix(k + kGamma * (uint64_t)(s.scen + 1));
  k = sm_mix(k + kGamma * (uint64_t)(c + 1));
  k = sm_mix(k + kGamma * (uint64_t)((int64_t)job + 1));
  k = sm_mix(k + kGamma * (uint64_t)((int64_t)cbl * 64 + item + 1));
  return W - (int64_t)(k % (uint64_t)(W - lo + 1));
}

// Bucket level of chain c on accelerator a: chains with a segment on a,
// ranked by priority, rank r of m on level floor(r n / m).
__device__ int level_of(const Sim &s, const uint8_t *amask, int c, int a) {
  const DevBatch &b = *s.b;
  const int rc = b.rank0[s.c0 + c];
  int m = 0, r = 0;
  for (int d = 0; d < s.C; ++d)
    if ((amask[d] >> a) & 1) {
      ++m;
      r += b.rank0[s.c0 + d] < rc;
    }
  return (int)((int64_t)r * b.buckets[s.a0 + a] / m);
}

__device__ void simulate(const Sim &s, const int64_t *offs, int64_t *obs, int8_t *status) {
  const DevBatch &b = *s.b;
  const paam_des_opts &o = *s.o;
  const int C = s.C, X = s.X, NA = s.NA;
  const int64_t hop = b.eps_hop[s.set];
  Slot sl[kSlots];
  int64_t rel[kDesChains], worst[kDesChains];
  int32_t njob[kDesChains];
  uint8_t amask[kDesChains];
  int8_t run[kDesExec], wait[kDesExec], cur[kMaxAccel * kDesLevels];
  for (int i = 0; i < 2 * C; ++i) sl[i].state = kFree, sl[i].queued = 0;
  for (int c = 0; c < C; ++c) {
    rel[c] = offs[c];
    worst[c] = -1;
    njob[c] = 0;
    amask[c] = 0;
  }
  // accelerator use per chain (segments are grouped by chain in set order)
  {
    const int64_t gs = b.set_seg_off[s.set], ge = b.set_seg_off[s.set + 1];
    for (int64_t g = gs; g < ge; ++g) amask[b.seg_chain[g]] |= (uint8_t)(1u << b.seg_accel[g]);
  }
  for (int e = 0; e < X; ++e) run[e] = -1, wait[e] = 0;
  for (int i = 0; i < NA * kDesLevels; ++i) cur[i] = -1;
  int32_t seq = 0;
  int64_t t = 0, steps = 0;
  int8_t st = 0;

  for (;;) {
    bool changed = true;
    while (changed) {
      changed = false;
      // releases
      for (int c = 0; c < C; ++c)
        while (rel[c] <= t && rel[c] <= o.horizon) {
          const int32_t k = njob[c]++;
          Slot &x = sl[2 * c + (k & 1)];
          if (x.state != kFree) {
            st = 1;
            goto done;
          }
          x.release = rel[c];
          x.job = k;
          x.cb = b.chain_cb_lo[s.c0 + c];
          x.state = kReady;
          x.exec = b.cb_exec[s.j0 + x.cb];
          x.queued = 0;
          x.pos = 0;
          x.left = -1;
          rel[c] += b.T[s.c0 + c];
          changed = true;
        }
      // hop arrivals
      for (int i = 0; i < 2 * C; ++i)
        if (sl[i].state == kHop && sl[i].left <= t) {
          sl[i].state = kReady;
          sl[i].exec = b.cb_exec[s.j0 + sl[i].cb];
          changed = true;
        }
      // executors
      for (int e = 0; e < X; ++e) {
        if (run[e] < 0) {
          int best = -1, brank = 0;
          for (int i = 0; i < 2 * C; ++i) {
            if (sl[i].state != kReady || sl[i].exec != e) continue;
            const int ri = b.rank0[s.c0 + (i >> 1)];
            if (best < 0 || ri < brank || (ri == brank && sl[i].release < sl[best].release)) {
              best = i;
              brank = ri;
            }
          }
          if (best >= 0) {
            run[e] = (int8_t)best;
            sl[best].state = kRun;
            sl[best].pos = 0;
            sl[best].left = -1;
            changed = true;
          }
        }
        if (run[e] >= 0 && !wait[e]) {
          Slot &x = sl[run[e]];
          const int c = run[e] >> 1;
          const int64_t g0 = b.cb_seg_off[s.j0 + x.cb];
          const int eta = (int)(b.cb_seg_off[s.j0 + x.cb + 1] - g0);
          const int cb_lo = b.chain_cb_lo[s.c0 + c];
          const int cb_hi = c + 1 < C ? b.chain_cb_lo[s.c0 + c + 1] : s.n_cb;
          const int cbl = x.cb - cb_lo;
          const int n_items = 1 + 3 * eta;
          for (;;) {
            if (x.pos >= n_items) {  // the callback completes
              run[e] = -1;
              wait[e] = 0;
              if (x.cb + 1 == cb_hi) {
                const int64_t r = t - x.release;
                if (r > worst[c]) worst[c] = r;
                x.state = kFree;
              } else {
                x.cb += 1;
                const int nx = b.cb_exec[s.j0 + x.cb];
                if (nx != e && hop > 0) {
                  x.state = kHop;
                  x.left = t + hop;
                } else {
                  x.state = kReady;
                  x.exec = (int8_t)nx;
                }
              }
              changed = true;
              break;
            }
            const int ph = x.pos % 3;
            if (ph == 2) {  // an accelerator request
              if (x.left == -1) {
                const int k = (x.pos - 1) / 3;
                const int a = b.seg_accel[g0 + k];
                x.queued = 1;
                x.ra = (int8_t)a;
                x.rl = (int8_t)level_of(s, amask, c, a);
                x.rleft = actual(s, c, x.job, cbl, k, scaled(s, b.A[g0 + k])) + 2 * b.akappa[s.a0 + a];
                x.seq = seq++;
                x.left = -2;
                wait[e] = 1;
                changed = true;
              }
              break;
            }
            if (x.left == -1) {
              if (ph == 1) {
                x.left = b.aeps[s.a0 + b.seg_accel[g0 + (x.pos - 1) / 3]];
              } else {
                const int64_t E = actual(s, c, x.job, cbl, 63, scaled(s, b.E[s.j0 + x.cb]));
                const int p = x.pos / 3, parts = eta + 1;
                x.left = E / parts + (p < E % parts ? 1 : 0);
              }
            }
            if (x.left > 0) break;
            x.pos += 1;
            x.left = -1;
            changed = true;
          }
        }
      }
      // accelerators
      for (int a = 0; a < NA; ++a) {
        const int nb = b.buckets[s.a0 + a];
        for (int l = 0; l < nb; ++l) {
          int8_t &q = cur[a * kDesLevels + l];
          if (q < 0) {
            int best = -1, brank = 0;
            for (int i = 0; i < 2 * C; ++i) {
              if (!sl[i].queued || sl[i].ra != a || sl[i].rl != l) continue;
              const int ri = b.rank0[s.c0 + (i >> 1)];
              if (best < 0 || ri < brank || (ri == brank && sl[i].seq < sl[best].seq)) {
                best = i;
                brank = ri;
              }
            }
            if (best >= 0) {
              q = (int8_t)best;
              sl[best].queued = 0;
            }
          }
          if (q >= 0) {
            Slot &x = sl[q];
            if (x.rleft == 0) {
              q = -1;
              x.pos += 1;
              x.left = -1;
              wait[x.exec] = 0;
              changed = true;
            }
            break;
          }
        }
      }
    }
    if (t >= o.horizon) break;
    if (++steps > o.max_steps) {
      st = 2;
      break;
    }
    // the next event
    int64_t next = o.horizon;
    for (int c = 0; c < C; ++c) next = rel[c] < next ? rel[c] : next;
    for (int i = 0; i < 2 * C; ++i)
      if (sl[i].state == kHop && sl[i].left < next) next = sl[i].left;
    uint32_t going = 0;  // executors whose CPU piece advances
    for (int e = 0; e < X; ++e) {
      if (run[e] < 0 || wait[e]) continue;
      const uint32_t above = b.hpx_mask[s.x0 + e];
      bool beaten = false;
      for (int f = 0; f < X; ++f)
        if (((above >> f) & 1) && run[f] >= 0 && (!wait[f] || b.spin[s.c0 + (run[f] >> 1)]))
          beaten = true;
      if (!beaten) {
        going |= 1u << e;
        const int64_t end = t + sl[run[e]].left;
        next = end < next ? end : next;
      }
    }
    int served[kMaxAccel];
    for (int a = 0; a < NA; ++a) {
      served[a] = -1;
      const int nb = b.buckets[s.a0 + a];
      for (int l = 0; l < nb; ++l)
        if (cur[a * kDesLevels + l] >= 0) {
          served[a] = cur[a * kDesLevels + l];
          break;
        }
      if (served[a] >= 0) {
        const int64_t end = t + sl[served[a]].rleft;
        next = end < next ? end : next;
      }
    }
    const int64_t dt = next - t;
    for (int e = 0; e < X; ++e)
      if ((going >> e) & 1) sl[run[e]].left -= dt;
    for (int a = 0; a < NA; ++a)
      if (served[a] >= 0) sl[served[a]].rleft -= dt;
    t = next;
  }
done:
  for (int c = 0; c < C; ++c) obs[c] = worst[c];
  *status = st;
}

__global__ __launch_bounds__(kWave) void des_kernel(DesLaunch L) {
  const DevBatch &b = L.b;
  const int64_t per_set = (L.o.n_scen + kWave - 1) / kWave;
  const int64_t n_work = b.n_sets * per_set;
  for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const int64_t set = w / per_set;
    const int64_t scen = (w % per_set) * kWave + threadIdx.x;
    if (scen >= L.o.n_scen) continue;
    Sim s;
    s.b = &b;
    s.o = &L.o;
    s.set = set;
    s.scen = scen;
    s.c0 = b.set_chain_off[set];
    s.C = (int)(b.set_chain_off[set + 1] - s.c0);
    s.x0 = b.set_exec_off[set];
    s.X = (int)(b.set_exec_off[set + 1] - s.x0);
    s.a0 = b.set_accel_off[set];
    s.NA = (int)(b.set_accel_off[set + 1] - s.a0);
    s.j0 = b.set_cb_off[set];
    s.n_cb = (int)(b.set_cb_off[set + 1] - s.j0);
    const int64_t base = s.c0 * L.o.n_scen + scen * s.C;
    simulate(s, L.offsets + base, L.obs + base, L.status + set * L.o.n_scen + scen);
  }
}

}  // namespace

int launch_des(const DesLaunch &L, void *stream) {
  hipLaunchKernelGGL(des_kernel, dim3(L.grid), dim3(kWave), 0, (hipStream_t)stream, L);
  return (int)hipGetLastError();
}

}  // namespace paam
