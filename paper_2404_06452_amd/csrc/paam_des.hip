// Event-driven simulation of chain sets under the PAAM model, one lane per
// (set, scenario): the observed end-to-end latencies that the analysis of
// Sec. IV-F must bound (the paper's Case Study 1, Sec. V-A, checks the same
// property on real hardware).
//
// A wave takes 64 scenarios of one set, so every lane reads the same set
// tables while it runs its own timeline; lanes never synchronise.  A lane's
// job slots (two per chain) and the request served on every bucket level
// live in private arrays; which slots are live, ready, travelling or queued,
// which executors run or wait, and which levels are occupied are bit masks
// in registers.
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
  int8_t exec, pos, ra, rl;
};

struct Sim {
  const DevBatch *b;
  const paam_des_opts *o;
  const int16_t *rank;  // [C] priority rank of every chain (LDS)
  const int8_t *lev;    // [C][kMaxAccel] bucket level of a chain's requests (LDS)
  // the set's tables, staged in LDS once per wave (times already scaled by
  // util_permille): per callback E, first segment, executor; per segment A
  // and accelerator
  const int64_t *cbE, *segA;
  const int16_t *cbSeg;  // [n_cb + 1] set-local segment offsets
  const int8_t *cbExec, *segAcc;
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

// Slot sets, executor sets and occupied bucket levels are bit masks held in
// registers, so the per-instant scans touch only the slots that matter (the
// ready, travelling or queued ones); the per-slot fields live in private
// memory.  Executor e's running slot is byte e of run_lo/run_hi.
__device__ inline int run_slot(uint64_t lo, uint64_t hi, int e) {
  return (int)(((e < 8 ? lo : hi) >> (8 * (e & 7))) & 0xff);
}
__device__ inline void set_run_slot(uint64_t &lo, uint64_t &hi, int e, int v) {
  uint64_t &w = e < 8 ? lo : hi;
  const int sh = 8 * (e & 7);
  w = (w & ~(0xffull << sh)) | ((uint64_t)v << sh);
}

__device__ void simulate(const Sim &s, const int64_t *offs, int64_t *obs, int8_t *status) {
  const DevBatch &b = *s.b;
  const paam_des_opts &o = *s.o;
  const int C = s.C, X = s.X, NA = s.NA;
  const int64_t hop = b.eps_hop[s.set];
  Slot sl[kSlots];
  int64_t rel[kDesChains], worst[kDesChains];
  int32_t njob[kDesChains];
  int8_t cur[kMaxAccel * kDesLevels];
  uint64_t live = 0, ready = 0, hopm = 0, queued = 0, busy = 0;  // slots; levels a*8+l
  uint32_t runm = 0, waitm = 0, spinm = 0;                         // executors
  uint64_t run_lo = 0, run_hi = 0;
  int64_t next_rel = INT64_MAX;
  for (int c = 0; c < C; ++c) {
    rel[c] = offs[c];
    next_rel = rel[c] < next_rel ? rel[c] : next_rel;
    worst[c] = -1;
    njob[c] = 0;
  }
  int32_t seq = 0;
  int64_t t = 0, steps = 0;
  int8_t st = 0;

  for (;;) {
    bool changed = true;
    while (changed) {
      changed = false;
      // releases
      if (next_rel <= t) {
        next_rel = INT64_MAX;
        for (int c = 0; c < C; ++c) {
          while (rel[c] <= t && rel[c] <= o.horizon) {
            const int32_t k = njob[c]++;
            const int i = 2 * c + (k & 1);
            if ((live >> i) & 1) {
              st = 1;
              goto done;
            }
            Slot &x = sl[i];
            x.release = rel[c];
            x.job = k;
            x.cb = b.chain_cb_lo[s.c0 + c];
            x.exec = s.cbExec[x.cb];
            live |= 1ull << i;
            ready |= 1ull << i;
            rel[c] += b.T[s.c0 + c];
            changed = true;
          }
          next_rel = rel[c] < next_rel ? rel[c] : next_rel;
        }
      }
      // hop arrivals
      for (uint64_t m = hopm; m; m &= m - 1) {
        const int i = __builtin_ctzll(m);
        if (sl[i].left <= t) {
          hopm &= ~(1ull << i);
          ready |= 1ull << i;
          sl[i].exec = s.cbExec[sl[i].cb];
          changed = true;
        }
      }
      // executors
      for (int e = 0; e < X; ++e) {
        if (!((runm >> e) & 1) && ready) {
          int best = -1, brank = 0;
          for (uint64_t m = ready; m; m &= m - 1) {
            const int i = __builtin_ctzll(m);
            if (sl[i].exec != e) continue;
            const int ri = s.rank[i >> 1];
            if (best < 0 || ri < brank || (ri == brank && sl[i].release < sl[best].release)) {
              best = i;
              brank = ri;
            }
          }
          if (best >= 0) {
            ready &= ~(1ull << best);
            runm |= 1u << e;
            set_run_slot(run_lo, run_hi, e, best);
            if (b.spin[s.c0 + (best >> 1)]) spinm |= 1u << e; else spinm &= ~(1u << e);
            sl[best].pos = 0;
            sl[best].left = -1;
            changed = true;
          }
        }
        if (((runm & ~waitm) >> e) & 1) {
          const int i = run_slot(run_lo, run_hi, e);
          Slot &x = sl[i];
          const int c = i >> 1;
          const int g0 = s.cbSeg[x.cb];
          const int eta = s.cbSeg[x.cb + 1] - g0;
          const int cb_lo = b.chain_cb_lo[s.c0 + c];
          const int cb_hi = c + 1 < C ? b.chain_cb_lo[s.c0 + c + 1] : s.n_cb;
          const int cbl = x.cb - cb_lo;
          const int n_items = 1 + 3 * eta;
          for (;;) {
            if (x.pos >= n_items) {  // the callback completes
              runm &= ~(1u << e);
              waitm &= ~(1u << e);
              if (x.cb + 1 == cb_hi) {
                const int64_t r = t - x.release;
                if (r > worst[c]) worst[c] = r;
                live &= ~(1ull << i);
              } else {
                x.cb += 1;
                const int nx = s.cbExec[x.cb];
                if (nx != e && hop > 0) {
                  hopm |= 1ull << i;
                  x.left = t + hop;
                } else {
                  ready |= 1ull << i;
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
                const int a = s.segAcc[g0 + k];
                queued |= 1ull << i;
                x.ra = (int8_t)a;
                x.rl = s.lev[c * kMaxAccel + a];
                x.rleft = actual(s, c, x.job, cbl, k, s.segA[g0 + k]) + 2 * b.akappa[s.a0 + a];
                x.seq = seq++;
                x.left = -2;
                waitm |= 1u << e;
                changed = true;
              }
              break;
            }
            if (x.left == -1) {
              if (ph == 1) {
                x.left = b.aeps[s.a0 + s.segAcc[g0 + (x.pos - 1) / 3]];
              } else {
                const int64_t E = actual(s, c, x.job, cbl, 63, s.cbE[x.cb]);
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
          const int q = a * kDesLevels + l;
          if (!((busy >> q) & 1) && queued) {
            int best = -1, brank = 0;
            for (uint64_t m = queued; m; m &= m - 1) {
              const int i = __builtin_ctzll(m);
              if (sl[i].ra != a || sl[i].rl != l) continue;
              const int ri = s.rank[i >> 1];
              if (best < 0 || ri < brank || (ri == brank && sl[i].seq < sl[best].seq)) {
                best = i;
                brank = ri;
              }
            }
            if (best >= 0) {
              cur[q] = (int8_t)best;
              busy |= 1ull << q;
              queued &= ~(1ull << best);
            }
          }
          if ((busy >> q) & 1) {
            Slot &x = sl[cur[q]];
            if (x.rleft == 0) {
              busy &= ~(1ull << q);
              x.pos += 1;
              x.left = -1;
              waitm &= ~(1u << x.exec);
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
    int64_t next = next_rel < o.horizon ? next_rel : o.horizon;
    for (uint64_t m = hopm; m; m &= m - 1) {
      const int i = __builtin_ctzll(m);
      next = sl[i].left < next ? sl[i].left : next;
    }
    const uint32_t demand = (runm & ~waitm) | (waitm & spinm);
    uint32_t going = 0;  // executors whose CPU piece advances
    for (uint32_t m = runm & ~waitm; m; m &= m - 1) {
      const int e = __builtin_ctz(m);
      if (b.hpx_mask[s.x0 + e] & demand) continue;
      going |= 1u << e;
      const int64_t end = t + sl[run_slot(run_lo, run_hi, e)].left;
      next = end < next ? end : next;
    }
    int served[kMaxAccel];
    for (int a = 0; a < NA; ++a) {
      const uint32_t lv = (uint32_t)(busy >> (a * kDesLevels)) & 0xff;
      served[a] = lv ? cur[a * kDesLevels + __builtin_ctz(lv)] : -1;
      if (served[a] >= 0) {
        const int64_t end = t + sl[served[a]].rleft;
        next = end < next ? end : next;
      }
    }
    const int64_t dt = next - t;
    for (uint32_t m = going; m; m &= m - 1) sl[run_slot(run_lo, run_hi, __builtin_ctz(m))].left -= dt;
    for (int a = 0; a < NA; ++a)
      if (served[a] >= 0) sl[served[a]].rleft -= dt;
    t = next;
  }
done:
  for (int c = 0; c < C; ++c) obs[c] = worst[c];
  *status = st;
}

__global__ __launch_bounds__(kWave) void des_kernel(DesLaunch L) {
  __shared__ int16_t rank_s[kDesChains];
  __shared__ int32_t amask_s[kDesChains];
  __shared__ int8_t lev_s[kDesChains * kMaxAccel];
  extern __shared__ __attribute__((aligned(16))) unsigned char des_lds[];
  const DevBatch &b = L.b;
  // per set: E and first segment of every callback, A of every segment,
  // then the byte-wide executors and accelerators (sized for the batch)
  int64_t *cbE = reinterpret_cast<int64_t *>(des_lds);
  int64_t *segA = cbE + L.max_cbs;
  int16_t *cbSeg = reinterpret_cast<int16_t *>(segA + L.max_segs);
  int8_t *cbExec = reinterpret_cast<int8_t *>(cbSeg + L.max_cbs + 1);
  int8_t *segAcc = cbExec + L.max_cbs;
  const int lane = threadIdx.x;
  const int64_t per_set = (L.o.n_scen + kWave - 1) / kWave;
  const int64_t n_work = b.n_sets * per_set;
  for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const int64_t set = w / per_set;
    const int64_t scen = (w % per_set) * kWave + lane;
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
    // the set's tables, shared by the wave's scenarios: ranks, accelerators
    // used by every chain, and the bucket level of every (chain, accelerator)
    // user (Sec. IV-C: users ranked by priority, rank r of m on level
    // floor(r * n / m))
    for (int c = lane; c < s.C; c += kWave) {
      rank_s[c] = b.rank0[s.c0 + c];
      amask_s[c] = 0;
    }
    __syncthreads();
    for (int64_t g = b.set_seg_off[set] + lane; g < b.set_seg_off[set + 1]; g += kWave)
      atomicOr(&amask_s[b.seg_chain[g]], 1 << b.seg_accel[g]);
    __syncthreads();
    for (int i = lane; i < s.C * s.NA; i += kWave) {
      const int c = i / s.NA, a = i - c * s.NA;
      int m = 0, r = 0;
      for (int d = 0; d < s.C; ++d)
        if ((amask_s[d] >> a) & 1) {
          ++m;
          r += rank_s[d] < rank_s[c];
        }
      lev_s[c * kMaxAccel + a] =
          ((amask_s[c] >> a) & 1) ? (int8_t)((int64_t)r * b.buckets[s.a0 + a] / m) : (int8_t)-1;
    }
    __syncthreads();
    {
      const int64_t g0 = b.set_seg_off[set];
      const int nseg = (int)(b.set_seg_off[set + 1] - g0);
      for (int j = lane; j < s.n_cb; j += kWave) {
        cbE[j] = scaled(s, b.E[s.j0 + j]);
        cbSeg[j] = (int16_t)(b.cb_seg_off[s.j0 + j] - g0);
        cbExec[j] = b.cb_exec[s.j0 + j];
      }
      if (lane == 0) cbSeg[s.n_cb] = (int16_t)nseg;
      for (int g = lane; g < nseg; g += kWave) {
        segA[g] = scaled(s, b.A[g0 + g]);
        segAcc[g] = (int8_t)b.seg_accel[g0 + g];
      }
    }
    __syncthreads();
    s.rank = rank_s;
    s.lev = lev_s;
    s.cbE = cbE;
    s.segA = segA;
    s.cbSeg = cbSeg;
    s.cbExec = cbExec;
    s.segAcc = segAcc;
    if (scen < L.o.n_scen) {
      const int64_t base = s.c0 * L.o.n_scen + scen * s.C;
      simulate(s, L.offsets + base, L.obs + base, L.status + set * L.o.n_scen + scen);
    }
    __syncthreads();
  }
}

}  // namespace

size_t des_lds_bytes(int64_t max_cbs, int64_t max_segs) {
  return (size_t)max_cbs * 8 + (size_t)max_segs * 8 + (size_t)(max_cbs + 1) * 2 + (size_t)max_cbs +
         (size_t)max_segs + 16;
}

int launch_des(const DesLaunch &L, void *stream) {
  hipLaunchKernelGGL(des_kernel, dim3(L.grid), dim3(kWave), des_lds_bytes(L.max_cbs, L.max_segs),
                     (hipStream_t)stream, L);
  return (int)hipGetLastError();
}

}  // namespace paam
