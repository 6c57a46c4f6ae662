// Binding of accelerator segments to the units of their accelerator type.
//
// Sec. IV-E ("Managing Multiple Accelerators"): when a system has several
// units of one accelerator type, the server keeps one set of workers per
// unit, and every callback's accelerator segment is bound to one unit at
// registration by a bin-packing heuristic such as worst-fit decreasing, as
// in partitioned multiprocessor scheduling.  Each unit is then analysed as
// an accelerator of its own.
//
// The batch keeps the input type of every segment (seg_type) and the unit
// count of every type; this kernel writes the unit of every segment into the
// analysed-accelerator array (seg_accel) in place.  One wave per set:
//   1. every segment's item: the segment itself, or the segments of its
//      callback or chain on its type (keys are non-decreasing in segment
//      order, so an item's segments lie in one key range); the item's leader
//      is its first segment;
//   2. leaders sum their segments' A (saturating at 2^36) and take the size
//      floor(sum * 2^26 / T) clamped at 2^36;
//   3. each leader's place in the decreasing order (size, then higher chain
//      priority, then lower leader index) by counting the leaders before it;
//   4. lane 0 places the items in that order, each on the least-loaded unit
//      of its type (lowest unit on ties), loads being sums of sizes;
//   5. every segment takes its leader's unit.
// The arithmetic is integer throughout, so the result is bit-exact.
#include <hip/hip_runtime.h>

#include "paam_internal.h"

namespace paam {
namespace {

constexpr int kUnitShift = 26;
constexpr int64_t kUnitClamp = int64_t(1) << 36;

struct UnitLaunch {
  DevBatch b;
  int16_t *seg_accel;  // the arena's analysed accelerators (written)
};

// LDS per wave for sets of up to n segments: size (8 B), key and leader
// (4 B each), place (4 B), unit, type and chain rank (2 B each).
__host__ __device__ inline size_t unit_lds_bytes(int64_t n) {
  return (size_t)(n > 0 ? n : 1) * 26 + 64;
}

__global__ __launch_bounds__(kWave) void units_kernel(UnitLaunch L) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int64_t load[kMaxAccel];
  __shared__ int32_t ubase[kMaxAccel + 1];
  __shared__ int32_t n_items;
  const DevBatch &b = L.b;
  const int lane = threadIdx.x;
  const int64_t cap = b.max_segs;
  int64_t *size = reinterpret_cast<int64_t *>(lds);
  int32_t *key = reinterpret_cast<int32_t *>(size + cap);
  int32_t *lead = key + cap;
  int32_t *place = lead + cap;
  int16_t *unit = reinterpret_cast<int16_t *>(place + cap);
  int16_t *type = unit + cap;
  int16_t *crank = type + cap;

  for (int64_t s = blockIdx.x; s < b.n_sets; s += gridDim.x) {
    const int64_t g0 = b.set_seg_off[s];
    const int n = (int)(b.set_seg_off[s + 1] - g0);
    const int64_t c0 = b.set_chain_off[s];
    const int64_t t0 = b.set_type_off[s];
    const int NT = (int)(b.set_type_off[s + 1] - t0);
    if (lane == 0) {
      int acc = 0;
      for (int a = 0; a < NT; ++a) {
        ubase[a] = acc;
        acc += b.type_units[t0 + a];
      }
      ubase[NT] = acc;
      for (int u = 0; u < kMaxAccel; ++u) load[u] = 0;
      n_items = 0;
    }
    // 1. keys, types and chain ranks
    if (b.unit_group == PAAM_UNITS_CALLBACK) {
      const int64_t j0 = b.set_cb_off[s], j1 = b.set_cb_off[s + 1];
      for (int64_t j = j0 + lane; j < j1; j += kWave)
        for (int64_t g = b.cb_seg_off[j]; g < b.cb_seg_off[j + 1]; ++g)
          key[g - g0] = (int32_t)(j - j0);
    }
    for (int i = lane; i < n; i += kWave) {
      const int c = b.seg_chain[g0 + i];
      if (b.unit_group == PAAM_UNITS_SEGMENT) key[i] = i;
      if (b.unit_group == PAAM_UNITS_CHAIN) key[i] = c;
      type[i] = b.seg_type[g0 + i];
      crank[i] = b.rank0[c0 + c];
    }
    __syncthreads();
    // 1-2. leaders and their sizes
    for (int i = lane; i < n; i += kWave) {
      int l = i;
      for (int k = i - 1; k >= 0 && key[k] == key[i]; --k)
        if (type[k] == type[i]) l = k;
      lead[i] = l;
      if (l == i) {
        int64_t sum = 0;
        for (int k = i; k < n && key[k] == key[i]; ++k)
          if (type[k] == type[i]) {
            sum += b.A[g0 + k];
            if (sum > kUnitClamp) sum = kUnitClamp;
          }
        const int64_t T = b.T[c0 + b.seg_chain[g0 + i]];
        const int64_t sz = (sum << kUnitShift) / T;  // sum <= 2^36: no overflow
        size[i] = sz > kUnitClamp ? kUnitClamp : sz;
      }
    }
    __syncthreads();
    // 3. place of every leader in the decreasing order
    for (int i = lane; i < n; i += kWave) {
      if (lead[i] != i) continue;
      const int64_t si = size[i];
      const int ri = crank[i];
      int p = 0;
      for (int j = 0; j < n; ++j) {
        if (lead[j] != j || j == i) continue;
        const int64_t sj = size[j];
        p += sj > si || (sj == si && (crank[j] < ri || (crank[j] == ri && j < i)));
      }
      place[p] = i;
      atomicAdd(&n_items, 1);
    }
    __syncthreads();
    // 4. worst fit, in placement order
    if (lane == 0) {
      const int m = n_items;
      for (int p = 0; p < m; ++p) {
        const int i = place[p];
        const int a = type[i];
        const int u0 = ubase[a], u1 = ubase[a + 1];
        int best = u0;
        for (int u = u0 + 1; u < u1; ++u)
          if (load[u] < load[best]) best = u;
        load[best] += size[i];
        unit[i] = (int16_t)best;
      }
    }
    __syncthreads();
    // 5. every segment on its item's unit
    for (int i = lane; i < n; i += kWave) L.seg_accel[g0 + i] = unit[lead[i]];
    __syncthreads();
  }
}

}  // namespace

int launch_units(const DevBatch &b, int n_cus, void *stream) {
  if (b.unit_group < 0 || b.n_sets == 0) return hipSuccess;
  UnitLaunch L;
  L.b = b;
  L.seg_accel = const_cast<int16_t *>(b.seg_accel);
  const size_t lds = unit_lds_bytes(b.max_segs);
  const int64_t want = (int64_t)n_cus * 8;
  const int grid = (int)(b.n_sets < want ? b.n_sets : want);
  hipLaunchKernelGGL(units_kernel, dim3(grid), dim3(kWave), lds, (hipStream_t)stream, L);
  return (int)hipGetLastError();
}

size_t units_lds_bytes(int64_t max_segs) { return unit_lds_bytes(max_segs); }

}  // namespace paam
