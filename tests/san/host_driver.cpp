// Drives the host side of libpaam (validation, derivation and packing of a
// batch, run on up to 16 threads) without a GPU, under the address,
// undefined-behaviour or thread sanitizer (tests/test_sanitizers.py).
// Test infrastructure only: paam_chainset_bytes makes no HIP call.
#include <cstdio>
#include <cstring>
#include <vector>

#include "paam.h"
extern "C" {
#include "batch_io.h"
}

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  const char *d = argv[1];
  paam_chainset_host h;
  std::memset(&h, 0, sizeof h);
  h.n_sets = static_cast<int64_t *>(san_read(d, "n_sets", nullptr))[0];
#define RD(f) h.f = static_cast<decltype(h.f)>(san_read(d, #f, nullptr))
  RD(set_chain_off); RD(set_exec_off); RD(set_accel_off); RD(chain_cb_off); RD(cb_seg_off);
  RD(T); RD(D); RD(prio); RD(spin); RD(E); RD(exec); RD(A); RD(accel); RD(exec_core);
  RD(exec_prio); RD(accel_buckets); RD(accel_eps); RD(accel_kappa); RD(eps_hop);
#undef RD
  size_t n = 0;
  if (paam_chainset_bytes(&h, &n) != PAAM_OK || n == 0) {
    std::fprintf(stderr, "valid batch rejected: %s\n", paam_last_error());
    return 4;
  }
  // units of every accelerator, each grouping
  const int64_t NA = h.set_accel_off[h.n_sets];
  std::vector<int16_t> units(NA > 0 ? NA : 1, 2);
  h.accel_units = units.data();
  for (int g = 0; g < 3; ++g) {
    h.unit_group = g;
    size_t m = 0;
    if (paam_chainset_bytes(&h, &m) != PAAM_OK || m <= n) return 5;
  }
  h.unit_group = 7;
  if (paam_chainset_bytes(&h, &n) == PAAM_OK) return 6;
  h.accel_units = nullptr;
  h.unit_group = 0;
  // malformed copies, each rejected
  const int64_t last = h.set_chain_off[h.n_sets] - 1;
  std::vector<int32_t> prio(h.prio, h.prio + last + 1);
  prio[last] = prio[last - 1];
  const int32_t *keep_prio = h.prio;
  h.prio = prio.data();
  if (paam_chainset_bytes(&h, &n) != PAAM_E_INVAL) return 7;
  h.prio = keep_prio;
  std::vector<int64_t> D(h.D, h.D + last + 1);
  D[last / 2] = h.T[last / 2] + 1;
  const int64_t *keep_D = h.D;
  h.D = D.data();
  if (paam_chainset_bytes(&h, &n) != PAAM_E_INVAL) return 8;
  h.D = keep_D;
  std::vector<int64_t> T(h.T, h.T + last + 1);
  T[last / 3] = int64_t(1) << 36;
  const int64_t *keep_T = h.T;
  h.T = T.data();
  if (paam_chainset_bytes(&h, &n) != PAAM_E_RANGE) return 9;
  h.T = keep_T;
  std::printf("host driver ok: %lld sets\n", (long long)h.n_sets);
  return 0;
}
