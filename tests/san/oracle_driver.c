/* Runs every oracle entry point over a batch, for the address, undefined-
 * behaviour and thread sanitizers (tests/test_sanitizers.py).  Test
 * infrastructure only. */
#include <pthread.h>
#include <string.h>

#include "../../oracle/paam_oracle.h"
#include "batch_io.h"

static oracle_chainsets cs;
static int64_t *chain_R, *worst_R, *terms;
static int8_t *sched;
static int32_t *worst;

typedef struct {
  int64_t lo, hi;
  int rc;
} range_t;

static void *run_range(void *arg) {
  range_t *r = arg;
  oracle_opts o = {0, 2, 700, 1, 0};
  r->rc = oracle_wcrt_range(&cs, &o, r->lo, r->hi, chain_R, sched, worst, worst_R, terms);
  return NULL;
}

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  const char *d = argv[1];
  long nb;
  int64_t *n_sets = san_read(d, "n_sets", &nb);
  cs.n_sets = n_sets[0];
#define RD(f) cs.f = san_read(d, #f, NULL)
  RD(set_chain_off); RD(set_exec_off); RD(set_accel_off); RD(chain_cb_off); RD(cb_seg_off);
  RD(T); RD(D); RD(prio); RD(spin); RD(E); RD(exec); RD(A); RD(accel); RD(exec_core);
  RD(exec_prio); RD(accel_buckets); RD(accel_eps); RD(accel_kappa); RD(eps_hop);
#undef RD
  const int64_t S = cs.n_sets, NC = cs.set_chain_off[S], NA = cs.set_accel_off[S];
  const int64_t NG = cs.cb_seg_off[cs.chain_cb_off[NC]];
  chain_R = calloc((size_t)NC, 8); worst_R = calloc((size_t)S, 8); terms = calloc((size_t)S, 8);
  sched = calloc((size_t)S, 1); worst = calloc((size_t)S, 4);
  /* analysis on four threads (the oracle is re-entrant) */
  pthread_t th[4];
  range_t rg[4];
  for (int t = 0; t < 4; ++t) {
    rg[t].lo = S * t / 4;
    rg[t].hi = S * (t + 1) / 4;
    pthread_create(&th[t], NULL, run_range, &rg[t]);
  }
  for (int t = 0; t < 4; ++t) {
    pthread_join(th[t], NULL);
    if (rg[t].rc) return 4;
  }
  /* every option set on the first sets */
  for (int b = 0; b < 2; ++b)
    for (int bound = 0; bound < 3; ++bound)
      for (int full = 0; full < 2; ++full) {
        oracle_opts o = {b, 1 + 63 * full, 1000, full, bound};
        if (oracle_wcrt_range(&cs, &o, 0, S < 50 ? S : 50, chain_R, sched, worst, worst_R, terms))
          return 5;
      }
  oracle_opts o = {0, 1, 300, 0, 0};
  int32_t *found = calloc((size_t)S, 4), *n_eval = calloc((size_t)S, 4);
  if (oracle_search_range(&cs, &o, 8, 42, 0, S < 40 ? S : 40, found, n_eval, NULL)) return 6;
  int16_t *units = malloc((size_t)(NA > 0 ? NA : 1) * 2), *unit = malloc((size_t)(NG > 0 ? NG : 1) * 2);
  for (int64_t a = 0; a < NA; ++a) units[a] = (int16_t)(1 + a % 3);
  for (int g = 0; g < 3; ++g)
    if (oracle_wfd_range(&cs, units, g, 0, S, unit)) return 7;
  oracle_des_opts dopt = {4, 0, 600, 11, 300, 100000};
  int64_t maxT = 0;
  for (int64_t c = 0; c < NC; ++c) maxT = cs.T[c] > maxT ? cs.T[c] : maxT;
  dopt.horizon = maxT;
  const int64_t sim_sets = S < 30 ? S : 30;
  const int64_t sim_chains = cs.set_chain_off[sim_sets];
  int64_t *off = calloc((size_t)(sim_chains * dopt.n_scen + 1), 8);
  int64_t *obs = calloc((size_t)(sim_chains * dopt.n_scen + 1), 8);
  int8_t *st = calloc((size_t)(sim_sets * dopt.n_scen + 1), 1);
  for (int64_t i = 0; i < sim_chains * dopt.n_scen; ++i) off[i] = (i * 7919) % 1000;
  if (oracle_des_range(&cs, &dopt, off, 0, sim_sets, obs, st)) return 8;
  printf("oracle driver ok: %lld sets\n", (long long)S);
  return 0;
}
