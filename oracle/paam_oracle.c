/*
 * CPU oracle of the PAAM worst-case response-time analysis (paper Sec. IV-F).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.
 *
 * Plain and single-threaded on purpose.  Every recurrence is a Kleene
 * iteration from 0 that stops at equality or when an iterate exceeds the cap
 * of its chain (then the value is ORACLE_INF).  Sets of sub-chains are solved
 * in dependency order: per core, executors by process priority (highest
 * first); within an executor, chains by chain priority (highest first).
 */
#include "paam_oracle.h"

#include <stdlib.h>
#include <string.h>

#define INF ORACLE_INF

/* ---------- saturating int64 arithmetic on non-negative values ---------- */
static int64_t sat_add(int64_t a, int64_t b) {
  if (a == INF || b == INF || a > INF - b) return INF;
  return a + b;
}
/* a product with a zero factor is zero, also when the other factor is INF */
static int64_t sat_mul(int64_t a, int64_t b) {
  if (a == 0 || b == 0) return 0;
  if (a == INF || b == INF || a > INF / b) return INF;
  return a * b;
}
static int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }

/* Lemma 1, Eq. (2): requests of a chain with period T in a window of length
 * t: ceil(t/T) + 1, with ceil(0/T) = 0. */
static int64_t mu(int64_t t, int64_t T) {
  if (t == INF) return INF;
  return t / T + (t % T != 0 ? 1 : 0) + 1;
}

/* ------------------------------ one set ------------------------------- */
typedef struct {
  const oracle_chainsets *cs;
  const oracle_opts *opt;
  int32_t C, X, NA;
  int64_t c0, cb0, ncb, g0, nseg, x0, a0;
  int64_t *terms;

  int32_t *pi;       /* [C] priority, larger = higher */
  int64_t *cap;      /* [C] cap_mult * D */
  int64_t *Ecb;      /* [ncb] CPU WCET, scaled */
  int64_t *Astar;    /* [nseg] A* = A + 2 kappa (Sec. IV-F, before Eq. 1) */
  int32_t *seg_cb;   /* [nseg] owning callback (set-local) */
  int32_t *cb_chain; /* [ncb] owning chain */
  uint8_t *uses;     /* [C*NA] chain has a segment on the accelerator */
  int64_t *Ahat;     /* [C*NA] sum of A* of the chain's segments on it */
  int32_t *level;    /* [C*NA] bucket of the chain on the accelerator, 0 = top */
  int64_t *Bacc;     /* [nseg] blocking by one LP request of the same bucket */
  int64_t *H;        /* [nseg] Lemma 2 bound */

  uint8_t *on;       /* [C*X] chain has callbacks on the executor */
  int64_t *Ece;      /* [C*X] sum of the chain's CPU WCETs on the executor */
  int64_t *epsce;    /* [C*X] sum of epsilon over the chain's segments on it */
  int64_t *Hstar_ce; /* [C*X] sum of H* over the chain's sub-chains on it */

  int32_t nrun;      /* sub-chains: maximal runs of a chain on one executor */
  int32_t *run_chain, *run_exec, *run_cb_lo, *run_cb_hi; /* cb range set-local */
  int64_t *run_E, *run_L2, *run_A0, *run_eps, *run_B, *run_R;
  int32_t *run_delta;
  uint8_t *run_acc;  /* [nrun*NA] accelerators used by the sub-chain */
  int32_t *nsub;     /* [C] sub-chains per chain */
} setctx;

static int64_t scale(const setctx *s, int64_t x) {
  int64_t u = s->opt->util_permille;
  return u == 1000 ? x : (x * u) / 1000;
}

static int64_t chain_T(const setctx *s, int32_t c) { return s->cs->T[s->c0 + c]; }

/* Lemma 2, Eq. (3): handling time of segment g, with one term per higher
 * priority chain using the same accelerator (mu depends on the chain only). */
static int64_t lemma2(setctx *s, int64_t g) {
  const int32_t c = s->cb_chain[s->seg_cb[g]];
  const int32_t a = s->cs->accel[s->g0 + g];
  int64_t h = 0;
  for (;;) {
    int64_t nxt = sat_add(s->Astar[g], s->Bacc[g]);
    for (int32_t k = 0; k < s->C; ++k) {
      if (k == c || s->pi[k] <= s->pi[c] || !s->uses[k * s->NA + a]) continue;
      nxt = sat_add(nxt, sat_mul(mu(h, chain_T(s, k)), s->Ahat[k * s->NA + a]));
      ++*s->terms;
    }
    if (nxt > s->cap[c]) return INF;
    if (nxt == h) return h;
    h = nxt;
  }
}

/* Lemma 3, Eq. (4) for sub-chain r over a window t: its own requests with
 * their blocking, plus every HP request on the accelerators it uses, each
 * HP segment counted once. */
static int64_t lemma3(setctx *s, int32_t r, int64_t t) {
  const int32_t c = s->run_chain[r];
  int64_t v = s->run_A0[r];
  for (int32_t a = 0; a < s->NA; ++a) {
    if (!s->run_acc[r * s->NA + a]) continue;
    for (int32_t k = 0; k < s->C; ++k) {
      if (k == c || s->pi[k] <= s->pi[c] || !s->uses[k * s->NA + a]) continue;
      v = sat_add(v, sat_mul(mu(t, chain_T(s, k)), s->Ahat[k * s->NA + a]));
      ++*s->terms;
    }
  }
  return v;
}

/* Eq. (1) with H = min(Lemma 2 summed over the segments, Lemma 3). */
static int64_t hstar(setctx *s, int32_t r, int64_t t) {
  if (s->run_delta[r] == 0) return 0;
  int64_t Hc;
  if (s->opt->bound == 1) Hc = s->run_L2[r];
  else if (s->opt->bound == 2) Hc = lemma3(s, r, t);
  else Hc = min64(s->run_L2[r], lemma3(s, r, t));
  return sat_add(Hc, s->run_eps[r]);
}

/* Theorem 1, Eq. (6), right-hand side for sub-chain r at window t. */
static int64_t thm1_rhs(setctx *s, int32_t r, int64_t t) {
  const int32_t c = s->run_chain[r], e = s->run_exec[r];
  const oracle_chainsets *cs = s->cs;
  int64_t v = sat_add(sat_add(s->run_B[r], s->run_E[r]), hstar(s, r, t));
  /* hp(c): higher priority chains on the same executor */
  for (int32_t h = 0; h < s->C; ++h) {
    if (h == c || s->pi[h] <= s->pi[c] || !s->on[h * s->X + e]) continue;
    int64_t w = sat_add(s->Ece[h * s->X + e], s->Hstar_ce[h * s->X + e]);
    v = sat_add(v, sat_mul(mu(t, chain_T(s, h)), w));
    ++*s->terms;
  }
  /* hpp(c): chains of higher process priority executors on the same core */
  for (int32_t e2 = 0; e2 < s->X; ++e2) {
    if (e2 == e || cs->exec_core[s->x0 + e2] != cs->exec_core[s->x0 + e] ||
        cs->exec_prio[s->x0 + e2] <= cs->exec_prio[s->x0 + e])
      continue;
    for (int32_t h = 0; h < s->C; ++h) {
      if (h == c || !s->on[h * s->X + e2]) continue;
      int64_t sp = cs->spin[s->c0 + h] ? s->Hstar_ce[h * s->X + e2] : s->epsce[h * s->X + e2];
      int64_t w = sat_add(s->Ece[h * s->X + e2], sp);
      v = sat_add(v, sat_mul(mu(t, chain_T(s, h)), w));
      ++*s->terms;
    }
  }
  return v;
}

static int64_t solve_run(setctx *s, int32_t r) {
  const int64_t cap = s->cap[s->run_chain[r]];
  int64_t t = 0;
  for (;;) {
    int64_t nxt = thm1_rhs(s, r, t);
    if (nxt > cap) return INF;
    if (nxt == t) return t;
    t = nxt;
  }
}

static void *zalloc(size_t n) { return calloc(n ? n : 1, 1); }

static void ctx_free(setctx *s) {
  void *p[] = {s->pi, s->cap, s->Ecb, s->Astar, s->seg_cb, s->cb_chain, s->uses, s->Ahat,
               s->level, s->Bacc, s->H, s->on, s->Ece, s->epsce, s->Hstar_ce, s->run_chain,
               s->run_exec, s->run_cb_lo, s->run_cb_hi, s->run_E, s->run_L2, s->run_A0,
               s->run_eps, s->run_B, s->run_R, s->run_delta, s->run_acc, s->nsub};
  for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); ++i) free(p[i]);
}

/* Validates the set and derives everything that does not depend on R. */
static int ctx_init(setctx *s, const oracle_chainsets *cs, int64_t set, const int32_t *order,
                    const oracle_opts *opt, int64_t *terms) {
  memset(s, 0, sizeof(*s));
  s->cs = cs;
  s->opt = opt;
  s->terms = terms;
  if (set < 0 || set >= cs->n_sets || opt->cap_mult < 1 || opt->util_permille < 0 ||
      opt->bound < 0 || opt->bound > 2)
    return -1;
  s->c0 = cs->set_chain_off[set];
  s->C = (int32_t)(cs->set_chain_off[set + 1] - s->c0);
  s->x0 = cs->set_exec_off[set];
  s->X = (int32_t)(cs->set_exec_off[set + 1] - s->x0);
  s->a0 = cs->set_accel_off[set];
  s->NA = (int32_t)(cs->set_accel_off[set + 1] - s->a0);
  if (s->C < 1 || s->X < 1 || s->NA < 0) return -1;
  s->cb0 = cs->chain_cb_off[s->c0];
  s->ncb = cs->chain_cb_off[s->c0 + s->C] - s->cb0;
  s->g0 = cs->cb_seg_off[s->cb0];
  s->nseg = cs->cb_seg_off[s->cb0 + s->ncb] - s->g0;
  const int32_t C = s->C, X = s->X, NA = s->NA;
  const int64_t ncb = s->ncb, nseg = s->nseg;

  s->pi = zalloc(sizeof(int32_t) * C);
  s->cap = zalloc(sizeof(int64_t) * C);
  s->Ecb = zalloc(sizeof(int64_t) * ncb);
  s->Astar = zalloc(sizeof(int64_t) * nseg);
  s->seg_cb = zalloc(sizeof(int32_t) * nseg);
  s->cb_chain = zalloc(sizeof(int32_t) * ncb);
  s->uses = zalloc((size_t)C * NA);
  s->Ahat = zalloc(sizeof(int64_t) * C * NA);
  s->level = zalloc(sizeof(int32_t) * C * NA);
  s->Bacc = zalloc(sizeof(int64_t) * nseg);
  s->H = zalloc(sizeof(int64_t) * nseg);
  s->on = zalloc((size_t)C * X);
  s->Ece = zalloc(sizeof(int64_t) * C * X);
  s->epsce = zalloc(sizeof(int64_t) * C * X);
  s->Hstar_ce = zalloc(sizeof(int64_t) * C * X);
  s->nsub = zalloc(sizeof(int32_t) * C);

  /* chains: priorities, caps, validity (Sec. II-C: D <= T, unique priorities) */
  if (order) {
    for (int32_t c = 0; c < C; ++c) s->pi[c] = -1;
    for (int32_t p = 0; p < C; ++p) {
      if (order[p] < 0 || order[p] >= C || s->pi[order[p]] != -1) return -1;
      s->pi[order[p]] = C - p;
    }
  } else {
    for (int32_t c = 0; c < C; ++c) s->pi[c] = cs->prio[s->c0 + c];
  }
  for (int32_t c = 0; c < C; ++c) {
    const int64_t T = cs->T[s->c0 + c], D = cs->D[s->c0 + c];
    if (T <= 0 || D <= 0 || D > T) return -1;
    for (int32_t k = 0; k < c; ++k)
      if (s->pi[k] == s->pi[c]) return -1;
    s->cap[c] = D > INF / opt->cap_mult ? INF : D * opt->cap_mult;
    const int64_t lo = cs->chain_cb_off[s->c0 + c], hi = cs->chain_cb_off[s->c0 + c + 1];
    if (hi <= lo) return -1;
    for (int64_t j = lo; j < hi; ++j) s->cb_chain[j - s->cb0] = c;
  }
  for (int32_t e = 0; e < X; ++e)
    for (int32_t e2 = 0; e2 < e; ++e2)
      if (cs->exec_core[s->x0 + e] == cs->exec_core[s->x0 + e2] &&
          cs->exec_prio[s->x0 + e] == cs->exec_prio[s->x0 + e2])
        return -1;
  for (int32_t a = 0; a < NA; ++a)
    if (cs->accel_buckets[s->a0 + a] < 1 || cs->accel_eps[s->a0 + a] < 0 ||
        cs->accel_kappa[s->a0 + a] < 0)
      return -1;
  if (cs->eps_hop[set] < 0) return -1;

  /* callbacks and segments */
  for (int64_t j = 0; j < ncb; ++j) {
    const int64_t E = cs->E[s->cb0 + j];
    const int32_t e = cs->exec[s->cb0 + j];
    if (E < 0 || e < 0 || e >= X) return -1;
    s->Ecb[j] = scale(s, E);
    const int32_t c = s->cb_chain[j];
    s->on[c * X + e] = 1;
    s->Ece[c * X + e] = sat_add(s->Ece[c * X + e], s->Ecb[j]);
    for (int64_t g = cs->cb_seg_off[s->cb0 + j]; g < cs->cb_seg_off[s->cb0 + j + 1]; ++g) {
      const int64_t gl = g - s->g0;
      const int64_t A = cs->A[g];
      const int32_t a = cs->accel[g];
      if (A < 0 || a < 0 || a >= NA) return -1;
      s->seg_cb[gl] = (int32_t)j;
      s->Astar[gl] = sat_add(scale(s, A), sat_mul(2, cs->accel_kappa[s->a0 + a]));
      s->uses[c * NA + a] = 1;
      s->Ahat[c * NA + a] = sat_add(s->Ahat[c * NA + a], s->Astar[gl]);
      s->epsce[c * X + e] = sat_add(s->epsce[c * X + e], cs->accel_eps[s->a0 + a]);
    }
  }

  /* buckets (Sec. IV-C): chains using accelerator a, by priority, split into
   * n evenly sized groups; rank r of m goes to level floor(r*n/m), 0 = top */
  for (int32_t a = 0; a < NA; ++a) {
    int32_t m = 0;
    for (int32_t c = 0; c < C; ++c) m += s->uses[c * NA + a];
    for (int32_t c = 0; c < C; ++c) {
      if (!s->uses[c * NA + a]) { s->level[c * NA + a] = -1; continue; }
      int32_t rank = 0;
      for (int32_t k = 0; k < C; ++k)
        if (s->uses[k * NA + a] && s->pi[k] > s->pi[c]) ++rank;
      s->level[c * NA + a] = (int32_t)(((int64_t)rank * cs->accel_buckets[s->a0 + a]) / m);
    }
  }

  /* Eq. (3) first max term: the largest A* of an LP segment on the same
   * accelerator in the same bucket (other buckets are preempted, R4) */
  for (int64_t g = 0; g < nseg; ++g) {
    const int32_t c = s->cb_chain[s->seg_cb[g]], a = cs->accel[s->g0 + g];
    int64_t b = 0;
    for (int64_t g2 = 0; g2 < nseg; ++g2) {
      const int32_t l = s->cb_chain[s->seg_cb[g2]];
      if (cs->accel[s->g0 + g2] != a || s->pi[l] >= s->pi[c]) continue;
      if (s->level[l * NA + a] != s->level[c * NA + a]) continue;
      b = max64(b, s->Astar[g2]);
    }
    s->Bacc[g] = b;
  }

  /* sub-chains: maximal runs of consecutive callbacks on one executor */
  s->run_chain = zalloc(sizeof(int32_t) * ncb);
  s->run_exec = zalloc(sizeof(int32_t) * ncb);
  s->run_cb_lo = zalloc(sizeof(int32_t) * ncb);
  s->run_cb_hi = zalloc(sizeof(int32_t) * ncb);
  s->run_E = zalloc(sizeof(int64_t) * ncb);
  s->run_L2 = zalloc(sizeof(int64_t) * ncb);
  s->run_A0 = zalloc(sizeof(int64_t) * ncb);
  s->run_eps = zalloc(sizeof(int64_t) * ncb);
  s->run_B = zalloc(sizeof(int64_t) * ncb);
  s->run_R = zalloc(sizeof(int64_t) * ncb);
  s->run_delta = zalloc(sizeof(int32_t) * ncb);
  s->run_acc = zalloc((size_t)ncb * (NA ? NA : 1));
  s->nrun = 0;
  for (int64_t j = 0; j < ncb; ++j) {
    const int32_t c = s->cb_chain[j], e = cs->exec[s->cb0 + j];
    const int newrun = j == 0 || s->cb_chain[j - 1] != c || cs->exec[s->cb0 + j - 1] != e;
    if (newrun) {
      s->run_chain[s->nrun] = c;
      s->run_exec[s->nrun] = e;
      s->run_cb_lo[s->nrun] = (int32_t)j;
      s->nsub[c]++;
      s->nrun++;
    }
    s->run_cb_hi[s->nrun - 1] = (int32_t)j + 1;
  }
  return 0;
}

/* per-run quantities that need the Lemma 2 values */
static void derive_runs(setctx *s) {
  const oracle_chainsets *cs = s->cs;
  for (int32_t r = 0; r < s->nrun; ++r) {
    const int32_t c = s->run_chain[r], e = s->run_exec[r];
    int64_t E = 0, L2 = 0, A0 = 0, eps = 0;
    int32_t delta = 0;
    for (int32_t j = s->run_cb_lo[r]; j < s->run_cb_hi[r]; ++j) {
      E = sat_add(E, s->Ecb[j]);
      for (int64_t g = cs->cb_seg_off[s->cb0 + j]; g < cs->cb_seg_off[s->cb0 + j + 1]; ++g) {
        const int64_t gl = g - s->g0;
        const int32_t a = cs->accel[g];
        L2 = sat_add(L2, s->H[gl]);
        A0 = sat_add(A0, sat_add(s->Astar[gl], s->Bacc[gl]));
        eps = sat_add(eps, cs->accel_eps[s->a0 + a]);
        s->run_acc[r * s->NA + a] = 1;
        delta++;
      }
    }
    s->run_E[r] = E;
    s->run_L2[r] = L2;
    s->run_A0[r] = A0;
    s->run_eps[r] = eps;
    s->run_delta[r] = delta;
    /* blocking by one callback of a lower priority chain on the executor
     * (Eq. 5 / Eq. 6 first term); with blocking == 0 the callback also holds
     * the executor while its accelerator requests are handled */
    int64_t B = 0;
    for (int64_t j = 0; j < s->ncb; ++j) {
      const int32_t l = s->cb_chain[j];
      if (cs->exec[s->cb0 + j] != e || s->pi[l] >= s->pi[c]) continue;
      int64_t b = s->Ecb[j];
      if (s->opt->blocking == 0) {
        for (int64_t g = cs->cb_seg_off[s->cb0 + j]; g < cs->cb_seg_off[s->cb0 + j + 1]; ++g)
          b = sat_add(b, sat_add(s->H[g - s->g0], cs->accel_eps[s->a0 + cs->accel[g]]));
      }
      B = max64(B, b);
    }
    s->run_B[r] = B;
  }
}

static int worse(int64_t Ra, int64_t Da, int64_t Rb, int64_t Db) { /* Ra/Da > Rb/Db */
  if (Ra == INF) return Rb != INF;
  if (Rb == INF) return 0;
  return (__int128)Ra * Db > (__int128)Rb * Da;
}

int oracle_analyse_set(const oracle_chainsets *cs, int64_t set, const int32_t *order,
                       const oracle_opts *opt, int64_t *chain_R, int8_t *sched, int32_t *worst,
                       int64_t *worst_R, int64_t *terms) {
  int64_t local_terms = 0;
  setctx s;
  if (ctx_init(&s, cs, set, order, opt, terms ? terms : &local_terms)) {
    ctx_free(&s);
    return -1;
  }
  if (terms) *terms = 0;
  const int32_t C = s.C, X = s.X;

  for (int64_t g = 0; g < s.nseg; ++g) s.H[g] = lemma2(&s, g);
  derive_runs(&s);

  /* chains and executors in dependency order */
  int32_t *ex_order = zalloc(sizeof(int32_t) * X);
  int32_t *ch_order = zalloc(sizeof(int32_t) * C);
  int64_t *partial = zalloc(sizeof(int64_t) * C);
  for (int32_t e = 0; e < X; ++e) ex_order[e] = e;
  for (int32_t i = 1; i < X; ++i) { /* by core, then process priority descending */
    int32_t x = ex_order[i], j = i - 1;
    while (j >= 0) {
      int32_t y = ex_order[j];
      int16_t cy = cs->exec_core[s.x0 + y], cx = cs->exec_core[s.x0 + x];
      if (cy < cx || (cy == cx && cs->exec_prio[s.x0 + y] > cs->exec_prio[s.x0 + x])) break;
      ex_order[j + 1] = y;
      --j;
    }
    ex_order[j + 1] = x;
  }
  for (int32_t c = 0; c < C; ++c) ch_order[c] = c;
  for (int32_t i = 1; i < C; ++i) { /* chain priority descending */
    int32_t x = ch_order[i], j = i - 1;
    while (j >= 0 && s.pi[ch_order[j]] < s.pi[x]) { ch_order[j + 1] = ch_order[j]; --j; }
    ch_order[j + 1] = x;
  }

  const int64_t hop = cs->eps_hop[set];
  int missed = 0;
  for (int32_t xi = 0; xi < X && !missed; ++xi) {
    const int32_t e = ex_order[xi];
    for (int32_t ci = 0; ci < C && !missed; ++ci) {
      const int32_t c = ch_order[ci];
      if (!s.on[c * X + e]) continue;
      int64_t hs = 0;
      for (int32_t r = 0; r < s.nrun; ++r) {
        if (s.run_chain[r] != c || s.run_exec[r] != e) continue;
        s.run_R[r] = solve_run(&s, r);
        hs = sat_add(hs, hstar(&s, r, s.run_R[r])); /* Eq. (1) at the sub-chain's bound */
        partial[c] = sat_add(partial[c], s.run_R[r]);
        if (!opt->full) {
          const int64_t lb = sat_add(partial[c], sat_mul(s.nsub[c] - 1, hop));
          if (s.run_R[r] == INF || lb > cs->D[s.c0 + c]) { missed = 1; break; }
        }
      }
      s.Hstar_ce[c * X + e] = hs;
    }
  }

  int ok = !missed;
  int32_t w = -1;
  int64_t wR = INF;
  if (!missed) {
    /* end of Sec. IV-F: sum of the sub-chain bounds plus one communication
     * cost per hop between consecutive sub-chains */
    for (int32_t c = 0; c < C; ++c) {
      int64_t R = sat_add(partial[c], sat_mul(s.nsub[c] - 1, hop));
      if (R > s.cap[c]) R = INF;
      chain_R[c] = R;
      if (R > cs->D[s.c0 + c]) ok = 0;
    }
    if (ok || opt->full) {
      for (int32_t c = 0; c < C; ++c)
        if (w < 0 || worse(chain_R[c], cs->D[s.c0 + c], chain_R[w], cs->D[s.c0 + w])) w = c;
      wR = chain_R[w];
    }
  } else {
    for (int32_t c = 0; c < C; ++c) chain_R[c] = -1;
  }
  *sched = (int8_t)ok;
  *worst = w;
  *worst_R = wR;
  free(ex_order);
  free(ch_order);
  free(partial);
  ctx_free(&s);
  return 0;
}

int oracle_segment_H(const oracle_chainsets *cs, int64_t set, const int32_t *order,
                     const oracle_opts *opt, int64_t *seg_H) {
  int64_t t = 0;
  setctx s;
  if (ctx_init(&s, cs, set, order, opt, &t)) {
    ctx_free(&s);
    return -1;
  }
  for (int64_t g = 0; g < s.nseg; ++g) seg_H[g] = lemma2(&s, g);
  ctx_free(&s);
  return 0;
}

int oracle_wcrt_range(const oracle_chainsets *cs, const oracle_opts *opt, int64_t lo, int64_t hi,
                      int64_t *chain_R, int8_t *sched, int32_t *worst, int64_t *worst_R,
                      int64_t *terms) {
  for (int64_t set = lo; set < hi; ++set) {
    int64_t t = 0;
    int rc = oracle_analyse_set(cs, set, NULL, opt, chain_R + cs->set_chain_off[set], &sched[set],
                                &worst[set], &worst_R[set], &t);
    if (rc) return rc;
    if (terms) terms[set] = t;
  }
  return 0;
}

/* ------------------------- candidate orders --------------------------- */
#define GAMMA 0x9E3779B97F4A7C15ULL
static uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
/* output m of the SplitMix64 stream of a set: its state starts at
 * out(seed + GAMMA*(set+1)) and advances by GAMMA per output */
static uint64_t swap_draw(uint64_t seed, int64_t set, uint64_t m) {
  uint64_t s0 = splitmix_out(seed + GAMMA * (uint64_t)(set + 1));
  return splitmix_out(s0 + GAMMA * (m + 1));
}
static void apply_swap(int32_t *order, int32_t C, uint64_t seed, int64_t set, int64_t k) {
  if (C < 2) return;
  uint64_t u1 = swap_draw(seed, set, 2 * (uint64_t)(k - 1));
  uint64_t u2 = swap_draw(seed, set, 2 * (uint64_t)(k - 1) + 1);
  int32_t i = (int32_t)(u1 % (uint64_t)C);
  int32_t j = (int32_t)((i + 1 + (int64_t)(u2 % (uint64_t)(C - 1))) % C);
  int32_t tmp = order[i];
  order[i] = order[j];
  order[j] = tmp;
}
static int base_order(const oracle_chainsets *cs, int64_t set, int32_t *order) {
  const int64_t c0 = cs->set_chain_off[set];
  const int32_t C = (int32_t)(cs->set_chain_off[set + 1] - c0);
  for (int32_t c = 0; c < C; ++c) order[c] = c;
  for (int32_t i = 1; i < C; ++i) {
    int32_t x = order[i], j = i - 1;
    while (j >= 0 && cs->prio[c0 + order[j]] < cs->prio[c0 + x]) { order[j + 1] = order[j]; --j; }
    order[j + 1] = x;
  }
  return C;
}

int oracle_candidate_order(const oracle_chainsets *cs, int64_t set, uint64_t seed, int64_t k,
                           int32_t *order) {
  if (set < 0 || set >= cs->n_sets || k < 0) return -1;
  int32_t C = base_order(cs, set, order);
  for (int64_t q = 1; q <= k; ++q) apply_swap(order, C, seed, set, q);
  return 0;
}

int oracle_search_range(const oracle_chainsets *cs, const oracle_opts *opt, int32_t n_cand,
                        uint64_t seed, int64_t lo, int64_t hi, int32_t *found, int32_t *n_eval,
                        int64_t *terms) {
  oracle_opts o = *opt;
  o.full = 0;
  for (int64_t set = lo; set < hi; ++set) {
    const int32_t C = (int32_t)(cs->set_chain_off[set + 1] - cs->set_chain_off[set]);
    int32_t *order = zalloc(sizeof(int32_t) * C);
    int64_t *R = zalloc(sizeof(int64_t) * C);
    base_order(cs, set, order);
    found[set] = -1;
    n_eval[set] = 0;
    int64_t tsum = 0;
    for (int32_t k = 0; k < n_cand; ++k) {
      if (k > 0) apply_swap(order, C, seed, set, k);
      int8_t sc;
      int32_t w;
      int64_t wr, t = 0;
      if (oracle_analyse_set(cs, set, order, &o, R, &sc, &w, &wr, &t)) {
        free(order);
        free(R);
        return -1;
      }
      tsum += t;
      n_eval[set]++;
      if (sc) { found[set] = k; break; }
    }
    if (terms) terms[set] = tsum;
    free(order);
    free(R);
  }
  return 0;
}

/* ---------------- units of one accelerator type (Sec. IV-E) ---------------
 * When a set has several units of an accelerator type, its segments are bound
 * to units at registration by a bin-packing heuristic, worst-fit decreasing
 * (the paper's "Managing Multiple Accelerators").  An item is one segment, or
 * all segments of one callback or of one chain on one type (group 0, 1, 2).
 * Item size: its utilisation sum(A)/T in fixed point,
 * floor(min(sum(A), 2^36) * 2^26 / T), clamped at 2^36.  Items are placed
 * largest first (equal sizes: the item of the higher-priority chain, then the
 * one whose first segment comes first); each goes to the unit of its type
 * with the smallest load so far (ties: the lowest unit), and its load grows
 * by the item's size. */
#define WFD_SHIFT 26
#define WFD_CLAMP ((int64_t)1 << 36)

typedef struct {
  int64_t sum_A;  /* saturated at WFD_CLAMP */
  int64_t size;
  int32_t prio;
  int64_t first;  /* lowest global segment index of the item */
  int32_t type;
  int64_t key;    /* callback or chain (global), or segment */
  int64_t unit;
} wfd_item;

static int wfd_cmp(const void *pa, const void *pb) {
  const wfd_item *a = pa, *b = pb;
  if (a->size != b->size) return a->size > b->size ? -1 : 1;
  if (a->prio != b->prio) return a->prio > b->prio ? -1 : 1;
  return a->first < b->first ? -1 : (a->first > b->first);
}

int oracle_wfd_range(const oracle_chainsets *cs, const int16_t *units, int32_t group, int64_t lo,
                     int64_t hi, int16_t *unit) {
  if (group < 0 || group > 2) return -1;
  for (int64_t set = lo; set < hi; ++set) {
    const int64_t c0 = cs->set_chain_off[set], c1 = cs->set_chain_off[set + 1];
    const int64_t a0 = cs->set_accel_off[set], a1 = cs->set_accel_off[set + 1];
    const int64_t NA = a1 - a0;
    int64_t base[64], n_units = 0;
    if (NA > 64) return -1;
    for (int64_t a = 0; a < NA; ++a) {
      if (units[a0 + a] < 1) return -1;
      base[a] = n_units;
      n_units += units[a0 + a];
    }
    const int64_t g0 = cs->cb_seg_off[cs->chain_cb_off[c0]];
    const int64_t g1 = cs->cb_seg_off[cs->chain_cb_off[c1]];
    wfd_item *it = zalloc(sizeof(wfd_item) * (size_t)(g1 - g0));
    int64_t *item_of = zalloc(sizeof(int64_t) * (size_t)(g1 - g0));
    int64_t *load = zalloc(sizeof(int64_t) * (size_t)n_units);
    int64_t n = 0;
    /* gather the items: a segment joins the item of its (key, type) */
    for (int64_t c = c0; c < c1; ++c)
      for (int64_t j = cs->chain_cb_off[c]; j < cs->chain_cb_off[c + 1]; ++j)
        for (int64_t g = cs->cb_seg_off[j]; g < cs->cb_seg_off[j + 1]; ++g) {
          const int a = cs->accel[g];
          if (a < 0 || a >= NA) { free(it); free(item_of); free(load); return -1; }
          const int64_t key = group == 0 ? g : group == 1 ? j : c;
          int64_t k = 0;
          while (k < n && !(it[k].key == key && it[k].type == a)) ++k;
          if (k == n) {
            it[n].sum_A = 0;
            it[n].prio = cs->prio[c];
            it[n].first = g;
            it[n].type = a;
            it[n].key = key;
            ++n;
          }
          it[k].sum_A += cs->A[g];
          if (it[k].sum_A > WFD_CLAMP) it[k].sum_A = WFD_CLAMP;
          item_of[g - g0] = k;
          it[k].size = 0;
        }
    /* sizes need T of the item's chain */
    for (int64_t c = c0; c < c1; ++c)
      for (int64_t j = cs->chain_cb_off[c]; j < cs->chain_cb_off[c + 1]; ++j)
        for (int64_t g = cs->cb_seg_off[j]; g < cs->cb_seg_off[j + 1]; ++g) {
          wfd_item *x = &it[item_of[g - g0]];
          const int64_t sz = (x->sum_A << WFD_SHIFT) / cs->T[c]; /* sum_A <= 2^36 */
          x->size = sz > WFD_CLAMP ? WFD_CLAMP : sz;
        }
    /* the sort permutes the items; remember each item's place by its first segment */
    qsort(it, (size_t)n, sizeof(wfd_item), wfd_cmp);
    for (int64_t i = 0; i < n; ++i) {
      const int a = it[i].type;
      int64_t best = base[a];
      for (int64_t u = base[a] + 1; u < base[a] + units[a0 + a]; ++u)
        if (load[u] < load[best]) best = u;
      load[best] += it[i].size;
      it[i].unit = best;
    }
    for (int64_t c = c0; c < c1; ++c)
      for (int64_t j = cs->chain_cb_off[c]; j < cs->chain_cb_off[c + 1]; ++j)
        for (int64_t g = cs->cb_seg_off[j]; g < cs->cb_seg_off[j + 1]; ++g) {
          const int64_t key = group == 0 ? g : group == 1 ? j : c;
          for (int64_t i = 0; i < n; ++i)
            if (it[i].key == key && it[i].type == cs->accel[g]) { unit[g] = (int16_t)it[i].unit; break; }
        }
    free(it);
    free(item_of);
    free(load);
  }
  return 0;
}
