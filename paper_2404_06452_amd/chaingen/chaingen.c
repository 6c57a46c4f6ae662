/*
 * Seeded synthetic chain-set generator.
 *
 * Produces the inputs of the response-time analysis (the callback tuple and
 * the chain tuple of the paper's system model, Sec. II-C) for many independent
 * chain sets, in CSR form.  It holds none of the analysis arithmetic: only
 * random draws, UUniFast [Bini & Buttazzo 2005], log-uniform periods,
 * rate-monotonic priorities and the WCET split into CPU and accelerator parts.
 *
 * Every set draws from its own two counter-based SplitMix64 streams
 * [Steele, Lea & Flood 2014] keyed by (seed, set id): stream 0 decides the
 * structure (chain count, callbacks per chain, which callbacks carry
 * segments), stream 1 the values.  So any subset of sets regenerates
 * bit-identically without the others, and the count pass needs stream 0 only.
 *
 * Built with plain gcc (no fast-math) so that the floating-point steps are
 * deterministic; every time leaves as int64 nanoseconds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint64_t seed;
  int64_t set_begin;   /* first set id generated */
  int64_t n_sets;      /* number of sets */
  int32_t chains_lo, chains_hi;   /* chains per set, uniform integer */
  int32_t cbs_lo, cbs_hi;         /* callbacks per chain, uniform integer */
  int32_t n_exec;                 /* executors per set */
  int32_t n_accel;                /* accelerators per set */
  int32_t max_seg_per_cb;         /* segments of a segment-carrying callback: U{1..max} */
  int32_t n_buckets;              /* buckets of every accelerator */
  double util_lo, util_hi;        /* total utilisation per set, uniform */
  double pseg_lo, pseg_hi;        /* P(callback carries segments), drawn once per set */
  double frac_lo, frac_hi;        /* accelerator share of a callback's WCET, uniform */
  double T_lo, T_hi;              /* period range in ns, log-uniform */
  double spin_prob;               /* P(chain busy-waits during its accelerator requests) */
  int64_t eps, kappa, eps_hop;    /* per-request overhead, preemption cost, hop cost (ns) */
  int32_t exec_per_chain;         /* 1: every callback of chain c on executor c mod n_exec */
  int32_t own_cores;              /* 1: every executor alone on its core (else pairs share one) */
} chaingen_params;

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct { uint64_t state; } rng_t;

static inline rng_t rng_open(uint64_t seed, int64_t set_id, int stream) {
  rng_t r;
  uint64_t k = mix64(seed + GAMMA) ^ mix64(((uint64_t)set_id << 1 | (uint64_t)stream) + 0xD1B54A32D192ED03ULL);
  r.state = mix64(k);
  return r;
}
static inline uint64_t rng_u64(rng_t *r) { r->state += GAMMA; return mix64(r->state); }
static inline double rng_unit(rng_t *r) { return (double)(rng_u64(r) >> 11) * 0x1.0p-53; }
static inline double rng_uniform(rng_t *r, double lo, double hi) {
  return lo == hi ? lo : lo + (hi - lo) * rng_unit(r);
}
static inline int32_t rng_int(rng_t *r, int32_t lo, int32_t hi) { /* inclusive */
  if (hi <= lo) return lo;
  return lo + (int32_t)(rng_u64(r) % (uint64_t)(hi - lo + 1));
}

/* ---- structure stream: identical draws in the count and the fill pass ---- */
typedef struct { int32_t C; double pseg; } set_shape;

static set_shape draw_shape(const chaingen_params *p, rng_t *s) {
  set_shape sh;
  sh.C = rng_int(s, p->chains_lo, p->chains_hi);
  sh.pseg = rng_uniform(s, p->pseg_lo, p->pseg_hi);
  return sh;
}
/* callbacks of one chain, then per callback its segment count */
static int32_t draw_ncb(const chaingen_params *p, rng_t *s) { return rng_int(s, p->cbs_lo, p->cbs_hi); }
static int32_t draw_nseg(const chaingen_params *p, rng_t *s, double pseg) {
  double u = rng_unit(s);
  int32_t eta = rng_int(s, 1, p->max_seg_per_cb > 1 ? p->max_seg_per_cb : 1);
  return u < pseg ? eta : 0;
}

static int check_params(const chaingen_params *p) {
  if (p->n_sets < 0 || p->chains_lo < 1 || p->chains_hi < p->chains_lo || p->cbs_lo < 1 ||
      p->cbs_hi < p->cbs_lo || p->n_exec < 1 || p->n_exec > 32767 || p->n_accel < 1 ||
      p->n_accel > 32767 || p->n_buckets < 1 || p->max_seg_per_cb < 1 || !(p->T_lo > 0) ||
      p->T_hi < p->T_lo || p->util_lo < 0 || p->util_hi < p->util_lo || p->eps < 0 ||
      p->kappa < 0 || p->eps_hop < 0)
    return -1;
  return 0;
}

/* counts[3*i + {0,1,2}] = chains, callbacks, segments of set set_begin+i */
int chaingen_count(const chaingen_params *p, int64_t *counts) {
  if (check_params(p)) return -1;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < p->n_sets; ++i) {
    rng_t s = rng_open(p->seed, p->set_begin + i, 0);
    set_shape sh = draw_shape(p, &s);
    int64_t ncb = 0, nseg = 0;
    for (int32_t c = 0; c < sh.C; ++c) {
      int32_t n = draw_ncb(p, &s);
      ncb += n;
      for (int32_t j = 0; j < n; ++j) nseg += draw_nseg(p, &s, sh.pseg);
    }
    counts[3 * i] = sh.C;
    counts[3 * i + 1] = ncb;
    counts[3 * i + 2] = nseg;
  }
  return 0;
}

typedef struct {
  /* global offsets of every set, computed by the caller from chaingen_count */
  const int64_t *set_chain_off, *set_cb_off, *set_seg_off;   /* [n_sets+1] */
  /* outputs */
  int64_t *chain_cb_off;  /* [n_chains+1], global callback index */
  int64_t *cb_seg_off;    /* [n_callbacks+1], global segment index */
  int64_t *T, *D;         /* [n_chains] */
  int32_t *prio;          /* [n_chains], unique per set, larger = higher */
  uint8_t *spin;          /* [n_chains] */
  int64_t *E;             /* [n_callbacks] */
  int16_t *exec;          /* [n_callbacks], set-local executor */
  int64_t *A;             /* [n_segments] */
  int16_t *accel;         /* [n_segments], set-local accelerator */
  int16_t *exec_core;     /* [n_sets*n_exec] */
  int32_t *exec_prio;     /* [n_sets*n_exec] */
  int16_t *accel_buckets; /* [n_sets*n_accel] */
  int64_t *accel_eps, *accel_kappa;  /* [n_sets*n_accel] */
  int64_t *eps_hop;       /* [n_sets] */
} chaingen_out;

int chaingen_fill(const chaingen_params *p, const chaingen_out *o) {
  if (check_params(p)) return -1;
  int bad = 0;
#pragma omp parallel
  {
    int32_t cap = 0;
    int32_t *ncb = NULL, *order = NULL;
    double *ut = NULL;
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < p->n_sets; ++i) {
      rng_t s = rng_open(p->seed, p->set_begin + i, 0);
      rng_t v = rng_open(p->seed, p->set_begin + i, 1);
      set_shape sh = draw_shape(p, &s);
      const int32_t C = sh.C;
      if (C > cap) {
        cap = C;
        ncb = (int32_t *)realloc(ncb, sizeof(int32_t) * cap);
        order = (int32_t *)realloc(order, sizeof(int32_t) * cap);
        ut = (double *)realloc(ut, sizeof(double) * cap);
      }
      const int64_t c0 = o->set_chain_off[i], cb0 = o->set_cb_off[i], sg0 = o->set_seg_off[i];
      if (o->set_chain_off[i + 1] - c0 != C) { bad = 1; continue; }

      /* total utilisation and its UUniFast split over the chains */
      double U = rng_uniform(&v, p->util_lo, p->util_hi);
      double rest = U;
      for (int32_t c = 0; c < C - 1; ++c) {
        double next = rest * pow(rng_unit(&v), 1.0 / (double)(C - 1 - c));
        ut[c] = rest - next;
        rest = next;
      }
      ut[C - 1] = rest;

      /* periods (log-uniform), implicit deadlines, spin/suspend */
      const double lnlo = log(p->T_lo), lnhi = log(p->T_hi);
      for (int32_t c = 0; c < C; ++c) {
        int64_t T = (int64_t)llround(exp(rng_uniform(&v, lnlo, lnhi)));
        if (T < 1) T = 1;
        o->T[c0 + c] = T;
        o->D[c0 + c] = T;
        o->spin[c0 + c] = rng_unit(&v) < p->spin_prob ? 1 : 0;
      }

      /* callbacks and their segments */
      int64_t cb = cb0, sg = sg0;
      for (int32_t c = 0; c < C; ++c) {
        const int32_t n = draw_ncb(p, &s);
        o->chain_cb_off[c0 + c] = cb;
        const double W_real = ut[c] * (double)o->T[c0 + c] / (double)n;
        for (int32_t j = 0; j < n; ++j, ++cb) {
          int64_t W = (int64_t)llround(W_real);
          if (W < 1) W = 1;
          const int32_t eta = draw_nseg(p, &s, sh.pseg);
          const int32_t ex = (int32_t)rng_int(&v, 0, p->n_exec - 1);
          o->exec[cb] = (int16_t)(p->exec_per_chain ? c % p->n_exec : ex);
          o->cb_seg_off[cb] = sg;
          int64_t Atot = 0;
          if (eta > 0) {
            const double f = rng_uniform(&v, p->frac_lo, p->frac_hi);
            Atot = (int64_t)llround(f * (double)W);
            if (Atot > W) Atot = W;
            /* equal split of the accelerator time over the callback's segments */
            for (int32_t q = 0; q < eta; ++q, ++sg) {
              o->A[sg] = Atot / eta + (q < Atot % eta ? 1 : 0);
              o->accel[sg] = (int16_t)rng_int(&v, 0, p->n_accel - 1);
            }
          }
          o->E[cb] = W - Atot;
        }
      }
      if (cb != o->set_cb_off[i + 1] || sg != o->set_seg_off[i + 1]) { bad = 1; continue; }
      if (i == p->n_sets - 1) {
        o->chain_cb_off[c0 + C] = cb;
        o->cb_seg_off[cb] = sg;
      }

      /* rate-monotonic priorities: shorter period = higher; ties to the lower index */
      for (int32_t c = 0; c < C; ++c) order[c] = c;
      for (int32_t a = 1; a < C; ++a) { /* stable insertion sort by T */
        int32_t x = order[a];
        int32_t b = a - 1;
        while (b >= 0 && o->T[c0 + order[b]] > o->T[c0 + x]) { order[b + 1] = order[b]; --b; }
        order[b + 1] = x;
      }
      for (int32_t r = 0; r < C; ++r) o->prio[c0 + order[r]] = C - r;

      /* executors: pairs share a core (or each has its own); process priority
         decreases with the index */
      for (int32_t e = 0; e < p->n_exec; ++e) {
        o->exec_core[i * p->n_exec + e] = (int16_t)(p->own_cores ? e : e / 2);
        o->exec_prio[i * p->n_exec + e] = p->n_exec - e;
      }
      for (int32_t a = 0; a < p->n_accel; ++a) {
        o->accel_buckets[i * p->n_accel + a] = (int16_t)p->n_buckets;
        o->accel_eps[i * p->n_accel + a] = p->eps;
        o->accel_kappa[i * p->n_accel + a] = p->kappa;
      }
      o->eps_hop[i] = p->eps_hop;
    }
    free(ncb);
    free(order);
    free(ut);
  }
  return bad ? -2 : 0;
}
