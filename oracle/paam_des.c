/*
 * Event-driven simulation of chain sets under PAAM -- TEST INFRASTRUCTURE ONLY.
 *
 * The model is the one the analysis of Sec. IV-F bounds (Sec. II-C chains and
 * single-threaded executors, Sec. IV-C buckets, Sec. IV-D per-request overhead
 * and preemption cost, rules R1-R4 of Sec. IV-F):
 *  - chain c releases a job every T_c from its offset; a job runs the chain's
 *    callbacks in order; the next callback becomes ready on its executor when
 *    the previous one completes, after the hop cost when the executor changes;
 *  - an executor is non-preemptive: when idle it starts its ready callback of
 *    the highest chain priority (then the earliest release) and keeps it to
 *    the end, also while the callback's accelerator requests are served;
 *  - a callback is a CPU piece, then per segment: epsilon of CPU time, the
 *    request (A + 2 kappa on the device), a CPU piece; the CPU time E is split
 *    equally over the pieces (the first E mod (eta+1) pieces one longer);
 *  - a core runs, at every instant, its demanding executor of the highest
 *    process priority; an executor demands while it has CPU work, or while
 *    its request is served if its chain busy-waits;
 *  - an accelerator serves the highest bucket level holding a request; within
 *    a level requests run one at a time, highest chain priority first (then
 *    submission order), and a higher level preempts a lower one.
 * Instants are processed in a fixed order until nothing changes: releases,
 * hop arrivals, executors by index (start a callback, then move it past
 * finished pieces or submit its request), accelerators by index (the
 * highest occupied level: start its next request, or finish the served one).
 * Between instants time jumps to the next event.  A chain keeps at most two
 * live jobs; a release that would need a third ends the scenario (status 1),
 * and so does passing max_steps time advances (status 2).
 *
 * Actual execution times: with exec_permille = 1000 every job runs its WCET;
 * otherwise every CPU WCET E of a callback job and every segment WCET A is
 * replaced by a draw from [floor(W * exec_permille / 1000), W], taken from
 * SplitMix64 (Steele, Lea and Flood, 2014) keyed by (seed, set, scenario,
 * chain, job, callback, item), as W - (draw mod (W - lo + 1)).
 */
#include "paam_oracle.h"

#include <stdlib.h>
#include <string.h>

#define DES_J 2 /* live jobs per chain */

enum { J_FREE = 0, J_READY, J_HOP, J_RUN };

typedef struct {
  int state;
  int64_t release, jobidx, ready_at;
  int64_t cb;          /* global callback index */
  int pos;             /* item index */
  int64_t left;        /* remaining time of the current item; -1: not started; -2: request submitted */
  int exec;
  /* request */
  int queued, req_a, req_lev;
  int64_t req_left, req_seq;
} des_job;

#define DES_G 0x9E3779B97F4A7C15ULL
static uint64_t des_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct {
  const oracle_chainsets *cs;
  const oracle_des_opts *o;
  int64_t set, scen, c0, x0, a0;
  int C, X, NA;
  int lev[4096];      /* [chain * 8 + accel] bucket level */
} des_ctx;

static int64_t des_scale(const des_ctx *d, int64_t x) {
  return x * d->o->util_permille / 1000;
}

static int64_t des_actual(const des_ctx *d, int chain, int64_t job, int64_t cbl, int item,
                          int64_t W) {
  if (d->o->exec_permille >= 1000) return W;
  const int64_t lo = W * d->o->exec_permille / 1000;
  if (W <= lo) return W;
  uint64_t k = d->o->seed;
  k = des_mix(k + DES_G * (uint64_t)(d->set + 1));
  k = des_mix(k + DES_G * (uint64_t)(d->scen + 1));
  k = des_mix(k + DES_G * (uint64_t)(chain + 1));
  k = des_mix(k + DES_G * (uint64_t)(job + 1));
  k = des_mix(k + DES_G * (uint64_t)(cbl * 64 + item + 1));
  return W - (int64_t)(k % (uint64_t)(W - lo + 1));
}

/* length of item pos of the running callback of job j (chain c) */
static int64_t des_item_len(const des_ctx *d, const des_job *j, int c, int pos, int *is_seg,
                            int *seg_a) {
  const oracle_chainsets *cs = d->cs;
  const int64_t cb = j->cb;
  const int64_t g0 = cs->cb_seg_off[cb];
  const int eta = (int)(cs->cb_seg_off[cb + 1] - g0);
  const int64_t cbl = cb - cs->chain_cb_off[d->c0 + c];
  *is_seg = 0;
  if (pos % 3 == 0) { /* CPU piece pos/3 of eta+1 */
    const int64_t E = des_actual(d, c, j->jobidx, cbl, 63, des_scale(d, cs->E[cb]));
    const int p = pos / 3, parts = eta + 1;
    return E / parts + (p < E % parts ? 1 : 0);
  }
  const int k = (pos - 1) / 3;
  const int a = cs->accel[g0 + k];
  if (pos % 3 == 1) return cs->accel_eps[d->a0 + a];
  *is_seg = 1;
  *seg_a = a;
  return des_actual(d, c, j->jobidx, cbl, k, des_scale(d, cs->A[g0 + k])) +
         2 * cs->accel_kappa[d->a0 + a];
}

static void bucket_levels(des_ctx *d) {
  const oracle_chainsets *cs = d->cs;
  for (int a = 0; a < d->NA; ++a) {
    int users[4096], m = 0;
    for (int c = 0; c < d->C; ++c) {
      int uses = 0;
      for (int64_t jb = cs->chain_cb_off[d->c0 + c]; jb < cs->chain_cb_off[d->c0 + c + 1]; ++jb)
        for (int64_t g = cs->cb_seg_off[jb]; g < cs->cb_seg_off[jb + 1]; ++g)
          if (cs->accel[g] == a) uses = 1;
      if (uses) users[m++] = c;
    }
    /* rank users by decreasing priority */
    for (int i = 1; i < m; ++i) {
      int x = users[i], k = i - 1;
      while (k >= 0 && cs->prio[d->c0 + users[k]] < cs->prio[d->c0 + x]) { users[k + 1] = users[k]; --k; }
      users[k + 1] = x;
    }
    const int n = cs->accel_buckets[d->a0 + a];
    for (int r = 0; r < m; ++r) d->lev[users[r] * 8 + a] = (int)((int64_t)r * n / m);
  }
}

static int des_scenario(des_ctx *d, const int64_t *offs, int64_t *worst) {
  const oracle_chainsets *cs = d->cs;
  const oracle_des_opts *o = d->o;
  const int C = d->C, X = d->X, NA = d->NA;
  const int64_t hop = cs->eps_hop[d->set];
  des_job *jobs = calloc((size_t)C * DES_J, sizeof(des_job));
  int64_t *rel = calloc((size_t)C, sizeof(int64_t));
  int64_t *njob = calloc((size_t)C, sizeof(int64_t));
  int *running = malloc(sizeof(int) * (size_t)X);
  int *waiting = calloc((size_t)X, sizeof(int));
  int cur[8][8];
  int64_t seq = 0, steps = 0, t = 0;
  int status = 0;
  for (int e = 0; e < X; ++e) running[e] = -1;
  for (int a = 0; a < 8; ++a)
    for (int l = 0; l < 8; ++l) cur[a][l] = -1;
  for (int c = 0; c < C; ++c) {
    rel[c] = offs[c];
    worst[c] = -1;
  }
#define CHAIN_OF(i) ((i) / DES_J)
#define LAST_CB(c) (cs->chain_cb_off[d->c0 + (c) + 1] - 1)
  for (;;) {
    int changed = 1;
    while (changed) {
      changed = 0;
      /* releases */
      for (int c = 0; c < C; ++c)
        while (rel[c] <= t && rel[c] <= o->horizon) {
          const int64_t k = njob[c]++;
          des_job *j = &jobs[c * DES_J + (int)(k % DES_J)];
          if (j->state != J_FREE) { status = 1; goto done; }
          memset(j, 0, sizeof(*j));
          j->release = rel[c];
          j->jobidx = k;
          j->cb = cs->chain_cb_off[d->c0 + c];
          j->state = J_READY;
          j->exec = cs->exec[j->cb];
          rel[c] += cs->T[d->c0 + c];
          changed = 1;
        }
      /* hop arrivals */
      for (int i = 0; i < C * DES_J; ++i)
        if (jobs[i].state == J_HOP && jobs[i].ready_at <= t) {
          jobs[i].state = J_READY;
          jobs[i].exec = cs->exec[jobs[i].cb];
          changed = 1;
        }
      /* executors */
      for (int e = 0; e < X; ++e) {
        if (running[e] < 0) {
          int best = -1;
          for (int i = 0; i < C * DES_J; ++i) {
            if (jobs[i].state != J_READY || jobs[i].exec != e) continue;
            if (best < 0) { best = i; continue; }
            const int32_t pi = cs->prio[d->c0 + CHAIN_OF(i)], pb = cs->prio[d->c0 + CHAIN_OF(best)];
            if (pi > pb || (pi == pb && jobs[i].release < jobs[best].release)) best = i;
          }
          if (best >= 0) {
            running[e] = best;
            jobs[best].state = J_RUN;
            jobs[best].pos = 0;
            jobs[best].left = -1;
            changed = 1;
          }
        }
        if (running[e] >= 0 && !waiting[e]) {
          des_job *j = &jobs[running[e]];
          const int c = CHAIN_OF(running[e]);
          const int n_items = 1 + 3 * (int)(cs->cb_seg_off[j->cb + 1] - cs->cb_seg_off[j->cb]);
          for (;;) {
            if (j->pos >= n_items) { /* callback done */
              running[e] = -1;
              waiting[e] = 0;
              if (j->cb == LAST_CB(c)) {
                const int64_t r = t - j->release;
                if (r > worst[c]) worst[c] = r;
                j->state = J_FREE;
              } else {
                j->cb += 1;
                const int nx = cs->exec[j->cb];
                if (nx != e && hop > 0) {
                  j->state = J_HOP;
                  j->ready_at = t + hop;
                } else {
                  j->state = J_READY;
                  j->exec = nx;
                }
              }
              changed = 1;
              break;
            }
            int is_seg = 0, a = 0;
            const int64_t len = des_item_len(d, j, c, j->pos, &is_seg, &a);
            if (!is_seg) {
              if (j->left == -1) j->left = len;
              if (j->left > 0) break;
              j->pos += 1;
              j->left = -1;
              changed = 1;
              continue;
            }
            if (j->left == -1) { /* submit the request */
              j->queued = 1;
              j->req_a = a;
              j->req_lev = d->lev[c * 8 + a];
              j->req_left = len;
              j->req_seq = seq++;
              j->left = -2;
              waiting[e] = 1;
              changed = 1;
            }
            break;
          }
        }
      }
      /* accelerators */
      for (int a = 0; a < NA; ++a) {
        const int nb = cs->accel_buckets[d->a0 + a];
        for (int l = 0; l < nb; ++l) {
          if (cur[a][l] < 0) {
            int best = -1;
            for (int i = 0; i < C * DES_J; ++i) {
              if (!jobs[i].queued || jobs[i].req_a != a || jobs[i].req_lev != l) continue;
              if (best < 0) { best = i; continue; }
              const int32_t pi = cs->prio[d->c0 + CHAIN_OF(i)], pb = cs->prio[d->c0 + CHAIN_OF(best)];
              if (pi > pb || (pi == pb && jobs[i].req_seq < jobs[best].req_seq)) best = i;
            }
            if (best >= 0) {
              cur[a][l] = best;
              jobs[best].queued = 0;
            }
          }
          if (cur[a][l] >= 0) {
            des_job *j = &jobs[cur[a][l]];
            if (j->req_left == 0) {
              cur[a][l] = -1;
              j->pos += 1;
              j->left = -1;
              waiting[j->exec] = 0;
              changed = 1;
            }
            break;
          }
        }
      }
    }
    if (t >= o->horizon) break;
    if (++steps > o->max_steps) { status = 2; break; }
    /* next event */
    int64_t next = o->horizon;
    for (int c = 0; c < C; ++c)
      if (rel[c] < next) next = rel[c];
    for (int i = 0; i < C * DES_J; ++i)
      if (jobs[i].state == J_HOP && jobs[i].ready_at < next) next = jobs[i].ready_at;
    int runs[64];
    for (int e = 0; e < X; ++e) {
      runs[e] = 0;
      if (running[e] < 0 || waiting[e]) continue;
      int beaten = 0;
      for (int f = 0; f < X; ++f) {
        if (f == e || running[f] < 0) continue;
        if (cs->exec_core[d->x0 + f] != cs->exec_core[d->x0 + e]) continue;
        if (cs->exec_prio[d->x0 + f] <= cs->exec_prio[d->x0 + e]) continue;
        const int demands = !waiting[f] || cs->spin[d->c0 + CHAIN_OF(running[f])];
        if (demands) beaten = 1;
      }
      if (!beaten) {
        runs[e] = 1;
        if (t + jobs[running[e]].left < next) next = t + jobs[running[e]].left;
      }
    }
    int served[8];
    for (int a = 0; a < NA; ++a) {
      served[a] = -1;
      for (int l = 0; l < cs->accel_buckets[d->a0 + a]; ++l)
        if (cur[a][l] >= 0) { served[a] = cur[a][l]; break; }
      if (served[a] >= 0 && t + jobs[served[a]].req_left < next) next = t + jobs[served[a]].req_left;
    }
    const int64_t dt = next - t;
    for (int e = 0; e < X; ++e)
      if (runs[e]) jobs[running[e]].left -= dt;
    for (int a = 0; a < NA; ++a)
      if (served[a] >= 0) jobs[served[a]].req_left -= dt;
    t = next;
  }
done:
  free(jobs);
  free(rel);
  free(njob);
  free(running);
  free(waiting);
  return status;
#undef CHAIN_OF
#undef LAST_CB
}

int oracle_des_range(const oracle_chainsets *cs, const oracle_des_opts *o, const int64_t *offsets,
                     int64_t lo, int64_t hi, int64_t *obs, int8_t *status) {
  if (o->n_scen < 1 || o->horizon < 0) return -1;
  des_ctx *d = malloc(sizeof(des_ctx));
  for (int64_t set = lo; set < hi; ++set) {
    d->cs = cs;
    d->o = o;
    d->set = set;
    d->c0 = cs->set_chain_off[set];
    d->x0 = cs->set_exec_off[set];
    d->a0 = cs->set_accel_off[set];
    d->C = (int)(cs->set_chain_off[set + 1] - d->c0);
    d->X = (int)(cs->set_exec_off[set + 1] - d->x0);
    d->NA = (int)(cs->set_accel_off[set + 1] - d->a0);
    if (d->C > 512 || d->X > 64 || d->NA > 8) { free(d); return -1; }
    for (int a = 0; a < d->NA; ++a)
      if (cs->accel_buckets[d->a0 + a] > 8) { free(d); return -1; }
    bucket_levels(d);
    for (int64_t s = 0; s < o->n_scen; ++s) {
      d->scen = s;
      const int64_t base = d->c0 * o->n_scen + s * d->C;
      status[set * o->n_scen + s] = (int8_t)des_scenario(d, offsets + base, obs + base);
    }
  }
  free(d);
  return 0;
}
