"""Discrete-event simulator of chains under PAAM -- TEST INFRASTRUCTURE ONLY.

A brute-force behavioural model used to pin the analysis from the other side:
on tiny sets, every response time it observes must stay within the bound the
oracle computes (the paper's Case Study 1 checks the same property on real
hardware, Sec. V-A).  It shares nothing with the analysis code.

Model (paper Sec. II-C, IV-C, IV-D and rules R1-R4 of Sec. IV-F), in unit
time steps:
* A chain releases a job every T from its offset; the job runs its callbacks
  in order.  A callback is ready on its executor when its predecessor
  completes, plus the hop cost when the executor changes.
* An executor is single-threaded and non-preemptive: when idle it starts the
  ready callback of the highest chain priority and keeps it until it
  completes, including while its accelerator requests are served.
* A callback alternates CPU pieces and accelerator segments.  Before each
  request the client spends epsilon of CPU time (the per-request overhead);
  while a request is served a spinning chain keeps demanding its core, a
  suspending one does not.
* Cores run, at every instant, the demanding executor of the highest
  process priority (OS preemption).
* Each accelerator has n buckets (chains using it, ranked by priority, split
  into n groups).  Within a bucket requests run one at a time in chain
  priority order, non-preemptively; a request in a higher bucket preempts a
  lower bucket.  A segment occupies the device for its length plus 2 kappa.
"""
from __future__ import annotations

import heapq
import random


class _Req:
    __slots__ = ("job", "prio", "left", "seq")

    def __init__(self, job, prio, left, seq):
        self.job, self.prio, self.left, self.seq = job, prio, left, seq


class _Job:
    __slots__ = ("chain", "release", "cb", "items", "pos", "left", "exec", "done_at", "ready_at")

    def __init__(self, chain, release):
        self.chain, self.release = chain, release
        self.cb = 0
        self.items = None  # list of ("cpu", n) | ("eps", n) | ("seg", accel, n)
        self.pos = 0
        self.left = 0
        self.exec = None
        self.done_at = None
        self.ready_at = release


def _split(total, parts, rng):
    if parts == 1:
        return [total]
    if rng is None:
        base = [total // parts] * parts
        for i in range(total % parts):
            base[i] += 1
        return base
    cuts = sorted(rng.randint(0, total) for _ in range(parts - 1))
    return [b - a for a, b in zip([0] + cuts, cuts + [total])]


def bucket_levels(st):
    """Level of every (chain, accelerator) pair: users ranked by priority."""
    chains = st["chains"]
    n_acc = len(st.get("accel_buckets", [1]))
    lev = {}
    for a in range(n_acc):
        users = [i for i, ch in enumerate(chains)
                 if any(ai == a for cb in ch["cbs"] for _, ai in cb["segs"])]
        users.sort(key=lambda i: -chains[i]["prio"])
        n = st.get("accel_buckets", [1])[a]
        for r, i in enumerate(users):
            lev[(i, a)] = (r * n) // len(users)
    return lev


def simulate(st, offsets, horizon, rng=None, exec_frac=None):
    """Runs one scenario; returns the largest observed response per chain
    (None for chains with no completed job).

    offsets: first release per chain.  rng: None = every WCET in full with
    equal CPU splits; otherwise actual times uniform in [exec_frac*W, W] and
    random CPU splits around the segments."""
    chains = st["chains"]
    C = len(chains)
    X = len(st["exec_core"])
    eps = st.get("accel_eps", [0])
    kap = st.get("accel_kappa", [0])
    hop = st.get("eps_hop", 0)
    levels = bucket_levels(st)
    n_acc = len(st.get("accel_buckets", [1]))
    nb = st.get("accel_buckets", [1])

    def make_items(job):
        ch = chains[job.chain]
        cb = ch["cbs"][job.cb]
        E = cb["E"]
        segs = cb["segs"]
        if rng is not None and exec_frac is not None:
            E = rng.randint(int(E * exec_frac), E)
        pieces = _split(E, len(segs) + 1, rng)
        items = [("cpu", pieces[0])]
        for k, (A, a) in enumerate(segs):
            if rng is not None and exec_frac is not None:
                A = rng.randint(int(A * exec_frac), A)
            items.append(("eps", eps[a]))
            items.append(("seg", a, A + 2 * kap[a]))
            items.append(("cpu", pieces[k + 1]))
        return items

    ready = [[] for _ in range(X)]        # per executor: heap of (-prio, release, seq, job)
    running = [None] * X                  # job running on the executor
    waiting = [None] * X                  # True while its current item is a served request
    bucket_cur = [[None] * nb[a] for a in range(n_acc)]
    bucket_q = [[[] for _ in range(nb[a])] for a in range(n_acc)]
    pending_ready = []                    # heap of (time, seq, job)
    releases = [offsets[c] for c in range(C)]
    worst = [None] * C
    seq = [0]

    def nseq():
        seq[0] += 1
        return seq[0]

    def make_ready(job, t):
        job.exec = chains[job.chain]["cbs"][job.cb]["exec"]
        heapq.heappush(ready[job.exec], (-chains[job.chain]["prio"], job.release, nseq(), job))

    def callback_done(job, t):
        e = job.exec
        running[e] = None
        waiting[e] = None
        ch = chains[job.chain]
        if job.cb + 1 == len(ch["cbs"]):
            r = t - job.release
            if worst[job.chain] is None or r > worst[job.chain]:
                worst[job.chain] = r
            return
        nxt_exec = ch["cbs"][job.cb + 1]["exec"]
        job.cb += 1
        if nxt_exec != e and hop > 0:
            heapq.heappush(pending_ready, (t + hop, nseq(), job))
        else:
            make_ready(job, t)

    def advance_items(job, t):
        """Moves past finished items; submits requests.  True if something changed."""
        changed = False
        while True:
            if job.pos >= len(job.items):
                callback_done(job, t)
                return True
            it = job.items[job.pos]
            if it[0] in ("cpu", "eps"):
                if job.left is None:
                    job.left = it[1]
                if job.left > 0:
                    return changed
                job.pos += 1
                job.left = None
                changed = True
                continue
            # a segment: submit once, then wait for the server
            if job.left is None:
                a, n = it[1], it[2]
                lev = levels[(job.chain, a)]
                req = _Req(job, chains[job.chain]["prio"], n, nseq())
                heapq.heappush(bucket_q[a][lev], (-req.prio, req.seq, req))
                job.left = -1  # marks "submitted"
                waiting[job.exec] = True
                return True
            return changed

    t = 0
    while t <= horizon:
        # events at time t, until nothing changes
        changed = True
        while changed:
            changed = False
            for c in range(C):
                while releases[c] <= t and releases[c] <= horizon:
                    j = _Job(c, releases[c])
                    make_ready(j, t)
                    releases[c] += chains[c]["T"]
                    changed = True
            while pending_ready and pending_ready[0][0] <= t:
                _, _, j = heapq.heappop(pending_ready)
                make_ready(j, t)
                changed = True
            for e in range(X):
                if running[e] is None and ready[e]:
                    _, _, _, j = heapq.heappop(ready[e])
                    running[e] = j
                    j.items = make_items(j)
                    j.pos = 0
                    j.left = None
                    changed = True
                if running[e] is not None and not waiting[e]:
                    if advance_items(running[e], t):
                        changed = True
            for a in range(n_acc):
                # the device serves the highest bucket holding a request
                for lev in range(nb[a]):
                    if bucket_cur[a][lev] is None and bucket_q[a][lev]:
                        bucket_cur[a][lev] = heapq.heappop(bucket_q[a][lev])[2]
                    cur = bucket_cur[a][lev]
                    if cur is not None:
                        if cur.left == 0:
                            bucket_cur[a][lev] = None
                            job = cur.job
                            job.pos += 1
                            job.left = None
                            waiting[job.exec] = False
                            changed = True
                        break
        if t == horizon:
            break
        # one unit of execution
        for core in set(st["exec_core"]):
            best = None
            for e in range(X):
                if st["exec_core"][e] != core or running[e] is None:
                    continue
                j = running[e]
                demands = (not waiting[e] and j.left is not None and j.left > 0) or \
                          (waiting[e] and chains[j.chain].get("spin", 0))
                if demands and (best is None or st["exec_prio"][e] > st["exec_prio"][best]):
                    best = e
            if best is not None and not waiting[best]:
                running[best].left -= 1
        for a in range(n_acc):
            for lev in range(nb[a]):
                cur = bucket_cur[a][lev]
                if cur is not None:
                    cur.left -= 1
                    break
        t += 1
    return worst


def hyperperiod(st):
    from math import gcd
    h = 1
    for ch in st["chains"]:
        h = h * ch["T"] // gcd(h, ch["T"])
    return h


def observe(st, scenarios=20, seed=0, exec_frac=0.5):
    """Largest observed response per chain over the synchronous release, random
    offsets, and random execution times."""
    rng = random.Random(seed)
    C = len(st["chains"])
    H = hyperperiod(st)
    maxT = max(ch["T"] for ch in st["chains"])
    horizon = 2 * H + 2 * maxT
    best = [0] * C
    plans = [([0] * C, None)]
    for k in range(scenarios):
        offs = [rng.randrange(ch["T"]) for ch in st["chains"]]
        plans.append((offs, None))
        plans.append((offs, random.Random(rng.random())))
    for offs, r in plans:
        w = simulate(st, offs, horizon + max(offs), rng=r, exec_frac=exec_frac if r else None)
        for c in range(C):
            if w[c] is not None:
                best[c] = max(best[c], w[c])
    return best
