"""Per-chain features of a candidate priority order -- TEST INFRASTRUCTURE ONLY.

Plain-Python reference of the surrogate's input: 48 numbers per chain that
summarise, for one chain set under one priority order, the quantities the
response-time analysis of Sec. IV-F is built from (own demand, interference
of higher-priority chains on the same executor, blocking by one lower-priority
callback, OS-level preemption by higher process-priority executors on the same
core, accelerator interference and same-bucket blocking of Eq. (3) under the
bucket split of Sec. IV-C).  The features are not part of the paper's method:
they feed the learned ranking of candidate orders that sits on top of it.

Arithmetic (fixed so that any implementation reproduces every bit): each
feature is a ratio N / M of exact integers (or a fixed sum of two such
ratios), evaluated as (double)N / (double)M with both integers converted by
round-to-nearest-even and the quotient correctly rounded, then rounded to
float32 and from there to bfloat16, both round-to-nearest-even.  Utilisation
terms are fixed-point integers q = floor(x * 2^16 / T).  Times are scaled by
util_permille exactly as the analysis scales them (floor(x * u / 1000) for E
and A; kappa and epsilon are not scaled), and A* = A + 2 kappa (Sec. IV-D).

Every sum here is a literal loop over its definition: O(C^2 X) per order,
which is fine for the small cases the tests use.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 48
Q = 1 << 16          # fixed-point scale of utilisation terms
TOT_LIMIT = 1 << 40  # every set's total scaled demand must stay below this

NAMES = (
    "own_E", "own_Astar", "own_eps", "own_hop", "own_demand", "own_Emax", "runs", "segs",
    "callbacks", "exec_share", "D_over_T", "T_s", "spin", "own_util_cpu", "own_util_acc",
    "rank", "rank_rev", "is_top", "is_bottom", "hp_longer", "lp_shorter",
    "hp_util_cpu", "hp_util_acc", "hp_carry", "hp_util_max", "hp_sharing",
    "blk_paper", "blk_safe", "blk_max", "lp_sharing",
    "hpp_carry", "hpp_util",
    "acc_carry", "acc_util", "acc_bacc", "acc_level", "acc_sharing", "acc_hp_flag",
    "set_util", "set_util_max", "set_util_acc", "set_C", "set_X", "set_NA", "set_Tmin",
    "est_floor", "est_util", "demand_share",
)
assert len(NAMES) == N_FEAT


def ratio(n: int, m: int) -> float:
    """(double)n / (double)m, 0 when m == 0."""
    if m == 0:
        return 0.0
    return float(n) / float(m)


def _runs(cbs):
    """Maximal runs of consecutive callbacks on one executor: (exec, [cb ids])."""
    runs = []
    for j, cb in enumerate(cbs):
        if runs and runs[-1][0] == cb["exec"]:
            runs[-1][1].append(j)
        else:
            runs.append((cb["exec"], [j]))
    return runs


def chain_features(st: dict, order, util_permille: int = 1000) -> np.ndarray:
    """float64 [C, 48]: row c holds the features of chain c (set-local index)
    when the chains have the priorities of ``order`` (chain ids, highest
    priority first).  ``st`` is a set in the ``set_dict`` format."""
    chains = st["chains"]
    C = len(chains)
    X = len(st["exec_core"])
    NA = len(st["accel_buckets"])
    u = int(util_permille)
    kap = st["accel_kappa"]
    eps = st["accel_eps"]
    hop = int(st["eps_hop"])
    rank = [0] * C
    for r, c in enumerate(order):
        rank[int(c)] = r
    assert sorted(rank) == list(range(C))

    def sE(x):
        return (int(x) * u) // 1000

    def sAs(a, acc):
        return (int(a) * u) // 1000 + 2 * int(kap[acc])

    # per chain, per (chain, executor) and per (chain, accelerator) totals
    E_c = [0] * C; Ac_c = [0] * C; ep_c = [0] * C; S_c = [0] * C; dl_c = [0] * C
    n_c = [0] * C; Emax_c = [0] * C
    Ece = [[0] * X for _ in range(C)]; Acce = [[0] * X for _ in range(C)]
    epce = [[0] * X for _ in range(C)]; runsce = [[0] * X for _ in range(C)]
    blce = [[0] * X for _ in range(C)]; bSce = [[0] * X for _ in range(C)]
    Ahat = [[0] * max(NA, 1) for _ in range(C)]; dca = [[0] * max(NA, 1) for _ in range(C)]
    Amax = [[0] * max(NA, 1) for _ in range(C)]
    seg_list = [[] for _ in range(C)]  # (accel, A*) of every segment of the chain
    for c, ch in enumerate(chains):
        cbs = ch["cbs"]
        n_c[c] = len(cbs)
        for e, ids in _runs(cbs):
            S_c[c] += 1
            runsce[c][e] += 1
        for cb in cbs:
            e = cb["exec"]
            Ej = sE(cb["E"])
            E_c[c] += Ej
            Ece[c][e] += Ej
            Emax_c[c] = max(Emax_c[c], Ej)
            blce[c][e] = max(blce[c][e], Ej)
            bj = Ej
            for (a, acc) in cb["segs"]:
                As = sAs(a, acc)
                Ac_c[c] += As
                ep_c[c] += int(eps[acc])
                dl_c[c] += 1
                Acce[c][e] += As
                epce[c][e] += int(eps[acc])
                Ahat[c][acc] += As
                dca[c][acc] += 1
                Amax[c][acc] = max(Amax[c][acc], As)
                seg_list[c].append((acc, As))
                bj += As + int(eps[acc])
            bSce[c][e] = max(bSce[c][e], bj)
    T = [int(ch["T"]) for ch in chains]
    D = [int(ch["D"]) for ch in chains]
    spin = [int(ch.get("spin", 0)) for ch in chains]
    tot = sum(E_c) + sum(Ac_c) + sum(ep_c)
    if tot >= TOT_LIMIT:
        raise ValueError("set demand beyond the exact feature range")

    q = [[(Ece[c][e] * Q) // T[c] for e in range(X)] for c in range(C)]
    qa = [[((Acce[c][e] + epce[c][e]) * Q) // T[c] for e in range(X)] for c in range(C)]
    qA = [[(Ahat[c][a] * Q) // T[c] for a in range(max(NA, 1))] for c in range(C)]

    # buckets of every accelerator under this order (Sec. IV-C)
    level = [[-1] * max(NA, 1) for _ in range(C)]
    for a in range(NA):
        users = sorted([c for c in range(C) if dca[c][a] > 0], key=lambda c: rank[c])
        m = len(users)
        for r, c in enumerate(users):
            level[c][a] = (r * int(st["accel_buckets"][a])) // m
    # higher process-priority executors on the same core
    hpx = [[e2 for e2 in range(X) if e2 != e and st["exec_core"][e2] == st["exec_core"][e]
            and st["exec_prio"][e2] > st["exec_prio"][e]] for e in range(X)]

    F = np.zeros((C, N_FEAT), np.float64)
    for c in range(C):
        rho = rank[c]
        HP = [h for h in range(C) if rank[h] < rho]
        LP = [h for h in range(C) if rank[h] > rho]
        mine = [e for e in range(X) if runsce[c][e] > 0]
        uses = [a for a in range(NA) if dca[c][a] > 0]
        own = E_c[c] + Ac_c[c] + ep_c[c] + (S_c[c] - 1) * hop
        f = F[c]
        f[0] = ratio(E_c[c], D[c])
        f[1] = ratio(Ac_c[c], D[c])
        f[2] = ratio(ep_c[c], D[c])
        f[3] = ratio((S_c[c] - 1) * hop, D[c])
        f[4] = ratio(own, D[c])
        f[5] = ratio(Emax_c[c], D[c])
        f[6] = ratio(S_c[c], 16)
        f[7] = ratio(dl_c[c], 16)
        f[8] = ratio(n_c[c], 32)
        f[9] = ratio(len(mine), X)
        f[10] = ratio(D[c], T[c])
        f[11] = ratio(T[c], 1 << 30)
        f[12] = float(spin[c])
        f[13] = ratio(sum(q[c]), Q)
        f[14] = ratio(sum(qa[c]), Q)
        # position in the order
        f[15] = ratio(rho, C)
        f[16] = ratio(C - 1 - rho, C)
        f[17] = 1.0 if rho == 0 else 0.0
        f[18] = 1.0 if rho == C - 1 else 0.0
        f[19] = ratio(sum(1 for h in HP if T[h] > T[c]), C)
        f[20] = ratio(sum(1 for h in LP if T[h] < T[c]), C)
        # higher-priority chains on the chain's executors (hp of Eq. (6))
        f[21] = ratio(sum(q[h][e] for e in mine for h in HP), Q)
        f[22] = ratio(sum(qa[h][e] for e in mine for h in HP), Q)
        n_carry = sum(runsce[c][e] * 2 * (Ece[h][e] + Acce[h][e] + epce[h][e])
                      for e in range(X) for h in HP)
        f[23] = ratio(n_carry, D[c])
        f[24] = ratio(max([sum(q[h][e] + qa[h][e] for h in HP) for e in mine], default=0), Q)
        f[25] = ratio(sum(1 for e in mine for h in HP if runsce[h][e] > 0), C)
        # blocking by one lower-priority callback per sub-chain
        n_bp = sum(runsce[c][e] * max([blce[h][e] for h in LP], default=0) for e in range(X))
        n_bs = sum(runsce[c][e] * max([bSce[h][e] for h in LP], default=0) for e in range(X))
        f[26] = ratio(n_bp, D[c])
        f[27] = ratio(n_bs, D[c])
        f[28] = ratio(max([max([bSce[h][e] for h in LP], default=0) for e in mine], default=0),
                      D[c])
        f[29] = ratio(sum(1 for e in mine for h in LP if runsce[h][e] > 0), C)
        # OS preemption by higher process-priority executors (hpp of Eq. (6))
        n_hpp = 0
        q_hpp = 0
        for e in range(X):
            for e2 in hpx[e]:
                for h in range(C):
                    if h == c:
                        continue
                    sp = Ece[h][e2] + (Acce[h][e2] + epce[h][e2] if spin[h] else epce[h][e2])
                    n_hpp += runsce[c][e] * 2 * sp
                    if runsce[c][e] > 0:
                        q_hpp += q[h][e2] + (qa[h][e2] if spin[h] else 0)
        f[30] = ratio(n_hpp, D[c])
        f[31] = ratio(q_hpp, Q)
        # accelerators (Eq. (3) and (4)): two requests of every HP chain on
        # each accelerator a sub-chain uses, once per sub-chain
        n_acc = 0
        for e, ids in _runs(chains[c]["cbs"]):
            acc_s = sorted({acc for j in ids for (_a, acc) in chains[c]["cbs"][j]["segs"]})
            n_acc += sum(2 * Ahat[h][a] for a in acc_s for h in HP)
        f[32] = ratio(n_acc, D[c])
        f[33] = ratio(sum(qA[h][a] for a in uses for h in HP), Q)
        n_bacc = 0
        for (a, _As) in seg_list[c]:
            n_bacc += max([Amax[h][a] for h in LP if dca[h][a] > 0 and level[h][a] == level[c][a]],
                          default=0)
        f[34] = ratio(n_bacc, D[c])
        f[35] = max([ratio(level[c][a], int(st["accel_buckets"][a])) for a in uses], default=0.0)
        f[36] = ratio(sum(1 for a in uses for h in HP if dca[h][a] > 0), C)
        f[37] = 1.0 if any(Ahat[h][a] > 0 for a in uses for h in HP) else 0.0
        # the whole set
        f[38] = ratio(sum(sum(q[h]) for h in range(C)), X * Q)
        f[39] = ratio(max(sum(q[h][e] for h in range(C)) for e in range(X)), Q)
        f[40] = ratio(sum(sum(qA[h][:NA]) for h in range(C)), Q)
        f[41] = ratio(C, 256)
        f[42] = ratio(X, 8)
        f[43] = ratio(NA, 8)
        f[44] = ratio(min(T), T[c])
        # a floor of the bound: own demand, two jobs of every interfering chain
        # per sub-chain (hp, hpp, accelerator), SAFE blocking and same-bucket
        # blocking; then the same plus the utilisation terms
        n_est = own + n_carry + n_bs + n_hpp + n_acc + n_bacc
        f[45] = ratio(n_est, D[c])
        q_est = (sum(q[h][e] for e in mine for h in HP) + sum(qa[h][e] for e in mine for h in HP)
                 + q_hpp + sum(qA[h][a] for a in uses for h in HP))
        f[46] = ratio(n_est, D[c]) + ratio(q_est, Q)
        f[47] = ratio(E_c[c] + Ac_c[c], sum(E_c) + sum(Ac_c))
    return F


def to_float32(x) -> np.ndarray:
    """Round-to-nearest-even fp64 -> fp32 (numpy's cast is exactly that)."""
    return np.asarray(x, np.float64).astype(np.float32)


def bf16_round(x32) -> np.ndarray:
    """fp32 -> bfloat16 value (as float64), round to nearest, ties to even.

    Chooses between the two bfloat16 neighbours of each finite value by the
    exact distance in float64 (every float32 and bfloat16 is exact there)."""
    x = np.asarray(x32, np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    lo_bits = (bits & np.uint64(0xFFFF0000)).astype(np.uint32)
    hi_bits = (lo_bits.astype(np.uint64) + np.uint64(0x10000)).astype(np.uint32)
    lo = lo_bits.view(np.float32).astype(np.float64)
    hi = hi_bits.view(np.float32).astype(np.float64)
    xv = x.astype(np.float64)
    dlo = np.abs(xv - lo)
    dhi = np.abs(hi - xv)
    even_lo = ((lo_bits >> np.uint32(16)) & np.uint32(1)) == 0
    pick_lo = (dlo < dhi) | ((dlo == dhi) & even_lo)
    out = np.where(pick_lo, lo, hi)
    return np.where(np.isfinite(xv), out, xv)


def bf16_bits(vals) -> np.ndarray:
    """uint16 bit patterns of bfloat16 values given as float64."""
    v = np.asarray(vals, np.float64).astype(np.float32)
    return (v.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def features_bf16(st: dict, order, util_permille: int = 1000) -> np.ndarray:
    """uint16 [C, 48]: the bfloat16 bit patterns of ``chain_features``."""
    return bf16_bits(bf16_round(to_float32(chain_features(st, order, util_permille))))
