"""Invariants and reductions that pin the oracle independently of its code.

Each property follows from the structure of the recurrences in Sec. IV-F:
every term is a non-negative integer combination of the inputs, mu is
non-decreasing, and the double bound takes a minimum of two safe bounds."""
import numpy as np
import pytest

import oracle
from paper_2404_06452_amd import chaingen

INF = oracle.INF


def _small_batch(n=60, seed=7, **kw):
    p = chaingen.PRESETS["small"].replace(seed=seed, **kw)
    return chaingen.generate(p, n)


def _tiny_params(seed):
    # small periods keep the recurrences short and mixes schedulable sets in
    return chaingen.PRESETS["small"].replace(
        seed=seed, chains=(2, 5), cbs=(1, 3), n_exec=3, util=(0.05, 0.4), pseg=(0.5, 0.5),
        frac=(0.1, 0.6), T=(20.0, 400.0))


def _scaled(cs, k):
    sets = [cs.set_dict(s) for s in range(cs.n_sets)]
    for st in sets:
        for ch in st["chains"]:
            ch["T"] *= k
            ch["D"] *= k
            for cb in ch["cbs"]:
                cb["E"] *= k
                cb["segs"] = [(a * k, i) for a, i in cb["segs"]]
        st["accel_eps"] = [v * k for v in st["accel_eps"]]
        st["accel_kappa"] = [v * k for v in st["accel_kappa"]]
        st["eps_hop"] *= k
    return chaingen.from_sets(sets)


@pytest.mark.parametrize("preset", ["small", "small_overheads"])
def test_homogeneity(preset):
    cs = chaingen.generate(chaingen.PRESETS[preset].replace(seed=11), 80)
    for full in (True, False):
        a = oracle.wcrt(cs, full=full)
        b = oracle.wcrt(_scaled(cs, 7), full=full)
        ra, rb = a["chain_R"], b["chain_R"]
        fin = (ra != INF) & (ra >= 0)
        assert np.array_equal(rb[fin], ra[fin] * 7)
        assert np.array_equal(rb[~fin], ra[~fin])
        assert np.array_equal(a["sched"], b["sched"])
        assert np.array_equal(a["worst"], b["worst"])


def _bounds(cs, **kw):
    return oracle.wcrt(cs, full=True, **kw)["chain_R"]


def _leq(a, b):
    """a <= b with INF as the top element."""
    return bool(np.all((a <= b) | (b == INF)))


@pytest.mark.parametrize("field", ["E", "A", "accel_eps", "accel_kappa", "eps_hop"])
def test_monotone_in_every_time(field):
    rng = np.random.default_rng(3)
    for seed in range(4):
        cs = chaingen.generate(_tiny_params(100 + seed), 40)
        base = _bounds(cs)
        arr = getattr(cs, field)
        if arr.size == 0:
            continue
        bumped = arr.copy()
        idx = rng.choice(arr.size, size=max(1, arr.size // 5), replace=False)
        bumped[idx] += rng.integers(1, 30, size=idx.size)
        setattr(cs, field, bumped)
        assert _leq(base, _bounds(cs)), field


def test_adding_a_chain_never_lowers_a_bound():
    rng = np.random.default_rng(5)
    cs = chaingen.generate(_tiny_params(200), 40)
    base = oracle.wcrt(cs, full=True)["chain_R"]
    sets = []
    for s in range(cs.n_sets):
        st = cs.set_dict(s)
        C = len(st["chains"])
        newp = int(rng.integers(0, C + 1))  # priority slot of the new chain
        for ch in st["chains"]:
            ch["prio"] = ch["prio"] * 2 + 1
        X = len(st["exec_core"])
        st["chains"].append({"T": 300, "D": 300, "prio": 2 * newp, "spin": int(rng.integers(0, 2)),
                             "cbs": [{"E": int(rng.integers(1, 6)), "exec": int(rng.integers(0, X)),
                                      "segs": [(int(rng.integers(0, 5)), 0)]}]})
        sets.append(st)
    more = chaingen.from_sets(sets)
    r2 = oracle.wcrt(more, full=True)["chain_R"]
    for s in range(cs.n_sets):
        c0, c1 = cs.set_chain_off[s], cs.set_chain_off[s + 1]
        d0 = more.set_chain_off[s]
        assert _leq(base[c0:c1], r2[d0:d0 + (c1 - c0)]), s


def test_own_demand_floor_and_cap():
    cs = chaingen.generate(_tiny_params(300), 200)
    R = _bounds(cs, cap_mult=2)
    for s in range(cs.n_sets):
        st = cs.set_dict(s)
        c0 = cs.set_chain_off[s]
        for i, ch in enumerate(st["chains"]):
            r = R[c0 + i]
            if r == INF:
                continue
            assert r <= 2 * ch["D"]
            execs = [cb["exec"] for cb in ch["cbs"]]
            runs = 1 + sum(1 for a, b in zip(execs, execs[1:]) if a != b)
            demand = sum(cb["E"] for cb in ch["cbs"])
            demand += sum(a + 2 * st["accel_kappa"][ai] + st["accel_eps"][ai]
                          for cb in ch["cbs"] for a, ai in cb["segs"])
            demand += (runs - 1) * st["eps_hop"]
            assert r >= demand


def test_double_bound_is_below_each_bound():
    for preset in ("small", "small_overheads"):
        cs = chaingen.generate(chaingen.PRESETS[preset].replace(seed=21), 80)
        for cap in (1, 3):
            m = _bounds(cs, cap_mult=cap)
            assert _leq(m, _bounds(cs, cap_mult=cap, bound=oracle.BOUND_L2))
            assert _leq(m, _bounds(cs, cap_mult=cap, bound=oracle.BOUND_L3))


def test_paper_blocking_below_safe_blocking():
    cs = chaingen.generate(chaingen.PRESETS["small_overheads"].replace(seed=23), 80)
    for cap in (1, 3):
        assert _leq(_bounds(cs, cap_mult=cap, blocking=oracle.BLOCK_PAPER),
                    _bounds(cs, cap_mult=cap, blocking=oracle.BLOCK_SAFE))


def test_chain_permutation_permutes_results():
    rng = np.random.default_rng(9)
    cs = _small_batch(40, seed=31)
    base = oracle.wcrt(cs, full=True)
    sets, perms = [], []
    for s in range(cs.n_sets):
        st = cs.set_dict(s)
        p = rng.permutation(len(st["chains"]))
        st["chains"] = [st["chains"][i] for i in p]
        sets.append(st)
        perms.append(p)
    pc = chaingen.from_sets(sets)
    out = oracle.wcrt(pc, full=True)
    for s in range(cs.n_sets):
        c0 = cs.set_chain_off[s]
        p = perms[s]
        assert out["chain_R"][c0:c0 + len(p)].tolist() == base["chain_R"][c0 + p].tolist()
        assert out["sched"][s] == base["sched"][s]


def _jitter_rta(chains):
    """Textbook response-time analysis with release jitter (Audsley, Burns,
    Richardson, Tindell & Wellings 1993) for one non-preemptive executor on a
    core of its own: R = B + C + sum_hp ceil((R + J_h)/T_h) C_h with J_h = T_h
    and B the largest lower-priority WCET."""
    out = []
    for i, (T, Cc) in enumerate(chains):
        B = max([c for _, c in chains[i + 1:]], default=0)
        R = 0
        while True:
            nxt = B + Cc + sum(-(-(R + Th) // Th) * Ch for Th, Ch in chains[:i])
            if nxt > T:
                R = INF
                break
            if nxt == R:
                break
            R = nxt
        out.append(R)
    return out


def test_reduces_to_jitter_rta_without_accelerators():
    rng = np.random.default_rng(13)
    for _ in range(200):
        C = int(rng.integers(1, 7))
        chains = sorted([(int(rng.integers(5, 200)), int(rng.integers(1, 12))) for _ in range(C)])
        st = {"chains": [{"T": T, "D": T, "prio": C - i, "spin": 0,
                          "cbs": [{"E": Cc, "exec": 0, "segs": []}]}
                         for i, (T, Cc) in enumerate(chains)],
              "exec_core": [0], "exec_prio": [1]}
        cs = chaingen.from_sets([st])
        assert oracle.analyse_set(cs, 0, full=True)["chain_R"].tolist() == _jitter_rta(chains)


def test_single_chain_closed_form():
    rng = np.random.default_rng(17)
    for _ in range(100):
        n = int(rng.integers(1, 7))
        X = int(rng.integers(1, 4))
        eps, kap, hop = (int(v) for v in rng.integers(0, 4, size=3))
        cbs = [{"E": int(rng.integers(0, 9)), "exec": int(rng.integers(0, X)),
                "segs": [(int(rng.integers(0, 9)), 0) for _ in range(int(rng.integers(0, 3)))]}
               for _ in range(n)]
        st = {"chains": [{"T": 10**6, "D": 10**6, "prio": 1, "spin": 0, "cbs": cbs}],
              "exec_core": list(range(X)), "exec_prio": [1] * X, "accel_eps": [eps],
              "accel_kappa": [kap], "eps_hop": hop}
        execs = [cb["exec"] for cb in cbs]
        runs = 1 + sum(1 for a, b in zip(execs, execs[1:]) if a != b)
        want = (sum(cb["E"] for cb in cbs) + sum(a + 2 * kap + eps for cb in cbs for a, _ in cb["segs"])
                + (runs - 1) * hop)
        r = oracle.analyse_set(chaingen.from_sets([st]), 0, full=True)
        assert r["chain_R"].tolist() == [want]


def test_verdict_mode_agrees_with_full_mode():
    for preset in ("small", "small_overheads"):
        cs = chaingen.generate(_tiny_params(400) if preset == "small" else
                               chaingen.PRESETS[preset].replace(seed=41), 150)
        f = oracle.wcrt(cs, full=True)
        v = oracle.wcrt(cs, full=False)
        assert np.array_equal(f["sched"], v["sched"])
        ok = v["sched"] == 1
        assert np.array_equal(f["worst"][ok], v["worst"][ok])
        assert np.array_equal(f["worst_R"][ok], v["worst_R"][ok])
        assert np.all(v["worst"][~ok] == -1)
        assert np.all(v["terms"] <= f["terms"])


def test_candidate_orders_are_a_swap_walk():
    cs = chaingen.generate("search", 5)
    for s in range(cs.n_sets):
        c0, c1 = cs.set_chain_off[s], cs.set_chain_off[s + 1]
        base = np.argsort(-cs.prio[c0:c1], kind="stable")
        prev = oracle.candidate_order(cs, s, 99, 0)
        assert prev.tolist() == base.tolist()
        for k in range(1, 40):
            cur = oracle.candidate_order(cs, s, 99, k)
            assert sorted(cur.tolist()) == list(range(c1 - c0))
            assert int(np.sum(cur != prev)) == 2  # exactly one swap of two positions
            prev = cur


def test_search_matches_brute_force_over_candidates():
    p = chaingen.PRESETS["search"].replace(seed=51, util=(0.03, 0.15), chains=(4, 6))
    cs = chaingen.generate(p, 40)
    res = oracle.search(cs, 24, 1234)
    for s in range(cs.n_sets):
        want = -1
        for k in range(24):
            if oracle.analyse_set(cs, s, oracle.candidate_order(cs, s, 1234, k))["sched"]:
                want = k
                break
        assert res["found"][s] == want
        assert res["n_eval"][s] == (want + 1 if want >= 0 else 24)
