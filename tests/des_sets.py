"""Random sets for the simulation tests (shared by the CPU and GPU tests)."""


def tiny_set(rng):
    """A random set small enough for the unit-step simulator: 1-4 chains of
    1-3 callbacks with 0-2 segments, 1-3 executors on 1-3 cores, 1-2
    accelerators with 1-2 buckets, small overheads, hops and periods."""
    C, X = rng.randint(1, 4), rng.randint(1, 3)
    cores, NA = rng.randint(1, X), rng.randint(1, 2)
    exec_core = [rng.randrange(cores) for _ in range(X)]
    exec_prio = []
    for e in range(X):
        used = {exec_prio[f] for f in range(e) if exec_core[f] == exec_core[e]}
        p = rng.randint(1, 5)
        while p in used:
            p += 1
        exec_prio.append(p)
    prios = rng.sample(range(1, 20), C)
    chains = []
    for c in range(C):
        T = rng.randint(20, 80)
        cbs = [{"E": rng.randint(0, 3), "exec": rng.randrange(X),
                "segs": [[rng.randint(0, 3), rng.randrange(NA)] for _ in range(rng.randint(0, 2))]}
               for _ in range(rng.randint(1, 3))]
        chains.append({"T": T, "D": T, "prio": prios[c], "spin": rng.randint(0, 1), "cbs": cbs})
    return {"chains": chains, "exec_core": exec_core, "exec_prio": exec_prio,
            "accel_buckets": [rng.randint(1, 2) for _ in range(NA)],
            "accel_eps": [rng.randint(0, 2) for _ in range(NA)],
            "accel_kappa": [rng.randint(0, 1) for _ in range(NA)], "eps_hop": rng.randint(0, 2)}
