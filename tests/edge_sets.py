"""Chain sets at the edges of the input range, for the GPU parity tests.

Two regimes, never mixed within a set, so that every recurrence either
converges or passes its cap within a bounded number of iterations (a total
interference utilisation just below 1 with a cap near 2^42 ns would need
billions of iterations):
* tiny: periods of 1-1000 ns, deadlines down to 1 ns, times of 0-3 ns or a
  quarter of the period, so caps stay below 64,000 ns;
* huge: periods of 2^30 ns to just below 2^36 ns, every time either at most
  1/256 of its chain's period or an overload (2^36 - 1 ns, or overheads of
  that size), so a set either stays below 3/4 utilisation or passes its caps
  within a few iterations.
Zero-length callbacks and segments, up to 3 accelerators with several buckets,
executor pairs sharing a core, callbacks alternating between executors (many
sub-chains per chain) and hop costs up to 2^36 - 1 ns.  Built from a seeded
numpy generator; holds no analysis arithmetic."""
import numpy as np

LIM = (1 << 36) - 1


def edge_sets(n_sets=160, seed=2404):
    rng = np.random.default_rng(seed)
    sets = []
    for i in range(n_sets):
        tiny = i % 2 == 0
        C = int(rng.integers(1, 9))
        X = int(rng.integers(1, 5))
        NA = int(rng.integers(0, 4))
        alternate = rng.random() < 0.4
        chains = []
        for c in range(C):
            if tiny:
                T = int(rng.choice([1, 2, 3, 7, 1000]))
            else:
                T = int(rng.choice([LIM, LIM - 12345, (1 << 35) + 777,
                                    int(rng.integers(1 << 30, 1 << 35))]))
            D = T if rng.random() < 0.6 else max(1, T // 3)
            n = int(rng.integers(1, 13))

            def value():
                if tiny:
                    return int(rng.choice([0, 1, 3, T // 4]))
                return int(rng.choice([0, 1, T // 256, T // 1024, LIM], p=[.2, .2, .25, .25, .1]))

            cbs = []
            for j in range(n):
                e = (j % X) if alternate else int(rng.integers(0, X))
                segs = []
                if NA > 0:
                    for _ in range(int(rng.choice([0, 0, 1, 2]))):
                        segs.append((value(), int(rng.integers(0, NA))))
                cbs.append({"E": value(), "exec": e, "segs": segs})
            chains.append({"T": T, "D": D, "prio": 0, "spin": int(rng.integers(0, 2)), "cbs": cbs})
        for r, c in enumerate(rng.permutation(C)):
            chains[int(c)]["prio"] = C - r
        cores = list(range(X)) if rng.random() < 0.5 else [e // 2 for e in range(X)]
        over = [0, 1, 3] if tiny else [0, 1, 391_000, LIM]
        sets.append({
            "chains": chains,
            "exec_core": cores,
            "exec_prio": [X - e for e in range(X)],
            "accel_buckets": [int(rng.integers(1, 7)) for _ in range(NA)],
            "accel_eps": [int(rng.choice(over)) for _ in range(NA)],
            "accel_kappa": [int(rng.choice(over)) for _ in range(NA)],
            "eps_hop": int(rng.choice(over)),
        })
    return sets
