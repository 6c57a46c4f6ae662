"""Named GPU workloads for profiling runs (``python -m paper_2404_06452_amd.runs <name>``).

Each run uploads a seeded synthetic batch, calls the library a fixed number of
times and prints one line per call, so that a kernel profiler attached to the
process sees a known sequence of launches:

* ``sweep``  - the analysis of the utilisation sweep (every chain's bound, cap = D)
* ``search`` - plain priority-order search over 256 candidates per set
* ``score``  - network scores of every candidate (features + forward)
* ``guided`` - scoring followed by the guided search (top 16, with fallback)
* ``train``  - targets, then training steps of the ranking network
* ``large``  - sets of 256 chains: the uploaded order's analysis, scores of
  1,024 candidate orders per set, the exact confirmation of the top 32
* ``des``    - the simulation of the study's 8-chain sets, 64 scenarios each
  (synchronous release, then random offsets), horizon twice the longest period
* ``units``  - binding of the sweep sets' segments to 4 units per accelerator
"""
from __future__ import annotations

import argparse
import time


def main(argv=None):
    import torch

    from . import _paam, chaingen, surrogate

    ap = argparse.ArgumentParser()
    ap.add_argument("run", choices=("sweep", "search", "score", "guided", "train", "large", "des",
                                    "units"))
    ap.add_argument("--sets", type=int, default=100_000)
    ap.add_argument("--cand", type=int, default=256)
    ap.add_argument("--util", type=int, default=1000)
    ap.add_argument("--repeat", type=int, default=2)
    ap.add_argument("--samples", type=int, default=1 << 20)
    args = ap.parse_args(argv)
    seed = 77

    def timed(what, fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        print("%s %.4f s" % (what, time.perf_counter() - t), flush=True)
        return r

    if args.run == "sweep":
        cs = chaingen.generate("sweep", args.sets)
        dev = _paam.Chainset(cs, device="cuda:0")
        for u in chaingen.SWEEP_LEVELS[:: max(1, 18 // max(args.repeat, 1))]:
            timed("sweep level %d" % u, lambda: _paam.wcrt(dev, full=True, util_permille=u))
        return
    if args.run == "des":
        cs = chaingen.generate(chaingen.study_params(8, 1, 1), args.sets)
        dev = _paam.Chainset(cs, device="cuda:0")
        n_scen, horizon = 64, int(2 * cs.T.max())
        offs = torch.as_tensor(chaingen.release_offsets(cs, n_scen, 2404)).cuda()
        obs = torch.empty(cs.n_chains * n_scen, dtype=torch.int64, device="cuda:0")
        st = torch.empty(cs.n_sets * n_scen, dtype=torch.int8, device="cuda:0")
        for r in range(args.repeat):
            o = _paam.des_opts(n_scen, horizon, exec_permille=1000 if r % 2 == 0 else 500, seed=7)
            timed("simulation %d" % r, lambda: _paam.paam_des_batch(dev, o, offs, obs, st))
        print("scenarios %d, completed %d" % (cs.n_sets * n_scen, int((st == 0).sum())), flush=True)
        return
    if args.run == "units":
        import numpy as np
        cs = chaingen.generate("sweep", args.sets)
        units = np.full(int(cs.set_accel_off[-1]), 4, np.int16)
        dev = _paam.Chainset(cs, device="cuda:0", units=units, unit_group=_paam.PAAM_UNITS_CHAIN)
        for r in range(args.repeat):
            timed("binding %d" % r, lambda: dev.assign_units())
        return
    if args.run == "train":
        cs = chaingen.generate("sweep", args.sets)
        dev = _paam.Chainset(cs, device="cuda:0")
        net = _paam.Network(chaingen.mlp_init(seed), device="cuda:0")
        tr = surrogate.Trainer(dev, net, seed)
        pairs = torch.from_numpy(surrogate.recipe_pairs(cs.n_sets, args.samples, seed)).cuda()
        tg = timed("targets", lambda: tr.targets(pairs))
        for r in range(args.repeat):
            timed("epoch %d" % r, lambda: tr.fit(pairs, tg.ratio[:args.samples], 1, 1e-3, seed + r))
        return
    if args.run == "large":
        cs = chaingen.generate("large", args.sets)
        dev = _paam.Chainset(cs, device="cuda:0")
        net = _paam.Network(chaingen.mlp_init(1), device="cuda:0")
        for r in range(args.repeat):
            timed("RM analysis", lambda: _paam.wcrt(dev, full=False, util_permille=args.util))
            sc = timed("score", lambda: _paam.score(dev, net, args.cand, seed,
                                                    util_permille=args.util))
            timed("guided search", lambda: _paam.search(dev, args.cand, seed, scores=sc,
                                                        guided=True, top_k=32, fallback=False,
                                                        util_permille=args.util))
        return
    cs = chaingen.generate("search", args.sets)
    dev = _paam.Chainset(cs, device="cuda:0")
    net = _paam.Network(chaingen.mlp_init(1), device="cuda:0")
    for r in range(args.repeat):
        if args.run == "search":
            timed("plain search", lambda: _paam.search(dev, args.cand, seed,
                                                       util_permille=args.util))
        elif args.run == "score":
            timed("score", lambda: _paam.score(dev, net, args.cand, seed,
                                               util_permille=args.util))
        else:
            sc = timed("score", lambda: _paam.score(dev, net, args.cand, seed,
                                                    util_permille=args.util))
            timed("guided search", lambda: _paam.search(dev, args.cand, seed, scores=sc,
                                                        guided=True, top_k=16, fallback=True,
                                                        util_permille=args.util))


if __name__ == "__main__":
    main()
