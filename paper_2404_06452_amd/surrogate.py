"""Training and use of the candidate-ranking network on the GPU.

Every step runs in libpaam's kernels: targets come from the exact analysis
(``paam_candidate_wcrt``, every chain's bound at cap 2D, target =
min(max R/D, 2)), inputs from ``paam_features``, and the network is trained by
``paam_mlp_forward`` / ``paam_mlp_backward`` / ``paam_mlp_adam_step``.  This
module only orders the calls, draws nothing itself (pairs and initial weights
come from the seeded input generators) and moves batch indices around.
"""
from __future__ import annotations

import time

import numpy as np

from . import _paam


# Training recipe: sets of the utilisation-sweep generator (4-64 chains x 2-12
# callbacks, 4 executors) analysed at a utilisation scale drawn log-uniformly
# over 0.2-10 % of their U = 1 draw, so that the targets span the feasibility
# boundary (at the sweep's own levels 0.10-0.95 almost every candidate's
# largest R/D exceeds 2 and the target is constant); candidates k uniform over
# the walk's first 256; target min(max R/D, 2).
TRAIN_UTIL = (2, 100)
TRAIN_CAP = 2


def recipe_pairs(n_sets: int, n_samples: int, seed: int, n_cand: int = 256):
    from . import chaingen
    return chaingen.training_triples(n_sets, n_samples, n_cand, TRAIN_UTIL, seed)


class Trainer:
    """Mean-squared-error training of the ranking network on (set, k,
    util_permille) pairs of one uploaded batch."""

    def __init__(self, dev: _paam.Chainset, net: _paam.Network, seed: int, batch: int = 4096,
                 stream=None):
        import torch
        self.dev, self.net, self.seed, self.batch, self.stream = dev, net, seed, batch, stream
        d = dev.device
        self.rs = dev.max_chains
        self.feat = torch.zeros(batch * self.rs * _paam.N_FEAT, dtype=torch.int16, device=d)
        self.count = torch.zeros(batch, dtype=torch.int32, device=d)
        self.out = torch.zeros(batch, dtype=torch.float32, device=d)
        self.act = torch.zeros(batch * 512, dtype=torch.int16, device=d)
        self.grad = torch.zeros(_paam.MLP_PARAMS, dtype=torch.float32, device=d)
        self.loss = torch.zeros(1, dtype=torch.float32, device=d)
        self.fws = _paam.workspace(_paam.paam_features_bytes(dev, batch), d)
        self.bws = _paam.workspace(_paam.paam_mlp_backward_bytes(batch), d)

    def targets(self, pairs, cap_mult: int = TRAIN_CAP):
        """Exact-analysis targets of device pairs [n, 3]: float32 ratios."""
        o = _paam.wcrt_opts(cap_mult=cap_mult, full=True)
        n = int(pairs.shape[0])
        out = _paam.CandOut(n, self.dev.device)
        ws = _paam.workspace(_paam.paam_candidate_bytes(self.dev, o, n), self.dev.device)
        _paam.paam_candidate_wcrt(self.dev, o, self.seed, pairs, out, ws, self.stream)
        return out

    def _features(self, pairs):
        _paam.paam_features(self.dev, self.seed, pairs, self.rs, self.feat, self.count, self.fws,
                            self.stream)

    def step(self, pairs, target, lr: float) -> None:
        """One Adam step on a batch (device pairs [b, 3], target [b])."""
        b = int(pairs.shape[0])
        self._features(pairs)
        _paam.paam_mlp_forward(self.net.params, self.net.packed, self.feat, self.count, b, self.rs,
                               self.out, self.act, self.stream)
        _paam.paam_mlp_backward(self.net.params, self.net.packed, self.feat, self.count, b,
                                self.rs, self.out, target, self.act, self.grad, self.loss,
                                self.bws, self.stream)
        self.net.adam(self.grad, lr, stream=self.stream)

    def predict(self, pairs):
        """Network outputs for device pairs (float32 device tensor)."""
        import torch
        n = int(pairs.shape[0])
        res = torch.empty(n, dtype=torch.float32, device=self.dev.device)
        for i in range(0, n, self.batch):
            p = pairs[i:i + self.batch]
            b = int(p.shape[0])
            self._features(p)
            _paam.paam_mlp_forward(self.net.params, self.net.packed, self.feat, self.count, b,
                                   self.rs, res[i:i + b], None, self.stream)
        return res

    def fit(self, pairs, target, epochs: int, lr: float, order_seed: int, log=None,
            lr_final: float | None = None, start_epoch: int = 0, stop_epoch: int | None = None,
            checkpoint: str | None = None):
        """Epochs over device pairs/targets in a seeded shuffled order; the
        learning rate decays linearly to lr_final.  Returns the mean loss of
        every epoch run.

        start_epoch > 0 resumes a run whose first start_epoch epochs are
        already in the network (restored by load_checkpoint): the epoch
        orders and the learning-rate schedule continue where they stopped, so
        the result equals the uninterrupted run; stop_epoch ends a run early
        (the schedule still spans all epochs).  checkpoint: a path written
        after every epoch."""
        import torch

        from . import chaingen
        n = int(pairs.shape[0])
        per_epoch = sum(1 for i in range(0, n, self.batch) if min(self.batch, n - i) >= 2)
        steps = epochs * ((n + self.batch - 1) // self.batch)
        k = start_epoch * per_epoch
        losses = []
        for ep in range(start_epoch, epochs if stop_epoch is None else min(stop_epoch, epochs)):
            perm = torch.from_numpy(chaingen.shuffle_order(n, order_seed + ep)).to(pairs.device)
            acc = torch.zeros(1, dtype=torch.float64, device=pairs.device)
            t0 = time.perf_counter()
            nb = 0
            for i in range(0, n, self.batch):
                idx = perm[i:i + self.batch]
                if idx.numel() < 2:
                    continue
                cur = lr if lr_final is None else lr + (lr_final - lr) * k / max(steps - 1, 1)
                self.step(pairs[idx].contiguous(), target[idx].contiguous(), float(cur))
                acc += self.loss.double()
                nb += 1
                k += 1
            losses.append(float(acc.item()) / max(nb, 1))
            if checkpoint:
                save_checkpoint(checkpoint, self.net, epoch=ep + 1)
            if log:
                log("epoch %d: loss %.5f (%.1f s)" % (ep, losses[-1], time.perf_counter() - t0))
        return losses


CHECKPOINT_FORMAT = "paam-ranking-network-1"


def save_state(path: str, params, m, v, step: int, epoch: int | None = None) -> None:
    """Writes a training state (float32 master parameters, Adam moments, Adam
    step, epochs done) as a safetensors file."""
    from safetensors.numpy import save_file
    arrays = {k: np.ascontiguousarray(a, np.float32) for k, a in
              (("params", params), ("adam_m", m), ("adam_v", v))}
    for k, a in arrays.items():
        if a.shape != (_paam.MLP_PARAMS,):
            raise ValueError("%s has shape %s, expected (%d,)" % (k, a.shape, _paam.MLP_PARAMS))
    meta = {"format": CHECKPOINT_FORMAT, "step": str(int(step)),
            "epoch": "" if epoch is None else str(int(epoch))}
    tmp = path + ".tmp"
    save_file(arrays, tmp, metadata=meta)
    import os
    os.replace(tmp, path)


def load_state(path: str) -> dict:
    """Reads a file written by save_state (safetensors: no code runs on load)."""
    from safetensors import safe_open
    with safe_open(path, framework="numpy") as f:
        meta = f.metadata() or {}
        if meta.get("format") != CHECKPOINT_FORMAT:
            raise ValueError("%s is not a ranking-network checkpoint" % path)
        out = {k: f.get_tensor(k) for k in ("params", "adam_m", "adam_v")}
    for k, a in out.items():
        if a.dtype != np.float32 or a.shape != (_paam.MLP_PARAMS,):
            raise ValueError("%s: %s has dtype %s shape %s" % (path, k, a.dtype, a.shape))
    out["step"] = int(meta["step"])
    out["epoch"] = int(meta["epoch"]) if meta.get("epoch") else None
    return out


def save_checkpoint(path: str, net: _paam.Network, epoch: int | None = None) -> None:
    """Checkpoint of a device network: master weights, moments, step."""
    save_state(path, net.params.cpu().numpy(), net.m.cpu().numpy(), net.v.cpu().numpy(),
               net.step, epoch)


def load_checkpoint(path: str, device="cuda:0", stream=None):
    """A device network restored from a checkpoint (its bfloat16 copy repacked
    by the library), and the epochs it holds."""
    import torch
    st = load_state(path)
    net = _paam.Network(st["params"], device=device, stream=stream)
    net.m.copy_(torch.from_numpy(st["adam_m"]))
    net.v.copy_(torch.from_numpy(st["adam_v"]))
    net.step = st["step"]
    return net, st["epoch"]


def spearman(a, b) -> float:
    """Spearman rank correlation of two 1-D arrays (average ranks for ties)."""
    def ranks(x):
        x = np.asarray(x, np.float64)
        order = np.argsort(x, kind="stable")
        r = np.empty(len(x))
        r[order] = np.arange(len(x))
        # average ranks of ties
        xs = x[order]
        i = 0
        while i < len(xs):
            j = i
            while j + 1 < len(xs) and xs[j + 1] == xs[i]:
                j += 1
            if j > i:
                r[order[i:j + 1]] = (i + j) / 2.0
            i = j + 1
        return r
    ra, rb = ranks(a), ranks(b)
    ra -= ra.mean()
    rb -= rb.mean()
    den = np.sqrt((ra * ra).sum() * (rb * rb).sum())
    return float((ra * rb).sum() / den) if den > 0 else 0.0
