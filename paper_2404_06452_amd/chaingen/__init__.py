"""Seeded synthetic chain-set generator (input module shared by both sides).

Holds none of the analysis arithmetic: it draws chain sets (the callback and
chain tuples of the paper's system model, Sec. II-C) and returns them as a
``ChainSets`` of numpy CSR arrays.  Each set has its own counter-based
SplitMix64 streams keyed by (seed, set id), so ``generate(..., set_begin=i,
n_sets=1)`` reproduces set ``i`` of a large batch exactly.

Workload recipes (all times int64 ns; periods log-uniform over 10-1000 ms with
implicit deadlines; per-chain utilisation from UUniFast split equally over the
chain's callbacks; a segment-carrying callback's WCET W splits into
A = round(f*W) on the accelerator and E = W - A on the CPU; callbacks map
uniformly to executors; executor pairs share a core with process priority
decreasing in the executor index; half of the chains busy-wait; priorities are
rate-monotonic; one accelerator with one bucket and zero overheads unless a
preset says otherwise):

* ``small``  - 8 chains x 2-5 callbacks, 2 executors, U = 0.5, 30 % segments
  of 10-50 % of the WCET.
* ``sweep``  - 4-64 chains x 2-12 callbacks, 4 executors, drawn at U = 1 and
  scaled per utilisation level 0.10-0.95; segment share per set U(10, 60) %,
  segment length 5-80 % of the WCET.
* ``search`` - 16 chains x 2-8 callbacks, 4 executors, U ~ U(0.5, 0.9).
* ``large``  - 256 chains x 2-32 callbacks, 8 executors, U ~ U(0.3, 0.95),
  50 % segments.
* ``study_params(n, acc, cpu)`` - the analytical study of Sec. V: n chains
  of 4 callbacks, each with one segment, accelerator : CPU utilisation
  acc : cpu per chain, one executor per chain on its own core, UUniFast at
  0.05 per chain (readings documented at STUDY_CHAIN_UTIL).
* ``small_overheads`` - ``small`` with the paper's measured overheads: 6
  buckets (Sec. IV-C), epsilon = 391 us (Sec. V-C, worst request overhead),
  kappa = 129.18 us (Sec. V-C table, worst preemption delay), hop cost =
  epsilon.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chaingen.c")
_LIB = os.path.join(_HERE, "libchaingen.so")

SEED_BASE = 2404064520


@dataclass(frozen=True)
class GenParams:
    seed: int
    chains: tuple[int, int]
    cbs: tuple[int, int]
    n_exec: int
    util: tuple[float, float]
    pseg: tuple[float, float]
    frac: tuple[float, float]
    T: tuple[float, float] = (1.0e7, 1.0e9)
    n_accel: int = 1
    max_seg_per_cb: int = 1
    n_buckets: int = 1
    spin_prob: float = 0.5
    eps: int = 0
    kappa: int = 0
    eps_hop: int = 0
    exec_per_chain: bool = False  # every callback of chain c on executor c mod n_exec
    own_cores: bool = False       # every executor alone on its core

    def replace(self, **kw) -> "GenParams":
        return dataclasses.replace(self, **kw)


PRESETS: dict[str, GenParams] = {
    "small": GenParams(SEED_BASE + 0, (8, 8), (2, 5), 2, (0.5, 0.5), (0.3, 0.3), (0.1, 0.5)),
    "sweep": GenParams(SEED_BASE + 1, (4, 64), (2, 12), 4, (1.0, 1.0), (0.1, 0.6), (0.05, 0.8)),
    "search": GenParams(SEED_BASE + 2, (16, 16), (2, 8), 4, (0.5, 0.9), (0.3, 0.3), (0.1, 0.5)),
    "large": GenParams(SEED_BASE + 4, (256, 256), (2, 32), 8, (0.3, 0.95), (0.5, 0.5), (0.1, 0.5)),
}
PRESETS["small_overheads"] = PRESETS["small"].replace(
    n_buckets=6, eps=391_000, kappa=129_180, eps_hop=391_000)

# utilisation levels of the sweep, in permille: 0.10, 0.15, ..., 0.95
SWEEP_LEVELS = tuple(range(100, 951, 50))

# Analytical study of the paper's Sec. V (schedulability against the number of
# chains, and against the accelerator : CPU utilisation ratio).  The paper
# fixes 4 callbacks per chain, one accelerator, random periods and the
# per-chain ratio (1:1, then 1:9 ... 7:3) with each chain's utilisation split
# equally over its callbacks.  Readings for what it leaves open: every
# callback carries one segment (its accelerator share of the callback's
# utilisation is the ratio); each chain runs on a single-threaded executor of
# its own, alone on its core, so chains contend only on the shared
# accelerator; chain utilisations come from UUniFast at 0.05 per chain.
STUDY_CHAIN_UTIL = 0.05
STUDY_CHAINS = tuple(range(1, 17))
STUDY_RATIOS = ((1, 9), (2, 8), (3, 7), (4, 6), (5, 5), (6, 4), (7, 3))
STUDY_RATIO_CHAINS = 8


def study_params(n_chains: int, acc: int = 1, cpu: int = 1) -> GenParams:
    """Generator of the analytical study: n_chains chains of 4 callbacks,
    accelerator : CPU utilisation acc : cpu per chain."""
    u = STUDY_CHAIN_UTIL * n_chains
    f = acc / (acc + cpu)
    return GenParams(SEED_BASE + 5 + 1000 * n_chains + 100 * acc + cpu, (n_chains, n_chains),
                     (4, 4), n_chains, (u, u), (1.0, 1.0), (f, f), exec_per_chain=True,
                     own_cores=True)


@dataclass
class ChainSets:
    """CSR arrays of ``n_sets`` chain sets (global indices throughout)."""
    n_sets: int
    set_chain_off: np.ndarray
    set_exec_off: np.ndarray
    set_accel_off: np.ndarray
    chain_cb_off: np.ndarray
    cb_seg_off: np.ndarray
    T: np.ndarray
    D: np.ndarray
    prio: np.ndarray
    spin: np.ndarray
    E: np.ndarray
    exec: np.ndarray
    A: np.ndarray
    accel: np.ndarray
    exec_core: np.ndarray
    exec_prio: np.ndarray
    accel_buckets: np.ndarray
    accel_eps: np.ndarray
    accel_kappa: np.ndarray
    eps_hop: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_chains(self) -> int:
        return int(self.set_chain_off[-1])

    @property
    def n_callbacks(self) -> int:
        return int(self.chain_cb_off[-1])

    @property
    def n_segments(self) -> int:
        return int(self.cb_seg_off[-1])

    def nbytes(self) -> int:
        return sum(v.nbytes for v in vars(self).values() if isinstance(v, np.ndarray))

    def subset(self, sets) -> "ChainSets":
        """A new batch holding the listed sets, in that order."""
        return from_sets([self.set_dict(int(s)) for s in sets])

    def set_dict(self, s: int) -> dict:
        """One set as plain set-local lists (chains, callbacks, segments)."""
        c0, c1 = int(self.set_chain_off[s]), int(self.set_chain_off[s + 1])
        x0, x1 = int(self.set_exec_off[s]), int(self.set_exec_off[s + 1])
        a0, a1 = int(self.set_accel_off[s]), int(self.set_accel_off[s + 1])
        chains = []
        for c in range(c0, c1):
            cbs = []
            for j in range(int(self.chain_cb_off[c]), int(self.chain_cb_off[c + 1])):
                segs = [(int(self.A[g]), int(self.accel[g]))
                        for g in range(int(self.cb_seg_off[j]), int(self.cb_seg_off[j + 1]))]
                cbs.append({"E": int(self.E[j]), "exec": int(self.exec[j]), "segs": segs})
            chains.append({"T": int(self.T[c]), "D": int(self.D[c]), "prio": int(self.prio[c]),
                           "spin": int(self.spin[c]), "cbs": cbs})
        return {
            "chains": chains,
            "exec_core": [int(v) for v in self.exec_core[x0:x1]],
            "exec_prio": [int(v) for v in self.exec_prio[x0:x1]],
            "accel_buckets": [int(v) for v in self.accel_buckets[a0:a1]],
            "accel_eps": [int(v) for v in self.accel_eps[a0:a1]],
            "accel_kappa": [int(v) for v in self.accel_kappa[a0:a1]],
            "eps_hop": int(self.eps_hop[s]),
        }


def from_sets(sets: list[dict]) -> ChainSets:
    """Builds a batch from hand-written sets (the format of ``set_dict``).

    Used for the worked examples: chains list callbacks in precedence order;
    each callback has E, exec and a list of (A, accel) segments."""
    sco, seo, sao, cco, cso = [0], [0], [0], [0], [0]
    T, D, prio, spin, E, ex, A, acc = [], [], [], [], [], [], [], []
    core, eprio, nb, eps, kap, hop = [], [], [], [], [], []
    for st in sets:
        for ch in st["chains"]:
            T.append(ch["T"]); D.append(ch.get("D", ch["T"]))
            prio.append(ch["prio"]); spin.append(ch.get("spin", 0))
            for cb in ch["cbs"]:
                E.append(cb["E"]); ex.append(cb["exec"])
                for (a, ai) in cb.get("segs", []):
                    A.append(a); acc.append(ai)
                cso.append(len(A))
            cco.append(len(E))
        sco.append(len(T))
        core += st["exec_core"]; eprio += st["exec_prio"]
        seo.append(len(core))
        nb += st.get("accel_buckets", [1]); eps += st.get("accel_eps", [0])
        kap += st.get("accel_kappa", [0])
        sao.append(len(nb))
        hop.append(st.get("eps_hop", 0))
    i64 = lambda v: np.asarray(v, dtype=np.int64)
    return ChainSets(
        n_sets=len(sets), set_chain_off=i64(sco), set_exec_off=i64(seo), set_accel_off=i64(sao),
        chain_cb_off=i64(cco), cb_seg_off=i64(cso), T=i64(T), D=i64(D),
        prio=np.asarray(prio, np.int32), spin=np.asarray(spin, np.uint8), E=i64(E),
        exec=np.asarray(ex, np.int16), A=i64(A), accel=np.asarray(acc, np.int16),
        exec_core=np.asarray(core, np.int16), exec_prio=np.asarray(eprio, np.int32),
        accel_buckets=np.asarray(nb, np.int16), accel_eps=i64(eps), accel_kappa=i64(kap),
        eps_hop=i64(hop))


# ----------------------------------------------------------------- native part
class _Params(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64), ("set_begin", ctypes.c_int64), ("n_sets", ctypes.c_int64),
        ("chains_lo", ctypes.c_int32), ("chains_hi", ctypes.c_int32),
        ("cbs_lo", ctypes.c_int32), ("cbs_hi", ctypes.c_int32),
        ("n_exec", ctypes.c_int32), ("n_accel", ctypes.c_int32),
        ("max_seg_per_cb", ctypes.c_int32), ("n_buckets", ctypes.c_int32),
        ("util_lo", ctypes.c_double), ("util_hi", ctypes.c_double),
        ("pseg_lo", ctypes.c_double), ("pseg_hi", ctypes.c_double),
        ("frac_lo", ctypes.c_double), ("frac_hi", ctypes.c_double),
        ("T_lo", ctypes.c_double), ("T_hi", ctypes.c_double),
        ("spin_prob", ctypes.c_double),
        ("eps", ctypes.c_int64), ("kappa", ctypes.c_int64), ("eps_hop", ctypes.c_int64),
        ("exec_per_chain", ctypes.c_int32), ("own_cores", ctypes.c_int32),
    ]


class _Out(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "set_chain_off", "set_cb_off", "set_seg_off", "chain_cb_off", "cb_seg_off", "T", "D",
        "prio", "spin", "E", "exec", "A", "accel", "exec_core", "exec_prio", "accel_buckets",
        "accel_eps", "accel_kappa", "eps_hop")]


_lib = None


def build(force: bool = False) -> str:
    """Compiles the generator with gcc (plain C, OpenMP over sets)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.chaingen_count.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p]
        lib.chaingen_count.restype = ctypes.c_int
        lib.chaingen_fill.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Out)]
        lib.chaingen_fill.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def generate(params: GenParams | str, n_sets: int, set_begin: int = 0,
             seed: int | None = None) -> ChainSets:
    """Sets ``set_begin .. set_begin+n_sets-1`` of the stream ``params``."""
    if isinstance(params, str):
        params = PRESETS[params]
    if seed is not None:
        params = params.replace(seed=seed)
    lib = _load()
    p = _Params(
        seed=params.seed & (2**64 - 1), set_begin=set_begin, n_sets=n_sets,
        chains_lo=params.chains[0], chains_hi=params.chains[1],
        cbs_lo=params.cbs[0], cbs_hi=params.cbs[1], n_exec=params.n_exec,
        n_accel=params.n_accel, max_seg_per_cb=params.max_seg_per_cb,
        n_buckets=params.n_buckets, util_lo=params.util[0], util_hi=params.util[1],
        pseg_lo=params.pseg[0], pseg_hi=params.pseg[1], frac_lo=params.frac[0],
        frac_hi=params.frac[1], T_lo=params.T[0], T_hi=params.T[1],
        spin_prob=params.spin_prob, eps=params.eps, kappa=params.kappa, eps_hop=params.eps_hop,
        exec_per_chain=1 if params.exec_per_chain else 0, own_cores=1 if params.own_cores else 0)
    counts = np.zeros((n_sets, 3), dtype=np.int64)
    if lib.chaingen_count(ctypes.byref(p), _ptr(counts)) != 0:
        raise ValueError("invalid generator parameters")
    off = np.zeros((3, n_sets + 1), dtype=np.int64)
    np.cumsum(counts, axis=0, out=off[:, 1:].T)
    nC, nJ, nG = (int(v) for v in off[:, -1])
    X, NA = params.n_exec, params.n_accel
    cs = ChainSets(
        n_sets=n_sets,
        set_chain_off=np.ascontiguousarray(off[0]),
        set_exec_off=np.arange(n_sets + 1, dtype=np.int64) * X,
        set_accel_off=np.arange(n_sets + 1, dtype=np.int64) * NA,
        chain_cb_off=np.zeros(nC + 1, np.int64), cb_seg_off=np.zeros(nJ + 1, np.int64),
        T=np.zeros(nC, np.int64), D=np.zeros(nC, np.int64), prio=np.zeros(nC, np.int32),
        spin=np.zeros(nC, np.uint8), E=np.zeros(nJ, np.int64), exec=np.zeros(nJ, np.int16),
        A=np.zeros(nG, np.int64), accel=np.zeros(nG, np.int16),
        exec_core=np.zeros(n_sets * X, np.int16), exec_prio=np.zeros(n_sets * X, np.int32),
        accel_buckets=np.zeros(n_sets * NA, np.int16), accel_eps=np.zeros(n_sets * NA, np.int64),
        accel_kappa=np.zeros(n_sets * NA, np.int64), eps_hop=np.zeros(n_sets, np.int64),
        meta={"params": params, "set_begin": set_begin})
    set_cb_off = np.ascontiguousarray(off[1])
    set_seg_off = np.ascontiguousarray(off[2])
    o = _Out(set_chain_off=_ptr(cs.set_chain_off), set_cb_off=_ptr(set_cb_off),
             set_seg_off=_ptr(set_seg_off), chain_cb_off=_ptr(cs.chain_cb_off),
             cb_seg_off=_ptr(cs.cb_seg_off), T=_ptr(cs.T), D=_ptr(cs.D), prio=_ptr(cs.prio),
             spin=_ptr(cs.spin), E=_ptr(cs.E), exec=_ptr(cs.exec), A=_ptr(cs.A),
             accel=_ptr(cs.accel), exec_core=_ptr(cs.exec_core), exec_prio=_ptr(cs.exec_prio),
             accel_buckets=_ptr(cs.accel_buckets), accel_eps=_ptr(cs.accel_eps),
             accel_kappa=_ptr(cs.accel_kappa), eps_hop=_ptr(cs.eps_hop))
    if n_sets > 0:
        rc = lib.chaingen_fill(ctypes.byref(p), ctypes.byref(o))
        if rc != 0:
            raise RuntimeError("chaingen_fill failed (%d)" % rc)
    return cs


# ------------------------------------------------- random inputs of the ranking
# Draws that the surrogate part consumes as inputs: initial network parameters,
# the (set, candidate) pairs of a training run, and synthetic score vectors.
# Parameter layout: W1 [256][48] | b1 [256] | W2 [256][256] | b2 [256] |
# w3 [256] | b3 [1] (78,593 float32 values).
MLP_SHAPES = (((256, 48), 48), ((256,), 0), ((256, 256), 256), ((256,), 0), ((256,), 256),
              ((1,), 0))
MLP_PARAMS = 78593


def mlp_init(seed: int) -> np.ndarray:
    """He-uniform weights (limit sqrt(6 / fan_in)) and zero biases, float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, fan_in in MLP_SHAPES:
        if fan_in == 0:
            parts.append(np.zeros(shape))
        else:
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, size=shape))
    out = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert out.size == MLP_PARAMS
    return out


def training_pairs(n_sets: int, n_samples: int, n_cand: int, seed: int) -> np.ndarray:
    """int64 [n_samples, 2]: (set, candidate k) drawn uniformly."""
    rng = np.random.default_rng(seed)
    out = np.empty((n_samples, 2), np.int64)
    out[:, 0] = rng.integers(0, n_sets, n_samples)
    out[:, 1] = rng.integers(0, n_cand, n_samples)
    return out


def random_scores(n: int, seed: int, ties: bool = False) -> np.ndarray:
    """float32 [n] synthetic scores; with ``ties`` drawn from 8 values only."""
    rng = np.random.default_rng(seed)
    if ties:
        return rng.integers(0, 8, n).astype(np.float32) / 4.0
    return rng.uniform(0.0, 2.0, n).astype(np.float32)


def training_triples(n_sets: int, n_samples: int, n_cand: int, util_range: tuple[int, int],
                     seed: int) -> np.ndarray:
    """int64 [n_samples, 3]: (set, candidate k, util_permille), set and k
    uniform, util_permille log-uniform over util_range (integers)."""
    rng = np.random.default_rng(seed)
    out = np.empty((n_samples, 3), np.int64)
    out[:, 0] = rng.integers(0, n_sets, n_samples)
    out[:, 1] = rng.integers(0, n_cand, n_samples)
    lo, hi = np.log(util_range[0]), np.log(util_range[1] + 1)
    out[:, 2] = np.clip(np.floor(np.exp(rng.uniform(lo, hi, n_samples))), util_range[0],
                        util_range[1]).astype(np.int64)
    return out


def shuffle_order(n: int, seed: int) -> np.ndarray:
    """int64 [n]: a seeded permutation (the visiting order of one epoch)."""
    return np.random.default_rng(seed).permutation(n).astype(np.int64)


def release_offsets(cs: ChainSets, n_scen: int, seed: int) -> np.ndarray:
    """First release of every chain in every scenario of a simulation:
    scenario 0 releases every chain at 0 (the synchronous release), the
    others uniformly in [0, T_c).  Layout: per set a [n_scen][C] block at
    set_chain_off[set] * n_scen."""
    rng = np.random.default_rng(seed)
    out = np.empty(int(cs.set_chain_off[-1]) * n_scen, np.int64)
    for s in range(cs.n_sets):
        c0, c1 = int(cs.set_chain_off[s]), int(cs.set_chain_off[s + 1])
        T = np.asarray(cs.T[c0:c1], np.int64)
        blk = (rng.random((n_scen, c1 - c0)) * T).astype(np.int64)
        blk[0] = 0
        out[c0 * n_scen:c1 * n_scen] = blk.ravel()
    return out
