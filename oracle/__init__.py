"""CPU oracle of the PAAM response-time analysis -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never touches it.

``paam_oracle.c`` is a plain single-threaded C implementation of the paper's
Sec. IV-F analysis.  This module compiles it with gcc and exposes it on numpy
arrays of any object with the ``ChainSets`` attribute names (the generator's
output); it does not import the generator or the product package.

Other oracle modules: ``des`` (a discrete-event simulator used as a brute-force
soundness pin), ``features`` and ``mlp`` (FP64 references of the surrogate's
features and network).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "paam_oracle.c")
_SRC_DES = os.path.join(_HERE, "paam_des.c")
_HDR = os.path.join(_HERE, "paam_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")

INF = np.iinfo(np.int64).max
BLOCK_SAFE, BLOCK_PAPER = 0, 1
BOUND_MIN, BOUND_L2, BOUND_L3 = 0, 1, 2


class _CS(ctypes.Structure):
    _fields_ = [("n_sets", ctypes.c_int64)] + [(n, ctypes.c_void_p) for n in (
        "set_chain_off", "set_exec_off", "set_accel_off", "chain_cb_off", "cb_seg_off", "T", "D",
        "prio", "spin", "E", "exec", "A", "accel", "exec_core", "exec_prio", "accel_buckets",
        "accel_eps", "accel_kappa", "eps_hop")]


class _Opts(ctypes.Structure):
    _fields_ = [("blocking", ctypes.c_int32), ("cap_mult", ctypes.c_int32),
                ("util_permille", ctypes.c_int32), ("full", ctypes.c_int32),
                ("bound", ctypes.c_int32)]


class _DesOpts(ctypes.Structure):
    _fields_ = [("n_scen", ctypes.c_int32), ("horizon", ctypes.c_int64),
                ("exec_permille", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("util_permille", ctypes.c_int32), ("max_steps", ctypes.c_int64)]


_DTYPES = {
    "set_chain_off": np.int64, "set_exec_off": np.int64, "set_accel_off": np.int64,
    "chain_cb_off": np.int64, "cb_seg_off": np.int64, "T": np.int64, "D": np.int64,
    "prio": np.int32, "spin": np.uint8, "E": np.int64, "exec": np.int16, "A": np.int64,
    "accel": np.int16, "exec_core": np.int16, "exec_prio": np.int32, "accel_buckets": np.int16,
    "accel_eps": np.int64, "accel_kappa": np.int64, "eps_hop": np.int64,
}

_lib = None


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_DES), os.path.getmtime(_HDR))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp,
                               _SRC, _SRC_DES])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_analyse_set.argtypes = [ctypes.POINTER(_CS), ctypes.c_int64, P,
                                           ctypes.POINTER(_Opts), P, P, P, P, P]
        lib.oracle_segment_H.argtypes = [ctypes.POINTER(_CS), ctypes.c_int64, P,
                                         ctypes.POINTER(_Opts), P]
        lib.oracle_wcrt_range.argtypes = [ctypes.POINTER(_CS), ctypes.POINTER(_Opts),
                                          ctypes.c_int64, ctypes.c_int64, P, P, P, P, P]
        lib.oracle_candidate_order.argtypes = [ctypes.POINTER(_CS), ctypes.c_int64,
                                               ctypes.c_uint64, ctypes.c_int64, P]
        lib.oracle_search_range.argtypes = [ctypes.POINTER(_CS), ctypes.POINTER(_Opts),
                                            ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                                            ctypes.c_int64, P, P, P]
        lib.oracle_wfd_range.argtypes = [ctypes.POINTER(_CS), P, ctypes.c_int32, ctypes.c_int64,
                                         ctypes.c_int64, P]
        lib.oracle_des_range.argtypes = [ctypes.POINTER(_CS), ctypes.POINTER(_DesOpts), P,
                                         ctypes.c_int64, ctypes.c_int64, P, P]
        for f in ("oracle_analyse_set", "oracle_segment_H", "oracle_wcrt_range",
                  "oracle_candidate_order", "oracle_search_range", "oracle_wfd_range",
                  "oracle_des_range"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


class _Bound:
    """Keeps contiguous copies alive while C holds pointers to them."""

    def __init__(self, cs):
        self.arrays = {k: np.ascontiguousarray(getattr(cs, k), dtype=t) for k, t in _DTYPES.items()}
        self.s = _CS(n_sets=int(cs.n_sets), **{k: v.ctypes.data for k, v in self.arrays.items()})


def _opts(blocking=BLOCK_SAFE, cap_mult=1, util_permille=1000, full=False, bound=BOUND_MIN):
    return _Opts(blocking=blocking, cap_mult=cap_mult, util_permille=util_permille,
                 full=1 if full else 0, bound=bound)


def _ranges(n, parts):
    parts = max(1, min(parts, n))
    edges = np.linspace(0, n, parts + 1).astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def wcrt(cs, blocking=BLOCK_SAFE, cap_mult=1, util_permille=1000, full=False, bound=BOUND_MIN,
         sets=None, threads=1):
    """Analyses sets (all, or the range ``sets=(lo, hi)``).

    Returns a dict: ``chain_R`` [n_chains] (INF past the cap, -1 where a
    verdict-mode analysis stopped early), ``sched`` / ``worst`` / ``worst_R``
    / ``terms`` [n_sets] (entries outside the range are left at their fill)."""
    lib = _load()
    b = _Bound(cs)
    o = _opts(blocking, cap_mult, util_permille, full, bound)
    n = int(cs.n_sets)
    lo, hi = (0, n) if sets is None else sets
    out = {
        "chain_R": np.full(int(cs.set_chain_off[-1]), -1, np.int64),
        "sched": np.zeros(n, np.int8), "worst": np.full(n, -1, np.int32),
        "worst_R": np.full(n, -1, np.int64), "terms": np.zeros(n, np.int64),
    }
    ptrs = [out[k].ctypes.data for k in ("chain_R", "sched", "worst", "worst_R", "terms")]

    def run(r):
        rc = lib.oracle_wcrt_range(ctypes.byref(b.s), ctypes.byref(o), r[0], r[1], *ptrs)
        if rc != 0:
            raise ValueError("oracle rejected a set in [%d, %d)" % r)

    if threads <= 1:
        run((lo, hi))
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(run, [(lo + a, lo + b_) for a, b_ in _ranges(hi - lo, 8 * threads)]))
    return out


def analyse_set(cs, s, order=None, **kw):
    """One set under an explicit priority order (chain ids, highest first)."""
    lib = _load()
    b = _Bound(cs)
    o = _opts(**kw)
    C = int(cs.set_chain_off[s + 1] - cs.set_chain_off[s])
    R = np.zeros(C, np.int64)
    sched, worst, wR, terms = (np.zeros(1, t) for t in (np.int8, np.int32, np.int64, np.int64))
    op = None
    if order is not None:
        order = np.ascontiguousarray(order, np.int32)
        op = order.ctypes.data
    rc = lib.oracle_analyse_set(ctypes.byref(b.s), s, op, ctypes.byref(o), R.ctypes.data,
                                sched.ctypes.data, worst.ctypes.data, wR.ctypes.data,
                                terms.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected set %d" % s)
    return {"chain_R": R, "sched": int(sched[0]), "worst": int(worst[0]),
            "worst_R": int(wR[0]), "terms": int(terms[0])}


def segment_H(cs, s, order=None, **kw):
    lib = _load()
    b = _Bound(cs)
    o = _opts(**kw)
    c0, c1 = int(cs.set_chain_off[s]), int(cs.set_chain_off[s + 1])
    g0 = int(cs.cb_seg_off[cs.chain_cb_off[c0]])
    g1 = int(cs.cb_seg_off[cs.chain_cb_off[c1]])
    H = np.zeros(g1 - g0, np.int64)
    op = None
    if order is not None:
        order = np.ascontiguousarray(order, np.int32)
        op = order.ctypes.data
    if lib.oracle_segment_H(ctypes.byref(b.s), s, op, ctypes.byref(o), H.ctypes.data) != 0:
        raise ValueError("oracle rejected set %d" % s)
    return H


def candidate_order(cs, s, seed, k):
    lib = _load()
    b = _Bound(cs)
    C = int(cs.set_chain_off[s + 1] - cs.set_chain_off[s])
    order = np.zeros(C, np.int32)
    if lib.oracle_candidate_order(ctypes.byref(b.s), s, seed & (2**64 - 1), k,
                                  order.ctypes.data) != 0:
        raise ValueError("bad candidate request")
    return order


def search(cs, n_cand, seed, blocking=BLOCK_SAFE, cap_mult=1, util_permille=1000, sets=None,
           threads=1):
    """Plain search: smallest k in [0, n_cand) whose order meets all deadlines."""
    lib = _load()
    b = _Bound(cs)
    o = _opts(blocking, cap_mult, util_permille, False, BOUND_MIN)
    n = int(cs.n_sets)
    lo, hi = (0, n) if sets is None else sets
    found = np.full(n, -1, np.int32)
    n_eval = np.zeros(n, np.int32)
    terms = np.zeros(n, np.int64)

    def run(r):
        rc = lib.oracle_search_range(ctypes.byref(b.s), ctypes.byref(o), n_cand,
                                     seed & (2**64 - 1), r[0], r[1], found.ctypes.data,
                                     n_eval.ctypes.data, terms.ctypes.data)
        if rc != 0:
            raise ValueError("oracle rejected a set in [%d, %d)" % r)

    if threads <= 1:
        run((lo, hi))
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(run, [(lo + a, lo + b_) for a, b_ in _ranges(hi - lo, 8 * threads)]))
    return {"found": found, "n_eval": n_eval, "terms": terms}


def candidate_analysis(cs, pairs, seed, cap_mult=2, blocking=BLOCK_SAFE, bound=BOUND_MIN):
    """Exact analysis of (set, k, util_permille) triples: every chain's bound
    at cap cap_mult * D under candidate order k.  Returns sched, worst_R,
    worst_D and ratio = min(worst_R / worst_D, cap_mult) rounded to float32."""
    pairs = np.asarray(pairs, np.int64).reshape(-1, 3)
    n = len(pairs)
    out = {"sched": np.zeros(n, np.int8), "worst_R": np.zeros(n, np.int64),
           "worst_D": np.zeros(n, np.int64), "ratio": np.zeros(n, np.float32)}
    for i, (s, k, u) in enumerate(pairs):
        order = candidate_order(cs, int(s), seed, int(k))
        r = analyse_set(cs, int(s), order=order, full=True, cap_mult=cap_mult,
                        util_permille=int(u), blocking=blocking, bound=bound)
        c0 = int(cs.set_chain_off[s])
        w = r["worst"]
        D = int(cs.D[c0 + w])
        out["sched"][i] = r["sched"]
        out["worst_R"][i] = r["worst_R"]
        out["worst_D"][i] = D
        ratio = float(cap_mult) if r["worst_R"] == INF else min(float(r["worst_R"]) / float(D),
                                                                 float(cap_mult))
        out["ratio"][i] = np.float32(ratio)
    return out


def score_order(scores):
    """Candidate indices by ascending score, ties to the lower index; -0.0
    sorts before +0.0 and every NaN after all numbers (IEEE total order on
    the float32 values)."""
    s = np.asarray(scores, np.float32)
    keys = []
    for k, v in enumerate(s):
        if np.isnan(v):
            key = (1, 0.0, 0)
        else:
            key = (0, float(v), 0 if (v == 0.0 and np.signbit(v)) else 1)
        keys.append((key, k))
    return [k for _, k in sorted(keys)]


def guided_search(cs, n_cand, seed, scores, top_k, fallback=True, blocking=BLOCK_SAFE,
                  util_permille=1000, sets=None):
    """Guided search: the top_k candidates by score (score_order) analysed in
    that order; the first feasible one wins.  With fallback, the remaining
    candidates follow in index order.  scores: [n_sets * n_cand]."""
    scores = np.asarray(scores, np.float32).reshape(-1, n_cand)
    n = int(cs.n_sets)
    lo, hi = (0, n) if sets is None else sets
    found = np.full(n, -1, np.int32)
    n_eval = np.zeros(n, np.int32)
    for s in range(lo, hi):
        top = score_order(scores[s])[:min(top_k, n_cand)]
        seq = list(top)
        if fallback:
            chosen = set(top)
            seq += [k for k in range(n_cand) if k not in chosen]
        for k in seq:
            r = analyse_set(cs, s, order=candidate_order(cs, s, seed, k), full=False,
                            util_permille=util_permille, blocking=blocking)
            n_eval[s] += 1
            if r["sched"] != 0:
                found[s] = k if r["sched"] > 0 else -2
                break
    return {"found": found, "n_eval": n_eval}


UNITS_SEGMENT, UNITS_CALLBACK, UNITS_CHAIN = 0, 1, 2


def wfd_units(cs, units, group=UNITS_SEGMENT):
    """Worst-fit-decreasing binding of every segment to a unit of its
    accelerator type (Sec. IV-E, Managing Multiple Accelerators).

    ``units`` [n_accels]: units of each accelerator type; ``group``: an item
    is a segment, or a callback's or a chain's segments on one type.  Returns
    the set-local unit of every segment [n_segments]; the units of a set are
    numbered type by type."""
    lib = _load()
    b = _Bound(cs)
    u = np.ascontiguousarray(units, dtype=np.int16)
    out = np.full(int(cs.cb_seg_off[-1]), -1, np.int16)
    if lib.oracle_wfd_range(ctypes.byref(b.s), u.ctypes.data, int(group), 0, int(cs.n_sets),
                            out.ctypes.data) != 0:
        raise ValueError("oracle rejected the unit counts")
    return out


class _Split:
    pass


def split_units(cs, units, seg_unit):
    """The batch whose accelerators are the units: segment g runs on unit
    ``seg_unit[g]``; every unit keeps its type's buckets and overheads."""
    units = np.asarray(units, np.int64)
    out = _Split()
    for k in _DTYPES:
        setattr(out, k, np.asarray(getattr(cs, k)).copy())
    out.n_sets = int(cs.n_sets)
    out.accel = np.asarray(seg_unit, np.int16).copy()
    out.accel_buckets = np.repeat(np.asarray(cs.accel_buckets), units).astype(np.int16)
    out.accel_eps = np.repeat(np.asarray(cs.accel_eps), units).astype(np.int64)
    out.accel_kappa = np.repeat(np.asarray(cs.accel_kappa), units).astype(np.int64)
    per_set = np.add.reduceat(units, np.asarray(cs.set_accel_off[:-1])) if len(units) else \
        np.zeros(0, np.int64)
    off = np.asarray(cs.set_accel_off)
    counts = np.where(off[1:] > off[:-1], per_set[:len(off) - 1] if len(per_set) else 0, 0)
    out.set_accel_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return out


def event_sim(cs, offsets, n_scen, horizon, exec_permille=1000, seed=0, util_permille=1000,
        max_steps=1 << 40, sets=None, threads=1):
    """Event-driven simulation (paam_des.c) of sets (all, or ``sets=(lo, hi)``).

    ``offsets`` [n_chains * n_scen]: first releases, per set a [n_scen][C]
    block at ``set_chain_off[set] * n_scen``.  Returns ``obs`` (same layout:
    largest observed response, -1 none) and ``status`` [n_sets * n_scen]."""
    lib = _load()
    b = _Bound(cs)
    o = _DesOpts(n_scen=n_scen, horizon=horizon, exec_permille=exec_permille,
                 seed=seed & (2**64 - 1), util_permille=util_permille, max_steps=max_steps)
    n = int(cs.n_sets)
    lo, hi = (0, n) if sets is None else sets
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    obs = np.full(int(cs.set_chain_off[-1]) * n_scen, -1, np.int64)
    status = np.full(n * n_scen, -1, np.int8)

    def run(r):
        if lib.oracle_des_range(ctypes.byref(b.s), ctypes.byref(o), off.ctypes.data, r[0], r[1],
                                obs.ctypes.data, status.ctypes.data) != 0:
            raise ValueError("oracle simulation rejected a set in [%d, %d)" % r)

    if threads <= 1:
        run((lo, hi))
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(run, [(lo + a, lo + b_) for a, b_ in _ranges(hi - lo, 8 * threads)]))
    return {"obs": obs, "status": status}
