"""ctypes binding of libpaam (include/paam.h): argument marshalling only.

Every step of the analysis runs in the HIP kernels of libpaam.so.  PyTorch
supplies device memory (the arena, workspaces, outputs) and streams.  There is
no fallback: if the library is missing or the device is not gfx950 the calls
raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIBPAAM = os.path.join(PKG, "libpaam.so")

PAAM_OK = 0
PAAM_INF = np.iinfo(np.int64).max
PAAM_BLOCK_SAFE, PAAM_BLOCK_PAPER = 0, 1
PAAM_BOUND_MIN, PAAM_BOUND_L2, PAAM_BOUND_L3 = 0, 1, 2

EXPORTED = (
    "paam_chainset_bytes", "paam_chainset_upload", "paam_chainset_free", "paam_chainset_info",
    "paam_assign_units", "paam_chainset_seg_units", "paam_des_batch",
    "paam_wcrt_bytes", "paam_wcrt_batch", "paam_wcrt_batch_noalloc", "paam_wcrt_autotune",
    "paam_wcrt_schedule",
    "paam_search_bytes",
    "paam_priority_search", "paam_candidate_bytes", "paam_candidate_wcrt", "paam_features_bytes", "paam_features",
    "paam_mlp_pack", "paam_mlp_forward", "paam_mlp_backward_bytes", "paam_mlp_backward",
    "paam_mlp_adam_step", "paam_score_bytes", "paam_score_candidates",
    "paam_last_error", "paam_version",
)
N_FEAT = 48
MLP_PARAMS = 78593
MLP_PACKED = 82176


class PaamError(RuntimeError):
    pass


class paam_chainset_host(ctypes.Structure):
    _fields_ = [("n_sets", ctypes.c_int64)] + [(n, ctypes.c_void_p) for n in (
        "set_chain_off", "set_exec_off", "set_accel_off", "chain_cb_off", "cb_seg_off", "T", "D",
        "prio", "spin", "E", "exec", "A", "accel", "exec_core", "exec_prio", "accel_buckets",
        "accel_eps", "accel_kappa", "eps_hop", "accel_units")] + [("unit_group", ctypes.c_int32)]


PAAM_UNITS_SEGMENT, PAAM_UNITS_CALLBACK, PAAM_UNITS_CHAIN = 0, 1, 2


class paam_des_opts(ctypes.Structure):
    _fields_ = [("n_scen", ctypes.c_int32), ("exec_permille", ctypes.c_int32),
                ("horizon", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("util_permille", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("max_steps", ctypes.c_int64)]

class paam_wcrt_opts(ctypes.Structure):
    _fields_ = [("blocking", ctypes.c_int32), ("cap_mult", ctypes.c_int32),
                ("util_permille", ctypes.c_int32), ("full", ctypes.c_int32),
                ("bound", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32)]


class paam_search_opts(ctypes.Structure):
    _fields_ = [("n_cand", ctypes.c_int32), ("guided", ctypes.c_int32), ("top_k", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("d_scores", ctypes.c_void_p), ("wcrt", paam_wcrt_opts)]


_lib = None


def lib():
    """Loads libpaam.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPAAM):
            raise PaamError("libpaam.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIBPAAM)
        P, S = ctypes.c_void_p, ctypes.c_size_t
        L.paam_chainset_bytes.argtypes = [ctypes.POINTER(paam_chainset_host), ctypes.POINTER(S)]
        L.paam_chainset_upload.argtypes = [ctypes.POINTER(paam_chainset_host), P, S, P,
                                           ctypes.POINTER(P)]
        L.paam_chainset_free.argtypes = [P]
        L.paam_chainset_free.restype = None
        L.paam_chainset_info.argtypes = [P, P]
        L.paam_assign_units.argtypes = [P, P]
        L.paam_des_batch.argtypes = [P, ctypes.POINTER(paam_des_opts), P, P, P, P]
        L.paam_chainset_seg_units.argtypes = [P, P, P]
        L.paam_wcrt_bytes.argtypes = [P, ctypes.POINTER(paam_wcrt_opts), ctypes.POINTER(S)]
        L.paam_wcrt_batch.argtypes = [P, ctypes.POINTER(paam_wcrt_opts), P, P, P, P, P, S, P]
        L.paam_wcrt_batch_noalloc.argtypes = [P, ctypes.POINTER(paam_wcrt_opts), P, P, P, P, P]
        L.paam_wcrt_autotune.argtypes = [P, ctypes.POINTER(paam_wcrt_opts), P, ctypes.c_int32,
                                          ctypes.c_int32, P, P, P, P, P, S, P,
                                          ctypes.POINTER(ctypes.c_float)]
        L.paam_wcrt_autotune.restype = ctypes.c_int32
        L.paam_wcrt_schedule.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.paam_wcrt_schedule.restype = ctypes.c_int32
        L.paam_search_bytes.argtypes = [P, ctypes.POINTER(paam_search_opts), ctypes.POINTER(S)]
        L.paam_priority_search.argtypes = [P, ctypes.POINTER(paam_search_opts), P, P, P, P, S, P]
        I64, I32, U64, F = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_float
        L.paam_candidate_bytes.argtypes = [P, ctypes.POINTER(paam_wcrt_opts), I64,
                                           ctypes.POINTER(S)]
        L.paam_candidate_wcrt.argtypes = [P, ctypes.POINTER(paam_wcrt_opts), U64, P, I64, P, P, P,
                                          P, P, S, P]
        L.paam_features_bytes.argtypes = [P, I64, ctypes.POINTER(S)]
        L.paam_features.argtypes = [P, U64, P, I64, I32, P, P, P, S, P]
        L.paam_mlp_pack.argtypes = [P, P, P]
        L.paam_mlp_forward.argtypes = [P, P, P, P, I64, I32, P, P, P]
        L.paam_mlp_backward_bytes.argtypes = [I64, ctypes.POINTER(S)]
        L.paam_mlp_backward.argtypes = [P, P, P, P, I64, I32, P, P, P, P, P, P, S, P]
        L.paam_mlp_adam_step.argtypes = [P, P, P, P, P, F, F, F, F, I64, P]
        L.paam_score_bytes.argtypes = [P, ctypes.POINTER(paam_search_opts), ctypes.POINTER(S)]
        L.paam_score_candidates.argtypes = [P, ctypes.POINTER(paam_search_opts), P, P, P, P, S, P]
        for f in ("paam_candidate_bytes", "paam_candidate_wcrt", "paam_features_bytes",
                  "paam_features", "paam_mlp_pack", "paam_mlp_forward", "paam_mlp_backward_bytes",
                  "paam_mlp_backward", "paam_mlp_adam_step", "paam_score_bytes",
                  "paam_score_candidates"):
            getattr(L, f).restype = ctypes.c_int32
        L.paam_last_error.argtypes = []
        L.paam_last_error.restype = ctypes.c_char_p
        L.paam_version.argtypes = []
        L.paam_version.restype = ctypes.c_char_p
        for f in ("paam_chainset_bytes", "paam_chainset_upload", "paam_chainset_info",
                  "paam_assign_units", "paam_chainset_seg_units", "paam_des_batch",
                  "paam_wcrt_bytes", "paam_wcrt_batch", "paam_wcrt_batch_noalloc", "paam_search_bytes",
                  "paam_priority_search"):
            getattr(L, f).restype = ctypes.c_int32
        _lib = L
    return _lib


def check(status: int, what: str) -> None:
    if status != PAAM_OK:
        msg = lib().paam_last_error().decode(errors="replace")
        raise PaamError("%s failed (%d): %s" % (what, status, msg))


_HOST_DTYPES = {
    "set_chain_off": np.int64, "set_exec_off": np.int64, "set_accel_off": np.int64,
    "chain_cb_off": np.int64, "cb_seg_off": np.int64, "T": np.int64, "D": np.int64,
    "prio": np.int32, "spin": np.uint8, "E": np.int64, "exec": np.int16, "A": np.int64,
    "accel": np.int16, "exec_core": np.int16, "exec_prio": np.int32, "accel_buckets": np.int16,
    "accel_eps": np.int64, "accel_kappa": np.int64, "eps_hop": np.int64,
}


class HostBatch:
    """paam_chainset_host over contiguous numpy copies of a CSR batch.

    units: None, or the units of every accelerator type [n_accels]
    (Sec. IV-E); group: PAAM_UNITS_* (what the bin packing keeps together)."""

    def __init__(self, cs, units=None, group=PAAM_UNITS_SEGMENT):
        self.arrays = {k: np.ascontiguousarray(getattr(cs, k), dtype=t)
                       for k, t in _HOST_DTYPES.items()}
        self.n_sets = int(cs.n_sets)
        ptrs = {k: v.ctypes.data for k, v in self.arrays.items()}
        if units is not None:
            self.arrays["accel_units"] = np.ascontiguousarray(units, dtype=np.int16)
            ptrs["accel_units"] = self.arrays["accel_units"].ctypes.data
        self.struct = paam_chainset_host(n_sets=self.n_sets, unit_group=int(group), **ptrs)


def _stream_ptr(stream) -> int | None:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


class Chainset:
    """An uploaded batch: the device arena (a torch uint8 tensor) and the
    opaque library handle."""

    def __init__(self, cs, device="cuda:0", stream=None, units=None,
                 unit_group=PAAM_UNITS_SEGMENT):
        import torch
        self.host = HostBatch(cs, units, unit_group)
        n = ctypes.c_size_t(0)
        check(lib().paam_chainset_bytes(ctypes.byref(self.host.struct), ctypes.byref(n)),
              "paam_chainset_bytes")
        self.arena = torch.empty(int(n.value), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p(0)
        check(lib().paam_chainset_upload(ctypes.byref(self.host.struct), self.arena.data_ptr(),
                                         int(n.value), _stream_ptr(stream), ctypes.byref(h)),
              "paam_chainset_upload")
        self.handle = h
        self.device = device
        info = np.zeros(8, np.int64)
        check(lib().paam_chainset_info(self.handle, info.ctypes.data), "paam_chainset_info")
        (self.n_sets, self.n_chains, self.n_callbacks, self.n_segments, self.n_subchains,
         self.max_chains, self.max_subchains, self.max_segments) = (int(v) for v in info)

    def assign_units(self, stream=None):
        """Re-runs the unit binding on the device (paam_assign_units)."""
        check(lib().paam_assign_units(self.handle, _stream_ptr(stream)), "paam_assign_units")

    def seg_units(self, stream=None):
        """The analysed accelerator (set-local unit) of every segment, int16."""
        import torch
        out = torch.empty(max(self.n_segments, 1), dtype=torch.int16, device=self.device)
        check(lib().paam_chainset_seg_units(self.handle, out.data_ptr(), _stream_ptr(stream)),
              "paam_chainset_seg_units")
        return out[:self.n_segments]

    def free(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().paam_chainset_free(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def wcrt_opts(blocking=PAAM_BLOCK_SAFE, cap_mult=1, util_permille=1000, full=True,
              bound=PAAM_BOUND_MIN, waves_per_cu=0) -> paam_wcrt_opts:
    return paam_wcrt_opts(blocking=blocking, cap_mult=cap_mult, util_permille=util_permille,
                          full=1 if full else 0, bound=bound, waves_per_cu=waves_per_cu)


def paam_wcrt_bytes(cs: Chainset, opts: paam_wcrt_opts) -> int:
    n = ctypes.c_size_t(0)
    check(lib().paam_wcrt_bytes(cs.handle, ctypes.byref(opts), ctypes.byref(n)), "paam_wcrt_bytes")
    return int(n.value)


class WcrtOut:
    def __init__(self, cs: Chainset, full: bool):
        import torch
        d = cs.device
        self.set_sched = torch.empty(cs.n_sets, dtype=torch.int8, device=d)
        self.set_worst = torch.empty(cs.n_sets, dtype=torch.int32, device=d)
        self.set_worst_R = torch.empty(cs.n_sets, dtype=torch.int64, device=d)
        self.chain_R = torch.empty(max(cs.n_chains, 1), dtype=torch.int64, device=d) if full else None


def paam_wcrt_batch(cs: Chainset, opts: paam_wcrt_opts, out: WcrtOut, ws, stream=None) -> None:
    check(lib().paam_wcrt_batch(cs.handle, ctypes.byref(opts), out.set_sched.data_ptr(),
                                out.set_worst.data_ptr(), out.set_worst_R.data_ptr(),
                                _dev_ptr(out.chain_R), ws.data_ptr(), ws.numel(),
                                _stream_ptr(stream)),
          "paam_wcrt_batch")


def paam_wcrt_batch_noalloc(cs: Chainset, opts: paam_wcrt_opts, out: WcrtOut, stream=None) -> None:
    check(lib().paam_wcrt_batch_noalloc(cs.handle, ctypes.byref(opts), out.set_sched.data_ptr(),
                                        out.set_worst.data_ptr(), out.set_worst_R.data_ptr(),
                                        _dev_ptr(out.chain_R), _stream_ptr(stream)),
          "paam_wcrt_batch_noalloc")


def paam_wcrt_autotune(cs: Chainset, opts: paam_wcrt_opts, candidates, reps: int, out: WcrtOut,
                       ws, stream=None) -> float:
    """Sets opts.waves_per_cu to the fastest of the candidates; returns its
    mean launch time in ms."""
    cand = np.ascontiguousarray(candidates, np.int32)
    best = ctypes.c_float(0.0)
    check(lib().paam_wcrt_autotune(cs.handle, ctypes.byref(opts), cand.ctypes.data, len(cand), reps,
                                   out.set_sched.data_ptr(), out.set_worst.data_ptr(),
                                   out.set_worst_R.data_ptr(), _dev_ptr(out.chain_R),
                                   ws.data_ptr(), ws.numel(), _stream_ptr(stream),
                                   ctypes.byref(best)),
          "paam_wcrt_autotune")
    return float(best.value)


def paam_wcrt_schedule(cs: Chainset) -> list:
    """Per size class: (largest chain count, sets, waves per CU, evaluations
    per engine step) used when waves_per_cu is 0."""
    buf = np.zeros((16, 4), np.int32)
    n = ctypes.c_int32(0)
    check(lib().paam_wcrt_schedule(cs.handle, buf.ctypes.data, 16, ctypes.byref(n)),
          "paam_wcrt_schedule")
    return [tuple(int(v) for v in buf[k]) for k in range(min(n.value, 16))]


def workspace(nbytes: int, device="cuda:0"):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def wcrt(cs: Chainset, stream=None, **kw) -> dict:
    """One analysis of an uploaded batch; returns host numpy arrays."""
    import torch
    o = wcrt_opts(**kw)
    out = WcrtOut(cs, bool(o.full))
    ws = workspace(paam_wcrt_bytes(cs, o), cs.device)
    paam_wcrt_batch(cs, o, out, ws, stream)
    _sync(cs.device)
    res = {"sched": out.set_sched.cpu().numpy(), "worst": out.set_worst.cpu().numpy(),
           "worst_R": out.set_worst_R.cpu().numpy()}
    if out.chain_R is not None:
        res["chain_R"] = out.chain_R.cpu().numpy()[:cs.n_chains]
    return res


def search_opts(n_cand, seed, guided=False, top_k=1, fallback=True, scores=None,
                **wcrt_kw) -> paam_search_opts:
    return paam_search_opts(n_cand=n_cand, guided=1 if guided else 0, top_k=top_k,
                            fallback=1 if fallback else 0, seed=seed & (2**64 - 1),
                            d_scores=None if scores is None else scores.data_ptr(),
                            wcrt=wcrt_opts(full=False, **wcrt_kw))


def paam_search_bytes(cs: Chainset, opts: paam_search_opts) -> int:
    n = ctypes.c_size_t(0)
    check(lib().paam_search_bytes(cs.handle, ctypes.byref(opts), ctypes.byref(n)),
          "paam_search_bytes")
    return int(n.value)


class SearchOut:
    def __init__(self, cs: Chainset, with_prio: bool = True):
        import torch
        d = cs.device
        self.found = torch.empty(cs.n_sets, dtype=torch.int32, device=d)
        self.n_exact = torch.empty(cs.n_sets, dtype=torch.int32, device=d)
        self.found_prio = (torch.zeros(max(cs.n_chains, 1), dtype=torch.int32, device=d)
                           if with_prio else None)


def paam_priority_search(cs: Chainset, opts: paam_search_opts, out: SearchOut, ws,
                         stream=None) -> None:
    check(lib().paam_priority_search(cs.handle, ctypes.byref(opts), out.found.data_ptr(),
                                     out.n_exact.data_ptr(), _dev_ptr(out.found_prio),
                                     ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
          "paam_priority_search")


def search(cs: Chainset, n_cand: int, seed: int, stream=None, scores=None, guided=False,
           top_k=1, fallback=True, **wcrt_kw) -> dict:
    """One priority-order search over an uploaded batch; host numpy results."""
    import torch
    o = search_opts(n_cand, seed, guided=guided, top_k=top_k, fallback=fallback, scores=scores,
                    **wcrt_kw)
    out = SearchOut(cs)
    ws = workspace(paam_search_bytes(cs, o), cs.device)
    paam_priority_search(cs, o, out, ws, stream)
    _sync(cs.device)
    return {"found": out.found.cpu().numpy(), "n_exact": out.n_exact.cpu().numpy(),
            "found_prio": out.found_prio.cpu().numpy()[:cs.n_chains]}


# ------------------------------------------------------------ candidate ranking

def _size(fn, *args) -> int:
    n = ctypes.c_size_t(0)
    check(getattr(lib(), fn)(*args, ctypes.byref(n)), fn)
    return int(n.value)


def paam_candidate_bytes(cs: Chainset, opts: paam_wcrt_opts, n_pairs: int) -> int:
    return _size("paam_candidate_bytes", cs.handle, ctypes.byref(opts), n_pairs)


class CandOut:
    def __init__(self, n: int, device):
        import torch
        self.sched = torch.empty(max(n, 1), dtype=torch.int8, device=device)
        self.worst_R = torch.empty(max(n, 1), dtype=torch.int64, device=device)
        self.worst_D = torch.empty(max(n, 1), dtype=torch.int64, device=device)
        self.ratio = torch.empty(max(n, 1), dtype=torch.float32, device=device)


def paam_candidate_wcrt(cs: Chainset, opts: paam_wcrt_opts, seed: int, pairs, out: CandOut, ws,
                        stream=None) -> None:
    n = int(pairs.shape[0])
    check(lib().paam_candidate_wcrt(cs.handle, ctypes.byref(opts), seed & (2**64 - 1),
                                    pairs.data_ptr(), n, out.sched.data_ptr(),
                                    out.worst_R.data_ptr(), out.worst_D.data_ptr(),
                                    out.ratio.data_ptr(), ws.data_ptr(), ws.numel(),
                                    _stream_ptr(stream)),
          "paam_candidate_wcrt")


def paam_features_bytes(cs: Chainset, n_pairs: int) -> int:
    return _size("paam_features_bytes", cs.handle, n_pairs)


def paam_features(cs: Chainset, seed: int, pairs, row_stride: int, feat, count, ws,
                  stream=None) -> None:
    check(lib().paam_features(cs.handle, seed & (2**64 - 1), pairs.data_ptr(),
                              int(pairs.shape[0]), row_stride, feat.data_ptr(), count.data_ptr(),
                              ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
          "paam_features")


def paam_mlp_pack(params, packed, stream=None) -> None:
    check(lib().paam_mlp_pack(params.data_ptr(), packed.data_ptr(), _stream_ptr(stream)),
          "paam_mlp_pack")


def paam_mlp_forward(params, packed, feat, count, n: int, row_stride: int, out, act=None,
                     stream=None) -> None:
    check(lib().paam_mlp_forward(params.data_ptr(), packed.data_ptr(), feat.data_ptr(),
                                 count.data_ptr(), n, row_stride, out.data_ptr(), _dev_ptr(act),
                                 _stream_ptr(stream)),
          "paam_mlp_forward")


def paam_mlp_backward_bytes(n: int) -> int:
    return _size("paam_mlp_backward_bytes", n)


def paam_mlp_backward(params, packed, feat, count, n: int, row_stride: int, out, target, act,
                      grad, loss, ws, stream=None) -> None:
    check(lib().paam_mlp_backward(params.data_ptr(), packed.data_ptr(), feat.data_ptr(),
                                  count.data_ptr(), n, row_stride, out.data_ptr(),
                                  target.data_ptr(), act.data_ptr(), grad.data_ptr(),
                                  _dev_ptr(loss), ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
          "paam_mlp_backward")


def paam_mlp_adam_step(params, packed, m, v, grad, lr, beta1, beta2, eps, step,
                       stream=None) -> None:
    check(lib().paam_mlp_adam_step(params.data_ptr(), packed.data_ptr(), m.data_ptr(),
                                   v.data_ptr(), grad.data_ptr(), lr, beta1, beta2, eps, step,
                                   _stream_ptr(stream)),
          "paam_mlp_adam_step")


def paam_score_bytes(cs: Chainset, opts: paam_search_opts) -> int:
    return _size("paam_score_bytes", cs.handle, ctypes.byref(opts))


def paam_score_candidates(cs: Chainset, opts: paam_search_opts, params, packed, scores, ws,
                          stream=None) -> None:
    check(lib().paam_score_candidates(cs.handle, ctypes.byref(opts), params.data_ptr(),
                                      packed.data_ptr(), scores.data_ptr(), ws.data_ptr(),
                                      ws.numel(), _stream_ptr(stream)),
          "paam_score_candidates")


def candidates(cs: Chainset, pairs, seed: int, stream=None, **wcrt_kw) -> dict:
    """Exact analysis of explicit (set, k, util_permille) pairs; host results."""
    import torch
    pairs = torch.as_tensor(np.ascontiguousarray(pairs, np.int64)).to(cs.device)
    o = wcrt_opts(**wcrt_kw)
    n = int(pairs.shape[0])
    out = CandOut(n, cs.device)
    ws = workspace(paam_candidate_bytes(cs, o, n), cs.device)
    paam_candidate_wcrt(cs, o, seed, pairs, out, ws, stream)
    _sync(cs.device)
    return {k: getattr(out, k).cpu().numpy()[:n] for k in ("sched", "worst_R", "worst_D", "ratio")}


def features(cs: Chainset, pairs, seed: int, row_stride=None, stream=None) -> dict:
    """Features of explicit pairs; host uint16 [n, row_stride, 48] and counts."""
    import torch
    pairs = torch.as_tensor(np.ascontiguousarray(pairs, np.int64)).to(cs.device)
    n = int(pairs.shape[0])
    rs = cs.max_chains if row_stride is None else row_stride
    feat = torch.zeros(max(n, 1) * rs * N_FEAT, dtype=torch.int16, device=cs.device)
    count = torch.empty(max(n, 1), dtype=torch.int32, device=cs.device)
    ws = workspace(paam_features_bytes(cs, n), cs.device)
    paam_features(cs, seed, pairs, rs, feat, count, ws, stream)
    _sync(cs.device)
    return {"feat": feat.cpu().numpy().view(np.uint16)[:n * rs * N_FEAT].reshape(n, rs, N_FEAT),
            "count": count.cpu().numpy()[:n]}


def _sync(device):
    import torch
    if str(device).startswith("cuda"):
        torch.cuda.synchronize()


class Network:
    """Device state of the ranking network: float32 master parameters, the
    packed bfloat16 weights and the Adam moments (all torch tensors)."""

    def __init__(self, params, device="cuda:0", stream=None):
        import torch
        p = np.ascontiguousarray(params, np.float32)
        assert p.size == MLP_PARAMS
        self.device = device
        self.params = torch.from_numpy(p.copy()).to(device)
        self.packed = torch.zeros(MLP_PACKED, dtype=torch.int16, device=device)
        self.m = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=device)
        self.v = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=device)
        self.step = 0
        paam_mlp_pack(self.params, self.packed, stream)

    def adam(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        paam_mlp_adam_step(self.params, self.packed, self.m, self.v, grad, lr, beta1, beta2, eps,
                           self.step, stream)


def score(cs: Chainset, net: Network, n_cand: int, seed: int, stream=None, **wcrt_kw):
    """Network scores of every candidate of every set: device float32
    [n_sets * n_cand]."""
    import torch
    o = search_opts(n_cand, seed, **wcrt_kw)
    scores = torch.empty(max(cs.n_sets * n_cand, 1), dtype=torch.float32, device=cs.device)
    ws = workspace(paam_score_bytes(cs, o), cs.device)
    paam_score_candidates(cs, o, net.params, net.packed, scores, ws, stream)
    return scores


def des_opts(n_scen, horizon, exec_permille=1000, seed=0, util_permille=1000,
             max_steps=1 << 40) -> paam_des_opts:
    return paam_des_opts(n_scen=n_scen, exec_permille=exec_permille, horizon=horizon,
                         seed=seed & (2**64 - 1), util_permille=util_permille, reserved=0,
                         max_steps=max_steps)


def paam_des_batch(cs: Chainset, opts: paam_des_opts, offsets, obs, status, stream=None) -> None:
    check(lib().paam_des_batch(cs.handle, ctypes.byref(opts), offsets.data_ptr(), obs.data_ptr(),
                               status.data_ptr(), _stream_ptr(stream)), "paam_des_batch")


def simulate(cs: Chainset, offsets, n_scen, horizon, stream=None, **kw) -> dict:
    """Event-driven simulation of every set in n_scen scenarios
    (paam_des_batch); offsets [n_chains * n_scen] int64 (per set a
    [n_scen][C] block).  Returns host arrays obs (same layout) and status."""
    import torch
    o = des_opts(n_scen, horizon, **kw)
    off = torch.as_tensor(np.ascontiguousarray(offsets, np.int64)).to(cs.device)
    obs = torch.empty(max(cs.n_chains * n_scen, 1), dtype=torch.int64, device=cs.device)
    status = torch.empty(max(cs.n_sets * n_scen, 1), dtype=torch.int8, device=cs.device)
    paam_des_batch(cs, o, off, obs, status, stream)
    _sync(cs.device)
    return {"obs": obs.cpu().numpy()[:cs.n_chains * n_scen],
            "status": status.cpu().numpy()[:cs.n_sets * n_scen]}
