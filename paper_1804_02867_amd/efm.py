"""Python binding of libefm.so (include/efm.h): argument marshalling only.

Every step of the traversal runs in the library's HIP kernels.  PyTorch supplies
device memory (the workspace tensor) and the HIP stream.  There is no fallback:
if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libefm.so")

OK, EINVAL, ENOMEM, EDEVICE, EOVERFLOW = 0, -1, -2, -3, -4
COMPLETE, DEPTH_CAPPED, FRONTIER_TRUNCATED = 0, 1, 2
OPT_NO_PRUNE, OPT_EXACT_RANK, OPT_TIME_KERNELS, OPT_NO_GF2, OPT_AUTOTUNE = 1, 2, 4, 8, 16
OPT_LEARNED = 32
MAX_DEPTH = 64
FEAT_MAX = 512
TRACE_WORDS = 16
HIDDEN = 256

EXPORTS = ["efm_network_create", "efm_network_destroy", "efm_workspace_query", "efm_enumerate",
           "efm_result_info", "efm_result_stats", "efm_result_bitsets", "efm_result_fluxes",
           "efm_result_destroy", "efm_status_string", "efm_last_error",
           "efm_batch_create", "efm_batch_run", "efm_batch_result", "efm_batch_latency",
           "efm_batch_config_get", "efm_batch_destroy",
           "efm_traces_create", "efm_traces_destroy", "efm_traces_info", "efm_trace_collect",
           "efm_traces_append", "efm_traces_fetch",
           "efm_model_create", "efm_model_destroy", "efm_model_info", "efm_model_get_params",
           "efm_model_set_params", "efm_model_save", "efm_model_load", "efm_model_score",
           "efm_model_score_keys", "efm_model_grad", "efm_model_train", "efm_enumerate_learned"]


class EnumOpts(ctypes.Structure):
    _fields_ = [("depth_cap", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("frontier_cap", ctypes.c_int64), ("unique_cap", ctypes.c_int64),
                ("found_cap", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("reserved1", ctypes.c_uint32), ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class LevelStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("parents", "children", "unique", "row_closed", "pruned", "independent", "emitted",
                 "kept")] + [(k, ctypes.c_double) for k in
                             ("ms_expand", "ms_rank", "ms_exact", "ms_select", "ms_materialize")] + [
                    ("rank_rows", ctypes.c_int64)]


class EfmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"efm error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (no GPU needed) and declare the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -m paper_1804_02867_amd.build)")
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "efm_network_create": ([I32, I32, P, P, P, ctypes.POINTER(P)], I32),
        "efm_network_destroy": ([P], I32),
        "efm_workspace_query": ([P, ctypes.POINTER(EnumOpts), ctypes.POINTER(ctypes.c_size_t)], I32),
        "efm_enumerate": ([P, I32, ctypes.POINTER(EnumOpts), ctypes.POINTER(P)], I32),
        "efm_result_info": ([P, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_uint32),
                             ctypes.POINTER(I32)], I32),
        "efm_result_stats": ([P, ctypes.POINTER(LevelStats), I32], I32),
        "efm_result_bitsets": ([P, P, I64], I32),
        "efm_result_fluxes": ([P, P, I64], I32),
        "efm_result_destroy": ([P], I32),
        "efm_status_string": ([I32], ctypes.c_char_p),
        "efm_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        lib = load()
        raise EfmError(rc, lib.efm_last_error().decode())


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the traversal runs only in the HIP library")
    return torch


class Network:
    """Device copy of a network (efm_network_create)."""

    def __init__(self, S, rev, ext):
        _require_gpu()
        lib = load()
        self.S = np.ascontiguousarray(S, dtype=np.int32)
        self.rev = np.ascontiguousarray(rev, dtype=np.uint8)
        self.ext = np.ascontiguousarray(ext, dtype=np.uint8)
        self.m, self.n = self.S.shape
        h = ctypes.c_void_p()
        _check(lib.efm_network_create(self.m, self.n, self.S.ctypes.data, self.rev.ctypes.data,
                                      self.ext.ctypes.data, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().efm_network_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Result:
    keys: np.ndarray       # uint64 [count, W], canonical order
    flux: np.ndarray       # int64 [count, n]
    status: int
    levels: list           # dicts per level (index 0 = one-reaction sets)

    @property
    def count(self) -> int:
        return int(self.keys.shape[0])


def make_opts(depth_cap=0, frontier_cap=0, unique_cap=0, found_cap=0, flags=0) -> EnumOpts:
    o = EnumOpts()
    o.depth_cap, o.frontier_cap, o.unique_cap, o.found_cap, o.flags = (
        int(depth_cap), int(frontier_cap), int(unique_cap), int(found_cap), int(flags))
    return o


def workspace_bytes(net: Network, opts: EnumOpts) -> int:
    size = ctypes.c_size_t()
    _check(load().efm_workspace_query(net._h, ctypes.byref(opts), ctypes.byref(size)))
    return int(size.value)


def enumerate_pathways(net: Network, target: int, depth_cap=0, frontier_cap=0, unique_cap=0,
                       found_cap=0, flags=0, workspace=None, stream=None) -> Result:
    """efm_enumerate with a torch-allocated workspace on the current (or given) stream."""
    torch = _require_gpu()
    lib = load()
    opts = make_opts(depth_cap, frontier_cap, unique_cap, found_cap, flags)
    need = workspace_bytes(net, opts)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    st = stream if stream is not None else torch.cuda.current_stream()
    opts.stream = ctypes.c_void_p(st.cuda_stream)
    opts.workspace = ctypes.c_void_p(workspace.data_ptr())
    opts.workspace_bytes = need
    res = ctypes.c_void_p()
    _check(lib.efm_enumerate(net._h, int(target), ctypes.byref(opts), ctypes.byref(res)))
    try:
        cnt, W, status, nl = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_uint32(), ctypes.c_int32()
        _check(lib.efm_result_info(res, ctypes.byref(cnt), ctypes.byref(W), ctypes.byref(status),
                                   ctypes.byref(nl)))
        keys = np.zeros((cnt.value, W.value), np.uint64)
        flux = np.zeros((cnt.value, net.n), np.int64)
        _check(lib.efm_result_bitsets(res, keys.ctypes.data, keys.size))
        _check(lib.efm_result_fluxes(res, flux.ctypes.data, flux.size))
        arr = (LevelStats * max(nl.value, 1))()
        _check(lib.efm_result_stats(res, arr, nl.value))
        levels = [{f: getattr(arr[i], f) for f, _ in LevelStats._fields_} for i in range(nl.value)]
        return Result(keys, flux, int(status.value), levels)
    finally:
        lib.efm_result_destroy(res)


# ------------------------------------------------------------------- batches

class BatchConfig(ctypes.Structure):
    _fields_ = [("waves_per_network", ctypes.c_int32), ("networks_per_cu", ctypes.c_int32)]


def _load_batch(lib):
    if getattr(lib, "_batch_sigs", False):
        return lib
    P, I32 = ctypes.c_void_p, ctypes.c_int32
    sig = {
        "efm_batch_create": ([P, P, I32, ctypes.POINTER(EnumOpts), ctypes.POINTER(P)], I32),
        "efm_batch_run": ([P, P], I32),
        "efm_batch_result": ([P, I32, ctypes.POINTER(P)], I32),
        "efm_batch_latency": ([P, P], I32),
        "efm_batch_config_get": ([P, ctypes.POINTER(BatchConfig)], I32),
        "efm_batch_destroy": ([P], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    lib._batch_sigs = True
    return lib


def _fetch(lib, res, n):
    cnt, W, status, nl = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_uint32(), ctypes.c_int32()
    _check(lib.efm_result_info(res, ctypes.byref(cnt), ctypes.byref(W), ctypes.byref(status), ctypes.byref(nl)))
    keys = np.zeros((cnt.value, W.value), np.uint64)
    flux = np.zeros((cnt.value, n), np.int64)
    _check(lib.efm_result_bitsets(res, keys.ctypes.data, keys.size))
    _check(lib.efm_result_fluxes(res, flux.ctypes.data, flux.size))
    arr = (LevelStats * max(nl.value, 1))()
    _check(lib.efm_result_stats(res, arr, nl.value))
    levels = [{f: getattr(arr[i], f) for f, _ in LevelStats._fields_} for i in range(nl.value)]
    return Result(keys, flux, int(status.value), levels)


class Batch:
    """efm_batch_*: many networks in one persistent launch, replayed as a HIP graph."""

    def __init__(self, nets, targets, depth_cap=0, frontier_cap=0, unique_cap=0, found_cap=0, flags=0):
        _require_gpu()
        self._lib = _load_batch(load())
        self.nets = list(nets)
        self.n = [g.n for g in self.nets]
        handles = (ctypes.c_void_p * len(self.nets))(*[g._h.value for g in self.nets])
        tg = np.ascontiguousarray(targets, dtype=np.int32)
        opts = make_opts(depth_cap, frontier_cap, unique_cap, found_cap, flags)
        h = ctypes.c_void_p()
        _check(self._lib.efm_batch_create(ctypes.cast(handles, ctypes.c_void_p), tg.ctypes.data, len(self.nets),
                                          ctypes.byref(opts), ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        st = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(self._lib.efm_batch_run(self._h, st))

    def config(self):
        c = BatchConfig()
        _check(self._lib.efm_batch_config_get(self._h, ctypes.byref(c)))
        return c.waves_per_network, c.networks_per_cu

    def result(self, i) -> Result:
        res = ctypes.c_void_p()
        _check(self._lib.efm_batch_result(self._h, int(i), ctypes.byref(res)))
        try:
            return _fetch(self._lib, res, self.n[i])
        finally:
            self._lib.efm_result_destroy(res)

    def latency_ns(self) -> np.ndarray:
        out = np.zeros(len(self.nets), np.int64)
        _check(self._lib.efm_batch_latency(self._h, out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.efm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------- learned ordering

class TraceOpts(ctypes.Structure):
    _fields_ = [("neg_per_pos", ctypes.c_double), ("neg_min", ctypes.c_int64), ("pos_max", ctypes.c_int64),
                ("seed", ctypes.c_uint64)]


class TraceInfo(ctypes.Structure):
    _fields_ = [("states", ctypes.c_int64), ("positives", ctypes.c_int64), ("recorded", ctypes.c_int64),
                ("pathways", ctypes.c_int64), ("status", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("pos_weight", ctypes.c_float), ("reserved", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_void_p)]


class TrainStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("ms", ctypes.c_double)]


def _load_learn(lib):
    if getattr(lib, "_learn_sigs", False):
        return lib
    P, I32, I64, F32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    sig = {
        "efm_traces_create": ([I32, I32, I64, ctypes.POINTER(P)], I32),
        "efm_traces_destroy": ([P], I32),
        "efm_traces_info": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64)], I32),
        "efm_trace_collect": ([P, P, I32, ctypes.POINTER(EnumOpts), ctypes.POINTER(TraceOpts),
                               ctypes.POINTER(TraceInfo)], I32),
        "efm_traces_append": ([P, P, P, P, I64], I32),
        "efm_traces_fetch": ([P, I64, I64, P, P, P, P], I32),
        "efm_model_create": ([I32, I32, I32, ctypes.c_uint64, ctypes.POINTER(P)], I32),
        "efm_model_destroy": ([P], I32),
        "efm_model_info": ([P, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(I32),
                            ctypes.POINTER(I32)], I32),
        "efm_model_get_params": ([P, P, I64], I32),
        "efm_model_set_params": ([P, P, I64], I32),
        "efm_model_save": ([P, ctypes.c_char_p], I32),
        "efm_model_load": ([ctypes.c_char_p, ctypes.POINTER(P)], I32),
        "efm_model_score": ([P, P, I64, I64, P], I32),
        "efm_model_score_keys": ([P, P, I32, P, I64, P], I32),
        "efm_model_grad": ([P, P, I64, I64, F32, P, ctypes.POINTER(ctypes.c_double)], I32),
        "efm_model_train": ([P, P, ctypes.POINTER(TrainOpts), ctypes.POINTER(TrainStats)], I32),
        "efm_enumerate_learned": ([P, I32, I64, P, ctypes.POINTER(EnumOpts), ctypes.POINTER(P)], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    lib._learn_sigs = True
    return lib


class Traces:
    """efm_traces_*: labelled partial pathways in model-input form (device memory)."""

    def __init__(self, in_bits=1024, in_counts=400, capacity=1 << 18):
        _require_gpu()
        self._lib = _load_learn(load())
        h = ctypes.c_void_p()
        _check(self._lib.efm_traces_create(int(in_bits), int(in_counts), int(capacity), ctypes.byref(h)))
        self._h = h
        self.in_bits, self.in_counts = int(in_bits), int(in_counts)

    def collect(self, net: "Network", target: int, depth_cap=0, frontier_cap=0, unique_cap=0, found_cap=0,
                flags=0, neg_per_pos=4.0, neg_min=64, pos_max=0, seed=0) -> dict:
        opts = make_opts(depth_cap, frontier_cap, unique_cap, found_cap, flags)
        to = TraceOpts(float(neg_per_pos), int(neg_min), int(pos_max), int(seed))
        info = TraceInfo()
        _check(self._lib.efm_trace_collect(self._h, net._h, int(target), ctypes.byref(opts), ctypes.byref(to),
                                           ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in TraceInfo._fields_ if f != "reserved"}

    def append(self, entries, lengths, labels):
        ent = np.ascontiguousarray(entries, dtype=np.uint16)
        ln = np.ascontiguousarray(lengths, dtype=np.uint16)
        lb = np.ascontiguousarray(labels, dtype=np.uint8)
        if ent.ndim != 2 or ent.shape[1] != FEAT_MAX or ent.shape[0] != ln.size or ln.size != lb.size:
            raise ValueError("entries must be (count, FEAT_MAX), lengths and labels (count,)")
        _check(self._lib.efm_traces_append(self._h, ent.ctypes.data, ln.ctypes.data, lb.ctypes.data, ln.size))

    def info(self):
        c, p = ctypes.c_int64(), ctypes.c_int64()
        _check(self._lib.efm_traces_info(self._h, ctypes.byref(c), ctypes.byref(p)))
        return c.value, p.value

    def __len__(self):
        return self.info()[0]

    def fetch(self, first=0, count=None):
        if count is None:
            count = len(self) - first
        ent = np.zeros((count, FEAT_MAX), np.uint16)
        ln = np.zeros(count, np.uint16)
        lb = np.zeros(count, np.uint8)
        keys = np.zeros((count, TRACE_WORDS), np.uint64)
        _check(self._lib.efm_traces_fetch(self._h, int(first), int(count), ent.ctypes.data, ln.ctypes.data,
                                          lb.ctypes.data, keys.ctypes.data))
        return ent, ln, lb, keys

    def close(self):
        if getattr(self, "_h", None):
            self._lib.efm_traces_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """efm_model_*: the frontier-scoring perceptron (fp32 master weights, bf16 kernel copies)."""

    def __init__(self, in_bits=1024, in_counts=400, seed=0, _handle=None):
        _require_gpu()
        self._lib = _load_learn(load())
        if _handle is None:
            h = ctypes.c_void_p()
            _check(self._lib.efm_model_create(int(in_bits), int(in_counts), HIDDEN, int(seed), ctypes.byref(h)))
            _handle = h
        self._h = _handle
        n, ib, ic, hd = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.efm_model_info(self._h, ctypes.byref(n), ctypes.byref(ib), ctypes.byref(ic),
                                        ctypes.byref(hd)))
        self.n_params, self.in_bits, self.in_counts, self.hidden = n.value, ib.value, ic.value, hd.value

    @classmethod
    def load(cls, path):
        _require_gpu()
        lib = _load_learn(load())
        h = ctypes.c_void_p()
        _check(lib.efm_model_load(os.fsencode(path), ctypes.byref(h)))
        return cls(_handle=h)

    def save(self, path):
        _check(self._lib.efm_model_save(self._h, os.fsencode(path)))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        _check(self._lib.efm_model_get_params(self._h, out.ctypes.data, out.size))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(self._lib.efm_model_set_params(self._h, p.ctypes.data, p.size))

    def score(self, traces: Traces, first=0, count=None) -> np.ndarray:
        if count is None:
            count = len(traces) - first
        out = np.zeros(count, np.float32)
        _check(self._lib.efm_model_score(self._h, traces._h, int(first), int(count), out.ctypes.data))
        return out

    def score_keys(self, net: "Network", target: int, keys) -> np.ndarray:
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.zeros(k.shape[0], np.float32)
        _check(self._lib.efm_model_score_keys(self._h, net._h, int(target), k.ctypes.data, k.shape[0],
                                              out.ctypes.data))
        return out

    def grad(self, traces: Traces, first=0, count=None, pos_weight=1.0):
        if count is None:
            count = len(traces) - first
        g = np.zeros(self.n_params, np.float32)
        loss = ctypes.c_double()
        _check(self._lib.efm_model_grad(self._h, traces._h, int(first), int(count), float(pos_weight),
                                        g.ctypes.data, ctypes.byref(loss)))
        return loss.value, g

    def train(self, traces: Traces, epochs=1, batch=1024, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              pos_weight=0.0, seed=0, stream=None) -> dict:
        st = stream.cuda_stream if stream is not None else None
        o = TrainOpts(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps),
                      float(pos_weight), 0, int(seed), st)
        stats = TrainStats()
        _check(self._lib.efm_model_train(self._h, traces._h, ctypes.byref(o), ctypes.byref(stats)))
        return {f: getattr(stats, f) for f, _ in TrainStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.efm_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def enumerate_learned(net: Network, target: int, budget: int, model: Model, depth_cap=0, unique_cap=0,
                      found_cap=0, flags=0, workspace=None, stream=None) -> Result:
    """efm_enumerate_learned: the traversal with the learned ordering of a
    `budget`-item frontier."""
    torch = _require_gpu()
    lib = _load_learn(load())
    opts = make_opts(depth_cap, budget, unique_cap, found_cap, flags | OPT_LEARNED)
    need = workspace_bytes(net, opts)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    st = stream if stream is not None else torch.cuda.current_stream()
    opts.stream = ctypes.c_void_p(st.cuda_stream)
    opts.workspace = ctypes.c_void_p(workspace.data_ptr())
    opts.workspace_bytes = need
    res = ctypes.c_void_p()
    _check(lib.efm_enumerate_learned(net._h, int(target), int(budget), model._h, ctypes.byref(opts),
                                     ctypes.byref(res)))
    try:
        return _fetch(lib, res, net.n)
    finally:
        lib.efm_result_destroy(res)
