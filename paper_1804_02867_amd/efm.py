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
MAX_DEPTH = 64

EXPORTS = ["efm_network_create", "efm_network_destroy", "efm_workspace_query", "efm_enumerate",
           "efm_result_info", "efm_result_stats", "efm_result_bitsets", "efm_result_fluxes",
           "efm_result_destroy", "efm_status_string", "efm_last_error",
           "efm_batch_create", "efm_batch_run", "efm_batch_result", "efm_batch_latency",
           "efm_batch_config_get", "efm_batch_destroy"]


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
                             ("ms_expand", "ms_rank", "ms_exact", "ms_select", "ms_materialize")]


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
