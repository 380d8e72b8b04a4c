"""CPU oracle of the exhaustive AND/OR pathway traversal (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the GPU library: the C source in this folder is
compiled on its own with gcc, and this wrapper only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "efm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

COMPLETE = 0
DEPTH_CAPPED = 1
FRONTIER_TRUNCATED = 2

_ERRORS = {-1: "invalid argument", -2: "out of memory", -4: "int128 overflow"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, portable code)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def bind(path: str):
    """Load an oracle shared library from `path` and declare its signatures."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.orc_enumerate.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int64, ctypes.POINTER(P)]
    lib.orc_enumerate.restype = ctypes.c_int
    lib.orc_count.argtypes = [P]
    lib.orc_count.restype = ctypes.c_int64
    lib.orc_status.argtypes = [P]
    lib.orc_status.restype = ctypes.c_uint32
    lib.orc_words.argtypes = [P]
    lib.orc_words.restype = ctypes.c_int
    lib.orc_n_levels.argtypes = [P]
    lib.orc_n_levels.restype = ctypes.c_int
    lib.orc_copy.argtypes = [P, P, P]
    lib.orc_copy.restype = None
    lib.orc_levels.argtypes = [P, P]
    lib.orc_levels.restype = None
    lib.orc_free.argtypes = [P]
    lib.orc_free.restype = None
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = bind(_LIB)
    return _lib


@dataclass
class OracleResult:
    keys: np.ndarray      # uint64 [count, W], canonical order
    flux: np.ndarray      # int64 [count, n]
    status: int
    levels: np.ndarray    # int64 [n_levels, 6]: parents, children, unique, independent, emitted, kept

    @property
    def count(self) -> int:
        return int(self.keys.shape[0])


def enumerate_pathways(S, rev, ext, target: int, depth_cap: int = 0,
                       frontier_cap: int = 0, lib=None) -> OracleResult:
    """All elementary pathways producing external metabolite `target` (see efm_oracle.c).
    `lib` may name another build of the same source (bind())."""
    lib = lib or _load()
    S = np.ascontiguousarray(S, dtype=np.int32)
    rev = np.ascontiguousarray(rev, dtype=np.uint8)
    ext = np.ascontiguousarray(ext, dtype=np.uint8)
    m, n = S.shape
    out = ctypes.c_void_p()
    rc = lib.orc_enumerate(m, n, S.ctypes.data, rev.ctypes.data, ext.ctypes.data, int(target),
                           int(depth_cap), int(frontier_cap), ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"oracle failed: {_ERRORS.get(rc, rc)}")
    try:
        cnt = lib.orc_count(out)
        W = lib.orc_words(out)
        keys = np.zeros((cnt, W), np.uint64)
        flux = np.zeros((cnt, n), np.int64)
        lib.orc_copy(out, keys.ctypes.data, flux.ctypes.data)
        nl = lib.orc_n_levels(out)
        lv = np.zeros((nl, 6), np.int64)
        lib.orc_levels(out, lv.ctypes.data)
        return OracleResult(keys, flux, int(lib.orc_status(out)), lv)
    finally:
        lib.orc_free(out)
