"""ctypes binding of libhrcpu.so (include/hrcpu.h): the multi-core SIMD CPU
search, on numpy arrays in host memory (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhrcpu.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hrcpu.h")
EXPORTS = ("hrc_simd_width", "hrc_filter", "hrc_search")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.hrc_simd_width.restype = i32
        L.hrc_simd_width.argtypes = []
        L.hrc_filter.restype = i32
        L.hrc_filter.argtypes = [P, P, P, u64, P, P, u32, P, P, P, i32]
        L.hrc_search.restype = i32
        L.hrc_search.argtypes = [P, P, P, u64, P, P, u32, P, P, P, P, u64, P, i32]
        _lib = L
    return _lib


def _p(x):
    if x is None:
        return None
    assert x.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(x.ctypes.data)


def _arr(x, dtype):
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


def simd_width() -> int:
    return lib().hrc_simd_width()


def filter_regular(a, b, N, d, lo=None, group=None, threads=0):
    """(pass uint8, d uint64, iters uint32) of the regular test per instance."""
    a, b, N = _arr(a, np.uint64), _arr(b, np.uint64), _arr(N, np.uint32)
    n = len(a)
    group = group or max(n, 1)
    d = _arr(np.broadcast_to(d, (-(-n // group),)) if np.ndim(d) == 0 else d, np.uint64)
    lo = None if lo is None else _arr(np.broadcast_to(lo, d.shape) if np.ndim(lo) == 0 else lo,
                                      np.uint64)
    ok = np.empty(n, np.uint8)
    dv = np.empty(n, np.uint64)
    it = np.empty(n, np.uint32)
    st = lib().hrc_filter(_p(a), _p(b), _p(N), n, _p(lo), _p(d), group, _p(ok), _p(dv), _p(it),
                          threads)
    if st != 0:
        raise RuntimeError(f"hrc_filter failed ({st})")
    return ok, dv, it


def search(a, b, N, d, lo=None, group=None, cap=1 << 20, threads=0):
    """(counts, offsets, hits) as hr_search, computed on the host cores."""
    a, b, N = _arr(a, np.uint64), _arr(b, np.uint64), _arr(N, np.uint32)
    n = len(a)
    group = group or max(n, 1)
    d = _arr(np.broadcast_to(d, (-(-n // group),)) if np.ndim(d) == 0 else d, np.uint64)
    lo = None if lo is None else _arr(np.broadcast_to(lo, d.shape) if np.ndim(lo) == 0 else lo,
                                      np.uint64)
    counts = np.empty(n, np.uint32)
    offsets = np.empty(n, np.uint64)
    total = np.zeros(1, np.uint64)
    while True:
        hits = np.empty(max(cap, 1), np.uint32)
        st = lib().hrc_search(_p(a), _p(b), _p(N), n, _p(lo), _p(d), group, _p(counts),
                              _p(offsets), _p(hits), None, cap, _p(total), threads)
        if st == 0:
            return counts, offsets, hits[: int(total[0])]
        if st != -2:
            raise RuntimeError(f"hrc_search failed ({st})")
        cap = int(total[0])
