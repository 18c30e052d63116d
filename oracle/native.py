"""Loader for the C part of the oracle (oracle/c/hr_oracle.c).

``build()`` compiles it with gcc into oracle/_build/liboracle.so; ``lib()``
loads it (building on first use).  Test infrastructure only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "c", "hr_oracle.c")
_OUT = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    if force or not os.path.exists(_OUT):
        tmp = _OUT + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                        "-o", tmp, _SRC], check=True)
        os.replace(tmp, _OUT)
    return _OUT


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_OUT):
            build(force=False)
        L = ctypes.CDLL(_OUT)
        P = ctypes.c_void_p
        L.oracle_brute_hits.restype = ctypes.c_uint64
        L.oracle_brute_hits.argtypes = [P, P, P, P, P, ctypes.c_uint64, P, P, P,
                                        ctypes.c_uint64, ctypes.c_int]
        L.oracle_exhaustive_many.restype = ctypes.c_uint64
        L.oracle_exhaustive_many.argtypes = [P, P, P, P, P, P, ctypes.c_uint64,
                                             ctypes.c_int, ctypes.c_int, P, P, P,
                                             ctypes.c_uint64, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads_default() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def brute_hits_many(A, B, N, lo, D, threads: int | None = None):
    """Brute-force hit lists of many instances (M = 2^64).

    A, B, lo, D: uint64 arrays (lo, D per instance); N: uint32 array.
    Returns (counts uint32[n], offsets uint64[n], ks uint32[total]); the hits
    of instance i are ks[offsets[i] : offsets[i] + counts[i]], ordered by
    (distance, k).
    """
    A = np.ascontiguousarray(A, np.uint64)
    B = np.ascontiguousarray(B, np.uint64)
    N = np.ascontiguousarray(N, np.uint32)
    lo = np.ascontiguousarray(lo, np.uint64)
    D = np.ascontiguousarray(D, np.uint64)
    n = A.size
    counts = np.zeros(n, np.uint32)
    offsets = np.zeros(max(n, 1), np.uint64)
    cap = 1 << 16
    while True:
        ks = np.zeros(cap, np.uint32)
        total = lib().oracle_brute_hits(_ptr(A), _ptr(B), _ptr(N), _ptr(lo), _ptr(D), n,
                                        _ptr(counts), _ptr(offsets), _ptr(ks), cap,
                                        threads or threads_default())
        if total <= cap:
            return counts, offsets[:n], ks[:total]
        cap = int(total)


def exhaustive_many(rows, N, hr_lo, hr_hi, rej_lo, rej_hi, delta: int, L: int,
                    threads: int | None = None):
    """Phase-3 exhaustive scan of many pieces (see oracle_exhaustive_many).

    rows: uint64 array of shape (n_pieces, delta+1, L) (little-endian limbs).
    Returns (counts uint32[n], xs uint32[total], cls uint8[total]).
    """
    rows = np.ascontiguousarray(rows, np.uint64)
    n = rows.shape[0]
    arrs = [np.ascontiguousarray(x, np.uint64) for x in (hr_lo, hr_hi, rej_lo, rej_hi)]
    N = np.ascontiguousarray(N, np.uint32)
    counts = np.zeros(max(n, 1), np.uint32)
    cap = 1 << 16
    while True:
        xs = np.zeros(cap, np.uint32)
        cl = np.zeros(cap, np.uint8)
        total = lib().oracle_exhaustive_many(_ptr(rows), _ptr(N), *[_ptr(a) for a in arrs],
                                             n, delta, L, _ptr(counts), _ptr(xs), _ptr(cl),
                                             cap, threads or threads_default())
        if total == (1 << 64) - 1:
            raise ValueError("degree or width out of range")
        if total <= cap:
            return counts[:n], xs[:total], cl[:total]
        cap = int(total)
