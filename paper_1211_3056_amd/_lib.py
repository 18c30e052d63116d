"""Thin ctypes binding of libhrsearch.so (include/hrsearch.h).

Argument marshalling only: every entry point takes torch tensors (device
memory) and passes their data pointers and the current HIP stream to the C
ABI.  There is no CPU fallback: if the library is missing, loading fails
loudly.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhrsearch.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hrsearch.h")

HR_OK, HR_EINVAL, HR_ECAPACITY, HR_EDEVICE, HR_ENOMEM, HR_ESCRATCH = 0, -1, -2, -3, -4, -5
HR_STATIC_MAX_INSTANCES = ((1 << 20) // 8 - 1) * 256
HR_WAVES_FILL = 0xFFFFFFFF

_lib = None


class HRError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f"{fn} failed: {status_str(status)} ({status})")
        self.status = status


class hr_result(ctypes.Structure):
    _fields_ = [("job", ctypes.c_uint32), ("sub", ctypes.c_uint32), ("piece", ctypes.c_uint32),
                ("k", ctypes.c_uint32), ("cls", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("value", ctypes.c_uint64)]


class hr_item(ctypes.Structure):
    _fields_ = [("table", ctypes.c_uint64), ("win_lo", ctypes.c_uint64), ("win_d", ctypes.c_uint64),
                ("thr", ctypes.c_uint64 * 4), ("job", ctypes.c_uint32), ("sub", ctypes.c_uint32),
                ("piece0", ctypes.c_uint32), ("npieces", ctypes.c_uint32), ("nu", ctypes.c_uint32),
                ("N", ctypes.c_uint32), ("last_piece", ctypes.c_uint32), ("last_N", ctypes.c_uint32)]


RESULT_BYTES = ctypes.sizeof(hr_result)
ITEM_BYTES = ctypes.sizeof(hr_item)
EXPORTS = ("hr_abi_version", "hr_status_str", "hr_create", "hr_destroy", "hr_search", "hr_batch_run",
           "hr_tabulate", "hr_recheck", "hr_pipeline", "hr_quot_check", "hr_subtables",
           "hr_search_static", "hr_search_steps", "hr_filter", "hr_batch_open", "hr_batch_submit",
           "hr_batch_poll", "hr_batch_wait", "hr_batch_close")
HR_FILTER_LEFEVRE, HR_FILTER_REGULAR = 1, 2


def lib():
    """Load libhrsearch.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.hr_abi_version.restype = i32
    L.hr_abi_version.argtypes = []
    L.hr_status_str.restype = ctypes.c_char_p
    L.hr_status_str.argtypes = [i32]
    L.hr_create.restype = i32
    L.hr_create.argtypes = [ctypes.POINTER(P), i32]
    L.hr_destroy.restype = i32
    L.hr_destroy.argtypes = [P]
    L.hr_search.restype = i32
    L.hr_search.argtypes = [P, P, P, P, u64, P, P, u32, P, P, P, P, u64, P, P]
    L.hr_search_static.restype = i32
    L.hr_search_static.argtypes = [P, P, P, P, u64, P, P, u32, P, P, P, P, u64, P, P]
    L.hr_batch_open.restype = i32
    L.hr_batch_open.argtypes = [P, u32, ctypes.POINTER(P)]
    L.hr_batch_submit.restype = i32
    L.hr_batch_submit.argtypes = [P, P, P, u32, u32, u32, P, u64, P, P, ctypes.POINTER(u64)]
    L.hr_batch_poll.restype = i32
    L.hr_batch_poll.argtypes = [P, ctypes.POINTER(u64)]
    L.hr_batch_wait.restype = i32
    L.hr_batch_wait.argtypes = [P, u64]
    L.hr_batch_close.restype = i32
    L.hr_batch_close.argtypes = [P]
    L.hr_filter.restype = i32
    L.hr_filter.argtypes = [P, i32, P, P, P, u64, P, P, u32, P, P, P, P]
    L.hr_search_steps.restype = i32
    L.hr_search_steps.argtypes = [P, P, P, P, u64, P, P, u32, P, P]
    L.hr_tabulate.restype = i32
    L.hr_tabulate.argtypes = [P, P, u32, u32, u32, u32, P, P, P]
    L.hr_recheck.restype = i32
    L.hr_recheck.argtypes = [P, P, u32, u32, u32, u32, P, P, u64, u32, P, P, P, P]
    L.hr_pipeline.restype = i32
    L.hr_pipeline.argtypes = [P, P, u32, u32, u32, u32, u32, P, P, P, u64, P, P, P]
    L.hr_quot_check.restype = i32
    L.hr_quot_check.argtypes = [P, P, P, u64, P, P, u64, P]
    L.hr_subtables.restype = i32
    L.hr_subtables.argtypes = [P, P, u32, u32, P, u32, P, u32, u32, u32, u32, u32, u32, P, P]
    L.hr_batch_run.restype = i32
    L.hr_batch_run.argtypes = [P, P, P, u32, u32, u32, u32, P, u64, P, P, P]
    _lib = L
    return L


def status_str(status: int) -> str:
    return lib().hr_status_str(status).decode()


def _check(fn, status):
    if status != HR_OK:
        raise HRError(fn, status)


def _p(t):
    """Data pointer of a tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """An hr_ctx on one device (hr_create / hr_destroy)."""

    def __init__(self, device: int = 0):
        self.device = device
        h = ctypes.c_void_p()
        _check("hr_create", lib().hr_create(ctypes.byref(h), device))
        self.handle = h

    def close(self):
        if self.handle:
            lib().hr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hr_search(ctx, a, b, N, win_lo, win_d, group, counts, offsets, hits, hit_inst, cap, total,
              stream=None):
    _check("hr_search", lib().hr_search(ctx.handle, _p(a), _p(b), _p(N), a.numel(), _p(win_lo),
                                        _p(win_d), group, _p(counts), _p(offsets), _p(hits),
                                        _p(hit_inst), cap, _p(total), _stream(stream)))


def hr_search_static(ctx, a, b, N, win_lo, win_d, group, counts, offsets, hits, hit_inst, cap,
                     total, stream=None):
    _check("hr_search_static", lib().hr_search_static(
        ctx.handle, _p(a), _p(b), _p(N), a.numel(), _p(win_lo), _p(win_d), group, _p(counts),
        _p(offsets), _p(hits), _p(hit_inst), cap, _p(total), _stream(stream)))


def hr_filter(ctx, alg, a, b, N, win_lo, win_d, group, passed, d_out=None, iters=None,
              stream=None):
    _check("hr_filter", lib().hr_filter(ctx.handle, alg, _p(a), _p(b), _p(N), a.numel(),
                                        _p(win_lo), _p(win_d), group, _p(passed), _p(d_out),
                                        _p(iters), _stream(stream)))


def hr_search_steps(ctx, a, b, N, win_lo, win_d, group, steps, stream=None):
    _check("hr_search_steps", lib().hr_search_steps(ctx.handle, _p(a), _p(b), _p(N), a.numel(),
                                                    _p(win_lo), _p(win_d), group, _p(steps),
                                                    _stream(stream)))


def hr_tabulate(ctx, table, n_sub, degree, tau, width, a_out, b_out, stream=None):
    _check("hr_tabulate", lib().hr_tabulate(ctx.handle, _p(table), n_sub, degree, tau, width,
                                            _p(a_out), _p(b_out), _stream(stream)))


def hr_recheck(ctx, table, n_sub, degree, tau, width, cand_inst, cand_k, max_k, thr,
               value_out, class_out, stream=None):
    _check("hr_recheck", lib().hr_recheck(ctx.handle, _p(table), n_sub, degree, tau, width,
                                          _p(cand_inst), _p(cand_k), cand_k.numel(), max_k,
                                          _p(thr), _p(value_out), _p(class_out), _stream(stream)))


def _stats_ok(stats):
    if stats is not None and stats.numel() < 8:
        raise ValueError("stats needs 8 uint64 entries")


def hr_pipeline(ctx, table, n_sub, degree, tau, width, N, win, thr, out, cap, count, stats,
                stream=None):
    _stats_ok(stats)
    _check("hr_pipeline", lib().hr_pipeline(ctx.handle, _p(table), n_sub, degree, tau, width, N,
                                            _p(win), _p(thr), _p(out), cap, _p(count), _p(stats),
                                            _stream(stream)))


def hr_batch_run(ctx, pool, items, n_items, width, degree, waves, out, cap, count, stats,
                 stream=None):
    _stats_ok(stats)
    _check("hr_batch_run", lib().hr_batch_run(ctx.handle, _p(pool), _p(items), n_items, width,
                                              degree, waves, _p(out), cap, _p(count), _p(stats),
                                              _stream(stream)))


def hr_subtables(ctx, upper, upper_degree, upper_width, t_idx, t0, N_per, N, max_t, max_N,
                 n_sub, degree, width, table_out, stream=None):
    _check("hr_subtables", lib().hr_subtables(ctx.handle, _p(upper), upper_degree, upper_width,
                                              _p(t_idx), t0, _p(N_per), N, max_t, max_N, n_sub,
                                              degree, width, _p(table_out), _stream(stream)))


def hr_quot_check(ctx, num, den, cap, out, rem=None, stream=None):
    _check("hr_quot_check", lib().hr_quot_check(ctx.handle, _p(num), _p(den), cap, _p(out),
                                                _p(rem) if rem is not None else None,
                                                num.numel(), _stream(stream)))


class BatchStream:
    """An hr_batch (hr_batch_open .. hr_batch_close): queued persistent
    launches with tickets."""

    def __init__(self, ctx, slots: int = 8):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check("hr_batch_open", lib().hr_batch_open(ctx.handle, slots, ctypes.byref(h)))
        self.handle = h

    def submit(self, pool, items, n_items, width, degree, out, cap, count, after_stream=None):
        """Queue one launch; returns its ticket, or None while every slot it
        could use is still running."""
        t = ctypes.c_uint64()
        after = ctypes.c_void_p(after_stream.cuda_stream) if after_stream is not None else None
        st = lib().hr_batch_submit(self.handle, _p(pool), _p(items), n_items, width, degree,
                                   _p(out), cap, _p(count), after, ctypes.byref(t))
        if st == HR_ECAPACITY:
            return None
        _check("hr_batch_submit", st)
        return t.value

    def poll(self) -> int:
        d = ctypes.c_uint64()
        _check("hr_batch_poll", lib().hr_batch_poll(self.handle, ctypes.byref(d)))
        return d.value

    def wait(self, ticket: int):
        _check("hr_batch_wait", lib().hr_batch_wait(self.handle, ticket))

    def close(self):
        if self.handle:
            lib().hr_batch_close(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
