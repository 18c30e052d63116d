"""Convenience layer over the C ABI: allocates outputs as torch device tensors
and handles the search's capacity protocol.  All computation happens in the
HIP library; this module only sizes buffers, launches and reads back counts.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib

_default_ctx = {}


def context(device: int = 0) -> _lib.Context:
    ctx = _default_ctx.get(device)
    if ctx is None:
        ctx = _default_ctx[device] = _lib.Context(device)
    return ctx


def to_dev(x, dtype, device="cuda"):
    """numpy array / list -> contiguous device tensor of the given dtype."""
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    np_dtype = {torch.uint64: np.uint64, torch.uint32: np.uint32, torch.uint8: np.uint8}[dtype]
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np_dtype))).to(device)


def to_dev_async(x, dtype, device="cuda"):
    """Like to_dev, through pinned host memory and a copy queued on the
    current stream: the host does not wait for work already queued there
    (a copy from pageable memory would).  The pinned buffer stays reserved
    until the copy has run."""
    np_dtype = {torch.uint64: np.uint64, torch.uint32: np.uint32, torch.uint8: np.uint8}[dtype]
    h = torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np_dtype))).pin_memory()
    return h.to(device, non_blocking=True)


def _u64_scalar(t: torch.Tensor) -> int:
    return int(t.cpu().numpy()[0])


def search(a, b, N, d, lo=None, group=None, cap=None, with_inst=False, ctx=None, stream=None):
    """Degree-1 search (hr_search).  a, b: uint64, N: uint32 device tensors.

    d and lo: python ints (one window for all instances) or uint64 tensors of
    ceil(n / group) entries.  Returns (counts, offsets, hits, inst or None),
    hits trimmed to the exact total.
    """
    ctx = ctx or context()
    dev = a.device
    n = a.numel()
    if group is None:
        group = max(n, 1)
    ng = (n + group - 1) // group if n else 1
    if not isinstance(d, torch.Tensor):
        d = to_dev(np.full(max(ng, 1), d, np.uint64), torch.uint64, dev)
    if lo is not None and not isinstance(lo, torch.Tensor):
        lo = to_dev(np.full(max(ng, 1), lo, np.uint64), torch.uint64, dev)
    counts = torch.empty(n, dtype=torch.uint32, device=dev)
    offsets = torch.empty(n, dtype=torch.uint64, device=dev)
    total = torch.zeros(1, dtype=torch.uint64, device=dev)
    if cap is None:
        cap = 1 << 16
    while True:
        hits = torch.empty(max(cap, 1), dtype=torch.uint32, device=dev)
        inst = torch.empty(max(cap, 1), dtype=torch.uint32, device=dev) if with_inst else None
        _lib.hr_search(ctx, a, b, N, lo, d, group, counts, offsets, hits, inst, cap, total, stream)
        torch.cuda.synchronize(dev)
        tot = _u64_scalar(total)
        if tot <= cap:
            return counts, offsets, hits[:tot], (inst[:tot] if with_inst else None)
        cap = tot


def tabulate(table, n_sub, degree, tau, width, ctx=None, stream=None):
    ctx = ctx or context()
    dev = table.device
    a = torch.empty(n_sub * tau, dtype=torch.uint64, device=dev)
    b = torch.empty(n_sub * tau, dtype=torch.uint64, device=dev)
    _lib.hr_tabulate(ctx, table, n_sub, degree, tau, width, a, b, stream)
    return a, b


def subtables(upper, upper_degree, upper_width, n_sub, degree, width, N, t0=0, t_idx=None,
              max_t=None, max_N=None, ctx=None, stream=None, out=None):
    """Sub-interval tables from an upper table (hr_subtables).  N: an int
    (every table) or a uint32 device tensor (one per table); t_idx: None
    (tables t0 .. t0 + n_sub - 1) or a uint32 device tensor.  Returns the
    uint64 table tensor (n_sub * E * width/64 limbs)."""
    ctx = ctx or context()
    dev = upper.device
    E = (degree + 1) * (degree + 2) // 2
    if out is None:
        out = torch.empty(max(n_sub, 1) * E * (width // 64), dtype=torch.uint64, device=dev)
    N_per = N if isinstance(N, torch.Tensor) else None
    N0 = 0 if N_per is not None else int(N)
    if max_t is None:
        max_t = t0 + n_sub - 1 if t_idx is None else int(t_idx.to(torch.int64).max().item())
    if max_N is None:
        max_N = N0 if N_per is None else int(N_per.to(torch.int64).max().item())
    _lib.hr_subtables(ctx, upper, upper_degree, upper_width, t_idx, t0, N_per, N0, max_t, max_N,
                      n_sub, degree, width, out, stream)
    return out


def recheck(table, n_sub, degree, tau, width, cand_inst, cand_k, max_k, thr, ctx=None,
            stream=None):
    ctx = ctx or context()
    dev = table.device
    n = cand_k.numel()
    value = torch.empty(max(n, 1), dtype=torch.uint64, device=dev)
    cls = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    _lib.hr_recheck(ctx, table, n_sub, degree, tau, width, cand_inst, cand_k, max_k, thr,
                    value, cls, stream)
    return value[:n], cls[:n]


from .plan import ITEM_DTYPE, RESULT_DTYPE  # noqa: E402,F401


def pipeline(table, n_sub, degree, tau, width, N, win, thr, cap=1 << 16, ctx=None, stream=None):
    """Fused tabulate + search + recheck (hr_pipeline).

    Returns (results as a numpy structured array sorted by (sub, piece, k),
    stats dict).  Retries once with the exact capacity if needed.
    """
    ctx = ctx or context()
    dev = table.device
    while True:
        out = torch.empty(max(cap, 1) * _lib.RESULT_BYTES, dtype=torch.uint8, device=dev)
        count = torch.zeros(1, dtype=torch.uint64, device=dev)
        stats = torch.zeros(8, dtype=torch.uint64, device=dev)
        _lib.hr_pipeline(ctx, table, n_sub, degree, tau, width, N, win, thr, out, cap, count,
                         stats, stream)
        torch.cuda.synchronize(dev)
        c = _u64_scalar(count)
        if c <= cap:
            res = out[: c * _lib.RESULT_BYTES].cpu().numpy().view(RESULT_DTYPE)
            res = np.sort(res, order=["sub", "piece", "k"])
            st = stats.cpu().numpy()
            return res, {"pieces": int(st[0]), "candidates": int(st[1]), "results": int(st[2])}
        cap = c
