"""End-to-end HR-case search of one job on the GPU.

prepare (host tables, windows, thresholds) -> device: either the fused
kernel (hr_pipeline, one launch) or the plain launch chain
(hr_tabulate -> hr_search -> hr_recheck) -> host decision of the few
undecided values -> sorted HR offsets m (argument X0 + m h).

With an upper table (``form="upper"``) the host prepares only the range's
upper table and one window; the sub-interval tables are made on the device
(hr_subtables) and fed to the fused kernel.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api
from .prep import JobSpec, Prepared, is_hr, prepare, upper_table, upper_windows


def upload(P: Prepared, device="cuda"):
    table = api.to_dev(P.tables.reshape(-1), torch.uint64, device)
    win = api.to_dev(P.win.reshape(-1), torch.uint64, device)
    thr = api.to_dev(P.thr.reshape(-1), torch.uint64, device)
    return table, win, thr


def _finish(P: Prepared, subs_idx, piece, k, cls):
    """Global offsets of certain HR cases plus host-decided undecided ones."""
    spec = P.spec
    base = P.subs[subs_idx].astype(np.int64) * spec.per_sub + piece.astype(np.int64) * spec.N
    m = base + k.astype(np.int64)
    out = [int(x) for x in m[cls == 1]]
    undecided = [int(x) for x in m[cls == 2]]
    out += [x for x in undecided if is_hr(spec, x, P.uf)]
    return sorted(out), len(undecided)


def run_fused(P: Prepared, dev_args=None, ctx=None):
    spec = P.spec
    table, win, thr = dev_args or upload(P)
    res, stats = api.pipeline(table, len(P.subs), spec.delta, spec.tau, spec.W, spec.N, win, thr,
                              ctx=ctx)
    hr, n_und = _finish(P, res["sub"], res["piece"], res["k"], res["cls"])
    stats["undecided"] = n_und
    return hr, stats


def run_plain(P: Prepared, dev_args=None, ctx=None):
    spec = P.spec
    table, win, thr = dev_args or upload(P)
    n_sub = len(P.subs)
    a, b = api.tabulate(table, n_sub, spec.delta, spec.tau, spec.W, ctx=ctx)
    N = api.to_dev(np.full(n_sub * spec.tau, spec.N, np.uint32), torch.uint32, a.device)
    lo = api.to_dev(P.win[:, 0], torch.uint64, a.device)
    d = api.to_dev(P.win[:, 1], torch.uint64, a.device)
    # expected candidates: every argument of a sub-interval lands in its
    # window with probability d / 2^64; size the buffer for one pass
    expect = float(P.win[:, 1].astype(np.float64).sum()) / 2.0 ** 64 * spec.per_sub
    cap = int(expect * 1.25) + (1 << 16)
    counts, offsets, hits, inst = api.search(a, b, N, d, lo=lo, group=spec.tau, with_inst=True,
                                             cap=cap, ctx=ctx)
    value, cls = api.recheck(table, n_sub, spec.delta, spec.tau, spec.W, inst, hits, spec.N - 1,
                             thr, ctx=ctx)
    cls_h = cls.cpu().numpy()
    keep = cls_h != 0
    inst_h = inst.cpu().numpy()[keep].astype(np.int64)
    k_h = hits.cpu().numpy()[keep]
    hr, n_und = _finish(P, inst_h // spec.tau, inst_h % spec.tau, k_h, cls_h[keep])
    return hr, {"pieces": n_sub * spec.tau, "candidates": int(hits.numel()),
                "results": int(keep.sum()), "undecided": n_und}


class UpperPrepared:
    """Host part of a job whose sub-interval tables the device makes: the
    range's upper table, and the window and thresholds shared by all its
    sub-intervals (same fields as Prepared where the finish step reads them)."""

    def __init__(self, spec: JobSpec, Du: int, Wu: int):
        self.spec = spec
        self.Du, self.Wu = Du, Wu
        self.U = upper_table(spec.fname, spec.X0, spec.count, spec.s, spec.mode, spec.per_sub,
                             Du, Wu)
        self.win, self.thr, self.mu = upper_windows(self.U, spec.N, spec.tau, spec.delta, spec.W)
        self.subs = np.arange(spec.n_sub, dtype=np.int64)
        self.uf = self.U.uf


def upload_upper(Pu: UpperPrepared, device="cuda"):
    """Upper table, and per-sub-interval window and threshold arrays (the
    shared values repeated), on the device."""
    n = Pu.spec.n_sub
    upper = api.to_dev_async(Pu.U.words.reshape(-1), torch.uint64, device)
    win = api.to_dev_async(Pu.win, torch.uint64, device).repeat(n)
    thr = api.to_dev_async(Pu.thr, torch.uint64, device).repeat(n)
    return upper, win, thr


def make_tables(Pu: UpperPrepared, upper, ctx=None, stream=None, out=None):
    spec = Pu.spec
    return api.subtables(upper, Pu.Du, Pu.Wu, spec.n_sub, spec.delta, spec.W, spec.N, ctx=ctx,
                         stream=stream, out=out)


def run_upper(Pu: UpperPrepared, ctx=None):
    upper, win, thr = upload_upper(Pu)
    table = make_tables(Pu, upper, ctx=ctx)
    return run_fused(Pu, dev_args=(table, win, thr), ctx=ctx)


def search_job(spec: JobSpec, form: str = "fused", subs=None, ctx=None, Du=None, Wu=None):
    if form == "upper":
        from .autotune import choose_upper_degree, choose_upper_width
        Du = Du or choose_upper_degree(spec.fname, spec.X0, spec.count, spec.s, spec.delta)
        Wu = Wu or choose_upper_width(Du, spec.n_sub, spec.N, spec.tau, spec.delta, spec.s)
        return run_upper(UpperPrepared(spec, Du, Wu), ctx=ctx)
    P = prepare(spec, subs)
    return (run_fused if form == "fused" else run_plain)(P, ctx=ctx)
