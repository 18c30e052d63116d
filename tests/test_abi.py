"""CPU checks of the C ABI: the library loads and exports what the header declares."""
import ctypes
import re

import pytest

from paper_1211_3056_amd import _lib


def _declared():
    text = open(_lib.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hr_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(_lib.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_version_and_status_strings():
    L = _lib.lib()
    assert L.hr_abi_version() == 1
    assert _lib.status_str(0) == "ok"
    assert "invalid" in _lib.status_str(-1)
    assert _lib.status_str(12345) == "unknown status"


def test_invalid_arguments_rejected_before_any_device_call():
    L = _lib.lib()
    P = ctypes.c_void_p
    assert L.hr_create(None, 0) == _lib.HR_EINVAL
    assert L.hr_search(None, None, None, None, 0, None, None, 1, None, None, None, None, 0, None, None) == _lib.HR_EINVAL
    assert L.hr_tabulate(None, None, 1, 3, 16, 192, None, None, None) == _lib.HR_EINVAL
    assert L.hr_destroy(None) == _lib.HR_OK


def test_record_layouts():
    from paper_1211_3056_amd import api
    assert _lib.RESULT_BYTES == 32 == api.RESULT_DTYPE.itemsize
    assert _lib.ITEM_BYTES == 88 == api.ITEM_DTYPE.itemsize
    # field offsets of the numpy views match the C structs
    for name, _ in _lib.hr_item._fields_:
        assert getattr(_lib.hr_item, name).offset == api.ITEM_DTYPE.fields[name][1]
    for name, _ in _lib.hr_result._fields_:
        assert getattr(_lib.hr_result, name).offset == api.RESULT_DTYPE.fields[name][1]


def _params():
    """Parameter count of every function the header declares."""
    text = open(_lib.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for name, args in re.findall(r"\b(hr_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", text):
        args = args.strip()
        out[name] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_argument_counts_match_header():
    L = _lib.lib()
    for name, n in _params().items():
        assert len(getattr(L, name).argtypes) == n, name


def test_header_constants_match_binding():
    text = open(_lib.HEADER).read()
    fill = int(re.search(r"#define HR_WAVES_FILL\s+(0x[0-9a-fA-F]+)u", text).group(1), 16)
    assert fill == _lib.HR_WAVES_FILL
    assert int(re.search(r"#define HR_FILTER_LEFEVRE (\d+)", text).group(1)) == _lib.HR_FILTER_LEFEVRE
    assert int(re.search(r"#define HR_FILTER_REGULAR (\d+)", text).group(1)) == _lib.HR_FILTER_REGULAR
    codes = dict(re.findall(r"\b(HR_E[A-Z]+|HR_OK)\s*=\s*(-?\d+)", text))
    assert {k: int(v) for k, v in codes.items()} == {
        "HR_OK": _lib.HR_OK, "HR_EINVAL": _lib.HR_EINVAL, "HR_ECAPACITY": _lib.HR_ECAPACITY,
        "HR_EDEVICE": _lib.HR_EDEVICE, "HR_ENOMEM": _lib.HR_ENOMEM,
        "HR_ESCRATCH": _lib.HR_ESCRATCH}
    sbytes = int(re.search(r"#define HR_STATIC_SCRATCH_BYTES \(1u << (\d+)\)", text).group(1))
    assert _lib.HR_STATIC_MAX_INSTANCES == ((1 << sbytes) // 8 - 1) * 256


def _gpu_visible():
    import torch
    return torch.cuda.is_available()


@pytest.mark.skipif(_gpu_visible(), reason="stand-in context is only safe where no device exists")
def test_each_parameter_check_returns_before_the_device():
    """One invalid parameter per call, every other argument plausible: each
    entry point rejects it on the host.  The context is a zeroed stand-in
    and the buffers are host memory; a check that let the call through would
    reach hipSetDevice, which fails here (no device) with HR_EDEVICE instead
    of HR_EINVAL.  Empty inputs return HR_OK the same way."""
    L = _lib.lib()
    ctx = ctypes.create_string_buffer(256)
    buf = ctypes.create_string_buffer(1 << 12)
    c, p = ctypes.addressof(ctx), ctypes.addressof(buf)
    E, OK, DEV = _lib.HR_EINVAL, _lib.HR_OK, _lib.HR_EDEVICE
    big = (1 << 32) - 1                     # big^5 >= 2^128, big^4 < 2^128

    def tab(deg=3, tau=16, width=128, table=p, n_sub=1):
        return L.hr_tabulate(c, table, n_sub, deg, tau, width, p, p, None)
    assert tab() == DEV             # all valid: reaches the device
    for kw in ({"deg": 0}, {"deg": 7}, {"width": 64}, {"width": 320}, {"tau": 0},
               {"deg": 5, "tau": big}, {"table": None}):
        assert tab(**kw) == E, kw
    assert tab(n_sub=0) == OK

    def rck(deg=3, tau=16, width=128, max_k=100, thr=p, n_cand=1):
        return L.hr_recheck(c, p, 1, deg, tau, width, p, p, n_cand, max_k, thr, p, p, None)
    assert rck() == DEV
    for kw in ({"deg": 7}, {"width": 0}, {"tau": 0}, {"deg": 5, "max_k": big},
               {"deg": 5, "tau": big}, {"thr": None}):
        assert rck(**kw) == E, kw
    assert rck(n_cand=0) == OK

    def pip(deg=3, tau=16, width=128, N=1 << 10, win=p, out=p, cap=1, count=p, n_sub=1):
        return L.hr_pipeline(c, p, n_sub, deg, tau, width, N, win, p, out, cap, count, None, None)
    assert pip() == DEV
    for kw in ({"deg": 0}, {"width": 192 + 1}, {"tau": 0}, {"N": 0}, {"deg": 5, "N": big},
               {"count": None}, {"win": None}, {"out": None}):
        assert pip(**kw) == E, kw
    assert pip(out=None, cap=0) == DEV     # no output wanted: no buffer needed
    assert pip(n_sub=0) == OK

    def qck(cap=1 << 10, out=p, n=1):
        return L.hr_quot_check(c, p, p, cap, out, None, n, None)
    assert qck() == DEV
    for kw in ({"cap": 0}, {"cap": 1 << 32}, {"out": None}):
        assert qck(**kw) == E, kw
    assert qck(n=0) == OK

    def bat(n_items=1, width=128, deg=3, items=p, out=p, cap=1, count=p):
        return L.hr_batch_run(c, p, items, n_items, width, deg, 0, out, cap, count, None, None)
    assert bat() == DEV
    for kw in ({"n_items": 1 << 31}, {"deg": 0}, {"width": 100}, {"count": None},
               {"items": None}, {"out": None}):
        assert bat(**kw) == E, kw
    assert bat(n_items=0) == OK

    def sch(n=1, group=1, win_d=p, total=p, hits=p, cap=1, counts=p):
        return L.hr_search(c, p, p, p, n, p, win_d, group, counts, p, hits, p, cap, total, None)
    assert sch() == DEV
    for kw in ({"group": 0}, {"n": 1 << 32}, {"win_d": None}, {"total": None},
               {"hits": None}, {"counts": None}):
        assert sch(**kw) == E, kw

    def sub(du=7, wu=320, deg=4, width=256, max_t=4095, max_N=1 << 18, N=1 << 18, n_sub=1,
            upper=p, out=p, t_idx=None, N_per=None, t0=0):
        return L.hr_subtables(c, upper, du, wu, t_idx, t0, N_per, N, max_t, max_N, n_sub, deg,
                              width, out, None)
    assert sub() == DEV
    for kw in ({"du": 0}, {"du": 11}, {"wu": 200}, {"wu": 512}, {"wu": 128}, {"deg": 0},
               {"deg": 8}, {"width": 320}, {"width": 64}, {"du": 3, "deg": 4},
               {"wu": 192, "width": 256}, {"max_t": (1 << 32) - 1},
               {"max_N": 0}, {"max_N": (1 << 32) - 1, "N": 5, "du": 10},
               {"N": 0}, {"N": (1 << 18) + 1}, {"t0": 4095, "n_sub": 2},
               {"upper": None}, {"out": None}):
        assert sub(**kw) == E, kw
    assert sub(t_idx=p, t0=1 << 20, n_sub=2) == DEV     # t from the device array
    assert sub(N_per=p, N=0) == DEV                     # N from the device array
    assert sub(n_sub=0) == OK

    def sst(n=1, group=1, win_d=p, total=p, hits=p, cap=1, counts=p):
        return L.hr_search_static(c, p, p, p, n, p, win_d, group, counts, p, hits, p, cap, total,
                                  None)
    assert sst() == DEV
    for kw in ({"group": 0}, {"n": 1 << 32}, {"win_d": None}, {"total": None},
               {"hits": None}, {"counts": None}):
        assert sst(**kw) == E, kw
    assert sst(n=_lib.HR_STATIC_MAX_INSTANCES + 1) == _lib.HR_ESCRATCH
    assert sst(n=_lib.HR_STATIC_MAX_INSTANCES) == DEV

    def sps(n=1, group=1, win_d=p, steps=p):
        return L.hr_search_steps(c, p, p, p, n, p, win_d, group, steps, None)
    assert sps() == DEV
    for kw in ({"group": 0}, {"n": 1 << 32}, {"win_d": None}, {"steps": None}):
        assert sps(**kw) == E, kw
    assert sps(n=0) == OK

    def flt(alg=1, n=1, group=1, win_d=p, passed=p):
        return L.hr_filter(c, alg, p, p, p, n, p, win_d, group, passed, None, None, None)
    assert flt() == DEV and flt(alg=2) == DEV
    for kw in ({"alg": 0}, {"alg": 3}, {"group": 0}, {"n": 1 << 32}, {"win_d": None},
               {"passed": None}):
        assert flt(**kw) == E, kw
    assert flt(n=0) == OK

    # streamed launches: every check before the device
    h = ctypes.c_void_p()
    assert L.hr_batch_open(None, 4, ctypes.byref(h)) == E
    assert L.hr_batch_open(c, 0, ctypes.byref(h)) == E
    assert L.hr_batch_open(c, 2000, ctypes.byref(h)) == E
    assert L.hr_batch_open(c, 4, None) == E
    assert L.hr_batch_open(c, 4, ctypes.byref(h)) == DEV
    t = ctypes.c_uint64()
    assert L.hr_batch_submit(None, p, p, 1, 128, 3, p, 1, p, None, ctypes.byref(t)) == E
    assert L.hr_batch_poll(None, ctypes.byref(t)) == E
    assert L.hr_batch_wait(None, 1) == E
    assert L.hr_batch_close(None) == OK
