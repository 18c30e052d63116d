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
    codes = dict(re.findall(r"\b(HR_E[A-Z]+|HR_OK)\s*=\s*(-?\d+)", text))
    assert {k: int(v) for k, v in codes.items()} == {
        "HR_OK": _lib.HR_OK, "HR_EINVAL": _lib.HR_EINVAL, "HR_ECAPACITY": _lib.HR_ECAPACITY,
        "HR_EDEVICE": _lib.HR_EDEVICE, "HR_ENOMEM": _lib.HR_ENOMEM}
