"""Host-side checks of the C-ABI library (no GPU needed): it loads and exports every entry
point that include/drt.h declares; host-only helpers behave; a missing library fails loudly."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "drt.h")
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared(headers=(HEADER,)):
    names = set()
    for h in headers:
        text = open(h).read()
        names |= set(re.findall(r"^\s*(?:int|double|const char \*)\s*(drt_\w+)\s*\(", text, re.M))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("drt_create", "drt_destroy", "drt_load_scene", "drt_unload_scene", "drt_extrapolate",
              "drt_cfr", "drt_submit", "drt_poll", "drt_strerror", "drt_last_error", "drt_now"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2205_00237_amd import _abi
    lib = ctypes.CDLL(_abi.LIB_PATH)
    every = _declared(HEADERS)
    assert len(every) > len(_declared())
    for n in every:
        assert hasattr(lib, n), n
    assert set(_abi.EXPORTS) == set(_declared())
    assert set(_abi.EXPORTS) | set(_abi.PROBE_EXPORTS) == set(every)


def test_host_only_helpers():
    from paper_2205_00237_amd import _abi
    assert _abi.LIB.drt_strerror(_abi.DRT_E_DEGENERATE).decode() == "degenerate ray at t0"
    assert _abi.LIB.drt_strerror(12345).decode() == "unknown status"
    t1 = _abi.drt_now()
    t2 = _abi.drt_now()
    assert t2 >= t1 > 0


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2205_00237_amd import _abi
    monkeypatch.setattr(_abi, "LIB_PATH", os.path.join(ROOT, "no_such_libdrt.so"))
    with pytest.raises(ImportError):
        _abi._load()


def test_struct_layouts_match_the_header():
    """ctypes mirrors of the C structs: sizes fixed by the header's member lists (x86-64 ABI)."""
    from paper_2205_00237_amd import _abi
    assert ctypes.sizeof(_abi.TimeGrid) == 16
    assert ctypes.sizeof(_abi.FreqGrid) == 24
    assert ctypes.sizeof(_abi.RayOut) == 64
    assert ctypes.sizeof(_abi.Request) == 4 + 4 + 16 + 24 + 4 + 4 + 8
    assert ctypes.sizeof(_abi.ReqStat) == 32
