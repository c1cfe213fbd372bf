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
              "drt_cfr", "drt_cfr_nufft", "drt_power_profiles", "drt_trace", "drt_scene_rays",
              "drt_segments", "drt_submit", "drt_poll", "drt_strerror", "drt_last_error", "drt_now"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2205_00237_amd import _abi
    lib = ctypes.CDLL(_abi.LIB_PATH)
    every = _declared(HEADERS)
    for n in every:
        assert hasattr(lib, n), n
    assert set(_abi.EXPORTS) == set(every)
    assert not any(n.startswith("drt_probe") for n in every)


def test_probe_library_is_separate():
    """The hardware probes live in a test-only library with its own header under tests/."""
    import probe
    hdr = os.path.join(ROOT, "tests", "probe", "drt_probe.h")
    assert set(_declared((hdr,))) == set(probe.EXPORTS)
    lib = ctypes.CDLL(probe.PATH)
    for n in probe.EXPORTS:
        assert hasattr(lib, n), n
    from paper_2205_00237_amd import _abi
    main = ctypes.CDLL(_abi.LIB_PATH)
    for n in probe.EXPORTS:
        assert not hasattr(main, n), n


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


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of the C structs: size and every member offset equal to what a C
    compiler makes of include/drt.h."""
    import shutil
    import subprocess
    from paper_2205_00237_amd import _abi
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    pairs = [("drt_scene_desc", _abi.SceneDesc), ("drt_time_grid", _abi.TimeGrid),
             ("drt_freq_grid", _abi.FreqGrid), ("drt_ray_out", _abi.RayOut),
             ("drt_request", _abi.Request), ("drt_req_stat", _abi.ReqStat),
             ("drt_profile", _abi.Profile), ("drt_serving_stats", _abi.ServingStats),
             ("drt_bins", _abi.Bins), ("drt_power_out", _abi.PowerOut),
             ("drt_trace_opts", _abi.TraceOpts), ("drt_trace_info", _abi.TraceInfo),
             ("drt_refresh_opts", _abi.RefreshOpts)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "drt.h"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'  printf("{cname}.{f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for cname, cls in pairs:
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert int(got[f"{cname}.{f[0]}"]) == getattr(cls, f[0]).offset, (cname, f[0])
