"""Host code of the library under the sanitizers, on the CPU.

AddressSanitizer and UndefinedBehaviorSanitizer (g++, every finding fatal):

* the shared device header's field functions (transition function, UTD coefficient,
  Fresnel, effective-roughness normalisation, the bounded binary32 sin/cos) over the input
  ranges the kernels see, including the shadow-boundary limits, grazing and normal
  incidence, zero and huge transition arguments;
* the scene loader (validation and packing, the t0 solve of every ray, the by-value copy of
  a description and its carriage to another instant) and the per-ray geometry the kernels
  evaluate, on every signature class, moving and rotating bodies, facets and edge segments,
  dipole antennas and two-edge rays, against the oracle; and every rejection of a bad
  description, each with its error code.

Every array the probe hands the loader is allocated at exactly its length, so a read past
what the description holds is a sanitizer error.

ThreadSanitizer (clang's runtime, which intercepts the condition-variable waits of
libstdc++): the runtime's host code, scheduler included, built against a host stand-in of the
HIP API (tests/host/fake_hip: work completes at once, device memory is host memory, graph
capture records its nodes) and driven by tests/host/serve_stress.cpp: three submitter
threads, a poller, a direct drt_cfr / drt_extrapolate caller and the scheduler thread at once,
the served results compared with drt_cfr, then a context destroyed with requests queued.
Linked with the real ROCm runtime, the sanitizer's shadow mappings leave the runtime no GPU
(it reports no device), hence the stand-in."""
import math
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2205_00237_amd import scenes
from paper_2205_00237_amd._abi import DRT_E_INVAL, DRT_E_DEGENERATE, DRT_E_INCONSISTENT

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_oracle_polar import _with_dipoles  # noqa: E402
from test_oracle_double_diffraction import _two_screens  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C0 = 299_792_458.0
SAN = ["-O1", "-g", "-std=c++20", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
       "-I", os.path.join(ROOT, "paper_2205_00237_amd", "csrc"), "-x", "c++"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _build(tmp_path_factory, src, name):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("g++ or the HIP headers not available")
    exe = str(tmp_path_factory.mktemp("asan") / name)
    r = subprocess.run([gxx] + SAN + [os.path.join(ROOT, "tests", "host", src), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, text):
    r = subprocess.run([exe], input=text, capture_output=True, text=True, env=ENV)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, \
        f"exit {r.returncode}\n{r.stderr[-3000:]}"
    return r.stdout.strip().splitlines()


@pytest.fixture(scope="module")
def field_probe(tmp_path_factory):
    return _build(tmp_path_factory, "geom_probe.cpp", "geom_probe_asan")


@pytest.fixture(scope="module")
def loader_probe(tmp_path_factory):
    return _build(tmp_path_factory, "loader_probe.cpp", "loader_probe_asan")


def test_field_functions_clean_under_sanitizers(field_probe):
    rng = np.random.default_rng(5)
    lines = []
    for X in np.concatenate([[0.0, 1e-300, 1e-30, 1e-9, 3.99999, 4.0, 4.00001, 11.99, 12.0, 39.9, 40.0, 1e8, 1e300],
                             np.logspace(-12, 12, 200)]):
        lines += [f"F64 {X!r}", f"F32 {X!r}"]
    for _ in range(300):
        n = rng.choice([1.0 + 1e-9, 1.5, 2.0, rng.uniform(1.05, 2.0)])
        phi, php = rng.uniform(0, n * math.pi, 2)
        sb, k, Ld, pol = rng.uniform(1e-6, 1), rng.uniform(1.0, 3e3), rng.uniform(1e-9, 1e4), int(rng.integers(2))
        args = " ".join(repr(float(v)) for v in (phi, php, sb, n, k, Ld))
        lines += [f"D64 {args} {pol}", f"D32 {args} {pol}"]
    for pol in (0, 1):
        for php in (0.0, 0.3, math.pi / 2, 1.1):
            for phi in (math.pi + php, math.pi - php, 0.0, 1.5 * math.pi):
                lines += [f"D64 {phi!r} {php!r} 1.0 1.5 586.7 12.0 {pol}", f"D32 {phi!r} {php!r} 1.0 1.5 586.7 12.0 {pol}"]
    for ct in (0.0, 1e-12, 0.5, 1.0):
        for pec in (0, 1):
            for pol in (0, 1):
                lines += [f"G64 {ct!r} 4.0 0.5 0.01 {pec} {pol}", f"G32 {ct!r} 4.0 0.5 0.01 {pec} {pol}"]
    for x in np.linspace(-8, 8, 101):
        lines.append(f"SC32 {float(x)!r}")
    for alpha in range(0, 9):
        for ct in (1e-9, 0.3, 1.0):
            lines.append(f"ER64 {alpha} {ct!r}")
    out = _run(field_probe, "\n".join(lines) + "\n")
    assert len(out) == len(lines)
    vals = np.array([float(v) for l in out for v in l.split()])
    assert np.isfinite(vals).all()


# ----------------------------------------------------------------------------------------
# the loader

_F64 = ("t0", "tx_p", "tx_v", "tx_a", "rx_p", "rx_v", "rx_a", "body_O0", "body_v0", "body_a", "body_axis",
        "body_w0", "body_wdot", "mat_eps_r", "mat_sigma", "plane_p0", "plane_n0", "plane_facet", "edge_a0",
        "edge_e0", "edge_t0", "edge_n0", "edge_wedge_n", "edge_zlim", "tile_c0", "tile_n0", "tile_area",
        "tile_S", "tile_phase0", "ray_q0", "tx_ant", "rx_ant")
_INT = ("mat_pec", "plane_body", "plane_mat", "edge_body", "tile_body", "tile_alpha", "tile_model",
        "ray_nint", "ray_kind", "ray_pol", "ray_prim")


def _scene_text(s, null=()):
    out = []
    for k in _F64 + _INT:
        if k in null or k not in s:
            out.append(f"A {k} -1")
        else:
            a = np.asarray(s[k]).ravel()
            if k in _INT:
                vals = " ".join(str(int(v)) for v in a)
            else:
                vals = " ".join(repr(float(v)) for v in a.astype(np.float64))
            out.append(f"A {k} {a.size} {vals}")
    return "\n".join(out) + "\n"


def _status(line):
    w = line.split(" ", 2)
    assert w[0] == "status", line
    return int(w[1]), (w[2] if len(w) > 2 else "")


def _parse(lines, R, T):
    a = np.array([[float(v) for v in l.split()] for l in lines])
    assert a.shape == (R * T, 11)
    return a.reshape(R, T, 11)


def _compare(got, ref, f_c, g64, where):
    valid = got[..., 8].astype(bool)
    assert np.array_equal(valid, ref["valid"]), f"{where}: valid differs at {np.argwhere(valid != ref['valid'])[:5]}"
    ib = got[..., 9].astype(bool)
    near = np.abs(ref["bounds_margin"]) < 1e-9
    assert not ((ib != ref["in_bounds"]) & ~near).any(), f"{where}: in_bounds differs"
    v = ref["valid"]
    assert np.abs(got[..., 0][v] - ref["L"][v]).max(initial=0) <= 1e-9, f"{where}: L"
    assert (np.abs(got[..., 1] - ref["dop"])[v] <= 1e-6 + 1e-9 * np.abs(ref["dop"][v])).all(), f"{where}: doppler"
    for j, k in enumerate(("aod_az", "aod_el", "aoa_az", "aoa_el")):
        d = np.abs(got[..., 4 + j] - ref[k])
        d = np.minimum(d, 2 * math.pi - d)[v]
        assert (d <= (1e-9 if g64 else 1e-6)).all(), f"{where}: {k} {d.max(initial=0)}"
    g = (got[..., 2] + 1j * got[..., 3])[v]
    gr = ref["gain"][v]
    if g64:
        tol = 1e-9 * np.abs(gr) + 1e-12 * np.abs(gr).max(initial=0)
    else:
        fs = (C0 / f_c) / (4 * math.pi * ref["L"][v])
        tol = 1e-5 * np.abs(gr) + 3e-6 * fs + 1e-12 * np.abs(gr).max(initial=0)
    assert (np.abs(g - gr) <= tol).all(), f"{where}: gain {(np.abs(g - gr) / np.abs(gr)).max(initial=0)}"


def _subset_by_class(s, per_class, seed=0):
    rng = np.random.default_rng(seed)
    sig = np.array([scenes.signature(s, r) for r in range(len(s["ray_nint"]))])
    pick = []
    for c in np.unique(sig):
        idx = np.flatnonzero(sig == c)
        pick += list(rng.choice(idx, min(per_class, idx.size), replace=False))
    return scenes.subset_rays(s, np.sort(np.array(pick)))


def _case(name):
    if name in ("config1", "dipoles"):
        s, tg, fg = scenes.config1()
        if name == "dipoles":
            return _with_dipoles(s, (0.3, 0.2, 1.0), (-0.2, 0.5, 1.0)), fg.f_c, np.array([0.0, 0.05])
        return s, fg.f_c, np.arange(0, 100, 9) * tg.dt
    if name == "urban":
        s, tg, fg = scenes.config2(scale=1)
        return _subset_by_class(s, 25), fg.f_c, np.array([0.0, 0.013, 0.05, 0.099])
    if name == "scattering":
        s, tg, fg = scenes.config3(n_boxes=4, tiles_per_box=40, n_steps=20)
        return _subset_by_class(s, 80), fg.f_c, np.array([0.0, 0.004, 0.019])
    s, _ = _two_screens()
    return dict(s, tx_v=np.array([1.0, 0.5, 0.0]), rx_v=np.array([-2.0, 0.0, 0.1])), 3e9, np.array([0.0, 0.2, 0.5])


@pytest.mark.parametrize("case", ["config1", "urban", "scattering", "dipoles", "two-edge"])
def test_loader_and_geometry_clean_under_sanitizers(loader_probe, case):
    name = case
    s, f_c, ts = _case(case)
    R, T = len(s["ray_nint"]), len(ts)
    shift = ts[len(ts) // 2]
    later = ts[ts >= shift]
    tline = " ".join(repr(float(t)) for t in ts)
    lline = " ".join(repr(float(t - shift)) for t in later)
    text = (_scene_text(s) + f"FC {float(f_c)!r}\nPACK\nEVAL 64 {T} {tline}\nEVAL 32 {T} {tline}\n"
            f"REBASE {float(shift)!r}\nEVAL 64 {len(later)} {lline}\n")
    out = _run(loader_probe, text)
    st, msg = _status(out[0])
    assert st == 0, msg
    ref = oracle.extrapolate(s, ts, f_c)
    assert ref["valid"].mean() > 0.3, f"{name}: too few valid rays to compare"
    _compare(_parse(out[1:1 + R * T], R, T), ref, f_c, True, f"{name} binary64")
    _compare(_parse(out[1 + R * T:1 + 2 * R * T], R, T), ref, f_c, False, f"{name} binary32 field")
    st, msg = _status(out[1 + 2 * R * T])
    assert st == 0, msg
    k = np.flatnonzero(ts >= shift)
    sub = {key: v[:, k] for key, v in ref.items() if isinstance(v, np.ndarray) and v.ndim == 2}
    _compare(_parse(out[2 + 2 * R * T:], R, len(later)), sub, f_c, True, f"{name} carried to t0 + {shift}")


def _bad(s, **kw):
    s = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in s.items()}
    for k, f in kw.items():
        f(s)
    return s


def _set(key, idx, val):
    def f(s):
        s[key][idx] = val
    return f


def _bad_descriptions():
    s, _, _ = scenes.config1()
    nr = len(s["ray_nint"])
    q0 = oracle.extrapolate(s, np.array([0.0]), 28e9, keep_points=True)["points"]
    yield "null body array", s, {"body_v0"}, None, DRT_E_INVAL
    yield "axis not unit", _bad(s, a=_set("body_axis", (1, 2), 0.9)), (), None, DRT_E_INVAL
    yield "plane body range", _bad(s, a=_set("plane_body", 2, 7)), (), None, DRT_E_INVAL
    yield "plane material range", _bad(s, a=_set("plane_mat", 0, -1)), (), None, DRT_E_INVAL
    yield "material", _bad(s, a=_set("mat_eps_r", 0, -2.0)), (), None, DRT_E_INVAL
    yield "edge wedge", _bad(s, a=_set("edge_wedge_n", 1, 2.5)), (), None, DRT_E_INVAL
    yield "edge limits", _bad(s, a=_set("edge_zlim", (0, 0), 9.0)), (), None, DRT_E_INVAL
    yield "tile alpha", _bad(s, a=_set("tile_alpha", 3, 9)), (), None, DRT_E_INVAL
    yield "tile area", _bad(s, a=_set("tile_area", 0, 0.0)), (), None, DRT_E_INVAL
    yield "facet sides", _bad(s, a=_set("plane_facet", (1, 2), s["plane_facet"][1, 1])), (), None, DRT_E_INVAL
    yield "too many interactions", _bad(s, a=_set("ray_nint", 1, 5)), (), None, DRT_E_INVAL
    yield "interaction kind", _bad(s, a=_set("ray_kind", (1, 0), 7)), (), None, DRT_E_INVAL
    yield "primitive range", _bad(s, a=_set("ray_prim", (1, 0), 10 ** 6)), (), None, DRT_E_INVAL
    yield "polarisation flag", _bad(s, a=_set("ray_pol", (2, 0), 3)), (), None, DRT_E_INVAL
    yield "scatter not alone", _bad(s, a=_set("ray_nint", nr - 1, 2)), (), None, DRT_E_INVAL
    one_antenna = dict(s, tx_ant=np.array([0.0, 0.0, 1.0, 1.0]))
    yield "one antenna", one_antenna, (), None, DRT_E_INVAL
    # both terminals on the ground plane: the ground reflection is degenerate at t0
    on_ground = dict(s, tx_p=np.array([0.0, 0.0, 0.0]), rx_p=np.array([50.0, 0.0, 0.0]))
    yield "terminals on a wall", on_ground, (), None, DRT_E_DEGENERATE
    pts = [[np.asarray(p)[0] for p in (q0[r] or [])] for r in range(nr)]
    yield "consistent points", s, (), pts, 0
    wall = int(np.flatnonzero(np.asarray(s["ray_nint"]) == 1)[0])
    moved = [list(p) for p in pts]
    moved[wall][0] = moved[wall][0] + np.array([0.0, 0.0, 1e-3])
    yield "inconsistent points", s, (), moved, DRT_E_INCONSISTENT


def _q0_array(pts, nr):
    q = np.zeros((nr, 4, 3))
    for r, p in enumerate(pts):
        for i, x in enumerate(p):
            q[r, i] = x
    return q


def test_loader_rejections_clean_under_sanitizers(loader_probe):
    cases = list(_bad_descriptions())
    text = ""
    for name, s, null, q, code in cases:
        s2 = dict(s)
        if q is not None:
            s2["ray_q0"] = _q0_array(q, len(s["ray_nint"]))
        text += _scene_text(s2, null=null) + "PACK\n"
    out = _run(loader_probe, text)
    assert len(out) == len(cases)
    for (name, s, null, q, code), line in zip(cases, out):
        st, msg = _status(line)
        assert st == code, f"{name}: status {st} ({msg}), expected {code}"


def test_scheduler_under_thread_sanitizer(tmp_path):
    clang = "/opt/rocm/lib/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("clang++ not available")
    exe = str(tmp_path / "serve_stress_tsan")
    csrc = os.path.join(ROOT, "paper_2205_00237_amd", "csrc")
    host = os.path.join(ROOT, "tests", "host")
    cmd = [clang, "-O1", "-g", "-std=c++20", "-fsanitize=thread", "-fno-omit-frame-pointer",
           "-I", os.path.join(host, "fake_hip"), "-I", os.path.join(ROOT, "include"), "-I", csrc,
           "-idirafter", "/opt/rocm/include",
           "-x", "c++", os.path.join(csrc, "runtime.hip"), "-x", "c++", os.path.join(csrc, "plan.hip"),
           "-x", "c++", os.path.join(host, "fake_kernels.cpp"), "-x", "c++", os.path.join(host, "serve_stress.cpp"),
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert "ThreadSanitizer" not in r.stderr and r.returncode == 0, r.stderr[-4000:]
    assert "served requests equal to drt_cfr" in r.stdout
