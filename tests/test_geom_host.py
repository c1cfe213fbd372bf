"""CPU check of the field-coefficient functions of the kernels' shared header
(paper_2205_00237_amd/csrc/drt_geom.h), compiled for the host, against the oracle."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import em

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("probe") / "geom_probe")
    cmd = [HIPCC, "-O2", "-std=c++20", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
           "-I", os.path.join(ROOT, "paper_2205_00237_amd", "csrc"), "-x", "c++",
           os.path.join(ROOT, "tests", "host", "geom_probe.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

    def run(lines):
        out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
        return [list(map(float, l.split())) for l in out.stdout.strip().splitlines()]
    return run


def test_transition_function(probe):
    X = np.concatenate([np.logspace(-9, 6, 300), [4.4999999, 4.5, 4.5000001, 4.0, 3.99999]])
    got64 = probe([f"F64 {float(x)!r}" for x in X])
    got32 = probe([f"F32 {float(x)!r}" for x in X])
    ref = em.utd_transition(X)
    for x, g, g32, r in zip(X, got64, got32, ref):
        assert abs(complex(*g) - r) <= 1e-13 * abs(r) + 1e-300, (x, g, r)
        assert abs(complex(*g32) - r) <= 3e-6 * abs(r), (x, g32, r)


def test_wedge_coefficient(probe):
    rng = np.random.default_rng(0)
    lines, args = [], []
    for _ in range(400):
        n = rng.choice([1.5, 2.0, rng.uniform(1.1, 2.0)])
        phi, php = rng.uniform(0, n * math.pi, 2)
        sb, k, Ld, pol = rng.uniform(0.2, 1), rng.choice([125.7, 586.7, 1257.0]), rng.uniform(0.1, 300), int(rng.integers(2))
        lines.append("D64 " + " ".join(repr(float(v)) for v in (phi, php, sb, n, k, Ld)) + f" {pol}")
        args.append((phi, php, sb, n, k, Ld, pol))
    # exactly on the incidence and reflection shadow boundaries (limit branch)
    for pol in (0, 1):
        for php in (0.3, 1.1):
            for phi in (math.pi + php, math.pi - php):
                lines.append(f"D64 {phi!r} {php!r} 1.0 1.5 586.7 12.0 {pol}")
                args.append((phi, php, 1.0, 1.5, 586.7, 12.0, pol))
    got = probe(lines)
    got32 = probe([l.replace("D64", "D32") for l in lines])
    for a, g, g32 in zip(args, got, got32):
        r = complex(em.utd_coefficient(*a))
        assert abs(complex(*g) - r) <= 1e-11 * abs(r), (a, g, r)
        # binary32 field arithmetic on binary64-formed boundary distances (split mode):
        # relative to the size of the four cot*F terms, which can cancel to a small D
        phi, php, sb, n, k, Ld, pol = a
        terms = sum(abs(complex(em._cot_F(b, sg, n, k * Ld))) for b in (phi - php, phi + php) for sg in (1.0, -1.0))
        pre = 1.0 / (2 * n * math.sqrt(2 * math.pi * k) * sb)
        assert abs(complex(*g32) - r) <= 3e-6 * abs(r) + 3e-7 * pre * terms, (a, g32, r)


def test_bounded_sincos32(probe):
    """The binary32 sin / cos of the field code against the binary64 library on |x| <= 8:
    absolute error near rounding, and relative accuracy of sin kept near zero."""
    x = np.concatenate([np.linspace(-8, 8, 4001), [0.0, 1e-30, -1e-20, 1e-8, 3e-5, -2e-3],
                        np.pi / 2 * np.arange(-5, 6)]).astype(np.float32)
    got = np.array(probe([f"SC32 {float(v)!r}" for v in x]))
    xd = x.astype(np.float64)
    assert np.abs(got[:, 0] - np.sin(xd)).max() < 4e-7
    assert np.abs(got[:, 1] - np.cos(xd)).max() < 4e-7
    small = np.abs(xd) < 0.5
    nz = small & (xd != 0)
    assert (np.abs(got[nz, 0] / np.sin(xd[nz]) - 1) < 3e-7).all()
    assert (got[xd == 0, 0] == 0).all()


def test_fresnel32(probe):
    """Binary32 Fresnel coefficients (fast reciprocals) against the oracle."""
    rng = np.random.default_rng(3)
    lines, refs = [], []
    for _ in range(300):
        ct, er, sg, lam = rng.uniform(0, 1), rng.uniform(1, 20), rng.uniform(0, 2), rng.uniform(0.001, 0.1)
        pec, pol = int(rng.random() < 0.2), int(rng.integers(2))
        lines.append("G32 " + " ".join(repr(float(v)) for v in (ct, er, sg, lam)) + f" {pec} {pol}")
        refs.append(complex(em.fresnel_gamma(ct, er, sg, lam, bool(pec), pol)))
    for g, r in zip(probe(lines), refs):
        assert abs(complex(*g) - r) <= 2e-6, (g, r)


def test_fresnel_and_er_norm(probe):
    rng = np.random.default_rng(1)
    lines, refs = [], []
    for _ in range(300):
        ct, er, sg, lam = rng.uniform(0, 1), rng.uniform(1, 20), rng.uniform(0, 2), rng.uniform(0.001, 0.1)
        pec, pol = int(rng.random() < 0.2), int(rng.integers(2))
        lines.append("G64 " + " ".join(repr(float(v)) for v in (ct, er, sg, lam)) + f" {pec} {pol}")
        refs.append(complex(em.fresnel_gamma(ct, er, sg, lam, bool(pec), pol)))
    for g, r in zip(probe(lines), refs):
        assert abs(complex(*g) - r) <= 1e-14, (g, r)
    lines, refs = [], []
    for alpha in range(0, 9):
        for ct in np.linspace(0.01, 1, 23):
            lines.append(f"ER64 {alpha} {float(ct)!r}")
            refs.append(float(em.er_norm_directive(alpha, ct)))
    for g, r in zip(probe(lines), refs):
        assert abs(g[0] - r) <= 1e-14 * r
