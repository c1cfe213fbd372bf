"""Pins of the oracle's field coefficients (Fresnel, UTD, Effective Roughness) against
independent physics: refraction and power balance, a high-precision complementary error
function, the asymptotic forms of the transition function, continuity of the total
field across the shadow boundaries of a wedge, and power balance of the scattering
patterns by quadrature."""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate

from oracle import em


# ------------------------------------------------------------------ Fresnel

@pytest.mark.parametrize("eps_r", [2.0, 5.0, 9.0])
def test_fresnel_power_balance_with_snell_refraction(eps_r):
    """Lossless: |G|^2 + (n cos t_t / cos t_i) |t|^2 = 1 with t from refraction at
    sin t_t = sin t_i / n (TE: t = 2 cos_i/(cos_i + n cos_t); TM: 2 cos_i/(n cos_i + cos_t))."""
    n = math.sqrt(eps_r)
    for th in np.linspace(0.01, 1.55, 40):
        ci = math.cos(th)
        ct = math.sqrt(1 - (math.sin(th) / n) ** 2)
        t_te = 2 * ci / (ci + n * ct)
        t_tm = 2 * ci / (n * ci + ct)
        g_te = em.fresnel_gamma(ci, eps_r, 0.0, 0.1, False, 0)
        g_tm = em.fresnel_gamma(ci, eps_r, 0.0, 0.1, False, 1)
        assert abs(abs(g_te) ** 2 + n * ct / ci * t_te ** 2 - 1) < 1e-13
        assert abs(abs(g_tm) ** 2 + n * ct / ci * t_tm ** 2 - 1) < 1e-13


def test_fresnel_special_angles():
    eps = 5.0 - 0.3j
    g = em.fresnel_gamma(1.0, 5.0, 0.3 / (60 * 0.01), 0.01, False, 0)
    assert abs(g - (1 - np.sqrt(eps)) / (1 + np.sqrt(eps))) < 1e-14            # normal incidence
    th_b = math.atan(math.sqrt(4.0))
    assert abs(em.fresnel_gamma(math.cos(th_b), 4.0, 0.0, 0.1, False, 1)) < 1e-14   # Brewster
    for pol in (0, 1):
        assert abs(em.fresnel_gamma(1e-9, 4.0, 0.2, 0.1, False, pol) + 1) < 1e-8  # grazing -> -1
    rng = np.random.default_rng(0)
    ci = rng.uniform(0, 1, 500)
    for pol in (0, 1):
        g = em.fresnel_gamma(ci, rng.uniform(1, 20, 500), rng.uniform(0, 1, 500), 0.01, False, pol)
        assert (np.abs(g) <= 1 + 1e-14).all()
    # PEC flag and the highly conducting limit agree in sign convention
    for pol, ref in ((0, -1.0), (1, 1.0)):
        assert em.fresnel_gamma(0.6, 3.0, 0.0, 0.01, True, pol) == ref
        assert abs(em.fresnel_gamma(0.6, 3.0, 1e12, 0.01, False, pol) - ref) < 1e-5


# ------------------------------------------------------------------ UTD transition function

def _F_mp(X):
    """F(X) via the complementary error function at 40 digits:
    int_x^inf e^{-j t^2} dt = (sqrt(pi)/2) e^{-j pi/4} erfc(e^{j pi/4} x)."""
    mpmath.mp.dps = 40
    x = mpmath.sqrt(mpmath.mpf(X))
    w = mpmath.exp(1j * mpmath.pi / 4)
    tail = mpmath.sqrt(mpmath.pi) / 2 / w * mpmath.erfc(w * x)
    val = 2j * x * mpmath.exp(1j * mpmath.mpf(X)) * tail
    return complex(val)


def test_transition_function_against_high_precision():
    for X in [1e-8, 1e-4, 0.01, 0.1, 0.3, 1.0, 2.0, 5.0, 10.0, 50.0, 300.0, 3e3, 1e5]:
        ref = _F_mp(X)
        got = complex(em.utd_transition(X))
        assert abs(got - ref) < 1e-12 * max(1.0, abs(ref)), (X, got, ref)


def test_transition_function_asymptotes():
    for X in [200.0, 1e3, 1e4]:
        big = 1 + 1j / (2 * X) - 3 / (4 * X * X)
        assert abs(complex(em.utd_transition(X)) - big) < 20 / X ** 3
    for X in [1e-6, 1e-5, 1e-4]:
        small = (math.sqrt(math.pi * X) - 2 * X * np.exp(1j * math.pi / 4)
                 - 2 / 3 * X * X * np.exp(-1j * math.pi / 4)) * np.exp(1j * (math.pi / 4 + X))
        assert abs(complex(em.utd_transition(X)) - small) < 10 * X ** 2.5
    assert em.utd_transition(0.0) == 0


# ------------------------------------------------------------------ UTD wedge coefficient

def _total_field(phi, phi_p, n, k, sp, s, pol, diffracted=True):
    """GO (direct + 0-face reflection) plus diffracted field around a wedge whose edge is
    the z axis, 0-face on the +x half-plane, exterior region 0 <= phi <= n pi; point
    source at (sp, phi_p), observer at (s, phi), both in the plane z = 0."""
    src = sp * np.array([math.cos(phi_p), math.sin(phi_p)])
    obs = s * np.array([math.cos(phi), math.sin(phi)])
    U = 0j
    if phi < math.pi + phi_p:                       # lit by the source
        R = np.linalg.norm(obs - src)
        U += np.exp(-1j * k * R) / R
    if phi < math.pi - phi_p:                       # lit by the 0-face reflection
        img = np.array([src[0], -src[1]])
        R = np.linalg.norm(obs - img)
        U += (1.0 if pol == 1 else -1.0) * np.exp(-1j * k * R) / R
    if not diffracted:
        return U
    Ld = s * sp / (s + sp)
    D = complex(em.utd_coefficient(phi, phi_p, 1.0, n, k, Ld, pol))
    U += np.exp(-1j * k * sp) / sp * D * math.sqrt(sp / (s * (s + sp))) * np.exp(-1j * k * s)
    return U


@pytest.mark.parametrize("n", [1.5, 2.0, 1.8])
@pytest.mark.parametrize("pol", [0, 1])
def test_total_field_continuous_across_shadow_boundaries(n, pol):
    k = 2 * math.pi / 0.0107
    sp, s, phi_p = 12.0, 7.0, math.radians(50)
    for bnd in (math.pi + phi_p, math.pi - phi_p):
        for d in (1e-6, 1e-9):       # direct formula, then the boundary limit
            U = [_total_field(bnd + m * d, phi_p, n, k, sp, s, pol) for m in (-3, -1, 1, 3)]
            # jump at the boundary with the smooth (linear) variation taken out
            jump = (U[2] - U[1]) - 0.5 * ((U[3] - U[2]) + (U[1] - U[0]))
            jump_go = abs(_total_field(bnd + d, phi_p, n, k, sp, s, pol, False)
                          - _total_field(bnd - d, phi_p, n, k, sp, s, pol, False))
            assert jump_go > 0.02          # the GO field alone jumps by about 1/R
            assert abs(jump) < 1e-6 * jump_go, (bnd, d, abs(jump), jump_go)


def test_diffraction_exactly_at_boundary_uses_limit():
    k, sp, s, phi_p = 2 * math.pi / 0.0107, 12.0, 7.0, math.radians(50)
    at = complex(em.utd_coefficient(math.pi + phi_p, phi_p, 1.0, 1.5, k, s * sp / (s + sp), 0))
    assert np.isfinite(at.real) and np.isfinite(at.imag)


def test_utd_reciprocity():
    rng = np.random.default_rng(4)
    for _ in range(100):
        n = rng.uniform(1.2, 2.0)
        phi, phi_p = rng.uniform(0.05, n * math.pi - 0.05, 2)
        k, Ld, sb = 600.0, rng.uniform(1, 50), rng.uniform(0.3, 1)
        for pol in (0, 1):
            a = complex(em.utd_coefficient(phi, phi_p, sb, n, k, Ld, pol))
            b = complex(em.utd_coefficient(phi_p, phi, sb, n, k, Ld, pol))
            assert abs(a - b) < 1e-12 * abs(a)


# ------------------------------------------------------------------ Effective Roughness

@pytest.mark.parametrize("alpha", [1, 2, 3, 4])
def test_er_directive_norm_matches_quadrature(alpha):
    for th in (0.0, 0.4, 0.9, 1.3):
        r = np.array([math.sin(th), 0.0, math.cos(th)])     # specular direction
        f = lambda p, t: ((1 + (math.sin(t) * math.cos(p) * r[0] + math.cos(t) * r[2])) / 2) ** alpha * math.sin(t)
        q, _ = integrate.dblquad(f, 0, math.pi / 2, 0, 2 * math.pi, epsabs=1e-12, epsrel=1e-12)
        assert abs(em.er_norm_directive(alpha, math.cos(th)) - q) < 1e-9 * q


@pytest.mark.parametrize("model,alpha", [(0, 1), (1, 1), (1, 2), (1, 3), (1, 4)])
def test_er_pattern_reradiates_S2_of_intercepted_power(model, alpha):
    """sum over the hemisphere of |a|^2 (4 pi/lambda)^2 r_i^2 r_s^2 dOmega = S^2 dS cos t_i."""
    lam, S, dS, ri, rs = 0.005, 0.37, 2e-4, 3.0, 4.0
    for th_i in (0.2, 0.8):
        ci = math.cos(th_i)
        spec = np.array([math.sin(th_i), 0.0, math.cos(th_i)])
        def power(p, t):
            ks = np.array([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)])
            a = em.er_gain(model, alpha, S, dS, 0.0, ci, ks[2], float(spec @ ks), ri, rs, lam)
            return abs(complex(a)) ** 2 * (4 * math.pi / lam) ** 2 * ri ** 2 * rs ** 2 * math.sin(t)
        q, _ = integrate.dblquad(power, 0, math.pi / 2, 0, 2 * math.pi, epsabs=1e-14, epsrel=1e-10)
        assert abs(q - S ** 2 * dS * ci) < 1e-8 * S ** 2 * dS * ci


def test_er_behind_tile_is_zero():
    assert em.er_gain(1, 2, 0.3, 1e-4, 0.0, -0.1, 0.5, 0.2, 1.0, 1.0, 0.01) == 0
    assert em.er_gain(0, 2, 0.3, 1e-4, 0.0, 0.5, -0.5, 0.2, 1.0, 1.0, 0.01) == 0
    assert abs(em.er_norm_directive(0, 0.3) - 2 * math.pi) < 1e-15
