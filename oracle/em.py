"""Field coefficients of one ray at the carrier (oracle step O7).  TEST INFRASTRUCTURE ONLY.

The paper recomputes the field of every extrapolated ray "as in standard ray tracing"
(Sec. III-A.2: Fresnel reflection coefficients and the ray divergence factor; Sec. III-B:
updated UTD coefficients, ref. [UTD] = Kouyoumjian and Pathak 1974; Sec. III-C: the
Effective Roughness model, ref. [vitucci2019]) without printing formulas.  The readings
used here are the textbook ones:

* Fresnel: eps_c = eps_r - j 60 sigma lambda (time convention e^{+j w t});
  G_perp = (cos t - sqrt(eps_c - sin^2 t)) / (cos t + sqrt(eps_c - sin^2 t)),
  G_par  = (eps_c cos t - sqrt(eps_c - sin^2 t)) / (eps_c cos t + sqrt(eps_c - sin^2 t)),
  principal square root; a perfect conductor gives G_perp = -1, G_par = +1.
* UTD wedge diffraction coefficient of a perfectly conducting wedge of exterior angle
  n*pi, with the transition function F(X) = 2j sqrt(X) e^{jX} int_{sqrt X}^inf e^{-j tau^2}
  d tau; "-" (soft) for perpendicular and "+" (hard) for parallel polarisation.
* Effective Roughness: Lambertian or single-lobe directive pattern, normalised so that
  the tile re-radiates S^2 of the power it intercepts.
"""
import math

import numpy as np
from scipy.special import wofz as _faddeeva

# Below this |eps| the product cot(.) F(.) at a shadow or reflection boundary is replaced
# by its small-argument limit (both sides of the parity check use the same switch).
UTD_EPS = 1e-8


def fresnel_gamma(cos_t, eps_r, sigma, lam, pec, pol):
    """Fresnel reflection coefficient for incidence cosine cos_t (measured from the normal).

    pol: 0 perpendicular (TE), 1 parallel (TM); pec: boolean perfect-conductor flag."""
    cos_t = np.asarray(cos_t, dtype=np.float64)
    eps_c = np.asarray(eps_r, dtype=np.complex128) - 1j * 60.0 * np.asarray(sigma) * lam
    root = np.sqrt(eps_c - (1.0 - cos_t * cos_t))
    with np.errstate(divide="ignore", invalid="ignore"):
        g_perp = (cos_t - root) / (cos_t + root)
        g_par = (eps_c * cos_t - root) / (eps_c * cos_t + root)
    pol = np.asarray(pol)
    g = np.where(pol == 1, g_par, g_perp)
    return np.where(np.asarray(pec, dtype=bool), np.where(pol == 1, 1.0 + 0j, -1.0 + 0j), g)


def utd_transition(X):
    """UTD transition function F(X) for real X >= 0 (F(0) = 0, F -> 1 as X -> inf).

    The tail integral is a complementary error function,
    int_x^inf e^{-j tau^2} d tau = (sqrt(pi)/2) e^{-j pi/4} erfc(e^{j pi/4} x), and
    erfc(z) = e^{-z^2} w(jz) with w the Faddeeva function; the factor e^{jX} cancels,
    leaving F(X) = sqrt(pi X) e^{j pi/4} w(e^{j 3pi/4} sqrt(X))."""
    X = np.asarray(X, dtype=np.float64)
    x = np.sqrt(X)
    return math.sqrt(math.pi) * x * np.exp(1j * math.pi / 4) * _faddeeva(np.exp(3j * math.pi / 4) * x)


def _cot_F(beta, sgn, n, kL):
    """cot((pi + sgn*beta)/(2n)) F(kL a^sgn(beta)) with its boundary limit."""
    N = np.round((beta + sgn * math.pi) / (2.0 * math.pi * n))
    a = 2.0 * np.cos((2.0 * n * math.pi * N - beta) / 2.0) ** 2
    eps = math.pi + sgn * beta - sgn * 2.0 * math.pi * n * N
    with np.errstate(divide="ignore", invalid="ignore"):
        direct = utd_transition(kL * a) / np.tan((math.pi + sgn * beta) / (2.0 * n))
    limit = n * (np.sqrt(2.0 * math.pi * kL) * np.sign(eps)
                 - 2.0 * kL * eps * np.exp(1j * math.pi / 4)) * np.exp(1j * math.pi / 4)
    return np.where(np.abs(eps) < UTD_EPS, limit, direct)


def utd_coefficient(phi, phi_p, sin_b0, n, k, Ld, pol):
    """Kouyoumjian-Pathak diffraction coefficient D_s (pol 0) or D_h (pol 1)."""
    bm = phi - phi_p
    bp = phi + phi_p
    kL = k * Ld
    t_m = _cot_F(bm, 1.0, n, kL) + _cot_F(bm, -1.0, n, kL)
    t_p = _cot_F(bp, 1.0, n, kL) + _cot_F(bp, -1.0, n, kL)
    sign = np.where(np.asarray(pol) == 1, 1.0, -1.0)
    pre = -np.exp(-1j * math.pi / 4) / (2.0 * n * math.sqrt(2.0 * math.pi * k) * sin_b0)
    return pre * (t_m + sign * t_p)


def er_norm_directive(alpha, cos_ti):
    """F_alpha = integral over the scattering hemisphere of ((1 + cos psi_R)/2)^alpha dOmega,
    psi_R the angle to the specular direction (closed form for integer alpha)."""
    alpha = int(alpha)
    cos_ti = np.asarray(cos_ti, dtype=np.float64)
    sin2 = 1.0 - cos_ti * cos_ti
    total = np.zeros_like(cos_ti)
    for j in range(alpha + 1):
        if j % 2 == 0:
            Ij = 2.0 * math.pi / (j + 1)
        else:
            acc = np.zeros_like(cos_ti)
            for w in range((j - 1) // 2 + 1):
                acc = acc + math.comb(2 * w, w) * sin2 ** w / 4.0 ** w
            Ij = 2.0 * math.pi / (j + 1) * cos_ti * acc
        total = total + math.comb(alpha, j) * Ij
    return total / 2.0 ** alpha


def er_gain(model, alpha, S, dS, phase0, cos_ti, cos_ts, cos_psi, r_i, r_s, lam):
    """Channel coefficient of one Effective-Roughness tile (zero when a terminal is behind).

    Lambertian: S sqrt(dS cos_i cos_s / pi) / (r_i r_s);
    directive:  S sqrt(dS cos_i / F_alpha) ((1 + cos psi_R)/2)^(alpha/2) / (r_i r_s);
    both times lambda/(4 pi) e^{j phase0}."""
    cos_ti = np.asarray(cos_ti, dtype=np.float64)
    cos_ts = np.asarray(cos_ts, dtype=np.float64)
    ok = (cos_ti > 0.0) & (cos_ts > 0.0)
    ci = np.where(ok, cos_ti, 1.0)
    cs = np.where(ok, cos_ts, 1.0)
    if int(model) == 0:
        amp = S * np.sqrt(dS * ci * cs / math.pi)
    else:
        lobe = np.maximum((1.0 + cos_psi) / 2.0, 0.0) ** (0.5 * alpha)
        amp = S * np.sqrt(dS * ci / er_norm_directive(alpha, ci)) * lobe
    a = lam / (4.0 * math.pi) * np.exp(1j * phase0) * amp / (r_i * r_s)
    return np.where(ok, a, 0.0 + 0j)
