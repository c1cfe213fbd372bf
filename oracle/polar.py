"""Polarimetric field coefficients with half-wave dipole antennas (the dipoles of the
measurement comparison, Sec. IV-B; the interactions of Sec. III in vector form).  TEST
INFRASTRUCTURE ONLY.

A scene carries this model when it has "tx_ant" and "rx_ant" = (p_x, p_y, p_z, kind) with
kind 1 (a half-wave dipole along the unit vector p).  The field leaves the transmitter
along the first segment direction k as the dipole's vector pattern

    e(p, k) = sqrt(1.64) cos((pi/2) cos(theta)) / sin(theta) theta_hat,
    cos(theta) = p . k,  theta_hat = ((p . k) k - p) / sin(theta)

(1.64 the dipole's directivity), is carried through every interaction by a dyadic, and is
received by projecting onto the receiving dipole's pattern in the arrival direction,
e(p_rx, -k_last) (the same function at both ends, so the coefficient is reciprocal):

* reflection on a wall with normal n, incidence k_in, reflection k_out:
  e_perp = (k_in x n)/|k_in x n|, e_par_in = e_perp x k_in, e_par_out = e_perp x k_out,
  E -> G_perp (E . e_perp) e_perp + G_par (E . e_par_in) e_par_out with the Fresnel
  coefficients of em.py (a perfect conductor: G_perp = -1, G_par = +1; tangential E cancels);
* diffraction at an edge along e, incidence s_in, diffraction s_out (Keller cone):
  e_phi_in = (e x s_in)/|e x s_in|, e_beta_in = s_in x e_phi_in, and likewise e_phi_out,
  e_beta_out = s_out x e_phi_out; E -> D_s (E . e_beta_in) e_beta_out + D_h (E . e_phi_in)
  e_phi_out with the UTD coefficients of em.py (the component along the edge sees the soft
  coefficient, the one across it the hard one, as the scalar problems for E_z and H_z);
* diffuse scattering keeps the field (the tile's effective-roughness amplitude is scalar).

With both antennas vertical and every wall vertical (or every edge vertical) the field
stays along z and the coefficient reduces to the scalar model's perpendicular one times the
two dipole gains.
"""
import math

import numpy as np

DIPOLE_GAIN = 1.64


def _dot(a, b):
    return np.sum(a * b, axis=-1)


def _unit(v):
    n = np.sqrt(_dot(v, v))[..., None]
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(n > 0, v / np.where(n > 0, n, 1.0), 0.0)


def dipole_pattern(p, k):
    """Vector pattern of a half-wave dipole along the unit p towards the unit directions k."""
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), k.shape)
    c = _dot(p, k)
    t = c[..., None] * k - p
    s2 = _dot(t, t)
    # cos((pi/2) c) / sin^2 = sin((pi/2) (1 - |c|)) / s^2 with 1 - |c| = s^2 / (1 + |c|): no
    # cancellation near the axis, where the pattern goes to zero with s
    x = s2 / (1.0 + np.abs(c))
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.where(s2 > 0, np.sin(0.5 * math.pi * x) / np.where(s2 > 0, s2, 1.0), 0.5 * math.pi / (1.0 + np.abs(c)))
    return math.sqrt(DIPOLE_GAIN) * amp[..., None] * t


def _perp_basis(k_in, n):
    e = np.cross(k_in, n)
    # normal incidence: any unit vector in the wall will do (both coefficients agree there
    # up to the basis orientation, which cancels)
    alt = np.cross(n, np.where(np.abs(n[..., 2:3]) < 0.9, [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]))
    small = _dot(e, e) < 1e-24
    return _unit(np.where(small[..., None], alt, e))


def reflect(E, k_in, k_out, n, g_perp, g_par):
    ep = _perp_basis(k_in, n)
    return (g_perp * _dot(E, ep))[..., None] * ep + (g_par * _dot(E, np.cross(ep, k_in)))[..., None] * np.cross(ep, k_out)


def diffract(E, s_in, s_out, e, d_soft, d_hard):
    phi_i = _unit(np.cross(e, s_in))
    phi_o = _unit(np.cross(e, s_out))
    beta_i = np.cross(s_in, phi_i)
    beta_o = np.cross(s_out, phi_o)
    return (d_soft * _dot(E, beta_i))[..., None] * beta_o + (d_hard * _dot(E, phi_i))[..., None] * phi_o


def antennas(scene):
    """(p_tx, p_rx) when the scene carries dipoles, else None."""
    if "tx_ant" not in scene or "rx_ant" not in scene:
        return None
    ta, ra = np.asarray(scene["tx_ant"], float), np.asarray(scene["rx_ant"], float)
    if ta[3] == 0 and ra[3] == 0:
        return None
    return ta[:3], ra[:3]


def transport(ants, kinds, khat, coef):
    """e(p_rx, -k_last) . (product of the interaction dyadics) e(p_tx, k_first).

    coef[i]: for a reflection (G_perp, G_par, n), for a diffraction (D_s, D_h, e), None for
    a scattering tile."""
    p_t, p_r = ants
    E = dipole_pattern(p_t, khat[0]).astype(np.complex128)
    for i, kd in enumerate(kinds):
        if kd == 1:
            g_perp, g_par, n = coef[i]
            E = reflect(E, khat[i], khat[i + 1], n, g_perp, g_par)
        elif kd == 2:
            d_s, d_h, e = coef[i]
            E = diffract(E, khat[i], khat[i + 1], e, d_s, d_h)
    return _dot(dipole_pattern(p_r, -khat[-1]), E)
