"""Pins of the diffusely scattered ray as the oracle assembles it in `extrapolate` (Sec. III-C:
the tile centroid acts as a virtual source carried with its body; ref. [vitucci2019], the
Effective Roughness model): which incidence and scattering cosines, which distances and which
specular direction enter the Lambertian and directive patterns.  The geometry is worked out
by hand (3-4-5 and 6-8-10 triangles); the pattern normalisation F_alpha itself is pinned
against quadrature in test_oracle_em.py."""
import math

import numpy as np
import pytest

import oracle
from oracle.em import er_norm_directive
from paper_2205_00237_amd.scenes import SceneBuilder, KIND_S, POL_PERP

C0 = 299_792_458.0
F_C = 28e9
LAM = C0 / F_C


def _tile_ray(tx, rx, model, alpha, S=0.35, dS=1e-4, phase0=0.7, body=None, dt=(0.0,)):
    b = SceneBuilder()
    bd = 0 if body is None else b.add_body(**body)
    t = b.add_tile(bd, (0, 0, 0), (0, 0, 1), dS, S, alpha, model, phase0)
    b.add_ray([KIND_S], [t], [POL_PERP])
    s = b.build(tx_p=tx, rx_p=rx)
    return oracle.extrapolate(s, np.asarray(dt, dtype=np.float64), F_C)


# (tx, rx, cos_i, cos_s, cos_psi, r_i, r_s) for a tile at the origin facing +z
CASES = [
    # k_in = (3,0,-4)/5, k_out = (0,0,1), specular (3,0,4)/5
    ((-3.0, 0.0, 4.0), (0.0, 0.0, 2.0), 0.8, 1.0, 0.8, 5.0, 2.0),
    # k_in = (0,4,-3)/5, k_out = (6,0,8)/10, specular (0,4,3)/5
    ((0.0, -4.0, 3.0), (6.0, 0.0, 8.0), 0.6, 0.8, 0.48, 5.0, 10.0),
    # k_in = (0,-4,-3)/5 (from the +y side), k_out = (0,-6,8)/10, specular (0,-4,3)/5
    ((0.0, 4.0, 3.0), (0.0, -6.0, 8.0), 0.6, 0.8, 0.96, 5.0, 10.0),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_lambertian_tile(case):
    tx, rx, ci, cs, _, ri, rs = CASES[case]
    S, dS, ph = 0.35, 1e-4, 0.7
    out = _tile_ray(tx, rx, 0, 1, S, dS, ph)
    ref = LAM / (4 * math.pi) * np.exp(1j * ph) * S * math.sqrt(dS * ci * cs / math.pi) / (ri * rs)
    assert out["valid"][0, 0]
    assert abs(out["gain"][0, 0] - ref) < 1e-13 * abs(ref)
    assert abs(out["L"][0, 0] - (ri + rs)) < 1e-14


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("alpha", [1, 2, 4])
def test_directive_tile(case, alpha):
    tx, rx, ci, cs, cpsi, ri, rs = CASES[case]
    S, dS, ph = 0.35, 1e-4, 0.7
    out = _tile_ray(tx, rx, 1, alpha, S, dS, ph)
    lobe = ((1 + cpsi) / 2) ** (alpha / 2)
    ref = (LAM / (4 * math.pi) * np.exp(1j * ph) * S
           * math.sqrt(dS * ci / float(er_norm_directive(alpha, ci))) * lobe / (ri * rs))
    assert abs(out["gain"][0, 0] - ref) < 1e-13 * abs(ref)


def test_terminal_behind_the_tile_is_inconsistent():
    for tx, rx in (((-3.0, 0.0, -4.0), (0.0, 0.0, 2.0)), ((-3.0, 0.0, 4.0), (0.0, 1.0, -2.0))):
        out = _tile_ray(tx, rx, 1, 2)
        assert not out["valid"][0, 0] and out["gain"][0, 0] == 0


def test_tile_carried_by_its_body():
    """A tile on a body translating at (1, 0, 0) m/s and turning about z through the tile at
    pi/2 rad/s: after 1 s the centroid is at (1, 0, 0) with the same normal, so with TX at
    (-2, 0, 4) and RX at (1, 0, 2) the first case's geometry shifted by one metre applies."""
    body = dict(O0=(0, 0, 0), v0=(1, 0, 0), axis=(0, 0, 1), w0=math.pi / 2)
    out = _tile_ray((-2.0, 0.0, 4.0), (1.0, 0.0, 2.0), 0, 1, body=body, dt=(1.0,))
    ref = LAM / (4 * math.pi) * np.exp(0.7j) * 0.35 * math.sqrt(1e-4 * 0.8 * 1.0 / math.pi) / 10.0
    assert abs(out["gain"][0, 0] - ref) < 1e-12 * abs(ref)
    assert abs(out["L"][0, 0] - 7.0) < 1e-12
