"""Pins of the oracle's angles of departure and arrival (Sec. I: the angular dispersion of
the multipath; the reading fixes azimuth in (-pi, pi] from +x towards +y and elevation
above the horizontal plane, the departure direction from TX towards the first point and
the arrival direction from RX towards the last point) against values worked out by hand."""
import math

import numpy as np
import pytest

import oracle
from oracle.geometry import direction_angles
from paper_2205_00237_amd.scenes import SceneBuilder, KIND_R, POL_PERP

Q = math.pi / 4
E35 = math.atan(1.0 / math.sqrt(2.0))          # elevation of (1, 1, 1): 35.26 degrees


@pytest.mark.parametrize("v,az,el", [
    ((1, 0, 0), 0.0, 0.0),
    ((0, 2, 0), 2 * Q, 0.0),
    ((-3, 0, 0), math.pi, 0.0),
    ((0, -1, 0), -2 * Q, 0.0),
    ((1, 1, 0), Q, 0.0),
    ((-1, 1, 0), 3 * Q, 0.0),
    ((-1, -1, 0), -3 * Q, 0.0),
    ((1, 0, 1), 0.0, Q),
    ((0, 1, -1), 2 * Q, -Q),
    ((-1, -1, math.sqrt(2)), -3 * Q, Q),
    ((2, 2, 2), Q, E35),
    ((0, 0, 5), 0.0, 2 * Q),
    ((0, 0, -1), 0.0, -2 * Q),
])
def test_direction_angles_cardinal(v, az, el):
    a, e = direction_angles(np.asarray(v, dtype=np.float64))
    assert abs(a - az) < 1e-15 and abs(e - el) < 1e-15


def _ray_angles(tx, rx, walls=(), tx_v=(0, 0, 0), dt=(0.0,)):
    b = SceneBuilder()
    m = b.add_material(4.0, 0.0)
    ids = [b.add_plane(0, m, p, n) for p, n in walls]
    b.add_ray([KIND_R] * len(ids), ids, [POL_PERP] * len(ids))
    s = b.build(tx_p=tx, rx_p=rx, tx_v=tx_v)
    out = oracle.extrapolate(s, np.asarray(dt, dtype=np.float64), 28e9)
    assert out["valid"].all()
    return out


def test_line_of_sight_angles():
    """TX at the origin, RX at (3, 3, 3 sqrt 2): departure towards +x+y, 45 degrees up;
    arrival (from RX back towards TX) towards -x-y, 45 degrees down."""
    out = _ray_angles((0, 0, 0), (3, 3, 3 * math.sqrt(2)))
    assert abs(out["aod_az"][0, 0] - Q) < 1e-15 and abs(out["aod_el"][0, 0] - Q) < 1e-15
    assert abs(out["aoa_az"][0, 0] + 3 * Q) < 1e-15 and abs(out["aoa_el"][0, 0] + Q) < 1e-15


def test_reflection_on_axis_aligned_wall_angles():
    """TX (0,0,0), RX (10,0,10), wall y = 5: the image of TX is (0,10,0), the line from RX
    to it crosses the wall half-way, at Q = (5,5,5).  Departure along (1,1,1): azimuth 45
    degrees, elevation atan(1/sqrt 2); arrival from RX towards Q along (-1,1,-1): azimuth
    135 degrees, elevation -atan(1/sqrt 2)."""
    out = _ray_angles((0, 0, 0), (10, 0, 10), walls=[((0, 5, 0), (0, -1, 0))])
    assert abs(out["aod_az"][0, 0] - Q) < 1e-14 and abs(out["aod_el"][0, 0] - E35) < 1e-14
    assert abs(out["aoa_az"][0, 0] - 3 * Q) < 1e-14 and abs(out["aoa_el"][0, 0] + E35) < 1e-14


def test_two_wall_angles_and_moving_terminal():
    """Walls y = 5 and x = 20 (a corner), TX (0,0,0), RX (10,0,0), all in the plane z = 0:
    TX' = (0,10,0), TX'' = (40,10,0); the last point lies on x = 20 where the line from RX
    to TX'' crosses it, (20, 10/3, 0), and the first where the line from that point to TX'
    crosses y = 5, (15, 5, 0).  Departure along (15,5,0); arrival from RX towards
    (20, 10/3, 0), i.e. along (3, 1, 0): a corner returns the ray antiparallel, both
    azimuths are atan(1/3).  After 1 s with TX moving at (2,0,0) m/s: TX'' = (38,10,0),
    last point (20, 25/7, 0), first point (16, 5, 0): departure along (14, 5, 0), arrival
    along (10, 25/7, 0), both at azimuth atan(5/14)."""
    walls = [((0, 5, 0), (0, -1, 0)), ((20, 0, 0), (-1, 0, 0))]
    out = _ray_angles((0, 0, 0), (10, 0, 0), walls=walls, tx_v=(2, 0, 0), dt=(0.0, 1.0))
    assert abs(out["aod_az"][0, 0] - math.atan(1.0 / 3.0)) < 1e-14
    assert abs(out["aoa_az"][0, 0] - math.atan(1.0 / 3.0)) < 1e-14
    assert abs(out["aod_az"][0, 1] - math.atan(5.0 / 14.0)) < 1e-14
    assert abs(out["aoa_az"][0, 1] - math.atan(5.0 / 14.0)) < 1e-14
    assert np.abs(out["aod_el"]).max() < 1e-15 and np.abs(out["aoa_el"]).max() < 1e-15


def test_arrival_points_from_receiver_not_towards_it():
    """A receiver north-west of the transmitter at the same height: departure azimuth 135
    degrees, arrival azimuth -45 degrees (the arrival direction points back along the path,
    from RX towards TX)."""
    out = _ray_angles((0, 0, 1), (-25, 25, 1))
    assert abs(out["aod_az"][0, 0] - 3 * Q) < 1e-15
    assert abs(out["aoa_az"][0, 0] + Q) < 1e-15
