"""Property tests (hypothesis) of the oracle on random tiny scenes: one wall carried by a
body that translates with constant acceleration and turns about a fixed axis with constant
angular acceleration (Sec. III-A.1), terminals with their own velocities (eq. Taylor).
Wherever the oracle finds the reflection, it must satisfy, at every instant:

* the reflection point lies on the wall as turned and moved by the rigid-body law, written
  here with scipy's rotation vectors (not the oracle's Rodrigues form);
* Snell's law there: the outgoing direction is the incoming one mirrored in that wall;
* Fermat: the length is the sum of the two legs and equals the distance from the receiver
  to the image of the transmitter;
* the Doppler shift of App. A equals -(f_c / c) dL/dt by central differences of the
  oracle's own lengths;
* a wall sliding in its own plane (static terminals) gives no Doppler shift; a wall turning
  about a line in it shifts it as the length of its image path changes (Sec. IV-A).
"""
import math

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st
from scipy.spatial.transform import Rotation

import oracle
from paper_2205_00237_amd.scenes import SceneBuilder, KIND_R, POL_PERP

C0 = 299_792_458.0
F_C = 28e9

coord = st.floats(-30, 30, allow_nan=False)
vec = st.tuples(coord, coord, coord)
small = st.tuples(*[st.floats(-3, 3, allow_nan=False)] * 3)
unitish = st.tuples(*[st.floats(-1, 1, allow_nan=False)] * 3).filter(lambda v: sum(x * x for x in v) > 0.05)


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def _wall_scene(p0, n0, tx_off, rx_off, hT, hR, body):
    n0 = _unit(n0)
    p0 = np.asarray(p0, float)
    tx = p0 + hT * n0 + np.asarray(tx_off) - np.dot(tx_off, n0) * n0
    rx = p0 + hR * n0 + np.asarray(rx_off) - np.dot(rx_off, n0) * n0
    b = SceneBuilder()
    mat = b.add_material(5.0, 0.02)
    bd = b.add_body(body["O0"], v0=body["v0"], a=body["a"], axis=body["axis"], w0=body["w0"], wdot=body["wdot"])
    pl = b.add_plane(bd, mat, p0, n0)
    b.add_ray((KIND_R,), (pl,), (POL_PERP,))
    return b.build(tx_p=tx, rx_p=rx, tx_v=body["tx_v"], rx_v=body["rx_v"]), p0, n0


def _wall_at(t, p0, n0, body):
    """Wall point and normal at t by the rigid-body law (translation of the rotation centre,
    turn by w0 t + wdot t^2 / 2 about the fixed axis through it)."""
    th = body["w0"] * t + 0.5 * body["wdot"] * t * t
    Rm = Rotation.from_rotvec(th * _unit(body["axis"])).as_matrix()
    O0 = np.asarray(body["O0"], float)
    O = O0 + np.asarray(body["v0"]) * t + 0.5 * np.asarray(body["a"]) * t * t
    return O + Rm @ (p0 - O0), Rm @ n0


bodies = st.fixed_dictionaries({
    "O0": vec, "v0": st.tuples(*[st.floats(-20, 20, allow_nan=False)] * 3), "a": small, "axis": unitish,
    "w0": st.floats(-1, 1, allow_nan=False), "wdot": st.floats(-0.5, 0.5, allow_nan=False),
    "tx_v": st.tuples(*[st.floats(-15, 15, allow_nan=False)] * 3), "rx_v": st.tuples(*[st.floats(-15, 15, allow_nan=False)] * 3)})


@settings(max_examples=80, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.filter_too_much])
@given(p0=vec, n0=unitish, tx_off=vec, rx_off=vec, hT=st.floats(0.5, 30), hR=st.floats(0.5, 30), body=bodies)
def test_single_reflection_invariants(p0, n0, tx_off, rx_off, hT, hR, body):
    s, p0, n0 = _wall_scene(p0, n0, tx_off, rx_off, hT, hR, body)
    t = np.array([0.0, 0.01, 0.05, 0.1, 0.2])
    out = oracle.extrapolate(s, t, F_C, keep_points=True)
    assert out["valid"][0, 0]                                  # built valid at t0
    Q = out["points"][0][0]
    TX = s["tx_p"] + np.outer(t, s["tx_v"])
    RX = s["rx_p"] + np.outer(t, s["rx_v"])
    for j in np.flatnonzero(out["valid"][0]):
        p, n = _wall_at(t[j], p0, n0, body)
        scale = 1.0 + np.abs(Q[j]).max()
        assert abs(np.dot(Q[j] - p, n)) < 1e-11 * scale        # on the moved wall
        leg = min(np.linalg.norm(Q[j] - TX[j]), np.linalg.norm(RX[j] - Q[j]))
        if leg < 1e-6:                 # a terminal on the wall: no direction to check
            continue
        u_in = _unit(Q[j] - TX[j])
        u_out = _unit(RX[j] - Q[j])
        # Snell; the directions carry the points' rounding divided by the leg length
        assert np.abs(u_out - (u_in - 2 * np.dot(u_in, n) * n)).max() < 1e-10 + 1e-13 * scale / leg
        L = np.linalg.norm(Q[j] - TX[j]) + np.linalg.norm(RX[j] - Q[j])
        img = TX[j] - 2 * np.dot(TX[j] - p, n) * n
        assert abs(out["L"][0, j] - L) < 1e-11 * scale                          # Fermat
        assert abs(out["L"][0, j] - np.linalg.norm(RX[j] - img)) < 1e-10 * scale
    # Doppler against central differences of the length
    h = 1e-5
    tc = np.array([0.05, 0.1])
    lo = oracle.extrapolate(s, tc - h, F_C)
    mid = oracle.extrapolate(s, tc, F_C)
    hi = oracle.extrapolate(s, tc + h, F_C)
    for j in range(len(tc)):
        if lo["valid"][0, j] and mid["valid"][0, j] and hi["valid"][0, j]:
            dLdt = (hi["L"][0, j] - lo["L"][0, j]) / (2 * h)
            assert abs(mid["dop"][0, j] + F_C / C0 * dLdt) < 1e-3 + 1e-7 * abs(mid["dop"][0, j])


def _length_independent(s, t, p0, n0, body):
    """|RX - image of TX| in the wall as carried by the rigid-body law (scipy rotations)."""
    TX = s["tx_p"] + s["tx_v"] * t
    RX = s["rx_p"] + s["rx_v"] * t
    p, n = _wall_at(t, p0, n0, body)
    return np.linalg.norm(RX - (TX - 2 * np.dot(TX - p, n) * n))


@settings(max_examples=40, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.filter_too_much])
@given(p0=vec, n0=unitish, tx_off=vec, rx_off=vec, hT=st.floats(0.5, 30), hR=st.floats(0.5, 30),
       slide=st.floats(-20, 20), w0=st.floats(0.05, 1.0), wdot=st.floats(-0.5, 0.5))
def test_turning_wall_doppler(p0, n0, tx_off, rx_off, hT, hR, slide, w0, wdot):
    n0 = _unit(n0)
    along = np.cross(n0, _unit([0.3, -0.5, 0.8]))
    if np.linalg.norm(along) < 0.1:
        along = np.cross(n0, [1.0, 0.0, 0.0])
    along = _unit(along)                                           # a direction in the wall
    still = {"O0": p0, "v0": tuple(slide * along), "a": (0, 0, 0), "axis": tuple(n0), "w0": 0.0, "wdot": 0.0,
             "tx_v": (0, 0, 0), "rx_v": (0, 0, 0)}
    s, q0, m0 = _wall_scene(p0, n0, tx_off, rx_off, hT, hR, still)
    t = np.array([0.0, 0.1, 0.3])
    out = oracle.extrapolate(s, t, F_C)
    # sliding in its own plane leaves an infinite wall, and so the path, unchanged
    assert out["valid"][0, 0]
    assert np.abs(out["dop"][0][out["valid"][0]]).max() < 1e-6
    # turning about a line in the wall: the Doppler shift follows the length of the
    # independently carried image path
    turning = dict(still, axis=tuple(along), w0=w0, wdot=wdot, v0=(0, 0, 0))
    s, q0, m0 = _wall_scene(p0, n0, tx_off, rx_off, hT, hR, turning)
    tc = np.array([0.0, 0.05, 0.1])
    out = oracle.extrapolate(s, tc, F_C)
    h = 1e-5
    for j in np.flatnonzero(out["valid"][0]):
        dLdt = (_length_independent(s, tc[j] + h, q0, m0, turning)
                - _length_independent(s, tc[j] - h, q0, m0, turning)) / (2 * h)
        assert abs(out["dop"][0, j] + F_C / C0 * dLdt) < 1e-3 + 1e-7 * abs(out["dop"][0, j])
