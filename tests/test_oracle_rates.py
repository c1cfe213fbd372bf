"""Pins of the oracle's interaction-point velocities and accelerations and the Doppler rate
(eqs. ref_point_velo / ref_point_acc, App. B and C): symbolic differentiation of the same
construction (sympy), the App. B closed form, finite differences of the re-solved points,
dL/dt against the Doppler of App. A, and the O(dt^3) error of the second-order Taylor
extrapolation of the points."""
import math

import numpy as np
import pytest

import oracle
from paper_2205_00237_amd import scenes
from paper_2205_00237_amd.scenes import SceneBuilder, KIND_R, KIND_D, POL_PERP

C0 = 299_792_458.0


def _moving_scene(seed, kinds):
    """A wall and an edge on one rotating, accelerating body plus a static wall; moving
    accelerated terminals; one ray with the interaction kinds `kinds`."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    mat = b.add_material(4.0, 0.01)
    ax = rng.normal(size=3)
    body = b.add_body((30.0, 8.0, 2.0), v0=rng.normal(size=3) * 5, a=rng.normal(size=3),
                      axis=ax, w0=rng.uniform(-0.8, 0.8), wdot=rng.uniform(-0.5, 0.5))
    walls = [b.add_plane(0, mat, (60.0, 0, 0), (-1.0, 0.1 * rng.normal(), 0)),
             b.add_plane(body, mat, (30.0, 6.0, 2.0), (0.2 * rng.normal(), -1.0, 0.1 * rng.normal()))]
    edge = b.add_edge(body, (25.0, 6.0, 1.0), (0.1 * rng.normal(), 0.1 * rng.normal(), 1.0), (1.0, 0, 0),
                      (0, -1.0, 0), 1.5)
    prims = []
    wi = 0
    for k in kinds:
        if k == KIND_D:
            prims.append(edge)
        else:
            prims.append(walls[wi % 2])
            wi += 1
    b.add_ray(kinds, prims, [POL_PERP] * len(kinds))
    return b.build(tx_p=(0, 0, 1.5), tx_v=rng.normal(size=3) * 8, tx_a=rng.normal(size=3),
                   rx_p=(40, -10, 1.7), rx_v=rng.normal(size=3) * 8, rx_a=rng.normal(size=3))


@pytest.mark.parametrize("kinds", [(KIND_R,), (KIND_R, KIND_R), (KIND_D,), (KIND_R, KIND_D)])
def test_points_match_extrapolation_and_finite_differences(kinds):
    s = _moving_scene(3, kinds)
    t = np.array([0.0, 0.013, 0.2])
    rts = oracle.rates(s, t, 28e9)
    ext = oracle.extrapolate(s, t, 28e9, keep_points=True)
    n = len(kinds)
    for i in range(n):
        assert np.abs(rts["Q"][0, :, i] - ext["points"][0][i]).max() < 1e-12
    h = 2e-3
    for j, tj in enumerate(t):
        P = [oracle.extrapolate(s, np.array([tj + m * h]), 28e9, keep_points=True)["points"][0]
             for m in (-2, -1, 0, 1, 2)]
        for i in range(n):
            q = [p[i][0] for p in P]
            v_fd = (-q[4] + 8 * q[3] - 8 * q[1] + q[0]) / (12 * h)
            a_fd = (-q[4] + 16 * q[3] - 30 * q[2] + 16 * q[1] - q[0]) / (12 * h * h)
            v, a = rts["dQ"][0, j, i], rts["ddQ"][0, j, i]
            assert np.abs(v_fd - v).max() < 1e-6 * (1 + np.abs(v).max()), (i, v_fd, v)
            assert np.abs(a_fd - a).max() < 1e-4 * (1 + np.abs(a).max()), (i, a_fd, a)


def test_symbolic_single_reflection_on_rotating_wall():
    """The image construction written in sympy for a wall rotating about a fixed axis with
    angular acceleration and translating with acceleration, accelerated terminals."""
    sp = pytest.importorskip("sympy")
    t = sp.symbols("t")
    s = _moving_scene(5, (KIND_R,))
    pl = int(s["ray_prim"][0, 0])
    b = int(s["plane_body"][pl])
    vec = lambda a: sp.Matrix([sp.Float(float(x), 30) for x in a])
    TX = vec(s["tx_p"]) + vec(s["tx_v"]) * t + vec(s["tx_a"]) * t ** 2 / 2
    RX = vec(s["rx_p"]) + vec(s["rx_v"]) * t + vec(s["rx_a"]) * t ** 2 / 2
    O = vec(s["body_O0"][b]) + vec(s["body_v0"][b]) * t + vec(s["body_a"][b]) * t ** 2 / 2
    th = sp.Float(float(s["body_w0"][b]), 30) * t + sp.Float(float(s["body_wdot"][b]), 30) * t ** 2 / 2
    k = vec(s["body_axis"][b])
    K = sp.Matrix([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    Rm = sp.eye(3) + sp.sin(th) * K + (1 - sp.cos(th)) * K * K
    p = O + Rm * (vec(s["plane_p0"][pl]) - vec(s["body_O0"][b]))
    n = Rm * vec(s["plane_n0"][pl])
    A = TX - 2 * ((TX - p).dot(n)) * n
    sc = ((RX - p).dot(n)) / ((RX - A).dot(n))
    Q = RX + sc * (A - RX)
    dQ, ddQ = Q.diff(t), Q.diff(t, 2)
    for tv in (0.0, 0.07, 0.31):
        rts = oracle.rates(s, np.array([tv]), 28e9)
        q1 = np.array([float(x) for x in dQ.subs(t, tv).evalf(25)])
        q2 = np.array([float(x) for x in ddQ.subs(t, tv).evalf(25)])
        assert np.abs(rts["dQ"][0, 0, 0] - q1).max() < 1e-10 * (1 + np.abs(q1).max())
        assert np.abs(rts["ddQ"][0, 0, 0] - q2).max() < 1e-9 * (1 + np.abs(q2).max())


def test_appendix_b_velocity_static_wall():
    """App. B closed form of v_Q,x for a static wall y = 0 (see test_oracle_reflection)."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        b = SceneBuilder()
        mat = b.add_material(3.0, 0.0)
        pl = b.add_plane(0, mat, (0, 0, 0), (0, 1, 0))
        b.add_ray((KIND_R,), (pl,), (POL_PERP,))
        tx = np.array([rng.uniform(-20, 20), rng.uniform(1, 20), 0.0])
        rx = np.array([rng.uniform(-20, 20), rng.uniform(1, 20), 0.0])
        vt = np.array([rng.normal() * 10, rng.normal() * 10, 0.0])
        vr = np.array([rng.normal() * 10, rng.normal() * 10, 0.0])
        s = b.build(tx_p=tx, rx_p=rx, tx_v=vt, rx_v=vr)
        v = oracle.rates(s, np.array([0.0]), 3e9)["dQ"][0, 0, 0]
        yT, yR, xT, xR = tx[1], rx[1], tx[0], rx[0]
        den = yT + yR
        v_app = ((1 - yT / den) * vt[0] + yR * (xR - xT) / den ** 2 * vt[1]
                 + yT / den * vr[0] - yT * (xR - xT) / den ** 2 * vr[1])
        assert abs(v[0] - v_app) < 1e-12 * (1 + abs(v_app))


@pytest.mark.parametrize("which", ["config1", "config2"])
def test_dL_dt_equals_doppler(which):
    """dL/dt from the differentiated construction against the App. A Doppler, which the
    oracle forms from the material velocities at the points (a different formula)."""
    if which == "config1":
        s, tg, fg = scenes.config1()
        rays = None
    else:
        s, tg, fg = scenes.config2()
        rays = np.arange(0, 5000, 7)
    t = np.array([0.0, 0.05, 0.099])
    rts = oracle.rates(s, t, fg.f_c, rays=rays)
    ext = oracle.extrapolate(s, t, fg.f_c, rays=rays)
    v = ext["valid"]
    dLdt = -ext["dop"] * C0 / fg.f_c
    assert np.abs(rts["dL"][v] - dLdt[v]).max() < 1e-9 * (1 + np.abs(dLdt).max())


def test_taylor_extrapolation_error_is_third_order():
    """Second-order Taylor extrapolation of the points from t0 (the alternative to
    re-solving) errs by O(dt^3): halving dt divides the error by ~8."""
    s = _moving_scene(7, (KIND_R, KIND_R))
    dts = np.array([0.0, 0.01, 0.02, 0.04])
    rts = oracle.rates(s, dts, 28e9)
    tay = oracle.taylor_points(rts, 0, dts)
    err = np.linalg.norm(tay[0, :, :2] - rts["Q"][0, :, :2], axis=-1).max(axis=-1)
    assert err[0] == 0.0
    r1, r2 = err[2] / err[1], err[3] / err[2]
    assert 6.0 < r1 < 10.0 and 6.0 < r2 < 10.0, err
