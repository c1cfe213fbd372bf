"""Pins of the oracle's kinematics (Sec. II eq. Taylor; Sec. III-A.1 rotation angle and
eq. RigidBodyMotion) against independent constructions."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from oracle import kinematics as kin


def test_rotation_orthonormal_and_matches_quaternion():
    rng = np.random.default_rng(0)
    for _ in range(20):
        k = rng.normal(size=3)
        k /= np.linalg.norm(k)
        th = rng.uniform(-7, 7, 50)
        R = kin.rodrigues(k, th)
        eye = np.einsum("tij,tkj->tik", R, R)
        assert np.abs(eye - np.eye(3)).max() < 1e-14
        assert np.abs(np.linalg.det(R) - 1).max() < 1e-14
        Rq = Rotation.from_rotvec(th[:, None] * k[None]).as_matrix()
        assert np.abs(R - Rq).max() < 1e-14


def test_paper_clockwise_z_example():
    # Sec. III-A.1: clockwise rotation about z by theta has rows (c, s, 0), (-s, c, 0), (0, 0, 1)
    th = np.array([0.3])
    R = kin.rodrigues(np.array([0.0, 0.0, -1.0]), th)[0]
    c, s = math.cos(0.3), math.sin(0.3)
    assert np.allclose(R, [[c, s, 0], [-s, c, 0], [0, 0, 1]], atol=1e-15)


def test_identity_at_t0_and_taylor_second_derivative():
    rng = np.random.default_rng(1)
    p0, v0, a = rng.normal(size=(3, 3))
    P, V = kin.terminal_state(p0, v0, a, np.array([0.0]))
    assert np.array_equal(P[0], p0) and np.array_equal(V[0], v0)
    h, t = 1e-3, 0.37
    P, _ = kin.terminal_state(p0, v0, a, np.array([t - h, t, t + h]))
    acc = (P[2] - 2 * P[1] + P[0]) / h ** 2
    assert np.allclose(acc, a, atol=1e-6)
    Pv, Vv = kin.terminal_state(p0, v0, a, np.array([t - h, t + h]))
    assert np.allclose((Pv[1] - Pv[0]) / (2 * h), kin.terminal_state(p0, v0, a, np.array([t]))[1][0],
                       atol=1e-9)


def _body_scene(rng):
    from paper_2205_00237_amd.scenes import SceneBuilder
    b = SceneBuilder()
    k = rng.normal(size=3)
    b.add_body(rng.normal(size=3) * 10, v0=rng.normal(size=3) * 5, a=rng.normal(size=3),
               axis=k, w0=rng.normal(), wdot=rng.normal())
    return b.build(tx_p=(0, 0, 0), rx_p=(1, 0, 0))


def test_rigid_point_matches_angle_law_and_velocity_is_derivative():
    rng = np.random.default_rng(2)
    for _ in range(10):
        s = _body_scene(rng)
        X0 = rng.normal(size=3) * 5
        dt = np.array([0.0, 0.2, 0.5])
        O, R, V, W = kin.body_poses(s, dt)
        X = kin.place_points(X0, s["body_O0"][1], O[1], R[1])
        assert np.allclose(X[0], X0, atol=1e-14)
        # rotation angle omega*dt + omega_dot*dt^2/2 about the fixed axis, built independently
        w0, wd = s["body_w0"][1], s["body_wdot"][1]
        th = w0 * dt + 0.5 * wd * dt ** 2
        Rq = Rotation.from_rotvec(th[:, None] * s["body_axis"][1][None]).as_matrix()
        Oref = s["body_O0"][1] + s["body_v0"][1] * dt[:, None] + 0.5 * s["body_a"][1] * dt[:, None] ** 2
        Xref = Oref + np.einsum("tij,j->ti", Rq, X0 - s["body_O0"][1])
        assert np.abs(X - Xref).max() < 1e-12
        # eq. RigidBodyMotion equals the time derivative of the carried point
        h = 1e-5
        for t in (0.1, 0.4):
            Oh, Rh, Vh, Wh = kin.body_poses(s, np.array([t - h, t, t + h]))
            Xh = kin.place_points(X0, s["body_O0"][1], Oh[1], Rh[1])
            fd = (Xh[2] - Xh[0]) / (2 * h)
            u = kin.material_velocity(Xh[1], Oh[1][1], Vh[1][1], Wh[1][1], s["body_axis"][1])
            assert np.allclose(u, fd, rtol=1e-7, atol=1e-7)
