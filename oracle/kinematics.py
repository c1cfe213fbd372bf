"""Kinematics of terminals and rigid bodies (oracle step O1).  TEST INFRASTRUCTURE ONLY.

* Terminals follow the second-order Taylor formula of Sec. II (eq. Taylor): position
  r(t0+dt) = r + v*dt + a*dt^2/2 and velocity v + a*dt (the jerk is neglected).
* A rigid body translates its reference point O (on its rotation axis) with constant
  acceleration and rotates about a fixed unit axis k by the angle
  theta = omega*dt + omega_dot*dt^2/2 (Sec. III-A.1, rotation-angle formula), with
  instantaneous v(t) = v0 + a*dt and omega(t) = omega0 + omega_dot*dt.
* A point rigidly attached to a body: X(t) = O(t) + R(t) (X0 - O0) (eq. coordinate_transf,
  written in the global frame); a direction d(t) = R(t) d0.
* The velocity of a material point is v_Q = v_Pi + omega x O^I Q (eq. RigidBodyMotion).
R(t) is the rotation by theta about k (Rodrigues' formula).
"""
import numpy as np


def terminal_state(p0, v0, a, dt):
    """Position and velocity of a terminal at the offsets dt (T,) -> (T,3), (T,3)."""
    dt = np.asarray(dt, dtype=np.float64)[:, None]
    p0, v0, a = (np.asarray(x, dtype=np.float64) for x in (p0, v0, a))
    return p0 + v0 * dt + 0.5 * a * dt * dt, v0 + a * dt


def _skew(k):
    k = np.asarray(k, dtype=np.float64)
    return np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])


def rodrigues(k, theta):
    """Rotation matrices (T,3,3) by angles theta (T,) about the fixed unit axis k."""
    theta = np.asarray(theta, dtype=np.float64)
    K = _skew(k)
    s = np.sin(theta)[:, None, None]
    c1 = (1.0 - np.cos(theta))[:, None, None]
    return np.eye(3)[None] + s * K[None] + c1 * (K @ K)[None]


def body_poses(scene, dt):
    """Per body b and time offset: O (nb,T,3), R (nb,T,3,3), v (nb,T,3), omega (nb,T)."""
    dt = np.asarray(dt, dtype=np.float64)
    nb = scene["body_O0"].shape[0]
    T = dt.shape[0]
    O = np.empty((nb, T, 3))
    R = np.empty((nb, T, 3, 3))
    V = np.empty((nb, T, 3))
    W = np.empty((nb, T))
    for b in range(nb):
        O[b], V[b] = terminal_state(scene["body_O0"][b], scene["body_v0"][b],
                                    scene["body_a"][b], dt)
        w0, wd = scene["body_w0"][b], scene["body_wdot"][b]
        R[b] = rodrigues(scene["body_axis"][b], w0 * dt + 0.5 * wd * dt * dt)
        W[b] = w0 + wd * dt
    return O, R, V, W


def place_points(X0, O0, O, R):
    """Rigidly carried points: X0 (...,3) at t0 -> O + R (X0 - O0), broadcasting over time."""
    return O + np.einsum("...ij,...j->...i", R, X0 - O0)


def rotate(d0, R):
    """Rigidly carried directions d0 (...,3) -> R d0."""
    return np.einsum("...ij,...j->...i", R, d0)


def material_velocity(X, O, V, W, k):
    """Velocity of the body's material point at X: v + omega k x (X - O)."""
    return V + W[..., None] * np.cross(k, X - O)
