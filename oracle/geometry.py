"""Interaction-point solves on the displaced geometry (oracle step O3).  TEST INFRASTRUCTURE
ONLY.

Reflections (Sec. III-A.1 eq. ref_point and Sec. III-A.2): the reflection point on one
wall lies where the line from the receiver to the image of the transmitter crosses the
wall; for several walls the transmitter is imaged wall after wall (TX', TX'', ...) and
the points are found by back-tracking from the receiver, each found point acting as the
virtual receiver of the previous wall.  Written in the global frame: image
A_m = A_{m-1} - 2((A_{m-1}-p_m).n_m) n_m, and Q_m = Q_{m+1} + s_m (A_m - Q_{m+1}) with
s_m = ((Q_{m+1}-p_m).n_m) / ((Q_{m+1}-A_m).n_m).  A chain is geometrically consistent
when every 0 < s_m < 1 (each point strictly between its virtual receiver and image).

Diffraction (Sec. III-B, eqs. dist2D_TXRX and diff_point): in a frame whose z axis runs
along the edge, the point Q_D divides the unfolded ray by similar triangles:
z_Q = z_B + rho_B (z_A - z_B) / (rho_A + rho_B), where rho are the distances of the
(image) source A and (image) receiver B from the edge line.
"""
import numpy as np


def dot(a, b):
    return np.sum(a * b, axis=-1)


def norm(a):
    return np.sqrt(dot(a, a))


def mirror(X, p, n):
    """Image of the point X in the plane through p with unit normal n."""
    return X - 2.0 * dot(X - p, n)[..., None] * n


def reflection_chain(src, dst, planes, return_den=False):
    """Reflection points from `src` to `dst` over the walls `planes` = [(p, n), ...].

    Returns (points [Q_1..Q_m], images [A_1..A_m], valid) where valid is the boolean
    0 < s_m < 1 for every wall (all arrays broadcast over the leading dims); with
    return_den=True also the denominators (Q_{m+1}-A_m).n_m (zero: image line parallel
    to the wall, a degenerate chain)."""
    images = []
    A = src
    for p, n in planes:
        A = mirror(A, p, n)
        images.append(A)
    points = [None] * len(planes)
    valid = np.ones(np.broadcast_shapes(src.shape, dst.shape)[:-1], dtype=bool)
    nxt = dst
    dens = [None] * len(planes)
    for m in range(len(planes) - 1, -1, -1):
        p, n = planes[m]
        num = dot(nxt - p, n)
        den = dot(nxt - images[m], n)
        dens[m] = den
        with np.errstate(divide="ignore", invalid="ignore"):
            s = num / den
        ok = np.isfinite(s) & (s > 0.0) & (s < 1.0)
        valid &= ok
        s = np.where(np.isfinite(s), s, 0.0)
        Q = nxt + s[..., None] * (images[m] - nxt)
        points[m] = Q
        nxt = Q
    if return_den:
        return points, images, valid, dens
    return points, images, valid


def edge_point(A, B, a, e):
    """Diffraction point on the edge line a + z e for the (image) source A and receiver B.

    Returns (Q, z_A, z_B, rho_A, rho_B)."""
    zA = dot(A - a, e)
    zB = dot(B - a, e)
    rA = norm((A - a) - zA[..., None] * e)
    rB = norm((B - a) - zB[..., None] * e)
    with np.errstate(divide="ignore", invalid="ignore"):
        zQ = zB + rB * (zA - zB) / (rA + rB)
    zQ = np.where(np.isfinite(zQ), zQ, 0.0)
    return a + zQ[..., None] * e, zA, zB, rA, rB


def direction_angles(v):
    """Azimuth atan2(y, x) in (-pi, pi] and elevation atan2(z, hypot(x, y)) of v (...,3)."""
    return np.arctan2(v[..., 1], v[..., 0]), np.arctan2(v[..., 2], np.hypot(v[..., 0], v[..., 1]))
