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


def double_edge_points(A, B, a1, e1, a2, e2, iters=60):
    """Points Q1 = a1 + z1 e1 and Q2 = a2 + z2 e2 of the path A -> Q1 -> Q2 -> B over two
    edges (the multiple-diffraction extension of Sec. III-B): the stationary, here shortest,
    length |Q1 - A| + |Q2 - Q1| + |B - Q2| (Fermat; Keller's law at both edges), a convex
    function of (z1, z2).  Newton's method with step halving from the single-edge points.

    Returns (Q1, Q2, z1, z2, converged) broadcast over the leading dims."""
    def length(z1, z2):
        Q1 = a1 + z1[..., None] * e1
        Q2 = a2 + z2[..., None] * e2
        return norm(Q1 - A) + norm(Q2 - Q1) + norm(B - Q2)

    z1 = edge_point(A, B, a1, e1)[0]
    z2 = edge_point(A, B, a2, e2)[0]
    z1 = dot(z1 - a1, e1)
    z2 = dot(z2 - a2, e2)
    f = length(z1, z2)
    g1 = g2 = np.ones_like(z1)
    for _ in range(iters):
        Q1 = a1 + z1[..., None] * e1
        Q2 = a2 + z2[..., None] * e2
        d0, d1, d2 = Q1 - A, Q2 - Q1, B - Q2
        l0, l1, l2 = norm(d0), norm(d1), norm(d2)
        c0, c1a, c1b, c2 = dot(d0, e1) / l0, dot(d1, e1) / l1, dot(d1, e2) / l1, dot(d2, e2) / l2
        g1 = c0 - c1a
        g2 = c1b - c2
        h11 = (1.0 - c0 * c0) / l0 + (1.0 - c1a * c1a) / l1
        h22 = (1.0 - c1b * c1b) / l1 + (1.0 - c2 * c2) / l2
        h12 = -(dot(e1, e2) - c1a * c1b) / l1
        det = h11 * h22 - h12 * h12
        with np.errstate(divide="ignore", invalid="ignore"):
            s1 = -(h22 * g1 - h12 * g2) / det
            s2 = -(h11 * g2 - h12 * g1) / det
        s1 = np.where(np.isfinite(s1), s1, -g1)
        s2 = np.where(np.isfinite(s2), s2, -g2)
        lam = np.ones_like(z1)
        for _ in range(40):          # halve while the length increases beyond its rounding
            fn = length(z1 + lam * s1, z2 + lam * s2)
            bad = fn > f * (1.0 + 1e-12)
            if not bad.any():
                break
            lam = np.where(bad, 0.5 * lam, lam)
        z1, z2, f = z1 + lam * s1, z2 + lam * s2, length(z1 + lam * s1, z2 + lam * s2)
    Q1 = a1 + z1[..., None] * e1
    Q2 = a2 + z2[..., None] * e2
    conv = (np.abs(g1) < 1e-12) & (np.abs(g2) < 1e-12)
    return Q1, Q2, z1, z2, conv
