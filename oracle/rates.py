"""Time derivatives of the interaction points and of the path length (the velocity and
acceleration of reflection and diffraction points of Sec. III-A.1, eqs. ref_point_velo and
ref_point_acc with App. B, and Sec. III-B with App. C; the Doppler rate).  TEST
INFRASTRUCTURE ONLY.

Every quantity is carried as a triple (x, x', x'') of its value and first and second time
derivatives, and each step of the oracle's construction (kinematics.py, geometry.py) is
differentiated by the product, quotient and square-root rules written out below, so the
derivatives are exact up to rounding:

* terminals and body reference points: (p + v dt + a dt^2/2, v + a dt, a) (eq. Taylor);
* body rotation R(theta) = I + sin(theta) K + (1 - cos(theta)) K^2 about the fixed axis k
  (K = [k]x), theta = w0 dt + wdot dt^2/2: R' = R_theta theta', R'' = R_thetatheta theta'^2
  + R_theta theta'' with R_theta = cos(theta) K + sin(theta) K^2 and
  R_thetatheta = -sin(theta) K + cos(theta) K^2;
* carried points O + R (X0 - O0) and directions R d0;
* images, back-tracked reflection points, the edge point and the segment lengths;
* the two points of a two-edge chain by Newton steps in triple arithmetic.

The Doppler rate is -(f_c / c) d^2 L / dt^2.
"""
import math

import numpy as np

from .kinematics import _skew
from .geometry import double_edge_points

C0 = 299_792_458.0
KIND_R, KIND_D, KIND_S = 1, 2, 3


def _dot(a, b):
    return np.sum(a * b, axis=-1)


# ---------------------------------------------------------------------------- triples

def t_add(a, b):
    return tuple(x + y for x, y in zip(a, b))


def t_sub(a, b):
    return tuple(x - y for x, y in zip(a, b))


def t_dot(a, b):
    """(a . b, (a . b)', (a . b)'') for vector triples."""
    return (_dot(a[0], b[0]),
            _dot(a[1], b[0]) + _dot(a[0], b[1]),
            _dot(a[2], b[0]) + 2.0 * _dot(a[1], b[1]) + _dot(a[0], b[2]))


def t_mul(a, b):
    """Product of scalar triples."""
    return (a[0] * b[0], a[1] * b[0] + a[0] * b[1], a[2] * b[0] + 2.0 * a[1] * b[1] + a[0] * b[2])


def t_scale(s, v):
    """Scalar triple times vector triple."""
    e = lambda x: x[..., None]
    return (e(s[0]) * v[0], e(s[1]) * v[0] + e(s[0]) * v[1],
            e(s[2]) * v[0] + 2.0 * e(s[1]) * v[1] + e(s[0]) * v[2])


def t_div(a, b):
    """a / b for scalar triples: from a = q b, q' = (a' - q b') / b, q'' = (a'' - 2 q' b' - q b'') / b."""
    with np.errstate(divide="ignore", invalid="ignore"):
        q = a[0] / b[0]
        q1 = (a[1] - q * b[1]) / b[0]
        q2 = (a[2] - 2.0 * q1 * b[1] - q * b[2]) / b[0]
    return q, q1, q2


def t_sqrt(a):
    """sqrt of a scalar triple: from r^2 = a, r' = a' / 2r, r'' = (a'' - 2 r'^2) / 2r."""
    r = np.sqrt(a[0])
    with np.errstate(divide="ignore", invalid="ignore"):
        r1 = a[1] / (2.0 * r)
        r2 = (a[2] - 2.0 * r1 * r1) / (2.0 * r)
    return r, r1, r2


def t_norm(v):
    return t_sqrt(t_dot(v, v))


def t_const(x):
    z = np.zeros_like(x)
    return (x, z, z)


# ---------------------------------------------------------------------------- kinematics

def terminal_triple(p0, v0, a, dt):
    dt = np.asarray(dt, dtype=np.float64)[:, None]
    p0, v0, a = (np.asarray(x, dtype=np.float64) for x in (p0, v0, a))
    return (p0 + v0 * dt + 0.5 * a * dt * dt, v0 + a * dt + 0.0 * dt, a + 0.0 * dt)


def body_triples(scene, dt):
    """O (nb,T,3) and R (nb,T,3,3) of every body as triples."""
    dt = np.asarray(dt, dtype=np.float64)
    nb, T = scene["body_O0"].shape[0], dt.shape[0]
    O = [np.empty((nb, T, 3)) for _ in range(3)]
    R = [np.empty((nb, T, 3, 3)) for _ in range(3)]
    for b in range(nb):
        o = terminal_triple(scene["body_O0"][b], scene["body_v0"][b], scene["body_a"][b], dt)
        for i in range(3):
            O[i][b] = o[i]
        w0, wd = scene["body_w0"][b], scene["body_wdot"][b]
        th, th1, th2 = w0 * dt + 0.5 * wd * dt * dt, w0 + wd * dt, wd + 0.0 * dt
        K = _skew(scene["body_axis"][b])
        K2 = K @ K
        s, c = np.sin(th)[:, None, None], np.cos(th)[:, None, None]
        R0 = np.eye(3)[None] + s * K[None] + (1.0 - c) * K2[None]
        Rt = c * K[None] + s * K2[None]
        Rtt = -s * K[None] + c * K2[None]
        R[0][b] = R0
        R[1][b] = Rt * th1[:, None, None]
        R[2][b] = Rtt * (th1 * th1)[:, None, None] + Rt * th2[:, None, None]
    return tuple(O), tuple(R)


def _mv(M, x):
    return np.einsum("...ij,...j->...i", M, x)


def carried_point(X0, O0, Ob, Rb):
    """O + R (X0 - O0) as a triple; X0, O0 (Ng,1,3), Ob/Rb triples indexed per ray."""
    d = X0 - O0
    return tuple(Ob[i] + _mv(Rb[i], d) for i in range(3))


def carried_dir(d0, Rb):
    return tuple(_mv(Rb[i], d0) for i in range(3))


# ---------------------------------------------------------------------------- chain

def _mirror(X, p, n):
    g = t_dot(t_sub(X, p), n)
    return t_sub(X, t_scale(tuple(2.0 * x for x in g), n))


def _chain(src, dst, planes):
    """Back-tracked reflection points (triples) from src to dst over planes [(p, n)]."""
    images, A = [], src
    for p, n in planes:
        A = _mirror(A, p, n)
        images.append(A)
    pts = [None] * len(planes)
    nxt = dst
    for m in range(len(planes) - 1, -1, -1):
        p, n = planes[m]
        s = t_div(t_dot(t_sub(nxt, p), n), t_dot(t_sub(nxt, images[m]), n))
        pts[m] = t_add(nxt, t_scale(s, t_sub(images[m], nxt)))
        nxt = pts[m]
    return pts


def _edge_point(A, B, a, e):
    zA = t_dot(t_sub(A, a), e)
    zB = t_dot(t_sub(B, a), e)
    rA = t_norm(t_sub(t_sub(A, a), t_scale(zA, e)))
    rB = t_norm(t_sub(t_sub(B, a), t_scale(zB, e)))
    zQ = t_add(zB, t_div(t_mul(rB, t_sub(zA, zB)), t_add(rA, rB)))
    return t_add(a, t_scale(zQ, e))


def _double_edge(A, B, a1, e1, a2, e2, steps=6):
    """The two-edge points as triples: the values from geometry.double_edge_points, then
    Newton steps on the stationarity conditions in triple arithmetic, which carry the first
    and second time derivatives of (z1, z2) to convergence (the conditions hold at every
    instant, so their jets vanish)."""
    _, _, z1v, z2v, _ = double_edge_points(A[0], B[0], a1[0], e1[0], a2[0], e2[0])
    z1, z2 = t_const(z1v), t_const(z2v)
    one = t_const(np.ones_like(z1v))
    for _ in range(steps):
        Q1 = t_add(a1, t_scale(z1, e1))
        Q2 = t_add(a2, t_scale(z2, e2))
        d0, d1, d2 = t_sub(Q1, A), t_sub(Q2, Q1), t_sub(B, Q2)
        l0, l1, l2 = t_norm(d0), t_norm(d1), t_norm(d2)
        c0, c1a = t_div(t_dot(d0, e1), l0), t_div(t_dot(d1, e1), l1)
        c1b, c2 = t_div(t_dot(d1, e2), l1), t_div(t_dot(d2, e2), l2)
        g1, g2 = t_sub(c0, c1a), t_sub(c1b, c2)
        h11 = t_add(t_div(t_sub(one, t_mul(c0, c0)), l0), t_div(t_sub(one, t_mul(c1a, c1a)), l1))
        h22 = t_add(t_div(t_sub(one, t_mul(c1b, c1b)), l1), t_div(t_sub(one, t_mul(c2, c2)), l2))
        h12 = t_div(t_sub(t_mul(c1a, c1b), t_dot(e1, e2)), l1)
        det = t_sub(t_mul(h11, h22), t_mul(h12, h12))
        s1 = t_div(t_sub(t_mul(h12, g2), t_mul(h22, g1)), det)
        s2 = t_div(t_sub(t_mul(h12, g1), t_mul(h11, g2)), det)
        z1, z2 = t_add(z1, s1), t_add(z2, s2)
    return t_add(a1, t_scale(z1, e1)), t_add(a2, t_scale(z2, e2))


def _group(scene, rays, kinds, TX, RX, O, R):
    n = len(kinds)
    Ng, T = len(rays), TX[0].shape[0]
    bc = lambda tr: tuple(np.broadcast_to(x[None], (Ng, T, 3)) for x in tr)
    TXg, RXg = bc(TX), bc(RX)
    prims = scene["ray_prim"][rays, :n]
    slots = []
    for i, kind in enumerate(kinds):
        pr = prims[:, i]
        if kind == KIND_R:
            body = scene["plane_body"][pr]
            Ob, Rb = tuple(x[body] for x in O), tuple(x[body] for x in R)
            O0 = scene["body_O0"][body][:, None, :]
            slots.append({"p": carried_point(scene["plane_p0"][pr][:, None, :], O0, Ob, Rb),
                          "n": carried_dir(scene["plane_n0"][pr][:, None, :], Rb)})
        elif kind == KIND_D:
            body = scene["edge_body"][pr]
            Ob, Rb = tuple(x[body] for x in O), tuple(x[body] for x in R)
            O0 = scene["body_O0"][body][:, None, :]
            slots.append({"a": carried_point(scene["edge_a0"][pr][:, None, :], O0, Ob, Rb),
                          "e": carried_dir(scene["edge_e0"][pr][:, None, :], Rb)})
        else:
            body = scene["tile_body"][pr]
            Ob, Rb = tuple(x[body] for x in O), tuple(x[body] for x in R)
            O0 = scene["body_O0"][body][:, None, :]
            slots.append({"c": carried_point(scene["tile_c0"][pr][:, None, :], O0, Ob, Rb)})
    if n == 0:
        pts = []
    elif kinds == (KIND_S,):
        pts = [slots[0]["c"]]
    elif kinds == (KIND_D, KIND_D):
        pts = list(_double_edge(TXg, RXg, slots[0]["a"], slots[0]["e"], slots[1]["a"], slots[1]["e"]))
    elif KIND_D in kinds:
        d = kinds.index(KIND_D)
        A = TXg
        for i in range(d):
            A = _mirror(A, slots[i]["p"], slots[i]["n"])
        B = RXg
        for i in range(n - 1, d, -1):
            B = _mirror(B, slots[i]["p"], slots[i]["n"])
        QD = _edge_point(A, B, slots[d]["a"], slots[d]["e"])
        pts = (_chain(TXg, QD, [(slots[i]["p"], slots[i]["n"]) for i in range(d)]) + [QD]
               + _chain(QD, RXg, [(slots[i]["p"], slots[i]["n"]) for i in range(d + 1, n)]))
    else:
        pts = _chain(TXg, RXg, [(s["p"], s["n"]) for s in slots])
    verts = [TXg] + pts + [RXg]
    L = t_const(np.zeros((Ng, T)))
    for i in range(1, n + 2):
        L = t_add(L, t_norm(t_sub(verts[i], verts[i - 1])))
    return pts, L


def rates(scene, dt, f_c, rays=None):
    """Interaction points and their first and second time derivatives, dL/dt, d2L/dt2 and
    the Doppler rate at the offsets dt.  Returns dict: Q, dQ, ddQ (R,T,4,3; zero for unused
    slots), dL, ddL, dop_rate (R,T).  Values are returned whatever the chain's validity."""
    dt = np.atleast_1d(np.asarray(dt, dtype=np.float64))
    if rays is None:
        rays = np.arange(scene["ray_nint"].shape[0])
    rays = np.asarray(rays)
    Rn, T = len(rays), len(dt)
    TX = terminal_triple(scene["tx_p"], scene["tx_v"], scene["tx_a"], dt)
    RX = terminal_triple(scene["rx_p"], scene["rx_v"], scene["rx_a"], dt)
    O, Rm = body_triples(scene, dt)
    out = {k: np.zeros((Rn, T, 4, 3)) for k in ("Q", "dQ", "ddQ")}
    for k in ("dL", "ddL"):
        out[k] = np.zeros((Rn, T))
    sigs = {}
    for pos, r in enumerate(rays):
        nint = int(scene["ray_nint"][r])
        sigs.setdefault(tuple(int(x) for x in scene["ray_kind"][r, :nint]), []).append(pos)
    for kinds, positions in sigs.items():
        positions = np.asarray(positions)
        pts, L = _group(scene, rays[positions], kinds, TX, RX, O, Rm)
        for i, q in enumerate(pts):
            out["Q"][positions, :, i] = q[0]
            out["dQ"][positions, :, i] = q[1]
            out["ddQ"][positions, :, i] = q[2]
        out["dL"][positions] = L[1]
        out["ddL"][positions] = L[2]
    out["dop_rate"] = -(f_c / C0) * out["ddL"]
    return out


def taylor_points(rts, j0, dt):
    """Second-order Taylor extrapolation of the interaction points from instant index j0:
    Q(t) ~ Q + dQ (t - t_j0) + ddQ (t - t_j0)^2 / 2 (the alternative to re-solving)."""
    d = (np.asarray(dt, dtype=np.float64) - dt[j0])[None, :, None, None]
    return (rts["Q"][:, j0:j0 + 1] + rts["dQ"][:, j0:j0 + 1] * d + 0.5 * rts["ddQ"][:, j0:j0 + 1] * d * d)
