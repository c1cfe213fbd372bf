"""Snapshot ray tracing at one instant: the image method with visibility on polyhedral
scenes, the conventional RT whose ray set DRT extrapolates (Sec. II: the t0 trace and its
refresh at the end of each multipath lifetime T_C).  TEST INFRASTRUCTURE ONLY.

The scene's primitives are first moved to the instant t (kinematics.py).  A candidate is an
interaction sequence; it is a path when:

* reflections (walls w_1..w_n, consecutive walls distinct): with the images of TX through
  the walls in order and the points back-tracked from RX (geometry.reflection_chain), every
  parameter s lies in (0, 1), every point lies in its wall's facet (a parallelogram, edges
  included; a wall without a facet is unbounded) and both neighbouring vertices lie on the
  wall's front side by more than 1e-9 m, n . (P - Q) > 1e-9 (a wall that contains the
  ray's diffracting edge puts the segment between them inside the wall: not a path);
* one diffraction, with reflections before and after it: the edge point comes from the
  unfolded closed form (eq. diff_point) between the image of TX through the walls before the
  edge and the image of RX through the walls after it; it lies on the edge segment, and the
  directions towards both neighbours lie in the wedge's exterior, their angle from the
  0-face (atan2 of the components along the 0-face normal and tangent) in [0, n pi];
  reflection points as above, back-tracked towards the edge point from both sides;
* two diffractions (consecutive edges distinct): the points of the shortest path over both
  edge lines (geometry.double_edge_points), each on its segment with its neighbours in its
  wedge's exterior;
* diffuse scattering from a tile whose front faces both terminals;
* line of sight;

and, in every case, no segment of the path is obstructed: no wall's facet (or unbounded
plane) crosses the segment more than 1e-7 m from both of its ends.

Polarisation flags follow the scalar model: perpendicular for walls with |n_z| <= 0.5 and
for edges with |e_z| > 0.5 (vertical), parallel otherwise; perpendicular for tiles.
"""
import itertools
import math

import numpy as np

from .kinematics import terminal_state, body_poses, place_points, rotate
from .geometry import dot, norm, reflection_chain, edge_point, double_edge_points
from .drt import extrapolate

KIND_R, KIND_D, KIND_S = 1, 2, 3
POL_PERP, POL_PAR = 0, 1
SEG_EPS = 1e-7
FRONT_EPS = 1e-9   # a neighbour this close to a wall's plane is grazing, not in front


def moved_scene(scene, t):
    """Primitives, terminals and facet data at the instant t0 + t."""
    O, R, _, _ = body_poses(scene, np.array([float(t)]))
    O, R = O[:, 0], R[:, 0]
    O0 = scene["body_O0"]
    ms = {}
    pb = scene["plane_body"]
    ms["p"] = place_points(scene["plane_p0"], O0[pb], O[pb], R[pb])
    ms["n"] = rotate(scene["plane_n0"], R[pb])
    npl = len(pb)
    F = scene.get("plane_facet", np.zeros((npl, 3, 3)))
    ms["bounded"] = np.any(F[:, 1] != 0.0, axis=1) | np.any(F[:, 2] != 0.0, axis=1)
    ms["corner"] = place_points(F[:, 0], O0[pb], O[pb], R[pb])
    ms["u"] = rotate(F[:, 1], R[pb])
    ms["v"] = rotate(F[:, 2], R[pb])
    eb = scene["edge_body"]
    ms["a"] = place_points(scene["edge_a0"], O0[eb], O[eb], R[eb])
    ms["e"] = rotate(scene["edge_e0"], R[eb])
    ms["et"] = rotate(scene["edge_t0"], R[eb])
    ms["en"] = rotate(scene["edge_n0"], R[eb])
    ms["wn"] = scene["edge_wedge_n"]
    ms["zlim"] = scene.get("edge_zlim", np.tile([-np.inf, np.inf], (len(eb), 1)))
    tb = scene["tile_body"]
    ms["c"] = place_points(scene["tile_c0"], O0[tb], O[tb], R[tb])
    ms["cn"] = rotate(scene["tile_n0"], R[tb])
    tt = np.array([float(t)])
    ms["tx"] = terminal_state(scene["tx_p"], scene["tx_v"], scene["tx_a"], tt)[0][0]
    ms["rx"] = terminal_state(scene["rx_p"], scene["rx_v"], scene["rx_a"], tt)[0][0]
    return ms


def facet_coords(ms, planes, X):
    """(s, w) with X - corner = s u + w v + (normal part), by the 2x2 Gram system."""
    u, v = ms["u"][planes], ms["v"][planes]
    x = X - ms["corner"][planes]
    uu, uv, vv = dot(u, u), dot(u, v), dot(v, v)
    xu, xv = dot(x, u), dot(x, v)
    det = uu * vv - uv * uv
    with np.errstate(divide="ignore", invalid="ignore"):
        s = (vv * xu - uv * xv) / det
        w = (uu * xv - uv * xu) / det
    return s, w


def in_facet(ms, planes, X):
    s, w = facet_coords(ms, planes, X)
    inside = (s >= 0.0) & (s <= 1.0) & (w >= 0.0) & (w <= 1.0)
    return np.where(ms["bounded"][planes], inside, True)


def obstructed(ms, A, B, chunk=2048):
    """(M,) True where some wall crosses the segment A -> B (M,3) away from its ends."""
    A, B = np.atleast_2d(A), np.atleast_2d(B)
    out = np.zeros(A.shape[0], dtype=bool)
    P, N = ms["p"], ms["n"]
    allp = np.arange(P.shape[0])
    for c0 in range(0, A.shape[0], chunk):
        a, b = A[c0:c0 + chunk], B[c0:c0 + chunk]
        d = b - a
        ln = norm(d)[:, None]
        den = d @ N.T
        num = np.einsum("pk,pk->p", P, N)[None, :] - a @ N.T
        with np.errstate(divide="ignore", invalid="ignore"):
            tau = num / den
        cross = np.isfinite(tau) & (tau * ln > SEG_EPS) & ((1.0 - tau) * ln > SEG_EPS)
        H = a[:, None, :] + np.where(cross, tau, 0.0)[..., None] * d[:, None, :]
        hit = cross & in_facet(ms, allp[None, :], H)
        out[c0:c0 + chunk] = hit.any(axis=1)
    return out


def _front(ms, pl, X, Q):
    return dot(X - Q, ms["n"][pl]) > FRONT_EPS


def _wedge_angle(ms, ed, Q, X):
    u = X - Q
    u = u - dot(u, ms["e"][ed])[..., None] * ms["e"][ed]
    return np.mod(np.arctan2(dot(u, ms["en"][ed]), dot(u, ms["et"][ed])), 2.0 * math.pi)


def path_exists(ms, kinds, prims, visibility=True):
    """Vectorised over M candidates of one signature: prims (M, n).  Returns (exists (M,),
    L (M,), vertices list of (M,3) from TX to RX).  visibility=False skips the wedge-exterior
    and obstruction tests (the geometric existence of the interaction points alone)."""
    prims = np.asarray(prims, dtype=np.int64)
    assert prims.ndim == 2 and prims.shape[1] == len(kinds)
    M, n = prims.shape
    TX = np.broadcast_to(ms["tx"], (M, 3))
    RX = np.broadcast_to(ms["rx"], (M, 3))
    ok = np.ones(M, dtype=bool)
    if n == 0:
        pts = []
    elif kinds == (KIND_S,):
        c, cn = ms["c"][prims[:, 0]], ms["cn"][prims[:, 0]]
        ok &= (dot(TX - c, cn) > 0.0) & (dot(RX - c, cn) > 0.0)
        pts = [c]
    elif kinds == (KIND_D, KIND_D):
        e1, e2 = prims[:, 0], prims[:, 1]
        Q1, Q2, z1, z2, conv = double_edge_points(TX, RX, ms["a"][e1], ms["e"][e1], ms["a"][e2], ms["e"][e2])
        ok &= conv
        for ed, z in ((e1, z1), (e2, z2)):
            ok &= (z >= ms["zlim"][ed, 0]) & (z <= ms["zlim"][ed, 1])
        if visibility:
            for ed, Q, prev, nxt in ((e1, Q1, TX, Q2), (e2, Q2, Q1, RX)):
                lim = ms["wn"][ed] * math.pi
                ok &= (_wedge_angle(ms, ed, Q, prev) <= lim) & (_wedge_angle(ms, ed, Q, nxt) <= lim)
        pts = [Q1, Q2]
    elif KIND_D in kinds:
        d = kinds.index(KIND_D)
        before = [(ms["p"][prims[:, i]], ms["n"][prims[:, i]]) for i in range(d)]
        after = [(ms["p"][prims[:, i]], ms["n"][prims[:, i]]) for i in range(d + 1, n)]
        _, imA, _ = reflection_chain(TX, TX, before) if before else (None, [TX], None)
        A = imA[-1]
        _, imB, _ = reflection_chain(RX, RX, after[::-1]) if after else (None, [RX], None)
        B = imB[-1]
        ed = prims[:, d]
        QD, zA, zB, rA, rB = edge_point(A, B, ms["a"][ed], ms["e"][ed])
        ok &= (rA > 0.0) & (rB > 0.0)
        zQ = dot(QD - ms["a"][ed], ms["e"][ed])
        ok &= (zQ >= ms["zlim"][ed, 0]) & (zQ <= ms["zlim"][ed, 1])
        if visibility:
            lim = ms["wn"][ed] * math.pi
            ok &= (_wedge_angle(ms, ed, QD, A) <= lim) & (_wedge_angle(ms, ed, QD, B) <= lim)
        p1, _, v1 = reflection_chain(TX, QD, before)
        p2, _, v2 = reflection_chain(QD, RX, after)
        ok &= v1 & v2
        pts = p1 + [QD] + p2
    else:
        planes = [(ms["p"][prims[:, i]], ms["n"][prims[:, i]]) for i in range(n)]
        pts, _, v = reflection_chain(TX, RX, planes)
        ok &= v
    verts = [TX] + pts + [RX]
    for i, k in enumerate(kinds):
        if k == KIND_R:
            pl = prims[:, i]
            Q = verts[i + 1]
            ok &= in_facet(ms, pl, Q) & _front(ms, pl, verts[i], Q) & _front(ms, pl, verts[i + 2], Q)
    L = np.zeros(M)
    for i in range(1, len(verts)):
        L += norm(verts[i] - verts[i - 1])
    idx = np.nonzero(ok)[0] if visibility else np.zeros(0, dtype=np.int64)
    for i in range(1, len(verts)):
        if idx.size:
            blk = obstructed(ms, verts[i - 1][idx], verts[i][idx])
            ok[idx[blk]] = False
            idx = idx[~blk]
    return ok, L, verts


def pols_of(ms, kinds, prims):
    out = []
    for k, p in zip(kinds, prims):
        if k == KIND_R:
            out.append(POL_PAR if abs(ms["n"][p][2]) > 0.5 else POL_PERP)
        elif k == KIND_D:
            out.append(POL_PERP if abs(ms["e"][p][2]) > 0.5 else POL_PAR)
        else:
            out.append(POL_PERP)
    return tuple(out)


def signatures(max_refl, max_refl_diff, scattering, los, double_diff=False):
    """Signature tuples in the tracer's order: LoS; reflections by count; one diffraction
    with 0..max_refl_diff reflections, the edge at every position; two diffractions;
    scattering."""
    sigs = [()] if los else []
    for n in range(1, max_refl + 1):
        sigs.append((KIND_R,) * n)
    for n in range(0, max_refl_diff + 1):
        for d in range(n + 1):
            sigs.append((KIND_R,) * d + (KIND_D,) + (KIND_R,) * (n - d))
    if double_diff:
        sigs.append((KIND_D, KIND_D))
    if scattering:
        sigs.append((KIND_S,))
    return sigs


def candidates(ms, kinds):
    """Every primitive sequence of the signature, consecutive walls distinct, in
    lexicographic order of the primitive indices."""
    npl, ned, nti = ms["p"].shape[0], ms["a"].shape[0], ms["c"].shape[0]
    ranges = [range(npl) if k == KIND_R else range(ned) if k == KIND_D else range(nti) for k in kinds]
    out = []
    for seq in itertools.product(*ranges):
        if any(kinds[i] == kinds[i + 1] != KIND_S and seq[i] == seq[i + 1] for i in range(len(seq) - 1)):
            continue
        out.append(seq)
    return np.array(out, dtype=np.int64).reshape(len(out), len(kinds))


def trace(scene, t=0.0, max_refl=2, max_refl_diff=1, scattering=True, los=True, double_diff=False):
    """All paths at the instant t0 + t: list of (kinds, prims, pols, L) in the tracer's
    order (signature order of signatures(), then primitive indices lexicographically)."""
    ms = moved_scene(scene, t)
    out = []
    for kinds in signatures(max_refl, max_refl_diff, scattering, los, double_diff):
        cand = candidates(ms, kinds)
        if cand.shape[0] == 0:
            continue
        ok, L, _ = path_exists(ms, kinds, cand)
        for i in np.nonzero(ok)[0]:
            prims = tuple(int(x) for x in cand[i])
            out.append((kinds, prims, pols_of(ms, kinds, prims), float(L[i])))
    return out


def rebase(scene, t):
    """The scene carried to the instant t0 + t: terminals by eq. Taylor; each body's
    reference point, velocity and angular speed advanced; every primitive placed with its
    body's pose at t (kinematics.py); rays unchanged."""
    t = float(t)
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    out["t0"] = scene.get("t0", 0.0) + t
    for w in ("tx", "rx"):
        p, v = terminal_state(scene[w + "_p"], scene[w + "_v"], scene[w + "_a"], np.array([t]))
        out[w + "_p"], out[w + "_v"] = p[0], v[0]
    O, R, V, W = body_poses(scene, np.array([t]))
    O, R = O[:, 0], R[:, 0]
    O0 = scene["body_O0"]
    out["body_O0"] = O
    out["body_v0"] = V[:, 0]
    out["body_w0"] = W[:, 0]
    pb, eb, tb = scene["plane_body"], scene["edge_body"], scene["tile_body"]
    out["plane_p0"] = place_points(scene["plane_p0"], O0[pb], O[pb], R[pb])
    out["plane_n0"] = rotate(scene["plane_n0"], R[pb])
    if "plane_facet" in scene:
        F = scene["plane_facet"]
        out["plane_facet"] = np.stack([place_points(F[:, 0], O0[pb], O[pb], R[pb]),
                                       rotate(F[:, 1], R[pb]), rotate(F[:, 2], R[pb])], axis=1)
    out["edge_a0"] = place_points(scene["edge_a0"], O0[eb], O[eb], R[eb])
    for k in ("edge_e0", "edge_t0", "edge_n0"):
        out[k] = rotate(scene[k], R[eb])
    out["tile_c0"] = place_points(scene["tile_c0"], O0[tb], O[tb], R[tb])
    out["tile_n0"] = rotate(scene["tile_n0"], R[tb])
    return out


def with_rays(scene, paths):
    """The scene with its rays replaced by the traced paths [(kinds, prims, pols, L)]."""
    out = dict(scene)
    n = len(paths)
    out["ray_nint"] = np.array([len(k) for k, *_ in paths], np.uint8).reshape(n)
    out["ray_kind"] = np.zeros((n, 4), np.uint8)
    out["ray_prim"] = np.zeros((n, 4), np.int32)
    out["ray_pol"] = np.zeros((n, 4), np.uint8)
    for r, (k, p, q, _) in enumerate(paths):
        out["ray_kind"][r, :len(k)] = k
        out["ray_prim"][r, :len(k)] = p
        out["ray_pol"][r, :len(k)] = q
    return out


def segments(scene, dt, n_steps, f_c, trace_opts, threshold_db, max_steps, min_steps=1):
    """Multipath lifetimes (Sec. II: the extrapolation holds over T_C while no major path
    disappears; at its end the conventional trace is run again).  From instant j (starting
    at 0): trace at t0 + j dt, carry the scene there, extrapolate its rays over the next
    m = min(max_steps, n_steps - j) instants with the validity monitor; the major rays are
    those whose power at instant j is within threshold_db of the strongest; the segment
    lasts until the first instant at which a major ray is out of bounds, at least min_steps
    and at most m instants.  Returns [(j, length, paths)]."""
    j, out = 0, []
    while j < n_steps:
        paths = trace(scene, j * dt, **trace_opts)
        m = min(max_steps, n_steps - j)
        length = m
        if paths:
            sc = with_rays(rebase(scene, j * dt), paths)
            ex = extrapolate(sc, np.arange(m) * dt, f_c)
            p0 = np.abs(ex["gain"][:, 0]) ** 2
            major = p0 >= p0.max() * 10.0 ** (-threshold_db / 10.0)
            length = int(min(m, max(min_steps, ex["first_out"][major].min())))
        out.append((j, length, paths))
        j += length
    return out
