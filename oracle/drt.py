"""Per-(ray, time) extrapolation and the time-variant transfer function (oracle steps O1-O8).
TEST INFRASTRUCTURE ONLY.

For each time instant the oracle displaces terminals and bodies (kinematics.py), moves the
primitives of each ray's interaction sequence rigidly with their body, re-solves the
interaction points (geometry.py), and evaluates:

* path length L = sum |Q_i - Q_{i-1}| over TX, Q_1..Q_n, RX and delay L/c (Sec. II: the
  total field, transfer function, Doppler shifts and delays are extrapolated per instant);
* Doppler (Appendix A): the multi-bounce product formula is, to first order in v/c,
  f_D = -(f_c/c) dL/dt with dL/dt = sum_i k_i . (u_i - u_{i-1}), u_0 = v_TX,
  u_{n+1} = v_RX and u_i the velocity of the body's material point at Q_i (eq.
  RigidBodyMotion).  The sliding part of a reflection (diffraction) point's velocity lies
  in the wall (along the edge) and cancels by Snell's law (Keller's law), so the material
  velocity gives the same dL/dt as the sliding-point velocities of Appendices B and C;
* angles of departure and arrival (azimuth, elevation) of the first and last segment;
* the channel coefficient at the carrier (em.py), zero for an inconsistent chain;
* H(t_j, f_k) = sum_r a_r(t_j) exp(-j 2 pi frac(f_k L_r(t_j) / c)), with f_k L / c formed
  and reduced modulo one cycle in float64, one direct complex exponential per sample.

A chain is inconsistent (valid = 0, every output 0) when a reflection parameter leaves
(0, 1), a diffraction source or receiver lies on the edge line, or a scattering tile faces
away from a terminal.

Validity monitor (the multipath lifetime T_C of Sec. II: the extrapolation holds while no
path disappears).  A consistent chain is in bounds at an instant when, on the geometry
displaced to that instant, every reflection point lies in its wall's facet (the
parallelogram corner + s u + w v, 0 <= s, w <= 1, carried with the wall's body) with both
neighbouring vertices on the front side of the wall (n . (P - Q) >= 0), and every
diffraction point lies on its edge segment (z_lo <= (Q_D - a) . e <= z_hi).  Walls without a
facet and edges without limits are unbounded.  `bounds_margin` is the smallest of these
signed distances in metres (facet coordinates scaled by the side lengths), `first_out` the
first instant index at which a ray is not in bounds (the number of instants if never).
"""
import math

import numpy as np

from .kinematics import terminal_state, body_poses, place_points, rotate, material_velocity
from .geometry import (dot, norm, mirror, reflection_chain, edge_point, double_edge_points,
                       direction_angles)
from .em import fresnel_gamma, utd_coefficient, er_gain
from . import polar

C0 = 299_792_458.0
KIND_R, KIND_D, KIND_S = 1, 2, 3
RHO_MIN = 1e-9  # a diffraction source/receiver closer than this to the edge line is degenerate
# A wedge angle (Sec. III-B, the UTD angles from the 0-face) measured inside the wedge body
# within this many radians of the 0-face is a direction along that face whose sign rounding
# decided: it is read as on the face (a tiny negative angle, where the coefficient is
# continuous) instead of near 2 pi.  Two edges of one face (a path along a roof) need this.
FACE_EPS = 1e-5


def freq_axis(f_c, bandwidth, n_sub):
    """f_k = f_c + (k - n_sub//2) * (bandwidth / n_sub), k = 0..n_sub-1."""
    k = np.arange(n_sub, dtype=np.float64)
    return f_c + (k - (n_sub // 2)) * (bandwidth / n_sub)


def _unit(v):
    return v / norm(v)[..., None]


def _wedge_angle(u, ed, wn):
    """Angle of the edge-normal component u from the 0-face (tangent t towards normal n) in
    [0, 2 pi), except inside the wedge body within FACE_EPS of 2 pi, read as on the 0-face."""
    phi = np.mod(np.arctan2(dot(u, ed["n"]), dot(u, ed["t"])), 2.0 * math.pi)
    return np.where((phi > wn * math.pi) & (phi > 2.0 * math.pi - FACE_EPS), phi - 2.0 * math.pi, phi)


def _moved(scene, kind, prim, poses, k_axis):
    """Primitive data of one interaction slot moved to every time: dict of (Ng,T,...) arrays."""
    O, R, V, W = poses
    if kind == KIND_R:
        body = scene["plane_body"][prim]
        Ob, Rb = O[body], R[body]
        O0 = scene["body_O0"][body][:, None, :]
        return {"body": body, "p": place_points(scene["plane_p0"][prim][:, None, :], O0, Ob, Rb),
                "n": rotate(scene["plane_n0"][prim][:, None, :], Rb)}
    if kind == KIND_D:
        body = scene["edge_body"][prim]
        Ob, Rb = O[body], R[body]
        O0 = scene["body_O0"][body][:, None, :]
        return {"body": body, "a": place_points(scene["edge_a0"][prim][:, None, :], O0, Ob, Rb),
                "e": rotate(scene["edge_e0"][prim][:, None, :], Rb),
                "t": rotate(scene["edge_t0"][prim][:, None, :], Rb),
                "n": rotate(scene["edge_n0"][prim][:, None, :], Rb)}
    body = scene["tile_body"][prim]
    Ob, Rb = O[body], R[body]
    O0 = scene["body_O0"][body][:, None, :]
    return {"body": body, "c": place_points(scene["tile_c0"][prim][:, None, :], O0, Ob, Rb),
            "n": rotate(scene["tile_n0"][prim][:, None, :], Rb)}


def _bounds_margin(scene, kinds, prims, slots, verts, pts, poses):
    """Smallest signed distance [m] of the chain's points to the edges of their facets /
    segments and of the neighbouring vertices to the front side of each wall; +inf when
    nothing bounds the chain."""
    O, R, V, W = poses
    Ng, T = verts[0].shape[:2]
    margin = np.full((Ng, T), np.inf)
    facets = scene.get("plane_facet")
    zlim = scene.get("edge_zlim")
    for i, kind in enumerate(kinds):
        if kind == KIND_R:
            nn = slots[i]["n"]
            margin = np.minimum(margin, dot(verts[i] - pts[i], nn))        # previous vertex
            margin = np.minimum(margin, dot(verts[i + 2] - pts[i], nn))    # next vertex
            if facets is None:
                continue
            fac = facets[prims[:, i]]                                       # (Ng,3,3) corner, u, v
            body = slots[i]["body"]
            O0 = scene["body_O0"][body][:, None, :]
            corner = place_points(fac[:, 0][:, None, :], O0, O[body], R[body])
            u = rotate(fac[:, 1][:, None, :], R[body])
            v = rotate(fac[:, 2][:, None, :], R[body])
            d = pts[i] - corner
            uu, uv, vv = dot(u, u), dot(u, v), dot(v, v)
            du, dv = dot(d, u), dot(d, v)
            bounded = (uu > 0) & (vv > 0)
            with np.errstate(divide="ignore", invalid="ignore"):
                det = uu * vv - uv * uv
                cs = (vv * du - uv * dv) / det          # d = cs u + cw v (in the wall plane)
                cw = (uu * dv - uv * du) / det
            lu, lv = np.sqrt(uu), np.sqrt(vv)
            m = np.minimum(np.minimum(cs, 1.0 - cs) * lu, np.minimum(cw, 1.0 - cw) * lv)
            margin = np.where(bounded, np.minimum(margin, m), margin)
        elif kind == KIND_D and zlim is not None:
            z = dot(pts[i] - slots[i]["a"], slots[i]["e"])
            lim = zlim[prims[:, i]]
            margin = np.minimum(margin, np.minimum(z - lim[:, 0:1], lim[:, 1:2] - z))
    return margin


def _solve_group(scene, rays, kinds, TX, VTX, RX, VRX, poses, f_c):
    """Outputs for the rays `rays` (all with interaction kinds `kinds`) at every time."""
    O, R, V, W = poses
    axis = scene["body_axis"]
    n = len(kinds)
    Ng, T = len(rays), TX.shape[0]
    TXg = np.broadcast_to(TX[None], (Ng, T, 3))
    RXg = np.broadcast_to(RX[None], (Ng, T, 3))
    prims = scene["ray_prim"][rays, :n]
    pols = scene["ray_pol"][rays, :n]
    slots = [_moved(scene, kinds[i], prims[:, i], poses, axis) for i in range(n)]
    valid = np.ones((Ng, T), dtype=bool)
    degen = np.zeros((Ng, T), dtype=bool)   # a chain no instant can solve (diagnostic)
    extra = {}

    if n == 0:
        pts = []
    elif kinds == (KIND_S,):
        pts = [slots[0]["c"]]
    elif kinds == (KIND_D, KIND_D):
        # two edges: the coupled stationary-length solve (geometry.double_edge_points)
        e1, e2 = slots[0], slots[1]
        Q1, Q2, _, _, conv = double_edge_points(TXg, RXg, e1["a"], e1["e"], e2["a"], e2["e"])
        pts = [Q1, Q2]

        def rho(X, ed):
            w = X - ed["a"]
            return norm(w - dot(w, ed["e"])[..., None] * ed["e"])
        far = ((rho(TXg, e1) > RHO_MIN) & (rho(Q2, e1) > RHO_MIN) & (rho(Q1, e2) > RHO_MIN)
               & (rho(RXg, e2) > RHO_MIN))
        valid &= conv & far
        degen = ~far
        extra = {"dd": True}
    elif KIND_D in kinds:
        d = kinds.index(KIND_D)
        before = [(slots[i]["p"], slots[i]["n"]) for i in range(d)]
        after = [(slots[i]["p"], slots[i]["n"]) for i in range(d + 1, n)]
        A = TXg
        for p, nn in before:
            A = mirror(A, p, nn)
        B = RXg
        for p, nn in reversed(after):
            B = mirror(B, p, nn)
        ed = slots[d]
        QD, zA, zB, rA, rB = edge_point(A, B, ed["a"], ed["e"])
        pb, _, v1, d1 = reflection_chain(TXg, QD, before, return_den=True)
        pa, _, v2, d2 = reflection_chain(QD, RXg, after, return_den=True)
        pts = pb + [QD] + pa
        valid &= v1 & v2 & (rA > RHO_MIN) & (rB > RHO_MIN)
        degen = ~((rA > RHO_MIN) & (rB > RHO_MIN))
        for den in d1 + d2:
            degen |= den == 0
        extra = {"d": d, "A": A, "B": B, "QD": QD}
    else:
        pts, _, v, dens = reflection_chain(TXg, RXg, [(s["p"], s["n"]) for s in slots], return_den=True)
        valid &= v
        for den in dens:
            degen |= den == 0

    verts = [TXg] + pts + [RXg]
    segs = [verts[i] - verts[i - 1] for i in range(1, n + 2)]
    lens = [norm(s) for s in segs]
    with np.errstate(divide="ignore", invalid="ignore"):
        khat = [s / l[..., None] for s, l in zip(segs, lens)]
    L = np.sum(lens, axis=0)
    for ln in lens:
        degen |= ~(ln > 0)

    # Doppler from the material velocities of the interaction points
    u = [np.broadcast_to(VTX[None], (Ng, T, 3))]
    for i in range(n):
        body = slots[i]["body"]
        u.append(material_velocity(pts[i], O[body], V[body], W[body], axis[body][:, None, :]))
    u.append(np.broadcast_to(VRX[None], (Ng, T, 3)))
    dLdt = np.sum([dot(khat[i], u[i + 1] - u[i]) for i in range(n + 1)], axis=0)
    dop = -(f_c / C0) * dLdt

    aod_az, aod_el = direction_angles(khat[0])
    aoa_az, aoa_el = direction_angles(-khat[-1])

    # field coefficient at the carrier: the scalar model multiplies the coefficient of each
    # interaction's polarisation flag; with dipole antennas (polar.py) both coefficients of
    # every interaction enter the dyadic transport instead
    lam = C0 / f_c
    k = 2.0 * math.pi / lam
    ants = polar.antennas(scene)
    coef = [None] * n
    gam = np.ones((Ng, T), dtype=np.complex128)
    for i in range(n):
        if kinds[i] != KIND_R:
            continue
        pl = prims[:, i]
        mat = scene["plane_mat"][pl]
        cos_t = np.abs(dot(khat[i], slots[i]["n"]))
        args = (cos_t, scene["mat_eps_r"][mat][:, None], scene["mat_sigma"][mat][:, None], lam,
                scene["mat_pec"][mat][:, None] != 0)
        if ants is None:
            gam = gam * fresnel_gamma(*args, pols[:, i][:, None])
        else:
            coef[i] = (fresnel_gamma(*args, 0), fresnel_gamma(*args, 1), slots[i]["n"])
    if ants is not None:
        if KIND_D not in kinds:
            gam = polar.transport(ants, kinds, khat, coef)
    if n == 0 or (KIND_D not in kinds and KIND_S not in kinds):
        a = gam * lam / (4.0 * math.pi * L)
    elif KIND_S in kinds:
        t = prims[:, 0]
        nt = slots[0]["n"]
        cos_ti = -dot(khat[0], nt)
        cos_ts = dot(khat[1], nt)
        spec = khat[0] - 2.0 * dot(khat[0], nt)[..., None] * nt
        cos_psi = dot(spec, khat[1])
        a = np.zeros((Ng, T), dtype=np.complex128)
        for g in range(Ng):
            tt = t[g]
            a[g] = er_gain(scene["tile_model"][tt], scene["tile_alpha"][tt], scene["tile_S"][tt],
                           scene["tile_area"][tt], scene["tile_phase0"][tt], cos_ti[g],
                           cos_ts[g], cos_psi[g], lens[0][g], lens[1][g], lam)
        if ants is not None:
            a = a * gam
        valid &= (cos_ti > 0.0) & (cos_ts > 0.0)
    elif "dd" in extra:
        # UTD for successive edges, non-slope.  The field diffracted by the first edge
        # reaches the second as an astigmatic wave: one caustic on the first edge (principal
        # radius s1), the other at the source's distance s0 + s1, which for parallel edges is
        # also its radius of curvature in the second edge's plane of incidence.  The
        # Kouyoumjian-Pathak distance parameter of such a wave,
        # L = s (r_e + s) r_1 r_2 sin^2 b / (r_e (r_1 + s) (r_2 + s)), then gives
        # L1 = s0 s1 sin^2 b1 / (s0 + s1) (a point source) and L2 = s1 s2 sin^2 b2 / (s1 + s2),
        # and the spreading sqrt(r_e / (s (r_e + s))) of each edge gives
        # 1 / sqrt(s0 s1 s2 (s0 + s1 + s2)) overall (exact for parallel edges, an
        # approximation otherwise)
        s0, s1, s2 = lens
        Ds, Ls = [], [s0 * s1 / (s0 + s1), s1 * s2 / (s1 + s2)]
        for j in range(2):
            ed = slots[j]
            e = ed["e"]
            prev, nxt = verts[j], verts[j + 2]
            Q = pts[j]
            cos_b0 = dot(_unit(Q - prev), e)
            sin_b0 = np.sqrt(np.maximum(1.0 - cos_b0 * cos_b0, 0.0))
            up = (prev - Q) - dot(prev - Q, e)[..., None] * e
            uo = (nxt - Q) - dot(nxt - Q, e)[..., None] * e
            wn = scene["edge_wedge_n"][prims[:, j]][:, None]
            phi_p = _wedge_angle(up, ed, wn)
            phi = _wedge_angle(uo, ed, wn)
            Ld = Ls[j] * sin_b0 ** 2
            if ants is None:
                Ds.append(utd_coefficient(phi, phi_p, sin_b0, wn, k, Ld, pols[:, j][:, None]))
            else:
                coef[j] = (utd_coefficient(phi, phi_p, sin_b0, wn, k, Ld, 0),
                           utd_coefficient(phi, phi_p, sin_b0, wn, k, Ld, 1), e)
        D = Ds[0] * Ds[1] if ants is None else polar.transport(ants, kinds, khat, coef)
        a = lam / (4.0 * math.pi) * D / np.sqrt(s0 * s1 * s2 * (s0 + s1 + s2))
    else:
        d = extra["d"]
        ed = slots[d]
        QD, A, B = extra["QD"], extra["A"], extra["B"]
        sp = norm(A - QD)
        s = norm(B - QD)
        e = ed["e"]
        cos_b0 = dot(_unit(QD - A), e)
        sin_b0 = np.sqrt(np.maximum(1.0 - cos_b0 * cos_b0, 0.0))
        up = (A - QD) - dot(A - QD, e)[..., None] * e
        uo = (B - QD) - dot(B - QD, e)[..., None] * e
        wn = scene["edge_wedge_n"][prims[:, d]][:, None]
        phi_p = _wedge_angle(up, ed, wn)
        phi = _wedge_angle(uo, ed, wn)
        Ld = s * sp * sin_b0 ** 2 / (s + sp)
        if ants is None:
            D = utd_coefficient(phi, phi_p, sin_b0, wn, k, Ld, pols[:, d][:, None])
        else:
            coef[d] = (utd_coefficient(phi, phi_p, sin_b0, wn, k, Ld, 0),
                       utd_coefficient(phi, phi_p, sin_b0, wn, k, Ld, 1), e)
            D = polar.transport(ants, kinds, khat, coef)
        a = gam * lam / (4.0 * math.pi) * D / np.sqrt(sp * s * (sp + s))

    margin = _bounds_margin(scene, kinds, prims, slots, verts, pts, poses)

    out = {"L": L, "dop": dop, "aod_az": aod_az, "aod_el": aod_el, "aoa_az": aoa_az,
           "aoa_el": aoa_el, "gain": a, "valid": valid}
    for key in out:
        if key == "valid":
            continue
        out[key] = np.where(valid, out[key], 0)
    out["bounds_margin"] = margin
    out["in_bounds"] = valid & (margin >= 0.0)
    out["degenerate"] = degen
    out["_pts"] = pts
    out["_khat"] = khat
    return out


def extrapolate(scene, dt, f_c, rays=None, chunk=256, keep_points=False):
    """Per-(ray, time) outputs at the time offsets dt (T,) for the rays `rays`
    (default all): dict of (R,T) arrays L [m], tau [s], dop [Hz], aod_az, aod_el, aoa_az,
    aoa_el [rad], gain (complex), valid (bool), in_bounds (bool), bounds_margin [m], and
    first_out (R,) of the validity monitor.  With keep_points=True, also "points":
    list per ray of the (T,3) interaction points and "khat": the unit segment directions."""
    dt = np.atleast_1d(np.asarray(dt, dtype=np.float64))
    if rays is None:
        rays = np.arange(scene["ray_nint"].shape[0])
    rays = np.asarray(rays)
    R, T = len(rays), len(dt)
    TX, VTX = terminal_state(scene["tx_p"], scene["tx_v"], scene["tx_a"], dt)
    RX, VRX = terminal_state(scene["rx_p"], scene["rx_v"], scene["rx_a"], dt)
    poses = body_poses(scene, dt)
    out = {k: np.zeros((R, T)) for k in ("L", "dop", "aod_az", "aod_el", "aoa_az", "aoa_el")}
    out["gain"] = np.zeros((R, T), dtype=np.complex128)
    out["valid"] = np.zeros((R, T), dtype=bool)
    out["degenerate"] = np.zeros((R, T), dtype=bool)
    out["in_bounds"] = np.zeros((R, T), dtype=bool)
    out["bounds_margin"] = np.zeros((R, T))
    if keep_points:
        out["points"] = [None] * R
        out["khat"] = [None] * R
    sigs = {}
    for pos, r in enumerate(rays):
        nint = int(scene["ray_nint"][r])
        sigs.setdefault(tuple(int(x) for x in scene["ray_kind"][r, :nint]), []).append(pos)
    for kinds, positions in sigs.items():
        positions = np.asarray(positions)
        for c0 in range(0, len(positions), chunk):
            pos = positions[c0:c0 + chunk]
            g = _solve_group(scene, rays[pos], kinds, TX, VTX, RX, VRX, poses, f_c)
            for key in out:
                if key in ("points", "khat"):
                    continue
                out[key][pos] = g[key]
            if keep_points:
                for j, p in enumerate(pos):
                    out["points"][p] = [q[j] for q in g["_pts"]]
                    out["khat"][p] = [q[j] for q in g["_khat"]]
    out["tau"] = out["L"] / C0
    ib = out["in_bounds"]
    out["first_out"] = np.where(ib.all(axis=1), T, np.argmin(ib, axis=1)).astype(np.int64)
    return out


def cfr(L, gain, f):
    """H[j, k] = sum_r gain[r, j] exp(-j 2 pi frac(f[k] L[r, j] / c)) as complex128 (T,K)."""
    L = np.asarray(L, dtype=np.float64)
    gain = np.asarray(gain, dtype=np.complex128)
    T = L.shape[1]
    H = np.zeros((T, f.shape[0]), dtype=np.complex128)
    for j in range(T):
        cyc = np.multiply.outer(L[:, j], f) / C0
        frac = cyc - np.floor(cyc)
        H[j] = np.sum(gain[:, j, None] * np.exp(-2j * math.pi * frac), axis=0)
    return H


def run(scene, tgrid, fgrid, t_index=None, rays=None):
    """Extrapolate every ray over the time grid (or the rows t_index) and synthesise H.

    Returns (per-ray outputs dict, H (T', K) complex128)."""
    j = np.arange(tgrid.n_steps) if t_index is None else np.asarray(t_index)
    dt = j * tgrid.dt
    out = extrapolate(scene, dt, fgrid.f_c, rays=rays)
    H = cfr(out["L"], out["gain"], freq_axis(fgrid.f_c, fgrid.bandwidth, fgrid.n_sub))
    return out, H
