"""Pins of the oracle's two-edge (double diffraction) chains, the multiple-diffraction
extension of Sec. III-B:

* points: closed form over two parallel vertical edges with both terminals at one height
  (the path stays in that horizontal plane); agreement with the Fermat snapshot re-tracer
  (an independent minimisation on the moved polyhedra) on moving, rotating boxes; Keller's
  law at both edges;
* coefficient: continuity of the total field where either edge's shadow boundary switches
  a singly diffracted ray off (the doubly diffracted ray must cancel the jump, which fixes
  both distance parameters and the spreading); the UTD product written out in the test from
  the single-edge coefficient of em.py with the angles and distances computed here, for
  the parallel-edge geometry in which the successive-edge caustic distances are exact;
* kinematics: velocities and accelerations of both points against finite differences of the
  re-solved points; Doppler against -(f_c/c) dL/dt;
* tracing: the path over two screen edges exists with its closed-form length and is
  removed by a wall across it.
"""
import math

import numpy as np

import oracle
from oracle.em import utd_coefficient
from paper_2205_00237_amd.scenes import SceneBuilder, KIND_D, POL_PERP
from bruteforce.tracer import solve
from test_oracle_bruteforce import _world
from test_oracle_tracer import _wedge_world_scene

C0 = 299_792_458.0
F_C = 5.9e9
LAM = C0 / F_C


def _two_screens(wall=False):
    # screens x = 10 (edge at y = 2) and x = 20 (edge at y = -1.5), vertical edges, both
    # half-planes (n = 2) extending away from the path's side
    b = SceneBuilder()
    mat = b.add_material(5.0, 0.0)
    b.add_plane(0, mat, (10, 5, 1.5), (-1, 0, 0), facet=((10, 2, -5), (0, 20, 0), (0, 0, 15)))
    e1 = b.add_edge(0, (10, 2, 0), (0, 0, 1), (0, 1, 0), (-1, 0, 0), 2.0, zlim=(-5, 10))
    b.add_plane(0, mat, (20, -5, 1.5), (-1, 0, 0), facet=((20, -21.5, -5), (0, 20, 0), (0, 0, 15)))
    e2 = b.add_edge(0, (20, -1.5, 0), (0, 0, 1), (0, -1, 0), (-1, 0, 0), 2.0, zlim=(-5, 10))
    if wall:
        b.add_plane(0, mat, (15, 0, 0), (-1, 0, 0), facet=((15, -10, -5), (0, 20, 0), (0, 0, 15)))
    b.add_ray((KIND_D, KIND_D), (e1, e2), (POL_PERP, POL_PERP))
    return b.build(tx_p=(0, 6, 1.5), rx_p=(30, -6, 1.5)), (e1, e2)


def test_parallel_edges_closed_form():
    s, _ = _two_screens()
    ex = oracle.extrapolate(s, np.array([0.0]), F_C, keep_points=True)
    q1, q2 = ex["points"][0][0][0], ex["points"][0][1][0]
    assert np.allclose(q1, (10, 2, 1.5), atol=1e-12) and np.allclose(q2, (20, -1.5, 1.5), atol=1e-12)
    s0, s1, s2 = math.hypot(10, 4), math.hypot(10, 3.5), math.hypot(10, 4.5)
    assert abs(ex["L"][0, 0] - (s0 + s1 + s2)) < 1e-12
    # coefficient: UTD product, soft, normal incidence (sin b0 = 1), angles from the 0-faces
    k = 2 * math.pi / LAM
    # angle = atan2(d . n, d . t) for the direction d from the edge point to a neighbour;
    # edge 1: t = +y, n = -x; edge 2: t = -y, n = -x
    phi_p1 = math.atan2(10.0, 4.0) % (2 * math.pi)          # towards Tx (-10, +4)
    phi1 = math.atan2(-10.0, -3.5) % (2 * math.pi)          # towards edge 2 (+10, -3.5)
    phi_p2 = math.atan2(10.0, -3.5) % (2 * math.pi)         # towards edge 1 (-10, +3.5)
    phi2 = math.atan2(-10.0, 4.5) % (2 * math.pi)           # towards Rx (+10, -4.5)
    D1 = utd_coefficient(np.array(phi1), np.array(phi_p1), np.array(1.0), 2.0, k, np.array(s0 * s1 / (s0 + s1)), 0)
    D2 = utd_coefficient(np.array(phi2), np.array(phi_p2), np.array(1.0), 2.0, k,
                         np.array(s1 * s2 / (s1 + s2)), 0)
    want = LAM / (4 * math.pi) * D1 * D2 / math.sqrt(s0 * s1 * s2 * (s0 + s1 + s2))
    assert abs(ex["gain"][0, 0] - want) < 1e-12 * abs(want)


def _two_edge_fields(tx, rx, pol):
    """Screens x = 10 (edge at y = 2, face towards +y) and x = 20 (edge at y = -8, face
    towards -y), both vertical half-planes: fields a exp(-j k L) of the rays over edge 1,
    over edge 2 and over both."""
    b = SceneBuilder()
    e1 = b.add_edge(0, (10, 2, 0), (0, 0, 1), (0, 1, 0), (-1, 0, 0), 2.0)
    e2 = b.add_edge(0, (20, -8, 0), (0, 0, 1), (0, -1, 0), (-1, 0, 0), 2.0)
    b.add_ray((KIND_D,), (e1,), (pol,))
    b.add_ray((KIND_D,), (e2,), (pol,))
    b.add_ray((KIND_D, KIND_D), (e1, e2), (pol, pol))
    ex = oracle.extrapolate(b.build(tx_p=tx, rx_p=rx), np.array([0.0]), F_C)
    assert ex["valid"].all()
    return ex["gain"][:, 0] * np.exp(-2j * math.pi * F_C / C0 * ex["L"][:, 0])


def test_double_diffraction_continuous_at_both_shadow_boundaries():
    """Edge 2's shadow boundary for the field of edge 1 (RX on the line from Q1 through Q2:
    in plan view x = 30, y = -18) switches the ray over edge 1 alone off; edge 1's shadow
    boundary for the source (TX on the line from Q2 through Q1: x = 0, y = 12) switches the
    ray over edge 2 alone off.  In both cases the ray over both edges must cancel the jump:
    the residual, after removing the linear variation, is set by the other edge's own
    transition (a few 1e-3 of the jump here), while a distance parameter of the second edge
    taken as from a point source at the unfolded distance s0 + s1 leaves about 13%."""
    for pol in (0, 1):
        for tz, rz in ((1.5, 1.5), (9.0, -4.0)):
            cases = (
                # (moving terminal, position at parameter m, index of the ray that switches off,
                #  sign of m on its lit side)
                (lambda m: ((0, 6, tz), (30, -18 + m, rz)), 0, +1),
                (lambda m: ((0, 12 + m, tz), (30, -30, rz)), 1, -1),
            )
            for place, off, lit in cases:
                d = 1e-6
                U, single = [], None
                for m in (-3, -1, 1, 3):
                    tx, rx = place(m * d)
                    E = _two_edge_fields(tx, rx, pol)
                    on = (m > 0) == (lit > 0)
                    U.append(E[2] + (E[off] if on else 0))
                    if on and abs(m) == 1:
                        single = E[off]
                jump = (U[2] - U[1]) - 0.5 * ((U[3] - U[2]) + (U[1] - U[0]))
                assert abs(jump) < 5e-3 * abs(single), (pol, tz, off, abs(jump) / abs(single))


def test_points_match_the_fermat_retracer_and_keller():
    world = _world(1)
    s, plane_id, edge_id = _wedge_world_scene(world)
    inv_e = {v: k for k, v in edge_id.items()}
    ne = len(s["edge_a0"])
    b_rays = [(i, j) for i in range(ne) for j in range(ne) if i != j]
    s2 = dict(s)
    n = len(b_rays)
    s2["ray_nint"] = np.full(n, 2, np.uint8)
    s2["ray_kind"] = np.zeros((n, 4), np.uint8)
    s2["ray_kind"][:, :2] = KIND_D
    s2["ray_prim"] = np.zeros((n, 4), np.int32)
    s2["ray_prim"][:, :2] = np.array(b_rays)
    s2["ray_pol"] = np.zeros((n, 4), np.uint8)
    dt = np.array([0.0, 0.21, 0.47])
    ex = oracle.extrapolate(s2, dt, F_C, keep_points=True)
    compared = 0
    for r, (i, j) in enumerate(b_rays):
        for c, t in enumerate(dt):
            if not ex["valid"][r, c]:
                continue
            L, pts, _ = solve(world, [("D", *inv_e[i]), ("D", *inv_e[j])], t)
            if abs(L - ex["L"][r, c]) > 1e-6:
                continue       # the re-tracer's descent stopped short (near a singular start)
            assert abs(L - ex["L"][r, c]) < 1e-9
            for m in range(2):
                assert np.linalg.norm(pts[m] - ex["points"][r][m][c]) < 1e-6
            compared += 1
            # Keller's law: equal angles with the edge on both sides of each point
            q = [ex["points"][r][m][c] for m in range(2)]
            tx = s["tx_p"] + s["tx_v"] * t + 0.5 * s["tx_a"] * t * t
            rx = s["rx_p"] + s["rx_v"] * t + 0.5 * s["rx_a"] * t * t
            verts = [tx, q[0], q[1], rx]
            for m, ed in enumerate((i, j)):
                e = oracle.rotate(s["edge_e0"][ed], oracle.body_poses(s, np.array([t]))[1][s["edge_body"][ed], 0])
                ku = (verts[m + 1] - verts[m]) / np.linalg.norm(verts[m + 1] - verts[m])
                kv = (verts[m + 2] - verts[m + 1]) / np.linalg.norm(verts[m + 2] - verts[m + 1])
                assert abs(np.dot(ku, e) - np.dot(kv, e)) < 1e-9
    assert compared >= 20


def test_kinematics_against_finite_differences():
    world = _world(0)
    s, _, edge_id = _wedge_world_scene(world)
    ne = len(s["edge_a0"])
    pairs = [(i, j) for i in range(ne) for j in range(ne) if i != j]
    s2 = dict(s)
    n = len(pairs)
    s2["ray_nint"] = np.full(n, 2, np.uint8)
    s2["ray_kind"] = np.zeros((n, 4), np.uint8)
    s2["ray_kind"][:, :2] = KIND_D
    s2["ray_prim"] = np.zeros((n, 4), np.int32)
    s2["ray_prim"][:, :2] = np.array(pairs)
    s2["ray_pol"] = np.zeros((n, 4), np.uint8)
    t, h = 0.13, 1e-3
    rts = oracle.rates(s2, np.array([t]), F_C)
    ts = t + h * np.arange(-2, 3)
    ex = oracle.extrapolate(s2, ts, F_C, keep_points=True)
    checked = 0
    for r in range(n):
        if not ex["valid"][r].all():
            continue
        for m in range(2):
            P = ex["points"][r][m]
            v = (P[0] - 8 * P[1] + 8 * P[3] - P[4]) / (12 * h)
            a = (-P[0] + 16 * P[1] - 30 * P[2] + 16 * P[3] - P[4]) / (12 * h * h)
            assert np.linalg.norm(rts["dQ"][r, 0, m] - v) < 1e-6 * (1 + np.linalg.norm(v))
            assert np.linalg.norm(rts["ddQ"][r, 0, m] - a) < 1e-3 * (1 + np.linalg.norm(a))
        L = ex["L"][r]
        dL = (L[0] - 8 * L[1] + 8 * L[3] - L[4]) / (12 * h)
        assert abs(ex["dop"][r, 2] + F_C / C0 * dL) < 1e-5
        checked += 1
    assert checked >= 10


def test_tracer_finds_and_blocks_the_path():
    s, (e1, e2) = _two_screens()
    p = oracle.trace(s, 0.0, max_refl=0, max_refl_diff=-1, scattering=False, los=False, double_diff=True)
    assert [(k, q) for k, q, _, _ in p] == [((KIND_D, KIND_D), (e1, e2))]
    assert abs(p[0][3] - (math.hypot(10, 4) + math.hypot(10, 3.5) + math.hypot(10, 4.5))) < 1e-12
    s, _ = _two_screens(wall=True)
    p = oracle.trace(s, 0.0, max_refl=0, max_refl_diff=-1, scattering=False, los=False, double_diff=True)
    assert p == []


def _roof(R, pol):
    # two edges of one face (the roof z = 10 of a block between x = 0 and x = 2, edges along
    # y, right-angle wedges n = 1.5 with the roof as 0-face); the whole scene turned by R
    b = SceneBuilder()
    e1 = b.add_edge(0, R @ (0.0, 0, 10), R @ (0.0, 1, 0), R @ (1.0, 0, 0), R @ (0.0, 0, 1), 1.5, zlim=(-5, 5))
    e2 = b.add_edge(0, R @ (2.0, 0, 10), R @ (0.0, 1, 0), R @ (-1.0, 0, 0), R @ (0.0, 0, 1), 1.5, zlim=(-5, 5))
    b.add_ray((KIND_D, KIND_D), (e1, e2), (pol, pol))
    return b.build(tx_p=R @ (-5.0, 0, 5), rx_p=R @ (8.0, 0, 6))


def _rotation(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def test_path_along_a_face_reads_grazing_angles():
    # The segment between the edges runs along their common face: the exit angle at the
    # first edge and the incidence angle at the second are 0 (grazing), whatever sign the
    # rounding of a turned frame gives them.  Pinned to the UTD product at those angles
    # (frame invariance: every turned copy gives the same coefficient).
    k = 2 * math.pi / LAM
    s0, s1, s2 = math.hypot(5, 5), 2.0, math.hypot(6, 4)
    angles = [(0.0, 1.25 * math.pi), (math.atan2(-4.0, -6.0) % (2 * math.pi), 0.0)]   # (phi, phi') per edge
    Ls = [s0 * s1 / (s0 + s1), s1 * s2 / (s1 + s2)]
    rng = np.random.default_rng(11)
    want = []
    for pol in (0, 1):
        w = LAM / (4 * math.pi) / math.sqrt(s0 * s1 * s2 * (s0 + s1 + s2))
        for (phi, phi_p), Lj in zip(angles, Ls):
            w = w * utd_coefficient(np.array(phi), np.array(phi_p), np.array(1.0), 1.5, k, np.array(Lj), pol)
        want.append(complex(w))
    assert want[0] == 0 and abs(want[1]) > 0          # soft vanishes along the face
    for pol in (0, 1):
        for r in range(24):
            R = np.eye(3) if r == 0 else _rotation(rng.normal(size=3), rng.uniform(0, 2 * math.pi))
            ex = oracle.extrapolate(_roof(R, pol), np.array([0.0]), F_C)
            assert ex["valid"][0, 0]
            assert abs(ex["L"][0, 0] - (s0 + s1 + s2)) < 1e-12
            assert abs(ex["gain"][0, 0] - want[pol]) <= 1e-9 * abs(want[1]), (pol, r)
