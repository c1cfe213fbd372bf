"""The paper's validation protocol (Sec. IV-A.1): DRT extrapolation against conventional
ray tracing repeated at every snapshot.  The oracle's extrapolated rays are compared with
an independent snapshot re-tracer (tests/bruteforce) on tiny scenes: every ray that both
consider present must agree in path length within 1e-9 m, and its Doppler must equal the
time derivative of the re-traced length."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2205_00237_amd.scenes import SceneBuilder, KIND_R, KIND_D, KIND_S, POL_PERP
from bruteforce.tracer import World, Body, box_poly, rect_poly, solve

C0 = 299_792_458.0


def _world(seed):
    rng = np.random.default_rng(seed)
    centre = np.array([20.0 + rng.normal(), 6.0 + rng.normal(), 1.2])
    box_body = Body(centre, np.array([-8.0 + rng.normal(), rng.normal(), 0.0]),
                    np.array([rng.normal(), rng.normal() * 0.3, 0.0]), np.array([0.0, 0.0, 1.0]),
                    rng.uniform(-0.4, 0.4), rng.uniform(-0.2, 0.2))
    if seed % 2:   # a tumbling box: rotation about a tilted axis
        ax = np.array([0.3, -0.2, 1.0])
        box_body.axis = ax / np.linalg.norm(ax)
    bodies = [None, box_body]
    polys = [
        rect_poly((-100, -100, 0), (200, 0, 0), (0, 200, 0)),                # ground, normal +z
        rect_poly((60, -40, 0), (0, 80, 0), (0, 0, 20)),                      # wall x = 60, normal... set below
        box_poly(centre, (4.5, 1.8, 1.5), rng.uniform(0, 2 * math.pi), 1),
    ]
    # the wall must face the terminals (-x): order its loop accordingly
    w = polys[1]
    n = np.cross(w.verts[1] - w.verts[0], w.verts[2] - w.verts[0])
    if n[0] > 0:
        w.faces[0].reverse()
    tx = (np.array([0.0, 0.0, 1.5]), np.array([12.0, rng.normal(), 0.0]), np.array([rng.normal(), 0, 0]))
    rx = (np.array([35.0, -3.0, 1.7]), np.array([-9.0, rng.normal(), 0.0]), np.array([0, rng.normal(), 0]))
    return World(bodies, polys, tx, rx)


def _drt_scene(world, seqs):
    """The same scene for the oracle: planes and edges taken from the polyhedra at t0."""
    b = SceneBuilder()
    bb = world.bodies[1]
    b.add_body(bb.O0, bb.v0, bb.a, bb.axis, bb.w0, bb.wdot)
    mat = b.add_material(5.0, 0.01)
    plane_id, edge_id = {}, {}
    for pi, P in enumerate(world.polys):
        body = P.body
        for fi in range(len(P.faces)):
            loop, n = world.face(pi, fi, 0.0)
            plane_id[(pi, fi)] = b.add_plane(body, mat, loop.mean(axis=0), n)
        for ei in range(len(P.edges)):
            a, c = world.edge(pi, ei, 0.0)
            e = (c - a) / np.linalg.norm(c - a)
            # 0-face data are irrelevant for lengths; any perpendicular pair will do
            t0 = np.cross(e, [1.0, 0.0, 0.0]) if abs(e[0]) < 0.9 else np.cross(e, [0.0, 1.0, 0.0])
            t0 /= np.linalg.norm(t0)
            edge_id[(pi, ei)] = b.add_edge(body, a, e, t0, np.cross(e, t0), 1.5)
    for seq in seqs:
        kinds, prims = [], []
        for kind, pi, ii in seq:
            if kind == "R":
                kinds.append(KIND_R)
                prims.append(plane_id[(pi, ii)])
            else:
                kinds.append(KIND_D)
                prims.append(edge_id[(pi, ii)])
        b.add_ray(kinds, prims, [POL_PERP] * len(kinds))
    return b.build(tx_p=world.tx[0], tx_v=world.tx[1], tx_a=world.tx[2],
                   rx_p=world.rx[0], rx_v=world.rx[1], rx_a=world.rx[2])


def _candidates(world):
    faces = [("R", pi, fi) for pi, P in enumerate(world.polys) for fi in range(len(P.faces))]
    edges = [("D", pi, ei) for pi, P in enumerate(world.polys) for ei in range(len(P.edges))]
    seqs = [[f] for f in faces] + [[e] for e in edges]
    seqs += [[f, g] for f, g in itertools.permutations(faces, 2)]
    seqs += [[f, e] for f in faces for e in edges] + [[e, f] for f in faces for e in edges]
    return seqs


@pytest.mark.parametrize("seed", [0, 1])
def test_drt_matches_snapshot_retracing(seed):
    world = _world(seed)
    present = [s for s in _candidates(world) if solve(world, s, 0.0)[2]]
    assert len(present) >= 8
    scene = _drt_scene(world, present)
    dt = np.arange(0, 20) * 1e-2
    out = oracle.extrapolate(scene, dt, 5.9e9)
    compared = 0
    for r, seq in enumerate(present):
        for j, t in enumerate(dt):
            L, _, ok = solve(world, seq, t)
            if ok and out["valid"][r, j]:
                assert abs(out["L"][r, j] - L) < 1e-9, (seq, t, out["L"][r, j] - L)
                compared += 1
    assert compared > 0.5 * len(present) * len(dt)


@pytest.mark.parametrize("seed", [1])
def test_doppler_matches_snapshot_derivative(seed):
    world = _world(seed)
    present = [s for s in _candidates(world) if solve(world, s, 0.0)[2]][:40]
    scene = _drt_scene(world, present)
    h, f_c = 1e-3, 5.9e9
    for t in (0.02, 0.11):
        out = oracle.extrapolate(scene, np.array([t]), f_c)
        for r, seq in enumerate(present):
            Ls = [solve(world, seq, t + m * h) for m in (-2, -1, 1, 2)]
            if not all(x[2] for x in Ls) or not out["valid"][r, 0]:
                continue
            dLdt = (-Ls[3][0] + 8 * Ls[2][0] - 8 * Ls[1][0] + Ls[0][0]) / (12 * h)
            assert abs(out["dop"][r, 0] + f_c / C0 * dLdt) < 1e-5
