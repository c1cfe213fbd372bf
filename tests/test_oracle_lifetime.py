"""Pins of the oracle's validity monitor (multipath lifetime, Sec. II: the extrapolation
holds while no path disappears): closed forms for a wall facet sliding past its reflection
point and an edge segment sliding past its diffraction point, the front-side rule on the
tiny scene, and agreement with the independent snapshot re-tracer's existence test
(polygon, front side, edge segment) on displaced polyhedra."""
import math

import numpy as np
import pytest

import oracle
from paper_2205_00237_amd.scenes import SceneBuilder, add_box, config1, KIND_R, KIND_D, POL_PERP
from bruteforce.tracer import solve
from test_oracle_bruteforce import _world, _candidates


def test_facet_sliding_past_reflection_point():
    # Tx, Rx symmetric about x = 0 at 1.5 m; the -y face of a box (y = 4.1, z in [0.3, 1.8])
    # translates along +x with v = 10 m/s, a = 2 m/s^2: the specular point stays at (0, 4.1,
    # 1.5) and leaves the facet when the trailing edge x_c(t) - 2.25 passes 0.
    b = SceneBuilder()
    pec = b.add_material(1.0, 0.0, True)
    body = b.add_body((0.0, 5.0, 1.05), v0=(10.0, 0, 0), a=(2.0, 0, 0))
    bx = add_box(b, body, pec, (0.0, 5.0, 1.05), (4.5, 1.8, 1.5))
    b.add_ray((KIND_R,), (bx["faces"]["-y"],), (POL_PERP,))
    s = b.build(tx_p=(-5, 0, 1.5), rx_p=(5, 0, 1.5))
    dt = np.arange(400) * 1e-3
    out = oracle.extrapolate(s, dt, 28e9)
    xc = 10.0 * dt + dt * dt
    expect = np.minimum(0.3, 2.25 - xc)
    assert np.abs(out["bounds_margin"][0] - expect).max() < 1e-12
    t_out = (-10.0 + math.sqrt(100.0 + 4 * 2.25)) / 2.0
    assert out["first_out"][0] == math.floor(t_out / 1e-3) + 1
    assert out["valid"][0].all()      # the chain itself stays consistent


def test_edge_segment_sliding_past_diffraction_point():
    # Tx and Rx at 1.5 m: the diffraction point on a vertical edge stays at z = 1.5 while the
    # box rises at 2 m/s, so the segment [z_c - 0.75, z_c + 0.75] leaves it at t = 0.6 s.
    b = SceneBuilder()
    pec = b.add_material(1.0, 0.0, True)
    body = b.add_body((0.0, 0.0, 1.05), v0=(0, 0, 2.0))
    bx = add_box(b, body, pec, (0.0, 0.0, 1.05), (4.5, 1.8, 1.5))
    e = bx["edges"][1]          # (+x, -y) corner
    b.add_ray((KIND_D,), (e,), (POL_PERP,))
    s = b.build(tx_p=(-10, -3, 1.5), rx_p=(10, -4, 1.5))
    dt = np.arange(800) * 1e-3
    out = oracle.extrapolate(s, dt, 28e9)
    expect = np.minimum(1.2 - 2.0 * dt, 0.3 + 2.0 * dt)
    assert np.abs(out["bounds_margin"][0] - expect).max() < 1e-12
    assert out["first_out"][0] == 601


def test_front_side_rule_on_tiny_scene():
    s, tg, fg = config1()
    out = oracle.extrapolate(s, np.arange(tg.n_steps) * tg.dt, fg.f_c)
    fo = out["first_out"]
    # LoS, ground and front-face reflections, the front edges and the front-face tiles hold;
    # the rear, side and top reflections have the terminals behind their wall from t0
    assert fo[0] == fo[1] == fo[2] == tg.n_steps
    assert (fo[3:7] == 0).all()
    assert (fo[7:] == tg.n_steps).all()


def _facet_scene(world, seqs):
    """The re-tracer's polyhedra as oracle primitives with facets and edge segments."""
    b = SceneBuilder()
    bb = world.bodies[1]
    b.add_body(bb.O0, bb.v0, bb.a, bb.axis, bb.w0, bb.wdot)
    mat = b.add_material(5.0, 0.01)
    plane_id, edge_id = {}, {}
    for pi, P in enumerate(world.polys):
        for fi in range(len(P.faces)):
            loop, n = world.face(pi, fi, 0.0)
            assert len(loop) == 4
            plane_id[(pi, fi)] = b.add_plane(P.body, mat, loop.mean(axis=0), n,
                                             facet=(loop[0], loop[1] - loop[0], loop[3] - loop[0]))
        for ei in range(len(P.edges)):
            a, c = world.edge(pi, ei, 0.0)
            ln = np.linalg.norm(c - a)
            e = (c - a) / ln
            t0 = np.cross(e, [1.0, 0.0, 0.0]) if abs(e[0]) < 0.9 else np.cross(e, [0.0, 1.0, 0.0])
            t0 /= np.linalg.norm(t0)
            edge_id[(pi, ei)] = b.add_edge(P.body, a, e, t0, np.cross(e, t0), 1.5, zlim=(0.0, ln))
    for seq in seqs:
        kinds = [KIND_R if k == "R" else KIND_D for k, _, _ in seq]
        prims = [plane_id[(pi, ii)] if k == "R" else edge_id[(pi, ii)] for k, pi, ii in seq]
        b.add_ray(kinds, prims, [POL_PERP] * len(seq))
    return b.build(tx_p=world.tx[0], tx_v=world.tx[1], tx_a=world.tx[2],
                   rx_p=world.rx[0], rx_v=world.rx[1], rx_a=world.rx[2])


@pytest.mark.parametrize("seed", [1])
def test_matches_snapshot_retracer_existence(seed):
    world = _world(seed)
    cand = _candidates(world)
    seqs = [s for s in cand if len(s) == 1] + [s for s in cand if len(s) == 2][::7]
    scene = _facet_scene(world, seqs)
    dt = np.arange(0, 20) * 5e-2
    out = oracle.extrapolate(scene, dt, 5.9e9)
    compared = changed = 0
    for r, seq in enumerate(seqs):
        states = []
        for j, t in enumerate(dt):
            if abs(out["bounds_margin"][r, j]) < 1e-6:
                continue          # on a boundary: either answer is right
            L, _, exists = solve(world, seq, t)
            if out["valid"][r, j] and abs(L - out["L"][r, j]) > 1e-9:
                continue          # the re-tracer's descent stopped short of the stationary path
            assert bool(out["in_bounds"][r, j]) == exists, (seq, t, out["bounds_margin"][r, j])
            states.append(exists)
            compared += 1
        changed += len(set(states)) > 1
    assert compared > 0.85 * len(seqs) * len(dt)
    assert changed >= 1        # some ray appears or disappears within the window
