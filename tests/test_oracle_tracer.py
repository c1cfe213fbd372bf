"""Pins of the oracle's snapshot tracer (image method with visibility) against things it
does not compute itself:

* the shoebox room: every image of the lattice of mirrored rooms is a valid path, so the
  paths with n reflections are exactly the images with n mirrorings, 4 n^2 + 2 of them, at
  the lattice distances (the classical image-source count);
* obstruction closed forms: a screen across the line of sight, a screen placed on a known
  single-reflection point and then moved clear of it, a terminal inside a box (no diffraction
  through the wedge interior);
* the vertex-based snapshot re-tracer (Fermat minimisation on moved polyhedra, scipy
  rotations): the same sequences exist, at the same lengths, on moving-box scenes at several
  instants (obstruction and wedge tests off, which the re-tracer does not make).
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle.tracer import path_exists, moved_scene, signatures, candidates
from paper_2205_00237_amd.scenes import SceneBuilder, add_box, KIND_R, KIND_D, KIND_S
from bruteforce.tracer import solve, box_poly, rect_poly, World, Body
from test_oracle_bruteforce import _world

ROOM = (7.0, 5.0, 3.0)


def _shoebox(tx, rx):
    b = SceneBuilder()
    mat = b.add_material(4.0, 0.01)
    Lx, Ly, Lz = ROOM
    X, Y, Z = np.eye(3)
    for axis, size, (u, su), (v, sv) in ((X, Lx, (Y, Ly), (Z, Lz)), (Y, Ly, (X, Lx), (Z, Lz)),
                                          (Z, Lz, (X, Lx), (Y, Ly))):
        # the wall at coordinate 0 (normal +axis) and at `size` (normal -axis)
        b.add_plane(0, mat, 0 * axis, axis, facet=(0 * axis, su * u, sv * v))
        b.add_plane(0, mat, size * axis, -axis, facet=(size * axis, su * u, sv * v))
    return b.build(tx_p=tx, rx_p=rx)


def _lattice_lengths(tx, rx, n):
    """Distances from RX to the images of TX with exactly n mirrorings in the shoebox."""
    per_axis = []
    for a in range(3):
        L = ROOM[a]
        opts = []
        for m in range(-n - 1, n + 2):
            opts.append((2 * m * L + tx[a], abs(2 * m)))
            opts.append((2 * m * L - tx[a], abs(2 * m - 1)))
        per_axis.append(opts)
    out = []
    for (x, cx), (y, cy), (z, cz) in itertools.product(*per_axis):
        if cx + cy + cz == n:
            out.append(math.dist((x, y, z), rx))
    return sorted(out)


@pytest.mark.parametrize("seed", [0, 1])
def test_shoebox_image_counts_and_lengths(seed):
    rng = np.random.default_rng(seed)
    tx = rng.uniform(0.3, 0.9, 3) * ROOM
    rx = rng.uniform(0.1, 0.9, 3) * ROOM
    s = _shoebox(tx, rx)
    paths = oracle.trace(s, 0.0, max_refl=3, max_refl_diff=-1, scattering=False, los=True)
    for n in range(0, 4):
        got = sorted(L for k, _, _, L in paths if len(k) == n)
        want = _lattice_lengths(tx, rx, n)
        assert len(got) == (1 if n == 0 else 4 * n * n + 2) == len(want)
        assert np.abs(np.array(got) - np.array(want)).max() < 1e-9


def _screen_scene(screen_centre, tx=(0, 0, 1.5), rx=(20, 0, 1.5)):
    """A ground-free scene: a reflecting wall y = 6 (normal -y, 40 x 10 m) and a 2 x 3 m
    screen in the plane x = x_c (normal -x) centred at screen_centre."""
    b = SceneBuilder()
    mat = b.add_material(5.0, 0.0)
    b.add_plane(0, mat, (10, 6, 0), (0, -1, 0), facet=((-10, 6, -2), (40, 0, 0), (0, 0, 10)))
    c = np.asarray(screen_centre, float)
    b.add_plane(0, mat, c, (-1, 0, 0), facet=(c - (0, 1, 1.5), (0, 2, 0), (0, 0, 3)))
    b.add_edge(0, c + (0, 1, 0), (0, 0, 1), (0, -1, 0), (-1, 0, 0), 2.0, zlim=(-1.5, 1.5))
    return b.build(tx_p=tx, rx_p=rx)


def test_screens_obstruct_closed_form():
    # screen on the line of sight: LoS gone, the wall reflection (point (10, 6, 1.5)) stays
    s = _screen_scene((10, 0, 1.5))
    p = oracle.trace(s, 0.0, max_refl=1, max_refl_diff=-1, scattering=False)
    assert [k for k, *_ in p] == [(KIND_R,)] and p[0][1] == (0,)
    # screen on the reflection point's path (TX -> (10, 6, 1.5) crosses x = 5 at y = 3):
    # the reflection is gone, LoS stays
    s = _screen_scene((5, 3, 1.5))
    p = oracle.trace(s, 0.0, max_refl=1, max_refl_diff=-1, scattering=False)
    assert [k for k, *_ in p] == [()]
    # moved 1.5 m further out (covers y in [3.5, 5.5] at x = 5): both paths exist
    s = _screen_scene((5, 4.5, 1.5))
    p = oracle.trace(s, 0.0, max_refl=1, max_refl_diff=-1, scattering=False)
    assert [k for k, *_ in p] == [(), (KIND_R,)]
    # the screen's edge at (5, 5.5, z) diffracts with the closed-form length
    p = oracle.trace(s, 0.0, max_refl=0, max_refl_diff=0, scattering=False, los=False)
    assert len(p) == 1 and p[0][0] == (KIND_D,)
    assert abs(p[0][3] - (math.hypot(5, 5.5) + math.hypot(15, 5.5))) < 1e-12


def test_no_diffraction_through_a_wedge_interior():
    b = SceneBuilder()
    pec = b.add_material(1.0, 0.0, True)
    bx = add_box(b, 0, pec, (10.0, 0.0, 1.5), (4.0, 4.0, 3.0))
    inside = b.build(tx_p=(10.5, 0.3, 1.5), rx_p=(20.0, 5.0, 1.5))
    outside = b.build(tx_p=(0.0, 0.2, 1.5), rx_p=(20.0, 5.0, 1.5))
    ms_in, ms_out = moved_scene(inside, 0.0), moved_scene(outside, 0.0)
    edges = np.array(bx["edges"])[:, None]
    ok_in, _, _ = path_exists(ms_in, (KIND_D,), edges)
    ok_out, _, _ = path_exists(ms_out, (KIND_D,), edges)
    assert not ok_in.any()
    # box x in [8, 12], y in [-2, 2]: Tx (0, 0.2) -> corner (12, +-2) crosses the box at
    # x = 8 (y = 1.4, -1.27); corner (8, -2) -> Rx (20, 5) crosses it at x = 12 (y = 0.33);
    # only corner (8, 2) is seen by both terminals
    a = moved_scene(outside, 0.0)["a"][bx["edges"]]
    seen = [tuple(float(x) for x in np.round(a[i, :2], 6)) for i in np.nonzero(ok_out)[0]]
    assert seen == [(8.0, 2.0)]


def _wedge_world_scene(world):
    """The re-tracer's polyhedra as tracer primitives: facets, edge segments, and each
    edge's true 0-face (the first face holding both its vertices) and wedge index."""
    b = SceneBuilder()
    for bb in world.bodies[1:]:
        b.add_body(bb.O0, bb.v0, bb.a, bb.axis, bb.w0, bb.wdot)
    mat = b.add_material(5.0, 0.01)
    plane_id, edge_id = {}, {}
    for pi, P in enumerate(world.polys):
        for fi in range(len(P.faces)):
            loop, n = world.face(pi, fi, 0.0)
            plane_id[(pi, fi)] = b.add_plane(P.body, mat, loop.mean(axis=0), n,
                                             facet=(loop[0], loop[1] - loop[0], loop[3] - loop[0]))
        for ei, (i, j) in enumerate(P.edges):
            a, c = world.edge(pi, ei, 0.0)
            ln = np.linalg.norm(c - a)
            e = (c - a) / ln
            f0 = next(f for f in range(len(P.faces)) if i in P.faces[f] and j in P.faces[f])
            loop, n0 = world.face(pi, f0, 0.0)
            t0 = loop.mean(axis=0) - a
            t0 -= np.dot(t0, e) * e
            t0 /= np.linalg.norm(t0)
            nfaces = sum(1 for f in P.faces if i in f and j in f)
            wn = 1.5 if nfaces == 2 else 2.0     # box corner or a free screen edge
            edge_id[(pi, ei)] = b.add_edge(P.body, a, e, t0, n0, wn, zlim=(0.0, ln))
    s = b.build(tx_p=world.tx[0], tx_v=world.tx[1], tx_a=world.tx[2],
                rx_p=world.rx[0], rx_v=world.rx[1], rx_a=world.rx[2])
    return s, plane_id, edge_id


@pytest.mark.parametrize("seed", [0, 1])
def test_existence_matches_snapshot_retracer(seed):
    world = _world(seed)
    s, plane_id, edge_id = _wedge_world_scene(world)
    inv_p = {v: k for k, v in plane_id.items()}
    inv_e = {v: k for k, v in edge_id.items()}
    checked = present = 0
    for t in (0.0, 0.37):
        ms = moved_scene(s, t)
        for kinds in signatures(2, 1, False, False):
            cand = candidates(ms, kinds)
            ok, L, _ = path_exists(ms, kinds, cand, visibility=False)
            for c, o, l in zip(cand, ok, L):
                seq = [("R", *inv_p[int(p)]) if k == KIND_R else ("D", *inv_e[int(p)]) for k, p in zip(kinds, c)]
                Lb, _, exists = solve(world, seq, t)
                if exists and o:
                    assert abs(Lb - l) < 1e-9, (seq, t)
                if exists != bool(o):
                    # the re-tracer's descent can stop short of a stationary path lying
                    # within rounding of a facet boundary: only a near-boundary miss is allowed
                    assert exists is False and abs(Lb - l) > 1e-6, (seq, t, Lb, l)
                checked += 1
                present += bool(o)
    assert checked >= 300 and present >= 15


def test_traced_paths_reproduce_extrapolation_at_t0():
    # the traced rays, loaded as a scene, give the tracer's lengths at t0 through the
    # extrapolation oracle (a different code path for the same points)
    world = _world(1)
    s, _, _ = _wedge_world_scene(world)
    paths = oracle.trace(s, 0.0, max_refl=2, max_refl_diff=1, scattering=False)
    assert len(paths) >= 8
    s2 = dict(s)
    n = len(paths)
    s2["ray_nint"] = np.array([len(k) for k, *_ in paths], np.uint8)
    s2["ray_kind"] = np.zeros((n, 4), np.uint8)
    s2["ray_prim"] = np.zeros((n, 4), np.int32)
    s2["ray_pol"] = np.zeros((n, 4), np.uint8)
    for r, (k, p, q, _) in enumerate(paths):
        s2["ray_kind"][r, :len(k)] = k
        s2["ray_prim"][r, :len(k)] = p
        s2["ray_pol"][r, :len(k)] = q
    ex = oracle.extrapolate(s2, np.array([0.0]), 5.9e9)
    assert ex["valid"][:, 0].all() and ex["in_bounds"][:, 0].all()
    assert np.abs(ex["L"][:, 0] - np.array([L for *_, L in paths])).max() < 1e-9
