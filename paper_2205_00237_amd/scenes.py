"""Seeded synthetic scene and request generators for the dynamic-ray-tracing hot path.

This module only *constructs inputs*: polyhedral geometry at the snapshot time t0, the
rigid-body dynamics of every object and terminal (Sec. II: the dynamic environment
database has a geometric part at t0 and a part with translation velocity, rotation axis,
angular velocity and the corresponding accelerations), and the interaction sequence of
every ray of the t0 multipath.  It holds none of the method's arithmetic: no image
method, no interaction-point solve, no field or channel computation.  Both the GPU path
and the CPU oracle consume the dictionaries built here.

Scene dictionary (all float arrays are float64, vectors are unit where stated):
    t0                                 snapshot time [s]
    tx_p tx_v tx_a rx_p rx_v rx_a      (3,) terminal position / velocity / acceleration at t0
    body_O0 body_v0 body_a body_axis   (nb,3) rotation centre on the axis, translation v and a,
                                       fixed unit rotation axis k; body 0 is the static world
    body_w0 body_wdot                  (nb,) angular speed and acceleration about k [rad/s, rad/s^2]
    mat_eps_r mat_sigma mat_pec        (nm,) relative permittivity, conductivity [S/m], PEC flag
    plane_body plane_mat               (np,) int32
    plane_p0 plane_n0                  (np,3) a point of the plane and its unit normal at t0
    edge_body                          (ne,) int32
    edge_a0 edge_e0                    (ne,3) a point of the edge line and its unit direction
    edge_t0 edge_n0                    (ne,3) unit tangent of the 0-face (in the face, pointing away
                                       from the edge) and the 0-face outward unit normal
    edge_wedge_n                       (ne,) wedge index n (exterior wedge angle = n*pi)
    tile_body tile_alpha tile_model    (nt,) int32 / int32 / uint8 (0 Lambertian, 1 directive)
    tile_c0 tile_n0                    (nt,3) centroid and outward unit normal at t0
    tile_area tile_S tile_phase0       (nt,) area dS [m^2], scattering coefficient S, phase [rad]
    plane_facet (optional)             (np,3,3) the wall's facet at t0: corner, u, v (the
                                       parallelogram corner + s u + w v, 0 <= s, w <= 1);
                                       zero u and v: unbounded wall
    edge_zlim (optional)               (ne,2) the edge segment z_lo <= (X - a0) . e0 <= z_hi;
                                       (-inf, inf): unbounded edge
    ray_nint                           (nr,) uint8, 0..4 interactions (0 = line of sight)
    ray_kind ray_pol ray_prim          (nr,4) uint8 kind (1 R, 2 D, 3 S) / uint8 polarisation
                                       (0 perpendicular = soft, 1 parallel = hard) / int32 primitive
                                       index into planes, edges or tiles; unused slots are 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KIND_R, KIND_D, KIND_S = 1, 2, 3
POL_PERP, POL_PAR = 0, 1
MAX_INT = 4
C0 = 299_792_458.0

SCENE_KEYS = (
    "tx_p", "tx_v", "tx_a", "rx_p", "rx_v", "rx_a",
    "body_O0", "body_v0", "body_a", "body_axis", "body_w0", "body_wdot",
    "mat_eps_r", "mat_sigma", "mat_pec",
    "plane_body", "plane_mat", "plane_p0", "plane_n0",
    "edge_body", "edge_a0", "edge_e0", "edge_t0", "edge_n0", "edge_wedge_n",
    "tile_body", "tile_alpha", "tile_model", "tile_c0", "tile_n0", "tile_area", "tile_S",
    "tile_phase0",
    "ray_nint", "ray_kind", "ray_pol", "ray_prim",
)


@dataclass
class TimeGrid:
    """t_j = t0 + j*dt, j = 0..n_steps-1 (relative to the scene's snapshot time)."""
    dt: float
    n_steps: int


@dataclass
class FreqGrid:
    """f_k = f_c + (k - n_sub//2) * bandwidth / n_sub, k = 0..n_sub-1."""
    f_c: float
    bandwidth: float
    n_sub: int


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


@dataclass
class SceneBuilder:
    """Accumulates primitives and rays, then packs them into the scene dictionary."""
    bodies: list = field(default_factory=list)
    mats: list = field(default_factory=list)
    planes: list = field(default_factory=list)
    edges: list = field(default_factory=list)
    tiles: list = field(default_factory=list)
    rays: list = field(default_factory=list)

    def __post_init__(self):
        self.add_body((0.0, 0.0, 0.0))  # body 0: the static world

    def add_body(self, O0, v0=(0, 0, 0), a=(0, 0, 0), axis=(0, 0, 1), w0=0.0, wdot=0.0):
        self.bodies.append((np.asarray(O0, float), np.asarray(v0, float), np.asarray(a, float),
                            _unit(axis), float(w0), float(wdot)))
        return len(self.bodies) - 1

    def add_material(self, eps_r, sigma, pec=False):
        self.mats.append((float(eps_r), float(sigma), int(bool(pec))))
        return len(self.mats) - 1

    def add_plane(self, body, mat, p0, n0, facet=None):
        """facet: optional (corner, u, v) of the wall's parallelogram at t0."""
        f = np.zeros((3, 3)) if facet is None else np.array([np.asarray(x, float) for x in facet])
        self.planes.append((body, mat, np.asarray(p0, float), _unit(n0), f))
        return len(self.planes) - 1

    def add_edge(self, body, a0, e0, t0, n0, wedge_n, zlim=None):
        """zlim: optional (z_lo, z_hi) of the edge segment along e0 from a0."""
        z = (-np.inf, np.inf) if zlim is None else (float(zlim[0]), float(zlim[1]))
        self.edges.append((body, np.asarray(a0, float), _unit(e0), _unit(t0), _unit(n0),
                           float(wedge_n), z))
        return len(self.edges) - 1

    def add_tile(self, body, c0, n0, area, S, alpha, model, phase0):
        self.tiles.append((body, np.asarray(c0, float), _unit(n0), float(area), float(S),
                           int(alpha), int(model), float(phase0)))
        return len(self.tiles) - 1

    def add_ray(self, kinds=(), prims=(), pols=()):
        assert len(kinds) == len(prims) == len(pols) <= MAX_INT
        self.rays.append((tuple(kinds), tuple(prims), tuple(pols)))
        return len(self.rays) - 1

    def build(self, tx_p, rx_p, tx_v=(0, 0, 0), tx_a=(0, 0, 0), rx_v=(0, 0, 0),
              rx_a=(0, 0, 0), t0=0.0):
        f8 = np.float64
        s = {"t0": float(t0)}
        for k, v in (("tx_p", tx_p), ("tx_v", tx_v), ("tx_a", tx_a),
                     ("rx_p", rx_p), ("rx_v", rx_v), ("rx_a", rx_a)):
            s[k] = np.asarray(v, dtype=f8).reshape(3).copy()
        B = self.bodies
        s["body_O0"] = np.array([b[0] for b in B], f8).reshape(-1, 3)
        s["body_v0"] = np.array([b[1] for b in B], f8).reshape(-1, 3)
        s["body_a"] = np.array([b[2] for b in B], f8).reshape(-1, 3)
        s["body_axis"] = np.array([b[3] for b in B], f8).reshape(-1, 3)
        s["body_w0"] = np.array([b[4] for b in B], f8)
        s["body_wdot"] = np.array([b[5] for b in B], f8)
        M = self.mats or [(1.0, 0.0, 1)]
        s["mat_eps_r"] = np.array([m[0] for m in M], f8)
        s["mat_sigma"] = np.array([m[1] for m in M], f8)
        s["mat_pec"] = np.array([m[2] for m in M], np.uint8)
        P = self.planes
        s["plane_body"] = np.array([p[0] for p in P], np.int32)
        s["plane_mat"] = np.array([p[1] for p in P], np.int32)
        s["plane_p0"] = np.array([p[2] for p in P], f8).reshape(-1, 3)
        s["plane_n0"] = np.array([p[3] for p in P], f8).reshape(-1, 3)
        if any(np.any(p[4] != 0) for p in P):
            s["plane_facet"] = np.array([p[4] for p in P], f8).reshape(-1, 3, 3)
        E = self.edges
        s["edge_body"] = np.array([e[0] for e in E], np.int32)
        s["edge_a0"] = np.array([e[1] for e in E], f8).reshape(-1, 3)
        s["edge_e0"] = np.array([e[2] for e in E], f8).reshape(-1, 3)
        s["edge_t0"] = np.array([e[3] for e in E], f8).reshape(-1, 3)
        s["edge_n0"] = np.array([e[4] for e in E], f8).reshape(-1, 3)
        s["edge_wedge_n"] = np.array([e[5] for e in E], f8)
        if any(np.isfinite(e[6][0]) or np.isfinite(e[6][1]) for e in E):
            s["edge_zlim"] = np.array([e[6] for e in E], f8).reshape(-1, 2)
        T = self.tiles
        s["tile_body"] = np.array([t[0] for t in T], np.int32)
        s["tile_c0"] = np.array([t[1] for t in T], f8).reshape(-1, 3)
        s["tile_n0"] = np.array([t[2] for t in T], f8).reshape(-1, 3)
        s["tile_area"] = np.array([t[3] for t in T], f8)
        s["tile_S"] = np.array([t[4] for t in T], f8)
        s["tile_alpha"] = np.array([t[5] for t in T], np.int32)
        s["tile_model"] = np.array([t[6] for t in T], np.uint8)
        s["tile_phase0"] = np.array([t[7] for t in T], f8)
        nr = len(self.rays)
        s["ray_nint"] = np.zeros(nr, np.uint8)
        s["ray_kind"] = np.zeros((nr, MAX_INT), np.uint8)
        s["ray_pol"] = np.zeros((nr, MAX_INT), np.uint8)
        s["ray_prim"] = np.zeros((nr, MAX_INT), np.int32)
        for i, (k, p, q) in enumerate(self.rays):
            n = len(k)
            s["ray_nint"][i] = n
            s["ray_kind"][i, :n] = k
            s["ray_prim"][i, :n] = p
            s["ray_pol"][i, :n] = q
        return s


# ----------------------------------------------------------------------------------------
# box vehicles


def box_frame(heading):
    """Local axes of a box whose +x axis points along the horizontal heading angle."""
    c, s = math.cos(heading), math.sin(heading)
    return (np.array([c, s, 0.0]), np.array([-s, c, 0.0]), np.array([0.0, 0.0, 1.0]))


def add_box(b: SceneBuilder, body, mat, centre, dims, axes=None, heading=0.0):
    """Six face planes (outward normals, each with its rectangular facet) and four edges
    parallel to the local z axis (segments of the box height).

    Returns {"faces": {name: plane}, "edges": [edge...], "face_geom": {name: (centre,
    normal, u, v, half_u, half_v)}} where u, v span the face.  Each edge's 0-face is the
    adjacent +-x face; the exterior wedge angle of a box corner is 3*pi/2 (n = 1.5)."""
    centre = np.asarray(centre, float)
    ex, ey, ez = axes if axes is not None else box_frame(heading)
    hx, hy, hz = 0.5 * np.asarray(dims, float)
    faces, geom = {}, {}
    for name, n, h, u, hu, v, hv in (
            ("+x", ex, hx, ey, hy, ez, hz), ("-x", -ex, hx, ey, hy, ez, hz),
            ("+y", ey, hy, ex, hx, ez, hz), ("-y", -ey, hy, ex, hx, ez, hz),
            ("+z", ez, hz, ex, hx, ey, hy), ("-z", -ez, hz, ex, hx, ey, hy)):
        c = centre + h * n
        faces[name] = b.add_plane(body, mat, c, n, facet=(c - hu * u - hv * v, 2 * hu * u, 2 * hv * v))
        geom[name] = (c, n, u, v, hu, hv)
    edges = []
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            a0 = centre + sx * hx * ex + sy * hy * ey
            edges.append(b.add_edge(body, a0, ez, -sy * ey, sx * ex, 1.5, zlim=(-hz, hz)))
    return {"faces": faces, "edges": edges, "face_geom": geom}


def _pol_for_normal(n):
    return POL_PAR if abs(float(n[2])) > 0.5 else POL_PERP


# ----------------------------------------------------------------------------------------
# configuration 1: tiny scene (computed in FP64)


def config1(seed=1):
    """Static Tx/Rx 50 m apart at 1.5 m, 28 GHz; one 4.5 x 1.8 x 1.5 m PEC box raised
    0.3 m above a static ground, driving at 15 m/s towards the link and yawing at
    0.2 rad/s about its vertical centre axis.  Rays: LoS, 6 single reflections (ground,
    front, rear, both sides, top), 2 diffractions at the vertical edges of the front face
    and 16 diffuse-scattering tiles (4 x 4 on the front face, directive, alpha = 2,
    S = 0.3).  The only random draw is the tile phases."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    ground_mat = b.add_material(5.0, 0.5, False)
    pec = b.add_material(1.0, 0.0, True)
    ground = b.add_plane(0, ground_mat, (0, 0, 0), (0, 0, 1))
    centre = np.array([70.0, 0.0, 1.05])
    box = b.add_body(centre, v0=(-15.0, 0, 0), axis=(0, 0, 1), w0=0.2)
    bx = add_box(b, box, pec, centre, (4.5, 1.8, 1.5), heading=math.pi)
    F = bx["faces"]
    b.add_ray()  # LoS
    b.add_ray((KIND_R,), (ground,), (POL_PAR,))
    for name in ("+x", "-x", "+y", "-y", "+z"):
        n = bx["face_geom"][name][1]
        b.add_ray((KIND_R,), (F[name],), (_pol_for_normal(n),))
    # the two vertical edges of the front (+x local) face: edges 0 and 1 of add_box
    for e in bx["edges"][:2]:
        b.add_ray((KIND_D,), (e,), (POL_PERP,))
    c, n, u, v, hu, hv = bx["face_geom"]["+x"]
    phases = rng.uniform(0.0, 2 * math.pi, 16)
    k = 0
    for i in range(4):
        for j in range(4):
            tc = c + (-hu + (i + 0.5) * hu / 2) * u + (-hv + (j + 0.5) * hv / 2) * v
            t = b.add_tile(box, tc, n, (2 * hu / 4) * (2 * hv / 4), 0.3, 2, 1, phases[k])
            b.add_ray((KIND_S,), (t,), (POL_PERP,))
            k += 1
    scene = b.build(tx_p=(0, 0, 1.5), rx_p=(50, 0, 1.5))
    return scene, TimeGrid(1e-3, 100), FreqGrid(28e9, 100e6, 64)


# ----------------------------------------------------------------------------------------
# configuration 2: urban vehicular (FP32 with split phase)

CONFIG2_MIX = (("", 1), ("R", 499), ("RR", 1500), ("RRR", 1800), ("D", 200),
               ("RD", 200), ("DR", 200), ("2R+D", 400), ("3R+D", 200))


def _moving_terminal(rng, p):
    psi = rng.uniform(0, 2 * math.pi)
    d = np.array([math.cos(psi), math.sin(psi), 0.0])
    return p, rng.uniform(0, 20) * d, rng.normal(0, 1) * d


def config2(seed=2, scale=1, separation=None, bearing=None, n_facades=200, n_boxes=20,
            f_c=28e9, n_steps=1000, dt=0.5e-3, bandwidth=400e6, n_sub=1024):
    """Urban vehicular scene on [0,500]^2: 200 static vertical facades (x- or y-aligned,
    width U(10,50) m, height U(10,30) m, eps_r U(3,9), sigma 0, both vertical edges
    n = 1.5 wedges, normals facing the Tx-Rx midpoint) and 20 PEC box vehicles (4.5 x
    1.8 x 1.5 m, 0.3 m clearance, heading U[0,2pi), speed U(0,20) m/s and acceleration
    N(0,1) m/s^2 along the heading, yaw rate U(-0.3,0.3) rad/s).  Tx and Rx at 1.5 m,
    separated by U(10,500) m, each moving like a vehicle.  Rays follow the signature mix
    (LoS 1, R 499, RR 1500, RRR 1800, D 200, RD 200, DR 200, 2R+D 400, 3R+D 200) times
    `scale`; reflections pick a facade with probability 0.8 else a box face, diffractions
    a facade edge with probability 0.7 else a box edge.  `separation`/`bearing` pin the
    Tx-Rx geometry (precision sweep)."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    pec = b.add_material(1.0, 0.0, True)
    tx = np.array([rng.uniform(50, 450), rng.uniform(50, 450), 1.5])
    if bearing is None:
        bearing = rng.uniform(0, 2 * math.pi)
    d = separation if separation is not None else rng.uniform(10, 500)
    rx = tx + d * np.array([math.cos(bearing), math.sin(bearing), 0.0])
    mid = 0.5 * (tx + rx)
    tx_p, tx_v, tx_a = _moving_terminal(rng, tx)
    rx_p, rx_v, rx_a = _moving_terminal(rng, rx)

    facade_planes, facade_edges = [], []
    for _ in range(n_facades):
        c = np.array([rng.uniform(0, 500), rng.uniform(0, 500), 0.0])
        w, h = rng.uniform(10, 50), rng.uniform(10, 30)
        c[2] = 0.5 * h
        axis = np.array([1.0, 0.0, 0.0]) if rng.random() < 0.5 else np.array([0.0, 1.0, 0.0])
        n = axis if np.dot(mid - c, axis) >= 0 else -axis
        along = np.array([-n[1], n[0], 0.0])
        mat = b.add_material(rng.uniform(3, 9), 0.0, False)
        up = np.array([0.0, 0.0, 1.0])
        facade_planes.append(b.add_plane(0, mat, c, n, facet=(c - 0.5 * w * along - 0.5 * h * up, w * along, h * up)))
        for sgn in (1.0, -1.0):
            a0 = c + sgn * 0.5 * w * along
            facade_edges.append(b.add_edge(0, a0, (0, 0, 1), -sgn * along, n, 1.5, zlim=(-0.5 * h, 0.5 * h)))

    box_planes, box_edges = [], []
    for _ in range(n_boxes):
        centre = np.array([rng.uniform(0, 500), rng.uniform(0, 500), 0.3 + 0.75])
        psi = rng.uniform(0, 2 * math.pi)
        hd = np.array([math.cos(psi), math.sin(psi), 0.0])
        body = b.add_body(centre, v0=rng.uniform(0, 20) * hd, a=rng.normal(0, 1) * hd,
                          axis=(0, 0, 1), w0=rng.uniform(-0.3, 0.3))
        bx = add_box(b, body, pec, centre, (4.5, 1.8, 1.5), heading=psi)
        for name, pl in bx["faces"].items():
            box_planes.append((pl, _pol_for_normal(bx["face_geom"][name][1])))
        box_edges.extend(bx["edges"])

    def coplanar(p, q):
        # two walls on one plane in succession: the second image undoes the first
        n1, n2 = b.planes[p][3], b.planes[q][3]
        return abs(abs(np.dot(n1, n2)) - 1.0) < 1e-12 and abs(np.dot(b.planes[q][2] - b.planes[p][2], n1)) < 1e-9

    def horizontal(p):
        return abs(b.planes[p][3][2]) > 0.5

    def pick_plane(prev, n_horizontal):
        # at most one horizontal box face per ray: all roofs (floors) share one height and
        # both terminals are 1.5 m high, so two horizontal mirrors cancel in z and leave the
        # last image line parallel to its wall at every instant
        while True:
            if rng.random() < 0.8:
                pl, pol = facade_planes[rng.integers(len(facade_planes))], POL_PERP
            else:
                pl, pol = box_planes[rng.integers(len(box_planes))]
            if n_horizontal and horizontal(pl):
                continue
            if prev < 0 or not coplanar(prev, pl):
                return pl, pol

    def pick_edge():
        if rng.random() < 0.7:
            return facade_edges[rng.integers(len(facade_edges))]
        return box_edges[rng.integers(len(box_edges))]

    def edge_in_plane(e, p):
        # a reflection on a wall that contains the ray's diffracting edge makes two
        # interaction points coincide
        a0, e0 = b.edges[e][1], b.edges[e][2]
        p0, n0 = b.planes[p][2], b.planes[p][3]
        return abs(np.dot(e0, n0)) < 1e-12 and abs(np.dot(a0 - p0, n0)) < 1e-9

    def compatible(kinds, prims):
        # no wall of the ray may contain the ray's diffracting edge
        for i, (ki, pi) in enumerate(zip(kinds, prims)):
            if ki != KIND_D:
                continue
            for kj, pj in zip(kinds, prims):
                if kj == KIND_R and edge_in_plane(pi, pj):
                    return False
        return True

    for sig, count in CONFIG2_MIX:
        for _ in range(count * scale):
            if sig == "":
                b.add_ray()
                continue
            if sig == "2R+D":
                slots = ["R", "R"]
                slots.insert(int(rng.integers(3)), "D")
            elif sig == "3R+D":
                slots = ["R", "R", "R"]
                slots.insert(int(rng.integers(4)), "D")
            else:
                slots = list(sig)
            while True:
                kinds, prims, pols, prev, nh = [], [], [], -1, 0
                for k in slots:
                    if k == "R":
                        pl, pol = pick_plane(prev, nh)
                        nh += horizontal(pl)
                        kinds.append(KIND_R)
                        prims.append(pl)
                        pols.append(pol)
                        prev = pl
                    else:
                        kinds.append(KIND_D)
                        prims.append(pick_edge())
                        pols.append(POL_PERP)
                        prev = -1
                if compatible(kinds, prims):
                    break
            b.add_ray(kinds, prims, pols)
    scene = b.build(tx_p=tx_p, tx_v=tx_v, tx_a=tx_a, rx_p=rx_p, rx_v=rx_v, rx_a=rx_a)
    return scene, TimeGrid(dt, n_steps), FreqGrid(f_c, bandwidth, n_sub)


# ----------------------------------------------------------------------------------------
# configuration 3: scattering-heavy, 60 GHz


def _random_axis(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def config3(seed=3, n_boxes=50, tiles_per_box=4000, n_steps=500, dt=1e-3,
            f_c=60e9, bandwidth=2e9, n_sub=256):
    """50 moving and rotating boxes (sides U(0.5,5) m, centres in [0,100]^2 x [0.5,3] m at
    least 2 m from the terminals, speed U(0,20) m/s and acceleration N(0,1) m/s^2 along a
    horizontal heading; half rotate about z, half about a random unit axis, omega
    U(-1,1) rad/s).  Tx static at (0,0,10); Rx from (60,40,1.5) moving at (10,0,0) m/s.
    4000 diffuse-scattering tiles per box, area-weighted over the faces, kept where both
    terminals lie more than 0.05 in cosine above the face at t0; dS U(0.5,1.5) cm^2,
    alpha U{1..4}, S U(0.1,0.5), Lambertian or directive with probability 1/2, phase
    U[0,2pi)."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    pec = b.add_material(1.0, 0.0, True)
    tx = np.array([0.0, 0.0, 10.0])
    rx = np.array([60.0, 40.0, 1.5])
    rx_v = np.array([10.0, 0.0, 0.0])
    for ib in range(n_boxes):
        while True:
            dims = rng.uniform(0.5, 5.0, 3)
            centre = np.array([rng.uniform(0, 100), rng.uniform(0, 100), rng.uniform(0.5, 3)])
            if min(np.linalg.norm(centre - tx), np.linalg.norm(centre - rx)) < 2.0 + 0.5 * np.linalg.norm(dims):
                continue
            psi = rng.uniform(0, 2 * math.pi)
            axes = box_frame(psi)
            # faces eligible for tiles: both terminals in front of the face plane
            cand = []
            for sgn, ax, h, (u, hu), (v, hv) in (
                    (1, 0, dims[0], (1, dims[1]), (2, dims[2])),
                    (-1, 0, dims[0], (1, dims[1]), (2, dims[2])),
                    (1, 1, dims[1], (0, dims[0]), (2, dims[2])),
                    (-1, 1, dims[1], (0, dims[0]), (2, dims[2])),
                    (1, 2, dims[2], (0, dims[0]), (1, dims[1])),
                    (-1, 2, dims[2], (0, dims[0]), (1, dims[1]))):
                n = sgn * axes[ax]
                fc = centre + 0.5 * h * n
                cand.append((fc, n, axes[u], 0.5 * hu, axes[v], 0.5 * hv))
            if any(np.dot(_unit(tx - c[0]), c[1]) > 0.05 and np.dot(_unit(rx - c[0]), c[1]) > 0.05
                   for c in cand):
                break
        psi_v = rng.uniform(0, 2 * math.pi)
        hd = np.array([math.cos(psi_v), math.sin(psi_v), 0.0])
        axis = (0, 0, 1) if ib < n_boxes // 2 else _random_axis(rng)
        body = b.add_body(centre, v0=rng.uniform(0, 20) * hd, a=rng.normal(0, 1) * hd,
                          axis=axis, w0=rng.uniform(-1, 1))
        areas = np.array([4 * c[3] * c[5] for c in cand])
        made = 0
        while made < tiles_per_box:
            m = 4 * (tiles_per_box - made) + 16
            fi = rng.choice(len(cand), size=m, p=areas / areas.sum())
            su = rng.uniform(-1, 1, m)
            sv = rng.uniform(-1, 1, m)
            for q in range(m):
                fc, n, u, hu, v, hv = cand[fi[q]]
                p = fc + su[q] * hu * u + sv[q] * hv * v
                if np.dot(_unit(tx - p), n) <= 0.05 or np.dot(_unit(rx - p), n) <= 0.05:
                    continue
                t = b.add_tile(body, p, n, rng.uniform(0.5e-4, 1.5e-4), rng.uniform(0.1, 0.5),
                               int(rng.integers(1, 5)), int(rng.random() < 0.5),
                               rng.uniform(0, 2 * math.pi))
                b.add_ray((KIND_S,), (t,), (POL_PERP,))
                made += 1
                if made == tiles_per_box:
                    break
    scene = b.build(tx_p=tx, rx_p=rx, rx_v=rx_v)
    return scene, TimeGrid(dt, n_steps), FreqGrid(f_c, bandwidth, n_sub)


# ----------------------------------------------------------------------------------------
# configuration 4: precision sweep on configuration 2's generator

SWEEP_DISTANCES = (10.0, 30.0, 100.0, 300.0, 500.0)
SWEEP_CARRIERS = (6e9, 28e9, 60e9, 140e9)


def config4(distance, f_c, seed=4, **kw):
    """Configuration 2's scene, seed 4, with Rx at `distance` along a fixed bearing."""
    return config2(seed=seed, separation=distance, bearing=0.6, f_c=f_c, **kw)


# ----------------------------------------------------------------------------------------
# configuration 5: serving mix


@dataclass
class Request:
    arrival: float        # scheduled arrival time [s] from the start of the stream
    scene: int
    n_rays: int
    n_steps: int
    dt: float
    f_c: float
    bandwidth: float
    n_sub: int


def street_canyon(seed=6, n_segments=8, n_vehicles=6, f_c=5.9e9, n_steps=400, dt=2.5e-3):
    """A street between two rows of building facades (dense multi-bounce traffic for the
    snapshot tracer): an unbounded ground (eps_r 5, sigma 0.05), facade segments 20 m long
    along x with 2 m alleys at y = +-10 m (heights U(8, 20) m, normals into the street,
    eps_r U(3, 7)), each with its two vertical building-corner edges (n = 1.5, 0-face the
    facade), and box vehicles (4.5 x 1.8 x 1.5 m, PEC) in the lanes y = +-2.5 m driving
    along x at U(5, 15) m/s.  Tx and Rx at 1.5 m in the street, Tx moving at 10 m/s.  The
    scene has no rays: trace it."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    ground_mat = b.add_material(5.0, 0.05, False)
    b.add_plane(0, ground_mat, (0, 0, 0), (0, 0, 1))
    for side in (1.0, -1.0):
        n = np.array([0.0, -side, 0.0])
        for i in range(n_segments):
            x0, h = 22.0 * i, rng.uniform(8.0, 20.0)
            mat = b.add_material(rng.uniform(3.0, 7.0), 0.0, False)
            c = np.array([x0 + 10.0, side * 10.0, 0.5 * h])
            b.add_plane(0, mat, c, n, facet=((x0, side * 10.0, 0.0), (20.0, 0.0, 0.0), (0.0, 0.0, h)))
            for xe, t in ((x0, (1.0, 0.0, 0.0)), (x0 + 20.0, (-1.0, 0.0, 0.0))):
                b.add_edge(0, (xe, side * 10.0, 0.5 * h), (0, 0, 1), t, n, 1.5, zlim=(-0.5 * h, 0.5 * h))
    pec = b.add_material(1.0, 0.0, True)
    for _ in range(n_vehicles):
        lane = 2.5 if rng.random() < 0.5 else -2.5
        centre = np.array([rng.uniform(10.0, 22.0 * n_segments - 10.0), lane, 1.05])
        speed = rng.uniform(5.0, 15.0) * (1.0 if lane < 0 else -1.0)
        body = b.add_body(centre, v0=(speed, 0, 0))
        add_box(b, body, pec, centre, (4.5, 1.8, 1.5))
    L = 22.0 * n_segments
    tx = (rng.uniform(0.2, 0.4) * L, -4.5, 1.5)
    rx = (rng.uniform(0.6, 0.8) * L, 4.5, 1.5)
    scene = b.build(tx_p=tx, rx_p=rx, tx_v=(10.0, 0, 0))
    return scene, TimeGrid(dt, n_steps), FreqGrid(f_c, 240e6, 256)


def config5_scenes(n_scenes=64, scale=4):
    """64 resident urban scenes of 20 000 rays (configuration 2's mix times 4)."""
    return [config2(seed=5000 + i, scale=scale)[0] for i in range(n_scenes)]


def config5_requests(n_requests=4096, n_scenes=64, rate=2000.0, seed=5, max_rays=20000):
    """Poisson arrivals at `rate`/s; per request: scene U{0..63}, ray count log-uniform
    50..20000, horizon U{10..1000} steps of 1 ms, subcarriers U{64,256,1024,2048},
    carrier U{28,60} GHz, 400 MHz bandwidth."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    out = []
    for i in range(n_requests):
        n = int(math.floor(math.exp(rng.uniform(math.log(50), math.log(max_rays)))))
        out.append(Request(float(arrivals[i]), int(rng.integers(n_scenes)), max(1, min(n, max_rays)),
                           int(rng.integers(10, 1001)), 1e-3,
                           float((28e9, 60e9)[rng.integers(2)]), 400e6,
                           int((64, 256, 1024, 2048)[rng.integers(4)])))
    return out


def subset_rays(scene, idx):
    """A scene restricted to the rays `idx` (same primitives and dynamics)."""
    s = dict(scene)
    for k in ("ray_nint", "ray_kind", "ray_pol", "ray_prim"):
        s[k] = np.ascontiguousarray(scene[k][idx])
    return s


def signature(scene, r):
    """Interaction signature of ray r as a string over {R, D, S} ('' for LoS)."""
    n = int(scene["ray_nint"][r])
    return "".join("?RDS"[int(k)] for k in scene["ray_kind"][r, :n])
