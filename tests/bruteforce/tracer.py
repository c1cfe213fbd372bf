"""Snapshot re-tracer for tiny polyhedral scenes (test infrastructure).

This is the "conventional RT at every snapshot" side of the paper's own validation
(Sec. IV-A.1, absolute error of DRT against multiple-run RT).  It shares nothing with the
oracle's formulation: at each instant it moves the *vertices* of every polyhedron (the
rotation is built by scipy from a rotation vector), rebuilds face planes and edges from
the moved vertices, and finds each interaction sequence's path by Fermat's principle,
minimising the total length over points constrained to the face planes / edge lines
with a damped Newton iteration on the (convex) length function.  A path exists when
every reflection point lies inside its face polygon with both neighbours in front of the
face and every diffraction point lies on its edge segment.
"""
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation


@dataclass
class Body:
    O0: np.ndarray
    v0: np.ndarray
    a: np.ndarray
    axis: np.ndarray
    w0: float
    wdot: float

    def transform(self, t):
        O = self.O0 + self.v0 * t + 0.5 * self.a * t * t
        th = self.w0 * t + 0.5 * self.wdot * t * t
        Rm = Rotation.from_rotvec(th * self.axis).as_matrix()
        return lambda X: O + (np.asarray(X) - self.O0) @ Rm.T


@dataclass
class Poly:
    """Vertices (n,3) at t0, faces as counter-clockwise vertex loops seen from outside,
    edges as vertex pairs, all carried by `body`."""
    verts: np.ndarray
    faces: list
    edges: list
    body: int


@dataclass
class World:
    bodies: list
    polys: list
    tx: tuple   # (p0, v0, a)
    rx: tuple
    tiles: list = field(default_factory=list)   # (poly, face, 4 corner points at t0)

    def terminal(self, which, t):
        p, v, a = self.tx if which == "tx" else self.rx
        return p + v * t + 0.5 * a * t * t

    def moved_verts(self, pi, t):
        P = self.polys[pi]
        if P.body == 0:
            return P.verts
        return self.bodies[P.body].transform(t)(P.verts)

    def face(self, pi, fi, t):
        V = self.moved_verts(pi, t)
        loop = V[self.polys[pi].faces[fi]]
        n = np.cross(loop[1] - loop[0], loop[2] - loop[0])
        return loop, n / np.linalg.norm(n)

    def edge(self, pi, ei, t):
        V = self.moved_verts(pi, t)
        i, j = self.polys[pi].edges[ei]
        return V[i], V[j]

    def tile_centroid(self, k, t):
        pi, fi, corners = self.tiles[k]
        P = self.polys[pi]
        if P.body == 0:
            return corners.mean(axis=0)
        return self.bodies[P.body].transform(t)(corners).mean(axis=0)


def _in_polygon(q, loop, n):
    for i in range(len(loop)):
        a, b = loop[i], loop[(i + 1) % len(loop)]
        if np.dot(np.cross(b - a, q - a), n) < -1e-12:
            return False
    return True


def solve(world, seq, t, iters=60):
    """Path for the interaction sequence seq = [("R", poly, face) | ("D", poly, edge), ...].

    Returns (L, points, exists)."""
    tx, rx = world.terminal("tx", t), world.terminal("rx", t)
    cons = []   # each: (origin, basis (k,3)) so that Q = origin + basis^T u
    checks = []
    for kind, pi, ii in seq:
        if kind == "R":
            loop, n = world.face(pi, ii, t)
            e1 = loop[1] - loop[0]
            e1 /= np.linalg.norm(e1)
            e2 = np.cross(n, e1)
            cons.append((loop.mean(axis=0), np.stack([e1, e2])))
            checks.append(("R", loop, n))
        else:
            a, b = world.edge(pi, ii, t)
            e = (b - a) / np.linalg.norm(b - a)
            cons.append((0.5 * (a + b), e[None]))
            checks.append(("D", a, b))
    dims = [c[1].shape[0] for c in cons]
    u = np.zeros(sum(dims))

    def points(u):
        out, o = [], 0
        for (c, B), d in zip(cons, dims):
            out.append(c + B.T @ u[o:o + d])
            o += d
        return out

    def length_grad_hess(u):
        V = [tx] + points(u) + [rx]
        Lsum = 0.0
        g = np.zeros_like(u)
        H = np.zeros((u.size, u.size))
        offs = np.concatenate([[0], np.cumsum(dims)])
        for s in range(1, len(V)):
            d = V[s] - V[s - 1]
            ln = max(np.linalg.norm(d), 1e-300)
            Lsum += ln
            k = d / ln
            P = (np.eye(3) - np.outer(k, k)) / ln
            # segment s joins vertex s-1 and s; vertex m (1..n) is constrained point m-1
            ends = []
            if s - 1 >= 1:
                ends.append((s - 2, -1.0))
            if s <= len(seq):
                ends.append((s - 1, 1.0))
            for (m, sg) in ends:
                Bm = cons[m][1]
                g[offs[m]:offs[m + 1]] += sg * (Bm @ k)
                for (m2, sg2) in ends:
                    B2 = cons[m2][1]
                    H[offs[m]:offs[m + 1], offs[m2]:offs[m2 + 1]] += sg * sg2 * (Bm @ P @ B2.T)
        return Lsum, g, H

    L, g, H = length_grad_hess(u)
    for _ in range(iters):
        if not (np.isfinite(H).all() and np.isfinite(g).all()):
            return L, points(u), False      # a segment collapsed: no such path
        step = np.linalg.lstsq(H, -g, rcond=None)[0]
        lam = 1.0
        while lam > 1e-12:
            Ln, gn, Hn = length_grad_hess(u + lam * step)
            if Ln <= L + 1e-15 * abs(L):
                break
            lam *= 0.5
        u = u + lam * step
        L, g, H = Ln, gn, Hn
        if np.abs(g).max() < 1e-14:
            break
    pts = points(u)
    V = [tx] + pts + [rx]
    exists = bool(np.abs(g).max() < 1e-9)
    for m, chk in enumerate(checks):
        q = pts[m]
        if chk[0] == "R":
            _, loop, n = chk
            front_prev = np.dot(V[m] - q, n) > 0
            front_next = np.dot(V[m + 2] - q, n) > 0
            exists &= bool(front_prev and front_next and _in_polygon(q, loop, n))
        else:
            _, a, b = chk
            z = np.dot(q - a, (b - a) / np.linalg.norm(b - a))
            exists &= bool(0.0 <= z <= np.linalg.norm(b - a))
    return L, pts, exists


def box_poly(centre, dims, heading, body):
    """A box as a polyhedron: 8 vertices, 6 outward-oriented faces, 4 vertical edges."""
    c, s = np.cos(heading), np.sin(heading)
    ex, ey, ez = np.array([c, s, 0.0]), np.array([-s, c, 0.0]), np.array([0.0, 0.0, 1.0])
    hx, hy, hz = 0.5 * np.asarray(dims, float)
    V = []
    for sz in (-1, 1):
        for sy in (-1, 1):
            for sx in (-1, 1):
                V.append(centre + sx * hx * ex + sy * hy * ey + sz * hz * ez)
    V = np.array(V)
    idx = lambda sx, sy, sz: ((sz > 0) * 4 + (sy > 0) * 2 + (sx > 0))
    faces = [
        [idx(1, -1, -1), idx(1, 1, -1), idx(1, 1, 1), idx(1, -1, 1)],        # +x
        [idx(-1, 1, -1), idx(-1, -1, -1), idx(-1, -1, 1), idx(-1, 1, 1)],    # -x
        [idx(1, 1, -1), idx(-1, 1, -1), idx(-1, 1, 1), idx(1, 1, 1)],        # +y
        [idx(-1, -1, -1), idx(1, -1, -1), idx(1, -1, 1), idx(-1, -1, 1)],    # -y
        [idx(-1, -1, 1), idx(1, -1, 1), idx(1, 1, 1), idx(-1, 1, 1)],        # +z
        [idx(-1, 1, -1), idx(1, 1, -1), idx(1, -1, -1), idx(-1, -1, -1)],    # -z
    ]
    for f in faces:   # orient every loop so that its normal points out of the box
        n = np.cross(V[f[1]] - V[f[0]], V[f[2]] - V[f[0]])
        if np.dot(n, V[f].mean(axis=0) - centre) < 0:
            f.reverse()
    edges = [(idx(sx, sy, -1), idx(sx, sy, 1)) for sx in (1, -1) for sy in (1, -1)]
    return Poly(V, faces, edges, body)


def rect_poly(corner, u, v, body=0):
    """A single-face rectangle corner, corner+u, corner+u+v, corner+v (normal u x v) with
    its two edges parallel to v."""
    corner, u, v = (np.asarray(x, float) for x in (corner, u, v))
    V = np.array([corner, corner + u, corner + u + v, corner + v])
    return Poly(V, [[0, 1, 2, 3]], [(0, 3), (1, 2)], body)
