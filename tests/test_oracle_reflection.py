"""Pins of the oracle's reflection chains (Sec. III-A eq. ref_point, Sec. III-A.2, App. B)
against closed forms, Snell's law, Fermat's principle and the paper's local-frame form."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from oracle.geometry import reflection_chain, mirror
from paper_2205_00237_amd.scenes import SceneBuilder, KIND_R, POL_PERP, TimeGrid, FreqGrid

C0 = 299_792_458.0


def _rand_frame(rng):
    return Rotation.random(random_state=rng.integers(1 << 30)).as_matrix()


def test_eq_ref_point_local_frame_equals_global_image_method():
    """Eq. ref_point: in the wall frame (wall y = 0, TX/RX in front) the point is
    x_Q = x_TX + (x_RX - x_TX) y_TX/(y_RX + y_TX) and likewise for z."""
    rng = np.random.default_rng(10)
    for _ in range(200):
        Rw = _rand_frame(rng)           # columns: wall-frame axes in world coordinates
        o = rng.normal(size=3) * 50
        tx_l = np.array([rng.uniform(-50, 50), rng.uniform(0.5, 40), rng.uniform(-20, 20)])
        rx_l = np.array([rng.uniform(-50, 50), rng.uniform(0.5, 40), rng.uniform(-20, 20)])
        den = rx_l[1] + tx_l[1]
        q_l = np.array([tx_l[0] + (rx_l[0] - tx_l[0]) / den * tx_l[1], 0.0,
                        tx_l[2] + (rx_l[2] - tx_l[2]) / den * tx_l[1]])
        to_w = lambda v: o + Rw @ v
        p = to_w(np.array([rng.normal(), 0.0, rng.normal()]))   # any point of the wall
        n = Rw[:, 1]
        pts, _, ok = reflection_chain(to_w(tx_l), to_w(rx_l), [(p, n)])
        assert ok
        assert np.abs(pts[0] - to_w(q_l)).max() < 1e-11


def test_translating_plane_closed_form():
    """Static TX/RX at heights h_T, h_R above a wall moving along its normal at v_n:
    L(t) = sqrt(d^2 + (h_T + h_R - 2 v_n t)^2), f_D = 2 v_n cos(theta_i) f_c / c."""
    hT, hR, d, vn, f_c = 7.0, 3.0, 40.0, 12.0, 28e9
    b = SceneBuilder()
    mat = b.add_material(4.0, 0.01)
    body = b.add_body((0, 0, 0), v0=(0, 0, vn))
    pl = b.add_plane(body, mat, (0, 0, 0), (0, 0, 1))
    b.add_ray((KIND_R,), (pl,), (POL_PERP,))
    s = b.build(tx_p=(0, 0, hT), rx_p=(d, 0, hR))
    t = np.linspace(0, 0.2, 31)
    out = oracle.extrapolate(s, t, f_c)
    Lref = np.sqrt(d ** 2 + (hT + hR - 2 * vn * t) ** 2)
    assert np.abs(out["L"][0] - Lref).max() < 1e-12
    cos_i = (hT + hR - 2 * vn * t) / Lref
    assert np.abs(out["dop"][0] - 2 * vn * cos_i * f_c / C0).max() < 1e-9
    assert out["valid"].all()


def _random_valid_chain(rng, m):
    """TX, RX and m walls arranged as a zig-zag corridor so that the chain is consistent."""
    while True:
        tx = rng.normal(size=3) * 3
        rx = tx + rng.normal(size=3) * 3 + np.array([30.0, 0, 0])
        planes = []
        for i in range(m):
            n = rng.normal(size=3) * 0.3
            n[1] = 1.0 if i % 2 == 0 else -1.0
            n /= np.linalg.norm(n)
            p = np.array([rng.uniform(0, 30), -n[1] * rng.uniform(8, 15), 0.0])
            planes.append((p, n))
        pts, imgs, ok = reflection_chain(tx, rx, planes)
        verts = [tx] + pts + [rx]
        if ok and min(np.linalg.norm(verts[i] - verts[i - 1]) for i in range(1, m + 2)) > 0.5:
            return tx, rx, planes, pts, imgs


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_snell_fermat_and_image_identity(m):
    rng = np.random.default_rng(100 + m)
    for _ in range(50):
        tx, rx, planes, pts, imgs = _random_valid_chain(rng, m)
        verts = [tx] + pts + [rx]
        k = [(verts[i] - verts[i - 1]) / np.linalg.norm(verts[i] - verts[i - 1])
             for i in range(1, m + 2)]
        L = sum(np.linalg.norm(verts[i] - verts[i - 1]) for i in range(1, m + 2))
        # image identity: the unfolded length equals |RX - A_m|
        assert abs(L - np.linalg.norm(rx - imgs[-1])) < 1e-10
        for i, (p, n) in enumerate(planes):
            q = pts[i]
            assert abs(np.dot(q - p, n)) < 1e-10                           # on the wall
            assert np.linalg.norm(np.cross(k[i] - k[i + 1], n)) < 1e-12     # Snell: k_in - k_out || n
            assert abs(abs(np.dot(k[i], n)) - abs(np.dot(k[i + 1], n))) < 1e-12   # equal angles
            # Fermat: L is stationary for tangential moves of Q_i
            t1 = np.cross(n, [1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.cross(n, [0.0, 1.0, 0.0])
            t1 /= np.linalg.norm(t1)
            t2 = np.cross(n, t1)
            for tt in (t1, t2):
                h = 1e-4
                def length(qq):
                    vv = list(verts)
                    vv[i + 1] = qq
                    return sum(np.linalg.norm(vv[j] - vv[j - 1]) for j in range(1, m + 2))
                g = (length(q + h * tt) - length(q - h * tt)) / (2 * h)
                assert abs(g) < 1e-7


def test_appendix_b_reflection_point_velocity():
    """App. B: with a static wall y = 0, v_{Q,x} = sum of dx_Q/d(coord) * v(coord) where
    dx/dx_TX = 1 - y_TX/(y_TX+y_RX), dx/dy_TX = y_RX (x_RX-x_TX)/(y_RX+y_TX)^2,
    dx/dx_RX = y_TX/(y_TX+y_RX), dx/dy_RX = -y_TX (x_RX-x_TX)/(y_RX+y_TX)^2 (the printed
    numerator -y_RX of the last term is a misprint: it follows from differentiating
    eq. ref_point).  Checked against a finite difference of the oracle's point."""
    rng = np.random.default_rng(7)
    for _ in range(30):
        b = SceneBuilder()
        mat = b.add_material(3.0, 0.0)
        pl = b.add_plane(0, mat, (0, 0, 0), (0, 1, 0))
        b.add_ray((KIND_R,), (pl,), (POL_PERP,))
        tx = np.array([rng.uniform(-20, 20), rng.uniform(1, 20), 0.0])
        rx = np.array([rng.uniform(-20, 20), rng.uniform(1, 20), 0.0])
        vt = np.array([rng.normal() * 10, rng.normal() * 10, 0.0])
        vr = np.array([rng.normal() * 10, rng.normal() * 10, 0.0])
        s = b.build(tx_p=tx, rx_p=rx, tx_v=vt, rx_v=vr)
        h = 1e-5
        out = oracle.extrapolate(s, np.array([-h, 0.0, h]), 3e9, keep_points=True)
        Q = out["points"][0][0]
        vfd = (Q[2] - Q[0]) / (2 * h)
        yT, yR, xT, xR = tx[1], rx[1], tx[0], rx[0]
        den = yT + yR
        v_app = ((1 - yT / den) * vt[0] + yR * (xR - xT) / den ** 2 * vt[1]
                 + yT / den * vr[0] - yT * (xR - xT) / den ** 2 * vr[1])
        assert abs(vfd[0] - v_app) < 1e-6 * (1 + abs(v_app))


def test_inconsistent_chain_is_flagged_and_zeroed():
    b = SceneBuilder()
    mat = b.add_material(3.0, 0.0)
    pl = b.add_plane(0, mat, (0, 0, 0), (0, 1, 0))
    b.add_ray((KIND_R,), (pl,), (POL_PERP,))
    s = b.build(tx_p=(0, 5, 0), rx_p=(10, -5, 0))     # opposite sides of the wall
    out = oracle.extrapolate(s, np.array([0.0]), 28e9)
    assert not out["valid"][0, 0]
    assert out["L"][0, 0] == 0 and out["gain"][0, 0] == 0
