"""Pins of the oracle's diffraction points (Sec. III-B eqs. dist2D_TXRX, diff_point, App. C)
and Doppler (App. A eq. doppler_freq) against the paper's closed forms, Keller's law,
Fermat's principle and finite differences."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from oracle.geometry import edge_point
from paper_2205_00237_amd import scenes
from paper_2205_00237_amd.scenes import SceneBuilder, KIND_R, KIND_D, POL_PERP, POL_PAR

C0 = 299_792_458.0


def test_eq_diff_point_in_edge_frame():
    """z_QD = z_RX + d_RX (z_TX - z_RX)/(d_TX + d_RX) with d the 2D distances to the edge."""
    rng = np.random.default_rng(20)
    for _ in range(200):
        Rw = Rotation.random(random_state=rng.integers(1 << 30)).as_matrix()
        o = rng.normal(size=3) * 30
        tx_l = rng.normal(size=3) * 20
        rx_l = rng.normal(size=3) * 20
        dT = math.hypot(tx_l[0], tx_l[1])
        dR = math.hypot(rx_l[0], rx_l[1])
        zq = rx_l[2] + dR * (tx_l[2] - rx_l[2]) / (dT + dR)
        to_w = lambda v: o + Rw @ v
        a = to_w(np.array([0.0, 0.0, rng.normal() * 5]))
        e = Rw[:, 2] * (1 if rng.random() < 0.5 else -1)
        Q, *_ = edge_point(to_w(tx_l), to_w(rx_l), a, e)
        assert np.abs(Q - to_w(np.array([0, 0, zq]))).max() < 1e-11


def _diff_scene(rng, sig, moving=True):
    """A vertical wedge edge of a moving, yawing box plus a ground plane and a side wall,
    with Tx/Rx placed so that chains of the signature `sig` are consistent."""
    b = SceneBuilder()
    gm = b.add_material(5.0, 0.05)
    wm = b.add_material(6.0, 0.0)
    ground = b.add_plane(0, gm, (0, 0, 0), (0, 0, 1))
    wall = b.add_plane(0, wm, (0, 30, 0), (0, -1, 0))
    centre = np.array([0.0, 5.0, 2.0])
    body = b.add_body(centre, v0=(rng.normal() * 5 if moving else 0, 0, 0),
                      a=(rng.normal() if moving else 0, 0, 0), axis=(0, 0, 1),
                      w0=rng.uniform(-0.3, 0.3) if moving else 0.0)
    pec = b.add_material(1, 0, True)
    bx = scenes.add_box(b, body, pec, centre, (4.0, 2.0, 3.0), heading=0.0)
    edge = bx["edges"][3]    # corner at (-2, 4): exposed towards -x, -y
    planes = {"G": ground, "W": wall}
    kinds, prims, pols = [], [], []
    for ch in sig:
        if ch == "D":
            kinds.append(KIND_D)
            prims.append(edge)
            pols.append(POL_PERP if rng.random() < 0.5 else POL_PAR)
        else:
            kinds.append(KIND_R)
            prims.append(planes[ch])
            pols.append(POL_PAR if ch == "G" else POL_PERP)
    b.add_ray(kinds, prims, pols)
    tx = np.array([-25.0 + rng.normal(), -3.0 + rng.normal(), rng.uniform(1.0, 12.0)])
    rx = np.array([-4.0 + rng.normal(), 12.0 + rng.normal(), rng.uniform(0.5, 12.0)])
    return b.build(tx_p=tx, rx_p=rx, tx_v=rng.normal(size=3) * 3, rx_v=rng.normal(size=3) * 3)


@pytest.mark.parametrize("sig", ["D", "GD", "DG", "WD", "GDW", "GWD"])
def test_keller_fermat_unfolded_length(sig):
    rng = np.random.default_rng(sum(map(ord, sig)))
    checked = 0
    for _ in range(100):
        s = _diff_scene(rng, sig)
        dt = np.linspace(0.0, 0.2, 5)
        out = oracle.extrapolate(s, dt, 28e9, keep_points=True)
        if not out["valid"].all():
            continue
        d = sig.index("D")
        e_id = s["ray_prim"][0, d]
        O, R, V, W = oracle.body_poses(s, dt)
        b = s["edge_body"][e_id]
        e = np.einsum("tij,j->ti", R[b], s["edge_e0"][e_id])
        pts = out["points"][0]
        kh = out["khat"][0]
        for j in range(len(dt)):
            assert abs(np.dot(kh[d][j], e[j]) - np.dot(kh[d + 1][j], e[j])) < 1e-12   # Keller cone
            # Fermat along the edge: moving Q_D along e leaves L stationary
            TX = s["tx_p"] + s["tx_v"] * dt[j]
            RX = s["rx_p"] + s["rx_v"] * dt[j]
            verts = [TX] + [p[j] for p in pts] + [RX]
            def length(q):
                vv = list(verts)
                vv[d + 1] = q
                return sum(np.linalg.norm(vv[i] - vv[i - 1]) for i in range(1, len(vv)))
            h = 1e-4
            g = (length(verts[d + 1] + h * e[j]) - length(verts[d + 1] - h * e[j])) / (2 * h)
            assert abs(g) < 1e-7
        checked += 1
    assert checked >= 5


def test_unfolded_length_identity():
    """L = sqrt((rho_A + rho_B)^2 + (z_A - z_B)^2) for the unfolded diffracted ray."""
    rng = np.random.default_rng(3)
    for _ in range(100):
        A, B = rng.normal(size=(2, 3)) * 20
        a = rng.normal(size=3)
        e = rng.normal(size=3)
        e /= np.linalg.norm(e)
        Q, zA, zB, rA, rB = edge_point(A, B, a, e)
        L = np.linalg.norm(A - Q) + np.linalg.norm(B - Q)
        assert abs(L - math.hypot(rA + rB, zA - zB)) < 1e-11


def test_appendix_c_diffraction_point_velocity():
    """App. C: for an edge at rest along z, v_QD,z = v_RX,z + d_RX/(d_RX+d_TX)(v_TX,z - v_RX,z)
    + (z_TX - z_RX) d/dt[d_RX/(d_TX+d_RX)] with d' = ((x - x_Q) v_x + (y - y_Q) v_y)/d."""
    rng = np.random.default_rng(5)
    for _ in range(30):
        b = SceneBuilder()
        e = b.add_edge(0, (0, 0, 0), (0, 0, 1), (1, 0, 0), (0, 1, 0), 1.5)
        b.add_ray((KIND_D,), (e,), (POL_PERP,))
        tx, rx = rng.normal(size=(2, 3)) * 10
        vt, vr = rng.normal(size=(2, 3)) * 10
        s = b.build(tx_p=tx, rx_p=rx, tx_v=vt, rx_v=vr)
        h = 1e-5
        out = oracle.extrapolate(s, np.array([-h, 0.0, h]), 3e9, keep_points=True)
        Q = out["points"][0][0]
        vfd = (Q[2, 2] - Q[0, 2]) / (2 * h)
        dT, dR = math.hypot(tx[0], tx[1]), math.hypot(rx[0], rx[1])
        ddT = (tx[0] * vt[0] + tx[1] * vt[1]) / dT
        ddR = (rx[0] * vr[0] + rx[1] * vr[1]) / dR
        dfrac = (ddR * (dR + dT) - (ddR + ddT) * dR) / (dT + dR) ** 2
        v_app = vr[2] + dR / (dR + dT) * (vt[2] - vr[2]) + (tx[2] - rx[2]) * dfrac
        assert abs(vfd - v_app) < 1e-6 * (1 + abs(v_app))


def _fd4(f, h):
    return (-f[4] + 8 * f[3] - 8 * f[1] + f[0]) / (12 * h)


@pytest.mark.parametrize("which", ["config1", "config2"])
def test_doppler_equals_minus_dL_dt_over_lambda(which):
    if which == "config1":
        s, tg, fg = scenes.config1()
        rays = np.arange(25)
    else:
        s, tg, fg = scenes.config2()
        rays = np.random.default_rng(0).choice(5000, 300, replace=False)
    h = 1e-3
    for t in (0.0, 0.037, 0.09):
        dt = t + h * np.arange(-2, 3)
        out = oracle.extrapolate(s, dt, fg.f_c, rays=rays)
        ok = out["valid"].all(axis=1)
        dLdt = _fd4(out["L"].T, h)
        fd = -(fg.f_c / C0) * dLdt
        err = np.abs(out["dop"][:, 2] - fd)[ok]
        assert ok.sum() > 0.3 * len(rays) if which == "config2" else ok.sum() >= 20
        assert err.max() < 2e-5, err.max()


def test_doppler_product_formula_with_sliding_points():
    """Eq. doppler_freq with the velocities of the (sliding) interaction points, taken by
    finite differences of the solved points, agrees with -(f_c/c) dL/dt to O(v/c)."""
    s, tg, fg = scenes.config2()
    rays = np.random.default_rng(1).choice(5000, 200, replace=False)
    h = 1e-4
    dt = 0.05 + h * np.arange(-2, 3)
    out = oracle.extrapolate(s, dt, fg.f_c, rays=rays, keep_points=True)
    TX, VTX = oracle.terminal_state(s["tx_p"], s["tx_v"], s["tx_a"], dt)
    RX, VRX = oracle.terminal_state(s["rx_p"], s["rx_v"], s["rx_a"], dt)
    n_checked = 0
    for i in range(len(rays)):
        if not out["valid"][i].all():
            continue
        pts = out["points"][i]
        vel = [VTX[2]] + [_fd4(p, h) for p in pts] + [VRX[2]]
        verts = [TX[2]] + [p[2] for p in pts] + [RX[2]]
        ratio = 1.0
        for m in range(1, len(verts)):
            k = (verts[m] - verts[m - 1]) / np.linalg.norm(verts[m] - verts[m - 1])
            ratio *= (C0 - np.dot(vel[m], k)) / (C0 - np.dot(vel[m - 1], k))
        fD_prod = fg.f_c * (ratio - 1.0)
        fD = out["dop"][i, 2]
        assert abs(fD_prod - fD) < 1e-6 * abs(fD) + 1e-3
        n_checked += 1
    assert n_checked > 50


def test_los_doppler_textbook_and_sign():
    """LoS (App. A): f' = f0 (c - v_RX.k)/(c - v_TX.k); approaching terminals give f_D > 0."""
    b = SceneBuilder()
    b.add_ray()
    s = b.build(tx_p=(0, 0, 1.5), rx_p=(100, 0, 1.5), tx_v=(13.9, 0, 0), rx_v=(-10, 0, 0))
    out = oracle.extrapolate(s, np.array([0.0, 1.0]), 3e9)
    k = np.array([1.0, 0, 0])
    f_text = 3e9 * (C0 - np.dot(s["rx_v"], k)) / (C0 - np.dot(s["tx_v"], k)) - 3e9
    assert out["dop"][0, 0] > 0
    assert abs(out["dop"][0, 0] - f_text) < 1e-6 * abs(f_text)
