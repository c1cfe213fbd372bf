"""Pins of the oracle's power-Doppler and power-delay profiles (Sec. IV-A, IV-B) against
closed forms that share nothing with its chain solver: the two-ray model over a perfectly
conducting ground (direct path and ground image, free-space power (lambda / 4 pi d)^2, Doppler
-(f_c/c) dd/dt from the hand-differentiated distances), the sign change of the direct ray's
Doppler when two vehicles pass (Sec. IV-A), out-of-range samples kept in the per-bin total,
and the validity monitor removing a reflection once its point leaves a bounded ground."""
import math

import numpy as np

import oracle
from oracle.profiles import edge_distance
from paper_2205_00237_amd.scenes import SceneBuilder, KIND_R, POL_PAR

C = 299_792_458.0
F_C = 5.9e9
LAM = C / F_C


def _two_ray(v_tx, v_rx, facet=None):
    b = SceneBuilder()
    pec = b.add_material(1.0, 0.0, True)
    g = b.add_plane(0, pec, (0, 0, 0), (0, 0, 1), facet=facet)
    b.add_ray()                                   # line of sight
    b.add_ray((KIND_R,), (g,), (POL_PAR,))        # ground reflection
    return b.build(tx_p=(-50.0, 0.0, 1.5), rx_p=(49.95, 3.5, 1.5), tx_v=v_tx, rx_v=v_rx)


def _closed_form(t, vx_tx, vx_rx):
    """Per ray (direct, ground image): distance, power and Doppler at the instants t."""
    dx = 99.95 + (vx_rx - vx_tx) * t            # x_RX - x_TX
    dvx = vx_rx - vx_tx
    out = []
    for dz in (0.0, 3.0):                         # Rx minus Tx height, or minus the image's
        d = np.sqrt(dx * dx + 3.5 ** 2 + dz * dz)
        dd = dx * dvx / d
        out.append((d, (LAM / (4.0 * math.pi * d)) ** 2, -(F_C / C) * dd))
    return out


def _bins(**kw):
    b = dict(steps_per_bin=20, n_dop=64, dop_lo=-458.88, dop_step=14.34,
             n_delay=96, delay_lo=0.0, delay_step=1.0 / 240e6, in_bounds_only=0)
    b.update(kw)
    return b


def _expected(t, rays, bins):
    n_tb = (len(t) - 1) // bins["steps_per_bin"] + 1
    pdfp, pdp, tot = np.zeros((n_tb, bins["n_dop"])), np.zeros((n_tb, bins["n_delay"])), np.zeros(n_tb)
    for d, p, fd in rays:
        for j in range(len(t)):
            b = j // bins["steps_per_bin"]
            tot[b] += p[j]
            kd = math.floor((fd[j] - bins["dop_lo"]) / bins["dop_step"])
            kt = math.floor((d[j] / C - bins["delay_lo"]) / bins["delay_step"])
            if 0 <= kd < bins["n_dop"]:
                pdfp[b, kd] += p[j]
            if 0 <= kt < bins["n_delay"]:
                pdp[b, kt] += p[j]
    return pdfp, pdp, tot


def _clear_of_edges(rays, bins):
    for d, _, fd in rays:
        assert edge_distance(fd, bins["dop_lo"], bins["dop_step"]).min() > 1e-6
        assert edge_distance(d / C, bins["delay_lo"], bins["delay_step"]).min() > 1e-15


def test_two_ray_passing_vehicles_match_closed_form():
    # Tx and Rx drive towards each other at 10 m/s in lanes 3.5 m apart and pass at
    # t = 4.9975 s, between two instants; 10 ms instants, 200 ms x 14.34 Hz bins as in
    # Sec. IV-A, 1/240 MHz delay bins
    s = _two_ray((10.0, 0, 0), (-10.0, 0, 0))
    j = np.arange(1000)
    t = j * 1e-2
    bins = _bins()
    rays = _closed_form(t, 10.0, -10.0)
    _clear_of_edges(rays, bins)
    pdfp, pdp, tot = _expected(t, rays, bins)
    o = oracle.power_profiles(s, j, 1e-2, F_C, bins)
    scale = tot.max()
    assert np.abs(o["total"] - tot).max() < 1e-12 * scale
    assert np.abs(o["pdfp"] - pdfp).max() < 1e-12 * scale
    assert np.abs(o["pdp"] - pdp).max() < 1e-12 * scale
    # the direct ray's Doppler is positive while approaching and negative after passing
    k0 = int(round(-bins["dop_lo"] / bins["dop_step"]))      # first bin at or above 0 Hz
    assert np.all(o["pdfp"][:25, :k0] == 0.0) and np.all(o["pdfp"][25:, k0:] == 0.0)
    # highest |f_D| = f_c v_rel / c at the start: 20 m/s closing, nearly head-on
    fmax = F_C * 20.0 / C
    assert abs(np.abs(o["dop"]).max() - fmax * 99.95 / math.hypot(99.95, 3.5)) < 1e-9


def test_out_of_range_samples_stay_in_total():
    s = _two_ray((10.0, 0, 0), (-10.0, 0, 0))
    j = np.arange(0, 1000, 7)
    t = j * 1e-2
    bins = _bins(steps_per_bin=50, n_dop=10, dop_lo=-71.7, n_delay=20, delay_lo=150e-9)
    rays = _closed_form(t, 10.0, -10.0)
    _clear_of_edges(rays, bins)
    # the instants are a subset of the grid: time bins follow the grid index j
    n_tb = j.max() // 50 + 1
    pdfp, pdp, tot = np.zeros((n_tb, 10)), np.zeros((n_tb, 20)), np.zeros(n_tb)
    for d, p, fd in rays:
        for c, jj in enumerate(j):
            b = jj // 50
            tot[b] += p[c]
            kd = math.floor((fd[c] + 71.7) / 14.34)
            kt = math.floor((d[c] / C - 150e-9) * 240e6)
            if 0 <= kd < 10:
                pdfp[b, kd] += p[c]
            if 0 <= kt < 20:
                pdp[b, kt] += p[c]
    o = oracle.power_profiles(s, j, 1e-2, F_C, bins)
    scale = tot.max()
    assert np.abs(o["total"] - tot).max() < 1e-12 * scale
    assert np.abs(o["pdfp"] - pdfp).max() < 1e-12 * scale
    assert np.abs(o["pdp"] - pdp).max() < 1e-12 * scale
    assert o["pdfp"].sum() < 0.9 * o["total"].sum() and o["pdp"].sum() < 0.9 * o["total"].sum()


def test_bounded_ground_drops_reflection_after_it_leaves():
    # Rx parked, Tx at 20 m/s: equal heights put the ground point at x = (x_TX + x_RX) / 2 =
    # 10 t - 0.025, which leaves the facet x in [-20, 20] after t = 2.0025 s
    s = _two_ray((20.0, 0, 0), (0.0, 0, 0), facet=((-20, -5, 0), (40, 0, 0), (0, 15, 0)))
    j = np.arange(400)
    t = j * 1e-2
    bins = _bins(steps_per_bin=10, in_bounds_only=1)
    direct, ground = _closed_form(t, 20.0, 0.0)
    _clear_of_edges((direct, ground), bins)
    inside = 10.0 * t - 0.025 <= 20.0
    ground = (ground[0], np.where(inside, ground[1], 0.0), ground[2])
    pdfp, pdp, tot = _expected(t, (direct, ground), bins)
    o = oracle.power_profiles(s, j, 1e-2, F_C, bins)
    scale = tot.max()
    assert np.abs(o["total"] - tot).max() < 1e-12 * scale
    assert np.abs(o["pdfp"] - pdfp).max() < 1e-12 * scale
    assert np.abs(o["pdp"] - pdp).max() < 1e-12 * scale
    # without the gate the reflection keeps its power over the whole span
    o2 = oracle.power_profiles(s, j, 1e-2, F_C, _bins(steps_per_bin=10))
    assert o2["total"][-1] > o["total"][-1] * 1.5
