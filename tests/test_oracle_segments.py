"""Pins of the oracle's scene carrying and multipath-lifetime segmentation (Sec. II: the
extrapolation holds while no major path disappears, then the trace is run again):

* carrying a scene to t0 + t and extrapolating it by tau reproduces the original scene's
  paths at t + tau (bodies translating, accelerating and rotating about tilted axes);
* a box sliding past its reflection point with constant acceleration: the first lifetime
  ends at the closed-form instant, the next trace no longer finds the reflection, and the
  line of sight then runs in segments of max_steps;
* a threshold that leaves the reflection out of the major rays removes that boundary.
"""
import math

import numpy as np

import oracle
from paper_2205_00237_amd.scenes import SceneBuilder, add_box, KIND_R
from test_oracle_bruteforce import _world
from test_oracle_tracer import _wedge_world_scene


def test_carried_scene_continues_the_motion():
    for seed in (0, 1):
        s, _, _ = _wedge_world_scene(_world(seed))
        paths = oracle.trace(s, 0.0, max_refl=2, max_refl_diff=1, scattering=False)
        s = oracle.with_rays(s, paths)
        tau = np.arange(30) * 7e-3
        for t in (0.2, 0.55):
            a = oracle.extrapolate(s, t + tau, 5.9e9)
            b = oracle.extrapolate(oracle.rebase(s, t), tau, 5.9e9)
            assert np.array_equal(a["valid"], b["valid"])
            v = a["valid"]
            assert np.abs(a["L"] - b["L"])[v].max() < 1e-9
            assert np.abs(a["dop"] - b["dop"])[v].max() < 1e-6
            assert np.abs(a["gain"] - b["gain"])[v].max() < 1e-9 * np.abs(a["gain"]).max()


def _sliding(eps_r=1.0, pec=True):
    # Tx, Rx symmetric about x = 0 at 1.5 m; the -y face of a box (y = 4.1) translating along
    # +x at 10 m/s with 2 m/s^2: the specular point stays at (0, 4.1, 1.5) and leaves the
    # face when its trailing edge x_c(t) - 2.25 passes 0, at t = (-10 + sqrt(109)) / 2
    b = SceneBuilder()
    mat = b.add_material(eps_r, 0.0, pec)
    body = b.add_body((0.0, 5.0, 1.05), v0=(10.0, 0, 0), a=(2.0, 0, 0))
    add_box(b, body, mat, (0.0, 5.0, 1.05), (4.5, 1.8, 1.5))
    return b.build(tx_p=(-5, 0, 1.5), rx_p=(5, 0, 1.5))


OPTS = dict(max_refl=1, max_refl_diff=-1, scattering=False, los=True)


def test_lifetime_ends_when_the_reflection_leaves_its_facet():
    s = _sliding()
    dt = 1e-3
    t_out = (-10.0 + math.sqrt(109.0)) / 2.0
    j1 = math.floor(t_out / dt) + 1
    segs = oracle.segments(s, dt, 600, 28e9, OPTS, threshold_db=40.0, max_steps=250)
    assert [(j, n) for j, n, _ in segs] == [(0, j1), (j1, 250), (j1 + 250, 600 - j1 - 250)]
    kinds = [[k for k, *_ in p] for _, _, p in segs]
    assert kinds[0] == [(), (KIND_R,)] and kinds[1] == [()] and kinds[2] == [()]


def test_weak_reflection_is_not_major():
    # a weakly reflecting face (eps_r 1.05: |Gamma| ~ 0.01 near normal incidence, 40 dB
    # below the line of sight) is ignored with a 20 dB threshold
    s = _sliding(eps_r=1.05, pec=False)
    segs = oracle.segments(s, 1e-3, 600, 28e9, OPTS, threshold_db=20.0, max_steps=250)
    assert [(j, n) for j, n, _ in segs] == [(0, 250), (250, 250), (500, 100)]
    assert [k for k, *_ in segs[0][2]] == [(), (KIND_R,)]
