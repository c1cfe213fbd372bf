"""Interaction-point kinematics on the GPU (eqs. ref_point_velo, ref_point_acc; App. B, C):
positions, velocities and accelerations of every reflection and diffraction point and the
Doppler rate against the oracle's differentiated construction, in every precision mode;
and the O(dt^3) error of second-order Taylor extrapolation of the points against re-solving."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2205_00237_amd import scenes
from test_oracle_rates import _moving_scene
from paper_2205_00237_amd.scenes import KIND_R, KIND_D

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_00237_amd.drt import Context
    c = Context(0)
    yield c
    c.close()


def _check(out, ref, valid, where):
    m = valid[..., None, None]
    for k, kr, rel, ab in (("q_pos", "Q", 1e-12, 1e-9), ("q_vel", "dQ", 1e-9, 1e-9), ("q_acc", "ddQ", 1e-7, 1e-7)):
        g = out[k].cpu().numpy()
        r = np.where(m, ref[kr], 0.0)
        scale = np.abs(r).max()
        err = np.abs(np.where(m, g, 0.0) - r).max()
        assert err <= rel * scale + ab, f"{where}: {k} error {err} (scale {scale})"
    dr = out["dop_rate"].cpu().numpy().astype(np.float64)
    rr = np.where(valid, ref["dop_rate"], 0.0)
    err = np.abs(np.where(valid, dr, 0.0) - rr)
    assert (err <= 2.0 ** -22 * np.abs(rr) + 1e-3).all(), f"{where}: dop_rate {err.max()}"


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_kinematics_moving_bodies(ctx, prec):
    say(f"kinematics: rotating, accelerating bodies, precision {prec}")
    for kinds in ((KIND_R,), (KIND_R, KIND_R), (KIND_D,), (KIND_R, KIND_D), (KIND_D, KIND_R)):
        s = _moving_scene(3, kinds)
        tg = scenes.TimeGrid(2e-3, 130)
        sid = ctx.load_scene(s)
        out = ctx.extrapolate(sid, tg, 28e9, prec, kinematics=True)
        t = np.arange(tg.n_steps) * tg.dt
        ref = oracle.rates(s, t, 28e9)
        valid = oracle.extrapolate(s, t, 28e9)["valid"]
        _check(out, ref, valid, f"{kinds}")
        ctx.unload_scene(sid)


def test_kinematics_urban_and_tiny(ctx):
    say("kinematics: tiny and urban scenes")
    for s, tg, fg, nr in ((*scenes.config1(), None), (*scenes.config2(), 600)):
        T = min(tg.n_steps, 100)
        tg = scenes.TimeGrid(tg.dt, T)
        sid = ctx.load_scene(s)
        out = ctx.extrapolate(sid, tg, fg.f_c, 1, n_rays=nr, kinematics=True)
        rays = None if nr is None else np.arange(nr)
        t = np.arange(T) * tg.dt
        ref = oracle.rates(s, t, fg.f_c, rays=rays)
        valid = oracle.extrapolate(s, t, fg.f_c, rays=rays)["valid"]
        _check(out, ref, valid, "urban" if nr else "tiny")
        ctx.unload_scene(sid)


def test_taylor_extrapolation_error_is_third_order(ctx):
    """From the GPU's points, velocities and accelerations at t0, extrapolate the points to
    later instants by the second-order Taylor formula and compare with the re-solved points."""
    say("kinematics: Taylor error order")
    s = _moving_scene(3, (KIND_R, KIND_D))       # consistent over the window
    tg = scenes.TimeGrid(1e-2, 5)
    sid = ctx.load_scene(s)
    out = ctx.extrapolate(sid, tg, 28e9, 0, kinematics=True)
    assert out["valid"].cpu().numpy().all()
    q, v, a = (out[k].cpu().numpy()[0, :, :2] for k in ("q_pos", "q_vel", "q_acc"))
    d = (np.arange(tg.n_steps) * tg.dt)[:, None, None]
    tay = q[0] + v[0] * d + 0.5 * a[0] * d * d
    err = np.linalg.norm(tay - q, axis=-1).max(axis=-1)
    assert err[0] == 0.0
    assert 6.0 < err[2] / err[1] < 10.0 and 6.0 < err[4] / err[2] < 10.0, err
    ctx.unload_scene(sid)
