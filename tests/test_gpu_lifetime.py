"""The validity monitor on the GPU (multipath lifetime, Sec. II): closed-form instants at
which a wall facet and an edge segment slide off their interaction points, the tiny scene's
front-side classification, and the urban workload at full size against the oracle."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2205_00237_amd import scenes
from paper_2205_00237_amd.scenes import SceneBuilder, add_box, KIND_R, KIND_D, POL_PERP

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


def _sliding_scenes():
    b = SceneBuilder()
    pec = b.add_material(1.0, 0.0, True)
    body = b.add_body((0.0, 5.0, 1.05), v0=(10.0, 0, 0), a=(2.0, 0, 0))
    bx = add_box(b, body, pec, (0.0, 5.0, 1.05), (4.5, 1.8, 1.5))
    b.add_ray((KIND_R,), (bx["faces"]["-y"],), (POL_PERP,))
    facet = b.build(tx_p=(-5, 0, 1.5), rx_p=(5, 0, 1.5))
    b = SceneBuilder()
    pec = b.add_material(1.0, 0.0, True)
    body = b.add_body((0.0, 0.0, 1.05), v0=(0, 0, 2.0))
    bx = add_box(b, body, pec, (0.0, 0.0, 1.05), (4.5, 1.8, 1.5))
    b.add_ray((KIND_D,), (bx["edges"][1],), (POL_PERP,))
    edge = b.build(tx_p=(-10, -3, 1.5), rx_p=(10, -4, 1.5))
    return facet, edge


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_closed_form_lifetimes(ctx, prec):
    say(f"lifetime closed forms, precision {prec}")
    facet, edge = _sliding_scenes()
    t_facet = (-10.0 + math.sqrt(100.0 + 4 * 2.25)) / 2.0
    for s, T, expect in ((facet, 400, math.floor(t_facet / 1e-3) + 1), (edge, 800, 601)):
        sid = ctx.load_scene(s)
        out = ctx.extrapolate(sid, scenes.TimeGrid(1e-3, T), 28e9, prec)
        fo = int(out["first_out"].cpu().numpy()[0])
        ib = out["in_bounds"].cpu().numpy()[0]
        assert fo == expect, (fo, expect)
        assert ib[:fo].all() and not ib[fo:].any()
        ctx.unload_scene(sid)


def test_tiny_scene_monitor(ctx):
    say("lifetime: tiny scene")
    s, tg, fg = scenes.config1()
    sid = ctx.load_scene(s)
    ref = oracle.extrapolate(s, np.arange(tg.n_steps) * tg.dt, fg.f_c)
    for prec in (0, 1):
        out = ctx.extrapolate(sid, tg, fg.f_c, prec)
        fo = out["first_out"].cpu().numpy()
        assert np.array_equal(fo, ref["first_out"])
        assert np.array_equal(out["in_bounds"].cpu().numpy().astype(bool), ref["in_bounds"])
    ctx.unload_scene(sid)


def test_monitor_ragged_and_empty(ctx):
    say("lifetime: ragged / empty")
    s, _, fg = scenes.config1()
    sid = ctx.load_scene(s)
    out = ctx.extrapolate(sid, scenes.TimeGrid(1e-3, 0), fg.f_c, 1)
    assert (out["first_out"].cpu().numpy() == 0).all()       # no instants: first_out = n_steps = 0
    for T in (1, 63, 65, 130):
        out = ctx.extrapolate(sid, scenes.TimeGrid(7e-4, T), fg.f_c, 1, n_rays=11)
        ref = oracle.extrapolate(s, np.arange(T) * 7e-4, fg.f_c, rays=np.arange(11))
        assert np.array_equal(out["first_out"].cpu().numpy(), ref["first_out"]), T
    ctx.unload_scene(sid)
