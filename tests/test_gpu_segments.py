"""Multipath lifetimes on the GPU (Sec. II: trace, extrapolate while no major path
disappears, trace again) through the C ABI against the oracle: identical segment
boundaries and traced paths on the sliding-box scene, the moving-box scenes, the urban
scene and a street canyon, and H over the whole span assembled from the segments' scenes against the oracle's
H of the same segments (binary64: |dH| <= 1e-6 rms; split: the parity bar of the ray sum)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2205_00237_amd import scenes

pytestmark = pytest.mark.gpu

import sys
sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_oracle_segments import _sliding, OPTS  # noqa: E402
from test_oracle_tracer import _wedge_world_scene  # noqa: E402
from test_oracle_bruteforce import _world  # noqa: E402
from test_gpu_trace import gpu_paths  # noqa: E402


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


def h_errors(H, Href):
    rms = np.sqrt(np.mean(np.abs(Href) ** 2))
    m = np.abs(Href) >= 0.1 * rms
    return (np.abs(H - Href).max() / rms,
            (np.abs(np.abs(H[m]) - np.abs(Href[m])) / np.abs(Href[m])).max(),
            np.abs(np.angle(H[m] * np.conj(Href[m]))).max())


def run_case(ctx, s, tg, f_c, opts, thr, max_steps, where, fg=None):
    sid = ctx.load_scene(s)
    segs = ctx.segments(sid, tg, f_c, threshold_db=thr, max_steps=max_steps, **opts)
    ref = oracle.segments(s, tg.dt, tg.n_steps, f_c, opts, thr, max_steps)
    say(f"{where}: {len(segs)} segments {[n for _, n, _ in segs][:8]}")
    assert [(j, n) for j, n, _ in segs] == [(j, n) for j, n, _ in ref], where
    for (_, _, sc), (_, _, paths) in zip(segs, ref):
        assert gpu_paths(ctx, sc) == [(k, p, q) for k, p, q, _ in paths], where
    if fg is not None:
        f = oracle.freq_axis(fg.f_c, fg.bandwidth, fg.n_sub)
        Href = np.zeros((tg.n_steps, fg.n_sub), np.complex128)
        for j0, n, paths in ref:
            if paths:
                sc = oracle.with_rays(oracle.rebase(s, j0 * tg.dt), paths)
                ex = oracle.extrapolate(sc, np.arange(n) * tg.dt, fg.f_c)
                Href[j0:j0 + n] = oracle.cfr(ex["L"], ex["gain"], f)
        for prec in (0, 1):
            H = ctx.cfr_segments(segs, tg, fg, precision=prec).cpu().numpy().astype(np.complex128)
            e_all, e_mag, e_arg = h_errors(H, Href)
            say(f"  H prec={prec}: {e_all:.3g} {e_mag:.3g} {e_arg:.3g}")
            if prec == 0:
                assert e_all <= 1e-6
            else:
                assert e_all <= 1e-4 and e_mag <= 1e-4 and e_arg <= 1e-3
    for _, _, sc in segs:
        ctx.unload_scene(sc)
    ctx.unload_scene(sid)
    return segs


def test_sliding_box(ctx):
    s = _sliding()
    segs = run_case(ctx, s, scenes.TimeGrid(1e-3, 600), 28e9, OPTS, 40.0, 250, "sliding",
                    fg=scenes.FreqGrid(28e9, 100e6, 64))
    t_out = (-10.0 + math.sqrt(109.0)) / 2.0
    assert segs[0][1] == math.floor(t_out / 1e-3) + 1


@pytest.mark.parametrize("seed", [0, 1])
def test_moving_boxes(ctx, seed):
    s, _, _ = _wedge_world_scene(_world(seed))
    opts = dict(max_refl=2, max_refl_diff=1, scattering=False, los=True)
    run_case(ctx, s, scenes.TimeGrid(5e-3, 200), 5.9e9, opts, 30.0, 60, f"world {seed}",
             fg=scenes.FreqGrid(5.9e9, 240e6, 128))


def test_urban(ctx):
    s, tg, fg = scenes.config2()
    opts = dict(max_refl=2, max_refl_diff=1, scattering=False, los=True)
    run_case(ctx, s, tg, fg.f_c, opts, 10.0, 250, "urban", fg=scenes.FreqGrid(fg.f_c, fg.bandwidth, 256))


def test_street_canyon(ctx):
    s, tg, fg = scenes.street_canyon()
    opts = dict(max_refl=2, max_refl_diff=1, scattering=False, los=True)
    run_case(ctx, s, tg, fg.f_c, opts, 20.0, 100, "canyon", fg=fg)


def test_errors(ctx):
    from paper_2205_00237_amd._abi import DrtError, drt_segments
    s = _sliding()
    sid = ctx.load_scene(s)
    tg = scenes.TimeGrid(1e-3, 600)
    with pytest.raises(DrtError):
        drt_segments(ctx.ctx, sid, tg.dt, tg.n_steps, 28e9, OPTS, 40.0, 250, max_segments=2)
    for bad in (dict(threshold_db=-1.0), dict(max_steps=0), dict(min_steps=300, max_steps=250)):
        kw = dict(threshold_db=40.0, max_steps=250, min_steps=1)
        kw.update(bad)
        with pytest.raises(DrtError):
            ctx.segments(sid, tg, 28e9, **kw, **OPTS)
    assert ctx.segments(sid, scenes.TimeGrid(1e-3, 0), 28e9, **OPTS) == []
    ctx.unload_scene(sid)
