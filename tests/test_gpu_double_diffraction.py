"""Two-edge (double diffraction) rays on the GPU through the C ABI against the oracle: every
per-(ray, instant) output, the monitor and H on the parallel-screen scene and on every edge
pair of the moving-box scenes (binary64 and split), the interaction-point kinematics, the
polarimetric coefficients with dipoles, the snapshot tracer's two-edge paths (screens,
moving boxes, street canyon), and the loader's checks."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2205_00237_amd import scenes
from paper_2205_00237_amd.scenes import KIND_D, KIND_R, POL_PERP

pytestmark = pytest.mark.gpu

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_gpu_parity import check_extrapolation, h_errors  # noqa: E402
from test_oracle_double_diffraction import _two_screens  # noqa: E402
from test_oracle_tracer import _wedge_world_scene  # noqa: E402
from test_oracle_bruteforce import _world  # noqa: E402
from test_oracle_polar import _with_dipoles  # noqa: E402
from test_gpu_trace import check_trace  # noqa: E402


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


def _edge_pairs(seed):
    s, _, _ = _wedge_world_scene(_world(seed))
    ne = len(s["edge_a0"])
    pairs = [(i, j) for i in range(ne) for j in range(ne) if i != j]
    s = dict(s)
    n = len(pairs)
    s["ray_nint"] = np.full(n, 2, np.uint8)
    s["ray_kind"] = np.zeros((n, 4), np.uint8)
    s["ray_kind"][:, :2] = KIND_D
    s["ray_prim"] = np.zeros((n, 4), np.int32)
    s["ray_prim"][:, :2] = np.array(pairs)
    s["ray_pol"] = np.zeros((n, 4), np.uint8)
    return s


def _compare(ctx, s, tg, fg, where):
    sid = ctx.load_scene(s)
    ref, Href = oracle.run(s, tg, fg)
    assert ref["valid"].sum() >= 10, where
    for prec in (0, 1):
        out = ctx.extrapolate(sid, tg, fg.f_c, precision=prec)
        check_extrapolation(out, ref, prec, f"{where} prec={prec}", fg.f_c)
        H = ctx.cfr(sid, tg, fg, precision=prec).cpu().numpy().astype(np.complex128)
        e_all, e_mag, e_arg = h_errors(H, Href)
        say(f"  {where} H prec={prec}: {e_all:.3g} {e_mag:.3g} {e_arg:.3g}")
        if prec == 0:
            assert e_all <= 1e-6
        else:
            assert e_all <= 1e-4 and e_mag <= 1e-4 and e_arg <= 1e-3
    ctx.unload_scene(sid)


def test_two_screens(ctx):
    s, _ = _two_screens()
    s = dict(s)
    s["tx_v"] = np.array([0.0, -4.0, 0.5])
    _compare(ctx, s, scenes.TimeGrid(5e-3, 70), scenes.FreqGrid(5.9e9, 240e6, 64), "screens")


@pytest.mark.parametrize("seed", [0, 1])
def test_edge_pairs_on_moving_boxes(ctx, seed):
    s = _edge_pairs(seed)
    _compare(ctx, s, scenes.TimeGrid(7e-3, 65), scenes.FreqGrid(5.9e9, 240e6, 96), f"pairs {seed}")
    _compare(ctx, _with_dipoles(s, (0.2, 0.1, 1.0), (0.9, -0.3, 0.3)), scenes.TimeGrid(7e-3, 40),
             scenes.FreqGrid(5.9e9, 240e6, 64), f"pairs {seed} dipoles")


def test_kinematics(ctx):
    s = _edge_pairs(0)
    sid = ctx.load_scene(s)
    tg = scenes.TimeGrid(5e-3, 40)
    out = ctx.extrapolate(sid, tg, 5.9e9, precision=0, kinematics=True)
    t = np.arange(tg.n_steps) * tg.dt
    ref = oracle.rates(s, t, 5.9e9)
    valid = oracle.extrapolate(s, t, 5.9e9)["valid"]
    assert valid.sum() >= 50
    for k, rel in (("q_pos", 1e-12), ("q_vel", 1e-9), ("q_acc", 1e-7)):
        g = out[k].cpu().numpy()[:, :, :2][valid]
        r = ref[{"q_pos": "Q", "q_vel": "dQ", "q_acc": "ddQ"}[k]][:, :, :2][valid]
        err = np.abs(g - r).max() / (np.abs(r).max() + 1e-30)
        say(f"  {k}: {err:.3g}")
        assert err < rel, k
    ctx.unload_scene(sid)


def test_tracer_two_edges(ctx):
    s, _ = _two_screens()
    check_trace(ctx, s, 0.0, "screens", max_refl=0, max_refl_diff=-1, scattering=False, los=False,
                double_diff=True)
    s, _ = _two_screens(wall=True)
    check_trace(ctx, s, 0.0, "screens + wall", max_refl=0, max_refl_diff=-1, scattering=False, los=False,
                double_diff=True)
    ws, _, _ = _wedge_world_scene(_world(1))
    for t in (0.0, 0.37):
        check_trace(ctx, ws, t, f"world t={t}", max_refl=1, max_refl_diff=1, scattering=False, los=True,
                    double_diff=True)
    cs, _, _ = scenes.street_canyon()
    new, ref, _ = check_trace(ctx, cs, 0.0, "canyon", max_refl=2, max_refl_diff=1, scattering=False, los=True,
                              double_diff=True)
    assert sum(1 for k, *_ in ref if k == (KIND_D, KIND_D)) >= 10
    ctx.unload_scene(new)


def test_loader_checks(ctx):
    from paper_2205_00237_amd._abi import DrtError
    s, (e1, e2) = _two_screens()
    bad = dict(s)
    bad["ray_prim"] = s["ray_prim"].copy()
    bad["ray_prim"][0, 1] = e1            # the same edge twice
    with pytest.raises(DrtError):
        ctx.load_scene(bad)
    bad = dict(s)
    bad["ray_nint"] = np.array([3], np.uint8)
    bad["ray_kind"] = np.array([[KIND_D, KIND_D, KIND_R, 0]], np.uint8)
    bad["ray_prim"] = np.array([[e1, e2, 0, 0]], np.int32)
    bad["ray_pol"] = np.zeros((1, 4), np.uint8)
    with pytest.raises(DrtError):         # two edges with a reflection
        ctx.load_scene(bad)


def test_path_along_a_face(ctx):
    # two edges of one face in turned frames: the grazing angles' sign is rounding's, the
    # coefficient must not be
    from test_oracle_double_diffraction import _roof, _rotation
    rng = np.random.default_rng(11)
    tg = scenes.TimeGrid(2e-3, 16)
    t = np.arange(tg.n_steps) * tg.dt
    for r in range(12):
        R = np.eye(3) if r == 0 else _rotation(rng.normal(size=3), rng.uniform(0, 2 * np.pi))
        s = dict(_roof(R, 1))
        s["rx_v"] = R @ np.array([0.0, 3.0, -1.0])
        ref = oracle.extrapolate(s, t, 5.9e9)
        assert ref["valid"].all()
        sid = ctx.load_scene(s)
        for prec in (0, 1):
            out = ctx.extrapolate(sid, tg, 5.9e9, precision=prec)
            check_extrapolation(out, ref, prec, f"roof {r} prec={prec}", 5.9e9)
        ctx.unload_scene(sid)
