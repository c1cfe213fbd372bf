"""The seeded generators produce the workloads' shapes deterministically."""
import numpy as np

from paper_2205_00237_amd import scenes


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in scenes.SCENE_KEYS)


def test_config1_census():
    s, tg, fg = scenes.config1()
    sigs = [scenes.signature(s, r) for r in range(len(s["ray_nint"]))]
    assert sigs.count("") == 1 and sigs.count("R") == 6 and sigs.count("D") == 2 and sigs.count("S") == 16
    assert (tg.n_steps, tg.dt, fg.n_sub, fg.bandwidth, fg.f_c) == (100, 1e-3, 64, 100e6, 28e9)
    assert _same(s, scenes.config1()[0])


def test_config2_census_and_determinism():
    s, tg, fg = scenes.config2()
    assert len(s["ray_nint"]) == 5000
    assert s["plane_p0"].shape[0] == 200 + 120 and s["edge_a0"].shape[0] == 400 + 80
    assert s["body_O0"].shape[0] == 21
    n = s["ray_nint"]
    assert (n == 0).sum() == 1 and (n <= 4).all()
    assert ((s["ray_kind"] == scenes.KIND_D).sum(axis=1) <= 1).all()
    assert (tg.n_steps, fg.n_sub) == (1000, 1024)
    assert _same(s, scenes.config2()[0])
    assert not _same(s, scenes.config2(seed=3)[0])


def test_config3_tiles_face_both_terminals():
    s, tg, fg = scenes.config3(n_boxes=4, tiles_per_box=300)
    assert len(s["ray_nint"]) == 1200 and (s["ray_kind"][:, 0] == scenes.KIND_S).all()
    for i in range(0, 1200, 37):
        c, n = s["tile_c0"][i], s["tile_n0"][i]
        for p in (s["tx_p"], s["rx_p"]):
            assert np.dot((p - c) / np.linalg.norm(p - c), n) > 0.05
    assert set(np.unique(s["tile_alpha"])) <= {1, 2, 3, 4}


def test_config5_request_stream():
    req = scenes.config5_requests(200)
    arr = np.array([r.arrival for r in req])
    assert (np.diff(arr) > 0).all()
    assert all(50 <= r.n_rays <= 20000 and 10 <= r.n_steps <= 1000 for r in req)
    assert {r.n_sub for r in req} <= {64, 256, 1024, 2048}
