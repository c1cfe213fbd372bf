"""Serving loop (continuous batching): requests of different sizes submitted together
complete, and each result is bitwise the one the request gives alone."""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2205_00237_amd import scenes

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


def _wait(ctx, tickets, timeout=60.0):
    done = {}
    t_end = time.time() + timeout
    while len(done) < len(tickets):
        assert time.time() < t_end, "serving did not drain"
        for t in tickets:
            if t in done:
                continue
            st = ctx.poll(t)
            if st[0] == 2 or st[0] < 0:
                done[t] = st
        time.sleep(1e-4)
    return done


def test_alone_equals_in_mix(ctx):
    say("serving alone vs mix")
    s1, _, _ = scenes.config2(seed=11)
    s2, _, _ = scenes.config1()
    sid1, sid2 = ctx.load_scene(s1), ctx.load_scene(s2)
    rng = np.random.default_rng(0)
    reqs = []
    for i in range(12):
        sid, R = (sid1, int(rng.integers(50, 5000))) if i % 3 else (sid2, 25)
        T = int(rng.integers(10, 300))
        K = int((64, 256, 1024, 2048)[rng.integers(4)])
        reqs.append((sid, R, scenes.TimeGrid(1e-3, T), scenes.FreqGrid(float((28e9, 60e9)[i % 2]), 400e6, K)))
    alone = []
    for sid, R, tg, fg in reqs:
        alone.append(ctx.cfr(sid, tg, fg, 1, n_rays=R).clone())
    torch.cuda.synchronize()
    outs = [torch.zeros_like(a) for a in alone]
    tickets = [ctx.submit(sid, R, tg, fg, H) for (sid, R, tg, fg), H in zip(reqs, outs)]
    done = _wait(ctx, tickets)
    for t, a, o in zip(tickets, alone, outs):
        st, t_arr, t_adm, t_done = done[t]
        assert st == 2
        assert t_arr <= t_adm <= t_done
        assert torch.equal(a.view(torch.float32), o.view(torch.float32))
    ctx.unload_scene(sid1)
    ctx.unload_scene(sid2)


def test_admission_and_errors(ctx):
    say("serving admission / errors")
    from paper_2205_00237_amd.drt import Context
    from paper_2205_00237_amd._abi import DrtError, DRT_E_ADMISSION, DRT_E_NOTFOUND, DRT_E_BUSY
    s, tg, fg = scenes.config1()
    small = Context(0, hbm_cap_bytes=64 << 20)
    try:
        sid = small.load_scene(s)
        big_tg = scenes.TimeGrid(1e-3, 2_000_000)   # ~1.2 GB of per-(ray, instant) records
        H = torch.empty((1, 1), dtype=torch.complex64, device="cuda")
        with pytest.raises(DrtError) as e:
            small.submit(sid, 25, big_tg, scenes.FreqGrid(28e9, 1e8, 4096), H)
        assert e.value.status == DRT_E_ADMISSION
        with pytest.raises(DrtError) as e:
            small.poll(12345)
        assert e.value.status == DRT_E_NOTFOUND
        H = torch.empty((tg.n_steps, fg.n_sub), dtype=torch.complex64, device="cuda")
        t = small.submit(sid, 25, tg, fg, H)
        # the scene is referenced until the request completes
        try:
            small.unload_scene(sid)
            unloaded = True
        except DrtError as err:
            assert err.status == DRT_E_BUSY
            unloaded = False
        _wait(small, [t])
        if not unloaded:
            small.unload_scene(sid)
    finally:
        small.close()
