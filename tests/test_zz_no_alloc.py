"""drt_cfr_noalloc (static per-GPU scratch, no device allocation) against drt_cfr: bitwise
equal H through the C ABI, on two calls in a row (the second smaller, so that stale scratch
contents from the first would show), in both precisions, and a call that needs more scratch
than the static array holds is refused."""
import pytest

torch = pytest.importorskip("torch")

from paper_2205_00237_amd import scenes

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _both(ctx, sid, R, tg, fg, prec):
    from paper_2205_00237_amd import _abi
    dt = torch.complex128 if prec == 0 else torch.complex64
    ref = torch.empty((tg.n_steps, fg.n_sub), dtype=dt, device="cuda")
    got = torch.empty_like(ref)
    got.view(torch.float32).fill_(7.0)
    st = torch.cuda.current_stream().cuda_stream
    _abi.drt_cfr(ctx.ctx, sid, R, tg.dt, tg.n_steps, fg.f_c, fg.bandwidth, fg.n_sub, prec, ref.data_ptr(), st)
    _abi.drt_cfr_noalloc(ctx.ctx, sid, R, tg.dt, tg.n_steps, fg.f_c, fg.bandwidth, fg.n_sub, prec,
                         got.data_ptr(), st)
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_equals_cfr_twice_then_smaller():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_00237_amd.drt import Context
    s2, tg2, fg2 = scenes.config2()
    s1, tg1, fg1 = scenes.config1()
    with Context(0) as ctx:
        sid2, sid1 = ctx.load_scene(s2), ctx.load_scene(s1)
        cases = [
            (sid2, 5000, tg2, fg2, 1),                                             # the urban step, 201 MB
            (sid2, 1234, scenes.TimeGrid(5e-4, 333), scenes.FreqGrid(28e9, 400e6, 256), 1),   # smaller
            (sid2, 3000, scenes.TimeGrid(5e-4, 200), fg2, 0),                      # binary64
            (sid1, 25, tg1, fg1, 0),                                               # tiny, binary64
            (sid1, 7, scenes.TimeGrid(1e-3, 37), scenes.FreqGrid(28e9, 1e8, 50), 1),   # ragged
            (sid1, 0, tg1, fg1, 1),                                                # no rays: zeros
        ]
        for sid, R, tg, fg, prec in cases:
            say(f"noalloc vs cfr: R={R} T={tg.n_steps} K={fg.n_sub} prec={prec}")
            ref, got = _both(ctx, sid, R, tg, fg, prec)
            assert torch.equal(ref.view(torch.int32), got.view(torch.int32)), (R, tg.n_steps, fg.n_sub, prec)
        ctx.unload_scene(sid2)
        ctx.unload_scene(sid1)


def test_noalloc_refuses_oversize():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_00237_amd import _abi
    from paper_2205_00237_amd.drt import Context
    s2, tg2, fg2 = scenes.config2()
    with Context(0) as ctx:
        sid = ctx.load_scene(s2)
        H = torch.empty((2000, 1024), dtype=torch.complex64, device="cuda")
        say("noalloc: oversize request refused")
        with pytest.raises(_abi.DrtError) as e:
            _abi.drt_cfr_noalloc(ctx.ctx, sid, 5000, tg2.dt, 2000, fg2.f_c, fg2.bandwidth, 1024, 1,
                                 H.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert e.value.status == _abi.DRT_E_NOMEM
        assert "static scratch" in str(e.value)
        ctx.unload_scene(sid)
