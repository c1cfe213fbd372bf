"""The gfx950 builtins behind the ray-sum kernels: the lane layouts assumed for
v_mfma_f32_16x16x4_f32 and v_mfma_f32_16x16x32_f16 and the accuracy of v_sin_f32 /
v_cos_f32 on revolutions, through the test-only probe library tests/probe/libdrt_probe.so."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_mfma_16x16x4_lane_layout():
    print("probe: mfma 16x16x4 f32 layout", flush=True)
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import probe
    lib = probe.load()
    rng = np.random.default_rng(0)
    A = rng.integers(-8, 8, (16, 4)).astype(np.float32)    # small integers: exact products
    B = rng.integers(-8, 8, (4, 16)).astype(np.float32)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dD = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    probe.call(lib, "drt_probe_mfma_f32_16x16x4", dA.data_ptr(), dB.data_ptr(), dD.data_ptr())
    assert np.array_equal(dD.cpu().numpy(), A @ B)


def test_mfma_f16_16x16x32_lane_layout():
    print("probe: mfma 16x16x32 f16 layout", flush=True)
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import probe
    lib = probe.load()
    rng = np.random.default_rng(2)
    A = rng.integers(-8, 8, (16, 32)).astype(np.float16)
    B = rng.integers(-8, 8, (32, 16)).astype(np.float16)
    dA = torch.from_numpy(A.view(np.uint16).astype(np.int16)).cuda()
    dB = torch.from_numpy(B.view(np.uint16).astype(np.int16)).cuda()
    dD = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    probe.call(lib, "drt_probe_mfma_f16_16x16x32", dA.data_ptr(), dB.data_ptr(), dD.data_ptr())
    assert np.array_equal(dD.cpu().numpy(), A.astype(np.float32) @ B.astype(np.float32))


def test_mfma_f64_16x16x4_lane_layout():
    print("probe: mfma 16x16x4 f64 layout", flush=True)
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import probe
    lib = probe.load()
    rng = np.random.default_rng(3)
    A = rng.normal(size=(16, 4))
    B = rng.normal(size=(4, 16))
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dD = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    probe.call(lib, "drt_probe_mfma_f64_16x16x4", dA.data_ptr(), dB.data_ptr(), dD.data_ptr())
    assert np.abs(dD.cpu().numpy() - A @ B).max() < 1e-14


def test_hardware_sincos_on_revolutions():
    print("probe: v_sin/v_cos accuracy", flush=True)
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import probe
    lib = probe.load()
    # the ray-sum kernels pass revolutions up to 65 without reducing them first
    x = np.concatenate([np.linspace(0, 1, 200001, dtype=np.float32),
                        np.random.default_rng(1).random(100000).astype(np.float32),
                        np.random.default_rng(2).uniform(-70, 70, 100000).astype(np.float32),
                        np.float32([-256, -65.75, 64.25, 65.0, 255.5, 256])])
    dx = torch.from_numpy(x).cuda()
    ds, dc = torch.empty_like(dx), torch.empty_like(dx)
    probe.call(lib, "drt_probe_sincos_rev", dx.data_ptr(), x.size, ds.data_ptr(), dc.data_ptr())
    xs = x.astype(np.float64)
    es = np.abs(ds.cpu().numpy() - np.sin(2 * np.pi * xs)).max()
    ec = np.abs(dc.cpu().numpy() - np.cos(2 * np.pi * xs)).max()
    print(f"  max abs error: sin {es:.3g}, cos {ec:.3g}", flush=True)
    assert es < 1e-5 and ec < 1e-5
