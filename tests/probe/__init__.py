"""ctypes loader of the test-only probe library (tests/probe/libdrt_probe.so, built beside
libdrt.so by paper_2205_00237_amd.build): self-tests of the gfx950 builtins that the ray-sum
kernels rely on.  Not part of the product library."""
import ctypes as C
import os

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdrt_probe.so")
EXPORTS = ("drt_probe_mfma_f32_16x16x4", "drt_probe_mfma_f16_16x16x32", "drt_probe_mfma_f64_16x16x4",
           "drt_probe_sincos_rev")


def load():
    if not os.path.exists(PATH):
        raise ImportError(f"{PATH} not found: run paper_2205_00237_amd.build.build() first")
    lib = C.CDLL(PATH)
    vp = C.c_void_p
    for name, args in (("drt_probe_mfma_f32_16x16x4", [vp, vp, vp]),
                       ("drt_probe_mfma_f16_16x16x32", [vp, vp, vp]),
                       ("drt_probe_mfma_f64_16x16x4", [vp, vp, vp]),
                       ("drt_probe_sincos_rev", [vp, C.c_int32, vp, vp])):
        f = getattr(lib, name)
        f.restype = C.c_int
        f.argtypes = args
    return lib


def call(lib, name, *args):
    """Call one probe with integer device pointers / sizes; raise on a nonzero status."""
    conv = [C.c_void_p(int(a)) if i != 1 or name != "drt_probe_sincos_rev" else int(a)
            for i, a in enumerate(args)]
    st = getattr(lib, name)(*conv)
    if st != 0:
        raise RuntimeError(f"{name}: status {st}")
