"""Build libdrt.so in-tree for gfx950 with hipcc (no JIT cache, no pip install)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdrt.so")
SOURCES = ("kernels_geom.hip", "kernels_geom_more.hip", "kernels_cfr.hip", "kernels_batch.hip", "plan.hip",
           "runtime.hip", "trace.hip", "nufft.hip")
# test-only hardware probes (MFMA lane layouts, v_sin/v_cos): their own library under tests/
PROBE_SRC = os.path.join(os.path.dirname(HERE), "tests", "probe", "probe.hip")
PROBE_OUT = os.path.join(os.path.dirname(PROBE_SRC), "libdrt_probe.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(os.path.dirname(HERE), "include"),
]


def build(verbose=True, jobs=2):
    """Compile every HIP source to an object in parallel, then link libdrt.so; the test-only
    probe library is compiled alongside."""
    objs, procs = [], []
    probe_tmp = PROBE_OUT + ".tmp"
    probe_cmd = [HIPCC] + FLAGS + [PROBE_SRC, "-o", probe_tmp]
    procs.append((probe_cmd, subprocess.Popen(probe_cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for src in SOURCES:
        obj = os.path.join(SRC, src.replace(".hip", ".o"))
        cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + ["-c", os.path.join(SRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    for cmd, p in procs:
        out, _ = p.communicate()
        text = "\n".join(l for l in out.decode(errors="replace").splitlines()
                         if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed: {' '.join(cmd)}\n{text}")
        if verbose and text.strip():
            print(text, file=sys.stderr)
    os.replace(probe_tmp, PROBE_OUT)
    tmp = OUT + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread", "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(link)}\n{r.stdout}{r.stderr}")
    os.replace(tmp, OUT)
    for o in objs:
        os.remove(o)
    return OUT


if __name__ == "__main__":
    print(build())
