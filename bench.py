#!/usr/bin/env python3
"""Throughput of the DRT hot path on one MI355X.

A step is one drt_cfr call over the urban vehicular workload (5000 rays up to three
reflections plus one diffraction among 20 moving boxes and 200 facades, 1000 instants of
0.5 ms, 1024 subcarriers over 400 MHz at 28 GHz): body poses, per-(ray, instant)
extrapolation and field coefficients, and the ray sum H(t, f), in split precision (binary64
geometry and phase reduction, binary32 field coefficients, ray sum as complex GEMMs on the
binary16 matrix cores with hi/lo operand splits, three products per tile, accumulated in
binary32).  The metric is ray x time x frequency samples of H per second, with inputs
resident in device memory.  Beside it: the accuracy of the timed step against the binary64
oracle on sampled instants, the binary64 GPU paths on the same workload, the kernel-level
roofline of the dominant kernel (timed with HIP events on its own stream), the scattering
workload at full size and the tiny workload's latency, the CPU oracle on a bounded sample
(one core and all cores), the serving mix (4096 Poisson requests over 64 resident scenes,
200 GB admission cap) with p50 / p99 latency, and the other calls on the urban scene:
drt_extrapolate with the validity monitor, the interaction-point kinematics, the
power-Doppler and power-delay profiles, the snapshot trace and the multipath-lifetime
refresh, and H by the non-uniform FFT.  Prints one JSON line.
"""
import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12      # MI355X published dense vector fp32 [flop/s]
PEAK_FP64_VECTOR = 78.6e12
PEAK_FP16_MFMA = 2.5e15          # dense binary16 matrix cores
PEAK_HBM = 8e12                  # HBM3E [B/s]
PEAK_FP32_MFMA = 157.3e12        # dense binary32 matrix cores
FLOP_PER_SAMPLE = 8              # one complex rotation (6) + one complex accumulate (2)
KERNEL_SOURCE = os.path.join(ROOT, "paper_2205_00237_amd", "csrc", "dev_cfr.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_cfr_urban_5000x1000x1024.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def kernel_source_hash():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE counter
    summary, or None when there is none or the kernel source changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        src = kernel_source_hash()
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("source_sha256_16") != src:
        return None
    return rec.get("hbm_bytes_per_launch")


def _oracle_rows(job):
    import oracle
    scene, tg, fg, idx = job
    oracle.run(scene, tg, fg, t_index=idx)
    return len(idx)


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(), "model": model}


def cpu_baseline(scene, tg, fg, budget_s=15.0, max_workers=16):
    """The oracle (numpy float64, unchanged) on whole time rows of the same workload: first
    on one core, then on every core of the host's share (a fork pool of one process per core,
    each taking its own rows).  Must run before the GPU is initialised (fork)."""
    import multiprocessing as mp
    import numpy as np
    import oracle
    R, K = len(scene["ray_nint"]), fg.n_sub
    oracle.run(scene, tg, fg, t_index=np.array([0]))       # warm the imports and caches
    rows1 = 6
    idx = np.linspace(0, tg.n_steps - 1, rows1).astype(int)
    t = time.perf_counter()
    oracle.run(scene, tg, fg, t_index=idx)
    one = (time.perf_counter() - t) / rows1
    single = R * K / one
    info = cpu_info()
    workers = max(1, min(max_workers, info["nproc"]))
    per = max(1, min(tg.n_steps // workers, int(budget_s / one)))
    rows = np.linspace(0, tg.n_steps - 1, per * workers).astype(int)
    jobs = [(scene, tg, fg, rows[w::workers]) for w in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_oracle_rows, [(scene, tg, fg, rows[:1])] * workers)   # start every worker
        t = time.perf_counter()
        done = sum(pool.map(_oracle_rows, jobs, chunksize=1))
        el = time.perf_counter() - t
    return {"value": R * done * K / el, "unit": "samples/s", "cores": workers, "kind": "oracle",
            "sample": f"{done} of {tg.n_steps} instants, all {R} rays and {K} subcarriers, spread over "
                      f"{workers} processes ({el:.1f} s wall, numpy float64); one core alone: "
                      f"{rows1} instants",
            "single_core_value": single, "host": info}


def oracle_sample(scene, tg, fg, rows):
    """Oracle per-(ray, instant) outputs and H on the instants `rows`, for the accuracy of the
    timed step."""
    import numpy as np
    import oracle
    out, H = oracle.run(scene, tg, fg, t_index=np.asarray(rows))
    return {"L": out["L"], "dop": out["dop"], "valid": out["valid"], "H": H}


def accuracy(ref, rows, H, ext):
    """Errors of the timed split step against the binary64 oracle on the sampled instants:
    per (ray, instant) where both sides find the chain consistent, and on H (|H| and arg H
    where |H_ref| >= 0.1 rms, |dH| / rms everywhere)."""
    import numpy as np
    C0 = 299792458.0
    Hg = H[rows].cpu().numpy().astype(np.complex128)
    Hr = ref["H"]
    L = ext["L"][:, rows].cpu().numpy()
    dop = ext["dop"][:, rows].cpu().numpy().astype(np.float64)
    v = (ext["valid"][:, rows].cpu().numpy() != 0) & ref["valid"]
    rms = float(np.sqrt(np.mean(np.abs(Hr) ** 2)))
    m = np.abs(Hr) >= 0.1 * rms
    dL = float(np.abs(L - ref["L"])[v].max())
    return {"instants": [int(r) for r in rows], "ray_instants_compared": int(v.sum()),
            "valid_mismatch": int(((ext["valid"][:, rows].cpu().numpy() != 0) != ref["valid"]).sum()),
            "L_m": dL, "tau_s": dL / C0, "doppler_hz": float(np.abs(dop - ref["dop"])[v].max()),
            "H_mag_rel": float((np.abs(np.abs(Hg[m]) - np.abs(Hr[m])) / np.abs(Hr[m])).max()),
            "H_arg_rad": float(np.abs(np.angle(Hg[m] * np.conj(Hr[m]))).max()),
            "H_err_over_rms": float(np.abs(Hg - Hr).max() / rms),
            "tolerance": {"H_mag_rel": 1e-4, "H_arg_rad": 1e-3}}


def serving(ctx, torch, sids, n_requests, burst=False):
    """Serving mix: Poisson arrivals at 2000/s over 64 resident 20000-ray scenes (burst: the
    same kind of requests all submitted at once, which measures the served throughput)."""
    import numpy as np
    from paper_2205_00237_amd import scenes
    from paper_2205_00237_amd._abi import drt_now
    from paper_2205_00237_amd.drt import DRT_SPLIT
    reqs = scenes.config5_requests(n_requests)
    if burst:
        for q in reqs:
            q.arrival = 0.0
    # the client stays out of the measurement's way: every output buffer and grid is made
    # before the clock starts (a device allocation inside the loop can stall it for
    # milliseconds), due requests are always submitted before any polling, and each pass
    # polls at most 32 of the pending tickets, oldest first
    Hs = [torch.empty((q.n_steps, q.n_sub), dtype=torch.complex64, device="cuda") for q in reqs]
    grids = [(scenes.TimeGrid(q.dt, q.n_steps), scenes.FreqGrid(q.f_c, q.bandwidth, q.n_sub)) for q in reqs]
    # the first submission on a context starts the serving loop (its thread, slot streams and
    # captured batch graphs); do that before the clock, with one request run to completion
    tk = ctx.submit(sids[reqs[0].scene], reqs[0].n_rays, grids[0][0], grids[0][1], Hs[0], DRT_SPLIT)
    while True:
        st = ctx.poll(tk)[0]
        if st == 2 or st < 0:
            break
        time.sleep(1e-4)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()   # a collection pause inside the loop would delay submissions by milliseconds
    stats0 = ctx.serving_stats()
    pending, lat, samples, t_last = {}, [], 0, 0.0
    t_start = drt_now() + 0.05
    i = 0
    while i < len(reqs) or pending:
        now = drt_now()
        while i < len(reqs) and t_start + reqs[i].arrival <= now:
            q = reqs[i]
            tk = ctx.submit(sids[q.scene], q.n_rays, grids[i][0], grids[i][1], Hs[i], DRT_SPLIT)
            pending[tk] = q
            i += 1
        for tk in list(pending)[:32]:
            st = ctx.poll(tk)
            if st[0] == 2 or st[0] < 0:
                q = pending.pop(tk)
                if st[0] < 0:
                    raise RuntimeError(f"request failed with status {st[0]}")
                lat.append(st[3] - (t_start + q.arrival))
                samples += q.n_rays * q.n_steps * q.n_sub
                t_last = max(t_last, st[3])
            if i < len(reqs) and t_start + reqs[i].arrival <= drt_now():
                break   # a request is due: submit it first
        if i < len(reqs) and not pending:
            time.sleep(max(0.0, min(1e-4, t_start + reqs[i].arrival - drt_now())))
    gc.enable()
    stats1 = ctx.serving_stats()
    nb = stats1["batches"] - stats0["batches"]
    lat = np.array(lat)
    span = t_last - (t_start + reqs[0].arrival)
    arrivals = "all submitted at once" if burst else "Poisson 2000/s"
    return {"workload": f"{len(reqs)} requests, {arrivals}, 64 resident scenes of 20000 rays, "
                        "rays log-uniform 50-20000, 10-1000 instants of 1 ms, 64-2048 subcarriers, "
                        "28/60 GHz, 400 MHz, split precision",
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "max_ms": float(lat.max() * 1e3), "samples_per_s": samples / span,
            "offered_samples_per_s": (None if burst else samples / (reqs[-1].arrival - reqs[0].arrival)),
            "graph_batches": nb,
            "mean_batch": (stats1["batched_requests"] - stats0["batched_requests"]) / max(1, nb),
            "max_batch": stats1["max_batch"],
            "requests_alone": stats1["single_launches"] - stats0["single_launches"]}


def extras(ctx, torch, sid, scene, tg, fg, args, sec64=None):
    """The other calls on the urban scene: drt_extrapolate, the kinematics, the power
    profiles, the snapshot trace and lifetime refresh, and H by the non-uniform FFT."""
    from paper_2205_00237_amd.drt import DRT_SPLIT
    R, T, K = len(scene["ray_nint"]), tg.n_steps, fg.n_sub
    res = {}
    # drt_extrapolate alone (every per-(ray, instant) output and the validity monitor):
    # 8 + 4 + 16 + 8 + 1 + 1 = 38 B per (ray, instant) and 4 B per ray
    ext = ctx.extrapolate(sid, tg, fg.f_c, DRT_SPLIT)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    sec_ext = timed_steps(lambda: ctx.extrapolate(sid, tg, fg.f_c, DRT_SPLIT, out=ext), args.steps, 2, torch)
    prof_ext = ctx.profile_read(reset=True)
    ctx.profile(False)
    ext_bytes = R * T * 38 + R * 4
    ext_kernel_ms = (prof_ext["pose"][0] + prof_ext["geom"][0]) / max(1, prof_ext["pose"][1])
    res["extrapolate"] = {"ms_per_call": sec_ext * 1e3, "ray_instants_per_s": R * T / sec_ext,
                          "bytes_written": ext_bytes, "write_GB_per_s": ext_bytes / sec_ext / 1e9,
                          "hbm_frac": ext_bytes / sec_ext / PEAK_HBM, "kernel_ms": ext_kernel_ms,
                          "outputs": "L f64, f_D, 4 angles f32, gain c64, valid, in_bounds u8 per "
                                     "(ray, instant); first_out i32 per ray"}
    log(f"extrapolate: {res['extrapolate']}")
    del ext
    # kinematics of the interaction points (second-order jets): positions, velocities,
    # accelerations (3 x 96 B) and the Doppler rate (4 B) per (ray, instant)
    kin = {k: torch.empty((R, T, 4, 3), dtype=torch.float64, device="cuda") for k in ("q_pos", "q_vel", "q_acc")}
    kin["dop_rate"] = torch.empty((R, T), dtype=torch.float32, device="cuda")
    kin["valid"] = torch.empty((R, T), dtype=torch.uint8, device="cuda")
    sec_kin = timed_steps(lambda: ctx.extrapolate(sid, tg, fg.f_c, DRT_SPLIT, out=kin),
                          max(3, args.steps // 4), 1, torch)
    # second-order Taylor extrapolation of the points from t0 against the re-solved points
    ok = kin["valid"].bool().all(dim=1)
    q0, v0, a0 = (kin[k][:, 0] for k in ("q_pos", "q_vel", "q_acc"))
    taylor = {}
    for j in (20, 100, 200):
        d = j * tg.dt
        err = torch.linalg.vector_norm(q0 + v0 * d + 0.5 * a0 * d * d - kin["q_pos"][:, j], dim=-1).amax(dim=-1)
        taylor[f"{d * 1e3:g} ms"] = float(err[ok].max()) if bool(ok.any()) else None
    kin_bytes = R * T * (3 * 96 + 4 + 1)
    res["kinematics"] = {"ms_per_call": sec_kin * 1e3, "ray_instants_per_s": R * T / sec_kin,
                         "bytes_written": kin_bytes, "write_GB_per_s": kin_bytes / sec_kin / 1e9,
                         "taylor_point_error_m": taylor, "rays_valid_throughout": int(ok.sum())}
    log(f"kinematics: {res['kinematics']}")
    del kin
    # power-Doppler and power-delay profiles (incoherent bin sums of |a|^2) over 10 ms x 100 Hz
    # and 10 ms x 2.5 ns bins: the geometry and field work of extrapolate, binned in-kernel
    pbins = dict(steps_per_bin=20, n_dop=512, dop_lo=-25600.0, dop_step=100.0,
                 n_delay=2048, delay_lo=0.0, delay_step=2.5e-9, in_bounds_only=0)
    pp = ctx.power_profiles(sid, tg, fg.f_c, pbins)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    sec_pp = timed_steps(lambda: ctx.power_profiles(sid, tg, fg.f_c, pbins, out=pp), args.steps, 2, torch)
    prof_pp = ctx.profile_read(reset=True)
    gated = dict(pbins, in_bounds_only=1)
    sec_ppg = timed_steps(lambda: ctx.power_profiles(sid, tg, fg.f_c, gated, out=pp), args.steps, 2, torch)
    ctx.profile(False)
    res["power_profiles"] = {"ms_per_call": sec_pp * 1e3, "ray_instants_per_s": R * T / sec_pp,
                             "geom_kernel_ms": prof_pp["geom"][0] / max(1, prof_pp["pose"][1]),
                             "gated_ms_per_call": sec_ppg * 1e3,
                             "bins": {"time_bins": (T + 19) // 20, "doppler": 512, "delay": 2048,
                                      "time_s": 20 * tg.dt, "doppler_hz": 100.0, "delay_s": 2.5e-9},
                             "gated_counted_power": float(pp["total"].sum())}
    log(f"power profiles: {res['power_profiles']}")
    del pp
    # snapshot tracing (the conventional RT that DRT extrapolates) and the lifetime refresh
    topts = dict(max_refl=3, max_refl_diff=1, scattering=False, los=True)
    t_tr = []
    for _ in range(4):
        t = time.perf_counter()
        new, info = ctx.trace(sid, 0.0, **topts)
        t_tr.append(time.perf_counter() - t)
        ctx.unload_scene(new)
    trace_s = sorted(t_tr[1:])[1]
    sopts = dict(max_refl=2, max_refl_diff=1, scattering=False, los=True)
    t = time.perf_counter()
    segs = ctx.segments(sid, tg, fg.f_c, threshold_db=10.0, max_steps=250, **sopts)
    seg_s = time.perf_counter() - t
    Hs = torch.empty((T, K), dtype=torch.complex64, device="cuda")
    sec_hs = timed_steps(lambda: ctx.cfr_segments(segs, tg, fg, DRT_SPLIT, out=Hs), 5, 1, torch)
    for _, _, s_id in segs:
        ctx.unload_scene(s_id)
    res["tracer"] = {"trace_ms": trace_s * 1e3, "orders": "LoS, 1-3 reflections, 1 diffraction with 0-1 reflections",
                     "candidates": info["candidates"], "candidates_per_s": info["candidates"] / trace_s,
                     "geometric": info["geometric"], "paths": info["n_paths"],
                     "segments": len(segs), "segment_instants": [n for _, n, _ in segs],
                     "segments_s": seg_s, "cfr_over_segments_ms": sec_hs * 1e3}
    log(f"tracer: {res['tracer']}")
    del Hs
    # the same H by the type-1 non-uniform FFT along f (binary64, kernel accuracy 1e-9 of
    # sum |a|): a variant with per-instant work R w + 5 M log2 M instead of R K
    Hn = torch.empty((T, K), dtype=torch.complex128, device="cuda")
    ctx.profile(True)
    ctx.profile_read(reset=True)
    sec_nu = timed_steps(lambda: ctx.cfr_nufft(sid, tg, fg, eps=1e-9, out=Hn), args.steps, 2, torch)
    prof_nu = ctx.profile_read(reset=True)
    ctx.profile(False)
    nufft = {"ms_per_step": sec_nu * 1e3, "samples_per_s": R * T * K / sec_nu, "eps": 1e-9, "dtype": "f64",
             "kernels": {k: {"avg_ms": v[0] / max(1, v[1]), "launches": v[1]} for k, v in prof_nu.items() if v[1]},
             "per_instant_work": "spread 5000 rays x 10 kernel points, FFT of 2048, 1024 outputs"}
    if sec64:
        nufft["speedup_vs_fp64_direct"] = sec64 / (sec_nu * 1e3)
    res["nufft"] = nufft
    log(f"nufft: {nufft}")
    del Hn
    return res


def scattering(ctx, torch, args):
    """The scattering workload at full size: 2e5 tiles (and rays) on 50 moving boxes, 500
    instants x 1 ms, 256 subcarriers over 2 GHz at 60 GHz (2.56e10 samples), split and
    binary64."""
    from paper_2205_00237_amd import scenes
    from paper_2205_00237_amd.drt import DRT_FP64, DRT_SPLIT
    t = time.perf_counter()
    s3, tg3, fg3 = scenes.config3()
    gen_s = time.perf_counter() - t
    t = time.perf_counter()
    sid3 = ctx.load_scene(s3)
    load_s = time.perf_counter() - t
    R, T, K = len(s3["ray_nint"]), tg3.n_steps, fg3.n_sub
    res = {"workload": "scattering: 200000 effective-roughness tiles on 50 moving, turning boxes, 500 instants "
                       "x 1 ms, 256 subcarriers / 2 GHz at 60 GHz", "rays": R, "instants": T, "subcarriers": K,
           "samples": R * T * K, "scene_gen_s": gen_s, "scene_load_s": load_s}
    for prec, nm, dt in ((DRT_SPLIT, "split", torch.complex64), (DRT_FP64, "fp64", torch.complex128)):
        H3 = torch.empty((T, K), dtype=dt, device="cuda")
        sec3 = timed_steps(lambda: ctx.cfr(sid3, tg3, fg3, prec, out=H3), max(3, args.steps // 4), 2, torch)
        res[nm] = {"ms_per_step": sec3 * 1e3, "samples_per_s": R * T * K / sec3}
        del H3
    res["split_speedup"] = res["fp64"]["ms_per_step"] / res["split"]["ms_per_step"]
    ctx.unload_scene(sid3)
    log(f"scattering: {res}")
    return res


def timed_calls(fn, n, torch):
    """Wall time of n synchronous calls (launch to completion), each timed alone."""
    out = []
    for _ in range(n):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        out.append(time.perf_counter() - t)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline step, its accuracy, the binary64 paths and the roofline")
    ap.add_argument("--serving-requests", type=int, default=4096)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (reference dispatch for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: the library runs the hot path on a single MI355X and "
              f"has no multi-GPU path (asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_2205_00237_amd import scenes

    scene, tg, fg = scenes.config2()
    R, T, K = len(scene["ray_nint"]), tg.n_steps, fg.n_sub
    samples = R * T * K
    # CPU work first, while no process has touched the GPU (the all-core oracle forks)
    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(scene, tg, fg)
        log(f"cpu baseline: {cpu}")
    acc_rows = [0, 63, 64, 311, 500, 777, 998, 999]
    ref = oracle_sample(scene, tg, fg, acc_rows)

    import torch
    from paper_2205_00237_amd.drt import Context, DRT_FP64, DRT_SPLIT

    ctx = Context(0)
    t = time.perf_counter()
    sid = ctx.load_scene(scene)
    load_s = time.perf_counter() - t

    H = torch.empty((T, K), dtype=torch.complex64, device="cuda")
    step = lambda: ctx.cfr(sid, tg, fg, DRT_SPLIT, out=H)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the step as a user runs it (no per-kernel events), then the same steps again with
    # per-kernel HIP events for the kernel figures and the roofline
    sec = timed_steps(step, args.steps, 0, torch)
    ctx.profile(True)
    ctx.profile_read(reset=True)
    sec_prof = timed_steps(step, args.steps, 0, torch)
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    log(f"split: {sec * 1e3:.3f} ms/step ({sec_prof * 1e3:.3f} with per-kernel events), kernels {prof}")
    # accuracy of what was timed: H of the last step, geometry of drt_extrapolate (split)
    ext = ctx.extrapolate(sid, tg, fg.f_c, DRT_SPLIT)
    torch.cuda.synchronize()
    acc = accuracy(ref, acc_rows, H, ext)
    log(f"accuracy: {acc}")

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    fp64 = None
    if not args.no_fp64:
        # both binary64 ray sums, each in a context of its own (the kernel is chosen at
        # context creation): the subcarrier walk on the vector ALU, and the split path's GEMM
        # factorisation on the binary64 matrix cores
        fp64 = {"dtype": "f64"}
        for kern, what in (("valu", "k_cfr<0, 32>: 32 subcarriers per lane, three-term phasor recurrence"),
                           ("mfma64", "k_cfr_mfma64<1, 8>: complex GEMM U (16 x R) . V (R x 64) per instant "
                                      "on v_mfma_f64_16x16x4_f64, K/B + B = 80 phasors per (ray, instant)")):
            os.environ["DRT_FP64_KERNEL"] = kern
            c64 = Context(0)
            sid64 = c64.load_scene(scene)
            H64 = torch.empty((T, K), dtype=torch.complex128, device="cuda")
            step64 = lambda: c64.cfr(sid64, tg, fg, DRT_FP64, out=H64)
            sec64 = timed_steps(step64, max(3, args.steps // 2), 1, torch)
            c64.profile(True)
            c64.profile_read(reset=True)
            timed_steps(step64, max(3, args.steps // 2), 0, torch)
            prof64 = c64.profile_read(reset=True)
            c64.profile(False)
            log(f"fp64 {kern}: {sec64 * 1e3:.3f} ms/step, kernels {prof64}")
            rms64 = float(np.sqrt(np.mean(np.abs(ref["H"]) ** 2)))
            fp64[kern] = {"value": samples / sec64, "ms_per_step": sec64 * 1e3, "kernel": what,
                          "kernels": {k: {"avg_ms": v[0] / max(1, v[1]), "launches": v[1]}
                                      for k, v in prof64.items() if v[1]},
                          "H_err_over_rms": float(np.abs(H64[acc_rows].cpu().numpy() - ref["H"]).max()) / rms64}
            c64.unload_scene(sid64)
            c64.close()
            del H64
        os.environ.pop("DRT_FP64_KERNEL", None)
        best = min(("valu", "mfma64"), key=lambda k: fp64[k]["ms_per_step"])
        fp64.update({"value": fp64[best]["value"], "ms_per_step": fp64[best]["ms_per_step"], "fastest": best,
                     "split_speedup": fp64[best]["ms_per_step"] / (sec * 1e3)})

    # dominant kernel of the split step (largest time per launch), against its roofline;
    # its average launch time comes from HIP events recorded on the stream it runs on
    name = max(prof, key=lambda k: prof[k][0] / max(1, prof[k][1]))
    ms_avg = prof[name][0] / max(1, prof[name][1])
    if name == "cfr":
        path = os.environ.get("DRT_CFR_KERNEL", "mfma16")
        kern, bound, peak = {"mfma16": ("k_cfr_mfma16", "mfma", PEAK_FP16_MFMA),
                             "mfma32": ("k_cfr_mfma", "mfma", PEAK_FP32_MFMA),
                             "valu": ("k_cfr", "alu", PEAK_FP32_VECTOR)}[path]
        achieved = FLOP_PER_SAMPLE * samples / (ms_avg * 1e-3)
        roof = {"kernel": kern, "bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": measured_traffic(kern),
                "avg_ms": ms_avg, "launches_timed": prof[name][1],
                "per_unit": f"{FLOP_PER_SAMPLE} flop per (ray, instant, subcarrier) sample "
                            f"(complex multiply-accumulate), {samples} samples per launch"}
    else:
        roof = {"kernel": name, "bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "avg_ms": ms_avg}
    # the whole step against the direct-sum vector roofline (8 binary32 flop per sample)
    path_roof = {"bound": "alu", "achieved": FLOP_PER_SAMPLE * samples / sec / 1e12,
                 "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                 "frac": FLOP_PER_SAMPLE * samples / sec / PEAK_FP32_VECTOR}
    kernels = {k: {"avg_ms": v[0] / max(1, v[1]), "launches": v[1]} for k, v in prof.items() if v[1]}

    out = {
        "metric": "ray*time*freq samples/s of H(t,f), split-precision vs FP64 GPU; p99 latency",
        "value": samples / sec, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 geometry + f32 field + f16 hi/lo x3 MFMA (f32 accumulate)",
        "data": "synthetic",
        "config": {"workload": "urban vehicular: 5000 rays <= 3R+1D, 20 moving boxes, "
                               "200 facades, 1000 instants x 0.5 ms, 1024 subcarriers / 400 MHz at 28 GHz; "
                               "split precision: binary64 geometry and carrier-phase reduction, binary32 "
                               "field coefficients, ray sum as complex GEMMs on the binary16 matrix cores "
                               "(each binary32 operand split hi + lo in binary16, three products per tile, "
                               "binary32 accumulation)",
                   "rays": R, "instants": T, "subcarriers": K, "parallelism": "single GPU"},
        "accuracy": acc,
        "fp64_gpu": fp64,
        "roofline": roof,
        "step_vs_direct_sum_roofline": path_roof,
        "kernels": kernels,
        "ms_per_step_with_kernel_events": sec_prof * 1e3,
        "scene_load_s": load_s,
    }

    # the tiny workload: latency of one call (launch to completion), binary64 and split
    s1, tg1, fg1 = scenes.config1()
    sid1 = ctx.load_scene(s1)
    lat = {}
    for prec, nm in ((DRT_FP64, "fp64"), (DRT_SPLIT, "split")):
        for _ in range(5):
            ctx.cfr(sid1, tg1, fg1, prec)
        torch.cuda.synchronize()
        w = np.array(timed_calls(lambda: ctx.cfr(sid1, tg1, fg1, prec), 200, torch)) * 1e3
        lat[nm] = {"p50_ms": float(np.percentile(w, 50)), "p99_ms": float(np.percentile(w, 99))}
    ctx.unload_scene(sid1)
    out["tiny_latency"] = {"workload": "tiny: 25 rays (LoS, 6 R, 2 D, 16 S), 100 instants x 1 ms, "
                                       "64 subcarriers / 100 MHz at 28 GHz",
                           "samples": len(s1["ray_nint"]) * tg1.n_steps * fg1.n_sub, **lat}
    log(f"tiny latency: {out['tiny_latency']}")

    if not args.no_extras:
        out.update(extras(ctx, torch, sid, scene, tg, fg, args, sec64=(fp64 or {}).get("ms_per_step")))
    ctx.unload_scene(sid)
    if not args.no_extras:
        out["scattering"] = scattering(ctx, torch, args)
    ctx.close()
    if not args.no_serving:
        log("serving mix ...")
        cap = 200e9
        sctx = Context(0, hbm_cap_bytes=int(cap))
        t = time.perf_counter()
        sids = [sctx.load_scene(s) for s in scenes.config5_scenes()]
        load5 = time.perf_counter() - t
        out["serving"] = serving(sctx, torch, sids, args.serving_requests)
        out["serving"]["scene_load_s"] = load5
        out["serving"]["hbm_cap_bytes"] = cap
        log(f"serving: {out['serving']}")
        log("serving burst ...")
        out["serving_burst"] = serving(sctx, torch, sids, 512, burst=True)
        out["serving_burst"]["hbm_cap_bytes"] = cap
        log(f"serving burst: {out['serving_burst']}")
        for s in sids:
            sctx.unload_scene(s)
        sctx.close()
        out["p99_latency_ms"] = out["serving"]["p99_ms"]
        out["p50_latency_ms"] = out["serving"]["p50_ms"]
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
