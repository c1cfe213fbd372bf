#!/usr/bin/env python3
"""Throughput of the DRT hot path on one MI355X.

A step is one drt_cfr call over the urban vehicular workload (5000 rays up to three
reflections plus one diffraction among 20 moving boxes and 200 facades, 1000 instants of
0.5 ms, 1024 subcarriers over 400 MHz at 28 GHz): body poses, per-(ray, instant)
extrapolation and field coefficients, and the ray sum H(t, f), in split precision.  The
metric is ray x time x frequency samples of H per second, with inputs resident in device
memory.  Beside it: the binary64 GPU path on the same workload, the kernel-level roofline
of the dominant kernel (timed with HIP events on its own stream), the CPU oracle on a
bounded sample, the serving mix (4096 Poisson requests over 64 resident scenes) with
p50 / p99 latency, and the other calls on the same scene: drt_extrapolate with the
validity monitor, the interaction-point kinematics, the power-Doppler and power-delay
profiles, the snapshot trace and the multipath-lifetime refresh, and H by the non-uniform
FFT.  Prints one JSON line.
"""
import argparse
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
KERNEL_SOURCE = os.path.join(ROOT, "paper_2205_00237_amd", "csrc", "kernels.hip")
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


def cpu_baseline(scene, tg, fg, budget_s=15.0):
    """The oracle (numpy, one thread) on whole time rows of the same workload."""
    import numpy as np
    import oracle
    R, K = len(scene["ray_nint"]), fg.n_sub
    t = time.perf_counter()
    oracle.run(scene, tg, fg, t_index=np.array([0]))
    one = time.perf_counter() - t
    rows = max(1, min(tg.n_steps, int(budget_s / max(one, 1e-3))))
    idx = np.linspace(0, tg.n_steps - 1, rows).astype(int)
    t = time.perf_counter()
    oracle.run(scene, tg, fg, t_index=idx)
    el = time.perf_counter() - t
    return {"value": R * rows * K / el, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} of {tg.n_steps} instants, all {R} rays and {K} subcarriers "
                      f"({el:.1f} s, numpy float64, single thread)"}


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
    stats0 = ctx.serving_stats()
    pending, lat, samples, t_last = {}, [], 0, 0.0
    t_start = drt_now() + 0.05
    i = 0
    while i < len(reqs) or pending:
        now = drt_now()
        while i < len(reqs) and t_start + reqs[i].arrival <= now:
            q = reqs[i]
            H = torch.empty((q.n_steps, q.n_sub), dtype=torch.complex64, device="cuda")
            tk = ctx.submit(sids[q.scene], q.n_rays, scenes.TimeGrid(q.dt, q.n_steps),
                            scenes.FreqGrid(q.f_c, q.bandwidth, q.n_sub), H, DRT_SPLIT)
            pending[tk] = (q, H)
            i += 1
        for tk in list(pending):
            st = ctx.poll(tk)
            if st[0] == 2 or st[0] < 0:
                q, _ = pending.pop(tk)
                if st[0] < 0:
                    raise RuntimeError(f"request failed with status {st[0]}")
                lat.append(st[3] - (t_start + q.arrival))
                samples += q.n_rays * q.n_steps * q.n_sub
                t_last = max(t_last, st[3])
        if i < len(reqs) and not pending:
            time.sleep(max(0.0, min(1e-4, t_start + reqs[i].arrival - drt_now())))
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
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

    import torch
    from paper_2205_00237_amd import scenes
    from paper_2205_00237_amd.drt import Context, DRT_FP64, DRT_SPLIT

    scene, tg, fg = scenes.config2()
    R, T, K = len(scene["ray_nint"]), tg.n_steps, fg.n_sub
    samples = R * T * K
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

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # drt_extrapolate alone (every per-(ray, instant) output and the validity monitor), the
    # HBM-write-bound call: 8 + 4 + 16 + 8 + 1 + 1 = 38 B per (ray, instant) and 4 B per ray
    ext = ctx.extrapolate(sid, tg, fg.f_c, DRT_SPLIT)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    sec_ext = timed_steps(lambda: ctx.extrapolate(sid, tg, fg.f_c, DRT_SPLIT, out=ext), args.steps, 2, torch)
    prof_ext = ctx.profile_read(reset=True)
    ctx.profile(False)
    ext_bytes = R * T * 38 + R * 4
    ext_kernel_ms = (prof_ext["pose"][0] + prof_ext["geom"][0]) / max(1, prof_ext["pose"][1])
    extrap = {"ms_per_call": sec_ext * 1e3, "ray_instants_per_s": R * T / sec_ext,
              "bytes_written": ext_bytes, "write_GB_per_s": ext_bytes / sec_ext / 1e9,
              "hbm_frac": ext_bytes / sec_ext / PEAK_HBM, "kernel_ms": ext_kernel_ms,
              "outputs": "L f64, f_D, 4 angles f32, gain c64, valid, in_bounds u8 per (ray, instant); "
                         "first_out i32 per ray"}
    log(f"extrapolate: {extrap}")
    del ext
    # kinematics of the interaction points (second-order jets): positions, velocities,
    # accelerations (3 x 96 B) and the Doppler rate (4 B) per (ray, instant)
    kin = {k: torch.empty((R, T, 4, 3), dtype=torch.float64, device="cuda") for k in ("q_pos", "q_vel", "q_acc")}
    kin["dop_rate"] = torch.empty((R, T), dtype=torch.float32, device="cuda")
    kin["valid"] = torch.empty((R, T), dtype=torch.uint8, device="cuda")
    sec_kin = timed_steps(lambda: ctx.extrapolate(sid, tg, fg.f_c, DRT_SPLIT, out=kin), max(3, args.steps // 4), 1, torch)
    # second-order Taylor extrapolation of the points from t0 against the re-solved points
    ok = kin["valid"].bool().all(dim=1)
    q0, v0, a0 = (kin[k][:, 0] for k in ("q_pos", "q_vel", "q_acc"))
    taylor = {}
    for j in (20, 100, 200):
        d = j * tg.dt
        err = torch.linalg.vector_norm(q0 + v0 * d + 0.5 * a0 * d * d - kin["q_pos"][:, j], dim=-1).amax(dim=-1)
        taylor[f"{d * 1e3:g} ms"] = float(err[ok].max()) if bool(ok.any()) else None
    kin_bytes = R * T * (3 * 96 + 4 + 1)
    kinematics = {"ms_per_call": sec_kin * 1e3, "ray_instants_per_s": R * T / sec_kin,
                  "bytes_written": kin_bytes, "write_GB_per_s": kin_bytes / sec_kin / 1e9,
                  "taylor_point_error_m": taylor, "rays_valid_throughout": int(ok.sum())}
    log(f"kinematics: {kinematics}")
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
    counted = float(pp["total"].sum())
    profiles = {"ms_per_call": sec_pp * 1e3, "ray_instants_per_s": R * T / sec_pp,
                "geom_kernel_ms": prof_pp["geom"][0] / max(1, prof_pp["pose"][1]),
                "gated_ms_per_call": sec_ppg * 1e3,
                "bins": {"time_bins": (T + 19) // 20, "doppler": 512, "delay": 2048,
                         "time_s": 20 * tg.dt, "doppler_hz": 100.0, "delay_s": 2.5e-9},
                "gated_counted_power": counted}
    log(f"power profiles: {profiles}")
    del pp
    # snapshot tracing (the conventional RT that DRT extrapolates) and the lifetime refresh;
    # against it, the paper's comparison: a snapshot trace at every instant (timed on 20
    # instants spread over the span, scaled to all of them) versus DRT, a trace per lifetime
    # plus extrapolation, both followed by the same ray sum over the span
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
    t = time.perf_counter()
    for j in range(0, T, T // 20):
        new, _ = ctx.trace(sid, j * tg.dt, **sopts)
        ctx.unload_scene(new)
    snap_s = (time.perf_counter() - t) / len(range(0, T, T // 20)) * T
    for _, _, s_id in segs:
        ctx.unload_scene(s_id)
    tracer = {"trace_ms": trace_s * 1e3, "orders": "LoS, 1-3 reflections, 1 diffraction with 0-1 reflections",
              "candidates": info["candidates"], "candidates_per_s": info["candidates"] / trace_s,
              "geometric": info["geometric"], "paths": info["n_paths"],
              "segments": len(segs), "segment_instants": [n for _, n, _ in segs],
              "segments_s": seg_s, "cfr_over_segments_ms": sec_hs * 1e3,
              "snapshot_trace_every_instant_s": snap_s,
              "drt_vs_snapshot_speedup": (snap_s + sec_hs) / (seg_s + sec_hs)}
    log(f"tracer: {tracer}")
    del Hs
    sec64 = None
    if not args.no_fp64:
        H64 = torch.empty((T, K), dtype=torch.complex128, device="cuda")
        step64 = lambda: ctx.cfr(sid, tg, fg, DRT_FP64, out=H64)
        sec64 = timed_steps(step64, max(3, args.steps // 2), 1, torch)
        ctx.profile(True)
        ctx.profile_read(reset=True)
        timed_steps(step64, max(3, args.steps // 2), 0, torch)
        prof64 = ctx.profile_read(reset=True)
        ctx.profile(False)
        log(f"fp64: {sec64 * 1e3:.3f} ms/step, kernels {prof64}")
    # the same H by the type-1 non-uniform FFT along f (binary64, kernel accuracy 1e-9 of
    # sum |a|): a variant with per-instant work R w + 5 M log2 M instead of R K; its error is
    # taken against the binary64 direct sum
    Hn = torch.empty((T, K), dtype=torch.complex128, device="cuda")
    ctx.profile(True)
    ctx.profile_read(reset=True)
    sec_nu = timed_steps(lambda: ctx.cfr_nufft(sid, tg, fg, eps=1e-9, out=Hn), args.steps, 2, torch)
    prof_nu = ctx.profile_read(reset=True)
    ctx.profile(False)
    nufft = {"ms_per_step": sec_nu * 1e3, "samples_per_s": samples / sec_nu, "eps": 1e-9, "dtype": "f64",
             "kernels": {k: {"avg_ms": v[0] / max(1, v[1]), "launches": v[1]} for k, v in prof_nu.items() if v[1]},
             "per_instant_work": "spread 5000 rays x 10 kernel points, FFT of 2048, 1024 outputs"}
    if sec64:
        ref_rms = float(torch.sqrt(torch.mean(torch.abs(H64) ** 2)))
        nufft["max_err_vs_fp64_direct_rel_rms"] = float(torch.max(torch.abs(Hn - H64))) / ref_rms
        nufft["speedup_vs_fp64_direct"] = sec64 / sec_nu
    log(f"nufft: {nufft}")
    del Hn

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
                "avg_ms": ms_avg,
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
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "urban vehicular: 5000 rays <= 3R+1D, 20 moving boxes, "
                               "200 facades, 1000 instants x 0.5 ms, 1024 subcarriers / 400 MHz at 28 GHz, "
                               "split precision (f64 phase reduction, f32 phasor arithmetic)",
                   "rays": R, "instants": T, "subcarriers": K, "parallelism": "single GPU"},
        "fp64_gpu": ({"value": samples / sec64, "ms_per_step": sec64 * 1e3, "dtype": "f64",
                      "split_speedup": sec64 / sec} if sec64 else None),
        "roofline": roof,
        "step_vs_direct_sum_roofline": path_roof,
        "extrapolate": extrap,
        "kinematics": kinematics,
        "power_profiles": profiles,
        "tracer": tracer,
        "nufft": nufft,
        "kernels": kernels,
        "ms_per_step_with_kernel_events": sec_prof * 1e3,
        "scene_load_s": load_s,
    }
    ctx.unload_scene(sid)
    if not args.no_serving:
        log("serving mix ...")
        from paper_2205_00237_amd import scenes as sc5
        t = time.perf_counter()
        sids = [ctx.load_scene(s) for s in sc5.config5_scenes()]
        load5 = time.perf_counter() - t
        out["serving"] = serving(ctx, torch, sids, args.serving_requests)
        out["serving"]["scene_load_s"] = load5
        log(f"serving: {out['serving']}")
        log("serving burst ...")
        out["serving_burst"] = serving(ctx, torch, sids, 512, burst=True)
        log(f"serving burst: {out['serving_burst']}")
        for s in sids:
            ctx.unload_scene(s)
        out["p99_latency_ms"] = out["serving"]["p99_ms"]
        out["p50_latency_ms"] = out["serving"]["p50_ms"]
    ctx.close()
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(scene, tg, fg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
