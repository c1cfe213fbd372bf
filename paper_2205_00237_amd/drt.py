"""PyTorch-facing convenience layer over the C ABI (argument marshalling only).

PyTorch provides the device memory (output tensors) and the stream handle; every step of
the hot path runs in libdrt's HIP kernels.
"""
import numpy as np
import torch

from . import _abi
from ._abi import DRT_FP64, DRT_SPLIT, DRT_NAIVE32, DrtError  # noqa: F401

_STREAM_NULL = 0


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class Context:
    """One libdrt context on one device."""

    def __init__(self, device=0, hbm_cap_bytes=0):
        self.device = torch.device("cuda", device)
        self.ctx = _abi.drt_create(device, hbm_cap_bytes)
        self.n_rays = {}

    def close(self):
        if self.ctx is not None:
            _abi.drt_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def load_scene(self, scene, ray_q0=None):
        sid = _abi.drt_load_scene(self.ctx, scene, ray_q0)
        self.n_rays[sid] = int(np.asarray(scene["ray_nint"]).shape[0])
        return sid

    def unload_scene(self, sid):
        _abi.drt_unload_scene(self.ctx, sid)
        self.n_rays.pop(sid, None)

    def extrapolate(self, sid, tgrid, f_c, precision=DRT_SPLIT, n_rays=None, stream=None, out=None,
                    kinematics=False):
        """Per-(ray, instant) outputs as device tensors [n_rays][n_steps] (first_out: [n_rays]);
        with kinematics=True also q_pos, q_vel, q_acc [n_rays][n_steps][4][3] and dop_rate.
        `out` may pass a dict of preallocated tensors (any subset) to write instead."""
        R = self.n_rays[sid] if n_rays is None else int(n_rays)
        T = int(tgrid.n_steps)
        dev = self.device
        gdt = torch.complex128 if precision == DRT_FP64 else torch.complex64
        if out is not None:
            _abi.drt_extrapolate(self.ctx, sid, R, tgrid.dt, T, f_c, precision,
                                 {k: v.data_ptr() for k, v in out.items()}, _stream(stream))
            return out
        out = {"L": torch.empty((R, T), dtype=torch.float64, device=dev),
               "dop": torch.empty((R, T), dtype=torch.float32, device=dev),
               "aod_az": torch.empty((R, T), dtype=torch.float32, device=dev),
               "aod_el": torch.empty((R, T), dtype=torch.float32, device=dev),
               "aoa_az": torch.empty((R, T), dtype=torch.float32, device=dev),
               "aoa_el": torch.empty((R, T), dtype=torch.float32, device=dev),
               "gain": torch.empty((R, T), dtype=gdt, device=dev),
               "valid": torch.empty((R, T), dtype=torch.uint8, device=dev),
               "in_bounds": torch.empty((R, T), dtype=torch.uint8, device=dev),
               "first_out": torch.empty((R,), dtype=torch.int32, device=dev)}
        if kinematics:
            for k in ("q_pos", "q_vel", "q_acc"):
                out[k] = torch.empty((R, T, 4, 3), dtype=torch.float64, device=dev)
            out["dop_rate"] = torch.empty((R, T), dtype=torch.float32, device=dev)
        _abi.drt_extrapolate(self.ctx, sid, R, tgrid.dt, T, f_c, precision,
                             {k: v.data_ptr() for k, v in out.items()}, _stream(stream))
        return out

    def trace(self, sid, t=0.0, max_refl=2, max_refl_diff=1, scattering=True, los=True, double_diff=False):
        """Snapshot trace at the scene's t0 + t: a new resident scene (the primitives carried
        to that instant, one ray per path found).  Returns (new scene id, info dict)."""
        new, info = _abi.drt_trace(self.ctx, sid, t, max_refl, max_refl_diff, scattering, los, double_diff)
        self.n_rays[new] = info["n_paths"]
        return new, info

    def segments(self, sid, tgrid, f_c, threshold_db=10.0, max_steps=200, min_steps=1, **trace_opts):
        """Multipath lifetimes over the time grid, each traced afresh at its start:
        [(first instant, length, resident scene id)]; the caller unloads the scenes."""
        segs = _abi.drt_segments(self.ctx, sid, tgrid.dt, tgrid.n_steps, f_c, trace_opts, threshold_db,
                                 max_steps, min_steps)
        for _, _, s in segs:
            self.n_rays[s] = int(_abi.drt_scene_rays(self.ctx, s)[0].shape[0])
        return segs

    def cfr_segments(self, segs, tgrid, fgrid, precision=DRT_SPLIT, out=None, stream=None):
        """H over the whole time grid, rows of each segment from the scene traced at its start."""
        T, K = int(tgrid.n_steps), int(fgrid.n_sub)
        if out is None:
            out = torch.empty((T, K), dtype=torch.complex128 if precision == DRT_FP64 else torch.complex64,
                              device=self.device)
        for j0, n, s in segs:
            rows = out[j0:j0 + n]
            _abi.drt_cfr(self.ctx, s, self.n_rays[s], tgrid.dt, n, fgrid.f_c, fgrid.bandwidth, K, precision,
                         rows.data_ptr(), _stream(stream))
        return out

    def scene_rays(self, sid):
        """Interaction sequences of a resident scene: nint, kind, prim, pol (numpy)."""
        return _abi.drt_scene_rays(self.ctx, sid)

    def power_profiles(self, sid, tgrid, f_c, bins, precision=DRT_SPLIT, n_rays=None, stream=None, out=None):
        """Power-Doppler profile pdfp [n_tb][n_dop], power-delay profile pdp [n_tb][n_delay] and
        per-time-bin total [n_tb] as binary64 device tensors; bins: dict of steps_per_bin,
        n_dop, dop_lo, dop_step, n_delay, delay_lo, delay_step and optionally in_bounds_only.
        `out` may pass a dict of preallocated tensors (any subset) to write instead."""
        R = self.n_rays[sid] if n_rays is None else int(n_rays)
        T = int(tgrid.n_steps)
        if out is None:
            n_tb = (T + int(bins["steps_per_bin"]) - 1) // max(int(bins["steps_per_bin"]), 1)
            f8 = dict(dtype=torch.float64, device=self.device)
            out = {"pdfp": torch.empty((n_tb, int(bins["n_dop"])), **f8),
                   "pdp": torch.empty((n_tb, int(bins["n_delay"])), **f8),
                   "total": torch.empty((n_tb,), **f8)}
        _abi.drt_power_profiles(self.ctx, sid, R, tgrid.dt, T, f_c, precision, bins,
                                {k: v.data_ptr() for k, v in out.items()}, _stream(stream))
        return out

    def cfr(self, sid, tgrid, fgrid, precision=DRT_SPLIT, n_rays=None, out=None, stream=None):
        """H(t_j, f_k) as a device tensor [n_steps][n_sub] (complex128 for FP64, else complex64)."""
        R = self.n_rays[sid] if n_rays is None else int(n_rays)
        T, K = int(tgrid.n_steps), int(fgrid.n_sub)
        if out is None:
            out = torch.empty((T, K), dtype=torch.complex128 if precision == DRT_FP64 else torch.complex64,
                              device=self.device)
        _abi.drt_cfr(self.ctx, sid, R, tgrid.dt, T, fgrid.f_c, fgrid.bandwidth, K, precision,
                     out.data_ptr(), _stream(stream))
        return out

    def cfr_nufft(self, sid, tgrid, fgrid, eps=1e-9, n_rays=None, out=None, stream=None):
        """H(t_j, f_k) [n_steps][n_sub] complex128 by the type-1 non-uniform FFT along f."""
        R = self.n_rays[sid] if n_rays is None else int(n_rays)
        T, K = int(tgrid.n_steps), int(fgrid.n_sub)
        if out is None:
            out = torch.empty((T, K), dtype=torch.complex128, device=self.device)
        _abi.drt_cfr_nufft(self.ctx, sid, R, tgrid.dt, T, fgrid.f_c, fgrid.bandwidth, K, eps, out.data_ptr(),
                           _stream(stream))
        return out

    def submit(self, sid, n_rays, tgrid, fgrid, H, precision=DRT_SPLIT):
        return _abi.drt_submit(self.ctx, sid, n_rays, tgrid.dt, tgrid.n_steps, fgrid.f_c,
                               fgrid.bandwidth, fgrid.n_sub, precision, H.data_ptr())

    def poll(self, ticket):
        return _abi.drt_poll(self.ctx, ticket)

    def serving_stats(self):
        """Batches replayed, requests inside them, requests run alone, largest batch, slots."""
        return _abi.drt_serving_stats_get(self.ctx)

    def profile(self, on=True):
        _abi.drt_profile_enable(self.ctx, on)

    def profile_read(self, reset=True):
        return _abi.drt_profile_read(self.ctx, reset)
