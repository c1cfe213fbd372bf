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
