"""ctypes binding of libdrt (include/drt.h).

Argument marshalling only: every computation runs in the HIP library.  Device buffers are
passed as raw pointers (a PyTorch CUDA tensor's data_ptr()) and streams as hipStream_t
handles (torch.cuda.current_stream().cuda_stream).  Importing this module loads the
library built in-tree by paper_2205_00237_amd/build.py and fails loudly when it is missing.
"""
import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdrt.so")

DRT_OK = 0
DRT_E_INVAL = -1
DRT_E_DEGENERATE = -2
DRT_E_NOMEM = -3
DRT_E_ADMISSION = -4
DRT_E_NOTFOUND = -5
DRT_E_BUSY = -6
DRT_E_DEVICE = -7
DRT_E_INCONSISTENT = -8
DRT_E_CANCELLED = -9

DRT_FP64, DRT_SPLIT, DRT_NAIVE32 = 0, 1, 2

EXPORTS = ("drt_create", "drt_destroy", "drt_load_scene", "drt_unload_scene", "drt_extrapolate",
           "drt_power_profiles", "drt_trace", "drt_scene_rays", "drt_segments", "drt_cfr_nufft",
           "drt_cfr", "drt_cfr_noalloc", "drt_submit", "drt_poll", "drt_now", "drt_strerror", "drt_last_error",
           "drt_profile_enable", "drt_profile_read", "drt_serving_stats_get")
KERNELS = ("pose", "geom", "cfr", "reduce")

_dp = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)
_i32p = C.POINTER(C.c_int32)


class SceneDesc(C.Structure):
    _fields_ = [
        ("t0", C.c_double),
        ("tx_p", C.c_double * 3), ("tx_v", C.c_double * 3), ("tx_a", C.c_double * 3),
        ("rx_p", C.c_double * 3), ("rx_v", C.c_double * 3), ("rx_a", C.c_double * 3),
        ("n_bodies", C.c_int32),
        ("body_O0", _dp), ("body_v0", _dp), ("body_a", _dp), ("body_axis", _dp),
        ("body_w0", _dp), ("body_wdot", _dp),
        ("n_mat", C.c_int32),
        ("mat_eps_r", _dp), ("mat_sigma", _dp), ("mat_pec", _u8p),
        ("n_planes", C.c_int32),
        ("plane_body", _i32p), ("plane_mat", _i32p), ("plane_p0", _dp), ("plane_n0", _dp),
        ("n_edges", C.c_int32),
        ("edge_body", _i32p), ("edge_a0", _dp), ("edge_e0", _dp), ("edge_t0", _dp), ("edge_n0", _dp),
        ("edge_wedge_n", _dp),
        ("n_tiles", C.c_int32),
        ("tile_body", _i32p), ("tile_alpha", _i32p), ("tile_model", _u8p),
        ("tile_c0", _dp), ("tile_n0", _dp), ("tile_area", _dp), ("tile_S", _dp), ("tile_phase0", _dp),
        ("n_rays", C.c_int32),
        ("ray_nint", _u8p), ("ray_kind", _u8p), ("ray_pol", _u8p), ("ray_prim", _i32p),
        ("ray_q0", _dp),
        ("plane_facet", _dp), ("edge_zlim", _dp),
        ("tx_ant", _dp), ("rx_ant", _dp),
    ]


class TimeGrid(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_steps", C.c_int32)]


class FreqGrid(C.Structure):
    _fields_ = [("f_c", C.c_double), ("bandwidth", C.c_double), ("n_sub", C.c_int32)]


class RayOut(C.Structure):
    _fields_ = [("L", C.c_void_p), ("dop", C.c_void_p), ("aod_az", C.c_void_p), ("aod_el", C.c_void_p),
                ("aoa_az", C.c_void_p), ("aoa_el", C.c_void_p), ("gain", C.c_void_p), ("valid", C.c_void_p),
                ("in_bounds", C.c_void_p), ("first_out", C.c_void_p),
                ("q_pos", C.c_void_p), ("q_vel", C.c_void_p), ("q_acc", C.c_void_p), ("dop_rate", C.c_void_p)]


class TraceOpts(C.Structure):
    _fields_ = [("max_refl", C.c_int32), ("max_refl_diff", C.c_int32), ("scattering", C.c_int32),
                ("los", C.c_int32), ("double_diff", C.c_int32)]


class TraceInfo(C.Structure):
    _fields_ = [("n_paths", C.c_int32), ("n_los", C.c_int32), ("n_refl", C.c_int32), ("n_diff", C.c_int32),
                ("n_scat", C.c_int32), ("candidates", C.c_int64), ("geometric", C.c_int64)]


class RefreshOpts(C.Structure):
    _fields_ = [("threshold_db", C.c_double), ("max_steps", C.c_int32), ("min_steps", C.c_int32)]


class Bins(C.Structure):
    _fields_ = [("dop_lo", C.c_double), ("dop_step", C.c_double), ("delay_lo", C.c_double),
                ("delay_step", C.c_double), ("steps_per_bin", C.c_int32), ("n_dop", C.c_int32),
                ("n_delay", C.c_int32), ("in_bounds_only", C.c_int32)]


class PowerOut(C.Structure):
    _fields_ = [("pdfp", C.c_void_p), ("pdp", C.c_void_p), ("total", C.c_void_p)]


class Request(C.Structure):
    _fields_ = [("scene", C.c_uint32), ("n_rays", C.c_int32), ("tg", TimeGrid), ("fg", FreqGrid),
                ("precision", C.c_int32), ("H", C.c_void_p)]


class ReqStat(C.Structure):
    _fields_ = [("state", C.c_int32), ("t_arrive", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]


class ServingStats(C.Structure):
    _fields_ = [("batches", C.c_int64), ("batched_requests", C.c_int64), ("single_launches", C.c_int64),
                ("max_batch", C.c_int32), ("slots", C.c_int32), ("failed_nomem", C.c_int64)]


class Profile(C.Structure):
    _fields_ = [("ms", C.c_double * 4), ("launches", C.c_int64 * 4)]


class DrtError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {LIB.drt_strerror(status).decode()} ({status}): "
                         f"{LIB.drt_last_error().decode()}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libdrt.so not found at {LIB_PATH}: run paper_2205_00237_amd.build.build() "
                          "(or __graft_entry__.build()) first; there is no fallback path")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "drt_create": (C.c_int, [C.c_int, C.c_uint64, C.POINTER(vp)]),
        "drt_destroy": (C.c_int, [vp]),
        "drt_load_scene": (C.c_int, [vp, C.POINTER(SceneDesc), C.POINTER(C.c_uint32)]),
        "drt_unload_scene": (C.c_int, [vp, C.c_uint32]),
        "drt_extrapolate": (C.c_int, [vp, C.c_uint32, C.c_int32, C.POINTER(TimeGrid), C.c_double,
                                      C.c_int32, C.POINTER(RayOut), vp]),
        "drt_cfr": (C.c_int, [vp, C.c_uint32, C.c_int32, C.POINTER(TimeGrid), C.POINTER(FreqGrid),
                              C.c_int32, vp, vp]),
        "drt_cfr_noalloc": (C.c_int, [vp, C.c_uint32, C.c_int32, C.POINTER(TimeGrid), C.POINTER(FreqGrid),
                                      C.c_int32, vp, vp]),
        "drt_cfr_nufft": (C.c_int, [vp, C.c_uint32, C.c_int32, C.POINTER(TimeGrid), C.POINTER(FreqGrid),
                                    C.c_double, vp, vp]),
        "drt_trace": (C.c_int, [vp, C.c_uint32, C.c_double, C.POINTER(TraceOpts), C.POINTER(C.c_uint32),
                                C.POINTER(TraceInfo)]),
        "drt_segments": (C.c_int, [vp, C.c_uint32, C.POINTER(TimeGrid), C.c_double, C.POINTER(TraceOpts),
                                   C.POINTER(RefreshOpts), C.c_int32, vp, vp, vp, C.POINTER(C.c_int32)]),
        "drt_scene_rays": (C.c_int, [vp, C.c_uint32, C.c_int32, C.POINTER(C.c_int32), vp, vp, vp, vp]),
        "drt_power_profiles": (C.c_int, [vp, C.c_uint32, C.c_int32, C.POINTER(TimeGrid), C.c_double,
                                         C.c_int32, C.POINTER(Bins), C.POINTER(PowerOut), vp]),
        "drt_submit": (C.c_int, [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]),
        "drt_poll": (C.c_int, [vp, C.c_uint64, C.POINTER(ReqStat)]),
        "drt_serving_stats_get": (C.c_int, [vp, C.POINTER(ServingStats)]),
        "drt_now": (C.c_double, []),
        "drt_strerror": (C.c_char_p, [C.c_int]),
        "drt_last_error": (C.c_char_p, []),
        "drt_profile_enable": (C.c_int, [vp, C.c_int]),
        "drt_profile_read": (C.c_int, [vp, C.POINTER(Profile), C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def _check(status, where):
    if status != DRT_OK:
        raise DrtError(status, where)


def _arr(a, dtype, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    if shape is not None:
        a = a.reshape(shape)
    return a


def scene_desc(scene, ray_q0=None):
    """Build a drt_scene_desc over numpy copies of a scene dictionary.  Returns (desc, keep)
    where `keep` holds the arrays that the pointers reference."""
    keep = {}

    def p(key, dtype, ctype):
        a = _arr(scene[key], dtype)
        keep[key] = a
        return a.ctypes.data_as(C.POINTER(ctype)) if a.size else C.POINTER(ctype)()

    d = SceneDesc()
    d.t0 = float(scene.get("t0", 0.0))
    for k in ("tx_p", "tx_v", "tx_a", "rx_p", "rx_v", "rx_a"):
        setattr(d, k, (C.c_double * 3)(*[float(x) for x in np.asarray(scene[k]).reshape(3)]))
    d.n_bodies = int(np.asarray(scene["body_w0"]).shape[0])
    for k in ("body_O0", "body_v0", "body_a", "body_axis", "body_w0", "body_wdot"):
        setattr(d, k, p(k, np.float64, C.c_double))
    d.n_mat = int(np.asarray(scene["mat_eps_r"]).shape[0])
    d.mat_eps_r = p("mat_eps_r", np.float64, C.c_double)
    d.mat_sigma = p("mat_sigma", np.float64, C.c_double)
    d.mat_pec = p("mat_pec", np.uint8, C.c_uint8)
    d.n_planes = int(np.asarray(scene["plane_body"]).shape[0])
    d.plane_body = p("plane_body", np.int32, C.c_int32)
    d.plane_mat = p("plane_mat", np.int32, C.c_int32)
    d.plane_p0 = p("plane_p0", np.float64, C.c_double)
    d.plane_n0 = p("plane_n0", np.float64, C.c_double)
    d.n_edges = int(np.asarray(scene["edge_body"]).shape[0])
    d.edge_body = p("edge_body", np.int32, C.c_int32)
    for k in ("edge_a0", "edge_e0", "edge_t0", "edge_n0", "edge_wedge_n"):
        setattr(d, k, p(k, np.float64, C.c_double))
    d.n_tiles = int(np.asarray(scene["tile_body"]).shape[0])
    d.tile_body = p("tile_body", np.int32, C.c_int32)
    d.tile_alpha = p("tile_alpha", np.int32, C.c_int32)
    d.tile_model = p("tile_model", np.uint8, C.c_uint8)
    for k in ("tile_c0", "tile_n0", "tile_area", "tile_S", "tile_phase0"):
        setattr(d, k, p(k, np.float64, C.c_double))
    d.n_rays = int(np.asarray(scene["ray_nint"]).shape[0])
    d.ray_nint = p("ray_nint", np.uint8, C.c_uint8)
    d.ray_kind = p("ray_kind", np.uint8, C.c_uint8)
    d.ray_pol = p("ray_pol", np.uint8, C.c_uint8)
    d.ray_prim = p("ray_prim", np.int32, C.c_int32)
    if ray_q0 is not None:
        q = _arr(ray_q0, np.float64, (d.n_rays, 4, 3))
        keep["ray_q0"] = q
        d.ray_q0 = q.ctypes.data_as(_dp)
    if "plane_facet" in scene and d.n_planes:
        f = _arr(scene["plane_facet"], np.float64, (d.n_planes, 3, 3))
        keep["plane_facet"] = f
        d.plane_facet = f.ctypes.data_as(_dp)
    if "edge_zlim" in scene and d.n_edges:
        z = _arr(scene["edge_zlim"], np.float64, (d.n_edges, 2))
        keep["edge_zlim"] = z
        d.edge_zlim = z.ctypes.data_as(_dp)
    for k in ("tx_ant", "rx_ant"):        # the library checks that both or neither are given
        if k in scene:
            a = _arr(scene[k], np.float64, (4,))
            keep[k] = a
            setattr(d, k, a.ctypes.data_as(_dp))
    return d, keep


# ----------------------------------------------------------------------------- C names

def drt_create(device=0, hbm_cap_bytes=0):
    ctx = C.c_void_p()
    _check(LIB.drt_create(int(device), int(hbm_cap_bytes), C.byref(ctx)), "drt_create")
    return ctx


def drt_destroy(ctx):
    _check(LIB.drt_destroy(ctx), "drt_destroy")


def drt_load_scene(ctx, scene, ray_q0=None):
    d, keep = scene_desc(scene, ray_q0)
    sid = C.c_uint32()
    _check(LIB.drt_load_scene(ctx, C.byref(d), C.byref(sid)), "drt_load_scene")
    return sid.value


def drt_unload_scene(ctx, sid):
    _check(LIB.drt_unload_scene(ctx, int(sid)), "drt_unload_scene")


def drt_extrapolate(ctx, sid, n_rays, dt, n_steps, f_c, precision, out_ptrs, stream=0):
    """out_ptrs: dict with any of L, dop, aod_az, aod_el, aoa_az, aoa_el, gain, valid, in_bounds,
    first_out, q_pos, q_vel, q_acc, dop_rate -> device pointer."""
    tg = TimeGrid(float(dt), int(n_steps))
    o = RayOut(**{k: int(v) for k, v in out_ptrs.items() if v})
    _check(LIB.drt_extrapolate(ctx, int(sid), int(n_rays), C.byref(tg), float(f_c), int(precision),
                               C.byref(o), C.c_void_p(int(stream))), "drt_extrapolate")


def drt_trace(ctx, sid, t, max_refl, max_refl_diff, scattering, los, double_diff=False):
    """Returns (new scene id, info dict)."""
    o = TraceOpts(int(max_refl), int(max_refl_diff), int(bool(scattering)), int(bool(los)), int(bool(double_diff)))
    new, info = C.c_uint32(), TraceInfo()
    _check(LIB.drt_trace(ctx, int(sid), float(t), C.byref(o), C.byref(new), C.byref(info)), "drt_trace")
    return new.value, {k: getattr(info, k) for k, _ in TraceInfo._fields_}


def drt_segments(ctx, sid, dt, n_steps, f_c, trace_opts, threshold_db, max_steps, min_steps=1,
                 max_segments=4096):
    """[(first instant, length, scene id)] of the multipath lifetimes."""
    import numpy as np
    o = TraceOpts(int(trace_opts.get("max_refl", 2)), int(trace_opts.get("max_refl_diff", 1)),
                  int(bool(trace_opts.get("scattering", True))), int(bool(trace_opts.get("los", True))),
                  int(bool(trace_opts.get("double_diff", False))))
    r = RefreshOpts(float(threshold_db), int(max_steps), int(min_steps))
    start = np.zeros(max_segments, np.int32)
    length = np.zeros(max_segments, np.int32)
    scene = np.zeros(max_segments, np.uint32)
    n = C.c_int32()
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    _check(LIB.drt_segments(ctx, int(sid), C.byref(TimeGrid(float(dt), int(n_steps))), float(f_c), C.byref(o),
                            C.byref(r), int(max_segments), ptr(start), ptr(length), ptr(scene), C.byref(n)),
           "drt_segments")
    return [(int(start[k]), int(length[k]), int(scene[k])) for k in range(n.value)]


def drt_scene_rays(ctx, sid):
    """(nint [n], kind [n][4], prim [n][4], pol [n][4]) numpy arrays of a resident scene."""
    import numpy as np
    n = C.c_int32()
    _check(LIB.drt_scene_rays(ctx, int(sid), 0, C.byref(n), None, None, None, None), "drt_scene_rays")
    nint = np.zeros(n.value, np.uint8)
    kind = np.zeros((n.value, 4), np.uint8)
    prim = np.zeros((n.value, 4), np.int32)
    pol = np.zeros((n.value, 4), np.uint8)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    _check(LIB.drt_scene_rays(ctx, int(sid), n.value, C.byref(n), ptr(nint), ptr(kind), ptr(prim), ptr(pol)),
           "drt_scene_rays")
    return nint, kind, prim, pol


def drt_power_profiles(ctx, sid, n_rays, dt, n_steps, f_c, precision, bins, out_ptrs, stream=0):
    """bins: dict of the drt_bins fields; out_ptrs: dict with any of pdfp, pdp, total -> device pointer."""
    tg = TimeGrid(float(dt), int(n_steps))
    b = Bins(float(bins["dop_lo"]), float(bins["dop_step"]), float(bins["delay_lo"]),
             float(bins["delay_step"]), int(bins["steps_per_bin"]), int(bins["n_dop"]),
             int(bins["n_delay"]), int(bins.get("in_bounds_only", 0)))
    o = PowerOut(**{k: int(v) for k, v in out_ptrs.items() if v})
    _check(LIB.drt_power_profiles(ctx, int(sid), int(n_rays), C.byref(tg), float(f_c), int(precision),
                                  C.byref(b), C.byref(o), C.c_void_p(int(stream))), "drt_power_profiles")


def drt_cfr(ctx, sid, n_rays, dt, n_steps, f_c, bandwidth, n_sub, precision, H_ptr, stream=0):
    tg = TimeGrid(float(dt), int(n_steps))
    fg = FreqGrid(float(f_c), float(bandwidth), int(n_sub))
    _check(LIB.drt_cfr(ctx, int(sid), int(n_rays), C.byref(tg), C.byref(fg), int(precision),
                       C.c_void_p(int(H_ptr)), C.c_void_p(int(stream))), "drt_cfr")


def drt_cfr_noalloc(ctx, sid, n_rays, dt, n_steps, f_c, bandwidth, n_sub, precision, H_ptr, stream=0):
    tg = TimeGrid(float(dt), int(n_steps))
    fg = FreqGrid(float(f_c), float(bandwidth), int(n_sub))
    _check(LIB.drt_cfr_noalloc(ctx, int(sid), int(n_rays), C.byref(tg), C.byref(fg), int(precision),
                               C.c_void_p(int(H_ptr)), C.c_void_p(int(stream))), "drt_cfr_noalloc")


def drt_cfr_nufft(ctx, sid, n_rays, dt, n_steps, f_c, bandwidth, n_sub, eps, H_ptr, stream=0):
    tg = TimeGrid(float(dt), int(n_steps))
    fg = FreqGrid(float(f_c), float(bandwidth), int(n_sub))
    _check(LIB.drt_cfr_nufft(ctx, int(sid), int(n_rays), C.byref(tg), C.byref(fg), float(eps),
                             C.c_void_p(int(H_ptr)), C.c_void_p(int(stream))), "drt_cfr_nufft")


def drt_submit(ctx, sid, n_rays, dt, n_steps, f_c, bandwidth, n_sub, precision, H_ptr):
    r = Request(int(sid), int(n_rays), TimeGrid(float(dt), int(n_steps)),
                FreqGrid(float(f_c), float(bandwidth), int(n_sub)), int(precision), C.c_void_p(int(H_ptr)))
    t = C.c_uint64()
    _check(LIB.drt_submit(ctx, C.byref(r), C.byref(t)), "drt_submit")
    return t.value


def drt_poll(ctx, ticket):
    st = ReqStat()
    _check(LIB.drt_poll(ctx, int(ticket), C.byref(st)), "drt_poll")
    return st.state, st.t_arrive, st.t_admit, st.t_done


def drt_serving_stats_get(ctx):
    st = ServingStats()
    _check(LIB.drt_serving_stats_get(ctx, C.byref(st)), "drt_serving_stats_get")
    return {k: getattr(st, k) for k, _ in ServingStats._fields_}


def drt_now():
    return LIB.drt_now()


def drt_profile_enable(ctx, on):
    _check(LIB.drt_profile_enable(ctx, int(bool(on))), "drt_profile_enable")


def drt_profile_read(ctx, reset=True):
    """{kernel name: (total ms, launches)} since the last reset."""
    p = Profile()
    _check(LIB.drt_profile_read(ctx, C.byref(p), int(bool(reset))), "drt_profile_read")
    return {k: (p.ms[i], p.launches[i]) for i, k in enumerate(KERNELS)}

