"""MI355X (gfx950) tracking hot path of IMU-seeded, median-filtered,
regularised KinectFusion ICP (Giancola et al. 2018).

A thin ctypes binding over ``_lib/libicp_mi355x.so`` whose functions carry the
names of the C ABI in ``include/icp.h``.  It only marshals arguments: device
memory comes from torch tensors (``data_ptr()``), the stream is torch's current
HIP stream, and every step of the registration runs in the library's kernels.
There is no fallback: if the library is missing or no GPU is present, the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libicp_mi355x.so")

ICP_ABI_VERSION = 5
MAX_LEVELS = 4
HIST_BINS = 1024
OK, EINVAL, ENOMEM, EDEVICE, ETIMEOUT = 0, -1, -2, -3, -4
LEVEL_OK, TOO_FEW_CORR, ILL_COND, NONFINITE = range(4)
LAMBDA_CONST, LAMBDA_C_OVER_SQRT_N, LAMBDA_C_OVER_N, LAMBDA_C_OVER_N2 = range(4)
PX_INVALID_LIVE, PX_BEHIND, PX_OUTSIDE, PX_INVALID_MODEL, PX_FAR, PX_ANGLE, PX_GATED = range(7)

# symbols of include/icp.h
EXPORTS = (
    "icp_abi_version", "icp_strerror", "icp_last_error", "icp_ctx_create", "icp_ctx_destroy",
    "icp_ctx_workspace_bytes", "icp_workspace_bytes", "icp_params_default", "icp_validate_problem", "icp_register",
    "icp_register_async", "icp_register_noalloc", "icp_register_batch", "icp_register_batch_async", "icp_ctx_set_timing", "icp_ctx_get_timing", "icp_ctx_set_graphs",
    "icp_stage_prepare", "icp_stage_level",
    "icp_stage_associate", "icp_stage_moments", "icp_stage_single_pass", "icp_stage_solve", "icp_live_maps", "icp_autotune_tiles",
    "icp_server_config_default", "icp_server_clock", "icp_server_create", "icp_server_destroy",
    "icp_server_last_error", "icp_server_open_stream", "icp_server_close_stream", "icp_server_submit",
    "icp_server_poll", "icp_server_get_counters", "icp_tsdf_bytes", "icp_tsdf_brick_bytes", "icp_tsdf_reset",
    "icp_tsdf_integrate", "icp_tsdf_raycast",
)


class IcpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"icp error {code}: {msg}")
        self.code = code


class icp_intrinsics(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class icp_tsdf(C.Structure):
    _fields_ = [("voxels", C.c_void_p), ("dim", C.c_int32), ("pad_", C.c_int32), ("size", C.c_double),
                ("origin", C.c_double * 3), ("mu", C.c_double), ("max_weight", C.c_double), ("bricks", C.c_void_p)]


class icp_params(C.Structure):
    _fields_ = [
        ("levels", C.c_int32), ("iters", C.c_int32 * MAX_LEVELS), ("dist_max", C.c_double),
        ("cos_angle_max", C.c_double), ("band_beta", C.c_double), ("use_median_filter", C.c_int32),
        ("use_imu_seed", C.c_int32), ("lambda_mode", C.c_int32), ("lambda_c", C.c_double),
        ("min_corr", C.c_int32), ("ill_cond_eps", C.c_double), ("converge_window", C.c_int32),
        ("reduce_mode", C.c_int32), ("pass_mode", C.c_int32), ("tile_px", C.c_int32 * MAX_LEVELS),
        ("depth_filter", C.c_int32), ("filter_radius", C.c_int32), ("filter_sigma_px", C.c_double),
        ("filter_sigma_m", C.c_double), ("normal_mode", C.c_int32), ("normal_radius", C.c_int32),
        ("anchor_to_imu", C.c_int32), ("reserved", C.c_int32),
    ]


class icp_level_stats(C.Structure):
    _fields_ = [("iters_run", C.c_int32), ("status", C.c_int32), ("n_gated", C.c_int64), ("n_kept", C.c_int64),
                ("k_med", C.c_int32), ("pad", C.c_int32), ("rmse", C.c_double)]


class icp_stats(C.Structure):
    _fields_ = [("level", icp_level_stats * MAX_LEVELS), ("status", C.c_int32), ("iters_total", C.c_int32)]


class icp_problem(C.Structure):
    _fields_ = [("live_depth", C.c_void_p), ("model_vtx", C.c_void_p), ("model_nrm", C.c_void_p),
                ("W", C.c_int32), ("H", C.c_int32), ("K", icp_intrinsics), ("imu_R", C.c_double * 9),
                ("init_pose", C.c_double * 16)]


class icp_kernel_time(C.Structure):
    _fields_ = [("total_ms", C.c_double), ("launches", C.c_int64), ("pixels", C.c_int64)]


TIME_FRONT_END, TIME_PASS1, TIME_BAND, TIME_PASS2, TIME_SOLVE = range(5)
TIME_KINDS = 5


class icp_result(C.Structure):
    _fields_ = [("pose", C.c_double * 16), ("stats", icp_stats)]


class icp_server_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_batch", C.c_int32), ("slots", C.c_int32), ("use_graphs", C.c_int32),
                ("frames_in_flight", C.c_int32), ("pad", C.c_int32), ("hbm_budget_bytes", C.c_size_t),
                ("params", icp_params)]


class icp_server_result(C.Structure):
    _fields_ = [("stream_id", C.c_int32), ("status", C.c_int32), ("frame", C.c_uint64), ("tag", C.c_uint64),
                ("pose_rel", C.c_double * 16), ("pose_world", C.c_double * 16), ("stats", icp_stats),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("batch_size", C.c_int32), ("pad", C.c_int32)]


class icp_server_counters(C.Structure):
    _fields_ = [("batches", C.c_uint64), ("frames", C.c_uint64), ("registrations", C.c_uint64),
                ("busy_s", C.c_double), ("resident_bytes", C.c_size_t), ("workspace_bytes", C.c_size_t),
                ("streams_open", C.c_int32), ("pad", C.c_int32), ("workspace_held_bytes", C.c_size_t)]


_lib = None


def lib():
    """Load the HIP library (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads torch's HIP runtime first)
        if not os.path.exists(LIB_PATH):
            # nothing built yet: compile it in-tree (hipcc for gfx950); a failed
            # build is an error, there is no other implementation to fall back on
            from . import build as _build
            try:
                _build.build()
            except Exception as e:
                raise ImportError(f"{LIB_PATH} is not built and building it failed: {e}") from e
        L = C.CDLL(LIB_PATH)
        P, I, D, Z = C.c_void_p, C.c_int, C.c_double, C.c_size_t
        sig = {
            "icp_abi_version": (I, []),
            "icp_strerror": (C.c_char_p, [I]),
            "icp_last_error": (C.c_char_p, [P]),
            "icp_ctx_create": (I, [I, Z, C.POINTER(P)]),
            "icp_ctx_destroy": (None, [P]),
            "icp_ctx_workspace_bytes": (Z, [P]),
            "icp_workspace_bytes": (Z, [I, P, P, I]),
            "icp_params_default": (None, [C.POINTER(icp_params)]),
            "icp_validate_problem": (I, [C.POINTER(icp_problem), C.POINTER(icp_params), C.c_char_p, Z]),
            "icp_register": (I, [P, P, I, I, P, P, C.POINTER(icp_intrinsics), P, P, C.POINTER(icp_params), P,
                                 C.POINTER(icp_stats), P]),
            "icp_register_async": (I, [P, P, I, I, P, P, C.POINTER(icp_intrinsics), P, P,
                                       C.POINTER(icp_params), P, P]),
            "icp_register_noalloc": (I, [P, I, I, P, P, C.POINTER(icp_intrinsics), P, P, C.POINTER(icp_params), P,
                                         P]),
            "icp_register_batch": (I, [P, I, P, C.POINTER(icp_params), P, P]),
            "icp_register_batch_async": (I, [P, I, P, C.POINTER(icp_params), P, P]),
            "icp_ctx_set_timing": (I, [P, I]),
            "icp_ctx_set_graphs": (I, [P, I]),
            "icp_ctx_get_timing": (I, [P, P]),
            "icp_stage_prepare": (I, [P, P, I, I, P, P, C.POINTER(icp_intrinsics), I, P, P]),
            "icp_stage_level": (I, [P, I, P, P, P, P, P, P]),
            "icp_stage_associate": (I, [P, I, P, C.POINTER(icp_params), P, P, P, P, P]),
            "icp_stage_moments": (I, [P, I, P, C.POINTER(icp_params), I, I, P, P, P]),
            "icp_stage_solve": (I, [P, P, C.c_int64, P, C.POINTER(icp_params), P, P, P, P]),
            "icp_stage_single_pass": (I, [P, I, P, C.POINTER(icp_params), I, I, I, P, P, C.POINTER(I), P, P, P]),
            "icp_live_maps": (I, [P, P, I, I, C.POINTER(icp_intrinsics), P, P, P]),
            "icp_autotune_tiles": (I, [P, I, P, C.POINTER(icp_params), I, P, C.POINTER(D), P]),
            "icp_tsdf_bytes": (Z, [I]),
            "icp_tsdf_brick_bytes": (Z, [I]),
            "icp_tsdf_reset": (I, [P, C.POINTER(icp_tsdf), P]),
            "icp_tsdf_integrate": (I, [P, C.POINTER(icp_tsdf), P, I, I, C.POINTER(icp_intrinsics), P, P]),
            "icp_tsdf_raycast": (I, [P, C.POINTER(icp_tsdf), I, I, C.POINTER(icp_intrinsics), P, D, D, P, P, P]),
            "icp_server_config_default": (None, [C.POINTER(icp_server_config)]),
            "icp_server_clock": (D, []),
            "icp_server_create": (I, [C.POINTER(icp_server_config), C.POINTER(P)]),
            "icp_server_destroy": (None, [P]),
            "icp_server_last_error": (C.c_char_p, [P]),
            "icp_server_open_stream": (I, [P, I, I, C.POINTER(icp_intrinsics), C.POINTER(I)]),
            "icp_server_close_stream": (I, [P, I]),
            "icp_server_submit": (I, [P, I, P, P, C.c_uint64, D]),
            "icp_server_poll": (I, [P, P, I, I]),
            "icp_server_get_counters": (I, [P, C.POINTER(icp_server_counters)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.icp_abi_version() != ICP_ABI_VERSION:
            raise ImportError("libicp_mi355x ABI version mismatch")
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers

def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype_name, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device (HIP) tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"{name} must be {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _maps_match(live_depth, model_vtx, model_nrm):
    """(H, W) of a problem after checking that the model maps are (H, W, 3)
    like the depth (the library reads H*W*3 floats from each)."""
    if live_depth.dim() != 2:
        raise ValueError(f"live_depth must be (H, W), got {tuple(live_depth.shape)}")
    H, W = live_depth.shape
    for name, t in (("model_vtx", model_vtx), ("model_nrm", model_nrm)):
        if tuple(t.shape) != (H, W, 3):
            raise ValueError(f"{name} must have shape ({H}, {W}, 3), got {tuple(t.shape)}")
    return H, W


def _f64(a, n, name):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if a.size != n:
        raise ValueError(f"{name} must have {n} values")
    return a


def _np_ptr(a):
    """Address of a numpy array's data (the caller keeps `a` alive for the call)."""
    return C.c_void_p(a.ctypes.data)


def _check(ctx, rc):
    if rc != OK:
        L = lib()
        msg = L.icp_last_error(ctx.handle if isinstance(ctx, Context) else ctx)
        raise IcpError(rc, (msg or L.icp_strerror(rc)).decode())


def stats_to_dict(st, levels=MAX_LEVELS):
    return dict(status=st.status, iters_total=st.iters_total,
                levels=[dict(iters_run=s.iters_run, status=s.status, n_gated=s.n_gated, n_kept=s.n_kept,
                             k_med=s.k_med, rmse=s.rmse) for s in st.level[:levels]])


# ---------------------------------------------------------------- API

def icp_params_default(**over):
    p = icp_params()
    lib().icp_params_default(C.byref(p))
    for k, v in over.items():
        if k in ("iters", "tile_px"):
            arr = getattr(p, k)
            for j in range(MAX_LEVELS):
                arr[j] = int(v[j]) if j < len(v) else 0
        else:
            setattr(p, k, v)
    return p


def icp_validate_problem(W, H, K, imu_R, init_pose, params=None):
    """Host-only check of a problem's sizes, intrinsics and rotations and of
    the parameters (the checks icp_register makes); returns (code, message).
    The map pointers are placeholders: they are compared with NULL only."""
    p = params if params is not None else icp_params_default()
    q = icp_problem()
    q.live_depth = q.model_vtx = q.model_nrm = 256
    q.W, q.H = int(W), int(H)
    q.K = make_intrinsics(K)
    q.imu_R[:] = [float(v) for v in _f64(imu_R, 9, "imu_R")]
    q.init_pose[:] = [float(v) for v in _f64(init_pose, 16, "init_pose")]
    buf = C.create_string_buffer(256)
    rc = lib().icp_validate_problem(C.byref(q), C.byref(p), buf, 256)
    return rc, buf.value.decode()


def make_intrinsics(K):
    fx, fy, cx, cy = (float(v) for v in K)
    return icp_intrinsics(fx, fy, cx, cy)


class Context:
    """An icp_ctx on one HIP device (created lazily by icp_ctx_create)."""

    def __init__(self, handle, device):
        self.handle = handle
        self.device = device

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.icp_ctx_destroy(self.handle)
            self.handle = None

    def workspace_bytes(self):
        return int(lib().icp_ctx_workspace_bytes(self.handle))


def icp_ctx_create(device=0, hbm_budget_bytes=0):
    h = C.c_void_p()
    rc = lib().icp_ctx_create(int(device), int(hbm_budget_bytes), C.byref(h))
    if rc != OK:
        raise IcpError(rc, lib().icp_strerror(rc).decode())
    return Context(h, device)


def icp_workspace_bytes(sizes, levels=3):
    W = np.array([s[0] for s in sizes], np.int32)
    H = np.array([s[1] for s in sizes], np.int32)
    return int(lib().icp_workspace_bytes(len(sizes), _np_ptr(W), _np_ptr(H), levels))


def icp_register(ctx, live_depth, model_vtx, model_nrm, K, imu_R, init_pose, params=None, stream=None):
    """Register one frame; returns (4x4 pose ndarray, stats dict)."""
    H, W = _maps_match(live_depth, model_vtx, model_nrm)
    p = params if params is not None else icp_params_default()
    Kc = make_intrinsics(K)
    R = _f64(imu_R, 9, "imu_R")
    T0 = _f64(init_pose, 16, "init_pose")
    pose = np.zeros(16)
    st = icp_stats()
    rc = lib().icp_register(ctx.handle, _dev_ptr(live_depth, "float32", "live_depth"), W, H,
                            _dev_ptr(model_vtx, "float32", "model_vtx"), _dev_ptr(model_nrm, "float32", "model_nrm"),
                            C.byref(Kc), _np_ptr(R), _np_ptr(T0), C.byref(p), _np_ptr(pose), C.byref(st),
                            _stream(stream))
    _check(ctx, rc)
    return pose.reshape(4, 4), stats_to_dict(st, p.levels)


def icp_register_async(ctx, live_depth, model_vtx, model_nrm, K, imu_R, init_pose, result_dev, params=None,
                       stream=None):
    """Asynchronous register; result_dev is a uint8 device tensor of at least
    sizeof(icp_result) bytes that receives the icp_result."""
    res_ptr = _dev_ptr(result_dev, "uint8", "result_dev")
    H, W = _maps_match(live_depth, model_vtx, model_nrm)
    p = params if params is not None else icp_params_default()
    if result_dev.numel() * result_dev.element_size() < C.sizeof(icp_result):
        raise ValueError("result_dev too small")
    Kc = make_intrinsics(K)
    R = _f64(imu_R, 9, "imu_R")
    T0 = _f64(init_pose, 16, "init_pose")
    rc = lib().icp_register_async(ctx.handle, _dev_ptr(live_depth, "float32", "live_depth"), W, H,
                                  _dev_ptr(model_vtx, "float32", "model_vtx"),
                                  _dev_ptr(model_nrm, "float32", "model_nrm"), C.byref(Kc), _np_ptr(R),
                                  _np_ptr(T0), C.byref(p), res_ptr, _stream(stream))
    _check(ctx, rc)


def icp_register_noalloc(live_depth, model_vtx, model_nrm, K, imu_R, init_pose, result_dev, params=None,
                         stream=None):
    """icp_register_noalloc: the registration of icp_register_async with no
    context and no device allocation (a static 32 MiB device array per GPU);
    result_dev is a uint8 device tensor of at least sizeof(icp_result) bytes.
    Raises IcpError (no context, so the message is the code's)."""
    res_ptr = _dev_ptr(result_dev, "uint8", "result_dev")
    H, W = _maps_match(live_depth, model_vtx, model_nrm)
    p = params if params is not None else icp_params_default()
    if result_dev.numel() * result_dev.element_size() < C.sizeof(icp_result):
        raise ValueError("result_dev too small")
    Kc = make_intrinsics(K)
    R = _f64(imu_R, 9, "imu_R")
    T0 = _f64(init_pose, 16, "init_pose")
    rc = lib().icp_register_noalloc(_dev_ptr(live_depth, "float32", "live_depth"), W, H,
                                    _dev_ptr(model_vtx, "float32", "model_vtx"),
                                    _dev_ptr(model_nrm, "float32", "model_nrm"), C.byref(Kc), _np_ptr(R),
                                    _np_ptr(T0), C.byref(p), res_ptr, _stream(stream))
    if rc != OK:
        raise IcpError(rc, lib().icp_strerror(rc).decode())


def result_from_bytes(buf):
    """Decode an icp_result from host bytes: (4x4 pose, stats dict)."""
    r = icp_result.from_buffer_copy(bytes(buf))
    return np.array(r.pose[:]).reshape(4, 4), stats_to_dict(r.stats)


class ProblemArray:
    """A ctypes icp_problem array built once from problem dicts, reusable in
    icp_register_batch while its tensors stay alive."""

    def __init__(self, problems):
        self.n = len(problems)
        self.arr = _problem_array(problems)
        self.keep = [(q["live_depth"], q["model_vtx"], q["model_nrm"]) for q in problems]


def _problem_array(problems):
    n = len(problems)
    arr = (icp_problem * n)()
    for i, q in enumerate(problems):
        d = q["live_depth"]
        H, W = _maps_match(d, q["model_vtx"], q["model_nrm"])
        a = arr[i]
        a.live_depth = _dev_ptr(d, "float32", "live_depth").value
        a.model_vtx = _dev_ptr(q["model_vtx"], "float32", "model_vtx").value
        a.model_nrm = _dev_ptr(q["model_nrm"], "float32", "model_nrm").value
        a.W, a.H = W, H
        a.K = make_intrinsics(q["K"])
        a.imu_R[:] = list(_f64(q["imu_R"], 9, "imu_R"))
        a.init_pose[:] = list(_f64(q["init_pose"], 16, "init_pose"))
    return arr


def icp_register_batch(ctx, problems, params=None, stream=None):
    """problems: a ProblemArray or a sequence of dicts with live_depth,
    model_vtx, model_nrm (device tensors), K, imu_R, init_pose.  Returns a
    list of (pose, stats)."""
    p = params if params is not None else icp_params_default()
    if isinstance(problems, ProblemArray):
        n, arr = problems.n, problems.arr
    else:
        n, arr = len(problems), _problem_array(problems)
    res = (icp_result * n)()
    rc = lib().icp_register_batch(ctx.handle, n, C.cast(arr, C.c_void_p), C.byref(p), C.cast(res, C.c_void_p),
                                  _stream(stream))
    _check(ctx, rc)
    return [(np.array(r.pose[:]).reshape(4, 4), stats_to_dict(r.stats, p.levels)) for r in res]


def icp_register_batch_async(ctx, problems, results_dev, params=None, stream=None):
    """Queue a batched registration on the stream and return: results_dev is
    a uint8 device tensor of at least n * sizeof(icp_result) bytes that the
    stream fills (decode with results_from_bytes once it has finished).  The
    problems' tensors and results_dev must stay alive until then."""
    res_ptr = _dev_ptr(results_dev, "uint8", "results_dev")
    p = params if params is not None else icp_params_default()
    if isinstance(problems, ProblemArray):
        n, arr = problems.n, problems.arr
    else:
        n, arr = len(problems), _problem_array(problems)
    if results_dev.numel() * results_dev.element_size() < n * C.sizeof(icp_result):
        raise ValueError("results_dev too small")
    rc = lib().icp_register_batch_async(ctx.handle, n, C.cast(arr, C.c_void_p), C.byref(p),
                                        res_ptr, _stream(stream))
    _check(ctx, rc)


def results_from_bytes(buf, n, levels=MAX_LEVELS):
    """Decode n consecutive icp_result records from host bytes: [(pose, stats)]."""
    arr = (icp_result * n).from_buffer_copy(bytes(buf)[:n * C.sizeof(icp_result)])
    return [(np.array(r.pose[:]).reshape(4, 4), stats_to_dict(r.stats, levels)) for r in arr]


def icp_autotune_tiles(ctx, problems, params=None, reps=3, stream=None):
    """Per-level tile sizes picked by timing the batch (see include/icp.h);
    returns (tile_px tuple of MAX_LEVELS, ms per registration of the batch)."""
    p = params if params is not None else icp_params_default()
    if isinstance(problems, ProblemArray):
        n, arr = problems.n, problems.arr
    else:
        n, arr = len(problems), _problem_array(problems)
    out = (C.c_int32 * MAX_LEVELS)()
    ms = C.c_double(0.0)
    rc = lib().icp_autotune_tiles(ctx.handle, n, C.cast(arr, C.c_void_p), C.byref(p), int(reps),
                                  C.cast(out, C.c_void_p), C.byref(ms), _stream(stream))
    _check(ctx, rc)
    return tuple(out[:]), ms.value


def icp_ctx_set_graphs(ctx, enable):
    _check(ctx, lib().icp_ctx_set_graphs(ctx.handle, 1 if enable else 0))


def icp_ctx_set_timing(ctx, enable):
    _check(ctx, lib().icp_ctx_set_timing(ctx.handle, 1 if enable else 0))


def icp_ctx_get_timing(ctx):
    """{kind: dict(total_ms, launches, pixels)} per kernel kind."""
    arr = (icp_kernel_time * TIME_KINDS)()
    _check(ctx, lib().icp_ctx_get_timing(ctx.handle, C.cast(arr, C.c_void_p)))
    names = ("front_end", "pass1", "band", "pass2", "solve")
    return {names[k]: dict(total_ms=arr[k].total_ms, launches=arr[k].launches, pixels=arr[k].pixels)
            for k in range(TIME_KINDS)}


# ---------------------------------------------------------------- stage access

def icp_stage_prepare(ctx, live_depth, model_vtx, model_nrm, K, levels=3, params=None, stream=None):
    H, W = _maps_match(live_depth, model_vtx, model_nrm)
    Kc = make_intrinsics(K)
    prm = C.byref(params) if params is not None else None
    rc = lib().icp_stage_prepare(ctx.handle, _dev_ptr(live_depth, "float32", "live_depth"), W, H,
                                 _dev_ptr(model_vtx, "float32", "model_vtx"),
                                 _dev_ptr(model_nrm, "float32", "model_nrm"), C.byref(Kc), levels, prm,
                                 _stream(stream))
    _check(ctx, rc)


def icp_stage_level(ctx, level, H, W, stream=None):
    """Level maps as device tensors: depth (H_l, W_l), live vertex and normal
    (3, H_l, W_l) planes, model vertex and normal (H_l, W_l, 3) interleaved."""
    import torch
    Hl, Wl = H >> level, W >> level
    dev = torch.device("cuda", ctx.device)
    D = torch.empty((Hl, Wl), dtype=torch.float32, device=dev)
    maps = [torch.empty((3, Hl, Wl), dtype=torch.float32, device=dev) for _ in range(2)]
    maps += [torch.empty((Hl, Wl, 3), dtype=torch.float32, device=dev) for _ in range(2)]
    rc = lib().icp_stage_level(ctx.handle, level, C.c_void_p(D.data_ptr()),
                               *[C.c_void_p(m.data_ptr()) for m in maps], _stream(stream))
    _check(ctx, rc)
    return D, maps[0], maps[1], maps[2], maps[3]


def icp_stage_associate(ctx, level, pose, H, W, params=None, stream=None):
    """Per-pixel codes and bins (device tensors), histogram and band (host)."""
    import torch
    p = params if params is not None else icp_params_default()
    Hl, Wl = H >> level, W >> level
    dev = torch.device("cuda", ctx.device)
    code = torch.empty((Hl, Wl), dtype=torch.uint8, device=dev)
    bins = torch.empty((Hl, Wl), dtype=torch.int32, device=dev)
    hist = np.zeros(HIST_BINS, np.uint32)
    band = np.zeros(4, np.int64)
    P12 = _f64(np.asarray(pose, dtype=np.float64)[:3, :4], 12, "pose")
    rc = lib().icp_stage_associate(ctx.handle, level, _np_ptr(P12), C.byref(p), C.c_void_p(code.data_ptr()),
                                   C.c_void_p(bins.data_ptr()), _np_ptr(hist), _np_ptr(band), _stream(stream))
    _check(ctx, rc)
    return code, bins, hist, band


def icp_stage_moments(ctx, level, pose, k_lo, k_hi, params=None, stream=None):
    p = params if params is not None else icp_params_default()
    P12 = _f64(np.asarray(pose, dtype=np.float64)[:3, :4], 12, "pose")
    M = np.zeros(28)
    n = np.zeros(1, np.int64)
    rc = lib().icp_stage_moments(ctx.handle, level, _np_ptr(P12), C.byref(p), int(k_lo), int(k_hi), _np_ptr(M),
                                 _np_ptr(n), _stream(stream))
    _check(ctx, rc)
    return M, int(n[0])


def icp_stage_single_pass(ctx, level, pose, iter=0, pred_hi=-1, pred_hw=24, params=None, stream=None):
    """Single-pass iteration at `level`: returns (hit, band[4], window(h0, width), moments[28], n)."""
    p = params if params is not None else icp_params_default()
    P12 = _f64(np.asarray(pose, dtype=np.float64)[:3, :4], 12, "pose")
    band = np.zeros(4, np.int64)
    win = np.zeros(2, np.int32)
    hit = C.c_int(0)
    M = np.zeros(28)
    n = np.zeros(1, np.int64)
    rc = lib().icp_stage_single_pass(ctx.handle, level, _np_ptr(P12), C.byref(p), int(iter), int(pred_hi),
                                     int(pred_hw), _np_ptr(band), _np_ptr(win), C.byref(hit), _np_ptr(M), _np_ptr(n),
                                     _stream(stream))
    _check(ctx, rc)
    return bool(hit.value), band, (int(win[0]), int(win[1])), M, int(n[0])


def icp_stage_solve(ctx, moments, n, pose, params=None, stream=None):
    p = params if params is not None else icp_params_default()
    M = _f64(moments, 28, "moments")
    P12 = _f64(np.asarray(pose, dtype=np.float64)[:3, :4], 12, "pose")
    out = np.zeros(12)
    x = np.zeros(6)
    st = C.c_int(0)
    rc = lib().icp_stage_solve(ctx.handle, _np_ptr(M), int(n), _np_ptr(P12), C.byref(p), _np_ptr(out), _np_ptr(x),
                               C.byref(st), _stream(stream))
    _check(ctx, rc)
    T = np.eye(4)
    T[:3, :4] = out.reshape(3, 4)
    return st.value, T, x


# ---------------------------------------------------------------- model maps

def icp_live_maps(ctx, depth, K, stream=None):
    """Interleaved (H, W, 3) vertex and normal maps of a device depth image."""
    import torch
    H, W = depth.shape
    dev = torch.device("cuda", ctx.device)
    vtx = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    nrm = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    Kc = make_intrinsics(K)
    rc = lib().icp_live_maps(ctx.handle, _dev_ptr(depth, "float32", "depth"), W, H, C.byref(Kc),
                             C.c_void_p(vtx.data_ptr()), C.c_void_p(nrm.data_ptr()), _stream(stream))
    _check(ctx, rc)
    return vtx, nrm


# ---------------------------------------------------------------- TSDF model

class TsdfVolume:
    """A TSDF volume in a device tensor of (dim, dim, dim, 2) float32 pairs
    (tsdf, weight), indexed [k][j][i] (x fastest).  mu defaults to 4 voxels.
    With bricks=True (the default) it also holds the per-brick buffer that
    lets the ray cast skip free and unobserved space (same results)."""

    def __init__(self, ctx, dim=512, size=6.0, origin=(-3.0, -3.0, -3.0), mu=None, max_weight=128.0, bricks=True):
        import torch
        self.ctx = ctx
        self.dim, self.size = int(dim), float(size)
        self.origin = tuple(float(o) for o in origin)
        self.mu = float(mu) if mu is not None else 4.0 * self.size / self.dim
        self.max_weight = float(max_weight)
        if lib().icp_tsdf_bytes(self.dim) == 0:
            raise IcpError(EINVAL, "TSDF dim must be in 2..1024")
        dev = torch.device("cuda", ctx.device)
        self.voxels = torch.empty((self.dim, self.dim, self.dim, 2), dtype=torch.float32, device=dev)
        self.bricks = (torch.empty(lib().icp_tsdf_brick_bytes(self.dim), dtype=torch.uint8, device=dev)
                       if bricks else None)
        self.desc = icp_tsdf(voxels=self.voxels.data_ptr(), dim=self.dim, pad_=0, size=self.size,
                             origin=(C.c_double * 3)(*self.origin), mu=self.mu, max_weight=self.max_weight,
                             bricks=self.bricks.data_ptr() if bricks else None)
        self.reset()

    def reset(self, stream=None):
        _check(self.ctx, lib().icp_tsdf_reset(self.ctx.handle, C.byref(self.desc), _stream(stream)))

    def integrate(self, depth, K, T_wc, stream=None):
        H, W = depth.shape
        T = _f64(T_wc, 16, "T_wc")
        Kc = make_intrinsics(K)
        _check(self.ctx, lib().icp_tsdf_integrate(self.ctx.handle, C.byref(self.desc), _dev_ptr(depth, "float32", "depth"),
                                                  W, H, C.byref(Kc), _np_ptr(T), _stream(stream)))

    def raycast(self, W, H, K, T_wc, tmin=0.4, tmax=8.0, out=None, stream=None):
        """Interleaved (H, W, 3) vertex and normal maps in the camera of T_wc."""
        import torch
        if out is None:
            dev = torch.device("cuda", self.ctx.device)
            out = (torch.empty((H, W, 3), dtype=torch.float32, device=dev),
                   torch.empty((H, W, 3), dtype=torch.float32, device=dev))
        vtx, nrm = out
        for name, t in (("vtx", vtx), ("nrm", nrm)):
            if tuple(t.shape) != (H, W, 3):
                raise ValueError(f"{name} must have shape ({H}, {W}, 3), got {tuple(t.shape)}")
        T = _f64(T_wc, 16, "T_wc")
        Kc = make_intrinsics(K)
        _check(self.ctx, lib().icp_tsdf_raycast(self.ctx.handle, C.byref(self.desc), W, H, C.byref(Kc), _np_ptr(T),
                                                float(tmin), float(tmax), _dev_ptr(vtx, "float32", "vtx"),
                                                _dev_ptr(nrm, "float32", "nrm"), _stream(stream)))
        return vtx, nrm

    def brick_state(self):
        """Host copies of the per-brick counts of observed voxels with
        tsdf <= 0, shape (nb, nb, nb) indexed [bz][by][bx], and the skip flags
        (1 = skippable), same shape."""
        nb = (self.dim + 7) // 8
        raw = self.bricks.cpu().numpy()
        cnt_bytes = (nb ** 3 * 4 + 255) // 256 * 256
        cnt = raw[:nb ** 3 * 4].view(np.int32).reshape(nb, nb, nb)
        flags = raw[cnt_bytes:cnt_bytes + nb ** 3].reshape(nb, nb, nb)
        return cnt, flags

    def host_arrays(self):
        """(tsdf, weight) as flat float32 host arrays in voxel order."""
        v = self.voxels.cpu().numpy().reshape(-1, 2)
        return np.ascontiguousarray(v[:, 0]), np.ascontiguousarray(v[:, 1])


# ---------------------------------------------------------------- serving

def icp_server_config_default(**over):
    cfg = icp_server_config()
    lib().icp_server_config_default(C.byref(cfg))
    for k, v in over.items():
        if k == "params":
            cfg.params = v
        else:
            setattr(cfg, k, v)
    return cfg


def icp_server_clock():
    return lib().icp_server_clock()


def server_result_dict(r):
    return dict(stream_id=r.stream_id, status=r.status, frame=r.frame, tag=r.tag,
                pose_rel=np.array(r.pose_rel[:]).reshape(4, 4), pose_world=np.array(r.pose_world[:]).reshape(4, 4),
                stats=stats_to_dict(r.stats), t_submit=r.t_submit, t_start=r.t_start, t_done=r.t_done,
                batch_size=r.batch_size)


class Server:
    """Frame server (icp_server_*): frame-to-frame tracking of many camera
    streams with continuous batching; see include/icp.h."""

    def __init__(self, config=None, **over):
        cfg = config if config is not None else icp_server_config_default(**over)
        h = C.c_void_p()
        rc = lib().icp_server_create(C.byref(cfg), C.byref(h))
        if rc != OK:
            raise IcpError(rc, "icp_server_create failed")
        self.handle = h
        self.config = cfg
        self.sizes = {}  # open stream id -> (H, W): a submitted frame must have that shape

    def _check(self, rc):
        if rc < 0:
            msg = lib().icp_server_last_error(self.handle)
            raise IcpError(rc, msg.decode() if msg else "")
        return rc

    def open_stream(self, W, H, K):
        sid = C.c_int(-1)
        Kc = make_intrinsics(K)
        self._check(lib().icp_server_open_stream(self.handle, W, H, C.byref(Kc), C.byref(sid)))
        self.sizes[sid.value] = (H, W)
        return sid.value

    def close_stream(self, sid):
        self._check(lib().icp_server_close_stream(self.handle, sid))
        self.sizes.pop(sid, None)

    def submit(self, sid, depth, imu_rel_R, tag=0, t_submit=0.0):
        d = np.ascontiguousarray(depth, dtype=np.float32)
        if sid in self.sizes and d.shape != self.sizes[sid]:  # the library copies H*W floats from it
            raise ValueError(f"depth must have shape {self.sizes[sid]}, got {d.shape}")
        R = np.ascontiguousarray(imu_rel_R, dtype=np.float64).reshape(9)
        self._check(lib().icp_server_submit(self.handle, sid, d.ctypes.data_as(C.c_void_p),
                                            R.ctypes.data_as(C.c_void_p), int(tag), float(t_submit)))

    def poll(self, max_results=256, timeout_ms=0):
        buf = (icp_server_result * max_results)()
        n = self._check(lib().icp_server_poll(self.handle, C.cast(buf, C.c_void_p), max_results, int(timeout_ms)))
        return [server_result_dict(buf[i]) for i in range(n)]

    def counters(self):
        c = icp_server_counters()
        self._check(lib().icp_server_get_counters(self.handle, C.byref(c)))
        return {k: getattr(c, k) for k, _ in icp_server_counters._fields_ if k != "pad"}

    def close(self):
        if self.handle:
            lib().icp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
