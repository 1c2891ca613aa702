"""ctypes wrapper of the plain FP64 CPU oracle (``icp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The GPU package never imports this module and
shares no code with it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD_DIR = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(BUILD_DIR, "libicp_oracle.so")
SOURCES = [os.path.join(HERE, "icp_oracle.c")]

MAX_LEVELS = 4
BINS = 1024
BIN_W = 1.0 / 8192.0

INVALID_LIVE, BEHIND, OUTSIDE, INVALID_MODEL, FAR, ANGLE, GATED = range(7)
LEVEL_OK, TOO_FEW_CORR, ILL_COND, NONFINITE = range(4)
LAMBDA_CONST, LAMBDA_C_OVER_SQRT_N, LAMBDA_C_OVER_N, LAMBDA_C_OVER_N2 = range(4)


def build(force=True):
    """Compile the oracle with gcc (FP64, no contraction, no fast-math)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fno-fast-math", "-ffp-contract=off",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [
        ("levels", C.c_int), ("iters", C.c_int * MAX_LEVELS),
        ("dist_max", C.c_double), ("cos_angle_max", C.c_double), ("band_beta", C.c_double),
        ("use_median_filter", C.c_int), ("use_imu_seed", C.c_int), ("lambda_mode", C.c_int),
        ("lambda_c", C.c_double), ("min_corr", C.c_int), ("ill_cond_eps", C.c_double),
        ("converge_window", C.c_int), ("depth_filter", C.c_int), ("filter_radius", C.c_int),
        ("filter_sigma_px", C.c_double), ("filter_sigma_m", C.c_double), ("normal_mode", C.c_int),
        ("normal_radius", C.c_int), ("anchor_to_imu", C.c_int),
    ]


class LevelStats(C.Structure):
    _fields_ = [("iters_run", C.c_int32), ("status", C.c_int32), ("n_gated", C.c_int64),
                ("n_kept", C.c_int64), ("k_med", C.c_int32), ("pad", C.c_int32), ("rmse", C.c_double)]


class IterTrace(C.Structure):
    _fields_ = [("level", C.c_int32), ("iter", C.c_int32), ("status", C.c_int32), ("k_med", C.c_int32),
                ("k_lo", C.c_int32), ("k_hi", C.c_int32), ("n_gated", C.c_int64), ("n_kept", C.c_int64),
                ("x", C.c_double * 6), ("pose", C.c_double * 12)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        stale = not os.path.exists(LIB_PATH) or any(
            os.path.getmtime(src) > os.path.getmtime(LIB_PATH)
            for src in SOURCES + [os.path.join(HERE, "icp_oracle.h")])
        if stale:
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        d = C.c_double
        i = C.c_int
        L.or_params_default.argtypes = [C.POINTER(Params)]
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]
        L.or_level_intrinsics.argtypes = [P, i, P]
        L.or_depth_down.argtypes = [P, i, i, P]
        L.or_live_vn.argtypes = [P, i, i, P, P, P]
        L.or_bilateral.argtypes = [P, i, i, i, d, d, P]
        L.or_tsdf_integrate.argtypes = [P, P, i, d, P, d, d, P, i, i, P, P]
        L.or_tsdf_raycast.argtypes = [P, P, i, d, P, d, d, i, i, P, P, P, P]
        L.or_live_vn_box.argtypes = [P, i, i, P, i, P, P]
        L.or_model_l0.argtypes = [P, P, i, i, P, P]
        L.or_model_down.argtypes = [P, P, i, i, P, P]
        L.or_associate.argtypes = [P, P, P, P, i, i, P, P, d, d, P, P, P, P]
        L.or_band.argtypes = [P, i, d, P]
        L.or_bin_of.argtypes = [d]
        L.or_bin_of.restype = i
        L.or_pairs.argtypes = [P, P, P, P, i, i, P, P, d, d, P, P, P, P, P]
        L.or_moments.argtypes = [P, P, P, P, i, i, P, P, d, d, i, i, P, P]
        L.or_solve_update.argtypes = [P, C.c_int64, P, i, d, i, d, P, P]
        L.or_solve_update.restype = i
        L.or_se3_exp.argtypes = [P, P, P, P]
        L.or_so3_log.argtypes = [P, P]
        L.or_solve_update_anchor.argtypes = [P, C.c_int64, P, i, d, i, d, P, P, P]
        L.or_solve_update_anchor.restype = i
        L.or_icp_register.argtypes = [P, i, i, P, P, P, P, P, C.POINTER(Params), P, P, P, i]
        L.or_icp_register.restype = i
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_params(**over):
    p = Params()
    lib().or_params_default(C.byref(p))
    for k, v in over.items():
        if k == "iters":
            for j in range(MAX_LEVELS):
                p.iters[j] = int(v[j]) if j < len(v) else 0
        else:
            setattr(p, k, v)
    return p


def params_like(p):
    """Oracle parameters with the values of any object that has the same
    field names (e.g. the GPU library's icp_params)."""
    q = Params()
    lib().or_params_default(C.byref(q))
    for name, _ in Params._fields_:
        if name == "iters":
            for j in range(MAX_LEVELS):
                q.iters[j] = int(p.iters[j])
        else:
            setattr(q, name, getattr(p, name))
    return q


def num_threads():
    return int(lib().or_num_threads())


def set_num_threads(n):
    """Threads of the oracle's later calls (for timing; results do not depend on it)."""
    lib().or_set_num_threads(int(n))


def level_intrinsics(K, level):
    out = np.zeros(4)
    lib().or_level_intrinsics(_p(_f64(K)), level, _p(out))
    return out


def pose12(T):
    """3x4 row-major [R | t] of a 4x4 (or 3x4) pose."""
    return _f64(np.asarray(T, dtype=np.float64)[:3, :4]).reshape(12).copy()


# ---------------------------------------------------------------- stages

def depth_down(D):
    D = _f32(D)
    H, W = D.shape
    out = np.empty((H // 2, W // 2), np.float32)
    lib().or_depth_down(_p(D), W, H, _p(out))
    return out


def live_vn(D, K):
    """SoA vertex and normal maps (3, H, W) float32 of one level."""
    D = _f32(D)
    H, W = D.shape
    V = np.empty((3, H, W), np.float32)
    N = np.empty((3, H, W), np.float32)
    lib().or_live_vn(_p(D), W, H, _p(_f64(K)), _p(V), _p(N))
    return V, N


def bilateral(D, r=3, sigma_px=4.5, sigma_m=0.05):
    """Bilateral smoothing of a depth image (Gaussian spatial, biweight range)."""
    D = _f32(D)
    H, W = D.shape
    out = np.empty((H, W), np.float32)
    lib().or_bilateral(_p(D), W, H, int(r), C.c_double(sigma_px), C.c_double(sigma_m), _p(out))
    return out


def live_vn_box(D, K, r=2):
    """Vertex planes and box-average 3D-gradient normal planes (3, H, W)."""
    D = _f32(D)
    H, W = D.shape
    V = np.empty((3, H, W), np.float32)
    N = np.empty((3, H, W), np.float32)
    lib().or_live_vn_box(_p(D), W, H, _p(_f64(K)), int(r), _p(V), _p(N))
    return V, N


class Tsdf:
    """TSDF volume held as host arrays (test infrastructure)."""

    def __init__(self, dim=64, size=3.0, origin=(-1.5, -1.5, 0.5), mu=None, max_weight=128.0):
        self.dim, self.size = int(dim), float(size)
        self.origin = np.ascontiguousarray(origin, dtype=np.float64)
        self.mu = float(mu) if mu is not None else 4.0 * self.size / self.dim
        self.max_weight = float(max_weight)
        self.tsdf = np.zeros(self.dim ** 3, np.float32)
        self.weight = np.zeros(self.dim ** 3, np.float32)

    def integrate(self, depth, K, T_wc):
        depth = _f32(depth)
        H, W = depth.shape
        lib().or_tsdf_integrate(_p(self.tsdf), _p(self.weight), self.dim, C.c_double(self.size), _p(self.origin),
                                C.c_double(self.mu), C.c_double(self.max_weight), _p(depth), W, H,
                                _p(_f64(K)), _p(_f64(np.asarray(T_wc, dtype=np.float64).reshape(16))))

    def raycast(self, W, H, K, T_wc, tmin=0.4, tmax=8.0):
        vtx = np.empty((H, W, 3), np.float32)
        nrm = np.empty((H, W, 3), np.float32)
        lib().or_tsdf_raycast(_p(self.tsdf), _p(self.weight), self.dim, C.c_double(self.size), _p(self.origin),
                              C.c_double(tmin), C.c_double(tmax), W, H, _p(_f64(K)),
                              _p(_f64(np.asarray(T_wc, dtype=np.float64).reshape(16))), _p(vtx), _p(nrm))
        return vtx, nrm


def model_l0(vtx, nrm):
    vtx, nrm = _f32(vtx), _f32(nrm)
    H, W, _ = vtx.shape
    V = np.empty((3, H, W), np.float32)
    N = np.empty((3, H, W), np.float32)
    lib().or_model_l0(_p(vtx), _p(nrm), W, H, _p(V), _p(N))
    return V, N


def model_down(V, N):
    V, N = _f32(V), _f32(N)
    _, H, W = V.shape
    Vn = np.empty((3, H // 2, W // 2), np.float32)
    Nn = np.empty((3, H // 2, W // 2), np.float32)
    lib().or_model_down(_p(V), _p(N), W, H, _p(Vn), _p(Nn))
    return Vn, Nn


def pyramids(depth, vtx, nrm, K, levels):
    """Per level: dict(D, LV, LN, MV, MN, K)."""
    out = []
    D = _f32(depth)
    MV, MN = model_l0(vtx, nrm)
    for lvl in range(levels):
        if lvl > 0:
            D = depth_down(D)
            MV, MN = model_down(MV, MN)
        Kl = level_intrinsics(K, lvl)
        LV, LN = live_vn(D, Kl)
        out.append(dict(D=D, LV=LV, LN=LN, MV=MV, MN=MN, K=Kl))
    return out


def associate(lvl, T, dist_max=0.10, cos_max=None):
    """Per-pixel code, bin, margin (H, W) and the histogram for pose T."""
    if cos_max is None:
        cos_max = default_params().cos_angle_max
    LV, LN, MV, MN = (_f32(lvl[k]) for k in ("LV", "LN", "MV", "MN"))
    _, H, W = LV.shape
    code = np.empty((H, W), np.uint8)
    bins = np.empty((H, W), np.int32)
    margin = np.empty((H, W), np.float64)
    hist = np.empty(BINS, np.uint32)
    lib().or_associate(_p(LV), _p(LN), _p(MV), _p(MN), W, H, _p(_f64(lvl["K"])), _p(pose12(T)),
                       dist_max, cos_max, _p(code), _p(bins), _p(margin), _p(hist))
    return code, bins, margin, hist


def bin_of(d2):
    return int(lib().or_bin_of(float(d2)))


def pairs(lvl, T, dist_max=0.10, cos_max=None):
    """Per-pixel code, bin and (GATED pixels) p', q, n_q arrays (H*W, 3)."""
    if cos_max is None:
        cos_max = default_params().cos_angle_max
    LV, LN, MV, MN = (_f32(lvl[k]) for k in ("LV", "LN", "MV", "MN"))
    _, H, W = LV.shape
    code = np.empty(H * W, np.uint8)
    bins = np.empty(H * W, np.int32)
    pp = np.full((H * W, 3), np.nan)
    q = np.full((H * W, 3), np.nan)
    nq = np.full((H * W, 3), np.nan)
    lib().or_pairs(_p(LV), _p(LN), _p(MV), _p(MN), W, H, _p(_f64(lvl["K"])), _p(pose12(T)), dist_max, cos_max,
                   _p(code), _p(bins), _p(pp), _p(q), _p(nq))
    return code, bins, pp, q, nq


def band(hist, use_filter=1, beta=1.0):
    out = np.zeros(4, np.int64)
    lib().or_band(_p(np.ascontiguousarray(hist, dtype=np.uint32)), use_filter, beta, _p(out))
    return out


def moments(lvl, T, k_lo, k_hi, dist_max=0.10, cos_max=None):
    if cos_max is None:
        cos_max = default_params().cos_angle_max
    LV, LN, MV, MN = (_f32(lvl[k]) for k in ("LV", "LN", "MV", "MN"))
    _, H, W = LV.shape
    M = np.zeros(28)
    n = np.zeros(1, np.int64)
    lib().or_moments(_p(LV), _p(LN), _p(MV), _p(MN), W, H, _p(_f64(lvl["K"])), _p(pose12(T)),
                     dist_max, cos_max, int(k_lo), int(k_hi), _p(M), _p(n))
    return M, int(n[0])


def solve_update(M, n, T, lambda_mode=LAMBDA_CONST, lambda_c=5.0, min_corr=6, eps=1e-12, imu_R=None):
    """Regularised solve and update; with imu_R the damping is anchored to it."""
    Tout = np.zeros(12)
    x = np.zeros(6)
    if imu_R is None:
        st = lib().or_solve_update(_p(_f64(M)), int(n), _p(pose12(T)), lambda_mode, lambda_c, min_corr, eps,
                                   _p(Tout), _p(x))
    else:
        st = lib().or_solve_update_anchor(_p(_f64(M)), int(n), _p(pose12(T)), lambda_mode, lambda_c, min_corr,
                                          eps, _p(_f64(imu_R)), _p(Tout), _p(x))
    P = np.eye(4)
    P[:3, :4] = Tout.reshape(3, 4)
    return st, P, x


def so3_log(R):
    w = np.zeros(3)
    lib().or_so3_log(_p(_f64(R)), _p(w))
    return w


def se3_exp(w, tau):
    R = np.zeros(9)
    t = np.zeros(3)
    lib().or_se3_exp(_p(_f64(w)), _p(_f64(tau)), _p(R), _p(t))
    return R.reshape(3, 3), t


def tri_index(i, j):
    """Position of entry (i, j), i <= j, in the 28-moment vector."""
    return i * 7 - i * (i - 1) // 2 + (j - i)


def register(depth, vtx, nrm, K, imu_R, init_pose, params=None, trace_cap=64):
    """Whole registration. Returns (pose 4x4, list of level-stat dicts, trace list)."""
    p = params if params is not None else default_params()
    depth, vtx, nrm = _f32(depth), _f32(vtx), _f32(nrm)
    H, W = depth.shape
    pose = np.zeros(16)
    stats = (LevelStats * MAX_LEVELS)()
    trace = (IterTrace * trace_cap)()
    nt = lib().or_icp_register(_p(depth), W, H, _p(vtx), _p(nrm), _p(_f64(K)), _p(_f64(imu_R)),
                               _p(_f64(init_pose)), C.byref(p), _p(pose), C.cast(stats, C.c_void_p),
                               C.cast(trace, C.c_void_p), trace_cap)
    st = [dict(iters_run=s.iters_run, status=s.status, n_gated=s.n_gated, n_kept=s.n_kept, k_med=s.k_med,
               rmse=s.rmse) for s in stats[:p.levels]]
    tr = []
    for t in trace[:min(nt, trace_cap)]:
        P = np.eye(4)
        P[:3, :4] = np.array(t.pose[:]).reshape(3, 4)
        tr.append(dict(level=t.level, iter=t.iter, status=t.status, k_med=t.k_med, k_lo=t.k_lo, k_hi=t.k_hi,
                       n_gated=t.n_gated, n_kept=t.n_kept, x=np.array(t.x[:]), pose=P))
    return pose.reshape(4, 4), st, tr


def register_problem(prob, params=None, trace_cap=64):
    return register(prob.live_depth, prob.model_vtx, prob.model_nrm, prob.K, prob.imu_R, prob.init_pose,
                    params, trace_cap)


# ---------------------------------------------------------------- analysis helpers

def levels_of(prob, p):
    """The pyramids of a problem with the front end of parameters p (oracle or
    icp parameters: the same field names), as or_icp_register builds them."""
    D = prob.live_depth
    if p.depth_filter:
        D = bilateral(D, p.filter_radius, p.filter_sigma_px, p.filter_sigma_m)
    MV, MN = model_l0(prob.model_vtx, prob.model_nrm)
    out = []
    for lvl in range(p.levels):
        if lvl:
            D = depth_down(D)
            MV, MN = model_down(MV, MN)
        Kl = level_intrinsics(prob.K, lvl)
        if p.normal_mode == 1:
            LV, LN = live_vn_box(D, Kl, p.normal_radius)
        else:
            LV, LN = live_vn(D, Kl)
        out.append(dict(D=D, LV=LV, LN=LN, MV=MV, MN=MN, K=Kl))
    return out


def seed_pose(prob, p):
    """The pose a registration starts from: [imu_R | t_init] with the IMU seed, else init_pose."""
    T = np.array(prob.init_pose, dtype=np.float64).reshape(4, 4).copy()
    if p.use_imu_seed:
        T[:3, :3] = prob.imu_R
    return T


def _rot_angle(R):
    c = (np.trace(R) - 1.0) / 2.0
    s = 0.5 * np.linalg.norm([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    return float(np.arctan2(s, c))


def sensitivity(prob, p, rel=1e-6, seeds=(0, 1)):
    """How far the final pose moves when every iteration's moments are
    perturbed by `rel` relative (the size of an FP32 reduction's rounding):
    the largest (rotation rad, translation m) change over the seeds, with the
    fixed cadence of p.  A registration whose pose moves by more than a
    comparison tolerance under this perturbation is ill-conditioned (too few
    constraints for its regularisation): its result depends on rounding."""
    lv = levels_of(prob, p)

    def run(seed):
        rng = np.random.default_rng(seed)
        T = seed_pose(prob, p)
        for lvl in range(p.levels - 1, -1, -1):
            for _ in range(p.iters[lvl]):
                _, _, _, hist = associate(lv[lvl], T, p.dist_max, p.cos_angle_max)
                N, kmed, klo, khi = band(hist, p.use_median_filter, p.band_beta)
                M, n = moments(lv[lvl], T, klo, khi, p.dist_max, p.cos_angle_max)
                if seed is not None:
                    M = M * (1.0 + rel * rng.standard_normal(28))
                st, T1, _ = solve_update(M, n, T, p.lambda_mode, p.lambda_c, p.min_corr, p.ill_cond_eps,
                                         prob.imu_R if p.anchor_to_imu else None)
                if st != LEVEL_OK:
                    break
                T = T1
        return T

    base = run(None)
    worst = (0.0, 0.0)
    for sd in seeds:
        T = run(sd)
        worst = (max(worst[0], _rot_angle(T[:3, :3] @ base[:3, :3].T)),
                 max(worst[1], float(np.linalg.norm(T[:3, 3] - base[:3, 3]))))
    return worst
