"""Shared checks of GPU registrations against the FP64 oracle.

A registration's per-level statistics (median bin, gated and kept counts of
the last iteration run, iterations, status) must equal the oracle's exactly,
except where a pixel's deciding quantity lies within EXCUSE_M of its
threshold at the pose that entered that iteration: the two sides' poses
differ by rounding (about 1e-10), so only such pixels can be decided
differently.  Those pixels are counted from the oracle's margins and
reported; with none, equality is exact.
"""
import numpy as np

import oracle
from tests.poseutil import pose_err

EXCUSE_M = 1e-6
POSE_TOL = 1e-5


def oracle_params(p):
    """Oracle parameters equal to an icp_params."""
    return oracle.default_params(levels=p.levels, iters=list(p.iters), dist_max=p.dist_max,
                                 cos_angle_max=p.cos_angle_max, band_beta=p.band_beta,
                                 use_median_filter=p.use_median_filter, use_imu_seed=p.use_imu_seed,
                                 lambda_mode=p.lambda_mode, lambda_c=p.lambda_c, min_corr=p.min_corr,
                                 ill_cond_eps=p.ill_cond_eps, converge_window=p.converge_window,
                                 depth_filter=p.depth_filter, filter_radius=p.filter_radius,
                                 filter_sigma_px=p.filter_sigma_px, filter_sigma_m=p.filter_sigma_m,
                                 normal_mode=p.normal_mode, normal_radius=p.normal_radius,
                                 anchor_to_imu=p.anchor_to_imu)


def oracle_levels(prob, p):
    """The oracle's pyramids of a problem with the front end of params p."""
    D = prob.live_depth
    if p.depth_filter:
        D = oracle.bilateral(D, p.filter_radius, p.filter_sigma_px, p.filter_sigma_m)
    MV, MN = oracle.model_l0(prob.model_vtx, prob.model_nrm)
    out = []
    for lvl in range(p.levels):
        if lvl:
            D = oracle.depth_down(D)
            MV, MN = oracle.model_down(MV, MN)
        Kl = oracle.level_intrinsics(prob.K, lvl)
        if p.normal_mode == 1:
            LV, LN = oracle.live_vn_box(D, Kl, p.normal_radius)
        else:
            LV, LN = oracle.live_vn(D, Kl)
        out.append(dict(D=D, LV=LV, LN=LN, MV=MV, MN=MN, K=Kl))
    return out


def _seed_pose(prob, p):
    T = np.array(prob.init_pose, dtype=np.float64).reshape(4, 4).copy()
    if p.use_imu_seed:
        T[:3, :3] = prob.imu_R
    return T


def entering_poses(prob, p, trace):
    """Pose entering each traced iteration (the oracle's)."""
    T = _seed_pose(prob, p)
    out = []
    for t in trace:
        out.append(T)
        T = t["pose"]
    return out


def assert_stats_match(prob, p, sg, so, trace, tag=""):
    """Per-level statistics of a GPU registration (stats dict of the binding)
    against the oracle's (list of level dicts and its iteration trace, which
    must cover every iteration).  Returns the number of excused pixels."""
    levels = None
    enter = entering_poses(prob, p, trace)
    excused_total = 0
    for lvl in range(p.levels):
        g, o = sg["levels"][lvl], so[lvl]
        assert g["iters_run"] == o["iters_run"], (tag, lvl, g["iters_run"], o["iters_run"])
        assert g["status"] == o["status"], (tag, lvl, g["status"], o["status"])
        same = (g["k_med"] == o["k_med"] and g["n_gated"] == o["n_gated"] and g["n_kept"] == o["n_kept"])
        if same:
            continue
        # which pixels could the rounding of the pose have decided differently?
        idx = max(i for i, t in enumerate(trace) if t["level"] == lvl)
        if levels is None:
            levels = oracle_levels(prob, p)
        _, _, margin, _ = oracle.associate(levels[lvl], enter[idx], p.dist_max, p.cos_angle_max)
        excused = int((margin < EXCUSE_M).sum())
        excused_total += excused
        print(f"{tag} level {lvl}: gpu {g} oracle {o}, {excused} pixels within {EXCUSE_M} m of a threshold")
        assert excused > 0, (tag, lvl, g, o)
        assert abs(g["n_gated"] - o["n_gated"]) <= excused, (tag, lvl)
    return excused_total


def oracle_register(prob, p, trace_cap=512):
    """The oracle's registration of a problem with params p: (pose, level stats, trace)."""
    To, so, trace = oracle.register_problem(prob, oracle_params(p), trace_cap=trace_cap)
    assert len(trace) == sum(s["iters_run"] for s in so)
    return To, so, trace


def assert_registration_matches(prob, p, Tg, sg, tag="", ref=None):
    """Pose within POSE_TOL of the oracle's and statistics per
    assert_stats_match (ref: a precomputed oracle_register result); returns
    (rotation error, translation error)."""
    To, so, trace = ref if ref is not None else oracle_register(prob, p)
    ang, dt = pose_err(Tg, To)
    assert ang < POSE_TOL and dt < POSE_TOL, (tag, ang, dt)
    assert_stats_match(prob, p, sg, so, trace, tag)
    return ang, dt


def oracle_sensitivity(prob, p, rel=1e-6, seeds=(0, 1)):
    """How far the oracle's own final pose moves when every iteration's
    moments are perturbed by `rel` relative (the size of an FP32 reduction's
    rounding): the largest (rotation, translation) change over the seeds.
    An ill-conditioned registration (few constraints, no regularisation)
    amplifies rounding without bound; a comparison with the GPU at POSE_TOL
    is only meaningful when this stays well below it."""
    levels = oracle_levels(prob, p)

    def run(seed):
        rng = np.random.default_rng(seed)
        T = _seed_pose(prob, p)
        for lvl in range(p.levels - 1, -1, -1):
            for _ in range(p.iters[lvl]):
                _, _, _, hist = oracle.associate(levels[lvl], T, p.dist_max, p.cos_angle_max)
                N, kmed, klo, khi = oracle.band(hist, p.use_median_filter, p.band_beta)
                M, n = oracle.moments(levels[lvl], T, klo, khi, p.dist_max, p.cos_angle_max)
                if seed is not None:
                    M = M * (1.0 + rel * rng.standard_normal(28))
                st, T1, _ = oracle.solve_update(M, n, T, p.lambda_mode, p.lambda_c, p.min_corr, p.ill_cond_eps,
                                                prob.imu_R if p.anchor_to_imu else None)
                if st != oracle.LEVEL_OK:
                    break
                T = T1
                # the convergence rule is not replayed: a fixed cadence is what is perturbed
        return T

    base = run(None)
    worst = (0.0, 0.0)
    for sd in seeds:
        a, d = pose_err(run(sd), base)
        worst = (max(worst[0], a), max(worst[1], d))
    return worst
