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
    return oracle.params_like(p)


def oracle_levels(prob, p):
    """The oracle's pyramids of a problem with the front end of params p."""
    return oracle.levels_of(prob, p)


def _seed_pose(prob, p):
    return oracle.seed_pose(prob, p)


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
    """The oracle's own pose change under FP32-sized moment perturbations
    (oracle.sensitivity): a comparison with the GPU at POSE_TOL is only
    meaningful when this stays well below it."""
    return oracle.sensitivity(prob, p, rel, seeds)
