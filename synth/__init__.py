"""Seeded synthetic inputs (depth frames, model maps, motions, IMU priors)."""
from .scene import (  # noqa: F401
    DEG, Problem, RoomSequence, pair_problem, uneven_problem, three_plane_problem,
    centred_intrinsics, rot_from_rotvec, pose_matrix, random_unit, render,
)
