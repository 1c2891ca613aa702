"""Pose-error metrics shared by the tests (no step of the method in here)."""
import math

import numpy as np


def rot_angle(R):
    """Rotation angle of R, accurate for tiny angles (atan2 of the skew part)."""
    s = 0.5 * np.linalg.norm([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    c = 0.5 * (np.trace(R) - 1.0)
    return math.atan2(s, c)


def pose_err(A, B):
    """(angle of R_A R_B^T in rad, |t_A - t_B| in m)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    return rot_angle(A[:3, :3] @ B[:3, :3].T), float(np.linalg.norm(A[:3, 3] - B[:3, 3]))
