"""Seeded camera streams for the serving workload.

Each stream looks at a scene of the single-frame-pair type (3 random planes
and 4 spheres, placed for its own resolution with f = 525 H / 480) from a
slow, smooth, periodic camera path: the pose repeats every `period` frames,
so a stream of any length is made of `period` distinct depth images.  Depth
has Kinect-like axial noise and dropouts, drawn per distinct frame.  The IMU
gives each frame's orientation perturbed by a small random rotation; the
prior of registration k (frame k against frame k-1) is the IMU rotation of
frame k relative to frame k-1.  Nothing here computes any part of the
registration itself.
"""
from __future__ import annotations

import math

import numpy as np

from .scene import (DEG, Plane, Sphere, _rng, add_sensor_noise, centred_intrinsics, pose_matrix, random_planes,
                    random_spheres, rot_from_rotvec)

SERVING_RESOLUTIONS = ((320, 240), (640, 480), (848, 480), (1280, 720))


def serving_mix(n_streams=32, proportions=(1, 2, 1, 1)):
    """Resolutions of n streams split by largest remainder in the given
    proportions, listed smallest first (32 streams: 7, 13, 6, 6)."""
    total = float(sum(proportions))
    exact = [n_streams * p / total for p in proportions]
    counts = [int(math.floor(e)) for e in exact]
    order = sorted(range(len(exact)), key=lambda i: exact[i] - counts[i], reverse=True)
    for i in order[:n_streams - sum(counts)]:
        counts[i] += 1
    out = []
    for (W, H), c in zip(SERVING_RESOLUTIONS, counts):
        out += [(W, H)] * c
    return out


def render_depth(prims, W, H, K, cam_pose, zmin=0.5, zmax=4.0):
    """Z-depth (float64, 0 = no hit or outside [zmin, zmax]) of planes and
    spheres seen from cam_pose (camera -> world), ray-cast in the camera frame
    where the ray of pixel (u, v) is z (x_u, y_v, 1)."""
    fx, fy, cx, cy = K
    R = np.asarray(cam_pose, dtype=np.float64)[:3, :3]
    t = np.asarray(cam_pose, dtype=np.float64)[:3, 3]
    xs = (np.arange(W, dtype=np.float64) - cx) / fx
    ys = (np.arange(H, dtype=np.float64) - cy) / fy
    best = np.full((H, W), np.inf)
    for p in prims:
        if isinstance(p, Plane):
            n = R.T @ p.n
            c = p.c - p.n @ t
            den = (n[1] * ys)[:, None] + (n[0] * xs)[None, :] + n[2]
            with np.errstate(divide="ignore", invalid="ignore"):
                z = c / den
            z = np.where(z > 0, z, np.inf)
        elif isinstance(p, Sphere):
            C = R.T @ (p.centre - t)
            dd = (ys * ys)[:, None] + (xs * xs)[None, :] + 1.0
            dc = (C[1] * ys)[:, None] + (C[0] * xs)[None, :] + C[2]
            disc = dc * dc - dd * (C @ C - p.radius * p.radius)
            with np.errstate(invalid="ignore"):
                z = (dc - np.sqrt(disc)) / dd
            z = np.where((disc >= 0) & (z > 0), z, np.inf)
        else:
            raise TypeError(type(p))
        best = np.minimum(best, z)
    return np.where((best >= zmin) & (best <= zmax), best, 0.0)


class CameraStream:
    """Frames of one camera stream (depth float32 on the host)."""

    def __init__(self, index, W, H, seed=0, period=60, rot_amp_deg=4.0, trans_amp_m=0.04, imu_deg=0.5):
        rng = _rng(5, seed, index)
        self.index, self.W, self.H, self.period = index, W, H, period
        self.K = centred_intrinsics(W, H, 525.0 * H / 480.0)
        self.prims = random_planes(rng, self.K, W, H) + random_spheres(rng, self.K, W, H)
        a1 = rng.normal(size=3)
        a2 = rng.normal(size=3)
        a1 *= rot_amp_deg * DEG / np.linalg.norm(a1)
        a2 *= 0.5 * rot_amp_deg * DEG / np.linalg.norm(a2)
        b1 = rng.normal(size=3)
        b2 = rng.normal(size=3)
        b1 *= trans_amp_m / np.linalg.norm(b1)
        b2 *= 0.5 * trans_amp_m / np.linalg.norm(b2)
        ph = rng.uniform(0, 2 * math.pi)
        self.poses = []
        self.imu = []
        for k in range(period):
            s = 2 * math.pi * k / period
            w = a1 * math.sin(s) + a2 * math.sin(2 * s + ph)
            tr = b1 * (1.0 - math.cos(s)) + b2 * math.sin(2 * s + ph)
            R = rot_from_rotvec(w)
            self.poses.append(pose_matrix(R, tr))
            g = rng.normal(size=3)
            self.imu.append(rot_from_rotvec(g / np.linalg.norm(g) * imu_deg * DEG) @ R)
        self.noise_seeds = rng.integers(0, 2**63 - 1, size=period)
        self._cache = {}

    def depth(self, k):
        j = k % self.period
        if j not in self._cache:
            d = render_depth(self.prims, self.W, self.H, self.K, self.poses[j])
            d = add_sensor_noise(d, np.random.default_rng(int(self.noise_seeds[j])))
            self._cache[j] = d.astype(np.float32)
        return self._cache[j]

    def imu_rel(self, k):
        """IMU rotation of frame k relative to frame k-1 (k >= 1)."""
        a, b = self.imu[(k - 1) % self.period], self.imu[k % self.period]
        return a[:3, :3].T @ b[:3, :3]

    def truth_rel(self, k):
        """Camera k in camera k-1 (4x4)."""
        a, b = self.poses[(k - 1) % self.period], self.poses[k % self.period]
        return np.linalg.inv(a) @ b
