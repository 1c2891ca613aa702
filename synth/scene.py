"""Seeded synthetic depth scenes shaped like the paper's Kinect workloads.

This module only *generates inputs*: analytic ray casting of planes, spheres
and axis-aligned boxes, the Kinect-like depth noise model, dropouts, camera
motions and IMU orientation draws.  It computes no step of the registration
method itself; the FP64 oracle and the GPU path both consume the arrays it
returns and neither shares any code with it beyond that.

Conventions
-----------
* Camera frame: x right, y down, z forward.  Pixel (u, v) has its centre at
  integer coordinates; its ray is ((u - cx)/fx, (v - cy)/fy, 1), so the ray
  parameter of a hit equals its z-depth.
* A camera pose is a 4x4 camera-to-world matrix.  The model camera of a
  registration problem is its reference frame; the ground-truth pose maps
  live-camera coordinates to model-camera coordinates (X_model = R X_live + t).
* Depth maps are float32 (H, W), metres, 0 where invalid.  Model vertex and
  normal maps are float32 (H, W, 3) in the model camera frame, NaN where
  invalid; normals are unit length and face the camera.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

DEG = math.pi / 180.0


# ----------------------------------------------------------------------------
# small geometry helpers used to *draw* motions (not the method's update)
# ----------------------------------------------------------------------------

def skew(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def rot_from_rotvec(w):
    """Rotation matrix of the rotation vector w (axis * angle), Rodrigues."""
    w = np.asarray(w, dtype=np.float64)
    th = float(np.linalg.norm(w))
    if th < 1e-12:
        return np.eye(3) + skew(w)
    k = skew(w / th)
    return np.eye(3) + math.sin(th) * k + (1.0 - math.cos(th)) * (k @ k)


def random_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def pose_matrix(R, t):
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def centred_intrinsics(W, H, fx, fy=None):
    """(fx, fy, cx, cy) with the principal point at the image centre."""
    fy = fx if fy is None else fy
    return (float(fx), float(fy), (W - 1) / 2.0, (H - 1) / 2.0)


# ----------------------------------------------------------------------------
# primitives (world frame)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Plane:
    n: np.ndarray  # unit normal
    c: float       # plane: n . X = c


@dataclasses.dataclass
class Sphere:
    centre: np.ndarray
    radius: float


@dataclasses.dataclass
class Box:
    lo: np.ndarray
    hi: np.ndarray


def _box_corners(lo, hi):
    return np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])])


def _pixel_window(prim, W, H, K, R_cw, t_cw):
    """Pixel rectangle that can see a compact primitive: None if it lies
    entirely behind the camera, the full image if it straddles the image
    plane."""
    if isinstance(prim, Plane):
        return 0, W, 0, H
    if isinstance(prim, Sphere):
        r = prim.radius
        corners = _box_corners(prim.centre - r, prim.centre + r)
    else:
        corners = _box_corners(prim.lo, prim.hi)
    Xc = (corners - t_cw) @ R_cw  # world -> camera: R^T (X - t)
    if np.all(Xc[:, 2] <= 0.0):
        return None
    if np.any(Xc[:, 2] < 0.05):
        return 0, W, 0, H
    fx, fy, cx, cy = K
    u = fx * Xc[:, 0] / Xc[:, 2] + cx
    v = fy * Xc[:, 1] / Xc[:, 2] + cy
    u0 = max(0, int(math.floor(u.min())) - 1)
    u1 = min(W, int(math.ceil(u.max())) + 2)
    v0 = max(0, int(math.floor(v.min())) - 1)
    v1 = min(H, int(math.ceil(v.max())) + 2)
    if u0 >= u1 or v0 >= v1:
        return None
    return u0, u1, v0, v1


def render(prims, W, H, K, cam_pose, zmin=0.5, zmax=4.0):
    """Ray-cast the primitives from a camera.

    Works in the camera frame, where the ray of pixel (u, v) is s * (xu, yv, 1)
    and every intersection term is separable in u and v.  Returns (depth,
    vertex, normal, prim_id) in float64: depth (H, W) with 0 for no hit or a
    hit outside [zmin, zmax]; vertex and normal (H, W, 3) in the camera frame,
    NaN where invalid, normals facing the camera; prim_id (H, W) int, -1 where
    invalid.
    """
    fx, fy, cx, cy = K
    R = np.asarray(cam_pose, dtype=np.float64)[:3, :3]
    t = np.asarray(cam_pose, dtype=np.float64)[:3, 3]
    us = (np.arange(W, dtype=np.float64) - cx) / fx
    vs = (np.arange(H, dtype=np.float64) - cy) / fy
    best = np.full((H, W), np.inf)
    nrm = np.zeros((H, W, 3))
    pid = np.full((H, W), -1, dtype=np.int64)
    for idx, prim in enumerate(prims):
        win = _pixel_window(prim, W, H, K, R, t)
        if win is None:
            continue
        u0, u1, v0, v1 = win
        xu = us[None, u0:u1]
        yv = vs[v0:v1, None]
        shape = (v1 - v0, u1 - u0)
        if isinstance(prim, Plane):
            nc = R.T @ prim.n            # plane in the camera frame: nc . X = cc
            cc = prim.c - prim.n @ t
            den = nc[0] * xu + nc[1] * yv + nc[2]
            with np.errstate(divide="ignore", invalid="ignore"):
                s = cc / den
            s = np.where(np.isfinite(s) & (s > 0), s, np.inf)
            nsel = lambda mask: nc  # noqa: E731
        elif isinstance(prim, Sphere):
            C = R.T @ (prim.centre - t)
            a = xu * xu + yv * yv + 1.0
            b = xu * C[0] + yv * C[1] + C[2]
            disc = b * b - a * (C @ C - prim.radius ** 2)
            ok = disc >= 0
            sq = np.sqrt(np.where(ok, disc, 0.0))
            s1 = (b - sq) / a
            s2 = (b + sq) / a
            s = np.where(s1 > 0, s1, s2)
            s = np.where(ok & (s > 0), s, np.inf)

            def nsel(mask, s=s, C=C, r=prim.radius, xu=xu, yv=yv):
                xx = np.broadcast_to(xu, shape)[mask]
                yy = np.broadcast_to(yv, shape)[mask]
                ss = s[mask]
                return np.stack([ss * xx - C[0], ss * yy - C[1], ss - C[2]], axis=-1) / r
        else:
            tmin = np.full(shape, -np.inf)
            tmax = np.full(shape, np.inf)
            axis = np.zeros(shape, dtype=np.int64)
            gs = []
            for i in range(3):
                g = R[i, 0] * xu + R[i, 1] * yv + R[i, 2]  # world axis i . ray
                g = np.broadcast_to(g, shape)
                gs.append(g)
                with np.errstate(divide="ignore", invalid="ignore"):
                    t1 = (prim.lo[i] - t[i]) / g
                    t2 = (prim.hi[i] - t[i]) / g
                tn = np.where(np.isnan(t1), -np.inf, np.minimum(t1, t2))
                tf = np.where(np.isnan(t1), np.inf, np.maximum(t1, t2))
                upd = tn > tmin
                axis = np.where(upd, i, axis)
                tmin = np.maximum(tmin, tn)
                tmax = np.minimum(tmax, tf)
            ok = (tmax >= tmin) & (tmin > 0)
            s = np.where(ok, tmin, np.inf)
            gsel = np.stack(gs, axis=-1)

            def nsel(mask, axis=axis, gsel=gsel):
                ax = axis[mask]
                g = np.take_along_axis(gsel[mask], ax[:, None], axis=-1)[:, 0]
                return -np.sign(g)[:, None] * R[ax, :]
        region = best[v0:v1, u0:u1]
        closer = s < region
        region[closer] = s[closer]
        nrm[v0:v1, u0:u1][closer] = nsel(closer)
        pid[v0:v1, u0:u1][closer] = idx
    valid = np.isfinite(best) & (best >= zmin) & (best <= zmax)
    depth = np.where(valid, best, 0.0)
    vtx = np.empty((H, W, 3))
    vtx[..., 0] = depth * us[None, :]
    vtx[..., 1] = depth * vs[:, None]
    vtx[..., 2] = depth
    side = nrm[..., 0] * vtx[..., 0] + nrm[..., 1] * vtx[..., 1] + nrm[..., 2] * vtx[..., 2]
    nrm *= np.where(side > 0, -1.0, 1.0)[..., None]
    vtx = np.where(valid[..., None], vtx, np.nan)
    nrm = np.where(valid[..., None], nrm, np.nan)
    pid = np.where(valid, pid, -1)
    return depth, vtx, nrm, pid


def add_sensor_noise(depth, rng, sigma_coeff=0.0012, dropout=0.02):
    """Kinect-like axial noise N(0, (c z^2)^2) plus uniform zero dropouts."""
    valid = depth > 0
    noisy = depth + rng.normal(size=depth.shape) * (sigma_coeff * depth * depth)
    noisy = np.where(valid, noisy, 0.0)
    drop = rng.random(size=depth.shape) < dropout
    return np.where(drop, 0.0, noisy)


# ----------------------------------------------------------------------------
# registration problems
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    """One frame-to-model registration problem (all arrays host numpy)."""
    live_depth: np.ndarray   # (H, W) float32, 0 invalid
    model_vtx: np.ndarray    # (H, W, 3) float32, NaN invalid
    model_nrm: np.ndarray    # (H, W, 3) float32, NaN invalid
    K: tuple                 # (fx, fy, cx, cy) of the full-resolution image
    imu_R: np.ndarray        # (3, 3) float64 prior for the live->model rotation
    init_pose: np.ndarray    # (4, 4) float64
    T_gt: np.ndarray         # (4, 4) float64 ground truth live->model
    name: str = ""

    @property
    def W(self):
        return self.live_depth.shape[1]

    @property
    def H(self):
        return self.live_depth.shape[0]


def _rng(*key):
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def random_planes(rng, K, W, H, n_planes=3, cone_deg=45.0, z_axis=(2.5, 3.8),
                  min_cover=0.05, min_pair_deg=0.0, tries=500):
    """Planes with normals within `cone_deg` of -z, crossing the optical axis at
    depth U(z_axis); rejection-sampled until each is the nearest plane on at
    least `min_cover` of the pixels and pairwise normal angles exceed
    `min_pair_deg`."""
    cos_cone = math.cos(cone_deg * DEG)
    for _ in range(tries):
        planes = []
        for _ in range(n_planes):
            ct = rng.uniform(cos_cone, 1.0)
            st = math.sqrt(max(0.0, 1.0 - ct * ct))
            ph = rng.uniform(0.0, 2 * math.pi)
            n = np.array([st * math.cos(ph), st * math.sin(ph), -ct])
            z0 = rng.uniform(*z_axis)
            planes.append(Plane(n=n, c=float(n[2] * z0)))
        ok = True
        for i in range(n_planes):
            for j in range(i + 1, n_planes):
                ang = math.degrees(math.acos(np.clip(planes[i].n @ planes[j].n, -1, 1)))
                if ang <= min_pair_deg:
                    ok = False
        if not ok:
            continue
        _, _, _, pid = render(planes, W, H, K, np.eye(4), zmin=0.0, zmax=np.inf)
        cover = [(pid == i).mean() for i in range(n_planes)]
        if min(cover) >= min_cover:
            return planes
    raise RuntimeError("could not draw a plane arrangement with the requested coverage")


def random_spheres(rng, K, W, H, n=4, r_range=(0.2, 0.5), z_range=(1.0, 3.0)):
    fx, fy, cx, cy = K
    out = []
    for _ in range(n):
        u = rng.uniform(0, W - 1)
        v = rng.uniform(0, H - 1)
        z = rng.uniform(*z_range)
        c = z * np.array([(u - cx) / fx, (v - cy) / fy, 1.0])
        out.append(Sphere(centre=c, radius=float(rng.uniform(*r_range))))
    return out


def make_pair_problem(prims, W, H, K, T_gt, imu_R, rng, noise=True, dropout=0.02,
                      zmin=0.5, zmax=4.0, name=""):
    """Model maps rendered noise-free at the identity, live depth at T_gt."""
    _, mv, mn, _ = render(prims, W, H, K, np.eye(4), zmin, zmax)
    ld, _, _, _ = render(prims, W, H, K, T_gt, zmin, zmax)
    if noise:
        ld = add_sensor_noise(ld, rng, dropout=dropout)
    return Problem(live_depth=ld.astype(np.float32), model_vtx=mv.astype(np.float32),
                   model_nrm=mn.astype(np.float32), K=K, imu_R=imu_R, init_pose=np.eye(4),
                   T_gt=T_gt, name=name)


def pair_problem(seed=0, W=160, H=120, f=130.0, rot_deg=2.0, trans_m=0.02,
                    imu_deg=0.5, noise=True, spheres=True):
    """Single frame pair, plain method: 3 random planes plus 4 spheres, 2 deg /
    2 cm ground-truth motion, IMU prior perturbed by 0.5 deg."""
    rng = _rng(1, seed)
    K = centred_intrinsics(W, H, f)
    prims = random_planes(rng, K, W, H)
    if spheres:
        prims += random_spheres(rng, K, W, H)
    R_gt = rot_from_rotvec(random_unit(rng) * rot_deg * DEG)
    t_gt = random_unit(rng) * trans_m
    T_gt = pose_matrix(R_gt, t_gt)
    imu_R = rot_from_rotvec(random_unit(rng) * imu_deg * DEG) @ R_gt
    return make_pair_problem(prims, W, H, K, T_gt, imu_R, rng, noise=noise,
                             dropout=0.02 if noise else 0.0, name=f"pair/seed{seed}")


def three_plane_problem(seed=0, W=160, H=120, f=130.0, rot_deg=2.0, trans_m=0.02):
    """Noiseless scene of three planes in general position (pairwise normal
    angle above 30 degrees, each covering at least 15% of the image)."""
    rng = _rng(11, seed)
    K = centred_intrinsics(W, H, f)
    planes = random_planes(rng, K, W, H, cone_deg=60.0, min_cover=0.15, min_pair_deg=30.0,
                           tries=5000)
    R_gt = rot_from_rotvec(random_unit(rng) * rot_deg * DEG)
    t_gt = random_unit(rng) * trans_m
    T_gt = pose_matrix(R_gt, t_gt)
    return make_pair_problem(planes, W, H, K, T_gt, R_gt.copy(), rng, noise=False, dropout=0.0,
                             name=f"planes3/seed{seed}")


BATCH_RESOLUTIONS = ((320, 240), (640, 480), (848, 480), (1280, 720))


def uneven_problem(index, seed=0):
    """One of the 64 uneven batched problems: resolution uniform over
    320x240 / 640x480 / 848x480 / 1280x720, f = 525 H / 480, single-pair scene
    type, motion up to 5 deg / 5 cm, IMU prior noise U(0.3, 1.0) deg."""
    rng = _rng(4, seed, index)
    W, H = BATCH_RESOLUTIONS[int(rng.integers(0, len(BATCH_RESOLUTIONS)))]
    K = centred_intrinsics(W, H, 525.0 * H / 480.0)
    prims = random_planes(rng, K, W, H) + random_spheres(rng, K, W, H)
    R_gt = rot_from_rotvec(random_unit(rng) * rng.uniform(0.0, 5.0) * DEG)
    t_gt = random_unit(rng) * rng.uniform(0.0, 0.05)
    T_gt = pose_matrix(R_gt, t_gt)
    imu_R = rot_from_rotvec(random_unit(rng) * rng.uniform(0.3, 1.0) * DEG) @ R_gt
    return make_pair_problem(prims, W, H, K, T_gt, imu_R, rng, name=f"uneven/{index}")


# ----------------------------------------------------------------------------
# Kinect-scale room sequence
# ----------------------------------------------------------------------------

ROOM_HALF = np.array([3.0, 1.5, 3.0])  # 6 m x 3 m x 6 m, y down


def room_scene(rng, n_objects=20):
    """Six inward-facing walls plus random boxes and spheres (0.2-0.8 m)."""
    prims = []
    for ax in range(3):
        for sgn in (-1.0, 1.0):
            # wall X_ax = sgn * half with inward normal -sgn e_ax: n.X = -half
            n = np.zeros(3)
            n[ax] = -sgn
            prims.append(Plane(n=n, c=float(-ROOM_HALF[ax])))
    placed = 0
    while placed < n_objects:
        size = rng.uniform(0.2, 0.8)
        pos = rng.uniform(-ROOM_HALF + 0.5, ROOM_HALF - 0.5)
        if math.hypot(pos[0], pos[2]) < 1.6:
            continue  # keep the camera's working volume clear
        if rng.random() < 0.5:
            prims.append(Sphere(centre=pos, radius=size / 2))
        else:
            half = rng.uniform(0.1, 0.4, size=3)
            prims.append(Box(lo=pos - half, hi=pos + half))
        placed += 1
    return prims


def room_trajectory(rng, n_frames, max_deg=3.0, max_m=0.03):
    """Smooth random camera-to-world poses; per-frame steps are at most
    `max_deg` degrees and `max_m` metres.  Angular and linear velocities follow
    low-pass filtered random walks with a pull toward a level camera near the
    room centre."""
    R = np.eye(3)
    t = np.zeros(3)
    w = np.zeros(3)
    v = np.zeros(3)
    poses = [pose_matrix(R, t)]
    for _ in range(n_frames - 1):
        # body-frame angular velocity, yaw-dominant
        w = 0.9 * w + 0.1 * rng.normal(size=3) * np.array([1.0, 4.0, 1.0]) * DEG
        # pull pitch/roll back: rotate the camera's y axis toward world down
        down_c = R.T @ np.array([0.0, 1.0, 0.0])
        w += 0.02 * np.cross(np.array([0.0, 1.0, 0.0]), down_c)
        ang = np.linalg.norm(w)
        if ang > max_deg * DEG:
            w *= max_deg * DEG / ang
        # world-frame linear velocity with a spring toward the centre
        v = 0.9 * v + 0.1 * (rng.normal(size=3) * 0.03 - 0.1 * t * np.array([1.0, 2.0, 1.0]))
        mag = np.linalg.norm(v)
        if mag > max_m:
            v *= max_m / mag
        R = R @ rot_from_rotvec(w)
        t = t + v
        poses.append(pose_matrix(R, t))
    return poses


class RoomSequence:
    """Kinect-scale sequence: 640x480, fx = fy = 525, a 6x3x6 m room with 20
    objects, smooth trajectory (<= 3 deg, <= 3 cm per frame), sensor noise and
    2% dropouts, IMU = truth perturbed by a N(0, (0.5 deg)^2) angle about a
    random axis.  Registration k (1 <= k < n_frames) aligns frame k against
    model maps rendered at the previous true pose, so all registrations are
    independent."""

    def __init__(self, seed=0, n_frames=300, W=640, H=480, f=525.0, imu_sigma_deg=0.5):
        self.seed, self.n_frames, self.W, self.H = seed, n_frames, W, H
        self.K = centred_intrinsics(W, H, f)
        rng = _rng(2, seed)
        self.prims = room_scene(rng)
        self.poses = room_trajectory(rng, n_frames)
        self.imu_sigma = imu_sigma_deg * DEG
        self._cache = {}

    def __len__(self):
        return self.n_frames - 1

    def _render(self, i):
        """Noise-free render at true pose i; the last two are kept so that a
        sequential walk renders each pose once."""
        hit = self._cache.get(i)
        if hit is None:
            hit = render(self.prims, self.W, self.H, self.K, self.poses[i])
            self._cache = {j: v for j, v in self._cache.items() if j >= i - 1}
            self._cache[i] = hit
        return hit

    def frame(self, k):
        """Frame k for tracking against a reconstruction: (noisy depth float32,
        IMU orientation in the world, true camera-to-world pose).  For k >= 1
        the depth and IMU equal those of problem(k - 1)."""
        if not 0 <= k < self.n_frames:
            raise IndexError(k)
        rng = _rng(2, self.seed, k) if k > 0 else _rng(2, self.seed, 0, 1)
        P = self.poses[k]
        d, _, _, _ = self._render(k)
        d = add_sensor_noise(d, rng)
        R_imu_world = rot_from_rotvec(random_unit(rng) * rng.normal() * self.imu_sigma) @ P[:3, :3]
        return d.astype(np.float32), R_imu_world, P

    def problem(self, k):
        """Registration of frame k+1 against model maps of frame k (0-based k)."""
        if not 0 <= k < self.n_frames - 1:
            raise IndexError(k)
        rng = _rng(2, self.seed, k + 1)
        P0, P1 = self.poses[k], self.poses[k + 1]
        _, mv, mn, _ = self._render(k)
        ld, _, _, _ = self._render(k + 1)
        ld = add_sensor_noise(ld, rng)
        T_rel = np.linalg.inv(P0) @ P1
        R_imu_world = rot_from_rotvec(random_unit(rng) * rng.normal() * self.imu_sigma) @ P1[:3, :3]
        imu_R = P0[:3, :3].T @ R_imu_world
        return Problem(live_depth=ld.astype(np.float32), model_vtx=mv.astype(np.float32),
                       model_nrm=mn.astype(np.float32), K=self.K, imu_R=imu_R,
                       init_pose=np.eye(4), T_gt=T_rel, name=f"room/{self.seed}/{k + 1}")
