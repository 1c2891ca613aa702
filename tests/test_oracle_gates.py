"""Pins of the oracle's projective association (paper Sec. 3: the live point
moved by the current pose, projected into the model image, paired with the
model point and normal at the nearest pixel, then gated), of the per-level
intrinsics of the pyramid, and of the margin that the GPU parity tests use to
excuse decisions within rounding of a threshold.

Every case is a hand-made level whose values are dyadic, so each deciding
quantity is known exactly and sits just inside, exactly on, or just outside
its threshold.  The plausible mistakes each case rules out are named in its
docstring.
"""
import math

import numpy as np

import oracle
from synth.scene import centred_intrinsics

BIN_W = 2.0 ** -13


def _level(W, H, K):
    nan = np.full((3, H, W), np.nan, np.float32)
    return dict(LV=nan.copy(), LN=nan.copy(), MV=nan.copy(), MN=nan.copy(), K=np.asarray(K, np.float64))


def _set(m, u, v, xyz):
    m[:, v, u] = np.asarray(xyz, np.float32)


def _pose(R=None, t=(0.0, 0.0, 0.0)):
    T = np.eye(4)
    if R is not None:
        T[:3, :3] = R
    T[:3, 3] = t
    return T


def _one(lvl, T, dist_max=0.10, cos_max=None, u=0, v=0):
    code, bins, margin, hist = oracle.associate(lvl, T, dist_max=dist_max, cos_max=cos_max)
    return int(code[v, u]), int(bins[v, u]), float(margin[v, u]), hist


def _pair(W, H, K, p, n, q, nq, live_uv=(0, 0), model_uv=None):
    """A level with one live pixel (vertex p, normal n) and, when model_uv is
    given, one valid model pixel (q, n_q); everything else is NaN."""
    lvl = _level(W, H, K)
    _set(lvl["LV"], *live_uv, p)
    _set(lvl["LN"], *live_uv, n)
    if model_uv is not None:
        _set(lvl["MV"], *model_uv, q)
        _set(lvl["MN"], *model_uv, nq)
    return lvl


# K = (fx, fy, cx, cy) with powers of two, so projections are exact
K_EXACT = (128.0, 128.0, 3.0, 2.0)
Z = 2.0
DOWN = (0.0, 0.0, -1.0)


def test_distance_gate_is_strict_on_the_squared_distance():
    """Gate d^2 < d_max^2.  With d_max = 1/16 (its square exact) a pair at
    exactly 1/16 is FAR and one at the next float32 below it is GATED; with
    d_max = 0.1 the float32 neighbours of 0.1 fall on either side.  Rules out
    `<=` for `<` and comparing d^2 with d_max unsquared (which would gate a
    pair at 0.1 + 1 ulp)."""
    W, H = 8, 5
    p = (0.0, 0.0, Z)  # projects onto the principal point (3, 2)
    cases = [
        (0.0625, np.float32(0.0625), oracle.FAR),
        (0.0625, np.nextafter(np.float32(0.0625), np.float32(0)), oracle.GATED),
        (0.10, np.nextafter(np.float32(0.1), np.float32(1)), oracle.FAR),
        (0.10, np.float32(0.1), oracle.FAR),  # float32(0.1) = 0.100000001490116...
        (0.10, np.nextafter(np.float32(0.1), np.float32(0)), oracle.GATED),
    ]
    for dmax, dx, want in cases:
        q = (float(dx), 0.0, Z)
        lvl = _pair(W, H, K_EXACT, p, DOWN, q, DOWN, live_uv=(1, 1), model_uv=(3, 2))
        code, b, _, _ = _one(lvl, _pose(), dist_max=dmax, u=1, v=1)
        assert code == want, (dmax, float(dx), code)
        if want == oracle.GATED:
            # bin of d: the unique k with (k w)^2 <= d^2 < ((k+1) w)^2
            assert b == math.floor(float(dx) / BIN_W)


def _tilt(m, towards, theta):
    """Unit vector at angle theta from m, in the plane of m and `towards`
    (towards it for theta > 0, away for theta < 0)."""
    e = towards - np.dot(towards, m) * m
    e /= np.linalg.norm(e)
    return math.cos(theta) * m + math.sin(theta) * e


def _rot_z(phi):
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def test_angle_gate_uses_the_rotated_live_normal():
    """Gate (R n) . n_q >= cos 20 deg.  The live point sits on the optical axis
    and the pose rotates about that axis by 60 deg, so p' = p while R n is
    29 deg away from n.  A model normal 19.99 deg from R n (tilted away from
    n) is GATED and one 20.01 deg from it (tilted towards n) is ANGLE; testing
    the unrotated normal n would give the opposite code in both cases."""
    W, H = 8, 5
    cos20 = math.cos(math.radians(20.0))
    a = math.radians(30.0)
    n = np.array([math.sin(a), 0.0, -math.cos(a)])
    R = _rot_z(math.radians(60.0))
    m = R @ n
    assert math.degrees(math.acos(np.dot(n, m))) > 28.9
    p = (0.0, 0.0, Z)
    for deg, sign, want in [(19.99, -1.0, oracle.GATED), (20.01, +1.0, oracle.ANGLE)]:
        nq = _tilt(m, n, sign * math.radians(deg))
        lvl = _pair(W, H, K_EXACT, p, n, p, nq, live_uv=(0, 0), model_uv=(3, 2))
        code, b, _, _ = _one(lvl, _pose(R), cos_max=cos20)
        assert code == want, (deg, code)
        # the mistaken gate on the unrotated normal decides the other way
        unrot = float(np.dot(n, nq.astype(np.float32)))
        assert (unrot >= cos20) == (want != oracle.GATED)


def test_angle_gate_is_inclusive():
    """cos exactly equal to the threshold is GATED (>=, not >): n = (0,0,-1)
    and n_q = (sqrt(3)/2, 0, -1/2) give a dot product of exactly 1/2."""
    W, H = 8, 5
    p = (0.0, 0.0, Z)
    nq = (math.sqrt(3.0) / 2.0, 0.0, -0.5)
    lvl = _pair(W, H, K_EXACT, p, DOWN, p, nq, model_uv=(3, 2))
    assert _one(lvl, _pose(), cos_max=0.5)[0] == oracle.GATED
    assert _one(lvl, _pose(), cos_max=np.nextafter(0.5, 1.0))[0] == oracle.ANGLE


def test_behind_the_camera():
    """p'_z <= 0 is BEHIND (p'_z = 0 included; `p'_z >= 0` would let it
    through to a division by zero); p'_z = 1/16 projects normally.  The margin
    of a BEHIND pixel is |p'_z|."""
    W, H = 8, 5
    p = (0.0, 0.0, Z)
    for tz, want in [(-3.0, oracle.BEHIND), (-2.0, oracle.BEHIND), (-1.9375, oracle.GATED)]:
        lvl = _pair(W, H, K_EXACT, p, DOWN, (0.0, 0.0, Z + tz), DOWN, model_uv=(3, 2))
        code, _, margin, _ = _one(lvl, _pose(t=(0.0, 0.0, tz)))
        assert code == want, (tz, code)
        if want == oracle.BEHIND:
            assert margin == abs(Z + tz)


def test_invalid_live_and_model_pixels():
    """A NaN in any one of the six model components makes the pixel
    INVALID_MODEL; a NaN in the live vertex or normal makes it INVALID_LIVE
    (checked before anything else)."""
    W, H = 8, 5
    p = (0.0, 0.0, Z)
    lvl = _pair(W, H, K_EXACT, p, DOWN, p, DOWN, model_uv=(3, 2))
    assert _one(lvl, _pose())[0] == oracle.GATED
    for which in ("MV", "MN"):
        for c in range(3):
            bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in lvl.items()}
            bad[which][c, 2, 3] = np.nan
            assert _one(bad, _pose())[0] == oracle.INVALID_MODEL, (which, c)
    for which in ("LV", "LN"):
        for c in range(3):
            bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in lvl.items()}
            bad[which][c, 0, 0] = np.nan
            assert _one(bad, _pose())[0] == oracle.INVALID_LIVE, (which, c)


def test_half_pixel_projections_round_up():
    """iu = floor(u + 1/2): a projection exactly on u = 4.5 pairs with column 5
    (round-half-to-even and truncation would take column 4), u = -0.5 lands
    in column 0 (rounding half away from zero would leave the image), and
    u = W - 1/2 falls outside.  The same holds for rows.  Every model pixel is
    valid and lies 4 (1 + u + W v) bins from p', so the bin names the pixel
    the rounding picked."""
    W, H = 8, 6
    fx = 128.0
    half = 0.5 * Z / fx  # lateral offset of half a pixel at depth Z: 2^-7
    # (cx, cy, x, y) -> expected model pixel (None: OUTSIDE)
    cases = [
        ((4.0, 2.0), (+half, 0.0), (5, 2)),
        ((0.0, 2.0), (-half, 0.0), (0, 2)),
        ((W - 1.0, 2.0), (+half, 0.0), None),
        ((3.0, 3.0), (0.0, +half), (3, 4)),
        ((3.0, 0.0), (0.0, -half), (3, 0)),
        ((3.0, H - 1.0), (0.0, +half), None),
    ]
    for (cx, cy), (x, y), want in cases:
        K = (fx, fx, cx, cy)
        p = (x, y, Z)
        lvl = _level(W, H, K)
        _set(lvl["LV"], 0, 0, p)
        _set(lvl["LN"], 0, 0, DOWN)
        for vv in range(H):
            for uu in range(W):
                dk = 4.0 * (1 + uu + W * vv) * BIN_W
                assert float(np.float32(x + dk)) == x + dk
                _set(lvl["MV"], uu, vv, (x + dk, y, Z))
                _set(lvl["MN"], uu, vv, DOWN)
        code, b, _, _ = _one(lvl, _pose())
        if want is None:
            assert code == oracle.OUTSIDE, (cx, cy, x, y)
            continue
        assert code == oracle.GATED, (cx, cy, x, y, code)
        uu, vv = want
        assert b == 4 * (1 + uu + W * vv), (cx, cy, x, y, b)


def test_level_intrinsics_hand_values():
    """The level intrinsics of the 160x120 pair (f = 130, centre (79.5, 59.5)):
    level 1 is (65, 65, 39.5, 29.5) and level 2 (32.5, 32.5, 19.5, 14.5) --
    the centre of the level-(l+1) pixel is the mean of its four children's
    centres, so it stays the image centre ((W_l - 1)/2)."""
    K0 = (130.0, 130.0, 79.5, 59.5)
    assert list(oracle.level_intrinsics(K0, 0)) == list(K0)
    assert list(oracle.level_intrinsics(K0, 1)) == [65.0, 65.0, 39.5, 29.5]
    assert list(oracle.level_intrinsics(K0, 2)) == [32.5, 32.5, 19.5, 14.5]
    K = centred_intrinsics(640, 480, 525.0)
    for lvl in range(4):
        Kl = oracle.level_intrinsics(K, lvl)
        assert Kl[2] == ((640 >> lvl) - 1) / 2 and Kl[3] == ((480 >> lvl) - 1) / 2


def test_coarse_vertices_are_the_mean_of_their_children():
    """Pixel-centre convention of the pyramid: for a constant-depth image (a
    fronto-parallel plane) the vertex that level l back-projects from the
    2x2-averaged depth is the mean of the 2^l x 2^l level-0 vertices it covers.
    Scaling the principal point as c / 2^l instead would shift every coarse
    vertex by half a fine pixel."""
    W, H = 32, 24
    K = (40.0, 36.0, 13.25, 10.5)  # off-centre on purpose
    z = np.float32(2.0)
    depth = np.full((H, W), z, np.float32)
    lv = oracle.pyramids(depth, np.zeros((H, W, 3), np.float32), np.zeros((H, W, 3), np.float32), K, 3)
    V0 = lv[0]["LV"].astype(np.float64)
    for lvl in (1, 2):
        s = 1 << lvl
        Vl = lv[lvl]["LV"].astype(np.float64)
        mean = V0.reshape(3, H // s, s, W // s, s).mean(axis=(2, 4))
        assert np.max(np.abs(Vl - mean)) < 1e-6, lvl


def test_margin_closed_form():
    """The margin of a GATED pixel is the smallest of: p'_z, the lateral metres
    to the pixel-rounding edge ((1/2 - |u - iu|) z / f, both axes), |d - d_max|,
    |cos - cos_max| and the distances of d to its bin's two edges.  Each case
    makes a different one the smallest, with dyadic values so it is exact."""
    W, H = 8, 6
    fx = 128.0
    cos_max = 0.5
    # (x, y) of p' (depth Z, principal point (0, 0)), d along x, n_q, d_max -> expected margin
    w = BIN_W
    s = float(np.float32(math.sqrt(1.0 - (0.5 + 2.0 ** -20) ** 2)))
    cases = [
        # bin edges: d = 192.5 w, half a bin from each edge; u = 2.25
        (2.25, 1.0, 192.5 * w, DOWN, 0.10, 0.5 * w),
        # pixel edge: u = 2.5 - 2^-12 -> (2^-12) * Z / fx = 2^-18
        (2.5 - 2.0 ** -12, 1.0, 100.5 * w, DOWN, 0.10, 2.0 ** -12 * Z / fx),
        # row edge: v = 1.5 - 2^-11 -> 2^-17
        (2.0, 1.5 - 2.0 ** -11, 100.5 * w, DOWN, 0.10, 2.0 ** -11 * Z / fx),
        # angle: cos = 1/2 + 2^-20 -> 2^-20
        (2.0, 1.0, 100.5 * w, (s, 0.0, -(0.5 + 2.0 ** -20)), 0.10, 2.0 ** -20),
        # distance gate: d = d_max - 2^-22 with d_max = 1/16 - 2^-16
        (2.0, 1.0, 2.0 ** -4 - 2.0 ** -16 - 2.0 ** -22, DOWN, 2.0 ** -4 - 2.0 ** -16, 2.0 ** -22),
    ]
    for u, v, d, nq, dmax, want in cases:
        x, y = u * Z / fx, v * Z / fx
        p = (x, y, Z)
        q = (x + d, y, Z)
        K = (fx, fx, 0.0, 0.0)
        iu, iv = math.floor(u + 0.5), math.floor(v + 0.5)
        lvl = _pair(W, H, K, p, DOWN, q, nq, model_uv=(iu, iv))
        assert float(np.float32(x)) == x and float(np.float32(x + d)) == x + d
        code, b, margin, _ = _one(lvl, _pose(), dist_max=dmax, cos_max=cos_max)
        assert code == oracle.GATED, (u, v, d, code)
        assert margin == want, (u, v, d, margin, want)


def test_histogram_counts_exactly_the_gated_pixels():
    """The histogram holds one count per GATED pixel, in its bin, and nothing
    for pixels with any other code.  Live pixels of one level are made to end
    with every code: GATED at several distances, FAR, ANGLE, OUTSIDE, BEHIND,
    INVALID_MODEL and INVALID_LIVE."""
    W, H = 8, 6
    lvl = _level(W, H, K_EXACT)
    _set(lvl["MV"], 3, 2, (0.05, 0.0, Z))  # the model pixel under the principal point
    _set(lvl["MN"], 3, 2, DOWN)
    tilt = (math.sin(math.radians(45.0)), 0.0, -math.cos(math.radians(45.0)))
    kinds = []
    for k in range(W * H):
        u, v = k % W, k // W
        kind = k % 7
        p, n = (0.0, 0.0, Z + 2.0 ** -9 * (k % 5)), DOWN  # GATED at distances hypot(0.05, dz)
        if kind == 1:
            p = (0.0, 0.0, Z + 0.25)  # FAR
        elif kind == 2:
            n = tilt  # ANGLE
        elif kind == 3:
            p = (2.0, 0.0, Z)  # OUTSIDE (u = 131)
        elif kind == 4:
            p = (0.0, 0.0, -1.0)  # BEHIND
        elif kind == 5:
            p = (Z / 128.0, 0.0, Z)  # projects onto (4, 2): INVALID_MODEL
        elif kind == 6:
            n = (np.nan, 0.0, -1.0)  # INVALID_LIVE
        _set(lvl["LV"], u, v, p)
        _set(lvl["LN"], u, v, n)
        kinds.append(kind)
    code, bins, _, hist = oracle.associate(lvl, _pose())
    want_code = [oracle.GATED, oracle.FAR, oracle.ANGLE, oracle.OUTSIDE, oracle.BEHIND, oracle.INVALID_MODEL,
                 oracle.INVALID_LIVE]
    assert [int(c) for c in code.reshape(-1)] == [want_code[k] for k in kinds]
    gated = code == oracle.GATED
    assert len(set(bins[gated].tolist())) > 2
    assert np.array_equal(hist, np.bincount(bins[gated], minlength=oracle.BINS))
    assert np.all(bins[~gated] == -1)
