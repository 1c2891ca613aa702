"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-worked
fixtures, closed forms, exact rational arithmetic, library routines (lstsq,
expm, partition) and invariants the method must satisfy.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth
from synth.scene import Plane, centred_intrinsics, render
from tests.poseutil import pose_err, rot_angle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


# --------------------------------------------------------------- pyramids

def test_depth_pyramid_golden():
    rows = _golden_rows("pyramid_4x4.txt")
    depth = np.array([[float(x) for x in r.split()] for r in rows[:4]], np.float32)
    want = np.array([[float(x) for x in r.split()] for r in rows[4:6]], np.float32)
    got = oracle.depth_down(depth)
    assert np.array_equal(got, want)


def test_depth_pyramid_invalid_children():
    d = np.full((4, 4), 2.0, np.float32)
    d[0, 0] = np.nan
    d[2, 3] = -1.0
    d[3, 0] = np.inf
    got = oracle.depth_down(d)
    assert got[0, 0] == 0 and got[1, 1] == 0 and got[1, 0] == 0 and got[0, 1] == 2.0


def test_model_pyramid_mean_and_normal():
    V = np.zeros((3, 2, 4), np.float32)
    N = np.zeros((3, 2, 4), np.float32)
    # left quad: vertices around (2, 1, 2); normals three times -z and one tilted
    V[:, 0, 0] = (1, 0, 2)
    V[:, 0, 1] = (3, 0, 2)
    V[:, 1, 0] = (1, 2, 2)
    V[:, 1, 1] = (3, 2, 2)
    for (v, u) in [(0, 0), (0, 1), (1, 0)]:
        N[:, v, u] = (0, 0, -1)
    N[:, 1, 1] = (0.6, 0.0, -0.8)
    # right quad: one child invalid
    V[:, :, 2:] = 1.0
    N[:, :, 2:] = (np.array([0, 0, -1.0], np.float32))[:, None, None]
    V[1, 1, 3] = np.nan
    vtx = np.moveaxis(V, 0, -1)
    nrm = np.moveaxis(N, 0, -1)
    MV, MN = oracle.model_l0(vtx, nrm)
    assert np.all(np.isnan(MV[:, 1, 3])) and np.all(np.isnan(MN[:, 1, 3]))
    Vn, Nn = oracle.model_down(MV, MN)
    assert np.array_equal(Vn[:, 0, 0], np.array([2, 1, 2], np.float32))
    s = np.array([0.6, 0.0, -3.8])
    n = Nn[:, 0, 0].astype(np.float64)
    assert abs(np.linalg.norm(n) - 1) < 1e-7
    assert np.linalg.norm(np.cross(n, s)) < 1e-6 * np.linalg.norm(s) and n @ s > 0
    assert np.all(np.isnan(Vn[:, 0, 1])) and np.all(np.isnan(Nn[:, 0, 1]))


def _plane_depth(W, H, K, n, c):
    pl = Plane(n=np.asarray(n, float) / np.linalg.norm(n), c=c)
    d, _, _, _ = render([pl], W, H, K, np.eye(4), zmin=0.0, zmax=np.inf)
    return pl, d.astype(np.float32)


def test_live_maps_on_plane():
    """P1: back-projected vertices lie on the rendered plane and on their pixel
    rays; forward-difference normals equal the plane normal (facing the camera);
    the last row and column have no normal."""
    W, H = 40, 30
    K = centred_intrinsics(W, H, 35.0)
    pl, d = _plane_depth(W, H, K, (0.3, -0.2, -1.0), -2.5)
    V, N = oracle.live_vn(d, K)
    assert np.array_equal(V[2], d)
    Vd = V.astype(np.float64)
    assert np.max(np.abs(np.einsum("k,khw->hw", pl.n, Vd) - pl.c)) < 4e-7 * 4
    u = np.arange(W)[None, :]
    v = np.arange(H)[:, None]
    assert np.max(np.abs(Vd[0] / Vd[2] - (u - K[2]) / K[0])) < 1e-6
    assert np.max(np.abs(Vd[1] / Vd[2] - (v - K[3]) / K[1])) < 1e-6
    Ni = N[:, :-1, :-1].astype(np.float64)
    want = pl.n if pl.n[2] < 0 else -pl.n
    assert np.max(np.abs(Ni - want[:, None, None])) < 1e-4
    assert np.all(np.einsum("khw,khw->hw", Ni, Vd[:, :-1, :-1]) < 0)
    assert np.all(np.isnan(N[:, -1, :])) and np.all(np.isnan(N[:, :, -1]))


def test_bilateral_keeps_constants_steps_and_holes():
    """P13: a constant image is a fixed point; across a depth step larger than
    the range cut-off no weight flows, so two constant sides stay exact; an
    invalid pixel stays invalid (0) and is not used by its neighbours."""
    D = np.full((30, 40), 2.0, np.float32)
    D[:, 20:] = 2.3  # 0.3 m step > 0.05 m cut-off
    D[10, 5] = 0.0
    D[12, 30] = np.nan
    out = oracle.bilateral(D, r=3, sigma_px=4.5, sigma_m=0.05)
    valid = np.isfinite(D) & (D > 0)
    assert np.array_equal(out[valid], D[valid])
    assert out[10, 5] == 0.0 and out[12, 30] == 0.0


def test_bilateral_reproduces_a_ramp_and_smooths_noise():
    """P14: with symmetric weights a linear depth ramp is reproduced away from
    the border (to rounding), and zero-mean noise shrinks: the filter is a
    normalised, symmetric local average."""
    H, W = 40, 60
    u = np.arange(W)[None, :]
    v = np.arange(H)[:, None]
    ramp = (2.0 + 0.001 * u + 0.0005 * v).astype(np.float32) + np.zeros((H, W), np.float32)
    out = oracle.bilateral(ramp, r=3, sigma_px=4.5, sigma_m=0.05)
    inner = (slice(3, H - 3), slice(3, W - 3))
    assert np.max(np.abs(out[inner].astype(np.float64) - ramp[inner])) < 1e-6
    rng = np.random.default_rng(4)
    noisy = (2.0 + rng.normal(0, 0.005, (H, W))).astype(np.float32)
    sm = oracle.bilateral(noisy, r=3, sigma_px=4.5, sigma_m=0.05)
    assert np.std(sm[inner] - 2.0) < 0.3 * np.std(noisy[inner] - 2.0)


def test_box_normals_on_plane_and_holes():
    """P15: box-average 3D-gradient normals equal the normal of a rendered
    plane (facing the camera); pixels whose box leaves the image or contains
    an invalid pixel have none (a hole removes exactly its (2r+1)^2 box)."""
    W, H, r = 40, 30, 2
    K = centred_intrinsics(W, H, 35.0)
    pl, d = _plane_depth(W, H, K, (0.3, -0.2, -1.0), -2.5)
    V, N = oracle.live_vn_box(d, K, r)
    Vf, _ = oracle.live_vn(d, K)
    assert np.array_equal(V, Vf)  # same vertices as the forward-difference maps
    want = pl.n if pl.n[2] < 0 else -pl.n
    inner = N[:, r:H - r, r:W - r].astype(np.float64)
    assert np.max(np.abs(inner - want[:, None, None])) < 1e-5
    assert np.all(np.isnan(N[:, :r, :])) and np.all(np.isnan(N[:, :, -r:]))
    # holes: a pixel keeps its normal while half of each half box is valid;
    # the means over valid pixels still give the plane normal
    d2 = d.copy()
    d2[15, 20] = 0.0
    d2[15, 21] = 0.0
    _, N2 = oracle.live_vn_box(d2, K, r)
    assert np.isnan(N2[0, 15, 20]) and np.isnan(N2[0, 15, 21])
    ok = ~np.isnan(N2[0])
    assert ok[14, 20] and ok[16, 21]
    assert np.max(np.abs(N2[:, ok].astype(np.float64) - want[:, None])) < 1e-5
    d3 = d.copy()
    d3[10:20, 19:22] = 0.0  # an invalid block, columns 19..21
    _, N3 = oracle.live_vn_box(d3, K, r)
    assert np.isnan(N3[0, 15, 18])  # right half (columns 19..20) all invalid
    assert not np.isnan(N3[0, 15, 17])  # right half (columns 18..19): 5 of 10 valid, enough



def test_paper_front_end_registration():
    """P16: with box normals the oracle recovers the true motion of a noiseless
    three-plane scene exactly as with forward differences (the live normals
    only gate; the residuals vanish at the truth); with the bilateral filter as
    well it stays within the bias the smoothing puts on the creases between
    planes (0.5 mrad, 1 mm); on a noisy config-1 scene more pairs pass the
    normal gate than with raw forward differences."""
    prob = synth.three_plane_problem(2)
    p = oracle.default_params(normal_mode=1, lambda_c=0.0, iters=(20, 10, 10))
    T, st, _ = oracle.register_problem(prob, p)
    ang, dt = pose_err(T, prob.T_gt)
    assert ang < 1e-6 and dt < 1e-6, (ang, dt)
    p = oracle.default_params(depth_filter=1, normal_mode=1, lambda_c=0.0, iters=(20, 10, 10))
    T, st, _ = oracle.register_problem(prob, p)
    ang, dt = pose_err(T, prob.T_gt)
    assert ang < 5e-4 and dt < 1e-3, (ang, dt)
    noisy = synth.pair_problem(3)
    _, s0, _ = oracle.register_problem(noisy, oracle.default_params())
    _, s1, _ = oracle.register_problem(noisy, oracle.default_params(depth_filter=1, normal_mode=1))
    assert s1[0]["n_gated"] > s0[0]["n_gated"]


# --------------------------------------------------------------- bins / band

def test_bin_is_exact_definition():
    """k is the unique integer with (k w)^2 <= d^2 < ((k+1) w)^2, checked in
    exact rational arithmetic, including values on and next to bin edges."""
    rng = np.random.default_rng(5)
    w = Fraction(1, 8192)
    vals = list(rng.uniform(0, 0.1, 2000) ** 2)
    for k in [0, 1, 2, 31, 500, 818, 819]:
        e = float((k * w) ** 2)
        vals += [e, np.nextafter(e, 0.0), np.nextafter(e, 1.0)]
    for d2 in vals:
        k = oracle.bin_of(d2)
        f = Fraction(d2)
        assert (k * w) ** 2 <= f < ((k + 1) * w) ** 2, (d2, k)


def test_band_golden():
    for row in _golden_rows("band_cases.txt"):
        beta, pairs, want = (s.strip() for s in row.split(";"))
        hist = np.zeros(oracle.BINS, np.uint32)
        for pr in pairs.split():
            k, c = pr.split(":")
            hist[int(k)] = int(c)
        got = oracle.band(hist, 1, float(beta))
        assert list(got) == [int(x) for x in want.split()], row


def test_band_median_matches_partition():
    """The median bin equals the lower median (np.partition) of the multiset of
    bin indices the histogram counts."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        n = int(rng.integers(1, 3000))
        samples = np.minimum(rng.gamma(2.0, 40.0, n).astype(int), oracle.BINS - 1)
        hist = np.bincount(samples, minlength=oracle.BINS).astype(np.uint32)
        N, kmed, klo, khi = oracle.band(hist)
        m = (n + 1) // 2
        assert N == n
        assert kmed == np.partition(samples, m - 1)[m - 1]
        assert klo == 0 and khi == min(oracle.BINS - 1, 2 * kmed + 1)
    N, kmed, klo, khi = oracle.band(np.zeros(oracle.BINS, np.uint32))
    assert N == 0 and kmed == -1 and khi < klo
    N, kmed, klo, khi = oracle.band(np.bincount([3, 9], minlength=oracle.BINS), use_filter=0)
    assert (klo, khi) == (0, oracle.BINS - 1)


def test_band_properties_over_beta():
    """For any histogram and any band factor beta >= 0 the band contains the
    median bin, beta = 0 keeps exactly the median bin, beta >= 1 starts at bin
    0, and the kept count never shrinks as beta grows (hypothesis-generated
    histograms)."""
    from hypothesis import given, settings, strategies as st

    @settings(max_examples=150, deadline=None)
    @given(st.lists(st.integers(0, oracle.BINS - 1), min_size=1, max_size=400),
           st.lists(st.floats(0.0, 3.0, allow_nan=False), min_size=2, max_size=6))
    def check(samples, betas):
        hist = np.bincount(samples, minlength=oracle.BINS).astype(np.uint32)
        cdf = np.cumsum(hist)
        kept_prev = -1
        for beta in sorted(betas):
            N, kmed, klo, khi = oracle.band(hist, 1, beta)
            assert N == len(samples) and klo <= kmed <= khi <= oracle.BINS - 1
            if beta == 0.0:
                assert klo == kmed == khi
            if beta >= 1.0:
                assert klo == 0
            kept = int(cdf[khi] - (cdf[klo - 1] if klo > 0 else 0))
            assert kept >= kept_prev and kept >= int(hist[kmed]) > 0
            kept_prev = kept
        N, kmed, klo, khi = oracle.band(hist, 1, 0.0)
        assert cdf[kmed] >= (N + 1) // 2 and (kmed == 0 or cdf[kmed - 1] < (N + 1) // 2)

    check()


# --------------------------------------------------------------- association

def _tiny_level(W=24, H=18, f=20.0, seed=3, T=None):
    """One pyramid level of a tiny config-1-like scene (planes plus spheres)."""
    rng = np.random.default_rng(seed)
    K = centred_intrinsics(W, H, f)
    from synth.scene import random_planes, random_spheres
    prims = random_planes(rng, K, W, H) + random_spheres(rng, K, W, H)
    T = np.eye(4) if T is None else T
    _, mv, mn, _ = render(prims, W, H, K, np.eye(4))
    ld, _, _, _ = render(prims, W, H, K, T)
    return oracle.pyramids(ld, mv, mn, K, 1)[0]


def test_identity_case():
    """P3: live maps used as model maps at T = I: every live pixel with a vertex
    and a normal matches itself, d = 0, median bin 0, b = 0, x = 0."""
    W, H = 32, 24
    K = centred_intrinsics(W, H, 25.0)
    d = _tiny_level(W, H, 25.0)["D"]
    LV, LN = oracle.live_vn(d, K)
    lvl = oracle.pyramids(d, np.moveaxis(LV, 0, -1), np.moveaxis(LN, 0, -1), K, 1)[0]
    code, bins, _, hist = oracle.associate(lvl, np.eye(4))
    has = np.isfinite(LV[0]) & np.isfinite(LN[0])
    assert has.sum() > 300
    assert np.all(code[has] == oracle.GATED) and np.all(code[~has] == oracle.INVALID_LIVE)
    assert np.all(bins[has] == 0) and hist[0] == has.sum() and hist.sum() == has.sum()
    N, kmed, klo, khi = oracle.band(hist)
    assert kmed == 0
    M, n = oracle.moments(lvl, np.eye(4), klo, khi)
    assert n == has.sum()
    assert all(M[oracle.tri_index(i, 6)] == 0.0 for i in range(7))
    st, T1, x = oracle.solve_update(M, n, np.eye(4), lambda_c=0.0)
    assert st == oracle.LEVEL_OK and np.all(x == 0.0) and np.array_equal(T1, np.eye(4))


def test_projection_closed_form():
    """P4: fronto-parallel plane at z0, model = live, lateral shift of
    3.25 z0/fx: interior pixels pair with the model pixel three columns to the
    right at distance 0.25 z0/fx, so every one lands in bin
    floor(0.25 z0/fx * 8192); the last three columns fall outside the image."""
    W, H, f, z0 = 40, 20, 130.0, 2.0
    K = centred_intrinsics(W, H, f)
    _, d = _plane_depth(W, H, K, (0, 0, -1.0), -z0)
    LV, LN = oracle.live_vn(d, K)
    _, mv, mn, _ = render([Plane(n=np.array([0, 0, -1.0]), c=-z0)], W, H, K, np.eye(4))
    lvl = oracle.pyramids(d, mv, mn, K, 1)[0]
    T = np.eye(4)
    T[0, 3] = 3.25 * z0 / f
    code, bins, margin, hist = oracle.associate(lvl, T)
    kexp = math.floor(0.25 * z0 / f * 8192)
    for v in range(H):
        for u in range(W):
            if u == W - 1 or v == H - 1:
                assert code[v, u] == oracle.INVALID_LIVE
            elif u >= W - 3:
                assert code[v, u] == oracle.OUTSIDE
            else:
                assert code[v, u] == oracle.GATED and bins[v, u] == kexp
    assert hist[kexp] == (W - 3) * (H - 1) and hist.sum() == hist[kexp]
    _, _, pp, q, nq = oracle.pairs(lvl, T)
    g = np.isfinite(pp[:, 0])
    assert np.allclose(np.linalg.norm(q[g] - pp[g], axis=1), 0.25 * z0 / f, atol=1e-6)


# --------------------------------------------------------------- moments / solve

def _kept_pairs(lvl, T):
    code, bins, pp, q, nq = oracle.pairs(lvl, T)
    hist = np.bincount(bins[code == oracle.GATED], minlength=oracle.BINS)
    N, kmed, klo, khi = oracle.band(hist)
    keep = (code == oracle.GATED) & (bins >= klo) & (bins <= khi)
    return pp[keep], q[keep], nq[keep], klo, khi


def _eq2_matrix(x):
    """The small-angle transform of Eq. (2), written as printed."""
    a, b, g, tx, ty, tz = x
    return np.array([[1, -g, b, tx], [g, 1, -a, ty], [-b, a, 1, tz], [0, 0, 0, 1.0]])


def _sym(M):
    H = np.zeros((7, 7))
    for i in range(7):
        for j in range(i, 7):
            H[i, j] = H[j, i] = M[oracle.tri_index(i, j)]
    return H


def test_moments_reproduce_point_to_plane_objective():
    """P6: for any increment x, the 28 moments give the Eq. (1) objective of the
    kept pairs under the Eq. (2) transform: sum (n.(M^ p' - q))^2 =
    x^T A^T A x - 2 x^T A^T b + b^T b.  Also: A^T A equals the explicit
    brute-force sum over rows, is symmetric and positive semi-definite."""
    T = synth.pose_matrix(synth.rot_from_rotvec([0.01, -0.02, 0.015]), [0.01, 0.0, -0.02])
    lvl = _tiny_level(T=T)
    pp, q, nq, klo, khi = _kept_pairs(lvl, np.eye(4))
    assert len(pp) > 50
    M, n = oracle.moments(lvl, np.eye(4), klo, khi)
    assert n == len(pp)
    S = _sym(M)
    rng = np.random.default_rng(0)
    for _ in range(60):
        x = rng.normal(size=6) * np.array([0.05, 0.05, 0.05, 0.1, 0.1, 0.1])
        Mh = _eq2_matrix(x)
        r = np.einsum("ik,ik->i", nq, pp @ Mh[:3, :3].T + Mh[:3, 3] - q)
        xe = np.append(x, -1.0)
        assert abs(np.sum(r * r) - xe @ S @ xe) <= 1e-10 * max(1.0, np.sum(r * r))
    A = np.hstack([np.cross(pp, nq), nq])
    b = np.einsum("ik,ik->i", nq, q - pp)
    assert np.allclose(S[:6, :6], A.T @ A, rtol=1e-12, atol=1e-12)
    assert np.allclose(S[:6, 6], A.T @ b, rtol=1e-12, atol=1e-15)
    ev = np.linalg.eigvalsh(S[:6, :6])
    assert ev.min() >= -1e-12 * ev.max()


@pytest.mark.parametrize("mode,c", [(oracle.LAMBDA_CONST, 0.0), (oracle.LAMBDA_CONST, 5.0),
                                    (oracle.LAMBDA_C_OVER_SQRT_N, 2.0), (oracle.LAMBDA_C_OVER_N, 1.0),
                                    (oracle.LAMBDA_C_OVER_N2, 0.2)])
def test_regularised_solve_matches_lstsq(mode, c):
    """P7/P8: x minimises Eq. (4), i.e. the least-squares solution (SVD, as in
    the paper) of [A; sqrt(2 n lambda) P] x = [b; 0] with P = [I3 | 0]; lambda = 0
    is plain point-to-plane least squares.  The update composes Exp(x) on the
    left of the pose."""
    T = synth.pose_matrix(synth.rot_from_rotvec([0.02, 0.01, -0.01]), [0.02, -0.01, 0.01])
    lvl = _tiny_level(T=T, seed=4)
    pp, q, nq, klo, khi = _kept_pairs(lvl, np.eye(4))
    M, n = oracle.moments(lvl, np.eye(4), klo, khi)
    A = np.hstack([np.cross(pp, nq), nq])
    b = np.einsum("ik,ik->i", nq, q - pp)
    lam = {oracle.LAMBDA_CONST: c, oracle.LAMBDA_C_OVER_SQRT_N: c / math.sqrt(n),
           oracle.LAMBDA_C_OVER_N: c / n, oracle.LAMBDA_C_OVER_N2: c / n ** 2}[mode]
    P = np.hstack([np.eye(3), np.zeros((3, 3))])
    As = np.vstack([A, math.sqrt(2 * n * lam) * P])
    bs = np.concatenate([b, np.zeros(3)])
    xref = np.linalg.lstsq(As, bs, rcond=None)[0]
    T0 = synth.pose_matrix(synth.rot_from_rotvec([0.1, 0.2, -0.3]), [0.5, -0.2, 1.0])
    st, T1, x = oracle.solve_update(M, n, T0, lambda_mode=mode, lambda_c=c)
    assert st == oracle.LEVEL_OK
    assert np.allclose(x, xref, rtol=1e-8, atol=1e-12)
    E = np.zeros((4, 4))
    E[:3, :3] = np.array([[0, -x[2], x[1]], [x[2], 0, -x[0]], [-x[1], x[0], 0]])
    E[:3, 3] = x[3:]
    assert np.allclose(T1, scipy.linalg.expm(E) @ T0, rtol=0, atol=1e-13)


def test_solver_flags_degenerate_systems():
    M = np.zeros(28)
    st, T1, x = oracle.solve_update(M, 100, np.eye(4), lambda_c=1.0)
    assert st == oracle.ILL_COND and np.array_equal(T1, np.eye(4))
    st, _, _ = oracle.solve_update(M, 5, np.eye(4))
    assert st == oracle.TOO_FEW_CORR


def test_se3_exp_matches_expm():
    """P10: the exponential of the 4x4 twist matrix (scipy expm), RtR = I, det 1."""
    rng = np.random.default_rng(1)
    for th in [0.0, 1e-9, 1e-7, 1e-6, 1.1e-6, 1e-5, 1e-3, 0.1, 1.0, 3.0]:
        for _ in range(5):
            ax = rng.normal(size=3)
            w = ax / np.linalg.norm(ax) * th
            tau = rng.normal(size=3)
            R, t = oracle.se3_exp(w, tau)
            E = np.zeros((4, 4))
            E[:3, :3] = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
            E[:3, 3] = tau
            X = scipy.linalg.expm(E)
            assert np.allclose(R, X[:3, :3], rtol=0, atol=2e-15)
            assert np.allclose(t, X[:3, 3], rtol=0, atol=1e-14 * max(1, np.linalg.norm(tau)))
            assert np.allclose(R.T @ R, np.eye(3), atol=1e-15) and abs(np.linalg.det(R) - 1) < 1e-15


# --------------------------------------------------------------- whole loop

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_truth_recovery_three_planes(seed):
    """P11: on noiseless renders of three planes in general position the loop
    converges to the ground-truth motion.  The floor is FP32 storage of the
    maps; the 2-degree normal gate drops the pixels on plane intersections whose
    forward-difference normals straddle two planes."""
    prob = synth.three_plane_problem(seed)
    p = oracle.default_params(lambda_c=0.0, cos_angle_max=math.cos(math.radians(2.0)))
    pose, st, _ = oracle.register_problem(prob, p)
    ang, dt = pose_err(pose, prob.T_gt)
    assert ang < 1e-6 and dt < 1e-6, (ang, dt)
    assert all(s["status"] == oracle.LEVEL_OK for s in st)


def test_large_lambda_pins_rotation_to_imu():
    """P9: lambda -> infinity keeps the rotation at the IMU seed; the loop then
    solves for the translation alone (its last increment vanishes)."""
    prob = synth.pair_problem(0)
    p = oracle.default_params(lambda_c=1e12, iters=(30, 5, 4))
    pose, st, tr = oracle.register_problem(prob, p)
    assert rot_angle(pose[:3, :3] @ prob.imu_R.T) < 1e-9
    assert np.linalg.norm(tr[-1]["x"][3:]) < 1e-6
    assert np.linalg.norm(tr[-1]["x"][:3]) < 1e-12


def test_so3_log_inverts_the_exponential():
    """P20: the rotation vector of Exp(w) is w again, from 1e-13 rad to nearly
    pi, and agrees with scipy's rotation vector of the same matrix."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(20)
    for ang in [0.0, 1e-13, 1e-9, 1e-5, 0.01, 0.3, 1.0, 2.0, 3.1]:
        ax = rng.normal(size=3)
        w = ax / np.linalg.norm(ax) * ang
        R, _ = oracle.se3_exp(w, np.zeros(3))
        v = oracle.so3_log(R)
        assert np.abs(v - w).max() <= 1e-14 * max(1.0, ang) + 1e-300, (ang, v, w)
        assert np.abs(v - Rotation.from_matrix(R).as_rotvec()).max() <= 1e-14, ang


def test_anchored_regulariser_stationarity():
    """P21: with the damping anchored to the IMU rotation (the reading that
    penalises the deviation w + Log(R imu_R^T) instead of each increment w),
    the iteration converges to the point where the moments' rotation rows
    equal 2 lambda n Log(R imu_R^T) and the translation rows vanish: the
    stationarity condition of (1/2n)|Ax - b|^2 + lambda |w + d|^2 at x = 0.
    Lambda = 0 leaves plain ICP, identical to the literal form."""
    prob = synth.pair_problem(3, noise=False)
    lam = 50.0
    p = oracle.default_params(levels=1, iters=[60], lambda_c=lam, anchor_to_imu=1)
    pose, st, tr = oracle.register_problem(prob, p)
    assert st[0]["status"] == oracle.LEVEL_OK and np.abs(tr[-1]["x"]).max() < 1e-12
    lv = oracle.pyramids(prob.live_depth, prob.model_vtx, prob.model_nrm, prob.K, 1)[0]
    _, _, _, hist = oracle.associate(lv, pose)
    _, _, klo, khi = oracle.band(hist)
    M, n = oracle.moments(lv, pose, klo, khi)
    g = np.array([M[oracle.tri_index(i, 6)] for i in range(6)])
    d = oracle.so3_log(pose[:3, :3] @ prob.imu_R.T)
    assert np.linalg.norm(g[:3]) > 1.0  # a real balance between the data and the prior
    assert np.abs(g[:3] - 2.0 * lam * n * d).max() < 1e-9 * np.abs(g[:3]).max()
    assert np.abs(g[3:]).max() < 1e-9 * np.abs(g[:3]).max()
    # the literal form with the same lambda ends farther from the IMU rotation
    pl, _, _ = oracle.register_problem(prob, oracle.default_params(levels=1, iters=[60], lambda_c=lam))
    assert rot_angle(pose[:3, :3] @ prob.imu_R.T) < 0.2 * rot_angle(pl[:3, :3] @ prob.imu_R.T)
    # lambda = 0: the anchor has no weight
    a0, _, _ = oracle.register_problem(prob, oracle.default_params(lambda_c=0.0, anchor_to_imu=1))
    l0, _, _ = oracle.register_problem(prob, oracle.default_params(lambda_c=0.0))
    assert np.array_equal(a0, l0)
    # the one-step solve: anchored right-hand side against lstsq of the stacked system
    T0 = np.eye(4)
    T0[:3, :3] = prob.imu_R @ synth.rot_from_rotvec([0.01, -0.02, 0.015])
    code, bins, pp, q, nq = oracle.pairs(lv, T0)
    keep = code.reshape(-1) == 6
    A = np.hstack([np.cross(pp[keep], nq[keep]), nq[keep]])
    b = np.einsum("ij,ij->i", nq[keep], q[keep] - pp[keep])
    nk = int(keep.sum())
    Mk = np.zeros(28)
    Ab = np.hstack([A, b[:, None]])
    for i in range(7):
        for j in range(i, 7):
            Mk[oracle.tri_index(i, j)] = Ab[:, i] @ Ab[:, j]
    _, _, x = oracle.solve_update(Mk, nk, T0, lambda_c=lam, imu_R=prob.imu_R)
    d0 = oracle.so3_log(T0[:3, :3] @ prob.imu_R.T)
    s = np.sqrt(2.0 * lam * nk)
    A_st = np.vstack([A, np.hstack([s * np.eye(3), np.zeros((3, 3))])])
    b_st = np.concatenate([b, -s * d0])
    x_ls = np.linalg.lstsq(A_st, b_st, rcond=None)[0]
    assert np.abs(x - x_ls).max() < 1e-9 * np.abs(x_ls).max()


def test_lambda_zero_corrects_imu_error():
    """Sec. 4.1: without regularisation the IMU error is corrected; with a large
    lambda the IMU rotation is kept."""
    prob = synth.pair_problem(0)
    imu_err = rot_angle(prob.imu_R @ prob.T_gt[:3, :3].T)
    pose0, _, _ = oracle.register_problem(prob, oracle.default_params(lambda_c=0.0))
    pose5, _, _ = oracle.register_problem(prob, oracle.default_params(lambda_c=5.0))
    e0 = pose_err(pose0, prob.T_gt)[0]
    e5 = pose_err(pose5, prob.T_gt)[0]
    assert e0 < 0.3 * imu_err and e0 < e5 <= imu_err * 1.01


def test_imu_seed_sets_initial_rotation():
    prob = synth.pair_problem(0)
    init = synth.pose_matrix(synth.rot_from_rotvec([0.1, 0, 0]), [0.1, 0.2, 0.3])
    p = oracle.default_params(iters=(0, 0, 0))
    pose, st, tr = oracle.register(prob.live_depth, prob.model_vtx, prob.model_nrm, prob.K, prob.imu_R, init, p)
    assert np.array_equal(pose[:3, :3], prob.imu_R) and np.array_equal(pose[:3, 3], init[:3, 3])
    p = oracle.default_params(iters=(0, 0, 0), use_imu_seed=0)
    pose, st, tr = oracle.register(prob.live_depth, prob.model_vtx, prob.model_nrm, prob.K, prob.imu_R, init, p)
    assert np.array_equal(pose, init)


def test_convergence_rule_stops_on_settled_median():
    """P12 (Sec. 3.4): with a window of 3 a level stops right after the first
    iteration whose median bin equals those of the two before it."""
    p = oracle.default_params(converge_window=3, iters=(30, 30, 30), lambda_c=0.0)
    early = 0
    for seed in range(3):
        prob = synth.pair_problem(seed)
        _, st, tr = oracle.register_problem(prob, p, trace_cap=128)
        for lvl in range(3):
            ks = [t["k_med"] for t in tr if t["level"] == lvl]
            stop = next((i for i in range(2, len(ks)) if ks[i] == ks[i - 1] == ks[i - 2]), None)
            # a median that keeps moving runs the whole cap
            assert len(ks) == (30 if stop is None else stop + 1), ks
            assert st[lvl]["iters_run"] == len(ks)
            early += stop is not None
    assert early >= 3


def test_failure_cases():
    prob = synth.pair_problem(0)
    z = np.zeros_like(prob.live_depth)
    pose, st, _ = oracle.register(z, prob.model_vtx, prob.model_nrm, prob.K, prob.imu_R, prob.init_pose)
    assert all(s["status"] == oracle.TOO_FEW_CORR and s["iters_run"] == 1 for s in st)
    assert np.array_equal(pose[:3, :3], prob.imu_R)
    # a single fronto-parallel plane leaves the in-plane translation free
    W, H = 40, 30
    K = centred_intrinsics(W, H, 35.0)
    _, d = _plane_depth(W, H, K, (0, 0, -1.0), -2.0)
    _, mv, mn, _ = render([Plane(n=np.array([0, 0, -1.0]), c=-2.0)], W, H, K, np.eye(4))
    pose, st, _ = oracle.register(d, mv, mn, K, np.eye(3), np.eye(4), oracle.default_params(levels=1))
    assert st[0]["status"] == oracle.ILL_COND


# --------------------------------------------------------------- TSDF model

def test_tsdf_plane_integration_and_raycast():
    """P17: one view of a fronto-parallel plane at 2 m: the observed voxels in
    front of it hold min(1, (2 - z)/mu) (the projective signed distance), those
    more than mu behind it stay unobserved; integrating the same view again
    keeps the values and doubles the weights; ray casting from the same camera
    finds the plane at 2 m with normal (0, 0, -1)."""
    W, H = 80, 60
    K = centred_intrinsics(W, H, 70.0)
    d = np.full((H, W), 2.0, np.float32)
    vol = oracle.Tsdf(dim=64, size=3.2, origin=(-1.6, -1.6, 0.4))
    vol.integrate(d, K, np.eye(4))
    side = vol.size / vol.dim
    t = vol.tsdf.reshape(vol.dim, vol.dim, vol.dim)  # [k][j][i]
    w = vol.weight.reshape(vol.dim, vol.dim, vol.dim)
    zc = vol.origin[2] + (np.arange(vol.dim) + 0.5) * side
    ic = jc = vol.dim // 2  # the central column projects inside the image
    for k in range(vol.dim):
        if 2.0 - zc[k] < -vol.mu:
            assert w[k, jc, ic] == 0
        else:
            assert w[k, jc, ic] == 1
            assert abs(t[k, jc, ic] - min(1.0, (2.0 - zc[k]) / vol.mu)) < 1e-6
    before = vol.tsdf.copy()
    vol.integrate(d, K, np.eye(4))
    assert np.array_equal(vol.tsdf, before) and np.max(vol.weight) == 2
    vtx, nrm = vol.raycast(W, H, K, np.eye(4), tmin=0.5, tmax=3.0)
    hit = ~np.isnan(vtx[..., 2])
    assert hit[4:-4, 4:-4].all()
    # a third view of the plane at 2.1 m: the weighted running average
    vol2 = oracle.Tsdf(dim=64, size=3.2, origin=(-1.6, -1.6, 0.4))
    vol2.tsdf[:], vol2.weight[:] = vol.tsdf, vol.weight
    vol2.integrate(np.full((H, W), 2.1, np.float32), K, np.eye(4))
    t2 = vol2.tsdf.reshape(vol.dim, vol.dim, vol.dim)
    for k in range(vol.dim):
        f_new = min(1.0, (np.float32(2.1) - zc[k]) / vol.mu)
        if f_new < -1.0:
            continue
        want = (f_new if w[k, jc, ic] == 0 else (2 * min(1.0, (2.0 - zc[k]) / vol.mu) + f_new) / 3)
        assert abs(t2[k, jc, ic] - want) < 1e-6, k  # only rays along the frustum's edge meet unobserved voxels
    assert np.max(np.abs(vtx[hit][:, 2] - 2.0)) < 1e-6
    assert np.max(np.abs(nrm[hit] - np.array([0, 0, -1.0]))) < 1e-6


def test_tsdf_sphere_raycast_lies_on_the_sphere():
    """P18: a sphere seen from one camera (pixels finer than the voxels),
    integrated and ray cast back from a slightly moved camera: where the
    surface faces the camera (within 45 deg; towards the silhouette the
    projective distance of a single view grows with the grazing angle) the
    points lie on the sphere to a small fraction of a voxel and the normals
    are radial within a few degrees."""
    K = centred_intrinsics(320, 240, 266.0)
    c, rad = np.array([0.05, -0.03, 2.0]), 0.5
    sph = synth.scene.Sphere(centre=c, radius=rad)
    d, _, _, _ = render([sph], 320, 240, K, np.eye(4), zmin=0.5, zmax=4.0)
    vol = oracle.Tsdf(dim=96, size=1.6, origin=(-0.75, -0.83, 1.2))
    vol.integrate(d.astype(np.float32), K, np.eye(4))
    W, H = 96, 72
    T = synth.pose_matrix(synth.rot_from_rotvec([0.0, 0.01, 0.0]), [0.01, 0.0, 0.0])
    vtx, nrm = vol.raycast(W, H, centred_intrinsics(W, H, 80.0), T, tmin=0.5, tmax=3.0)
    hit = ~np.isnan(vtx[..., 2])
    assert hit.sum() > 500
    pw = vtx[hit].astype(np.float64) @ T[:3, :3].T + T[:3, 3]
    r_err = np.linalg.norm(pw - c, axis=1) - rad
    side = vol.size / vol.dim
    radial = (pw - c) / np.linalg.norm(pw - c, axis=1)[:, None]
    view = pw / np.linalg.norm(pw, axis=1)[:, None]
    facing = -np.sum(radial * view, axis=1) > math.cos(math.radians(45))
    assert facing.sum() > 300
    assert np.max(np.abs(r_err[facing])) < 0.15 * side
    nw = nrm[hit].astype(np.float64) @ T[:3, :3].T
    assert np.min(np.sum(nw * radial, axis=1)[facing]) > math.cos(math.radians(5))

def test_tsdf_oblique_plane_from_off_axis_cameras():
    """P22: the ray cast's grid-coordinate march (camera centre
    gc = (t - origin)/side - 1/2, direction gd = R d / side, voxel centres on
    integers) against a closed form.  A plane whose normal has three nonzero
    components of one sign is fused from three rotated, translated views and
    ray cast from a fourth: every hit lies on the plane within a tenth of a
    voxel and every normal is the plane's within 2 deg.  Dropping the half-
    voxel offset of gc would move the surface by 0.8 voxel along the normal;
    marching the camera-frame direction instead of the world one, or mixing up
    the voxel index order, would put the hits off the plane altogether."""
    nw = np.array([-0.4, -0.5, -1.0])
    nw /= np.linalg.norm(nw)
    c = float(nw @ np.array([0.02, -0.03, 2.0]))
    plane = Plane(n=nw, c=c)
    K = centred_intrinsics(640, 480, 560.0)
    vol = oracle.Tsdf(dim=64, size=1.6, origin=(-0.8, -0.8, 1.2))
    side = vol.size / vol.dim
    views = [([0.06, -0.08, 0.03], [0.05, 0.04, -0.1]), ([-0.07, 0.05, -0.04], [-0.06, 0.03, 0.05]),
             ([0.03, 0.09, 0.06], [0.02, -0.07, 0.0])]
    for w, t in views:
        T = synth.pose_matrix(synth.rot_from_rotvec(w), t)
        d, _, _, _ = render([plane], 640, 480, K, T, zmin=0.3, zmax=5.0)
        vol.integrate(d.astype(np.float32), K, T)
    T = synth.pose_matrix(synth.rot_from_rotvec([-0.05, 0.07, -0.08]), [0.04, 0.05, 0.02])
    W, H = 96, 72
    vtx, nrm = vol.raycast(W, H, centred_intrinsics(W, H, 84.0), T, tmin=0.5, tmax=4.0)
    hit = ~np.isnan(vtx[..., 2])
    assert hit.sum() > 0.5 * W * H
    pw = vtx[hit].astype(np.float64) @ T[:3, :3].T + T[:3, 3]
    assert np.max(np.abs(pw @ nw - c)) < 0.1 * side
    n_world = nrm[hit].astype(np.float64) @ T[:3, :3].T
    assert np.min(n_world @ nw) > math.cos(math.radians(2.0))


def test_band_keeps_about_three_quarters_of_the_pairs():
    """P19: the band rule against the paper's one quantitative statement about
    the filter (Sec. 3.3, the caption of its median-filtering figure: about 75%
    of the pairs kept in the example shown).  On room registrations the finest
    level keeps between 60% and 90% of the gated pairs; a band a few bins wide
    around the median, no band at all, or one that never reaches above the
    median would fall outside."""
    seq = synth.RoomSequence(0, n_frames=6)
    fracs = []
    for k in (0, 2, 4):
        _, st, _ = oracle.register_problem(seq.problem(k))
        fracs.append(st[0]["n_kept"] / st[0]["n_gated"])
    assert all(0.6 < f < 0.9 for f in fracs), fracs


def test_division_by_a_correctly_rounded_reciprocal(tmp_path):
    """The bilateral filter's range quotient dz / c is formed on the GPU as
    q = RN(dz y), t = RN(q + RN(dz - c q) y) with y = RN(1/c) (Markstein's
    correction); it must equal the IEEE quotient for the filter's inputs.  A
    plain C check over a million FP32 depth differences within the cut-off,
    for several cut-offs (including ones whose reciprocal is inexact)."""
    import subprocess
    src = tmp_path / "m.c"
    src.write_text(r'''
#include <math.h>
#include <stdint.h>
#include <stdio.h>
static uint64_t s = 88172645463325252ull;
static uint64_t xr(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double u01(void) { return (xr() >> 11) * 0x1.0p-53; }
int main(void) {
    const double cs[] = {0.05, 0.03, 0.1, 0.0123456789, 1.0 / 3.0};
    long bad = 0, n = 0;
    for (int ci = 0; ci < 5; ++ci) {
        const double c = cs[ci], y = 1.0 / c;
        for (long k = 0; k < 200000; ++k) {
            const float z = (float)(0.3 + 9.7 * u01());
            float zq = (k & 1) ? nextafterf(z, (k & 2) ? 100.0f : 0.0f) : (float)(z + (2.0 * u01() - 1.0) * c);
            const double dz = (double)zq - (double)z;
            if (!(fabs(dz) < c)) continue;
            const double q = dz * y;
            ++n;
            bad += fma(fma(-q, c, dz), y, q) != dz / c;
        }
    }
    printf("%ld %ld\n", n, bad);
    return 0;
}
''')
    exe = tmp_path / "m"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", str(exe), str(src), "-lm"], check=True)
    n, bad = (int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split())
    assert n > 500000 and bad == 0


def test_back_projection_quotients_without_division(tmp_path):
    """The pixel passes form the back-projection quotient (t - c)/f of the
    front end's tables (t a pixel column or row, c the level's principal
    point, f its focal length) as RN(q + RN(a - f q) y), q = RN(a y),
    y = RN(1/f), a = RN(t - c).  A plain C check that this equals the IEEE
    quotient for every column and row of the benchmark geometries' levels and
    for random focal lengths and principal points."""
    import subprocess
    src = tmp_path / "b.c"
    src.write_text(r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
static uint64_t s = 0xD1B54A32D192ED03ull;
static uint64_t xr(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double u01(void) { return (xr() >> 11) * 0x1.0p-53; }
static long n = 0, bad = 0;
static void run(double f, double c, int T) {
    const double y = 1.0 / f;
    for (int t = 0; t <= T; ++t) {
        const double a = (double)t - c, q = a * y;
        ++n; bad += fma(fma(-q, f, a), y, q) != a / f;
    }
}
int main(void) {
    const double fs[] = {525.0, 130.0, 570.3, 1000.0, 481.2};
    const int Ws[] = {160, 320, 640, 848, 1280, 120, 240, 480, 720};
    for (int fi = 0; fi < 5; ++fi)
        for (int l = 0; l < 5; ++l)
            for (int wi = 0; wi < 9; ++wi) {
                const double p = (double)(1 << l);
                run(fs[fi] / p, ((Ws[wi] - 1) * 0.5 + 0.5) / p - 0.5, (Ws[wi] >> l) + 1);
            }
    for (long k = 0; k < 40000; ++k) {
        const double p = (double)(1 << (int)(xr() % 5));
        const double c0 = 2000.0 * u01();
        run((20.0 + 3000.0 * u01()) / p, (k & 1) ? c0 : (c0 + 0.5) / p - 0.5, (int)(1300 / p));
    }
    printf("%ld %ld\n", n, bad);
    return 0;
}
""")
    exe = tmp_path / "b"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", str(exe), str(src), "-lm"], check=True)
    n, bad = (int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split())
    assert n > 10000000 and bad == 0


def test_normalisation_by_one_division(tmp_path):
    """The live normals and the model pyramid's normals divide each component
    c_k of a vector by its length len = sqrt((c0 c0 + c1 c1) + c2 c2) as
    RN(q + RN(c_k - len q) y), q = RN(c_k y), with the one division
    y = RN(1/len).  A plain C check that this equals the IEEE quotient for
    vectors over 80 binades, with components down to 1e-6 of the others and
    exact zeros."""
    import subprocess
    src = tmp_path / "n.c"
    src.write_text(r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
static uint64_t s = 0x853c49e6748fea9bull;
static uint64_t xr(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double u01(void) { return (xr() >> 11) * 0x1.0p-53; }
int main(void) {
    long n = 0, bad = 0;
    for (long t = 0; t < 4000000; ++t) {
        const double sc = ldexp(1.0, (int)(xr() % 80) - 60);
        double c[3];
        for (int k = 0; k < 3; ++k) c[k] = (2.0 * u01() - 1.0) * sc * ((xr() & 7) == 0 ? 1e-6 : 1.0);
        if (t & 1) c[xr() % 3] = 0.0;
        const double len2 = (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2];
        if (!(len2 > 0.0) || !isfinite(len2)) continue;
        const double len = sqrt(len2), y = 1.0 / len;
        for (int k = 0; k < 3; ++k) {
            const double q = c[k] * y;
            ++n; bad += fma(fma(-q, len, c[k]), y, q) != c[k] / len;
        }
    }
    printf("%ld %ld\n", n, bad);
    return 0;
}
""")
    exe = tmp_path / "n"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", str(exe), str(src), "-lm"], check=True)
    n, bad = (int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split())
    assert n > 10000000 and bad == 0


def test_reciprocal_division_over_the_tsdf_ranges(tmp_path):
    """The TSDF integration forms its quotients the same way: x/z and y/z
    share y = RN(1/z) (z from 2^-900 to 20 m, numerators up to 20 m in
    magnitude down to 1e-12), sdf/mu uses RN(1/mu), and the running average
    divides by an integer count k = 1..256 through a table of RN(1/k).  A
    plain C check that every such quotient equals the IEEE one."""
    import subprocess
    src = tmp_path / "t.c"
    src.write_text(r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint64_t xr(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double u01(void) { return (xr() >> 11) * 0x1.0p-53; }
static double mq(double a, double b, double y) { const double q = a * y; return fma(fma(-q, b, a), y, q); }
int main(void) {
    long bad = 0, n = 0;
    for (long t = 0; t < 2000000; ++t) {          /* projection: shared divisor */
        const double b = (t & 1) ? 0.01 + 20.0 * u01() : ldexp(1.0 + u01(), -(int)(900.0 * u01()));
        const double a = (2.0 * u01() - 1.0) * ((t & 2) ? 20.0 : ldexp(1.0, -(int)(40.0 * u01())));
        const double y = 1.0 / b;
        ++n; bad += mq(a, b, y) != a / b;
    }
    const double mus[] = {0.05, 0.0125 * 4, 0.03, 0.1, 1.0 / 3.0, 0.0173};
    for (int m = 0; m < 6; ++m) {                  /* sdf / mu */
        const double mu = mus[m], y = 1.0 / mu;
        for (long t = 0; t < 300000; ++t) {
            const double z = (double)(float)(0.3 + 9.7 * u01()), xc = 0.3 + 9.7 * u01();
            const double sdf = z - xc;
            if (sdf < -mu) continue;
            ++n; bad += mq(sdf, mu, y) != sdf / mu;
        }
    }
    for (int k = 1; k <= 256; ++k) {               /* running average by the count */
        const double y = 1.0 / (double)k;
        for (long t = 0; t < 20000; ++t) {
            const double w = (double)(k - 1);
            const double a = (double)(float)(2.0 * u01() - 1.0) * w + (2.0 * u01() - 1.0);
            ++n; bad += mq(a, (double)k, y) != a / (double)k;
        }
    }
    printf("%ld %ld\n", n, bad);
    return 0;
}
""")
    exe = tmp_path / "t"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", str(exe), str(src), "-lm"], check=True)
    n, bad = (int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split())
    assert n > 7000000 and bad == 0
