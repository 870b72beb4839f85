"""Pins of the measurement-confidence oracle (Sec. II.2, Eq. 3) and of the E_MC evaluator
oracle (Sec. III, Eq. 12): closed forms, special cases and brute force on tiny inputs."""
import math

import numpy as np
import pytest

from oracle import core as O
from oracle import measures as M
from synth.scenes import make_camera

F32 = np.float32


# ------------------------------------------------------------------ Eq. 3

def test_flat_depth_has_full_confidence():
    # G = 0 and sigma_local = 0: (alpha + gamma) / (alpha + gamma) = 1 exactly
    C = M.confidence_eq3(np.full((7, 9), 2.5, F32))
    assert np.all(C == F32(1))


def _eq3(G, sd, a=0.5, b=0.5, g=1.0, d=1.0):
    return (a / (1 + b * G) + g / (1 + d * sd)) / (a + g)


def test_linear_ramp_closed_form():
    # D = 2 + s x: interior G = s, window values D(x) + {-s, 0, s} in 3 rows -> population
    # std s sqrt(2/3); at the left and right borders one-sided G = s and the window holds
    # two columns -> std s / 2
    s = 0.25
    H, W = 6, 11
    D = (2 + s * np.arange(W, dtype=np.float64))[None, :].repeat(H, 0).astype(F32)
    C = M.confidence_eq3(D)
    interior = _eq3(s, s * math.sqrt(2 / 3))
    border = _eq3(s, s / 2)
    assert np.allclose(C[:, 1:-1], interior, rtol=2e-7, atol=0)
    assert np.allclose(C[:, [0, -1]], border, rtol=2e-7, atol=0)
    # un-normalised Eq. 3 spans (0, alpha + gamma]: the normalisation divides by 1.5
    assert abs(float(C[2, 5]) * 1.5 - (0.5 / (1 + 0.5 * s) + 1 / (1 + s * math.sqrt(2 / 3)))) < 1e-6


def test_invalid_and_isolated_pixels():
    D = np.zeros((5, 5), F32)
    D[2, 2] = 3.0                       # one valid pixel: G = 0, sigma = 0
    D[0, 0] = np.nan
    D[4, 4] = -1.0
    C = M.confidence_eq3(D)
    assert C[2, 2] == F32(1)
    assert np.count_nonzero(C) == 1


def test_weights_enter_as_written():
    # planted gradient only (rows constant in y, step in x at the centre) with beta = 0:
    # the gradient term is alpha for any G, so C depends on sigma alone
    D = np.array([[1, 1, 2, 2]] * 3, F32)
    C0 = M.confidence_eq3(D, beta=0.0)
    C1 = M.confidence_eq3(D, beta=0.0, delta=0.0)
    assert np.all(C1 == F32(1))         # both terms constant: (alpha + gamma) / (alpha + gamma)
    assert np.all(C0 <= F32(1)) and np.all(C0[:, 1:3] < F32(1))


@pytest.mark.parametrize("seed", range(3))
def test_bruteforce_agrees(seed):
    rng = np.random.default_rng(seed)
    D = (1 + 3 * rng.random((9, 12))).astype(F32)
    D[rng.random(D.shape) < 0.15] = 0
    D[rng.random(D.shape) < 0.05] = np.inf
    assert np.array_equal(M.confidence_eq3(D), M.confidence_eq3_bruteforce(D))


def test_range_and_noise_monotonicity():
    rng = np.random.default_rng(5)
    base = np.full((64, 64), 3.0)
    quiet = (base + 0.001 * rng.standard_normal(base.shape)).astype(F32)
    noisy = (base + 0.05 * rng.standard_normal(base.shape)).astype(F32)
    cq, cn = M.confidence_eq3(quiet), M.confidence_eq3(noisy)
    for c in (cq, cn):
        assert np.all(c > 0) and np.all(c <= 1)
    assert cn.mean() < cq.mean()


# ------------------------------------------------------------------ Eq. 12

def _plane_rig(Z0=3.0, W=40, H=30):
    cam = make_camera(W, H, np.array([0.0, -Z0, 0.0]), np.zeros(3))
    depth = np.full((H, W), Z0, F32)
    return cam, depth


def _points_at(cam, depth_val, W, H):
    """World points on camera rays at z-depth `depth_val` (back-projection, Eq. 8)."""
    cf = O.camera_f32(cam)
    yy, xx = np.mgrid[0:H, 0:W]
    p = O.backproject(cf, xx.ravel(), yy.ravel(), np.full(W * H, depth_val, F32))
    return np.stack(p, 1).astype(F32)


def test_emc_zero_for_the_observed_surface():
    cam, D = _plane_rig()
    P = _points_at(cam, 3.0, 40, 30)
    r = M.emc([cam], [D], P)
    assert r["points"] == 40 * 30 and r["mean_visible"] == 1.0
    assert r["emc_m"] < 1e-6


@pytest.mark.parametrize("delta", [0.01, 0.05])
def test_emc_planted_offset_in_front(delta):
    # points delta in front of the observed plane: visible, error delta per point
    cam, D = _plane_rig()
    P = _points_at(cam, 3.0 - delta, 40, 30)
    r = M.emc([cam], [D], P)
    assert r["points"] == 40 * 30
    assert abs(r["emc_m"] - delta) < 1e-5


def test_emc_occluded_points_are_not_visible():
    # points 0.2 m behind the surface (beyond 3 * 0.001 z^2 = 0.03 m): no camera sees them
    cam, D = _plane_rig()
    P = _points_at(cam, 3.2, 40, 30)
    r = M.emc([cam], [D], P)
    assert r["points"] == 0 and r["emc_m"] == 0.0
    # within the tolerance they count
    P = _points_at(cam, 3.02, 40, 30)
    r = M.emc([cam], [D], P)
    assert r["points"] == 40 * 30 and abs(r["emc_m"] - 0.02) < 1e-5


def test_emc_two_cameras_average_per_point():
    # the same plane seen by a second camera 1 m further back: per point the mean of the
    # two absolute depth errors
    cam0, D0 = _plane_rig(3.0)
    cam1 = make_camera(40, 30, np.array([0.0, -4.0, 0.0]), np.zeros(3))
    D1 = np.full((30, 40), 4.0, F32)
    P = _points_at(cam0, 2.9, 40, 30)     # 0.1 m in front of the plane for both cameras
    r = M.emc([cam0, cam1], [D0, D1], P)
    assert r["points"] == 40 * 30
    assert abs(r["emc_m"] - 0.1) < 1e-5
    assert 1.0 < r["mean_visible"] <= 2.0


def _emc_bruteforce(cams, depth, P, c_occ=M.C_OCC):
    tot, n = 0.0, 0
    cfs = [O.camera_f32(c) for c in cams]
    for p in np.asarray(P, F32):
        s, k = 0.0, 0
        for cf, D in zip(cfs, depth):
            X = [F32(F32(F32(cf.R[a, 0] * p[0]) + F32(cf.R[a, 1] * p[1])) + F32(cf.R[a, 2] * p[2]))
                 for a in range(3)]
            X = [F32(X[a] + cf.t[a]) for a in range(3)]
            if not X[2] > 0:
                continue
            u = F32(F32(cf.fx * F32(X[0] / X[2])) + cf.cx)
            v = F32(F32(cf.fy * F32(X[1] / X[2])) + cf.cy)
            fu, fv = np.floor(F32(u + F32(0.5))), np.floor(F32(v + F32(0.5)))
            if not (0 <= fu < cf.width and 0 <= fv < cf.height):
                continue
            d = D[int(fv), int(fu)]
            if not (np.isfinite(d) and d > 0):
                continue
            if not X[2] <= F32(d + F32(F32(F32(c_occ) * X[2]) * X[2])):
                continue
            s += abs(float(X[2]) - float(d))
            k += 1
        if k:
            tot += s / k
            n += 1
    return tot / n if n else 0.0, n


def test_emc_bruteforce_agrees():
    rng = np.random.default_rng(11)
    from synth import make_config
    f = make_config("c1")
    fused = O.fuse_frame(f)
    idx = rng.choice(len(fused["xyz"]), 300, replace=False)
    P = fused["xyz"][np.sort(idx)]
    r = M.emc(f.cams, f.depth, P)
    e, n = _emc_bruteforce(f.cams, f.depth, P)
    assert r["points"] == n and abs(r["emc_m"] - e) <= 1e-12 * max(1.0, e)
    r2 = M.emc(f.cams, f.depth, P, stride=3)
    e2, n2 = _emc_bruteforce(f.cams, f.depth, P[::3])
    assert r2["points"] == n2 and abs(r2["emc_m"] - e2) <= 1e-12 * max(1.0, e2)
