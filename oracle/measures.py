"""CPU oracle of the measurement-confidence model and of the evaluation metric
(test infrastructure only).

Like ``oracle.core`` this is the plain reference the GPU library is checked against; only
the test suite, the smoke check and the benchmark's CPU-baseline leg may import it, and it
shares no code with the HIP library.

  Sec. II.2, Eq. 2-3   per-pixel measurement confidence   -> ``confidence_eq3``
  Sec. III, Eq. 12     multi-camera depth consistency     -> ``emc``

Readings of what the paper leaves open:
  * Eq. 3's depth gradient G is the magnitude of the central-difference gradient in metres
    per pixel, sqrt(gx^2 + gy^2) with gx = (D(x+1) - D(x-1)) / 2; where only one horizontal
    (vertical) neighbour has a valid depth the one-sided difference with it is used, where
    neither has, that component is 0.
  * sigma_local is the population standard deviation of the valid depths in the 3x3
    window centred on the pixel (the pixel included); the paper's symbol is a standard
    deviation although its text says "variance".
  * Eq. 3 with alpha = beta = 0.5, gamma = delta = 1 spans (0, 1.5], against Eq. 2's
    [0, 1]: the result is divided by alpha + gamma.  Pixels without a valid depth (not
    finite or <= 0) get C = 0.
  * Eq. 12's visible set gamma(P): cameras where the point is in front (z > 0), its nearest
    pixel is inside the image, the depth there is valid, and the point is not occluded:
    z <= D + c_occ z^2 (c_occ = 3 x 0.001 /m, three times the depth-noise coefficient of the
    synthetic sensor).  Points with an empty visible set are left out of rho; rho is every
    `stride`-th fused point.
  * Decisions (visibility, pixel) use the same float32 arithmetic as the fusion oracle; the
    error sums are float64.
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np

from oracle.core import F32, camera_f32, project

# Eq. 3 weights of the paper (Sec. II.2)
ALPHA, BETA, GAMMA, DELTA = 0.5, 0.5, 1.0, 1.0
C_OCC = 0.003   # occlusion tolerance coefficient of the visible set (1/m)


def _valid(d):
    return np.isfinite(d) & (d > 0)


def confidence_eq3(depth: np.ndarray, alpha: float = ALPHA, beta: float = BETA,
                   gamma: float = GAMMA, delta: float = DELTA) -> np.ndarray:
    """Eq. 3 per pixel of one depth map (H x W float32), normalised into (0, 1]; 0 where the
    depth is invalid.  float32, one rounding per operation in the order written."""
    with np.errstate(over="ignore", invalid="ignore"):
        return _confidence_eq3(np.asarray(depth, F32), alpha, beta, gamma, delta)


def _confidence_eq3(D, alpha, beta, gamma, delta):
    # huge depths may overflow to inf in the squares: inf is what IEEE float32 gives
    H, W = D.shape
    ok = _valid(D)
    Dz = np.where(ok, D, F32(0))
    a, b, g, dl = F32(alpha), F32(beta), F32(gamma), F32(delta)

    def shifted(arr, dy, dx, fill):
        out = np.full_like(arr, fill)
        ys = slice(max(0, -dy), H - max(0, dy))
        xs = slice(max(0, -dx), W - max(0, dx))
        yd = slice(max(0, dy), H - max(0, -dy) if max(0, -dy) else H)
        xd = slice(max(0, dx), W - max(0, -dx) if max(0, -dx) else W)
        out[ys, xs] = arr[yd, xd]
        return out

    def grad(dy, dx):
        # neighbour values at +1 and -1 along the axis
        vp, op = shifted(Dz, dy, dx, F32(0)), shifted(ok, dy, dx, False)
        vm, om = shifted(Dz, -dy, -dx, F32(0)), shifted(ok, -dy, -dx, False)
        both = (vp - vm) * F32(0.5)
        right = vp - Dz
        left = Dz - vm
        return np.where(op & om, both, np.where(op, right, np.where(om, left, F32(0)))).astype(F32)

    gx = grad(0, 1)
    gy = grad(1, 0)
    G = np.sqrt((gx * gx + gy * gy).astype(F32)).astype(F32)

    # 3x3 window, row-major order, valid pixels only
    offs = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    n = np.zeros((H, W), F32)
    s = np.zeros((H, W), F32)
    vals = []
    for dy, dx in offs:
        v, o = shifted(Dz, dy, dx, F32(0)), shifted(ok, dy, dx, False)
        vals.append((v, o))
        n = np.where(o, n + F32(1), n).astype(F32)
        s = np.where(o, s + v, s).astype(F32)
    nn = np.where(n > 0, n, F32(1))
    mean = (s / nn).astype(F32)
    acc = np.zeros((H, W), F32)
    for v, o in vals:
        e = (v - mean).astype(F32)
        acc = np.where(o, acc + e * e, acc).astype(F32)
    sd = np.sqrt((acc / nn).astype(F32)).astype(F32)

    t1 = (a / (F32(1) + b * G)).astype(F32)
    t2 = (g / (F32(1) + dl * sd)).astype(F32)
    C = ((t1 + t2) / (a + g)).astype(F32)
    return np.where(ok, C, F32(0)).astype(F32)


def confidence_eq3_bruteforce(depth: np.ndarray, alpha: float = ALPHA, beta: float = BETA,
                              gamma: float = GAMMA, delta: float = DELTA) -> np.ndarray:
    """The same definition written as plain loops over pixels with float32 scalars (slow;
    tiny images only): an independent check of the vectorised form."""
    D = np.asarray(depth, F32)
    H, W = D.shape
    a, b, g, dl = F32(alpha), F32(beta), F32(gamma), F32(delta)
    out = np.zeros((H, W), F32)

    def okat(y, x):
        return 0 <= y < H and 0 <= x < W and np.isfinite(D[y, x]) and D[y, x] > 0

    for y in range(H):
        for x in range(W):
            if not okat(y, x):
                continue
            d = D[y, x]
            comps = []
            for dy, dx in ((0, 1), (1, 0)):
                p, m = okat(y + dy, x + dx), okat(y - dy, x - dx)
                if p and m:
                    comps.append(F32(D[y + dy, x + dx] - D[y - dy, x - dx]) * F32(0.5))
                elif p:
                    comps.append(F32(D[y + dy, x + dx] - d))
                elif m:
                    comps.append(F32(d - D[y - dy, x - dx]))
                else:
                    comps.append(F32(0))
            G = np.sqrt(F32(F32(comps[0] * comps[0]) + F32(comps[1] * comps[1])))
            win = [D[y + dy, x + dx] for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                   if okat(y + dy, x + dx)]
            s = F32(0)
            for v in win:
                s = F32(s + v)
            mean = F32(s / F32(len(win)))
            acc = F32(0)
            for v in win:
                e = F32(v - mean)
                acc = F32(acc + F32(e * e))
            sd = np.sqrt(F32(acc / F32(len(win))))
            t1 = F32(a / F32(F32(1) + F32(b * G)))
            t2 = F32(g / F32(F32(1) + F32(dl * sd)))
            out[y, x] = F32(F32(t1 + t2) / F32(a + g))
    return out


def emc(cams_in, depth: Sequence[np.ndarray], xyz: np.ndarray, c_occ: float = C_OCC,
        stride: int = 1) -> Dict:
    """Eq. 12 over every `stride`-th point of a fused cloud (S x 3 float32): the mean over
    points of the mean |z(T_i P) - D_i(pi(T_i P))| over the cameras that see the point.
    Returns E_MC in metres, the number of points used and their mean visible-camera count."""
    cams = [camera_f32(c) for c in cams_in]
    P = np.asarray(xyz, F32).reshape(-1, 3)[::max(1, int(stride))]
    n = len(P)
    err = np.zeros(n, np.float64)
    cnt = np.zeros(n, np.int64)
    k = F32(c_occ)
    for cam, D in zip(cams, depth):
        D = np.asarray(D, F32)
        ok, px, py, Z = _project_z(cam, P)
        d = np.where(ok, D[np.where(ok, py, 0), np.where(ok, px, 0)], F32(0))
        vis = ok & np.isfinite(d) & (d > 0)
        tol = ((k * Z).astype(F32) * Z).astype(F32)
        vis &= Z <= (d + tol).astype(F32)
        err += np.where(vis, np.abs(Z.astype(np.float64) - d.astype(np.float64)), 0.0)
        cnt += vis
    used = cnt > 0
    per_point = err[used] / cnt[used]
    total = 0.0
    for v in per_point:        # sequential, in point order
        total += v
    m = int(used.sum())
    return dict(emc_m=total / m if m else 0.0, points=m,
                mean_visible=float(cnt[used].mean()) if m else 0.0)


def _project_z(cam, P):
    """Nearest pixel of world points in one camera (the fusion oracle's projection, Eq. 4)
    and their camera-frame depth z, in float32."""
    cols = [P[:, 0].astype(F32), P[:, 1].astype(F32), P[:, 2].astype(F32)]
    ok, px, py = project(cam, cols)
    R, t = cam.R, cam.t
    Z = (((R[2, 0] * cols[0] + R[2, 1] * cols[1]) + R[2, 2] * cols[2]) + t[2]).astype(F32)
    return ok, px, py, Z
