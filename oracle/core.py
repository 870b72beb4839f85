"""CPU oracle of the FUSE-Flow per-frame fusion path (test infrastructure only).

This module is the plain, slow reference that the GPU library is checked against.  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does.  It shares no code with the HIP library.

It follows the method of the paper (Sec. II) step by step:

  Eq. 9   confidence gate                 -> ``gate``
  Eq. 8   pixel-wise back-projection      -> ``backproject``
  II.5(1) adaptive spatial partition      -> ``extents``, ``coarse_exponent``,
          (a..e)                             ``coarse_cells``, ``levels``, ``cell_keys``
  II.5(2)a  top-3 representatives by C    -> ``representatives``
  II.5(2)b  local camera constraint       -> ``select_views`` (uses Eq. 4)
  Eq. 5-7 distance consistency            -> ``consistency``
  Eq. 10-11 joint weight, fusion          -> ``fuse_cells``

Arithmetic convention.  Every quantity that feeds a discrete decision (point coordinates,
which decide cell keys; projections, which decide pixels; camera ranking) is computed in
IEEE float32 with one rounding per +, -, *, / in exactly the order written here, with no
fused multiply-add (NumPy float32 ufuncs applied one at a time).  Continuous quantities
(squared distances, consistency, fusion) are computed in float64.

Readings of points the paper leaves open (each repeated at the function that implements
it):
  * T_i is world->camera [R | t]; Eq. 8 applies its inverse (R^T, c = -R^T t).
  * pi^-1(K, [x, y, 1], d) = d * K^-1 [x, y, 1]: depth is z-depth, pixel centres are at
    integer coordinates.
  * Eq. 9's "0 otherwise" means the point is dropped, not placed at the origin; a point
    also needs a finite positive depth and finite coordinates.
  * Coarse grid: ``coarse_res`` cells along the longest AABB axis, cell edge rounded up to a
    power of two (so that all later scalings are exact).
  * Refinement rule: level L(c) = smallest L in [0, max_level] with
    n(c) <= target_per_cell * 4^L (surfaces are 2-D: halving the edge quarters the count).
  * Representative order: C descending, then x, y, z ascending, then pixel id.
  * Local views: cameras whose image contains the projection (in front, nearest pixel in
    bounds), ranked by squared distance from the point to the camera centre (ties: centre
    x, y, z, then camera index); the first K - 1 are used; a view whose depth at that
    pixel is missing (not finite or <= 0) contributes nothing.
  * Eq. 7's 1/(K - 1) is taken as 1/m with m the number of views that contributed
    (equal to 1/(K-1) whenever K - 1 views contribute); m = 0 gives V = 1.
  * Eq. 11 is normalised (the text calls it weighted averaging): xyz = sum(w p) / sum(w),
    evaluated as a softmax of log-weights; output weight = mean of w over the
    representatives; colour fused with the same normalised weights.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

F32 = np.float32
PAD = np.uint32(0xFFFFFFFF)

FF_NO_MF = 1   # ablation: no measurement confidence (C := 1, gate on depth only)
FF_NO_DC = 2   # ablation: no distance consistency (V := 1)
FF_NO_SA = 4   # ablation: no spatial-hash aggregation (every point is its own cell)
FF_CONF_EQ3 = 8  # confidence from the depth maps by Eq. 3 (``oracle.measures``), not given

E_MIN, E_MAX = -24, 100   # clamp of the coarse-cell exponent (degenerate extents only)


@dataclasses.dataclass
class Params:
    tau: float = 0.6            # Eq. 9 threshold (Sec. II.4 sets 0.6)
    k_views: int = 4            # K of Eq. 7 / II.5(2)b, own camera included
    sigma: float = 0.02         # Eq. 7 tolerance, metres
    coarse_res: int = 64        # coarse cells along the longest AABB axis (power of two)
    max_level: int = 6          # deepest refinement level
    target_per_cell: int = 16   # refinement target occupancy
    level_override: int = -1    # >= 0: force this level in every coarse cell
    flags: int = 0              # FF_NO_MF | FF_NO_DC | FF_NO_SA | FF_CONF_EQ3


@dataclasses.dataclass
class CameraF32:
    """Camera parameters cast to float32, with the inverse transform (Eq. 8's T^-1)."""
    width: int
    height: int
    fx: np.float32
    fy: np.float32
    cx: np.float32
    cy: np.float32
    R: np.ndarray      # (3, 3) float32, world -> camera rotation
    t: np.ndarray      # (3,) float32
    centre: np.ndarray  # (3,) float32, c = -R^T t (canonical order)


def camera_f32(cam) -> CameraF32:
    """Cast a camera to float32 and invert its extrinsics.

    The world->camera transform is [R | t]; its inverse maps camera points to the world as
    p = R^T X + c with c = -R^T t (Sec. II.4, Eq. 8).  c is evaluated as
    -((R00 t0 + R10 t1) + R20 t2) (and likewise per axis) in float32.
    """
    T = np.asarray(cam.world_to_cam, dtype=F32)
    R = T[:, :3].copy()
    t = T[:, 3].copy()
    c = np.empty(3, F32)
    for a in range(3):
        c[a] = -((R[0, a] * t[0] + R[1, a] * t[1]) + R[2, a] * t[2])
    return CameraF32(int(cam.width), int(cam.height), F32(cam.fx), F32(cam.fy),
                     F32(cam.cx), F32(cam.cy), R, t, c)


# ------------------------------------------------------------------ Sec. II.4, Eq. 8 and 9

def backproject(cam: CameraF32, x, y, d):
    """Eq. 8: P = T^-1 pi^-1(K, [x, y, 1], d), all float32, canonical order.

    pi^-1 gives the camera-frame point (d (x - cx)/fx, d (y - cy)/fy, d); the inverse
    extrinsics give p_a = ((R0a X + R1a Y) + R2a Z) + c_a.
    """
    x = np.asarray(x, F32)
    y = np.asarray(y, F32)
    d = np.asarray(d, F32)
    xn = (x - cam.cx) / cam.fx
    yn = (y - cam.cy) / cam.fy
    X = xn * d
    Y = yn * d
    Z = d
    R, c = cam.R, cam.centre
    return [((R[0, a] * X + R[1, a] * Y) + R[2, a] * Z) + c[a] for a in range(3)]


def gate(depth: np.ndarray, conf: np.ndarray, params: Params) -> np.ndarray:
    """Eq. 9: keep a pixel when its confidence exceeds tau (strictly) and its depth is a
    finite positive number.  With FF_NO_MF the confidence test is skipped."""
    ok = np.isfinite(depth) & (depth > 0)
    if not params.flags & FF_NO_MF:
        ok &= conf > F32(params.tau)
    return ok


def generate_points(cams: Sequence[CameraF32], depth, conf, params: Params) -> Dict:
    """Sec. II.4: back-project every pixel of every camera, gate it (Eq. 9), and keep the
    survivors in pixel-id order (camera-major, then row-major)."""
    ids, cam_idx, xs, ys, zs, cs = [], [], [], [], [], []
    offset = 0
    for k, cam in enumerate(cams):
        D = np.asarray(depth[k], F32)
        C = np.asarray(conf[k], F32)
        assert D.shape == (cam.height, cam.width) and C.shape == D.shape
        ok = gate(D, C, params)
        yy, xx = np.nonzero(ok)
        d = D[yy, xx]
        p = backproject(cam, xx.astype(F32), yy.astype(F32), d)
        fin = np.isfinite(p[0]) & np.isfinite(p[1]) & np.isfinite(p[2])
        c = np.ones(len(d), F32) if params.flags & FF_NO_MF else C[yy, xx]
        ids.append((offset + yy.astype(np.int64) * cam.width + xx)[fin])
        cam_idx.append(np.full(int(fin.sum()), k, np.int64))
        xs.append(p[0][fin]); ys.append(p[1][fin]); zs.append(p[2][fin]); cs.append(c[fin])
        offset += cam.width * cam.height
    cat = lambda v, dt: np.concatenate(v).astype(dt) if v else np.zeros(0, dt)
    return dict(pix=cat(ids, np.int64), cam=cat(cam_idx, np.int64),
                xyz=np.stack([cat(xs, F32), cat(ys, F32), cat(zs, F32)], axis=1),
                conf=cat(cs, F32))


# ------------------------------------------------------------ Sec. II.5(1) partition

def extents(xyz: np.ndarray):
    """II.5(1)b: componentwise min and max over all points."""
    return xyz.min(axis=0), xyz.max(axis=0)


def coarse_exponent(bmin: np.ndarray, bmax: np.ndarray, coarse_res: int) -> int:
    """II.5(1)c: the coarse cell edge is s0 = 2^e, the smallest power of two with
    coarse_res * s0 >= the longest extent (float32 extent, exact frexp arithmetic)."""
    with np.errstate(over="ignore"):
        ext = float(np.max(bmax - bmin))      # float32 subtraction, then exact widening
    if ext == 0.0:
        return E_MIN
    if not math.isfinite(ext):
        return E_MAX
    m, x = math.frexp(ext)                    # ext = m 2^x, 0.5 <= m < 1
    ceil_log2 = x - 1 if m == 0.5 else x
    e = ceil_log2 - int(round(math.log2(coarse_res)))
    return max(E_MIN, min(E_MAX, e))


def coarse_cells(xyz: np.ndarray, bmin: np.ndarray, e: int, coarse_res: int):
    """II.5(1)c: scaled offsets q = (p - bmin) 2^-e (float32; the scaling is exact) and the
    coarse cell index floor(q), clamped to coarse_res - 1, per axis."""
    scale = F32(2.0 ** (-e))
    q = (xyz - bmin[None, :].astype(F32)) * scale
    ci = np.minimum(np.floor(q), F32(coarse_res - 1)).astype(np.int64)
    return q, ci


def coarse_linear(ci: np.ndarray, coarse_res: int) -> np.ndarray:
    return (ci[:, 2] * coarse_res + ci[:, 1]) * coarse_res + ci[:, 0]


def levels(counts: np.ndarray, params: Params) -> np.ndarray:
    """II.5(1)d: refinement level per coarse cell: the smallest L in [0, max_level] with
    count <= target_per_cell * 4^L (max_level if none); level_override forces one level."""
    if params.level_override >= 0:
        return np.full(counts.shape, params.level_override, np.int64)
    L = np.full(counts.shape, params.max_level, np.int64)
    for lev in range(params.max_level, -1, -1):
        L[counts <= params.target_per_cell * 4 ** lev] = lev
    return L


def cell_keys(q: np.ndarray, ci: np.ndarray, L: np.ndarray, params: Params):
    """II.5(1)e: assign each point to its cell at its coarse cell's level.

    Fine coordinates f = floor(q 2^L) (exact scaling), clamped into the coarse cell, local
    offsets l = f - ci 2^L in [0, 2^L).  The key is
    (coarse_linear << 3 Lmax) | (l_z << 2 Lmax) | (l_y << Lmax) | l_x, which orders cells
    by coarse cell, then z, y, x.
    """
    G, Lm = params.coarse_res, params.max_level
    s = (2.0 ** L).astype(F32)[:, None]
    f = np.floor(q * s)
    f = np.minimum(f, (ci + 1).astype(F32) * s - F32(1))
    loc = f.astype(np.int64) - ci * (2 ** L)[:, None]
    key = ((coarse_linear(ci, G) << (3 * Lm)) | (loc[:, 2] << (2 * Lm))
           | (loc[:, 1] << Lm) | loc[:, 0])
    return key.astype(np.uint64), loc


def group(keys: np.ndarray):
    """Cells = runs of equal keys after a stable sort; returns (order, cell keys, offsets)."""
    order = np.argsort(keys, kind="stable")
    sk = keys[order]
    if len(sk) == 0:
        return order, sk, np.zeros(1, np.int64)
    head = np.ones(len(sk), bool)
    head[1:] = sk[1:] != sk[:-1]
    starts = np.flatnonzero(head)
    offsets = np.append(starts, len(sk)).astype(np.int64)
    return order, sk[starts], offsets


# ------------------------------------------------------------ Sec. II.5(2) representatives

def _zero_sign(v):
    return v + F32(0.0)     # -0 + 0 = +0: orders -0 and +0 as equal


def representatives(order, offsets, pts: Dict, top: int = 3):
    """II.5(2)a: per cell, the ``top`` members with the highest confidence.

    Ties in C are broken by position (x, y, z ascending) and then pixel id, so the choice does
    not depend on the order in which cameras are listed.  Returns (rep_index (S, top) into
    the point arrays with -1 padding, member count (S,)).
    """
    S = len(offsets) - 1
    M = len(order)
    cell_of = np.repeat(np.arange(S), np.diff(offsets))
    xyz, C, pix = pts["xyz"], pts["conf"], pts["pix"]
    mem = order                                  # members grouped by cell
    rank_order = np.lexsort((pix[mem], _zero_sign(xyz[mem, 2]), _zero_sign(xyz[mem, 1]),
                             _zero_sign(xyz[mem, 0]), -C[mem], cell_of))
    ranked = mem[rank_order]
    pos = np.arange(M) - offsets[cell_of[rank_order]]
    reps = np.full((S, top), -1, np.int64)
    sel = pos < top
    reps[cell_of[rank_order][sel], pos[sel]] = ranked[sel]
    return reps, np.diff(offsets)


def _camera_rank(cams: Sequence[CameraF32]) -> np.ndarray:
    """Rank of each camera under (centre x, y, z, index) — the distance tie-break."""
    cx = np.array([c.centre for c in cams], F32).reshape(-1, 3)
    order = np.lexsort((np.arange(len(cams)), _zero_sign(cx[:, 2]), _zero_sign(cx[:, 1]),
                        _zero_sign(cx[:, 0])))
    rank = np.empty(len(cams), np.int64)
    rank[order] = np.arange(len(cams))
    return rank


def project(cam: CameraF32, p):
    """Eq. 4: camera-frame point X = R p + t (canonical float32 order), then the nearest
    pixel of u = fx X/Z + cx, v = fy Y/Z + cy.  Returns (in_view, px, py): in_view needs
    Z > 0 and the nearest pixel floor(u + 1/2), floor(v + 1/2) inside the image."""
    R, t = cam.R, cam.t
    X = [((R[a, 0] * p[0] + R[a, 1] * p[1]) + R[a, 2] * p[2]) + t[a] for a in range(3)]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        u = cam.fx * (X[0] / X[2]) + cam.cx
        v = cam.fy * (X[1] / X[2]) + cam.cy
        fu = np.floor(u + F32(0.5))
        fv = np.floor(v + F32(0.5))
        ok = (X[2] > 0) & (fu >= 0) & (fu < F32(cam.width)) & (fv >= 0) & (fv < F32(cam.height))
    px = np.where(ok, fu, 0).astype(np.int64)
    py = np.where(ok, fv, 0).astype(np.int64)
    return ok, px, py


def select_views(rep_cam, rep_xyz, cams: Sequence[CameraF32], k_views: int):
    """II.5(2)b: for each representative, the cameras (other than its own) whose view
    contains the point (Eq. 4), ranked by squared distance from the point to the camera
    centre; the first min(K, N) - 1 are kept.  Returns (views (R, K-1) with -1 padding,
    px, py) of the kept views."""
    N = len(cams)
    R = len(rep_cam)
    keep = max(0, min(k_views, N) - 1)
    if keep == 0 or R == 0:
        z = np.zeros((R, keep), np.int64)
        return z - 1, z, z
    p = [rep_xyz[:, 0], rep_xyz[:, 1], rep_xyz[:, 2]]
    ok = np.zeros((R, N), bool)
    dist2 = np.zeros((R, N), F32)
    PX = np.zeros((R, N), np.int64)
    PY = np.zeros((R, N), np.int64)
    for j, cam in enumerate(cams):
        vj, px, py = project(cam, p)
        ok[:, j] = vj & (rep_cam != j)
        with np.errstate(over="ignore", invalid="ignore"):
            dx = p[0] - cam.centre[0]
            dy = p[1] - cam.centre[1]
            dz = p[2] - cam.centre[2]
            dist2[:, j] = (dx * dx + dy * dy) + dz * dz
        PX[:, j], PY[:, j] = px, py
    crank = np.broadcast_to(_camera_rank(cams)[None, :], (R, N))
    order = np.lexsort((crank, dist2, ~ok), axis=1)[:, :keep]
    sel_ok = np.take_along_axis(ok, order, 1)
    views = np.where(sel_ok, order, -1)
    return (views, np.take_along_axis(PX, order, 1), np.take_along_axis(PY, order, 1))


def consistency(rep_cam, rep_xyz, views, px, py, cams, depth, params: Params):
    """Eq. 5-7: reconstruct Q_j = T_j^-1 pi^-1(K_j, u_j, D_j(u_j)) in each kept view,
    d_ij = ||p - Q_j|| (float64), V = exp(-(sum d^2) / (m sigma^2)) over the m views with a
    finite positive depth at u_j; V = 1 when m = 0.

    Returns (sum of d^2, m, V), all per representative."""
    R = len(rep_cam)
    s = np.zeros(R)
    m = np.zeros(R, np.int64)
    for slot in range(views.shape[1]):
        for j, cam in enumerate(cams):
            sel = np.flatnonzero(views[:, slot] == j)
            if len(sel) == 0:
                continue
            D = np.asarray(depth[j], F32)
            d = D[py[sel, slot], px[sel, slot]]
            good = np.isfinite(d) & (d > 0)
            sel, d = sel[good], d[good]
            Q = backproject(cam, px[sel, slot].astype(F32), py[sel, slot].astype(F32), d)
            d2 = np.zeros(len(sel))
            for a in range(3):
                diff = rep_xyz[sel, a].astype(np.float64) - Q[a].astype(np.float64)
                d2 = d2 + diff * diff
            s[sel] += d2
            m[sel] += 1
    sig = float(F32(params.sigma))            # the library takes sigma as float32
    sig2 = sig * sig
    with np.errstate(divide="ignore", invalid="ignore"):
        expo = np.where(m > 0, s / (np.maximum(m, 1) * sig2), 0.0)
    if params.flags & FF_NO_DC:
        expo = np.zeros(R)
    return s, m, expo


# ------------------------------------------------------------ Sec. II.5(2)c, II.5(3)

def fuse_cells(reps: np.ndarray, expo: np.ndarray, pts: Dict, rgb_pts: Optional[np.ndarray]):
    """Eq. 10-11: joint weight w = C V per representative and the normalised weighted mean
    of the representatives' positions (log-domain softmax, float64), output weight = mean w,
    colour = rint of the same weighted mean of colours.

    ``reps`` (S, 3) indexes the point arrays (-1 padding); ``expo`` is -ln V per entry of
    ``reps`` (same shape)."""
    S = reps.shape[0]
    valid = reps >= 0
    idx = np.where(valid, reps, 0)
    C = pts["conf"][idx].astype(np.float64)
    with np.errstate(divide="ignore"):
        a = np.where(valid, np.log(C) - expo, -np.inf)
    amax = a.max(axis=1, keepdims=True)
    ex = np.where(valid, np.exp(a - amax), 0.0)
    pi = ex / ex.sum(axis=1, keepdims=True)
    P = pts["xyz"][idx].astype(np.float64)
    xyz = np.zeros((S, 3))
    for r in range(reps.shape[1]):
        xyz += pi[:, r:r + 1] * np.where(valid[:, r:r + 1], P[:, r], 0.0)
    w = np.where(valid, C * np.exp(-expo), 0.0).sum(axis=1) / valid.sum(axis=1)
    rgb = None
    if rgb_pts is not None:
        col = rgb_pts[idx].astype(np.float64)
        acc = np.zeros((S, 3))
        for r in range(reps.shape[1]):
            acc += pi[:, r:r + 1] * np.where(valid[:, r:r + 1], col[:, r], 0.0)
        rgb = np.clip(np.rint(acc), 0, 255).astype(np.uint8)
    return xyz.astype(F32), w.astype(F32), rgb


# ------------------------------------------------------------ the whole frame

def _rgb_of_points(frame_rgb, cams, pix):
    if frame_rgb is None:
        return None
    flat = np.concatenate([np.asarray(r, np.uint8).reshape(-1, 3) for r in frame_rgb])
    return flat[pix]


def validate_camera(cam) -> None:
    """What the method needs of a camera (Sec. II.1): finite intrinsics and extrinsics and an
    image of at least one pixel on each side.  Any narrower range a particular
    implementation admits is that implementation's limit, not the method's."""
    vals = [float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy)]
    T = np.asarray(cam.world_to_cam, np.float32)
    if not (int(cam.width) >= 1 and int(cam.height) >= 1):
        raise ValueError("image sides must be at least 1")
    if not all(math.isfinite(v) for v in vals):
        raise ValueError("intrinsics must be finite")
    if T.shape != (3, 4) or not np.all(np.isfinite(T)):
        raise ValueError("extrinsics must be a finite 3x4 matrix")


def validate(params: Params, cams) -> None:
    """Reject parameter sets the key layout or the method cannot represent."""
    G = params.coarse_res
    if G < 1 or G & (G - 1) or G > 1024:
        raise ValueError("coarse_res must be a power of two in [1, 1024]")
    if not 0 <= params.max_level <= 16:
        raise ValueError("max_level out of range")
    if 3 * (int(round(math.log2(G))) + params.max_level) > 56:
        raise ValueError("3 (log2 coarse_res + max_level) must be <= 56")
    if not -1 <= params.level_override <= params.max_level:
        raise ValueError("level_override must be -1 or in [0, max_level]")
    if params.target_per_cell < 1 or not 1 <= params.k_views <= 16:
        raise ValueError("target_per_cell >= 1 and k_views in [1, 16] required")
    if not params.sigma > 0:
        raise ValueError("sigma must be positive")
    if sum(int(c.width) * int(c.height) for c in cams) >= 2 ** 32:
        raise ValueError("a frame must have fewer than 2^32 pixels")
    for c in cams:
        validate_camera(c)
    if params.flags & ~(FF_NO_MF | FF_NO_DC | FF_NO_SA | FF_CONF_EQ3):
        raise ValueError("unknown flag")


def fuse(cams_in, depth: Sequence[np.ndarray], conf: Sequence[np.ndarray],
         rgb: Optional[Sequence[np.ndarray]] = None, params: Optional[Params] = None,
         debug: bool = False) -> Dict:
    """Fuse one frame of N cameras into one weighted point per adaptive cell.

    Inputs: cameras (width, height, fx, fy, cx, cy, world_to_cam 3x4), per-camera z-depth
    and confidence (H, W) float32, optional RGB (H, W, 3) uint8.
    Output dict (cells in ascending key order): xyz (S, 3) f32, weight (S,) f32,
    rgb (S, 3) u8 or None, n_members (S,) u32, reps (S, 3) u32 frame pixel ids padded with
    0xFFFFFFFF, keys (S,) u64, member_offsets (S+1,) u32, member_ids (M,) u32 (members of
    each cell in pixel-id order).  With ``debug`` also the intermediate quantities.
    """
    params = params or Params()
    validate(params, cams_in)
    cams = [camera_f32(c) for c in cams_in]
    if params.flags & FF_CONF_EQ3:
        # Sec. II.2: the confidence is computed from the depth maps (Eq. 3), not given
        from oracle.measures import confidence_eq3
        conf = [confidence_eq3(d) for d in depth]
    pts = generate_points(cams, depth, conf, params)
    M = len(pts["pix"])
    rgb_pts = _rgb_of_points(rgb, cams, pts["pix"])
    out: Dict = {}
    dbg: Dict = dict(M=M, pix=pts["pix"], xyz_pts=pts["xyz"], conf_pts=pts["conf"])

    if params.flags & FF_NO_SA:
        # point-wise fusion: every gated point is its own cell, in pixel-id order
        reps = np.arange(M)[:, None]
        views, px, py = select_views(pts["cam"], pts["xyz"], cams, params.k_views)
        _, m, expo = consistency(pts["cam"], pts["xyz"], views, px, py, cams, depth, params)
        xyz, w, frgb = fuse_cells(reps, expo[:, None], pts, rgb_pts)
        out = dict(xyz=xyz, weight=w, rgb=frgb, n_members=np.ones(M, np.uint32),
                   reps=np.concatenate([pts["pix"][:, None].astype(np.uint32),
                                        np.full((M, 2), PAD)], axis=1),
                   keys=pts["pix"].astype(np.uint64),
                   member_offsets=np.arange(M + 1, dtype=np.uint32),
                   member_ids=pts["pix"].astype(np.uint32))
        dbg.update(views=views, m=m, expo=expo)
        if debug:
            out["debug"] = dbg
        return out

    if M == 0:
        out = dict(xyz=np.zeros((0, 3), F32), weight=np.zeros(0, F32),
                   rgb=None if rgb is None else np.zeros((0, 3), np.uint8),
                   n_members=np.zeros(0, np.uint32), reps=np.zeros((0, 3), np.uint32),
                   keys=np.zeros(0, np.uint64), member_offsets=np.zeros(1, np.uint32),
                   member_ids=np.zeros(0, np.uint32))
        if debug:
            out["debug"] = dbg
        return out

    G = params.coarse_res
    bmin, bmax = extents(pts["xyz"])                                   # II.5(1)b
    e = coarse_exponent(bmin, bmax, G)                                 # II.5(1)c
    q, ci = coarse_cells(pts["xyz"], bmin, e, G)
    cl = coarse_linear(ci, G)
    counts = np.bincount(cl, minlength=G ** 3)
    lev_cell = levels(counts, params)                                  # II.5(1)d
    L = lev_cell[cl]
    keys, loc = cell_keys(q, ci, L, params)                            # II.5(1)e
    order, ckeys, offsets = group(keys)
    reps, nmem = representatives(order, offsets, pts)                  # II.5(2)a
    S = len(ckeys)
    flat = reps.reshape(-1)
    rsel = flat >= 0
    ridx = flat[rsel]
    views, px, py = select_views(pts["cam"][ridx], pts["xyz"][ridx], cams,
                                 params.k_views)                       # II.5(2)b, Eq. 4
    s, m, expo_r = consistency(pts["cam"][ridx], pts["xyz"][ridx], views, px, py, cams,
                               depth, params)                          # Eq. 5-7
    expo = np.zeros(flat.shape)
    expo[rsel] = expo_r
    xyz, w, frgb = fuse_cells(reps, expo.reshape(reps.shape), pts, rgb_pts)  # Eq. 10-11

    rep_pix = np.where(reps >= 0, pts["pix"][np.where(reps >= 0, reps, 0)], -1)
    out = dict(xyz=xyz, weight=w, rgb=frgb, n_members=nmem.astype(np.uint32),
               reps=np.where(rep_pix >= 0, rep_pix, PAD).astype(np.uint32), keys=ckeys,
               member_offsets=offsets.astype(np.uint32),
               member_ids=pts["pix"][order].astype(np.uint32))
    if debug:
        sq = np.full(flat.shape, np.nan)
        sq[rsel] = s
        mm = np.zeros(flat.shape, np.int64)
        mm[rsel] = m
        dbg.update(bmin=bmin, bmax=bmax, e=e, q=q, ci=ci, counts=counts,
                   levels=lev_cell, point_level=L, point_keys=keys, loc=loc, order=order,
                   offsets=offsets, rep_index=reps, views=views, rep_sum_d2=sq.reshape(reps.shape),
                   rep_m=mm.reshape(reps.shape), rep_expo=expo.reshape(reps.shape))
        out["debug"] = dbg
    return out


def fuse_frame(frame, params: Optional[Params] = None, debug: bool = False,
               with_rgb: bool = True) -> Dict:
    """Convenience wrapper for a ``synth.Frame``-like object."""
    return fuse(frame.cams, frame.depth, frame.conf, frame.rgb if with_rgb else None,
                params, debug)


def sample_cells(n_members: np.ndarray, n_sample: int, seed: int) -> np.ndarray:
    """Cell indices for a sampled comparison: the first and last cells, the largest cells,
    cells with one, two and three members, and a seeded uniform draw; sorted, unique."""
    S = len(n_members)
    if S == 0:
        return np.zeros(0, np.int64)
    rng = np.random.default_rng(seed)
    pick = [np.array([0, S - 1]), np.argsort(-n_members.astype(np.int64), kind="stable")[:8]]
    for n in (1, 2, 3):
        pick.append(np.flatnonzero(n_members == n)[:4])
    pick.append(rng.choice(S, min(S, n_sample), replace=False))
    return np.unique(np.concatenate(pick).astype(np.int64))


def fuse_sample(cams_in, depth: Sequence[np.ndarray], conf: Sequence[np.ndarray],
                rgb: Optional[Sequence[np.ndarray]] = None, params: Optional[Params] = None,
                n_sample: int = 4000, seed: int = 0) -> Dict:
    """The steps of ``fuse`` with the per-cell work (representatives, views, consistency,
    fusion: Sec. II.5(2)-(3)) done for a sample of cells only, for frames too large for the
    whole oracle to finish quickly.

    The partition (Sec. II.5(1)) and grouping are computed for every point, so ``keys``,
    ``n_members``, ``member_offsets`` and ``member_ids`` cover the whole frame as in
    ``fuse``; ``cells`` (sorted indices into them) names the sampled cells, and ``xyz``,
    ``weight``, ``rgb`` and ``reps`` hold the outputs of those cells in that order.  Each
    sampled cell's outputs are the ones ``fuse`` computes for it: a cell's result depends
    only on its own members and the depth maps."""
    params = params or Params()
    validate(params, cams_in)
    if params.flags & FF_NO_SA:
        raise ValueError("fuse_sample covers the aggregated path only")
    cams = [camera_f32(c) for c in cams_in]
    if params.flags & FF_CONF_EQ3:
        from oracle.measures import confidence_eq3
        conf = [confidence_eq3(d) for d in depth]
    pts = generate_points(cams, depth, conf, params)
    M = len(pts["pix"])
    if M == 0:
        z = np.zeros(0, np.int64)
        return dict(keys=np.zeros(0, np.uint64), n_members=np.zeros(0, np.uint32),
                    member_offsets=np.zeros(1, np.uint32), member_ids=np.zeros(0, np.uint32),
                    cells=z, xyz=np.zeros((0, 3), F32), weight=np.zeros(0, F32),
                    rgb=None if rgb is None else np.zeros((0, 3), np.uint8),
                    reps=np.zeros((0, 3), np.uint32))
    G = params.coarse_res
    bmin, bmax = extents(pts["xyz"])                                   # II.5(1)b
    e = coarse_exponent(bmin, bmax, G)                                 # II.5(1)c
    q, ci = coarse_cells(pts["xyz"], bmin, e, G)
    cl = coarse_linear(ci, G)
    counts = np.bincount(cl, minlength=G ** 3)
    L = levels(counts, params)[cl]                                     # II.5(1)d
    keys, _ = cell_keys(q, ci, L, params)                              # II.5(1)e
    order, ckeys, offsets = group(keys)
    nmem = np.diff(offsets)
    cells = sample_cells(nmem, n_sample, seed)

    # the sampled cells' members, regrouped as a smaller partition
    lens = nmem[cells]
    sub_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    sub_order = np.concatenate([order[offsets[c]:offsets[c + 1]] for c in cells])
    keep = np.unique(sub_order)                                        # pixel-id order
    remap = np.full(M, -1, np.int64)
    remap[keep] = np.arange(len(keep))
    spts = {k: v[keep] for k, v in pts.items()}
    reps, _ = representatives(remap[sub_order], sub_off, spts)         # II.5(2)a
    flat = reps.reshape(-1)
    rsel = flat >= 0
    ridx = flat[rsel]
    views, px, py = select_views(spts["cam"][ridx], spts["xyz"][ridx], cams,
                                 params.k_views)                       # II.5(2)b, Eq. 4
    _, _, expo_r = consistency(spts["cam"][ridx], spts["xyz"][ridx], views, px, py, cams,
                               depth, params)                          # Eq. 5-7
    expo = np.zeros(flat.shape)
    expo[rsel] = expo_r
    rgb_pts = _rgb_of_points(rgb, cams, spts["pix"])
    xyz, w, frgb = fuse_cells(reps, expo.reshape(reps.shape), spts, rgb_pts)  # Eq. 10-11
    rep_pix = np.where(reps >= 0, spts["pix"][np.where(reps >= 0, reps, 0)], -1)
    return dict(keys=ckeys, n_members=nmem.astype(np.uint32),
                member_offsets=offsets.astype(np.uint32),
                member_ids=pts["pix"][order].astype(np.uint32), cells=cells,
                xyz=xyz, weight=w, rgb=frgb,
                reps=np.where(rep_pix >= 0, rep_pix, PAD).astype(np.uint32))


def fuse_frame_sample(frame, params: Optional[Params] = None, n_sample: int = 4000,
                      seed: int = 0, with_rgb: bool = True) -> Dict:
    """``fuse_sample`` for a ``synth.Frame``-like object."""
    return fuse_sample(frame.cams, frame.depth, frame.conf, frame.rgb if with_rgb else None,
                       params, n_sample, seed)
