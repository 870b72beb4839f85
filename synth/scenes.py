"""Seeded synthetic rigs shaped like the workloads of the FUSE-Flow evaluation.

The paper evaluates on real multi-camera captures that were never released (Sec. III.1),
so every input here is synthetic: analytic scenes (a ground plane, spheres and axis-aligned
boxes) ray-cast into z-depth maps, with depth noise, outliers and per-pixel confidence.

Conventions
-----------
* World frame: right-handed, z up, metres.
* Camera frame: OpenCV (x right, y down, z forward).  ``world_to_cam`` is the 3x4 matrix
  [R | t] with t = -R c, i.e. it maps world points into the camera frame; the fusion
  method applies its inverse to go from camera to world (Sec. II.4, Eq. 8).
* Depth is the z-depth of the nearest hit (not the ray length), 0 where a ray hits nothing.
* Intrinsics: fx = fy = 300 * W / 320, cx = W / 2, cy = H / 2 (a 56 degree horizontal
  field of view at every resolution).
* Cameras sit on a ring of radius 3 m at height 0.5 m, yaw 2*pi*k/N, looking at the origin.
* The ground is a square floor at z = -1 m (half-width 8 m; 16 m for c3) and the sensor
  returns nothing beyond a z-depth of 10 m (16 m for c3), as real RGB-D sensors do.

Configs (see ``CONFIGS``)
-------------------------
c1  2 x 320x240, ground + 3 spheres, sigma_z = 0.001 z^2, no outliers, C ~ U[0.5, 1].
c2  4 x 640x480 ring with jitter, ground + 10 spheres + 1 box, 2 % outliers in
    U[0.3, 8] m, C ~ Beta(5, 2), 0 on no-hit pixels, halved next to depth jumps > 5 cm.
c3  8 x 1280x720, 200 primitives: 140 small ones (0.05-0.2 m) in a 1.2 m ball round the
    origin and 60 large ones (0.3-1 m) at 5-12 m range; 3 % outliers; C as c2; RGB.
c4  16 cameras (6 x 640x480, 6 x 1280x720, 4 x 1920x1080, seeded order round the ring),
    c2 scene family with spheres moving at 0.5 m/s and reflecting off the [-2, 2]^3 walls;
    frame f is at t = f / 30 s.
c5  serving rigs 0..3 with 2, 6, 12, 32 cameras, each camera's resolution drawn from
    {640x480, 1280x720, 1920x1080}; dynamic c2 scene family.

Seeds: config k uses scene seed 1000 k + 100 * rig (rig 0 for single-rig configs); the
per-frame noise/confidence draw uses scene seed + frame.  Everything is NumPy PCG64.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = ["Camera", "Frame", "Primitive", "ring_cameras", "render", "make_frame",
           "make_config", "CONFIGS"]


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    world_to_cam: np.ndarray  # (3, 4) float32, [R | t]

    @property
    def pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Primitive:
    kind: str                 # "plane" | "sphere" | "box"
    centre: np.ndarray        # (3,) float64 (plane: unused)
    size: np.ndarray          # sphere: (1,) radius; box: (3,) half extents; plane: (1,) height
    colour: np.ndarray        # (3,) in [0, 1]
    velocity: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))


@dataclasses.dataclass
class Frame:
    cams: List[Camera]
    depth: List[np.ndarray]            # (H, W) float32
    conf: List[np.ndarray]             # (H, W) float32
    rgb: Optional[List[np.ndarray]]    # (H, W, 3) uint8
    label: List[np.ndarray]            # (H, W) int32: -1 no hit, else primitive index
    clean_depth: List[np.ndarray]      # (H, W) float64 noise-free z-depth (inf = no hit)
    outlier: List[np.ndarray]          # (H, W) bool
    prims: List[Primitive]

    @property
    def pixels(self) -> int:
        return sum(c.pixels for c in self.cams)


# ----------------------------------------------------------------------------- cameras

def _look_at(c: np.ndarray, target: np.ndarray) -> np.ndarray:
    f = target - c
    f = f / np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0])
    r = np.cross(f, up)
    r = r / np.linalg.norm(r)
    d = np.cross(f, r)
    return np.stack([r, d, f])          # rows: camera x (right), y (down), z (forward)


def make_camera(width: int, height: int, centre: np.ndarray, target: np.ndarray) -> Camera:
    R = _look_at(np.asarray(centre, np.float64), np.asarray(target, np.float64))
    t = -R @ np.asarray(centre, np.float64)
    T = np.concatenate([R, t[:, None]], axis=1).astype(np.float32)
    f = 300.0 * width / 320.0
    return Camera(width, height, f, f, width / 2.0, height / 2.0, T)


def ring_cameras(resolutions: Sequence[Tuple[int, int]], radius: float = 3.0,
                 height: float = 0.5, jitter_pos: float = 0.0, jitter_target: float = 0.0,
                 rng: Optional[np.random.Generator] = None) -> List[Camera]:
    n = len(resolutions)
    cams = []
    for k, (w, h) in enumerate(resolutions):
        yaw = 2.0 * np.pi * k / n
        c = np.array([radius * np.cos(yaw), radius * np.sin(yaw), height])
        tgt = np.zeros(3)
        if jitter_pos > 0:
            c = c + rng.uniform(-jitter_pos, jitter_pos, 3)
        if jitter_target > 0:
            tgt = tgt + rng.uniform(-jitter_target, jitter_target, 3)
        cams.append(make_camera(w, h, c, tgt))
    return cams


def _cam64(cam: Camera):
    T = cam.world_to_cam.astype(np.float64)
    R, t = T[:, :3], T[:, 3]
    return R, t, -R.T @ t


# ----------------------------------------------------------------------------- ray casting

def _rect(cam: Camera, R, t, lo, hi):
    """Conservative pixel rectangle containing the image of the box [lo, hi]."""
    corners = np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1])
                        for z in (lo[2], hi[2])])
    X = corners @ R.T + t
    if np.all(X[:, 2] <= 0.0):
        return 0, 0, 0, 0                      # entirely behind the camera
    if np.any(X[:, 2] <= 1e-3):
        return 0, cam.width, 0, cam.height
    u = cam.fx * X[:, 0] / X[:, 2] + cam.cx
    v = cam.fy * X[:, 1] / X[:, 2] + cam.cy
    x0 = int(max(0, np.floor(u.min()) - 1))
    x1 = int(min(cam.width, np.ceil(u.max()) + 2))
    y0 = int(max(0, np.floor(v.min()) - 1))
    y1 = int(min(cam.height, np.ceil(v.max()) + 2))
    return x0, x1, y0, y1


def render(cam: Camera, prims: Sequence[Primitive], max_range: float = np.inf):
    """Ray-cast one camera: returns (z-depth float64 with inf for no hit, label, shade).
    Hits farther than ``max_range`` (z-depth) return nothing, like a real depth sensor."""
    R, t, c = _cam64(cam)
    H, W = cam.height, cam.width
    xs = (np.arange(W, dtype=np.float64) - cam.cx) / cam.fx
    ys = (np.arange(H, dtype=np.float64) - cam.cy) / cam.fy
    # world-space ray direction for camera-frame direction (xs, ys, 1): d = R^T [xs, ys, 1]
    dirs = (xs[None, :, None] * R[0][None, None, :] + ys[:, None, None] * R[1][None, None, :]
            + R[2][None, None, :])                      # (H, W, 3)
    depth = np.full((H, W), np.inf)
    label = np.full((H, W), -1, np.int32)
    cosang = np.zeros((H, W))
    for k, p in enumerate(prims):
        if p.kind == "plane":
            h, half = float(p.size[0]), float(p.size[1])
            dz = dirs[..., 2]
            with np.errstate(divide="ignore", invalid="ignore"):
                tt = (h - c[2]) / dz
            gx = c[0] + tt * dirs[..., 0]
            gy = c[1] + tt * dirs[..., 1]
            hit = ((tt > 0) & np.isfinite(tt) & (tt < depth) & (np.abs(gx) <= half)
                   & (np.abs(gy) <= half))
            depth[hit] = tt[hit]
            label[hit] = k
            dn = np.abs(dirs[..., 2]) / np.linalg.norm(dirs, axis=-1)
            cosang[hit] = dn[hit]
            continue
        if p.kind == "sphere":
            r = float(p.size[0])
            lo, hi = p.centre - r, p.centre + r
        else:
            lo, hi = p.centre - p.size, p.centre + p.size
        x0, x1, y0, y1 = _rect(cam, R, t, lo, hi)
        if x0 >= x1 or y0 >= y1:
            continue
        d = dirs[y0:y1, x0:x1]
        cur = depth[y0:y1, x0:x1]
        if p.kind == "sphere":
            oc = c - p.centre
            a = np.einsum("hwk,hwk->hw", d, d)
            b = d @ oc
            cc = oc @ oc - r * r
            disc = b * b - a * cc
            ok = disc >= 0
            sq = np.sqrt(np.where(ok, disc, 0.0))
            t1 = (-b - sq) / a
            t2 = (-b + sq) / a
            tt = np.where(t1 > 0, t1, t2)
            hit = ok & (tt > 0) & (tt < cur)
            if not hit.any():
                continue
            P = c + tt[..., None] * d
            n = (P - p.centre) / r
        else:
            with np.errstate(divide="ignore", invalid="ignore"):
                dd = np.where(np.abs(d) < 1e-12, 1e-12, d)
                ta = (lo - c) / dd
                tb = (hi - c) / dd
            tmin = np.minimum(ta, tb)
            tmax = np.maximum(ta, tb)
            tnear = tmin.max(axis=-1)
            tfar = tmax.min(axis=-1)
            axis = tmin.argmax(axis=-1)
            tt = np.where(tnear > 0, tnear, tfar)
            hit = (tnear <= tfar) & (tt > 0) & (tt < cur)
            if not hit.any():
                continue
            n = np.zeros(d.shape)
            sgn = -np.sign(np.take_along_axis(d, axis[..., None], -1))[..., 0]
            np.put_along_axis(n, axis[..., None], sgn[..., None], -1)
        cur[hit] = tt[hit]
        label[y0:y1, x0:x1][hit] = k
        dn = np.abs(np.einsum("hwk,hwk->hw", n, d)) / np.linalg.norm(d, axis=-1)
        cosang[y0:y1, x0:x1][hit] = dn[hit]
    far = depth > max_range
    depth[far] = np.inf
    label[far] = -1
    return depth, label, cosang


# ----------------------------------------------------------------------------- scenes

def _far_enough(centre, reach, cams, margin=0.3):
    for cam in cams:
        _, _, c = _cam64(cam)
        if np.linalg.norm(centre - c) - reach < margin:
            return False
    return True


def _sample_prims(rng, cams, n, kind_fn, size_fn, centre_fn, velocity=0.0):
    prims = []
    while len(prims) < n:
        kind = kind_fn()
        size = size_fn(kind)
        centre = centre_fn()
        reach = float(np.linalg.norm(size)) if kind == "box" else float(size[0])
        if not _far_enough(centre, reach, cams):
            continue
        vel = np.zeros(3)
        if velocity > 0:
            v = rng.normal(size=3)
            vel = velocity * v / np.linalg.norm(v)
        prims.append(Primitive(kind, centre, size, rng.uniform(0.2, 1.0, 3), vel))
    return prims


def _ground(half: float = 8.0):
    """Square floor at z = -1 m, |x|, |y| <= half."""
    return Primitive("plane", np.zeros(3), np.array([-1.0, half]), np.array([0.6, 0.6, 0.6]))


def _reflect(x, lo, hi):
    span = hi - lo
    y = np.mod(x - lo, 2.0 * span)
    return lo + np.where(y > span, 2.0 * span - y, y)


def _at_time(prims, tsec):
    out = []
    for p in prims:
        if p.kind == "plane" or not np.any(p.velocity):
            out.append(p)
            continue
        r = float(p.size[0]) if p.kind == "sphere" else float(np.max(p.size))
        lo, hi = -2.0 + r, 2.0 - r
        c = _reflect(p.centre + p.velocity * tsec, lo, hi) if hi > lo else p.centre
        out.append(dataclasses.replace(p, centre=c))
    return out


def _scene_c1(rng, cams):
    return [_ground()] + _sample_prims(
        rng, cams, 3, lambda: "sphere", lambda k: np.array([rng.uniform(0.3, 0.8)]),
        lambda: rng.uniform(-2.0, 2.0, 3))


def _scene_c2(rng, cams, velocity=0.0):
    spheres = _sample_prims(
        rng, cams, 10, lambda: "sphere", lambda k: np.array([rng.uniform(0.3, 0.8)]),
        lambda: rng.uniform(-2.0, 2.0, 3), velocity=velocity)
    box = _sample_prims(rng, cams, 1, lambda: "box", lambda k: rng.uniform(0.2, 0.6, 3),
                        lambda: rng.uniform(-2.0, 2.0, 3))
    return [_ground()] + spheres + box


def _ball(rng, radius):
    while True:
        p = rng.uniform(-radius, radius, 3)
        if np.linalg.norm(p) <= radius:
            return p


def _scene_c3(rng, cams):
    kind = lambda: "sphere" if rng.random() < 0.5 else "box"

    def size_near(k):
        return np.array([rng.uniform(0.05, 0.2)]) if k == "sphere" else rng.uniform(0.05, 0.2, 3)

    def size_far(k):
        return np.array([rng.uniform(0.3, 1.0)]) if k == "sphere" else rng.uniform(0.3, 1.0, 3)

    def centre_far():
        rr, az = rng.uniform(5.0, 12.0), rng.uniform(0.0, 2.0 * np.pi)
        return np.array([rr * np.cos(az), rr * np.sin(az), rng.uniform(-1.0, 2.0)])

    near = _sample_prims(rng, cams, 140, kind, size_near, lambda: _ball(rng, 1.2))
    far = _sample_prims(rng, cams, 60, kind, size_far, centre_far)
    return [_ground(16.0)] + near + far


# ----------------------------------------------------------------------------- frames

def _discontinuity(clean: np.ndarray, thresh: float = 0.05) -> np.ndarray:
    """True where the noise-free depth jumps by more than ``thresh`` to a 4-neighbour
    (a neighbour without a hit counts as a jump)."""
    jump = np.zeros(clean.shape, bool)
    for axis in (0, 1):
        a = np.swapaxes(clean, 0, axis)
        j = np.swapaxes(jump, 0, axis)
        with np.errstate(invalid="ignore"):
            diff = np.abs(a[1:] - a[:-1])
        big = ~(diff <= thresh)          # NaN/inf (no hit) counts as a jump
        j[1:] |= big
        j[:-1] |= big
    return jump


def make_frame(cams: Sequence[Camera], prims: Sequence[Primitive], seed: int, *,
               outlier_frac: float = 0.0, conf_model: str = "uniform",
               noise: bool = True, with_rgb: bool = True, max_range: float = 10.0) -> Frame:
    """Render every camera and draw noise, outliers and confidence with ``seed``."""
    rng = np.random.default_rng(seed)
    depth, conf, rgb, labels, cleans, outs = [], [], [], [], [], []
    # ray casting draws no random numbers, so cameras render in parallel threads
    # (NumPy releases the GIL); noise and confidence are drawn afterwards in camera order
    with concurrent.futures.ThreadPoolExecutor(min(len(cams), os.cpu_count() or 1)) as ex:
        rendered = list(ex.map(lambda cam: render(cam, prims, max_range), cams))
    for cam, (clean, label, cosang) in zip(cams, rendered):
        hit = np.isfinite(clean)
        H, W = clean.shape
        z = np.where(hit, clean, 0.0)
        eps = rng.standard_normal((H, W))
        d = z + eps * 0.001 * z * z if noise else z.copy()
        out = np.zeros((H, W), bool)
        if outlier_frac > 0:
            out = rng.random((H, W)) < outlier_frac
            d[out] = rng.uniform(0.3, 8.0, int(out.sum()))
        d[(~hit) & (~out)] = 0.0
        d[d <= 0] = 0.0
        d32 = d.astype(np.float32)
        if conf_model == "uniform":
            c = rng.uniform(0.5, 1.0, (H, W)).astype(np.float32)
        else:
            c = rng.beta(5.0, 2.0, (H, W)).astype(np.float32)
            c[~hit] = 0.0
            c[_discontinuity(clean)] *= np.float32(0.5)
        depth.append(d32)
        conf.append(c)
        labels.append(label)
        cleans.append(clean)
        outs.append(out)
        if with_rgb:
            base = np.stack([prims[k].colour if k >= 0 else np.zeros(3)
                             for k in range(len(prims))] + [np.zeros(3)])
            col = base[label] * (0.25 + 0.75 * cosang)[..., None]
            rgb.append(np.clip(np.rint(col * 255.0), 0, 255).astype(np.uint8))
    return Frame(list(cams), depth, conf, rgb if with_rgb else None, labels, cleans,
                 outs, list(prims))


_RES = [(640, 480), (1280, 720), (1920, 1080)]

CONFIGS = ("c1", "c2", "c3", "c4", "c5")


def make_config(name: str, frame: int = 0, rig: int = 0, *, with_rgb: bool = True,
                noise: bool = True) -> Frame:
    """Build frame ``frame`` of config ``name`` (for c3 and c5, of rig ``rig``)."""
    if name == "c1":
        seed = 1000 + 100 * rig
        rng = np.random.default_rng(seed)
        cams = ring_cameras([(320, 240)] * 2)
        prims = _scene_c1(rng, cams)
        return make_frame(cams, prims, seed + frame, conf_model="uniform",
                          noise=noise, with_rgb=with_rgb)
    if name == "c2":
        seed = 2000 + 100 * rig
        rng = np.random.default_rng(seed)
        cams = ring_cameras([(640, 480)] * 4, jitter_pos=0.1, jitter_target=0.2, rng=rng)
        prims = _scene_c2(rng, cams)
        return make_frame(cams, prims, seed + frame, outlier_frac=0.02 if noise else 0.0,
                          conf_model="beta", noise=noise, with_rgb=with_rgb)
    if name == "c3":
        seed = 3000 + 100 * rig
        rng = np.random.default_rng(seed)
        cams = ring_cameras([(1280, 720)] * 8)
        prims = _scene_c3(rng, cams)
        return make_frame(cams, prims, seed + frame, outlier_frac=0.03 if noise else 0.0,
                          conf_model="beta", noise=noise, with_rgb=with_rgb, max_range=16.0)
    if name == "c4":
        seed = 4000 + 100 * rig
        rng = np.random.default_rng(seed)
        res = [_RES[0]] * 6 + [_RES[1]] * 6 + [_RES[2]] * 4
        res = [res[i] for i in rng.permutation(len(res))]
        cams = ring_cameras(res, jitter_pos=0.1, jitter_target=0.2, rng=rng)
        prims = _at_time(_scene_c2(rng, cams, velocity=0.5), frame / 30.0)
        return make_frame(cams, prims, seed + frame, outlier_frac=0.02 if noise else 0.0,
                          conf_model="beta", noise=noise, with_rgb=with_rgb)
    if name == "c5":
        n = (2, 6, 12, 32)[rig]
        seed = 5000 + 100 * rig
        rng = np.random.default_rng(seed)
        res = [_RES[i] for i in rng.integers(0, 3, n)]
        cams = ring_cameras(res, jitter_pos=0.1, jitter_target=0.2, rng=rng)
        prims = _at_time(_scene_c2(rng, cams, velocity=0.5), frame / 30.0)
        return make_frame(cams, prims, seed + frame, outlier_frac=0.02 if noise else 0.0,
                          conf_model="beta", noise=noise, with_rgb=with_rgb)
    raise ValueError(f"unknown config {name!r}")


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process, seeded (serving streams use 7000 + rig)."""
    rng = np.random.default_rng(seed)
    n = int(rate_hz * duration_s * 2 + 20)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    return t[t < duration_s]
