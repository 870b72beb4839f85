"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a hand-derived worked
example, a closed form, a brute-force recomputation written differently, or an invariant.
None of these tests touches the GPU library.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import core as O
from synth import make_config, make_frame, ring_cameras
from synth.scenes import Camera, Primitive, make_camera, _scene_c1

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F32 = np.float32


def _cam(d):
    return Camera(d["width"], d["height"], d["fx"], d["fy"], d["cx"], d["cy"],
                  np.array(d["world_to_cam"], np.float32))


# ---------------------------------------------------------------- P1: Eq. 8 back-projection

def test_backproject_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "backproject_worked_example.json")))
    cam = O.camera_f32(_cam(g["camera"]))
    assert list(cam.centre) == g["centre"]
    for case in g["cases"]:
        p = O.backproject(cam, [case["x"]], [case["y"]], [case["d"]])
        assert [float(v[0]) for v in p] == case["world"]


def test_paper_constants():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert O.Params().tau == g["tau"]["value"]
    # top-3 representatives: a cell of 5 points keeps exactly 3
    pts = dict(xyz=np.zeros((5, 3), F32), conf=np.array([.7, .8, .9, .65, .95], F32),
               pix=np.arange(5))
    reps, n = O.representatives(np.arange(5), np.array([0, 5]), pts)
    assert (reps >= 0).sum() == g["representatives_per_cell"]["value"]
    assert list(reps[0]) == [4, 2, 1]


def test_points_lie_on_their_primitives():
    """Noise-free rig: every gated point back-projects onto the analytic surface that the
    renderer hit at that pixel (plane or sphere), to float32 accuracy."""
    f = make_config("c1", noise=False, with_rgb=False)
    cams = [O.camera_f32(c) for c in f.cams]
    P = O.Params()
    for k, cam in enumerate(cams):
        ok = O.gate(f.depth[k], f.conf[k], P)
        yy, xx = np.nonzero(ok)
        p = np.stack(O.backproject(cam, xx.astype(F32), yy.astype(F32),
                                   f.depth[k][yy, xx]), 1).astype(np.float64)
        z = f.depth[k][yy, xx].astype(np.float64)
        lab = f.label[k][yy, xx]
        for li in np.unique(lab):
            prim = f.prims[li]
            sel = lab == li
            if prim.kind == "plane":
                err = np.abs(p[sel, 2] - prim.size[0])
            else:
                err = np.abs(np.linalg.norm(p[sel] - prim.centre, axis=1) - prim.size[0])
            assert np.all(err <= 2e-6 * z[sel] + 1e-6), (prim.kind, err.max())


# ---------------------------------------------------------------- P2: Eq. 4 projection

def test_projection_round_trip(frame_c2):
    """project(backproject(x, y, d)) returns (x, y) in the same camera for every pixel."""
    for k, c in enumerate(frame_c2.cams):
        cam = O.camera_f32(c)
        yy, xx = np.nonzero(frame_c2.depth[k] > 0)
        p = O.backproject(cam, xx.astype(F32), yy.astype(F32), frame_c2.depth[k][yy, xx])
        ok, px, py = O.project(cam, p)
        assert ok.all() and (px == xx).all() and (py == yy).all()


def test_projection_rejects_points_behind_and_outside():
    g = json.load(open(os.path.join(GOLDEN, "backproject_worked_example.json")))
    cam = O.camera_f32(_cam(g["camera"]))
    # camera at (-2, 1, 0.5) looks along +x: a point at x = -3 is behind it
    ok, _, _ = O.project(cam, [np.array([-3.0], F32), np.array([1.0], F32), np.array([0.5], F32)])
    assert not ok[0]
    # far off to the side: outside the 8x6 image
    ok, _, _ = O.project(cam, [np.array([0.0], F32), np.array([-50.0], F32), np.array([0.5], F32)])
    assert not ok[0]
    # the worked-example point projects back to pixel (6, 1)
    ok, px, py = O.project(cam, [np.array([0.5], F32), np.array([-0.25], F32), np.array([3.0], F32)])
    assert ok[0] and px[0] == 6 and py[0] == 1


# ---------------------------------------------------------------- P3: Eq. 9 gate

def test_gate_planted_values():
    D = np.array([[1.0, 1.0, 1.0, 1.0, np.nan, np.inf, -1.0, 0.0, 1.0]], F32)
    C = np.array([[0.6, np.nextafter(F32(0.6), F32(1)), 1.0, np.nan, 0.9, 0.9, 0.9, 0.9, 0.59]], F32)
    ok = O.gate(D, C, O.Params())
    assert ok.tolist() == [[False, True, True, False, False, False, False, False, False]]
    ok = O.gate(D, C, O.Params(flags=O.FF_NO_MF))
    assert ok.tolist() == [[True, True, True, True, False, False, False, False, True]]


def test_gate_fraction_matches_distributions(frame_c1):
    """tau = 0.6 on C ~ U[0.5, 1] keeps 80 % of valid depths; on Beta(5, 2) it keeps
    1 - I_0.6(5, 2) = 1 - (6 x^5 - 5 x^6)|_0.6 = 0.76672."""
    valid = np.concatenate([(d > 0).ravel() for d in frame_c1.depth])
    C = np.concatenate([c.ravel() for c in frame_c1.conf])
    kept = O.gate(np.concatenate([d.ravel() for d in frame_c1.depth]), C, O.Params())
    frac = kept.sum() / valid.sum()
    n = valid.sum()
    assert abs(frac - 0.8) < 5 * math.sqrt(0.16 / n)
    rng = np.random.default_rng(5)
    b = rng.beta(5, 2, 400000).astype(F32)
    frac = O.gate(np.ones_like(b), b, O.Params()).mean()
    x = 0.6
    assert abs(frac - (1 - (6 * x ** 5 - 5 * x ** 6))) < 5 * math.sqrt(0.25 / len(b))


# ---------------------------------------------------------------- P4: II.5(1) partition

def test_coarse_exponent_closed_forms():
    z = np.zeros(3, F32)
    e = lambda ext, G=64: O.coarse_exponent(z, np.array([ext, 0, 0], F32), G)
    assert e(3.0) == -4            # 64 * 2^-4 = 4 >= 3 > 2
    assert e(4.0) == -4            # exactly 64 cells
    assert e(float(np.nextafter(F32(4), F32(5)))) == -3
    assert e(1.0, G=1) == 0 and e(1.5, G=1) == 1
    assert O.coarse_exponent(z, z, 64) == O.E_MIN
    big = np.array([3e38, 0, 0], F32)
    assert O.coarse_exponent(-big, big, 64) == O.E_MAX   # extent overflows float32


def test_levels_lattice():
    counts = np.array([0, 1, 16, 17, 64, 65, 256, 257, 1024, 1025, 10 ** 9])
    assert O.levels(counts, O.Params()).tolist() == [0, 0, 0, 1, 1, 2, 2, 3, 3, 4, 6]
    assert O.levels(counts, O.Params(level_override=2)).tolist() == [2] * len(counts)
    P = O.Params(target_per_cell=4, max_level=2)
    assert O.levels(np.array([4, 5, 16, 17, 65]), P).tolist() == [0, 1, 1, 2, 2]


def _tiny_points(seed, n=1500):
    rng = np.random.default_rng(seed)
    # clustered points: a dense blob, a plane patch and sparse outliers
    a = rng.normal(0, 0.05, (n // 2, 3))
    b = np.c_[rng.uniform(-1, 1, (n // 3, 2)), np.full(n // 3, 0.3)]
    c = rng.uniform(-3, 3, (n - len(a) - len(b), 3))
    return np.concatenate([a, b, c]).astype(F32)


@pytest.mark.parametrize("seed", [0, 1])
def test_partition_brute_force(seed):
    """Brute force over all pairs of a tiny cloud: equal keys <=> equal (coarse, fine)
    integer cells; every point lies inside its cell's box; levels from direct counts."""
    xyz = _tiny_points(seed)
    P = O.Params(target_per_cell=4, max_level=5)
    bmin, bmax = O.extents(xyz)
    assert (bmin == xyz.min(0)).all() and (bmax == xyz.max(0)).all()
    e = O.coarse_exponent(bmin, bmax, P.coarse_res)
    s0 = 2.0 ** e
    ext = float((bmax - bmin).max())
    assert P.coarse_res * s0 >= ext > P.coarse_res * s0 / 2
    q, ci = O.coarse_cells(xyz, bmin, e, P.coarse_res)
    cl = O.coarse_linear(ci, P.coarse_res)
    counts = np.bincount(cl, minlength=P.coarse_res ** 3)
    L = O.levels(counts, P)[cl]
    keys, loc = O.cell_keys(q, ci, L, P)
    # brute-force counts and levels
    direct = {}
    for t in map(tuple, ci):
        direct[t] = direct.get(t, 0) + 1
    for i in range(len(xyz)):
        n = direct[tuple(ci[i])]
        lev = 0
        while lev < P.max_level and n > P.target_per_cell * 4 ** lev:
            lev += 1
        assert L[i] == lev
    # every point inside its cell box (float64), up to one float32 rounding of p - bmin
    s = s0 / 2.0 ** L
    fine = ci * (2 ** L)[:, None] + loc
    lo = bmin.astype(np.float64) + fine * s[:, None]
    slack = np.abs(xyz.astype(np.float64) - bmin) * 2.0 ** -23 + 1e-30
    assert np.all(xyz >= lo - slack) and np.all(xyz <= lo + s[:, None] + slack)
    # pairwise: same key <=> same (coarse cell, level, local offset)
    ident = [tuple(ci[i]) + (int(L[i]),) + tuple(loc[i]) for i in range(len(xyz))]
    for i in range(len(xyz)):
        same_key = keys == keys[i]
        same_cell = np.array([ident[j] == ident[i] for j in range(len(xyz))])
        assert (same_key == same_cell).all()
        d = np.linalg.norm(xyz[same_key].astype(np.float64) - xyz[i], axis=1)
        assert d.max() <= math.sqrt(3) * s[i] * (1 + 1e-6) + 1e-6
    # key order = (coarse linear, z, y, x) lexicographic
    order = np.lexsort((loc[:, 0], loc[:, 1], loc[:, 2], cl))
    assert (np.diff(keys[order].astype(np.float64)) >= 0).all()


def test_key_layout_bits():
    P = O.Params()
    q = np.array([[63.99, 0.0, 63.99]], F32)
    ci = np.array([[63, 0, 63]])
    key, loc = O.cell_keys(q, ci, np.array([6]), P)
    assert loc.tolist() == [[63, 0, 63]]
    assert int(key[0]) == (((63 * 64 + 0) * 64 + 63) << 18) | (63 << 12) | (0 << 6) | 63


# ---------------------------------------------------------------- P5: II.5(2)a top-3

def test_representatives_brute_force():
    rng = np.random.default_rng(3)
    n = 400
    conf = rng.choice(np.array([0.7, 0.8, 0.9, 0.95], F32), n)    # many ties
    xyz = rng.choice(np.array([-1, 0, 1], F32), (n, 3))             # ties in position too
    xyz[rng.random(n) < 0.2, 0] = F32(-0.0)
    pix = rng.permutation(10 * n)[:n]
    keys = rng.integers(0, 40, n).astype(np.uint64)
    order, ck, off = O.group(keys)
    reps, nm = O.representatives(order, off, dict(xyz=xyz, conf=conf, pix=pix))
    for s, k in enumerate(ck):
        mem = [i for i in range(n) if keys[i] == k]
        best = sorted(mem, key=lambda i: (-float(conf[i]), float(xyz[i, 0]) + 0.0,
                                          float(xyz[i, 1]), float(xyz[i, 2]), int(pix[i])))
        assert list(reps[s][:min(3, len(mem))]) == best[:3]
        assert nm[s] == len(mem)
    # members listed in input order within each cell (stable grouping)
    for s in range(len(ck)):
        mem = order[off[s]:off[s + 1]]
        assert (np.diff(mem) > 0).all()


# ---------------------------------------------------------------- P6: II.5(2)b views

def test_view_selection_brute_force():
    f = make_config("c2", noise=False, with_rgb=False)
    cams = [O.camera_f32(c) for c in f.cams]
    rng = np.random.default_rng(7)
    k = 1
    yy, xx = np.nonzero(f.depth[k] > 0)
    pick = rng.choice(len(yy), 300, replace=False)
    p = np.stack(O.backproject(cams[k], xx[pick].astype(F32), yy[pick].astype(F32),
                               f.depth[k][yy[pick], xx[pick]]), 1)
    for K in (2, 3, 4, 8):
        views, px, py = O.select_views(np.full(len(pick), k), p, cams, K)
        for r in range(len(pick)):
            cand = []
            for j, cam in enumerate(cams):
                if j == k:
                    continue
                X = [float(v) for v in (cam.R.astype(np.float64) @ p[r].astype(np.float64)
                                        + cam.t)]
                if X[2] <= 0:
                    continue
                u = cam.fx * (X[0] / X[2]) + cam.cx
                v = cam.fy * (X[1] / X[2]) + cam.cy
                if not (0 <= math.floor(u + .5) < cam.width and 0 <= math.floor(v + .5) < cam.height):
                    continue
                dist = float(np.sum((p[r].astype(np.float64) - cam.centre) ** 2))
                cand.append((dist, j))
            cand.sort()
            want = [j for _, j in cand[:min(K, len(cams)) - 1]]
            got = [int(j) for j in views[r] if j >= 0]
            assert got == want, (r, got, want)


def test_all_views_pass_picks_nearest_centres():
    # eight cameras on a ring all looking at a point near the origin: every view passes,
    # and the kept views are the K - 1 nearest other cameras
    cams_in = ring_cameras([(64, 48)] * 8)
    cams = [O.camera_f32(c) for c in cams_in]
    p = np.array([[0.5, 0.1, 0.0]], F32)
    views, _, _ = O.select_views(np.array([0]), p, cams, 4)
    d = [float(np.sum((p[0].astype(np.float64) - c.centre) ** 2)) for c in cams]
    want = sorted(range(1, 8), key=lambda j: d[j])[:3]
    assert views[0].tolist() == want


# ---------------------------------------------------------------- P7: Eq. 5-7 closed form

def _stereo_plane(n_extra, delta, Z=2.0, b=0.5, f=100.0, W=160, H=120):
    """Camera 0 looks along world +z at a fronto-parallel plane at depth Z; cameras 1..n are
    camera 0 shifted by b, 2b, ... along its x axis (same orientation), so that a pixel
    shifts by exactly b f / Z = 25 columns per camera."""
    cams = []
    for k in range(n_extra + 1):
        c = np.array([k * b, 0.0, 0.0])
        R = np.eye(3)
        t = -R @ c
        cams.append(Camera(W, H, f, f, W / 2.0, H / 2.0,
                           np.concatenate([R, t[:, None]], 1).astype(np.float32)))
    depth = [np.full((H, W), Z, F32)] + [np.full((H, W), Z + delta, F32)] * n_extra
    return cams, depth


@pytest.mark.parametrize("n_extra", [1, 2, 3])
def test_consistency_closed_form(n_extra):
    delta, Z, sigma = 0.01, 2.0, 0.02
    cams_in, depth = _stereo_plane(n_extra, delta)
    cams = [O.camera_f32(c) for c in cams_in]
    x, y = 150, 70                                # visible in every shifted view
    p = np.stack(O.backproject(cams[0], [x], [y], [Z]), 1)
    P = O.Params(sigma=sigma, k_views=n_extra + 1)
    views, px, py = O.select_views(np.array([0]), p, cams, P.k_views)
    assert sorted(views[0].tolist()) == list(range(1, n_extra + 1))
    assert all(px[0, s] == x - 25 * views[0, s] for s in range(n_extra))
    s, m, expo = O.consistency(np.array([0]), p, views, px, py, cams, depth, P)
    # Q_j lies on camera j's ray through p at depth Z + delta: d_j = delta |p - c_j| / Z
    d2 = [(delta * np.linalg.norm(p[0].astype(np.float64) - cams[j].centre) / Z) ** 2
          for j in range(1, n_extra + 1)]
    assert m[0] == n_extra
    assert s[0] == pytest.approx(sum(d2), rel=1e-4)
    V = math.exp(-expo[0])
    assert V == pytest.approx(math.exp(-np.mean(d2) / sigma ** 2), rel=1e-4)


def test_duplicate_camera_gives_unit_consistency():
    f = make_config("c1", with_rgb=False)
    cams_in = [f.cams[0], f.cams[0]]
    depth = [f.depth[0], f.depth[0]]
    cams = [O.camera_f32(c) for c in cams_in]
    yy, xx = np.nonzero(f.depth[0] > 0)
    p = np.stack(O.backproject(cams[0], xx.astype(F32), yy.astype(F32),
                               f.depth[0][yy, xx]), 1)
    views, px, py = O.select_views(np.zeros(len(xx), np.int64), p, cams, 4)
    s, m, expo = O.consistency(np.zeros(len(xx), np.int64), p, views, px, py, cams, depth,
                               O.Params())
    assert (m == 1).all() and (s == 0).all() and (expo == 0).all()


def test_consistency_skips_missing_depth():
    delta = 0.01
    cams_in, depth = _stereo_plane(2, delta)
    depth[1] = np.zeros_like(depth[1])             # view 1 has no depth anywhere
    cams = [O.camera_f32(c) for c in cams_in]
    p = np.stack(O.backproject(cams[0], [150], [70], [2.0]), 1)
    views, px, py = O.select_views(np.array([0]), p, cams, 3)
    s, m, expo = O.consistency(np.array([0]), p, views, px, py, cams, depth, O.Params())
    assert m[0] == 1          # only view 2 contributes: the normalisation uses m, not K-1


# ---------------------------------------------------------------- P8: Eq. 10-11 fusion

def test_fusion_closed_forms():
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0], [5, 5, 5]], F32)
    conf = np.array([0.8, 0.8, 0.8, 0.7], F32)
    pts = dict(xyz=xyz, conf=conf, pix=np.arange(4))
    reps = np.array([[0, 1, 2], [3, -1, -1], [0, 1, -1]])
    expo = np.array([[0.0, 0.0, 0.0], [0.5, 0, 0], [0.0, math.log(3.0), 0]])
    out, w, _ = O.fuse_cells(reps, expo, pts, None)
    # equal weights: centroid
    assert np.allclose(out[0], [1 / 3, 2 / 3, 0], atol=1e-7)
    assert w[0] == pytest.approx(0.8, rel=1e-7)
    # a single representative returns its own point exactly and w = C V
    assert out[1].tolist() == [5, 5, 5]
    assert w[1] == pytest.approx(0.7 * math.exp(-0.5), rel=1e-7)
    # weights 0.8 and 0.8/3: x = (1/3) / (1 + 1/3) = 0.25
    assert out[2][0] == pytest.approx(0.25, rel=1e-7)
    assert w[2] == pytest.approx((0.8 + 0.8 / 3) / 2, rel=1e-7)


def test_fusion_colour_closed_forms():
    """Eq. 11 applied to colour: rint of the same normalised weights pi_r = w_r / sum w,
    w_r = C_r V_r (Eq. 10), clamped to [0, 255].  Each case is worked by hand, and chosen so
    that a plausible slip gives another value: raw weights w instead of pi, confidence
    without V, truncation instead of rounding, or rounding half away from zero."""
    n = 12
    xyz = np.zeros((n, 3), F32)
    conf = np.array([0.8, 0.4, 0.8, 0.8, 0.9, 0.6, 0.3, 0.5, 0.5, 0.5, 0.5, 0.7], F32)
    rgb = np.array([[30, 0, 101], [60, 255, 100],        # cell 0: pi = 2/3, 1/3
                    [40, 7, 200], [80, 11, 0],           # cell 1: pi = 3/4, 1/4
                    [0, 8, 200], [100, 8, 100], [255, 8, 0],   # cell 2: 1/4, 1/2, 1/4
                    [10, 11, 254], [11, 12, 255],        # cell 3: 1/2, 1/2 (ties to even)
                    [255, 255, 255], [255, 255, 255],    # cell 4: the top of the range
                    [7, 8, 9]], np.uint8)                # cell 5: one representative
    pts = dict(xyz=xyz, conf=conf, pix=np.arange(n))
    reps = np.array([[0, 1, -1], [2, 3, -1], [4, 5, 6], [7, 8, -1], [9, 10, -1],
                     [11, -1, -1]])
    ln3 = math.log(3.0)
    expo = np.array([[0, 0, 0], [0, ln3, 0], [ln3, 0, 0], [0, 0, 0], [0.25, 0.25, 0],
                     [40.0, 0, 0]], np.float64)
    _, w, col = O.fuse_cells(reps, expo, pts, rgb)
    expect = np.array([
        # 2/3 (30, 0, 101) + 1/3 (60, 255, 100) = (40, 85, 100.67) -> (40, 85, 101)
        # (raw weights 0.8, 0.4 would give 48; truncation would give 100 in blue)
        [40, 85, 101],
        # w = (0.8, 0.8/3): 3/4 (40, 7, 200) + 1/4 (80, 11, 0) = (50, 8, 150)
        # (C alone would give pi = 1/2: 60 in red)
        [50, 8, 150],
        # w = (0.3, 0.6, 0.3): (0 + 50 + 63.75, 8, 50 + 50) -> (114, 8, 100)
        [114, 8, 100],
        # halves round to even: (10.5, 11.5, 254.5) -> (10, 12, 254)
        [10, 12, 254],
        [255, 255, 255],
        [7, 8, 9]], np.uint8)
    assert (col == expect).all(), col
    assert w[0] == pytest.approx((0.8 + 0.4) / 2, rel=1e-7)
    assert w[2] == pytest.approx(0.4, rel=1e-6)
    assert w[5] == pytest.approx(0.7 * math.exp(-40.0), rel=1e-6)


def test_fusion_convexity(frame_c2):
    r = O.fuse_frame(frame_c2, debug=True)
    d = r["debug"]
    reps = d["rep_index"]
    P = d["xyz_pts"]
    valid = reps >= 0
    idx = np.where(valid, reps, 0)
    lo = np.where(valid[..., None], P[idx], np.inf).min(1)
    hi = np.where(valid[..., None], P[idx], -np.inf).max(1)
    tol = 1e-6 * np.maximum(1, np.abs(r["xyz"]))
    assert np.all(r["xyz"] >= lo - tol) and np.all(r["xyz"] <= hi + tol)
    assert np.all(r["weight"] >= 0) and np.all(r["weight"] <= 1)
    assert (r["n_members"] >= (r["reps"] != O.PAD).sum(1)).all()


# ---------------------------------------------------------------- P9: identity fusion

def test_identity_fusion_single_camera():
    rng = np.random.default_rng(1000)
    cams = ring_cameras([(320, 240)] * 2)
    prims = _scene_c1(rng, cams)
    f = make_frame(cams[:1], prims, 1000, noise=False)
    P = O.Params(level_override=6)
    r = O.fuse(f.cams, f.depth, f.conf, f.rgb, P, debug=True)
    assert r["n_members"].max() == 1                        # precondition
    d = r["debug"]
    M = d["M"]
    assert len(r["keys"]) == M
    # output multiset == gated input: map each cell back to its single pixel
    pid = r["reps"][:, 0].astype(np.int64)
    order = np.argsort(d["pix"])
    at = order[np.searchsorted(d["pix"], pid, sorter=order)]
    assert (r["xyz"] == d["xyz_pts"][at]).all()
    assert (r["weight"] == d["conf_pts"][at]).all()         # N = 1: V = 1, w = C
    rgb = f.rgb[0].reshape(-1, 3)[pid]
    assert (r["rgb"] == rgb).all()
    assert sorted(pid.tolist()) == sorted(d["pix"].tolist())


# ---------------------------------------------------------------- P10, P11

def _canon(r, cams):
    """Per-cell (key, reps as (camera-centre tuple, y, x)) — independent of camera order."""
    off = np.cumsum([0] + [c.width * c.height for c in cams])
    out = []
    for s in range(len(r["keys"])):
        reps = []
        for pid in r["reps"][s]:
            if pid == O.PAD:
                continue
            k = int(np.searchsorted(off, pid, side="right") - 1)
            loc = int(pid - off[k])
            reps.append((k, loc // cams[k].width, loc % cams[k].width))
        out.append((int(r["keys"][s]), reps))
    return out


def test_camera_permutation_invariance(frame_c2):
    perm = [2, 0, 3, 1]
    f = frame_c2
    a = O.fuse_frame(f)
    b = O.fuse([f.cams[i] for i in perm], [f.depth[i] for i in perm],
               [f.conf[i] for i in perm], [f.rgb[i] for i in perm])
    assert (a["keys"] == b["keys"]).all()
    assert (a["xyz"] == b["xyz"]).all() and (a["weight"] == b["weight"]).all()
    assert (a["n_members"] == b["n_members"]).all() and (a["rgb"] == b["rgb"]).all()
    ca = _canon(a, f.cams)
    cb = _canon(b, [f.cams[i] for i in perm])
    cb = [(k, [(perm[c], y, x) for c, y, x in reps]) for k, reps in cb]
    assert ca == cb


def test_oracle_deterministic(frame_c1):
    a = O.fuse_frame(frame_c1)
    b = O.fuse_frame(frame_c1)
    for k in a:
        if a[k] is not None:
            assert np.array_equal(a[k], b[k])


# ---------------------------------------------------------------- ablations and edges

def test_ablation_flags(frame_c1):
    full = O.fuse_frame(frame_c1, debug=True)
    no_dc = O.fuse_frame(frame_c1, O.Params(flags=O.FF_NO_DC))
    assert (no_dc["keys"] == full["keys"]).all()
    # without DC every weight is the mean confidence of the representatives
    d = full["debug"]
    reps = d["rep_index"]
    C = np.where(reps >= 0, d["conf_pts"][np.where(reps >= 0, reps, 0)], 0).astype(np.float64)
    assert np.allclose(no_dc["weight"], C.sum(1) / (reps >= 0).sum(1), rtol=1e-6)
    no_mf = O.fuse_frame(frame_c1, O.Params(flags=O.FF_NO_MF | O.FF_NO_DC))
    assert (no_mf["weight"] == 1).all()
    no_sa = O.fuse_frame(frame_c1, O.Params(flags=O.FF_NO_SA))
    assert len(no_sa["keys"]) == d["M"]
    assert (no_sa["xyz"] == d["xyz_pts"]).all()


def test_empty_and_degenerate_frames():
    cam = make_camera(16, 8, np.array([0.0, -3, 0]), np.zeros(3))
    D = np.zeros((8, 16), F32)
    C = np.ones((8, 16), F32)
    r = O.fuse([cam], [D], [C])
    assert len(r["keys"]) == 0 and r["member_offsets"].tolist() == [0]
    # a single valid pixel: one cell, its own point, weight C
    D[3, 5] = 2.0
    C[3, 5] = 0.75
    r = O.fuse([cam], [D], [C], debug=True)
    assert len(r["keys"]) == 1 and r["weight"][0] == F32(0.75)
    assert r["debug"]["e"] == O.E_MIN and r["reps"][0].tolist() == [3 * 16 + 5, O.PAD, O.PAD]


def _bad_cameras(cam):
    """Cameras the library rejects: non-finite parameters, and (its own limits) focal
    lengths outside [2^-20, 2^20] px and a principal point beyond +-16384 px."""
    import dataclasses
    T = cam.world_to_cam.copy()
    T[1, 3] = np.inf
    return [dataclasses.replace(cam, fx=0.0), dataclasses.replace(cam, fy=2.0 ** -21),
            dataclasses.replace(cam, fx=2.0 ** 21), dataclasses.replace(cam, fx=np.nan),
            dataclasses.replace(cam, cx=16385.0), dataclasses.replace(cam, cy=-np.inf),
            dataclasses.replace(cam, world_to_cam=T)]


def test_camera_validation():
    """The oracle rejects only what the method cannot use: non-finite parameters and empty
    images.  Focal lengths and principal points of any finite value are accepted."""
    import dataclasses
    cam = make_camera(4, 4, np.array([0.0, -3, 0]), np.zeros(3))
    D = [np.ones((4, 4), F32)]
    C = [np.ones((4, 4), F32)]
    T = cam.world_to_cam.copy()
    T[1, 3] = np.inf
    for bad in (dataclasses.replace(cam, fx=np.nan), dataclasses.replace(cam, cy=-np.inf),
                dataclasses.replace(cam, world_to_cam=T)):
        with pytest.raises(ValueError):
            O.fuse([bad], D, C)
    for bad in (dataclasses.replace(cam, width=0), dataclasses.replace(cam, height=-1)):
        with pytest.raises(ValueError):
            O.validate_camera(bad)
    # finite parameters far outside any implementation range are the method's business
    for ok in (dataclasses.replace(cam, fx=2.0 ** 30, fy=-(2.0 ** -30), cx=1e6, cy=-1e6),
               dataclasses.replace(cam, fx=0.0)):
        r = O.fuse([ok], D, C)
        assert r["weight"].dtype == np.float32
    # a zero focal length sends every ray to (x - cx)/0, infinite or (at x = cx) 0/0:
    # no point is finite, so all are dropped
    z = dataclasses.replace(cam, fx=0.0, cx=2.0, cy=2.0)
    r = O.fuse([z], D, C, debug=True)
    assert r["debug"]["M"] == 0 and len(r["keys"]) == 0


def test_parameter_validation():
    cam = make_camera(4, 4, np.array([0.0, -3, 0]), np.zeros(3))
    D = [np.ones((4, 4), F32)]
    C = [np.ones((4, 4), F32)]
    for bad in (O.Params(coarse_res=48), O.Params(max_level=13), O.Params(level_override=7),
                O.Params(sigma=0.0), O.Params(k_views=0)):
        with pytest.raises(ValueError):
            O.fuse([cam], D, C, params=bad)


@pytest.mark.parametrize("target,max_level", [(16, 6), (1, 6), (4, 3), (64, 6), (16, 0), (3, 5)])
def test_dense_key_range_bound(target, max_level):
    """The sort is planned for at most ceil(log2 T) key bits with T, the dense key range
    (sum over occupied coarse cells of 8^L), bounded by M max(1, ceil(2^(Lmax+2) / target)):
    a cell refined to L >= 1 holds more than target 4^(L-1) points.  Checked on random and
    on worst-case count vectors through the oracle's level rule."""
    p = O.Params(target_per_cell=target, max_level=max_level)
    per = max(1, -(-(2 ** (max_level + 2)) // target))
    rng = np.random.default_rng(target * 7 + max_level)
    worst = [target * 4 ** (L - 1) + 1 for L in range(1, max_level + 1)]
    cases = [rng.integers(0, 5000, 4096), rng.integers(0, 50, 4096),
             np.array(worst + [1, 1, 0], np.int64), np.array([worst[-1]] * 5 if worst else [1])]
    for counts in cases:
        counts = np.asarray(counts, np.int64)
        L = O.levels(counts, p)
        T = int(np.sum(np.where(counts > 0, 8 ** L, 0)))
        M = int(counts.sum())
        assert T <= M * per, (counts[:8], T, M * per)
