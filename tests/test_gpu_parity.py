"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by element.

Bit-exact: point counts, cell keys, membership, representative ids.  Within 1e-5
(relative): fused coordinates and weights.  Every case prints its name before the GPU step.
"""
import dataclasses

import numpy as np
import pytest

from oracle import core as O
from synth import make_config, make_frame, ring_cameras
from synth.scenes import Camera, Primitive, make_camera, _scene_c1, _scene_c2
from tests.conftest import cached_frame
from tests.gpu_helpers import compare, oracle_params, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2602_01035_amd as ff
    return ff


@pytest.fixture(scope="module")
def ctx(ff):
    c = ff.Context(max_pixels=16_000_000, max_cameras=64, max_frames=8)
    yield c
    c.close()


def _case(ctx, ff, frame, label, params=None, with_rgb=True, batch=False):
    print(f"[case] {label}", flush=True)
    p = params or ff.Params()
    g = run_gpu(ctx, frame, p, with_rgb=with_rgb, batch=batch)
    o = O.fuse_frame(frame, oracle_params(p), with_rgb=with_rgb)
    compare(g, o, label=label)
    return g, o


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_configs_full(ctx, ff, name):
    _case(ctx, ff, cached_frame(name), name)


def test_c3_full(ctx, ff):
    g, o = _case(ctx, ff, cached_frame("c3"), "c3")
    assert g["info"][0] == len(o["member_ids"])          # M
    assert g["info"][2] == (o["reps"] != O.PAD).sum()    # R


@pytest.mark.parametrize("flags", [1, 2, 3, 4, 5])
def test_ablation_flags(ctx, ff, flags):
    _case(ctx, ff, cached_frame("c1"), f"c1 flags={flags}", ff.Params(flags=flags))


@pytest.mark.parametrize("kw", [dict(k_views=1), dict(k_views=2), dict(k_views=8),
                                dict(level_override=0), dict(level_override=6),
                                dict(coarse_res=16), dict(coarse_res=128, max_level=4),
                                dict(target_per_cell=1), dict(sigma=0.5, tau=0.8),
                                dict(sigma=1e-4),      # weights underflow: log-domain mean
                                dict(coarse_res=1, max_level=10)])
def test_parameter_variants(ctx, ff, kw):
    _case(ctx, ff, cached_frame("c2"), f"c2 {kw}", ff.Params(**kw))


@pytest.mark.parametrize("seed", range(4))
def test_random_small_rigs(ctx, ff, seed):
    """Ragged sizes (not multiples of 4 or of the 4096-pixel tile), odd camera counts."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 6))
    res = [(int(rng.integers(3, 300)), int(rng.integers(2, 200))) for _ in range(n)]
    cams = ring_cameras(res, jitter_pos=0.2, jitter_target=0.3, rng=rng)
    prims = _scene_c2(rng, cams)
    f = make_frame(cams, prims, 9000 + seed, outlier_frac=0.05, conf_model="beta")
    _case(ctx, ff, f, f"random rig {seed} {res}")


def _admissible_extremes_frame(seed):
    """A small rig with half of its cameras given intrinsics drawn across the whole range
    the boundary admits (|f| log-uniform in [2^-20, 2^20], either sign, principal point off
    the image), and random blocks of subnormal, tiny or far depths."""
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(2, 6))
    res = [(int(rng.integers(1, 300)), int(rng.integers(1, 300))) for _ in range(n)]
    base = ring_cameras(res, radius=float(rng.uniform(1.5, 4.0)), jitter_pos=0.4,
                        jitter_target=0.5, rng=rng)
    cams = []
    for (w, h), b in zip(res, base):
        if rng.random() < 0.5:
            e = rng.uniform(-20, 20)
            fx = float(2.0 ** e) * (1 if rng.random() < 0.8 else -1)
            fy = float(2.0 ** float(np.clip(e + rng.uniform(-2, 2), -20, 20)))
            cx = float(np.clip(rng.uniform(-2 * w, 3 * w), -16384, 16384))
            cy = float(np.clip(rng.uniform(-2 * h, 3 * h), -16384, 16384))
            cams.append(Camera(w, h, fx, fy, cx, cy, b.world_to_cam))
        else:
            cams.append(b)
    prims = _scene_c2(rng, base)
    fr = make_frame(cams, prims, 7000 + seed, outlier_frac=0.03, conf_model="beta")
    D = [d.copy() for d in fr.depth]
    C = [c.copy() for c in fr.conf]
    for d, c in zip(D, C):
        for _ in range(int(rng.integers(0, 3))):
            H, W = d.shape
            y0, x0 = int(rng.integers(0, H)), int(rng.integers(0, W))
            d[y0:y0 + 3, x0:x0 + 5] = np.float32(rng.choice([1e-39, 1.4e-45, 3e-30, 40.0]))
            c[y0:y0 + 3, x0:x0 + 5] = np.float32(rng.uniform(0.61, 1.0))
    return dataclasses.replace(fr, depth=D, conf=C)


@pytest.mark.parametrize("seed", range(64))
def test_admissible_extremes(ctx, ff, seed):
    f = _admissible_extremes_frame(seed)
    desc = [(c.width, c.height, f"{c.fx:.3g}") for c in f.cams]
    for prm in (ff.Params(), ff.Params(level_override=6)):
        _case(ctx, ff, f, f"admissible extremes {seed} {desc}", prm)


@pytest.mark.parametrize("first", [0, 8, 16, 24])
def test_admissible_extremes_batched(ctx, ff, first):
    """Eight of those rigs in one batched call: frames of very different extents, levels
    and camera counts share every launch, and each must equal its own oracle result."""
    frames = [_admissible_extremes_frame(seed) for seed in range(first, first + 8)]
    print(f"[case] admissible extremes batched {first}..{first + 7}", flush=True)
    outs = ctx.fuse_batch([ff.to_device(f) for f in frames], members=True)
    for k, (f, out) in enumerate(zip(frames, outs)):
        compare(out.result(), O.fuse_frame(f), label=f"batched extremes frame {first + k}")


def _random_params(ff, seed):
    """Parameters drawn across the ranges the library admits (coarse_res a power of two up
    to 128 and K up to 8, as its header states; level limits, target count, sigma, tau and
    ablation flags over the method's ranges)."""
    rng = np.random.default_rng(6000 + seed)
    lg = int(rng.integers(0, 8))                          # coarse_res 1 .. 128
    lmax = int(rng.integers(0, min(16, 56 // 3 - lg) + 1))
    lo = -1 if rng.random() < 0.7 else int(rng.integers(0, lmax + 1))
    flags = int(rng.choice([0, 0, 0, 1, 2, 3, 4]))
    return ff.Params(coarse_res=1 << lg, max_level=lmax, level_override=lo,
                     target_per_cell=int(rng.integers(1, 65)), k_views=int(rng.integers(1, 9)),
                     sigma=float(10.0 ** rng.uniform(-4, 0)), tau=float(rng.uniform(0.0, 0.95)),
                     flags=flags)


@pytest.mark.parametrize("seed", range(24))
def test_random_parameters(ctx, ff, seed):
    f = cached_frame("c1")
    p = _random_params(ff, seed)
    label = (f"random parameters {seed}: G {p.coarse_res} Lmax {p.max_level} "
             f"override {p.level_override} target {p.target_per_cell} K {p.k_views} "
             f"flags {p.flags}")
    _case(ctx, ff, f, label, p)
    _case(ctx, ff, f, label + " batched", p, batch=True)


@pytest.mark.parametrize("seed", range(16))
def test_admissible_extremes_random_parameters(ctx, ff, seed):
    """The extreme-intrinsics rigs under random parameter sets."""
    f = _admissible_extremes_frame(100 + seed)
    p = _random_params(ff, 100 + seed)
    _case(ctx, ff, f, f"extremes {100 + seed} with random parameters {100 + seed}", p)


@pytest.mark.parametrize("n_cams,res", [(9, (160, 120)), (12, (128, 96)), (20, (96, 64))])
def test_frames_with_many_cameras(ctx, ff, n_cams, res):
    """More than 8 cameras in a frame: every camera is tested for the local views."""
    rng = np.random.default_rng(300 + n_cams)
    cams = ring_cameras([res] * n_cams, jitter_pos=0.3, jitter_target=0.2, rng=rng)
    prims = _scene_c2(rng, cams)
    f = make_frame(cams, prims, 9100 + n_cams, outlier_frac=0.03, conf_model="beta")
    _case(ctx, ff, f, f"{n_cams} cameras {res}", ff.Params(k_views=6))
    _case(ctx, ff, f, f"{n_cams} cameras {res} batched", ff.Params(k_views=6), batch=True)


def test_empty_and_single_pixel(ctx, ff):
    cam = make_camera(37, 5, np.array([0.0, -3, 0]), np.zeros(3))
    D = np.zeros((5, 37), np.float32)
    C = np.ones((5, 37), np.float32)

    class Fr:
        cams, depth, conf, rgb = [cam], [D], [C], None
    g, o = _case(ctx, ff, Fr, "empty frame", with_rgb=False)
    assert g["count"] == 0
    D[2, 11] = 2.0
    C[2, 11] = 0.75
    g, o = _case(ctx, ff, Fr, "single pixel", with_rgb=False)
    assert g["count"] == 1 and g["weight"][0] == np.float32(0.75)


def test_batch_with_empty_frames(ctx, ff):
    """Frames without a single gated point between others in one batched call: every
    frame's compacted positions start after the points of the frames before it."""
    import synth
    cam = make_camera(37, 5, np.array([0.0, -3, 0]), np.zeros(3))
    empty = synth.Frame([cam], [np.zeros((5, 37), np.float32)], [np.ones((5, 37), np.float32)],
                        None, None, None, None, [])
    D1 = np.zeros((5, 37), np.float32)
    C1 = np.ones((5, 37), np.float32)
    D1[2, 11] = 2.0
    C1[2, 11] = 0.75
    single = synth.Frame([cam], [D1], [C1], None, None, None, None, [])
    frames = [empty, cached_frame("c1"), empty, single, cached_frame("c1", frame=1), empty]
    print("[case] batch of 6 with empty frames", flush=True)
    devs = [ff.to_device(f, with_rgb=False) for f in frames]
    outs = ctx.fuse_batch(devs, members=True)
    for i, (f, out) in enumerate(zip(frames, outs)):
        g = out.result()
        compare(g, O.fuse_frame(f, with_rgb=False), label=f"frame {i}")
    assert outs[0].result()["count"] == 0 and outs[3].result()["count"] == 1


def test_nonfinite_inputs(ctx, ff):
    f = make_config("c1")
    D = [d.copy() for d in f.depth]
    C = [c.copy() for c in f.conf]
    D[0][10, :50] = np.nan
    D[0][11, :50] = np.inf
    D[0][12, :50] = -1.0
    C[1][20, :] = np.nan
    C[1][21, :] = np.float32(0.6)          # exactly tau: excluded
    D[1][22, :3] = np.float32(3e38)        # finite depth, far point

    class Fr:
        cams, depth, conf, rgb = f.cams, D, C, f.rgb
    _case(ctx, ff, Fr, "non-finite inputs")


def test_identity_fusion(ctx, ff):
    rng = np.random.default_rng(1000)
    cams = ring_cameras([(320, 240)] * 2)
    prims = _scene_c1(rng, cams)
    f = make_frame(cams[:1], prims, 1000, noise=False)
    g, o = _case(ctx, ff, f, "identity", ff.Params(level_override=6))
    assert g["n_members"].max() == 1


def _border_band_pairs(frame, margin=0.0625):
    """(point, other camera) pairs whose u + 1/2 or v + 1/2 lies within `margin` px of that
    camera's image border, in the oracle's float32 arithmetic: the cases the field-of-view
    test must settle with the exact quotients."""
    cams = [O.camera_f32(c) for c in frame.cams]
    pts = O.generate_points(cams, frame.depth, frame.conf, O.Params())
    F = np.float32
    n = 0
    for j, cm in enumerate(cams):
        p = pts["xyz"][pts["cam"] != j]
        X = [((cm.R[a, 0] * p[:, 0] + cm.R[a, 1] * p[:, 1]) + cm.R[a, 2] * p[:, 2]) + cm.t[a]
             for a in range(3)]
        with np.errstate(all="ignore"):
            u = cm.fx * (X[0] / X[2]) + cm.cx + F(0.5)
            v = cm.fy * (X[1] / X[2]) + cm.cy + F(0.5)
        W, H = F(cm.width), F(cm.height)
        near_u = (np.abs(u) < margin) | (np.abs(u - W) < margin)
        near_v = (np.abs(v) < margin) | (np.abs(v - H) < margin)
        in_u = (u > -margin) & (u < W + margin)
        in_v = (v > -margin) & (v < H + margin)
        n += int(((X[2] > 0) & ((near_u & in_v) | (near_v & in_u))).sum())
    return n


def test_field_of_view_border_band(ctx, ff):
    """A fine camera over a plane and two coarse cameras that each see part of it: the fine
    camera's points fall densely across the coarse cameras' image borders, so hundreds of
    representatives lie within 1/16 px of a border (Eq. 4 visibility decided by the exact
    quotients), and with K - 1 = 2 both other cameras are kept whenever visible, so every
    such decision changes V."""
    A = make_camera(160, 120, np.array([0.0, -1.0, 2.0]), np.array([0.0, 0.3, 0.0]))
    B = make_camera(40, 30, np.array([0.45, -1.2, 2.6]), np.array([0.55, 0.5, 0.0]))
    C = make_camera(40, 30, np.array([-0.4, -0.8, 2.4]), np.array([-0.5, 0.1, 0.0]))
    plane = Primitive("plane", np.zeros(3), np.array([0.0, 5.0]), np.array([0.5, 0.5, 0.5]))
    f = make_frame([A, B, C], [plane], 4242)
    assert _border_band_pairs(f) >= 150
    # level 6 everywhere: nearly every point is its own cell's representative
    g, o = _case(ctx, ff, f, "field-of-view border band", ff.Params(level_override=6))
    assert (o["reps"] != O.PAD).sum() > 0.9 * len(o["member_ids"])


def test_cameras_at_the_range_limits(ctx, ff):
    """Cameras at the limits the boundary admits: a 16384 x 1 strip, a 1 x 4000 strip,
    |f| = 2^20 with the principal point at -16000 (a sliver of view, u far from the
    principal point) and |f| = 2^-20 (a near-hemispherical view), beside an ordinary
    camera.  Tiles, pixel coordinates and the field-of-view fast path at its error bound
    must all agree with the oracle."""
    def strip(base, w, h, fx, cx, cy):
        return Camera(w, h, float(fx), float(fx), float(cx), float(cy), base.world_to_cam)

    c0 = make_camera(320, 240, np.array([0.0, -3.0, 0.6]), np.array([0.0, 0.0, 0.0]))
    b1 = make_camera(8, 8, np.array([2.5, -1.5, 0.4]), np.array([0.1, 0.1, 0.0]))
    b2 = make_camera(8, 8, np.array([-2.2, -1.8, 0.8]), np.array([-0.1, 0.2, 0.1]))
    b3 = make_camera(8, 8, np.array([0.3, 2.8, 0.5]), np.array([0.0, -0.1, 0.0]))
    b4 = make_camera(8, 8, np.array([-2.0, 2.0, 1.2]), np.array([0.0, 0.0, -0.2]))
    cams = [c0, strip(b1, 16384, 1, 4000.0, 8192.0, 0.5), strip(b2, 1, 4000, 300.0, 0.5, 2000.0),
            strip(b3, 64, 48, 2.0 ** 20, -16000.0, 24.0), strip(b4, 40, 30, 2.0 ** -20, 20.0, 15.0)]
    rng = np.random.default_rng(5)
    prims = [Primitive("plane", np.zeros(3), np.array([-1.0, 8.0]), np.array([0.5, 0.5, 0.5]))]
    for c, r in (([0.3, 0.2, -0.4], 0.5), ([-0.5, 0.6, 0.1], 0.35), ([0.6, -0.4, 0.3], 0.3)):
        prims.append(Primitive("sphere", np.array(c), np.array([r]), rng.uniform(0.2, 1, 3)))
    f = make_frame(cams, prims, 31)
    pts = O.generate_points([O.camera_f32(c) for c in f.cams], f.depth, f.conf, O.Params())
    assert np.all(np.bincount(pts["cam"], minlength=len(cams)) > 100)   # every camera counts
    for prm in (ff.Params(), ff.Params(level_override=6), ff.Params(k_views=5)):
        _case(ctx, ff, f, "cameras at the range limits", prm)


@pytest.mark.parametrize("kind", ["subnormal", "huge"])
def test_extreme_depths(ctx, ff, kind):
    """Two cameras at the world origin (t = 0 exactly) and a third elsewhere.  "subnormal":
    blocks of subnormal depths (down to the smallest one) give points within 1e-38 of the
    origin, equal in confidence, so their cell is ranked on subnormal positions, and their
    camera-frame Z in the other origin camera is subnormal (the approximate reciprocal is
    infinite and the exact quotients decide).  "huge": depths of 1e30 give points near
    1e30 (the coarse exponent clamps) and 3e38 overflows when back-projected (gated out)."""
    A = make_camera(160, 120, np.array([0.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.1]))
    B = make_camera(160, 120, np.array([0.0, 0.0, 0.0]), np.array([0.4, 1.0, 0.0]))
    C = make_camera(160, 120, np.array([0.0, -1.5, 0.4]), np.array([0.0, 1.0, 0.0]))
    rng = np.random.default_rng(8)
    prims = [Primitive("plane", np.zeros(3), np.array([-1.0, 8.0]), np.array([0.5, 0.5, 0.5]))]
    for c, r in (([0.0, 2.0, 0.0], 0.5), ([0.6, 2.5, 0.3], 0.4), ([-0.5, 1.8, -0.2], 0.3)):
        prims.append(Primitive("sphere", np.array(c), np.array([r]), rng.uniform(0.2, 1, 3)))
    f = make_frame([A, B, C], prims, 12)
    d0, c0 = f.depth[0].copy(), f.conf[0].copy()
    d1, c1 = f.depth[1].copy(), f.conf[1].copy()
    if kind == "subnormal":
        sub = np.float32(1e-39) * np.arange(1, 11, dtype=np.float32)
        d0[40:50, 60:100] = np.resize(sub, (10, 40))
        c0[40:50, 60:100] = 0.9
        d1[70:75, 70:90] = np.float32(1.4e-45)
        c1[70:75, 70:90] = 0.8
    else:
        d0[60:62, 10:20] = np.float32(1e30)
        c0[60:62, 10:20] = 0.95
        d0[62, 10:20] = np.float32(3e38)
        c0[62, 10:20] = 0.95
    g = dataclasses.replace(f, depth=[d0, d1, f.depth[2]], conf=[c0, c1, f.conf[2]])
    for prm in (ff.Params(), ff.Params(level_override=6)):
        _case(ctx, ff, g, f"{kind} depths", prm)


def test_exact_distance_ties_between_views(ctx, ff):
    """Two cameras mirrored in x about a centre camera whose middle column back-projects to
    x = 0 exactly: those points are at exactly the same squared distance from both mirrored
    centres (152 of them visible in both).  With K = 2 one view is kept, so the camera
    rank (centre x first) decides which, and the scene is asymmetric, so the choice changes
    V.  Every point is its own cell."""
    A = make_camera(320, 240, np.array([0.0, -3.0, 0.5]), np.array([0.0, 0.0, 0.0]))
    B = make_camera(320, 240, np.array([1.5, -2.5, 0.5]), np.array([0.2, 0.0, 0.0]))
    C = make_camera(320, 240, np.array([-1.5, -2.5, 0.5]), np.array([-0.2, 0.0, 0.0]))
    rng = np.random.default_rng(77)
    prims = [Primitive("plane", np.zeros(3), np.array([-1.0, 6.0]), np.array([0.5, 0.5, 0.5]))]
    for c, r in (([0.35, 0.4, -0.3], 0.45), ([-0.6, 0.9, 0.2], 0.3), ([0.1, -0.5, 0.4], 0.25),
                 ([0.9, 0.2, 0.6], 0.35)):
        prims.append(Primitive("sphere", np.array(c), np.array([r]), rng.uniform(0.2, 1, 3)))
    f = make_frame([A, B, C], prims, 99)
    # the ties are there: exact equal squared distances, both mirrored cameras in view
    cams = [O.camera_f32(c) for c in f.cams]
    pts = O.generate_points(cams, f.depth, f.conf, O.Params())
    p = pts["xyz"][pts["cam"] == 0]

    def d2(c):
        return ((p[:, 0] - c[0]) ** 2 + (p[:, 1] - c[1]) ** 2) + (p[:, 2] - c[2]) ** 2

    both = O.project(cams[1], p.T)[0] & O.project(cams[2], p.T)[0]
    assert int(((d2(cams[1].centre) == d2(cams[2].centre)) & both).sum()) >= 100
    _case(ctx, ff, f, "exact distance ties", ff.Params(k_views=2, level_override=6))


def test_duplicate_cameras(ctx, ff):
    """c1 with its first camera twice (same pose, depth, confidence and colour): every point
    of that camera has an exact twin, so cells hold members equal in confidence and
    position and the full order falls through to the pixel id; the twin cameras' ranks
    tie on the centre and fall to the index; and a twin is always the nearest other view,
    where its depth reprojects the point exactly."""
    f = cached_frame("c1")
    g = dataclasses.replace(f, cams=[f.cams[0], f.cams[0], f.cams[1]],
                            depth=[f.depth[0], f.depth[0].copy(), f.depth[1]],
                            conf=[f.conf[0], f.conf[0].copy(), f.conf[1]],
                            rgb=[f.rgb[0], f.rgb[0].copy(), f.rgb[1]])
    for level in (None, 6):
        prm = ff.Params() if level is None else ff.Params(level_override=level)
        _case(ctx, ff, g, f"c1 with a duplicated camera, level {level}", prm)


@pytest.mark.parametrize("steps", [16, 1024])
def test_quantised_confidences(ctx, ff, steps):
    """Confidences rounded to multiples of 1/steps: equal confidences among a cell's best
    three are common (about 81,000 cells of c2 at 1/16, 2,300 at 1/1024), so the ranking
    must fall back to the full order (position, then pixel id) both in the three-member
    path and in the four-lanes-per-cell path, and the tie must be detected per member."""
    f = cached_frame("c2")
    conf = [(np.round(c.astype(np.float64) * steps) / steps).astype(np.float32) for c in f.conf]
    g, o = _case(ctx, ff, dataclasses.replace(f, conf=conf), f"c2 confidences in 1/{steps}")
    # the ties are really there
    call = np.concatenate([c.ravel() for c in conf])
    mo, mi = o["member_offsets"], o["member_ids"]
    n = np.diff(mo)
    tied = 0
    for s in np.flatnonzero(n >= 2):
        cs = np.sort(call[mi[mo[s]:mo[s + 1]]])[::-1]
        k = min(3, len(cs))
        if len(np.unique(cs[:k])) < k or (len(cs) > k and cs[k] == cs[k - 1]):
            tied += 1
    assert tied >= (50_000 if steps == 16 else 1_000), tied


def test_batch_equals_single(ctx, ff):
    frames = [cached_frame("c1"), cached_frame("c2"), cached_frame("c1", frame=1)]
    print("[case] batch of c1, c2, c1/1", flush=True)
    devs = [ff.to_device(f) for f in frames]
    outs = ctx.fuse_batch(devs, members=True)
    for f, out in zip(frames, outs):
        g = out.result()
        o = O.fuse_frame(f)
        compare(g, o, label="batched")
        s = run_gpu(ctx, f)
        for k in ("keys", "xyz", "weight", "reps", "n_members", "rgb", "member_ids"):
            assert np.array_equal(g[k], s[k]), k


@pytest.mark.skip(reason="the single persistent launch that runs every phase in one kernel "
                  "did not finish on the device in two runs; it is not built until its "
                  "cause is shown on the CPU (per-phase kernels under a graph replace it)")
def test_persistent_single_launch(ctx, ff):
    raise AssertionError("not built")


def test_deterministic_repeat(ctx, ff):
    f = cached_frame("c2")
    print("[case] repeat c2 x3", flush=True)
    a = run_gpu(ctx, f)
    for _ in range(2):
        b = run_gpu(ctx, f)
        for k in ("keys", "xyz", "weight", "reps", "n_members", "rgb", "member_ids"):
            assert np.array_equal(a[k], b[k]), k


def test_capacity_overflow_reported(ctx, ff):
    import torch
    f = cached_frame("c1")
    print("[case] capacity overflow", flush=True)
    dev = ff.to_device(f)
    o = O.fuse_frame(f)
    S = len(o["keys"])
    out = ff.Output(S // 2, rgb=True)
    ctx.fuse(dev["cams"], dev["depth"], dev["conf"], dev["rgb"], out=out)
    g = out.result()
    assert g["status"] == 1 and g["count"] == S
    n = S // 2
    assert np.array_equal(g["keys"], o["keys"][:n])
    assert np.array_equal(g["reps"], o["reps"][:n])


def test_unaligned_inputs(ctx, ff):
    """Depth/confidence views that are not 16-byte aligned take the scalar load path."""
    import torch
    f = cached_frame("c1")
    print("[case] unaligned views", flush=True)
    dev = ff.to_device(f)
    D = [torch.cat([torch.zeros(1, device="cuda"), d.reshape(-1)])[1:].view_as(d) for d in dev["depth"]]
    C = [torch.cat([torch.zeros(1, device="cuda"), c.reshape(-1)])[1:].view_as(c) for c in dev["conf"]]
    assert D[0].data_ptr() % 16 != 0
    out = ctx.fuse(dev["cams"], D, C, dev["rgb"], members=True)
    compare(out.result(), O.fuse_frame(f), label="unaligned")


def test_bad_arguments_raise(ctx, ff):
    import torch
    f = cached_frame("c1")
    dev = ff.to_device(f)
    with pytest.raises(ValueError):
        ctx.fuse(dev["cams"], [d.cpu() for d in dev["depth"]], dev["conf"])
    with pytest.raises(ff.FuseFlowError):
        ctx.fuse(dev["cams"], dev["depth"], dev["conf"], params=ff.Params(coarse_res=48))
    with pytest.raises(ff.FuseFlowError):
        ctx.fuse(dev["cams"], dev["depth"], dev["conf"], params=ff.Params(k_views=9))
    with pytest.raises(ff.FuseFlowError):     # above the library's coarse grid limit (128)
        ctx.fuse(dev["cams"], dev["depth"], dev["conf"], params=ff.Params(coarse_res=256))
    small = ff.Context(max_pixels=1000, max_cameras=2)
    with pytest.raises(ff.FuseFlowError):
        small.fuse(dev["cams"], dev["depth"], dev["conf"])
    small.close()
    # cameras outside the admitted range (the oracle rejects the same ones)
    from tests.test_oracle_pins import _bad_cameras
    for bad in _bad_cameras(dev["cams"][0]):
        with pytest.raises(ff.FuseFlowError):
            ctx.fuse([bad] + dev["cams"][1:], dev["depth"], dev["conf"])


def _scattered_frame(seed, n_cams=4):
    """Cameras of 64 x 64 px (one 4,096-px tile each, 90-degree field of view) with
    independent random depths in [1, 30] m: under a 128^3 coarse grid nearly every pixel
    lands in a coarse cell of its own, about 3,900 per camera."""
    rng = np.random.default_rng(seed)
    base = ring_cameras([(64, 64)] * n_cams, radius=3.0)
    cams = [Camera(64, 64, 32.0, 32.0, 32.0, 32.0, c.world_to_cam) for c in base]
    fr = make_frame(cams, _scene_c1(rng, cams), seed)
    D = [rng.uniform(1.0, 30.0, (64, 64)).astype(np.float32) for _ in cams]
    C = [rng.uniform(0.61, 1.0, (64, 64)).astype(np.float32) for _ in cams]
    return dataclasses.replace(fr, depth=D, conf=C)


@pytest.mark.parametrize("hist_tiles", [1, 2])
def test_coarse_histogram_hash_overflow(ff, hist_tiles):
    """Sec. II.5(1)c counts with more distinct coarse cells per histogram workgroup than its
    LDS hash holds (2,048): the overflow goes straight to the global counts.  With two tiles
    per workgroup a batched workgroup also spans two frames, whose counts it flushes apart."""
    f = _scattered_frame(5, n_cams=3)          # 3 tiles per frame: pairs of tiles straddle
    p = ff.Params(coarse_res=128)
    op = oracle_params(p)
    pts = O.generate_points([O.camera_f32(c) for c in f.cams], f.depth, f.conf, op)
    lo, _ = O.extents(pts["xyz"])
    e = O.coarse_exponent(*O.extents(pts["xyz"]), op.coarse_res)
    lin = O.coarse_linear(O.coarse_cells(pts["xyz"], lo, e, op.coarse_res)[1], op.coarse_res)
    cam = pts["pix"] // (64 * 64)
    assert min(len(np.unique(lin[cam == k])) for k in range(len(f.cams))) > 2048
    print(f"[case] coarse histogram hash overflow, {hist_tiles} tiles per workgroup", flush=True)
    c = ff.Context(max_pixels=2 * 3 * 64 * 64, max_cameras=8, max_frames=2)
    c.set_tuning(hist_tiles=hist_tiles)
    d = ff.to_device(f)
    o = O.fuse_frame(f, op)
    compare(c.fuse(d["cams"], d["depth"], d["conf"], d["rgb"], params=p, members=True).result(),
            o, label=f"overflow plain {hist_tiles}")
    for k, out in enumerate(c.fuse_batch([d, d], params=p, members=True)):
        compare(out.result(), o, label=f"overflow batched frame {k}, {hist_tiles}")
    c.close()
