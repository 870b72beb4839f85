"""GPU parity of the Eq. 3 confidence (bit-exact: it feeds the gate and the ranking), of the
fusion path with the confidence computed on the device (FF_CONF_EQ3), and of the E_MC
evaluator (Eq. 12), each against the CPU oracle."""
import numpy as np
import pytest

from oracle import core as O
from oracle import measures as M
from synth.scenes import make_camera
from tests.conftest import cached_frame
from tests.gpu_helpers import compare, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2602_01035_amd as ff
    return ff


@pytest.fixture(scope="module")
def ctx(ff):
    c = ff.Context(max_pixels=4_000_000, max_cameras=16, max_frames=4)
    yield c
    c.close()


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_confidence_maps_bit_exact(ff, name):
    print(f"[case] Eq. 3 maps {name}", flush=True)
    f = cached_frame(name)
    dev = ff.to_device(f)
    out = ff.confidence(dev["cams"], dev["depth"])
    for k, D in enumerate(f.depth):
        g = out[k].cpu().numpy()
        o = M.confidence_eq3(D)
        assert np.array_equal(g, o), (k, np.abs(g - o).max(), int((g != o).sum()))


def test_confidence_edge_cases(ff):
    import torch
    print("[case] Eq. 3 edge cases", flush=True)
    rng = np.random.default_rng(3)
    cases = [np.full((1, 1), 2.0), np.zeros((3, 4)), (1 + rng.random((1, 37))),
             (1 + rng.random((29, 1))), (1 + 5 * rng.random((17, 23)))]
    special = (1 + rng.random((9, 11)))
    special[2, 3] = np.nan
    special[4, :] = np.inf
    special[6, 6] = -2.0
    special[0, 0] = 3e38
    cases.append(special)
    for D in cases:
        D = D.astype(np.float32)
        H, W = D.shape
        cam = make_camera(W, H, np.array([0.0, -3.0, 0.0]), np.zeros(3))
        d = torch.from_numpy(D).cuda()
        for kw in ({}, dict(alpha=0.2, beta=3.0, gamma=0.7, delta=10.0)):
            g = ff.confidence([cam], [d], **kw)[0].cpu().numpy()
            assert np.array_equal(g, M.confidence_eq3(D, **kw)), (D.shape, kw)


@pytest.mark.parametrize("name,batch", [("c1", False), ("c2", False), ("c2", True)])
def test_fusion_with_device_confidence(ctx, ff, name, batch):
    print(f"[case] fusion with Eq. 3 confidence {name} batch={batch}", flush=True)
    f = cached_frame(name)
    dev = ff.to_device(f)
    p = ff.Params(flags=ff.FF_CONF_EQ3)
    if batch:
        g = ctx.fuse_batch([dict(cams=dev["cams"], depth=dev["depth"], rgb=dev["rgb"])],
                           params=p, members=True)[0].result()
    else:
        g = ctx.fuse(dev["cams"], dev["depth"], None, dev["rgb"], params=p,
                     members=True).result()
    compare(g, O.fuse_frame(f, oracle_params(p)), label=f"{name} eq3")


@pytest.mark.parametrize("name,stride", [("c1", 1), ("c2", 1), ("c2", 3)])
def test_emc_matches_oracle(ctx, ff, name, stride):
    print(f"[case] E_MC {name} stride {stride}", flush=True)
    f = cached_frame(name)
    dev = ff.to_device(f)
    out = ctx.fuse(dev["cams"], dev["depth"], dev["conf"], dev["rgb"])
    r = ctx.emc(dev["cams"], dev["depth"], out, stride=stride)
    xyz = out.result()["xyz"]
    o = M.emc(f.cams, f.depth, xyz, stride=stride)
    assert r["points"] == o["points"] > 0
    assert abs(r["emc_m"] - o["emc_m"]) <= 1e-12 + 1e-9 * o["emc_m"]
    assert abs(r["mean_visible"] - o["mean_visible"]) <= 1e-9 * o["mean_visible"]
    assert 0 < r["emc_m"] < 1.0


def test_emc_orders_the_ablations(ctx, ff):
    """Method sanity, not parity: on the scene with outliers (c2) the full method is the
    most consistent with the views, and dropping the distance consistency hurts most, in
    the order of Table II (E_MC: full < no MF < no DC < neither)."""
    print("[case] E_MC of the ablations on c2", flush=True)
    f = cached_frame("c2")
    dev = ff.to_device(f)
    e = {}
    for flags in (0, ff.FF_NO_MF, ff.FF_NO_DC, ff.FF_NO_MF | ff.FF_NO_DC):
        out = ctx.fuse(dev["cams"], dev["depth"], dev["conf"], params=ff.Params(flags=flags))
        e[flags] = ctx.emc(dev["cams"], dev["depth"], out)["emc_m"]
    assert e[0] < e[ff.FF_NO_MF] < e[ff.FF_NO_DC] < e[ff.FF_NO_MF | ff.FF_NO_DC], e


def test_emc_planted_offset(ctx, ff):
    import torch
    print("[case] E_MC planted offset", flush=True)
    W, H, Z0, delta = 64, 48, 3.0, 0.02
    cam = make_camera(W, H, np.array([0.0, -Z0, 0.0]), np.zeros(3))
    D = torch.full((H, W), Z0, dtype=torch.float32, device="cuda")
    cf = O.camera_f32(cam)
    yy, xx = np.mgrid[0:H, 0:W]
    P = np.stack(O.backproject(cf, xx.ravel(), yy.ravel(),
                               np.full(W * H, Z0 - delta, np.float32)), 1).astype(np.float32)
    out = ff.Output(W * H)
    out.xyz.copy_(torch.from_numpy(P))
    out.count.fill_(W * H)
    r = ctx.emc([cam], [D], out)
    assert r["points"] == W * H and abs(r["emc_m"] - delta) < 1e-5 and r["mean_visible"] == 1.0
    out.count.fill_(10)                      # only the first 10 points
    assert ctx.emc([cam], [D], out)["points"] == 10


def test_bad_arguments(ctx, ff):
    import torch
    f = cached_frame("c1")
    dev = ff.to_device(f)
    out = ctx.fuse(dev["cams"], dev["depth"], dev["conf"])
    with pytest.raises(ff.FuseFlowError):
        ctx.emc(dev["cams"], dev["depth"], out, stride=0)
    with pytest.raises(ff.FuseFlowError):
        ctx.emc(dev["cams"], dev["depth"], out, c_occ=-1.0)
    with pytest.raises(ff.FuseFlowError):
        ff.confidence(dev["cams"], dev["depth"], alpha=float("nan"))
    with pytest.raises(ff.FuseFlowError):       # without FF_CONF_EQ3 the confidence is needed
        ctx.fuse(dev["cams"], dev["depth"], None)


def test_server_with_device_confidence(ff):
    """Frames without a confidence map, served with FF_CONF_EQ3, equal the plain call."""
    print("[case] server with Eq. 3 confidence", flush=True)
    f = cached_frame("c1")
    dev = ff.to_device(f)
    frame = dict(cams=dev["cams"], depth=dev["depth"], rgb=dev["rgb"])
    p = ff.Params(flags=ff.FF_CONF_EQ3)
    ctx = ff.Context(max_pixels=f.pixels, max_cameras=4)
    a = ctx.fuse(dev["cams"], dev["depth"], None, dev["rgb"], params=p).result()
    ctx.close()
    srv = ff.Server(hbm_budget_bytes=1 << 30, lanes=2, max_batch_frames=2)
    outs = [ff.Output(f.pixels, rgb=True) for _ in range(3)]
    for o in outs:
        srv.submit(0, frame, o, params=p)
    srv.drain()
    srv.close()
    for o in outs:
        g = o.result()
        for k in ("keys", "xyz", "weight", "reps", "n_members", "rgb"):
            assert np.array_equal(g[k], a[k]), k
