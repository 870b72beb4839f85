"""GPU tests of the batched path and the continuous-batching server.

Each frame's result must be identical alone (ff_fuse) and in the mix (batched with other
rigs' frames, overlapping on several streams); the oracle pins the alone result.
"""
import numpy as np
import pytest

from oracle import core as O
from tests.conftest import cached_frame
from tests.gpu_helpers import compare, oracle_params

pytestmark = pytest.mark.gpu

KEYS = ("keys", "xyz", "weight", "reps", "n_members", "rgb")


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2602_01035_amd as ff
    return ff


def _alone(ff, dev):
    ctx = ff.Context(max_pixels=4_000_000, max_cameras=16)
    r = ctx.fuse(dev["cams"], dev["depth"], dev["conf"], dev.get("rgb")).result()
    ctx.close()
    return r


def _frames():
    # three rigs with different camera counts and resolutions, two frames each
    return [cached_frame("c1", frame=f, rig=r) for r in (0, 1) for f in (0, 1)] + \
           [cached_frame("c2", frame=f) for f in (0, 1)]


@pytest.mark.parametrize("use_graph", [1, 0])
def test_batched_matches_alone_and_oracle(ff, use_graph):
    print(f"[case] batch of 6 frames, graph={use_graph}", flush=True)
    frames = _frames()
    devs = [ff.to_device(f) for f in frames]
    ctx = ff.Context(max_pixels=8_000_000, max_cameras=32, max_frames=8)
    ctx.set_tuning(use_graph=use_graph)
    for rep in range(3):                     # replays of the cached graph
        outs = ctx.fuse_batch(devs)
        for f, d, out in zip(frames, devs, outs):
            g = out.result()
            a = _alone(ff, d)
            for k in KEYS:
                assert np.array_equal(g[k], a[k]), (rep, k)
    compare(outs[0].result(), O.fuse_frame(frames[0]), label="batched vs oracle")
    ctx.close()


def test_graph_replay_follows_view_budget(ff):
    """The same batch shape with a different K must not replay a graph captured for another
    per-cell kernel variant."""
    print("[case] graph replay across k_views", flush=True)
    frames = [cached_frame("c2")]
    devs = [ff.to_device(f) for f in frames]
    ctx = ff.Context(max_pixels=2_000_000, max_cameras=8, max_frames=2)
    for k in (4, 8, 2, 4):
        p = ff.Params(k_views=k)
        g = ctx.fuse_batch(devs, params=p)[0].result()
        compare(g, O.fuse_frame(frames[0], oracle_params(p)), label=f"k_views={k}")
    ctx.close()


def test_graph_replay_follows_key_width(ff):
    """The same batch shape with level limits that change the sort's pass count and key
    width (the scatter's LDS holds 4- or 8-byte keys by the host's key-width bound) must
    not replay a graph captured for other ones.  Level 12 everywhere on one coarse cell
    needs 36-bit keys, so the 64-bit path runs too; every result against the oracle."""
    print("[case] graph replay across key widths", flush=True)
    f = cached_frame("c2")
    devs = [ff.to_device(f)]
    ctx = ff.Context(max_pixels=2_000_000, max_cameras=8, max_frames=2)
    wide = dict(coarse_res=1, max_level=12, level_override=12)
    for kw in (dict(), wide, dict(), dict(max_level=10, target_per_cell=1),
               dict(level_override=0), wide):
        p = ff.Params(**kw)
        g = ctx.fuse_batch(devs, params=p)[0].result()
        compare(g, O.fuse_frame(f, oracle_params(p)), label=f"batched {kw}")
    p = ff.Params(**wide)
    d = devs[0]
    g = ctx.fuse(d["cams"], d["depth"], d["conf"], d.get("rgb"), params=p).result()
    compare(g, O.fuse_frame(f, oracle_params(p)), check_members=False, label="plain, 36-bit keys")
    ctx.close()


@pytest.mark.parametrize("tuning", [dict(radix_bits=6, sort_items=8),
                                    dict(radix_bits=8, sort_items=16),
                                    dict(radix_bits=10, sort_items=8),
                                    dict(hist_tiles=1), dict(hist_tiles=3), dict(hist_tiles=8),
                                    dict(cell_groups=64), dict(cell_groups=777),
                                    dict(cell_groups=4096),
                                    dict(radix_bits=7, sort_items=16, hist_tiles=2,
                                         cell_groups=300, use_graph=0)])
def test_tuning_does_not_change_results(ff, tuning):
    """Every knob of the tuning changes only the launch shapes: results equal the oracle's,
    plain and batched."""
    print(f"[case] tuning {tuning}", flush=True)
    f = cached_frame("c2")
    d = ff.to_device(f)
    ctx = ff.Context(max_pixels=4_000_000, max_cameras=8, max_frames=2)
    ctx.set_tuning(**tuning)
    o = O.fuse_frame(f)
    compare(ctx.fuse_batch([d])[0].result(), o, label=f"batched {tuning}")
    compare(ctx.fuse(d["cams"], d["depth"], d["conf"], d["rgb"]).result(), o,
            check_members=False, label=f"plain {tuning}")
    outs = ctx.fuse_batch([d, d])
    for out in outs:
        compare(out.result(), o, check_members=False, label=f"batch of two {tuning}")
    ctx.close()


def test_autotune_caches_per_shape_and_persists(ff, tmp_path):
    """ff_autotune caches its choice for the batch's shape only; the cache survives a JSON
    round trip into a fresh context and ignores entries of another device; a malformed
    text is refused.  Tuned calls keep the oracle's results."""
    print("[case] autotune cache", flush=True)
    f1, f2 = cached_frame("c1"), cached_frame("c2")
    d1, d2 = ff.to_device(f1), ff.to_device(f2)
    ctx = ff.Context(max_pixels=4_000_000, max_cameras=8, max_frames=2)
    assert ctx.tuning_for([d1]) is None and ctx.tuning_for([d2]) is None
    chosen = ctx.autotune([d1])
    assert ctx.tuning_for([d1]) == chosen
    assert ctx.tuning_for([d2]) is None and ctx.tuning_for([d1, d1]) is None
    compare(ctx.fuse_batch([d1])[0].result(), O.fuse_frame(f1), label="tuned c1")
    text = ctx.export_tuning()
    assert '"entries"' in text and f1.cams[0].width.__str__() in text
    path = tmp_path / "tuning.json"
    ctx.save_tuning(str(path))
    fresh = ff.Context(max_pixels=4_000_000, max_cameras=8, max_frames=2)
    assert fresh.load_tuning(str(path)) == 1
    assert fresh.tuning_for([d1]) == chosen
    import json
    other = json.loads(text)
    other["device"] = "some other device"
    other["entries"][0]["shape"] = "1x1,;|G64|L6|f0|w0"
    assert fresh.import_tuning(json.dumps(other)) == 0
    with pytest.raises(ff.FuseFlowError):
        fresh.import_tuning('{"device": "x", "entries": [{"shape": "1x1,;", "radix_bits": 99}]}')
    compare(fresh.fuse_batch([d1])[0].result(), O.fuse_frame(f1), label="imported tuning")
    fresh.close()
    ctx.close()


def test_server_autotunes_each_new_shape(ff):
    """A server with autotuning tunes the first batch of each shape and shares the tuning
    between lanes; results stay identical to ff_fuse."""
    print("[case] server autotune", flush=True)
    frames = [cached_frame("c1"), cached_frame("c2")]
    devs = [ff.to_device(f) for f in frames]
    alone = [_alone(ff, d) for d in devs]
    srv = ff.Server(hbm_budget_bytes=2 << 30, lanes=2, max_batch_frames=1, autotune=True)
    outs = []
    for rep in range(3):
        for i, d in enumerate(devs):
            out = ff.Output(sum(c.width * c.height for c in d["cams"]), rgb=True)
            srv.submit(i, d, out)
            outs.append((i, out))
    srv.drain()
    for i, out in outs:
        g = out.result()
        for k in KEYS:
            assert np.array_equal(g[k], alone[i][k]), (i, k)
    srv.close()


@pytest.mark.parametrize("plain", [False, True])
def test_server_results_same_alone_and_in_mix(ff, plain):
    print(f"[case] server plain={plain}", flush=True)
    frames = _frames()
    devs = [ff.to_device(f) for f in frames]
    alone = [_alone(ff, d) for d in devs]
    srv = ff.Server(hbm_budget_bytes=2 << 30, lanes=2, max_batch_frames=4, plain=plain)
    tickets, outs = [], []
    for rep in range(2):
        for i, d in enumerate(devs):
            out = ff.Output(sum(c.width * c.height for c in d["cams"]), rgb=True)
            # arrivals spread over 20 ms so that batches form and overlap
            tickets.append(srv.submit(rig=i % 3, frame=d, out=out, arrival_s=srv.now() + 0.002 * i))
            outs.append((i, out))
    srv.drain()
    for i, out in outs:
        g = out.result()
        for k in KEYS:
            assert np.array_equal(g[k], alone[i][k]), (i, k)
    st = srv.stats()
    assert st["frames"] == len(outs) and st["p99_ms"] >= st["p50_ms"] > 0
    if plain:
        assert st["mean_batch_frames"] == 1.0
    # the per-frame samples: one per completed frame with its rig, agreeing with the stats
    rigs, lat = srv.latencies()
    assert len(lat) == len(outs)
    assert sorted(np.bincount(rigs).tolist()) == sorted(
        np.bincount([i % 3 for i, _ in outs]).tolist())
    assert lat.max() == pytest.approx(st["max_ms"]) and lat.mean() == pytest.approx(st["mean_ms"])
    assert np.sort(lat)[int(np.ceil(0.5 * len(lat))) - 1] == pytest.approx(st["p50_ms"])
    srv.reset_stats()
    assert len(srv.latencies()[1]) == 0
    srv.close()


def test_server_admission_by_footprint(ff):
    print("[case] admission", flush=True)
    with pytest.raises(ff.FuseFlowError) as e:
        ff.Server(hbm_budget_bytes=64 << 10, lanes=2)          # not even one small frame
    assert e.value.status == ff.FF_ERR_OOM
    f = cached_frame("c2")                                     # 1.2 Mpx
    d = ff.to_device(f)
    srv = ff.Server(hbm_budget_bytes=24 << 20, lanes=1, max_batch_frames=2)
    assert srv.max_pixels < f.pixels
    with pytest.raises(ff.FuseFlowError) as e:
        srv.submit(0, d, ff.Output(16))
    assert e.value.status == ff.FF_ERR_OOM
    small = cached_frame("c1")
    ds = ff.to_device(small)
    out = ff.Output(small.pixels)
    t = srv.submit(0, ds, out)
    srv.wait(t)
    with pytest.raises(ff.FuseFlowError) as e:      # a waited ticket is forgotten
        srv.poll(t)
    assert e.value.status == ff.FF_ERR_NOT_FOUND
    assert out.result()["count"] == len(O.fuse_frame(small)["keys"])
    srv.close()


def test_server_reserve_sizes_idle_lanes(ff):
    """ff_server_reserve gives every lane a workspace for the stated batch up front; frames
    and batches that fit it then run without any workspace growing (the footprint stays
    put), with the same results as ff_fuse; a budget too small for every lane stops with
    FF_ERR_OOM after the lanes that fit."""
    print("[case] reserve", flush=True)
    big, small = cached_frame("c2"), cached_frame("c1")
    db, ds = ff.to_device(big), ff.to_device(small)
    ref_b, ref_s = _alone(ff, db), _alone(ff, ds)
    px, nc = big.pixels, len(big.cams)
    want = 2 * px + (2 * px) // 4          # two large frames, with the lanes' pixel headroom
    lane = int(ff.lib().ff_workspace_bytes(want, 2 * nc, 2))
    srv = ff.Server(hbm_budget_bytes=4 * lane, lanes=3, max_batch_frames=2)
    with pytest.raises(ff.FuseFlowError) as e:
        srv.reserve(px, nc, 3)                               # beyond the batch limit
    assert e.value.status == ff.FF_ERR_INVALID_ARG
    srv.reserve(2 * px, 2 * nc, 2)
    used = srv.stats()["hbm_used_bytes"]
    assert used == 3 * lane
    outs = []
    for rep in range(2):
        for name, d, P in (("b", db, big.pixels), ("s", ds, small.pixels), ("b", db, big.pixels)):
            o = ff.Output(P, rgb=True)
            srv.submit(rep, d, o)
            outs.append((name, o))
    srv.drain()
    st = srv.stats()
    assert st["frames"] == 6 and st["hbm_used_bytes"] == used and st["hbm_peak_bytes"] == used
    for name, o in outs:
        g, r = o.result(), (ref_s if name == "s" else ref_b)
        for k in KEYS:
            assert np.array_equal(g[k], r[k]), (name, k)
    srv.close()
    one = int(ff.lib().ff_workspace_bytes(px + px // 4, nc, 1))
    two = ff.Server(hbm_budget_bytes=2 * one + one // 2, lanes=3, max_batch_frames=1)
    with pytest.raises(ff.FuseFlowError) as e:
        two.reserve(px, nc, 1)
    assert e.value.status == ff.FF_ERR_OOM
    assert two.stats()["hbm_used_bytes"] == 2 * one
    o = ff.Output(big.pixels, rgb=True)
    two.submit(0, db, o)
    two.drain()
    assert np.array_equal(o.result()["keys"], ref_b["keys"])
    two.close()


def test_server_admits_by_each_frames_footprint(ff):
    """The budget holds one large frame's workspace or several small ones, not both: small
    frames run side by side on the lanes, a large frame waits until they are done (idle
    lanes give their workspaces back), the device bytes of all workspaces never exceed the
    budget, and every result equals ff_fuse."""
    print("[case] footprint admission", flush=True)
    big, small = cached_frame("c2"), cached_frame("c1")
    db, ds = ff.to_device(big), ff.to_device(small)
    wb = int(ff.lib().ff_workspace_bytes(big.pixels, len(big.cams), 1))
    ws = int(ff.lib().ff_workspace_bytes(small.pixels, len(small.cams), 1))
    budget = int(wb * 1.3)                 # the large frame with headroom, or 2+ small ones
    assert budget < wb + 2 * ws and budget > 2 * ws
    ref_b, ref_s = _alone(ff, db), _alone(ff, ds)
    srv = ff.Server(hbm_budget_bytes=budget, lanes=3, max_batch_frames=1)
    outs = []
    for rep in range(3):
        for name, d, P in (("s", ds, small.pixels), ("s", ds, small.pixels), ("b", db, big.pixels)):
            o = ff.Output(P, rgb=True)
            srv.submit(0, d, o)
            outs.append((name, o))
    srv.drain()
    st = srv.stats()
    assert st["frames"] == 9 and 0 < st["hbm_peak_bytes"] <= budget, st
    for name, o in outs:
        g, r = o.result(), (ref_s if name == "s" else ref_b)
        for k in KEYS:
            assert np.array_equal(g[k], r[k]), (name, k)
    # a frame larger than the whole budget is refused; the server keeps serving
    tiny = ff.Server(hbm_budget_bytes=ws + ws // 2, lanes=2, max_batch_frames=1)
    with pytest.raises(ff.FuseFlowError) as e:
        tiny.submit(0, db, ff.Output(big.pixels))
    assert e.value.status == ff.FF_ERR_OOM
    o = ff.Output(small.pixels, rgb=True)
    tiny.wait(tiny.submit(0, ds, o))
    assert np.array_equal(o.result()["keys"], ref_s["keys"])
    tiny.close()
    srv.close()


def test_server_back_pressure(ff):
    print("[case] back-pressure", flush=True)
    small = cached_frame("c1")
    ds = ff.to_device(small)
    srv = ff.Server(hbm_budget_bytes=1 << 30, lanes=1, max_batch_frames=1, max_pending=2)
    later = srv.now() + 0.5                                     # not yet arrived
    outs = [ff.Output(small.pixels) for _ in range(3)]
    srv.submit(0, ds, outs[0], arrival_s=later)
    srv.submit(0, ds, outs[1], arrival_s=later)
    with pytest.raises(ff.FuseFlowError) as e:
        srv.submit(0, ds, outs[2], arrival_s=later)
    assert e.value.status == ff.FF_ERR_BUSY
    srv.drain()
    assert srv.stats()["frames"] == 2
    srv.close()


@pytest.mark.parametrize("slot", [13, 18])
def test_probe_keeps_results_and_counts_launches(ff, slot):
    """Timing one kernel splits the cached graph around it; results must not change."""
    print(f"[case] probe slot {slot}", flush=True)
    frames = _frames()[:3]
    devs = [ff.to_device(f) for f in frames]
    ctx = ff.Context(max_pixels=4_000_000, max_cameras=16, max_frames=4)
    ref = [o.result() for o in ctx.fuse_batch(devs)]
    ctx.probe(slot)
    for rep in range(3):
        outs = ctx.fuse_batch(devs)
        for g, r in zip((o.result() for o in outs), ref):
            for k in KEYS:
                assert np.array_equal(g[k], r[k]), (rep, k)
    p = ctx.probe_read()
    assert p["slot"] == slot and p["launches"] == 3 and p["frames"] == 9
    assert p["pixels"] == 3 * sum(f.pixels for f in frames)
    assert 0 < p["mean_ms"] < 1000
    ctx.probe(-1)
    ctx.fuse_batch(devs)
    assert ctx.probe_read()["launches"] == 0
    ctx.close()


def test_server_probe(ff):
    print("[case] server probe", flush=True)
    frames = _frames()
    devs = [ff.to_device(f) for f in frames]
    srv = ff.Server(hbm_budget_bytes=2 << 30, lanes=2, max_batch_frames=4)
    srv.probe(13)
    for i, d in enumerate(devs):
        srv.submit(0, d, ff.Output(sum(c.width * c.height for c in d["cams"])))
    srv.drain()
    p = srv.probe_read()
    assert p["frames"] == len(devs) and p["launches"] == srv.stats()["batches"]
    assert p["total_ms"] > 0
    srv.close()


def test_serving_at_benchmark_scale(ff):
    """The configuration bench.py times: four 8 x 1280x720 rigs through the serving path
    (2 lanes, batches of up to 4 frames).  Every frame equals its standalone ff_fuse result
    bit for bit, and one of them equals the oracle."""
    print("[case] serving, four 8x1280x720 rigs", flush=True)
    frames = [cached_frame("c3", rig=r) for r in range(4)]
    devs = [ff.to_device(f) for f in frames]
    P = frames[0].pixels
    ctx = ff.Context(max_pixels=P, max_cameras=8)
    alone = []
    for d in devs:
        alone.append(ctx.fuse(d["cams"], d["depth"], d["conf"], d["rgb"]).result())
    ctx.close()
    srv = ff.Server(hbm_budget_bytes=8 << 30, lanes=2, max_batch_frames=4, max_pending=64)
    outs = [[ff.Output(P, rgb=True) for _ in range(2)] for _ in devs]
    for rep in range(2):
        for i, d in enumerate(devs):
            srv.submit(i, d, outs[i][rep])
    srv.drain()
    assert srv.stats()["mean_batch_frames"] > 1.0
    srv.close()
    for i in range(len(devs)):
        for rep in range(2):
            g = outs[i][rep].result()
            for k in KEYS:
                assert np.array_equal(g[k], alone[i][k]), (i, rep, k)
    compare(outs[2][1].result(), O.fuse_frame(frames[2]), label="c3 rig 2 served")


def test_batch_at_frame_limit(ff):
    """64 frames (the per-batch maximum) of one small camera each, ragged sizes."""
    print("[case] batch of 64 frames", flush=True)
    from synth import make_frame, ring_cameras
    from synth.scenes import _scene_c1
    rng = np.random.default_rng(64)
    frames = []
    for i in range(64):
        W, H = int(rng.integers(20, 90)), int(rng.integers(10, 60))
        cams = ring_cameras([(W, H)] * 2, rng=rng, jitter_pos=0.2)
        frames.append(make_frame(cams[:1 + i % 2], _scene_c1(rng, cams), 6400 + i))
    devs = [ff.to_device(f) for f in frames]
    ctx = ff.Context(max_pixels=sum(f.pixels for f in frames), max_cameras=128, max_frames=64)
    outs = ctx.fuse_batch(devs, members=True)
    for i in (0, 1, 17, 63):
        compare(outs[i].result(), O.fuse_frame(frames[i]), label=f"frame {i} of 64")
    for i, (d, o) in enumerate(zip(devs, outs)):
        a = ctx.fuse(d["cams"], d["depth"], d["conf"], d["rgb"]).result()
        g = o.result()
        for k in KEYS:
            assert np.array_equal(g[k], a[k]), (i, k)
    ctx.close()


def test_server_rejects_a_bad_frame_alone(ff):
    """A frame the host checks reject (no confidence without FF_CONF_EQ3) is refused at its
    own submit; frames before and after it are accepted and complete normally."""
    print("[case] server error path", flush=True)
    f = cached_frame("c1")
    dev = ff.to_device(f)
    srv = ff.Server(hbm_budget_bytes=1 << 30, lanes=2, max_batch_frames=2)
    outs = [ff.Output(f.pixels) for _ in range(2)]
    t0 = srv.submit(0, dev, outs[0])
    with pytest.raises(ff.FuseFlowError) as e:
        srv.submit(1, dict(cams=dev["cams"], depth=dev["depth"]), ff.Output(f.pixels))
    assert e.value.status == ff.FF_ERR_INVALID_ARG
    t1 = srv.submit(0, dev, outs[1])
    srv.wait(t0)
    done = False
    while not done:
        done = srv.poll(t1)
    srv.drain()
    ref = O.fuse_frame(f)
    for o in outs:
        compare(o.result(), ref, check_members=False, label="around a rejected frame")
    srv.close()


def test_server_default_arrival_is_the_submit(ff):
    """A submit without an arrival time arrives when it is made: its latency is at most the
    wall time from the submit to its completion, however long the server existed before."""
    import time
    print("[case] default arrival", flush=True)
    f = cached_frame("c1")
    dev = ff.to_device(f)
    srv = ff.Server(hbm_budget_bytes=1 << 30, lanes=2, max_batch_frames=2)
    time.sleep(0.3)
    out = ff.Output(f.pixels)
    t = time.perf_counter()
    tk = srv.submit(0, dev, out)
    srv.wait(tk)
    wall_ms = (time.perf_counter() - t) * 1e3
    st = srv.stats()
    assert st["frames"] == 1 and 0 < st["max_ms"] <= wall_ms + 0.5, (st, wall_ms)
    srv.close()


def test_server_waits_for_the_callers_stream(ff):
    """Inputs written by torch on a side stream right before the submit (with that stream
    passed) are complete when the server reads them: the result equals ff_fuse of the same
    frame.  The outputs are cleared on that stream too."""
    import torch
    print("[case] caller stream ordering", flush=True)
    f = cached_frame("c2")
    src = ff.to_device(f)
    ref = _alone(ff, src)
    srv = ff.Server(hbm_budget_bytes=2 << 30, lanes=2, max_batch_frames=2)
    side = torch.cuda.Stream()
    for rep in range(3):
        dst = dict(cams=src["cams"], depth=[torch.empty_like(d) for d in src["depth"]],
                   conf=[torch.empty_like(c) for c in src["conf"]],
                   rgb=[torch.empty_like(r) for r in src["rgb"]])
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            big = torch.empty(64 << 20, device="cuda")
            for _ in range(8):            # keep the side stream busy before the copies
                big.mul_(1.0001)
            for k in ("depth", "conf", "rgb"):
                for a, b in zip(dst[k], src[k]):
                    a.copy_(b)
            out = ff.Output(f.pixels, rgb=True)
            out.count.fill_(0)
        tk = srv.submit(0, dst, out, stream=side)
        srv.wait(tk)
        g = out.result()
        for k in KEYS:
            assert np.array_equal(g[k], ref[k]), (rep, k)
        del big
    srv.close()
