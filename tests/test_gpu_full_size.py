"""GPU parity at the full sizes of the two largest workloads, in their own launch
configurations, against the sampled oracle (whole partition bit for bit, per-cell outputs
on a few thousand sampled cells including the first, last and largest ones):

  * 16 cameras at mixed resolutions (6 x 640x480, 6 x 1280x720, 4 x 1920x1080), four
    frames of the moving-sphere sequence in one batched call, after the autotuner picked
    the tile and digit sizes;
  * four rigs of 2, 6, 12 and 32 cameras at resolutions drawn from {640x480, 1280x720,
    1920x1080} (36.6 Mpx for the 32-camera frame) through the continuous-batching server.
"""
import numpy as np
import pytest

from oracle import core as O
from tests.conftest import cached_frame
from tests.gpu_helpers import compare_sample

pytestmark = pytest.mark.gpu

KEYS = ("keys", "xyz", "weight", "reps", "n_members", "rgb")


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2602_01035_amd as ff
    return ff


def test_sixteen_camera_sequence_batched(ff):
    frames = [cached_frame("c4", frame=i) for i in range(4)]
    P = sum(f.pixels for f in frames)
    print(f"[case] 16 mixed-resolution cameras, 4 frames ({P} px) in one batched call",
          flush=True)
    devs = [ff.to_device(f) for f in frames]
    ctx = ff.Context(max_pixels=P, max_cameras=64, max_frames=4)
    tuned = ctx.autotune(devs)
    print(f"[case] tuned {tuned}", flush=True)
    outs = ctx.fuse_batch(devs, members=True)
    res = [o.result() for o in outs]
    for i, (f, g) in enumerate(zip(frames, res)):
        compare_sample(g, O.fuse_frame_sample(f, n_sample=3000, seed=i), label=f"frame {i}")
    # the same frame alone equals its result in the batch
    d = devs[2]
    a = ctx.fuse(d["cams"], d["depth"], d["conf"], d["rgb"]).result()
    for k in KEYS:
        assert np.array_equal(res[2][k], a[k]), k
    ctx.close()


def test_four_rigs_served(ff):
    frames = [cached_frame("c5", rig=r) for r in range(4)]
    print("[case] served rigs of " + ", ".join(
        f"{len(f.cams)} cams / {f.pixels} px" for f in frames), flush=True)
    devs = [ff.to_device(f) for f in frames]
    srv = ff.Server(hbm_budget_bytes=16 << 30, lanes=2, max_batch_frames=4, max_pending=64)
    outs = [ff.Output(f.pixels, rgb=True) for f in frames]
    for i, d in enumerate(devs):
        srv.submit(i, d, outs[i])
    srv.drain()
    srv.close()
    for i, (f, o) in enumerate(zip(frames, outs)):
        compare_sample(o.result(), O.fuse_frame_sample(f, n_sample=3000, seed=10 + i),
                       label=f"rig {i}")
