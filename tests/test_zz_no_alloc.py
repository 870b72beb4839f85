"""The allocation-free E_MC entry point (ff_emc_noalloc) against ff_emc, through the C ABI.

Two calls in a row on the same device, the second with a smaller input (fewer cameras and
a smaller cloud), each compared with ff_emc on the same input: the same kernels run on a
static scratch array instead of a context workspace, so the results are bit-identical.
"""
import numpy as np
import pytest

from tests.conftest import cached_frame

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2602_01035_amd as ff
    return ff


def _fused(ff, dev, ctx):
    return ctx.fuse(dev["cams"], dev["depth"], dev["conf"], dev.get("rgb"))


def test_emc_noalloc_matches_emc_on_two_calls(ff):
    import torch
    print("[case] ff_emc_noalloc vs ff_emc, c2 then c1", flush=True)
    big = ff.to_device(cached_frame("c2"))          # 4 cameras, 1.2 Mpx
    small = ff.to_device(cached_frame("c1"))        # 2 cameras, 154 kpx
    ctx = ff.Context(max_pixels=2_000_000, max_cameras=8)
    results = []
    for dev, stride in ((big, 1), (small, 3)):
        out = _fused(ff, dev, ctx)
        ref = ctx.emc(dev["cams"], dev["depth"], out, stride=stride)
        res = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
        ff.emc_noalloc(dev["cams"], dev["depth"], out.xyz, out.count, out.capacity, res,
                       stride=stride)
        got = res.cpu().tolist()
        results.append(got)
        assert got[1] == ref["points"] and got[1] > 0, (got, ref)
        assert got[0] == ref["emc_m"] and got[2] == ref["mean_visible"], (got, ref)
    assert results[0] != results[1]
    ctx.close()


def test_emc_noalloc_rejects_too_many_cameras(ff):
    import torch
    print("[case] ff_emc_noalloc camera limit", flush=True)
    dev = ff.to_device(cached_frame("c1"))
    cams = list(dev["cams"]) * 33                   # 66 cameras > 64
    depth = list(dev["depth"]) * 33
    xyz = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    res = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(ff.FuseFlowError) as e:
        ff.emc_noalloc(cams, depth, xyz, cnt, 4, res)
    assert e.value.status == ff.FF_ERR_INVALID_ARG
