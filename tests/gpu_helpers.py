"""Shared helpers of the GPU tests: run the library, compare against the oracle."""
import numpy as np

from oracle import core as O

# Parity bar.  Integer/index results are compared bit for bit.  Floating point: the oracle
# accumulates in float64 and the library's float64 continuous part differs only in the
# last bits of exp/log, so 1e-5 relative (floor 1 m for coordinates, 1e-6 for weights) is
# far above the expected gap while far below any plausible arithmetic mistake.
XYZ_RTOL = 1e-5
W_RTOL = 1e-5


def oracle_params(p):
    """library Params -> oracle Params"""
    return O.Params(tau=float(np.float32(p.tau)), k_views=p.k_views, sigma=float(np.float32(p.sigma)),
                    coarse_res=p.coarse_res, max_level=p.max_level,
                    target_per_cell=p.target_per_cell, level_override=p.level_override,
                    flags=p.flags)


def run_gpu(ctx, frame, params=None, members=True, with_rgb=True, batch=False, stream=None):
    import paper_2602_01035_amd as ff
    dev = ff.to_device(frame, with_rgb=with_rgb)
    if batch:
        out = ctx.fuse_batch([dev], params=params, members=members, stream=stream)[0]
    else:
        out = ctx.fuse(dev["cams"], dev["depth"], dev["conf"], dev.get("rgb"), params=params,
                       members=members, stream=stream)
    return out.result()


def compare(g, o, check_members=True, label=""):
    """Assert GPU result g == oracle result o to the parity bar."""
    S = len(o["keys"])
    assert g["status"] == 0, (label, "status", g["status"])
    assert g["count"] == S, (label, "S", g["count"], S)
    assert np.array_equal(g["keys"], o["keys"]), (label, "keys")
    assert np.array_equal(g["n_members"], o["n_members"]), (label, "n_members")
    assert np.array_equal(g["reps"], o["reps"]), (label, "reps")
    if check_members and "member_ids" in g:
        assert np.array_equal(g["member_offsets"], o["member_offsets"]), (label, "offsets")
        assert np.array_equal(g["member_ids"], o["member_ids"]), (label, "member ids")
    if S:
        gx, ox = g["xyz"].astype(np.float64), np.asarray(o["xyz"], np.float64)
        gw, ow = g["weight"].astype(np.float64), np.asarray(o["weight"], np.float64)
        # a NaN on one side only is a mismatch (a comparison with NaN is never "too far")
        assert np.array_equal(np.isnan(gx), np.isnan(ox)), (label, "xyz NaN positions")
        assert np.array_equal(np.isnan(gw), np.isnan(ow)), (label, "weight NaN positions")
        assert np.array_equal(np.isinf(gx), np.isinf(ox)), (label, "xyz inf positions")
        fin = np.isfinite(ox)
        scale = np.maximum(np.abs(np.where(fin, ox, 0.0)).max(axis=1), 1.0)
        err = np.where(fin, np.abs(gx - np.where(fin, ox, 0.0)), 0.0).max(axis=1)
        bad = np.flatnonzero(err > XYZ_RTOL * scale)
        assert len(bad) == 0, (label, "xyz", bad[:5], err[bad[:5]])
        wfin = np.isfinite(ow)
        werr = np.where(wfin, np.abs(gw - np.where(wfin, ow, 0.0)), 0.0)
        wbad = np.flatnonzero(werr > W_RTOL * np.maximum(np.where(wfin, ow, 0.0), 1e-6))
        assert len(wbad) == 0, (label, "weight", wbad[:5], g["weight"][wbad[:5]],
                                o["weight"][wbad[:5]])
        if o.get("rgb") is not None and g.get("rgb") is not None:
            d = np.abs(g["rgb"].astype(int) - o["rgb"].astype(int))
            assert d.max() <= 1, (label, "rgb")


def compare_sample(g, s, label=""):
    """Assert GPU result g == the sampled oracle result s (``O.fuse_sample``): the whole
    partition bit for bit (count, keys, member counts, membership when g carries it), the
    per-cell outputs on the sampled cells."""
    S = len(s["keys"])
    assert g["status"] == 0, (label, "status", g["status"])
    assert g["count"] == S, (label, "S", g["count"], S)
    assert np.array_equal(g["keys"], s["keys"]), (label, "keys")
    assert np.array_equal(g["n_members"], s["n_members"]), (label, "n_members")
    if "member_ids" in g:
        assert np.array_equal(g["member_offsets"], s["member_offsets"]), (label, "offsets")
        assert np.array_equal(g["member_ids"], s["member_ids"]), (label, "member ids")
    c = s["cells"]
    sub = dict(keys=s["keys"][c], n_members=s["n_members"][c], reps=s["reps"], xyz=s["xyz"],
               weight=s["weight"], rgb=s["rgb"])
    gs = dict(status=g["status"], count=len(c), keys=g["keys"][c],
              n_members=g["n_members"][c], reps=g["reps"][c], xyz=g["xyz"][c],
              weight=g["weight"][c], rgb=None if g.get("rgb") is None else g["rgb"][c])
    compare(gs, sub, check_members=False, label=label)
