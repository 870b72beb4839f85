"""The sampled oracle (per-cell work on a sample of cells, used for the largest frames)
gives exactly the whole oracle's results on the cells it samples, and the whole partition."""
import numpy as np
import pytest

from oracle import core as O
from tests.conftest import cached_frame


@pytest.mark.parametrize("name,flags", [("c1", 0), ("c2", 0), ("c1", O.FF_NO_MF | O.FF_NO_DC)])
def test_sample_equals_whole(name, flags):
    f = cached_frame(name)
    p = O.Params(flags=flags)
    full = O.fuse_frame(f, p)
    s = O.fuse_frame_sample(f, p, n_sample=400, seed=7)
    for k in ("keys", "n_members", "member_offsets", "member_ids"):
        assert np.array_equal(full[k], s[k]), k
    c = s["cells"]
    assert np.all(np.diff(c) > 0) and c[0] == 0 and c[-1] == len(full["keys"]) - 1
    for k in ("xyz", "weight", "rgb", "reps"):
        assert np.array_equal(full[k][c], s[k]), k


def test_sample_covers_edge_cells():
    n = np.array([5, 1, 2, 9, 3, 1, 40, 2, 3, 7], np.uint32)
    c = O.sample_cells(n, 2, seed=0)
    assert {0, 9, 6, 3}.issubset(set(c.tolist()))          # ends and the largest cells
    assert {1, 2, 4}.issubset(set(c.tolist()))             # one, two, three members
    assert len(O.sample_cells(np.zeros(0, np.uint32), 5, 0)) == 0
