import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases (still minutes, not hours)")


@functools.lru_cache(maxsize=None)
def cached_frame(name, frame=0, rig=0, noise=True, with_rgb=True):
    from synth import make_config
    return make_config(name, frame=frame, rig=rig, noise=noise, with_rgb=with_rgb)


@pytest.fixture(scope="session")
def frame_c1():
    return cached_frame("c1")


@pytest.fixture(scope="session")
def frame_c2():
    return cached_frame("c2")
