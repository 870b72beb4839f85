"""Host-side checks of the C ABI (no GPU needed): the built library loads and exports every
function that include/fuseflow.h declares, and the Python binding's struct layouts agree
with the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fuseflow.h")
LIB = os.path.join(ROOT, "paper_2602_01035_amd", "libfuseflow.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ff_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ff_context_create", "ff_context_destroy", "ff_params_default", "ff_fuse",
                 "ff_fuse_batch", "ff_status_string", "ff_autotune",
                 "ff_server_create", "ff_server_submit", "ff_server_poll", "ff_server_wait",
                 "ff_server_stats", "ff_server_destroy", "ff_confidence", "ff_emc"):
        assert must in names, must


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_defaults_and_status_strings():
    import paper_2602_01035_amd as ff
    p = ff.Params()
    assert abs(p.tau - 0.6) < 1e-7 and p.k_views == 4 and abs(p.sigma - 0.02) < 1e-9
    assert p.coarse_res == 64 and p.max_level == 6 and p.target_per_cell == 16
    assert p.level_override == -1 and p.flags == 0
    assert ff.lib().ff_status_string(0) == b"ok"
    assert ff.lib().ff_status_string(1) == b"invalid argument"
    assert b"gfx950" in ff.lib().ff_version()
    # workspace sizing is a pure function of the limits
    b1 = ff.lib().ff_workspace_bytes(1 << 20, 8, 1)
    b2 = ff.lib().ff_workspace_bytes(1 << 21, 8, 1)
    assert 0 < b1 < b2


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_struct_sizes_match_header():
    import paper_2602_01035_amd as ff
    assert ctypes.sizeof(ff.ff_camera) == 4 * (2 + 4 + 12)
    assert ctypes.sizeof(ff.ff_view) == 3 * 8
    assert ctypes.sizeof(ff.ff_params) == 8 * 4
    assert ctypes.sizeof(ff.ff_output) == 8 * 8 + 2 * 4 + 3 * 8
    assert ctypes.sizeof(ff.ff_frame) == 8 + 2 * 8


STRUCTS = ("ff_camera", "ff_view", "ff_params", "ff_output", "ff_frame", "ff_tuning",
           "ff_trace", "ff_probe", "ff_server_config", "ff_stats", "ff_conf_params",
           "ff_emc_params")


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_struct_layouts_match_c_compiler(tmp_path):
    """Size and every field offset of each ctypes struct against gcc on the header."""
    import shutil
    import subprocess
    import paper_2602_01035_amd as ff
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "fuseflow.h"',
             'int main(void) {']
    for name in STRUCTS:
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in getattr(ff, name)._fields_:
            lines.append(f'printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True,
                             text=True).stdout.splitlines():
        a, b, v = ln.split()
        got[(a, b)] = int(v)
    for name in STRUCTS:
        cls = getattr(ff, name)
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert got[(name, fname)] == getattr(cls, fname).offset, (name, fname)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_invalid_arguments_rejected_without_gpu_work():
    import paper_2602_01035_amd as ff
    h = ctypes.c_void_p()
    # null output pointer, bad sizes: rejected before any device is touched
    assert ff.lib().ff_context_create(None, 0, 100, 1, 1) == ff.FF_ERR_INVALID_ARG
    assert ff.lib().ff_fuse(None, 1, None, None, None, None, None) == ff.FF_ERR_INVALID_ARG
    assert ff.lib().ff_fuse_batch(None, 1, None, None, None, None) == ff.FF_ERR_INVALID_ARG
