"""CPU oracle for the FUSE-Flow fusion path — test infrastructure only.

Imported by the test suite, the smoke check and the benchmark's CPU baseline; the GPU
library never imports or calls it.
"""
from .core import (Params, fuse, fuse_frame, validate, FF_NO_MF, FF_NO_DC, FF_NO_SA,
                   camera_f32, backproject, project, gate, generate_points, extents,
                   coarse_exponent, coarse_cells, coarse_linear, levels, cell_keys, group,
                   representatives, select_views, consistency, fuse_cells, PAD)
