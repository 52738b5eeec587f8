"""MI355X-native direct volume rendering of LR-spline volumes.

C ABI: include/lrvr.h; HIP kernels and host builders: csrc/; binding: _lib;
Python API: api (Volume, Scene, render, RenderFunction, ExtractFunction, trace,
lookup).
"""
from .api import (ExtractFunction, Forest, Octree, RenderFunction, RenderParams, Scene, Volume, bezier_stride,  # noqa: F401
                  build_forest_device, lookup, render, render_workspace,
                  render_backward, streamlines, support_csr, trace, unpack)
from ._build import build  # noqa: F401
