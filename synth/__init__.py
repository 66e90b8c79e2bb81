"""Seeded synthetic inputs for the adaptive bilateral filter.

This module only draws images and parameter maps. It holds none of the
filter's arithmetic, so both the CPU oracle (``oracle/``) and the GPU
library's tests and benchmark can use it without sharing any step of the
method.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` and returns
float32 arrays with ``-0.0`` canonicalised to ``+0.0``. Intensities live on
[0, 255] as in the paper's experiments (Sec. III: sigma values are quoted on
the 8-bit scale).

The workloads stand in for the paper's test images, which are not available:
- ``rect_scene``  — piecewise-constant rectangles plus Gaussian noise
  (classical-filter timing image of Table 2 / Fig. 3 is replaced by this);
- ``gauss_field`` — a smooth sum of Gaussian blobs plus noise
  (the sharpening images of Figs. 4-5 are replaced by this);
- ``voronoi``     — piecewise-constant Voronoi cells plus noise;
- ``texture_frames`` — textured regions (checker / stripes) over
  piecewise-constant cells (the texture-filtering images of Figs. 9-10).
"""
from .generators import (  # noqa: F401
    smooth_field,
    rect_scene,
    gauss_field,
    voronoi,
    block_constant,
    texture_frames,
    workload,
    WORKLOADS,
    serving_requests,
)
