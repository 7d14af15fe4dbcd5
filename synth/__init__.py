"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only *generates* inputs: disparity maps of ground-plus-box road
scenes, camera presets, the default model parameters and the workload
descriptions.  It holds none of the stixel method's arithmetic (no data
costs, no prefix sums, no dynamic programme), so that the CPU oracle and the
HIP path can both consume it without sharing any of the computation.
"""

from .configs import (  # noqa: F401
    DEFAULT_MODEL,
    CAMERA_1024x440,
    camera_for_size,
    make_params,
    WORKLOADS,
)
from .scenes import (  # noqa: F401
    SceneSpec,
    generate_frame,
    generate_workload,
    workload_frame,
    random_columns_frame,
)
