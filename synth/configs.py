"""Camera presets, default model parameters and the named synthetic workloads.

The paper fixes the camera geometry only implicitly (a flat ground seen from a
stereo rig, with the ground slope and horizon known per image, Sec. 3) and
defers the prior model and its constants to Pfeiffer's thesis, which is not
available.  The values below are therefore stated *inputs*: both the CPU oracle
and the HIP library receive them from the caller and derive everything else on
their own.

Class order everywhere is (object, ground, sky), the order of the class set in
Sec. 3.1.  ``trans_cost[prev][cur]`` is the pairwise prior of a stixel of class
``cur`` sitting directly above one of class ``prev``; ``math.inf`` marks a
transition the staggering constraint forbids (Sec. 3, constraint 4).
"""

from __future__ import annotations

import copy
import math

INF = math.inf

#: Default prior / sensor-model parameters.  Not from the paper (it defers them
#: to Pfeiffer's thesis); chosen once for the synthetic ground-plus-box scenes.
DEFAULT_MODEL = {
    # sensor model, Eq. 3-4
    "p_out": 0.15,                 # outlier rate
    "sigma_disp": 1.0,             # disparity measurement noise [px]
    "sigma_sky": 0.8,              # sky model standard deviation [px]
    "ground_slope_noise": 0.05,    # relative slope uncertainty of the ground model
    "object_depth_extent_m": 0.3,  # depth extent of an object stixel [m]
    # prior model, Sec. 3 constraints (1)-(5)
    "bic_cost": 3.0,                     # (1) cost per stixel
    "first_cost": [1.0, 0.0, 10.0],      # prior of the bottom stixel, per class
    "trans_cost": [[0.5, 1.0, 0.0],      # object -> (object, ground, sky)
                   [0.0, INF, 0.0],      # ground -> ...
                   [2.0, INF, INF]],     # sky    -> ...
    "ordering_cost": 4.0,     # (3) upper object closer than the lower one
    "ordering_tol_px": 1,     #     tolerance in disparity steps (integer)
    "gravity_cost": 3.0,      # (2) object on ground but far behind it (floating)
    "gravity_tol_px": 2.0,
    "diving_cost": 20.0,      # (5) object base closer than the ground below it
    "diving_tol_px": 2.0,
}

#: The paper's headline camera: 1024x440 disparity, stixel width 5.
CAMERA_1024x440 = {
    "focal_px": 700.0,
    "baseline_m": 0.3,
    "cam_height_m": 1.2,
    "horizon_row": 180.0,   # top-down image row of the horizon
    "pitch_rad": 0.0,
}


def camera_for_size(width: int, height: int) -> dict:
    """Camera preset scaled to an image size: focal 700 px per 1024 columns and
    the horizon at the same relative height as row 180 of 440."""
    cam = dict(CAMERA_1024x440)
    cam["focal_px"] = 700.0 * width / 1024.0
    cam["horizon_row"] = float(round(180.0 * height / 440.0))
    return cam


def make_params(camera: dict | None = None, model: dict | None = None, *,
                stixel_width: int = 5, max_disparity: int = 128,
                max_width: int = 1024, max_height: int = 440,
                max_stixels_per_column: int = 0, reduce_mode: int = 0,
                cost_grid_log2: int = 10, flags: int = 0, subpixel_log2: int = 0) -> dict:
    """Full parameter set handed to both the oracle and the HIP library.

    reduce_mode: 0 = lower median of the valid pixels of each row strip,
                 1 = mean (the paper's Sec. 4.1 operator).
    cost_grid_log2: every cost table and prior constant is rounded to a
                 multiple of 2**-cost_grid_log2 nats.
    max_stixels_per_column: output capacity per column, 0 means the height.
    flags: library handle flags (1 = batch API only: no per-frame workspace);
                 the oracle ignores them.
    subpixel_log2: disparities in bins of 2^-subpixel_log2 px (0 = whole px);
                 max_disparity stays in px.
    """
    return {
        "camera": dict(camera if camera is not None else CAMERA_1024x440),
        "model": copy.deepcopy(model if model is not None else DEFAULT_MODEL),
        "stixel_width": int(stixel_width),
        "max_disparity": int(max_disparity),
        "max_width": int(max_width),
        "max_height": int(max_height),
        "max_stixels_per_column": int(max_stixels_per_column),
        "reduce_mode": int(reduce_mode),
        "cost_grid_log2": int(cost_grid_log2),
        "flags": int(flags),
        "subpixel_log2": int(subpixel_log2),
    }


#: Named workloads.  Frame sizes, camera scaling and scene statistics follow
#: the paper's headline case (1024x440, stixel width 5) and its resolution sweep.
WORKLOADS = {
    "frame_1024x440": dict(sizes=[(1024, 440)], frames=1, widths=[5], d_max=128,
                           boxes=(4, 12), sigma=(0.8, 0.8), invalid=(0.05, 0.05),
                           seeds=[0]),
    "batch64_1024x440": dict(sizes=[(1024, 440)], frames=64, widths=[5], d_max=128,
                             boxes=(4, 12), sigma=(0.8, 0.8), invalid=(0.05, 0.05),
                             seeds=list(range(64))),
    "hires16_2048x880": dict(sizes=[(2048, 880)], frames=16, widths=[3, 5], d_max=256,
                             boxes=(4, 12), sigma=(0.8, 0.8), invalid=(0.05, 0.05),
                             seeds=list(range(16))),
    "uneven256": dict(sizes=[(640, 240), (1024, 440), (1280, 720), (2048, 880)],
                      frames=256, widths=[3, 5, 7], d_max=None,
                      boxes=(0, 20), sigma=(0.5, 1.5), invalid=(0.0, 0.15),
                      seeds=[1000 + i for i in range(256)]),
}
