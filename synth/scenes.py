"""Seeded synthetic disparity maps shaped like the paper's road scenes.

A flat ground plane seen from a stereo rig, fronto-parallel box obstacles
standing on it, sky (disparity 0) above, Gaussian measurement noise and a
fraction of invalid pixels (disparity -1).  This stands in for the SYNTHIA and
real stereo frames of the paper's evaluation, which are not available.

Every frame is a float32 array of shape (height, width), row 0 at the top.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .configs import CAMERA_1024x440, WORKLOADS, camera_for_size


@dataclass
class SceneSpec:
    width: int = 1024
    height: int = 440
    d_max: int = 128
    camera: dict = field(default_factory=lambda: dict(CAMERA_1024x440))
    boxes: tuple = (4, 12)          # inclusive range of the obstacle count
    sigma: float = 0.8              # Gaussian disparity noise [px]
    p_invalid: float = 0.05         # fraction of pixels set to -1
    seed: int = 0


def generate_frame(spec: SceneSpec, return_labels: bool = False):
    """Render one frame.  With ``return_labels`` also return the noise-free
    disparity and a per-pixel class image (0 object, 1 ground, 2 sky)."""
    rng = np.random.default_rng(spec.seed)
    W, H = spec.width, spec.height
    cam = spec.camera
    f, B, Hc, hr = cam["focal_px"], cam["baseline_m"], cam["cam_height_m"], cam["horizon_row"]
    rows = np.arange(H, dtype=np.float64)[:, None]
    # ground: disparity grows linearly below the horizon, sky (0) above it
    ground = np.where(rows > hr, (B / Hc) * (rows - hr), 0.0) * np.ones((1, W))
    disp = ground.copy()
    label = np.where(rows > hr, 1, 2) * np.ones((1, W), dtype=np.int8)
    nb = int(rng.integers(spec.boxes[0], spec.boxes[1] + 1))
    for _ in range(nb):
        Z = rng.uniform(5.0, 60.0)
        d = f * B / Z
        r_b = hr + f * Hc / Z
        height_m = rng.uniform(0.5, 3.0)
        r_t = r_b - f * height_m / Z
        bw = rng.uniform(16.0, 160.0) * W / 1024.0
        c0 = rng.uniform(0.0, max(W - bw, 0.0))
        c_lo, c_hi = int(np.floor(c0)), int(np.ceil(c0 + bw))
        r_lo, r_hi = int(np.ceil(r_t)), int(np.floor(r_b))
        c_lo, c_hi = max(c_lo, 0), min(c_hi, W)
        r_lo, r_hi = max(r_lo, 0), min(r_hi, H - 1)
        if c_lo >= c_hi or r_lo > r_hi:
            continue
        win = disp[r_lo:r_hi + 1, c_lo:c_hi]
        closer = d >= win            # z-buffer: the larger disparity is in front
        win[closer] = d
        label[r_lo:r_hi + 1, c_lo:c_hi][closer] = 0
    clean = disp.copy()
    noisy = disp + spec.sigma * rng.standard_normal(disp.shape)
    noisy = np.clip(noisy, 0.0, spec.d_max - 1)
    invalid = rng.random(disp.shape) < spec.p_invalid
    noisy[invalid] = -1.0
    out = noisy.astype(np.float32)
    if return_labels:
        return out, clean.astype(np.float32), label
    return out


def workload_frame(name: str, index: int):
    """Frame ``index`` of a named workload.

    Returns ``(frame, info)`` where ``info`` holds width, height, d_max,
    stixel_width and the camera used to render it.
    """
    w = WORKLOADS[name]
    seed = w["seeds"][index % len(w["seeds"])]
    if name == "uneven256":
        rng = np.random.default_rng(seed)
        W, H = w["sizes"][int(rng.integers(len(w["sizes"])))]
        s = int(w["widths"][int(rng.integers(len(w["widths"])))])
        d_max = 256 if W == 2048 else 128
        cam = camera_for_size(W, H)
        sigma = float(rng.uniform(*w["sigma"]))
        p_inv = float(rng.uniform(*w["invalid"]))
        spec = SceneSpec(W, H, d_max, cam, w["boxes"], sigma, p_inv, seed)
    else:
        W, H = w["sizes"][0]
        s = int(w["widths"][index % len(w["widths"])]) if name != "hires16_2048x880" else int(w["widths"][0])
        d_max = int(w["d_max"])
        cam = camera_for_size(W, H)
        spec = SceneSpec(W, H, d_max, cam, w["boxes"], w["sigma"][0], w["invalid"][0], seed)
    info = dict(width=W, height=H, d_max=d_max, stixel_width=s, camera=cam, seed=seed)
    return generate_frame(spec), info


def generate_workload(name: str):
    """All frames of a named workload, as a list of ``(frame, info)``."""
    return [workload_frame(name, i) for i in range(WORKLOADS[name]["frames"])]


def random_columns_frame(seed: int, width: int, height: int, d_max: int,
                         p_invalid: float = 0.1):
    """Adversarial frame for parity testing: columns of assorted structure.

    Column strips are drawn from: uniform random disparities, piecewise
    constant runs, all-invalid strips, strips with NaN/inf/negative values,
    exact ground ramps and values beyond ``d_max`` (which clamp).
    """
    rng = np.random.default_rng(seed)
    out = np.empty((height, width), dtype=np.float32)
    for c in range(width):
        kind = int(rng.integers(7))
        if kind == 0:
            col = rng.uniform(0, d_max - 1, height)
        elif kind == 1:
            cuts = np.sort(rng.integers(0, height, int(rng.integers(1, 6))))
            vals = rng.uniform(0, d_max - 1, len(cuts) + 1)
            col = vals[np.searchsorted(cuts, np.arange(height), side="right")]
            col = col + 0.3 * rng.standard_normal(height)
        elif kind == 2:
            col = -np.ones(height)
        elif kind == 3:
            col = rng.uniform(0, d_max - 1, height)
            bad = rng.random(height)
            col[bad < 0.1] = np.nan
            col[(bad >= 0.1) & (bad < 0.15)] = np.inf
            col[(bad >= 0.15) & (bad < 0.2)] = -np.inf
            col[(bad >= 0.2) & (bad < 0.25)] = -3.5
        elif kind == 4:
            col = np.maximum(0.25 * (np.arange(height) - height * 0.4), 0.0)
        elif kind == 5:
            col = rng.uniform(0, 4 * d_max, height)
        else:
            col = np.round(rng.uniform(0, d_max - 1, height)) + 0.5  # exact .5 ties
        inv = rng.random(height) < p_invalid
        col = np.where(inv, -1.0, col)
        out[:, c] = col
    return out
