"""Seeded synthetic rectified stereo pairs of the road scenes.

The disparity stage upstream of the stixel path (semi-global matching, cited
by the paper as its real-time source of disparity maps) needs image pairs.
They are rendered here from the same ground-plus-box scenes as the disparity
maps in ``scenes.py``: every surface is fronto-parallel along an image row
(the ground's disparity is constant along a row, the boxes face the camera),
so with whole-pixel disparities the right view is an exact warp of the left
one.  This module only renders images; it holds none of the matching
arithmetic.

Every image is uint8 of shape (height, width), row 0 at the top.  The right
image is the view from the camera one baseline to the right: the left pixel
(r, c) of disparity d appears at (r, c - d).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .scenes import SceneSpec, generate_frame


@dataclass
class StereoSpec:
    scene: SceneSpec
    image_noise: float = 1.0        # Gaussian noise added to both images [gray levels]
    sky_texture: float = 24.0       # amplitude of the sky's (weak) texture


def _texture(rng, shape, lo, hi):
    """Random texture: uniform noise averaged over 2x2 blocks of pixels."""
    t = rng.uniform(lo, hi, (shape[0] + 1, shape[1] + 1))
    return 0.25 * (t[:-1, :-1] + t[1:, :-1] + t[:-1, 1:] + t[1:, 1:])


def generate_stereo(spec: StereoSpec):
    """Render a stereo pair.

    Returns ``(left, right, truth)``: uint8 images and the whole-pixel
    disparity of every left pixel (int16), -1 where the left pixel is not
    seen by the right camera (it leaves the image, or a nearer surface covers
    it there)."""
    sc = spec.scene
    _, clean, label = generate_frame(sc, return_labels=True)
    H, W = clean.shape
    d = np.clip(np.rint(clean), 0, sc.d_max - 1).astype(np.int64)
    rng = np.random.default_rng(10_000_019 + sc.seed)
    left = _texture(rng, (H, W), 20.0, 235.0)
    sky = label == 2
    left[sky] = 128.0 + _texture(rng, (H, W), -spec.sky_texture, spec.sky_texture)[sky]

    # right view: the nearest left pixel that lands on each right column
    right = _texture(rng, (H, W), 20.0, 235.0)      # what only the right camera sees
    best = np.full((H, W), -1, np.int64)            # disparity of the visible left pixel
    src = np.full((H, W), -1, np.int64)
    cols = np.arange(W)
    for r in range(H):
        x = cols - d[r]
        ok = x >= 0
        # visit in increasing disparity so that the nearest surface is written last
        order = np.argsort(d[r][ok], kind="stable")
        cs, xs = cols[ok][order], x[ok][order]
        best[r, xs] = d[r, cs]
        src[r, xs] = cs
    seen = src >= 0
    rr, xx = np.nonzero(seen)
    right[rr, xx] = left[rr, src[rr, xx]]

    truth = np.full((H, W), -1, np.int16)
    for r in range(H):
        c = cols
        x = c - d[r]
        ok = x >= 0
        vis = np.zeros(W, bool)
        vis[ok] = src[r, x[ok]] == c[ok]
        truth[r, vis] = d[r, vis]

    def quantise(img):
        img = img + spec.image_noise * rng.standard_normal(img.shape)
        return np.clip(np.rint(img), 0, 255).astype(np.uint8)

    return quantise(left), quantise(right), truth
