"""GPU parity of finer disparity bins (2^-k px; Sec. 3.4 rounds pixels and
object means to whole px, the variant resolves them finer): per-frame staged
and fused paths and a batch, against the oracle with the same bins, bit for
bit, both reductions."""

import numpy as np
import pytest

import oracle
import synth
import paper_1610_04124_amd as P
from gpu_helpers import announce, assert_frames_equal, gpu_frame, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,D,mode,path", [
    (1, 128, 0, 1), (1, 128, 1, 2), (2, 64, 0, 2), (3, 32, 1, 1), (1, 64, 0, 1),
])
def test_subpixel_frame_vs_oracle(k, D, mode, path):
    announce(f"subpixel k={k} D={D} mode={mode} path={path}")
    cam = synth.camera_for_size(1024, 440)
    p = synth.make_params(camera=cam, max_disparity=D, subpixel_log2=k, reduce_mode=mode)
    h = P.Stixels(p)
    h.set_frame_path(path)
    disp = synth.generate_frame(synth.SceneSpec(1024, 440, D, cam, seed=40 + k))
    got = gpu_frame(h, disp)
    ref = oracle.frame(p, disp)
    assert_frames_equal(got, ref, f"subpixel k={k}")
    # objects' means are bin indices: finer than whole px somewhere
    recs = np.concatenate([ref["records"][i, :ref["counts"][i]] for i in range(len(ref["counts"]))])
    obj = recs[recs["cls"] == 0]
    assert np.any(obj["disparity"] % (1 << k) != 0)


def test_subpixel_batch_with_whole_px_frames():
    """One launch over frames with 2^-1 px bins and frames with whole px."""
    announce("subpixel batch")
    import torch
    cam = synth.camera_for_size(1024, 440)
    p1 = synth.make_params(camera=cam, subpixel_log2=1, flags=1)
    p0 = synth.make_params(camera=cam, flags=1)
    h1, h0 = P.Stixels(p1), P.Stixels(p0)
    items, refs = [], []
    for i in range(6):
        p, h = (p1, h1) if i % 2 == 0 else (p0, h0)
        disp = synth.generate_frame(synth.SceneSpec(seed=500 + i))
        items.append((h, to_device(disp), h.new_output(1024, 440)))
        refs.append((p, disp))
    b = P.Batch(6, 6 * 204, 440, 256)
    b.compute(items)
    torch.cuda.synchronize()
    for i, ((_, _, out), (p, disp)) in enumerate(zip(items, refs)):
        assert_frames_equal(out.to_host(), oracle.frame(p, disp), f"subpixel batch job {i}")


@pytest.mark.parametrize("kw", [dict(), dict(subpixel_log2=1), dict(cost_grid_log2=6),
                                dict(max_disparity=256, max_width=2048, max_height=880)])
def test_online_object_costs_equal_offline_lut(kw):
    """Sec. 3.4: the staged table build with Eq. 4 evaluated online per
    (pixel, mean) gives the offline LUT's prefix tables and stixels bit for
    bit."""
    announce(f"online object LUT {kw}")
    W, H = kw.get("max_width", 1024), kw.get("max_height", 440)
    cam = synth.camera_for_size(W, H)
    p = synth.make_params(camera=cam, **{"max_width": W, "max_height": H, **kw})
    h = P.Stixels(p)
    h.set_frame_path(1)
    disp = synth.generate_frame(synth.SceneSpec(W, H, p["max_disparity"], cam, seed=70))
    off = gpu_frame(h, disp)
    po_off = h.debug_stage(3, W, H)
    h.set_object_lut(1)
    on = gpu_frame(h, disp)
    po_on = h.debug_stage(3, W, H)
    rng = h.debug_stage(2, W, H)
    for i in range(len(rng)):
        n = rng[i, 1] - rng[i, 0] + 1
        assert np.array_equal(po_on[i, :n], po_off[i, :n]), i
    assert_frames_equal(on, oracle.frame(p, disp), "online LUT")
    assert_frames_equal(off, oracle.frame(p, disp), "offline LUT")
