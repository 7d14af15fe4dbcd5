"""GPU parity of the per-frame fused path (stixels_compute as one launch of the
persistent kernel), of the one-call batch (stixels_compute_batch) and of the
table and size queries added with them, against the CPU oracle and against
the staged per-frame path, bit for bit."""

import numpy as np
import pytest

import oracle
import synth
import paper_1610_04124_amd as P
from paper_1610_04124_amd import binding as B
from gpu_helpers import announce, assert_frames_equal, device, gpu_frame, to_device

pytestmark = pytest.mark.gpu


def handle_for(W, H, s=5, D=128, **kw):
    cam = kw.pop("camera", None) or synth.camera_for_size(W, H)
    p = synth.make_params(camera=cam, stixel_width=s, max_disparity=D, max_width=W,
                          max_height=H, **kw)
    return p, P.Stixels(p)


def fused_frame(h, disp, waves=None, capacity=None):
    h.set_frame_path(2)
    try:
        return gpu_frame(h, disp, capacity=capacity, waves=waves)
    finally:
        h.set_frame_path(0)


@pytest.mark.parametrize("seed,waves", [(0, 1), (1, 2), (2, 4)])
def test_fused_frame_1024x440(seed, waves):
    announce(f"fused frame 1024x440 seed={seed} waves={waves}")
    p, h = handle_for(1024, 440)
    assert h.frame_path() == 1
    disp = synth.generate_frame(synth.SceneSpec(seed=seed))
    got = fused_frame(h, disp, waves=waves)
    assert_frames_equal(got, oracle.frame(p, disp), f"fused seed {seed} waves {waves}")
    assert_frames_equal(got, gpu_frame(h, disp), "fused vs staged")


def fused_cases():
    rng = np.random.default_rng(4040)
    out = []
    for H in (1, 2, 63, 64, 65, 129, 300, 513, 880, 1024):
        s = int(rng.choice([1, 3, 5, 7, 16]))
        W = int(s * rng.integers(1, 30) + rng.integers(0, s))
        D = int(rng.choice([16, 128, 256]))
        out.append((W, H, s, D, int(rng.integers(0, 2)), int(rng.integers(1 << 30))))
    return out


@pytest.mark.parametrize("W,H,s,D,mode,seed", fused_cases())
def test_fused_frame_adversarial(W, H, s, D, mode, seed):
    """Heights around the slot boundaries up to the maximum, ragged widths,
    every kind of invalid pixel, both reductions, d_range up to 256."""
    announce(f"fused adversarial W={W} H={H} s={s} D={D} mode={mode} seed={seed}")
    cam = dict(synth.CAMERA_1024x440, horizon_row=float(seed % max(H, 1)))
    p, h = handle_for(W, H, s=s, D=D, reduce_mode=mode, camera=cam)
    disp = synth.random_columns_frame(seed, W, H, D)
    assert_frames_equal(fused_frame(h, disp), oracle.frame(p, disp), f"fused {W}x{H}")


def test_fused_frame_capacity_and_reuse():
    announce("fused capacity")
    p, h = handle_for(1024, 440)
    disp = synth.generate_frame(synth.SceneSpec(seed=7))
    for cap in (1, 3):
        assert_frames_equal(fused_frame(h, disp, capacity=cap), oracle.frame(p, disp, cap=cap),
                            f"fused cap {cap}")
    # a narrower frame on the same handle after a wider one
    small = disp[:, :333]
    assert_frames_equal(fused_frame(h, small), oracle.frame(p, small), "fused narrower")


def test_debug_stage_needs_the_staged_path():
    announce("debug stage after fused")
    p, h = handle_for(200, 100)
    disp = synth.random_columns_frame(1, 200, 100, 128)
    fused_frame(h, disp)
    with pytest.raises(B.StixelsError):
        h.debug_stage(B.STAGE_REDUCED, 200, 100)
    gpu_frame(h, disp)
    assert h.debug_stage(B.STAGE_REDUCED, 200, 100).shape == (40, 100)


def test_compute_batch_one_call_grows():
    """stixels_compute_batch: uneven frames of several cameras in one call,
    then a bigger call on the same first handle (the internal batch grows)."""
    import torch
    announce("compute_batch one call")
    items, refs = [], []
    for i in range(6):
        disp, info = synth.workload_frame("uneven256", i)
        W, H = info["width"], info["height"]
        p = synth.make_params(camera=info["camera"], stixel_width=info["stixel_width"],
                              max_disparity=info["d_max"], max_width=W, max_height=H)
        h = P.Stixels(p)
        items.append((h, to_device(disp), h.new_output(W, H)))
        refs.append((p, disp))
    P.compute_batch(items[:2])
    torch.cuda.synchronize()
    for (h, d, out), (p, disp) in zip(items[:2], refs[:2]):
        assert_frames_equal(out.to_host(), oracle.frame(p, disp), "compute_batch small")
    first = items[0]
    bigger = [first] + items[2:]
    P.compute_batch(bigger)
    torch.cuda.synchronize()
    for (h, d, out), (p, disp) in zip(bigger, [refs[0]] + refs[2:]):
        assert_frames_equal(out.to_host(), oracle.frame(p, disp), "compute_batch grown")


def test_debug_tables_and_output_bytes():
    announce("debug tables, output bytes")
    p, h = handle_for(1024, 440)
    allt = h.debug_tables()
    for which in range(5):
        assert np.array_equal(allt[which], h.debug_table(which))
    ncols, cap = 204, 440
    assert h.output_bytes(1024, 440) == ncols * (4 + 12 * cap + 4 + 1)
    with pytest.raises(B.StixelsError):
        h.output_bytes(4, 440)


def test_binding_rejects_mismatched_outputs():
    announce("binding output checks")
    p, h = handle_for(1024, 440)
    disp = to_device(synth.generate_frame(synth.SceneSpec(seed=1)))
    wrong = h.new_output(1000, 440)            # 200 columns, the frame has 204
    with pytest.raises(B.StixelsError):
        h.compute(disp, wrong)
    with pytest.raises(B.StixelsError):
        P.Batch(1, 204, 440, 128).compute([(h, disp, wrong)])
