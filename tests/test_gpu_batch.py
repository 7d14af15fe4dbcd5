"""GPU parity of the persistent batched launch: against the oracle, against
the per-frame path (bitwise), across uneven frame sizes / stixel widths /
cameras, across workgroup counts, and through HIP graph replays."""

import numpy as np
import pytest

import oracle
import synth
import paper_1610_04124_amd as P
from gpu_helpers import announce, assert_frames_equal, device, gpu_frame, to_device

pytestmark = pytest.mark.gpu


def frame_setup(n, seeds=None):
    p = synth.make_params()
    h = P.Stixels(p)
    seeds = seeds if seeds is not None else list(range(n))
    frames = [synth.generate_frame(synth.SceneSpec(seed=s)) for s in seeds]
    return p, h, frames


def run_batch(items, workgroups=0, max_h=440, max_d=128, waves=1, columns=1):
    import torch
    b = P.Batch(len(items), sum(h.num_columns(d.shape[1]) for h, d, _ in items), max_h, max_d,
                workgroups)
    b.set_waves(waves)
    b.set_columns(columns)
    b.compute(items)
    torch.cuda.synchronize()
    assert b.waves() == waves
    assert b.columns() == columns
    return b


def test_batch64_matches_oracle_and_per_frame():
    """64 frames of 1024x440, stixel width 5 (the batched headline workload)."""
    import torch
    announce("batch 64 x 1024x440")
    p, h, frames = frame_setup(64)
    dev = device()
    outs = [h.new_output(1024, 440) for _ in frames]
    items = [(h, to_device(f), o) for f, o in zip(frames, outs)]
    b = run_batch(items)
    g, t = b.info()
    assert t == 64 * 204 and g >= 1
    for i in (0, 17, 63):
        assert_frames_equal(outs[i].to_host(), oracle.frame(p, frames[i]), f"batch frame {i}")
    for i, f in enumerate(frames):
        assert_frames_equal(outs[i].to_host(), gpu_frame(h, f), f"batch vs per-frame {i}")


@pytest.mark.parametrize("waves", [2, 4])
def test_batch_waves_match_per_frame(waves):
    """16 frames of 1024x440 with several wavefronts per column: bitwise
    equal to the one-wave per-frame path."""
    announce(f"batch 16 x 1024x440 waves={waves}")
    p, h, frames = frame_setup(16)
    outs = [h.new_output(1024, 440) for _ in frames]
    items = [(h, to_device(f), o) for f, o in zip(frames, outs)]
    run_batch(items, waves=waves)
    for i, f in enumerate(frames):
        assert_frames_equal(outs[i].to_host(), gpu_frame(h, f, waves=1), f"waves {waves} frame {i}")
    assert_frames_equal(outs[3].to_host(), oracle.frame(p, frames[3]), "oracle frame 3")


def test_batch_mean_reduction_matches_oracle():
    """The paper's mean reduction (reduce_mode 1) through the batched launch
    at the headline size."""
    announce("batch 8 x 1024x440 mean reduction")
    p = synth.make_params(reduce_mode=1)
    h = P.Stixels(p)
    frames = [synth.generate_frame(synth.SceneSpec(seed=s)) for s in range(40, 48)]
    outs = [h.new_output(1024, 440) for _ in frames]
    run_batch([(h, to_device(f), o) for f, o in zip(frames, outs)])
    for i in (0, 5):
        assert_frames_equal(outs[i].to_host(), oracle.frame(p, frames[i]), f"mean frame {i}")
    for i, f in enumerate(frames):
        assert_frames_equal(outs[i].to_host(), gpu_frame(h, f), f"mean batch vs per-frame {i}")


def test_batch_two_columns_per_wave_matches_per_frame():
    """Two columns of a frame per wave64 (one per 32-lane half): bitwise equal
    to the per-frame path, with even (204) and odd (341) column counts."""
    announce("batch two columns per wave")
    p, h, frames = frame_setup(12)
    outs = [h.new_output(1024, 440) for _ in frames]
    run_batch([(h, to_device(f), o) for f, o in zip(frames, outs)], columns=2)
    for i, f in enumerate(frames):
        assert_frames_equal(outs[i].to_host(), gpu_frame(h, f), f"pairs frame {i}")
    assert_frames_equal(outs[7].to_host(), oracle.frame(p, frames[7]), "pairs oracle frame 7")
    p3 = synth.make_params(stixel_width=3)
    h3 = P.Stixels(p3)
    outs3 = [h3.new_output(1024, 440) for _ in frames[:4]]
    run_batch([(h3, to_device(f), o) for f, o in zip(frames[:4], outs3)], columns=2)
    for i, f in enumerate(frames[:4]):
        assert h3.num_columns(1024) % 2 == 1
        assert_frames_equal(outs3[i].to_host(), oracle.frame(p3, f), f"pairs s=3 frame {i}")


@pytest.mark.parametrize("H", [1, 31, 32, 33, 63, 64, 65, 95, 129, 257, 300, 511, 512])
def test_batch_two_columns_per_wave_heights(H):
    """Heights around the 32-row slot boundaries, adversarial columns, odd
    and even column counts."""
    announce(f"pairs height {H}")
    W = 5 * (7 + H % 4)
    cam = dict(synth.CAMERA_1024x440, horizon_row=float((H * 7) // 10))
    p = synth.make_params(camera=cam, stixel_width=5, max_disparity=128, max_width=W,
                          max_height=H)
    h = P.Stixels(p)
    disps = [synth.random_columns_frame(100 + H + i, W, H, 128) for i in range(3)]
    outs = [h.new_output(W, H) for _ in disps]
    run_batch([(h, to_device(d), o) for d, o in zip(disps, outs)], max_h=H, columns=2)
    for i, d in enumerate(disps):
        assert_frames_equal(outs[i].to_host(), oracle.frame(p, d), f"pairs H={H} frame {i}")


def uneven_items(n):
    """Frames of the uneven workload: four sizes, stixel widths 3/5/7, their
    own cameras and disparity ranges, one handle per frame."""
    items, refs = [], []
    for i in range(n):
        disp, info = synth.workload_frame("uneven256", i)
        W, H = info["width"], info["height"]
        p = synth.make_params(camera=info["camera"], stixel_width=info["stixel_width"],
                              max_disparity=info["d_max"], max_width=W, max_height=H)
        h = P.Stixels(p)
        items.append((h, to_device(disp), h.new_output(W, H)))
        refs.append((p, disp))
    return items, refs


@pytest.mark.parametrize("workgroups,waves", [(0, 1), (7, 1), (0, 2), (5, 4)])
def test_uneven_batch_matches_oracle(workgroups, waves):
    announce(f"uneven batch workgroups={workgroups} waves={waves}")
    items, refs = uneven_items(10)
    run_batch(items, workgroups, max_h=880, max_d=256, waves=waves)
    for i, ((h, d, out), (p, disp)) in enumerate(zip(items, refs)):
        assert_frames_equal(out.to_host(), oracle.frame(p, disp), f"uneven frame {i}")


def test_uneven256_every_frame_in_one_launch():
    """The whole uneven workload (256 frames, four sizes, stixel widths 3/5/7,
    own camera and disparity range per size) in one persistent launch: every
    frame bitwise equal to the same frame through the per-frame path, and one
    frame of every (size, stixel width) pair equal to the oracle."""
    import torch
    announce("uneven256: 256 frames in one launch vs per frame; oracle per size x width")
    handles, items, infos = {}, [], []
    for i in range(256):
        disp, info = synth.workload_frame("uneven256", i)
        W, H, s = info["width"], info["height"], info["stixel_width"]
        key = (W, H, s, info["d_max"])
        if key not in handles:
            p = synth.make_params(camera=info["camera"], stixel_width=s,
                                  max_disparity=info["d_max"], max_width=W, max_height=H)
            handles[key] = (P.Stixels(p), p)
        h, p = handles[key]
        items.append((h, to_device(disp), h.new_output(W, H)))
        infos.append((key, p, disp))
    b = run_batch(items, 0, max_h=880, max_d=256)
    assert b.info()[1] == sum(h.num_columns(d.shape[1]) for h, d, _ in items)
    checked = set()
    for i, ((h, d, out), (key, p, disp)) in enumerate(zip(items, infos)):
        alone = h.new_output(key[0], key[1])
        h.compute(d, alone)
        torch.cuda.synchronize()
        got = out.to_host()
        assert_frames_equal(got, alone.to_host(), f"uneven256 frame {i} vs per frame")
        if key[:3] not in checked:
            checked.add(key[:3])
            assert_frames_equal(got, oracle.frame(p, disp), f"uneven256 frame {i} vs oracle")
    sizes = {(k[0], k[1]) for k in checked}
    assert len(sizes) == 4 and len({k[2] for k in checked}) == 3, checked


def test_graph_replays_are_stable_and_follow_inputs():
    """Capture once, replay several times with eager work and syncs between
    the replays; each replay equals the per-frame result of the inputs it
    saw, including after the inputs are rewritten in place."""
    import torch
    announce("graph replay")
    p, h, frames = frame_setup(8)
    dev_frames = [to_device(f) for f in frames]
    outs = [h.new_output(1024, 440) for _ in frames]
    items = list(zip([h] * 8, dev_frames, outs))
    b = P.Batch(8, 8 * 204, 440, 128)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    b.capture(items, stream)
    expect = [gpu_frame(h, f) for f in frames]
    for rep in range(3):
        for o in outs:
            o.counts.fill_(-1)
        torch.cuda.synchronize()
        b.replay(stream)
        torch.cuda.synchronize()
        _ = torch.ones(1024, device=dev_frames[0].device).sum().item()   # eager work between replays
        for i in range(8):
            assert_frames_equal(outs[i].to_host(), expect[i], f"replay {rep} frame {i}")
    # rewrite the inputs in place: the graph reads the same buffers
    new = [synth.generate_frame(synth.SceneSpec(seed=100 + i)) for i in range(8)]
    for df, nf in zip(dev_frames, new):
        df.copy_(torch.from_numpy(nf))
    torch.cuda.synchronize()
    b.replay(stream)
    torch.cuda.synchronize()
    for i in range(8):
        assert_frames_equal(outs[i].to_host(), gpu_frame(h, new[i]), f"new input frame {i}")


def test_batch_limits_are_enforced():
    announce("batch limits")
    p, h, frames = frame_setup(3)
    items = [(h, to_device(f), h.new_output(1024, 440)) for f in frames]
    b = P.Batch(2, 10000, 440, 128)
    with pytest.raises(P.StixelsError):
        b.compute(items)                      # more jobs than max_jobs
    b = P.Batch(3, 300, 440, 128)
    with pytest.raises(P.StixelsError):
        b.compute(items)                      # more columns than max_tasks
    b = P.Batch(3, 1000, 400, 128)
    with pytest.raises(P.StixelsError):
        b.compute(items)                      # taller than the batch's max_height
    with pytest.raises(P.StixelsError):
        P.Batch(1, 1, 440, 128).replay()      # nothing captured
    with pytest.raises(P.StixelsError):
        b.capture(items[:1], None)            # the null stream cannot be captured
