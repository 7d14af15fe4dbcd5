"""Serving on the GPU: 8 camera streams (1024x440, 1280x720, 2048x880, stixel
width 5) with Poisson arrivals, continuous batching over three streams.
Every served frame equals the same frame computed alone, bit for bit."""

import numpy as np
import pytest

import synth
from gpu_helpers import announce, to_device
import paper_1610_04124_amd as P
from paper_1610_04124_amd.serving import (GpuExecutor, Server, poisson_arrivals, serving_cameras,
                                          serving_params)

pytestmark = pytest.mark.gpu


def test_served_frames_equal_alone():
    import torch
    announce("serving 8 cameras")
    cams = serving_cameras(8)
    per_cam = 3
    frames = {}
    for c, cam in enumerate(cams):
        W, H, D = cam.width, cam.height, cam.handle.D
        for i in range(per_cam):
            disp = synth.generate_frame(synth.SceneSpec(W, H, D, synth.camera_for_size(W, H),
                                                        seed=1000 * c + i))
            frames[(c, i)] = to_device(disp)
    # alone: the per-frame path of a handle with the camera's parameters (the
    # serving handles are batch-only)
    solo = [P.Stixels(serving_params(c, batch_only=False)) for c in range(len(cams))]
    alone = {}
    for (c, i), f in frames.items():
        alone[(c, i)] = solo[c].compute(f)
    torch.cuda.synchronize()
    key_of = {f.data_ptr(): k for k, f in frames.items()}

    ex = GpuExecutor(cams, streams=3, max_frames=32)
    srv = Server(cams, ex, hbm_budget=8 << 30, max_batch=32)
    arrivals = poisson_arrivals([600.0] * 8, 0.4, [42 + c for c in range(8)], per_cam)
    srv.run_trace(arrivals, lambda c, i: frames[(c, i)])
    torch.cuda.synchronize()
    st = srv.stats()
    assert st["completed"] == len(arrivals) and st["rejected"] == 0
    assert st["frames_per_launch"] > 1.0
    for r in srv.completed:
        ref = alone[key_of[r.frame.data_ptr()]]
        for name in ("counts", "records", "total", "overflow"):
            assert torch.equal(getattr(r.out, name), getattr(ref, name)), (r.rid, name)
    assert all(r.latency > 0 for r in srv.completed)
