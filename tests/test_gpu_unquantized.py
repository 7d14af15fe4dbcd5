"""Costs off the grid (cost_grid_log2 = -1): FP32 tables and sums on the
device, FP64 in the oracle, so the two agree up to rounding.  The rule
(tolerances of the headline's parity contract):

  * every column total within 1e-4 relative of the oracle's C*;
  * where the stixel list equals the oracle's (boundaries, classes, means),
    every stixel cost within 1e-4 relative of the oracle's;
  * where it differs, the difference must be a near-tie: the device's list
    must be a valid segmentation (contiguous, legal transitions, ground at or
    below the horizon, object means equal to the rounded mean of their
    pixels) whose cost, evaluated in FP64 by direct sums over its pixels with
    each stixel's prior taken against its actual predecessor, lies within
    1e-5 relative of C*; its reported stixel costs must match those direct
    evaluations within 1e-4 relative.

The recurrence with stored links that these handles run is also checked bit
for bit on the grid: a batch mixing an exact handle with an off-grid one
runs the links kernel for both."""

import math

import numpy as np
import pytest

import oracle
import synth
import paper_1610_04124_amd as P
from bruteforce import GR, OB, Problem, stixel_cost
from gpu_helpers import announce, assert_frames_equal, gpu_frame, to_device

pytestmark = pytest.mark.gpu

REL_NEAR, REL_COST = 1e-5, 1e-4
TRANS_OK = None


def tol(x, rel):
    return rel * max(1.0, abs(x))


def check_off_grid(gpu, ref, params, disp):
    """Applies the rule above to every column; returns (columns, columns with
    a different list)."""
    H = disp.shape[0]
    q = oracle.reduce(params, disp)
    t = oracle.tables(params, H)
    T = params["model"]["trans_cost"]
    ncols = len(ref["counts"])
    differ = 0
    for i in range(ncols):
        cstar = float(ref["total"][i])
        assert abs(float(gpu["total"][i]) - cstar) <= tol(cstar, REL_COST), (i, gpu["total"][i], cstar)
        assert gpu["overflow"][i] == 0, i
        n, m = int(gpu["counts"][i]), int(ref["counts"][i])
        g, r = gpu["records"][i, :n], ref["records"][i, :m]
        same = n == m and all(np.array_equal(g[f], r[f]) for f in ("v_bottom", "v_top", "cls",
                                                                   "disparity"))
        if same:
            for a, b in zip(g["cost"], r["cost"]):
                assert abs(float(a) - float(b)) <= tol(float(b), REL_COST), (i, a, b)
            continue
        differ += 1
        pb = Problem(params, t, q[i])
        # valid segmentation, bottom-up, contiguous, covering the column
        assert int(g["v_bottom"][0]) == 0 and int(g["v_top"][-1]) == H - 1, i
        prev, total = None, 0.0
        for s in range(n):
            b, top, c, f = (int(g[k][s]) for k in ("v_bottom", "v_top", "cls", "disparity"))
            if s > 0:
                assert b == int(g["v_top"][s - 1]) + 1, (i, s)
                assert math.isfinite(T[prev[2]][c]), (i, s, "forbidden transition")
            if c == GR:
                assert top <= pb.vtop, (i, s, "ground above the horizon")
            cost, cur = stixel_cost(pb, prev, b, top, c)
            assert cur is not None and math.isfinite(cost), (i, s)
            if c == OB:
                assert f == cur[3], (i, s, "object mean")
            assert abs(float(g["cost"][s]) - cost) <= tol(cost, REL_COST), (i, s, g["cost"][s], cost)
            total += cost
            prev = cur
        assert abs(total - cstar) <= tol(cstar, REL_NEAR), (i, total, cstar, "not a near-tie")
    return ncols, differ


def off_grid_params(W=1024, H=440, D=128, **kw):
    cam = synth.camera_for_size(W, H)
    return synth.make_params(camera=cam, max_width=W, max_height=H, max_disparity=D,
                             cost_grid_log2=-1, **kw), cam


@pytest.mark.parametrize("seed,mode", [(0, 0), (1, 1)])
def test_off_grid_frame_1024x440(seed, mode):
    announce(f"off-grid frame seed={seed} mode={mode}")
    p, cam = off_grid_params(reduce_mode=mode)
    h = P.Stixels(p)
    assert h.frame_path() == 2
    disp = synth.generate_frame(synth.SceneSpec(seed=seed))
    cols, differ = check_off_grid(gpu_frame(h, disp), oracle.frame(p, disp), p, disp)
    print(f"off-grid seed {seed}: {differ} of {cols} columns differ by a near-tie")


def test_off_grid_frame_2048x880():
    announce("off-grid frame 2048x880")
    p, cam = off_grid_params(2048, 880, 256, stixel_width=5)
    h = P.Stixels(p)
    disp = synth.generate_frame(synth.SceneSpec(2048, 880, 256, cam, seed=9))
    cols, differ = check_off_grid(gpu_frame(h, disp), oracle.frame(p, disp), p, disp)
    print(f"off-grid 2048x880: {differ} of {cols} columns differ by a near-tie")


def test_links_kernel_is_exact_on_the_grid():
    """A batch with one off-grid job runs the links kernel for every job: the
    on-grid jobs must still equal the oracle bit for bit, the off-grid one
    must satisfy the rule."""
    announce("links kernel on the grid")
    import torch
    cam = synth.camera_for_size(1024, 440)
    pe = synth.make_params(camera=cam, flags=1)
    po, _ = off_grid_params(flags=1)
    he, ho = P.Stixels(pe), P.Stixels(po)
    items, refs = [], []
    for i in range(5):
        p, h = (po, ho) if i == 2 else (pe, he)
        disp = synth.generate_frame(synth.SceneSpec(seed=600 + i))
        items.append((h, to_device(disp), h.new_output(1024, 440)))
        refs.append((p, disp))
    b = P.Batch(5, 5 * 204, 440, 128)
    b.set_waves(2)          # ignored: the links kernel runs one wave per column
    b.compute(items)
    torch.cuda.synchronize()
    assert b.waves() == 1
    for i, ((_, _, out), (p, disp)) in enumerate(zip(items, refs)):
        got, ref = out.to_host(), oracle.frame(p, disp)
        if i == 2:
            check_off_grid(got, ref, p, disp)
        else:
            assert_frames_equal(got, ref, f"links kernel, exact job {i}")


def test_off_grid_adversarial_columns():
    """Ragged sizes, invalid strips, exact .5 values and ground ramps."""
    announce("off-grid adversarial")
    for (W, H, s, D, seed) in ((203, 129, 3, 64, 11), (97, 300, 7, 256, 12), (64, 65, 1, 16, 13)):
        cam = dict(synth.CAMERA_1024x440, horizon_row=float(seed * 7 % H))
        p = synth.make_params(camera=cam, stixel_width=s, max_disparity=D, max_width=W,
                              max_height=H, cost_grid_log2=-1)
        h = P.Stixels(p)
        disp = synth.random_columns_frame(seed, W, H, D)
        check_off_grid(gpu_frame(h, disp), oracle.frame(p, disp), p, disp)
