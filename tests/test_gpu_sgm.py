"""The semi-global matching stage on the GPU against the oracle, bit for bit
(integer arithmetic throughout): census words of both views, summed path
costs, the disparity map with its left-right check, several frames in one
call, the full 1024x440 size, the stereo pair -> stixels call, and the
degenerate cases (constant images, one-pixel images, widths below the
disparity range, zero penalties)."""

import numpy as np
import pytest

import oracle
from oracle import sgm as osgm
import synth
from synth.stereo import StereoSpec, generate_stereo
import paper_1610_04124_amd as P
from paper_1610_04124_amd import binding as B
from gpu_helpers import announce, assert_frames_equal, device

pytestmark = pytest.mark.gpu


def pair(W, H, D, seed, noise=1.0):
    cam = synth.camera_for_size(W, H)
    return generate_stereo(StereoSpec(synth.SceneSpec(W, H, D, cam, seed=seed), image_noise=noise))


def dev_u8(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint8)).to(device())


def run(m, left, right):
    import torch
    d = m.compute(dev_u8(left), dev_u8(right))
    torch.cuda.synchronize()
    return d.cpu().numpy()


@pytest.mark.parametrize("W,H,D", [(333, 121, 48), (260, 100, 128), (300, 80, 256)])
def test_census_costs_and_disparity_equal_oracle(W, H, D):
    left, right, _ = pair(W, H, D, seed=W + H)
    announce(f"sgm {W}x{H} D{D}")
    m = P.Sgm(W, H, D)
    got = run(m, left, right)
    want = osgm.disparity(left, right, D)
    cl, cr = osgm.census(left), osgm.census(right)
    assert np.array_equal(m.debug(B.SGM_LEFT_CENSUS, W, H), cl)
    assert np.array_equal(m.debug(B.SGM_RIGHT_CENSUS, W, H), cr)
    # the volume in HBM holds the top-down, bottom-up and right-to-left
    # terms; the left-to-right pass adds its own in registers
    three = sum(osgm.path(cl, cr, D, 10, 120, r).astype(np.int64) for r in (1, 2, 3))
    assert np.array_equal(m.debug(B.SGM_COSTS, W, H).astype(np.int64), three)
    assert np.array_equal(got, want)
    assert (got >= 0).mean() > 0.8
    m.close()


def test_several_frames_in_one_call():
    import torch
    W, H, D = 200, 72, 64
    pairs = [pair(W, H, D, seed=s) for s in (1, 2, 3)]
    L = dev_u8(np.stack([p[0] for p in pairs]))
    R = dev_u8(np.stack([p[1] for p in pairs]))
    announce("sgm 3 frames")
    m = P.Sgm(W, H, D, max_frames=3)
    got = m.compute(L, R)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    for i, (l, r, _) in enumerate(pairs):
        assert np.array_equal(got[i], osgm.disparity(l, r, D)), i
    m.close()


def test_full_size_frame():
    W, H, D = 1024, 440, 128
    left, right, truth = pair(W, H, D, seed=0)
    announce("sgm 1024x440 D128")
    m = P.Sgm(W, H, D)
    got = run(m, left, right)
    want = osgm.disparity(left, right, D)
    assert np.array_equal(got, want)
    seen = truth >= 0
    assert ((got == truth) & seen).sum() > 0.97 * seen.sum()
    m.close()


def test_stereo_pair_to_stixels_equals_oracle():
    import torch
    W, H, D = 640, 240, 128
    left, right, _ = pair(W, H, D, seed=5)
    cam = synth.camera_for_size(W, H)
    params = synth.make_params(camera=cam, max_width=W, max_height=H, max_disparity=D)
    h = P.Stixels(params)
    m = P.Sgm(W, H, D)
    announce("stereo -> stixels 640x240")
    out, disp = h.compute_stereo(m, dev_u8(left), dev_u8(right))
    torch.cuda.synchronize()
    want_disp = osgm.disparity(left, right, D)
    assert np.array_equal(disp.cpu().numpy(), want_disp)
    assert_frames_equal(out.to_host(), oracle.frame(params, want_disp), "stereo stixels")
    h.close()
    m.close()


@pytest.mark.parametrize("case", ["constant", "one_pixel", "narrow", "no_penalty"])
def test_degenerate_inputs(case):
    rng = np.random.default_rng(3)
    D, P1, P2 = 32, 10, 120
    if case == "constant":
        left = np.full((20, 40), 90, np.uint8)
        right = left.copy()
    elif case == "one_pixel":
        left = np.array([[7]], np.uint8)
        right = np.array([[200]], np.uint8)
    elif case == "narrow":                          # width below the disparity range
        left = rng.integers(0, 256, (30, 12), dtype=np.uint8)
        right = rng.integers(0, 256, (30, 12), dtype=np.uint8)
    else:
        left = rng.integers(0, 256, (25, 50), dtype=np.uint8)
        right = np.roll(left, -3, axis=1)
        P1 = P2 = 0
    H, W = left.shape
    announce(f"sgm degenerate {case}")
    m = P.Sgm(max(W, 8), max(H, 8), D, p1=P1, p2=P2)
    got = run(m, left, right)
    assert np.array_equal(got, osgm.disparity(left, right, D, P1, P2))
    m.close()


def test_bad_arguments_are_rejected():
    import torch
    for kw in [dict(max_disparity=30), dict(max_disparity=260), dict(p1=20, p2=10),
               dict(paths=8), dict(max_frames=0), dict(max_width=9000)]:
        args = dict(max_width=64, max_height=32, max_disparity=32, p1=10, p2=120, paths=4,
                    max_frames=1)
        args.update(kw)
        with pytest.raises(B.StixelsError):
            P.Sgm(**args)
    m = P.Sgm(64, 32, 32, max_frames=2)
    img = torch.zeros((3, 32, 64), dtype=torch.uint8, device=device())
    with pytest.raises(B.StixelsError):
        m.compute(img, img)                         # 3 frames > max_frames
    big = torch.zeros((32, 65), dtype=torch.uint8, device=device())
    with pytest.raises(B.StixelsError):
        m.compute(big, big)                         # wider than max_width
    m.close()
