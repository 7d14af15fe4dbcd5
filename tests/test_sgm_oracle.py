"""Pins of the semi-global matching oracle (the stereo stage upstream of the
stixel path) against what the definitions fix: the census transform by
impulses at every window offset, borders and ties; Hamming costs by Python's
bit counts; every path recurrence by the exhaustive minimum over all
disparity sequences along short paths; the selection by numpy's argmin; the
left-right check by hand-built cases; the whole stage by textured synthetic
pairs whose whole-pixel disparities are known."""

import itertools

import numpy as np
import pytest

import synth
from synth.stereo import StereoSpec, generate_stereo
from oracle import sgm


def bit_index(dy, dx):
    """Position of neighbour (dy, dx) in the row-major 9x7 window order that
    skips the centre."""
    k = (dy + 3) * 9 + (dx + 4)
    return k if k < 31 else k - 1


def test_census_constant_image_is_zero():
    assert not sgm.census(np.full((12, 15), 77, np.uint8)).any()


@pytest.mark.parametrize("dy", range(-3, 4))
def test_census_bit_order_by_impulses(dy):
    for dx in range(-4, 5):
        if dy == 0 and dx == 0:
            continue
        img = np.full((9, 11), 60, np.uint8)
        img[4, 5] = 50
        img[4 + dy, 5 + dx] = 40            # the one neighbour below the centre
        c = int(sgm.census(img)[4, 5])
        assert c == 1 << bit_index(dy, dx), (dy, dx, hex(c))


def test_census_comparison_is_strict_and_borders_read_zero():
    img = np.full((10, 10), 90, np.uint8)
    assert int(sgm.census(img)[5, 5]) == 0               # equal neighbours give 0
    img = np.full((10, 10), 10, np.uint8)
    img[0, 0] = 200
    c = int(sgm.census(img)[0, 0])
    inside = [(dy, dx) for dy in range(0, 4) for dx in range(0, 5) if (dy, dx) != (0, 0)]
    assert c == sum(1 << bit_index(dy, dx) for dy, dx in inside)
    assert bin(c).count("1") == 19


def test_costs_are_bit_counts():
    rng = np.random.default_rng(5)
    cl = rng.integers(0, 1 << 62, (6, 20), dtype=np.uint64)
    cr = rng.integers(0, 1 << 62, (6, 20), dtype=np.uint64)
    D = 9
    C = sgm.costs(cl, cr, D)
    for y in range(6):
        for x in range(20):
            for d in range(D):
                want = sgm.COST_OUT if x - d < 0 else (int(cl[y, x]) ^ int(cr[y, x - d])).bit_count()
                assert C[y, x, d] == want


def path_lines(H, W, dy, dx):
    """Every path of direction (dy, dx) as its list of pixels, first pixel
    first (a pixel whose predecessor lies outside the image starts one)."""
    lines = []
    for y in range(H):
        for x in range(W):
            if 0 <= y - dy < H and 0 <= x - dx < W:
                continue
            line, yy, xx = [], y, x
            while 0 <= yy < H and 0 <= xx < W:
                line.append((yy, xx))
                yy, xx = yy + dy, xx + dx
            lines.append(line)
    return lines


def penalty(a, b, P1, P2):
    return 0 if a == b else (P1 if abs(a - b) == 1 else P2)


@pytest.mark.parametrize("direction", range(8))
def test_path_is_the_minimum_over_disparity_sequences(direction):
    """L_r(p_t, d) = U_t(d) - min_k U_{t-1}(k), where U_t(d) is the smallest
    sum of costs and penalties over all disparity sequences along the path
    from its first pixel to p_t that end at d (L_r = U at the first pixel)."""
    rng = np.random.default_rng(100 + direction)
    H, W, D, P1, P2 = 5, 5, 3, 7, 25
    left = rng.integers(0, 256, (H, W), dtype=np.uint8)
    right = rng.integers(0, 256, (H, W), dtype=np.uint8)
    cl, cr = sgm.census(left), sgm.census(right)
    C = sgm.costs(cl, cr, D).astype(np.int64)
    L = sgm.path(cl, cr, D, P1, P2, direction).astype(np.int64)
    dy, dx = sgm.DIRECTIONS[direction]
    for line in path_lines(H, W, dy, dx):
        prev_min = None
        for t in range(len(line)):
            U = np.full(D, np.iinfo(np.int64).max)
            for seq in itertools.product(range(D), repeat=t + 1):
                v = sum(C[line[i]][seq[i]] for i in range(t + 1))
                v += sum(penalty(seq[i - 1], seq[i], P1, P2) for i in range(1, t + 1))
                U[seq[-1]] = min(U[seq[-1]], v)
            want = U if t == 0 else U - prev_min
            assert np.array_equal(L[line[t]], want), (direction, line[t], L[line[t]], want)
            prev_min = U.min()


def test_select_first_minimum_and_right_view_diagonal():
    rng = np.random.default_rng(9)
    H, W, D = 4, 13, 6
    S = rng.integers(0, 5, (H, W, D)).astype(np.uint16)      # many ties
    dL, dR = sgm.select(S)
    assert np.array_equal(dL, np.argmin(S, axis=2))
    for y in range(H):
        for x in range(W):
            n = min(D, W - x)
            diag = S[y, x + np.arange(n), np.arange(n)]
            assert dR[y, x] == int(np.argmin(diag))


def test_left_right_check_cases():
    dL = np.array([[0, 1, 2, 3, 2, 5]], np.int16)
    dR = np.array([[0, 3, 1, 0, 4, 0]], np.int16)
    got = sgm.check(dL, dR)
    # x=0: d 0, dR[0]=0 ok; x=1: d 1 -> dR[0]=0, |1-0|<=1 ok; x=2: d 2 -> dR[0]=0 fails;
    # x=3: d 3 -> dR[0]=0 fails; x=4: d 2 -> dR[2]=1 ok; x=5: d 5 -> dR[0]=0 fails
    assert got.tolist() == [[0.0, 1.0, -1.0, -1.0, 2.0, -1.0]]
    got = sgm.check(np.array([[4, 4]], np.int16), np.zeros((1, 2), np.int16))
    assert got.tolist() == [[-1.0, -1.0]]                   # x - d < 0


def stereo_pair(W, H, D, seed, noise=1.0):
    cam = synth.camera_for_size(W, H)
    spec = StereoSpec(synth.SceneSpec(W, H, D, cam, seed=seed), image_noise=noise)
    return generate_stereo(spec)


@pytest.mark.parametrize("npaths", [4, 8])
def test_textured_pairs_recover_the_known_disparity(npaths):
    left, right, truth = stereo_pair(256, 110, 48, seed=3)
    disp = sgm.disparity(left, right, 48, npaths=npaths)
    inner = np.zeros_like(truth, bool)
    inner[4:-4, 48:-5] = True
    seen = (truth >= 0) & inner
    correct = (disp == truth) & seen
    assert correct.sum() >= 0.93 * seen.sum(), correct.sum() / seen.sum()
    # what survives the left-right check is right almost everywhere
    kept = (disp >= 0) & seen
    assert (np.abs(disp - truth)[kept] <= 1).mean() >= 0.98


def test_disparity_equals_its_steps():
    left, right, _ = stereo_pair(96, 40, 24, seed=11)
    D, P1, P2 = 24, 10, 120
    disp, S = sgm.disparity(left, right, D, P1, P2, 8, return_costs=True)
    cl, cr = sgm.census(left), sgm.census(right)
    total = sum(sgm.path(cl, cr, D, P1, P2, r).astype(np.int64) for r in range(8))
    assert np.array_equal(S.astype(np.int64), total)
    dL, dR = sgm.select(S)
    assert np.array_equal(disp, sgm.check(dL, dR))


def test_bad_arguments_are_rejected():
    img = np.zeros((8, 8), np.uint8)
    with pytest.raises(ValueError):
        sgm.disparity(img, img, 16, npaths=5)
    with pytest.raises(ValueError):
        sgm.disparity(img, np.zeros((8, 9), np.uint8), 16)
