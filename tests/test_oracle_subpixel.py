"""Pins of the oracle's sub-pixel disparity bins (disparities resolved to
2^-subpixel_log2 px; a reading of the scope's finer-bin variant, the paper
itself rounds to whole px, Sec. 3.4).  Each function is pinned to an
independent computation: numpy's sort and fsum for the reduction, scipy's
normal distribution for every table entry at the bins' disparities, the
exhaustive search and the naive recurrence for the dynamic programme."""

import math

import numpy as np
import pytest

import oracle
import synth
from bruteforce import Problem, c_map
from naive_dp import NaiveColumn
from test_oracle_exhaustive import grid_value, random_model, scipy_cost
from test_oracle_pins import dp_path, random_column


@pytest.fixture(scope="module")
def build_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("bruteforce_subpixel"))


@pytest.mark.parametrize("sp", [1, 2, 3])
@pytest.mark.parametrize("mode", [0, 1])
def test_reduce_in_bins(sp, mode):
    rng = np.random.default_rng(10 * sp + mode)
    s, H, W, Dpx = 5, 30, 53, 32
    disp = (rng.integers(0, Dpx * 64 + 40, (H, W)) / 64.0).astype(np.float32)   # exact sums
    disp[rng.random((H, W)) < 0.15] = -1
    disp[3] = np.float32(5.0 + 0.5 ** (sp + 1))          # exact half-bin ties
    p = synth.make_params(stixel_width=s, max_disparity=Dpx, reduce_mode=mode, subpixel_log2=sp)
    q = oracle.reduce(p, disp)
    nb = Dpx << sp
    for i in range(W // s):
        for r in range(H):
            vals = [float(x) for x in disp[r, i * s:(i + 1) * s] if x >= 0]
            if not vals:
                exp = -1
            else:
                m = np.sort(vals)[(len(vals) - 1) // 2] if mode == 0 else math.fsum(vals) / len(vals)
                exp = int(min(np.rint(m * 2 ** sp), nb - 1))
            assert q[i, H - 1 - r] == exp


@pytest.mark.parametrize("sp", [1, 2])
def test_tables_in_bins_against_scipy(sp):
    W, H, D = 640, 240, 64
    cam = dict(synth.camera_for_size(W, H), pitch_rad=0.01)
    m = dict(synth.DEFAULT_MODEL)
    p = synth.make_params(camera=cam, model=m, max_disparity=D, max_width=W, max_height=H,
                          subpixel_log2=sp)
    t = oracle.tables(p, H)
    nb = D << sp
    assert t["S"].shape == (nb,) and t["O"].shape == (nb, nb) and t["G"].shape == (H, nb)
    g = p["cost_grid_log2"]
    pout, sd = m["p_out"], m["sigma_disp"]
    alpha = cam["baseline_m"] * math.cos(cam["pitch_rad"]) / cam["cam_height_m"]
    v_hor = (H - 1) - cam["horizon_row"]
    px = lambda i: i / 2.0 ** sp  # noqa: E731
    rng = np.random.default_rng(sp)
    for d in range(nb):
        want = grid_value(scipy_cost(px(d), 0.0, m["sigma_sky"], pout, D), g)
        if want is not None:
            assert t["S"][d] == want
    for v in rng.integers(0, int(v_hor) + 1, 12):
        mu = alpha * (v_hor - int(v))
        sg = math.sqrt(sd * sd + (m["ground_slope_noise"] * mu) ** 2)
        for d in range(0, nb, 3):
            want = grid_value(scipy_cost(px(d), mu, sg, pout, D), g)
            if want is not None:
                assert t["G"][int(v)][d] == want
    for f in rng.integers(0, nb, 10):
        f = int(f)
        so = math.sqrt(sd * sd + (px(f) ** 2 * m["object_depth_extent_m"]
                                  / (cam["focal_px"] * cam["baseline_m"])) ** 2)
        for d in range(0, nb, 3):
            want = grid_value(scipy_cost(px(d), px(f), so, pout, D), g)
            if want is not None:
                assert t["O"][d][f] == want
    # thresholds in bins: floor / ceil of (ground disparity +- tolerance) * 2^sp
    for b in range(0, H + 1, 7):
        fg = alpha * (v_hor - b)
        assert t["fg_hi"][b] == math.floor((fg + m["diving_tol_px"]) * 2 ** sp)
        assert t["fg_lo"][b] == math.ceil((fg - m["gravity_tol_px"]) * 2 ** sp)


def small_params_bins(sp, ordering, horizon, grid=10, D=16, model=None):
    cam = dict(focal_px=700.0, baseline_m=1.2, cam_height_m=0.3, horizon_row=horizon,
               pitch_rad=0.0)
    m = dict(model or synth.DEFAULT_MODEL)
    if not ordering:
        m["ordering_cost"] = 0.0
    return synth.make_params(camera=cam, model=m, max_disparity=D, max_height=16,
                             cost_grid_log2=grid, subpixel_log2=sp)


@pytest.mark.parametrize("sp", [1, 2])
@pytest.mark.parametrize("H", [9, 11])
def test_dp_in_bins_equals_exhaustive_map(build_dir, sp, H):
    rng = np.random.default_rng(100 * sp + H)
    for horizon in (0.0, float(H) / 2):
        for grid in (10, 0):
            p = small_params_bins(sp, False, horizon, grid)
            t = oracle.tables(p, H)
            for _ in range(3):
                q = random_column(rng, H, 16 << sp)
                res = oracle.column(p, q)
                best, lst, _, _ = c_map(build_dir, Problem(p, t, q))
                assert res["total"] == best
                assert dp_path(res) == [tuple(x) for x in lst]


@pytest.mark.parametrize("sp", [1, 2])
def test_naive_recurrence_in_bins(sp):
    """Every prior term on, the ordering tolerance in bins."""
    rng = np.random.default_rng(7 + sp)
    for case in range(40):
        H = int(rng.integers(1, 33))
        m = random_model(rng)
        p = small_params_bins(sp, True, float(rng.integers(-2, H + 2)), int(rng.choice([10, 0])),
                              D=16, model=m)
        q = random_column(rng, H, 16 << sp)
        t = oracle.tables(p, H)
        ref = NaiveColumn(p, t, q).solve()
        got = oracle.column(p, q)
        assert np.array_equal(got["C"], np.array(ref["C"])), case
        assert np.array_equal(got["fob"], np.array(ref["fob"])), case
        assert dp_path(got) == [(b, k, c, f) for b, k, c, f, _ in ref["stixels"]], case


def test_whole_px_is_one_bin():
    """subpixel_log2 = 0 is the whole-pixel method, bit for bit."""
    disp = synth.generate_frame(synth.SceneSpec(seed=4))
    a = oracle.frame(synth.make_params(), disp)
    b = oracle.frame(synth.make_params(subpixel_log2=0), disp)
    for k in ("counts", "records", "total", "overflow"):
        assert np.array_equal(a[k], b[k])
