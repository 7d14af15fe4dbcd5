"""Further pins of the CPU FP64 oracle, each against a computation that shares
nothing with it.

* Offline tables (Sec. 3.4, Eq. 4) against scipy's normal distribution:
  every entry of the sky, ground and object tables, with the per-class
  standard deviations written out here.
* The recurrence (Eq. 5-6) against exhaustive search (Eq. 1-2) over every
  segmentation of 9-12-row columns (tests/bruteforce_enum.c: direct sums,
  integer means).  Ordering prior off: exact MAP, so the cost and the first
  optimum in the tie order must agree exactly.  Ordering prior on: the
  recurrence charges the penalty against the stored best object stixel and
  is not MAP; its cost is the true cost of the list it returns and never
  below the MAP.
* The recurrence with every prior term on against a naive Python
  re-implementation of Eq. 5-6 (tests/naive_dp.py): cost table, links, best
  object means, stixels and costs, bit for bit.
"""

import math

import numpy as np
import pytest
from scipy.stats import norm

import oracle
import synth
from bruteforce import OB, Problem, c_map
from naive_dp import NaiveColumn
from test_oracle_pins import dp_path, random_column, small_params


@pytest.fixture(scope="module")
def build_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("bruteforce"))


# --------------------------------------------------------------- Eq. 4 tables

def scipy_cost(d, mu, sigma, p_out, D):
    """Eq. 4 written with scipy: the Gaussian branch is minus the log of the
    normal density truncated to [0, D] and weighted by 1 - p_out, the
    outlier branch minus the log of the uniform density p_out / D."""
    c_out = -math.log(p_out / D)
    mass = norm.cdf(D, mu, sigma) - norm.cdf(0.0, mu, sigma)
    if mass <= 0.0:
        return c_out
    gauss = -(math.log(1.0 - p_out) + norm.logpdf(d, mu, sigma) - math.log(mass))
    return min(c_out, gauss)


def grid_value(x, g):
    """x on the 2^-g grid, or None when x lies within 1e-9 of a rounding
    boundary (two correct evaluations may then round either way)."""
    y = math.ldexp(x, g)
    frac = y - math.floor(y)
    if abs(frac - 0.5) < 1e-9 * max(1.0, abs(y)):
        return None
    return math.ldexp(round(y), -g)


@pytest.mark.parametrize("W,H,D,pitch,eps_g", [(1024, 440, 128, 0.0, 0.05),
                                               (640, 240, 64, 0.02, 0.2),
                                               (2048, 880, 256, -0.01, 0.05)])
def test_tables_against_scipy(W, H, D, pitch, eps_g):
    cam = dict(synth.camera_for_size(W, H), pitch_rad=pitch)
    m = dict(synth.DEFAULT_MODEL, ground_slope_noise=eps_g)
    p = synth.make_params(camera=cam, model=m, max_disparity=D, max_width=W, max_height=H)
    t = oracle.tables(p, H)
    g = p["cost_grid_log2"]
    pout, sd = m["p_out"], m["sigma_disp"]
    alpha = cam["baseline_m"] * math.cos(pitch) / cam["cam_height_m"]
    v_hor = (H - 1) - cam["horizon_row"]
    rng = np.random.default_rng(H)
    checked = 0
    for d in range(D):
        want = grid_value(scipy_cost(d, 0.0, m["sigma_sky"], pout, D), g)
        if want is not None:
            assert t["S"][d] == want, d
            checked += 1
    for v in rng.integers(0, H, 40):
        v = int(v)
        if v > math.floor(v_hor):
            assert np.all(t["G"][v] == 0.0)           # above the horizon: never used
            continue
        mu = alpha * (v_hor - v)                      # ground model f_ground(v)
        sg = math.sqrt(sd * sd + (eps_g * mu) ** 2)
        for d in range(D):
            want = grid_value(scipy_cost(d, mu, sg, pout, D), g)
            if want is not None:
                assert t["G"][v][d] == want, (v, d)
                checked += 1
    for f in rng.integers(0, D, 24):
        f = int(f)
        so = math.sqrt(sd * sd + (f * f * m["object_depth_extent_m"]
                                  / (cam["focal_px"] * cam["baseline_m"])) ** 2)
        for d in range(D):
            want = grid_value(scipy_cost(d, float(f), so, pout, D), g)
            if want is not None:
                assert t["O"][d][f] == want, (d, f)
                checked += 1
    assert checked > 0.99 * D * (1 + 24) + 10


# --------------------------------------------------------------- brute force, 9-12 rows

def permissive_params(**kw):
    """Every transition finite, so the search walks all 3 * 4^(h-1) lists."""
    m = dict(synth.DEFAULT_MODEL)
    m["trans_cost"] = [[0.5, 1.0, 0.0], [0.0, 2.0, 0.0], [2.0, 3.0, 1.5]]
    m.update(kw)
    cam = dict(focal_px=700.0, baseline_m=1.2, cam_height_m=0.3, horizon_row=-40.0,
               pitch_rad=0.0)
    return synth.make_params(camera=cam, model=m, max_disparity=32, max_height=16)


def c_path(lst):
    return [tuple(x) for x in lst]


@pytest.mark.parametrize("H", [9, 10, 11, 12])
@pytest.mark.parametrize("grid", [10, 0])
def test_dp_equals_exhaustive_map_9_to_12_rows(build_dir, H, grid):
    """Ordering prior off: the recurrence is exact MAP.  Its total equals
    the exhaustive minimum and its list is the first optimum in the tie
    order (class then base of the top stixel, then of the next, ...); its
    per-stixel costs sum to the total.  grid 0 (integer costs) makes ties
    frequent."""
    rng = np.random.default_rng(1000 * H + grid)
    ties = 0
    for horizon in (0.0, float(H) / 2, float(H + 3)):
        p = small_params(ordering=False, grid=grid, horizon=horizon)
        t = oracle.tables(p, H)
        for _ in range(5):
            q = random_column(rng, H, 32)
            res = oracle.column(p, q)
            best, lst, n_lists, n_opt = c_map(build_dir, Problem(p, t, q))
            assert n_lists > 0
            assert res["total"] == best
            assert dp_path(res) == c_path(lst)
            assert math.fsum(float(s["cost"]) for s in res["stixels"]) == best
            ties += n_opt > 1
    if grid == 0:
        assert ties > 0                      # the tie order was exercised


@pytest.mark.parametrize("H", [9, 12])
def test_dp_equals_exhaustive_map_all_transitions(build_dir, H):
    """Every transition allowed and ground everywhere (horizon below the
    column): the search walks all 3 * 4^(h-1) lists (12.6 M at h = 12)."""
    rng = np.random.default_rng(H)
    for grid in (10, 0):
        p = permissive_params(ordering_cost=0.0)
        p["cost_grid_log2"] = grid
        t = oracle.tables(p, H)
        q = random_column(rng, H, 32)
        res = oracle.column(p, q)
        best, lst, n_lists, _ = c_map(build_dir, Problem(p, t, q))
        assert n_lists == 3 * 4 ** (H - 1)
        assert res["total"] == best
        assert dp_path(res) == c_path(lst)


@pytest.mark.parametrize("H", [9, 10, 11, 12])
def test_dp_with_full_prior_9_to_12_rows(build_dir, H):
    """Ordering prior on (Eq. 6 charges it against the stored best object
    stixel, so the recurrence is not MAP): its cost is never below the
    exhaustive minimum and equals the cost of its own list scored stixel by
    stixel against the actual stixel below each one."""
    rng = np.random.default_rng(77 + H)
    for horizon in (0.0, float(H) / 2, float(H + 3)):
        for c_ord in (4.0, 0.5):
            p = small_params(ordering=True, ordering_cost=c_ord, horizon=horizon)
            t = oracle.tables(p, H)
            for _ in range(3):
                q = random_column(rng, H, 32)
                res = oracle.column(p, q)
                pb = Problem(p, t, q)
                best, _, _, _ = c_map(build_dir, pb)
                assert res["total"] >= best
                prev, acc = None, []
                for (b, e, c, f) in dp_path(res):
                    d, f2 = pb.data(c, b, e)
                    assert c != OB or f2 == f
                    cur = (b, e, c, f)
                    acc.append(d + pb.prior(prev, cur))
                    prev = cur
                assert math.fsum(acc) == res["total"]
                assert [float(s["cost"]) for s in res["stixels"]] == acc


# --------------------------------------------------------------- naive Eq. 5-6

def random_model(rng):
    m = dict(synth.DEFAULT_MODEL)
    m["bic_cost"] = float(rng.uniform(0, 4))
    m["ordering_cost"] = float(rng.uniform(0.5, 8))
    m["ordering_tol_px"] = int(rng.integers(0, 3))
    m["gravity_cost"] = float(rng.uniform(0, 6))
    m["diving_cost"] = float(rng.uniform(0, 10))
    m["gravity_tol_px"] = float(rng.uniform(0, 3))
    m["diving_tol_px"] = float(rng.uniform(0, 3))
    m["first_cost"] = [float(x) for x in rng.uniform(0, 4, 3)]
    T = [[float(x) for x in row] for row in rng.uniform(0, 3, (3, 3))]
    if rng.random() < 0.5:
        T[1][1] = T[2][1] = T[2][2] = math.inf
    m["trans_cost"] = T
    return m


def structured_column(rng, H, D):
    """Ground ramp below a cut, one to three objects above it, sky (0) on
    top; rounding noise and invalid pixels."""
    col = np.zeros(H)
    a = int(rng.integers(0, H + 1))
    b = int(rng.integers(a, H + 1))
    col[:a] = 0.5 * (a - np.arange(a))
    cuts = np.sort(rng.integers(a, b + 1, int(rng.integers(0, 3))))
    edges = [a, *cuts.tolist(), b]
    for lo, hi in zip(edges[:-1], edges[1:]):
        col[lo:hi] = rng.integers(0, D)
    col = np.rint(col + rng.normal(0, 0.7, H))
    col[rng.random(H) < 0.1] = -1
    return np.clip(col, -1, D - 1).astype(np.int32)


def test_naive_recurrence_matches_oracle_bitwise():
    """A few hundred random columns (h <= 64) under random priors, every
    prior term on: cost table, links, best object means, stixels, costs."""
    rng = np.random.default_rng(20240)
    n = 0
    for case in range(240):
        H = int(rng.integers(1, 65)) if case % 4 else int(rng.integers(1, 9))
        D = int(rng.choice([16, 32, 64]))
        grid = int(rng.choice([10, 0, 4]))
        cam = dict(focal_px=700.0, baseline_m=0.6, cam_height_m=1.2,
                   horizon_row=float(rng.integers(-3, H + 3)), pitch_rad=0.0)
        p = synth.make_params(camera=cam, model=random_model(rng), max_disparity=D,
                              max_height=H, cost_grid_log2=grid)
        q = random_column(rng, H, D) if case % 2 else structured_column(rng, H, D)
        t = oracle.tables(p, H)
        ref = NaiveColumn(p, t, q).solve()
        got = oracle.column(p, q)
        assert np.array_equal(got["C"], np.array(ref["C"])), case
        assert np.array_equal(got["link_b"], np.array(ref["link_b"])), case
        assert np.array_equal(got["link_c"], np.array(ref["link_c"])), case
        assert np.array_equal(got["fob"], np.array(ref["fob"])), case
        assert got["total"] == ref["total"], case
        want = [(b, k, c, f) for b, k, c, f, _ in ref["stixels"]]
        assert dp_path(got) == want, case
        assert [float(s["cost"]) for s in got["stixels"]] == [x[4] for x in ref["stixels"]]
        n += 1
    assert n == 240
