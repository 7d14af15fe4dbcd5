"""Pins of the CPU FP64 oracle to things other than itself.

Each test ties one oracle function to the mathematics or to an independent
computation: closed forms of Eq. 4, the mixture of Eq. 3, numpy's sort,
rational arithmetic, direct sums instead of prefix sums, and brute-force
enumeration of every segmentation of short columns (Eq. 1-2).
"""

import json
import math
import os

import numpy as np
import pytest
from scipy.stats import norm

import oracle
import synth
from bruteforce import (GR, OB, SK, Problem, lexicographic_key, map_solutions,
                        rounded_mean)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- Eq. 3-4

def test_pixel_cost_closed_forms():
    """Closed forms of Eq. 4 (values derived by hand in golden/closed_forms.json)."""
    gold = json.load(open(os.path.join(GOLDEN, "closed_forms.json")))
    # Gaussian peak, mu far inside [0, 128], sigma 1: ln(sqrt(2 pi)) - ln(1 - 0.15)
    assert oracle.pixel_cost(50, 50, 1.0, 0.15, 128) == pytest.approx(
        gold["peak_sigma1_pout0.15"]["value"], abs=1e-12)
    # outlier branch: ln(128) - ln(0.15)
    assert oracle.pixel_cost(120, 10, 1.0, 0.15, 128) == pytest.approx(
        gold["outlier_d128_pout0.15"]["value"], abs=1e-12)
    assert oracle.pixel_cost(0, 200, 1.0, 0.15, 256) == pytest.approx(
        gold["outlier_d256_pout0.15"]["value"], abs=1e-12)
    # mu = 0: the Gaussian keeps half its mass inside [0, d_range]: + ln(1/2)
    assert oracle.pixel_cost(0, 0, 1.0, 0.15, 128) == pytest.approx(
        gold["sky_peak_sigma1_pout0.15"]["value"], abs=1e-12)


def test_pixel_cost_terms():
    """sigma and quadratic terms of Eq. 4, each isolated by a difference."""
    base = oracle.pixel_cost(60, 60, 1.0, 0.2, 128)
    assert oracle.pixel_cost(60, 60, 2.0, 0.2, 128) - base == pytest.approx(math.log(2.0), abs=1e-12)
    for dd, s in [(1, 1.0), (2, 1.5), (3, 2.0)]:
        diff = oracle.pixel_cost(60 + dd, 60, s, 0.2, 128) - oracle.pixel_cost(60, 60, s, 0.2, 128)
        assert diff == pytest.approx(dd * dd / (2 * s * s), abs=1e-12)
    # the branch switches exactly where the Gaussian cost reaches the outlier cost
    c_out = math.log(128) - math.log(0.2)
    for d in range(0, 128):
        c = oracle.pixel_cost(d, 60, 1.0, 0.2, 128)
        assert c <= c_out + 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_pixel_cost_vs_mixture(seed):
    """Eq. 4 is the max-approximation of -log of the mixture of Eq. 3: since
    a + b lies between max(a, b) and 2 max(a, b), the cost must lie within
    [-ln P, -ln P + ln 2], with P evaluated from Eq. 3 and a truncated normal."""
    rng = np.random.default_rng(seed)
    for _ in range(200):
        D = int(rng.choice([64, 128, 256]))
        mu = float(rng.uniform(0, D - 1))
        sig = float(rng.uniform(0.3, 6.0))
        pout = float(rng.uniform(0.01, 0.5))
        d = float(rng.integers(0, D))
        mass = norm.cdf(D, mu, sig) - norm.cdf(0, mu, sig)
        P = pout / D + (1 - pout) * norm.pdf(d, mu, sig) / mass
        c = oracle.pixel_cost(d, mu, sig, pout, D)
        assert -math.log(P) - 1e-9 <= c <= -math.log(P) + math.log(2) + 1e-9


def test_quantize_grid():
    for g in (0, 4, 10):
        for x in np.random.default_rng(0).uniform(-50, 50, 100):
            y = oracle.quantize(x, g)
            assert y * 2 ** g == round(y * 2 ** g)
            assert abs(y - x) <= 2.0 ** (-g - 1)
    assert oracle.quantize(math.inf, 10) == math.inf
    assert oracle.quantize(0.3, -1) == 0.3


# --------------------------------------------------------------- Sec. 3.4 tables

def test_tables_properties():
    p = synth.make_params()
    H = 440
    t = oracle.tables(p, H)
    D = p["max_disparity"]
    grid = 2.0 ** p["cost_grid_log2"]
    for name in ("S", "G", "O"):
        a = t[name]
        assert np.all(a * grid == np.round(a * grid)), name
    c_out = math.log(D) - math.log(p["model"]["p_out"])
    assert np.all(t["O"] <= c_out + 1e-12) and np.all(t["S"] <= c_out + 1e-12)
    # sky cost grows with disparity until it saturates at the outlier cost
    assert np.all(np.diff(t["S"]) >= 0)
    # object cost of mean f is smallest at pixel disparity d = f
    for f in range(D):
        assert t["O"][f, f] == t["O"][:, f].min()
    # ground: f_ground(v) = alpha (v_hor - v) with alpha = B/H_cam = 0.25 and
    # v_hor = 439 - 180 = 259; each row is cheapest at the nearest disparity
    alpha, vhor = 0.3 / 1.2, 439 - 180
    for v in range(0, 260, 7):
        mu = alpha * (vhor - v)
        near = [d for d in range(D) if abs(d - mu) == min(abs(e - mu) for e in range(D))]
        assert t["G"][v].argmin() in near
    assert np.all(t["G"][260:] == 0.0)
    # integer prior thresholds at the object base row b
    for b in range(0, H + 1, 11):
        fg = alpha * (vhor - b)
        assert t["fg_hi"][b] == math.floor(fg + 2.0)
        assert t["fg_lo"][b] == math.ceil(fg - 2.0)


def test_tables_match_pixel_cost():
    """The tables are Eq. 4 evaluated at each model disparity, then rounded."""
    p = synth.make_params(max_disparity=64)
    t = oracle.tables(p, 100)
    m = p["model"]
    for d in (0, 3, 17, 63):
        assert t["S"][d] == oracle.quantize(oracle.pixel_cost(d, 0, m["sigma_sky"], m["p_out"], 64), 10)
        f = 40
        so = math.sqrt(1.0 + (f * f * 0.3 / (700 * 0.3)) ** 2)
        assert t["O"][d, f] == oracle.quantize(oracle.pixel_cost(d, f, so, m["p_out"], 64), 10)


# --------------------------------------------------------------- Sec. 3.1 reduction

@pytest.mark.parametrize("s", [1, 2, 3, 5, 7, 8])
def test_reduce_median_vs_numpy(s):
    rng = np.random.default_rng(s)
    H, W = 37, 11 * s + (s - 1)          # trailing pixels beyond the last strip
    disp = rng.uniform(0, 140, (H, W)).astype(np.float32)
    bad = rng.random((H, W))
    disp[bad < 0.15] = -1
    disp[(bad > 0.15) & (bad < 0.2)] = np.nan
    disp[(bad > 0.2) & (bad < 0.22)] = np.inf
    disp[:, :s][:5] = -1                    # fully invalid strips
    disp[7] = np.round(disp[7]) + 0.5       # exact .5 ties -> half to even
    disp[9] = 0.0                           # zero disparity is valid (sky)
    disp[10, ::2] = -0.0                    # and so is negative zero
    p = synth.make_params(stixel_width=s, max_disparity=128)
    q = oracle.reduce(p, disp)
    ncols = W // s
    assert q.shape == (ncols, H)
    for i in range(ncols):
        for r in range(H):
            strip = disp[r, i * s:(i + 1) * s].astype(np.float64)
            ok = strip[np.isfinite(strip) & (strip >= 0)]
            if ok.size == 0:
                exp = -1
            else:
                med = np.sort(ok)[(ok.size - 1) // 2]
                exp = int(min(np.rint(med), 127))
            assert q[i, H - 1 - r] == exp


def test_reduce_mean_vs_fsum():
    rng = np.random.default_rng(3)
    s, H, W = 5, 20, 50
    disp = (rng.integers(0, 128 * 64, (H, W)) / 64.0).astype(np.float32)  # exact sums
    disp[rng.random((H, W)) < 0.2] = -1
    p = synth.make_params(stixel_width=s, reduce_mode=1)
    q = oracle.reduce(p, disp)
    for i in range(W // s):
        for r in range(H):
            vals = [float(x) for x in disp[r, i * s:(i + 1) * s] if x >= 0]
            exp = -1 if not vals else int(min(np.rint(math.fsum(vals) / len(vals)), 127))
            assert q[i, H - 1 - r] == exp


# --------------------------------------------------------------- prefix sums

def test_prefix_sums_equal_direct_sums():
    rng = np.random.default_rng(7)
    p = synth.make_params(max_disparity=64, camera=dict(synth.CAMERA_1024x440, horizon_row=20.0))
    H = 57
    q = rng.integers(-1, 64, H).astype(np.int32)
    r = oracle.column(p, q)
    t = oracle.tables(p, H)
    for (b, e) in [(0, 0), (0, H - 1), (3, 9), (10, 56), (20, 20)]:
        rows = range(b, e + 1)
        ok = [v for v in rows if q[v] >= 0]
        assert r["PG"][e + 1] - r["PG"][b] == math.fsum(t["G"][v, q[v]] for v in ok)
        assert r["PS"][e + 1] - r["PS"][b] == math.fsum(t["S"][q[v]] for v in ok)
        assert r["PD"][e + 1] - r["PD"][b] == sum(int(q[v]) for v in ok)
        assert r["PN"][e + 1] - r["PN"][b] == len(ok)
        for f in (0, 5, 31, 63):
            assert r["PO"][f, e + 1] - r["PO"][f, b] == math.fsum(t["O"][q[v], f] for v in ok)


# --------------------------------------------------------------- Eq. 5-6 vs brute force

def small_params(ordering=True, grid=10, D=32, horizon=3.0, **kw):
    cam = dict(focal_px=700.0, baseline_m=1.2, cam_height_m=0.3, horizon_row=horizon, pitch_rad=0.0)
    m = dict(synth.DEFAULT_MODEL)
    if not ordering:
        m["ordering_cost"] = 0.0
    m.update(kw)
    return synth.make_params(camera=cam, model=m, max_disparity=D, max_height=16,
                             cost_grid_log2=grid)


def random_column(rng, H, D):
    kind = rng.integers(3)
    if kind == 0:
        return rng.integers(-1, D, H).astype(np.int32)
    if kind == 1:
        cut = int(rng.integers(0, H + 1))
        a, b = rng.integers(0, D, 2)
        col = np.where(np.arange(H) < cut, a, b)
        col = col + rng.integers(-1, 2, H)
        col[rng.random(H) < 0.15] = -1
        return np.clip(col, -1, D - 1).astype(np.int32)
    col = np.full(H, -1, np.int32)
    col[rng.random(H) < 0.4] = rng.integers(0, D)
    return col


def dp_path(res):
    return [(int(s["v_bottom"]), int(s["v_top"]), int(s["cls"]), int(s["disparity"]))
            for s in res["stixels"]]


@pytest.mark.parametrize("H", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("grid", [10, 0])
def test_dp_equals_bruteforce_map_without_ordering(H, grid):
    """Without the ordering prior no term depends on a stored stixel, so the
    recurrence is exact MAP (Eq. 1): its cost equals the brute-force minimum
    and its segmentation is the first optimum in the tie order."""
    rng = np.random.default_rng(100 * H + grid)
    for horizon in (0.0, float(H) / 2, float(H + 3)):
        p = small_params(ordering=False, grid=grid, horizon=horizon)
        t = oracle.tables(p, H)
        for _ in range(6):
            q = random_column(rng, H, 32)
            res = oracle.column(p, q)
            pb = Problem(p, t, q)
            best, sols = map_solutions(pb)
            assert res["total"] == best
            winner = min(sols, key=lambda s: lexicographic_key(s[1]))
            assert dp_path(res) == [st for st, _ in winner[1]]
            assert [float(s["cost"]) for s in res["stixels"]] == [c for _, c in winner[1]]


@pytest.mark.parametrize("H", [2, 4, 6, 8])
def test_dp_with_ordering_prior(H):
    """With the ordering prior the recurrence charges it against the stored best
    object stixel (Eq. 6), so it is no longer exact MAP.  Its cost is still
    the true cost of the list it returns, and never below the MAP."""
    rng = np.random.default_rng(H)
    p = small_params(ordering=True, ordering_cost=4.0, horizon=float(H) / 2)
    t = oracle.tables(p, H)
    for _ in range(10):
        q = random_column(rng, H, 32)
        res = oracle.column(p, q)
        pb = Problem(p, t, q)
        best, _ = map_solutions(pb)
        assert res["total"] >= best
        # recompute the returned list's cost from scratch
        prev, acc = None, []
        for (b, e, c, f) in dp_path(res):
            d, f2 = pb.data(c, b, e)
            assert f2 == f or c != OB
            cur = (b, e, c, f)
            acc.append(d + pb.prior(prev, cur))
            prev = cur
        assert math.fsum(acc) == res["total"]


def test_ordering_penalty_binds():
    """Two stacked objects, the upper one closer: the recurrence keeps both and
    charges the ordering penalty on the upper one."""
    p = small_params(ordering=True, horizon=-5.0)   # no ground anywhere
    H = 10
    q = np.array([5] * 5 + [25] * 5, np.int32)
    res = oracle.column(p, q)
    path = dp_path(res)
    assert path == [(0, 4, OB, 5), (5, 9, OB, 25)]
    t = oracle.tables(p, H)
    pb = Problem(p, t, q)
    d_up, _ = pb.data(OB, 5, 9)
    assert res["stixels"][1]["cost"] == d_up + pb.T[OB][OB] + pb.beta + pb.c_ord


# --------------------------------------------------------------- special cases

def test_single_row_column():
    """h = 1: the result is argmin over classes of data + F[c] + beta."""
    p = small_params(horizon=0.0)
    t = oracle.tables(p, 1)
    for d in (-1, 0, 4, 17, 31):
        res = oracle.column(p, np.array([d], np.int32))
        data = [0.0, 0.0, 0.0] if d < 0 else [t["O"][d, d], t["G"][0, d], t["S"][d]]
        F = [oracle.quantize(x, 10) for x in p["model"]["first_cost"]]
        beta = oracle.quantize(p["model"]["bic_cost"], 10)
        costs = [data[c] + F[c] + beta for c in range(3)]
        c_best = int(np.argmin(costs))
        assert res["total"] == min(costs)
        assert dp_path(res) == [(0, 0, c_best, d if (c_best == OB and d >= 0) else 0)]


def test_all_invalid_column():
    """Every data term is 0, so the priors alone decide.  With the default
    model the single object stixel (F_OB + beta = 4) beats ground + sky (6),
    ground + object (6), object + sky (7) and sky alone (13)."""
    p = synth.make_params()
    res = oracle.column(p, np.full(440, -1, np.int32))
    assert res["total"] == 4.0
    assert dp_path(res) == [(0, 439, OB, 0)]


def test_constant_column_is_one_object():
    p = synth.make_params()
    res = oracle.column(p, np.full(440, 20, np.int32))
    assert dp_path(res) == [(0, 439, OB, 20)]


def test_exact_ground_column():
    """q follows the ground model below the horizon and is 0 above it: the
    result is one ground stixel ending at or below floor(v_hor), then sky."""
    p = synth.make_params()
    H, vhor = 440, 259
    q = np.array([int(np.rint(0.25 * (vhor - v))) if v <= vhor else 0 for v in range(H)], np.int32)
    path = dp_path(oracle.column(p, q))
    assert [c for _, _, c, _ in path] == [GR, SK]
    assert path[0][0] == 0 and path[0][1] <= vhor and path[1][1] == H - 1


def test_rounded_mean_reading():
    assert rounded_mean([1, 2]) == 2          # 1.5 rounds half up
    assert rounded_mean([2, 3, 3, 3]) == 3
    assert rounded_mean([0, 1, 1, 1]) == 1    # 0.75
    assert rounded_mean([]) == 0


# --------------------------------------------------------------- invariants / scenes

def check_invariants(p, disp, res, cap=None):
    H, W = disp.shape
    s = p["stixel_width"]
    q = oracle.reduce(p, disp)
    vtop = math.floor((H - 1) - p["camera"]["horizon_row"])
    T = p["model"]["trans_cost"]
    for i in range(W // s):
        st = oracle.column_stixels(res, i)
        assert len(st) >= 1
        if res["overflow"][i]:
            assert cap is not None and len(st) == cap
        else:
            assert st[0]["v_bottom"] == 0 and st[-1]["v_top"] == H - 1
            assert math.fsum(float(x) for x in st["cost"]) == res["total"][i]
        for a, b in zip(st[:-1], st[1:]):
            assert b["v_bottom"] == a["v_top"] + 1
            assert math.isfinite(T[a["cls"]][b["cls"]])
        for x in st:
            assert x["v_bottom"] <= x["v_top"]
            if x["cls"] == GR:
                assert x["v_top"] <= vtop
            if x["cls"] == OB:
                vals = [int(d) for d in q[i, x["v_bottom"]:x["v_top"] + 1] if d >= 0]
                assert x["disparity"] == rounded_mean(vals)


@pytest.mark.parametrize("seed", [0, 1])
def test_scene_invariants(seed):
    p = synth.make_params()
    disp = synth.generate_frame(synth.SceneSpec(seed=seed))
    res = oracle.frame(p, disp)
    check_invariants(p, disp, res)
    capped = oracle.frame(p, disp, cap=2)
    check_invariants(p, disp, capped, cap=2)
    for i in range(len(res["counts"])):
        n = res["counts"][i]
        assert capped["overflow"][i] == (n > 2)
        assert capped["counts"][i] == min(n, 2)
        assert np.array_equal(oracle.column_stixels(capped, i), oracle.column_stixels(res, i)[:2])
        assert capped["total"][i] == res["total"][i]


@pytest.mark.parametrize("seed", [0, 3])
def test_scene_recovery(seed):
    """Quality check of oracle + default parameters on ground-plus-box scenes:
    per-pixel class agreement with the scene generator's labels."""
    p = synth.make_params()
    disp, clean, lab = synth.generate_frame(synth.SceneSpec(seed=seed), return_labels=True)
    res = oracle.frame(p, disp)
    H, W = disp.shape
    s = p["stixel_width"]
    pred = np.full((H, W // s), -1)
    for i in range(W // s):
        for st in oracle.column_stixels(res, i):
            pred[H - 1 - st["v_top"]:H - st["v_bottom"], i] = st["cls"]
    gt = lab[:, s // 2::s][:, :W // s]
    assert (pred == gt).mean() > 0.97
    for c in (OB, GR, SK):
        hit = ((pred == c) & (gt == c)).sum()
        assert hit / max((gt == c).sum(), 1) > 0.9
        assert hit / max((pred == c).sum(), 1) > 0.9
    # objects carry the box disparity
    obj = (pred == OB) & (gt == OB)
    fpix = np.zeros_like(pred)
    for i in range(W // s):
        for st in oracle.column_stixels(res, i):
            fpix[H - 1 - st["v_top"]:H - st["v_bottom"], i] = st["disparity"]
    err = np.abs(fpix[obj] - clean[:, s // 2::s][:, :W // s][obj])
    assert np.median(err) <= 1.0


def test_rejects_bad_arguments():
    p = synth.make_params()
    with pytest.raises(ValueError):
        oracle.frame(p, np.zeros((10, 3), np.float32))       # narrower than one stixel
    bad = synth.make_params()
    bad["model"]["first_cost"] = [math.inf, 0.0, 1.0]
    with pytest.raises(ValueError):
        oracle.column(bad, np.zeros(5, np.int32))


@pytest.mark.parametrize("tol,penalised", [(20, False), (19, True)])
def test_ordering_tolerance_boundary(tol, penalised):
    """The ordering penalty applies only when the upper mean exceeds the lower
    one by strictly more than the tolerance."""
    p = small_params(ordering=True, horizon=-5.0, ordering_tol_px=tol)
    q = np.array([5] * 5 + [25] * 5, np.int32)
    res = oracle.column(p, q)
    assert dp_path(res) == [(0, 4, OB, 5), (5, 9, OB, 25)]
    pb = Problem(p, oracle.tables(p, 10), q)
    d_up, _ = pb.data(OB, 5, 9)
    expect = d_up + pb.T[OB][OB] + pb.beta + (pb.c_ord if penalised else 0.0)
    assert res["stixels"][1]["cost"] == expect


@pytest.mark.parametrize("obj_disp,penalty,dive_tol", [
    (5, "gravity_cost", 2.0), (14, None, 2.0), (30, "diving_cost", 2.0), (12, "gravity_cost", 2.0),
    (13, None, 2.0), (17, "diving_cost", 2.0), (20, None, 6.0), (21, "diving_cost", 6.0)])
def test_gravity_and_diving_penalties(obj_disp, penalty, dive_tol):
    """An object standing on the ground at base row 200, where the ground
    disparity is 0.25 * (259 - 200) = 14.75: far behind it (5 < 13) pays the
    gravity cost, in front of it (30 > 16) the diving cost, at it nothing.
    The thresholds are ceil(14.75 - 2) = 13 and floor(14.75 + 2) = 16, both
    strict: 12 and 17 pay, 13 does not; with a diving tolerance of 6 px the
    upper one is 20 (an object at 16 would absorb the ground rows below
    its base), so 20 does not pay and 21 does.
    The penalties are lowered so that the direct ground-to-object transition
    stays optimal and the penalty shows in the object's cost."""
    m = dict(synth.DEFAULT_MODEL, gravity_cost=1.0, diving_cost=1.5, diving_tol_px=dive_tol)
    p = synth.make_params(model=m)
    H, vhor = 440, 259
    q = np.array([int(np.rint(0.25 * (vhor - v))) for v in range(200)]
                 + [obj_disp] * 60 + [0] * 180, np.int32)
    res = oracle.column(p, q)
    path = dp_path(res)
    assert path[0] == (0, 199, GR, 0) and path[1] == (200, 259, OB, obj_disp)
    b = path[1][0]
    pb = Problem(p, oracle.tables(p, H), q)
    d_ob, _ = pb.data(OB, b, path[1][1])
    extra = 0.0 if penalty is None else oracle.quantize(p["model"][penalty], 10)
    assert res["stixels"][1]["cost"] == d_ob + pb.T[GR][OB] + pb.beta + extra
