"""Mutation check of the oracle's pins.

Each mutant plants one plausible mistake in a copy of oracle/stixel_oracle.c
(a dropped term, a wrong sign, index, comparison or rounding, a transposed
operand), builds it with gcc on the CPU, and runs a battery of the pins of
tests/test_oracle_pins.py and tests/test_oracle_exhaustive.py against it.
Every mutant must fail at least one pin; the unmutated copy, built the same
way, must pass them all.  The mistakes live only in the temporary copies.
"""

import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_exhaustive as EX
import test_oracle_pins as PIN
import test_oracle_subpixel as SUB
from naive_dp import NaiveColumn

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "stixel_oracle.c")

# (name, text in the oracle source, replacement); the text must occur once
MUTANTS = [
    ("bic dropped from the pair prior", "return t + x->beta + pen;", "return t + pen;"),
    ("bic dropped from the bottom prior", "return x->F[c] + x->beta; }", "return x->F[c]; }"),
    ("sign of ln A_norm", "double gauss = log(a_norm) +", "double gauss = -log(a_norm) +"),
    ("lower truncation bound of A_norm", "- normal_cdf(-mu / sigma);", "- normal_cdf(mu / sigma);"),
    ("last minimum wins", "if (cand < best) {", "if (cand <= best) {"),
    ("object table transposed", "(valid ? x->O[(size_t)d * D + f] : 0.0)",
     "(valid ? x->O[(size_t)f * D + d] : 0.0)"),
    ("mean truncated instead of rounded", "(2 * sum + n) / (2 * n)", "(2 * sum) / (2 * n)"),
    ("diving threshold off by one", "floor(ldexp(fg + p->diving_tol_px, p->subpixel_log2));",
     "floor(ldexp(fg + p->diving_tol_px, p->subpixel_log2)) + 1;"),
    ("gravity threshold rounded down", "ceil(ldexp(fg - p->gravity_tol_px, p->subpixel_log2));",
     "floor(ldexp(fg - p->gravity_tol_px, p->subpixel_log2));"),
    ("ordering comparison not strict", "f > f_prev + (x->p->ordering_tol_px",
     "f >= f_prev + (x->p->ordering_tol_px"),
    ("ordering tolerance not in bins", "(x->p->ordering_tol_px << x->p->subpixel_log2)",
     "x->p->ordering_tol_px"),
    ("thresholds not in bins", "floor(ldexp(fg + p->diving_tol_px, p->subpixel_log2));",
     "floor(fg + p->diving_tol_px);"),
    ("object table at bin indices, not px", "sigma_object(p, bin_px(p, f)), p->p_out, dr), g);",
     "sigma_object(p, f), p->p_out, dr), g);"),
    ("reduction not scaled to bins", "double rq = rint(ldexp(m, p->subpixel_log2));",
     "double rq = rint(m);"),
    ("gravity comparison not strict", "else if (f < x->fg_lo[b])", "else if (f <= x->fg_lo[b])"),
    ("diving comparison not strict", "if (f > x->fg_hi[b]) pen", "if (f >= x->fg_hi[b]) pen"),
    ("diving and gravity costs swapped",
     "if (f > x->fg_hi[b]) pen = x->c_dive;\n        else if (f < x->fg_lo[b]) pen = x->c_grav;",
     "if (f > x->fg_hi[b]) pen = x->c_grav;\n        else if (f < x->fg_lo[b]) pen = x->c_dive;"),
    ("predecessor mean read at the wrong row", "+ prior_pair(x, cp, c, fob[b - 1], f, b) + dat;",
     "+ prior_pair(x, cp, c, fob[b], f, b) + dat;"),
    ("stored mean of the whole column", "fob[k] = object_mean(x, bb, k);",
     "fob[k] = object_mean(x, 0, k);"),
    ("ground allowed one row above the horizon", "if (t > x->vtop) return INFINITY;",
     "if (t > x->vtop + 1) return INFINITY;"),
    ("ground top rounded up", "double vh = floor(horizon_v(p, H));",
     "double vh = ceil(horizon_v(p, H));"),
    ("ground slope noise not squared",
     "double e = p->ground_slope_noise * mu;\n    return sqrt(p->sigma_disp * p->sigma_disp + e * e);",
     "double e = p->ground_slope_noise * mu;\n    return sqrt(p->sigma_disp * p->sigma_disp + e);"),
    ("object depth term linear in f", "double e = f * f * p->object_depth_extent_m",
     "double e = f * p->object_depth_extent_m"),
    ("final class: last minimum", "if (C[(size_t)(H - 1) * NCLS + cc] < C[(size_t)(H - 1) * NCLS + c])",
     "if (C[(size_t)(H - 1) * NCLS + cc] <= C[(size_t)(H - 1) * NCLS + c])"),
    ("upper median", "m = vals[(n - 1) / 2];", "m = vals[n / 2];"),
    ("columns not flipped bottom-up", "q[(size_t)i * H + (H - 1 - r)] = out;",
     "q[(size_t)i * H + r] = out;"),
    ("zero disparity treated as invalid", "if (isfinite(x) && x >= 0.0) vals[n++] = x;",
     "if (isfinite(x) && x > 0.0) vals[n++] = x;"),
    ("grid rounding by floor", "return ldexp(rint(ldexp(x, g)), -g);",
     "return ldexp(floor(ldexp(x, g)), -g);"),
    ("invalid pixel charged as disparity 0", "(valid ? x->S[d] : 0.0);", "(valid ? x->S[d] : x->S[0]);"),
    ("invalid pixel counted in the mean", "x->PN[v + 1] = x->PN[v] + (valid ? 1 : 0);",
     "x->PN[v + 1] = x->PN[v] + 1;"),
    ("reported bottom stixel cost without bic", "+ (b == 0 ? prior_first(x, c)",
     "+ (b == 0 ? x->F[c]"),
]


def build(tmpdir, name, text):
    src = os.path.join(tmpdir, f"{name}.c")
    so = os.path.join(tmpdir, f"lib{name}.so")
    with open(src, "w") as f:
        f.write(text)
    inc = os.path.dirname(SRC)
    subprocess.run(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                    "-fopenmp", "-I", inc, src, "-o", so, "-lm"], check=True)
    return so


def naive_battery():
    rng = np.random.default_rng(5)
    for case in range(40):
        H = int(rng.integers(1, 24))
        D = 32
        cam = dict(focal_px=700.0, baseline_m=0.6, cam_height_m=1.2,
                   horizon_row=float(rng.integers(-3, H + 3)) + 0.5 * (case % 2), pitch_rad=0.0)
        p = oracle_params(cam, EX.random_model(rng), D, H, int(rng.choice([10, 0])))
        q = PIN.random_column(rng, H, D) if case % 2 else EX.structured_column(rng, H, D)
        t = oracle.tables(p, H)
        ref = NaiveColumn(p, t, q).solve()
        got = oracle.column(p, q)
        assert np.array_equal(got["C"], np.array(ref["C"]))
        assert np.array_equal(got["fob"], np.array(ref["fob"]))
        assert PIN.dp_path(got) == [(b, k, c, f) for b, k, c, f, _ in ref["stixels"]]
        assert [float(s["cost"]) for s in got["stixels"]] == [x[4] for x in ref["stixels"]]


def oracle_params(cam, model, D, H, grid):
    import synth
    return synth.make_params(camera=cam, model=model, max_disparity=D, max_height=H,
                             cost_grid_log2=grid)


BATTERY = [
    ("closed forms", PIN.test_pixel_cost_closed_forms),
    ("cost terms", PIN.test_pixel_cost_terms),
    ("grid", PIN.test_quantize_grid),
    ("median", lambda: PIN.test_reduce_median_vs_numpy(5)),
    ("mean", PIN.test_reduce_mean_vs_fsum),
    ("table properties", PIN.test_tables_properties),
    ("tables vs scipy", lambda: EX.test_tables_against_scipy(640, 240, 64, 0.02, 0.2)),
    ("prefix sums", PIN.test_prefix_sums_equal_direct_sums),
    ("single row", PIN.test_single_row_column),
    ("all invalid", PIN.test_all_invalid_column),
    ("exact ground", PIN.test_exact_ground_column),
    ("ordering boundary", lambda: (PIN.test_ordering_tolerance_boundary(20, False),
                                   PIN.test_ordering_tolerance_boundary(19, True))),
    ("gravity/diving", lambda: [PIN.test_gravity_and_diving_penalties(d, c, t) for d, c, t in
                                ((5, "gravity_cost", 2.0), (14, None, 2.0),
                                 (30, "diving_cost", 2.0), (12, "gravity_cost", 2.0),
                                 (13, None, 2.0), (17, "diving_cost", 2.0), (20, None, 6.0),
                                 (21, "diving_cost", 6.0))]),
    ("brute force, ordering off", lambda: [PIN.test_dp_equals_bruteforce_map_without_ordering(H, g)
                                           for H in (5, 7) for g in (10, 0)]),
    ("naive recurrence", naive_battery),
    ("bins: reduction", lambda: [SUB.test_reduce_in_bins(sp, m) for sp in (1, 2) for m in (0, 1)]),
    ("bins: tables", lambda: SUB.test_tables_in_bins_against_scipy(1)),
    ("bins: naive recurrence", lambda: SUB.test_naive_recurrence_in_bins(1)),
]


def run_battery():
    """Name of the first pin that fails, or None."""
    for name, fn in BATTERY:
        try:
            fn()
        except (AssertionError, ValueError, IndexError):
            return name
    return None


@pytest.fixture(scope="module")
def tmpdir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("mutants"))


def with_library(path, fn):
    saved = (oracle._lib, oracle.LIB_PATH)
    oracle._lib, oracle.LIB_PATH = None, path
    try:
        return fn()
    finally:
        oracle._lib, oracle.LIB_PATH = saved


def test_unmutated_copy_passes_the_battery(tmpdir):
    so = build(tmpdir, "control", open(SRC).read())
    assert with_library(so, run_battery) is None


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_killed(tmpdir, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site of '{name}' not found exactly once"
    so = build(tmpdir, "m" + str(abs(hash(name)) % 10 ** 8), text.replace(old, new))
    killed_by = with_library(so, run_battery)
    assert killed_by is not None, f"mutant '{name}' survived every pin"
