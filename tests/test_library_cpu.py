"""Host-side checks of the HIP library that need no GPU: the shared object
loads and exports every entry point its header declares, the ctypes structs
match the C layout, parameter validation and the exact-range checks, and the
library's host-built offline tables equal the oracle's bit for bit."""

import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import synth
import paper_1610_04124_amd as P
from paper_1610_04124_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stixels.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stixels_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    L = P.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(B.EXPORTS) == names


def test_phase_timing_library_exports_the_same_symbols():
    """The profiling build (kernels with phase stamps) is the same library:
    every declared entry point, loaded in a process of its own."""
    if not os.path.exists(B.PHASES_LIB_PATH):
        pytest.skip("libstixels_phases.so not built")
    code = ("import ctypes, sys; L = ctypes.CDLL(sys.argv[1]); "
            "print(' '.join(n for n in sys.argv[2:] if not hasattr(L, n)))")
    # torch first, as the binding does, so that the HIP runtime resolves
    out = subprocess.run(["python", "-c", "import torch; " + code, B.PHASES_LIB_PATH,
                          *declared_functions()], check=True, capture_output=True, text=True)
    assert out.stdout.strip() == ""


def test_phase_cycles_reject_bad_arguments():
    buf = (ctypes.c_uint64 * 7)()
    assert P.lib().stixels_batch_phase_cycles(None, buf, 7, 0) == B.E_INVALID_ARG


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "stixels.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu\\n\","
        "sizeof(stixels_params), sizeof(stixels_model), sizeof(stixels_record),"
        "sizeof(stixels_output), sizeof(stixels_job), sizeof(stixels_batch_config),"
        "offsetof(stixels_params, stixel_width), offsetof(stixels_model, ordering_tol_px));"
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [ctypes.sizeof(B.Params), ctypes.sizeof(B.Model), 12, ctypes.sizeof(B.Output),
            ctypes.sizeof(B.Job), ctypes.sizeof(B.BatchConfig), B.Params.stixel_width.offset,
            B.Model.ordering_tol_px.offset]
    assert got == want


@pytest.mark.parametrize("kw", [
    dict(), dict(max_disparity=256, max_height=880, max_width=2048, stixel_width=3),
    dict(max_disparity=64, max_height=100), dict(cost_grid_log2=6),
    dict(subpixel_log2=1), dict(max_disparity=64, subpixel_log2=2),
    dict(max_disparity=32, subpixel_log2=3, reduce_mode=1),
])
def test_host_tables_equal_oracle(kw):
    cam = synth.camera_for_size(kw.get("max_width", 1024), kw.get("max_height", 440))
    p = synth.make_params(camera=cam, **kw)
    H = p["max_height"]
    t = oracle.tables(p, H)
    S = P.host_table(p, B.TABLE_SKY)
    G = P.host_table(p, B.TABLE_GROUND)
    O = P.host_table(p, B.TABLE_OBJECT)
    hi = P.host_table(p, B.TABLE_FG_HI)
    lo = P.host_table(p, B.TABLE_FG_LO)
    # library: ground by top-down row, object as [f][d]; oracle: bottom-up, [d][f]
    assert np.array_equal(S.astype(np.float64), t["S"])
    assert np.array_equal(G[::-1].astype(np.float64), t["G"])
    assert np.array_equal(O.T.astype(np.float64), t["O"])
    assert np.array_equal(hi[::-1], t["fg_hi"][:H])
    assert np.array_equal(lo[::-1], t["fg_lo"][:H])


def _rc(params):
    try:
        P.host_table(params, B.TABLE_SKY)
        return 0
    except B.StixelsError as e:
        return e.code


@pytest.mark.parametrize("mutate,code", [
    (lambda p: p.update(stixel_width=0), B.E_INVALID_ARG),
    (lambda p: p.update(stixel_width=17), B.E_INVALID_ARG),
    (lambda p: p.update(max_height=1025), B.E_INVALID_ARG),
    (lambda p: p.update(max_disparity=257), B.E_INVALID_ARG),
    (lambda p: p.update(max_width=2), B.E_INVALID_ARG),
    (lambda p: p.update(reduce_mode=2), B.E_INVALID_ARG),
    (lambda p: p.update(cost_grid_log2=13), B.E_INVALID_ARG),
    (lambda p: p["camera"].update(horizon_row=180.3), B.E_INVALID_ARG),
    (lambda p: p["camera"].update(cam_height_m=0.0), B.E_INVALID_ARG),
    (lambda p: p["model"].update(p_out=1.0), B.E_INVALID_ARG),
    (lambda p: p["model"].update(first_cost=[math.inf, 0, 0]), B.E_INVALID_ARG),
    (lambda p: p["model"].update(trans_cost=[[math.inf, 1, 0], [0, math.inf, 0], [2, math.inf, math.inf]]),
     B.E_INVALID_ARG),
    (lambda p: p["model"].update(bic_cost=-1.0), B.E_INVALID_ARG),
    (lambda p: p["model"].update(trans_cost=[[0, 1, math.nan], [0, 0, 0], [0, 0, 0]]), B.E_INVALID_ARG),
    # exact-grid range: 2 (h+1) c_max must stay below 2^(24-g)
    (lambda p: p.update(cost_grid_log2=12), B.E_RANGE),
    (lambda p: p.update(max_height=1024, max_disparity=1024 // 4 + 1), B.E_INVALID_ARG),
])
def test_validation(mutate, code):
    p = synth.make_params()
    mutate(p)
    assert _rc(p) == code


def test_range_limits_at_paper_sizes():
    """The exact-arithmetic checks admit every workload size used here."""
    for (W, H, D) in [(1024, 440, 128), (2048, 880, 256), (1280, 720, 128), (640, 240, 128)]:
        p = synth.make_params(camera=synth.camera_for_size(W, H), max_width=W, max_height=H,
                              max_disparity=D)
        assert _rc(p) == 0
    p = synth.make_params(max_height=1024, max_disparity=256)
    assert _rc(p) == 0
    assert B.status_string(B.E_RANGE).startswith("parameters")


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        B.lib()


def test_record_decoding():
    raw = np.zeros((2, 3), np.int32)
    w = raw.view(np.uint32)
    w[0, 0] = 5 | (17 << 16)
    w[0, 1] = 0 | (42 << 8)
    raw[0, 2] = np.float32(12.5).view(np.int32)
    w[1, 0] = 18 | (439 << 16)
    w[1, 1] = 2
    raw[1, 2] = np.float32(-0.25).view(np.int32)
    d = B.decode_records(raw)
    assert list(d["v_bottom"]) == [5, 18] and list(d["v_top"]) == [17, 439]
    assert list(d["cls"]) == [0, 2] and list(d["disparity"]) == [42, 0]
    assert list(d["cost"]) == [12.5, -0.25]


def test_create_and_batch_reject_bad_arguments_without_a_device():
    """Validation happens before any HIP call, so it runs on the CPU."""
    import ctypes as C
    L = P.lib()
    p = synth.make_params()
    p["max_height"] = 2000
    h = C.c_void_p()
    assert L.stixels_create(C.byref(B.to_params(p)), C.byref(h)) == B.E_INVALID_ARG
    assert b"max_height" in L.stixels_last_error(None)
    assert L.stixels_create(None, C.byref(h)) == B.E_INVALID_ARG
    b = C.c_void_p()
    for cfg in [(0, 10, 440, 128), (1, 0, 440, 128), (1, 10, 1025, 128), (1, 10, 440, 300),
                (1, 10, 440, 1)]:
        c = B.BatchConfig()
        c.max_jobs, c.max_tasks, c.max_height, c.max_disparity = cfg
        assert L.stixels_batch_create(C.byref(c), C.byref(b)) == B.E_INVALID_ARG
    assert L.stixels_destroy(None) == 0 and L.stixels_batch_destroy(None) == 0
    assert L.stixels_set_waves(None, 1) == B.E_INVALID_ARG
    assert L.stixels_get_waves(None, 440, 1024) == 0
    assert L.stixels_set_po_placement(None, 1) == B.E_INVALID_ARG
    assert L.stixels_batch_set_waves(None, 2) == B.E_INVALID_ARG
    assert L.stixels_batch_waves(None) == 0
    assert L.stixels_batch_set_columns(None, 2) == B.E_INVALID_ARG
    assert L.stixels_batch_columns(None) == 0
    assert L.stixels_selftest_mean(1, 10, None) == B.E_INVALID_ARG
    n = C.c_int64()
    assert L.stixels_selftest_mean(256, 8192, C.byref(n)) == B.E_INVALID_ARG


@pytest.mark.parametrize("kw,code", [
    (dict(subpixel_log2=2), B.E_INVALID_ARG),            # 512 bins
    (dict(subpixel_log2=4, max_disparity=16), B.E_INVALID_ARG),
    (dict(subpixel_log2=-1), B.E_INVALID_ARG),
])
def test_subpixel_limits(kw, code):
    """Disparity bins (max_disparity << subpixel_log2) are limited to 256 and
    the exponent to 0..3."""
    p = synth.make_params(camera=synth.CAMERA_1024x440, **kw)
    with pytest.raises(B.StixelsError) as e:
        P.host_table(p, B.TABLE_SKY)
    assert e.value.code == code


def test_host_tables_off_the_grid_equal_oracle_in_fp32():
    """cost_grid_log2 = -1: no rounding onto a grid; the library's FP32
    tables are the oracle's FP64 values rounded once to FP32."""
    p = synth.make_params(camera=synth.CAMERA_1024x440, cost_grid_log2=-1)
    H = p["max_height"]
    t = oracle.tables(p, H)
    assert np.array_equal(P.host_table(p, B.TABLE_SKY), t["S"].astype(np.float32))
    assert np.array_equal(P.host_table(p, B.TABLE_GROUND)[::-1], t["G"].astype(np.float32))
    assert np.array_equal(P.host_table(p, B.TABLE_OBJECT).T, t["O"].astype(np.float32))
    assert np.array_equal(P.host_table(p, B.TABLE_FG_HI)[::-1], t["fg_hi"][:H])
    # some table value really is off the 2^-10 grid
    assert np.any(np.ldexp(t["S"], 10) != np.rint(np.ldexp(t["S"], 10)))


def test_bench_reads_the_active_shader_clock_level(tmp_path):
    """The bench's clock sampler parses the DPM level marked active."""
    import bench
    f = tmp_path / "pp_dpm_sclk"
    f.write_text("0: 500Mhz\n1: 1600Mhz\n2: 2400Mhz *\n")
    assert bench.read_sclk_mhz(str(f)) == 2400.0
    f.write_text("0: 500Mhz\n1: 1600Mhz\n")
    assert bench.read_sclk_mhz(str(f)) is None
    assert bench.read_sclk_mhz(str(tmp_path / "missing")) is None
    with bench.ClockSampler(None) as c:
        pass
    assert c.median() is None
