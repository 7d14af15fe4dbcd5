"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Everything the method computes is exact on the 2^-g cost grid, so the bar is
bit-exact equality: reduced disparities, offline and prefix tables, stixel
boundaries, classes, object disparities, per-stixel and per-column costs.
(This is stricter than a relative cost tolerance of 1e-4.)
"""

import math

import numpy as np
import pytest

import oracle
import synth
import paper_1610_04124_amd as P
from paper_1610_04124_amd import binding as B
from gpu_helpers import announce, assert_frames_equal, gpu_frame, to_device

pytestmark = pytest.mark.gpu


def handle_for(W, H, s=5, D=128, **kw):
    cam = kw.pop("camera", None) or synth.camera_for_size(W, H)
    model = kw.pop("model", None)
    p = synth.make_params(camera=cam, model=model, stixel_width=s, max_disparity=D,
                          max_width=W, max_height=H, **kw)
    return p, P.Stixels(p)


def test_selftest_rounded_mean():
    for D, Hm in [(128, 1024), (256, 1024), (2, 1024), (200, 880)]:
        announce(f"selftest_mean D={D} H={Hm}")
        assert P.selftest_mean(D, Hm) == 0


@pytest.mark.parametrize("W,H,D", [(1024, 440, 128), (2048, 880, 256)])
def test_device_tables_equal_oracle(W, H, D):
    announce(f"tables {W}x{H} D={D}")
    p, h = handle_for(W, H, D=D)
    t = oracle.tables(p, H)
    assert np.array_equal(h.debug_table(B.TABLE_SKY).astype(np.float64), t["S"])
    assert np.array_equal(h.debug_table(B.TABLE_GROUND)[::-1].astype(np.float64), t["G"])
    assert np.array_equal(h.debug_table(B.TABLE_OBJECT).T.astype(np.float64), t["O"])
    assert np.array_equal(h.debug_table(B.TABLE_FG_HI)[::-1], t["fg_hi"][:H])
    assert np.array_equal(h.debug_table(B.TABLE_FG_LO)[::-1], t["fg_lo"][:H])


STAGE_CASES = [
    # W, H, s, D, reduce_mode, seed
    (37, 1, 5, 64, 0, 1), (23, 2, 3, 32, 0, 2), (64, 63, 1, 128, 0, 3),
    (130, 64, 5, 128, 1, 4), (71, 65, 7, 256, 0, 5), (50, 129, 16, 128, 0, 6),
    (200, 200, 5, 128, 1, 7), (33, 440, 3, 128, 0, 8),
]


@pytest.mark.parametrize("W,H,s,D,mode,seed", STAGE_CASES)
def test_stage_parity(W, H, s, D, mode, seed):
    """Intermediates: reduction, the four small prefix tables, the column
    disparity range and the object prefix rows, against the oracle."""
    announce(f"stages W={W} H={H} s={s} D={D} mode={mode} seed={seed}")
    p, h = handle_for(W, H, s=s, D=D, reduce_mode=mode,
                      camera=dict(synth.CAMERA_1024x440, horizon_row=float(H // 3)))
    disp = synth.random_columns_frame(seed, W, H, D)
    gpu_frame(h, disp)
    q = oracle.reduce(p, disp)
    assert np.array_equal(h.debug_stage(B.STAGE_REDUCED, W, H).astype(np.int32), q)
    pre = h.debug_stage(B.STAGE_PREFIX, W, H).astype(np.float64)
    rng = h.debug_stage(B.STAGE_RANGE, W, H)
    po = h.debug_stage(B.STAGE_OBJECT_PREFIX, W, H).astype(np.float64)
    for i in range(W // s):
        c = oracle.column(p, q[i])
        assert np.array_equal(pre[0, i], c["PG"]), i
        assert np.array_equal(pre[1, i], c["PS"]), i
        assert np.array_equal(pre[2, i], 2 * c["PD"] + c["PN"]), i
        assert np.array_equal(pre[3, i], 2 * c["PN"]), i
        valid = q[i][q[i] >= 0]
        # the table starts at disparity 0 when the column has an invalid pixel
        lo, hi = (int(valid.min()), int(valid.max())) if valid.size else (0, 0)
        if valid.size < H:
            lo = 0
        assert tuple(rng[i]) == (lo, hi)
        assert np.array_equal(po[i, : hi - lo + 1], c["PO"][lo:hi + 1]), i


def small_cases():
    cases = []
    rng = np.random.default_rng(2024)
    for H in (1, 2, 3, 17, 63, 64, 65, 100, 127, 128, 129, 257, 300):
        s = int(rng.choice([1, 3, 5, 7, 16]))
        W = int(s * rng.integers(1, 40) + rng.integers(0, s))
        D = int(rng.choice([16, 64, 128, 256]))
        cases.append((W, H, s, D, int(rng.integers(0, 2)), int(rng.integers(1 << 30))))
    return cases


@pytest.mark.parametrize("W,H,s,D,mode,seed", small_cases())
def test_frame_parity_adversarial(W, H, s, D, mode, seed):
    """Ragged widths, heights around the 64-row slot boundaries, every kind of
    invalid pixel, both reduction operators."""
    announce(f"adversarial W={W} H={H} s={s} D={D} mode={mode} seed={seed}")
    cam = dict(synth.CAMERA_1024x440, horizon_row=float(int(seed % max(H, 1))))
    p, h = handle_for(W, H, s=s, D=D, reduce_mode=mode, camera=cam)
    disp = synth.random_columns_frame(seed, W, H, D)
    assert_frames_equal(gpu_frame(h, disp), oracle.frame(p, disp), f"adv {W}x{H}")


def perturbed_models():
    out = []
    rng = np.random.default_rng(7)
    for i in range(4):
        m = dict(synth.DEFAULT_MODEL)
        m["bic_cost"] = float(rng.uniform(0, 6))
        m["ordering_cost"] = float(rng.uniform(0, 8))
        m["ordering_tol_px"] = int(rng.integers(0, 4))
        m["gravity_cost"] = float(rng.uniform(0, 6))
        m["diving_cost"] = float(rng.uniform(0, 30))
        m["gravity_tol_px"] = float(rng.uniform(0, 4))
        m["diving_tol_px"] = float(rng.uniform(0, 4))
        m["sigma_disp"] = float(rng.uniform(0.5, 2))
        m["p_out"] = float(rng.uniform(0.05, 0.4))
        m["first_cost"] = [float(x) for x in rng.uniform(0, 5, 3)]
        T = [[float(x) for x in row] for row in rng.uniform(0, 3, (3, 3))]
        if i % 2 == 0:
            T[1][1] = T[2][1] = T[2][2] = math.inf
        m["trans_cost"] = T
        out.append(m)
    return out


@pytest.mark.parametrize("mi", range(4))
def test_frame_parity_perturbed_models(mi):
    m = perturbed_models()[mi]
    announce(f"perturbed model {mi}")
    p, h = handle_for(320, 200, s=5, D=128, model=m,
                      camera=synth.camera_for_size(320, 200))
    disp = synth.generate_frame(synth.SceneSpec(320, 200, 128, synth.camera_for_size(320, 200),
                                                seed=mi))
    assert_frames_equal(gpu_frame(h, disp), oracle.frame(p, disp), f"model {mi}")


@pytest.mark.parametrize("seed,waves", [(0, 1), (1, 2), (2, 4), (0, 4)])
def test_frame_parity_1024x440(seed, waves):
    """The paper's headline frame: 1024x440, stixel width 5, 204 columns,
    with 1, 2 and 4 wavefronts per column."""
    announce(f"1024x440 seed={seed} waves={waves}")
    p, h = handle_for(1024, 440)
    disp = synth.generate_frame(synth.SceneSpec(seed=seed))
    assert_frames_equal(gpu_frame(h, disp, waves=waves), oracle.frame(p, disp),
                        f"1024x440 seed {seed} waves {waves}")


def multiwave_cases():
    """Heights around the 64-row slot boundaries and slot counts that the
    waves do not divide (the last wave holds a padding slot)."""
    cases = []
    rng = np.random.default_rng(77)
    for H in (65, 127, 128, 129, 191, 193, 250, 257, 320, 449, 513, 700):
        for waves in (2, 4):
            if waves == 4 and H <= 192:
                continue
            s = int(rng.choice([1, 3, 5, 7]))
            W = int(s * rng.integers(2, 30) + rng.integers(0, s))
            D = int(rng.choice([64, 128, 256]))
            cases.append((W, H, s, D, waves, int(rng.integers(1 << 30))))
    return cases


@pytest.mark.parametrize("W,H,s,D,waves,seed", multiwave_cases())
def test_frame_parity_multiwave(W, H, s, D, waves, seed):
    announce(f"multiwave W={W} H={H} s={s} D={D} waves={waves} seed={seed}")
    cam = dict(synth.CAMERA_1024x440, horizon_row=float(seed % H))
    p, h = handle_for(W, H, s=s, D=D, camera=cam)
    disp = synth.random_columns_frame(seed, W, H, D)
    assert_frames_equal(gpu_frame(h, disp, waves=waves), oracle.frame(p, disp),
                        f"multiwave {W}x{H} waves {waves}")


@pytest.mark.parametrize("s,waves", [(3, 1), (5, 2), (5, 4)])
def test_frame_parity_2048x880(s, waves):
    """High resolution: 880 rows (14 row slots), d_range 256."""
    announce(f"2048x880 s={s} waves={waves}")
    W, H = 2048, 880
    cam = synth.camera_for_size(W, H)
    p, h = handle_for(W, H, s=s, D=256, camera=cam)
    disp = synth.generate_frame(synth.SceneSpec(W, H, 256, cam, seed=s))
    assert_frames_equal(gpu_frame(h, disp, waves=waves), oracle.frame(p, disp),
                        f"2048x880 s={s} waves={waves}")


@pytest.mark.parametrize("waves", [1, 4])
def test_frame_parity_max_height(waves):
    """h = 1024, the largest height a handle accepts (16 row slots)."""
    announce(f"max height 1024 waves={waves}")
    W, H = 45, 1024
    p, h = handle_for(W, H, s=5, D=128, camera=dict(synth.CAMERA_1024x440, horizon_row=400.0))
    disp = synth.random_columns_frame(11, W, H, 128)
    assert_frames_equal(gpu_frame(h, disp, waves=waves), oracle.frame(p, disp),
                        f"h=1024 waves {waves}")


def test_many_stixels_per_column():
    """Columns with more than 64 stixels take the second backtracking pass."""
    announce("many stixels")
    W, H = 15, 440
    m = dict(synth.DEFAULT_MODEL, bic_cost=0.0)
    p, h = handle_for(W, H, s=5, D=128, model=m,
                      camera=dict(synth.CAMERA_1024x440, horizon_row=500.0))
    rows = np.arange(H)
    col = np.where((rows // 3) % 2 == 0, 10.0, 100.0)
    disp = np.repeat(col[:, None], W, axis=1).astype(np.float32)
    ref = oracle.frame(p, disp)
    assert ref["counts"].max() > 64
    assert_frames_equal(gpu_frame(h, disp), ref, "many stixels")
    assert_frames_equal(gpu_frame(h, disp, waves=4), ref, "many stixels, 4 waves")
    h.set_waves(0)
    for cap in (1, 7, 100):
        assert_frames_equal(gpu_frame(h, disp, capacity=cap), oracle.frame(p, disp, cap=cap),
                            f"many stixels cap {cap}")


@pytest.mark.parametrize("cap", [1, 2, 3])
def test_capacity_truncation(cap):
    announce(f"capacity {cap}")
    p, h = handle_for(1024, 440)
    disp = synth.generate_frame(synth.SceneSpec(seed=5))
    assert_frames_equal(gpu_frame(h, disp, capacity=cap), oracle.frame(p, disp, cap=cap),
                        f"cap {cap}")


def test_all_invalid_and_degenerate_frames():
    announce("degenerate frames")
    p, h = handle_for(100, 120)
    for disp in (np.full((120, 100), -1, np.float32), np.zeros((120, 100), np.float32),
                 np.full((120, 100), np.nan, np.float32), np.full((120, 100), 1e30, np.float32)):
        assert_frames_equal(gpu_frame(h, disp), oracle.frame(p, disp), "degenerate")
    # a frame narrower than the handle's maximum, and W == s (one column)
    disp = synth.random_columns_frame(3, 5, 120, 128)
    assert_frames_equal(gpu_frame(h, disp), oracle.frame(p, disp), "one column")


def test_deterministic_and_reusable():
    announce("determinism")
    p, h = handle_for(1024, 440)
    disp = synth.generate_frame(synth.SceneSpec(seed=9))
    a = gpu_frame(h, disp)
    b = gpu_frame(h, disp)
    for k in ("counts", "total", "overflow"):
        assert np.array_equal(a[k], b[k])
    assert np.array_equal(a["records"], b["records"])


@pytest.mark.parametrize("W,H,s,D,waves,placement,seed", [
    (1024, 440, 5, 128, 1, 2, 0), (1024, 440, 5, 128, 4, 2, 1), (1024, 440, 5, 128, 1, 1, 2),
    (300, 440, 5, 256, 1, 2, 3), (300, 440, 5, 256, 2, 2, 4), (97, 129, 3, 64, 2, 2, 5),
    (50, 512, 5, 128, 4, 2, 6), (64, 1, 1, 16, 1, 2, 7), (80, 65, 5, 256, 1, 2, 8),
])
def test_frame_parity_po_placement(W, H, s, D, waves, placement, seed):
    """Object prefix table in LDS (where it fits, per column) or in HBM; the
    random-column frames mix tables that fit with tables that do not."""
    announce(f"po placement {placement} W={W} H={H} s={s} D={D} waves={waves} seed={seed}")
    if W == 1024:
        p, h = handle_for(W, H, s=s, D=D)
        disp = synth.generate_frame(synth.SceneSpec(seed=seed))
    else:
        cam = dict(synth.CAMERA_1024x440, horizon_row=float(seed * 37 % H))
        p, h = handle_for(W, H, s=s, D=D, camera=cam)
        disp = synth.random_columns_frame(seed, W, H, D)
    got = gpu_frame(h, disp, waves=waves, po_placement=placement)
    assert_frames_equal(got, oracle.frame(p, disp), f"po placement {placement} {W}x{H}")


def test_waves_setting():
    announce("waves setting")
    p, h = handle_for(1024, 440)
    for w in (1, 2, 4):
        h.set_waves(w)
        assert h.waves(1024, 440) == w
        assert h.waves(1024, 100) == min(w, 2)      # 2 row slots
        assert h.waves(1024, 64) == 1
    h.set_waves(0)
    assert h.waves(1024, 440) in (1, 2, 4)
    for bad in (3, 5, -1, 8):
        with pytest.raises(B.StixelsError) as ei:
            h.set_waves(bad)
        assert ei.value.code == B.E_INVALID_ARG
    for bad in (-1, 3):
        with pytest.raises(B.StixelsError) as ei:
            h.set_po_placement(bad)
        assert ei.value.code == B.E_INVALID_ARG


def test_errors_leave_outputs_untouched():
    import torch
    announce("error paths")
    p, h = handle_for(200, 100)
    out = P.FrameOutput(40, 100, torch.device("cuda", 0))
    out.counts.fill_(-7)
    good = to_device(np.zeros((100, 200), np.float32))
    for shape in [(100, 4), (101, 200), (100, 205), (0, 200)]:
        bad = to_device(np.zeros(shape, np.float32)) if shape[0] > 0 else good[:0]
        with pytest.raises(B.StixelsError) as ei:
            h.compute(bad, out)
        assert ei.value.code == B.E_INVALID_ARG
    out0 = P.FrameOutput(40, 0, torch.device("cuda", 0))
    with pytest.raises(B.StixelsError):
        h.compute(good, out0)
    torch.cuda.synchronize()
    assert bool((out.counts == -7).all())
