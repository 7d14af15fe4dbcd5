"""Benchmark: stixel frames/s at 1024x440, stixel width 5, on one MI355X.

One step = the whole hot path (column reduction, prefix tables, the
three-class recurrence and backtracking) over one batch of 64 synthetic
1024x440 frames (seeds 0..63), inputs resident in HBM.  The timed path is the
persistent batched launch replayed from a HIP graph.  Beside it: the plain
per-frame path (three staged kernels, and one fused launch) with per-frame
latency percentiles and the HBM fraction of its reduction and table kernels;
the 2048x880 batches; the 256-frame uneven batch; 64 stereo pairs through
the semi-global matching stage and on into stixels; serving of 8 camera
streams for 60 s; the CPU oracle on the host cores.

Prints one JSON line.  Roofline of the dominant kernel (the persistent
kernel): algorithmic work = 13 VALU lane-ops per (cut, row) pair of the
recurrence (ground, sky and object candidate: prefix differences, the
object mean, adds and minima), h(h+1)/2 pairs per column, against the plain
VALU issue peak of 256 CUs x 64 lanes x 2.4 GHz = 39.32 T lane-ops/s (the
recurrence is min-plus, not a contraction, so MFMA peaks do not apply).  The
fraction by the 7 lane-ops the object candidate alone needs (the ground and
sky minima are separable) is reported beside it, and the fraction at the
shader clock read from sysfs while the replays are timed.

    python bench.py [--steps K] [--warmup W]          the JSON line
    python bench.py --profile-mode MODE [--launches N] one workload for rocprofv3
    python bench.py --profile-mode batch --phase-timing the per-phase split of a task
"""

from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stixel frames/s @1024×440 w=5 (batched vs per-frame); p50/p99 frame latency"
W, H, S_WIDTH, D_RANGE, FRAMES = 1024, 440, 5, 128, 64
VALU_PEAK = 256 * 64 * 2.4e9              # lane-ops/s
HBM_PEAK = 8.0e12                         # bytes/s
OPS_PER_PAIR = 13                         # algorithmic lane-ops per (cut, row) pair
OPS_SEPARABLE = 7                         # the object candidate's share alone


def pairs_per_frame(W=W, H=H, s=S_WIDTH):
    return (W // s) * H * (H + 1) // 2


def kernel_source_hash():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1610_04124_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def profile_record(kernel, workgroups):
    """HBM bytes per launch of the persistent kernel (and its VALU busy
    fraction where taken) from the committed PMC summary, if it was taken on
    the current kernel sources and kernel variant and covers this number of
    workgroups: (bytes or None, busy or None)."""
    path = os.path.join(ROOT, "profiles", "batch_kernel_1024x440_b64_traffic.json")
    if not os.path.exists(path):
        return None, None
    try:
        d = json.load(open(path))
    except Exception:
        return None, None
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("kernel") != kernel:
        return None, None
    rec = d.get("by_workgroups", {}).get(str(workgroups))
    busy = d.get("valu_busy_by_workgroups", {}).get(str(workgroups))
    return (rec.get("hbm_bytes_per_launch") if rec else None), busy


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def r4(x):
    return None if x is None else round(float(x), 4)


def shader_clock_mhz():
    """Current shader clock from rocm-smi (run before this process touches
    the GPU), or None."""
    try:
        out = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True,
                             timeout=20).stdout
    except Exception:
        return None
    for line in out.splitlines():
        if "sclk" in line and "Mhz" in line:
            tok = line.split("(")[-1].split("Mhz")[0]
            try:
                return float(tok)
            except ValueError:
                continue
    return None


def sclk_sysfs_path(index=0):
    """sysfs file of the device's shader clock levels (the active one is
    marked '*'), found by the device's PCI address, or None."""
    import torch
    p = torch.cuda.get_device_properties(index)
    path = (f"/sys/bus/pci/devices/{p.pci_domain_id:04x}:{p.pci_bus_id:02x}:"
            f"{p.pci_device_id:02x}.0/pp_dpm_sclk")
    return path if os.path.exists(path) else None


def read_sclk_mhz(path):
    try:
        for line in open(path):
            if "*" in line:
                return float(line.split(":", 1)[1].lower().split("mhz")[0])
    except (OSError, ValueError, IndexError):
        pass
    return None


class ClockSampler:
    """Reads the active shader clock level from sysfs on a thread, every few
    milliseconds, while a timed region runs (a file read: no process is
    started).  median() is None where the file is not readable."""

    def __init__(self, path, period_s=0.002):
        self.path, self.period, self.samples = path, period_s, []

    def __enter__(self):
        import threading
        self.stop = threading.Event()
        self.thread = None
        if self.path:
            def run():
                while not self.stop.is_set():
                    v = read_sclk_mhz(self.path)
                    if v is not None:
                        self.samples.append(v)
                    self.stop.wait(self.period)
            self.thread = threading.Thread(target=run, daemon=True)
            self.thread.start()
        return self

    def __exit__(self, *exc):
        self.stop.set()
        if self.thread:
            self.thread.join()
        return False

    def median(self):
        return statistics.median(self.samples) if self.samples else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# ------------------------------------------------------------------ workloads

def headline_frames():
    import synth
    return [synth.generate_frame(synth.SceneSpec(seed=i)) for i in range(FRAMES)]


def uneven_items(dev, flags=0):
    """The 256 frames of the uneven workload (sizes 640x240 .. 2048x880,
    stixel widths 3/5/7, own camera per size) with one handle per (size,
    stixel width) and outputs; returns items and total (cut, row) pairs."""
    import torch

    import synth
    import paper_1610_04124_amd as P

    handles, items, pairs = {}, [], 0
    for i in range(256):
        disp, info = synth.workload_frame("uneven256", i)
        Wf, Hf, s = info["width"], info["height"], info["stixel_width"]
        key = (Wf, Hf, s)
        if key not in handles:
            p = synth.make_params(camera=info["camera"], stixel_width=s,
                                  max_disparity=info["d_max"], max_width=Wf, max_height=Hf,
                                  flags=flags)
            handles[key] = P.Stixels(p)
        h = handles[key]
        items.append((h, torch.from_numpy(disp).to(dev), h.new_output(Wf, Hf)))
        pairs += (Wf // s) * Hf * (Hf + 1) // 2
    return items, pairs


def time_replays(batch, stream, warmup, steps):
    """Graph replays timed with HIP events on the launch stream; returns
    (wall seconds, per-replay milliseconds)."""
    import torch
    for _ in range(warmup):
        batch.replay(stream)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        batch.replay(stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [s.elapsed_time(e) for s, e in zip(starts, ends)]


def tuned_capture(batch, items, stream, tune_launch):
    if tune_launch:
        from paper_1610_04124_amd.autotune import tune
        return tune(batch, items, stream, cache_path=None)
    batch.capture(items, stream)
    return None


def hires(warmup, steps, tune_launch=True):
    """16 frames of 2048x880 (d_range 256) at stixel widths 3 and 5, one
    batched graph replay per step."""
    import torch

    import synth
    import paper_1610_04124_amd as P

    dev = torch.device("cuda", 0)
    Wh, Hh = 2048, 880
    cam = synth.camera_for_size(Wh, Hh)
    frames = [torch.from_numpy(synth.generate_frame(synth.SceneSpec(Wh, Hh, 256, cam, seed=i))).to(dev)
              for i in range(16)]
    out = {}
    stream = torch.cuda.Stream()
    for s in (3, 5):
        params = synth.make_params(camera=cam, stixel_width=s, max_disparity=256, max_width=Wh,
                                   max_height=Hh, flags=P.binding.FLAG_BATCH_ONLY)
        h = P.Stixels(params)
        outs = [h.new_output(Wh, Hh) for _ in frames]
        b = P.Batch(16, 16 * (Wh // s), Hh, 256)
        torch.cuda.synchronize()
        tuned_capture(b, list(zip([h] * 16, frames, outs)), stream, tune_launch)
        wall, ms = time_replays(b, stream, warmup, steps)
        dt = wall / steps
        avg = statistics.mean(ms) * 1e-3
        pairs = 16 * (Wh // s) * Hh * (Hh + 1) // 2
        g, _ = b.info()
        out[f"s{s}"] = {"fps": round(16 / dt, 2), "ms_per_batch": round(dt * 1e3, 4),
                        "valu_frac": round(OPS_PER_PAIR * pairs / avg / VALU_PEAK, 4),
                        "valu_frac_7op": round(OPS_SEPARABLE * pairs / avg / VALU_PEAK, 4),
                        "waves_per_column": b.waves(), "columns_per_wave": b.columns(),
                        "workgroups": g}
    return out


def mean_mode(d_frames, warmup, steps, tune_launch=True):
    """The batched headline workload with the paper's own reduction (the
    mean of each strip's valid pixels, Sec. 4.1) instead of the median."""
    import torch

    import synth
    import paper_1610_04124_amd as P

    params = synth.make_params(reduce_mode=1, flags=P.binding.FLAG_BATCH_ONLY)
    h = P.Stixels(params)
    outs = [h.new_output(W, H) for _ in d_frames]
    stream = torch.cuda.Stream()
    b = P.Batch(FRAMES, FRAMES * (W // S_WIDTH), H, D_RANGE)
    torch.cuda.synchronize()
    tuned_capture(b, list(zip([h] * FRAMES, d_frames, outs)), stream, tune_launch)
    wall, _ = time_replays(b, stream, warmup, steps)
    dt = wall / steps
    g, _ = b.info()
    return {"fps": round(FRAMES / dt, 2), "ms_per_batch": round(dt * 1e3, 4),
            "waves_per_column": b.waves(), "workgroups": g,
            "reduction": "mean of the strip's valid pixels (reduce_mode 1)"}


def uneven(warmup, steps, tune_launch=True):
    """The 256-frame uneven batch in one autotuned persistent launch."""
    import torch

    import paper_1610_04124_amd as P

    dev = torch.device("cuda", 0)
    items, pairs = uneven_items(dev, flags=P.binding.FLAG_BATCH_ONLY)
    ntasks = sum(h.num_columns(d.shape[1]) for h, d, _ in items)
    b = P.Batch(256, ntasks, 880, 256)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    tuned = tuned_capture(b, items, stream, tune_launch)
    wall, ms = time_replays(b, stream, warmup, steps)
    avg = statistics.mean(ms) * 1e-3
    g, t = b.info()
    res = {"fps": round(256 * steps / wall, 2), "ms_per_batch": round(wall * 1e3 / steps, 4),
           "batch_latency_ms_p50": r4(percentile(ms, 0.5)),
           "batch_latency_ms_p99": r4(percentile(ms, 0.99)),
           "valu_frac": round(OPS_PER_PAIR * pairs / avg / VALU_PEAK, 4),
           "frames": 256, "tasks": t, "workgroups": g, "waves_per_column": b.waves(),
           "columns_per_wave": b.columns(),
           "sizes": "640x240, 1024x440, 1280x720, 2048x880; stixel widths 3/5/7; one launch"}
    if tuned is not None:
        res["autotune_tried_ms"] = tuned["tried"]
        res["autotune_refined_ms"] = tuned.get("refined")
    return res


def sgm_bytes_per_frame(W=W, H=H, D=D_RANGE):
    """Algorithmic HBM bytes of the matching stage per frame: census (both
    images read, both word arrays written), each of the four path passes
    reading both word arrays once, the summed costs written (first pass),
    read and written (two passes) and read (last pass), the map written."""
    n = W * H
    return 2 * n + 16 * n + 4 * 16 * n + 2 * n * D * (1 + 2 + 2 + 1) + 4 * n


def stereo(warmup, steps, tune_launch=True):
    """64 rectified stereo pairs of the headline scenes (1024x440, 128
    disparities): the semi-global matching stage alone, and stereo pairs to
    stixels (matching, then the batched stixel launch on its maps, replayed
    from a HIP graph)."""
    import numpy as np
    import torch

    import synth
    from synth.stereo import StereoSpec, generate_stereo
    import paper_1610_04124_amd as P

    dev = torch.device("cuda", 0)
    pairs = [generate_stereo(StereoSpec(synth.SceneSpec(seed=i))) for i in range(FRAMES)]
    L = torch.from_numpy(np.stack([p[0] for p in pairs])).to(dev)
    R = torch.from_numpy(np.stack([p[1] for p in pairs])).to(dev)
    truth = np.stack([p[2] for p in pairs])
    m = P.Sgm(W, H, D_RANGE, max_frames=FRAMES)
    disp = torch.empty((FRAMES, H, W), dtype=torch.float32, device=dev)
    stream = torch.cuda.Stream()
    for _ in range(warmup):
        m.compute(L, R, disp, stream)
    torch.cuda.synchronize()
    seen = truth >= 0
    got = disp.cpu().numpy()
    accuracy = float(((got == truth) & seen).sum() / seen.sum())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    for i in range(steps):
        ev[2 * i].record(stream)
        m.compute(L, R, disp, stream)
        ev[2 * i + 1].record(stream)
    torch.cuda.synchronize()
    sgm_ms = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(steps)]
    sgm_s = statistics.mean(sgm_ms) * 1e-3
    bytes_frame = sgm_bytes_per_frame()

    h = P.Stixels(synth.make_params(flags=P.binding.FLAG_BATCH_ONLY))
    outs = [h.new_output(W, H) for _ in range(FRAMES)]
    b = P.Batch(FRAMES, FRAMES * (W // S_WIDTH), H, D_RANGE)
    tuned_capture(b, list(zip([h] * FRAMES, [disp[i] for i in range(FRAMES)], outs)), stream,
                  tune_launch)
    for _ in range(warmup):
        m.compute(L, R, disp, stream)
        b.replay(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        m.compute(L, R, disp, stream)
        b.replay(stream)
    torch.cuda.synchronize()
    both = (time.perf_counter() - t0) / steps
    return {"sgm_fps": round(FRAMES / sgm_s, 2), "sgm_ms_per_batch": round(sgm_s * 1e3, 4),
            "stereo_to_stixels_fps": round(FRAMES / both, 2),
            "stereo_to_stixels_ms_per_batch": round(both * 1e3, 4),
            "sgm_roofline": {"bound": "hbm", "bytes_per_frame": bytes_frame,
                             "achieved_GBps": round(bytes_frame * FRAMES / sgm_s / 1e9, 1),
                             "peak_GBps": HBM_PEAK / 1e9,
                             "frac": round(bytes_frame * FRAMES / sgm_s / HBM_PEAK, 4)},
            "disparity_equal_to_scene": round(accuracy, 4),
            "frames": FRAMES, "max_disparity": D_RANGE, "paths": 4, "p1": 10, "p2": 120,
            "census": "9x7", "workspace_bytes": m.device_bytes()}


def per_frame_legs(h, d_frames, outs, stream, steps, latency_frames, tune_launch):
    """The per-frame paths: three staged kernels and one fused launch.  Per
    path: throughput with frames back to back, and latency per frame (HIP
    events around each call, a synchronisation between frames).  For the
    staged path also the time of each kernel and the HBM fraction of the
    reduction and table kernels."""
    import torch

    from paper_1610_04124_amd import binding as B

    res = {}
    frame_tuned = None
    if tune_launch:
        from paper_1610_04124_amd.autotune import tune_frame
        frame_tuned = tune_frame(h, d_frames[0], outs[0], stream)
    for name, path in (("staged", 1), ("fused", 2)):
        h.set_frame_path(path)
        for i in range(len(d_frames)):
            h.compute(d_frames[i], outs[i], stream)
        torch.cuda.synchronize()
        reps = max(1, steps // 5)
        t0 = time.perf_counter()
        for _ in range(reps):
            for i in range(len(d_frames)):
                h.compute(d_frames[i], outs[i], stream)
        torch.cuda.synchronize()
        fps = len(d_frames) * reps / (time.perf_counter() - t0)
        lat = []
        for i in range(latency_frames):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            h.compute(d_frames[i % len(d_frames)], outs[i % len(d_frames)], stream)
            b.record(stream)
            b.synchronize()
            lat.append(a.elapsed_time(b))
        res[name] = {"fps": round(fps, 2), "frame_latency_ms_p50": r4(percentile(lat, 0.5)),
                     "frame_latency_ms_p99": r4(percentile(lat, 0.99))}
    h.set_frame_path(0)
    res["waves_per_column"] = h.waves(W, H)
    if frame_tuned is not None:
        res["po_placement"] = "lds" if frame_tuned["po_placement"] == 2 else "hbm"
        res["autotune_tried_ms"] = frame_tuned["tried"]
    # stage split: kernel times between HIP events, median over frames
    times = [h.stage_times(d_frames[i % len(d_frames)], outs[i % len(d_frames)], stream)
             for i in range(32)]
    med = [statistics.median(t[k] for t in times) for k in range(3)]
    rows = h.debug_stage(B.STAGE_RANGE, W, H, stream)
    po_rows = int(sum(int(hi) - int(lo) + 1 for lo, hi in rows))
    ncols = W // S_WIDTH
    red_bytes = 4 * S_WIDTH * ncols * H + 2 * ncols * H
    tab_bytes = 2 * ncols * H + 4 * 4 * ncols * (H + 1) + 4 * po_rows * (H + 1)
    res["stages"] = {
        "reduce_kernel": {"us": round(med[0] * 1e3, 2), "bytes": red_bytes,
                          "hbm_frac": round(red_bytes / (med[0] * 1e-3) / HBM_PEAK, 4)},
        "tables_kernel": {"us": round(med[1] * 1e3, 2), "bytes": tab_bytes,
                          "object_prefix_rows": po_rows,
                          "hbm_frac": round(tab_bytes / (med[1] * 1e-3) / HBM_PEAK, 4)},
        "dp_kernel": {"us": round(med[2] * 1e3, 2),
                      "valu_frac": round(OPS_PER_PAIR * pairs_per_frame() / (med[2] * 1e-3)
                                         / VALU_PEAK, 4)},
        "share": [round(x / sum(med), 4) for x in med],
        "bytes_note": "reduction: strips read + reduced column written; tables: reduced "
                      "column read + four small prefix tables + the object prefix rows of each "
                      "column's own disparity range written (last frame's range)"}
    return res


def serve(seconds, rate_scale=1.0, budget_frames=None, pool=32):
    """8 cameras (1024x440, 1280x720, 2048x880 by camera index, stixel width
    5) at 30 Hz Poisson each (times rate_scale), served with continuous
    batching in real time; every camera draws from `pool` distinct frames.
    The HBM budget covers the resident tables and scratch plus the admitted
    frames: 64 GiB, or with budget_frames the resident bytes plus that many
    footprints of the largest camera's frame (so that admission binds)."""
    import torch

    import synth
    from paper_1610_04124_amd.serving import (GpuExecutor, Server, poisson_arrivals,
                                              serving_cameras)

    dev = torch.device("cuda", 0)
    cams = serving_cameras(8)
    frames = {}
    for c, cam in enumerate(cams):
        Wc, Hc, D = cam.width, cam.height, cam.handle.D
        for i in range(pool):
            spec = synth.SceneSpec(Wc, Hc, D, synth.camera_for_size(Wc, Hc), seed=1000 * c + i)
            frames[(c, i)] = torch.from_numpy(synth.generate_frame(spec)).to(dev)
    ex = GpuExecutor(cams, streams=3, max_frames=64)
    layout = ex.tune({c: [frames[(c, i)] for i in range(8)] for c in range(len(cams))})
    resident = ex.resident_bytes()
    frame_bytes = sum(frames[(c, 0)].numel() * 4 for c in range(8)) * pool
    budget = 64 << 30
    if budget_frames:
        budget = resident + budget_frames * max(c.footprint() for c in cams)
    srv = Server(cams, ex, hbm_budget=budget, max_batch=64, keep_outputs=False,
                 resident_bytes=resident)
    arrivals = poisson_arrivals([30.0 * rate_scale] * 8, seconds, [42 + c for c in range(8)], pool)
    torch.cuda.synchronize()
    srv.run_trace(arrivals, lambda c, i: frames[(c, i)])
    torch.cuda.synchronize()
    st = srv.stats()
    st = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
    st.update({"arrivals": len(arrivals), "cameras": 8, "rate_hz_per_camera": 30 * rate_scale,
               "seconds": seconds, "distinct_frames_per_camera": pool,
               "frame_pool_bytes": frame_bytes,
               "layout_by_height_class": {str(k): v for k, v in sorted(layout.items())},
               "sizes": "1024x440, 1280x720, 2048x880 by camera index; stixel width 5"})
    return st


def cpu_baseline(frames, params, seconds_all=12.0, seconds_one=10.0):
    """The FP64 oracle as it stands on the host cores: all cores (OpenMP over
    columns), then one core, each on as many of the 64 frames as fit the
    time given (a bounded sample)."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    out = {}
    for label, nt, budget in (("all", threads, seconds_all), ("one", 1, seconds_one)):
        oracle.frame(params, frames[0], nthreads=nt)                # load / warm
        n, t0 = 0, time.perf_counter()
        while n < len(frames) and (n == 0 or time.perf_counter() - t0 < budget):
            oracle.frame(params, frames[n], nthreads=nt)
            n += 1
        dt = time.perf_counter() - t0
        out[label] = (n / dt, nt, n, dt)
    fps, nt, n, dt = out["all"]
    fps1, _, n1, dt1 = out["one"]
    return {"value": round(fps, 3), "unit": "frames/s", "cores": nt, "kind": "oracle",
            "sample": f"{n} of the {FRAMES} 1024x440 frames (seeds 0..{n - 1}), C FP64 oracle, "
                      f"OpenMP over columns, {dt:.2f} s wall ({dt * nt:.0f} core-seconds)",
            "one_core": {"value": round(fps1, 3), "unit": "frames/s", "cores": 1,
                         "sample": f"{n1} frames, {dt1:.2f} s wall"},
            "cpu_model": cpu_model()}


# ------------------------------------------------------------------ profile modes

def profile_mode(args):
    """One workload, for rocprofv3 runs:
    batch   the persistent batched launch over 64 frames 1024x440 (stixel
            width 5), replayed from a HIP graph --launches times;
    hires   the same over 16 frames of 2048x880 (stixel width 5, d_range 256);
    uneven  the 256-frame uneven batch;
    frame   the staged per-frame path (three kernels) on the 64 frames;
    fused   the fused per-frame path (one launch per frame) on the 64 frames;
    sgm     the semi-global matching stage over 64 stereo pairs 1024x440;
    copy    a plain 256 MiB device-to-device copy, whose FETCH_SIZE and
            WRITE_SIZE readings calibrate the HBM byte counters."""
    import torch

    dev = torch.device("cuda", 0)
    if args.profile_mode == "copy":
        n = 256 * 1024 * 1024 // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(args.launches):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copied {n * 4} bytes x {args.launches}", flush=True)
        return

    import synth
    import paper_1610_04124_amd as P

    stream = torch.cuda.Stream()
    if args.profile_mode == "sgm":
        import numpy as np
        from synth.stereo import StereoSpec, generate_stereo
        pairs = [generate_stereo(StereoSpec(synth.SceneSpec(seed=i))) for i in range(FRAMES)]
        L = torch.from_numpy(np.stack([p[0] for p in pairs])).to(dev)
        R = torch.from_numpy(np.stack([p[1] for p in pairs])).to(dev)
        m = P.Sgm(W, H, D_RANGE, max_frames=FRAMES)
        disp = torch.empty((FRAMES, H, W), dtype=torch.float32, device=dev)
        for _ in range(args.launches):
            m.compute(L, R, disp, stream)
        torch.cuda.synchronize()
        print(f"sgm: {args.launches} launches over {FRAMES} stereo pairs", flush=True)
        return
    if args.profile_mode == "uneven":
        items, _ = uneven_items(dev)
        ntasks = sum(h.num_columns(d.shape[1]) for h, d, _ in items)
        b = P.Batch(256, ntasks, 880, 256, args.workgroups)
        b.set_waves(args.waves)
        torch.cuda.synchronize()
        b.capture(items, stream)
        for _ in range(args.launches):
            b.replay(stream)
        torch.cuda.synchronize()
        print(f"uneven: {args.launches} launches over 256 frames", flush=True)
        return
    if args.profile_mode == "hires":
        Wp, Hp, D, nframes = 2048, 880, 256, 16
        cam = synth.camera_for_size(Wp, Hp)
        params = synth.make_params(camera=cam, max_width=Wp, max_height=Hp, max_disparity=D)
        specs = [synth.SceneSpec(Wp, Hp, D, cam, seed=i) for i in range(nframes)]
    else:
        Wp, Hp, D, nframes = W, H, D_RANGE, FRAMES
        params = synth.make_params()
        specs = [synth.SceneSpec(seed=i) for i in range(nframes)]
    h = P.Stixels(params)
    h.set_waves(args.waves)
    h.set_po_placement(args.placement)
    frames = [torch.from_numpy(synth.generate_frame(sp)).to(dev) for sp in specs]
    outs = [h.new_output(Wp, Hp) for _ in frames]
    torch.cuda.synchronize()
    if args.profile_mode in ("batch", "hires"):
        b = P.Batch(len(frames), len(frames) * (Wp // 5), Hp, D, args.workgroups)
        b.set_waves(args.waves)
        b.capture(list(zip([h] * len(frames), frames, outs)), stream)
        if args.phase_timing:
            b.replay(stream)                         # warm, then count the timed launches only
            b.phase_cycles(reset=True)
        for _ in range(args.launches):
            b.replay(stream)
        if args.phase_timing:
            print(json.dumps(phase_split(b, args.launches)), flush=True)
    else:
        h.set_frame_path(1 if args.profile_mode == "frame" else 2)
        for _ in range(args.launches):
            for f, o in zip(frames, outs):
                h.compute(f, o, stream)
    torch.cuda.synchronize()
    print(f"{args.profile_mode}: {args.launches} launches over {len(frames)} frames", flush=True)


def phase_split(batch, launches):
    """Per-task shader cycles of each phase of the persistent kernel and its
    share of the tasks' summed time (a library built with phase timing)."""
    c = batch.phase_cycles()
    g, _ = batch.info()
    tasks = max(1, c["tasks"])
    names = ("reduce", "prefix_scans", "object_table", "recurrence", "backtracking")
    total = sum(c[n] for n in names)
    return {"workgroups": g, "launches": launches, "tasks": c["tasks"],
            "cycles_per_task": {n: round(c[n] / tasks, 1) for n in names},
            "share": {n: round(c[n] / max(1, total), 4) for n in names},
            "task_cycles_over_lifetime": round(total / max(1, c["workgroup_lifetime"]), 4)}


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--latency-frames", type=int, default=200)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--profile-mode", choices=["batch", "hires", "uneven", "frame", "fused", "copy",
                                               "sgm"])
    ap.add_argument("--launches", type=int, default=3)
    ap.add_argument("--waves", type=int, default=0,
                    help="profile modes: waves per column (0: automatic per frame, one batched)")
    ap.add_argument("--workgroups", type=int, default=0,
                    help="profile modes: resident workgroups of the batched launch (0: occupancy)")
    ap.add_argument("--placement", type=int, default=0,
                    help="profile modes: object prefix table placement (0 auto, 1 HBM, 2 LDS)")
    ap.add_argument("--phase-timing", action="store_true",
                    help="profile modes batch/hires: load the library built with phase timing "
                         "(python -m paper_1610_04124_amd.build --phase-timing) and print the "
                         "per-phase split of the column tasks")
    args = ap.parse_args()
    if args.phase_timing:
        os.environ["STIXELS_PHASE_TIMING"] = "1"        # before the binding loads a library
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(frames and columns are independent, see the design notes "
                                   "on sharding)"}))
        sys.exit(2)
    if args.profile_mode:
        profile_mode(args)
        return

    sclk = shader_clock_mhz()             # before this process touches the GPU

    import torch

    import synth
    import paper_1610_04124_amd as P

    dev = torch.device("cuda", 0)
    params = synth.make_params()
    frames = headline_frames()
    d_frames = [torch.from_numpy(f).to(dev) for f in frames]
    h = P.Stixels(params)
    outs = [h.new_output(W, H) for _ in range(FRAMES)]
    stream = torch.cuda.Stream()            # a created stream: graphs cannot capture the null stream
    torch.cuda.synchronize()
    tune_launch = not args.no_tune

    # ---------------- batched path: persistent launch replayed from a graph
    batch = P.Batch(FRAMES, FRAMES * (W // S_WIDTH), H, D_RANGE)
    items = list(zip([h] * FRAMES, d_frames, outs))
    tuned = tuned_capture(batch, items, stream, tune_launch)
    grid, ntasks = batch.info()
    waves = batch.waves()
    columns = batch.columns()
    with ClockSampler(sclk_sysfs_path()) as clock:
        wall, launch_ms = time_replays(batch, stream, args.warmup, args.steps)
    batched_fps = FRAMES * args.steps / wall
    ms_per_step = wall * 1e3 / args.steps
    avg_launch_s = statistics.mean(launch_ms) * 1e-3

    # ---------------- roofline of the persistent kernel
    pairs = pairs_per_frame() * FRAMES
    ops = OPS_PER_PAIR * pairs
    achieved = ops / avg_launch_s
    kernel = f"batch_kernel<7, 2, {waves}>" if columns == 1 else "batch_pair_kernel<7, 2>"
    traffic, valu_busy = profile_record(kernel, grid)
    roofline = {"bound": "alu", "achieved": round(achieved / 1e12, 4),
                "peak": round(VALU_PEAK / 1e12, 4), "unit": "TOP/s",
                "frac": round(achieved / VALU_PEAK, 4), "traffic": traffic,
                "kernel": kernel, "ops_per_pair": OPS_PER_PAIR, "pairs_per_launch": pairs,
                "ops_per_launch": ops, "avg_launch_ms": round(avg_launch_s * 1e3, 4),
                "frac_7op": round(OPS_SEPARABLE * pairs / avg_launch_s / VALU_PEAK, 4),
                "valu_busy_counters": valu_busy,
                "sclk_mhz_at_start": sclk,
                "sclk_mhz_during_timing": clock.median(),
                "sclk_samples": len(clock.samples)}
    if clock.median():
        # the same fraction against the VALU rate at the clock observed while timing
        roofline["frac_at_observed_sclk"] = round(
            achieved / (VALU_PEAK * clock.median() / 2400.0), 4)

    # ---------------- per-frame paths
    per_frame = per_frame_legs(h, d_frames, outs, stream, args.steps, args.latency_frames,
                               tune_launch)

    result = {
        "metric": METRIC, "value": round(batched_fps, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch64_1024x440", "frames_per_step": FRAMES, "width": W,
                   "height": H, "stixel_width": S_WIDTH, "max_disparity": D_RANGE,
                   "columns_per_frame": W // S_WIDTH,
                   "path": "persistent batched launch replayed from a HIP graph",
                   "workgroups": grid, "tasks": ntasks, "waves_per_column": waves,
                   "columns_per_wave": columns},
        "batched": {"fps": round(batched_fps, 2),
                    "batch_latency_ms_p50": r4(percentile(launch_ms, 0.5)),
                    "batch_latency_ms_p99": r4(percentile(launch_ms, 0.99))},
        "per_frame": per_frame,
        "roofline": roofline,
        "paper_context_fps": {"titan_x": 413, "tegra_x1": 26, "i7_980x_cpu": 13.3},
    }
    if tuned is not None:
        result["config"]["autotune_tried_ms"] = tuned["tried"]
        result["config"]["autotune_refined_ms"] = tuned.get("refined")
    print("[bench] batched and per-frame legs done", file=sys.stderr, flush=True)
    result["hires_2048x880"] = hires(args.warmup, max(3, args.steps // 5), tune_launch)
    result["batched_mean_reduction"] = mean_mode(d_frames, args.warmup, max(3, args.steps // 5),
                                                 tune_launch)
    result["uneven256"] = uneven(args.warmup, max(3, args.steps // 5), tune_launch)
    print("[bench] hires, mean and uneven legs done", file=sys.stderr, flush=True)
    result["stereo64_1024x440"] = stereo(args.warmup, max(3, args.steps // 5), tune_launch)
    print("[bench] stereo leg done", file=sys.stderr, flush=True)
    if args.serve_seconds > 0:
        result["serving"] = serve(args.serve_seconds)
        print("[bench] serving at 30 Hz done", file=sys.stderr, flush=True)
        # the same cameras at 16x the rate: continuous batching under load
        loaded_s = min(10.0, args.serve_seconds)
        result["serving_loaded"] = serve(loaded_s, rate_scale=16.0)
        # and with an HBM budget that binds: the resident bytes plus room for
        # 8 frames of the largest camera
        result["serving_admission_bound"] = serve(loaded_s, rate_scale=16.0, budget_frames=8)
        print("[bench] serving legs done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(frames, params)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
