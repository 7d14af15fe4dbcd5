"""Continuous-batching request loop for many camera streams.

Frames arrive from several cameras (each camera: one handle, i.e. its model
and offline tables resident in HBM).  Each request is admitted as soon as a
launch slot and HBM are free for it, and every admitted request that is
waiting when a launch slot frees up joins the next batched launch.  Launches
go out on several streams, so a batch admitted while others run overlaps
them on the device.  Admission charges each frame's HBM footprint (its input
and outputs) against a budget from which the resident bytes (the cameras'
tables and the batch objects' scratch) are taken once.  Latency is measured
from arrival to completion.

The loop is written against a small executor interface, so the admission
and batching logic can run against a mock executor on the CPU; the GPU
executor issues stixels_batch_compute on HIP streams.
"""

from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field


@dataclass
class CameraSpec:
    handle: object            # paper_1610_04124_amd.Stixels (or a stand-in for the mock)
    width: int
    height: int

    def ncols(self) -> int:
        return self.width // self.handle.s

    def height_class(self) -> int:
        """64-row slots per lane of the recurrence: frames of one class share
        a kernel variant and a batch object."""
        return (self.height + 63) // 64

    def footprint(self) -> int:
        """HBM bytes a frame of this camera holds while admitted: its input
        and the outputs allocated for it.  The tables and scratch the
        kernels use are resident (the handles' tables, the executor's batch
        objects) and are charged once, not per frame."""
        ncols, H = self.ncols(), self.height
        cap = H
        return 4 * self.width * H + ncols * (4 + 12 * cap + 4 + 1)


@dataclass(eq=False)
class Request:
    rid: int
    camera: int
    frame: object             # device tensor [H, W] (or any token for the mock)
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    out: object = None
    cancelled: bool = False

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class GpuExecutor:
    """Batched launches on `streams` HIP streams.  Every stream owns one batch
    object per height class, so the launches of one admission (one per
    class) never wait on each other's descriptor uploads."""

    def __init__(self, cameras, streams: int = 3, max_frames: int = 64):
        import torch

        import paper_1610_04124_amd as P

        self.cameras = cameras
        self.max_frames = max_frames
        self.classes = {}
        for c in cameras:
            k = c.height_class()
            hmax, dmax, cols = self.classes.get(k, (0, 0, 0))
            self.classes[k] = (max(hmax, c.height), max(dmax, c.handle.D), max(cols, c.ncols()))
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.batches = [{k: P.Batch(max_frames, max_frames * cols, hmax, dmax)
                         for k, (hmax, dmax, cols) in self.classes.items()}
                        for _ in range(streams)]
        self.free = list(range(streams))
        self._torch = torch
        self._P = P
        # launch layout of each height class: (columns per wave, waves per
        # column, workgroups); untuned classes use one wave per column for
        # up to 8 slots and two above, the autotuner's choice at 440 and 880
        # rows on MI355X, and the occupancy limit
        self.layout = {}

    def layout_for(self, k: int):
        return self.layout.get(k, (1, 1 if k <= 8 else 2, 0))

    def resident_bytes(self) -> int:
        """Device bytes held for the whole run: the batch objects and the
        cameras' handles (tables, and workspace unless batch-only)."""
        n = sum(b.device_bytes() for per in self.batches for b in per.values())
        seen = set()
        for c in self.cameras:
            if id(c.handle) not in seen:
                seen.add(id(c.handle))
                n += c.handle.device_bytes()
        return n

    def tune(self, frames_by_camera, max_frames: int = 16):
        """Time the launch layout of every height class on sample frames
        (camera index -> list of device frames) and keep the fastest."""
        from paper_1610_04124_amd.autotune import tune

        st = self.streams[0]
        members = {}
        for ci, frames in frames_by_camera.items():
            c = self.cameras[ci]
            for f in frames:
                members.setdefault(c.height_class(), []).append((c, f))
        for k, mem in members.items():
            mem = mem[:max_frames]
            items = [(c.handle, f, c.handle.new_output(c.width, c.height)) for c, f in mem]
            rec = tune(self.batches[0][k], items, st, replays=3, cache_path=None)
            self.layout[k] = (rec["columns"], rec["waves"], 0)
        self._torch.cuda.synchronize()
        return {k: {"columns": v[0], "waves": v[1]} for k, v in self.layout.items()}

    def slots(self) -> int:
        return len(self.free)

    def launch(self, reqs):
        """Allocate the requests' outputs and enqueue the batched launches,
        all on one stream (the allocation's zero fill is stream-ordered before
        the kernels that write the results).  Frames are grouped by height
        class, one launch per class, so short frames never run the
        register-heavy variant sized for tall ones."""
        i = self.free.pop()
        st = self.streams[i]
        with self._torch.cuda.stream(st):
            for r in reqs:
                c = self.cameras[r.camera]
                r.out = c.handle.new_output(c.width, c.height)
        groups = {}
        for r in reqs:
            groups.setdefault(self.cameras[r.camera].height_class(), []).append(r)
        for k in sorted(groups, reverse=True):
            items = [(self.cameras[r.camera].handle, r.frame, r.out) for r in groups[k]]
            b = self.batches[i][k]
            cols, waves, wg = self.layout_for(k)
            b.set_columns(cols)
            b.set_waves(waves)
            b.set_workgroups(wg)
            b.compute(items, st)
        ev = self._torch.cuda.Event()
        ev.record(st)
        return (i, ev)

    def finished(self, token) -> bool:
        i, ev = token
        if ev.query():
            self.free.append(i)
            return True
        return False


class Server:
    """Admission by HBM footprint + continuous batching over an executor."""

    def __init__(self, cameras, executor, hbm_budget: int, max_batch: int = 64,
                 clock=time.perf_counter, keep_outputs: bool = True, resident_bytes: int = 0):
        """hbm_budget covers everything the run holds on the device: the
        resident bytes (tables and batch scratch, charged once) plus the
        footprints of the admitted frames."""
        self.cameras = cameras
        self.ex = executor
        self.resident = int(resident_bytes)
        self.budget = int(hbm_budget) - self.resident
        self.max_batch = int(max_batch)
        self.clock = clock
        self.queue = collections.deque()
        self.inflight = []           # (token, [requests], bytes)
        self.in_use = 0
        self.completed = []
        self.rejected = []
        self._next = 0
        self.launches = 0
        self.max_in_use = 0
        self.max_inflight = 0
        self.max_queue = 0
        self.keep_outputs = keep_outputs
        for c in cameras:
            if c.footprint() > self.budget:
                raise ValueError("HBM budget smaller than the resident bytes plus one frame of "
                                 "a camera")

    # ---------------------------------------------------------------- API
    def submit(self, camera: int, frame, arrival: float | None = None) -> Request | None:
        """Queue a frame; malformed requests are rejected (returns None)."""
        t = self.clock() if arrival is None else arrival
        ok = 0 <= camera < len(self.cameras)
        if ok and hasattr(frame, "shape"):
            c = self.cameras[camera]
            ok = tuple(frame.shape) == (c.height, c.width)
        r = Request(self._next, camera, frame, t)
        self._next += 1
        if not ok:
            self.rejected.append(r)
            return None
        self.queue.append(r)
        self.max_queue = max(self.max_queue, len(self.queue))
        return r

    def cancel(self, req: Request) -> bool:
        """Drop a request that has not been admitted yet."""
        if req in self.queue:
            self.queue.remove(req)
            req.cancelled = True
            return True
        return False

    def poll(self) -> int:
        """Retire finished launches, then admit and launch waiting requests.
        Returns the number of requests launched."""
        now = self.clock()
        still = []
        for tok, reqs, nbytes in self.inflight:
            if self.ex.finished(tok):
                t = self.clock()
                for r in reqs:
                    r.done = t
                    if not self.keep_outputs:
                        r.out = None
                self.completed.extend(reqs)
                self.in_use -= nbytes
            else:
                still.append((tok, reqs, nbytes))
        self.inflight = still
        launched = 0
        while self.queue and self.ex.slots() > 0:
            batch, nbytes = [], 0
            while self.queue and len(batch) < self.max_batch:
                r = self.queue[0]
                fp = self.cameras[r.camera].footprint()
                if self.in_use + nbytes + fp > self.budget:
                    break
                self.queue.popleft()
                batch.append(r)
                nbytes += fp
            if not batch:
                break
            for r in batch:
                r.admitted = now
            tok = self.ex.launch(batch)
            self.in_use += nbytes
            self.max_in_use = max(self.max_in_use, self.in_use)
            self.inflight.append((tok, batch, nbytes))
            self.max_inflight = max(self.max_inflight, len(self.inflight))
            self.launches += 1
            launched += len(batch)
        return launched

    def drain(self, timeout: float = 60.0) -> None:
        t_end = self.clock() + timeout
        while (self.queue or self.inflight) and self.clock() < t_end:
            self.poll()
        if self.queue or self.inflight:
            raise TimeoutError("server did not drain")

    # ---------------------------------------------------------------- driver
    def run_trace(self, arrivals, frames_of) -> None:
        """Replay `arrivals` (sorted (time_offset, camera, index)) in real
        time: each request is submitted when its arrival time is reached."""
        t0 = self.clock()
        i = 0
        n = len(arrivals)
        while i < n or self.queue or self.inflight:
            now = self.clock() - t0
            while i < n and arrivals[i][0] <= now:
                off, cam, idx = arrivals[i]
                self.submit(cam, frames_of(cam, idx), arrival=t0 + off)
                i += 1
            self.poll()

    def stats(self) -> dict:
        lat = sorted(r.latency for r in self.completed)
        wait = sorted(r.admitted - r.arrival for r in self.completed)

        def pct(xs, q):
            if not xs:
                return None
            k = (len(xs) - 1) * q
            lo = int(k)
            hi = min(lo + 1, len(xs) - 1)
            return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)

        span = (max(r.done for r in self.completed) - min(r.arrival for r in self.completed)
                if self.completed else 0.0)
        ms = lambda x: None if x is None else 1e3 * x  # noqa: E731
        return {"completed": len(self.completed), "rejected": len(self.rejected),
                "launches": self.launches,
                "frames_per_launch": len(self.completed) / max(self.launches, 1),
                "throughput_fps": len(self.completed) / span if span > 0 else None,
                "latency_ms_p50": ms(pct(lat, 0.5)), "latency_ms_p99": ms(pct(lat, 0.99)),
                "admission_wait_ms_p50": ms(pct(wait, 0.5)),
                "admission_wait_ms_p99": ms(pct(wait, 0.99)),
                "max_queue": self.max_queue,
                "resident_bytes": self.resident, "budget_bytes": self.budget + self.resident,
                "peak_admitted_bytes": self.max_in_use,
                "max_launches_in_flight": self.max_inflight}


def poisson_arrivals(rates, seconds: float, seeds, frames_per_camera: int):
    """Merged arrival list of independent Poisson streams (rates in Hz):
    sorted (time, camera, frame index)."""
    import numpy as np

    out = []
    for cam, (rate, seed) in enumerate(zip(rates, seeds)):
        rng = np.random.default_rng(seed)
        t = 0.0
        n = 0
        while True:
            t += rng.exponential(1.0 / rate)
            if t >= seconds:
                break
            out.append((t, cam, n % frames_per_camera))
            n += 1
    out.sort()
    return out


# config of the serving workload: 8 cameras, frame size by camera index
SERVING_SIZES = [(1024, 440), (1280, 720), (2048, 880)]


def serving_params(camera: int, stixel_width: int = 5, batch_only: bool = True):
    """Parameters of serving camera `camera` (frame size by camera index).
    batch_only: a handle used through the batch API only, without a per-frame
    workspace."""
    import synth
    import paper_1610_04124_amd as P

    W, H = SERVING_SIZES[camera % len(SERVING_SIZES)]
    D = 256 if W == 2048 else 128
    return synth.make_params(camera=synth.camera_for_size(W, H), stixel_width=stixel_width,
                             max_disparity=D, max_width=W, max_height=H,
                             flags=P.binding.FLAG_BATCH_ONLY if batch_only else 0)


def serving_cameras(n_cameras: int = 8, stixel_width: int = 5):
    """Handles and frame sizes of the serving workload (one batch-only handle
    per camera)."""
    import paper_1610_04124_amd as P

    cams = []
    for i in range(n_cameras):
        W, H = SERVING_SIZES[i % len(SERVING_SIZES)]
        cams.append(CameraSpec(P.Stixels(serving_params(i, stixel_width)), W, H))
    return cams
