"""Thin ctypes binding of ``libstixels.so`` (include/stixels.h).

Argument marshalling only: every step of the segmentation runs in the HIP
kernels behind the C ABI.  Device buffers are torch tensors on a ROCm device;
streams are torch.cuda streams (HIP streams under ROCm).  When the shared
library is missing, loading fails loudly: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstixels.so")
#: the same library built with per-phase clock stamps in the persistent
#: kernel (profiling only); STIXELS_PHASE_TIMING=1 in the environment loads it
PHASES_LIB_PATH = os.path.join(_HERE, "libstixels_phases.so")

OK, E_INVALID_ARG, E_RANGE, E_HIP, E_NOMEM = 0, -1, -2, -3, -4
FLAG_BATCH_ONLY = 1
TABLE_SKY, TABLE_GROUND, TABLE_OBJECT, TABLE_FG_HI, TABLE_FG_LO = range(5)
STAGE_REDUCED, STAGE_PREFIX, STAGE_RANGE, STAGE_OBJECT_PREFIX = range(4)

#: every entry point declared in include/stixels.h
EXPORTS = (
    "stixels_create", "stixels_destroy", "stixels_num_columns", "stixels_output_capacity",
    "stixels_compute", "stixels_last_error", "stixels_status_string",
    "stixels_batch_create", "stixels_batch_destroy", "stixels_batch_compute",
    "stixels_batch_capture", "stixels_batch_replay", "stixels_batch_info",
    "stixels_batch_set_workgroups", "stixels_batch_set_waves", "stixels_batch_waves",
    "stixels_batch_set_columns", "stixels_batch_columns",
    "stixels_set_waves", "stixels_get_waves", "stixels_set_po_placement",
    "stixels_batch_last_error", "stixels_debug_table", "stixels_host_table",
    "stixels_debug_stage", "stixels_selftest_mean", "stixels_output_bytes",
    "stixels_compute_batch", "stixels_debug_tables", "stixels_set_frame_path",
    "stixels_get_frame_path", "stixels_device_bytes", "stixels_batch_device_bytes",
    "stixels_debug_stage_times", "stixels_compute_pose", "stixels_debug_pose_tables",
    "stixels_set_object_lut", "stixels_compute_noalloc",
    "stixels_sgm_create", "stixels_sgm_destroy", "stixels_sgm_last_error",
    "stixels_sgm_device_bytes", "stixels_sgm_compute", "stixels_sgm_debug",
    "stixels_compute_stereo", "stixels_batch_phase_cycles",
)


class StixelsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Camera(C.Structure):
    _fields_ = [("focal_px", C.c_double), ("baseline_m", C.c_double),
                ("cam_height_m", C.c_double), ("horizon_row", C.c_double),
                ("pitch_rad", C.c_double)]


class Model(C.Structure):
    _fields_ = [("p_out", C.c_double), ("sigma_disp", C.c_double), ("sigma_sky", C.c_double),
                ("ground_slope_noise", C.c_double), ("object_depth_extent_m", C.c_double),
                ("bic_cost", C.c_double), ("first_cost", C.c_double * 3),
                ("trans_cost", (C.c_double * 3) * 3), ("ordering_cost", C.c_double),
                ("gravity_cost", C.c_double), ("gravity_tol_px", C.c_double),
                ("diving_cost", C.c_double), ("diving_tol_px", C.c_double),
                ("ordering_tol_px", C.c_int32), ("reserved0", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("camera", Camera), ("model", Model), ("stixel_width", C.c_int32),
                ("max_disparity", C.c_int32), ("max_width", C.c_int32),
                ("max_height", C.c_int32), ("max_stixels_per_column", C.c_int32),
                ("reduce_mode", C.c_int32), ("cost_grid_log2", C.c_int32),
                ("flags", C.c_int32), ("subpixel_log2", C.c_int32), ("reserved1", C.c_int32)]


class Output(C.Structure):
    _fields_ = [("counts", C.c_void_p), ("records", C.c_void_p), ("total_cost", C.c_void_p),
                ("overflow", C.c_void_p), ("capacity", C.c_int32), ("reserved0", C.c_int32)]


class Pose(C.Structure):
    _fields_ = [("horizon_row", C.c_double), ("pitch_rad", C.c_double)]


class Job(C.Structure):
    _fields_ = [("handle", C.c_void_p), ("d_disparity", C.c_void_p), ("width", C.c_int32),
                ("height", C.c_int32), ("out", Output), ("pose", Pose),
                ("use_pose", C.c_int32), ("reserved0", C.c_int32)]


class BatchConfig(C.Structure):
    _fields_ = [("max_jobs", C.c_int32), ("max_tasks", C.c_int32), ("max_height", C.c_int32),
                ("max_disparity", C.c_int32), ("workgroups", C.c_int32), ("flags", C.c_int32)]


BATCH_POSES = 1


class SgmParams(C.Structure):
    _fields_ = [("max_width", C.c_int32), ("max_height", C.c_int32),
                ("max_disparity", C.c_int32), ("p1", C.c_int32), ("p2", C.c_int32),
                ("paths", C.c_int32), ("max_frames", C.c_int32)]


SGM_LEFT_CENSUS, SGM_RIGHT_CENSUS, SGM_COSTS = range(3)


def to_pose(pose) -> Pose:
    """(horizon_row, pitch_rad), or a dict with those keys, as a stixels_pose."""
    if isinstance(pose, dict):
        return Pose(float(pose["horizon_row"]), float(pose.get("pitch_rad", 0.0)))
    hr, pitch = pose
    return Pose(float(hr), float(pitch))


_lib = None


def lib():
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        path = PHASES_LIB_PATH if os.environ.get("STIXELS_PHASE_TIMING") == "1" else LIB_PATH
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with "
                              "`python -m paper_1610_04124_amd.build` (no CPU fallback exists)")
        # torch ships its own HIP runtime (SONAME libamdhip64.so.7) and loads
        # it under another file name; importing torch first lets this
        # library's libamdhip64.so.7 dependency bind to that same runtime, so
        # the process holds one HIP runtime and shares devices and streams.
        import torch  # noqa: F401
        L = C.CDLL(path)
        vp, i32, P = C.c_void_p, C.c_int32, C.POINTER
        L.stixels_create.argtypes = [P(Params), P(vp)]
        L.stixels_destroy.argtypes = [vp]
        L.stixels_num_columns.argtypes = [vp, i32, P(i32)]
        L.stixels_output_capacity.argtypes = [vp, i32, P(i32)]
        L.stixels_compute.argtypes = [vp, vp, i32, i32, vp, P(Output)]
        L.stixels_compute_pose.argtypes = [vp, vp, i32, i32, P(Pose), vp, P(Output)]
        L.stixels_compute_noalloc.argtypes = [vp, vp, i32, i32, vp, P(Output)]
        L.stixels_debug_pose_tables.argtypes = [vp, P(Pose), i32, vp, C.c_size_t, vp]
        L.stixels_last_error.argtypes = [vp]
        L.stixels_last_error.restype = C.c_char_p
        L.stixels_status_string.argtypes = [C.c_int]
        L.stixels_status_string.restype = C.c_char_p
        L.stixels_debug_table.argtypes = [vp, i32, vp, C.c_size_t]
        L.stixels_host_table.argtypes = [P(Params), i32, vp, C.c_size_t]
        L.stixels_debug_stage.argtypes = [vp, i32, vp, C.c_size_t, vp]
        L.stixels_selftest_mean.argtypes = [i32, i32, P(C.c_int64)]
        L.stixels_batch_create.argtypes = [P(BatchConfig), P(vp)]
        L.stixels_batch_destroy.argtypes = [vp]
        L.stixels_batch_compute.argtypes = [vp, P(Job), i32, vp]
        L.stixels_batch_capture.argtypes = [vp, P(Job), i32, vp]
        L.stixels_batch_replay.argtypes = [vp, vp]
        L.stixels_batch_info.argtypes = [vp, P(i32), P(i32)]
        L.stixels_batch_set_workgroups.argtypes = [vp, i32]
        L.stixels_batch_set_waves.argtypes = [vp, i32]
        L.stixels_batch_waves.argtypes = [vp]
        L.stixels_batch_set_columns.argtypes = [vp, i32]
        L.stixels_batch_columns.argtypes = [vp]
        L.stixels_set_waves.argtypes = [vp, i32]
        L.stixels_get_waves.argtypes = [vp, i32, i32]
        L.stixels_set_po_placement.argtypes = [vp, i32]
        L.stixels_output_bytes.argtypes = [vp, i32, i32, P(C.c_size_t)]
        L.stixels_compute_batch.argtypes = [P(Job), i32, vp]
        L.stixels_debug_tables.argtypes = [vp, vp, C.c_size_t]
        L.stixels_set_frame_path.argtypes = [vp, i32]
        L.stixels_set_object_lut.argtypes = [vp, i32]
        L.stixels_get_frame_path.argtypes = [vp]
        L.stixels_device_bytes.argtypes = [vp, P(C.c_size_t)]
        L.stixels_batch_device_bytes.argtypes = [vp, P(C.c_size_t)]
        L.stixels_debug_stage_times.argtypes = [vp, vp, i32, i32, vp, P(Output),
                                                P(C.c_float)]
        L.stixels_batch_phase_cycles.argtypes = [vp, P(C.c_uint64), i32, i32]
        L.stixels_batch_last_error.argtypes = [vp]
        L.stixels_batch_last_error.restype = C.c_char_p
        L.stixels_sgm_create.argtypes = [P(SgmParams), P(vp)]
        L.stixels_sgm_destroy.argtypes = [vp]
        L.stixels_sgm_last_error.argtypes = [vp]
        L.stixels_sgm_last_error.restype = C.c_char_p
        L.stixels_sgm_device_bytes.argtypes = [vp, P(C.c_size_t)]
        L.stixels_sgm_compute.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp]
        L.stixels_sgm_debug.argtypes = [vp, i32, vp, C.c_size_t]
        L.stixels_compute_stereo.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp, P(Output)]
        _lib = L
    return _lib


def bins(params: dict) -> int:
    """Disparity bins of a parameter set: max_disparity px in bins of
    2^-subpixel_log2 px (an out-of-range exponent is left to the library to
    reject)."""
    k = int(params.get("subpixel_log2", 0))
    return int(params["max_disparity"]) << k if 0 <= k <= 8 else int(params["max_disparity"])


def to_params(params: dict) -> Params:
    p = Params()
    for k in ("focal_px", "baseline_m", "cam_height_m", "horizon_row", "pitch_rad"):
        setattr(p.camera, k, float(params["camera"][k]))
    m = params["model"]
    for k in ("p_out", "sigma_disp", "sigma_sky", "ground_slope_noise", "object_depth_extent_m",
              "bic_cost", "ordering_cost", "gravity_cost", "gravity_tol_px", "diving_cost",
              "diving_tol_px"):
        setattr(p.model, k, float(m[k]))
    p.model.ordering_tol_px = int(m["ordering_tol_px"])
    for a in range(3):
        p.model.first_cost[a] = float(m["first_cost"][a])
        for b in range(3):
            p.model.trans_cost[a][b] = float(m["trans_cost"][a][b])
    for k in ("stixel_width", "max_disparity", "max_width", "max_height",
              "max_stixels_per_column", "reduce_mode", "cost_grid_log2"):
        setattr(p, k, int(params[k]))
    p.flags = int(params.get("flags", 0))
    p.subpixel_log2 = int(params.get("subpixel_log2", 0))
    return p


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _check_device_tensor(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor")


class FrameOutput:
    """Caller-owned device output of one frame (torch tensors)."""

    def __init__(self, ncols: int, capacity: int, device):
        import torch
        self.ncols, self.capacity = int(ncols), int(capacity)
        self.counts = torch.zeros(ncols, dtype=torch.int32, device=device)
        self.records = torch.zeros((ncols, capacity, 3), dtype=torch.int32, device=device)
        self.total = torch.zeros(ncols, dtype=torch.float32, device=device)
        self.overflow = torch.zeros(ncols, dtype=torch.uint8, device=device)

    def struct(self) -> Output:
        o = Output()
        o.counts = self.counts.data_ptr()
        o.records = self.records.data_ptr()
        o.total_cost = self.total.data_ptr()
        o.overflow = self.overflow.data_ptr()
        o.capacity = self.capacity
        return o

    def to_host(self) -> dict:
        """Decoded host copy: counts, records (structured, bottom-up), total, overflow."""
        rec = self.records.cpu().numpy()
        return dict(counts=self.counts.cpu().numpy(), records=decode_records(rec),
                    total=self.total.cpu().numpy(), overflow=self.overflow.cpu().numpy())


RECORD_DTYPE = np.dtype([("v_bottom", np.int32), ("v_top", np.int32), ("cls", np.int32),
                         ("disparity", np.int32), ("cost", np.float32)])


def decode_records(raw: np.ndarray) -> np.ndarray:
    """[..., 3] int32 words (stixels_record) -> structured array."""
    raw = np.ascontiguousarray(raw, dtype=np.int32)
    w = raw.view(np.uint32)
    out = np.zeros(raw.shape[:-1], RECORD_DTYPE)
    out["v_bottom"] = (w[..., 0] & 0xFFFF).astype(np.int16)
    out["v_top"] = (w[..., 0] >> 16).astype(np.int16)
    out["cls"] = w[..., 1] & 0xFF
    out["disparity"] = (w[..., 1] >> 8) & 0xFF
    out["cost"] = raw[..., 2].view(np.float32)
    return out


class Stixels:
    """One camera model: the resident offline tables and a per-frame workspace."""

    def __init__(self, params: dict):
        self.params = params
        self._p = to_params(params)
        h = C.c_void_p()
        rc = lib().stixels_create(C.byref(self._p), C.byref(h))
        if rc != OK:
            raise StixelsError(rc, "stixels_create: " + lib().stixels_last_error(None).decode())
        self.h = h
        self.s = int(params["stixel_width"])
        # disparity bins: max_disparity px in bins of 2^-subpixel_log2 px
        self.D = bins(params)
        self.max_height = int(params["max_height"])

    def close(self):
        if getattr(self, "h", None):
            lib().stixels_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc, what):
        raise StixelsError(rc, f"{what}: " + lib().stixels_last_error(self.h).decode())

    def num_columns(self, width: int) -> int:
        n = C.c_int32()
        rc = lib().stixels_num_columns(self.h, int(width), C.byref(n))
        if rc != OK:
            self._err(rc, "stixels_num_columns")
        return n.value

    def capacity(self, height: int) -> int:
        n = C.c_int32()
        rc = lib().stixels_output_capacity(self.h, int(height), C.byref(n))
        if rc != OK:
            self._err(rc, "stixels_output_capacity")
        return n.value

    def set_waves(self, waves: int) -> None:
        """Wavefronts per column of the recurrence (1, 2, 4; 0 = automatic)."""
        rc = lib().stixels_set_waves(self.h, int(waves))
        if rc != OK:
            self._err(rc, "stixels_set_waves")

    def set_po_placement(self, placement: int) -> None:
        """Object prefix table of the per-frame recurrence: 0 auto, 1 HBM, 2 LDS where it fits."""
        rc = lib().stixels_set_po_placement(self.h, int(placement))
        if rc != OK:
            self._err(rc, "stixels_set_po_placement")

    def waves(self, width: int, height: int) -> int:
        """Wavefronts per column that compute uses for a frame of this size."""
        return int(lib().stixels_get_waves(self.h, int(height), int(width)))

    def set_frame_path(self, path: int) -> None:
        """How compute runs a frame: 1 staged kernels, 2 one fused launch, 0 automatic."""
        rc = lib().stixels_set_frame_path(self.h, int(path))
        if rc != OK:
            self._err(rc, "stixels_set_frame_path")

    def set_object_lut(self, mode: int) -> None:
        """Object costs of the staged table build: 0 offline LUT, 1 online Eq. 4."""
        rc = lib().stixels_set_object_lut(self.h, int(mode))
        if rc != OK:
            self._err(rc, "stixels_set_object_lut")

    def frame_path(self) -> int:
        """The path (1 staged, 2 fused) compute takes under the current setting."""
        return int(lib().stixels_get_frame_path(self.h))

    def device_bytes(self) -> int:
        """Device bytes the handle holds (tables, workspace, internal batch)."""
        n = C.c_size_t()
        rc = lib().stixels_device_bytes(self.h, C.byref(n))
        if rc != OK:
            self._err(rc, "stixels_device_bytes")
        return n.value

    def output_bytes(self, width: int, height: int) -> int:
        """Device bytes of a frame's four output arrays."""
        n = C.c_size_t()
        rc = lib().stixels_output_bytes(self.h, int(width), int(height), C.byref(n))
        if rc != OK:
            self._err(rc, "stixels_output_bytes")
        return n.value

    def new_output(self, width: int, height: int, device=None) -> FrameOutput:
        import torch
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        return FrameOutput(self.num_columns(width), self.capacity(height), dev)

    def compute(self, disp, out: FrameOutput | None = None, stream=None,
                pose=None) -> FrameOutput:
        """Enqueue the segmentation of one device frame [height, width] float32,
        with the handle's camera or, given `pose` = (horizon_row, pitch_rad),
        with that frame's own pose (stixels_compute_pose)."""
        import torch
        _check_device_tensor(disp, torch.float32, "disparity")
        H, W = disp.shape
        if out is None:
            out = self.new_output(W, H, disp.device)
        self.check_output(out, W, disp.device)
        o = out.struct()
        if pose is None:
            rc = lib().stixels_compute(self.h, C.c_void_p(disp.data_ptr()), int(W), int(H),
                                       _stream_ptr(stream), C.byref(o))
        else:
            ps = to_pose(pose)
            rc = lib().stixels_compute_pose(self.h, C.c_void_p(disp.data_ptr()), int(W), int(H),
                                            C.byref(ps), _stream_ptr(stream), C.byref(o))
        if rc != OK:
            self._err(rc, "stixels_compute" if pose is None else "stixels_compute_pose")
        return out

    def compute_noalloc(self, disp, out: FrameOutput, stream=None) -> FrameOutput:
        """Enqueue one device frame through stixels_compute_noalloc (the fused
        kernel with the library's fixed per-GPU workspace; the caller brings
        the output, and calls that overlap on one GPU race)."""
        import torch
        _check_device_tensor(disp, torch.float32, "disparity")
        H, W = disp.shape
        self.check_output(out, W, disp.device)
        o = out.struct()
        rc = lib().stixels_compute_noalloc(self.h, C.c_void_p(disp.data_ptr()), int(W), int(H),
                                           _stream_ptr(stream), C.byref(o))
        if rc != OK:
            self._err(rc, "stixels_compute_noalloc")
        return out

    def compute_stereo(self, sgm: "Sgm", left, right, out: FrameOutput | None = None,
                       disparity=None, stream=None):
        """A device stereo pair (uint8 [height, width] each) through the
        matching stage and this handle's stixel path on one stream
        (stixels_compute_stereo).  Returns (stixels, disparity map)."""
        import torch
        _check_device_tensor(left, torch.uint8, "left image")
        _check_device_tensor(right, torch.uint8, "right image")
        if left.shape != right.shape or left.dim() != 2:
            raise StixelsError(E_INVALID_ARG, "left and right must be equal 2-D images")
        H, W = left.shape
        if out is None:
            out = self.new_output(W, H, left.device)
        self.check_output(out, W, left.device)
        if disparity is None:
            disparity = torch.empty((H, W), dtype=torch.float32, device=left.device)
        _check_device_tensor(disparity, torch.float32, "disparity")
        if tuple(disparity.shape) != (H, W):
            raise StixelsError(E_INVALID_ARG, "disparity map must match the images")
        o = out.struct()
        rc = lib().stixels_compute_stereo(self.h, sgm.h, C.c_void_p(left.data_ptr()),
                                          C.c_void_p(right.data_ptr()), int(W), int(H),
                                          _stream_ptr(stream), C.c_void_p(disparity.data_ptr()),
                                          C.byref(o))
        if rc != OK:
            self._err(rc, "stixels_compute_stereo")
        return out, disparity

    def debug_pose_tables(self, pose, height: int, stream=None):
        """The ground table [height][D] and diving / gravity thresholds
        [height] that the device builds for a frame pose (synchronises)."""
        H = int(height)
        buf = np.zeros(H * (4 * self.D + 8), np.uint8)
        ps = to_pose(pose)
        rc = lib().stixels_debug_pose_tables(self.h, C.byref(ps), H, buf.ctypes.data, buf.nbytes,
                                             _stream_ptr(stream))
        if rc != OK:
            self._err(rc, "stixels_debug_pose_tables")
        g = buf[:H * 4 * self.D].view(np.float32).reshape(H, self.D).copy()
        hi = buf[H * 4 * self.D:H * (4 * self.D + 4)].view(np.int32).copy()
        lo = buf[H * (4 * self.D + 4):].view(np.int32).copy()
        return g, hi, lo

    def check_output(self, out: FrameOutput, width: int, device) -> None:
        """The kernels write ncols columns of `capacity` records into the
        output's tensors; a mismatched output would be overrun on the device."""
        if out.ncols != self.num_columns(width):
            raise StixelsError(E_INVALID_ARG, f"output holds {out.ncols} columns, the frame "
                               f"has {self.num_columns(width)}")
        if out.counts.device != device:
            raise StixelsError(E_INVALID_ARG, "output and input are on different devices")
        if (out.records.shape != (out.ncols, out.capacity, 3) or out.counts.numel() != out.ncols
                or out.total.numel() != out.ncols or out.overflow.numel() != out.ncols):
            raise StixelsError(E_INVALID_ARG,
                               "output tensors do not match its column count and capacity")

    def compute_raw(self, disp_ptr: int, W: int, H: int, out: Output, stream_ptr) -> None:
        rc = lib().stixels_compute(self.h, C.c_void_p(disp_ptr), int(W), int(H), stream_ptr,
                                   C.byref(out))
        if rc != OK:
            self._err(rc, "stixels_compute")

    # ------------------------------------------------------------- debug
    def debug_table(self, which: int) -> np.ndarray:
        shape, dt = _table_shape(which, self.D, self.max_height)
        a = np.zeros(shape, dt)
        rc = lib().stixels_debug_table(self.h, int(which), a.ctypes.data, a.nbytes)
        if rc != OK:
            self._err(rc, "stixels_debug_table")
        return a

    def stage_times(self, disp, out: FrameOutput, stream=None):
        """Milliseconds of the staged path's reduction, tables and recurrence
        kernels for one frame (HIP events between them; synchronises)."""
        import torch
        _check_device_tensor(disp, torch.float32, "disparity")
        H, W = disp.shape
        self.check_output(out, W, disp.device)
        o = out.struct()
        ms = (C.c_float * 3)()
        rc = lib().stixels_debug_stage_times(self.h, C.c_void_p(disp.data_ptr()), int(W), int(H),
                                             _stream_ptr(stream), C.byref(o), ms)
        if rc != OK:
            self._err(rc, "stixels_debug_stage_times")
        return [float(x) for x in ms]

    def debug_tables(self) -> dict:
        """All offline tables in one call (stixels_debug_tables)."""
        shapes = [_table_shape(w, self.D, self.max_height) for w in range(5)]
        sizes = [int(np.prod(sh)) * np.dtype(dt).itemsize for sh, dt in shapes]
        buf = np.zeros(sum(sizes), np.uint8)
        rc = lib().stixels_debug_tables(self.h, buf.ctypes.data, buf.nbytes)
        if rc != OK:
            self._err(rc, "stixels_debug_tables")
        out, off = {}, 0
        for w, (sh, dt), n in zip(range(5), shapes, sizes):
            out[w] = buf[off:off + n].view(dt).reshape(sh).copy()
            off += n
        return out

    def debug_stage(self, which: int, W: int, H: int, stream=None) -> np.ndarray:
        ncols = W // self.s
        shape, dt = {STAGE_REDUCED: ((ncols, H), np.int16),
                     STAGE_PREFIX: ((4, ncols, H + 1), np.float32),
                     STAGE_RANGE: ((ncols, 2), np.int32),
                     STAGE_OBJECT_PREFIX: ((ncols, self.D, H + 1), np.float32)}[which]
        a = np.zeros(shape, dt)
        rc = lib().stixels_debug_stage(self.h, int(which), a.ctypes.data, a.nbytes,
                                       _stream_ptr(stream))
        if rc != OK:
            self._err(rc, "stixels_debug_stage")
        return a


def _table_shape(which, D, Hm):
    return {TABLE_SKY: ((D,), np.float32), TABLE_GROUND: ((Hm, D), np.float32),
            TABLE_OBJECT: ((D, D), np.float32), TABLE_FG_HI: ((Hm,), np.int32),
            TABLE_FG_LO: ((Hm,), np.int32)}[which]


def host_table(params: dict, which: int) -> np.ndarray:
    """An offline table built on the host by the library, without a device."""
    shape, dt = _table_shape(which, bins(params), int(params["max_height"]))
    a = np.zeros(shape, dt)
    p = to_params(params)
    rc = lib().stixels_host_table(C.byref(p), int(which), a.ctypes.data, a.nbytes)
    if rc != OK:
        raise StixelsError(rc, "stixels_host_table: " + lib().stixels_last_error(None).decode())
    return a


def selftest_mean(d_range: int, max_height: int) -> int:
    n = C.c_int64(-1)
    rc = lib().stixels_selftest_mean(int(d_range), int(max_height), C.byref(n))
    if rc != OK:
        raise StixelsError(rc, "stixels_selftest_mean")
    return n.value


def status_string(code: int) -> str:
    return lib().stixels_status_string(int(code)).decode()


def finite(x):
    return x if math.isfinite(x) else math.inf


def compute_batch(items, stream=None):
    """One-call batch (stixels_compute_batch): items as for Batch.compute; the
    batch object lives in the first item's handle."""
    arr, keep = Batch.make_jobs(items)
    rc = lib().stixels_compute_batch(arr, len(arr), _stream_ptr(stream))
    if rc != OK:
        raise StixelsError(rc, "stixels_compute_batch: " +
                           lib().stixels_last_error(items[0][0].h).decode())
    return keep


class Batch:
    """Persistent batched launch over many frames (possibly different cameras,
    sizes and stixel widths); see stixels_batch_* in include/stixels.h."""

    def __init__(self, max_jobs: int, max_tasks: int, max_height: int, max_disparity: int,
                 workgroups: int = 0, poses: bool = False):
        cfg = BatchConfig()
        cfg.max_jobs, cfg.max_tasks = int(max_jobs), int(max_tasks)
        cfg.max_height, cfg.max_disparity = int(max_height), int(max_disparity)
        cfg.workgroups = int(workgroups)
        cfg.flags = BATCH_POSES if poses else 0
        b = C.c_void_p()
        rc = lib().stixels_batch_create(C.byref(cfg), C.byref(b))
        if rc != OK:
            raise StixelsError(rc, "stixels_batch_create")
        self.b = b
        self.cfg = cfg
        self._keep = None

    def close(self):
        if getattr(self, "b", None):
            lib().stixels_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc, what):
        raise StixelsError(rc, f"{what}: " + lib().stixels_batch_last_error(self.b).decode())

    @staticmethod
    def make_jobs(items):
        """items: sequence of (Stixels, device frame tensor [H, W], FrameOutput)
        or (Stixels, frame, FrameOutput, pose) with pose = (horizon_row,
        pitch_rad) for a frame with its own camera pose (None = the handle's)."""
        import torch
        arr = (Job * len(items))()
        keep = []
        for i, item in enumerate(items):
            h, disp, out = item[:3]
            pose = item[3] if len(item) > 3 else None
            _check_device_tensor(disp, torch.float32, "disparity")
            H, W = disp.shape
            h.check_output(out, W, disp.device)
            arr[i].handle = h.h
            arr[i].d_disparity = disp.data_ptr()
            arr[i].width, arr[i].height = int(W), int(H)
            arr[i].out = out.struct()
            if pose is not None:
                arr[i].pose = to_pose(pose)
                arr[i].use_pose = 1
            keep.append((h, disp, out))
        return arr, keep

    def compute(self, items, stream=None):
        arr, keep = self.make_jobs(items)
        self._keep = keep
        rc = lib().stixels_batch_compute(self.b, arr, len(arr), _stream_ptr(stream))
        if rc != OK:
            self._err(rc, "stixels_batch_compute")

    def capture(self, items, stream=None):
        arr, keep = self.make_jobs(items)
        self._keep = keep
        rc = lib().stixels_batch_capture(self.b, arr, len(arr), _stream_ptr(stream))
        if rc != OK:
            self._err(rc, "stixels_batch_capture")

    def replay(self, stream=None):
        rc = lib().stixels_batch_replay(self.b, _stream_ptr(stream))
        if rc != OK:
            self._err(rc, "stixels_batch_replay")

    def set_waves(self, waves: int):
        """Wavefronts per column of later launches (1, 2, 4; 0 = 1)."""
        rc = lib().stixels_batch_set_waves(self.b, int(waves))
        if rc != OK:
            self._err(rc, "stixels_batch_set_waves")

    def waves(self) -> int:
        """Wavefronts per column of the last launch."""
        return int(lib().stixels_batch_waves(self.b))

    def set_columns(self, columns: int):
        """Columns per wave64 of later launches (1, 2; 0 = 1)."""
        rc = lib().stixels_batch_set_columns(self.b, int(columns))
        if rc != OK:
            self._err(rc, "stixels_batch_set_columns")

    def columns(self) -> int:
        """Columns per wave of the last launch."""
        return int(lib().stixels_batch_columns(self.b))

    def set_workgroups(self, n: int):
        rc = lib().stixels_batch_set_workgroups(self.b, int(n))
        if rc != OK:
            self._err(rc, "stixels_batch_set_workgroups")

    def device_bytes(self) -> int:
        """Device bytes the batch object holds."""
        n = C.c_size_t()
        rc = lib().stixels_batch_device_bytes(self.b, C.byref(n))
        if rc != OK:
            self._err(rc, "stixels_batch_device_bytes")
        return n.value

    def info(self):
        g, t = C.c_int32(), C.c_int32()
        rc = lib().stixels_batch_info(self.b, C.byref(g), C.byref(t))
        if rc != OK:
            self._err(rc, "stixels_batch_info")
        return g.value, t.value

    #: names of the values phase_cycles returns
    PHASES = ("reduce", "prefix_scans", "object_table", "recurrence", "backtracking",
              "tasks", "workgroup_lifetime")

    def phase_cycles(self, reset: bool = False) -> dict:
        """Shader-clock cycles per task phase summed over this batch's
        launches (the library built with phase timing only)."""
        buf = (C.c_uint64 * 7)()
        rc = lib().stixels_batch_phase_cycles(self.b, buf, 7, 1 if reset else 0)
        if rc != OK:
            self._err(rc, "stixels_batch_phase_cycles")
        return dict(zip(self.PHASES, (int(x) for x in buf)))


class Sgm:
    """Semi-global matching stage ahead of the stixel path (stixels_sgm_* in
    include/stixels.h): census 9x7 costs, four path directions, left-right
    check.  Argument marshalling only."""

    def __init__(self, max_width: int, max_height: int, max_disparity: int, p1: int = 10,
                 p2: int = 120, paths: int = 4, max_frames: int = 1):
        sp = SgmParams(int(max_width), int(max_height), int(max_disparity), int(p1), int(p2),
                       int(paths), int(max_frames))
        h = C.c_void_p()
        rc = lib().stixels_sgm_create(C.byref(sp), C.byref(h))
        if rc != OK:
            raise StixelsError(rc, "stixels_sgm_create: " + lib().stixels_sgm_last_error(None).decode())
        self.h = h
        self.D = int(max_disparity)
        self.max_frames = int(max_frames)

    def close(self):
        if getattr(self, "h", None):
            lib().stixels_sgm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self) -> int:
        b = C.c_size_t()
        rc = lib().stixels_sgm_device_bytes(self.h, C.byref(b))
        if rc != OK:
            raise StixelsError(rc, "stixels_sgm_device_bytes")
        return int(b.value)

    def compute(self, left, right, disparity=None, stream=None):
        """Enqueue the disparity of device stereo pairs: uint8 [H, W] or
        [n, H, W] each; returns the float32 map(s) of the same shape (-1
        where the left-right check fails)."""
        import torch
        _check_device_tensor(left, torch.uint8, "left image")
        _check_device_tensor(right, torch.uint8, "right image")
        if left.shape != right.shape or left.dim() not in (2, 3):
            raise StixelsError(E_INVALID_ARG, "left and right must be equal [H, W] or [n, H, W]")
        n = 1 if left.dim() == 2 else int(left.shape[0])
        H, W = int(left.shape[-2]), int(left.shape[-1])
        if disparity is None:
            disparity = torch.empty(tuple(left.shape), dtype=torch.float32, device=left.device)
        _check_device_tensor(disparity, torch.float32, "disparity")
        if tuple(disparity.shape) != tuple(left.shape) or disparity.device != left.device:
            raise StixelsError(E_INVALID_ARG, "disparity must match the images")
        rc = lib().stixels_sgm_compute(self.h, C.c_void_p(left.data_ptr()),
                                       C.c_void_p(right.data_ptr()), W, H, n,
                                       _stream_ptr(stream), C.c_void_p(disparity.data_ptr()))
        if rc != OK:
            raise StixelsError(rc, "stixels_sgm_compute: " + lib().stixels_sgm_last_error(self.h).decode())
        return disparity

    def debug(self, which: int, width: int, height: int) -> np.ndarray:
        """Census words (which 0 left, 1 right) or summed costs (2) of frame 0
        of the last compute, as host arrays (synchronises)."""
        if which == SGM_COSTS:
            a = np.zeros((height, width, self.D), np.uint16)
        else:
            a = np.zeros((height, width), np.uint64)
        rc = lib().stixels_sgm_debug(self.h, int(which), a.ctypes.data, a.nbytes)
        if rc != OK:
            raise StixelsError(rc, "stixels_sgm_debug")
        return a
