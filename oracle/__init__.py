"""ctypes binding of the CPU FP64 stixel oracle (``stixel_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the HIP library or its binding.

Parity status of the oracle's functions (how each one is pinned to something
other than itself is stated by the tests that do it):
  pixel_cost     closed forms of Eq. 4, the Eq. 3 mixture bound, the sigma and
                 quadratic terms isolated by differences
  quantize       grid membership and the half-step error bound
  tables         every table entry against Eq. 4 written with scipy's normal
                 distribution (with the ground and object sigmas spelled out),
                 monotonicity, the argmin of each row, the integer thresholds
  reduce         numpy sort (lower median) and fsum (mean) on random strips
  column/frame   prefix sums against direct sums; exhaustive search over every
                 segmentation of 1..12-row columns (ordering prior off: exact
                 cost and the first optimum in the tie order; on: the
                 recurrence's own list cost, never below the MAP); a naive
                 re-implementation of Eq. 5-6 with every prior term on, bit for
                 bit on 240 random columns of up to 64 rows; hand-solved special
                 cases and penalty boundaries; invariants and scene recovery.
A mutation check (tests/test_oracle_mutants.py) plants 27 plausible mistakes
in copies of the C source and requires each to fail one of these pins.
Parity unpinned: agreement with the paper's authors' outputs and with the
prior constants of Pfeiffer's thesis (neither is available).
"""

from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstixel_oracle.so")

OBJECT, GROUND, SKY = 0, 1, 2


class SoParams(C.Structure):
    _fields_ = [
        ("focal_px", C.c_double), ("baseline_m", C.c_double), ("cam_height_m", C.c_double),
        ("horizon_row", C.c_double), ("pitch_rad", C.c_double),
        ("p_out", C.c_double), ("sigma_disp", C.c_double), ("sigma_sky", C.c_double),
        ("ground_slope_noise", C.c_double), ("object_depth_extent_m", C.c_double),
        ("bic_cost", C.c_double),
        ("first_cost", C.c_double * 3),
        ("trans_cost", (C.c_double * 3) * 3),
        ("ordering_cost", C.c_double),
        ("gravity_cost", C.c_double), ("gravity_tol_px", C.c_double),
        ("diving_cost", C.c_double), ("diving_tol_px", C.c_double),
        ("ordering_tol_px", C.c_int32),
        ("stixel_width", C.c_int32), ("max_disparity", C.c_int32),
        ("max_stixels_per_column", C.c_int32), ("reduce_mode", C.c_int32),
        ("cost_grid_log2", C.c_int32), ("subpixel_log2", C.c_int32),
    ]


STIXEL_DTYPE = np.dtype([("v_bottom", np.int32), ("v_top", np.int32), ("cls", np.int32),
                         ("disparity", np.int32), ("cost", np.float64)])


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/libstixel_oracle.so``."""
    from .build import build_oracle
    return build_oracle(force=force)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp, ip, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.so_pixel_cost.restype = C.c_double
        L.so_pixel_cost.argtypes = [C.c_double] * 5
        L.so_quantize.restype = C.c_double
        L.so_quantize.argtypes = [C.c_double, C.c_int32]
        L.so_tables.argtypes = [C.POINTER(SoParams), C.c_int32, dp, dp, dp, ip, ip]
        L.so_reduce.argtypes = [C.POINTER(SoParams), C.c_void_p, C.c_int32, C.c_int32, ip]
        L.so_column.argtypes = [C.POINTER(SoParams), C.c_int32, ip, dp, dp, i64p, i64p, dp,
                                dp, ip, ip, ip, C.c_void_p, ip, dp]
        L.so_frame.argtypes = [C.POINTER(SoParams), C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                               ip, C.c_void_p, dp, C.POINTER(C.c_uint8), C.c_int32]
        _lib = L
    return _lib


def to_struct(params: dict) -> SoParams:
    cam, m = params["camera"], params["model"]
    p = SoParams()
    for k in ("focal_px", "baseline_m", "cam_height_m", "horizon_row", "pitch_rad"):
        setattr(p, k, float(cam[k]))
    for k in ("p_out", "sigma_disp", "sigma_sky", "ground_slope_noise", "object_depth_extent_m",
              "bic_cost", "ordering_cost", "gravity_cost", "gravity_tol_px", "diving_cost",
              "diving_tol_px"):
        setattr(p, k, float(m[k]))
    p.ordering_tol_px = int(m["ordering_tol_px"])
    for c in range(3):
        p.first_cost[c] = float(m["first_cost"][c])
        for cc in range(3):
            p.trans_cost[c][cc] = float(m["trans_cost"][c][cc])
    for k in ("stixel_width", "max_disparity", "max_stixels_per_column", "reduce_mode",
              "cost_grid_log2"):
        setattr(p, k, int(params[k]))
    p.subpixel_log2 = int(params.get("subpixel_log2", 0))
    return p


def bins(params: dict) -> int:
    """Disparity bins: max_disparity px in bins of 2^-subpixel_log2 px."""
    return int(params["max_disparity"]) << int(params.get("subpixel_log2", 0))


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")


def pixel_cost(d, mu, sigma, p_out, d_range) -> float:
    """Eq. 4 for one pixel, unquantized."""
    return lib().so_pixel_cost(float(d), float(mu), float(sigma), float(p_out), float(d_range))


def quantize(x: float, g: int) -> float:
    return lib().so_quantize(float(x), int(g))


def tables(params: dict, H: int) -> dict:
    """Offline LUTs for a frame of height H: S[d], G[v, d] (bottom-up v),
    O[d, f], fg_hi[b], fg_lo[b]; d and f are disparity bins."""
    D = bins(params)
    S = np.zeros(D, np.float64)
    G = np.zeros((H, D), np.float64)
    O = np.zeros((D, D), np.float64)
    hi = np.zeros(H + 1, np.int32)
    lo = np.zeros(H + 1, np.int32)
    p = to_struct(params)
    _check(lib().so_tables(C.byref(p), H, _ptr(S, C.c_double), _ptr(G, C.c_double),
                           _ptr(O, C.c_double), _ptr(hi, C.c_int32), _ptr(lo, C.c_int32)),
           "tables")
    return dict(S=S, G=G, O=O, fg_hi=hi, fg_lo=lo)


def reduce(params: dict, disp: np.ndarray) -> np.ndarray:
    """Reduced, transposed, bottom-up integer disparities q[col, v] (-1 invalid)."""
    disp = np.ascontiguousarray(disp, dtype=np.float32)
    H, W = disp.shape
    ncols = W // int(params["stixel_width"])
    q = np.zeros((ncols, H), np.int32)
    p = to_struct(params)
    _check(lib().so_reduce(C.byref(p), disp.ctypes.data, W, H, _ptr(q, C.c_int32)), "reduce")
    return q


def column(params: dict, q_col) -> dict:
    """Solve one reduced column; returns every intermediate of the method."""
    q = np.ascontiguousarray(q_col, dtype=np.int32)
    H = int(q.shape[0])
    D = bins(params)
    out = dict(
        PG=np.zeros(H + 1), PS=np.zeros(H + 1),
        PD=np.zeros(H + 1, np.int64), PN=np.zeros(H + 1, np.int64),
        PO=np.zeros((D, H + 1)),
        C=np.zeros((H, 3)), link_b=np.zeros((H, 3), np.int32), link_c=np.zeros((H, 3), np.int32),
        fob=np.zeros(H, np.int32),
    )
    st = np.zeros(H, STIXEL_DTYPE)
    n = C.c_int32(0)
    tot = C.c_double(0.0)
    p = to_struct(params)
    _check(lib().so_column(C.byref(p), H, _ptr(q, C.c_int32),
                           _ptr(out["PG"], C.c_double), _ptr(out["PS"], C.c_double),
                           _ptr(out["PD"], C.c_int64), _ptr(out["PN"], C.c_int64),
                           _ptr(out["PO"], C.c_double), _ptr(out["C"], C.c_double),
                           _ptr(out["link_b"], C.c_int32), _ptr(out["link_c"], C.c_int32),
                           _ptr(out["fob"], C.c_int32), st.ctypes.data, C.byref(n),
                           C.byref(tot)), "column")
    out["stixels"] = st[: n.value].copy()
    out["total"] = tot.value
    return out


def frame(params: dict, disp: np.ndarray, cap: int = 0, nthreads: int = 0) -> dict:
    """Whole frame: per column counts, stixel records (bottom-up), total cost
    and overflow flag.  ``cap`` 0 means the frame height."""
    disp = np.ascontiguousarray(disp, dtype=np.float32)
    H, W = disp.shape
    s = int(params["stixel_width"])
    if W < s or H < 1:
        raise ValueError("frame narrower than one stixel or empty")
    ncols = W // s
    cap = int(cap) if cap > 0 else H
    counts = np.zeros(ncols, np.int32)
    recs = np.zeros((ncols, cap), STIXEL_DTYPE)
    total = np.zeros(ncols, np.float64)
    ovf = np.zeros(ncols, np.uint8)
    p = to_struct(params)
    _check(lib().so_frame(C.byref(p), disp.ctypes.data, W, H, cap, _ptr(counts, C.c_int32),
                          recs.ctypes.data, _ptr(total, C.c_double), _ptr(ovf, C.c_uint8),
                          int(nthreads)), "frame")
    return dict(counts=counts, records=recs, total=total, overflow=ovf)


def column_stixels(result: dict, i: int):
    """Stixel records of column i of a ``frame`` result."""
    return result["records"][i, : result["counts"][i]]


def finite_or_inf(x):
    return x if math.isfinite(x) else math.inf
