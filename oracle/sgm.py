"""ctypes binding of the CPU semi-global matching oracle (``sgm_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the HIP library or its binding.

The stereo stage upstream of the stixel path: census 9x7 costs, path
recurrences with penalties P1 / P2 summed over 4 or 8 directions, the smallest
disparity of minimum summed cost, and a left-right check that marks failures
-1 (the stixel input's invalid value).  Integer arithmetic throughout.

Parity status (how each step is pinned to something other than itself is
stated by tests/test_sgm_oracle.py):
  census     constant images, an impulse at every window offset (bit order),
             image borders, the comparison's strictness
  costs      bit counts of random 64-bit words by Python's int.bit_count
  path       exhaustive minimum over every disparity sequence along short
             paths, for each of the eight directions
  select     numpy argmin (first minimum) and the right-view diagonal
  check      hand-built disparity pairs
  disparity  textured synthetic pairs with known whole-pixel disparity
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import lib as _stixel_lib

#: Hamming distance charged when x - d leaves the image (62 census bits)
COST_OUT = 62
CENSUS_BITS = 62
#: direction order of the paths (dy, dx)
DIRECTIONS = [(0, 1), (0, -1), (1, 0), (-1, 0), (1, 1), (1, -1), (-1, 1), (-1, -1)]

_ready = False


def _lib():
    global _ready
    L = _stixel_lib()
    if not _ready:
        u8p, u16p = C.POINTER(C.c_uint8), C.POINTER(C.c_uint16)
        u64p, i16p, fp = C.POINTER(C.c_uint64), C.POINTER(C.c_int16), C.POINTER(C.c_float)
        i = C.c_int
        L.sgm_census.argtypes = [u8p, i, i, u64p]
        L.sgm_census.restype = None
        L.sgm_costs.argtypes = [u64p, u64p, i, i, i, u8p]
        L.sgm_costs.restype = None
        L.sgm_path.argtypes = [u64p, u64p, i, i, i, i, i, i, u16p]
        L.sgm_path.restype = None
        L.sgm_select.argtypes = [u16p, i, i, i, i16p, i16p]
        L.sgm_select.restype = None
        L.sgm_check.argtypes = [i16p, i16p, i, i, fp]
        L.sgm_check.restype = None
        L.sgm_disparity.argtypes = [u8p, u8p, i, i, i, i, i, i, fp, u16p]
        L.sgm_disparity.restype = C.c_int
        _ready = True
    return L


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def census(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, np.uint8)
    H, W = img.shape
    out = np.zeros((H, W), np.uint64)
    _lib().sgm_census(_p(img, C.c_uint8), W, H, _p(out, C.c_uint64))
    return out


def costs(cl: np.ndarray, cr: np.ndarray, D: int) -> np.ndarray:
    cl = np.ascontiguousarray(cl, np.uint64)
    cr = np.ascontiguousarray(cr, np.uint64)
    H, W = cl.shape
    out = np.zeros((H, W, D), np.uint8)
    _lib().sgm_costs(_p(cl, C.c_uint64), _p(cr, C.c_uint64), W, H, D, _p(out, C.c_uint8))
    return out


def path(cl: np.ndarray, cr: np.ndarray, D: int, P1: int, P2: int, direction: int) -> np.ndarray:
    cl = np.ascontiguousarray(cl, np.uint64)
    cr = np.ascontiguousarray(cr, np.uint64)
    H, W = cl.shape
    out = np.zeros((H, W, D), np.uint16)
    _lib().sgm_path(_p(cl, C.c_uint64), _p(cr, C.c_uint64), W, H, D, P1, P2, direction,
                    _p(out, C.c_uint16))
    return out


def select(S: np.ndarray):
    S = np.ascontiguousarray(S, np.uint16)
    H, W, D = S.shape
    dL = np.zeros((H, W), np.int16)
    dR = np.zeros((H, W), np.int16)
    _lib().sgm_select(_p(S, C.c_uint16), W, H, D, _p(dL, C.c_int16), _p(dR, C.c_int16))
    return dL, dR


def check(dL: np.ndarray, dR: np.ndarray) -> np.ndarray:
    dL = np.ascontiguousarray(dL, np.int16)
    dR = np.ascontiguousarray(dR, np.int16)
    H, W = dL.shape
    out = np.zeros((H, W), np.float32)
    _lib().sgm_check(_p(dL, C.c_int16), _p(dR, C.c_int16), W, H, _p(out, C.c_float))
    return out


def disparity(left: np.ndarray, right: np.ndarray, D: int, P1: int = 10, P2: int = 120,
              npaths: int = 4, return_costs: bool = False):
    """Float32 disparity of the left view, -1 where the left-right check
    fails; with return_costs also the summed costs S [H][W][D]."""
    left = np.ascontiguousarray(left, np.uint8)
    right = np.ascontiguousarray(right, np.uint8)
    H, W = left.shape
    if right.shape != (H, W):
        raise ValueError("left and right images differ in size")
    disp = np.zeros((H, W), np.float32)
    S = np.zeros((H, W, D), np.uint16) if return_costs else None
    rc = _lib().sgm_disparity(_p(left, C.c_uint8), _p(right, C.c_uint8), W, H, D, P1, P2, npaths,
                              _p(disp, C.c_float),
                              _p(S, C.c_uint16) if S is not None else None)
    if rc != 0:
        raise ValueError("sgm_disparity rejected its arguments")
    return (disp, S) if return_costs else disp
