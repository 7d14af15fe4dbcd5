"""Brute-force MAP over every segmentation and labelling of a short column.

Independent of the oracle's dynamic programme: it enumerates stixel lists
(Sec. 3.1, Eq. 1-2) depth first and scores each complete list directly as
sum over stixels of (sum over its pixels of the per-pixel cost) + prior, with
the pairwise prior evaluated against the *actual* previous stixel of the list.
The per-pixel costs come from the offline tables (pinned on their own), and
the object mean is computed with exact rational arithmetic.
"""

from __future__ import annotations

import math
from fractions import Fraction

OB, GR, SK = 0, 1, 2


def quantize(x: float, g: int) -> float:
    if g < 0 or not math.isfinite(x):
        return x
    return math.ldexp(round(math.ldexp(x, g)), -g)  # round() is half-to-even


def rounded_mean(vals):
    """Mean of the valid disparities rounded half up; 0 for an empty list."""
    if not vals:
        return 0
    m = Fraction(sum(vals), len(vals))
    return math.floor(m + Fraction(1, 2))


class Problem:
    def __init__(self, params: dict, tables: dict, q):
        self.p = params
        self.m = params["model"]
        self.g = int(params["cost_grid_log2"])
        self.q = [int(x) for x in q]
        self.H = len(self.q)
        self.t = tables
        H = self.H
        v_hor = (H - 1) - params["camera"]["horizon_row"]
        self.vtop = math.floor(v_hor)
        qz = lambda x: quantize(float(x), self.g)  # noqa: E731
        self.F = [qz(x) for x in self.m["first_cost"]]
        self.T = [[qz(x) for x in row] for row in self.m["trans_cost"]]
        self.beta = qz(self.m["bic_cost"])
        self.c_ord = qz(self.m["ordering_cost"])
        self.c_grav = qz(self.m["gravity_cost"])
        self.c_dive = qz(self.m["diving_cost"])
        # ordering tolerance in disparity bins (2^-subpixel_log2 px)
        self.tau = int(self.m["ordering_tol_px"]) << int(params.get("subpixel_log2", 0))

    def mean(self, b, t):
        return rounded_mean([d for d in self.q[b:t + 1] if d >= 0])

    def data(self, c, b, t):
        """Direct sum of per-pixel costs of rows b..t (no prefix sums)."""
        f = self.mean(b, t) if c == OB else 0
        if c == GR and t > self.vtop:
            return math.inf, f
        terms = []
        for v in range(b, t + 1):
            d = self.q[v]
            if d < 0:
                continue
            if c == GR:
                terms.append(self.t["G"][v][d])
            elif c == SK:
                terms.append(self.t["S"][d])
            else:
                terms.append(self.t["O"][d][f])
        return math.fsum(terms), f

    def prior(self, prev, cur):
        """prev/cur are (b, t, c, f) tuples; prev None for the bottom stixel."""
        b, _, c, f = cur
        if prev is None:
            return self.F[c] + self.beta
        tr = self.T[prev[2]][c]
        if math.isinf(tr):
            return math.inf
        pen = 0.0
        if c == OB and prev[2] == OB and f > prev[3] + self.tau:
            pen = self.c_ord
        if c == OB and prev[2] == GR:
            if f > self.t["fg_hi"][b]:
                pen = self.c_dive
            elif f < self.t["fg_lo"][b]:
                pen = self.c_grav
        return tr + self.beta + pen


def stixel_cost(pb: Problem, prev, b, t, c):
    if c == GR and t > pb.vtop:
        return math.inf, None
    cache = pb.__dict__.setdefault("_data_cache", {})
    key = (c, b, t)
    if key not in cache:
        cache[key] = pb.data(c, b, t)
    d, f = cache[key]
    cur = (b, t, c, f)
    return d + pb.prior(prev, cur), cur


def enumerate_all(pb: Problem):
    """Yield (total_cost, [stixels bottom-up]) for every finite segmentation."""
    H = pb.H
    out = []

    def rec(b, prev, acc, path):
        for t in range(b, H):
            for c in (OB, GR, SK):
                cost, cur = stixel_cost(pb, prev, b, t, c)
                if math.isinf(cost):
                    continue
                path.append((cur, cost))
                if t == H - 1:
                    out.append((acc + cost, list(path)))
                else:
                    rec(t + 1, cur, acc + cost, path)
                path.pop()

    rec(0, None, 0.0, [])
    return out


def exact_total(items):
    return math.fsum(c for _, c in items)


def map_solutions(pb: Problem):
    """All segmentations attaining the minimum total (exact on the cost grid)."""
    sols = enumerate_all(pb)
    best = min(s[0] for s in sols)
    return best, [s for s in sols if s[0] == best]


def lexicographic_key(path):
    """Tie-break key of the recurrence read from the top: (c_N, b_N, c_{N-1},
    b_{N-1}, ...)."""
    key = []
    for (b, t, c, f), _ in reversed(path):
        key.extend([c, b])
    return tuple(key)


# --------------------------------------------------------------- C enumerator
# bruteforce_enum.c: the same exhaustive search in C (direct sums, integer
# half-up means), fast enough for 9-12-row columns (up to 3 * 4^11 lists).

_ENUM = None


def enumerator(build_dir: str):
    """Compile bruteforce_enum.c with gcc into build_dir (once per process)
    and return its ctypes handle."""
    global _ENUM
    if _ENUM is None:
        import ctypes as C
        import os
        import subprocess

        src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bruteforce_enum.c")
        so = os.path.join(build_dir, "libbruteforce_enum.so")
        subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", src, "-o", so,
                        "-lm"], check=True)
        L = C.CDLL(so)
        dp, ip, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.bf_map.argtypes = [C.c_int, ip, C.c_int, dp, dp, dp, ip, ip, C.c_int, dp, dp,
                             C.c_double, C.c_double, C.c_int, C.c_double, C.c_double, dp, ip,
                             ip, i64p, i64p]
        _ENUM = L
    return _ENUM


def c_map(build_dir: str, pb: Problem):
    """Exhaustive MAP of pb's column in C.  Returns (best total, best list
    bottom-up as (b, t, c, f) tuples, number of finite lists, number of
    optimal lists); the list is the first optimum in the tie order."""
    import ctypes as C

    import numpy as np

    L = enumerator(build_dir)
    H = pb.H
    D = len(pb.t["S"])
    q = np.ascontiguousarray(pb.q, dtype=np.int32)
    G = np.ascontiguousarray(pb.t["G"], dtype=np.float64)
    S = np.ascontiguousarray(pb.t["S"], dtype=np.float64)
    O = np.ascontiguousarray(pb.t["O"], dtype=np.float64)
    hi = np.ascontiguousarray(pb.t["fg_hi"], dtype=np.int32)
    lo = np.ascontiguousarray(pb.t["fg_lo"], dtype=np.int32)
    F = np.array(pb.F, np.float64)
    T = np.array(pb.T, np.float64).reshape(9)
    best = C.c_double()
    path = np.zeros(4 * H, np.int32)
    npath = C.c_int32()
    nl, no = C.c_int64(), C.c_int64()
    P = lambda a, t: a.ctypes.data_as(C.POINTER(t))  # noqa: E731
    rc = L.bf_map(H, P(q, C.c_int32), D, P(G, C.c_double), P(S, C.c_double), P(O, C.c_double),
                  P(hi, C.c_int32), P(lo, C.c_int32), int(pb.vtop), P(F, C.c_double),
                  P(T, C.c_double), pb.beta, pb.c_ord, int(pb.tau), pb.c_grav,
                  pb.c_dive, C.byref(best), P(path, C.c_int32), C.byref(npath), C.byref(nl),
                  C.byref(no))
    if rc != 0:
        raise ValueError("bf_map rejected its arguments")
    lst = [tuple(int(x) for x in path[4 * i:4 * i + 4]) for i in range(npath.value)]
    return best.value, lst, nl.value, no.value
