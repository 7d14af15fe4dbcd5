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
        if c == OB and prev[2] == OB and f > prev[3] + int(self.m["ordering_tol_px"]):
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
