"""A deliberately naive re-implementation of the recurrence of Eq. 5-6.

Written from the paper's Sec. 3.3, independently of the oracle's C code, to
pin the oracle with every prior term switched on (the ordering penalty makes
the recurrence depend on the stored best object stixel ob^{b-1}, so it is no
longer the MAP of Eq. 1 and brute force alone cannot pin it).

Nothing is clever here: the data term of a stixel is the direct sum of its
pixels' costs (no prefix sums), an object's mean is the half-up rounding of
an exact Fraction, and the candidates of every (row, class) are listed one by
one in the order Eq. 6 writes them -- the bottom stixel first, then the cut
positions b ascending, and for each b the predecessor classes object, ground,
sky -- with the first minimum kept.
"""

from __future__ import annotations

import math
from fractions import Fraction

OB, GR, SK = 0, 1, 2
INF = math.inf


def q_grid(x: float, g: int) -> float:
    """Round a prior constant onto the 2^-g grid (half to even), g < 0: none."""
    if g < 0 or not math.isfinite(x):
        return x
    return math.ldexp(round(math.ldexp(x, g)), -g)


class NaiveColumn:
    def __init__(self, params: dict, tables: dict, q):
        m = params["model"]
        g = int(params["cost_grid_log2"])
        self.q = [int(x) for x in q]
        self.H = len(self.q)
        self.S, self.G, self.O = tables["S"], tables["G"], tables["O"]
        self.hi, self.lo = tables["fg_hi"], tables["fg_lo"]
        v_hor = (self.H - 1) - float(params["camera"]["horizon_row"])
        self.top_ground = math.floor(v_hor)          # highest row a ground stixel may cover
        self.F = [q_grid(x, g) for x in m["first_cost"]]
        self.T = [[q_grid(x, g) for x in row] for row in m["trans_cost"]]
        self.beta = q_grid(m["bic_cost"], g)
        self.c_ord = q_grid(m["ordering_cost"], g)
        self.c_grav = q_grid(m["gravity_cost"], g)
        self.c_dive = q_grid(m["diving_cost"], g)
        # ordering tolerance in disparity bins of 2^-subpixel_log2 px
        self.tau = int(m["ordering_tol_px"]) << int(params.get("subpixel_log2", 0))

    def mean(self, b: int, k: int) -> int:
        vals = [d for d in self.q[b:k + 1] if d >= 0]
        if not vals:
            return 0
        return math.floor(Fraction(sum(vals), len(vals)) + Fraction(1, 2))

    def data(self, c: int, b: int, k: int, f: int) -> float:
        if c == GR and k > self.top_ground:
            return INF
        terms = []
        for v in range(b, k + 1):
            d = self.q[v]
            if d < 0:
                continue                              # invalid pixels cost nothing
            terms.append(self.O[d][f] if c == OB else (self.G[v][d] if c == GR else self.S[d]))
        return math.fsum(terms)

    def pair_prior(self, cp: int, c: int, f_prev: int, f: int, b: int) -> float:
        t = self.T[cp][c]
        if math.isinf(t):
            return INF
        pen = 0.0
        if c == OB and cp == OB and f > f_prev + self.tau:
            pen = self.c_ord                          # ordering
        if c == OB and cp == GR:
            if f > self.hi[b]:
                pen = self.c_dive                     # diving
            elif f < self.lo[b]:
                pen = self.c_grav                     # gravity
        return t + self.beta + pen

    def solve(self) -> dict:
        H = self.H
        C = [[INF] * 3 for _ in range(H)]
        link_b = [[0] * 3 for _ in range(H)]
        link_c = [[-1] * 3 for _ in range(H)]
        fob = [0] * H
        for k in range(H):
            for c in (OB, GR, SK):
                cands = []                             # (cost, b, predecessor class)
                f0 = self.mean(0, k) if c == OB else 0
                cands.append((self.data(c, 0, k, f0) + self.F[c] + self.beta, 0, -1))
                for b in range(1, k + 1):
                    f = self.mean(b, k) if c == OB else 0
                    dat = self.data(c, b, k, f)
                    for cp in (OB, GR, SK):
                        pr = self.pair_prior(cp, c, fob[b - 1], f, b)
                        cands.append((C[b - 1][cp] + pr + dat, b, cp))
                best = cands[0]
                for cand in cands[1:]:
                    if cand[0] < best[0]:
                        best = cand
                C[k][c], link_b[k][c], link_c[k][c] = best
                if c == OB:
                    fob[k] = self.mean(best[1], k)
        # backtracking from the first minimum of the top row
        c = min((OB, GR, SK), key=lambda x: (C[H - 1][x], x))
        total = C[H - 1][c]
        out = []
        k = H - 1
        while True:
            b, cp = link_b[k][c], link_c[k][c]
            f = fob[k] if c == OB else 0
            pr = self.F[c] + self.beta if b == 0 else self.pair_prior(cp, c, fob[b - 1], f, b)
            out.append((b, k, c, f, self.data(c, b, k, f) + pr))
            if b == 0:
                break
            k, c = b - 1, cp
        out.reverse()
        return dict(C=C, link_b=link_b, link_c=link_c, fob=fob, stixels=out, total=total)
