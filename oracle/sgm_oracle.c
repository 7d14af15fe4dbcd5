/* sgm_oracle.c -- plain CPU semi-global matching: the stereo stage the paper
 * names as the real-time source of its disparity maps (Sec. 1 and Sec. 5
 * cite a GPU semi-global matching with census costs; the method itself is
 * Hirschmuller's, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU baseline, never by the HIP library.  Every quantity is an
 * integer, so the library's result must equal this one exactly.
 *
 * Steps, in order:
 *   census      9 x 7 window; for each of the 62 neighbours q of p, in
 *               row-major window order skipping p itself, bit i is 1 iff
 *               q lies inside the image and I(q) < I(p)
 *   cost        C(p, d) = Hamming distance of the left census at (y, x) and
 *               the right census at (y, x - d); SGM_COST_OUT when x - d < 0
 *   paths       for each direction r: L_r(p, d) = C(p, d) for the first
 *               pixel of a path, otherwise
 *               C(p, d) + min(L_r(p-r, d), L_r(p-r, d-1) + P1,
 *                             L_r(p-r, d+1) + P1, M + P2) - M
 *               with M = min_k L_r(p-r, k) (the d-1 / d+1 terms only where
 *               they exist)
 *   sum         S(p, d) = sum over the paths of L_r(p, d)
 *   selection   d_L(y, x) = the smallest d minimising S((y, x), d);
 *               d_R(y, x) = the smallest d minimising S((y, x + d), d) over
 *               d with x + d < W
 *   check       disparity(y, x) = d_L if x - d_L >= 0 and
 *               |d_L - d_R(y, x - d_L)| <= 1, else -1 (invalid)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SGM_CENSUS_W 9
#define SGM_CENSUS_H 7
#define SGM_COST_OUT 62

/* direction order of the paths: left to right, right to left, top to
 * bottom, bottom to top, then the four diagonals */
static const int SGM_DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};
static const int SGM_DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};

void sgm_census(const uint8_t* img, int W, int H, uint64_t* out) {
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const int centre = img[y * W + x];
            uint64_t c = 0;
            int bit = 0;
            for (int dy = -(SGM_CENSUS_H / 2); dy <= SGM_CENSUS_H / 2; ++dy) {
                for (int dx = -(SGM_CENSUS_W / 2); dx <= SGM_CENSUS_W / 2; ++dx) {
                    if (dy == 0 && dx == 0) continue;
                    const int yy = y + dy, xx = x + dx;
                    int b = 0;
                    if (yy >= 0 && yy < H && xx >= 0 && xx < W) b = img[yy * W + xx] < centre;
                    if (b) c |= (uint64_t)1 << bit;
                    ++bit;
                }
            }
            out[y * W + x] = c;
        }
    }
}

static int hamming(uint64_t a, uint64_t b) {
    uint64_t v = a ^ b;
    int n = 0;
    for (int i = 0; i < 64; ++i) n += (int)((v >> i) & 1u);
    return n;
}

/* Matching cost of left pixel (y, x) at disparity d. */
static int cost(const uint64_t* cl, const uint64_t* cr, int W, int y, int x, int d) {
    if (x - d < 0) return SGM_COST_OUT;
    return hamming(cl[y * W + x], cr[y * W + x - d]);
}

void sgm_costs(const uint64_t* cl, const uint64_t* cr, int W, int H, int D, uint8_t* C) {
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int d = 0; d < D; ++d)
                C[((size_t)y * W + x) * D + d] = (uint8_t)cost(cl, cr, W, y, x, d);
}

/* L_r of one direction (index into the direction table) for every pixel and
 * disparity, [H][W][D].  Pixels are visited so that p - r always comes
 * before p. */
void sgm_path(const uint64_t* cl, const uint64_t* cr, int W, int H, int D, int P1, int P2,
              int dir, uint16_t* L) {
    const int dy = SGM_DY[dir], dx = SGM_DX[dir];
    for (int i = 0; i < H; ++i) {
        const int y = dy >= 0 ? i : H - 1 - i;
        for (int j = 0; j < W; ++j) {
            const int x = dx >= 0 ? j : W - 1 - j;
            uint16_t* cur = L + ((size_t)y * W + x) * D;
            const int py = y - dy, px = x - dx;
            if (py < 0 || py >= H || px < 0 || px >= W) {
                for (int d = 0; d < D; ++d) cur[d] = (uint16_t)cost(cl, cr, W, y, x, d);
                continue;
            }
            const uint16_t* prev = L + ((size_t)py * W + px) * D;
            int M = prev[0];
            for (int k = 1; k < D; ++k)
                if (prev[k] < M) M = prev[k];
            for (int d = 0; d < D; ++d) {
                int best = prev[d];
                if (d > 0 && prev[d - 1] + P1 < best) best = prev[d - 1] + P1;
                if (d + 1 < D && prev[d + 1] + P1 < best) best = prev[d + 1] + P1;
                if (M + P2 < best) best = M + P2;
                cur[d] = (uint16_t)(cost(cl, cr, W, y, x, d) + best - M);
            }
        }
    }
}

/* d_L and d_R from the summed costs S [H][W][D]. */
void sgm_select(const uint16_t* S, int W, int H, int D, int16_t* dL, int16_t* dR) {
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const uint16_t* s = S + ((size_t)y * W + x) * D;
            int b = 0;
            for (int d = 1; d < D; ++d)
                if (s[d] < s[b]) b = d;
            dL[y * W + x] = (int16_t)b;
            int br = 0, bv = -1;
            for (int d = 0; d < D && x + d < W; ++d) {
                const int v = S[((size_t)y * W + x + d) * D + d];
                if (bv < 0 || v < bv) { bv = v; br = d; }
            }
            dR[y * W + x] = (int16_t)br;
        }
    }
}

void sgm_check(const int16_t* dL, const int16_t* dR, int W, int H, float* disp) {
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const int d = dL[y * W + x];
            float v = -1.0f;
            if (x - d >= 0) {
                const int e = dR[y * W + x - d];
                if (abs(d - e) <= 1) v = (float)d;
            }
            disp[y * W + x] = v;
        }
    }
}

/* The whole stage; S (optional, [H][W][D]) receives the summed costs.
 * Returns 0, or -1 on bad arguments or allocation failure. */
int sgm_disparity(const uint8_t* left, const uint8_t* right, int W, int H, int D, int P1, int P2,
                  int npaths, float* disp, uint16_t* S_out) {
    if (W < 1 || H < 1 || D < 1 || (npaths != 4 && npaths != 8) || P1 < 0 || P2 < 0) return -1;
    const size_t n = (size_t)W * H, nd = n * (size_t)D;
    uint64_t* cl = malloc(n * sizeof(uint64_t));
    uint64_t* cr = malloc(n * sizeof(uint64_t));
    uint16_t* L = malloc(nd * sizeof(uint16_t));
    uint16_t* S = calloc(nd, sizeof(uint16_t));
    int16_t* dL = malloc(n * sizeof(int16_t));
    int16_t* dR = malloc(n * sizeof(int16_t));
    int rc = -1;
    if (cl && cr && L && S && dL && dR) {
        sgm_census(left, W, H, cl);
        sgm_census(right, W, H, cr);
        for (int r = 0; r < npaths; ++r) {
            sgm_path(cl, cr, W, H, D, P1, P2, r, L);
            for (size_t i = 0; i < nd; ++i) S[i] = (uint16_t)(S[i] + L[i]);
        }
        sgm_select(S, W, H, D, dL, dR);
        sgm_check(dL, dR, W, H, disp);
        if (S_out) memcpy(S_out, S, nd * sizeof(uint16_t));
        rc = 0;
    }
    free(cl);
    free(cr);
    free(L);
    free(S);
    free(dL);
    free(dR);
    return rc;
}
