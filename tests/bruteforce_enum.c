/*
 * bruteforce_enum.c -- exhaustive MAP search over every segmentation of one
 * short column (Eq. 1-2 of the paper: a column is a list of stixels, each
 * with a class, a base and a top row; its cost is the sum over stixels of
 * the data term plus the prior of the stixel given the one below it).
 *
 * Test infrastructure, independent of the oracle's dynamic programme: it
 * shares no code with oracle/ (it never includes or links it) and it does
 * not use prefix sums.  The data term of every candidate stixel is a direct
 * sum of per-pixel costs over its rows, and an object's mean disparity is
 * the half-up rounding of sum/n done by integer division and remainder.
 * The per-pixel cost tables are inputs (they are pinned on their own).
 *
 * The search walks the stixel lists depth first from the bottom, skips
 * transitions whose prior is infinite, and keeps the minimum total and,
 * among the lists attaining it, the one whose key read from the top
 * (class of the top stixel, its base, class of the next one down, its base,
 * ...) is lexicographically smallest.  With costs on a 2^-g grid every sum
 * is exact, so equality of totals is exact.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXH 16

typedef struct {
    int H, D, vtop, tau_ord;
    const int32_t *q;
    const double *G, *S, *O;        /* G[v*D+d] bottom-up rows, S[d], O[d*D+f] */
    const int32_t *fg_hi, *fg_lo;   /* per base row b, 0..H */
    double F[3], T[3][3], beta, c_ord, c_grav, c_dive;
    /* direct data terms and means of every (class, base, top) */
    double data[3][MAXH][MAXH];
    int mean[MAXH][MAXH];
    /* search state */
    int cur_b[MAXH], cur_t[MAXH], cur_c[MAXH], cur_f[MAXH];
    double best;
    int nbest;
    int best_b[MAXH], best_t[MAXH], best_c[MAXH], best_f[MAXH];
    int64_t n_lists, n_optimal;
} bf_state;

static int half_up_mean(int64_t sum, int64_t n)
{
    if (n == 0) return 0;
    int64_t f = sum / n, r = sum - f * n;   /* sum >= 0, n > 0 */
    if (2 * r >= n) ++f;
    return (int)f;
}

static void prepare(bf_state *s)
{
    for (int b = 0; b < s->H; ++b) {
        for (int t = b; t < s->H; ++t) {
            int64_t sum = 0, n = 0;
            for (int v = b; v <= t; ++v)
                if (s->q[v] >= 0) { sum += s->q[v]; ++n; }
            const int f = half_up_mean(sum, n);
            s->mean[b][t] = f;
            double g = 0.0, k = 0.0, o = 0.0;
            for (int v = b; v <= t; ++v) {
                const int d = s->q[v];
                if (d < 0) continue;
                g += s->G[(size_t)v * s->D + d];
                k += s->S[d];
                o += s->O[(size_t)d * s->D + f];
            }
            s->data[0][b][t] = o;
            s->data[1][b][t] = (t > s->vtop) ? INFINITY : g;
            s->data[2][b][t] = k;
        }
    }
}

/* prior of a stixel (class c, mean f, base b) above the n-th stixel of the
 * current list (n < 0: it is the bottom stixel) */
static double prior(const bf_state *s, int n, int c, int f, int b)
{
    if (n < 0) return s->F[c] + s->beta;
    const int cp = s->cur_c[n];
    const double t = s->T[cp][c];
    if (isinf(t)) return INFINITY;
    double pen = 0.0;
    if (c == 0 && cp == 0 && f > s->cur_f[n] + s->tau_ord) pen = s->c_ord;
    if (c == 0 && cp == 1) {
        if (f > s->fg_hi[b]) pen = s->c_dive;
        else if (f < s->fg_lo[b]) pen = s->c_grav;
    }
    return t + s->beta + pen;
}

/* key comparison from the top: (c_N, b_N, c_{N-1}, b_{N-1}, ...) */
static int key_less(const bf_state *s, int n)
{
    for (int i = n - 1, j = s->nbest - 1; i >= 0 && j >= 0; --i, --j) {
        if (s->cur_c[i] != s->best_c[j]) return s->cur_c[i] < s->best_c[j];
        if (s->cur_b[i] != s->best_b[j]) return s->cur_b[i] < s->best_b[j];
    }
    return 0;
}

static void search(bf_state *s, int b, int n, double acc)
{
    for (int t = b; t < s->H; ++t) {
        for (int c = 0; c < 3; ++c) {
            const double d = s->data[c][b][t];
            if (isinf(d)) continue;
            const int f = (c == 0) ? s->mean[b][t] : 0;
            const double p = prior(s, n - 1, c, f, b);
            if (isinf(p)) continue;
            s->cur_b[n] = b; s->cur_t[n] = t; s->cur_c[n] = c; s->cur_f[n] = f;
            const double tot = acc + (d + p);
            if (t == s->H - 1) {
                ++s->n_lists;
                if (tot < s->best || (tot == s->best && key_less(s, n + 1))) {
                    if (tot < s->best) s->n_optimal = 0;
                    s->best = tot;
                    s->nbest = n + 1;
                    memcpy(s->best_b, s->cur_b, sizeof s->best_b);
                    memcpy(s->best_t, s->cur_t, sizeof s->best_t);
                    memcpy(s->best_c, s->cur_c, sizeof s->best_c);
                    memcpy(s->best_f, s->cur_f, sizeof s->best_f);
                }
                if (tot == s->best) ++s->n_optimal;
            } else {
                search(s, t + 1, n + 1, tot);
            }
        }
    }
}

/* Returns 0, or -1 for bad arguments.  path receives the best list bottom-up
 * as (base, top, class, mean) quadruples; *n_lists counts the finite lists. */
int bf_map(int H, const int32_t *q, int D, const double *G, const double *S, const double *O,
           const int32_t *fg_hi, const int32_t *fg_lo, int vtop, const double *F,
           const double *T, double beta, double c_ord, int tau_ord, double c_grav,
           double c_dive, double *best, int32_t *path, int32_t *npath, int64_t *n_lists,
           int64_t *n_optimal)
{
    if (H < 1 || H > MAXH || D < 1) return -1;
    bf_state *s = (bf_state *)calloc(1, sizeof(bf_state));
    if (!s) return -1;
    s->H = H; s->D = D; s->vtop = vtop; s->tau_ord = tau_ord;
    s->q = q; s->G = G; s->S = S; s->O = O; s->fg_hi = fg_hi; s->fg_lo = fg_lo;
    for (int a = 0; a < 3; ++a) {
        s->F[a] = F[a];
        for (int c = 0; c < 3; ++c) s->T[a][c] = T[3 * a + c];
    }
    s->beta = beta; s->c_ord = c_ord; s->c_grav = c_grav; s->c_dive = c_dive;
    s->best = INFINITY;
    prepare(s);
    search(s, 0, 0, 0.0);
    *best = s->best;
    *npath = s->nbest;
    for (int i = 0; i < s->nbest; ++i) {
        path[4 * i + 0] = s->best_b[i];
        path[4 * i + 1] = s->best_t[i];
        path[4 * i + 2] = s->best_c[i];
        path[4 * i + 3] = s->best_f[i];
    }
    *n_lists = s->n_lists;
    *n_optimal = s->n_optimal;
    free(s);
    return 0;
}
