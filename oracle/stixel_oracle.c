/*
 * stixel_oracle.c -- plain CPU FP64 oracle of per-column multi-stixel
 * segmentation (Hernandez-Juarez et al., "GPU-accelerated real-time stixel
 * computation").
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * benchmark's CPU-baseline leg are its only callers.  It shares no code with
 * the HIP library and never calls it.
 *
 * It follows the paper's steps in order, slowly and literally:
 *   Sec. 3.1  column reduction to one pixel per row strip, ground model
 *             f_ground(v) = alpha (v_hor - v), sky model 0, object model = mean;
 *   Eq. 4     per-pixel data cost, min(outlier cost, Gaussian cost);
 *   Sec. 3.4  offline cost LUTs (ground/sky per disparity, object per
 *             (pixel disparity, mean disparity)), integer-rounded object mean,
 *             per-column prefix-sum LUTs;
 *   Eq. 5-6   the recurrence for OB^k, GR^k, SK^k over every cut position b
 *             and every predecessor class, cost table C plus index table;
 *   Sec. 3.3  backtracking from min(OB^{h-1}, GR^{h-1}, SK^{h-1}).
 *
 * Readings where the paper is silent or garbled (each one is listed with the
 * design notes):
 *   - a pixel is valid iff finite and >= 0; invalid pixels cost 0 in every
 *     class and are left out of every mean;
 *   - the reduction is the lower median of the valid pixels (reduce_mode 0) or
 *     their mean (reduce_mode 1, the paper's operator); the result is rounded
 *     half-to-even and clamped to d_range-1;
 *   - A_norm of Eq. 4 is the mass of the Gaussian on [0, d_range]; a Gaussian
 *     branch that is not finite (mass underflow) leaves the outlier cost;
 *   - the object mean f of a stixel is floor((2*sum + n) / (2*n)) (half up),
 *     f = 0 when the stixel holds no valid pixel;
 *   - a ground stixel must end at or below floor(v_hor);
 *   - the prior model (deferred by the paper to Pfeiffer's thesis) is a
 *     bottom-stixel cost F[c], a per-stixel BIC cost, a transition table
 *     T[prev][cur] with INFINITY for forbidden pairs, an ordering penalty on
 *     object-over-object when the upper mean exceeds the lower one by more
 *     than a tolerance, and a diving / gravity penalty on object-over-ground
 *     when the object mean is above / below the ground disparity at its base
 *     by more than a tolerance;
 *   - every table value and prior constant is rounded to a multiple of
 *     2^-cost_grid_log2 nats (cost_grid_log2 < 0 disables the rounding);
 *   - disparities may be resolved finer than 1 px: in bins of
 *     2^-subpixel_log2 px, the reduced pixel is rint(value * 2^subpixel_log2),
 *     object means are rounded to a bin, tables are evaluated at the bins'
 *     disparities in px, the diving / gravity thresholds are floor / ceil of
 *     the px bound times 2^subpixel_log2 and the ordering tolerance is
 *     ordering_tol_px bins times 2^subpixel_log2 (the outlier density stays
 *     uniform over [0, max_disparity] px);
 *   - ties go to the first candidate in the order of Eq. 6: the bottom-stixel
 *     candidate, then cut positions b ascending, then predecessor classes
 *     object, ground, sky; the final class is the first minimum in that order.
 */
#include "stixel_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NCLS 3

/* ---------------------------------------------------------------- Eq. 3-4 */

/* Standard normal cumulative distribution. */
static double normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

double so_pixel_cost(double d, double mu, double sigma, double p_out, double d_range)
{
    double outlier = log(d_range) - log(p_out);
    double a_norm = normal_cdf((d_range - mu) / sigma) - normal_cdf(-mu / sigma);
    double gauss = log(a_norm) + log(sigma * sqrt(2.0 * M_PI)) - log(1.0 - p_out)
                 + (d - mu) * (d - mu) / (2.0 * sigma * sigma);
    if (!(gauss == gauss) || isinf(gauss)) return outlier;
    return outlier < gauss ? outlier : gauss;
}

double so_quantize(double x, int32_t g)
{
    if (g < 0 || !isfinite(x)) return x;
    return ldexp(rint(ldexp(x, g)), -g);
}

/* ------------------------------------------------------------- Sec. 3.1 */

/* Disparity bins: max_disparity px in bins of 2^-subpixel_log2 px.  A bin
 * index i stands for the disparity i * 2^-subpixel_log2 px. */
static int32_t n_bins(const so_params *p) { return p->max_disparity << p->subpixel_log2; }

static double bin_px(const so_params *p, int32_t i) { return ldexp((double)i, -p->subpixel_log2); }

/* Ground disparity slope in px per row, from the camera (slope and horizon are
 * known per image, Sec. 3). */
static double ground_alpha(const so_params *p)
{
    return p->baseline_m * cos(p->pitch_rad) / p->cam_height_m;
}

/* Bottom-up row of the horizon for a column of height H. */
static double horizon_v(const so_params *p, int32_t H)
{
    return (double)(H - 1) - p->horizon_row;
}

/* f_ground(v) = alpha (v_hor - v) */
static double f_ground(const so_params *p, int32_t H, double v)
{
    return ground_alpha(p) * (horizon_v(p, H) - v);
}

/* Highest bottom-up row a ground stixel may reach. */
static int32_t ground_top(const so_params *p, int32_t H)
{
    double vh = floor(horizon_v(p, H));
    if (vh < -1.0) return -1;
    if (vh > (double)H) return H;
    return (int32_t)vh;
}

static double sigma_ground(const so_params *p, double mu)
{
    double e = p->ground_slope_noise * mu;
    return sqrt(p->sigma_disp * p->sigma_disp + e * e);
}

static double sigma_object(const so_params *p, double f)
{
    double e = f * f * p->object_depth_extent_m / (p->focal_px * p->baseline_m);
    return sqrt(p->sigma_disp * p->sigma_disp + e * e);
}

/* ------------------------------------------------------------- Sec. 3.4 */

int so_tables(const so_params *p, int32_t H, double *S, double *G, double *O,
              int32_t *fg_hi, int32_t *fg_lo)
{
    if (!p || H < 1 || p->max_disparity < 1 || p->subpixel_log2 < 0 || p->subpixel_log2 > 3)
        return SO_EINVAL;
    const int32_t D = n_bins(p);
    const double dr = (double)p->max_disparity;
    const int32_t g = p->cost_grid_log2;
    const int32_t vtop = ground_top(p, H);

    for (int32_t d = 0; d < D; ++d)
        S[d] = so_quantize(so_pixel_cost(bin_px(p, d), 0.0, p->sigma_sky, p->p_out, dr), g);

    for (int32_t v = 0; v < H; ++v) {
        double mu = f_ground(p, H, v);
        for (int32_t d = 0; d < D; ++d)
            G[(size_t)v * D + d] = (v <= vtop)
                ? so_quantize(so_pixel_cost(bin_px(p, d), mu, sigma_ground(p, mu), p->p_out, dr), g)
                : 0.0;
    }

    for (int32_t d = 0; d < D; ++d)
        for (int32_t f = 0; f < D; ++f)
            O[(size_t)d * D + f] =
                so_quantize(so_pixel_cost(bin_px(p, d), bin_px(p, f),
                                          sigma_object(p, bin_px(p, f)), p->p_out, dr), g);

    for (int32_t b = 0; b <= H; ++b) {
        double fg = f_ground(p, H, b);
        fg_hi[b] = (int32_t)floor(ldexp(fg + p->diving_tol_px, p->subpixel_log2));
        fg_lo[b] = (int32_t)ceil(ldexp(fg - p->gravity_tol_px, p->subpixel_log2));
    }
    return SO_OK;
}

/* Column reduction: one value per row of each s-pixel-wide strip, written
 * transposed and bottom-up (q[i*H + v], v = H-1-r). */
int so_reduce(const so_params *p, const float *disp, int32_t W, int32_t H, int32_t *q)
{
    if (!p || !disp || !q || p->subpixel_log2 < 0 || p->subpixel_log2 > 3) return SO_EINVAL;
    const int32_t s = p->stixel_width;
    if (s < 1 || W < s || H < 1) return SO_EINVAL;
    const int32_t ncols = W / s;
    double *vals = (double *)malloc(sizeof(double) * (size_t)s);
    if (!vals) return SO_EINVAL;
    for (int32_t i = 0; i < ncols; ++i) {
        for (int32_t r = 0; r < H; ++r) {
            int32_t n = 0;
            for (int32_t t = 0; t < s; ++t) {
                double x = disp[(size_t)r * W + (size_t)i * s + t];
                if (isfinite(x) && x >= 0.0) vals[n++] = x;
            }
            int32_t out = -1;
            if (n > 0) {
                double m;
                if (p->reduce_mode == 0) {
                    /* insertion sort, then the lower median */
                    for (int32_t a = 1; a < n; ++a) {
                        double key = vals[a];
                        int32_t c = a - 1;
                        while (c >= 0 && vals[c] > key) { vals[c + 1] = vals[c]; --c; }
                        vals[c + 1] = key;
                    }
                    m = vals[(n - 1) / 2];
                } else {
                    double sum = 0.0;
                    for (int32_t a = 0; a < n; ++a) sum += vals[a];
                    m = sum / (double)n;
                }
                double rq = rint(ldexp(m, p->subpixel_log2));
                double top = (double)(n_bins(p) - 1);
                out = (int32_t)(rq < top ? rq : top);
            }
            q[(size_t)i * H + (H - 1 - r)] = out;
        }
    }
    free(vals);
    return SO_OK;
}

/* ------------------------------------------------------------- Sec. 3.3 */

typedef struct {
    const so_params *p;
    int32_t H, D, vtop;
    const double *S, *G, *O;
    const int32_t *fg_hi, *fg_lo;
    double F[NCLS], T[NCLS][NCLS], beta, c_ord, c_grav, c_dive;
    /* per-column prefix-sum LUTs */
    double *PG, *PS, *PO;
    int64_t *PD, *PN;
} column_ctx;

/* Prefix sums of the per-pixel costs and of the disparities (Sec. 3.4):
 * entry v+1 accumulates rows 0..v, entry 0 is zero. */
static void build_prefix(column_ctx *x, const int32_t *q)
{
    const int32_t H = x->H, D = x->D;
    x->PG[0] = 0.0; x->PS[0] = 0.0; x->PD[0] = 0; x->PN[0] = 0;
    for (int32_t f = 0; f < D; ++f) x->PO[(size_t)f * (H + 1)] = 0.0;
    for (int32_t v = 0; v < H; ++v) {
        int32_t d = q[v];
        int valid = d >= 0;
        x->PG[v + 1] = x->PG[v] + (valid ? x->G[(size_t)v * D + d] : 0.0);
        x->PS[v + 1] = x->PS[v] + (valid ? x->S[d] : 0.0);
        x->PD[v + 1] = x->PD[v] + (valid ? d : 0);
        x->PN[v + 1] = x->PN[v] + (valid ? 1 : 0);
        for (int32_t f = 0; f < D; ++f) {
            size_t row = (size_t)f * (H + 1);
            x->PO[row + v + 1] = x->PO[row + v] + (valid ? x->O[(size_t)d * D + f] : 0.0);
        }
    }
}

/* Integer-rounded mean disparity of the valid pixels of rows b..t. */
static int32_t object_mean(const column_ctx *x, int32_t b, int32_t t)
{
    int64_t n = x->PN[t + 1] - x->PN[b];
    int64_t sum = x->PD[t + 1] - x->PD[b];
    if (n == 0) return 0;
    return (int32_t)((2 * sum + n) / (2 * n));
}

/* C_data of a stixel of class c over rows b..t, from two prefix entries. */
static double data_cost(const column_ctx *x, int32_t c, int32_t b, int32_t t, int32_t f)
{
    const int32_t H = x->H;
    switch (c) {
    case SO_GROUND:
        if (t > x->vtop) return INFINITY;
        return x->PG[t + 1] - x->PG[b];
    case SO_SKY:
        return x->PS[t + 1] - x->PS[b];
    default: {
        size_t row = (size_t)f * (H + 1);
        return x->PO[row + t + 1] - x->PO[row + b];
    }
    }
}

/* C_prior of the bottom stixel. */
static double prior_first(const column_ctx *x, int32_t c) { return x->F[c] + x->beta; }

/* C_prior(s_n, s_{n-1}) of a stixel of class c with mean f and base b on top
 * of the stored best stixel of class cp (object mean f_prev) ending at b-1. */
static double prior_pair(const column_ctx *x, int32_t cp, int32_t c, int32_t f_prev,
                         int32_t f, int32_t b)
{
    double t = x->T[cp][c];
    if (isinf(t)) return INFINITY;
    double pen = 0.0;
    if (c == SO_OBJECT && cp == SO_OBJECT &&
        f > f_prev + (x->p->ordering_tol_px << x->p->subpixel_log2))
        pen = x->c_ord;
    if (c == SO_OBJECT && cp == SO_GROUND) {
        if (f > x->fg_hi[b]) pen = x->c_dive;
        else if (f < x->fg_lo[b]) pen = x->c_grav;
    }
    return t + x->beta + pen;
}

/* Eq. 5-6: fills C, the index table and the object mean of each best object
 * stixel.  Candidates are visited in the order Eq. 6 lists them. */
static void solve_dp(const column_ctx *x, double *C, int32_t *link_b, int32_t *link_c,
                     int32_t *fob)
{
    const int32_t H = x->H;
    for (int32_t k = 0; k < H; ++k) {
        for (int32_t c = 0; c < NCLS; ++c) {
            int32_t f0 = (c == SO_OBJECT) ? object_mean(x, 0, k) : 0;
            double best = data_cost(x, c, 0, k, f0) + prior_first(x, c);
            int32_t bb = 0, bc = -1;
            for (int32_t b = 1; b <= k; ++b) {
                int32_t f = (c == SO_OBJECT) ? object_mean(x, b, k) : 0;
                double dat = data_cost(x, c, b, k, f);
                for (int32_t cp = 0; cp < NCLS; ++cp) {
                    double cand = C[(size_t)(b - 1) * NCLS + cp]
                                + prior_pair(x, cp, c, fob[b - 1], f, b) + dat;
                    if (cand < best) { best = cand; bb = b; bc = cp; }
                }
            }
            C[(size_t)k * NCLS + c] = best;
            link_b[(size_t)k * NCLS + c] = bb;
            link_c[(size_t)k * NCLS + c] = bc;
            if (c == SO_OBJECT) fob[k] = object_mean(x, bb, k);
        }
    }
}

/* Backtracking from the top row along the index table; returns the number of
 * stixels, written bottom-up into out[]. */
static int32_t backtrack(const column_ctx *x, const double *C, const int32_t *link_b,
                         const int32_t *link_c, const int32_t *fob, so_stixel *out,
                         double *total)
{
    const int32_t H = x->H;
    int32_t c = 0;
    for (int32_t cc = 1; cc < NCLS; ++cc)
        if (C[(size_t)(H - 1) * NCLS + cc] < C[(size_t)(H - 1) * NCLS + c]) c = cc;
    *total = C[(size_t)(H - 1) * NCLS + c];
    int32_t n = 0, k = H - 1;
    while (k >= 0) {
        int32_t b = link_b[(size_t)k * NCLS + c];
        int32_t cp = link_c[(size_t)k * NCLS + c];
        int32_t f = (c == SO_OBJECT) ? fob[k] : 0;
        double cost = data_cost(x, c, b, k, f)
                    + (b == 0 ? prior_first(x, c)
                              : prior_pair(x, cp, c, fob[b - 1], f, b));
        out[n].v_bottom = b;
        out[n].v_top = k;
        out[n].cls = c;
        out[n].disparity = f;
        out[n].cost = cost;
        ++n;
        if (b == 0) break;
        k = b - 1;
        c = cp;
    }
    /* top-down discovery order -> bottom-up output order */
    for (int32_t a = 0, z = n - 1; a < z; ++a, --z) {
        so_stixel tmp = out[a]; out[a] = out[z]; out[z] = tmp;
    }
    return n;
}

static int validate(const so_params *p)
{
    if (!p) return SO_EINVAL;
    if (p->max_disparity < 1 || p->stixel_width < 1) return SO_EINVAL;
    if (p->subpixel_log2 < 0 || p->subpixel_log2 > 3) return SO_EINVAL;
    if (!(p->p_out > 0.0 && p->p_out < 1.0)) return SO_EINVAL;
    if (!(p->sigma_disp > 0.0 && p->sigma_sky > 0.0)) return SO_EINVAL;
    if (!(p->cam_height_m > 0.0 && p->focal_px > 0.0 && p->baseline_m > 0.0)) return SO_EINVAL;
    for (int c = 0; c < NCLS; ++c) {
        if (!isfinite(p->first_cost[c])) return SO_EINVAL;
        if (!isfinite(p->trans_cost[c][SO_OBJECT])) return SO_EINVAL;
    }
    return SO_OK;
}

static void fill_ctx(column_ctx *x, const so_params *p, int32_t H)
{
    const int32_t g = p->cost_grid_log2;
    x->p = p;
    x->H = H;
    x->D = n_bins(p);
    x->vtop = ground_top(p, H);
    for (int c = 0; c < NCLS; ++c) {
        x->F[c] = so_quantize(p->first_cost[c], g);
        for (int cc = 0; cc < NCLS; ++cc) x->T[c][cc] = so_quantize(p->trans_cost[c][cc], g);
    }
    x->beta = so_quantize(p->bic_cost, g);
    x->c_ord = so_quantize(p->ordering_cost, g);
    x->c_grav = so_quantize(p->gravity_cost, g);
    x->c_dive = so_quantize(p->diving_cost, g);
}

int so_column(const so_params *p, int32_t H, const int32_t *q,
              double *PG, double *PS, int64_t *PD, int64_t *PN, double *PO,
              double *C, int32_t *link_b, int32_t *link_c, int32_t *fob,
              so_stixel *out, int32_t *n_out, double *total)
{
    if (validate(p) != SO_OK || H < 1 || !q) return SO_EINVAL;
    const int32_t D = n_bins(p);
    double *S = (double *)malloc(sizeof(double) * (size_t)D);
    double *G = (double *)malloc(sizeof(double) * (size_t)H * D);
    double *O = (double *)malloc(sizeof(double) * (size_t)D * D);
    int32_t *hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(H + 1));
    int32_t *lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(H + 1));
    int rc = SO_EINVAL;
    if (S && G && O && hi && lo && so_tables(p, H, S, G, O, hi, lo) == SO_OK) {
        column_ctx x;
        fill_ctx(&x, p, H);
        x.S = S; x.G = G; x.O = O; x.fg_hi = hi; x.fg_lo = lo;
        x.PG = PG; x.PS = PS; x.PD = PD; x.PN = PN; x.PO = PO;
        build_prefix(&x, q);
        solve_dp(&x, C, link_b, link_c, fob);
        *n_out = backtrack(&x, C, link_b, link_c, fob, out, total);
        rc = SO_OK;
    }
    free(S); free(G); free(O); free(hi); free(lo);
    return rc;
}

int so_frame(const so_params *p, const float *disp, int32_t W, int32_t H, int32_t cap,
             int32_t *counts, so_stixel *recs, double *total, uint8_t *overflow,
             int32_t nthreads)
{
    if (validate(p) != SO_OK || !disp || H < 1 || W < p->stixel_width) return SO_EINVAL;
    const int32_t D = n_bins(p);
    const int32_t ncols = W / p->stixel_width;
    if (cap <= 0) cap = H;
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncols * H);
    double *S = (double *)malloc(sizeof(double) * (size_t)D);
    double *G = (double *)malloc(sizeof(double) * (size_t)H * D);
    double *O = (double *)malloc(sizeof(double) * (size_t)D * D);
    int32_t *hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(H + 1));
    int32_t *lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(H + 1));
    int rc = SO_EINVAL;
    if (q && S && G && O && hi && lo && so_reduce(p, disp, W, H, q) == SO_OK &&
        so_tables(p, H, S, G, O, hi, lo) == SO_OK) {
        rc = SO_OK;
#ifdef _OPENMP
        int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
        for (int32_t i = 0; i < ncols; ++i) {
            column_ctx x;
            fill_ctx(&x, p, H);
            x.S = S; x.G = G; x.O = O; x.fg_hi = hi; x.fg_lo = lo;
            x.PG = (double *)malloc(sizeof(double) * (size_t)(H + 1));
            x.PS = (double *)malloc(sizeof(double) * (size_t)(H + 1));
            x.PD = (int64_t *)malloc(sizeof(int64_t) * (size_t)(H + 1));
            x.PN = (int64_t *)malloc(sizeof(int64_t) * (size_t)(H + 1));
            x.PO = (double *)malloc(sizeof(double) * (size_t)D * (H + 1));
            double *C = (double *)malloc(sizeof(double) * (size_t)H * NCLS);
            int32_t *lb = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * NCLS);
            int32_t *lc = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * NCLS);
            int32_t *fob = (int32_t *)malloc(sizeof(int32_t) * (size_t)H);
            so_stixel *col = (so_stixel *)malloc(sizeof(so_stixel) * (size_t)H);
            build_prefix(&x, q + (size_t)i * H);
            solve_dp(&x, C, lb, lc, fob);
            double tot;
            int32_t n = backtrack(&x, C, lb, lc, fob, col, &tot);
            int32_t m = n < cap ? n : cap;
            counts[i] = m;
            overflow[i] = (uint8_t)(n > cap);
            total[i] = tot;
            memcpy(recs + (size_t)i * cap, col, sizeof(so_stixel) * (size_t)m);
            free(x.PG); free(x.PS); free(x.PD); free(x.PN); free(x.PO);
            free(C); free(lb); free(lc); free(fob); free(col);
        }
    }
    (void)nthreads;
    free(q); free(S); free(G); free(O); free(hi); free(lo);
    return rc;
}
