/*
 * stixel_oracle.h -- plain CPU FP64 oracle of per-column multi-stixel
 * segmentation (Hernandez-Juarez et al., "GPU-accelerated real-time stixel
 * computation", Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only callers.  Nothing here is shared
 * with the HIP library: no header, table builder or helper.
 *
 * Conventions
 *   rows v are bottom-up inside a column (v = 0 is the bottom pixel, Sec. 3.1);
 *   disparities are integer bins of 2^-subpixel_log2 px (1 px by default);
 *   classes are 0 = object, 1 = ground, 2 = sky (the order of the class set);
 *   all costs are negative log-likelihoods in nats.
 */
#ifndef STIXEL_ORACLE_H
#define STIXEL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SO_OBJECT = 0, SO_GROUND = 1, SO_SKY = 2 };
enum { SO_OK = 0, SO_EINVAL = -1 };

typedef struct {
    /* camera; horizon_row is a top-down image row */
    double focal_px, baseline_m, cam_height_m, horizon_row, pitch_rad;
    /* sensor model (Eq. 3-4) */
    double p_out, sigma_disp, sigma_sky, ground_slope_noise, object_depth_extent_m;
    /* prior model (Sec. 3 constraints 1-5) */
    double bic_cost;
    double first_cost[3];
    double trans_cost[3][3];      /* [previous class][current class]; INFINITY = forbidden */
    double ordering_cost;
    double gravity_cost, gravity_tol_px, diving_cost, diving_tol_px;
    int32_t ordering_tol_px;
    /* geometry / numerics */
    int32_t stixel_width, max_disparity, max_stixels_per_column, reduce_mode, cost_grid_log2;
    /* disparity bins of 2^-subpixel_log2 px (0..3): pixel disparities, object
     * means and the rows of the object tables are bin indices; max_disparity
     * stays in px, so there are max_disparity << subpixel_log2 bins */
    int32_t subpixel_log2;
} so_params;

typedef struct {
    int32_t v_bottom, v_top, cls, disparity;
    double cost;
} so_stixel;

/* Eq. 4 for one pixel, unquantized. */
double so_pixel_cost(double d, double mu, double sigma, double p_out, double d_range);
/* Rounding of a table value onto the cost grid, 2^-g nats (g < 0: identity). */
double so_quantize(double x, int32_t g);

/* Offline tables for a frame of height H (Sec. 3.4), D = number of bins:
 *   S[d]        sky cost,                                      D values
 *   G[v*D + d]  ground cost at bottom-up row v (0 above horizon), H*D values
 *   O[d*D + f]  object cost of pixel disparity d, mean f,      D*D values
 *   fg_hi[b], fg_lo[b]  integer diving / gravity thresholds (in bins) for an
 *               object whose base is row b, b = 0..H           H+1 values each */
int so_tables(const so_params *p, int32_t H, double *S, double *G, double *O,
              int32_t *fg_hi, int32_t *fg_lo);

/* Column reduction + transpose (Sec. 3.1, Sec. 4.1): q[i*H + v], -1 = invalid. */
int so_reduce(const so_params *p, const float *disp, int32_t W, int32_t H, int32_t *q);

/* One column, every intermediate exposed.  Arrays:
 *   PG, PS [H+1]; PD, PN [H+1]; PO [D*(H+1)] (row f, column v);
 *   C [H*3]; link_b, link_c [H*3] (link_c = -1 for the bottom stixel); fob [H];
 *   out [H] stixels bottom-up, *n_out their number, *total the column cost. */
int so_column(const so_params *p, int32_t H, const int32_t *q,
              double *PG, double *PS, int64_t *PD, int64_t *PN, double *PO,
              double *C, int32_t *link_b, int32_t *link_c, int32_t *fob,
              so_stixel *out, int32_t *n_out, double *total);

/* Whole frame: reduction, tables, DP and backtracking for every column.
 * counts[ncols], recs[ncols*cap], total[ncols], overflow[ncols]; cap = 0
 * means H.  nthreads <= 0 uses the OpenMP default. */
int so_frame(const so_params *p, const float *disp, int32_t W, int32_t H, int32_t cap,
             int32_t *counts, so_stixel *recs, double *total, uint8_t *overflow,
             int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
