/*
 * stixels.h -- C ABI of the gfx950 multi-stixel segmentation library.
 *
 * The library segments every column of a dense disparity map into ground,
 * object and sky stixels (Hernandez-Juarez et al., "GPU-accelerated real-time
 * stixel computation", Sec. 3): a W x h disparity map, a stixel width s and a
 * camera whose ground slope and horizon are known go in (Sec. 3, Sec. 3.1);
 * per reduced column, an ordered list of stixels {v_bottom, v_top, class}
 * with an integer disparity for objects comes out (Sec. 3.3, Sec. 4.4).
 *
 * Conventions shared by every entry point
 *   - Pointers named d_* are device (HIP) memory owned by the caller; host
 *     pointers are named host_*.  The library never frees caller memory.
 *   - Rows inside a column are bottom-up (v = 0 is the bottom image row,
 *     Sec. 3.1); the input image itself is row-major, row 0 at the top.
 *   - Classes: 0 = object, 1 = ground, 2 = sky.  Costs are negative log
 *     likelihoods in nats.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Compute calls are asynchronous on that stream; results are valid once
 *     the stream has been synchronised.
 *   - Every call returns STIXELS_OK (0) or a negative STIXELS_E_* code; the
 *     text of the last error of a handle is available from
 *     stixels_last_error().  On error nothing is enqueued and no output is
 *     touched.
 */
#ifndef STIXELS_H
#define STIXELS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STIXELS_ABI_VERSION 1

enum {
    STIXELS_OK = 0,
    STIXELS_E_INVALID_ARG = -1, /* null pointer, size out of the handle's limits, bad parameter */
    STIXELS_E_RANGE = -2,       /* parameters would break exact arithmetic on the cost grid */
    STIXELS_E_HIP = -3,         /* a HIP call or kernel launch failed */
    STIXELS_E_NOMEM = -4        /* device or host allocation failed */
};

enum { STIXELS_OBJECT = 0, STIXELS_GROUND = 1, STIXELS_SKY = 2 };

/* Stereo camera.  The ground slope in disparity per row is
 * baseline * cos(pitch) / height and the ground disparity of top-down image
 * row r is slope * (r - horizon_row) (Sec. 3.1, ground model).  horizon_row
 * must be a multiple of 1/256 with |horizon_row| <= 2^20; |pitch| < pi/2. */
typedef struct {
    double focal_px, baseline_m, cam_height_m, horizon_row, pitch_rad;
} stixels_camera;

/* Sensor model (Eq. 3-4) and prior model (Sec. 3, constraints 1-5).
 * Class order of the arrays: object, ground, sky.  trans_cost[prev][cur] is
 * the prior of a `cur` stixel directly above a `prev` stixel; INFINITY marks
 * a forbidden pair.  Every prior value must be >= 0, first_cost must be
 * finite and trans_cost[*][object] finite (an object can always follow). */
typedef struct {
    double p_out;                 /* outlier rate, 0 < p_out < 1 */
    double sigma_disp;            /* disparity noise [px] */
    double sigma_sky;             /* sky model sigma [px] */
    double ground_slope_noise;    /* ground sigma = sqrt(sigma_disp^2 + (this * f_ground)^2) */
    double object_depth_extent_m; /* object sigma = sqrt(sigma_disp^2 + (f^2 * this / (focal * baseline))^2) */
    double bic_cost;              /* cost per stixel (constraint 1) */
    double first_cost[3];         /* prior of the bottom stixel */
    double trans_cost[3][3];      /* staggering (constraint 4) and pair costs */
    double ordering_cost;         /* object over object with larger mean (constraint 3) */
    double gravity_cost, gravity_tol_px; /* object over ground, mean below ground disparity (2) */
    double diving_cost, diving_tol_px;   /* object over ground, mean above ground disparity (5) */
    int32_t ordering_tol_px;      /* integer tolerance of the ordering constraint */
    int32_t reserved0;
} stixels_model;

typedef struct {
    stixels_camera camera;
    stixels_model model;
    int32_t stixel_width;        /* s: pixels reduced into one column, 1..16 */
    int32_t max_disparity;       /* d_range: disparities 0..d_range-1, 2..256 */
    int32_t max_width;           /* largest frame width accepted by stixels_compute */
    int32_t max_height;          /* largest frame height, 1..1024 */
    int32_t max_stixels_per_column; /* output records per column, 0 = the frame height */
    int32_t reduce_mode;         /* 0 = lower median of the valid pixels, 1 = mean (Sec. 4.1) */
    int32_t cost_grid_log2;      /* g: costs are multiples of 2^-g nats, 0..12; results then
                                    equal an FP64 evaluation bit for bit.  -1: costs off
                                    any grid (FP32 tables and sums, not exact): frames run
                                    the fused kernel with a stored index table (Sec. 3.3)
                                    for the backtracking, stixel costs are summed directly
                                    over their pixels, and results agree with FP64 up to
                                    near-ties and rounding */
    int32_t flags;               /* STIXELS_FLAG_* bits, 0 = none */
    int32_t subpixel_log2;       /* k, 0..3: disparities in bins of 2^-k px (Sec. 3.4 rounds
                                    pixels and object means to whole px; k > 0 resolves them
                                    finer).  Reduced pixels, object means, the record's
                                    disparity and the table rows are bin indices; Eq. 4 is
                                    evaluated at the bins' disparities in px.  There are
                                    max_disparity << k bins, at most 256. */
    int32_t reserved1;
} stixels_params;

/* stixels_params.flags: the handle is used only through the batch API
 * (stixels_batch_*, stixels_compute_batch), so stixels_create allocates no
 * per-frame workspace and stixels_compute returns STIXELS_E_INVALID_ARG. */
#define STIXELS_FLAG_BATCH_ONLY 1

/* One stixel, 12 bytes.  v_bottom..v_top are inclusive bottom-up rows;
 * disparity is the rounded mean of an object's valid pixels, 0 otherwise;
 * cost is the stixel's data term plus its prior (Sec. 3.3), so the costs of
 * a column sum to its total cost. */
typedef struct {
    int16_t v_bottom, v_top;
    uint8_t cls, disparity;
    uint16_t flags;              /* reserved, 0 */
    float cost;
} stixels_record;

/* Caller-owned device output of one frame with ncols = floor(width / s)
 * columns.  records holds `capacity` records per column; when a column has
 * more stixels than that, its bottom-most `capacity` stixels are kept, counts
 * is `capacity` and overflow is 1. */
typedef struct {
    int32_t *counts;             /* [ncols] */
    stixels_record *records;     /* [ncols][capacity], bottom-up within a column */
    float *total_cost;           /* [ncols], min(OB^{h-1}, GR^{h-1}, SK^{h-1}) */
    uint8_t *overflow;           /* [ncols]; 1 = truncated to capacity, 255 = backtracking
                                    found no predecessor (never expected; counts is 0) */
    int32_t capacity;
    int32_t reserved0;
} stixels_output;

typedef struct stixels_handle stixels_handle;

/* Camera pose of one frame.  The paper takes the ground slope and the
 * horizon as known for each image (Sec. 3); a frame that brings its own pose
 * is segmented with the ground model of that pose instead of the handle's
 * camera: slope baseline * cos(pitch_rad) / cam_height (focal, baseline and
 * height stay the handle's), horizon at top-down row horizon_row.  The
 * handle's ground table (Eq. 4 per row and pixel disparity) and the diving /
 * gravity thresholds are rebuilt on the device for the frame; the sky and
 * object tables do not depend on the pose.  Valid poses: horizon_row a
 * multiple of 1/256 with |horizon_row| <= 2^20, |pitch_rad| < pi/2
 * (finite), and a ground disparity at the frame's bottom row of at
 * most max_disparity. */
typedef struct {
    double horizon_row, pitch_rad;
} stixels_pose;

/* Validate the parameters, build the offline cost tables of Sec. 3.4 on the
 * host in FP64 (Eq. 4 for every pair of pixel disparity and model disparity,
 * rounded to the 2^-g grid), upload them and allocate a workspace for frames
 * up to max_width x max_height.  Must be called with the target device
 * current.  Returns STIXELS_E_RANGE when (max_height + 1) * (largest table
 * cost) plus the priors could leave the exact range of FP32 on the grid, or
 * when max_height * max_disparity > 2^20. */
int stixels_create(const stixels_params *params, stixels_handle **out);

/* Release the tables and the workspace.  NULL is accepted. */
int stixels_destroy(stixels_handle *h);

/* Device bytes the handle holds: its resident tables, its per-frame
 * workspace (none with STIXELS_FLAG_BATCH_ONLY) and the batch object of
 * stixels_compute_batch, if one exists. */
int stixels_device_bytes(const stixels_handle *h, size_t *bytes);

/* Number of reduced columns of a frame of this width: floor(width / s). */
int stixels_num_columns(const stixels_handle *h, int32_t width, int32_t *ncols);

/* Records per column that an output for a frame of this height must hold. */
int stixels_output_capacity(const stixels_handle *h, int32_t height, int32_t *capacity);

/* Device bytes of the four output arrays of a frame of this size (Sec. 4.4:
 * a fixed-capacity list per column): ncols * (4 counts + capacity * 12
 * records + 4 total + 1 overflow), ncols = floor(width / s) and capacity as
 * stixels_output_capacity.  The caller allocates them (one buffer or four)
 * and fills a stixels_output.  STIXELS_E_INVALID_ARG for a null handle or
 * pointer, width < s or height < 1. */
int stixels_output_bytes(const stixels_handle *h, int32_t width, int32_t height, size_t *bytes);

/* Segment one frame (Sec. 4.1-4.4): column reduction and transpose, the
 * per-column prefix-sum tables, the Eq. 5-6 recurrence and backtracking.
 * d_disparity: device float32 [height][width], row-major, dense; a pixel is
 * valid iff it is finite and >= 0.  width >= s, width <= max_width,
 * 1 <= height <= max_height; out->capacity >= 1.  Uses the handle's
 * workspace, so calls on one handle must not overlap (one handle per stream,
 * or the batch API).  Allocates nothing. */
int stixels_compute(stixels_handle *h, const float *d_disparity, int32_t width, int32_t height,
                    void *stream, const stixels_output *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * stixels_compute through the fused persistent kernel with its workspace in
 * a fixed device array of the library (64 MiB per GPU, held from the first
 * stixels_create on that GPU until the process ends) instead of the
 * handle's workspace, so it also runs on STIXELS_FLAG_BATCH_ONLY handles.
 * Arguments and output as stixels_compute; the handle's camera pose only.
 * The handle's device must be current.  Frames whose descriptor, task list
 * and one scratch slot (the four small prefix tables and room for the
 * object prefix table, about (bins + 1) * (height + 7) floats) exceed the array
 * return STIXELS_E_RANGE (no valid handle reaches that); a frame with more
 * columns than the array has slots runs on fewer workgroups.  Allocates
 * nothing.  Every call on one GPU shares that GPU's array, so calls that
 * overlap on one GPU (other streams, other threads, other handles) race and
 * must be ordered by the caller. */
int stixels_compute_noalloc(stixels_handle *h, const float *d_disparity, int32_t width,
                            int32_t height, void *stream, const stixels_output *out);

/* stixels_compute for a frame with its own camera pose (see stixels_pose):
 * the frame's ground table and thresholds are built on the device into the
 * handle's pose area, on `stream`, ahead of the frame's kernels.  Same
 * arguments, ownership and errors as stixels_compute, plus
 * STIXELS_E_INVALID_ARG for a null or invalid pose and STIXELS_E_RANGE when
 * the handle's cost range leaves no room for other poses.  pose equal to the
 * handle's camera gives the results of stixels_compute. */
int stixels_compute_pose(stixels_handle *h, const float *d_disparity, int32_t width,
                         int32_t height, const stixels_pose *pose, void *stream,
                         const stixels_output *out);

/* How stixels_compute runs a frame: 1 = three staged kernels (reduction and
 * transpose, prefix tables into the handle's workspace, recurrence and
 * backtracking: Sec. 4.1, 4.2, 4.3-4.4 as separate steps, as in the paper);
 * 2 = one launch of the persistent fused kernel of the batch API over the
 * frame's columns (each column reduced, tabulated, solved and backtracked
 * inside one workgroup, its tables in a scratch slot of the handle's
 * workspace); 0 (the default) = automatic (currently 1).  Results do not
 * depend on it.  The intermediates of stixels_debug_stage exist only after a
 * staged call.  STIXELS_E_INVALID_ARG for other values. */
int stixels_set_frame_path(stixels_handle *h, int32_t path);

/* Object costs of the staged path's prefix-table kernel (Sec. 4.2): 0 (the
 * default) = the offline LUT of Sec. 3.4, one table lookup per (pixel,
 * mean); 1 = Eq. 4 evaluated online per (pixel, mean) in FP64 from a per-mean
 * constant (its normalisation) and rounded to the grid, as the paper's
 * online alternative that its offline LUT replaced.  Results do not depend
 * on it (the online values equal the LUT's bit for bit); the fused and batch
 * paths always use the LUT.  STIXELS_E_INVALID_ARG for other values. */
int stixels_set_object_lut(stixels_handle *h, int32_t mode);

/* The path (1 or 2) stixels_compute takes under the current setting (0 for a
 * null handle). */
int stixels_get_frame_path(const stixels_handle *h);

/* Wavefronts per column of the recurrence in stixels_compute (Sec. 4.3
 * assigns one thread block per column; here a column's rows are shared by
 * 1, 2 or 4 wave64s, interleaved by 64-row slot).  0 (the default) picks
 * automatically from the frame's column count and the device's compute
 * units; a request is capped by the rows: 4 needs more than 192 rows, 2
 * more than 64.  Results do not depend on it.  STIXELS_E_INVALID_ARG for
 * other values. */
int stixels_set_waves(stixels_handle *h, int32_t waves);

/* Waves per column that stixels_compute uses for a frame of this size under
 * the current setting (0 for a null handle or a size below the minimum). */
int stixels_get_waves(const stixels_handle *h, int32_t height, int32_t width);

/* Placement of a column's object prefix table (Sec. 4.2 keeps LUT_object in
 * global memory) for the recurrence of stixels_compute: 1 = read from
 * global memory (HBM and the caches); 2 = copied into the workgroup's LDS
 * when the column's table (its disparity rows x (height+1) floats) fits,
 * else global memory; 0 (the default) = as 2 for heights up to 512, as 1
 * above.  The LDS copy applies to one wave per column and max_disparity
 * <= 128; other launches read global memory.  Results do not depend on it.
 * STIXELS_E_INVALID_ARG for other values. */
int stixels_set_po_placement(stixels_handle *h, int32_t placement);

/* Text of the last error reported on this handle ("" if none); with NULL,
 * the reason the last stixels_create or stixels_host_table of this thread
 * failed. */
const char *stixels_last_error(const stixels_handle *h);

/* Static description of a status code. */
const char *stixels_status_string(int code);

/* ------------------------------------------------------------------ batch
 * Many frames, possibly from different handles (cameras) and of different
 * sizes, in one persistent launch: every (frame, column) pair is a task,
 * tasks are ordered by decreasing h^2 (the cost of the recurrence, Sec. 3.3)
 * and pulled by resident workgroups from a device counter.  Results are
 * bitwise identical to stixels_compute on each frame alone. */
typedef struct {
    stixels_handle *handle;      /* camera model and tables; its workspace is not used */
    const float *d_disparity;    /* device [height][width] */
    int32_t width, height;
    stixels_output out;
    stixels_pose pose;           /* the frame's own camera pose, read when use_pose = 1 */
    int32_t use_pose;            /* 0 = the handle's camera, 1 = pose (needs a batch
                                    created with STIXELS_BATCH_POSES) */
    int32_t reserved0;
} stixels_job;

typedef struct {
    int32_t max_jobs;            /* frames per call */
    int32_t max_tasks;           /* (frame, column) pairs per call */
    int32_t max_height;          /* tallest frame */
    int32_t max_disparity;       /* most disparity bins of the handles used
                                    (max_disparity << subpixel_log2) */
    int32_t workgroups;          /* persistent workgroups, 0 = chosen by the library */
    int32_t flags;               /* STIXELS_BATCH_* bits */
} stixels_batch_config;

/* stixels_batch_config.flags: jobs may bring their own camera pose; the
 * batch then holds one ground table area per job, max_jobs * (max_height *
 * max_disparity * 4 + max_height * 8) bytes, filled on the device by a
 * table-building kernel that runs ahead of the persistent launch (and is
 * captured with it). */
#define STIXELS_BATCH_POSES 1

typedef struct stixels_batch stixels_batch;

/* Allocate the task list, descriptors and per-workgroup scratch. */
int stixels_batch_create(const stixels_batch_config *cfg, stixels_batch **out);
int stixels_batch_destroy(stixels_batch *b);

/* Enqueue one persistent launch over all jobs.  Jobs must fit the batch's
 * limits and each job the limits of its handle.  Calls on one batch object
 * must not overlap.  Host-side job descriptors are staged through pinned
 * memory owned by the batch; nothing is allocated per call. */
int stixels_batch_compute(stixels_batch *b, const stixels_job *jobs, int32_t n, void *stream);

/* Capture the launch of stixels_batch_compute for these jobs into a HIP
 * graph owned by the batch (replacing any previous one), then replay it with
 * stixels_batch_replay.  The graph reads the same device buffers on every
 * replay: refill the inputs in place between replays.  `stream` must be a
 * created stream, not the null stream (which cannot be captured). */
int stixels_batch_capture(stixels_batch *b, const stixels_job *jobs, int32_t n, void *stream);
int stixels_batch_replay(stixels_batch *b, void *stream);

/* Cap on the persistent workgroups of later calls (0 = as many as the
 * device keeps resident and the batch's scratch allows); used by the
 * autotuner.  Takes effect at the next compute or capture. */
int stixels_batch_set_workgroups(stixels_batch *b, int32_t workgroups);

/* Wavefronts per column of later calls (as in stixels_set_waves: 1, 2 or
 * 4, capped by the batch's row slots; 0 = 1); used by the autotuner.
 * Results do not depend on it.  Takes effect at the next compute or
 * capture. */
int stixels_batch_set_waves(stixels_batch *b, int32_t waves);

/* Waves per column of the last compute or capture (0 before the first). */
int stixels_batch_waves(const stixels_batch *b);

/* One-call form of the batch API: segment n frames (any cameras, sizes and
 * stixel widths) in one persistent launch on `stream`, as
 * stixels_batch_compute, through a batch object owned by the first job's
 * handle.  That object is created on the first call and grown (after a
 * device synchronisation) when a call needs more jobs, columns, rows or
 * disparities than every earlier one; other calls allocate nothing.  Calls
 * whose first job names the same handle must not overlap, like
 * stixels_compute on that handle.  Errors are reported on the first job's
 * handle (stixels_last_error). */
int stixels_compute_batch(const stixels_job *jobs, int32_t n, void *stream);

/* Columns per wave64 of later calls: 1, or 2 (two columns of one frame
 * share a wave, one per 32-lane half, so that the recurrence's per-step work
 * serves both), which applies where h <= 512 and d_range <= 128 and with
 * one wave per column; 0 = 1.  Results do not depend on it.  Used by the
 * autotuner; takes effect at the next compute or capture. */
int stixels_batch_set_columns(stixels_batch *b, int32_t columns);

/* Columns per wave of the last compute or capture (0 before the first). */
int stixels_batch_columns(const stixels_batch *b);

/* Device bytes the batch object holds (descriptors, task lists and the
 * per-workgroup scratch slots). */
int stixels_batch_device_bytes(const stixels_batch *b, size_t *bytes);

/* Workgroups of the persistent launch last used, and the number of
 * tasks (frame columns) of the last call. */
int stixels_batch_info(const stixels_batch *b, int32_t *workgroups, int32_t *tasks);
const char *stixels_batch_last_error(const stixels_batch *b);

/* Profiling only.  Shader-clock cycles that wave 0 of the persistent
 * kernel's workgroups spent in each phase of the column tasks of this
 * batch's launches (Sec. 4.1 reduction, the four small prefix scans and the
 * object prefix table of Sec. 4.2, the recurrence of Sec. 4.3, the
 * backtracking of Sec. 4.4), then the number of tasks and the workgroups'
 * summed lifetimes: 7 values into host_dst[0..n) (zeros past 7).
 * Synchronises the device; reset != 0 clears the sums.  Only a library
 * built with STX_PHASE_TIMING counts (python -m paper_1610_04124_amd.build
 * --phase-timing, which writes libstixels_phases.so); the regular library
 * returns STIXELS_E_INVALID_ARG. */
int stixels_batch_phase_cycles(stixels_batch *b, uint64_t *host_dst, int32_t n, int32_t reset);

/* ------------------------------------------------------------------ debug
 * Host copies of the handle's offline tables (Sec. 3.4), for parity tests.
 * Here and below d_range counts disparity bins (max_disparity <<
 * subpixel_log2).  which = STIXELS_TABLE_*; bytes must equal the table's size:
 *   SKY    float[d_range]                  cost of sky per pixel disparity
 *   GROUND float[max_height][d_range]      ground cost per top-down image row
 *   OBJECT float[d_range][d_range]         [f][d]: object of mean f, pixel disparity d
 *   FG_HI  int32[max_height]               diving threshold per top-down row
 *   FG_LO  int32[max_height]               gravity threshold per top-down row */
enum { STIXELS_TABLE_SKY = 0, STIXELS_TABLE_GROUND = 1, STIXELS_TABLE_OBJECT = 2,
       STIXELS_TABLE_FG_HI = 3, STIXELS_TABLE_FG_LO = 4 };
int stixels_debug_table(const stixels_handle *h, int32_t which, void *host_dst, size_t bytes);

/* All five tables above in one host buffer, in the order SKY, GROUND,
 * OBJECT, FG_HI, FG_LO, each laid out as for stixels_debug_table; bytes must
 * equal the sum of their sizes. */
int stixels_debug_tables(const stixels_handle *h, void *host_dst, size_t bytes);

/* The ground table and thresholds of a frame of this height under `pose`,
 * built on the device as stixels_compute_pose builds them (synchronises
 * `stream`): host_dst receives GROUND float[height][d_range] by top-down
 * row, then FG_HI int32[height] and FG_LO int32[height]; bytes must equal
 * height * (4 * d_range + 8).  Uses the handle's pose area (not with
 * STIXELS_FLAG_BATCH_ONLY). */
int stixels_debug_pose_tables(stixels_handle *h, const stixels_pose *pose, int32_t height,
                              void *host_dst, size_t bytes, void *stream);

/* The same tables built on the host from `params` alone, without a handle or
 * a device (validation and range checks as in stixels_create; the error
 * text is then available from stixels_last_error(NULL)). */
int stixels_host_table(const stixels_params *params, int32_t which, void *host_dst, size_t bytes);

/* Host copies of the intermediates of the last stixels_compute on this
 * handle, which must have taken the staged path (synchronises `stream`
 * first).  With ncols columns of height h:
 *   REDUCED  int16[ncols][h]               reduced bottom-up disparities, -1 invalid
 *   PREFIX   float[4][ncols][h+1]          ground, sky, 2*sum(q)+count, 2*count prefixes
 *   RANGE    int32[ncols][2]               smallest / largest valid q of each column
 *   OBJECT_PREFIX float[ncols][d_range][h+1] object prefix table, row f - fmin of
 *                                          each column (rows past fmax unused) */
enum { STIXELS_STAGE_REDUCED = 0, STIXELS_STAGE_PREFIX = 1, STIXELS_STAGE_RANGE = 2,
       STIXELS_STAGE_OBJECT_PREFIX = 3 };
int stixels_debug_stage(const stixels_handle *h, int32_t which, void *host_dst, size_t bytes,
                        void *stream);

/* One frame through the staged path of stixels_compute with HIP events on
 * `stream` between its three kernels; synchronises and writes the
 * milliseconds of the reduction (Sec. 4.1), the prefix tables (Sec. 4.2) and
 * the recurrence with backtracking (Sec. 4.3-4.4) to host_ms[0..2].  For
 * measurements; the results equal those of stixels_compute. */
int stixels_debug_stage_times(stixels_handle *h, const float *d_disparity, int32_t width,
                              int32_t height, void *stream, const stixels_output *out,
                              float *host_ms);

/* Exhaustive device check of the rounded object mean used by the recurrence:
 * for every count n in 1..max_height and every sum S in 0..n*(d_range-1),
 * compares the kernel's floor((2S+n)/(2n)) against integer division and
 * writes the number of mismatches to *host_mismatches.  Synchronous. */
int stixels_selftest_mean(int32_t d_range, int32_t max_height, int64_t *host_mismatches);

/* ------------------------------------------------------------------ stereo
 * Semi-global matching ahead of the stixel path.  The paper takes its
 * disparity maps from a GPU semi-global matching with census costs (Sec. 1,
 * Sec. 5) and leaves that stage out of its timings; this stage produces the
 * same kind of map on the device from a rectified stereo pair:
 *   census   9 x 7 window; bit i of a pixel's 62-bit word is 1 iff the i-th
 *            neighbour (row-major, centre skipped) lies inside the image and
 *            is darker than the centre
 *   cost     C(p, d) = Hamming distance of the left word at (y, x) and the
 *            right word at (y, x - d); 62 where x - d < 0
 *   paths    for the four axis directions r: L_r(p, d) = C(p, d) +
 *            min(L_r(p-r, d), L_r(p-r, d -+ 1) + p1, M + p2) - M with
 *            M = min_k L_r(p-r, k); L_r = C at a path's first pixel
 *   select   d_L = the smallest d minimising the summed cost S(p, d);
 *            d_R(y, x) = the smallest d minimising S((y, x + d), d)
 *   check    the output is d_L where x - d_L >= 0 and
 *            |d_L - d_R(y, x - d_L)| <= 1, else -1 (invalid)
 * All arithmetic is integer. */
typedef struct stixels_sgm stixels_sgm;

typedef struct {
    int32_t max_width, max_height;  /* largest frame; max_width <= 8192 (LDS of a row) */
    int32_t max_disparity;          /* disparities 0..max_disparity-1: a multiple of 4 in 4..256 */
    int32_t p1, p2;                 /* path penalties, 0 <= p1 <= p2 <= 1000 */
    int32_t paths;                  /* 4 */
    int32_t max_frames;             /* frames per stixels_sgm_compute call */
} stixels_sgm_params;

/* Validate, and allocate the workspace: both views' census words and the
 * summed costs, uint16 [max_frames][max_height][max_width][max_disparity]
 * (device bytes: stixels_sgm_device_bytes).  STIXELS_E_INVALID_ARG with the
 * reason in stixels_sgm_last_error(NULL), or STIXELS_E_NOMEM. */
int stixels_sgm_create(const stixels_sgm_params *params, stixels_sgm **out);
int stixels_sgm_destroy(stixels_sgm *m);
const char *stixels_sgm_last_error(const stixels_sgm *m);
int stixels_sgm_device_bytes(const stixels_sgm *m, size_t *bytes);

/* Disparity of `frames` stereo pairs stored back to back: d_left and
 * d_right device uint8 [frames][height][width] (row-major, row 0 at the
 * top), d_disparity device float32 [frames][height][width], caller-owned.
 * Asynchronous on `stream`; allocates nothing; calls on one handle must not
 * overlap (they share its workspace).  STIXELS_E_INVALID_ARG for null
 * pointers, sizes beyond the handle's or frames outside 1..max_frames. */
int stixels_sgm_compute(stixels_sgm *m, const uint8_t *d_left, const uint8_t *d_right,
                        int32_t width, int32_t height, int32_t frames, void *stream,
                        float *d_disparity);

/* Host copy of an intermediate of frame 0 of the last stixels_sgm_compute
 * (synchronises the device): which 0 = left census words, 1 = right census
 * words (uint64 [height][width]), 2 = the cost volume as the last pass finds
 * it (uint16 [height][width][max_disparity]): the sum of the top-to-bottom,
 * bottom-to-top and right-to-left path terms; the left-to-right pass, which
 * selects, adds its own term in registers and does not write it back. */
int stixels_sgm_debug(const stixels_sgm *m, int32_t which, void *host_dst, size_t bytes);

/* A stereo pair in, stixels out: stixels_sgm_compute of one frame into
 * d_disparity (caller-owned device float32 [height][width], which keeps the
 * map), then stixels_compute on it, both on `stream`.  The two handles must
 * share max_disparity (whole-pixel bins). */
int stixels_compute_stereo(stixels_handle *h, stixels_sgm *m, const uint8_t *d_left,
                           const uint8_t *d_right, int32_t width, int32_t height, void *stream,
                           float *d_disparity, const stixels_output *out);

#ifdef __cplusplus
}
#endif
#endif /* STIXELS_H */
