// batch.hip -- many frames in one persistent fused launch: job validation,
// the decreasing-height task list, descriptor staging, launches and HIP graph
// capture.  The kernel itself is in batch_kernel.h.
#include <algorithm>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "job_desc.h"
#include "kernel_table.h"
#include "launch.h"
#include "stixels.h"

using namespace stx;

namespace stx::persist {

// Resets the task counter before a launch (a kernel node, not a memset, so
// that a captured graph replays it correctly).
__global__ void reset_counter_kernel(unsigned int* c) { *c = 0u; }

hipError_t launch_pair_batch(int slots, int nch, int grid, hipStream_t st, const JobDesc* jobs,
                             const int2* tasks, int ntasks, unsigned int* counter, float* scratch,
                             long long stride, int hmax) {
    const void* f = batch_pair_kernel_ptr(slots, nch);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    void* args[] = {&jobs, &tasks, &ntasks, &counter, &scratch, &stride, &hmax};
    return hipLaunchKernel(f, dim3(grid), dim3(64), args, 0, st);
}

hipError_t launch_batch(int slots, int nch, int waves, bool links, int grid, hipStream_t st,
                        const JobDesc* jobs, const int2* tasks, int ntasks, unsigned int* counter,
                        float* scratch, long long stride, int hmax) {
    const void* f = links ? batch_links_kernel_ptr(slots, nch) : batch_kernel_ptr(slots, nch, waves);
    if (!f) return hipErrorInvalidValue;
    // stagger the XCDs' starts only where the tasks fill two rounds or more
    // of the resident workgroups (a shorter launch would only be delayed)
    unsigned int stagger = (ntasks >= 2 * grid) ? kXcdStaggerCycles : 0u;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    void* args[] = {&jobs, &tasks, &ntasks, &counter, &scratch, &stride, &hmax, &stagger};
    return hipLaunchKernel(f, dim3(grid), dim3(64 * waves), args, 0, st);
}

}  // namespace stx::persist

using namespace stx::persist;

struct stixels_batch {
    stixels_batch_config cfg{};
    int num_cu = 0;
    // descriptors of the eager path and of the captured graph
    JobDesc* d_jobs = nullptr;
    int2* d_tasks = nullptr;
    unsigned int* d_counter = nullptr;
    JobDesc* d_jobs_g = nullptr;
    int2* d_tasks_g = nullptr;
    unsigned int* d_counter_g = nullptr;
    float* d_scratch = nullptr;
    size_t scratch_floats = 0;
    JobDesc* h_jobs = nullptr;   // pinned staging
    int2* h_tasks = nullptr;
    // frames with their own pose (STIXELS_BATCH_POSES): one ground table
    // area per job slot, and the table builds of the eager path and the graph
    char* d_pose_area = nullptr;
    size_t pose_area_bytes = 0;  // per job slot
    PoseItem* d_pose_items = nullptr;
    PoseItem* d_pose_items_g = nullptr;
    PoseItem* h_pose_items = nullptr;
    int npose = 0, pose_hmax = 0;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int waves = 1;          // requested waves per column
    int columns = 1;        // requested columns per wave (2: the pair kernel where it exists)
    int last_columns = 0;
    int last_grid = 0, last_tasks = 0, last_waves = 0;
    bool links = false;     // the staged jobs need the recurrence with stored links
    unsigned long long* d_phase = nullptr;   // phase cycles (STX_PHASE_TIMING builds)
    std::string err;
};

namespace {

int bfail(stixels_batch* b, int code, const std::string& m) {
    if (b) b->err = m;
    return code;
}

// Waves per column for a launch of this slot count: the request, capped so
// that every wave owns at least one 64-row slot.
int batch_waves_for(const stixels_batch* b, int slots) {
    const int cap = slots >= 4 ? 4 : (slots >= 2 ? 2 : 1);
    return std::min(std::max(b->waves, 1), cap);
}

int occupancy_grid(stixels_batch* b, int slots, int nch, int waves, int* grid,
                   bool links = false) {
    int per_cu = 0;
    const void* f = links ? batch_links_kernel_ptr(slots, nch) : batch_kernel_ptr(slots, nch, waves);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 64 * waves, 0) != hipSuccess ||
        per_cu < 1)
        return bfail(b, STIXELS_E_HIP, "occupancy query failed");
    *grid = per_cu * b->num_cu;
    return STIXELS_OK;
}

// Validate the jobs and fill the pinned staging buffers: descriptors and the
// task list in decreasing-height order.
int stage(stixels_batch* b, const stixels_job* jobs, int32_t n, int* slots, int* nch,
          int* ntasks, long long* stride, int* hmax_out, bool want_pairs, bool* pairs_out) {
    if (!jobs || n < 1 || n > b->cfg.max_jobs)
        return bfail(b, STIXELS_E_INVALID_ARG, "job count outside [1, max_jobs]");
    int hmax = 0, dmax = 0;
    long long total = 0;
    for (int i = 0; i < n; ++i) {
        const stixels_job& j = jobs[i];
        const stixels_handle* h = j.handle;
        if (!h || !j.d_disparity || !j.out.counts || !j.out.records || !j.out.total_cost ||
            !j.out.overflow)
            return bfail(b, STIXELS_E_INVALID_ARG, "null handle, input or output in job " +
                                                       std::to_string(i));
        if (j.width < h->s || j.width > h->Wmax || j.height < 1 || j.height > h->Hmax ||
            j.height > b->cfg.max_height || h->D > b->cfg.max_disparity || j.out.capacity < 1)
            return bfail(b, STIXELS_E_INVALID_ARG, "job " + std::to_string(i) +
                                                       " outside its handle's or the batch's limits");
        hmax = std::max(hmax, (int)j.height);
        dmax = std::max(dmax, h->D);
        total += j.width / h->s;
    }
    if (total > b->cfg.max_tasks)
        return bfail(b, STIXELS_E_INVALID_ARG, "more frame columns than max_tasks");
    if (b->staged_pending) {
        if (hipEventSynchronize(b->staged) != hipSuccess)
            return bfail(b, STIXELS_E_HIP, "waiting for the previous upload failed");
        b->staged_pending = false;
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return jobs[a].height > jobs[c].height; });
    int t = 0;
    b->npose = 0;
    b->pose_hmax = 0;
    b->links = false;
    for (int i = 0; i < n; ++i) {
        const stixels_job& j = jobs[i];
        b->h_jobs[i] = make_job_desc(j.handle, j.d_disparity, j.width, j.height, j.out);
        b->h_jobs[i].phase = b->d_phase;
        b->links = b->links || !j.handle->prior.exact;
        if (!j.use_pose) continue;
        if (!b->d_pose_area)
            return bfail(b, STIXELS_E_INVALID_ARG, "job " + std::to_string(i) +
                                                       " has a pose: create the batch with STIXELS_BATCH_POSES");
        if (!j.handle->pose_in_range)
            return bfail(b, STIXELS_E_RANGE, "job " + std::to_string(i) +
                                                 ": its handle's cost range leaves no room for poses");
        char* area = b->d_pose_area + (size_t)i * b->pose_area_bytes;
        float* G = reinterpret_cast<float*>(area);
        int32_t* hi = reinterpret_cast<int32_t*>(
            area + (size_t)b->cfg.max_height * b->cfg.max_disparity * sizeof(float));
        int32_t* lo = hi + b->cfg.max_height;
        const char* why = "";
        const int rc = make_pose_item(j.handle->p, j.handle->D, j.pose, j.height, G, hi, lo,
                                      &b->h_pose_items[b->npose], &why);
        if (rc != STIXELS_OK) return bfail(b, rc, "job " + std::to_string(i) + ": " + why);
        ++b->npose;
        b->pose_hmax = std::max(b->pose_hmax, (int)j.height);
        b->h_jobs[i].ground = G;
        b->h_jobs[i].fg_hi = hi;
        b->h_jobs[i].fg_lo = lo;
        b->h_jobs[i].vtop = ground_top(j.pose.horizon_row, j.height);
    }
    // two columns per wave only where that kernel exists (h <= 512,
    // d_range <= 128); a task is then a (frame, even column) pair
    const bool pairs = want_pairs && !b->links && kernel_slots(hmax) <= 8 &&
                       kernel_chunks(dmax) == 2;
    for (int oi = 0; oi < n; ++oi) {
        const int i = order[oi];
        const int nc = b->h_jobs[i].ncols;
        for (int c = 0; c < nc; c += pairs ? 2 : 1) b->h_tasks[t++] = make_int2(i, c);
    }
    *slots = kernel_slots(hmax);
    *nch = kernel_chunks(dmax);
    *ntasks = t;
    *stride = pairs ? 2LL * (8 + dmax) * (hmax + 1) : slot_floats(hmax, dmax);
    *pairs_out = pairs;
    *hmax_out = hmax;
    return STIXELS_OK;
}

int pair_occupancy_grid(stixels_batch* b, int slots, int nch, int* grid) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_pair_kernel_ptr(slots, nch), 64,
                                                     0) != hipSuccess ||
        per_cu < 1)
        return bfail(b, STIXELS_E_HIP, "occupancy query failed");
    *grid = per_cu * b->num_cu;
    return STIXELS_OK;
}

int choose_grid(stixels_batch* b, int slots, int nch, int waves, bool pairs, long long stride,
                int ntasks, int* grid) {
    int g = 0;
    int rc = pairs ? pair_occupancy_grid(b, slots, nch, &g)
                   : occupancy_grid(b, slots, nch, waves, &g, b->links);
    if (rc != STIXELS_OK) return rc;
    if (b->cfg.workgroups > 0) g = std::min(g, (int)b->cfg.workgroups);
    const long long by_scratch = (long long)(b->scratch_floats / (size_t)stride);
    g = (int)std::min<long long>(g, by_scratch);
    g = std::min(g, ntasks);
    if (g < 1) return bfail(b, STIXELS_E_INVALID_ARG, "batch scratch too small for these jobs");
    *grid = g;
    return STIXELS_OK;
}

int upload(stixels_batch* b, JobDesc* dj, int2* dt, PoseItem* dp, int n, int ntasks,
           hipStream_t st) {
    if (hipMemcpyAsync(dj, b->h_jobs, sizeof(JobDesc) * n, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(dt, b->h_tasks, sizeof(int2) * ntasks, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        (b->npose > 0 && hipMemcpyAsync(dp, b->h_pose_items, sizeof(PoseItem) * b->npose,
                                        hipMemcpyHostToDevice, st) != hipSuccess))
        return bfail(b, STIXELS_E_HIP, "descriptor upload failed");
    if (hipEventRecord(b->staged, st) != hipSuccess)
        return bfail(b, STIXELS_E_HIP, "event record failed");
    b->staged_pending = true;
    return STIXELS_OK;
}

void destroy_graph(stixels_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

}  // namespace

extern "C" {

int stixels_batch_create(const stixels_batch_config* cfg, stixels_batch** out) {
    if (!cfg || !out) return STIXELS_E_INVALID_ARG;
    *out = nullptr;
    if (cfg->max_jobs < 1 || cfg->max_tasks < 1 || cfg->max_height < 1 ||
        cfg->max_height > kMaxHeight || cfg->max_disparity < 2 ||
        cfg->max_disparity > kMaxDisparity || cfg->workgroups < 0 ||
        (cfg->flags & ~STIXELS_BATCH_POSES))
        return STIXELS_E_INVALID_ARG;
    stixels_batch* b = new (std::nothrow) stixels_batch;
    if (!b) return STIXELS_E_NOMEM;
    b->cfg = *cfg;
    int dev = 0;
    int rc = STIXELS_OK;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess)
        rc = STIXELS_E_HIP;
    int grid = 0;
    const int slots = kernel_slots(cfg->max_height);
    // one-wave workgroups are the most that can be resident: the scratch
    // slots cover them, and so every later choice of waves per column
    if (rc == STIXELS_OK) rc = occupancy_grid(b, slots, kernel_chunks(cfg->max_disparity), 1, &grid);
    if (rc == STIXELS_OK && cfg->workgroups > 0) grid = std::min(grid, (int)cfg->workgroups);
    if (rc == STIXELS_OK) {
        b->scratch_floats = (size_t)grid *
                            (size_t)slot_floats(cfg->max_height, cfg->max_disparity);
        // the two-column kernel, where it exists, needs two (8 + D)(h+1)
        // column slots per resident workgroup
        int pgrid = 0;
        if (slots <= 8 && kernel_chunks(cfg->max_disparity) == 2 &&
            pair_occupancy_grid(b, slots, 2, &pgrid) == STIXELS_OK)
            b->scratch_floats = std::max(b->scratch_floats,
                                         (size_t)pgrid * 2 * (size_t)(8 + cfg->max_disparity) *
                                             (size_t)(cfg->max_height + 1));
        const bool ok =
            hipMalloc(reinterpret_cast<void**>(&b->d_jobs), sizeof(JobDesc) * cfg->max_jobs) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&b->d_tasks), sizeof(int2) * cfg->max_tasks) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&b->d_counter), sizeof(unsigned int)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&b->d_jobs_g), sizeof(JobDesc) * cfg->max_jobs) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&b->d_tasks_g), sizeof(int2) * cfg->max_tasks) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&b->d_counter_g), sizeof(unsigned int)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&b->d_scratch),
                      sizeof(float) * b->scratch_floats + kTableGuardBytes) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&b->h_jobs), sizeof(JobDesc) * cfg->max_jobs, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&b->h_tasks), sizeof(int2) * cfg->max_tasks, hipHostMallocDefault) == hipSuccess &&
            hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) == hipSuccess;
        if (!ok) rc = STIXELS_E_NOMEM;
    }
#ifdef STX_PHASE_TIMING
    if (rc == STIXELS_OK &&
        (hipMalloc(reinterpret_cast<void**>(&b->d_phase), sizeof(unsigned long long) * kPhaseSlots) !=
             hipSuccess ||
         hipMemset(b->d_phase, 0, sizeof(unsigned long long) * kPhaseSlots) != hipSuccess))
        rc = STIXELS_E_NOMEM;
#endif
    if (rc == STIXELS_OK && (cfg->flags & STIXELS_BATCH_POSES)) {
        b->pose_area_bytes = (size_t)cfg->max_height *
                             ((size_t)cfg->max_disparity * sizeof(float) + 2 * sizeof(int32_t));
        const bool ok =
            hipMalloc(reinterpret_cast<void**>(&b->d_pose_area),
                      b->pose_area_bytes * (size_t)cfg->max_jobs) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&b->d_pose_items), sizeof(PoseItem) * cfg->max_jobs) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&b->d_pose_items_g), sizeof(PoseItem) * cfg->max_jobs) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&b->h_pose_items), sizeof(PoseItem) * cfg->max_jobs,
                          hipHostMallocDefault) == hipSuccess;
        if (!ok) rc = STIXELS_E_NOMEM;
    }
    if (rc != STIXELS_OK) {
        stixels_batch_destroy(b);
        return rc;
    }
    *out = b;
    return STIXELS_OK;
}

int stixels_batch_destroy(stixels_batch* b) {
    if (!b) return STIXELS_OK;
    if (b->staged_pending) (void)hipEventSynchronize(b->staged);
    destroy_graph(b);
    (void)hipFree(b->d_jobs);
    (void)hipFree(b->d_tasks);
    (void)hipFree(b->d_counter);
    (void)hipFree(b->d_jobs_g);
    (void)hipFree(b->d_tasks_g);
    (void)hipFree(b->d_counter_g);
    (void)hipFree(b->d_phase);
    (void)hipFree(b->d_scratch);
    (void)hipFree(b->d_pose_area);
    (void)hipFree(b->d_pose_items);
    (void)hipFree(b->d_pose_items_g);
    if (b->h_pose_items) (void)hipHostFree(b->h_pose_items);
    if (b->h_jobs) (void)hipHostFree(b->h_jobs);
    if (b->h_tasks) (void)hipHostFree(b->h_tasks);
    if (b->staged) (void)hipEventDestroy(b->staged);
    delete b;
    return STIXELS_OK;
}

int stixels_batch_compute(stixels_batch* b, const stixels_job* jobs, int32_t n, void* stream) {
    if (!b) return STIXELS_E_INVALID_ARG;
    int slots = 0, nch = 0, ntasks = 0, grid = 0, hmax = 0;
    long long stride = 0;
    bool pairs = false;
    int rc = stage(b, jobs, n, &slots, &nch, &ntasks, &stride, &hmax, b->columns == 2, &pairs);
    const int waves = (pairs || b->links) ? 1 : batch_waves_for(b, slots);
    if (rc == STIXELS_OK) rc = choose_grid(b, slots, nch, waves, pairs, stride, ntasks, &grid);
    if (rc != STIXELS_OK) return rc;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    rc = upload(b, b->d_jobs, b->d_tasks, b->d_pose_items, n, ntasks, st);
    if (rc != STIXELS_OK) return rc;
    hipError_t e = launch_pose_tables(b->d_pose_items, b->npose, b->pose_hmax, st);
    if (e == hipSuccess)
        e = pairs ? launch_pair_batch(slots, nch, grid, st, b->d_jobs, b->d_tasks, ntasks,
                                  b->d_counter, b->d_scratch, stride, hmax)
              : launch_batch(slots, nch, waves, b->links, grid, st, b->d_jobs, b->d_tasks, ntasks,
                             b->d_counter, b->d_scratch, stride, hmax);
    if (e != hipSuccess)
        return bfail(b, STIXELS_E_HIP, std::string("batch launch failed: ") + hipGetErrorString(e));
    b->last_grid = grid;
    b->last_tasks = ntasks;
    b->last_waves = waves;
    b->last_columns = pairs ? 2 : 1;
    return STIXELS_OK;
}

int stixels_batch_capture(stixels_batch* b, const stixels_job* jobs, int32_t n, void* stream) {
    if (!b) return STIXELS_E_INVALID_ARG;
    if (!stream)
        return bfail(b, STIXELS_E_INVALID_ARG, "the null stream cannot be captured; pass a created stream");
    int slots = 0, nch = 0, ntasks = 0, grid = 0, hmax = 0;
    long long stride = 0;
    bool pairs = false;
    int rc = stage(b, jobs, n, &slots, &nch, &ntasks, &stride, &hmax, b->columns == 2, &pairs);
    const int waves = (pairs || b->links) ? 1 : batch_waves_for(b, slots);
    if (rc == STIXELS_OK) rc = choose_grid(b, slots, nch, waves, pairs, stride, ntasks, &grid);
    if (rc != STIXELS_OK) return rc;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    // the graph reads its own descriptor copy, uploaded once here
    rc = upload(b, b->d_jobs_g, b->d_tasks_g, b->d_pose_items_g, n, ntasks, st);
    if (rc != STIXELS_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess)
        return bfail(b, STIXELS_E_HIP, "synchronising the capture stream failed");
    b->staged_pending = false;
    destroy_graph(b);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bfail(b, STIXELS_E_HIP, "hipStreamBeginCapture failed");
    hipError_t e = launch_pose_tables(b->d_pose_items_g, b->npose, b->pose_hmax, st);
    if (e == hipSuccess)
        e = pairs ? launch_pair_batch(slots, nch, grid, st, b->d_jobs_g, b->d_tasks_g, ntasks,
                                  b->d_counter_g, b->d_scratch, stride, hmax)
              : launch_batch(slots, nch, waves, b->links, grid, st, b->d_jobs_g, b->d_tasks_g, ntasks,
                             b->d_counter_g, b->d_scratch, stride, hmax);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(b, STIXELS_E_HIP, "capturing the batch launch failed");
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        destroy_graph(b);
        return bfail(b, STIXELS_E_HIP, "hipGraphInstantiate failed");
    }
    b->last_grid = grid;
    b->last_tasks = ntasks;
    b->last_waves = waves;
    b->last_columns = pairs ? 2 : 1;
    return STIXELS_OK;
}

int stixels_batch_replay(stixels_batch* b, void* stream) {
    if (!b) return STIXELS_E_INVALID_ARG;
    if (!b->exec) return bfail(b, STIXELS_E_INVALID_ARG, "no captured batch to replay");
    if (hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)) != hipSuccess)
        return bfail(b, STIXELS_E_HIP, "hipGraphLaunch failed");
    return STIXELS_OK;
}

int stixels_batch_set_workgroups(stixels_batch* b, int32_t workgroups) {
    if (!b || workgroups < 0) return STIXELS_E_INVALID_ARG;
    b->cfg.workgroups = workgroups;
    return STIXELS_OK;
}

int stixels_batch_set_waves(stixels_batch* b, int32_t waves) {
    if (!b || (waves != 0 && waves != 1 && waves != 2 && waves != 4))
        return bfail(b, STIXELS_E_INVALID_ARG, "waves per column must be 0, 1, 2 or 4");
    b->waves = waves == 0 ? 1 : waves;
    return STIXELS_OK;
}

int stixels_batch_waves(const stixels_batch* b) { return b ? b->last_waves : 0; }

int stixels_batch_set_columns(stixels_batch* b, int32_t columns) {
    if (!b || columns < 0 || columns > 2)
        return bfail(b, STIXELS_E_INVALID_ARG, "columns per wave must be 0, 1 or 2");
    b->columns = columns == 0 ? 1 : columns;
    return STIXELS_OK;
}

int stixels_batch_columns(const stixels_batch* b) { return b ? b->last_columns : 0; }

int stixels_batch_device_bytes(const stixels_batch* b, size_t* bytes) {
    if (!b || !bytes) return STIXELS_E_INVALID_ARG;
    *bytes = 2 * (sizeof(JobDesc) * (size_t)b->cfg.max_jobs +
                  sizeof(int2) * (size_t)b->cfg.max_tasks + sizeof(unsigned int)) +
             sizeof(float) * b->scratch_floats + kTableGuardBytes;
    if (b->d_pose_area)
        *bytes += (b->pose_area_bytes + 2 * sizeof(PoseItem)) * (size_t)b->cfg.max_jobs;
    return STIXELS_OK;
}

int stixels_batch_info(const stixels_batch* b, int32_t* workgroups, int32_t* tasks) {
    if (!b) return STIXELS_E_INVALID_ARG;
    if (workgroups) *workgroups = b->last_grid;
    if (tasks) *tasks = b->last_tasks;
    return STIXELS_OK;
}

int stixels_compute_batch(const stixels_job* jobs, int32_t n, void* stream) {
    if (!jobs || n < 1 || !jobs[0].handle) return STIXELS_E_INVALID_ARG;
    stixels_handle* owner = jobs[0].handle;
    int hmax = 1, dmax = 2;
    long long tasks = 0;
    bool poses = false;
    for (int i = 0; i < n; ++i) {
        poses = poses || jobs[i].use_pose;
        const stixels_handle* h = jobs[i].handle;
        if (!h || jobs[i].width < h->s || jobs[i].height < 1 || jobs[i].height > h->Hmax) {
            owner->err = "job " + std::to_string(i) + ": null handle or size outside its limits";
            return STIXELS_E_INVALID_ARG;
        }
        hmax = std::max(hmax, (int)jobs[i].height);
        dmax = std::max(dmax, h->D);
        tasks += jobs[i].width / h->s;
    }
    if (tasks > INT_MAX) {
        owner->err = "too many frame columns in one call";
        return STIXELS_E_INVALID_ARG;
    }
    stixels_batch* b = owner->auto_batch;
    if (!b || b->cfg.max_jobs < n || b->cfg.max_tasks < tasks || b->cfg.max_height < hmax ||
        b->cfg.max_disparity < dmax || (poses && !(b->cfg.flags & STIXELS_BATCH_POSES))) {
        // grow: the new limits cover this call and every earlier one
        stixels_batch_config c{};
        c.max_jobs = b ? std::max((int)n, (int)b->cfg.max_jobs) : n;
        c.max_tasks = (int)(b ? std::max<long long>(tasks, b->cfg.max_tasks) : tasks);
        c.max_height = b ? std::max(hmax, (int)b->cfg.max_height) : hmax;
        c.max_disparity = b ? std::max(dmax, (int)b->cfg.max_disparity) : dmax;
        c.flags = (poses || (b && (b->cfg.flags & STIXELS_BATCH_POSES))) ? STIXELS_BATCH_POSES : 0;
        if (b) {
            // earlier launches may still read the old batch's buffers
            if (hipDeviceSynchronize() != hipSuccess) {
                owner->err = "synchronising before growing the batch failed";
                return STIXELS_E_HIP;
            }
            stixels_batch_destroy(b);
            owner->auto_batch = nullptr;
        }
        const int rc = stixels_batch_create(&c, &b);
        if (rc != STIXELS_OK) {
            owner->err = "creating the batch of stixels_compute_batch failed";
            return rc;
        }
        owner->auto_batch = b;
    }
    const int rc = stixels_batch_compute(b, jobs, n, stream);
    if (rc != STIXELS_OK) owner->err = b->err;
    return rc;
}

int stixels_batch_phase_cycles(stixels_batch* b, uint64_t* host_dst, int32_t n, int32_t reset) {
    if (!b || !host_dst || n < 1) return STIXELS_E_INVALID_ARG;
#ifdef STX_PHASE_TIMING
    unsigned long long h[kPhaseSlots] = {};
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(h, b->d_phase, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess ||
        (reset && hipMemset(b->d_phase, 0, sizeof(h)) != hipSuccess))
        return bfail(b, STIXELS_E_HIP, "reading the phase cycles failed");
    for (int i = 0; i < n; ++i) host_dst[i] = (i < kPhaseSlots) ? (uint64_t)h[i] : 0u;
    return STIXELS_OK;
#else
    (void)reset;
    return bfail(b, STIXELS_E_INVALID_ARG,
                 "this library was built without phase timing (STX_PHASE_TIMING)");
#endif
}

const char* stixels_batch_last_error(const stixels_batch* b) {
    return b ? b->err.c_str() : "";
}

}  // extern "C"
