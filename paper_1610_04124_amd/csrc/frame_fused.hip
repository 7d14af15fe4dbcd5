// frame_fused.hip -- the per-frame path as one launch of the persistent fused
// kernel (reduction, prefix tables, recurrence and backtracking per column
// in one workgroup, Sec. 4.1-4.4), with the job's descriptor and task list
// written on the device.
#include <algorithm>

#include "job_desc.h"
#include "kernel_table.h"

namespace stx::persist {

namespace {
constexpr size_t kHeaderBytes = 512;

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

__global__ __launch_bounds__(256) void stage_frame_kernel(JobDesc job, JobDesc* dst, int2* tasks,
                                                          int ntasks, unsigned int* counter) {
    if (threadIdx.x == 0) {
        *dst = job;
        *counter = 0u;
    }
    for (int t = threadIdx.x; t < ntasks; t += 256) tasks[t] = make_int2(0, t);
}

size_t frame_fused_bytes(int ncols, int H, int D, int slots) {
    const size_t stride = (size_t)slot_floats(H, D) * sizeof(float);
    return kHeaderBytes + round256(sizeof(int2) * (size_t)ncols) + stride * (size_t)slots +
           kTableGuardBytes;
}

hipError_t launch_frame_fused(const JobDesc& job, void* ws, size_t ws_bytes, int waves, int num_cu,
                              hipStream_t st, int* grid_out) {
    *grid_out = 0;
    const int slots = kernel_slots(job.H), nch = kernel_chunks(job.D);
    const int cap = slots >= 4 ? 4 : (slots >= 2 ? 2 : 1);
    // costs off the grid: the recurrence with stored links, one wave
    const bool links = !job.prior.exact;
    waves = links ? 1 : std::min(std::max(waves, 1), cap);
    const void* f = links ? batch_links_kernel_ptr(slots, nch) : batch_kernel_ptr(slots, nch, waves);
    if (!f || job.ncols < 1) return hipErrorInvalidValue;
    const size_t base = frame_fused_bytes(job.ncols, job.H, job.D, 0);
    if (ws_bytes < base) return hipErrorInvalidValue;
    long long stride = slot_floats(job.H, job.D);
    const long long by_ws = (long long)((ws_bytes - base) / ((size_t)stride * sizeof(float)));
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 64 * waves, 0);
    if (e != hipSuccess) return e;
    long long g = std::min<long long>((long long)per_cu * num_cu, job.ncols);
    g = std::min(g, by_ws);
    if (g < 1) return hipErrorInvalidValue;
    char* p = static_cast<char*>(ws);
    JobDesc* d_job = reinterpret_cast<JobDesc*>(p);
    unsigned int* d_counter = reinterpret_cast<unsigned int*>(p + 256);
    int2* d_tasks = reinterpret_cast<int2*>(p + kHeaderBytes);
    float* scratch = reinterpret_cast<float*>(p + kHeaderBytes +
                                              round256(sizeof(int2) * (size_t)job.ncols));
    int ntasks = job.ncols, hmax = job.H;
    unsigned int stagger = 0u;
    hipLaunchKernelGGL(stage_frame_kernel, dim3(1), dim3(256), 0, st, job, d_job, d_tasks, ntasks,
                       d_counter);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const JobDesc* jobs = d_job;
    const int2* tasks = d_tasks;
    void* args[] = {&jobs, &tasks, &ntasks, &d_counter, &scratch, &stride, &hmax, &stagger};
    e = hipLaunchKernel(f, dim3((unsigned)g), dim3(64 * waves), args, 0, st);
    if (e == hipSuccess) *grid_out = (int)g;
    return e;
}

}  // namespace stx::persist
