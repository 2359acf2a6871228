// Device side of the serving loop of the PHIA library for gfx950.
//
// k_argmin_many: the end-of-round read-out of many requests in one launch.
// Workgroup j takes request j's per-replica best energies and finds the
// lowest one, the lowest replica index on ties (the final choice of App. B,
// Table 3, state 5, as the single-problem argmin computes it), and copies
// the request's device error word (0 where it has none).  The requests come
// in the kernel arguments, kArgminJobs per launch, so a round needs no table
// upload; out receives (energy, replica) pairs and then the error words.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phia_internal.h"

namespace phia {

namespace {

constexpr int kArgminJobs = 64;

struct ArgminJobs {
    const int64_t* bestE[kArgminJobs];
    const int32_t* err[kArgminJobs];
    int32_t R[kArgminJobs];
};

__global__ void __launch_bounds__(256) k_argmin_many(ArgminJobs jobs, int64_t* pairs, int32_t* errs)
{
    __shared__ int64_t sE[256];
    __shared__ int64_t sR[256];
    const int j = blockIdx.x;
    const int64_t* bestE = jobs.bestE[j];
    const int32_t R = jobs.R[j];
    int64_t e = INT64_MAX, r = -1;
    for (int i = threadIdx.x; i < R; i += 256) {  // rising index: a tie keeps the first
        const int64_t v = bestE[i];
        if (r < 0 || v < e) {
            e = v;
            r = i;
        }
    }
    sE[threadIdx.x] = e;
    sR[threadIdx.x] = r;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const int64_t e2 = sE[threadIdx.x + w], r2 = sR[threadIdx.x + w];
            const int64_t e1 = sE[threadIdx.x], r1 = sR[threadIdx.x];
            if (r2 >= 0 && (r1 < 0 || e2 < e1 || (e2 == e1 && r2 < r1))) {
                sE[threadIdx.x] = e2;
                sR[threadIdx.x] = r2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pairs[2 * j] = sE[0];
        pairs[2 * j + 1] = sR[0];
        errs[j] = jobs.err[j] ? *jobs.err[j] : 0;
    }
}

}  // namespace

hipError_t launch_argmin_many(const int64_t* const* bestE, const int32_t* R, const int32_t* const* err, int n,
                              int64_t* pairs, int32_t* errs, hipStream_t st)
{
    for (int b = 0; b < n; b += kArgminJobs) {
        const int m = n - b < kArgminJobs ? n - b : kArgminJobs;
        ArgminJobs jobs{};
        for (int j = 0; j < m; ++j) {
            jobs.bestE[j] = bestE[b + j];
            jobs.err[j] = err[b + j];
            jobs.R[j] = R[b + j];
        }
        hipLaunchKernelGGL(k_argmin_many, dim3(static_cast<unsigned>(m)), dim3(256), 0, st, jobs, pairs + 2 * b,
                           errs + b);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace phia
