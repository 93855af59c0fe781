// Deterministic sum of per-cell values: one workgroup, every thread adds a
// fixed strided subset in FP64 in index order, then a fixed-shape tree in
// LDS.  The result depends only on the values and their count (no atomics,
// no dependence on scheduling), so repeated evaluations agree bit for bit.
#include "fe_device.h"

namespace fe {
namespace {

constexpr int SUM_THREADS = 1024;

template <typename T>
__global__ __launch_bounds__(SUM_THREADS) void k_sum_cells(const T *vals, int64_t n, double *total)
{
    __shared__ double part[SUM_THREADS];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += SUM_THREADS) s += static_cast<double>(vals[i]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = SUM_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) total[0] = part[0];
}

}  // namespace

int sum_cells(const void *vals, int prec, int64_t n, double *total, hipStream_t st)
{
    if (n < 0) return FE_ERR_INVALID_ARG;
    if (prec == FE_PREC_FP64)
        hipLaunchKernelGGL(k_sum_cells<double>, dim3(1), dim3(SUM_THREADS), 0, st, static_cast<const double *>(vals),
                           n, total);
    else
        hipLaunchKernelGGL(k_sum_cells<float>, dim3(1), dim3(SUM_THREADS), 0, st, static_cast<const float *>(vals),
                           n, total);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
}

}  // namespace fe
