// Work ordering of a size bucket between steps.  One workgroup per world
// and one resident workgroup per compute unit means a step ends when the
// slowest compute unit drains its share; the iteration counts of worlds
// persist from step to step (the same contact configurations stay hard), so
// dispatching the worlds in decreasing order of their last iteration count
// is a longest-processing-time-first schedule for the next step.  The order
// only decides which workgroup slot takes a world, never what it computes.
#include "kamx_internal.h"

namespace kamx {

namespace {

constexpr int kSchedThreads = 1024;
constexpr int kSchedBins = 256;

__device__ inline int cost_bin(int iters) {
    int it = iters < 0 ? 0 : (iters > 2047 ? 2047 : iters);
    return it >> 3;
}

// Counting sort of the bucket's worlds by cost bin, most expensive first.
// Positions inside a bin come from LDS atomics, so ties are ordered
// arbitrarily; results do not depend on the order.
__global__ __launch_bounds__(kSchedThreads) void lpt_order_kernel(const int32_t *worlds, int n,
                                                                  const int32_t *iters, int32_t *order) {
    __shared__ int hist[kSchedBins];
    const int tid = threadIdx.x;
    for (int k = tid; k < kSchedBins; k += kSchedThreads) hist[k] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += kSchedThreads) atomicAdd(&hist[cost_bin(iters[worlds[i]])], 1);
    __syncthreads();
    if (tid == 0) {
        int run = 0;  // start of bin k = number of worlds in the bins above k
        for (int k = kSchedBins - 1; k >= 0; --k) {
            int c = hist[k];
            hist[k] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int i = tid; i < n; i += kSchedThreads) {
        int w = worlds[i];
        int pos = atomicAdd(&hist[cost_bin(iters[w])], 1);
        order[pos] = w;
    }
}

// One thread: the step counter that keys the noise of the next step.
__global__ void advance_step_kernel(uint32_t *ctr, uint32_t inc) {
    if (threadIdx.x == 0) ctr[0] = ctr[0] + inc;
}

}  // namespace

hipError_t launch_advance_step(uint32_t *ctr, uint32_t inc, hipStream_t stream) {
    hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, stream, ctr, inc);
    return hipGetLastError();
}

hipError_t launch_lpt_order(const int32_t *worlds, int n, const int32_t *iters, int32_t *order, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(lpt_order_kernel, dim3(1), dim3(kSchedThreads), 0, stream, worlds, n, iters, order);
    return hipGetLastError();
}

}  // namespace kamx
