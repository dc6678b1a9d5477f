// Optimiser step and small bookkeeping kernels: the Adam update of the
// flat parameters (App. B), the device-resident step counters that let a
// captured HIP graph keep counting, and the non-finite count of a device
// array.
#include "kernels.h"

namespace vmc {

// *c += 1 (a device-resident Philox counter or Adam step, after the kernels
// of the call that read it)
__global__ void bump_counter(uint64_t *c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c += 1;
}

// Learning rate at update index k (Table III schedules): the first rate
// before t_switch and the second after it, divided by an inverse-time decay
// that starts at t_decay (tau = 0: none).
__device__ inline double adam_lr(const vmc_adam_cfg &c, int64_t k) {
    double lr = k < c.t_switch ? c.lr0 : c.lr1;
    if (c.tau > 0.0 && k > c.t_decay) lr /= 1.0 + (double)(k - c.t_decay) / c.tau;
    return lr;
}

// Adam (Kingma & Ba): moment updates and the bias-corrected step, FP64
// arithmetic on FP32 storage.  Every thread reads the step count from device
// memory; bump_counter advances it afterwards.
__global__ __launch_bounds__(256) void adam_kernel(int64_t n, float *__restrict__ p, const double *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   const int64_t *t_dev, vmc_adam_cfg c) {
    const int64_t t = *t_dev + 1;
    const double lr = adam_lr(c, t - 1);
    const double bc1 = 1.0 - pow(c.beta1, (double)t), bc2 = 1.0 - pow(c.beta2, (double)t);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double gi = g[i];
        const double mi = c.beta1 * (double)m[i] + (1.0 - c.beta1) * gi;
        const double vi = c.beta2 * (double)v[i] + (1.0 - c.beta2) * gi * gi;
        m[i] = (float)mi;
        v[i] = (float)vi;
        p[i] = (float)((double)p[i] - lr * (mi / bc1) / (sqrt(vi / bc2) + c.eps));
    }
}

// Number of non-finite entries of x, one work-group (a fixed reduction tree).
__global__ __launch_bounds__(1024) void count_nonfinite(const float *__restrict__ x, int64_t n,
                                                        unsigned long long *out) {
    __shared__ unsigned long long part[1024];
    unsigned long long c = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t u = __float_as_uint(x[i]);
        c += ((u & 0x7f800000u) == 0x7f800000u) ? 1ull : 0ull;
    }
    part[threadIdx.x] = c;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

hipError_t launch_bump(uint64_t *counter, hipStream_t st) {
    hipLaunchKernelGGL(bump_counter, dim3(1), dim3(64), 0, st, counter);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float *p, const double *g, float *m, float *v, int64_t *t_dev,
                       const vmc_adam_cfg &c, hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    const int grid = (int)(blocks > 4096 ? 4096 : blocks);
    hipLaunchKernelGGL(adam_kernel, dim3(grid), dim3(256), 0, st, n, p, g, m, v, (const int64_t *)t_dev, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_bump((uint64_t *)t_dev, st);
}

hipError_t launch_count_nonfinite(const float *x, int64_t n, unsigned long long *count, hipStream_t st) {
    hipLaunchKernelGGL(count_nonfinite, dim3(1), dim3(1024), 0, st, x, n, count);
    return hipGetLastError();
}

}  // namespace vmc
