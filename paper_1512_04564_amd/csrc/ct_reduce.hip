// FP64 reductions for the solver trace and the finiteness check (compiled with NaN semantics).
#include "ct_internal.hpp"

namespace ct {

namespace {

// Deterministic FP64 partial sums: one partial per block, then a single-block final pass.
constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 256;

__global__ __launch_bounds__(RED_THREADS) void k_trace_partial(const float *__restrict__ x,
                                                              const float *__restrict__ ref,
                                                              const float *__restrict__ gv,
                                                              const float *__restrict__ h, int nx, int ny, float dx,
                                                              float dy, float radius, double *__restrict__ part)
{
    const size_t n = (size_t)nx * ny;
    double s = 0.0, c = 0.0, bad = 0.0;
    for (size_t p = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; p < n; p += (size_t)RED_BLOCKS * RED_THREADS) {
        const int i = (int)(p / nx), j = (int)(p % nx);
        const float xv = x[p];
        if (!isfinite(xv) || (gv && !isfinite(gv[p])) || (h && !isfinite(h[p]))) bad += 1.0;
        if (ref) {
            const float px = ((float)j - 0.5f * (float)(nx - 1)) * dx;
            const float py = ((float)i - 0.5f * (float)(ny - 1)) * dy;
            if (radius <= 0.f || px * px + py * py <= radius * radius) {
                const double dd = (double)xv - (double)ref[p];
                s += dd * dd;
                c += 1.0;
            }
        }
    }
    __shared__ double sh[3][RED_THREADS];
    sh[0][threadIdx.x] = s;
    sh[1][threadIdx.x] = c;
    sh[2][threadIdx.x] = bad;
    __syncthreads();
    for (int st = RED_THREADS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) part[(size_t)q * RED_BLOCKS + blockIdx.x] = sh[q][0];
}

__global__ __launch_bounds__(RED_BLOCKS) void k_trace_final(const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double sh[3][RED_BLOCKS];
    for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = part[(size_t)q * RED_BLOCKS + threadIdx.x];
    __syncthreads();
    for (int st = RED_BLOCKS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) out[q] = sh[q][0];
}

}  // namespace

hipError_t launch_trace_reduce(const float *x, const float *ref, const float *gv, const float *h, int nx, int ny,
                               float dx, float dy, float radius, double *out, hipStream_t s)
{
    // out must hold 3 doubles followed by 3 * RED_BLOCKS doubles of scratch
    double *part = out + 3;
    hipLaunchKernelGGL(k_trace_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, ref, gv, h, nx, ny, dx, dy,
                       radius, part);
    hipLaunchKernelGGL(k_trace_final, dim3(1), dim3(RED_BLOCKS), 0, s, part, out);
    return hipGetLastError();
}

}  // namespace ct
