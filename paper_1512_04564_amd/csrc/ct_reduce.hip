// FP64 reductions: the solver trace (RMSD to a reference, finiteness) and the PWLS cost
// Psi(x) = 1/2 ||y - A x||_W^2 + R(x). Compiled with NaN semantics. Every reduction is deterministic:
// a fixed grid of block partials, each reduced in a fixed tree, then one block adds the partials in order.
#include "ct_internal.hpp"

namespace ct {

namespace {

constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 256;
constexpr int TRACE_Q = 4;   // FOV sum of squares, FOV count, non-finite count, whole-image sum of squares

template <int Q>
__device__ __forceinline__ void block_reduce_store(double (&v)[Q], double *__restrict__ part)
{
    __shared__ double sh[Q][RED_THREADS];
#pragma unroll
    for (int q = 0; q < Q; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int st = RED_THREADS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
#pragma unroll
            for (int q = 0; q < Q; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < Q; ++q) part[(size_t)q * RED_BLOCKS + blockIdx.x] = sh[q][0];
}

__global__ __launch_bounds__(RED_THREADS) void k_trace_partial(const float *__restrict__ x,
                                                              const float *__restrict__ ref,
                                                              const float *__restrict__ gv,
                                                              const float *__restrict__ h, int nx, int ny, float dx,
                                                              float dy, float radius, double *__restrict__ part)
{
    const size_t n = (size_t)nx * ny;
    double v[TRACE_Q] = {0.0, 0.0, 0.0, 0.0};
    for (size_t p = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; p < n; p += (size_t)RED_BLOCKS * RED_THREADS) {
        const int i = (int)(p / nx), j = (int)(p % nx);
        const float xv = x[p];
        if (!isfinite(xv) || (gv && !isfinite(gv[p])) || (h && !isfinite(h[p]))) v[2] += 1.0;
        if (ref) {
            const double dd = (double)xv - (double)ref[p];
            v[3] += dd * dd;
            const float px = ((float)j - 0.5f * (float)(nx - 1)) * dx;
            const float py = ((float)i - 0.5f * (float)(ny - 1)) * dy;
            if (radius <= 0.f || px * px + py * py <= radius * radius) {
                v[0] += dd * dd;
                v[1] += 1.0;
            }
        }
    }
    block_reduce_store<TRACE_Q>(v, part);
}

// out[q] = sum of the RED_BLOCKS partials of quantity q, in a fixed order
template <int Q>
__global__ __launch_bounds__(RED_BLOCKS) void k_final(const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double sh[Q][RED_BLOCKS];
    for (int q = 0; q < Q; ++q) sh[q][threadIdx.x] = part[(size_t)q * RED_BLOCKS + threadIdx.x];
    __syncthreads();
    for (int st = RED_BLOCKS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int q = 0; q < Q; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < Q; ++q) out[q] = sh[q][0];
}

// Potential phi(t) in FP64 (scaled to t^2 / 2 near 0): 0 hyperbola delta^2 (sqrt(1 + z^2) - 1), written as
// t^2 / (sqrt(1 + z^2) + 1) to avoid the cancellation; 1 Fair delta^2 (|z| - log(1 + |z|)); 2 q-GGMRF with
// p = 2, q = 1.2: t^2 / (2 (1 + |z|^0.8)). z = t / delta.
__device__ __forceinline__ double potential64(int kind, double delta, double t)
{
    const double z = t / delta;
    if (kind == 0) return t * t / (sqrt(1.0 + z * z) + 1.0);
    const double a = fabs(z);
    if (kind == 1) return delta * delta * (a - log1p(a));
    return 0.5 * t * t / (1.0 + pow(a, 0.8));
}

// Partials of the data term 1/2 sum w (p - y)^2 (quantity 0) and of R(x) (quantity 1): four directions
// (0,1), (1,0), (1,1), (1,-1), each pair once, beta / ||s|| per direction, kappa_j kappa_n per pair when
// kappa is given, a pair only when both pixels lie in the image.
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_cost_partial(const float *__restrict__ p, const T *__restrict__ y,
                                                             const T *__restrict__ w, size_t nsino,
                                                             const float *__restrict__ x,
                                                             const float *__restrict__ kappa, int nx, int ny,
                                                             int kind, double delta, double beta,
                                                             double *__restrict__ part)
{
    double v[2] = {0.0, 0.0};
    const size_t stride = (size_t)RED_BLOCKS * RED_THREADS;
    for (size_t i = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; i < nsino; i += stride) {
        const double r = (double)p[i] - (double)(float)y[i];
        v[0] += 0.5 * (double)(float)w[i] * r * r;
    }
    const int di[4] = {0, 1, 1, 1};
    const int dj[4] = {1, 0, 1, -1};
    const double bd[4] = {beta, beta, beta / sqrt(2.0), beta / sqrt(2.0)};
    const size_t n = (size_t)nx * ny;
    for (size_t q = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; q < n; q += stride) {
        const int i = (int)(q / nx), j = (int)(q % nx);
        const double xc = (double)x[q];
        for (int d = 0; d < 4; ++d) {
            const int i2 = i + di[d], j2 = j + dj[d];
            if (i2 >= ny || j2 < 0 || j2 >= nx) continue;
            const size_t q2 = (size_t)i2 * nx + j2;
            const double kk = kappa ? (double)kappa[q] * (double)kappa[q2] : 1.0;
            v[1] += bd[d] * kk * potential64(kind, delta, xc - (double)x[q2]);
        }
    }
    block_reduce_store<2>(v, part);
}

__global__ void k_cost_total(double *out) { out[2] = out[0] + out[1]; }

}  // namespace

hipError_t launch_trace_reduce(const float *x, const float *ref, const float *gv, const float *h, int nx, int ny,
                               float dx, float dy, float radius, double *out, hipStream_t s)
{
    // out holds kTraceOut doubles followed by TRACE_Q * RED_BLOCKS doubles of scratch
    double *part = out + kTraceOut;
    hipLaunchKernelGGL(k_trace_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, ref, gv, h, nx, ny, dx, dy,
                       radius, part);
    hipLaunchKernelGGL(k_final<TRACE_Q>, dim3(1), dim3(RED_BLOCKS), 0, s, part, out);
    return hipGetLastError();
}

hipError_t launch_cost_reduce(const float *p, const void *y, const void *w, int dtype, size_t nsino, const float *x,
                              const float *kappa, int nx, int ny, int kind, double delta, double beta, double *out,
                              hipStream_t s)
{
    double *part = out + kCostOut;
    const dim3 grid(RED_BLOCKS), block(RED_THREADS);
    if (dtype == CT_F16)
        hipLaunchKernelGGL(k_cost_partial<_Float16>, grid, block, 0, s, p, static_cast<const _Float16 *>(y),
                           static_cast<const _Float16 *>(w), nsino, x, kappa, nx, ny, kind, delta, beta, part);
    else if (dtype == CT_BF16)
        hipLaunchKernelGGL(k_cost_partial<__bf16>, grid, block, 0, s, p, static_cast<const __bf16 *>(y),
                           static_cast<const __bf16 *>(w), nsino, x, kappa, nx, ny, kind, delta, beta, part);
    else
        hipLaunchKernelGGL(k_cost_partial<float>, grid, block, 0, s, p, static_cast<const float *>(y),
                           static_cast<const float *>(w), nsino, x, kappa, nx, ny, kind, delta, beta, part);
    hipLaunchKernelGGL(k_final<2>, dim3(1), dim3(RED_BLOCKS), 0, s, part, out);
    hipLaunchKernelGGL(k_cost_total, dim3(1), dim3(1), 0, s, out);
    return hipGetLastError();
}

}  // namespace ct
