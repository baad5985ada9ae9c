// HIP kernels for gfx950: distance-driven projection pair, fused relaxed OS-LALM update, reductions.
//
// Forward projection (view-parallel): one workgroup per (block of 64 detector bins, view); its waves
// split the image lines of the view and reduce in LDS in a fixed order (deterministic, no atomics).
// Lanes are adjacent bins, so the per-line image reads of a wave are contiguous; column-sweep views read
// the transposed image so that every view reads its lines contiguously. The epilogue writes the
// weighted, subset-scaled residual M w (A_m x - y) directly (the seed of the subset gradient).
//
// Back-projection (gather, pixel-parallel, no atomics): one thread per pixel; for each view the
// candidate bins come from the detector coordinate of the pixel's two edges (+-1 bin of margin), and the
// overlaps are then evaluated from the same FP32 boundary table and the same fmaf sequence as the
// forward projector, so the back-projector is the transpose of the implemented forward operator up to
// the order of summation.
//
// The back-projection kernel also carries the rest of the subiteration (Algorithm 1 of the paper):
// the g and h recursions with rho_t, then the regularizer gradient / Huber curvature stencil and the
// clipped x-step of the next subiteration with rho_{t+1}, writing the new image and its transpose.
#include "ct_internal.hpp"

namespace ct {

namespace {

constexpr int FP_BINS = 64;   // bins per forward workgroup (one per lane)
constexpr int FP_WAVES = 8;   // waves per forward workgroup (line split)
constexpr int BP_TX = 16, BP_TY = 16;

__device__ __forceinline__ float rcp_approx(float v) { return __builtin_amdgcn_rcpf(v); }

template <int EPI, bool ONES>
__global__ __launch_bounds__(FP_BINS *FP_WAVES) void k_forward(GeomDev G, const float *__restrict__ img,
                                                                const float *__restrict__ imgT,
                                                                int vstart, int vstride,
                                                                const float *__restrict__ y,
                                                                const float *__restrict__ w, float mscale,
                                                                float *__restrict__ out)
{
    const int vi = blockIdx.y;
    const int v = vstart + vi * vstride;
    const int lane = threadIdx.x & (FP_BINS - 1);
    const int wave = threadIdx.x / FP_BINS;
    const int nb = G.nb;
    const int k = blockIdx.x * FP_BINS + lane;
    const bool row = G.rowsweep[v] != 0;
    const int NL = row ? G.ny : G.nx;
    const int NQ = row ? G.nx : G.ny;
    const float *src = row ? img : imgT;
    const float half = 0.5f * (float)NQ;
    const float lc0 = -0.5f * (float)(NL - 1);
    float acc = 0.f;
    if (k < nb) {
        const float2 b0 = G.bnd[(size_t)v * (nb + 1) + k];
        const float2 b1 = G.bnd[(size_t)v * (nb + 1) + k + 1];
        const int l0 = (wave * NL) / FP_WAVES, l1 = ((wave + 1) * NL) / FP_WAVES;
        for (int l = l0; l < l1; ++l) {
            const float lc = lc0 + (float)l;
            const float u0 = fmaf(lc, b0.y, b0.x);
            const float u1 = fmaf(lc, b1.y, b1.x);
            const float lo = fminf(u0, u1), hi = fmaxf(u0, u1);
            const float loc = fmaxf(lo, -half), hic = fminf(hi, half);
            if (loc < hic) {
                int q0 = (int)floorf(loc + half);
                if (loc < (float)q0 - half) --q0;              // exact correction of a rounded floor
                int q1 = (int)floorf(hic + half);
                if (hic > (float)(q1 + 1) - half) ++q1;
                q0 = max(q0, 0);
                q1 = min(q1, NQ - 1);
                float s = 0.f;
                if (ONES) {
                    // all-ones image: the clamped overlaps telescope to the clamped footprint
                    for (int q = q0; q <= q1; ++q) {
                        const float e0 = (float)q - half;
                        s += fmaxf(fminf(hic, e0 + 1.f) - fmaxf(loc, e0), 0.f);
                    }
                } else {
                    const float *line = src + (size_t)l * NQ;
                    for (int q = q0; q <= q1; ++q) {
                        const float e0 = (float)q - half;
                        const float ov = fminf(hic, e0 + 1.f) - fmaxf(loc, e0);
                        s = fmaf(fmaxf(ov, 0.f), line[q], s);
                    }
                }
                acc = fmaf(s, rcp_approx(hi - lo), acc);
            }
        }
    }
    __shared__ float red[FP_WAVES][FP_BINS];
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && k < nb) {
        float p = 0.f;
#pragma unroll
        for (int ww = 0; ww < FP_WAVES; ++ww) p += red[ww][lane];
        p *= G.scale[(size_t)v * nb + k];
        const size_t o = (size_t)vi * nb + k;
        const size_t si = (size_t)v * nb + k;
        if (EPI == FP_PLAIN) out[o] = p;
        else if (EPI == FP_RESIDUAL) out[o] = mscale * w[si] * (p - y[si]);
        else out[o] = w[si] * p;
    }
}

// Back-projection of one pixel over the views vstart + vi * vstride, vi < nv.
__device__ __forceinline__ float bp_pixel(const GeomDev &G, const float *__restrict__ r, int vstart, int vstride,
                                          int nv, int i, int j)
{
    const int nb = G.nb;
    float zeta = 0.f;
    for (int vi = 0; vi < nv; ++vi) {
        const int v = vstart + vi * vstride;
        const bool row = G.rowsweep[v] != 0;
        const int l = row ? i : j, q = row ? j : i;
        const int NL = row ? G.ny : G.nx, NQ = row ? G.nx : G.ny;
        const float lc = (float)l - 0.5f * (float)(NL - 1);
        const float e0 = (float)q - 0.5f * (float)NQ;
        const float e1 = e0 + 1.f;
        const float4 im = G.inv[v];
        const float nlc = lc * im.y;
        const float dlc = fmaf(lc, im.w, G.dso);
        const float num0 = fmaf(e0, im.x, nlc), den0 = fmaf(e0, im.z, dlc);
        const float num1 = fmaf(e1, im.x, nlc), den1 = fmaf(e1, im.z, dlc);
        float t0 = num0 / den0, t1 = num1 / den1;
        if (G.arc) {
            t0 = atanf(t0);
            t1 = atanf(t1);
        }
        float kf0 = fmaf(G.c_kf, t0, G.k0), kf1 = fmaf(G.c_kf, t1, G.k0);
        float kmn = fminf(kf0, kf1), kmx = fmaxf(kf0, kf1);
        kmn = fminf(fmaxf(kmn, -2.f), (float)nb + 2.f);
        kmx = fminf(fmaxf(kmx, -2.f), (float)nb + 2.f);
        const int ka = max((int)floorf(kmn) - 1, 0);
        const int kb = min((int)floorf(kmx) + 1, nb - 1);
        if (ka > kb) continue;
        const float2 *bv = G.bnd + (size_t)v * (nb + 1);
        const float *sv = G.scale + (size_t)v * nb;
        const float *rv = r + (size_t)vi * nb;
        float2 bp = bv[ka];
        float up = fmaf(lc, bp.y, bp.x);
        for (int k = ka; k <= kb; ++k) {
            const float2 bn = bv[k + 1];
            const float un = fmaf(lc, bn.y, bn.x);
            const float lo = fminf(up, un), hi = fmaxf(up, un);
            const float ov = fminf(hi, e1) - fmaxf(lo, e0);
            if (ov > 0.f) zeta = fmaf(rv[k] * sv[k], ov * rcp_approx(hi - lo), zeta);
            up = un;
        }
    }
    return zeta;
}

__device__ __forceinline__ void pot_terms(int potential, float delta, float t, float &dphi, float &omega)
{
    const float z = t / delta;
    if (potential == 0) {
        omega = rsqrtf(fmaf(z, z, 1.f));
    } else {
        omega = 1.f / (1.f + fabsf(z));
    }
    dphi = t * omega;
}

template <int MODE>
__global__ __launch_bounds__(BP_TX *BP_TY) void k_back_update(GeomDev G, const float *__restrict__ r, int vstart,
                                                              int vstride, int nv, float *__restrict__ out_back,
                                                              UpdateArgs U)
{
    const int tx = threadIdx.x % BP_TX, ty = threadIdx.x / BP_TX;
    const int j = blockIdx.x * BP_TX + tx, i = blockIdx.y * BP_TY + ty;
    const int nx = G.nx, ny = G.ny;
    __shared__ float tile[BP_TX][BP_TY + 1];
    const bool inside = i < ny && j < nx;
    float xn = 0.f;
    if (inside) {
        const size_t idx = (size_t)i * nx + j;
        float zeta = 0.f;
        if (MODE != BP_XSTEP) zeta = bp_pixel(G, r, vstart, vstride, nv, i, j);
        if (MODE == BP_BACK) {
            out_back[idx] = zeta;
        } else {
            const float xc = U.x[idx];
            const float d = U.dl[idx];
            float g = U.gv[idx], hh = U.h[idx];
            const long long t = (U.tbase ? (long long)(*U.tbase) : 0ll) + U.tofs;
            if (MODE == BP_INIT || MODE == BP_INIT_XSTEP) {
                g = zeta;
                hh = U.algorithm == 1 ? fmaf(d, xc, -zeta) : zeta;
                U.gv[idx] = g;
                U.h[idx] = hh;
            } else if (MODE == BP_FULL || MODE == BP_DUAL) {
                const float rho = U.rho[t];
                const float a = U.alpha;
                const float inv1 = 1.f / (rho + 1.f);
                const float gn = rho * inv1 * (a * zeta + (1.f - a) * g) + g * inv1;
                const float hn = U.algorithm == 1 ? a * fmaf(d, xc, -zeta) + (1.f - a) * hh : zeta;
                g = gn;
                hh = hn;
                U.gv[idx] = g;
                U.h[idx] = hh;
            }
            if (MODE == BP_FULL || MODE == BP_XSTEP || MODE == BP_INIT_XSTEP) {
                const long long tx1 = MODE == BP_FULL ? t + 1 : t;
                const float rho1 = U.rho[tx1];
                const float s = U.algorithm == 1 ? rho1 * fmaf(d, xc, -hh) + (1.f - rho1) * g
                                                 : rho1 * hh + (1.f - rho1) * g;
                // regularizer gradient and Huber curvature at xc (8 neighbours, 4 directions)
                float gr = 0.f, dr = 0.f;
                const float kc = U.kappa ? U.kappa[idx] : 1.f;
                const int di[8] = {0, 0, 1, -1, 1, -1, 1, -1};
                const int dj[8] = {1, -1, 0, 0, 1, -1, -1, 1};
#pragma unroll
                for (int n = 0; n < 8; ++n) {
                    const int i2 = i + di[n], j2 = j + dj[n];
                    if (i2 < 0 || i2 >= ny || j2 < 0 || j2 >= nx) continue;
                    const size_t i2x = (size_t)i2 * nx + j2;
                    const float bt = (n < 4 ? U.beta_ax : U.beta_dg) * (U.kappa ? kc * U.kappa[i2x] : 1.f);
                    float dphi, om;
                    pot_terms(U.potential, U.delta, xc - U.x[i2x], dphi, om);
                    gr = fmaf(bt, dphi, gr);
                    dr = fmaf(bt, 2.f * (U.huber ? om : 1.f), dr);
                }
                const float den = fmaf(rho1, d, dr);
                xn = den > 0.f ? fmaxf(xc - (s + gr) / den, 0.f) : xc;
                U.x_next[idx] = xn;
            }
        }
    }
    if (MODE == BP_FULL || MODE == BP_XSTEP || MODE == BP_INIT_XSTEP) {
        // transpose through LDS: write xT_next[j][i] in runs of BP_TY along i
        tile[tx][ty] = xn;
        __syncthreads();
        const int jj = blockIdx.x * BP_TX + ty;   // swapped roles
        const int ii = blockIdx.y * BP_TY + tx;
        if (jj < nx && ii < ny) U.xT_next[(size_t)jj * ny + ii] = tile[ty][tx];
    }
}

__global__ void k_transpose(const float *__restrict__ x, float *__restrict__ xT, int nx, int ny)
{
    __shared__ float tile[16][17];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    int j = blockIdx.x * 16 + tx, i = blockIdx.y * 16 + ty;
    if (i < ny && j < nx) tile[ty][tx] = x[(size_t)i * nx + j];
    __syncthreads();
    int ii = blockIdx.y * 16 + tx, jj = blockIdx.x * 16 + ty;
    if (ii < ny && jj < nx) xT[(size_t)jj * ny + ii] = tile[tx][ty];
}

__global__ void k_clip_copy(const float *__restrict__ in, float *__restrict__ out, float *__restrict__ outT, int nx,
                            int ny, int zero)
{
    __shared__ float tile[16][17];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    int j = blockIdx.x * 16 + tx, i = blockIdx.y * 16 + ty;
    float v = 0.f;
    if (i < ny && j < nx) {
        v = zero ? 0.f : fmaxf(in[(size_t)i * nx + j], 0.f);
        out[(size_t)i * nx + j] = v;
    }
    tile[ty][tx] = v;
    __syncthreads();
    int ii = blockIdx.y * 16 + tx, jj = blockIdx.x * 16 + ty;
    if (ii < ny && jj < nx) outT[(size_t)jj * ny + ii] = tile[tx][ty];
}

__global__ void k_scale(float *x, size_t n, float a)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] *= a;
}

__global__ void k_fill(float *x, size_t n, float a)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = a;
}

__global__ void k_kappa(const float *bw, const float *b1, float *kappa, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) kappa[i] = b1[i] > 0.f ? sqrtf(fmaxf(bw[i], 0.f) / b1[i]) : 0.f;
}

__global__ void k_add_counter(int *c, int add) { c[0] += add; }
__global__ void k_set_counter(int *c, int value) { c[0] = value; }

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

hipError_t launch_forward(const GeomDev &G, const float *img, const float *imgT, int ones, int vstart, int vstride,
                          int nv, int epi, const float *y, const float *w, float mscale, float *out, hipStream_t s)
{
    if (nv <= 0) return hipSuccess;
    dim3 grid((G.nb + FP_BINS - 1) / FP_BINS, nv), block(FP_BINS * FP_WAVES);
#define CT_FP_LAUNCH(E, O)                                                                                     \
    hipLaunchKernelGGL((k_forward<E, O>), grid, block, 0, s, G, img, imgT, vstart, vstride, y, w, mscale, out)
    if (ones) {
        if (epi == FP_PLAIN) CT_FP_LAUNCH(FP_PLAIN, true);
        else if (epi == FP_RESIDUAL) CT_FP_LAUNCH(FP_RESIDUAL, true);
        else CT_FP_LAUNCH(FP_WEIGHTED, true);
    } else {
        if (epi == FP_PLAIN) CT_FP_LAUNCH(FP_PLAIN, false);
        else if (epi == FP_RESIDUAL) CT_FP_LAUNCH(FP_RESIDUAL, false);
        else CT_FP_LAUNCH(FP_WEIGHTED, false);
    }
#undef CT_FP_LAUNCH
    return hipGetLastError();
}

hipError_t launch_back_update(const GeomDev &G, int mode, const float *r, int vstart, int vstride, int nv,
                              float *out_back, const UpdateArgs &U, hipStream_t s)
{
    dim3 grid((G.nx + BP_TX - 1) / BP_TX, (G.ny + BP_TY - 1) / BP_TY), block(BP_TX * BP_TY);
#define CT_BP_CASE(M)                                                                                          \
    case M: hipLaunchKernelGGL(k_back_update<M>, grid, block, 0, s, G, r, vstart, vstride, nv, out_back, U); break;
    switch (mode) {
        CT_BP_CASE(BP_BACK)
        CT_BP_CASE(BP_INIT)
        CT_BP_CASE(BP_FULL)
        CT_BP_CASE(BP_DUAL)
        CT_BP_CASE(BP_XSTEP)
        CT_BP_CASE(BP_INIT_XSTEP)
    default: return hipErrorInvalidValue;
    }
#undef CT_BP_CASE
    return hipGetLastError();
}

hipError_t launch_transpose(const float *x, float *xT, int nx, int ny, hipStream_t s)
{
    dim3 grid((nx + 15) / 16, (ny + 15) / 16);
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, x, xT, nx, ny);
    return hipGetLastError();
}

hipError_t launch_clip_copy(const float *in, float *out, float *outT, int nx, int ny, int zero, hipStream_t s)
{
    dim3 grid((nx + 15) / 16, (ny + 15) / 16);
    hipLaunchKernelGGL(k_clip_copy, grid, dim3(256), 0, s, in, out, outT, nx, ny, zero);
    return hipGetLastError();
}

hipError_t launch_scale(float *x, size_t n, float a, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, a);
    return hipGetLastError();
}

hipError_t launch_fill(float *x, size_t n, float a, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, a);
    return hipGetLastError();
}

hipError_t launch_kappa(const float *bw, const float *b1, float *kappa, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_kappa, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, bw, b1, kappa, n);
    return hipGetLastError();
}

hipError_t launch_add_counter(int *c, int add, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_counter, dim3(1), dim3(1), 0, s, c, add);
    return hipGetLastError();
}

hipError_t launch_set_counter(int *c, int value, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, s, c, value);
    return hipGetLastError();
}

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
