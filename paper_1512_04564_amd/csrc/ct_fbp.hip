// FBP-like start image for a flat fan-beam detector (Algorithm 1 starts from an FBP image).
//
// Per view, the data are cosine-weighted on the detector magnified to the isocentre
// (dso / sqrt(dso^2 + s^2), s the isocentre coordinate of the bin centre), filtered with the spatial
// Ram-Lak kernel on the isocentre grid (h(0) = 1/(4 d^2), h(n odd) = -1/(pi n d)^2, h(n even) = 0, scaled
// by d), then back-projected pixel by pixel with linear interpolation between bin centres and the fan
// weight (dso / L)^2, L the source-to-pixel distance along the central ray; a full scan measures every
// ray twice, hence the factor 1/2 with the angular step. The result is clipped at zero.
#include "ct_internal.hpp"

namespace ct {

namespace {

constexpr int FILT_THREADS = 256;

// q[v][k] = d * sum_k2 h(k - k2) cw(k2) y[v][k2]; the weighted row is staged in LDS. The kernel's DC gain is a
// near-exact cancellation of h(0) against the odd taps, so the coefficients and the sum are FP64: a one-ulp
// FP32 mismatch between h(0) and the odd taps leaks a DC offset that the view sum amplifies.
template <typename TY>
__global__ __launch_bounds__(FILT_THREADS) void k_fbp_filter(const TY *__restrict__ y, float *__restrict__ q,
                                                            int nb, double dui, float dso, float uoff_bins,
                                                            double h0, double hodd)
{
    // LDS: the weighted row (nb floats, padded to whole doubles), then the odd taps' coefficients
    // cf[m] = h(2m + 1) = hodd / (2m + 1)^2, m < nb / 2, divided once per workgroup instead of once per tap
    // and output (nb <= 8192: at most 64 KB)
    extern __shared__ double smem[];
    float *row = reinterpret_cast<float *>(smem);
    double *cf = smem + (nb + 1) / 2;
    const int v = blockIdx.y;
    const TY *yv = y + (size_t)v * nb;
    for (int k = threadIdx.x; k < nb; k += FILT_THREADS) {
        const float s = ((float)k + 0.5f - 0.5f * (float)nb + uoff_bins) * (float)dui;
        row[k] = (float)yv[k] * dso * rsqrtf(fmaf(s, s, dso * dso));
    }
    for (int m = threadIdx.x; m < nb / 2; m += FILT_THREADS) {
        const double n = 2.0 * (double)m + 1.0;
        cf[m] = hodd / (n * n);
    }
    __syncthreads();
    const int k = blockIdx.x * FILT_THREADS + threadIdx.x;
    if (k >= nb) return;
    double acc = h0 * row[k];
    // odd offsets n = k - k2 = +-1, +-3, ...: h(n) = hodd / n^2
    for (int n = 1; n <= k || n < nb - k; n += 2) {
        double pair = 0.0;
        if (n <= k) pair += row[k - n];
        if (k + n < nb) pair += row[k + n];
        acc = fma(cf[n >> 1], pair, acc);
    }
    q[(size_t)v * nb + k] = (float)(acc * dui);
}

// x(i, j) = max(0, fac * sum_v (dso / L)^2 q_v(s')), s' the isocentre coordinate of the ray through the pixel.
// The bin coordinate reaches several hundred bins and the filtered rows are steep at object edges, so the
// pixel-to-bin geometry and the view sum are carried in FP64 (FP32 coordinates alone cost ~3e-5 relative).
__global__ __launch_bounds__(256) void k_fbp_back(const float *__restrict__ q, const double2 *__restrict__ cs, int nx,
                                                  int ny, double dx, double dy, int nb, int nviews, double dui,
                                                  double dso, double k0, double fac, float *__restrict__ x)
{
    const int j = blockIdx.x * 16 + threadIdx.x % 16, i = blockIdx.y * 16 + threadIdx.x / 16;
    if (i >= ny || j >= nx) return;
    const double px = ((double)j - 0.5 * (double)(nx - 1)) * dx;
    const double py = ((double)i - 0.5 * (double)(ny - 1)) * dy;
    const double rdui = 1.0 / dui;
    double acc = 0.0;
    for (int v = 0; v < nviews; ++v) {
        const double2 c = cs[v];
        const double L = fma(px, c.x, fma(py, c.y, dso));
        const double t = fma(-px, c.y, py * c.x);
        const double invL = 1.0 / L;
        const double kf = fma(dso * t * invL, rdui, k0);   // bin-centre coordinate
        const double kfl = floor(kf);
        const int k = (int)kfl;
        if (k < 0 || k + 1 >= nb) continue;
        const double f = kf - kfl;
        const float *qv = q + (size_t)v * nb;
        const double q0 = qv[k], q1 = qv[k + 1];
        const double wgt = dso * invL;
        acc = fma(fma(f, q1 - q0, q0), wgt * wgt, acc);
    }
    x[(size_t)i * nx + j] = fmaxf((float)(fac * acc), 0.f);
}

}  // namespace

hipError_t launch_fbp(const ct_geom *g, const void *y, int ytype, float *q, const double2 *cs, float *x, hipStream_t s)
{
    const ct_geom_desc &d = g->desc;
    const double dui = d.du * d.dso / d.dsd;   // bin width at the isocentre
    const double pi = 3.14159265358979323846;
    dim3 gf((d.nb + FILT_THREADS - 1) / FILT_THREADS, d.nviews);
    const size_t lds = (size_t)((d.nb + 1) / 2 + d.nb / 2) * sizeof(double);   // row + odd-tap coefficients
    const double h0 = 1.0 / (4.0 * dui * dui), hodd = -1.0 / (pi * pi * dui * dui);
    if (ytype == CT_F32)
        hipLaunchKernelGGL(k_fbp_filter<float>, gf, dim3(FILT_THREADS), lds, s, static_cast<const float *>(y), q, d.nb,
                           dui, (float)d.dso, (float)d.u_offset, h0, hodd);
    else if (ytype == CT_F16)
        hipLaunchKernelGGL(k_fbp_filter<_Float16>, gf, dim3(FILT_THREADS), lds, s, static_cast<const _Float16 *>(y), q,
                           d.nb, dui, (float)d.dso, (float)d.u_offset, h0, hodd);
    else if (ytype == CT_BF16)
        hipLaunchKernelGGL(k_fbp_filter<__bf16>, gf, dim3(FILT_THREADS), lds, s, static_cast<const __bf16 *>(y), q, d.nb,
                           dui, (float)d.dso, (float)d.u_offset, h0, hodd);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double fac = 0.5 * d.span / d.nviews;
    const double k0 = 0.5 * d.nb - d.u_offset - 0.5;
    dim3 gb((d.nx + 15) / 16, (d.ny + 15) / 16);
    hipLaunchKernelGGL(k_fbp_back, gb, dim3(256), 0, s, q, cs, d.nx, d.ny, d.dx, d.dy, d.nb, d.nviews, dui, d.dso, k0,
                       fac, x);
    return hipGetLastError();
}

}  // namespace ct
