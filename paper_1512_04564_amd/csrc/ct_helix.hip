// 3-D helical cone-beam part of libctrlalm (include/ct_helix.h): device tables, the projector pair, the
// 26-neighbour relaxed update and the solver driver.
//
// Kernels (per-thread arithmetic in ct_helix_body.hpp):
//   k_hcum    cumulative form of the volume for the forward projector, in both layouts: per voxel the
//             FP64 sum of its column's voxels below it (rounded once) and the voxel itself.
//   k_hfp     forward projection of a view block: workgroup = (64 bins, HX_RB rows, view); its HX_FW waves
//             take interleaved planes, lanes are bins; each row of a meeting column is one evaluation of the
//             column's cumulative integral; the waves' partial sums are added in LDS in a fixed order; the epilogue writes A x, the weighted residual M w (A x - y), or w (A 1), the last two
//             optionally prescaled for the back-projector (hx_prescale).
//   k_hbp     gather back-projection, no atomics: a wave is an 8 x 8 tile of voxel columns, every lane the
//             same HX_ZG voxels in z of its column, so that the lanes of a wave meet the same few detector
//             rows and neighbouring bins of each view (a few cache lines per load) and enter and leave the
//             cone together; the 4 waves of a workgroup take 4 consecutive z groups of the tile. Workgroups
//             are ordered so that each XCD takes a contiguous band of tiles (its L2 then holds the detector
//             region that band projects to). Writes or accumulates A' r from the prescaled residual.
//   k_hprescale  r' = scale secphi r for a plain sinogram handed to the back-projector.
//   k_hupd    per voxel: the dual updates g+, h+ of subiteration t, then the clipped x-step of subiteration
//             t + 1 with the 26-neighbour regularizer gradient and Huber curvature; writes the new volume in
//             both projector layouts (canonical [nz][ny][nx] for row-sweep views, per-slice transposed
//             [nz][nx][ny] for column-sweep views, through LDS).
// Every launch is a plain stream-ordered launch (one subiteration = three launches).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ct_helix_internal.hpp"

struct ct_helix {
    ct_helix_desc desc{};
    int device = 0;
    double2 *bnd = nullptr;
    float *scale = nullptr;
    float4 *inv = nullptr;
    int *rowsweep = nullptr;
    float2 *cs = nullptr;
    float *zai = nullptr, *zaf = nullptr, *wr = nullptr, *secphi = nullptr;
    ct::HelixDev dev{};
    // workspace (allocated on first use)
    size_t nvox = 0;
    float *xa = nullptr, *xb = nullptr, *xta = nullptr, *xtb = nullptr;
    float *gv = nullptr, *h = nullptr, *dl = nullptr, *zeta = nullptr;
    float2 *cz = nullptr, *czT = nullptr;   // cumulative forms of the projected volume (both layouts, padded)
    float *r = nullptr;
    size_t r_cap = 0;
    double *red = nullptr;
};

namespace ct {

namespace {

enum HfpEpi { HFP_PLAIN = 0, HFP_RESIDUAL = 1, HFP_WEIGHTED_ONES = 2 };
enum HupdMode { HUPD_CLIP = 0, HUPD_INIT = 1, HUPD_FULL = 2, HUPD_XSTEP = 3 };

constexpr int HFP_THREADS = 64 * HX_FW;
constexpr int HBP_THREADS = 256;   // 4 waves; a wave = 8 x 8 columns x HX_ZG voxels
constexpr int HBP_ZSPAN = 4 * HX_ZG;
constexpr int HBP_XCDS = 8;
constexpr int HUPD_T = 16;         // update tile edge

// Forward projection of views vstart + vi * vstride (vi = blockIdx.z). Bins blockIdx.x * 64 + lane, rows
// blockIdx.y * HX_RB + rr. Output block out[vi][r][k]; y, w indexed by the full view v.
// Cumulative form (blockIdx.y = 0: in0 -> out0, 1: in1 -> out1) of a volume [nz][ncol], padded by one plane
// on each side: out[kz + 1][c] = (sum over k < kz of in[k][c], accumulated in FP64 and rounded once;
// in[kz][c]), out[0][c] = (0, 0), out[nz + 1][c] = (the column's sum, 0). One thread per column.
__global__ __launch_bounds__(256) void k_hcum(const float *__restrict__ in0, const float *__restrict__ in1, int ncol,
                                              int nz, float2 *__restrict__ out0, float2 *__restrict__ out1)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= ncol) return;
    const float *__restrict__ in = blockIdx.y ? in1 : in0;
    float2 *__restrict__ out = blockIdx.y ? out1 : out0;
    double acc = 0.0;
    out[c] = make_float2(0.f, 0.f);
    for (int kz = 0; kz < nz; ++kz) {
        const float v = in[(size_t)kz * ncol + c];
        out[(size_t)(kz + 1) * ncol + c] = make_float2((float)acc, v);
        acc += (double)v;
    }
    out[(size_t)(nz + 1) * ncol + c] = make_float2((float)acc, 0.f);
}

template <bool ONES>
__global__ __launch_bounds__(HFP_THREADS) void k_hfp(HelixDev G, const float2 *__restrict__ cz,
                                                     const float2 *__restrict__ czT, size_t nvox, int vstart,
                                                     int vstride, int epi, int prescale,
                                                     const float *__restrict__ y, const float *__restrict__ w,
                                                     float mscale, float *__restrict__ out)
{
    __shared__ float part[HX_FW][HX_RB][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + lane;
    const int r0 = blockIdx.y * HX_RB;
    const int vi = blockIdx.z;
    const int v = vstart + vi * vstride;
    const bool row = G.rowsweep[v] != 0;
    float acc[HX_RB];
#pragma unroll
    for (int rr = 0; rr < HX_RB; ++rr) acc[rr] = 0.f;
    if (k < G.nb) {
        const Ro<float2> C{row ? cz : czT, nvox + 2 * (size_t)G.nx * G.ny};   // padded by two planes
        hfp_lane<ONES>(G, C, v, k, r0, wave, HX_FW, acc);
    }
#pragma unroll
    for (int rr = 0; rr < HX_RB; ++rr) part[wave][rr][lane] = acc[rr];
    __syncthreads();
    for (int idx = threadIdx.x; idx < HX_RB * 64; idx += HFP_THREADS) {
        const int rr = idx >> 6, ln = idx & 63;
        const int kk = blockIdx.x * 64 + ln, r = r0 + rr;
        if (kk >= G.nb || r >= G.nr) continue;
        float s = part[0][rr][ln];
#pragma unroll
        for (int wv = 1; wv < HX_FW; ++wv) s += part[wv][rr][ln];
        const float sv = hx_prescale(G, v, r, kk);
        const float val = s * sv;
        const size_t o = ((size_t)vi * G.nr + r) * G.nb + kk;
        const size_t src = ((size_t)v * G.nr + r) * G.nb + kk;
        float res;
        if (epi == HFP_PLAIN) res = val;
        else if (epi == HFP_RESIDUAL) res = mscale * w[src] * (val - y[src]);
        else res = w[src] * val;
        out[o] = prescale ? res * sv : res;
    }
}

// Back-projection: blockIdx.x = 8 x 8 column tile (XCD-ordered), blockIdx.y = block of HBP_ZSPAN voxels in
// z. Wave w takes voxels (blockIdx.y * 4 + w) * HX_ZG .. of the 64 columns; lane l is column
// (8 ty + l / 8, 8 tx + l % 8). Rp is the prescaled residual; out = A' r (accumulate: out += A' r).
__global__ __launch_bounds__(HBP_THREADS) void k_hbp(HelixDev G, const float *__restrict__ rp, size_t rlen, int vstart,
                                                     int vstride, int nv, float *__restrict__ out, int accumulate)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_x = (G.nx + 7) >> 3, ntiles = tiles_x * ((G.ny + 7) >> 3);
    // workgroups go round-robin over the XCDs: give XCD x the tiles [x n / 8, (x + 1) n / 8)
    const int bid = blockIdx.x;
    const int full = ntiles - ntiles % HBP_XCDS;
    const int tile = bid < full ? (bid % HBP_XCDS) * (full / HBP_XCDS) + bid / HBP_XCDS : bid;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int j = tx * 8 + (lane & 7), i = ty * 8 + (lane >> 3);
    const int kz0 = (blockIdx.y * 4 + wave) * HX_ZG;
    if (i >= G.ny || j >= G.nx || kz0 >= G.nz) return;   // no barrier in this kernel
    float acc[HX_ZG];
#pragma unroll
    for (int b = 0; b < HX_ZG; ++b) acc[b] = 0.f;
    const Ro<float> R{rp, rlen};
    hbp_lane(G, R, vstart, vstride, nv, i, j, kz0, acc);
#pragma unroll
    for (int b = 0; b < HX_ZG; ++b) {
        const int kz = kz0 + b;
        if (kz >= G.nz) break;
        const size_t idx = ((size_t)kz * G.ny + i) * G.nx + j;
        out[idx] = accumulate ? out[idx] + acc[b] : acc[b];
    }
}

// r' = scale secphi r over the view block [nv][nr][nb] of views vstart + vi * vstride.
__global__ __launch_bounds__(256) void k_hprescale(HelixDev G, const float *__restrict__ r, int vstart, int vstride,
                                                   int nv, float *__restrict__ out)
{
    const size_t n = (size_t)nv * G.nr * G.nb;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        const int k = (int)(e % (size_t)G.nb);
        const size_t vr = e / (size_t)G.nb;
        const int rr = (int)(vr % (size_t)G.nr), vi = (int)(vr / (size_t)G.nr);
        out[e] = r[e] * hx_prescale(G, vstart + vi * vstride, rr, k);
    }
}

// Update over a 16 x 16 tile of slice blockIdx.z. Modes:
//   CLIP   x_next = max(x, 0) (zero: 0)
//   INIT   g = zeta, h = D_L x - zeta
//   FULL   g, h of subiteration t (rho_a = rho_t), then x_next = x-step of t + 1 (rho_b = rho_t+1) at x
//   XSTEP  x_next = x-step with rho_a from the current g, h
// CLIP, FULL and XSTEP also write x_next's per-slice transpose xT_next [nz][nx][ny].
__global__ __launch_bounds__(HUPD_T * HUPD_T) void k_hupd(HelixUpdate U, int mode, int zero, const float *__restrict__ x,
                                                          size_t nvox, const float *__restrict__ zeta,
                                                          float *__restrict__ gv, float *__restrict__ h,
                                                          const float *__restrict__ dl, float rho_a, float rho_b,
                                                          float *__restrict__ x_next, float *__restrict__ xT_next)
{
    __shared__ float tile[HUPD_T][HUPD_T + 1];
    const int tx = threadIdx.x % HUPD_T, ty = threadIdx.x / HUPD_T;
    const int j = blockIdx.x * HUPD_T + tx, i = blockIdx.y * HUPD_T + ty, kz = blockIdx.z;
    const bool valid = i < U.ny && j < U.nx;
    const size_t idx = ((size_t)kz * U.ny + i) * U.nx + j;
    float xn = 0.f;
    if (valid) {
        const float xc = x[idx];
        if (mode == HUPD_CLIP) {
            xn = zero ? 0.f : fmaxf(xc, 0.f);
        } else if (mode == HUPD_INIT) {
            const float z = zeta[idx];
            gv[idx] = z;
            h[idx] = fmaf(dl[idx], xc, -z);
        } else {
            float g = gv[idx], hh = h[idx];
            const float d = dl[idx];
            float rho = rho_a;
            if (mode == HUPD_FULL) {
                const float z = zeta[idx];
                const float inv1 = hx_rcp(rho_a + 1.f);
                const float gn = rho_a * inv1 * fmaf(U.alpha, z, (1.f - U.alpha) * g) + g * inv1;
                hh = fmaf(U.alpha, fmaf(d, xc, -z), (1.f - U.alpha) * hh);
                g = gn;
                gv[idx] = g;
                h[idx] = hh;
                rho = rho_b;
            }
            float gr, dr;
            reg26(U, Ro<float>{x, nvox}, kz, i, j, xc, gr, dr);
            xn = xstep(rho, xc, g, hh, d, gr, dr);
        }
        if (mode != HUPD_INIT) x_next[idx] = xn;
    }
    if (mode == HUPD_INIT) return;   // uniform over the workgroup: no barrier is skipped by part of it
    tile[ty][tx] = xn;
    __syncthreads();
    const int jt = blockIdx.x * HUPD_T + ty, it = blockIdx.y * HUPD_T + tx;
    if (jt < U.nx && it < U.ny) xT_next[((size_t)kz * U.nx + jt) * U.ny + it] = tile[tx][ty];
}

// Per-slice transpose x [nz][ny][nx] -> xT [nz][nx][ny].
__global__ __launch_bounds__(HUPD_T * HUPD_T) void k_htranspose(const float *__restrict__ x, float *__restrict__ xT, int nx,
                                                                int ny)
{
    __shared__ float tile[HUPD_T][HUPD_T + 1];
    const int tx = threadIdx.x % HUPD_T, ty = threadIdx.x / HUPD_T;
    const int j = blockIdx.x * HUPD_T + tx, i = blockIdx.y * HUPD_T + ty, kz = blockIdx.z;
    tile[ty][tx] = (i < ny && j < nx) ? x[((size_t)kz * ny + i) * nx + j] : 0.f;
    __syncthreads();
    const int jt = blockIdx.x * HUPD_T + ty, it = blockIdx.y * HUPD_T + tx;
    if (jt < nx && it < ny) xT[((size_t)kz * nx + jt) * ny + it] = tile[tx][ty];
}

template <typename T>
ct_status hx_alloc(T **p, size_t n)
{
    if (*p) return CT_OK;
    hipError_t e = hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? CT_ERR_OOM : CT_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return CT_OK;
}

template <typename T>
void hx_free(T **p)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
}

template <typename T>
ct_status upload(T **dst, const std::vector<T> &src)
{
    CT_TRY(hx_alloc(dst, src.size()));
    CT_HIP_CHECK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return CT_OK;
}

void free_helix(ct_helix *h)
{
    hx_free(&h->bnd);
    hx_free(&h->scale);
    hx_free(&h->inv);
    hx_free(&h->rowsweep);
    hx_free(&h->cs);
    hx_free(&h->zai);
    hx_free(&h->zaf);
    hx_free(&h->wr);
    hx_free(&h->secphi);
    hx_free(&h->xa);
    hx_free(&h->xb);
    hx_free(&h->xta);
    hx_free(&h->xtb);
    hx_free(&h->gv);
    hx_free(&h->h);
    hx_free(&h->dl);
    hx_free(&h->zeta);
    hx_free(&h->r);
    hx_free(&h->cz);
    hx_free(&h->czT);
    hx_free(&h->red);
}

ct_status ensure_views(ct_helix *h, int nv)
{
    const size_t need = (size_t)nv * h->desc.nr * h->desc.nb;
    if (need > h->r_cap) {
        hx_free(&h->r);
        h->r_cap = 0;
        CT_TRY(hx_alloc(&h->r, need));
        h->r_cap = need;
    }
    CT_TRY(hx_alloc(&h->xta, h->nvox));
    const size_t ncz = h->nvox + 2 * (size_t)h->desc.nx * h->desc.ny;   // two padding planes
    CT_TRY(hx_alloc(&h->cz, ncz));
    CT_TRY(hx_alloc(&h->czT, ncz));
    CT_TRY(hx_alloc(&h->red, kRedSize));
    return CT_OK;
}

ct_status subset_of(const ct_helix *h, int subset, int *vs, int *vst, int *nv)
{
    const int M = h->desc.nsubsets;
    if (subset == -1) {
        *vs = 0;
        *vst = 1;
        *nv = h->desc.nviews;
        return CT_OK;
    }
    if (subset < 0 || subset >= M) return fail(CT_ERR_INVALID_ARG, "subset must be -1 or in [0, M)");
    *vs = subset;
    *vst = M;
    *nv = h->desc.nviews / M;
    return CT_OK;
}

// Forward projection of the volume x (xT its per-slice transpose): the cumulative forms of both layouts,
// then the projection (the ones epilogue reads no volume and skips the first step). prescale: write
// r' = scale secphi (epilogue value), the back-projector's input.
hipError_t launch_hfp(const ct_helix *h, const float *x, const float *xT, int vs, int vst, int nv, int epi,
                      int prescale, const float *y, const float *w, float mscale, float *out, hipStream_t s)
{
    const ct_helix_desc &d = h->desc;
    if (epi != HFP_WEIGHTED_ONES) {
        const int ncol = d.nx * d.ny;
        hipLaunchKernelGGL(k_hcum, dim3((unsigned)((ncol + 255) / 256), 2), dim3(256), 0, s, x, xT, ncol, d.nz, h->cz,
                           h->czT);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)((d.nb + 63) / 64), (unsigned)((d.nr + HX_RB - 1) / HX_RB), (unsigned)nv);
    if (epi == HFP_WEIGHTED_ONES)
        hipLaunchKernelGGL(k_hfp<true>, grid, dim3(HFP_THREADS), 0, s, h->dev, h->cz, h->czT, h->nvox, vs, vst, epi,
                           prescale, y, w, mscale, out);
    else
        hipLaunchKernelGGL(k_hfp<false>, grid, dim3(HFP_THREADS), 0, s, h->dev, h->cz, h->czT, h->nvox, vs, vst, epi,
                           prescale, y, w, mscale, out);
    return hipGetLastError();
}

hipError_t launch_hprescale(const ct_helix *h, const float *r, int vs, int vst, int nv, float *out, hipStream_t s)
{
    const ct_helix_desc &d = h->desc;
    const size_t n = (size_t)nv * d.nr * d.nb;
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_hprescale, dim3(std::max(blocks, 1u)), dim3(256), 0, s, h->dev, r, vs, vst, nv, out);
    return hipGetLastError();
}

hipError_t launch_hbp(const ct_helix *h, const float *r, int vs, int vst, int nv, float *out, int accumulate,
                      hipStream_t s)
{
    const ct_helix_desc &d = h->desc;
    const unsigned tiles = (unsigned)(((d.nx + 7) / 8) * ((d.ny + 7) / 8));
    const dim3 grid(tiles, (unsigned)((d.nz + HBP_ZSPAN - 1) / HBP_ZSPAN));
    const size_t rlen = (size_t)nv * d.nr * d.nb;
    hipLaunchKernelGGL(k_hbp, grid, dim3(HBP_THREADS), 0, s, h->dev, r, rlen, vs, vst, nv, out, accumulate);
    return hipGetLastError();
}

hipError_t launch_hupd(const ct_helix *h, const HelixUpdate &U, int mode, int zero, const float *x, float rho_a,
                       float rho_b, float *x_next, float *xT_next, hipStream_t s)
{
    const ct_helix_desc &d = h->desc;
    const dim3 grid((unsigned)((d.nx + HUPD_T - 1) / HUPD_T), (unsigned)((d.ny + HUPD_T - 1) / HUPD_T), (unsigned)d.nz);
    hipLaunchKernelGGL(k_hupd, grid, dim3(HUPD_T * HUPD_T), 0, s, U, mode, zero, x, h->nvox, h->zeta, h->gv, h->h, h->dl,
                       rho_a, rho_b, x_next, xT_next);
    return hipGetLastError();
}

hipError_t launch_htranspose(const ct_helix *h, const float *x, float *xT, hipStream_t s)
{
    const ct_helix_desc &d = h->desc;
    const dim3 grid((unsigned)((d.nx + HUPD_T - 1) / HUPD_T), (unsigned)((d.ny + HUPD_T - 1) / HUPD_T), (unsigned)d.nz);
    hipLaunchKernelGGL(k_htranspose, grid, dim3(HUPD_T * HUPD_T), 0, s, x, xT, d.nx, d.ny);
    return hipGetLastError();
}

hipStream_t hs(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

}  // namespace ct

using namespace ct;

extern "C" {

ct_status ct_helix_create(const ct_helix_desc *desc, ct_helix **out)
{
    if (!out) return fail(CT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    CT_TRY(check_helix_desc(desc));
    HelixTables t;
    CT_TRY(helix_tables(*desc, t));
    ct_helix *h = new (std::nothrow) ct_helix();
    if (!h) return fail(CT_ERR_OOM, "host allocation failed");
    h->desc = *desc;
    (void)hipGetDevice(&h->device);
    h->nvox = (size_t)desc->nx * desc->ny * desc->nz;
    ct_status st = CT_OK;
    if (st == CT_OK) st = upload(&h->bnd, t.fan.bnd64);
    if (st == CT_OK) st = upload(&h->scale, t.fan.scale);
    if (st == CT_OK) st = upload(&h->inv, t.fan.inv);
    if (st == CT_OK) st = upload(&h->rowsweep, t.fan.rowsweep);
    if (st == CT_OK) st = upload(&h->cs, t.cs);
    if (st == CT_OK) st = upload(&h->zai, t.zai);
    if (st == CT_OK) st = upload(&h->zaf, t.zaf);
    if (st == CT_OK) st = upload(&h->wr, t.wr);
    if (st == CT_OK) st = upload(&h->secphi, t.secphi);
    if (st != CT_OK) {
        free_helix(h);
        delete h;
        return st;
    }
    const ct_helix_desc &d = *desc;
    HelixDev &G = h->dev;
    G.nx = d.nx;
    G.ny = d.ny;
    G.nz = d.nz;
    G.nb = d.nb;
    G.nr = d.nr;
    G.nviews = d.nviews;
    G.dx = (float)d.dx;
    G.dy = (float)d.dy;
    G.dso = (float)d.dso;
    G.c_kf = t.fan.c_kf;
    G.k0 = t.fan.k0;
    G.dwn = t.dwn;
    G.bnd = {h->bnd, t.fan.bnd64.size()};
    G.scale = {h->scale, t.fan.scale.size()};
    G.inv = {h->inv, t.fan.inv.size()};
    G.rowsweep = {h->rowsweep, t.fan.rowsweep.size()};
    G.cs = {h->cs, t.cs.size()};
    G.zai = {h->zai, t.zai.size()};
    G.zaf = {h->zaf, t.zaf.size()};
    G.wr = {h->wr, t.wr.size()};
    G.secphi = {h->secphi, t.secphi.size()};
    *out = h;
    return CT_OK;
}

void ct_helix_destroy(ct_helix *h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_helix(h);
    delete h;
}

ct_status ct_helix_forward(ct_helix *h, int subset, const float *x, float *p, void *stream)
{
    if (!h || !x || !p) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    int vs, vst, nv;
    CT_TRY(subset_of(h, subset, &vs, &vst, &nv));
    CT_TRY(ensure_views(h, 0));
    hipStream_t s = hs(stream);
    CT_HIP_CHECK(launch_htranspose(h, x, h->xta, s));
    CT_HIP_CHECK(launch_hfp(h, x, h->xta, vs, vst, nv, HFP_PLAIN, 0, nullptr, nullptr, 1.f, p, s));
    return CT_OK;
}

ct_status ct_helix_back(ct_helix *h, int subset, const float *r, float *x, void *stream)
{
    if (!h || !r || !x) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    int vs, vst, nv;
    CT_TRY(subset_of(h, subset, &vs, &vst, &nv));
    CT_TRY(ensure_views(h, nv));
    hipStream_t s = hs(stream);
    CT_HIP_CHECK(launch_hprescale(h, r, vs, vst, nv, h->r, s));
    CT_HIP_CHECK(launch_hbp(h, h->r, vs, vst, nv, x, 0, s));
    return CT_OK;
}

ct_status ct_helix_solve(ct_helix *h, const ct_rlalm_params *p, const float *y, const float *w, float *x,
                         void *stream)
{
    if (!h || !y || !w || !x) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    CT_TRY(check_params(p));
    if (p->algorithm != 1) return fail(CT_ERR_UNSUPPORTED, "the 3-D solver runs Algorithm 1 only");
    if (p->kappa) return fail(CT_ERR_UNSUPPORTED, "certainty weights are not available in 3-D");
    if (p->start != 0 && p->start != 1) return fail(CT_ERR_UNSUPPORTED, "the 3-D solver starts from x0 or zero");
    const ct_helix_desc &d = h->desc;
    const int M = d.nsubsets, nvm = d.nviews / M;
    hipStream_t s = hs(stream);
    const size_t nvox = h->nvox;
    CT_TRY(ensure_views(h, nvm));
    CT_TRY(hx_alloc(&h->xa, nvox));
    CT_TRY(hx_alloc(&h->xb, nvox));
    CT_TRY(hx_alloc(&h->xtb, nvox));
    CT_TRY(hx_alloc(&h->gv, nvox));
    CT_TRY(hx_alloc(&h->h, nvox));
    CT_TRY(hx_alloc(&h->dl, nvox));
    CT_TRY(hx_alloc(&h->zeta, nvox));
    const std::vector<int> order = subset_order(M, p->subset_order);
    HelixUpdate U;
    U.nx = d.nx;
    U.ny = d.ny;
    U.nz = d.nz;
    U.alpha = (float)p->alpha;
    U.potential = p->potential;
    U.huber = p->huber;
    U.delta = (float)p->delta;
    U.idelta = 1.f / U.delta;
    U.beta = (float)p->beta;
    // D_L = dl_scale * sum_m A_m' (w_m .* A_m 1)
    for (int m = 0; m < M; ++m) {
        // the ones pass reads no volume; zeta stands in as a valid pointer
        CT_HIP_CHECK(launch_hfp(h, h->zeta, h->zeta, m, M, nvm, HFP_WEIGHTED_ONES, 1, nullptr, w, 1.f, h->r, s));
        CT_HIP_CHECK(launch_hbp(h, h->r, m, M, nvm, h->dl, m > 0, s));
    }
    if (p->dl_scale != 1.0) CT_HIP_CHECK(launch_scale(h->dl, nvox, (float)p->dl_scale, s));
    // x^0 = max(x, 0) (or zero) in A, then zeta on the last subset of the order (or all views), g, h
    CT_HIP_CHECK(launch_hupd(h, U, HUPD_CLIP, p->start == 1, x, 0.f, 0.f, h->xa, h->xta, s));
    if (p->init_full) {
        for (int m = 0; m < M; ++m) {
            CT_HIP_CHECK(launch_hfp(h, h->xa, h->xta, m, M, nvm, HFP_RESIDUAL, 1, y, w, 1.f, h->r, s));
            CT_HIP_CHECK(launch_hbp(h, h->r, m, M, nvm, h->zeta, m > 0, s));
        }
    } else {
        const int m = order[(size_t)M - 1];
        CT_HIP_CHECK(launch_hfp(h, h->xa, h->xta, m, M, nvm, HFP_RESIDUAL, 1, y, w, (float)M, h->r, s));
        CT_HIP_CHECK(launch_hbp(h, h->r, m, M, nvm, h->zeta, 0, s));
    }
    CT_HIP_CHECK(launch_hupd(h, U, HUPD_INIT, 0, h->xa, 0.f, 0.f, nullptr, nullptr, s));
    const long long nsub = (long long)p->niters * M;
    float *xc = h->xa, *xcT = h->xta, *xo = h->xb, *xoT = h->xtb;
    if (nsub > 0) {
        // x^1 from the state at t = 0
        CT_HIP_CHECK(launch_hupd(h, U, HUPD_XSTEP, 0, xc, (float)rho_value(0, p), 0.f, xo, xoT, s));
        std::swap(xc, xo);
        std::swap(xcT, xoT);
        for (long long t = 0; t < nsub; ++t) {
            const int m = order[(size_t)(t % M)];
            CT_HIP_CHECK(launch_hfp(h, xc, xcT, m, M, nvm, HFP_RESIDUAL, 1, y, w, (float)M, h->r, s));
            CT_HIP_CHECK(launch_hbp(h, h->r, m, M, nvm, h->zeta, 0, s));
            CT_HIP_CHECK(launch_hupd(h, U, HUPD_FULL, 0, xc, (float)rho_value(t, p), (float)rho_value(t + 1, p), xo,
                                     xoT, s));
            std::swap(xc, xo);
            std::swap(xcT, xoT);
        }
        // x^(nsub) is the input of the last projection: the buffer before the last swap
        std::swap(xc, xo);
    }
    CT_HIP_CHECK(hipMemcpyAsync(x, xc, nvox * sizeof(float), hipMemcpyDeviceToDevice, s));
    CT_HIP_CHECK(launch_trace_reduce(x, nullptr, h->gv, h->h, d.nx, d.ny * d.nz, 1.f, 1.f, 0.f, h->red + kRedTrace, s));
    double host[kTraceOut];
    CT_HIP_CHECK(hipMemcpyAsync(host, h->red + kRedTrace, sizeof(host), hipMemcpyDeviceToHost, s));
    CT_HIP_CHECK(hipStreamSynchronize(s));
    if (host[2] != 0.0) return fail(CT_ERR_DIVERGED, "non-finite values in the final 3-D state");
    return CT_OK;
}

}  // extern "C"
