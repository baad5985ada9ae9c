// Learned warm start: a BF16 U-Net on the gfx950 matrix cores (include/ct_unet.h).
//
// The network maps the FBP-like image of a scan (units of mu_water) to a start image for the solve.
//
// Layout. Activations and their gradients are bfloat16 NHWC ([n][h][w][c], channels fastest); sums are
// float32. 3x3 convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (D[16 x 16] += A[16 x 32] *
// B[32 x 16]; lane l holds A[l%16][8(l/16) .. +7], B[8(l/16) .. +7][l%16] and D[4(l/16) + j][l%16]):
//   forward        D[c_out][pixel] = sum over (tap, c_in) of W[c_out][tap][c_in] * in[pixel + tap][c_in]
//   input gradient the same kernel on the output gradient with the weights stored [c_in][8 - tap][c_out]
//   weight gradient D[c_out][c_in] (one tap) = sum over pixels of dz[pixel][c_out] in[pixel + tap][c_in],
//                  split over pixel ranges (fixed-order reduction, no atomics); operand tiles are
//                  transposed through LDS so that every fragment is one 16-byte LDS read.
// The forward and input-gradient kernels read each operand fragment with one 16-byte load straight
// from memory (8 consecutive channels of one pixel, or of one weight row); the decoder's first
// convolution reads its concatenated input from two tensors, the upsampled one at half resolution
// (nearest neighbour: pixel (y, x) reads (y/2, x/2)), so neither the concatenation nor the upsampled
// tensor is materialised. The one-channel input layer and the 1x1 output layer are plain FP32 VALU
// kernels (9 and 32 multiply-adds per pixel). Parameters are kept in float32 (canonical layout) with
// Adam's moments; the bfloat16 weight copies in both GEMM layouts are refreshed after every update.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ct_internal.hpp"
#include "ct_unet_plan.hpp"
#include "../../include/ct_unet.h"

namespace ct {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

using unet_plan::kLayers;
using unet_plan::kShape;

// Input channels [0, c0) come from src0 (c0 channels; half resolution when up0), [c0, c0 + c1) from
// src1 (c1 channels, full resolution).
struct ConvSrc {
    const bf16 *src0;
    int c0, up0;
    const bf16 *src1;
    int c1;
};

__device__ __forceinline__ const bf16 *src_ptr(const ConvSrc &S, int ci0, int n, int y, int x, int h, int w)
{
    if (ci0 < S.c0) {
        if (S.up0) return S.src0 + (((size_t)n * (h >> 1) + (y >> 1)) * (w >> 1) + (x >> 1)) * S.c0 + ci0;
        return S.src0 + (((size_t)n * h + y) * w + x) * S.c0 + ci0;
    }
    return S.src1 + (((size_t)n * h + y) * w + x) * S.c1 + (ci0 - S.c0);
}

// 3x3 convolution, wave tile 32 output channels x 64 pixels. KS = 1: four waves per workgroup on
// consecutive pixel blocks. KS = 4 (layers with few tiles, the deep levels): the four waves share one
// tile and split the (tap, 32-channel chunk) steps into quarters; their partial tiles are added in LDS in
// a fixed order, wave w finishing pixel sub-block w. FWD: out = relu(conv + bias). !FWD (input gradient):
// out = conv * (mask > 0) (mask optional). Requires c_in, c_out multiples of 32. The pixel count n*h*w
// is arbitrary (deep levels of small images hold a handful of pixels): lanes past the last pixel read
// the last pixel's data and store nothing.
template <bool FWD, int KS>
__global__ __launch_bounds__(256) void k_conv3x3(ConvSrc S, const bf16 *__restrict__ wt, const float *__restrict__ bias,
                                                 const bf16 *__restrict__ mask, bf16 *__restrict__ out, int n, int h,
                                                 int w, int cout)
{
    __shared__ f32x4 red[KS > 1 ? KS * 8 * 64 : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cin = S.c0 + S.c1;
    const int hw = h * w, npix = n * hw;
    const int p0 = KS > 1 ? blockIdx.x * 64 : (blockIdx.x * 4 + wave) * 64;
    if (p0 >= npix) return;   // (KS > 1: the same for every wave of the workgroup)
    const int co0 = blockIdx.y * 32;
    const int g = lane >> 4, r = lane & 15;
    int pn[4], py[4], px[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int p = min(p0 + 16 * s + r, npix - 1);
        pn[s] = p / hw;
        const int rem = p - pn[s] * hw;
        py[s] = rem / w;
        px[s] = rem - py[s] * w;
    }
    f32x4 acc[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[m][s] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero8 = {};
    // steps (tap, chunk) in the order tap-major; this wave's range
    const int nch = cin / 32, T = 9 * nch;
    const int it0 = KS > 1 ? (wave * T) / KS : 0, it1 = KS > 1 ? ((wave + 1) * T) / KS : T;
    for (int it = it0; it < it1; ++it) {
        const int tap = it / nch, ci0 = (it - tap * nch) * 32;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        int ny_[4], nx_[4];
        bool ok[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int yy = py[s] + dy, xx = px[s] + dx;
            ok[s] = yy >= 0 && yy < h && xx >= 0 && xx < w;
            ny_[s] = ok[s] ? yy : py[s];   // in-range address for masked lanes
            nx_[s] = ok[s] ? xx : px[s];
        }
        bf16x8 a[2], b[4];
#pragma unroll
        for (int m = 0; m < 2; ++m)
            a[m] = *reinterpret_cast<const bf16x8 *>(wt + ((size_t)(co0 + 16 * m + r) * 9 + tap) * cin + ci0 + 8 * g);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bf16x8 v = *reinterpret_cast<const bf16x8 *>(src_ptr(S, ci0, pn[s], ny_[s], nx_[s], h, w) + 8 * g);
            b[s] = ok[s] ? v : zero8;
        }
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[m][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[s], acc[m][s], 0, 0, 0);
    }
    if (KS > 1) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int s = 0; s < 4; ++s) red[((wave * 2 + m) * 4 + s) * 64 + lane] = acc[m][s];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            f32x4 t = red[((0 * 2 + m) * 4 + wave) * 64 + lane];
#pragma unroll
            for (int k = 1; k < KS; ++k) t += red[((k * 2 + m) * 4 + wave) * 64 + lane];
            acc[m][0] = t;   // this wave's pixel sub-block, held in slot 0
        }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int co = co0 + 16 * m + 4 * g;
#pragma unroll
        for (int s = 0; s < (KS > 1 ? 1 : 4); ++s) {
            const int sb = KS > 1 ? wave : s;   // pixel sub-block
            if (p0 + 16 * sb + r >= npix) continue;
            const size_t o = (size_t)(p0 + 16 * sb + r) * cout + co;
            bf16x4 v;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float t = acc[m][s][j];
                if (FWD) t = fmaxf(t + bias[co + j], 0.f);
                else if (mask) t = (float)mask[o + j] > 0.f ? t : 0.f;
                v[j] = (bf16)t;
            }
            *reinterpret_cast<bf16x4 *>(out + o) = v;
        }
    }
}

// The same 3x3 convolution for large images, with the input staged in LDS: a workgroup computes 32 output
// channels of a 16 x 16 pixel tile (wave w: tile rows 4w .. 4w + 3, one 16-pixel row per operand block).
// For each 32-channel chunk the 18 x 18 input tile (one-pixel halo, zero outside the image) is loaded
// once into LDS, 64 bytes per pixel, and the nine taps read their 16-byte fragments from there, so each
// input value is read from memory once per chunk instead of once per tap and wave; the chunk's weights
// are staged alike, once per workgroup. FWD / !FWD as in k_conv3x3. Images of n planes; grid (tiles,
// c_out / 32).
constexpr int CT_T = 16;                     // tile width (pixels; one operand block per tile row)
constexpr int CT_HX = CT_T + 2;              // with halo
// TY: tile height, 16 (four rows per wave) or 8 (two rows per wave, for layers with few tiles)
// pooled (forward, may be null): also writes the 2 x 2 average of the output (h, w even), as k_pool would.
template <bool FWD, bool PF, int TY>
__global__ __launch_bounds__(256) void k_conv3x3_tile(ConvSrc S, const bf16 *__restrict__ wt,
                                                      const float *__restrict__ bias, const bf16 *__restrict__ mask,
                                                      bf16 *__restrict__ out, int n, int h, int w, int cout,
                                                      bf16 *__restrict__ pooled)
{
    constexpr int RW = TY / 4;                 // tile rows per wave
    constexpr int HY = TY + 2;                 // haloed rows
    __shared__ bf16x8 tile[HY * CT_HX * 4];    // [hy][hx][8-channel group]
    constexpr int WP = 9 * 4 + 1;              // weight row pitch (16-byte units), padded against bank conflicts
    __shared__ bf16x8 wts[32 * WP];            // [c_out of the block][tap][8-channel group]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cin = S.c0 + S.c1;
    const int tx = (w + CT_T - 1) / CT_T, ty = (h + TY - 1) / TY;
    int t = blockIdx.x;
    const int tix = t % tx;
    t /= tx;
    const int tiy = t % ty;
    const int pn = t / ty;
    const int x0 = tix * CT_T, y0 = tiy * TY;
    const int co0 = blockIdx.y * 32;
    const int g = lane >> 4, r = lane & 15;
    f32x4 acc[2][RW];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int s = 0; s < RW; ++s) acc[m][s] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero8 = {};
    auto taps = [&]() {
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;   // offsets into the haloed tile
            bf16x8 a[2], b[RW];
#pragma unroll
            for (int m = 0; m < 2; ++m) a[m] = wts[(16 * m + r) * WP + tap * 4 + g];
#pragma unroll
            for (int s = 0; s < RW; ++s) b[s] = tile[((RW * wave + s + dy) * CT_HX + r + dx) * 4 + g];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int s = 0; s < RW; ++s)
                    acc[m][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[s], acc[m][s], 0, 0, 0);
        }
    };
    if constexpr (PF) {
        // A chunk's input tile and weights go through registers: the next chunk's loads are issued before
        // the current chunk's taps, so that their latency overlaps the matrix work (ceil(HY * 18 * 4 / 256)
        // and ceil(32 * 9 * 4 / 256) = 5 values per thread). For layers with few workgroups per CU, which
        // have no other workgroup to run during a chunk's loads.
        constexpr int NT = (HY * CT_HX * 4 + 255) / 256, NW = (32 * 9 * 4 + 255) / 256;
        bf16x8 pt[NT], pw[NW];
        auto load_chunk = [&](int ci0) {
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                const int v = threadIdx.x + 256 * i;
                const int px = v >> 2, part = v & 3;
                const int yy = y0 - 1 + px / CT_HX, xx = x0 - 1 + px % CT_HX;
                pt[i] = zero8;
                if (v < HY * CT_HX * 4 && yy >= 0 && yy < h && xx >= 0 && xx < w)
                    pt[i] = *reinterpret_cast<const bf16x8 *>(src_ptr(S, ci0 + 8 * part, pn, yy, xx, h, w));
            }
#pragma unroll
            for (int i = 0; i < NW; ++i) {   // the chunk's weights
                const int v = threadIdx.x + 256 * i;
                const int co = v / 36, rem = v % 36;
                if (v < 32 * 9 * 4)
                    pw[i] = *reinterpret_cast<const bf16x8 *>(wt + ((size_t)(co0 + co) * 9 + rem / 4) * cin + ci0 +
                                                              8 * (rem % 4));
            }
        };
        load_chunk(0);
        for (int ci0 = 0; ci0 < cin; ci0 += 32) {
            __syncthreads();   // the previous chunk's reads are done
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                const int v = threadIdx.x + 256 * i;
                if (v < HY * CT_HX * 4) tile[v] = pt[i];
            }
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const int v = threadIdx.x + 256 * i;
                if (v < 32 * 9 * 4) wts[(v / 36) * WP + v % 36] = pw[i];
            }
            __syncthreads();
            if (ci0 + 32 < cin) load_chunk(ci0 + 32);
            taps();
        }
    } else {
        for (int ci0 = 0; ci0 < cin; ci0 += 32) {
            __syncthreads();   // the previous chunk's reads are done
            for (int v = threadIdx.x; v < HY * CT_HX * 4; v += 256) {
                const int px = v >> 2, part = v & 3;
                const int yy = y0 - 1 + px / CT_HX, xx = x0 - 1 + px % CT_HX;
                bf16x8 val = zero8;
                if (yy >= 0 && yy < h && xx >= 0 && xx < w)
                    val = *reinterpret_cast<const bf16x8 *>(src_ptr(S, ci0 + 8 * part, pn, yy, xx, h, w));
                tile[v] = val;
            }
            for (int v = threadIdx.x; v < 32 * 9 * 4; v += 256) {   // the chunk's weights, staged alike
                const int co = v / 36, rem = v % 36;
                wts[co * WP + rem] = *reinterpret_cast<const bf16x8 *>(wt + ((size_t)(co0 + co) * 9 + rem / 4) * cin +
                                                                       ci0 + 8 * (rem % 4));
            }
            __syncthreads();
            taps();
        }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int co = co0 + 16 * m + 4 * g;
#pragma unroll
        for (int s = 0; s < RW; ++s) {
            const int yy = y0 + RW * wave + s, xx = x0 + r;
            if (yy >= h || xx >= w) continue;
            const size_t o = (((size_t)pn * h + yy) * w + xx) * cout + co;
            bf16x4 v;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float tv = acc[m][s][j];
                if (FWD) tv = fmaxf(tv + bias[co + j], 0.f);
                else if (mask) tv = (float)mask[o + j] > 0.f ? tv : 0.f;
                v[j] = (bf16)tv;
            }
            *reinterpret_cast<bf16x4 *>(out + o) = v;
        }
        if (FWD && pooled) {
            // 2 x 2 average of the stored (rounded) outputs: rows s, s + 1 of this lane, columns r (even) and
            // r + 1 of the next lane, added in k_pool's order; every lane takes part in the exchange
#pragma unroll
            for (int s = 0; s < RW; s += 2) {
                const int yy = y0 + RW * wave + s, xx = x0 + r;
                bf16x4 q;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float v0 = (float)(bf16)fmaxf(acc[m][s][j] + bias[co + j], 0.f);
                    const float v1 = (float)(bf16)fmaxf(acc[m][s + 1][j] + bias[co + j], 0.f);
                    const float v01 = __shfl_xor(v0, 1), v11 = __shfl_xor(v1, 1);
                    q[j] = (bf16)(0.25f * (((v0 + v01) + v1) + v11));
                }
                if ((r & 1) == 0 && yy + 1 < h && xx + 1 < w) {
                    const int ho = h / 2, wo = w / 2;
                    *reinterpret_cast<bf16x4 *>(pooled + (((size_t)pn * ho + yy / 2) * wo + xx / 2) * cout + co) = q;
                }
            }
        }
    }
}

// Weight gradient partials of a 3x3 convolution: part[split][c_out][tap][c_in] over the pixels
// [split * pps, min((split + 1) * pps, npix)) (pps a multiple of 64; the last chunk of 64 may be
// partial, its missing pixels count as zero). One wave per (split, tap, 32 x 32 channel block); grid
// (splits, 9, (c_out / 32) * (c_in / 32)). Each LDS fill holds 64 pixels of both operands (two MFMA
// K-steps per pair of barriers).
__global__ __launch_bounds__(64) void k_conv3x3_wgrad(ConvSrc S, const bf16 *__restrict__ dz, int cout, int n, int h,
                                                      int w, int pps, float *__restrict__ part)
{
    constexpr int KC = 64;        // pixels per LDS fill
    constexpr int LD = KC + 8;    // padded LDS row (bf16): 144 bytes keeps rows 16-byte aligned
    __shared__ __attribute__((aligned(16))) bf16 sA[32 * LD];   // [c_out][pixel]
    __shared__ __attribute__((aligned(16))) bf16 sB[32 * LD];   // [c_in][pixel]
    const int lane = threadIdx.x;
    const int cin = S.c0 + S.c1;
    const int split = blockIdx.x, tap = blockIdx.y;
    const int nci = cin / 32;
    const int co0 = (blockIdx.z / nci) * 32, ci0 = (blockIdx.z % nci) * 32;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int hw = h * w, npix = n * hw;
    const int pb = split * pps, pe = min(pb + pps, npix);
    const int g = lane >> 4, r = lane & 15;
    f32x4 acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[m][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero8 = {};
    for (int pc = pb; pc < pe; pc += KC) {
        // 64 pixels x 32 channels of each operand: 256 16-byte pieces, four per lane; piece t of lane q is
        // channel group t of pixel q, so that each transposing write covers 64 consecutive pixels of one
        // channel (neighbouring LDS halves, no bank conflicts between the channel groups)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int q = lane, c8 = 8 * t;
            const bool in = pc + q < pe;
            const int p = in ? pc + q : pe - 1;
            const bf16x8 va0 = *reinterpret_cast<const bf16x8 *>(dz + (size_t)p * cout + co0 + c8);
            const int pn = p / hw, rem = p - pn * hw, py = rem / w, px = rem - py * w;
            const int yy = py + dy, xx = px + dx;
            const bool ok = in && yy >= 0 && yy < h && xx >= 0 && xx < w;
            const bf16x8 vb0 = *reinterpret_cast<const bf16x8 *>(
                src_ptr(S, ci0, pn, ok ? yy : py, ok ? xx : px, h, w) + c8);
            const bf16x8 va = in ? va0 : zero8;
            const bf16x8 vb = ok ? vb0 : zero8;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                sA[(c8 + i) * LD + q] = va[i];
                sB[(c8 + i) * LD + q] = vb[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KC / 32; ++kk) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int m = 0; m < 2; ++m) a[m] = *reinterpret_cast<const bf16x8 *>(sA + (16 * m + r) * LD + 32 * kk + 8 * g);
#pragma unroll
            for (int q = 0; q < 2; ++q) b[q] = *reinterpret_cast<const bf16x8 *>(sB + (16 * q + r) * LD + 32 * kk + 8 * g);
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc[m][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[q], acc[m][q], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int co = co0 + 16 * m + 4 * g + j, ci = ci0 + 16 * q + r;
                part[(((size_t)split * cout + co) * 9 + tap) * cin + ci] = acc[m][q][j];
            }
}

// Weight gradient partials of a 3x3 convolution, all nine taps per workgroup, for images whose width is a
// multiple of 64: part[split][c_out][tap][c_in] over the split's 64-pixel row segments [split * cps,
// min((split + 1) * cps, segments)). Workgroup = 4 waves = the 2 x 2 16 x 16 tiles of a 32 (c_out) x 32
// (c_in) block, grid (splits, (c_out / 32) * (c_in / 32)). Per segment the output gradient (32 channels x
// 64 pixels) and the input rows y - 1, y, y + 1 over the segment's pixels with one halo pixel on each side
// are staged in LDS, transposed to pixel-contiguous rows (the matrix cores take 8 consecutive pixels of
// one channel per lane). A wave reads its A operand once per 32-pixel K-step and, per input row, one
// window of 10 pixels per lane, from which the three horizontal taps' B operands come: pixels 0-7 (dx = -1),
// 1-8 (a 16-bit shift across the window's words, dx = 0) and 2-9 (dx = +1).
__global__ __launch_bounds__(256) void k_conv3x3_wgrad9(ConvSrc S, const bf16 *__restrict__ dz, int cout, int n,
                                                        int h, int w, int cps, float *__restrict__ part)
{
    constexpr int LD = 72;   // padded LDS row (bf16): 144 bytes keeps rows 16-byte aligned; 66 pixels used
    __shared__ __attribute__((aligned(16))) bf16 sA[32 * LD];       // [c_out][pixel]
    __shared__ __attribute__((aligned(16))) bf16 sB[3 * 32 * LD];   // [input row][c_in][halo pixel]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cin = S.c0 + S.c1;
    const int nci = cin / 32;
    const int co0 = (blockIdx.y / nci) * 32, ci0 = (blockIdx.y % nci) * 32;
    const int segs_row = w / 64, nseg = n * h * segs_row;
    const int s0 = blockIdx.x * cps, s1 = min(s0 + cps, nseg);
    const int g = lane >> 4, r = lane & 15;
    const int mt = wave & 1, qt = wave >> 1;   // the wave's c_out and c_in 16-tiles
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero8 = {};
    for (int sg = s0; sg < s1; ++sg) {
        const int row = sg / segs_row, px0 = (sg - row * segs_row) * 64;
        const int pn = row / h, py = row - pn * h;
        {   // output gradient: thread -> (pixel tid % 64, channels 8 (tid / 64) ..), 64 x 4 pieces: each wave
            // writes one channel group's rows over 64 consecutive pixels (neighbouring LDS halves)
            const int q = tid & 63, c8 = (tid >> 6) * 8;
            const bf16x8 v =
                *reinterpret_cast<const bf16x8 *>(dz + (((size_t)pn * h + py) * w + px0 + q) * cout + co0 + c8);
#pragma unroll
            for (int i = 0; i < 8; ++i) sA[(c8 + i) * LD + q] = v[i];
        }
        // input rows: 3 rows x 66 pixels x 4 channel groups
        for (int idx = tid; idx < 3 * 66 * 4; idx += 256) {
            const int c8 = (idx / 198) * 8, pr = idx % 198;   // channel group major, as above
            const int ry = pr / 66, j = pr - ry * 66;
            const int yy = py + ry - 1, xx = px0 + j - 1;
            const bool ok = yy >= 0 && yy < h && xx >= 0 && xx < w;
            const bf16x8 v = ok ? *reinterpret_cast<const bf16x8 *>(src_ptr(S, ci0, pn, yy, xx, h, w) + c8) : zero8;
#pragma unroll
            for (int i = 0; i < 8; ++i) sB[(ry * 32 + c8 + i) * LD + j] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(sA + (16 * mt + r) * LD + 32 * kk + 8 * g);
#pragma unroll
            for (int ry = 0; ry < 3; ++ry) {
                const bf16 *wp = sB + (ry * 32 + 16 * qt + r) * LD + 32 * kk + 8 * g;
                const uint4 w0 = *reinterpret_cast<const uint4 *>(wp);
                const unsigned w4 = *reinterpret_cast<const unsigned *>(wp + 8);
                const uint4 bc = {__builtin_amdgcn_alignbit(w0.y, w0.x, 16), __builtin_amdgcn_alignbit(w0.z, w0.y, 16),
                                  __builtin_amdgcn_alignbit(w0.w, w0.z, 16), __builtin_amdgcn_alignbit(w4, w0.w, 16)};
                const uint4 bp = {w0.y, w0.z, w0.w, w4};
                acc[3 * ry] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, w0), acc[3 * ry], 0,
                                                                      0, 0);
                acc[3 * ry + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, bc),
                                                                          acc[3 * ry + 1], 0, 0, 0);
                acc[3 * ry + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, bp),
                                                                          acc[3 * ry + 2], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = co0 + 16 * mt + 4 * g + j, ci = ci0 + 16 * qt + r;
            part[(((size_t)blockIdx.x * cout + co) * 9 + t) * cin + ci] = acc[t][j];
        }
}

// grad[co][ci][dy][dx] (canonical) = sum over splits of part[split][co][tap][ci]: 32 outputs per workgroup,
// consecutive in the partials' layout (so that each split's reads are coalesced; the one write per output
// goes to its canonical place), 8 lanes over the splits (k = lane, lane + 8, ...), added in lane order.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *__restrict__ part, int nsplit, int cout, int cin,
                                                      float *__restrict__ grad)
{
    __shared__ float red[8][32];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const size_t o = (size_t)blockIdx.x * 32 + tx;   // index in [c_out][tap][c_in]
    const size_t total = (size_t)cout * cin * 9;
    float s = 0.f;
    if (o < total) {
        // eight of the lane's partials in flight at once, then added in split order
        int k = ty;
        for (; k + 56 < nsplit; k += 64) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(k + 8 * u) * total + o];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; k < nsplit; k += 8) s += part[(size_t)k * total + o];
    }
    red[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && o < total) {
        float t = red[0][tx];
#pragma unroll
        for (int l = 1; l < 8; ++l) t += red[l][tx];
        const int ci = (int)(o % cin);
        const int tap = (int)((o / cin) % 9);
        const int co = (int)(o / (9 * (size_t)cin));
        grad[((size_t)co * cin + ci) * 9 + tap] = t;
    }
}

// Bias gradient partials: part[split][c] = sum over the split's pixels of dz[p][c] (c a multiple of 8,
// c / 8 dividing 256). The 256 threads are c / 8 channel groups (16-byte loads) x 2048 / c pixel lanes;
// the pixel lanes' sums are added in LDS in lane order.
__global__ __launch_bounds__(256) void k_bias_part(const bf16 *__restrict__ dz, int c, int npix, int pps,
                                                   float *__restrict__ part)
{
    __shared__ float red[256 * 8];
    const int ng = c / 8, nl = 256 / ng;
    const int cg = threadIdx.x % ng, pl = threadIdx.x / ng;
    const int pb = blockIdx.x * pps, pe = min(pb + pps, npix);
    float sum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int p = pb + pl;
    for (; p + 3 * nl < pe; p += 4 * nl) {   // four of the lane's pixels in flight, added in pixel order
        bf16x8 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = *reinterpret_cast<const bf16x8 *>(dz + (size_t)(p + u * nl) * c + 8 * cg);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int i = 0; i < 8; ++i) sum[i] += (float)v[u][i];
    }
    for (; p < pe; p += nl) {
        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(dz + (size_t)p * c + 8 * cg);
#pragma unroll
        for (int i = 0; i < 8; ++i) sum[i] += (float)v[i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) red[threadIdx.x * 8 + i] = sum[i];   // [pixel lane][channel]
    __syncthreads();
    for (int ch = threadIdx.x; ch < c; ch += 256) {
        float t = 0.f;
        for (int l = 0; l < nl; ++l) t += red[l * c + ch];
        part[(size_t)blockIdx.x * c + ch] = t;
    }
}

using unet_plan::bias_pps;

// out[i] = sum over k of part[k * n + i]: 32 outputs per workgroup, 8 lanes over the splits (k = lane,
// lane + 8, ...), their sums added in lane order.
__global__ __launch_bounds__(256) void k_sum_parts(const float *__restrict__ part, int nsplit, int n,
                                                   float *__restrict__ out)
{
    __shared__ float red[8][32];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int i = blockIdx.x * 32 + tx;
    float s = 0.f;
    if (i < n) {
        // eight of the lane's partials in flight at once, then added in split order
        int k = ty;
        for (; k + 56 < nsplit; k += 64) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(k + 8 * u) * n + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; k < nsplit; k += 8) s += part[(size_t)k * n + i];
    }
    red[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && i < n) {
        float t = red[0][tx];
#pragma unroll
        for (int l = 1; l < 8; ++l) t += red[l][tx];
        out[i] = t;
    }
}

// Sum of v over the 16 lanes of a wave that share lane % 4 (a butterfly: every such lane ends with the
// same bits, since each step adds the same two values on both sides).
__device__ __forceinline__ float sum16_of_4(float v)
{
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// Input layer (one channel, 32 outputs): out[p][co] = relu(b[co] + sum_tap W[co][tap] x[p + tap]).
// Four lanes per pixel, eight channels each, so that a wave's stores cover 1 KiB contiguously; the
// weights and bias are staged in LDS once per workgroup.
__global__ __launch_bounds__(256) void k_conv_in(const float *__restrict__ x, const float *__restrict__ W,
                                                 const float *__restrict__ b, bf16 *__restrict__ out, int n, int h,
                                                 int w)
{
    __shared__ float sw[32 * 9 + 32];
    for (int i = threadIdx.x; i < 32 * 9 + 32; i += 256) sw[i] = i < 32 * 9 ? W[i] : b[i - 32 * 9];
    __syncthreads();
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int hw = h * w;
    if (t >= (size_t)n * hw * 4) return;
    const int q = (int)(t & 3);
    const size_t p = t >> 2;
    const int pn = (int)(p / hw), rem = (int)(p - (size_t)pn * hw), py = rem / w, px = rem - py * w;
    float v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int yy = py + k / 3 - 1, xx = px + k % 3 - 1;
        v[k] = (yy >= 0 && yy < h && xx >= 0 && xx < w) ? x[(size_t)pn * hw + yy * w + xx] : 0.f;
    }
    bf16x8 o;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int co = 8 * q + i;
        float z = sw[32 * 9 + co];
#pragma unroll
        for (int k = 0; k < 9; ++k) z = fmaf(sw[co * 9 + k], v[k], z);
        o[i] = (bf16)fmaxf(z, 0.f);
    }
    *reinterpret_cast<bf16x8 *>(out + p * 32 + 8 * q) = o;
}

// Input layer weight / bias gradient partials part[split][320]: entries co * 9 + tap (co < 32, tap < 9)
// sum dz[p][co] x[p + tap offset], entries 288 + co sum dz[p][co]. Thread (pixel lane tid / 4, channel
// group tid % 4 of 8 channels) accumulates its pixels' 72 + 8 sums; the 16 pixel lanes of a wave are
// added by a butterfly, the four waves in LDS, in a fixed order.
__global__ __launch_bounds__(256) void k_conv_in_wgrad(const float *__restrict__ x, const bf16 *__restrict__ dz, int n,
                                                       int h, int w, int pps, float *__restrict__ part)
{
    __shared__ float red[4][320];
    const int cg = threadIdx.x & 3, pl = threadIdx.x >> 2, wave = threadIdx.x >> 6;
    const int hw = h * w, npix = n * hw;
    const int pb = blockIdx.x * pps, pe = min(pb + pps, npix);
    float sw[8][9], sb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        sb[i] = 0.f;
#pragma unroll
        for (int k = 0; k < 9; ++k) sw[i][k] = 0.f;
    }
    for (int p = pb + pl; p < pe; p += 64) {
        const int pn = p / hw, rem = p - pn * hw, py = rem / w, px = rem - py * w;
        float v[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int yy = py + k / 3 - 1, xx = px + k % 3 - 1;
            v[k] = (yy >= 0 && yy < h && xx >= 0 && xx < w) ? x[(size_t)pn * hw + yy * w + xx] : 0.f;
        }
        const bf16x8 d = *reinterpret_cast<const bf16x8 *>(dz + (size_t)p * 32 + 8 * cg);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float di = (float)d[i];
            sb[i] += di;
#pragma unroll
            for (int k = 0; k < 9; ++k) sw[i][k] = fmaf(di, v[k], sw[i][k]);
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        sb[i] = sum16_of_4(sb[i]);
#pragma unroll
        for (int k = 0; k < 9; ++k) sw[i][k] = sum16_of_4(sw[i][k]);
    }
    if ((threadIdx.x & 63) < 4) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int co = 8 * cg + i;
            red[wave][288 + co] = sb[i];
#pragma unroll
            for (int k = 0; k < 9; ++k) red[wave][co * 9 + k] = sw[i][k];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 320; t += 256)
        part[(size_t)blockIdx.x * 320 + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

// Output layer: out[p] = x[p] + b + sum_c W[c] a[p][c]. With a target: dy[p] = gscale (out - target)
// on masked pixels (0 elsewhere) and lpart[block] = sum over the block's masked pixels of
// (1000 (out - target))^2 in FP64.
__global__ __launch_bounds__(256) void k_conv_out(const bf16 *__restrict__ a, const float *__restrict__ x,
                                                  const float *__restrict__ W, const float *__restrict__ b,
                                                  float *__restrict__ out, const float *__restrict__ target,
                                                  const unsigned char *__restrict__ mask, float gscale,
                                                  float *__restrict__ dy, double *__restrict__ lpart, int npix, int hw)
{
    __shared__ double red[256];
    const int p = blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (p < npix) {
        float o = x[p] + b[0];
        for (int c8 = 0; c8 < 32; c8 += 8) {
            const bf16x8 v = *reinterpret_cast<const bf16x8 *>(a + (size_t)p * 32 + c8);
#pragma unroll
            for (int i = 0; i < 8; ++i) o = fmaf(W[c8 + i], (float)v[i], o);
        }
        out[p] = o;
        if (target) {
            const bool m = mask[p % hw] != 0;
            const float d = o - target[p];
            dy[p] = m ? gscale * d : 0.f;
            if (m) l = 1e6 * (double)d * (double)d;
        }
    }
    if (target) {
        red[threadIdx.x] = l;
        __syncthreads();
        for (int k = 128; k > 0; k >>= 1) {
            if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
    }
}

// Output layer backward: dz[p][c] = dy[p] W[c] (a[p][c] > 0); gradient partials part[split][33]
// (32 weights, then the bias): thread c < 32 sums dy[p] a[p][c], thread 32 sums dy[p].
__global__ void k_conv_out_back(const float *__restrict__ dy, const float *__restrict__ W, const bf16 *__restrict__ a,
                                bf16 *__restrict__ dz, int npix)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const float d = dy[p];
    for (int c8 = 0; c8 < 32; c8 += 8) {
        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(a + (size_t)p * 32 + c8);
        bf16x8 o;
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = (bf16)((float)v[i] > 0.f ? d * W[c8 + i] : 0.f);
        *reinterpret_cast<bf16x8 *>(dz + (size_t)p * 32 + c8) = o;
    }
}

// Output layer gradient partials part[split][33]: entry c < 32 sums dy[p] a[p][c], entry 32 sums dy[p].
// Thread (pixel lane tid / 4, channel group tid % 4) as in k_conv_in_wgrad.
__global__ __launch_bounds__(256) void k_conv_out_wgrad(const float *__restrict__ dy, const bf16 *__restrict__ a,
                                                        int npix, int pps, float *__restrict__ part)
{
    __shared__ float red[4][33];
    const int cg = threadIdx.x & 3, pl = threadIdx.x >> 2, wave = threadIdx.x >> 6;
    const int pb = blockIdx.x * pps, pe = min(pb + pps, npix);
    float sum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, sb = 0.f;
    for (int p = pb + pl; p < pe; p += 64) {
        const float d = dy[p];
        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(a + (size_t)p * 32 + 8 * cg);
#pragma unroll
        for (int i = 0; i < 8; ++i) sum[i] = fmaf(d, (float)v[i], sum[i]);
        sb += d;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) sum[i] = sum16_of_4(sum[i]);
    sb = sum16_of_4(sb);
    if ((threadIdx.x & 63) < 4) {
#pragma unroll
        for (int i = 0; i < 8; ++i) red[wave][8 * cg + i] = sum[i];
        if (cg == 0) red[wave][32] = sb;
    }
    __syncthreads();
    if (threadIdx.x < 33)
        part[(size_t)blockIdx.x * 33 + threadIdx.x] =
            ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// 2x2 average pooling, NHWC bf16: one thread per (output pixel, 8 channels).
__global__ void k_pool(const bf16 *__restrict__ in, bf16 *__restrict__ out, int n, int ho, int wo, int c)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c8n = c / 8;
    const size_t total = (size_t)n * ho * wo * c8n;
    if (i >= total) return;
    const int c8 = (int)(i % c8n) * 8;
    const size_t po = i / c8n;
    const int x = (int)(po % wo), y = (int)((po / wo) % ho), nn = (int)(po / ((size_t)wo * ho));
    const int wi = 2 * wo;
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const bf16x8 v = *reinterpret_cast<const bf16x8 *>(
                in + (((size_t)nn * 2 * ho + 2 * y + a) * wi + 2 * x + b) * c + c8);
#pragma unroll
            for (int k = 0; k < 8; ++k) s[k] += (float)v[k];
        }
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = (bf16)(0.25f * s[k]);
    *reinterpret_cast<bf16x8 *>(out + po * c + c8) = o;
}

// Gradient through the nearest upsampling into a ReLU output: dz[n][y][x][c] = (sum over the 2x2
// block of dcat[.][.][.][c]) * (act[n][y][x][c] > 0), c < c0; dcat has ccat channels at 2x resolution.
__global__ void k_up_back(const bf16 *__restrict__ dcat, int ccat, const bf16 *__restrict__ act, bf16 *__restrict__ dz,
                          int n, int hl, int wl, int c0)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c8n = c0 / 8;
    const size_t total = (size_t)n * hl * wl * c8n;
    if (i >= total) return;
    const int c8 = (int)(i % c8n) * 8;
    const size_t pl = i / c8n;
    const int x = (int)(pl % wl), y = (int)((pl / wl) % hl), nn = (int)(pl / ((size_t)wl * hl));
    const int wh = 2 * wl;
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const bf16x8 v = *reinterpret_cast<const bf16x8 *>(
                dcat + (((size_t)nn * 2 * hl + 2 * y + a) * wh + 2 * x + b) * ccat + c8);
#pragma unroll
            for (int k = 0; k < 8; ++k) s[k] += (float)v[k];
        }
    const bf16x8 av = *reinterpret_cast<const bf16x8 *>(act + pl * c0 + c8);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = (bf16)((float)av[k] > 0.f ? s[k] : 0.f);
    *reinterpret_cast<bf16x8 *>(dz + pl * c0 + c8) = o;
}

// Encoder output gradient: dz = (skip part of dcat + pooling backward of dpool) * (act > 0).
// act / dz: [n][h][w][c]; dcat: [n][h][w][ccat], skip channels at [c0, c0 + c); dpool: [n][h/2][w/2][c].
__global__ void k_skip_combine(const bf16 *__restrict__ dcat, int ccat, int c0, const bf16 *__restrict__ dpool,
                               const bf16 *__restrict__ act, bf16 *__restrict__ dz, int n, int h, int w, int c)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c8n = c / 8;
    const size_t total = (size_t)n * h * w * c8n;
    if (i >= total) return;
    const int c8 = (int)(i % c8n) * 8;
    const size_t p = i / c8n;
    const int x = (int)(p % w), y = (int)((p / w) % h), nn = (int)(p / ((size_t)w * h));
    const bf16x8 vs = *reinterpret_cast<const bf16x8 *>(dcat + p * ccat + c0 + c8);
    const bf16x8 vp = *reinterpret_cast<const bf16x8 *>(
        dpool + (((size_t)nn * (h / 2) + y / 2) * (w / 2) + x / 2) * c + c8);
    const bf16x8 va = *reinterpret_cast<const bf16x8 *>(act + p * c + c8);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = (bf16)((float)va[k] > 0.f ? (float)vs[k] + 0.25f * (float)vp[k] : 0.f);
    *reinterpret_cast<bf16x8 *>(dz + p * c + c8) = o;
}

__global__ void k_adam(float *__restrict__ th, float *__restrict__ m, float *__restrict__ v, const float *__restrict__ g,
                       size_t n, float lr, float bc1, float bc2)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

// bfloat16 copies of one 3x3 layer's canonical weights: wf[co][tap][ci] and wb[ci][8 - tap][co].
__global__ void k_pack(const float *__restrict__ th, int cout, int cin, bf16 *__restrict__ wf, bf16 *__restrict__ wb)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)cout * cin * 9) return;
    const int tap = (int)(i % 9);
    const int ci = (int)((i / 9) % cin);
    const int co = (int)(i / (9 * (size_t)cin));
    const bf16 v = (bf16)th[i];
    wf[((size_t)co * 9 + tap) * cin + ci] = v;
    wb[((size_t)ci * 9 + (8 - tap)) * cout + co] = v;
}

__global__ void k_scale_copy(const float *__restrict__ in, float a, float *__restrict__ out, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a * in[i];
}

__global__ void k_start(const float *__restrict__ o, float mu, float *__restrict__ x, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = mu * fmaxf(o[i], 0.f);
}

inline unsigned blocks(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

}  // namespace
}  // namespace ct

using namespace ct;

struct ct_unet {
    int max_n = 0, max_h = 0, max_w = 0;
    int device = 0;
    size_t off[kLayers + 1] = {};   // canonical offsets of each layer's weights (bias follows)
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    bf16 *wf[kLayers] = {}, *wb[kLayers] = {};
    long long step = 0;
    // activations (bf16 NHWC) per level
    bf16 *e1a = nullptr, *e1b = nullptr, *d1a = nullptr, *d1b = nullptr;
    bf16 *p1 = nullptr, *e2a = nullptr, *e2b = nullptr, *d2a = nullptr, *d2b = nullptr;
    bf16 *p2 = nullptr, *e3a = nullptr, *e3b = nullptr, *d3a = nullptr, *d3b = nullptr;
    bf16 *p3 = nullptr, *ba = nullptr, *bb = nullptr;
    float *out = nullptr;   // network output (training)
    // gradients
    bool train_alloc = false;
    bf16 *dzA[4] = {}, *dzB[4] = {}, *dcat[3] = {}, *dpool[3] = {};
    float *dy = nullptr, *part = nullptr;
    size_t part_cap = 0;
    double *lpart = nullptr;
    size_t lpart_cap = 0;
};

namespace {

template <typename T>
ct_status ualloc(T **p, size_t n)
{
    hipError_t e = hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? CT_ERR_OOM : CT_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return CT_OK;
}

template <typename T>
void ufree(T **p)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
}

size_t n_params()
{
    size_t s = 0;
    for (auto &L : kShape) s += (size_t)L[1] * L[0] * L[2] * L[2] + L[1];
    return s;
}

ct_status pack_weights(ct_unet *u, hipStream_t s)
{
    for (int l = 1; l < kLayers - 1; ++l) {
        const int ci = kShape[l][0], co = kShape[l][1];
        const size_t nw = (size_t)co * ci * 9;
        hipLaunchKernelGGL(k_pack, dim3(blocks(nw, 256)), dim3(256), 0, s, u->theta + u->off[l], co, ci, u->wf[l], u->wb[l]);
        CT_HIP_CHECK(hipGetLastError());
    }
    return CT_OK;
}

ct_status check_shape(const ct_unet *u, int n, int h, int w)
{
    if (n < 1 || n > u->max_n || h < 8 || w < 8 || h > u->max_h || w > u->max_w || h % 8 || w % 8)
        return fail(CT_ERR_INVALID_ARG, "batch shape must be 1..max_n images of 8..max size, multiples of 8");
    return CT_OK;
}

using unet_plan::kInPps;
using unet_plan::kLevel;
using unet_plan::kOutPps;
using unet_plan::wgrad9_splits;
using unet_plan::wgrad_splits;

// Largest partial-sum request of any backward launch for batches up to max_n x max_h x max_w. Every
// request grows with the pixel count, so the maximum batch bounds all smaller ones.
size_t part_need(const ct_unet *u) { return unet_plan::part_need(u->max_n, u->max_h, u->max_w); }

ct_status alloc_train(ct_unet *u)
{
    if (u->train_alloc) return CT_OK;
    u->part_cap = part_need(u);
    CT_TRY(ualloc(&u->part, u->part_cap));
    const size_t P1 = (size_t)u->max_n * u->max_h * u->max_w;
    const int ch[4] = {32, 64, 128, 256};
    for (int l = 0; l < 4; ++l) {
        const size_t P = P1 >> (2 * l);
        CT_TRY(ualloc(&u->dzA[l], P * ch[l]));
        CT_TRY(ualloc(&u->dzB[l], P * ch[l]));
    }
    const int ccat[3] = {96, 192, 384};
    const int cpool[3] = {32, 64, 128};
    for (int l = 0; l < 3; ++l) {
        CT_TRY(ualloc(&u->dcat[l], (P1 >> (2 * l)) * ccat[l]));
        CT_TRY(ualloc(&u->dpool[l], (P1 >> (2 * (l + 1))) * cpool[l]));
    }
    CT_TRY(ualloc(&u->dy, P1));
    u->train_alloc = true;
    return CT_OK;
}

// The partial-sum buffer is sized once (alloc_train) for the largest request at the maximum batch, so
// that it is never reallocated while earlier kernels on the stream may still read it.
ct_status ensure_part(ct_unet *u, size_t n)
{
    if (n <= u->part_cap) return CT_OK;
    return fail(CT_ERR_HIP, "internal: partial-sum buffer too small");
}

// The deep levels have too few 32 x 64 output tiles to fill the device: split each tile's steps over
// four waves when the tiles number fewer than 2048 (eight waves per CU).
bool split_k(size_t npix, int cout) { return ((npix + 63) / 64) * (size_t)(cout / 32) < 2048; }

// Layers with at least 64 workgroups of the LDS-tiled form (16 x 16 tiles, one workgroup per tile and 32
// output channels) use it; below four workgroups per CU it prefetches each channel chunk into registers,
// which hides the chunk loads well enough to beat the split form down to a quarter workgroup per CU.
int tiles16(int e) { return (e + 15) / 16; }
size_t tile_wgs(int n, int h, int w, int cout, int ty = 16)
{
    return (size_t)n * ((h + ty - 1) / ty) * tiles16(w) * (cout / 32);
}
bool use_tile(int n, int h, int w, int cout) { return tile_wgs(n, h, w, cout) >= 64; }
// fewer than two workgroups of 16 x 16 tiles per CU: 8-row tiles (twice the workgroups)
int tile_rows(int n, int h, int w, int cout) { return tile_wgs(n, h, w, cout) < 512 ? 8 : 16; }
bool tile_prefetch(int n, int h, int w, int cout) { return tile_wgs(n, h, w, cout, tile_rows(n, h, w, cout)) < 1024; }

// The tiled convolution for (n, h, w, c) with c output channels (forward) or input channels (data
// gradient): tile height and prefetch chosen as above.
template <bool FWD>
void launch_conv_tile(const ConvSrc &S, const bf16 *wt, const float *bias, const bf16 *mask, bf16 *out, int n, int h,
                      int w, int c, hipStream_t s, bf16 *pooled = nullptr)
{
    const int ty = tile_rows(n, h, w, c);
    dim3 grid(n * ((h + ty - 1) / ty) * tiles16(w), c / 32);
    const bool pf = tile_prefetch(n, h, w, c);
    if (ty == 8)
        hipLaunchKernelGGL((k_conv3x3_tile<FWD, true, 8>), grid, dim3(256), 0, s, S, wt, bias, mask, out, n, h, w, c,
                           pooled);
    else if (pf)
        hipLaunchKernelGGL((k_conv3x3_tile<FWD, true, 16>), grid, dim3(256), 0, s, S, wt, bias, mask, out, n, h, w, c,
                           pooled);
    else
        hipLaunchKernelGGL((k_conv3x3_tile<FWD, false, 16>), grid, dim3(256), 0, s, S, wt, bias, mask, out, n, h, w, c,
                           pooled);
}

ConvSrc one(const bf16 *src, int c) { return ConvSrc{src, c, 0, nullptr, 0}; }
ConvSrc cat(const bf16 *low, int cl, const bf16 *skip, int cs) { return ConvSrc{low, cl, 1, skip, cs}; }

// pooled (may be null): also the 2 x 2 average of the output, fused into the tiled form, else by k_pool
hipError_t conv_fwd(const ct_unet *u, int l, const ConvSrc &S, bf16 *out, int n, int h, int w, hipStream_t s,
                    bf16 *pooled = nullptr)
{
    const int cout = kShape[l][1];
    const size_t npix = (size_t)n * h * w;
    const float *bias = u->theta + u->off[l] + (size_t)cout * kShape[l][0] * 9;
    if (use_tile(n, h, w, cout)) {
        launch_conv_tile<true>(S, u->wf[l], bias, nullptr, out, n, h, w, cout, s, pooled);
        return hipGetLastError();
    } else if (split_k(npix, cout)) {
        dim3 grid(blocks(npix, 64), cout / 32);
        hipLaunchKernelGGL((k_conv3x3<true, 4>), grid, dim3(256), 0, s, S, u->wf[l], bias, nullptr, out, n, h, w, cout);
    } else {
        dim3 grid(blocks(npix, 256), cout / 32);
        hipLaunchKernelGGL((k_conv3x3<true, 1>), grid, dim3(256), 0, s, S, u->wf[l], bias, nullptr, out, n, h, w, cout);
    }
    if (pooled) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const size_t nq = (size_t)n * (h / 2) * (w / 2) * (cout / 8);
        hipLaunchKernelGGL(k_pool, dim3(blocks(nq, 256)), dim3(256), 0, s, out, pooled, n, h / 2, w / 2, cout);
    }
    return hipGetLastError();
}

// input gradient of layer l (3x3, c_in % 32 == 0) from dz, optionally masked by act
hipError_t conv_dgrad(const ct_unet *u, int l, const bf16 *dz, const bf16 *act, bf16 *out, int n, int h, int w,
                      hipStream_t s)
{
    const int cin = kShape[l][0], cout = kShape[l][1];
    const size_t npix = (size_t)n * h * w;
    if (use_tile(n, h, w, cin)) {
        launch_conv_tile<false>(one(dz, cout), u->wb[l], nullptr, act, out, n, h, w, cin, s);
    } else if (split_k(npix, cin)) {
        dim3 grid(blocks(npix, 64), cin / 32);
        hipLaunchKernelGGL((k_conv3x3<false, 4>), grid, dim3(256), 0, s, one(dz, cout), u->wb[l], nullptr, act, out, n,
                           h, w, cin);
    } else {
        dim3 grid(blocks(npix, 256), cin / 32);
        hipLaunchKernelGGL((k_conv3x3<false, 1>), grid, dim3(256), 0, s, one(dz, cout), u->wb[l], nullptr, act, out, n,
                           h, w, cin);
    }
    return hipGetLastError();
}



// weight and bias gradients of 3x3 layer l (c_in % 32 == 0) into u->grad
ct_status conv_wgrad(ct_unet *u, int l, const ConvSrc &S, const bf16 *dz, int n, int h, int w, hipStream_t s)
{
    const int cin = kShape[l][0], cout = kShape[l][1];
    const size_t npix = (size_t)n * h * w;
    int nsp;
    if (w % 64 == 0) {   // whole 64-pixel row segments: the nine-tap form
        int cps;
        wgrad9_splits(npix, cin, cout, &cps, &nsp);
        CT_TRY(ensure_part(u, (size_t)nsp * cout * 9 * cin));
        hipLaunchKernelGGL(k_conv3x3_wgrad9, dim3(nsp, (cout / 32) * (cin / 32)), dim3(256), 0, s, S, dz, cout, n, h, w,
                           cps, u->part);
    } else {
        int pps;
        wgrad_splits(npix, cin, cout, &pps, &nsp);
        CT_TRY(ensure_part(u, (size_t)nsp * cout * 9 * cin));
        hipLaunchKernelGGL(k_conv3x3_wgrad, dim3(nsp, 9, (cout / 32) * (cin / 32)), dim3(64), 0, s, S, dz, cout, n, h, w,
                           pps, u->part);
    }
    CT_HIP_CHECK(hipGetLastError());
    const size_t nw = (size_t)cout * cin * 9;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks(nw, 32)), dim3(256), 0, s, u->part, nsp, cout, cin, u->grad + u->off[l]);
    CT_HIP_CHECK(hipGetLastError());
    // bias
    const int bps = bias_pps(cout);
    const int nb = (int)((npix + bps - 1) / bps);
    CT_TRY(ensure_part(u, (size_t)nb * cout));
    hipLaunchKernelGGL(k_bias_part, dim3(nb), dim3(256), 0, s, dz, cout, (int)npix, bps, u->part);
    CT_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_sum_parts, dim3(blocks(cout, 32)), dim3(256), 0, s, u->part, nb, cout, u->grad + u->off[l] + nw);
    CT_HIP_CHECK(hipGetLastError());
    return CT_OK;
}

const float *bias_of(const ct_unet *u, int l)
{
    return u->theta + u->off[l] + (size_t)kShape[l][1] * kShape[l][0] * kShape[l][2] * kShape[l][2];
}

// Forward pass up to the last 3x3 layer (the output layer is run_output).
ct_status run_forward(ct_unet *u, const float *x, int n, int h, int w, hipStream_t s)
{
    const size_t P1 = (size_t)n * h * w;
    const int h2 = h / 2, w2 = w / 2, h3 = h / 4, w3 = w / 4, h4 = h / 8, w4 = w / 8;
    hipLaunchKernelGGL(k_conv_in, dim3(blocks(P1 * 4, 256)), dim3(256), 0, s, x, u->theta + u->off[0], bias_of(u, 0), u->e1a, n,
                       h, w);
    CT_HIP_CHECK(hipGetLastError());
    CT_HIP_CHECK(conv_fwd(u, 1, one(u->e1a, 32), u->e1b, n, h, w, s, u->p1));
    CT_HIP_CHECK(conv_fwd(u, 2, one(u->p1, 32), u->e2a, n, h2, w2, s));
    CT_HIP_CHECK(conv_fwd(u, 3, one(u->e2a, 64), u->e2b, n, h2, w2, s, u->p2));
    CT_HIP_CHECK(conv_fwd(u, 4, one(u->p2, 64), u->e3a, n, h3, w3, s));
    CT_HIP_CHECK(conv_fwd(u, 5, one(u->e3a, 128), u->e3b, n, h3, w3, s, u->p3));
    CT_HIP_CHECK(conv_fwd(u, 6, one(u->p3, 128), u->ba, n, h4, w4, s));
    CT_HIP_CHECK(conv_fwd(u, 7, one(u->ba, 256), u->bb, n, h4, w4, s));
    CT_HIP_CHECK(conv_fwd(u, 8, cat(u->bb, 256, u->e3b, 128), u->d3a, n, h3, w3, s));
    CT_HIP_CHECK(conv_fwd(u, 9, one(u->d3a, 128), u->d3b, n, h3, w3, s));
    CT_HIP_CHECK(conv_fwd(u, 10, cat(u->d3b, 128, u->e2b, 64), u->d2a, n, h2, w2, s));
    CT_HIP_CHECK(conv_fwd(u, 11, one(u->d2a, 64), u->d2b, n, h2, w2, s));
    CT_HIP_CHECK(conv_fwd(u, 12, cat(u->d2b, 64, u->e1b, 32), u->d1a, n, h, w, s));
    CT_HIP_CHECK(conv_fwd(u, 13, one(u->d1a, 32), u->d1b, n, h, w, s));
    return CT_OK;
}

// Output layer; with a target also the loss gradient dy (gscale = 2e6 / masked pixel count) and one
// FP64 loss partial per 256 pixels (their count is returned through nlpart).
ct_status run_output(ct_unet *u, const float *x, float *out, int n, int h, int w, const float *target,
                     const unsigned char *mask, float gscale, int *nlpart, hipStream_t s)
{
    const size_t P1 = (size_t)n * h * w;
    const int nbl = (int)blocks(P1, 256);   // <= lpart_cap (sized for the maximum batch at creation)
    if (nlpart) *nlpart = nbl;
    hipLaunchKernelGGL(k_conv_out, dim3(blocks(P1, 256)), dim3(256), 0, s, u->d1b, x, u->theta + u->off[14],
                       bias_of(u, 14), out, target, mask, gscale, u->dy, u->lpart, (int)P1, h * w);
    CT_HIP_CHECK(hipGetLastError());
    return CT_OK;
}

ct_status run_backward(ct_unet *u, const float *x, int n, int h, int w, hipStream_t s)
{
    const size_t P1 = (size_t)n * h * w;
    const int h2 = h / 2, w2 = w / 2, h3 = h / 4, w3 = w / 4, h4 = h / 8, w4 = w / 8;
    // output layer
    hipLaunchKernelGGL(k_conv_out_back, dim3(blocks(P1, 256)), dim3(256), 0, s, u->dy, u->theta + u->off[14], u->d1b,
                       u->dzA[0], (int)P1);
    CT_HIP_CHECK(hipGetLastError());
    {
        const int pps = kOutPps;
        const int nsp = (int)((P1 + pps - 1) / pps);
        CT_TRY(ensure_part(u, (size_t)nsp * 33));
        hipLaunchKernelGGL(k_conv_out_wgrad, dim3(nsp), dim3(256), 0, s, u->dy, u->d1b, (int)P1, pps, u->part);
        CT_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_sum_parts, dim3(blocks(33, 32)), dim3(256), 0, s, u->part, nsp, 33, u->grad + u->off[14]);
        CT_HIP_CHECK(hipGetLastError());
    }
    // decoder level 1
    CT_TRY(conv_wgrad(u, 13, one(u->d1a, 32), u->dzA[0], n, h, w, s));
    CT_HIP_CHECK(conv_dgrad(u, 13, u->dzA[0], u->d1a, u->dzB[0], n, h, w, s));
    CT_TRY(conv_wgrad(u, 12, cat(u->d2b, 64, u->e1b, 32), u->dzB[0], n, h, w, s));
    CT_HIP_CHECK(conv_dgrad(u, 12, u->dzB[0], nullptr, u->dcat[0], n, h, w, s));
    hipLaunchKernelGGL(k_up_back, dim3(blocks(P1 / 4 * 8, 256)), dim3(256), 0, s, u->dcat[0], 96, u->d2b, u->dzA[1], n, h2,
                       w2, 64);
    CT_HIP_CHECK(hipGetLastError());
    // decoder level 2
    CT_TRY(conv_wgrad(u, 11, one(u->d2a, 64), u->dzA[1], n, h2, w2, s));
    CT_HIP_CHECK(conv_dgrad(u, 11, u->dzA[1], u->d2a, u->dzB[1], n, h2, w2, s));
    CT_TRY(conv_wgrad(u, 10, cat(u->d3b, 128, u->e2b, 64), u->dzB[1], n, h2, w2, s));
    CT_HIP_CHECK(conv_dgrad(u, 10, u->dzB[1], nullptr, u->dcat[1], n, h2, w2, s));
    hipLaunchKernelGGL(k_up_back, dim3(blocks(P1 / 16 * 16, 256)), dim3(256), 0, s, u->dcat[1], 192, u->d3b, u->dzA[2], n,
                       h3, w3, 128);
    CT_HIP_CHECK(hipGetLastError());
    // decoder level 3
    CT_TRY(conv_wgrad(u, 9, one(u->d3a, 128), u->dzA[2], n, h3, w3, s));
    CT_HIP_CHECK(conv_dgrad(u, 9, u->dzA[2], u->d3a, u->dzB[2], n, h3, w3, s));
    CT_TRY(conv_wgrad(u, 8, cat(u->bb, 256, u->e3b, 128), u->dzB[2], n, h3, w3, s));
    CT_HIP_CHECK(conv_dgrad(u, 8, u->dzB[2], nullptr, u->dcat[2], n, h3, w3, s));
    hipLaunchKernelGGL(k_up_back, dim3(blocks(P1 / 64 * 32, 256)), dim3(256), 0, s, u->dcat[2], 384, u->bb, u->dzA[3], n,
                       h4, w4, 256);
    CT_HIP_CHECK(hipGetLastError());
    // bottleneck
    CT_TRY(conv_wgrad(u, 7, one(u->ba, 256), u->dzA[3], n, h4, w4, s));
    CT_HIP_CHECK(conv_dgrad(u, 7, u->dzA[3], u->ba, u->dzB[3], n, h4, w4, s));
    CT_TRY(conv_wgrad(u, 6, one(u->p3, 128), u->dzB[3], n, h4, w4, s));
    CT_HIP_CHECK(conv_dgrad(u, 6, u->dzB[3], nullptr, u->dpool[2], n, h4, w4, s));
    // encoder level 3
    hipLaunchKernelGGL(k_skip_combine, dim3(blocks(P1 / 16 * 16, 256)), dim3(256), 0, s, u->dcat[2], 384, 256, u->dpool[2],
                       u->e3b, u->dzA[2], n, h3, w3, 128);
    CT_HIP_CHECK(hipGetLastError());
    CT_TRY(conv_wgrad(u, 5, one(u->e3a, 128), u->dzA[2], n, h3, w3, s));
    CT_HIP_CHECK(conv_dgrad(u, 5, u->dzA[2], u->e3a, u->dzB[2], n, h3, w3, s));
    CT_TRY(conv_wgrad(u, 4, one(u->p2, 64), u->dzB[2], n, h3, w3, s));
    CT_HIP_CHECK(conv_dgrad(u, 4, u->dzB[2], nullptr, u->dpool[1], n, h3, w3, s));
    // encoder level 2
    hipLaunchKernelGGL(k_skip_combine, dim3(blocks(P1 / 4 * 8, 256)), dim3(256), 0, s, u->dcat[1], 192, 128, u->dpool[1],
                       u->e2b, u->dzA[1], n, h2, w2, 64);
    CT_HIP_CHECK(hipGetLastError());
    CT_TRY(conv_wgrad(u, 3, one(u->e2a, 64), u->dzA[1], n, h2, w2, s));
    CT_HIP_CHECK(conv_dgrad(u, 3, u->dzA[1], u->e2a, u->dzB[1], n, h2, w2, s));
    CT_TRY(conv_wgrad(u, 2, one(u->p1, 32), u->dzB[1], n, h2, w2, s));
    CT_HIP_CHECK(conv_dgrad(u, 2, u->dzB[1], nullptr, u->dpool[0], n, h2, w2, s));
    // encoder level 1
    hipLaunchKernelGGL(k_skip_combine, dim3(blocks(P1 * 4, 256)), dim3(256), 0, s, u->dcat[0], 96, 64, u->dpool[0], u->e1b,
                       u->dzA[0], n, h, w, 32);
    CT_HIP_CHECK(hipGetLastError());
    CT_TRY(conv_wgrad(u, 1, one(u->e1a, 32), u->dzA[0], n, h, w, s));
    CT_HIP_CHECK(conv_dgrad(u, 1, u->dzA[0], u->e1a, u->dzB[0], n, h, w, s));
    {
        const int pps = kInPps;
        const int nsp = (int)((P1 + pps - 1) / pps);
        CT_TRY(ensure_part(u, (size_t)nsp * 320));
        hipLaunchKernelGGL(k_conv_in_wgrad, dim3(nsp), dim3(256), 0, s, x, u->dzB[0], n, h, w, pps, u->part);
        CT_HIP_CHECK(hipGetLastError());
        // weights 0..287 (canonical [co][1][3][3] == [co][tap]), then biases 288..319
        hipLaunchKernelGGL(k_sum_parts, dim3(blocks(320, 32)), dim3(256), 0, s, u->part, nsp, 320, u->grad + u->off[0]);
        CT_HIP_CHECK(hipGetLastError());
    }
    return CT_OK;
}

// Loss and gradient of one batch: forward with the loss epilogue, then backward. Returns the loss
// partial count through nlp (the caller reduces u->lpart when it wants the loss).
ct_status loss_and_grad(ct_unet *u, const float *x, const float *target, const unsigned char *mask, int n, int h,
                        int w, int *nlp, hipStream_t s)
{
    CT_TRY(alloc_train(u));
    CT_TRY(run_forward(u, x, n, h, w, s));
    // masked pixel count (FP64-exact on the host from a one-off copy of the mask)
    std::vector<unsigned char> hm((size_t)h * w);
    CT_HIP_CHECK(hipMemcpyAsync(hm.data(), mask, hm.size(), hipMemcpyDeviceToHost, s));
    CT_HIP_CHECK(hipStreamSynchronize(s));
    size_t cnt = 0;
    for (unsigned char c : hm) cnt += c != 0;
    if (cnt == 0) return fail(CT_ERR_INVALID_ARG, "mask selects no pixel");
    const float gscale = (float)(2.0e6 / ((double)cnt * n));
    CT_TRY(run_output(u, x, u->out, n, h, w, target, mask, gscale, nlp, s));
    CT_TRY(run_backward(u, x, n, h, w, s));
    return CT_OK;
}

ct_status read_loss(ct_unet *u, int nlp, int n, int h, int w, const unsigned char *mask, double *loss, hipStream_t s)
{
    std::vector<double> lp((size_t)nlp);
    CT_HIP_CHECK(hipMemcpyAsync(lp.data(), u->lpart, lp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<unsigned char> hm((size_t)h * w);
    CT_HIP_CHECK(hipMemcpyAsync(hm.data(), mask, hm.size(), hipMemcpyDeviceToHost, s));
    CT_HIP_CHECK(hipStreamSynchronize(s));
    double sum = 0.0;
    for (double v : lp) sum += v;
    size_t cnt = 0;
    for (unsigned char c : hm) cnt += c != 0;
    *loss = sum / ((double)cnt * n);
    return CT_OK;
}

hipStream_t as_s(void *p) { return reinterpret_cast<hipStream_t>(p); }

}  // namespace

extern "C" {

size_t ct_unet_num_params(void) { return n_params(); }

void ct_unet_destroy(ct_unet *u)
{
    if (!u) return;
    (void)hipDeviceSynchronize();
    ufree(&u->theta);
    ufree(&u->m);
    ufree(&u->v);
    ufree(&u->grad);
    for (int l = 0; l < kLayers; ++l) {
        ufree(&u->wf[l]);
        ufree(&u->wb[l]);
    }
    bf16 **acts[] = {&u->e1a, &u->e1b, &u->d1a, &u->d1b, &u->p1, &u->e2a, &u->e2b, &u->d2a, &u->d2b,
                     &u->p2, &u->e3a, &u->e3b, &u->d3a, &u->d3b, &u->p3, &u->ba, &u->bb};
    for (bf16 **a : acts) ufree(a);
    for (int l = 0; l < 4; ++l) {
        ufree(&u->dzA[l]);
        ufree(&u->dzB[l]);
    }
    for (int l = 0; l < 3; ++l) {
        ufree(&u->dcat[l]);
        ufree(&u->dpool[l]);
    }
    ufree(&u->out);
    ufree(&u->dy);
    ufree(&u->part);
    ufree(&u->lpart);
    delete u;
}

ct_status ct_unet_set_params(ct_unet *u, const float *theta)
{
    if (!u || !theta) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    const size_t np = n_params();
    CT_HIP_CHECK(hipMemcpy(u->theta, theta, np * sizeof(float), hipMemcpyHostToDevice));
    CT_HIP_CHECK(hipMemset(u->m, 0, np * sizeof(float)));
    CT_HIP_CHECK(hipMemset(u->v, 0, np * sizeof(float)));
    u->step = 0;
    CT_TRY(pack_weights(u, nullptr));
    CT_HIP_CHECK(hipDeviceSynchronize());
    return CT_OK;
}

ct_status ct_unet_create(const float *theta, int max_n, int max_h, int max_w, ct_unet **out)
{
    if (!out || !theta) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (max_n < 1 || max_h < 8 || max_w < 8 || max_h % 8 || max_w % 8 || (size_t)max_n * max_h * max_w > (1ull << 31) / 96)
        return fail(CT_ERR_INVALID_ARG, "max sizes must be >= 8, multiples of 8, and bounded");
    ct_unet *u = new (std::nothrow) ct_unet();
    if (!u) return fail(CT_ERR_OOM, "host allocation failed");
    u->max_n = max_n;
    u->max_h = max_h;
    u->max_w = max_w;
    (void)hipGetDevice(&u->device);
    size_t o = 0;
    for (int l = 0; l < kLayers; ++l) {
        u->off[l] = o;
        o += (size_t)kShape[l][1] * kShape[l][0] * kShape[l][2] * kShape[l][2] + kShape[l][1];
    }
    u->off[kLayers] = o;
    auto fail_out = [&](ct_status st) {
        ct_unet_destroy(u);
        return st;
    };
    ct_status st;
#define U_TRY(e)                                                                                                      \
    if ((st = (e)) != CT_OK) return fail_out(st);
    U_TRY(ualloc(&u->theta, o));
    U_TRY(ualloc(&u->m, o));
    U_TRY(ualloc(&u->v, o));
    U_TRY(ualloc(&u->grad, o));
    for (int l = 1; l < kLayers - 1; ++l) {
        const size_t nw = (size_t)kShape[l][0] * kShape[l][1] * 9;
        U_TRY(ualloc(&u->wf[l], nw));
        U_TRY(ualloc(&u->wb[l], nw));
    }
    const size_t P1 = (size_t)max_n * max_h * max_w;
    const size_t P2 = P1 / 4, P3 = P1 / 16, P4 = P1 / 64;
    U_TRY(ualloc(&u->e1a, P1 * 32));
    U_TRY(ualloc(&u->e1b, P1 * 32));
    U_TRY(ualloc(&u->d1a, P1 * 32));
    U_TRY(ualloc(&u->d1b, P1 * 32));
    U_TRY(ualloc(&u->p1, P2 * 32));
    U_TRY(ualloc(&u->e2a, P2 * 64));
    U_TRY(ualloc(&u->e2b, P2 * 64));
    U_TRY(ualloc(&u->d2a, P2 * 64));
    U_TRY(ualloc(&u->d2b, P2 * 64));
    U_TRY(ualloc(&u->p2, P3 * 64));
    U_TRY(ualloc(&u->e3a, P3 * 128));
    U_TRY(ualloc(&u->e3b, P3 * 128));
    U_TRY(ualloc(&u->d3a, P3 * 128));
    U_TRY(ualloc(&u->d3b, P3 * 128));
    U_TRY(ualloc(&u->p3, P4 * 128));
    U_TRY(ualloc(&u->ba, P4 * 256));
    U_TRY(ualloc(&u->bb, P4 * 256));
    U_TRY(ualloc(&u->out, P1));
    u->lpart_cap = blocks(P1, 256);
    U_TRY(ualloc(&u->lpart, u->lpart_cap));
    U_TRY(ct_unet_set_params(u, theta));
#undef U_TRY
    *out = u;
    return CT_OK;
}

ct_status ct_unet_get_params(const ct_unet *u, float *theta)
{
    if (!u || !theta) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    CT_HIP_CHECK(hipDeviceSynchronize());
    CT_HIP_CHECK(hipMemcpy(theta, u->theta, n_params() * sizeof(float), hipMemcpyDeviceToHost));
    return CT_OK;
}

ct_status ct_unet_forward(ct_unet *u, const float *x, float *out, int n, int h, int w, void *stream)
{
    if (!u || !x || !out) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    if (x == out) return fail(CT_ERR_INVALID_ARG, "x and out may not alias");
    CT_TRY(check_shape(u, n, h, w));
    hipStream_t s = as_s(stream);
    CT_TRY(run_forward(u, x, n, h, w, s));
    CT_TRY(run_output(u, x, out, n, h, w, nullptr, nullptr, 0.f, nullptr, s));
    return CT_OK;
}

ct_status ct_unet_gradient(ct_unet *u, const float *x, const float *target, const unsigned char *mask, int n, int h,
                           int w, double *loss, float *grad, void *stream)
{
    if (!u || !x || !target || !mask) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    CT_TRY(check_shape(u, n, h, w));
    hipStream_t s = as_s(stream);
    int nlp = 0;
    CT_TRY(loss_and_grad(u, x, target, mask, n, h, w, &nlp, s));
    if (loss) CT_TRY(read_loss(u, nlp, n, h, w, mask, loss, s));
    if (grad) {
        CT_HIP_CHECK(hipMemcpyAsync(grad, u->grad, n_params() * sizeof(float), hipMemcpyDeviceToHost, s));
        CT_HIP_CHECK(hipStreamSynchronize(s));
    }
    return CT_OK;
}

ct_status ct_unet_train_step(ct_unet *u, const float *x, const float *target, const unsigned char *mask, int n, int h,
                             int w, float lr, double *loss, void *stream)
{
    if (!u || !x || !target || !mask) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    if (!(lr > 0.f)) return fail(CT_ERR_INVALID_ARG, "lr must be > 0");
    CT_TRY(check_shape(u, n, h, w));
    hipStream_t s = as_s(stream);
    int nlp = 0;
    CT_TRY(loss_and_grad(u, x, target, mask, n, h, w, &nlp, s));
    if (loss) CT_TRY(read_loss(u, nlp, n, h, w, mask, loss, s));
    u->step += 1;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)u->step));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)u->step));
    const size_t np = n_params();
    hipLaunchKernelGGL(k_adam, dim3(blocks(np, 256)), dim3(256), 0, s, u->theta, u->m, u->v, u->grad, np, lr, bc1, bc2);
    CT_HIP_CHECK(hipGetLastError());
    CT_TRY(pack_weights(u, s));
    return CT_OK;
}

ct_status ct_unet_input(ct_geom *g, const void *y, double mu_water, float *x_in, void *stream)
{
    if (!g || !y || !x_in) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    if (!(mu_water > 0)) return fail(CT_ERR_INVALID_ARG, "mu_water must be > 0");
    if (g->desc.det != CT_DET_FLAT) return fail(CT_ERR_UNSUPPORTED, "the network input needs the flat-detector FBP");
    return unet_input(g, y, 1.0 / mu_water, x_in, as_s(stream));
}

}  // extern "C"

namespace ct {

// x_in = factor * FBP-like image of y (flat detector)
ct_status unet_input(ct_geom *g, const void *y, double factor, float *x_in, hipStream_t s)
{
    CT_TRY(ensure_workspace(g, g->desc.nviews, 4));
    Workspace &W = g->ws;
    CT_HIP_CHECK(launch_fbp(g, y, g->desc.storage, W.r, g->cs, W.tmp, s));
    hipLaunchKernelGGL(k_scale_copy, dim3(blocks(W.npix, 256)), dim3(256), 0, s, W.tmp, (float)factor, x_in, W.npix);
    CT_HIP_CHECK(hipGetLastError());
    return CT_OK;
}

// Learned start of a solve: x = mu_water * max(network(FBP(y) / mu_water), 0). a and b: two [ny][nx]
// float32 scratch images.
ct_status learned_start(ct_geom *g, const ct_unet *uc, const void *y, double mu_water, float *x, float *a, float *b,
                        hipStream_t s)
{
    ct_unet *u = const_cast<ct_unet *>(uc);
    if (g->desc.det != CT_DET_FLAT) return fail(CT_ERR_UNSUPPORTED, "the learned start needs the flat-detector FBP");
    CT_TRY(unet_input(g, y, 1.0 / mu_water, a, s));
    CT_TRY(ct_unet_forward(u, a, b, 1, g->desc.ny, g->desc.nx, s));
    hipLaunchKernelGGL(k_start, dim3(blocks(g->ws.npix, 256)), dim3(256), 0, s, b, (float)mu_water, x, g->ws.npix);
    CT_HIP_CHECK(hipGetLastError());
    return CT_OK;
}

}  // namespace ct
