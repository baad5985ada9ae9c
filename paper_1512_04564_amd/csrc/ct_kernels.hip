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
//
// Storage: the sinogram inputs, the residual block and the forward projector's image copies may be
// float16 or bfloat16 (converted to float32 on load, rounded to nearest even on store); every sum and
// the image state x, g, h stay float32.
//
// Both hot kernels exist twice: for one launch described by kernel arguments, and batched, where a
// 1-D grid spans several independent slices (each with its own geometry and buffers) and every
// workgroup looks its slice up in a device table of workgroup ranges.
//
// This file is compiled without NaN semantics (-fno-honor-nans): min/max need no canonicalising moves.
// Finiteness checks live in ct_reduce.hip, which keeps them.
#include <type_traits>

#include "ct_grid_barrier.hpp"
#include "ct_internal.hpp"

namespace ct {

namespace {

constexpr int FP_BINS = 64;          // bins per forward workgroup (one per lane)
constexpr int FP_WAVES = 16;         // waves per forward workgroup (single launches); each streams its own lines
constexpr int FP_WIN = 128;          // LDS pixel window of one wave (floats)
constexpr int FP_PF = FP_WIN / 64;   // prefetch registers per lane
constexpr int FP_RING = 2;           // image lines in flight per wave (fast line loop)
constexpr int BP_TX = kBpTile, BP_TY = kBpTile;

__device__ __forceinline__ float rcp_approx(float v) { return __builtin_amdgcn_rcpf(v); }

// Read-only geometry entry at a wave-uniform index, through the constant address space (a scalar load)
template <typename T>
__device__ __forceinline__ T ld_uniform(const T *p, unsigned i)
{
    return reinterpret_cast<const __attribute__((address_space(4))) T *>(reinterpret_cast<size_t>(p))[i];
}

template <typename T>
__device__ __forceinline__ float ld(const void *p, size_t i)
{
    return (float)static_cast<const T *>(p)[i];
}
template <typename T>
__device__ __forceinline__ void st(void *p, size_t i, float v)
{
    static_cast<T *>(p)[i] = (T)v;
}

// The bits of one element of type T through a buffer resource (byte offset off), and their value as
// float. The two are separate so that a prefetch can keep the raw bits in flight: converting at load time
// would make the load wait for its data at once.
// (float32 elements are kept as float.)
template <typename T>
using RawT = std::conditional_t<sizeof(T) == 4, float, unsigned>;
template <typename T>
__device__ __forceinline__ RawT<T> buf_raw(__amdgpu_buffer_rsrc_t rs, unsigned off)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
    else
        return __builtin_amdgcn_raw_buffer_load_b16(rs, (int)off, 0, 0);
}
template <typename T>
__device__ __forceinline__ RawT<T> ld_raw(const T *p, unsigned i)
{
    if constexpr (sizeof(T) == 4)
        return p[i];
    else
        return __builtin_bit_cast(unsigned short, p[i]);
}
template <typename T>
__device__ __forceinline__ float from_raw(RawT<T> u)
{
    if constexpr (sizeof(T) == 4)
        return u;
    else
        return (float)__builtin_bit_cast(T, (unsigned short)u);
}

// Forward projection of the views vstart + vi * vstride (vi = blockIdx.y) for the 64 bins of block
// blockIdx.x. Each wave streams a contiguous range of image lines: the pixels of line l+1 that the
// block's footprint covers are loaded into registers (coalesced, clamped addresses) while line l is
// evaluated from the wave's LDS window. The windows of 64 lines at a time are computed one line per lane
// and read back with readlane. A bin's overlaps with its pixels are three branch-free taps from LDS (the
// window is padded, so taps past its end read finite data with zero weight); wider footprints (oblique
// lines) continue in a loop, and lines whose window exceeds the LDS slice read global memory.
template <int EPI, bool ONES, int WAVES, typename TI, typename TY, typename TO>
__device__ __forceinline__ void fp_body(const FpLaunch &a, const int bx, const int vi, const int half_of, float *win)
{
    const GeomDev &G = a.G;
    const int vstart = a.vstart, vstride = a.vstride;
    const TI *__restrict__ img = static_cast<const TI *>(a.img);
    const TI *__restrict__ imgT = static_cast<const TI *>(a.imgT);
    constexpr int PADW = FP_WIN + 4;
    const int v = vstart + vi * vstride;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform: line loop in SGPRs
    const int nb = G.nb;
    const int kblk = bx * FP_BINS;
    const int k = kblk + lane;
    const int kc = min(k, nb - 1);   // lanes past the last bin repeat it; their result is discarded
    const int klast = min(kblk + FP_BINS, nb);
    const bool row = G.rowsweep[v] != 0;
    const int NL = row ? G.ny : G.nx;
    const int NQ = row ? G.nx : G.ny;
    const bool even = (NQ & 1) == 0;
    const int hq = NQ / 2;
    const TI *src = row ? img : imgT;
    const float half = 0.5f * (float)NQ;
    const float lc0 = -0.5f * (float)(NL - 1);
    const float2 *bv = G.bnd + (size_t)v * (nb + 1);
    const float2 b0 = bv[kc], b1 = bv[kc + 1];
    const float2 bF = bv[kblk], bL = bv[klast];
    // operands of the epilogue (wave 0), loaded with the boundaries so that their latency overlaps
    float e_sc = 0.f, e_w = 0.f, e_y = 0.f;
    if (wave == 0 && k < nb) {
        const size_t si = (size_t)v * nb + k;
        e_sc = G.scale[si];
        if (EPI != FP_PLAIN) e_w = ld<TY>(a.w, si);
        if (EPI == FP_RESIDUAL) e_y = ld<TY>(a.y, si);
    }
    float *wl = win + wave * PADW;
    for (int t = lane; t < PADW; t += 64) wl[t] = ONES ? 1.f : 0.f;
    // the workgroup's lines: all, or half half_of (0: [0, NL / 2), 1: [NL / 2, NL)) of a split block
    const int lbeg = half_of == 1 ? NL / 2 : 0, nlw = half_of < 0 ? NL : (half_of == 0 ? NL / 2 : NL - NL / 2);
    const int l0 = lbeg + (wave * nlw) / WAVES, l1 = lbeg + ((wave + 1) * nlw) / WAVES;

    // pixels [ws, ws + wn) of line l that the block's bins can overlap (boundaries are monotone in k);
    // computed by lane (l - lb) for the 64 lines starting at lb
    int ws_v = 0, wn_v = 0;
    auto windows = [&](int lb) {
        const float lc = lc0 + (float)(lb + lane);
        const float uF = fmaf(lc, bF.y, bF.x), uL = fmaf(lc, bL.y, bL.x);
        const float lo = fmaxf(fminf(uF, uL), -half), hi = fminf(fmaxf(uF, uL), half);
        ws_v = max((int)floorf(lo + half) - 1, 0);
        const int we = min((int)floorf(hi + half) + 1, NQ - 1);
        wn_v = lo < hi ? we - ws_v + 1 : 0;
    };
    RawT<TI> pf[FP_PF];
    // Image lines are read through a buffer resource over the whole image: one scalar descriptor, a 32-bit
    // byte offset per lane (line base included, so the hardware range check covers every read) and reads
    // past the image returning 0. Reads past the end of a line only feed taps of zero weight (their
    // pixels lie beyond the clamped footprint), so no per-lane clamp is needed.
    const __amdgpu_buffer_rsrc_t img_rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<TI *>(src), 0, (int)((size_t)NL * NQ * sizeof(TI)), 0x00020000);
    const unsigned lane_off = (unsigned)lane * (unsigned)sizeof(TI);
    auto prefetch = [&](int l, int ws) {
        if (!ONES) {
            const unsigned base = ((unsigned)l * (unsigned)NQ + (unsigned)ws) * (unsigned)sizeof(TI);
#pragma unroll
            for (int j = 0; j < FP_PF; ++j) {
                pf[j] = buf_raw<TI>(img_rs, lane_off + base + (unsigned)(64 * j * sizeof(TI)));
            }
        }
    };

    // vmcnt(0): the boundary loads above are complete before the line loop, so that waiting on them
    // inside the loop cannot also drain the next line's prefetch (vector loads complete in order)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    float acc = 0.f;
    int lb = l0;
    windows(lb);
    if (l0 < l1) prefetch(l0, __builtin_amdgcn_readfirstlane(ws_v));
    float lc = lc0 + (float)l0;
    // Branch-free loop when every footprint of the block is at most two pixels wide (three taps suffice:
    // d < width + 1 < 3) and every line's window fits the LDS slice (its width is at most the span of the
    // block's outer boundaries + 4). Both widths are linear in the line coordinate, so their maxima over the
    // view's lines are at the first or the last line. It computes the same sums as the general loop below:
    // a footprint that misses the line gets zero weights, and the tap index is clamped into the padded
    // window, whose entries are finite.
    const float lcL = lc0 + (float)(NL - 1);
    // signed footprint width at the first and the last line (linear in between)
    const float sw0 = fmaf(lc0, b1.y - b0.y, b1.x - b0.x), sw1 = fmaf(lcL, b1.y - b0.y, b1.x - b0.x);
    const float fw = fmaxf(fabsf(sw0), fabsf(sw1));
    // The fast loop takes the lane's boundaries in a fixed order: where the footprint keeps one orientation
    // over all lines, by a margin far above the rounding of a boundary position, the order of the two
    // rounded positions is that of the exact ones on every line, which min / max would find.
    const bool ordered = (sw0 > 0.01f && sw1 > 0.01f) || (sw0 < -0.01f && sw1 < -0.01f);
    const float2 blo = sw0 > 0.f ? b0 : b1, bhi = sw0 > 0.f ? b1 : b0;
    const float bw = fmaxf(fabsf(fmaf(lc0, bL.y - bF.y, bL.x - bF.x)), fabsf(fmaf(lcL, bL.y - bF.y, bL.x - bF.x)));
    // first pixel q0 of a footprint starting at loc and its left edge e (exact)
    auto first_pixel = [&](float loc, int &q0, float &e, auto even_tag) {
        if (decltype(even_tag)::value) {   // pixel edges sit at integers: floor is exact
            e = floorf(loc);
            q0 = (int)e + hq;
        } else {
            q0 = (int)floorf(loc + half);
            e = (float)q0 - half;
            if (loc < e) {   // exact correction of a rounded floor
                --q0;
                e -= 1.f;
            }
        }
    };
    // FP_RING lines in flight: register set r serves the lines l0 + r, l0 + r + FP_RING, ..., with no moves
    // between sets; every step issues its loads (the last line repeats past the end) so that the loads in
    // flight are counted statically
    auto fast_lines = [&](auto even_tag) {
        RawT<TI> pr[FP_RING][FP_PF];
        int wsr[FP_RING];
        auto fetch_into = [&](int ll, RawT<TI> (&dst)[FP_PF], int &wsd) {
            ll = min(ll, l1 - 1);
            if (ll - lb == 64) {
                lb += 64;
                windows(lb);
            }
            wsd = __builtin_amdgcn_readlane(ws_v, ll - lb);
            prefetch(ll, wsd);
#pragma unroll
            for (int j = 0; j < FP_PF; ++j) dst[j] = pf[j];
        };
        // line coordinate lcl (exact: integers plus the half of lc0)
        auto step = [&](float lcl, const RawT<TI> (&src)[FP_PF], int ws) {
            if (!ONES) {
#pragma unroll
                for (int j = 0; j < FP_PF; ++j) wl[lane + 64 * j] = from_raw<TI>(src[j]);
            }
            __builtin_amdgcn_wave_barrier();
            const float lo = fmaf(lcl, blo.y, blo.x);
            const float hi = fmaf(lcl, bhi.y, bhi.x);
            // both ends clamped into the line: loc <= hic, so the first weight min(d, 1) - f is >= 0, and a
            // footprint that misses the line gets d = f = 0
            const float loc = __builtin_amdgcn_fmed3f(lo, -half, half), hic = __builtin_amdgcn_fmed3f(hi, -half, half);
            int q0;
            float e;
            first_pixel(loc, q0, e, even_tag);
            const float d = hic - e, f = loc - e;
            const float *tp = wl + min(max(q0 - ws, 0), FP_WIN);
            float s = (fminf(d, 1.f) - f) * tp[0];
            s = fmaf(__builtin_amdgcn_fmed3f(d - 1.f, 0.f, 1.f), tp[1], s);
            s = fmaf(__builtin_amdgcn_fmed3f(d - 2.f, 0.f, 1.f), tp[2], s);
            return s * rcp_approx(hi - lo);
        };
        // line l0 is already fetched into pf (by the caller's prefetch); lines l0 + 1 .. go to the other sets
        wsr[0] = __builtin_amdgcn_readlane(ws_v, l0 - lb);
#pragma unroll
        for (int j = 0; j < FP_PF; ++j) pr[0][j] = pf[j];
#pragma unroll
        for (int r = 1; r < FP_RING; ++r) fetch_into(l0 + r, pr[r], wsr[r]);
        // The loop body has no branch around a step, so that the wait before a set's use counts the other
        // sets' loads as still in flight (a conditional step would make the compiler wait for all of them);
        // the last lines (fewer than FP_RING) are taken after the loop, in line order.
        float lcl = lc0 + (float)l0;
        int l = l0;
        for (; l + FP_RING <= l1; l += FP_RING) {
#pragma unroll
            for (int r = 0; r < FP_RING; ++r) {
                const float c = step(lcl + (float)r, pr[r], wsr[r]);
                __builtin_amdgcn_wave_barrier();
                fetch_into(l + r + FP_RING, pr[r], wsr[r]);
                acc += c;
            }
            lcl += (float)FP_RING;
        }
#pragma unroll
        for (int r = 0; r + 1 < FP_RING; ++r)
            if (l + r < l1) acc += step(lcl + (float)r, pr[r], wsr[r]);
    };
    if (l0 < l1 && __ballot(fw > 1.99f || bw + 5.f > (float)FP_WIN || !ordered) == 0) {   // (waves with no lines skip both)
        if (even) fast_lines(std::true_type{});
        else fast_lines(std::false_type{});
    } else
    for (int l = l0; l < l1; ++l, lc += 1.f) {
        const int ws = __builtin_amdgcn_readlane(ws_v, l - lb);
        const int wn = __builtin_amdgcn_readlane(wn_v, l - lb);
        if (!ONES) {
#pragma unroll
            for (int j = 0; j < FP_PF; ++j) wl[lane + 64 * j] = from_raw<TI>(pf[j]);
        }
        // LDS operations of one wave complete in order: the window is readable by every lane below,
        // and the next line's stores cannot overtake these reads.
        __builtin_amdgcn_wave_barrier();
        if (l + 1 < l1) {
            if (l + 1 - lb == 64) {
                lb += 64;
                windows(lb);
            }
            prefetch(l + 1, __builtin_amdgcn_readlane(ws_v, l + 1 - lb));
        }
        if (wn > 0) {
            const float u0 = fmaf(lc, b0.y, b0.x);
            const float u1 = fmaf(lc, b1.y, b1.x);
            const float lo = fminf(u0, u1), hi = fmaxf(u0, u1);
            const float loc = fmaxf(lo, -half), hic = fminf(hi, half);
            if (loc < hic) {
                float e;   // left edge of pixel q0, the first pixel the footprint meets (exact)
                int q0;
                if (even) {   // pixel edges sit at integers: floor is exact
                    e = floorf(loc);
                    q0 = (int)e + hq;
                } else {
                    q0 = (int)floorf(loc + half);
                    if (loc < (float)q0 - half) --q0;   // exact correction of a rounded floor
                    e = (float)q0 - half;
                }
                // overlap of [loc, hic] with pixel q0 + i, pixel edges e + i: since e <= loc < e + 1,
                // pixel q0 takes min(d, 1) - f and pixel q0 + i (i >= 1) takes med3(d - i, 0, 1),
                // with d = hic - e and f = loc - e
                const float d = hic - e, f = loc - e;
                float s;
                if (wn <= FP_WIN) {
                    const float *tp = wl + (q0 - ws);  // q0 >= ws; three taps stay inside the padding
                    s = (fminf(d, 1.f) - f) * tp[0];
                    s = fmaf(__builtin_amdgcn_fmed3f(d - 1.f, 0.f, 1.f), tp[1], s);
                    s = fmaf(__builtin_amdgcn_fmed3f(d - 2.f, 0.f, 1.f), tp[2], s);
                    for (int i = 3; (float)i < d; ++i)   // footprint wider than three pixels
                        s = fmaf(fminf(d - (float)i, 1.f), tp[i], s);
                } else {
                    const TI *line = src + (size_t)l * NQ;
                    s = (fminf(d, 1.f) - f) * (ONES ? 1.f : (float)line[q0]);
                    for (int i = 1; (float)i < d; ++i)
                        s = fmaf(fminf(d - (float)i, 1.f), ONES ? 1.f : (float)line[q0 + i], s);
                }
                acc = fmaf(s, rcp_approx(hi - lo), acc);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    float *red = win;   // reuse: [WAVES][64]
    red[wave * 64 + lane] = acc;
    __syncthreads();
    if (wave == 0 && k < nb) {
        float p = 0.f;
#pragma unroll
        for (int ww = 0; ww < WAVES; ++ww) p += red[ww * 64 + lane];
        const float sc = e_sc;
        p *= sc;
        const size_t o = (size_t)vi * nb + k;
        if (EPI == FP_PLAIN) st<TO>(a.out, o, p);
        // the residual is stored multiplied by the bin scale, the factor the back-projector applies to it
        else if (EPI == FP_RESIDUAL) {
            if (half_of == 1) st<float>(a.out2, o, (a.mscale * e_w * p) * sc);   // the data term is in half 0
            else st<TO>(a.out, o, (a.mscale * e_w * (p - e_y)) * sc);
        }
        else st<TO>(a.out, o, e_w * p);
    }
}

// SPLIT: each block's lines split over two workgroups (grid x doubled; residual epilogue, float32)
template <int EPI, bool ONES, int WAVES, typename TI, typename TY, typename TO, bool SPLIT>
__global__ __launch_bounds__(FP_BINS *WAVES) void k_forward(FpLaunch a)
{
    __shared__ float win[WAVES * (FP_WIN + 4)];
    if constexpr (SPLIT) {
        const int nbx = (a.G.nb + FP_BINS - 1) / FP_BINS;
        fp_body<EPI, ONES, WAVES, TI, TY, TO>(a, blockIdx.x % nbx, blockIdx.y, (int)blockIdx.x / nbx, win);
    } else {
        fp_body<EPI, ONES, WAVES, TI, TY, TO>(a, blockIdx.x, blockIdx.y, -1, win);
    }
}

// Slice of workgroup b in a batched grid: the table holds ascending, contiguous workgroup ranges.
template <bool FP>
__device__ __forceinline__ int find_slice(const SliceDev *__restrict__ tab, int ns, int b)
{
    int s = 0;
    while (s + 1 < ns && b >= (FP ? tab[s].fp_end : tab[s].bp_end)) ++s;
    return s;
}

// Batched forward projection of subset m with the residual epilogue, every slice reading image buffer par:
// the work of workgroup b of the batched grid.
template <int WAVES, typename T>
__device__ __forceinline__ void forward_item(const SliceDev *__restrict__ tab, int ns, int m, int par, int b, float *win)
{
    const int s = find_slice<true>(tab, ns, b);
    const SliceDev &S = tab[s];
    FpLaunch a;
    a.G = S.G;
    a.img = S.xc[par];
    a.imgT = S.xt[par];
    a.y = S.y;
    a.w = S.w;
    a.out = S.r;
    a.out2 = S.r2;
    a.vstart = m;
    a.vstride = S.M;
    a.nv = S.nvm;
    a.mscale = (float)S.M;
    const int local = b - S.fp_begin;
    const int nbx = (S.G.nb + FP_BINS - 1) / FP_BINS, per_view = S.r2 ? 2 * nbx : nbx;
    const int rem = local % per_view;
    if (S.r2)   // split: float32 residual planes
        fp_body<FP_RESIDUAL, false, WAVES, T, T, float>(a, rem % nbx, local / per_view, rem / nbx, win);
    else
        fp_body<FP_RESIDUAL, false, WAVES, T, T, T>(a, rem % nbx, local / per_view, -1, win);
}

template <int WAVES, typename T>
__global__ __launch_bounds__(FP_BINS *WAVES) void k_forward_batch(const SliceDev *__restrict__ tab, int ns, int m,
                                                                   int par)
{
    __shared__ float win[WAVES * (FP_WIN + 4)];
    forward_item<WAVES, T>(tab, ns, m, par, blockIdx.x, win);
}

// Back-projection of one pixel for one view: bins whose interval meets the pixel [e0, e0 + 1] on line
// lc. The candidate range comes from the detector coordinate of the pixel's two edges (inverse map
// u = dsd (e na + lc nl) / (e da + lc dl + dso)), widened by 0.05 bin, which absorbs the FP32 error of the
// inverse map and of the boundary table (both far below it); the overlaps themselves are evaluated from
// the same boundary table and fmaf sequence as the forward projector. ab(k) returns the boundary
// coefficients of boundary k and rs(k) the residual of bin k premultiplied by its scale.
template <typename AB, typename RS>
__device__ __forceinline__ float bp_view(const GeomDev &G, const float4 im, float lc, float e0, int kw0, int kw1,
                                         AB ab, RS rs)
{
    const float nlc = lc * im.y;
    const float dlc = fmaf(lc, im.w, G.dso);
    const float num0 = fmaf(e0, im.x, nlc), den0 = fmaf(e0, im.z, dlc);
    const float num1 = num0 + im.x, den1 = den0 + im.z;
    float t0 = num0 * rcp_approx(den0), t1 = num1 * rcp_approx(den1);
    if (G.arc) {
        t0 = atanf(t0);
        t1 = atanf(t1);
    }
    const float kf0 = fmaf(G.c_kf, t0, G.k0), kf1 = fmaf(G.c_kf, t1, G.k0);
    const int ka = max((int)floorf(fminf(kf0, kf1) - 0.05f), kw0);
    const int kb = min((int)floorf(fmaxf(kf0, kf1) + 0.05f), kw1);
    if (ka > kb) return 0.f;   // the pixel meets no bin (ka <= kb <= kw1 below keeps every index in range)
    const float e1 = e0 + 1.f;
    // Bins ka, ka+1, ka+2 unconditionally (boundary indices clamped to the staged range [kw0, kw1 + 1]);
    // bins past kb lie at least 0.05 bin beyond the pixel, so their overlap is zero, and a clamped
    // zero-width interval contributes 0 * finite. Pixels that meet more bins continue in a loop.
    const int kt = kw1 + 1;
    const float2 b0 = ab(ka), b1 = ab(min(ka + 1, kt)), b2 = ab(min(ka + 2, kt)), b3 = ab(min(ka + 3, kt));
    const float u0 = fmaf(lc, b0.y, b0.x), u1 = fmaf(lc, b1.y, b1.x);
    const float u2 = fmaf(lc, b2.y, b2.x), u3 = fmaf(lc, b3.y, b3.x);
    auto tap = [&](float ua, float ub, int kk) {
        const float lo = fminf(ua, ub), hi = fmaxf(ua, ub);
        const float ov = fmaxf(fminf(hi, e1) - fmaxf(lo, e0), 0.f);
        return rs(min(kk, kw1)) * (ov * rcp_approx(fmaxf(hi - lo, 1e-30f)));
    };
    float zeta = tap(u0, u1, ka) + tap(u1, u2, ka + 1) + tap(u2, u3, ka + 2);
    float up = u3;
    for (int k = ka + 3; k <= kb; ++k) {
        const float2 b = ab(k + 1);
        const float un = fmaf(lc, b.y, b.x);
        zeta += tap(up, un, k);
        up = un;
    }
    return zeta;
}

// v clamped to [0, hi] (hi >= 0) in one instruction: the median of v, 0 and hi.
__device__ __forceinline__ int clamp_entry(int v, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(v), "v"(hi));
    return r;
}

// Cumulative form of the same back-projection, from a view staged in LDS. For the tile's bin window
// kw0 .. kw1 (n bins), entry e = k - kw0 (0 <= e <= n) holds s (A_k, B_k), the signed coefficients of
// boundary k (s = +1 or -1 the view's boundary order, so that s U_k increases with k), P_e, the sum of
// r_j * scale_j over the window's bins before k, and r_k * scale_k (0 at e = n). With
// F(u) = P_e + r_e (u - s U_k) / (s U_k+1 - s U_k) for u in bin k (clamped to the window), the pixel's
// value is F(s edge_hi) - F(s edge_lo): in exact arithmetic the sum over bins of the residual times
// overlap / footprint that the forward projector's weights define, evaluated at two points instead of
// once per bin. The bin of each edge comes from its detector coordinate; when that estimate misses the
// bin by a hair (FP32 error, far below one bin) the neighbouring entry is taken instead.
// Entry of the bin of the edge at signed coordinate u (detector coordinate kf, window-relative), with
// u's endpoints ua, ub on the line lc; returns whether the estimate missed that bin.
struct CumBin {
    float4 q;       // s A_k, s B_k, P_e, r_e
    float ua, ub;   // s U_k, s U_k+1 on the pixel's line
};
__device__ __forceinline__ CumBin cum_bin(const float4 *__restrict__ E, int e, float lc)
{
    CumBin c;
    c.q = E[e];
    const float2 b = *reinterpret_cast<const float2 *>(E + e + 1);
    c.ua = fmaf(lc, c.q.y, c.q.x);
    c.ub = fmaf(lc, b.y, b.x);
    return c;
}
__device__ __forceinline__ float cum_value(const CumBin &c, float u)
{
    return fmaf(c.q.w, __builtin_amdgcn_fmed3f((u - c.ua) * rcp_approx(c.ub - c.ua), 0.f, 1.f), c.q.z);
}

// Back-projection of view onto the NP pixels [ex + m, ex + m + 1] (m < NP) of line lc from the cumulative
// form: the NP + 1 edges are evaluated once each, one after the other, each pixel taking the difference
// of its two edges' values. kofs = k0 - kw0 (the detector coordinate from the window's first bin), n the
// window's bins, POS the view's boundary order (a template parameter, so that the sign flips are operand
// modifiers). POLY: the edges' detector coordinates come from the quadratic Taylor polynomial in m about
// the first edge (t(m) = a/c + K / (1 + eps m) along the line, so t'' / 2 = -eps t'); the host allows it
// only where the polynomial stays within a quarter bin of the true coordinate, and the step to the
// neighbouring entry below absorbs that as it absorbs the reciprocal's error. Otherwise one division per
// edge (and the arc detector's arctangent).
template <int NP, bool POS, bool POLY>
__device__ __forceinline__ void bp_line(const GeomDev &G, const float4 im, float lc, float ex, int n, float kofs,
                                        const float4 *__restrict__ E, float (&val)[NP])
{
    const float nlc = lc * im.y;
    const float dlc = fmaf(lc, im.w, G.dso);
    float K0 = 0.f, K1 = 0.f, K2 = 0.f;
    if constexpr (POLY) {
        const float rd = rcp_approx(fmaf(ex, im.z, dlc));
        const float t0 = fmaf(ex, im.x, nlc) * rd;
        K0 = fmaf(G.c_kf, t0, kofs);
        K1 = G.c_kf * (fmaf(-t0, im.z, im.x) * rd);   // d kf / dm at m = 0
        K2 = -K1 * (im.z * rd);                        // half the second derivative
    }
    float Fp = 0.f;
#pragma unroll
    for (int m = 0; m <= NP; ++m) {
        const float em = ex + (float)m;
        float kf;
        if constexpr (POLY) {
            kf = m == 0 ? K0 : fmaf((float)m, fmaf((float)m, K2, K1), K0);
        } else {
            float t = fmaf(em, im.x, nlc) * rcp_approx(fmaf(em, im.z, dlc));
            if (G.arc) t = atanf(t);
            kf = fmaf(G.c_kf, t, kofs);
        }
        const int e = clamp_entry((int)floorf(kf), n - 1);
        const float u = POS ? em : -em;   // the edge in signed coordinates
        CumBin c = cum_bin(E, e, lc);
        if ((u < c.ua) | (u > c.ub))   // the estimate missed its edge's bin: the neighbouring entry
            c = cum_bin(E, clamp_entry(u < c.ua ? e - 1 : e + 1, n - 1), lc);
        const float F = cum_value(c, u);
        if (m > 0) val[m - 1] = POS ? F - Fp : Fp - F;
        Fp = F;
    }
}

// Inclusive prefix sum over the 64 lanes of a wave: shifts within rows of 16 lanes, then the row totals
// broadcast into the following rows.
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_or_zero(T v)
{
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xF, true));
}
template <typename T>
__device__ __forceinline__ T wave_prefix_sum(T v)
{
    v += dpp_or_zero<0x111, 0xF>(v);   // row_shr:1
    v += dpp_or_zero<0x112, 0xF>(v);   // row_shr:2
    v += dpp_or_zero<0x114, 0xF>(v);   // row_shr:4
    v += dpp_or_zero<0x118, 0xF>(v);   // row_shr:8
    v += dpp_or_zero<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_or_zero<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}
// value of the lane below (0 in lane 0)
template <typename T>
__device__ __forceinline__ T wave_shift_up(T v)
{
    return dpp_or_zero<0x138, 0xF>(v);   // wave_shr:1
}

// idelta = 1 / delta (rounded once on the host: no division on the device).
template <int POT>
__device__ __forceinline__ void pot_terms(float idelta, float t, float &dphi, float &omega)
{
    const float z = t * idelta;
    if (POT == 0) {
        omega = rsqrtf(fmaf(z, z, 1.f));
    } else if (POT == 1) {
        omega = 1.f / (1.f + fabsf(z));
    } else {   // q-GGMRF, p = 2, q = 1.2: s = |z|^0.8 (0 at z = 0: exp2(-inf))
        const float s = exp2f(0.8f * log2f(fabsf(z)));
        const float u = 1.f + s;
        omega = fmaf(1.2f, s, 2.f) / (2.f * u * u);
    }
    dphi = t * omega;
}

// Detector-bin window [k0, k1] of the tile (pixel edges ti0..ti1 x tj0..tj1, tile-local) for view v:
// the central projection of a convex tile is spanned by the projections of its four corners; one bin of
// margin on each side absorbs FP32 error (k0 > k1: the tile misses the detector).
__device__ __forceinline__ int2 tile_window(const GeomDev &G, int v, int i0, int i1, int j0, int j1)
{
    const bool row = G.rowsweep[v] != 0;
    const float4 im = G.inv[v];
    // corner coordinates in the view's (along-line e, line lc) pixel units
    const float ea = row ? (float)j0 - 0.5f * G.nx : (float)i0 - 0.5f * G.ny;
    const float eb = row ? (float)j1 - 0.5f * G.nx : (float)i1 - 0.5f * G.ny;
    const float la = row ? (float)i0 - 0.5f * G.ny : (float)j0 - 0.5f * G.nx;
    const float lb = row ? (float)i1 - 0.5f * G.ny : (float)j1 - 0.5f * G.nx;
    float kmn = 3.0e38f, kmx = -3.0e38f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float e = (c & 1) ? eb : ea, lc = (c & 2) ? lb : la;
        const float num = fmaf(e, im.x, lc * im.y), den = fmaf(e, im.z, fmaf(lc, im.w, G.dso));
        float t = num * rcp_approx(den);   // the window's one-bin margin absorbs the reciprocal's error
        if (G.arc) t = atanf(t);
        const float kf = fmaf(G.c_kf, t, G.k0);
        kmn = fminf(kmn, kf);
        kmx = fmaxf(kmx, kf);
    }
    if (kmx < -1.f || kmn > (float)G.nb + 1.f) return make_int2(1, 0);
    return make_int2(max((int)floorf(kmn) - 1, 0), min((int)floorf(kmx) + 1, G.nb - 1));
}

// Fused back-projection and relaxed update over one 16 x 16 pixel tile. The workgroup's eight waves are
// view groups: wave w back-projects the views w, w + 8, w + 16, ... onto the whole tile, each lane four
// consecutive pixels along the view's lines (1 x 4 for row sweep views, 4 x 1 for column sweep views).
// Each wave computes its views' bin windows and descriptors one view per lane (read back with readlane)
// and stages its current view in its own LDS slot (boundaries, residual x scale and their running sum
// over the window: one wave prefix sum), the next view's loads in flight meanwhile; the view loop needs no
// workgroup barrier. The lane's four pixels share their inner edges, so a view costs five edge
// evaluations for four pixels. The eight partial sums are added in a fixed order, then the first 256
// threads carry out the update, one pixel each.
constexpr int BP_NT = BP_TX * BP_TY;
constexpr int BP_GROUPS = 8;    // view groups (waves) per workgroup
constexpr int BP_SWIN = 125;    // widest window staged (bins); wider ones read the tables directly
constexpr int BP_SLOT = 128;    // staged entries per view (n + 1 for a window of n bins)

// Regularizer gradient and Huber curvature at pixel (i, j) of value xc: the pair terms of neighbours
// 0 .. 3 (axial) or 4 .. 7 (diagonal) of the 8 (4 directions, each pair seen from both sides) with potential
// POT, weighted by beta and the kappa factors. The neighbours' loads (nbr_load) are issued together
// and ahead of the pixel's own stores (one memory latency, not one per neighbour): a neighbour outside the
// image reads the pixel itself and enters with weight 0, so that its term (difference 0) leaves both sums
// unchanged.
// Four neighbours of a pixel: N0 = 0 the axial ones, N0 = 4 the diagonal ones.
struct Nbrs4 {
    float x[4], k[4];   // values and kappa factors (1 without kappa)
    float kc;           // the pixel's own kappa factor
    unsigned in;        // bit n: neighbour n lies in the image
};
template <int N0>
__device__ __forceinline__ Nbrs4 nbr_load(const UpdateArgs &U, int i, int j, int nx, int ny, unsigned idx)
{
    constexpr int di[8] = {0, 0, 1, -1, 1, -1, 1, -1};
    constexpr int dj[8] = {1, -1, 0, 0, 1, -1, -1, 1};
    Nbrs4 q;
    unsigned k[4];
    q.in = 0u;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        bool in = true;
        if (di[N0 + n] > 0) in = in && i + 1 < ny;
        if (di[N0 + n] < 0) in = in && i > 0;
        if (dj[N0 + n] > 0) in = in && j + 1 < nx;
        if (dj[N0 + n] < 0) in = in && j > 0;
        q.in |= in ? 1u << n : 0u;
        k[n] = in ? idx + (unsigned)(di[N0 + n] * nx + dj[N0 + n]) : idx;
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) q.x[n] = U.x[k[n]];
    q.kc = 1.f;
    if (U.kappa) {   // uniform
        q.kc = U.kappa[idx];
#pragma unroll
        for (int n = 0; n < 4; ++n) q.k[n] = U.kappa[k[n]];
    } else {
#pragma unroll
        for (int n = 0; n < 4; ++n) q.k[n] = 1.f;
    }
    return q;
}
// beta: the four neighbours' direction weight (beta_ax or beta_dg)
template <int POT>
__device__ __forceinline__ void reg_terms(const UpdateArgs &U, const Nbrs4 &q, float beta, float xc, float &gr,
                                          float &dr)
{
    gr = 0.f;
    dr = 0.f;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const float bt = (q.in >> n) & 1u ? beta * (q.kc * q.k[n]) : 0.f;
        float dphi, om;
        pot_terms<POT>(U.idelta, xc - q.x[n], dphi, om);
        gr = fmaf(bt, dphi, gr);
        dr = fmaf(bt, 2.f * (U.huber ? om : 1.f), dr);
    }
}
__device__ __forceinline__ void reg_stencil_pot(const UpdateArgs &U, const Nbrs4 &q, float beta, float xc, float &gr,
                                                float &dr)
{
    // one uniform branch on the potential per pixel, not one per neighbour
    if (U.potential == 0) reg_terms<0>(U, q, beta, xc, gr, dr);
    else if (U.potential == 1) reg_terms<1>(U, q, beta, xc, gr, dr);
    else reg_terms<2>(U, q, beta, xc, gr, dr);
}

struct BpShared {
    float tile_t[BP_TX][BP_TY + 1];
    float4 ent[BP_GROUPS][BP_SLOT];   // per wave: the staged view, then the wave's partial sums
    float2 reg_part[BP_NT];           // the diagonal neighbours' regularizer terms, from the second half
};

// R2 = 1: the residual is the sum of the two float32 planes of a split forward projection (a.r, a.r2);
// R2 = 2: the same where a.r2 is set (the float32 batched kernel, whose slices differ).
template <int MODE, typename TR, typename TXC, int R2>
__device__ __forceinline__ void bp_body(const BpLaunch &a, const int bx, const int by, BpShared &sh)
{
    static_assert(R2 == 0 || std::is_same<TR, float>::value, "split residual planes are float32");
    // the solver's residual blocks come from the forward epilogue already multiplied by the bin scale
    constexpr bool PRESCALED = MODE == BP_INIT || MODE == BP_FULL;
    const GeomDev &G = a.G;
    const UpdateArgs &U = a.U;
    const int vstart = a.vstart, vstride = a.vstride, nv = a.nv;
    const TR *__restrict__ r = static_cast<const TR *>(a.r);
    const float *__restrict__ r2 = static_cast<const float *>(a.r2);
    // threads 0 .. 255 (hv = 0) update pixel tid of the tile after the back-projection
    const int hv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / BP_NT));
    const int tid = threadIdx.x % BP_NT;
    const int lane = threadIdx.x & 63;
    const int tx = tid % BP_TX, ty = tid / BP_TX;
    const int j = bx * BP_TX + tx, i = by * BP_TY + ty;
    const int nx = G.nx, ny = G.ny, nb = G.nb;
    auto &tile_t = sh.tile_t;
    const bool inside = i < ny && j < nx;
    float zeta = 0.f;
    if (MODE != BP_XSTEP) {
        const int ti0 = by * BP_TY, ti1 = min(ti0 + BP_TY, ny);
        const int tj0 = bx * BP_TX, tj1 = min(tj0 + BP_TX, nx);
        const int tilesx = (nx + BP_TX - 1) / BP_TX, ntiles = tilesx * ((ny + BP_TY - 1) / BP_TY);
        const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // view group
        // The lane's pixels are four consecutive pixels of one line of the view, so that five edges give four
        // pixels: for row sweep views tile row r4 = lane % 16, columns q4 + {0..3} (q4 = 4 (lane / 16)), edges
        // along x; for column sweep views tile column r4, rows q4 + {0..3}, edges along y. Row and column
        // views accumulate separately (acc_r, acc_c) and meet in the partial sums. Consecutive lanes take
        // neighbouring lines, whose edges fall in the same or nearby staged entries (fewer LDS bank
        // conflicts than lanes four pixels apart along one line).
        const int r4 = lane & 15, q4 = 4 * (lane >> 4);
        const float lc_row = (float)(ti0 + r4) - 0.5f * (float)(ny - 1), ex_row = (float)(tj0 + q4) - 0.5f * (float)nx;
        const float lc_col = (float)(tj0 + r4) - 0.5f * (float)(nx - 1), ex_col = (float)(ti0 + q4) - 0.5f * (float)ny;
        float acc_r[4] = {0.f, 0.f, 0.f, 0.f}, acc_c[4] = {0.f, 0.f, 0.f, 0.f};
        float4 *E = sh.ent[wave];
        const int nvw = nv > wave ? (nv - wave + BP_GROUPS - 1) / BP_GROUPS : 0;   // views of this group
        for (int c0 = 0; c0 < nvw; c0 += 64) {
            const int cn = min(64, nvw - c0);
            // view wave + 8 (c0 + q) in lane q: the tile's bin window and staged entries (0: window too wide
            // to stage); the view's inverse map, boundary order and sweep mode are read by scalar loads
            int2 wq = make_int2(1, 0);
            int nq = 0;
            if (lane < cn) {
                const int v = vstart + (wave + BP_GROUPS * (c0 + lane)) * vstride;
                wq = G.win ? G.win[(unsigned)v * (unsigned)ntiles + (unsigned)(by * tilesx + bx)]
                           : tile_window(G, v, ti0, ti1, tj0, tj1);
                const int n = wq.y - wq.x + 1;
                nq = n > 0 && n <= BP_SWIN ? n + 1 : 0;
            }
            // staging of view ci: lane L loads entries 2L and 2L + 1; the running sum is formed on store
            // (residuals are kept as their raw bits until stored, so that all of a view's loads are in
            // flight together)
            struct Fetch {
                float2 b0, b1;
                RawT<TR> r0, r1;
                float s0, s1;   // bin scales (modes whose residual is not prescaled)
            };
            auto fetch = [&](int ci) {
                Fetch q = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), 0, 0, 1.f, 1.f};
                const int ne = __builtin_amdgcn_readlane(nq, ci);
                if (ne == 0) return q;
                const int kw0 = __builtin_amdgcn_readlane(wq.x, ci);
                const unsigned vi = (unsigned)(wave + BP_GROUPS * (c0 + ci));
                const unsigned v = (unsigned)vstart + vi * (unsigned)vstride;
                const int e0i = 2 * lane, e1i = e0i + 1;
                // 32-bit element offsets (the geometry keeps nviews * (nb + 1) below 2^31)
                const unsigned kb = v * (unsigned)(nb + 1) + (unsigned)(kw0 + e0i);
                const unsigned kr = vi * (unsigned)nb + (unsigned)(kw0 + e0i);
                const unsigned ks = v * (unsigned)nb + (unsigned)(kw0 + e0i);
                if (e0i < ne) q.b0 = G.bnd[kb];
                if (e1i < ne) q.b1 = G.bnd[kb + 1];
                if (e0i < ne - 1) {
                    q.r0 = ld_raw<TR>(r, kr);
                    if (!PRESCALED) q.s0 = G.scale[ks];
                }
                if (e1i < ne - 1) {
                    q.r1 = ld_raw<TR>(r, kr + 1);
                    if (!PRESCALED) q.s1 = G.scale[ks + 1];
                }
                if constexpr (R2 != 0) {
                    if (R2 == 1 || r2) {   // the second plane of a split forward projection
                        if (e0i < ne - 1) q.r0 += r2[kr];
                        if (e1i < ne - 1) q.r1 += r2[kr + 1];
                    }
                }
                return q;
            };
            auto put = [&](int ci, const Fetch &q) {
                const int ne = __builtin_amdgcn_readlane(nq, ci);
                if (ne == 0) return;
                const float s = ld_uniform(G.sgn, (unsigned)(vstart + (wave + BP_GROUPS * (c0 + ci)) * vstride));
                const int e0i = 2 * lane, e1i = e0i + 1;
                const float r0 = from_raw<TR>(q.r0) * q.s0, r1 = from_raw<TR>(q.r1) * q.s1;
                const float p0 = wave_shift_up(wave_prefix_sum(r0 + r1));
                if (e0i < ne) E[e0i] = make_float4(s * q.b0.x, s * q.b0.y, p0, r0);
                if (e1i < ne) E[e1i] = make_float4(s * q.b1.x, s * q.b1.y, p0 + r0, r1);
            };
            for (int ci = 0; ci < cn; ++ci) {
                // LDS operations of one wave complete in order: the previous view's reads precede these
                // stores. (Other waves of the CU run while this one waits for its loads.)
                put(ci, fetch(ci));
                const int kw0 = __builtin_amdgcn_readlane(wq.x, ci), kw1 = __builtin_amdgcn_readlane(wq.y, ci);
                if (kw0 <= kw1) {
                    const unsigned vu = (unsigned)(vstart + (wave + BP_GROUPS * (c0 + ci)) * vstride);
                    const float *imv = reinterpret_cast<const float *>(G.inv);
                    const float4 im = make_float4(ld_uniform(imv, 4 * vu), ld_uniform(imv, 4 * vu + 1),
                                                  ld_uniform(imv, 4 * vu + 2), ld_uniform(imv, 4 * vu + 3));
                    const bool row = ld_uniform(G.rowsweep, vu) != 0;
                    const bool pos = ld_uniform(G.sgn, vu) > 0.f;
                    const int ne = __builtin_amdgcn_readlane(nq, ci);
                    const float lc0 = row ? lc_row : lc_col, ex = row ? ex_row : ex_col;
                    float val[4];   // the lane's four pixels along the line
                    if (ne > 0) {
                        const float kofs = G.k0 - (float)kw0;
                        if (G.poly) {
                            if (pos) bp_line<4, true, true>(G, im, lc0, ex, ne - 1, kofs, E, val);
                            else bp_line<4, false, true>(G, im, lc0, ex, ne - 1, kofs, E, val);
                        } else {
                            if (pos) bp_line<4, true, false>(G, im, lc0, ex, ne - 1, kofs, E, val);
                            else bp_line<4, false, false>(G, im, lc0, ex, ne - 1, kofs, E, val);
                        }
                    } else {   // window wider than the staging slots: read the tables directly
                        const int vi = wave + BP_GROUPS * (c0 + ci);
                        const int v = vstart + vi * vstride;
                        const float2 *bv = G.bnd + (size_t)v * (nb + 1);
                        const float *sv = G.scale + (size_t)v * nb;
                        const TR *rv = r + (size_t)vi * nb;
                        const float *rv2 = (R2 != 0 && r2) ? r2 + (size_t)vi * nb : nullptr;   // a split projection's second plane
                        auto rs = [&](int k) {
                            float rk = (float)rv[k];
                            if constexpr (R2 != 0) {
                                if (R2 == 1 || rv2) rk += rv2[k];
                            }
                            return PRESCALED ? rk : rk * sv[k];
                        };
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            val[m] = bp_view(G, im, lc0, ex + (float)m, kw0, kw1, [&](int k) { return bv[k]; }, rs);
                    }
                    if (row) {
#pragma unroll
                        for (int m = 0; m < 4; ++m) acc_r[m] += val[m];
                    } else {
#pragma unroll
                        for (int m = 0; m < 4; ++m) acc_c[m] += val[m];
                    }
                }
            }
        }
        // partial sums of the group, by tile pixel, in the wave's own slot (its staged reads are complete)
        // (row views' pixels (r4, q4 + m) first; then each lane adds its column views' pixels (q4 + m, r4):
        // every pixel of the tile takes one value of each kind, and the wave's LDS operations are in order)
        float *part = reinterpret_cast<float *>(E);
        *reinterpret_cast<float4 *>(part + r4 * BP_TX + q4) = make_float4(acc_r[0], acc_r[1], acc_r[2], acc_r[3]);
#pragma unroll
        for (int m = 0; m < 4; ++m) part[(q4 + m) * BP_TX + r4] += acc_c[m];
        __syncthreads();
        if (hv == 0) {
#pragma unroll
            for (int w = 0; w < BP_GROUPS; ++w) zeta += reinterpret_cast<const float *>(sh.ent[w])[tid];
        }
    }
    float xn = 0.f;
    // operands of the x-step, kept over the barrier below: s, rho1, d, xc and the axial regularizer terms
    float xs_s = 0.f, xs_rho1 = 0.f, xs_d = 0.f, xs_xc = 0.f, gr = 0.f, dr = 0.f;
    if (hv == 0 && inside) {   // half 1 only evaluates the diagonal regularizer terms from here on
        const unsigned idx = (unsigned)i * (unsigned)nx + (unsigned)j;
        if (MODE == BP_BACK) {
            a.out_back[idx] = zeta;
        } else {
            const float xc = U.x[idx];
            const float d = U.dl[idx];
            float g = U.gv[idx], hh = U.h[idx];
            Nbrs4 nb;   // the axial neighbours, loaded ahead of this pixel's stores
            if (MODE == BP_FULL || MODE == BP_XSTEP) nb = nbr_load<0>(U, i, j, nx, ny, idx);
            const long long t = (U.tbase ? (long long)(*U.tbase) : 0ll) + U.tofs;
            if (MODE == BP_INIT) {
                g = zeta;
                hh = U.algorithm == 1 ? fmaf(d, xc, -zeta) : zeta;
                U.gv[idx] = g;
                U.h[idx] = hh;
            } else if (MODE == BP_FULL) {
                const float rho = U.rho[t];
                const float a = U.alpha;
                const float inv1 = rcp_approx(rho + 1.f);
                const float gn = rho * inv1 * (a * zeta + (1.f - a) * g) + g * inv1;
                const float hn = U.algorithm == 1 ? a * fmaf(d, xc, -zeta) + (1.f - a) * hh : zeta;
                g = gn;
                hh = hn;
                U.gv[idx] = g;
                U.h[idx] = hh;
            }
            if (MODE == BP_FULL || MODE == BP_XSTEP) {
                const long long tx1 = MODE == BP_FULL ? t + 1 : t;
                const float rho1 = U.rho[tx1];
                const float s = U.algorithm == 1 ? rho1 * fmaf(d, xc, -hh) + (1.f - rho1) * g
                                                 : rho1 * hh + (1.f - rho1) * g;
                // regularizer gradient and Huber curvature at xc: the axial neighbours here, the diagonal
                // ones by the second half of the workgroup (below), added after the barrier
                reg_stencil_pot(U, nb, U.beta_ax, xc, gr, dr);
                xs_s = s;
                xs_rho1 = rho1;
                xs_d = d;
                xs_xc = xc;
            }
        }
    }
    if (MODE == BP_FULL || MODE == BP_XSTEP) {
        if (hv == 1 && inside) {
            const unsigned idx = (unsigned)i * (unsigned)nx + (unsigned)j;
            float g2, d2;
            reg_stencil_pot(U, nbr_load<4>(U, i, j, nx, ny, idx), U.beta_dg, U.x[idx], g2, d2);
            sh.reg_part[tid] = make_float2(g2, d2);
        }
        __syncthreads();
        if (hv == 0 && inside) {
            const unsigned idx = (unsigned)i * (unsigned)nx + (unsigned)j;
            const float2 q = sh.reg_part[tid];
            gr += q.x;
            dr += q.y;
            const float den = fmaf(xs_rho1, xs_d, dr);
            xn = den > 0.f ? fmaxf(xs_xc - (xs_s + gr) * rcp_approx(den), 0.f) : xs_xc;
            U.x_next[idx] = xn;
            if (!std::is_same<TXC, float>::value) st<TXC>(U.xc_next, idx, xn);
        }
        // transpose through LDS: write xT_next[j][i] in runs of BP_TY along i
        if (hv == 0) tile_t[tx][ty] = xn;
        __syncthreads();
        const int jj = bx * BP_TX + ty;   // swapped roles
        const int ii = by * BP_TY + tx;
        if (hv == 0 && jj < nx && ii < ny) st<TXC>(U.xT_next, (unsigned)jj * (unsigned)ny + (unsigned)ii, tile_t[ty][tx]);
    }
}

// Eight waves per SIMD (four workgroups per CU): the register budget is held to that occupancy.
template <int MODE, typename TR, typename TXC, int R2>
__global__ __launch_bounds__(2 * BP_TX *BP_TY) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_back_update(BpLaunch a)
{
    __shared__ BpShared sh;
    bp_body<MODE, TR, TXC, R2>(a, blockIdx.x, blockIdx.y, sh);
}

// The bin window of every (view, tile) pair, as bp_body would compute it: one thread per pair.
__global__ __launch_bounds__(256) void k_tile_windows(GeomDev G, int2 *__restrict__ out)
{
    const int tilesx = (G.nx + BP_TX - 1) / BP_TX, ntiles = tilesx * ((G.ny + BP_TY - 1) / BP_TY);
    const unsigned q = blockIdx.x * 256u + threadIdx.x;
    if (q >= (unsigned)G.nviews * (unsigned)ntiles) return;
    const int v = (int)(q / (unsigned)ntiles), tile = (int)(q % (unsigned)ntiles);
    const int bx = tile % tilesx, by = tile / tilesx;
    const int ti0 = by * BP_TY, ti1 = min(ti0 + BP_TY, G.ny);
    const int tj0 = bx * BP_TX, tj1 = min(tj0 + BP_TX, G.nx);
    out[q] = tile_window(G, v, ti0, ti1, tj0, tj1);
}

// Batched fused back-projection / relaxed update of subset m: every slice reads image buffer par and
// its residual block, and writes image buffer par ^ 1 (and its copies). The work of workgroup b.
template <typename T>
__device__ __forceinline__ void update_item(const SliceDev *__restrict__ tab, int ns, int m, int par,
                                            const BatchUpdate &u, int b, BpShared &sh)
{
    const int s = find_slice<false>(tab, ns, b);
    const SliceDev &S = tab[s];
    BpLaunch a;
    a.G = S.G;
    a.r = S.r;
    a.r2 = S.r2;
    a.vstart = m;
    a.vstride = S.M;
    a.nv = S.nvm;
    a.U.x = S.x[par];
    a.U.x_next = S.x[par ^ 1];
    a.U.xc_next = S.xc[par ^ 1];
    a.U.xT_next = S.xt[par ^ 1];
    a.U.gv = S.gv;
    a.U.h = S.h;
    a.U.dl = S.dl;
    a.U.kappa = S.kappa;
    a.U.rho = u.rho;
    a.U.tbase = u.tbase;
    a.U.tofs = u.tofs;
    a.U.alpha = u.alpha;
    a.U.algorithm = u.algorithm;
    a.U.potential = u.potential;
    a.U.delta = u.delta;
    a.U.idelta = u.idelta;
    a.U.beta_ax = u.beta_ax;
    a.U.beta_dg = u.beta_dg;
    a.U.huber = u.huber;
    const int local = b - S.bp_begin;
    const int tilesx = (S.G.nx + BP_TX - 1) / BP_TX;
    if constexpr (std::is_same<T, float>::value) {
        bp_body<BP_FULL, float, float, 2>(a, local % tilesx, local / tilesx, sh);
    } else {   // 16-bit slices: the two float32 residual planes of a split projection, or one 16-bit block
        if (S.r2) bp_body<BP_FULL, float, T, 1>(a, local % tilesx, local / tilesx, sh);
        else bp_body<BP_FULL, T, T, 0>(a, local % tilesx, local / tilesx, sh);
    }
}

template <typename T>
__global__ __launch_bounds__(2 * BP_TX *BP_TY) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_update_batch(const SliceDev *__restrict__ tab, int ns, int m,
                                                                    int par, BatchUpdate u)
{
    __shared__ BpShared sh;
    update_item<T>(tab, ns, m, par, u, blockIdx.x, sh);
}

// Memory operations of the grid barrier in a kernel: the workgroup's first thread arrives and waits with
// agent-scope atomics and fences (the release fence writes this XCD's L2 back, the acquire fence drops
// stale lines, so the next phase sees every workgroup's results on every XCD); the outcome reaches the
// other threads through LDS.
struct DevBarrierOps {
    int *flag;
    __device__ void block_sync() { __syncthreads(); }
    __device__ bool leader() { return threadIdx.x == 0; }
    __device__ int load(int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ int load_acquire(int *p) { return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ void store(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ void store_release(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ int fetch_add(int *p, int v)
    {
        return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ void release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
    __device__ void acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
    __device__ void pause() { __builtin_amdgcn_s_sleep(2); }
    __device__ void set_block_flag(int v) { *flag = v; }
    __device__ int block_flag() { return *flag; }
};

union PersistentShared {
    BpShared bp;
    float win[8 * (FP_WIN + 4)];
};

// The whole batched iteration in one launch: subiterations t0 .. t0 + nsub - 1, each a forward phase over
// the batched forward grid's nwg_fp work items and an update phase over the nwg_bp update tiles, the items
// taken by the resident workgroups in strides of the grid, with a grid barrier after each phase. The
// forward items run the 8-wave body (the workgroup is the update's 512 threads). Images ping-pong from
// buffer par0 at t0. state: 4 ints, zero at launch (barrier arrivals, generation, error flag in 1..3).
template <typename T>
__global__ __launch_bounds__(2 * BP_TX *BP_TY) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_batch_persistent(
    const SliceDev *__restrict__ tab, int ns, int nwg_fp, int nwg_bp, const int *__restrict__ order, int M, long long t0,
    long long nsub, int par0, BatchUpdate u, int *state, unsigned spin_limit)
{
    __shared__ PersistentShared sh;
    __shared__ int flag;
    DevBarrierOps ops{&flag};
    const int nblk = (int)gridDim.x;
    u.tbase = nullptr;   // rho index = tofs = t
    for (long long k = 0; k < nsub; ++k) {
        const long long t = t0 + k;
        const int m = order[(int)(t % M)];
        const int par = (par0 + (int)(k & 1)) & 1;
        for (int b = (int)blockIdx.x; b < nwg_fp; b += nblk) {
            forward_item<8, T>(tab, ns, m, par, b, sh.win);
            __syncthreads();
        }
        if (!grid_barrier(ops, state, nblk, spin_limit)) return;
        u.tofs = t;
        for (int b = (int)blockIdx.x; b < nwg_bp; b += nblk) {
            update_item<T>(tab, ns, m, par, u, b, sh.bp);
            __syncthreads();
        }
        if (!grid_barrier(ops, state, nblk, spin_limit)) return;
    }
}

__global__ void k_fill_int(int *p, int n, int v)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = v;
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

template <typename TXC>
__global__ void k_clip_copy(const float *__restrict__ in, float *__restrict__ out, void *__restrict__ outc,
                            void *__restrict__ outT, int nx, int ny, int zero)
{
    __shared__ float tile[16][17];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    int j = blockIdx.x * 16 + tx, i = blockIdx.y * 16 + ty;
    float v = 0.f;
    if (i < ny && j < nx) {
        v = zero ? 0.f : fmaxf(in[(size_t)i * nx + j], 0.f);
        out[(size_t)i * nx + j] = v;
        if (outc) st<TXC>(outc, (size_t)i * nx + j, v);
    }
    tile[ty][tx] = v;
    __syncthreads();
    int ii = blockIdx.y * 16 + tx, jj = blockIdx.x * 16 + ty;
    if (ii < ny && jj < nx) st<TXC>(outT, (size_t)jj * ny + ii, tile[tx][ty]);
}

template <typename T>
__global__ void k_to_float(const void *__restrict__ src, float *__restrict__ dst, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = ld<T>(src, i);
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

}  // namespace

int forward_workgroups(const GeomDev &G, int nv, int, bool split)
{
    return ((G.nb + FP_BINS - 1) / FP_BINS) * nv * (split ? 2 : 1);
}

// A float32 subset projection whose (block, view) workgroups would number fewer than two per CU (512 on
// the 256 CUs) splits each block's lines over two workgroups, which halves the chain of line steps that
// bounds a workgroup. The halves write two residual planes (the data term in the first), which the update
// kernel adds when it stages a view; both planes must fit the residual block of nviews views. The planes
// are float32 in every storage mode: two 16-bit partial residuals would round before they cancel.
bool split_eligible(const GeomDev &, int nv, int nviews, int) { return 2 * nv <= nviews; }
bool launch_underfills(int forward_wgs) { return forward_wgs < 512; }
bool forward_split(const GeomDev &G, int nv, int nviews, int dtype)
{
    return split_eligible(G, nv, nviews, dtype) && launch_underfills(((G.nb + FP_BINS - 1) / FP_BINS) * nv);
}

int update_workgroups(const GeomDev &G) { return ((G.nx + BP_TX - 1) / BP_TX) * ((G.ny + BP_TY - 1) / BP_TY); }

// Storage-typed instantiations: float32 keeps every epilogue; 16-bit storage needs the subset residual
// (image copy, y, w and r in 16 bits) and the weighted ones projection for D_L (w in 16 bits, output
// float32, so that the majorizer is computed from float32 sums).
hipError_t launch_forward(const FpLaunch &a, int ones, int epi, int dtype, hipStream_t s)
{
    if (a.nv <= 0) return hipSuccess;
    if (a.out2 && (epi != FP_RESIDUAL || ones)) return hipErrorInvalidValue;
    dim3 grid(((a.G.nb + FP_BINS - 1) / FP_BINS) * (a.out2 ? 2 : 1), a.nv), block(FP_BINS * FP_WAVES);
#define CT_FP(E, O, TI, TY, TO) hipLaunchKernelGGL((k_forward<E, O, FP_WAVES, TI, TY, TO, false>), grid, block, 0, s, a)
    if (a.out2) {   // split: float32 residual planes in every storage mode
        if (dtype == CT_F32)
            hipLaunchKernelGGL((k_forward<FP_RESIDUAL, false, FP_WAVES, float, float, float, true>), grid, block, 0, s, a);
        else if (dtype == CT_F16)
            hipLaunchKernelGGL((k_forward<FP_RESIDUAL, false, FP_WAVES, _Float16, _Float16, float, true>), grid, block, 0,
                               s, a);
        else if (dtype == CT_BF16)
            hipLaunchKernelGGL((k_forward<FP_RESIDUAL, false, FP_WAVES, __bf16, __bf16, float, true>), grid, block, 0, s,
                               a);
        else
            return hipErrorInvalidValue;
    } else if (dtype == CT_F32) {
        if (ones) {
            if (epi == FP_PLAIN) CT_FP(FP_PLAIN, true, float, float, float);
            else if (epi == FP_RESIDUAL) CT_FP(FP_RESIDUAL, true, float, float, float);
            else CT_FP(FP_WEIGHTED, true, float, float, float);
        } else {
            if (epi == FP_PLAIN) CT_FP(FP_PLAIN, false, float, float, float);
            else if (epi == FP_RESIDUAL) CT_FP(FP_RESIDUAL, false, float, float, float);
            else CT_FP(FP_WEIGHTED, false, float, float, float);
        }
    } else if (dtype == CT_F16) {
        if (!ones && epi == FP_RESIDUAL) CT_FP(FP_RESIDUAL, false, _Float16, _Float16, _Float16);
        else if (ones && epi == FP_WEIGHTED) CT_FP(FP_WEIGHTED, true, float, _Float16, float);
        else return hipErrorInvalidValue;
    } else if (dtype == CT_BF16) {
        if (!ones && epi == FP_RESIDUAL) CT_FP(FP_RESIDUAL, false, __bf16, __bf16, __bf16);
        else if (ones && epi == FP_WEIGHTED) CT_FP(FP_WEIGHTED, true, float, __bf16, float);
        else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
#undef CT_FP
    return hipGetLastError();
}

size_t tile_windows_count(const GeomDev &G)
{
    return (size_t)G.nviews * (size_t)((G.nx + BP_TX - 1) / BP_TX) * (size_t)((G.ny + BP_TY - 1) / BP_TY);
}

hipError_t launch_tile_windows(const GeomDev &G, int2 *out, hipStream_t s)
{
    const size_t n = tile_windows_count(G);
    if (n == 0 || n >= (size_t(1) << 31)) return hipErrorInvalidValue;   // 32-bit entry index
    hipLaunchKernelGGL(k_tile_windows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, out);
    return hipGetLastError();
}

// rtype: type of r (BP_BACK: float32 or storage type; update modes: storage type). ctype: type of the
// image copies written by the x-step.
hipError_t launch_back_update(const BpLaunch &a, int mode, int rtype, int ctype, hipStream_t s)
{
    dim3 grid((a.G.nx + BP_TX - 1) / BP_TX, (a.G.ny + BP_TY - 1) / BP_TY), block(2 * BP_TX * BP_TY);
#define CT_BP(M, TR, TC) hipLaunchKernelGGL((k_back_update<M, TR, TC, 0>), grid, block, 0, s, a)
#define CT_BP_ALL(T)                                                                                           \
    if (mode == BP_INIT) CT_BP(BP_INIT, T, T);                                                                 \
    else if (mode == BP_FULL) CT_BP(BP_FULL, T, T);                                                            \
    else if (mode == BP_XSTEP) CT_BP(BP_XSTEP, T, T);                                                          \
    else return hipErrorInvalidValue;
    if (a.r2) {   // a split forward projection's two float32 residual planes, any image-copy storage
#define CT_BP2(T)                                                                                              \
    if (mode == BP_INIT) hipLaunchKernelGGL((k_back_update<BP_INIT, float, T, 1>), grid, block, 0, s, a);      \
    else hipLaunchKernelGGL((k_back_update<BP_FULL, float, T, 1>), grid, block, 0, s, a);
        if (rtype != CT_F32 || (mode != BP_INIT && mode != BP_FULL)) return hipErrorInvalidValue;
        if (ctype == CT_F32) {
            CT_BP2(float)
        } else if (ctype == CT_F16) {
            CT_BP2(_Float16)
        } else if (ctype == CT_BF16) {
            CT_BP2(__bf16)
        } else {
            return hipErrorInvalidValue;
        }
#undef CT_BP2
    } else if (mode == BP_BACK) {
        if (rtype == CT_F32) CT_BP(BP_BACK, float, float);
        else if (rtype == CT_F16) CT_BP(BP_BACK, _Float16, float);
        else if (rtype == CT_BF16) CT_BP(BP_BACK, __bf16, float);
        else return hipErrorInvalidValue;
    } else {
        if (rtype != ctype) return hipErrorInvalidValue;
        if (ctype == CT_F32) {
            CT_BP_ALL(float)
        } else if (ctype == CT_F16) {
            CT_BP_ALL(_Float16)
        } else if (ctype == CT_BF16) {
            CT_BP_ALL(__bf16)
        } else {
            return hipErrorInvalidValue;
        }
    }
#undef CT_BP_ALL
#undef CT_BP
    return hipGetLastError();
}

hipError_t launch_forward_batch(const SliceDev *tab, int ns, int nwg_fp, int m, int par, int dtype, int fp_waves,
                                hipStream_t s)
{
    if (ns <= 0 || nwg_fp <= 0) return hipSuccess;
#define CT_FPB(W, T) hipLaunchKernelGGL((k_forward_batch<W, T>), dim3(nwg_fp), dim3(FP_BINS * W), 0, s, tab, ns, m, par)
#define CT_FPB_W(T)                                                                                            \
    if (fp_waves == 8) CT_FPB(8, T);                                                                           \
    else if (fp_waves == 16) CT_FPB(16, T);                                                                    \
    else return hipErrorInvalidValue;
    if (dtype == CT_F32) {
        CT_FPB_W(float)
    } else if (dtype == CT_F16) {
        CT_FPB_W(_Float16)
    } else if (dtype == CT_BF16) {
        CT_FPB_W(__bf16)
    } else {
        return hipErrorInvalidValue;
    }
#undef CT_FPB_W
#undef CT_FPB
    return hipGetLastError();
}

hipError_t launch_update_batch(const SliceDev *tab, int ns, int nwg_bp, int m, int par, const BatchUpdate &u,
                               int dtype, hipStream_t s)
{
    if (ns <= 0 || nwg_bp <= 0) return hipSuccess;
    dim3 grid(nwg_bp), block(2 * BP_TX * BP_TY);
    if (dtype == CT_F32) hipLaunchKernelGGL(k_update_batch<float>, grid, block, 0, s, tab, ns, m, par, u);
    else if (dtype == CT_F16) hipLaunchKernelGGL(k_update_batch<_Float16>, grid, block, 0, s, tab, ns, m, par, u);
    else if (dtype == CT_BF16) hipLaunchKernelGGL(k_update_batch<__bf16>, grid, block, 0, s, tab, ns, m, par, u);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

int persistent_blocks_per_cu(int dtype)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    if (dtype == CT_F32) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_persistent<float>, 2 * BP_TX * BP_TY, 0);
    else if (dtype == CT_F16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_persistent<_Float16>, 2 * BP_TX * BP_TY, 0);
    else if (dtype == CT_BF16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_persistent<__bf16>, 2 * BP_TX * BP_TY, 0);
    return e == hipSuccess ? n : 0;
}

hipError_t launch_batch_persistent(const SliceDev *tab, int ns, int nwg_fp, int nwg_bp, const int *order, int M,
                                   long long t0, long long nsub, int par0, const BatchUpdate &u, int *state,
                                   int blocks, int dtype, hipStream_t s)
{
    if (ns <= 0 || nsub <= 0) return hipSuccess;
    if (blocks < 1) return hipErrorInvalidValue;
    constexpr unsigned kSpinLimit = 1u << 20;   // polls of about 50 ns: a waiting workgroup gives up after ~50 ms
    const dim3 grid(blocks), block(2 * BP_TX * BP_TY);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, state, 4, 0);
#define CT_PB(T) hipLaunchKernelGGL(k_batch_persistent<T>, grid, block, 0, s, tab, ns, nwg_fp, nwg_bp, order, M, t0, nsub, \
                                    par0, u, state, kSpinLimit)
    if (dtype == CT_F32) CT_PB(float);
    else if (dtype == CT_F16) CT_PB(_Float16);
    else if (dtype == CT_BF16) CT_PB(__bf16);
    else return hipErrorInvalidValue;
#undef CT_PB
    return hipGetLastError();
}

hipError_t launch_transpose(const float *x, float *xT, int nx, int ny, hipStream_t s)
{
    dim3 grid((nx + 15) / 16, (ny + 15) / 16);
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, x, xT, nx, ny);
    return hipGetLastError();
}

hipError_t launch_clip_copy(const float *in, float *out, void *outc, void *outT, int nx, int ny, int zero, int ctype,
                            hipStream_t s)
{
    dim3 grid((nx + 15) / 16, (ny + 15) / 16);
    if (ctype == CT_F32) hipLaunchKernelGGL(k_clip_copy<float>, grid, dim3(256), 0, s, in, out, outc, outT, nx, ny, zero);
    else if (ctype == CT_F16)
        hipLaunchKernelGGL(k_clip_copy<_Float16>, grid, dim3(256), 0, s, in, out, outc, outT, nx, ny, zero);
    else if (ctype == CT_BF16)
        hipLaunchKernelGGL(k_clip_copy<__bf16>, grid, dim3(256), 0, s, in, out, outc, outT, nx, ny, zero);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_to_float(const void *src, int ctype, float *dst, size_t n, hipStream_t s)
{
    dim3 grid((unsigned)((n + 255) / 256));
    if (ctype == CT_F32) hipLaunchKernelGGL(k_to_float<float>, grid, dim3(256), 0, s, src, dst, n);
    else if (ctype == CT_F16) hipLaunchKernelGGL(k_to_float<_Float16>, grid, dim3(256), 0, s, src, dst, n);
    else if (ctype == CT_BF16) hipLaunchKernelGGL(k_to_float<__bf16>, grid, dim3(256), 0, s, src, dst, n);
    else return hipErrorInvalidValue;
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

}  // namespace ct
