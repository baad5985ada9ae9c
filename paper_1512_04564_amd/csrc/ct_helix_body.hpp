// Per-thread bodies of the 3-D helical projector pair and update (host + device).
//
// The kernels in ct_helix.hip wrap these functions; the same functions compiled for the host let a CPU
// emulation run every index computation of the kernels under bounds checks (Ro below checks its index on
// the host and compiles to a plain load on the device).
//
// Geometry (separable distance-driven helical cone-beam projector): view v sweeps voxel planes ("lines")
// y = y_i (row sweep) or x = x_j, as the fan-beam projector does. Within a plane, voxel column q and bin k
// overlap by f_t = |[q, q+1] cap [U_k, U_k+1]| / |U_k+1 - U_k| (voxel units along the line, U_k from the
// fan-beam boundary table: U_k = fmaf(lc, B_k, A_k) + NQ / 2, lc the centred line index). Row r of the
// detector meets voxel kz of that column by f_a = |[kz, kz+1] cap [z_r, z_r+1]| / |z_r+1 - z_r| with
// z_r = za_v + ell * wr_r (voxel units), ell = x_c cos b + y_c sin b + dso the depth of the column centre
// along the central ray and wr_r = w_r / (dsd dz). The weight is scale_k * secphi_rk * f_t * f_a.
// Precision: overlaps are taken where FP32 rounding stays relative to a voxel, not to the volume. Along the
// line the boundary crossings U_k reach hundreds of voxels, where FP32 would round them by 1e-5 voxel or
// more; they are evaluated in FP64 from an FP64 table, and the forward projector forms each overlap in
// FP64, the back-projector each crossing relative to the column's edge, before rounding to FP32. Along z
// the view's source height is split into an integer voxel index zai and a fraction zaf: voxel kz spans
// [kz - zai, kz - zai + 1] exactly, and the row boundaries zaf + ell wr_r stay within a few tens of voxels.
// The forward projector integrates a column along z from its cumulative form, whose partial sums are
// accumulated in FP64 and rounded once.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <cstddef>

namespace ct {

#if defined(__HIP_DEVICE_COMPILE__)
#define HX_CHECK(cond, idx) ((void)0)
#else
// Host emulation: out-of-range reads are counted and the first offending index kept; the read itself then
// returns element 0 instead.
inline long long &hx_oob_index()
{
    static long long v = -1;
    return v;
}
inline int &hx_oob_count()
{
    static int n = 0;
    return n;
}
#define HX_CHECK(cond, idx)                                  \
    do {                                                     \
        if (!(cond)) {                                       \
            if (::ct::hx_oob_count()++ == 0) ::ct::hx_oob_index() = (long long)(idx); \
        }                                                    \
    } while (0)
#endif

template <typename T>
struct Ro {
    const T *p;
    size_t n;
    __host__ __device__ T operator[](size_t i) const
    {
#if defined(__HIP_DEVICE_COMPILE__)
        return p[i];
#else
        HX_CHECK(i < n, i);
        return i < n ? p[i] : p[0];
#endif
    }
};

// Device view of a helical scan's tables.
struct HelixDev {
    int nx, ny, nz, nb, nr, nviews;
    float dx, dy;          // voxel size (mm): column centres
    float dso;             // source to isocentre (mm)
    float c_kf, k0;        // inverse map of the fan-beam tables: bin kf = c_kf * ratio + k0
    float dwn;             // wr_(r+1) - wr_r = dw / (dsd dz)
    Ro<double2> bnd;       // [nviews][nb + 1] (A, B) in FP64: U_k = A + lc B
    Ro<float> scale;       // [nviews][nb] plane spacing / |cos theta|
    Ro<float4> inv;        // [nviews] inverse map (na, nl, da, dl)
    Ro<int> rowsweep;      // [nviews]
    Ro<float2> cs;         // [nviews] (cos b, sin b)
    Ro<float> zai, zaf;    // [nviews] (S_z - z_lo) / dz split into its integer part and the fraction [0, 1)
    Ro<float> wr;          // [nr + 1] w_r / (dsd dz)
    Ro<float> secphi;      // [nr][nb]
};

__host__ __device__ inline int hx_min(int a, int b) { return a < b ? a : b; }

// Approximate reciprocal square root (one ulp on the device), for the potentials' weights.
__host__ __device__ inline float hx_rsqrt(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.f / sqrtf(x);
#endif
}

// Approximate reciprocal (one ulp on the device), for weights and candidate ranges.
__host__ __device__ inline float hx_rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.f / x;
#endif
}


// Rows per forward-projection workgroup and waves per forward workgroup; voxels per back-projection thread.
constexpr int HX_RB = 8;
constexpr int HX_FW = 4;
constexpr int HX_ZG = 8;
constexpr int HX_KC = 4;   // candidate bins per view kept in registers by the back-projector

// Centre of voxel column q on line lc (world mm) and its depth ell along the view's central ray.
__host__ __device__ inline float column_depth(const HelixDev &G, bool row, float lc, int q, float2 cs)
{
    const float xc = row ? ((float)q - 0.5f * (float)(G.nx - 1)) * G.dx : lc * G.dx;
    const float yc = row ? lc * G.dy : ((float)q - 0.5f * (float)(G.ny - 1)) * G.dy;
    return fmaf(xc, cs.x, fmaf(yc, cs.y, G.dso));
}

// Point z of the view's z frame (voxel kz spans [kz - zai, kz - zai + 1]) as a voxel index and the fraction
// above its lower face, clamped to the volume: below it (k, f) = (0, 0), above it (nz - 1, 1). The integer
// part and the fraction are taken in the view's frame, where |z| stays within the cone, so f is exact.
__host__ __device__ inline void hx_cum_point(float z, int zi, int nz, int &k, float &f)
{
    const float fl = floorf(z);
    k = (int)fl + zi;
    f = z - fl;
    if (k < 0) {
        k = 0;
        f = 0.f;
    } else if (k >= nz) {
        k = nz - 1;
        f = 1.f;
    }
}

__host__ __device__ inline int hx_clampi(int v, int lo, int hi)
{
    const int a = v < hi ? v : hi;
    return a > lo ? a : lo;
}

// a * b for a, b < 2^24 (the full-rate 24-bit multiply on the device); the product must fit 32 bits.
__host__ __device__ inline unsigned hx_mul24(unsigned a, unsigned b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul24(a, b);
#else
    return a * b;
#endif
}

// Forward projection, one lane: bin k of view v, rows r0 .. r0 + HX_RB - 1 (rows >= nr are skipped),
// lines l0, l0 + lstep, ... < NL. acc[rr] += f_t * (integral of the column over the row's z interval) /
// (row height) over the lane's lines; the caller multiplies by scale_k * secphi. Cz: the cumulative form of
// the volume in the view's sweep layout (x for row sweep views, its per-slice transpose for the others),
// padded by one plane on each side: Cz[kz + 1][col] = (sum of the column's voxels below kz, voxel kz) for
// kz in [0, nz), Cz[0] = (0, 0) and Cz[nz + 1] = (column sum, 0). The column's integral from the volume's
// lower face to height k + f is then C = S + f X at the index clamped to [-1, nz] (one integer clamp: the
// padding planes give 0 below the volume and the column sum above it), and a row costs one evaluation of
// C at its upper face (its lower face's value is the previous row's). ONES: every voxel is 1 (C = k + f
// clamped to [0, nz]; Cz is not read).
template <bool ONES>
__host__ __device__ inline void hfp_lane(const HelixDev &G, const Ro<float2> &Cz, int v, int k, int r0, int l0,
                                         int lstep, float (&acc)[HX_RB])
{
    const bool row = G.rowsweep[v] != 0;
    const int NL = row ? G.ny : G.nx, NQ = row ? G.nx : G.ny;
    const size_t bb = (size_t)v * (G.nb + 1) + k;
    const double2 b0 = G.bnd[bb], b1 = G.bnd[bb + 1];
    const float2 cs = G.cs[v];
    const int zi = (int)G.zai[v];
    const float zaf = G.zaf[v];
    float wr[HX_RB + 1];
#pragma unroll
    for (int rr = 0; rr <= HX_RB; ++rr) wr[rr] = G.wr[(size_t)hx_min(r0 + rr, G.nr)];
    const double halfq = 0.5 * (double)NQ, cl = 0.5 * (double)(NL - 1);
    const size_t plane = (size_t)NL * NQ;
    const float rdwn = 1.f / G.dwn;
    for (int l = l0; l < NL; l += lstep) {
        const double lcd = (double)l - cl;
        const float lc = (float)lcd;
        const double ua = fma(lcd, b0.y, b0.x), ub = fma(lcd, b1.y, b1.x);
        const double lo = fmin(ua, ub), hi = fmax(ua, ub);
        if (!(hi > lo)) continue;
        const float invt = hx_rcp((float)(hi - lo));
        const int qa = (int)floor(fmax(lo + halfq, 0.0));
        const int qb = (int)ceil(fmin(hi + halfq, (double)NQ)) - 1;
        for (int q = qa; q <= qb; ++q) {
            const double e0 = (double)q - halfq;   // the column spans [e0, e0 + 1] (exact)
            const float ft = (float)(fmin(hi, e0 + 1.0) - fmax(lo, e0)) * invt;
            if (!(ft > 0.f)) continue;
            const float ell = column_depth(G, row, lc, q, cs);
            const float w = ft * rdwn * hx_rcp(ell);
            const size_t col = (size_t)l * NQ + q;
            if (ONES) {
                int kp;
                float fp;
                hx_cum_point(fmaf(ell, wr[0], zaf), zi, G.nz, kp, fp);
#pragma unroll
                for (int rr = 0; rr < HX_RB; ++rr) {
                    int kn;
                    float fn;
                    hx_cum_point(fmaf(ell, wr[rr + 1], zaf), zi, G.nz, kn, fn);
                    if (r0 + rr < G.nr) acc[rr] = fmaf(w, (float)(kn - kp) + (fn - fp), acc[rr]);
                    kp = kn;
                    fp = fn;
                }
            } else {
                // 32-bit element index (the descriptor check keeps the padded volume below 2^31 elements
                // and a plane below 2^24)
                const unsigned col32 = (unsigned)col, plane32 = (unsigned)plane;
                auto cum = [&](float z) {
                    const float fl = floorf(z);
                    const unsigned kk = (unsigned)(hx_clampi((int)fl + zi, -1, G.nz) + 1);
                    const float2 c = Cz[hx_mul24(kk, plane32) + col32];
                    return fmaf(z - fl, c.y, c.x);
                };
                float Cp = cum(fmaf(ell, wr[0], zaf));
#pragma unroll
                for (int rr = 0; rr < HX_RB; ++rr) {
                    const float Cn = cum(fmaf(ell, wr[rr + 1], zaf));
                    if (r0 + rr < G.nr) acc[rr] = fmaf(w, Cn - Cp, acc[rr]);
                    Cp = Cn;
                }
            }
        }
    }
}

// Residual prescaling: the back-projector reads r'[v][r][k] = scale_vk secphi_rk r[v][r][k], so that its
// inner loop carries only the transaxial and axial overlaps. The forward epilogue writes r' directly when its
// output feeds the back-projector; a plain sinogram is prescaled by a separate pass.
__host__ __device__ inline float hx_prescale(const HelixDev &G, int v, int r, int k)
{
    return G.scale[(size_t)v * G.nb + k] * G.secphi[(size_t)r * G.nb + k];
}

__host__ __device__ inline float hx_clamp01(float x) { return fminf(fmaxf(x, 0.f), 1.f); }

// Back-projection, one lane: voxels kz0 .. kz0 + HX_ZG - 1 of column (i, j) (voxels >= nz are computed and
// dropped by the caller), views vstart + vi * vstride, vi < nv, reading the prescaled residual block
// Rp [nv][nr][nb]. acc[b] += sum over the views' cells of f_t f_a Rp.
//
// Per view: the candidate bins come from the inverse map at the column's two edges (widened by 0.05 bin);
// their boundary crossings are evaluated once each in FP64 (HX_KC + 1 of them) and the first HX_KC bins'
// transaxial weights kept in registers; a column that meets more bins (a depth close to the source, a coarse
// detector) re-evaluates the rest per row. Along z the thread walks the rows that can meet its voxels;
// row r spans [z_r, z_r+1] in the group's coordinates (voxel b spans [b, b+1]) and meets voxel b by
// clamp01(z_r+1 - b) - clamp01(z_r - b): the clamps at the row's upper face are those at the next row's lower
// face, so each (row, voxel) costs one clamp, one difference and one FMA.
__host__ __device__ inline void hbp_lane(const HelixDev &G, const Ro<float> &Rp, int vstart, int vstride, int nv, int i,
                                         int j, int kz0, float (&acc)[HX_ZG])
{
    for (int vi = 0; vi < nv; ++vi) {
        const int v = vstart + vi * vstride;
        const bool row = G.rowsweep[v] != 0;
        const int NL = row ? G.ny : G.nx, NQ = row ? G.nx : G.ny;
        const int line = row ? i : j, q = row ? j : i;
        const double lcd = (double)line - 0.5 * (double)(NL - 1);
        const float lc = (float)lcd;
        const float2 cs = G.cs[v];
        const float ell = column_depth(G, row, lc, q, cs);
        const float zai = G.zai[v], zaf = G.zaf[v];
        const float zg0 = (float)kz0 - zai;   // the group's voxels span [zg0, zg0 + HX_ZG] in the view's z
        const float hrow = ell * G.dwn;       // row height in voxels at this depth
        const float inva = hx_rcp(hrow);
        // rows that can meet them: z_r = zaf + ell wr_r increases with r
        const float rw0 = G.wr[0] / G.dwn;
        const float rz0 = (zg0 - zaf) * inva - rw0;
        const float rz1 = rz0 + (float)HX_ZG * inva;
        const int ra = (int)floorf(fmaxf(rz0 - 1.f, 0.f));
        const int rb = (int)floorf(fminf(rz1 + 1.f, (float)(G.nr - 1)));
        if (ra > rb) continue;
        // candidate bins of the voxel column in this view
        const float4 im = G.inv[v];
        const double e0d = (double)q - 0.5 * (double)NQ;   // the column spans [e0, e0 + 1] (exact)
        const float e0 = (float)e0d;
        const float nlc = lc * im.y, dlc = fmaf(lc, im.w, G.dso);
        const float t0 = fmaf(e0, im.x, nlc) * hx_rcp(fmaf(e0, im.z, dlc));
        const float t1 = fmaf(e0 + 1.f, im.x, nlc) * hx_rcp(fmaf(e0 + 1.f, im.z, dlc));
        const float kf0 = fmaf(G.c_kf, t0, G.k0), kf1 = fmaf(G.c_kf, t1, G.k0);
        const int ka = (int)floorf(fmaxf(fminf(kf0, kf1) - 0.05f, 0.f));
        const int kb = (int)floorf(fminf(fmaxf(kf0, kf1) + 0.05f, (float)(G.nb - 1)));
        if (ka > kb) continue;
        const size_t vb = (size_t)v * (G.nb + 1);
        // boundary crossings relative to the column's lower edge, in FP64: d_c = U_(ka+c) - e0
        float fk[HX_KC];
        double up;
        {
            const double2 b = G.bnd[vb + ka];
            up = fma(lcd, b.y, b.x) - e0d;
        }
#pragma unroll
        for (int c = 0; c < HX_KC; ++c) {
            const double2 b = G.bnd[vb + hx_min(ka + c + 1, kb + 1)];
            const double un = fma(lcd, b.y, b.x) - e0d;
            const float lo = (float)fmin(up, un), hi = (float)fmax(up, un), wd = (float)fabs(un - up);
            const float ov = fminf(hi, 1.f) - fmaxf(lo, 0.f);
            fk[c] = (ka + c <= kb && ov > 0.f && wd > 0.f) ? ov * hx_rcp(wd) * inva : 0.f;
            up = un;
        }
        const float zoff = zaf - zg0;   // row boundaries in the group's coordinates: fmaf(ell, wr_r, zoff)
        float cl[HX_ZG];
        {
            const float zl = fmaf(ell, G.wr[(size_t)ra], zoff);
#pragma unroll
            for (int b = 0; b < HX_ZG; ++b) cl[b] = hx_clamp01(zl - (float)b);
        }
        // 32-bit element offsets into the residual block (the descriptor check keeps nviews * nr * nb below
        // 2^31): the row's base advances by nb per row, the candidates' bins are fixed for the view
        unsigned kcand[HX_KC];
#pragma unroll
        for (int c = 0; c < HX_KC; ++c) kcand[c] = (unsigned)hx_min(ka + c, kb);
        unsigned rr = ((unsigned)vi * (unsigned)G.nr + (unsigned)ra) * (unsigned)G.nb;
        for (int r = ra; r <= rb; ++r, rr += (unsigned)G.nb) {
            const float zh = fmaf(ell, G.wr[(size_t)r + 1], zoff);
            float t = 0.f;
#pragma unroll
            for (int c = 0; c < HX_KC; ++c) t = fmaf(fk[c], Rp[rr + kcand[c]], t);
            for (int k = ka + HX_KC; k <= kb; ++k) {   // columns that meet more than HX_KC bins
                const double2 b0 = G.bnd[vb + k], b1 = G.bnd[vb + k + 1];
                const double ua = fma(lcd, b0.y, b0.x) - e0d, ub = fma(lcd, b1.y, b1.x) - e0d;
                const float lo = (float)fmin(ua, ub), hi = (float)fmax(ua, ub), wd = (float)fabs(ub - ua);
                const float ov = fminf(hi, 1.f) - fmaxf(lo, 0.f);
                if (ov > 0.f && wd > 0.f) t = fmaf(ov * hx_rcp(wd) * inva, Rp[rr + k], t);
            }
#pragma unroll
            for (int b = 0; b < HX_ZG; ++b) {
                const float ch = hx_clamp01(zh - (float)b);
                acc[b] = fmaf(t, ch - cl[b], acc[b]);
                cl[b] = ch;
            }
        }
    }
}

// Scalars of the 3-D update.
struct HelixUpdate {
    int nx, ny, nz;
    float alpha;
    int potential, huber;
    float delta, beta;
    float idelta;   // 1 / delta, rounded once on the host
};

// The 26-neighbour regularizer at voxel (kz, i, j) of X (canonical [nz][ny][nx]): gradient and Huber
// curvature diagonal (omega = 1 when huber == 0). Offsets of length 1, sqrt 2 and sqrt 3 (voxel units)
// carry beta, beta / sqrt 2 and beta / sqrt 3; a pair exists only when both voxels lie in the volume.
__host__ __device__ inline void reg26(const HelixUpdate &U, const Ro<float> &X, int kz, int i, int j, float xc,
                                      float &gr, float &dr)
{
    gr = 0.f;
    dr = 0.f;
    const float bnd[4] = {0.f, U.beta, U.beta * 0.70710678118654752f, U.beta * 0.57735026918962576f};
    // Every neighbour's value is loaded before the first term (one memory latency, not one per neighbour):
    // a neighbour outside the volume reads the voxel itself and takes weight 0, so that its term
    // (difference 0) leaves both sums unchanged; the terms are added in the same order as the loops.
    const size_t idx = ((size_t)kz * U.ny + i) * U.nx + j;
    float xn[26];
    unsigned in = 0u;
    int q = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int di = -1; di <= 1; ++di)
            for (int dj = -1; dj <= 1; ++dj) {
                if (dz == 0 && di == 0 && dj == 0) continue;
                const int k2 = kz + dz, i2 = i + di, j2 = j + dj;
                const bool ok = k2 >= 0 && k2 < U.nz && i2 >= 0 && i2 < U.ny && j2 >= 0 && j2 < U.nx;
                xn[q] = X[ok ? ((size_t)k2 * U.ny + i2) * U.nx + j2 : idx];
                in |= ok ? 1u << q : 0u;
                ++q;
            }
    q = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int di = -1; di <= 1; ++di)
            for (int dj = -1; dj <= 1; ++dj) {
                if (dz == 0 && di == 0 && dj == 0) continue;
                const int n = dz * dz + di * di + dj * dj;
                const float b = (in >> q) & 1u ? bnd[n] : 0.f;
                const float t = xc - xn[q];
                ++q;
                const float z = t * U.idelta;
                float om;
                if (U.potential == 0) om = hx_rsqrt(fmaf(z, z, 1.f));
                else if (U.potential == 1) om = hx_rcp(1.f + fabsf(z));
                else {
                    const float s = powf(fabsf(z), 0.8f);
                    om = fmaf(1.2f, s, 2.f) / (2.f * (1.f + s) * (1.f + s));
                }
                gr = fmaf(b * om, t, gr);
                dr = fmaf(b, 2.f * (U.huber ? om : 1.f), dr);
            }
}

// Clipped x-step at one voxel: x+ = max(0, (gamma + D_R x - grad R) / (rho D_L + D_R)), gamma = (rho - 1) g + rho h.
__host__ __device__ inline float xstep(float rho, float x, float gv, float h, float dl, float gr, float dr)
{
    const float gamma = fmaf(rho - 1.f, gv, rho * h);
    const float curv = fmaf(rho, dl, dr);
    const float xn = curv > 0.f ? (gamma + fmaf(dr, x, -gr)) * hx_rcp(curv) : x;
    return fmaxf(xn, 0.f);
}

}  // namespace ct
