// Host-side geometry tables for the distance-driven fan-beam projector (FP64 -> FP32 device tables).
//
// The projector is the distance-driven operator (the paper cites, but does not define, its projector):
// for a view whose central ray is within 45 degrees of the y axis ("row sweep"; decided here in FP64
// as |sin b| >= |cos b| - 1e-12) the image lines are rows, otherwise columns. Detector boundary k is the
// ray from the source through the detector point at u_k = (k - nb/2 + u_offset) du; it crosses line l
// at U_k(l), an affine function of the line index. The weight of pixel q of line l in bin k is
//     (line spacing / |cos theta_k|) * |[q, q+1] intersect [U_k(l), U_k+1(l)]| / |U_k+1(l) - U_k(l)|
// (pixel units), theta_k being the angle between the ray through the bin centre and the line normal.
//
// The kernels evaluate U_k(l) = fmaf(lc, B_k, A_k) from the FP32 (A_k, B_k) stored here, in the forward
// and in the back-projector alike, so both see bit-identical boundaries. Along every line of a view the
// boundaries are ordered the same way (the image lies between source and detector, so the boundary rays
// cross each line in their own order); sgn[v] = +1 when U_k increases with k, -1 otherwise, lets the
// back-projector work with increasing boundaries s U_k (a sign flip, exact).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ct_internal.hpp"

namespace ct {

namespace {

struct View64 {
    double c, s;        // central direction d = (c, s)
    double sx, sy;      // source
    bool row;
};

View64 view64(const ct_geom_desc &d, int v)
{
    View64 o;
    double beta = d.beta0 + d.span * (double)v / (double)d.nviews;
    o.c = std::cos(beta);
    o.s = std::sin(beta);
    o.sx = -d.dso * o.c;
    o.sy = -d.dso * o.s;
    o.row = std::fabs(o.s) >= std::fabs(o.c) - 1e-12;
    return o;
}

void det_point64(const ct_geom_desc &d, const View64 &o, double u, double *px, double *py)
{
    // detector axis e = (-s, c)
    if (d.det == CT_DET_FLAT) {
        double off = d.dsd - d.dso;
        *px = off * o.c - u * o.s;
        *py = off * o.s + u * o.c;
    } else {
        double gam = u / d.dsd;
        double cg = std::cos(gam), sg = std::sin(gam);
        *px = o.sx + d.dsd * (cg * o.c - sg * o.s);
        *py = o.sy + d.dsd * (cg * o.s + sg * o.c);
    }
}

}  // namespace

// Whether the back-projector may locate the bins of a lane's run of pixel edges by a quadratic in the
// edge index m = 0 .. 4 instead of one division per edge (flat detector only). Along a line the detector
// coordinate of edge m is t(m) = (n0 + a m) / (d0 + c m) = a/c + K / (1 + eps m), eps = c / d0, so the
// quadratic Taylor polynomial about m = 0 misses it by t'(0) eps^2 m^3 / (1 + eps m). With R the image's
// half diagonal, every depth d0 + c m is at least dso - R, |a|, |c| are at most the pixel size p and
// |t| at most R / (dso - R): |eps| <= p / (dso - R) and |t'| <= (1 + R / (dso - R)) p / (dso - R). The
// kernel's estimate only has to land within one bin of the true one (it then steps to the neighbour);
// the bound is required below a quarter bin.
static int quadratic_bin_estimate_ok(const ct_geom_desc &d)
{
    if (d.det == CT_DET_ARC) return 0;
    const double R = 0.5 * std::hypot(d.nx * d.dx, d.ny * d.dy);
    const double depth = d.dso - R;
    if (!(depth > 0.0)) return 0;
    const double p = std::max(d.dx, d.dy);
    const double eps = p / depth, np = 4.0;
    if (!(np * eps < 0.5)) return 0;
    const double slope = d.dsd / d.du * (1.0 + R / depth) * p / depth;   // bins per edge step, at most
    const double miss = slope * eps * eps * np * np * np / (1.0 - np * eps);
    return miss < 0.25 ? 1 : 0;
}

ct_status geometry_tables(const ct_geom_desc &d, GeomTables &t)
{
    const int nv = d.nviews, nb = d.nb;
    std::vector<float2> &bnd = t.bnd;
    std::vector<float> &scale = t.scale;
    std::vector<float4> &inv = t.inv;
    std::vector<double2> &cs = t.cs;
    std::vector<float> &sgn = t.sgn;
    bnd.assign((size_t)nv * (nb + 1), float2{});
    t.bnd64.assign((size_t)nv * (nb + 1), double2{});
    scale.assign((size_t)nv * nb, 0.f);
    inv.assign(nv, float4{});
    cs.assign(nv, double2{});
    sgn.assign(nv, 0.f);
    t.rowsweep.assign(nv, 0);
    for (int v = 0; v < nv; ++v) {
        View64 o = view64(d, v);
        t.rowsweep[v] = o.row ? 1 : 0;
        cs[v] = make_double2(o.c, o.s);
        for (int k = 0; k <= nb; ++k) {
            double u = ((double)k - 0.5 * nb + d.u_offset) * d.du;
            double px, py;
            det_point64(d, o, u, &px, &py);
            double A, B;
            if (o.row) {
                double slope = (px - o.sx) / (py - o.sy);       // dx/dy along the ray
                A = (o.sx - o.sy * slope) / d.dx;
                B = d.dy * slope / d.dx;
            } else {
                double slope = (py - o.sy) / (px - o.sx);       // dy/dx along the ray
                A = (o.sy - o.sx * slope) / d.dy;
                B = d.dx * slope / d.dy;
            }
            bnd[(size_t)v * (nb + 1) + k] = make_float2((float)A, (float)B);
            t.bnd64[(size_t)v * (nb + 1) + k] = make_double2(A, B);
        }
        // boundary order of the view, and every footprint positive in the kernels' FP32 evaluation at the
        // first and last line (U_k is affine in the line coordinate, so the extremes bound the rest)
        {
            const float2 *b = &bnd[(size_t)v * (nb + 1)];
            const int NL = o.row ? d.ny : d.nx;
            const float s = b[1].x > b[0].x ? 1.f : -1.f;   // order at the central line (lc = 0)
            sgn[v] = s;
            for (int side = 0; side < 2; ++side) {
                const float lc = (side ? 0.5f : -0.5f) * (float)(NL - 1);
                float up = std::fmaf(lc, b[0].y, b[0].x);
                for (int k = 1; k <= nb; ++k) {
                    const float un = std::fmaf(lc, b[k].y, b[k].x);
                    if (!(s * (un - up) > 1e-6f))
                        return fail(CT_ERR_UNSUPPORTED, "detector bins too narrow for the projector's FP32 boundary table");
                    up = un;
                }
            }
        }
        for (int k = 0; k < nb; ++k) {
            double u = ((double)k + 0.5 - 0.5 * nb + d.u_offset) * d.du;
            double cx, cy;
            det_point64(d, o, u, &cx, &cy);
            double rx = cx - o.sx, ry = cy - o.sy, len = std::sqrt(rx * rx + ry * ry);
            scale[(size_t)v * nb + k] = (float)(o.row ? d.dy * len / std::fabs(ry) : d.dx * len / std::fabs(rx));
        }
        // inverse map: point at along-line coordinate e and line coordinate lc (view pixel units)
        double ex = -o.s, ey = o.c;
        if (o.row)  // X = e dx, Y = lc dy
            inv[v] = make_float4((float)(d.dx * ex), (float)(d.dy * ey), (float)(d.dx * o.c), (float)(d.dy * o.s));
        else        // X = lc dx, Y = e dy
            inv[v] = make_float4((float)(d.dy * ey), (float)(d.dx * ex), (float)(d.dy * o.s), (float)(d.dx * o.c));
    }
    t.c_kf = (float)(d.dsd / d.du);
    t.k0 = (float)(0.5 * nb - d.u_offset);
    t.poly = quadratic_bin_estimate_ok(d);
    return CT_OK;
}

ct_status build_geometry(ct_geom *g)
{
    const ct_geom_desc &d = g->desc;
    const int nv = d.nviews, nb = d.nb;
    GeomTables t;
    CT_TRY(geometry_tables(d, t));
    const std::vector<float2> &bnd = t.bnd;
    const std::vector<float> &scale = t.scale;
    const std::vector<float4> &inv = t.inv;
    const std::vector<double2> &cs = t.cs;
    const std::vector<float> &sgn = t.sgn;
    g->rowsweep = t.rowsweep;
    CT_HIP_CHECK(hipMalloc(&g->bnd, bnd.size() * sizeof(float2)));
    CT_HIP_CHECK(hipMalloc(&g->scale, scale.size() * sizeof(float)));
    CT_HIP_CHECK(hipMalloc(&g->inv, inv.size() * sizeof(float4)));
    CT_HIP_CHECK(hipMalloc(&g->d_rowsweep, nv * sizeof(int)));
    CT_HIP_CHECK(hipMalloc(&g->cs, nv * sizeof(double2)));
    CT_HIP_CHECK(hipMalloc(&g->sgn, nv * sizeof(float)));
    CT_HIP_CHECK(hipMemcpy(g->sgn, sgn.data(), nv * sizeof(float), hipMemcpyHostToDevice));
    CT_HIP_CHECK(hipMemcpy(g->cs, cs.data(), nv * sizeof(double2), hipMemcpyHostToDevice));
    CT_HIP_CHECK(hipMemcpy(g->bnd, bnd.data(), bnd.size() * sizeof(float2), hipMemcpyHostToDevice));
    CT_HIP_CHECK(hipMemcpy(g->scale, scale.data(), scale.size() * sizeof(float), hipMemcpyHostToDevice));
    CT_HIP_CHECK(hipMemcpy(g->inv, inv.data(), inv.size() * sizeof(float4), hipMemcpyHostToDevice));
    CT_HIP_CHECK(hipMemcpy(g->d_rowsweep, g->rowsweep.data(), nv * sizeof(int), hipMemcpyHostToDevice));
    GeomDev &G = g->dev;
    G.nx = d.nx;
    G.ny = d.ny;
    G.nb = nb;
    G.nviews = nv;
    G.arc = d.det == CT_DET_ARC;
    G.poly = t.poly;
    G.dso = (float)d.dso;
    G.c_kf = t.c_kf;
    G.k0 = t.k0;
    G.bnd = g->bnd;
    G.scale = g->scale;
    G.inv = g->inv;
    G.rowsweep = g->d_rowsweep;
    G.sgn = g->sgn;
    G.win = nullptr;   // filled by the caller once the kernels are at hand (ct_geom_create)
    return CT_OK;
}

void free_geometry(ct_geom *g)
{
    if (g->bnd) (void)hipFree(g->bnd);
    if (g->scale) (void)hipFree(g->scale);
    if (g->inv) (void)hipFree(g->inv);
    if (g->d_rowsweep) (void)hipFree(g->d_rowsweep);
    if (g->cs) (void)hipFree(g->cs);
    if (g->sgn) (void)hipFree(g->sgn);
    if (g->win) (void)hipFree(g->win);
    g->win = nullptr;
    g->dev.win = nullptr;
    g->cs = nullptr;
    g->sgn = nullptr;
    g->bnd = nullptr;
    g->scale = nullptr;
    g->inv = nullptr;
    g->d_rowsweep = nullptr;
}

std::vector<int> subset_order(int M, int kind)
{
    std::vector<int> o;
    if (kind == CT_ORDER_BITREV) {
        int P = 1, bits = 0;
        while (P < M) { P <<= 1; ++bits; }
        for (int i = 0; i < P; ++i) {
            int r = 0;
            for (int b = 0; b < bits; ++b)
                if (i & (1 << b)) r |= 1 << (bits - 1 - b);
            if (r < M) o.push_back(r);
        }
    } else {
        for (int m = 0; m < M; ++m) o.push_back(m);
    }
    return o;
}

}  // namespace ct
