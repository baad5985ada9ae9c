// Host-side tables of the 3-D helical projector (FP64 geometry, stored FP32).
//
// Transaxially every view is a fan-beam view: the fan-beam tables of ct_geom.cpp serve the helical scan
// as a multi-turn fan (span 2 pi nviews / views_per_turn). Axially: za_v = (S_z(v) - z_lo) / dz, the source
// height in voxel units from the volume's lower face (stored as integer part and fraction); wr_r = w_r / (dsd dz), so that row boundary r passes
// a column of depth ell at height za_v + ell wr_r; sec phi at each cell centre.
#include <cmath>

#include "ct_helix_internal.hpp"

namespace ct {

ct_geom_desc helix_fan_desc(const ct_helix_desc &d)
{
    ct_geom_desc f{};
    f.nx = d.nx;
    f.ny = d.ny;
    f.dx = d.dx;
    f.dy = d.dy;
    f.nb = d.nb;
    f.du = d.du;
    f.u_offset = d.u_offset;
    f.det = CT_DET_FLAT;
    f.nviews = d.nviews;
    f.beta0 = d.beta0;
    f.span = 2.0 * M_PI * (double)d.nviews / (double)d.views_per_turn;
    f.dso = d.dso;
    f.dsd = d.dsd;
    f.nsubsets = d.nsubsets;
    f.storage = CT_F32;
    return f;
}

ct_status check_helix_desc(const ct_helix_desc *d)
{
    if (!d) return fail(CT_ERR_INVALID_ARG, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nx > 4096 || d->ny > 4096 || d->nz < 1 || d->nz > 2048)
        return fail(CT_ERR_INVALID_ARG, "nx, ny must be in [1, 4096] and nz in [1, 2048]");
    if (!(d->dx > 0) || !(d->dy > 0) || !(d->dz > 0) || !(d->du > 0) || !(d->dw > 0))
        return fail(CT_ERR_INVALID_ARG, "dx, dy, dz, du, dw must be > 0");
    if (d->nb < 1 || d->nb > 8192 || d->nr < 1 || d->nr > 1024)
        return fail(CT_ERR_INVALID_ARG, "nb must be in [1, 8192] and nr in [1, 1024]");
    if (d->nviews < 1 || d->views_per_turn < 1 || d->nviews > (1 << 20))
        return fail(CT_ERR_INVALID_ARG, "nviews and views_per_turn must be >= 1 (nviews <= 2^20)");
    // the back-projector indexes a residual block (up to all views) in 32 bits
    if ((long long)d->nviews * (d->nb + 1) >= (1ll << 31) || (long long)d->nviews * d->nr * d->nb >= (1ll << 31))
        return fail(CT_ERR_INVALID_ARG, "sinogram too large: nviews * nr * nb must be below 2^31");
    // the forward projector indexes the padded cumulative volume ((nz + 2) planes) in 32 bits, a plane by a
    // 24-bit multiply
    if ((long long)d->nx * d->ny >= (1ll << 24) || (long long)(d->nz + 2) * d->nx * d->ny >= (1ll << 31))
        return fail(CT_ERR_INVALID_ARG, "volume too large: nx * ny must be below 2^24 and (nz + 2) * nx * ny below 2^31");
    if (d->nsubsets < 1 || d->nviews % d->nsubsets != 0)
        return fail(CT_ERR_INVALID_ARG, "nsubsets must be >= 1 and divide nviews");
    if (!(d->dso > 0) || !(d->dsd > d->dso)) return fail(CT_ERR_INVALID_ARG, "need dsd > dso > 0");
    const double hx = 0.5 * d->nx * d->dx, hy = 0.5 * d->ny * d->dy;
    if (std::sqrt(hx * hx + hy * hy) >= 0.95 * d->dso)
        return fail(CT_ERR_INVALID_ARG, "the volume must lie well inside the source circle");
    if (!std::isfinite(d->beta0) || !std::isfinite(d->z0) || !std::isfinite(d->feed) || !std::isfinite(d->zc) ||
        !std::isfinite(d->u_offset) || !std::isfinite(d->w_offset))
        return fail(CT_ERR_INVALID_ARG, "non-finite angle, height or offset");
    const double half = (0.5 * d->nb + std::fabs(d->u_offset)) * d->du;
    if (std::atan(half / d->dsd) > 35.0 * M_PI / 180.0) return fail(CT_ERR_INVALID_ARG, "fan half-angle must be <= 35 degrees");
    const double halfw = (0.5 * d->nr + std::fabs(d->w_offset)) * d->dw;
    if (std::atan(halfw / d->dsd) > 30.0 * M_PI / 180.0) return fail(CT_ERR_INVALID_ARG, "cone half-angle must be <= 30 degrees");
    return CT_OK;
}

ct_status helix_tables(const ct_helix_desc &d, HelixTables &t)
{
    CT_TRY(check_helix_desc(&d));
    CT_TRY(geometry_tables(helix_fan_desc(d), t.fan));
    const int nv = d.nviews;
    t.cs.resize(nv);
    t.zai.resize(nv);
    t.zaf.resize(nv);
    const double zlo = d.zc - 0.5 * d.nz * d.dz;
    for (int v = 0; v < nv; ++v) {
        const double beta = d.beta0 + 2.0 * M_PI * (double)v / (double)d.views_per_turn;
        t.cs[v] = make_float2((float)std::cos(beta), (float)std::sin(beta));
        const double sz = d.z0 + d.feed * (double)v / (double)d.views_per_turn;
        const double za = (sz - zlo) / d.dz, zi = std::floor(za);
        t.zai[v] = (float)zi;
        t.zaf[v] = (float)(za - zi);
    }
    t.wr.resize(d.nr + 1);
    for (int r = 0; r <= d.nr; ++r) t.wr[r] = (float)(((double)r - 0.5 * d.nr + d.w_offset) * d.dw / (d.dsd * d.dz));
    t.dwn = (float)(d.dw / (d.dsd * d.dz));
    t.secphi.resize((size_t)d.nr * d.nb);
    for (int r = 0; r < d.nr; ++r) {
        const double wc = ((double)r + 0.5 - 0.5 * d.nr + d.w_offset) * d.dw;
        for (int k = 0; k < d.nb; ++k) {
            const double uc = ((double)k + 0.5 - 0.5 * d.nb + d.u_offset) * d.du;
            t.secphi[(size_t)r * d.nb + k] = (float)std::sqrt(1.0 + wc * wc / (d.dsd * d.dsd + uc * uc));
        }
    }
    return CT_OK;
}

}  // namespace ct
