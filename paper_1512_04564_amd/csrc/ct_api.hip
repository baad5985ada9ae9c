// C ABI of libctrlalm (include/ct.h): argument checking, workspace, and the relaxed OS-LALM driver.
//
// One subiteration is two kernels: the forward projection of subset m(t) with the fused residual
// epilogue, then the fused back-projection / relaxed-update kernel (dual update of subiteration t and
// x-step of subiteration t+1). An outer iteration (M subiterations) is captured once as a hipGraph and
// replayed; the subiteration index is read from a device counter that a one-thread kernel at the end of
// the graph advances, so one captured graph serves every iteration.
#include <sys/stat.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "ct_internal.hpp"

namespace ct {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

ct_status fail(ct_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

namespace {

template <typename T>
ct_status dev_alloc(T **p, size_t n)
{
    if (*p) return CT_OK;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T) > 0 ? n * sizeof(T) : sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? CT_ERR_OOM : CT_ERR_HIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return CT_OK;
}

template <typename T>
void dev_free(T **p)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
}

ct_status check_desc(const ct_geom_desc *d)
{
    if (!d) return fail(CT_ERR_INVALID_ARG, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nx > 4096 || d->ny > 4096) return fail(CT_ERR_INVALID_ARG, "nx, ny must be in [1, 4096]");
    if (!(d->dx > 0) || !(d->dy > 0) || !(d->du > 0)) return fail(CT_ERR_INVALID_ARG, "dx, dy, du must be > 0");
    if (d->nb < 1 || d->nb > 8192) return fail(CT_ERR_INVALID_ARG, "nb must be in [1, 8192]");
    if (d->nviews < 1 || d->nviews > (1 << 20)) return fail(CT_ERR_INVALID_ARG, "nviews must be in [1, 2^20]");
    if ((long long)d->nviews * (d->nb + 1) >= (1ll << 31))
        return fail(CT_ERR_INVALID_ARG, "nviews * (nb + 1) must stay below 2^31");
    if (d->nsubsets < 1 || d->nviews % d->nsubsets != 0)
        return fail(CT_ERR_INVALID_ARG, "nsubsets must be >= 1 and divide nviews");
    if (!(d->dso > 0) || !(d->dsd > d->dso)) return fail(CT_ERR_INVALID_ARG, "need dsd > dso > 0");
    if (d->det != CT_DET_FLAT && d->det != CT_DET_ARC) return fail(CT_ERR_INVALID_ARG, "det must be flat or arc");
    if (d->storage != CT_F32 && d->storage != CT_F16 && d->storage != CT_BF16)
        return fail(CT_ERR_INVALID_ARG, "storage must be CT_F32, CT_F16 or CT_BF16");
    double hx = 0.5 * d->nx * d->dx, hy = 0.5 * d->ny * d->dy;
    if (std::sqrt(hx * hx + hy * hy) >= 0.95 * d->dso)
        return fail(CT_ERR_INVALID_ARG, "the image must lie well inside the source circle");
    if (!std::isfinite(d->beta0) || !std::isfinite(d->span) || !std::isfinite(d->u_offset))
        return fail(CT_ERR_INVALID_ARG, "non-finite angle or offset");
    // Half the detector's fan must stay below 80 degrees so that boundary rays never run parallel to a line.
    double half = (0.5 * d->nb + std::fabs(d->u_offset)) * d->du;
    double gam = d->det == CT_DET_FLAT ? std::atan(half / d->dsd) : half / d->dsd;
    if (gam > 35.0 * M_PI / 180.0) return fail(CT_ERR_INVALID_ARG, "fan half-angle must be <= 35 degrees");
    return CT_OK;
}

}  // namespace

ct_status check_params(const ct_rlalm_params *p)
{
    if (!p) return fail(CT_ERR_INVALID_ARG, "params is NULL");
    if (!(p->alpha >= 1.0 && p->alpha < 2.0)) return fail(CT_ERR_INVALID_ARG, "alpha must be in [1, 2)");
    if (p->niters < 0) return fail(CT_ERR_INVALID_ARG, "niters must be >= 0");
    if (p->rho_mode != 0 && p->rho_mode != 1) return fail(CT_ERR_INVALID_ARG, "rho_mode must be 0 or 1");
    if (p->rho_mode == 1 && !(p->rho_fixed > 0)) return fail(CT_ERR_INVALID_ARG, "rho_fixed must be > 0");
    if (p->potential < 0 || p->potential > 2) return fail(CT_ERR_INVALID_ARG, "potential must be 0, 1 or 2");
    if (!(p->delta > 0) || !(p->beta >= 0)) return fail(CT_ERR_INVALID_ARG, "need delta > 0, beta >= 0");
    if (p->algorithm != 1 && p->algorithm != 2) return fail(CT_ERR_INVALID_ARG, "algorithm must be 1 or 2");
    if (p->subset_order != CT_ORDER_SEQUENTIAL && p->subset_order != CT_ORDER_BITREV)
        return fail(CT_ERR_INVALID_ARG, "unknown subset order");
    if (!(p->dl_scale > 0)) return fail(CT_ERR_INVALID_ARG, "dl_scale must be > 0");
    if (p->start < 0 || p->start > 3) return fail(CT_ERR_INVALID_ARG, "start must be 0, 1, 2 or 3");
    if (p->start == 3 && !p->unet) return fail(CT_ERR_INVALID_ARG, "start == 3 needs a network (unet)");
    if (p->forward_split < -1 || p->forward_split > 1) return fail(CT_ERR_INVALID_ARG, "forward_split must be -1, 0 or 1");
    if (p->diverge_window < 0) return fail(CT_ERR_INVALID_ARG, "diverge_window must be >= 0");
    if (p->diverge_window > 0 && !(p->diverge_factor > 1.0))
        return fail(CT_ERR_INVALID_ARG, "diverge_factor must be > 1 when diverge_window > 0");
    return CT_OK;
}

double rho_value(long long k, const ct_rlalm_params *p)
{
    if (p->rho_mode == 1) return p->rho_fixed;
    if (k == 0) return 1.0;
    double a = M_PI / (p->alpha * (double)(k + 1));
    double b = M_PI / (2.0 * p->alpha * (double)(k + 1));
    return a * std::sqrt(1.0 - b * b);
}

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

ct_status ensure_workspace(ct_geom *g, size_t r_views, size_t rho_len)
{
    Workspace &W = g->ws;
    const ct_geom_desc &d = g->desc;
    const size_t npix = (size_t)d.nx * d.ny;
    W.npix = npix;
    CT_TRY(dev_alloc(&W.xa, npix));
    CT_TRY(dev_alloc(&W.xb, npix));
    CT_TRY(dev_alloc(&W.xta, npix));
    CT_TRY(dev_alloc(&W.xtb, npix));
    if (d.storage != CT_F32) {
        CT_TRY(dev_alloc(reinterpret_cast<uint16_t **>(&W.xca), npix));
        CT_TRY(dev_alloc(reinterpret_cast<uint16_t **>(&W.xcb), npix));
    }
    CT_TRY(dev_alloc(&W.tmp, npix));
    CT_TRY(dev_alloc(&W.tbase, 4));
    CT_TRY(dev_alloc(&W.red, kRedSize));
    const size_t need_r = r_views * (size_t)d.nb;
    if (need_r > W.r_cap) {
        dev_free(&W.r);
        CT_TRY(dev_alloc(&W.r, need_r));
        W.r_cap = need_r;
    }
    if (rho_len > W.rho_cap) {
        dev_free(&W.rho);
        CT_TRY(dev_alloc(&W.rho, rho_len));
        W.rho_cap = rho_len;
    }
    return CT_OK;
}

void free_workspace(ct_geom *g)
{
    Workspace &W = g->ws;
    dev_free(&W.xa);
    dev_free(&W.xb);
    dev_free(&W.xta);
    dev_free(&W.xtb);
    dev_free(&W.xca);
    dev_free(&W.xcb);
    dev_free(&W.tmp);
    dev_free(&W.r);
    dev_free(&W.rho);
    dev_free(&W.tbase);
    dev_free(&W.red);
    dev_free(&W.dl);
    dev_free(&W.kappa);
    dev_free(&W.gv);
    dev_free(&W.h);
    W.r_cap = W.rho_cap = 0;
}

}  // namespace ct

using namespace ct;

// ------------------------------------------------------------------------------------------------
// Graph cache: one executable graph per (ping-pong parity) for a given set of pointers and params.
// ------------------------------------------------------------------------------------------------
namespace {

bool params_equal(const ct_rlalm_params &a, const ct_rlalm_params &b)
{
    return a.alpha == b.alpha && a.rho_mode == b.rho_mode && a.rho_fixed == b.rho_fixed &&
           a.potential == b.potential && a.delta == b.delta && a.beta == b.beta && a.huber == b.huber &&
           a.algorithm == b.algorithm && a.subset_order == b.subset_order && a.kappa == b.kappa &&
           a.forward_split == b.forward_split;
}

bool key_equal(const GraphKey &a, const GraphKey &b)
{
    return a.y == b.y && a.w == b.w && a.dl == b.dl && a.kappa == b.kappa && a.gv == b.gv && a.h == b.h &&
           a.rho == b.rho && a.r == b.r && a.t0mod == b.t0mod && a.parity == b.parity && a.len == b.len &&
           params_equal(a.p, b.p);
}

void drop_graph_cache(ct_geom *g)
{
    GraphCache &c = g->graphs;
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 2; ++i)
            if (c.exec[k][i]) (void)hipGraphExecDestroy(c.exec[k][i]);
    if (c.cap) (void)hipStreamDestroy(c.cap);
    c = GraphCache();
}

struct Ctx {
    ct_geom *g;
    const ct_rlalm_params *p;
    const void *y, *w;   // storage type
    const float *dl, *kappa;
    float *gv, *h;
    std::vector<int> order;
    int M, nvm, dtype;
};

// The forward projector's input copies of ping-pong buffer A (a != 0) or B: float32 storage reads the
// image itself, 16-bit storage its rounded copy; the transposed copy is always in the storage type.
const void *proj_img(const Workspace &W, int dtype, int a) { return dtype == CT_F32 ? (a ? W.xa : W.xb) : (a ? W.xca : W.xcb); }
void *proj_imgT(const Workspace &W, int a) { return a ? W.xta : W.xtb; }
void *proj_copy(const Workspace &W, int dtype, int a) { return dtype == CT_F32 ? nullptr : (a ? W.xca : W.xcb); }

FpLaunch fp_launch(const GeomDev &G, const void *img, const void *imgT, int vstart, int vstride, int nv, const void *y,
                   const void *w, float mscale, void *out)
{
    FpLaunch a;
    a.G = G;
    a.img = img;
    a.imgT = imgT;
    a.y = y;
    a.w = w;
    a.out = out;
    a.vstart = vstart;
    a.vstride = vstride;
    a.nv = nv;
    a.mscale = mscale;
    return a;
}

BpLaunch bp_launch(const GeomDev &G, const void *r, int vstart, int vstride, int nv, float *out_back,
                   const UpdateArgs &U)
{
    BpLaunch a;
    a.G = G;
    a.r = r;
    a.vstart = vstart;
    a.vstride = vstride;
    a.nv = nv;
    a.out_back = out_back;
    a.U = U;
    return a;
}

// The second residual plane of a subset projection of nv views when it is split, right after the first in
// the residual block; nullptr otherwise. A single slice's launch decides for itself (forward_split); a
// batched launch passes its own decision (batch_split).
float *split_plane(const Ctx &c, int nv, int batch_split = -1)
{
    const ct_geom_desc &d = c.g->desc;
    const int mode = c.p->forward_split;
    bool split = false;
    if (mode == 1) split = split_eligible(c.g->dev, nv, d.nviews, c.dtype);
    else if (mode == -1)
        split = batch_split >= 0 ? batch_split && split_eligible(c.g->dev, nv, d.nviews, c.dtype)
                                 : forward_split(c.g->dev, nv, d.nviews, c.dtype);
    return split ? c.g->ws.r + (size_t)nv * d.nb : nullptr;
}

UpdateArgs make_update(const Ctx &c)
{
    UpdateArgs U;
    U.gv = c.gv;
    U.h = c.h;
    U.dl = c.dl;
    U.kappa = c.kappa;
    U.rho = c.g->ws.rho;
    U.tbase = c.g->ws.tbase;
    U.alpha = (float)c.p->alpha;
    U.algorithm = c.p->algorithm;
    U.potential = c.p->potential;
    U.delta = (float)c.p->delta;
    U.idelta = 1.f / U.delta;   // the correctly rounded float32 quotient, as a device division would give
    U.beta_ax = (float)c.p->beta;
    U.beta_dg = (float)(c.p->beta / std::sqrt(2.0));
    U.huber = c.p->huber;
    return U;
}

// One subiteration t (relative offset tofs from the device counter): FP of subset m(t) on cur, then the
// fused BP + dual(t) + x-step(t+1) writing nxt.
hipError_t launch_subiter_part(const Ctx &c, long long t_abs, long long tofs, int cur_is_a, int part, hipStream_t s)
{
    Workspace &W = c.g->ws;
    const GeomDev &G = c.g->dev;
    const int m = c.order[(size_t)(t_abs % c.M)];
    float *r2 = split_plane(c, c.nvm);
    if (part == 0) {
        FpLaunch a = fp_launch(G, proj_img(W, c.dtype, cur_is_a), proj_imgT(W, cur_is_a), m, c.M, c.nvm, c.y, c.w,
                               (float)c.M, W.r);
        a.out2 = r2;
        return launch_forward(a, 0, FP_RESIDUAL, c.dtype, s);
    }
    UpdateArgs U = make_update(c);
    U.x = cur_is_a ? W.xa : W.xb;
    U.x_next = cur_is_a ? W.xb : W.xa;
    U.xc_next = proj_copy(W, c.dtype, !cur_is_a);
    U.xT_next = proj_imgT(W, !cur_is_a);
    U.tofs = tofs;
    BpLaunch b = bp_launch(G, W.r, m, c.M, c.nvm, nullptr, U);
    b.r2 = r2;
    return launch_back_update(b, BP_FULL, r2 ? CT_F32 : c.dtype, c.dtype, s);
}

hipError_t launch_subiter(const Ctx &c, long long t_abs, long long tofs, int cur_is_a, hipStream_t s)
{
    hipError_t e = launch_subiter_part(c, t_abs, tofs, cur_is_a, 0, s);
    if (e != hipSuccess) return e;
    return launch_subiter_part(c, t_abs, tofs, cur_is_a, 1, s);
}

// The rho table of rho_k (k < len) in FP64, stored as float32 on the device. Uploaded from a pinned staging
// buffer without waiting for the device; skipped when the device already holds this table.
ct_status upload_rho(ct_geom *g, const ct_rlalm_params *p, long long len, hipStream_t s)
{
    std::vector<float> tab((size_t)len);
    for (long long k = 0; k < len; ++k) tab[(size_t)k] = (float)rho_value(k, p);
    const float *old_ptr = g->ws.rho;
    CT_TRY(ensure_workspace(g, g->desc.nviews, (size_t)len));
    if (g->ws.rho != old_ptr) g->rho_on_device.clear();
    if (g->rho_on_device.size() >= tab.size() && std::equal(tab.begin(), tab.end(), g->rho_on_device.begin()))
        return CT_OK;
    if (!g->rho_ev) CT_HIP_CHECK(hipEventCreateWithFlags(&g->rho_ev, hipEventDisableTiming));
    else CT_HIP_CHECK(hipEventSynchronize(g->rho_ev));   // the staging buffer's last upload has been done
    if (tab.size() > g->rho_host_cap) {
        if (g->rho_host) (void)hipHostFree(g->rho_host);
        g->rho_host = nullptr;
        g->rho_host_cap = 0;
        CT_HIP_CHECK(hipHostMalloc((void **)&g->rho_host, tab.size() * sizeof(float), hipHostMallocDefault));
        g->rho_host_cap = tab.size();
    }
    std::copy(tab.begin(), tab.end(), g->rho_host);
    g->rho_on_device.clear();
    CT_HIP_CHECK(hipMemcpyAsync(g->ws.rho, g->rho_host, tab.size() * sizeof(float), hipMemcpyHostToDevice, s));
    CT_HIP_CHECK(hipEventRecord(g->rho_ev, s));
    g->rho_on_device = std::move(tab);
    return CT_OK;
}

// Cost Psi(x) of the float32 image x (eq. ct_problem) into the cost region of the reduction buffer
// (W.red + kRedCost: kCostOut doubles + scratch): all-view projection into the residual buffer (through the
// transposed copy in tmp), then the FP64 reductions. The workspace is allocated here first, so callers read
// the result's address only after this returns.
ct_status do_cost(ct_geom *g, const ct_rlalm_params *p, const void *y, const void *w, const float *x,
                  const float *kappa, hipStream_t s)
{
    CT_TRY(ensure_workspace(g, g->desc.nviews, 4));
    Workspace &W = g->ws;
    if (!W.red || !W.r || !W.tmp) return fail(CT_ERR_HIP, "cost: workspace missing");
    double *out = W.red + kRedCost;
    const ct_geom_desc &d = g->desc;
    CT_HIP_CHECK(launch_transpose(x, W.tmp, d.nx, d.ny, s));
    CT_HIP_CHECK(launch_forward(fp_launch(g->dev, x, W.tmp, 0, 1, d.nviews, nullptr, nullptr, 1.f, W.r), 0, FP_PLAIN,
                                CT_F32, s));
    CT_HIP_CHECK(launch_cost_reduce(W.r, y, w, d.storage, (size_t)d.nviews * d.nb, x, kappa, d.nx, d.ny, p->potential,
                                    p->delta, p->beta, out, s));
    return CT_OK;
}

// Advance (x in buffer A on entry) from state t0 by nsub subiterations. On exit the buffer holding
// x^(t0+nsub) is returned through final_is_a.
ct_status run_subiters(const Ctx &c, long long t0, long long nsub, int use_graph, hipStream_t s, int *final_is_a,
                       ct_trace_row *trace, const ct_rlalm_params *p, std::chrono::steady_clock::time_point tstart,
                       float *x_out = nullptr)
{
    ct_geom *g = c.g;
    Workspace &W = g->ws;
    const GeomDev &G = g->dev;
    // x-step of subiteration t0 from the state (x^t0 in A): writes x^(t0+1) into B
    {
        CT_HIP_CHECK(launch_set_counter(W.tbase, 0, s));
        UpdateArgs U = make_update(c);
        U.x = W.xa;
        U.x_next = W.xb;
        U.xc_next = proj_copy(W, c.dtype, 0);
        U.xT_next = W.xtb;
        U.tofs = t0;
        CT_HIP_CHECK(launch_back_update(bp_launch(G, nullptr, 0, 1, 0, nullptr, U), BP_XSTEP, c.dtype, c.dtype, s));
    }
    int cur_a = 0;  // x^(t0+1) is in B
    long long t = t0;
    const long long tend = t0 + nsub;
    const int M = c.M;
    // graph length: one iteration, doubled when M is odd so that the ping-pong parity is preserved
    const int L = (M % 2 == 0) ? M : 2 * M;
    const bool traced = trace != nullptr;
    double cost_min = INFINITY;
    int grown = 0;
    auto trace_point = [&](long long t_done) -> ct_status {
        // called when t_done subiterations are complete and t_done % M == 0
        if (!traced || t_done % M != 0 || t_done == 0) return CT_OK;
        long long it = t_done / M;
        if (it < 1 || it > p->niters) return CT_OK;
        // x^(t_done) is the input of the last projection: the "cur" buffer before the last swap
        const float *xcur = cur_a ? W.xb : W.xa;  // after the swap below, the previous cur is the other one
        const ct_geom_desc &d = g->desc;
        double *tr = W.red + kRedTrace, *co = W.red + kRedCost;
        CT_HIP_CHECK(launch_trace_reduce(xcur, p->x_ref, c.gv, c.h, d.nx, d.ny, (float)d.dx, (float)d.dy,
                                         (float)p->fov_radius, tr, s));
        // the residual block and tmp are free between iterations: the next projection rewrites them
        CT_TRY(do_cost(g, p, c.y, c.w, xcur, c.kappa, s));
        double host[kTraceOut + kCostOut];
        CT_HIP_CHECK(hipMemcpyAsync(host, tr, kTraceOut * sizeof(double), hipMemcpyDeviceToHost, s));
        CT_HIP_CHECK(hipMemcpyAsync(host + kTraceOut, co, kCostOut * sizeof(double), hipMemcpyDeviceToHost, s));
        CT_HIP_CHECK(hipStreamSynchronize(s));
        ct_trace_row &row = trace[it - 1];
        row.iter = (int)it;
        row.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tstart).count();
        const double hu = 1000.0 / p->mu_water;
        row.rmsd_hu = (p->x_ref && host[1] > 0) ? hu * std::sqrt(host[0] / host[1]) : NAN;
        row.rmsd_hu_all = p->x_ref ? hu * std::sqrt(host[3] / (double)W.npix) : NAN;
        row.rho = rho_value(t_done - 1, p);
        row.finite = host[2] == 0.0 && std::isfinite(host[kTraceOut + 2]);
        row.cost = host[kTraceOut + 2];
        if (!row.finite)
            return fail(CT_ERR_DIVERGED, "non-finite values after iteration " + std::to_string(it) +
                                             "; x holds the last finite traced iterate");
        // x holds the latest finite traced iterate
        CT_HIP_CHECK(hipMemcpyAsync(x_out, xcur, W.npix * sizeof(float), hipMemcpyDeviceToDevice, s));
        cost_min = std::min(cost_min, row.cost);
        grown = row.cost > p->diverge_factor * cost_min ? grown + 1 : 0;
        if (p->diverge_window > 0 && grown >= p->diverge_window) {
            CT_HIP_CHECK(hipStreamSynchronize(s));
            return fail(CT_ERR_DIVERGED, "cost grew above " + std::to_string(p->diverge_factor) +
                                             " times its lowest traced value for " + std::to_string(grown) +
                                             " iterations in a row (iteration " + std::to_string(it) + ")");
        }
        return CT_OK;
    };
    auto plain_one = [&]() -> ct_status {
        CT_HIP_CHECK(launch_set_counter(W.tbase, 0, s));
        CT_HIP_CHECK(launch_subiter(c, t, t, cur_a, s));
        cur_a ^= 1;
        ++t;
        return trace_point(t);
    };
    if (use_graph && nsub >= L) {
        // plain launches until t is at an iteration boundary relative to t0 (keeps traces aligned)
        while (t < tend && (t % M) != 0) CT_TRY(plain_one());
        GraphCache &gc = g->graphs;
        if (!gc.cap) CT_HIP_CHECK(hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking));
        const int chunk = traced ? M : L;  // traced runs replay per iteration, still needing parity graphs
        // untraced runs replay runs of about 400 subiterations as one graph while enough remain (fewer
        // replays, each with its counter reset), then single chunks
        const int nlong = traced ? 1 : std::max(1, 400 / chunk);
        while (tend - t >= chunk) {
            const int kind = nlong > 1 && tend - t >= (long long)chunk * nlong ? 1 : 0;
            const int len = kind ? chunk * nlong : chunk;
            const int parity = cur_a;
            GraphKey key{c.y, c.w, c.dl, c.kappa, c.gv, c.h, W.rho, W.r, (int)(t % M), parity, len, *p};
            if (!gc.valid[kind][parity] || !key_equal(gc.key[kind][parity], key)) {
                if (gc.exec[kind][parity]) (void)hipGraphExecDestroy(gc.exec[kind][parity]);
                gc.exec[kind][parity] = nullptr;
                gc.valid[kind][parity] = false;
                hipGraph_t graph;
                CT_HIP_CHECK(hipStreamBeginCapture(gc.cap, hipStreamCaptureModeThreadLocal));
                int ca = parity;
                hipError_t e = hipSuccess;
                for (int j = 0; j < len && e == hipSuccess; ++j) {
                    e = launch_subiter(c, t + j, j, ca, gc.cap);
                    ca ^= 1;
                }
                if (e == hipSuccess) e = launch_add_counter(W.tbase, len, gc.cap);
                hipError_t e2 = hipStreamEndCapture(gc.cap, &graph);
                if (e != hipSuccess) return fail(CT_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
                if (e2 != hipSuccess) return fail(CT_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
                hipError_t e3 = hipGraphInstantiate(&gc.exec[kind][parity], graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e3 != hipSuccess) return fail(CT_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
                gc.key[kind][parity] = key;
                gc.valid[kind][parity] = true;
            }
            CT_HIP_CHECK(launch_set_counter(W.tbase, (int)t, s));
            CT_HIP_CHECK(hipGraphLaunch(gc.exec[kind][parity], s));
            if (len % 2) cur_a ^= 1;
            t += len;
            CT_TRY(trace_point(t));
        }
    }
    while (t < tend) CT_TRY(plain_one());
    // x^(tend) is the input of the last projection
    *final_is_a = nsub > 0 ? (cur_a ^ 1) : 1;  // with nsub == 0 nothing ran; caller keeps its x
    if (nsub == 0) *final_is_a = -1;
    return CT_OK;
}

// Kernel timing: replay the two kernels of subiteration t (input image in A when cur_is_a) kTimingReps
// times each, back to back between one hipEvent pair per kernel, on the solve's stream. Runs after the
// solve's result has been copied out; it only rewrites solve-owned workspace (g, h, the spare image).
constexpr int kTimingReps = 50;

ct_status time_last_subiteration(const Ctx &c, long long t, int cur_is_a, hipStream_t s)
{
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    ct_status st = CT_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) st = fail(CT_ERR_HIP, "hipEventCreate failed");
    if (st == CT_OK) {
        hipError_t e = launch_set_counter(c.g->ws.tbase, 0, s);
        if (e == hipSuccess) e = hipEventRecord(ev[0], s);
        for (int r = 0; r < kTimingReps && e == hipSuccess; ++r) e = launch_subiter_part(c, t, t, cur_is_a, 0, s);
        if (e == hipSuccess) e = hipEventRecord(ev[1], s);
        for (int r = 0; r < kTimingReps && e == hipSuccess; ++r) e = launch_subiter_part(c, t, t, cur_is_a, 1, s);
        if (e == hipSuccess) e = hipEventRecord(ev[2], s);
        if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
        float f = 0.f, u = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, ev[0], ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&u, ev[1], ev[2]);
        if (e != hipSuccess) st = fail(CT_ERR_HIP, std::string("kernel timing: ") + hipGetErrorString(e));
        else {
            c.g->ktimes.n_forward = kTimingReps;
            c.g->ktimes.n_update = kTimingReps;
            c.g->ktimes.ms_forward = f;
            c.g->ktimes.ms_update = u;
            c.g->ktimes_valid = true;
        }
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return st;
}

Ctx make_ctx(ct_geom *g, const ct_rlalm_params *p, const void *y, const void *w, const float *dl, const float *kappa,
             float *gv, float *h)
{
    Ctx c;
    c.g = g;
    c.p = p;
    c.y = y;
    c.w = w;
    c.dtype = g->desc.storage;
    c.dl = dl;
    c.kappa = (p->kappa && kappa) ? kappa : nullptr;
    c.gv = gv;
    c.h = h;
    c.M = g->desc.nsubsets;
    c.nvm = g->desc.nviews / c.M;
    c.order = subset_order(c.M, p->subset_order);
    return c;
}

ct_status do_prepare(ct_geom *g, const ct_rlalm_params *p, const void *w, float *dl, float *kappa, hipStream_t s)
{
    CT_TRY(ensure_workspace(g, g->desc.nviews, 4));
    Workspace &W = g->ws;
    const GeomDev &G = g->dev;
    const int nv = g->desc.nviews;
    const int dt = g->desc.storage;
    const size_t npix = W.npix;
    UpdateArgs U;
    // D_L = A' (w .* A 1) over all views (float32 intermediate whatever the storage type)
    CT_HIP_CHECK(launch_forward(fp_launch(G, nullptr, nullptr, 0, 1, nv, nullptr, w, 1.f, W.r), 1, FP_WEIGHTED, dt, s));
    CT_HIP_CHECK(launch_back_update(bp_launch(G, W.r, 0, 1, nv, dl, U), BP_BACK, CT_F32, CT_F32, s));
    if (p->dl_scale != 1.0) CT_HIP_CHECK(launch_scale(dl, npix, (float)p->dl_scale, s));
    if (p->kappa && kappa) {
        // kappa = sqrt(A'w / A'1)
        CT_HIP_CHECK(launch_back_update(bp_launch(G, w, 0, 1, nv, kappa, U), BP_BACK, dt, CT_F32, s));
        CT_HIP_CHECK(launch_fill(W.r, (size_t)nv * g->desc.nb, 1.f, s));
        CT_HIP_CHECK(launch_back_update(bp_launch(G, W.r, 0, 1, nv, W.tmp, U), BP_BACK, CT_F32, CT_F32, s));
        CT_HIP_CHECK(launch_kappa(kappa, W.tmp, kappa, npix, s));
    }
    return CT_OK;
}

// x (caller) -> clipped copy in A (+ transpose); then the initial gradient and g, h.
ct_status do_init(const Ctx &c, const float *x_in, int zero_start, hipStream_t s)
{
    ct_geom *g = c.g;
    Workspace &W = g->ws;
    const GeomDev &G = g->dev;
    CT_HIP_CHECK(launch_clip_copy(x_in, W.xa, proj_copy(W, c.dtype, 1), W.xta, g->desc.nx, g->desc.ny, zero_start,
                                  c.dtype, s));
    UpdateArgs U = make_update(c);
    U.x = W.xa;
    const void *img = proj_img(W, c.dtype, 1);
    if (c.p->init_full) {
        const int nv = g->desc.nviews;
        CT_HIP_CHECK(launch_forward(fp_launch(G, img, W.xta, 0, 1, nv, c.y, c.w, 1.f, W.r), 0, FP_RESIDUAL, c.dtype, s));
        CT_HIP_CHECK(launch_back_update(bp_launch(G, W.r, 0, 1, nv, nullptr, U), BP_INIT, c.dtype, c.dtype, s));
    } else {
        const int m = c.order[(size_t)c.M - 1];
        FpLaunch a = fp_launch(G, img, W.xta, m, c.M, c.nvm, c.y, c.w, (float)c.M, W.r);
        a.out2 = split_plane(c, c.nvm);
        CT_HIP_CHECK(launch_forward(a, 0, FP_RESIDUAL, c.dtype, s));
        BpLaunch b = bp_launch(G, W.r, m, c.M, c.nvm, nullptr, U);
        b.r2 = a.out2;
        CT_HIP_CHECK(launch_back_update(b, BP_INIT, b.r2 ? CT_F32 : c.dtype, c.dtype, s));
    }
    return CT_OK;
}

// ---- batched solve ----------------------------------------------------------------------------

// Slice table of a batch in a given slice order, with contiguous workgroup ranges. Buffer index 0 is
// ping-pong buffer A, 1 is B.
// split_mode: the forward launch's split of each block's lines over two workgroups, -1 automatic (decided
// for the launch as a whole: when all of its unsplit forward workgroups would underfill the device), 0
// never, 1 always (where eligible); a solve's own forward_split setting other than -1 overrides it.
std::vector<SliceDev> slice_table(const std::vector<Ctx> &cs, const std::vector<int> &order, int fp_waves,
                                  int split_mode, int *nwg_fp, int *nwg_bp)
{
    std::vector<SliceDev> tab;
    int fp = 0, bp = 0;
    int fp_all = 0;
    for (int i : order) fp_all += forward_workgroups(cs[(size_t)i].g->dev, cs[(size_t)i].nvm, fp_waves, false);
    const int batch_split = split_mode >= 0 ? split_mode : (launch_underfills(fp_all) ? 1 : 0);
    for (int i : order) {
        const Ctx &c = cs[(size_t)i];
        const Workspace &W = c.g->ws;
        SliceDev S;
        S.G = c.g->dev;
        S.M = c.M;
        S.nvm = c.nvm;
        S.y = c.y;
        S.w = c.w;
        S.r = W.r;
        S.r2 = split_plane(c, c.nvm, batch_split);
        S.x[0] = W.xa;
        S.x[1] = W.xb;
        S.xc[0] = const_cast<void *>(proj_img(W, c.dtype, 1));
        S.xc[1] = const_cast<void *>(proj_img(W, c.dtype, 0));
        S.xt[0] = W.xta;
        S.xt[1] = W.xtb;
        S.gv = c.gv;
        S.h = c.h;
        S.dl = c.dl;
        S.kappa = c.kappa;
        S.fp_begin = fp;
        fp += forward_workgroups(S.G, S.nvm, fp_waves, S.r2 != nullptr);
        S.fp_end = fp;
        S.bp_begin = bp;
        bp += update_workgroups(S.G);
        S.bp_end = bp;
        tab.push_back(S);
    }
    *nwg_fp = fp;
    *nwg_bp = bp;
    return tab;
}

BatchUpdate batch_update(const Ctx &c, long long tofs)
{
    const UpdateArgs U = make_update(c);
    BatchUpdate u;
    u.rho = U.rho;
    u.tbase = U.tbase;
    u.tofs = tofs;
    u.alpha = U.alpha;
    u.algorithm = U.algorithm;
    u.potential = U.potential;
    u.huber = U.huber;
    u.delta = U.delta;
    u.idelta = U.idelta;
    u.beta_ax = U.beta_ax;
    u.beta_dg = U.beta_dg;
    return u;
}

// One batched subiteration (subset m; tofs relative to the device counter), images in buffer par.
hipError_t batch_subiter(const SliceDev *dtab, int ns, int nwg_fp, int nwg_bp, int m, int par, const BatchUpdate &u,
                         int dtype, int fp_waves, hipStream_t s)
{
    hipError_t e = launch_forward_batch(dtab, ns, nwg_fp, m, par, dtype, fp_waves, s);
    if (e != hipSuccess) return e;
    return launch_update_batch(dtab, ns, nwg_bp, m, par, u, dtype, s);
}

struct BatchKey {
    int device;
    std::vector<int> shape;
    bool operator<(const BatchKey &o) const { return device != o.device ? device < o.device : shape < o.shape; }
};

std::mutex g_tune_mu;
std::map<BatchKey, ct_batch_config> g_tune_cache;

// Device copy of a slice table (caller frees).
ct_status upload_table(const std::vector<SliceDev> &tab, SliceDev **dtab, hipStream_t s)
{
    CT_TRY(dev_alloc(dtab, tab.size()));
    CT_HIP_CHECK(hipMemcpyAsync(*dtab, tab.data(), tab.size() * sizeof(SliceDev), hipMemcpyHostToDevice, s));
    CT_HIP_CHECK(hipStreamSynchronize(s));   // the host table may go out of scope
    return CT_OK;
}

// Times each candidate launch shape of the selected forms on the prepared slices (two subiterations of
// warm-up, then kReps timed); it overwrites the slices' ping-pong images, g, h and residual blocks, which
// the initialisation that follows rewrites.
ct_status tune_batch(const std::vector<Ctx> &cs, hipStream_t s, ct_batch_config *best, bool lockstep, bool persistent)
{
    constexpr int kReps = 6;
    const int n = (int)cs.size();
    std::vector<int> given(n), largest(n);
    std::iota(given.begin(), given.end(), 0);
    largest = given;
    std::stable_sort(largest.begin(), largest.end(), [&](int a, int b) {
        auto work = [&](int i) {
            const ct_geom_desc &d = cs[(size_t)i].g->desc;
            return (double)d.nx * d.ny * cs[(size_t)i].nvm;
        };
        return work(a) > work(b);
    });
    for (const Ctx &c : cs) {   // zero images and copies, so that the timed launches read defined data
        const Workspace &W = c.g->ws;
        CT_HIP_CHECK(launch_clip_copy(W.xa, W.xa, proj_copy(W, c.dtype, 1), W.xta, c.g->desc.nx, c.g->desc.ny, 1,
                                      c.dtype, s));
        CT_HIP_CHECK(launch_clip_copy(W.xb, W.xb, proj_copy(W, c.dtype, 0), W.xtb, c.g->desc.nx, c.g->desc.ny, 1,
                                      c.dtype, s));
        CT_HIP_CHECK(launch_fill(c.gv, W.npix, 0.f, s));
        CT_HIP_CHECK(launch_fill(c.h, W.npix, 0.f, s));
    }
    CT_HIP_CHECK(launch_set_counter(cs[0].g->ws.tbase, 0, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CT_HIP_CHECK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(CT_ERR_HIP, "hipEventCreate failed");
    }
    ct_status st = CT_OK;
    best->ms_subiteration = 1e30;
    const int M = cs[0].M;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
    const int max_bpc = persistent_blocks_per_cu(cs[0].dtype);
    std::vector<int> ord(cs[0].order);
    int *dorder = nullptr;
    if (persistent && cus > 0 && max_bpc > 0) {
        st = dev_alloc(&dorder, ord.size());
        if (st == CT_OK && hipMemcpy(dorder, ord.data(), ord.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
            st = fail(CT_ERR_HIP, "batch tuning: order upload failed");
    }
    for (int lf = 0; lf < 2 && st == CT_OK; ++lf) {
        if (lf == 1 && largest == given) continue;
        // the persistent launch: 1, 2 or 4 resident workgroups per CU (within the occupancy limit)
        for (int bpc : {1, 2, 4}) {
            if (!dorder || bpc > max_bpc || st != CT_OK) continue;
            int nfp = 0, nbp = 0;
            std::vector<SliceDev> tab = slice_table(cs, lf ? largest : given, 8, -1, &nfp, &nbp);
            SliceDev *dtab = nullptr;
            st = upload_table(tab, &dtab, s);
            if (st != CT_OK) break;
            const BatchUpdate u = batch_update(cs[0], 0);
            int *state = cs[0].g->ws.tbase;
            hipError_t e = launch_batch_persistent(dtab, n, nfp, nbp, dorder, M, 0, 2, 1, u, state, bpc * cus,
                                                   cs[0].dtype, s);
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            if (e == hipSuccess)
                e = launch_batch_persistent(dtab, n, nfp, nbp, dorder, M, 0, kReps, 1, u, state, bpc * cus,
                                            cs[0].dtype, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            int flag = 0;
            if (e == hipSuccess) e = hipMemcpy(&flag, state + 3, sizeof(int), hipMemcpyDeviceToHost);
            (void)hipFree(dtab);
            if (e != hipSuccess) {
                st = fail(CT_ERR_HIP, std::string("batch tuning: ") + hipGetErrorString(e));
                break;
            }
            const double per = ms / kReps;
            if (flag == 0 && per < best->ms_subiteration) {
                best->ms_subiteration = per;
                best->fp_waves = 8;
                best->largest_first = lf;
                best->persistent = 1;
                best->blocks_per_cu = bpc;
                best->forward_split = -1;
            }
        }
        // lockstep: 16 or 8 forward waves per workgroup, each with the forward split never and always (when
        // the solve leaves the split to the library; otherwise its own setting)
        const bool tune_split = cs[0].p->forward_split == -1;
        for (int cand = 0; cand < 4 && lockstep; ++cand) {
            const int waves = cand < 2 ? 16 : 8, split = tune_split ? (cand & 1) : -1;
            if (!tune_split && (cand & 1)) continue;
            int nfp = 0, nbp = 0;
            std::vector<SliceDev> tab = slice_table(cs, lf ? largest : given, waves, split, &nfp, &nbp);
            SliceDev *dtab = nullptr;
            st = upload_table(tab, &dtab, s);
            if (st != CT_OK) break;
            const BatchUpdate u = batch_update(cs[0], 0);
            hipError_t e = hipSuccess;
            int par = 1;
            for (int r = 0; r < 2 + kReps && e == hipSuccess; ++r) {
                if (r == 2) e = hipEventRecord(e0, s);
                if (e == hipSuccess)
                    e = batch_subiter(dtab, n, nfp, nbp, cs[0].order[(size_t)(r % M)], par, u, cs[0].dtype, waves, s);
                par ^= 1;
            }
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            (void)hipFree(dtab);
            if (e != hipSuccess) {
                st = fail(CT_ERR_HIP, std::string("batch tuning: ") + hipGetErrorString(e));
                break;
            }
            const double per = ms / kReps;
            if (per < best->ms_subiteration) {
                best->ms_subiteration = per;
                best->fp_waves = waves;
                best->largest_first = lf;
                best->persistent = 0;
                best->blocks_per_cu = 0;
                best->forward_split = split;
            }
        }
    }
    if (dorder) (void)hipFree(dorder);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

// On-disk cache of tuned launch shapes: one text file per (device architecture, slice-shape set) under
// $CTRLALM_TUNE_DIR, else $XDG_CACHE_HOME/ctrlalm/tune, else ~/.cache/ctrlalm/tune. Empty path: no cache.
std::string tune_file(int device, const BatchKey &key)
{
    std::string dir;
    if (const char *e = std::getenv("CTRLALM_TUNE_DIR")) dir = e;
    else if (const char *x = std::getenv("XDG_CACHE_HOME")) dir = std::string(x) + "/ctrlalm/tune";
    else if (const char *h = std::getenv("HOME")) dir = std::string(h) + "/.cache/ctrlalm/tune";
    if (dir.empty()) return std::string();
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return std::string();
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    unsigned long long h = 1469598103934665603ull;   // FNV-1a of the shape set
    for (int v : key.shape) {
        h ^= (unsigned long long)(unsigned)v;
        h *= 1099511628211ull;
    }
    char name[64];
    std::snprintf(name, sizeof(name), "/%016llx.txt", h);
    return dir + "/" + arch + name;
}

bool read_tuned(const std::string &path, ct_batch_config *cfg, int max_bpc)
{
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    ct_batch_config c{};
    const int got = std::fscanf(f, "fp_waves %d largest_first %d persistent %d blocks_per_cu %d forward_split %d ms %lf",
                                &c.fp_waves, &c.largest_first, &c.persistent, &c.blocks_per_cu, &c.forward_split,
                                &c.ms_subiteration);
    std::fclose(f);
    const bool ok = got == 6 && (c.fp_waves == 8 || c.fp_waves == 16) && (c.largest_first == 0 || c.largest_first == 1) &&
                    (c.persistent == 0 || (c.persistent == 1 && c.blocks_per_cu >= 1 && c.blocks_per_cu <= max_bpc)) &&
                    c.forward_split >= -1 && c.forward_split <= 1;
    if (ok) *cfg = c;
    return ok;
}

void write_tuned(const std::string &path, const ct_batch_config &c)
{
    // create the directories on the way (best effort: without them the cache is simply not written)
    for (size_t pos = path.find('/', 1); pos != std::string::npos; pos = path.find('/', pos + 1))
        (void)mkdir(path.substr(0, pos).c_str(), 0755);
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "fp_waves %d largest_first %d persistent %d blocks_per_cu %d forward_split %d ms %.6f\n",
                 c.fp_waves, c.largest_first, c.persistent, c.blocks_per_cu, c.forward_split, c.ms_subiteration);
    std::fclose(f);
    (void)std::rename(tmp.c_str(), path.c_str());
}

// The batched solve as one captured graph: every slice's initialisation and first x-step, then one
// persistent launch of all nsub subiterations. Waits for the device at the end (finiteness and the
// barrier's error flag).
template <typename Init>
ct_status persistent_batched(ct_geom *const *gs, int n, const ct_rlalm_params *p, float *const *x,
                             const std::vector<Ctx> &cs, const ct_batch_config &cfg, int cus, Init init_all,
                             hipStream_t s)
{
    const Workspace &W0 = gs[0]->ws;
    const long long nsub = (long long)p->niters * cs[0].M;
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    if (cfg.largest_first)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            auto work = [&](int i) { return (double)gs[i]->desc.nx * gs[i]->desc.ny * cs[(size_t)i].nvm; };
            return work(a) > work(b);
        });
    int nfp = 0, nbp = 0;
    std::vector<SliceDev> tab = slice_table(cs, order, 8, -1, &nfp, &nbp);
    SliceDev *dtab = nullptr;
    CT_TRY(upload_table(tab, &dtab, s));
    int *dorder = nullptr;
    ct_status st = dev_alloc(&dorder, cs[0].order.size());
    if (st == CT_OK &&
        hipMemcpy(dorder, cs[0].order.data(), cs[0].order.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        st = fail(CT_ERR_HIP, "order upload failed");
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (st == CT_OK && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        st = fail(CT_ERR_HIP, "capture stream");
    if (st == CT_OK) {
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) st = fail(CT_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        if (st == CT_OK) st = init_all(cap);
        if (st == CT_OK) {
            e = launch_batch_persistent(dtab, n, nfp, nbp, dorder, cs[0].M, 0, nsub, 1, batch_update(cs[0], 0), W0.tbase,
                                        cfg.blocks_per_cu * cus, cs[0].dtype, cap);
            if (e != hipSuccess) st = fail(CT_ERR_HIP, std::string("persistent launch: ") + hipGetErrorString(e));
        }
        e = hipStreamEndCapture(cap, &graph);
        if (st == CT_OK && e != hipSuccess) st = fail(CT_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        if (st == CT_OK && (e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess)
            st = fail(CT_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        if (st == CT_OK && (e = hipGraphLaunch(exec, s)) != hipSuccess)
            st = fail(CT_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    }
    // x^(nsub) is the input of the last projection: buffer B (index 1) after an odd number of
    // subiterations' swaps from B, A otherwise (nothing ran: A)
    const int fin = nsub > 0 ? (int)((1 + nsub - 1) & 1) : 0;
    std::vector<double> host(3 * (size_t)n);
    int flag = 0;
    for (int i = 0; i < n && st == CT_OK; ++i) {
        ct_geom *g = gs[i];
        Workspace &W = g->ws;
        hipError_t e = hipMemcpyAsync(x[i], fin ? W.xb : W.xa, W.npix * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = launch_trace_reduce(x[i], nullptr, W.gv, W.h, g->desc.nx, g->desc.ny, (float)g->desc.dx,
                                    (float)g->desc.dy, 0.f, W.red, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&host[3 * (size_t)i], W.red, 3 * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) st = fail(CT_ERR_HIP, std::string("batched result: ") + hipGetErrorString(e));
    }
    if (st == CT_OK && hipMemcpyAsync(&flag, W0.tbase + 3, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        st = fail(CT_ERR_HIP, "barrier flag readback");
    const hipError_t es = hipStreamSynchronize(s);
    if (st == CT_OK && es != hipSuccess) st = fail(CT_ERR_HIP, std::string("batched solve: ") + hipGetErrorString(es));
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    if (dorder) (void)hipFree(dorder);
    (void)hipFree(dtab);
    if (st != CT_OK) return st;
    if (flag) return fail(CT_ERR_HIP, "persistent batched launch: a grid barrier wait gave up (workgroups not resident)");
    for (int i = 0; i < n; ++i)
        if (host[3 * (size_t)i + 2] != 0.0)
            return fail(CT_ERR_DIVERGED, "non-finite values in the final state of slice " + std::to_string(i));
    return CT_OK;
}

}  // namespace

extern "C" {

const char *ct_last_error(void) { return g_last_error.c_str(); }

ct_status ct_rlalm_kernel_times(const ct_geom *g, ct_kernel_times *out)
{
    if (!g || !out) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    if (!g->ktimes_valid) return fail(CT_ERR_INVALID_ARG, "no solve with time_kernels = 1 on this handle");
    *out = g->ktimes;
    return CT_OK;
}

void ct_rlalm_params_default(ct_rlalm_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->alpha = 1.999;
    p->niters = 20;
    p->rho_mode = 0;
    p->rho_fixed = 0.05;
    p->potential = 0;
    p->delta = 1e-4;
    p->beta = 1024.0;
    p->huber = 1;
    p->algorithm = 1;
    p->subset_order = CT_ORDER_SEQUENTIAL;
    p->kappa = 0;
    p->start = 0;
    p->init_full = 0;
    p->dl_scale = 1.0;
    p->x_ref = nullptr;
    p->mu_water = 0.02;
    p->fov_radius = 0.0;
    p->use_graph = 1;
    p->time_kernels = 0;
    p->forward_split = -1;
    p->diverge_factor = 2.0;
    p->diverge_window = 3;
}

// The update kernel's bin windows, once per geometry (7.9 MB for 512^2 pixels and 984 views); above
// 256 MiB the kernel computes them itself, as it would without the table.
static ct_status build_tile_windows(ct_geom *g)
{
    const size_t nwin = tile_windows_count(g->dev);
    if (nwin * sizeof(int2) > (size_t(256) << 20)) return CT_OK;
    CT_HIP_CHECK(hipMalloc(&g->win, nwin * sizeof(int2)));
    CT_HIP_CHECK(launch_tile_windows(g->dev, g->win, nullptr));
    CT_HIP_CHECK(hipStreamSynchronize(nullptr));
    g->dev.win = g->win;
    return CT_OK;
}

ct_status ct_geom_create(const ct_geom_desc *desc, ct_geom **out)
{
    if (!out) return fail(CT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    CT_TRY(check_desc(desc));
    ct_geom *g = new (std::nothrow) ct_geom();
    if (!g) return fail(CT_ERR_OOM, "host allocation failed");
    g->desc = *desc;
    (void)hipGetDevice(&g->device);
    ct_status st = build_geometry(g);
    if (st == CT_OK) st = build_tile_windows(g);
    if (st != CT_OK) {
        free_geometry(g);
        delete g;
        return st;
    }
    *out = g;
    return CT_OK;
}

void ct_geom_destroy(ct_geom *g)
{
    if (!g) return;
    (void)hipDeviceSynchronize();
    drop_graph_cache(g);
    free_workspace(g);
    free_geometry(g);
    if (g->status_host) (void)hipHostFree(g->status_host);
    if (g->rho_host) (void)hipHostFree(g->rho_host);
    if (g->status_ev) (void)hipEventDestroy(g->status_ev);
    if (g->rho_ev) (void)hipEventDestroy(g->rho_ev);
    delete g;
}

static ct_status subset_range(const ct_geom *g, int subset, int *vstart, int *vstride, int *nv)
{
    const int M = g->desc.nsubsets;
    if (subset == -1) {
        *vstart = 0;
        *vstride = 1;
        *nv = g->desc.nviews;
        return CT_OK;
    }
    if (subset < 0 || subset >= M) return fail(CT_ERR_INVALID_ARG, "subset must be -1 or in [0, M)");
    *vstart = subset;
    *vstride = M;
    *nv = g->desc.nviews / M;
    return CT_OK;
}

ct_status ct_forward(const ct_geom *gc, int subset, const float *x, float *p, void *stream)
{
    if (!gc || !x || !p) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    ct_geom *g = const_cast<ct_geom *>(gc);
    int vs, vst, nv;
    CT_TRY(subset_range(g, subset, &vs, &vst, &nv));
    CT_TRY(ensure_workspace(g, 0, 4));
    hipStream_t s = as_stream(stream);
    CT_HIP_CHECK(launch_transpose(x, g->ws.tmp, g->desc.nx, g->desc.ny, s));
    CT_HIP_CHECK(launch_forward(fp_launch(g->dev, x, g->ws.tmp, vs, vst, nv, nullptr, nullptr, 1.f, p), 0, FP_PLAIN,
                                CT_F32, s));
    return CT_OK;
}

}  // extern "C"

// Scratch of ct_forward_noalloc: the projector's transposed image copy, in a file-scope device array that
// each GPU holds until the process ends. Host code never uses the array's name as an address: its device
// address is looked up once per device (hipGetSymbolAddress, with that device current) and kept.
namespace {

constexpr size_t kNoAllocFloats = (size_t)4 << 20;   // 16 MiB: images up to 4 Mi pixels (2048 x 2048)
__device__ __align__(256) float scratch[kNoAllocFloats];

std::mutex g_scratch_mu;
std::map<int, float *> g_scratch_addr;

ct_status scratch_address(int device, float **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return CT_OK;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(CT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[device] = static_cast<float *>(ptr);
    *out = static_cast<float *>(ptr);
    return CT_OK;
}

}  // namespace

extern "C" {

ct_status ct_forward_noalloc(const ct_geom *gc, int subset, const float *x, float *p, void *stream)
{
    if (!gc || !x || !p) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    int vs, vst, nv;
    CT_TRY(subset_range(gc, subset, &vs, &vst, &nv));
    const size_t npix = (size_t)gc->desc.nx * gc->desc.ny;
    if (npix > kNoAllocFloats)
        return fail(CT_ERR_INVALID_ARG, "image of " + std::to_string(npix) + " pixels exceeds the " +
                                            std::to_string(kNoAllocFloats) + "-pixel scratch of ct_forward_noalloc");
    int dev = -1;
    CT_HIP_CHECK(hipGetDevice(&dev));
    if (dev != gc->device) return fail(CT_ERR_INVALID_ARG, "the geometry's device must be the current device");
    float *xt = nullptr;
    CT_TRY(scratch_address(dev, &xt));
    hipStream_t s = as_stream(stream);
    CT_HIP_CHECK(launch_transpose(x, xt, gc->desc.nx, gc->desc.ny, s));
    CT_HIP_CHECK(launch_forward(fp_launch(gc->dev, x, xt, vs, vst, nv, nullptr, nullptr, 1.f, p), 0, FP_PLAIN, CT_F32,
                                s));
    return CT_OK;
}

ct_status ct_back(const ct_geom *gc, int subset, const float *r, float *x, void *stream)
{
    if (!gc || !r || !x) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    ct_geom *g = const_cast<ct_geom *>(gc);
    int vs, vst, nv;
    CT_TRY(subset_range(g, subset, &vs, &vst, &nv));
    UpdateArgs U;
    CT_HIP_CHECK(launch_back_update(bp_launch(g->dev, r, vs, vst, nv, x, U), BP_BACK, CT_F32, CT_F32, as_stream(stream)));
    return CT_OK;
}

ct_status ct_fbp(const ct_geom *gc, const void *y, float *x, void *stream)
{
    if (!gc || !y || !x) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    ct_geom *g = const_cast<ct_geom *>(gc);
    if (g->desc.det != CT_DET_FLAT) return fail(CT_ERR_UNSUPPORTED, "the FBP-like start supports the flat detector only");
    CT_TRY(ensure_workspace(g, g->desc.nviews, 4));
    CT_HIP_CHECK(launch_fbp(g, y, g->desc.storage, g->ws.r, g->cs, x, as_stream(stream)));
    return CT_OK;
}

ct_status ct_rlalm_prepare(ct_geom *g, const ct_rlalm_params *p, const void *w, float *dl, float *kappa, void *stream)
{
    if (!g || !w || !dl) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    CT_TRY(check_params(p));
    return do_prepare(g, p, w, dl, kappa, as_stream(stream));
}

ct_status ct_rlalm_init(ct_geom *g, const ct_rlalm_params *p, const void *y, const void *w, const float *dl, float *x,
                        float *gv, float *h, void *stream)
{
    if (!g || !y || !w || !dl || !x || !gv || !h) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    CT_TRY(check_params(p));
    CT_TRY(ensure_workspace(g, g->desc.nviews, 4));
    hipStream_t s = as_stream(stream);
    Ctx c = make_ctx(g, p, y, w, dl, nullptr, gv, h);
    CT_TRY(do_init(c, x, p->start == 1, s));
    CT_HIP_CHECK(hipMemcpyAsync(x, g->ws.xa, g->ws.npix * sizeof(float), hipMemcpyDeviceToDevice, s));
    return CT_OK;
}

ct_status ct_rlalm_iterate(ct_geom *g, const ct_rlalm_params *p, const void *y, const void *w, const float *dl,
                           const float *kappa, float *x, float *gv, float *h, long long t0, long long nsub,
                           void *stream)
{
    if (!g || !y || !w || !dl || !x || !gv || !h) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    CT_TRY(check_params(p));
    if (t0 < 0 || nsub < 0 || t0 + nsub + 2 > (1ll << 30)) return fail(CT_ERR_INVALID_ARG, "bad t0 / nsub");
    if (p->kappa && !kappa) return fail(CT_ERR_INVALID_ARG, "kappa requested but NULL");
    if (nsub == 0) return CT_OK;
    hipStream_t s = as_stream(stream);
    CT_TRY(ensure_workspace(g, g->desc.nviews, (size_t)(t0 + nsub + 2)));
    CT_TRY(upload_rho(g, p, t0 + nsub + 2, s));
    Ctx c = make_ctx(g, p, y, w, dl, kappa, gv, h);
    CT_HIP_CHECK(hipMemcpyAsync(g->ws.xa, x, g->ws.npix * sizeof(float), hipMemcpyDeviceToDevice, s));
    int fin = 1;
    CT_TRY(run_subiters(c, t0, nsub, p->use_graph, s, &fin, nullptr, p, std::chrono::steady_clock::now()));
    if (fin >= 0)
        CT_HIP_CHECK(hipMemcpyAsync(x, fin ? g->ws.xa : g->ws.xb, g->ws.npix * sizeof(float), hipMemcpyDeviceToDevice, s));
    return CT_OK;
}

ct_status ct_rlalm_solve(ct_geom *g, const ct_rlalm_params *p, const void *y, const void *w, float *x,
                         ct_trace_row *trace, void *stream)
{
    auto tstart = std::chrono::steady_clock::now();
    if (!g || !y || !w || !x) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    CT_TRY(check_params(p));
    hipStream_t s = as_stream(stream);
    const long long nsub = (long long)p->niters * g->desc.nsubsets;
    CT_TRY(ensure_workspace(g, g->desc.nviews, (size_t)(nsub + 2)));
    Workspace &W = g->ws;
    CT_TRY(dev_alloc(&W.dl, W.npix));
    CT_TRY(dev_alloc(&W.gv, W.npix));
    CT_TRY(dev_alloc(&W.h, W.npix));
    if (p->kappa) CT_TRY(dev_alloc(&W.kappa, W.npix));
    CT_TRY(upload_rho(g, p, nsub + 2, s));
    if (p->start == 2) {   // FBP-like start image, written into x
        if (g->desc.det != CT_DET_FLAT) return fail(CT_ERR_UNSUPPORTED, "the FBP-like start supports the flat detector only");
        CT_HIP_CHECK(launch_fbp(g, y, g->desc.storage, W.r, g->cs, x, s));
    }
    CT_TRY(do_prepare(g, p, w, W.dl, p->kappa ? W.kappa : nullptr, s));
    if (p->start == 3) {
        if (g->desc.det != CT_DET_FLAT) return fail(CT_ERR_UNSUPPORTED, "the learned start supports the flat detector only");
        CT_TRY(learned_start(g, p->unet, y, p->mu_water, x, W.xa, W.xb, s));
    }
    Ctx c = make_ctx(g, p, y, w, W.dl, W.kappa, W.gv, W.h);
    CT_TRY(do_init(c, x, p->start == 1, s));
    if (trace)
        for (int i = 0; i < p->niters; ++i) trace[i] = ct_trace_row{0, 0.0, NAN, NAN, 0, NAN, NAN};
    int fin = -1;
    if (nsub > 0) CT_TRY(run_subiters(c, 0, nsub, p->use_graph, s, &fin, trace, p, tstart, x));
    const float *xf = fin == 0 ? W.xb : W.xa;
    CT_HIP_CHECK(hipMemcpyAsync(x, xf, W.npix * sizeof(float), hipMemcpyDeviceToDevice, s));
    // finiteness of the final state: an FP64 reduction on the device, read back without waiting
    CT_HIP_CHECK(launch_trace_reduce(x, nullptr, W.gv, W.h, g->desc.nx, g->desc.ny, (float)g->desc.dx,
                                     (float)g->desc.dy, 0.f, W.red + kRedTrace, s));
    if (!g->status_host)
        CT_HIP_CHECK(hipHostMalloc((void **)&g->status_host, kTraceOut * sizeof(double), hipHostMallocDefault));
    if (!g->status_ev) CT_HIP_CHECK(hipEventCreateWithFlags(&g->status_ev, hipEventDisableTiming));
    CT_HIP_CHECK(hipMemcpyAsync(g->status_host, W.red + kRedTrace, kTraceOut * sizeof(double), hipMemcpyDeviceToHost, s));
    CT_HIP_CHECK(hipEventRecord(g->status_ev, s));
    g->status_pending = true;
    if (trace || p->time_kernels) CT_TRY(ct_rlalm_status(g));
    if (p->time_kernels && nsub > 0) CT_TRY(time_last_subiteration(c, nsub - 1, fin == 0 ? 0 : 1, s));
    return CT_OK;
}

ct_status ct_rlalm_status(ct_geom *g)
{
    if (!g) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    if (!g->status_pending) return CT_OK;
    CT_HIP_CHECK(hipEventSynchronize(g->status_ev));
    if (g->status_host[2] != 0.0) return fail(CT_ERR_DIVERGED, "non-finite values in the final state");
    return CT_OK;
}

ct_status ct_cost(ct_geom *g, const ct_rlalm_params *p, const void *y, const void *w, const float *x,
                  const float *kappa, double *out, void *stream)
{
    if (!g || !y || !w || !x || !out) return fail(CT_ERR_INVALID_ARG, "NULL argument");
    CT_TRY(check_params(p));
    hipStream_t s = as_stream(stream);
    CT_TRY(do_cost(g, p, y, w, x, kappa, s));
    CT_HIP_CHECK(hipMemcpyAsync(out, g->ws.red + kRedCost, kCostOut * sizeof(double), hipMemcpyDeviceToDevice, s));
    return CT_OK;
}

ct_status ct_rlalm_solve_batched(ct_geom *const *gs, int n, const ct_rlalm_params *p, const void *const *y,
                                 const void *const *w, float *const *x, int autotune, ct_batch_config *chosen,
                                 void *stream)
{
    if (!gs || !y || !w || !x || n < 1) return fail(CT_ERR_INVALID_ARG, "NULL argument or n < 1");
    CT_TRY(check_params(p));
    if (p->time_kernels) return fail(CT_ERR_UNSUPPORTED, "time_kernels is not available in the batched solve");
    if (autotune < 0 || autotune > 2) return fail(CT_ERR_INVALID_ARG, "autotune must be 0, 1 or 2");
    for (int i = 0; i < n; ++i) {
        if (!gs[i] || !y[i] || !w[i] || !x[i]) return fail(CT_ERR_INVALID_ARG, "NULL slice argument");
        if (gs[i]->desc.nsubsets != gs[0]->desc.nsubsets || gs[i]->desc.storage != gs[0]->desc.storage)
            return fail(CT_ERR_INVALID_ARG, "all slices must share nsubsets and storage");
        if (gs[i]->device != gs[0]->device) return fail(CT_ERR_INVALID_ARG, "all slices must be on one device");
        if ((p->start == 2 || p->start == 3) && gs[i]->desc.det != CT_DET_FLAT)
            return fail(CT_ERR_UNSUPPORTED, "the FBP-like and learned starts support the flat detector only");
        for (int j = 0; j < i; ++j)
            if (gs[j] == gs[i]) return fail(CT_ERR_INVALID_ARG, "each slice needs its own handle");
    }
    hipStream_t s = as_stream(stream);
    const long long nsub = (long long)p->niters * gs[0]->desc.nsubsets;
    std::vector<Ctx> cs;
    for (int i = 0; i < n; ++i) {
        ct_geom *g = gs[i];
        CT_TRY(ensure_workspace(g, g->desc.nviews, (size_t)(nsub + 2)));
        Workspace &W = g->ws;
        CT_TRY(dev_alloc(&W.dl, W.npix));
        CT_TRY(dev_alloc(&W.gv, W.npix));
        CT_TRY(dev_alloc(&W.h, W.npix));
        if (p->kappa) CT_TRY(dev_alloc(&W.kappa, W.npix));
        if (i == 0) CT_TRY(upload_rho(g, p, nsub + 2, s));
        if (p->start == 2) CT_HIP_CHECK(launch_fbp(g, y[i], g->desc.storage, W.r, g->cs, x[i], s));
        CT_TRY(do_prepare(g, p, w[i], W.dl, p->kappa ? W.kappa : nullptr, s));
        if (p->start == 3) CT_TRY(learned_start(g, p->unet, y[i], p->mu_water, x[i], W.xa, W.xb, s));
        cs.push_back(make_ctx(g, p, y[i], w[i], W.dl, W.kappa, W.gv, W.h));
    }
    // every slice reads the rho table and subiteration counter of slice 0
    const Workspace &W0 = gs[0]->ws;

    ct_batch_config cfg{16, 0, 0.0, 0, 0, -1};
    int dev = 0, cus = 0;
    CT_HIP_CHECK(hipGetDevice(&dev));
    CT_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (autotune == 1) {
        BatchKey key{gs[0]->device, {}};
        for (int i = 0; i < n; ++i) {
            const ct_geom_desc &d = gs[i]->desc;
            key.shape.insert(key.shape.end(), {d.nx, d.ny, d.nb, d.nviews, d.nsubsets, d.storage});
        }
        bool have = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                cfg = it->second;
                have = true;
            }
        }
        const std::string path = tune_file(dev, key);
        if (!have && !path.empty()) have = read_tuned(path, &cfg, persistent_blocks_per_cu(cs[0].dtype));
        if (!have) {
            CT_TRY(tune_batch(cs, s, &cfg, true, true));
            if (!path.empty()) write_tuned(path, cfg);
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = cfg;
    } else if (autotune == 2) {
        // the persistent launch, its workgroups per CU and slice order tuned on this batch (not cached)
        if (persistent_blocks_per_cu(cs[0].dtype) < 1)
            return fail(CT_ERR_UNSUPPORTED, "the persistent batched kernel cannot be resident on this device");
        CT_TRY(tune_batch(cs, s, &cfg, false, true));
        if (cfg.persistent != 1) return fail(CT_ERR_HIP, "no persistent launch shape completed its grid barriers");
    }
    if (chosen) *chosen = cfg;

    // initial state of every slice, then the x-step of subiteration 0 (A -> B): eager for the lockstep
    // launches, part of the one captured graph for the persistent launch
    auto init_all = [&](hipStream_t st) -> ct_status {
        for (int i = 0; i < n; ++i) {
            const Ctx &c = cs[(size_t)i];
            CT_TRY(do_init(c, x[i], p->start == 1, st));
            Workspace &W = c.g->ws;
            UpdateArgs U = make_update(c);
            U.rho = W0.rho;
            U.tbase = W0.tbase;
            U.x = W.xa;
            U.x_next = W.xb;
            U.xc_next = proj_copy(W, c.dtype, 0);
            U.xT_next = W.xtb;
            U.tofs = 0;
            CT_HIP_CHECK(launch_set_counter(W0.tbase, 0, st));
            CT_HIP_CHECK(launch_back_update(bp_launch(c.g->dev, nullptr, 0, 1, 0, nullptr, U), BP_XSTEP, c.dtype, c.dtype,
                                            st));
        }
        return CT_OK;
    };
    if (cfg.persistent) return persistent_batched(gs, n, p, x, cs, cfg, cus, init_all, s);
    CT_TRY(init_all(s));
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    if (cfg.largest_first)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            auto work = [&](int i) { return (double)gs[i]->desc.nx * gs[i]->desc.ny * cs[(size_t)i].nvm; };
            return work(a) > work(b);
        });
    int nfp = 0, nbp = 0;
    std::vector<SliceDev> tab = slice_table(cs, order, cfg.fp_waves, cfg.forward_split, &nfp, &nbp);
    SliceDev *dtab = nullptr;
    CT_TRY(upload_table(tab, &dtab, s));
    struct Guard {
        SliceDev *p;
        ~Guard() { if (p) (void)hipFree(p); }
    } guard{dtab};

    const int M = cs[0].M;
    const int dt = cs[0].dtype;
    const std::vector<int> &sub = cs[0].order;
    int par = 1;   // x^(1) is in B
    long long t = 0;
    const int L = (M % 2 == 0) ? M : 2 * M;
    if (p->use_graph && nsub >= L) {
        hipStream_t cap = nullptr;
        CT_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        for (int j = 0; j < L && e == hipSuccess; ++j)
            e = batch_subiter(dtab, n, nfp, nbp, sub[(size_t)(j % M)], (par + j) & 1, batch_update(cs[0], j), dt,
                              cfg.fp_waves, cap);
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        for (; e == hipSuccess && nsub - t >= L; t += L) {
            e = launch_set_counter(W0.tbase, (int)t, s);
            if (e == hipSuccess) e = hipGraphLaunch(exec, s);
        }
        hipError_t e3 = hipStreamSynchronize(s);
        if (e == hipSuccess) e = e3;
        if (exec) (void)hipGraphExecDestroy(exec);
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess) return fail(CT_ERR_HIP, std::string("batched graph: ") + hipGetErrorString(e));
        // L is even: the parity of the images is unchanged by whole graphs
    }
    CT_HIP_CHECK(launch_set_counter(W0.tbase, 0, s));
    for (; t < nsub; ++t) {
        CT_HIP_CHECK(batch_subiter(dtab, n, nfp, nbp, sub[(size_t)(t % M)], par, batch_update(cs[0], t), dt,
                                   cfg.fp_waves, s));
        par ^= 1;
    }
    // x^(nsub) is the input of the last projection: buffer par ^ 1 (par itself when nothing ran)
    const int fin = nsub > 0 ? (par ^ 1) : 0;
    std::vector<double> host(3 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        ct_geom *g = gs[i];
        Workspace &W = g->ws;
        CT_HIP_CHECK(hipMemcpyAsync(x[i], fin ? W.xb : W.xa, W.npix * sizeof(float), hipMemcpyDeviceToDevice, s));
        CT_HIP_CHECK(launch_trace_reduce(x[i], nullptr, W.gv, W.h, g->desc.nx, g->desc.ny, (float)g->desc.dx,
                                         (float)g->desc.dy, 0.f, W.red, s));
        CT_HIP_CHECK(hipMemcpyAsync(&host[3 * (size_t)i], W.red, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    CT_HIP_CHECK(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i)
        if (host[3 * (size_t)i + 2] != 0.0)
            return fail(CT_ERR_DIVERGED, "non-finite values in the final state of slice " + std::to_string(i));
    return CT_OK;
}

}  // extern "C"
