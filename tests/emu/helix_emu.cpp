// Host emulation of the 3-D helical kernels (test infrastructure): runs the per-thread bodies of
// ct_helix_body.hpp over the same grids as the kernels in ct_helix.hip, with every table and volume read
// bounds-checked, so that index arithmetic and results can be checked on a CPU against the FP64 oracle.
// Built by tests/test_helix_emulation.py with g++; no GPU is touched.
#include <string>
#include <vector>

#include "../../paper_1512_04564_amd/csrc/ct_helix_internal.hpp"

namespace ct {
static std::string g_err;
void set_error(const std::string &m) { g_err = m; }
ct_status fail(ct_status st, const std::string &m)
{
    g_err = m;
    return st;
}
}  // namespace ct

using namespace ct;

namespace {

struct Emu {
    HelixTables t;
    HelixDev G{};
};

int setup(const ct_helix_desc *d, Emu &e)
{
    if (helix_tables(*d, e.t) != CT_OK) return 1;
    HelixDev &G = e.G;
    G.nx = d->nx;
    G.ny = d->ny;
    G.nz = d->nz;
    G.nb = d->nb;
    G.nr = d->nr;
    G.nviews = d->nviews;
    G.dx = (float)d->dx;
    G.dy = (float)d->dy;
    G.dso = (float)d->dso;
    G.c_kf = e.t.fan.c_kf;
    G.k0 = e.t.fan.k0;
    G.dwn = e.t.dwn;
    G.bnd = {e.t.fan.bnd64.data(), e.t.fan.bnd64.size()};
    G.scale = {e.t.fan.scale.data(), e.t.fan.scale.size()};
    G.inv = {e.t.fan.inv.data(), e.t.fan.inv.size()};
    G.rowsweep = {e.t.fan.rowsweep.data(), e.t.fan.rowsweep.size()};
    G.cs = {e.t.cs.data(), e.t.cs.size()};
    G.zai = {e.t.zai.data(), e.t.zai.size()};
    G.zaf = {e.t.zaf.data(), e.t.zaf.size()};
    G.wr = {e.t.wr.data(), e.t.wr.size()};
    G.secphi = {e.t.secphi.data(), e.t.secphi.size()};
    return 0;
}

void reset_oob()
{
    hx_oob_count() = 0;
    hx_oob_index() = -1;
}

}  // namespace

extern "C" {

const char *hemu_error(void) { return g_err.c_str(); }

// p[vi][r][k] = A x over views vs + vi * vst (the k_hfp grid, plain epilogue). Returns the number of
// out-of-range reads (-1 for a rejected descriptor); *first receives the first offending index.
int hemu_forward(const ct_helix_desc *d, int vs, int vst, int nv, const float *x, float *p, long long *first)
{
    Emu e;
    if (setup(d, e)) return -1;
    const HelixDev &G = e.G;
    const size_t nvox = (size_t)d->nx * d->ny * d->nz;
    std::vector<float> xT(nvox);
    for (int kz = 0; kz < d->nz; ++kz)
        for (int i = 0; i < d->ny; ++i)
            for (int j = 0; j < d->nx; ++j)
                xT[((size_t)kz * d->nx + j) * d->ny + i] = x[((size_t)kz * d->ny + i) * d->nx + j];
    // the k_hcum pass: padded cumulative forms of both layouts (one thread per column)
    const int ncol = d->nx * d->ny;
    const size_t ncz = nvox + 2 * (size_t)ncol;
    std::vector<float2> cz(ncz), czT(ncz);
    for (int layout = 0; layout < 2; ++layout) {
        const float *in = layout ? xT.data() : x;
        float2 *out = layout ? czT.data() : cz.data();
        for (int c = 0; c < ncol; ++c) {
            double acc = 0.0;
            out[c] = make_float2(0.f, 0.f);
            for (int kz = 0; kz < d->nz; ++kz) {
                const float v = in[(size_t)kz * ncol + c];
                out[(size_t)(kz + 1) * ncol + c] = make_float2((float)acc, v);
                acc += (double)v;
            }
            out[(size_t)(d->nz + 1) * ncol + c] = make_float2((float)acc, 0.f);
        }
    }
    reset_oob();
    for (int vi = 0; vi < nv; ++vi) {
        const int v = vs + vi * vst;
        for (int bx = 0; bx < (d->nb + 63) / 64; ++bx)
            for (int by = 0; by < (d->nr + HX_RB - 1) / HX_RB; ++by) {
                static float part[HX_FW][HX_RB][64];
                const int r0 = by * HX_RB;
                const bool row = G.rowsweep[v] != 0;
                const Ro<float2> X{row ? cz.data() : czT.data(), ncz};
                for (int wave = 0; wave < HX_FW; ++wave)
                    for (int lane = 0; lane < 64; ++lane) {
                        const int k = bx * 64 + lane;
                        float acc[HX_RB];
                        for (int rr = 0; rr < HX_RB; ++rr) acc[rr] = 0.f;
                        if (k < G.nb) hfp_lane<false>(G, X, v, k, r0, wave, HX_FW, acc);
                        for (int rr = 0; rr < HX_RB; ++rr) part[wave][rr][lane] = acc[rr];
                    }
                for (int idx = 0; idx < HX_RB * 64; ++idx) {
                    const int rr = idx >> 6, ln = idx & 63;
                    const int kk = bx * 64 + ln, r = r0 + rr;
                    if (kk >= G.nb || r >= G.nr) continue;
                    float s = part[0][rr][ln];
                    for (int wv = 1; wv < HX_FW; ++wv) s += part[wv][rr][ln];
                    p[((size_t)vi * G.nr + r) * G.nb + kk] =
                        s * G.scale[(size_t)v * G.nb + kk] * G.secphi[(size_t)r * G.nb + kk];
                }
            }
    }
    *first = hx_oob_index();
    return hx_oob_count();
}

// x = A' r over views vs + vi * vst, r [nv][nr][nb]: the k_hprescale pass, then the k_hbp grid with its
// XCD-ordered tiles (every tile must be visited exactly once).
int hemu_back(const ct_helix_desc *d, int vs, int vst, int nv, const float *r, float *x, long long *first)
{
    Emu e;
    if (setup(d, e)) return -1;
    const HelixDev &G = e.G;
    const size_t n = (size_t)nv * d->nr * d->nb;
    std::vector<float> rp(n);
    reset_oob();
    for (size_t el = 0; el < n; ++el) {
        const int k = (int)(el % (size_t)G.nb);
        const size_t vr = el / (size_t)G.nb;
        const int rr = (int)(vr % (size_t)G.nr), vi = (int)(vr / (size_t)G.nr);
        rp[el] = r[el] * hx_prescale(G, vs + vi * vst, rr, k);
    }
    const Ro<float> R{rp.data(), n};
    const int tiles_x = (G.nx + 7) >> 3, ntiles = tiles_x * ((G.ny + 7) >> 3);
    const int zblocks = (G.nz + 4 * HX_ZG - 1) / (4 * HX_ZG);
    std::vector<int> seen((size_t)ntiles, 0);
    for (int bid = 0; bid < ntiles; ++bid) {
        const int full = ntiles - ntiles % 8;
        const int tile = bid < full ? (bid % 8) * (full / 8) + bid / 8 : bid;
        if (tile < 0 || tile >= ntiles || seen[(size_t)tile]++) {
            g_err = "back-projection tile order is not a permutation";
            return -1;
        }
        const int tx = tile % tiles_x, ty = tile / tiles_x;
        for (int by = 0; by < zblocks; ++by)
            for (int tid = 0; tid < 256; ++tid) {
                const int lane = tid & 63, wave = tid >> 6;
                const int j = tx * 8 + (lane & 7), i = ty * 8 + (lane >> 3);
                const int kz0 = (by * 4 + wave) * HX_ZG;
                if (i >= G.ny || j >= G.nx || kz0 >= G.nz) continue;
                float acc[HX_ZG];
                for (int b = 0; b < HX_ZG; ++b) acc[b] = 0.f;
                hbp_lane(G, R, vs, vst, nv, i, j, kz0, acc);
                for (int b = 0; b < HX_ZG; ++b) {
                    const int kz = kz0 + b;
                    if (kz >= G.nz) break;
                    x[((size_t)kz * G.ny + i) * G.nx + j] = acc[b];
                }
            }
    }
    *first = hx_oob_index();
    return hx_oob_count();
}

// Regularizer gradient and curvature at every voxel (the k_hupd stencil).
int hemu_reg(int nx, int ny, int nz, const float *x, int potential, double delta, double beta, int huber, float *gr,
             float *dr, long long *first)
{
    HelixUpdate U;
    U.nx = nx;
    U.ny = ny;
    U.nz = nz;
    U.alpha = 1.f;
    U.potential = potential;
    U.huber = huber;
    U.delta = (float)delta;
    U.idelta = 1.f / U.delta;
    U.beta = (float)beta;
    const size_t nvox = (size_t)nx * ny * nz;
    reset_oob();
    for (int kz = 0; kz < nz; ++kz)
        for (int i = 0; i < ny; ++i)
            for (int j = 0; j < nx; ++j) {
                const size_t idx = ((size_t)kz * ny + i) * nx + j;
                reg26(U, Ro<float>{x, nvox}, kz, i, j, x[idx], gr[idx], dr[idx]);
            }
    *first = hx_oob_index();
    return hx_oob_count();
}

}  // extern "C"
