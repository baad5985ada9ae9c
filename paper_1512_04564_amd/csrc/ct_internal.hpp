// Internal declarations shared by the libctrlalm sources (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ct.h"

namespace ct {

// Thread-local last-error message (ct_last_error).
void set_error(const std::string &msg);
ct_status fail(ct_status st, const std::string &msg);

#define CT_HIP_CHECK(expr)                                                                         \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return ::ct::fail(CT_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

#define CT_TRY(expr)                                                                               \
    do {                                                                                           \
        ct_status s_ = (expr);                                                                     \
        if (s_ != CT_OK) return s_;                                                                \
    } while (0)

// Device view of the per-view geometry tables. All tables cover every view of the scan.
//   bnd[v*(nb+1) + k] = (A, B): boundary ray k of view v crosses image line l at
//       U = fmaf(lc, B, A),  lc = l - (NL-1)/2,
//   in pixel units along the line, centred so that pixel q spans [q - NQ/2, q + 1 - NQ/2].
//   Lines are image rows (NL = ny, NQ = nx) for row-sweep views and columns otherwise.
//   scale[v*nb + k] = line spacing / |cos theta|, theta the angle between the ray through the bin
//       centre and the line normal (mm per line).
//   inv[v] = (na, nl, da, dl): detector coordinate of the point at (along-line e, line lc), both in
//       the view's own pixel units, is u = dsd * (e na + lc nl) / (e da + lc dl + dso);
//       bin index kf = u / du + nb/2 - u_offset (arc: atan of the same ratio).
//   rowsweep[v] = 1 for row-sweep views.
constexpr int kBpTile = 16;   // back-projection tile edge (pixels)

struct GeomDev {
    int nx, ny, nb, nviews;
    int arc;
    float dso;
    float c_kf;   // dsd / du
    float k0;     // nb/2 - u_offset
    const float2 *bnd;
    const float *scale;
    const float4 *inv;
    const int *rowsweep;
};

struct Workspace {
    size_t npix = 0;
    float *xa = nullptr, *xb = nullptr;     // ping-pong images
    float *xta = nullptr, *xtb = nullptr;   // their transposes [nx][ny]
    float *r = nullptr;                     // residual block, [max views per launch][nb]
    size_t r_cap = 0;                       // floats
    float *rho = nullptr;                   // rho table
    size_t rho_cap = 0;
    int *tbase = nullptr;                   // device subiteration base counter (graph replays)
    double *red = nullptr;                  // reduction scratch (trace / finiteness)
    size_t red_cap = 0;
    float *dl = nullptr, *kappa = nullptr, *gv = nullptr, *h = nullptr;  // solve-owned state
    float *tmp = nullptr;                   // scratch image
};

// Cached executable graphs of one outer iteration, one per ping-pong parity of the image buffers.
struct GraphKey {
    const void *y, *w, *dl, *kappa, *gv, *h, *rho, *r;
    int t0mod, parity, len;
    ct_rlalm_params p;
};

struct GraphCache {
    bool valid[2] = {false, false};
    GraphKey key[2]{};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipStream_t cap = nullptr;
};

}  // namespace ct

struct ct_geom {
    ct_geom_desc desc;
    int device = 0;
    // host copies (FP64-derived)
    std::vector<int> rowsweep;
    // device tables
    float2 *bnd = nullptr;
    float *scale = nullptr;
    float4 *inv = nullptr;
    int *d_rowsweep = nullptr;
    double2 *cs = nullptr;  // per view (cos beta, sin beta) in FP64, for the FBP-like start
    ct::GeomDev dev{};
    ct::Workspace ws;
    ct::GraphCache graphs;
    ct_kernel_times ktimes{};
    bool ktimes_valid = false;
};

namespace ct {

ct_status build_geometry(ct_geom *g);
void free_geometry(ct_geom *g);
ct_status ensure_workspace(ct_geom *g, size_t r_views, size_t rho_len);
void free_workspace(ct_geom *g);

// subset order m(t mod M)
std::vector<int> subset_order(int M, int kind);

// ---- kernel launchers (ct_kernels.hip) ----
enum FpEpilogue { FP_PLAIN = 0, FP_RESIDUAL = 1, FP_WEIGHTED = 2 };
// Views v = vstart + vi * vstride for vi in [0, nv). img / imgT: image and its transpose (may be the same
// pointer semantics as documented in ct_kernels.hip). ones != 0 projects the all-ones image.
hipError_t launch_forward(const GeomDev &G, const float *img, const float *imgT, int ones, int vstart, int vstride,
                          int nv, int epi, const float *y, const float *w, float mscale, float *out, hipStream_t s);

enum BpMode { BP_BACK = 0, BP_INIT = 1, BP_FULL = 2, BP_DUAL = 3, BP_XSTEP = 4, BP_INIT_XSTEP = 5 };

struct UpdateArgs {
    const float *x = nullptr;      // current x^(t+1) (input of the projection just done)
    float *x_next = nullptr;       // x-step output
    float *xT_next = nullptr;      // its transpose
    float *gv = nullptr;
    float *h = nullptr;
    const float *dl = nullptr;
    const float *kappa = nullptr;  // nullptr: kappa = 1
    const float *rho = nullptr;    // rho table, indexed by t
    const int *tbase = nullptr;    // t = *tbase + tofs
    long long tofs = 0;
    float alpha = 1.999f;
    int algorithm = 1;
    int potential = 0;
    float delta = 1e-4f;
    float beta_ax = 1024.f, beta_dg = 1024.f / 1.41421356f;
    int huber = 1;
};

hipError_t launch_back_update(const GeomDev &G, int mode, const float *r, int vstart, int vstride, int nv,
                              float *out_back, const UpdateArgs &U, hipStream_t s);

hipError_t launch_transpose(const float *x, float *xT, int nx, int ny, hipStream_t s);
// FBP-like image of sinogram y into x (flat detector); q is an [nviews][nb] scratch sinogram.
hipError_t launch_fbp(const ct_geom *g, const float *y, float *q, const double2 *cs, float *x, hipStream_t s);
hipError_t launch_clip_copy(const float *in, float *out, float *outT, int nx, int ny, int zero, hipStream_t s);
hipError_t launch_scale(float *x, size_t n, float a, hipStream_t s);
hipError_t launch_fill(float *x, size_t n, float a, hipStream_t s);
hipError_t launch_kappa(const float *bw, const float *b1, float *kappa, size_t n, hipStream_t s);
hipError_t launch_add_counter(int *c, int add, hipStream_t s);
hipError_t launch_set_counter(int *c, int value, hipStream_t s);
// FP64 reduction: out[0] += sum over masked pixels of (x - ref)^2, out[1] += count, out[2] += nonfinite count
hipError_t launch_trace_reduce(const float *x, const float *ref, const float *gv, const float *h, int nx, int ny,
                               float dx, float dy, float radius, double *out, hipStream_t s);

}  // namespace ct
