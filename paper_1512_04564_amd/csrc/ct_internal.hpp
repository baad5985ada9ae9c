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
//   sgn[v] = +1 if U_k increases with k along the lines of view v, -1 if it decreases.
constexpr int kBpTile = 16;   // back-projection tile edge (pixels)

struct GeomDev {
    int nx, ny, nb, nviews;
    int arc;
    int poly;     // the back-projector may estimate edge bins by a quadratic along the line (see ct_geom.cpp)
    float dso;
    float c_kf;   // dsd / du
    float k0;     // nb/2 - u_offset
    const float2 *bnd;
    const float *scale;
    const float4 *inv;
    const int *rowsweep;
    const float *sgn;
    // bin window [x, y] of every (view, 16 x 16 tile) pair of the fused back-projection, at
    // win[view * tiles + tile] (tiles in row-major order), filled when the geometry is created; nullptr
    // where the table would exceed its size limit (the kernel then computes each window itself)
    const int2 *win;
};

struct Workspace {
    size_t npix = 0;
    float *xa = nullptr, *xb = nullptr;     // ping-pong images
    float *xta = nullptr, *xtb = nullptr;   // transposed projector copies [nx][ny] (storage type)
    void *xca = nullptr, *xcb = nullptr;    // projector copies [ny][nx] of 16-bit storage (else unused)
    float *r = nullptr;                     // residual block, [max views per launch][nb] (float32 capacity)
    size_t r_cap = 0;                       // floats
    float *rho = nullptr;                   // rho table
    size_t rho_cap = 0;
    int *tbase = nullptr;                   // device subiteration base counter (graph replays)
    double *red = nullptr;                  // reduction scratch (trace / finiteness)
    size_t red_cap = 0;
    float *dl = nullptr, *kappa = nullptr, *gv = nullptr, *h = nullptr;  // solve-owned state
    float *tmp = nullptr;                   // scratch image
};

// Cached executable graphs of a solve's subiterations, per kind (0: one iteration, doubled for an odd subset
// count; 1: a run of such graphs as one, for untraced solves) and per ping-pong parity of the image buffers.
struct GraphKey {
    const void *y, *w, *dl, *kappa, *gv, *h, *rho, *r;
    int t0mod, parity, len;
    ct_rlalm_params p;
};

struct GraphCache {
    bool valid[2][2] = {{false, false}, {false, false}};
    GraphKey key[2][2]{};
    hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
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
    float *sgn = nullptr;   // per view boundary order (+1 increasing, -1 decreasing)
    int2 *win = nullptr;    // the fused back-projection's per (view, tile) bin windows (GeomDev::win)
    ct::GeomDev dev{};
    ct::Workspace ws;
    ct::GraphCache graphs;
    ct_kernel_times ktimes{};
    bool ktimes_valid = false;
    // Untraced solves end without waiting for the device: the final finiteness reduction is copied to
    // pinned host memory and an event recorded after the copy (ct_rlalm_status waits for it).
    double *status_host = nullptr;
    hipEvent_t status_ev = nullptr;
    bool status_pending = false;   // an untraced solve has recorded status_ev
    // rho table staging: pinned host buffer, the event after its last upload, and the table the device
    // holds (empty: unknown), so that an unchanged table is not uploaded again.
    float *rho_host = nullptr;
    size_t rho_host_cap = 0;
    hipEvent_t rho_ev = nullptr;
    std::vector<float> rho_on_device;
};

namespace ct {

// Host tables of the fan-beam projector (FP64 geometry, stored FP32; cs in FP64): the device tables of
// GeomDev before upload.
struct GeomTables {
    std::vector<float2> bnd;
    std::vector<double2> bnd64;   // the same boundary coefficients in FP64 (the helical projector's table)
    std::vector<float> scale;
    std::vector<float4> inv;
    std::vector<double2> cs;
    std::vector<float> sgn;
    std::vector<int> rowsweep;
    float c_kf = 0.f, k0 = 0.f;
    int poly = 0;
};
ct_status geometry_tables(const ct_geom_desc &d, GeomTables &t);
// Argument check of solver parameters; rho_k of eq. dec_rho (FP64; rho_fixed in fixed mode).
ct_status check_params(const ct_rlalm_params *p);
double rho_value(long long k, const ct_rlalm_params *p);
ct_status build_geometry(ct_geom *g);
void free_geometry(ct_geom *g);
ct_status ensure_workspace(ct_geom *g, size_t r_views, size_t rho_len);
void free_workspace(ct_geom *g);

// subset order m(t mod M)
std::vector<int> subset_order(int M, int kind);

// ---- kernel launchers (ct_kernels.hip) ----
// Storage types: sinogram inputs y, w, the residual block r and the forward projector's image copy are
// stored as ct_dtype (float32, float16 or bfloat16); accumulation and the image state x, g, h are float32.
enum FpEpilogue { FP_PLAIN = 0, FP_RESIDUAL = 1, FP_WEIGHTED = 2 };

// One forward projection: views v = vstart + vi * vstride, vi in [0, nv), of the image img (row-sweep
// views) / its transpose imgT (column-sweep views). Epilogues: PLAIN out = A x (float32); RESIDUAL
// out = mscale * w (A x - y) * scale (storage type; multiplied by the bin scale for the back-projector's
// solver modes); WEIGHTED out = w * A 1 (float32, ones image).
struct FpLaunch {
    GeomDev G;
    const void *img = nullptr, *imgT = nullptr;
    const void *y = nullptr, *w = nullptr;
    void *out = nullptr;
    // Residual epilogue with the block's lines split over two workgroups (see forward_split): the first
    // half of the lines writes M w (p_1 - y) s to out, the second half M w p_2 s to out2 (float32).
    void *out2 = nullptr;
    int vstart = 0, vstride = 1, nv = 0;
    float mscale = 1.f;
};

enum BpMode { BP_BACK = 0, BP_INIT = 1, BP_FULL = 2, BP_XSTEP = 3 };

struct UpdateArgs {
    const float *x = nullptr;      // current x^(t+1) (input of the projection just done), float32
    float *x_next = nullptr;       // x-step output, float32
    void *xc_next = nullptr;       // its forward-projector copy (storage type; unused for float32)
    void *xT_next = nullptr;       // its transposed copy (storage type)
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
    float idelta = 1e4f;           // 1 / delta, rounded once on the host
    float beta_ax = 1024.f, beta_dg = 1024.f / 1.41421356f;
    int huber = 1;
};

// One back-projection (BP_BACK: out_back = A' r, r float32 or storage type) or fused back-projection
// and relaxed update (the other modes, whose r is the RESIDUAL epilogue's, already multiplied by the bin
// scale) over views vstart + vi * vstride, vi in [0, nv).
struct BpLaunch {
    GeomDev G;
    const void *r = nullptr;
    const void *r2 = nullptr;   // second residual plane of a split forward projection (float32), added to r
    int vstart = 0, vstride = 1, nv = 0;
    float *out_back = nullptr;
    UpdateArgs U;
};

// One slice of a batched solve: everything a batched launch needs to address the slice. The images
// ping-pong between index 0 and 1; the forward projector reads xc / xt (xc == x for float32 storage).
struct SliceDev {
    GeomDev G;
    int M = 1, nvm = 0;
    const void *y = nullptr, *w = nullptr;
    void *r = nullptr;
    void *r2 = nullptr;   // second residual plane when the slice's forward projection is split
    float *x[2] = {nullptr, nullptr};
    void *xc[2] = {nullptr, nullptr};
    void *xt[2] = {nullptr, nullptr};
    float *gv = nullptr, *h = nullptr;
    const float *dl = nullptr, *kappa = nullptr;
    int fp_begin = 0, fp_end = 0;   // workgroup range of the slice in a batched forward grid
    int bp_begin = 0, bp_end = 0;   // ... and in a batched update grid
};

// Scalars shared by every slice of a batched update launch.
struct BatchUpdate {
    const float *rho = nullptr;
    const int *tbase = nullptr;
    long long tofs = 0;
    float alpha = 1.999f;
    int algorithm = 1, potential = 0, huber = 1;
    float delta = 1e-4f, idelta = 1e4f, beta_ax = 1024.f, beta_dg = 1024.f / 1.41421356f;
};

// dtype: ct_dtype of the storage-typed operands (y, w, residual, image copies).
hipError_t launch_forward(const FpLaunch &a, int ones, int epi, int dtype, hipStream_t s);
hipError_t launch_back_update(const BpLaunch &a, int mode, int rtype, int ctype, hipStream_t s);
// The bin windows of the fused back-projection's tiles for every view of G into out (G.nviews x tiles
// entries), by the function the kernel would evaluate; tile_windows_count gives the number of entries.
size_t tile_windows_count(const GeomDev &G);
hipError_t launch_tile_windows(const GeomDev &G, int2 *out, hipStream_t s);
// Batched subiteration kernels over slices [0, ns) of the device table tab: the forward projection of
// subset m (views m + vi * M) from image buffer par with the residual epilogue, and the fused
// back-projection / relaxed update reading buffer par and writing buffer par ^ 1. nwg_*: grid sizes
// (tab[ns - 1].fp_end, bp_end). fp_waves selects the forward workgroup shape (8 or 16 waves).
hipError_t launch_forward_batch(const SliceDev *tab, int ns, int nwg_fp, int m, int par, int dtype, int fp_waves,
                                hipStream_t s);
hipError_t launch_update_batch(const SliceDev *tab, int ns, int nwg_bp, int m, int par, const BatchUpdate &u,
                               int dtype, hipStream_t s);
// The whole batched iteration as one persistent launch of `blocks` workgroups (at most the resident
// capacity: persistent_blocks_per_cu per CU), subiterations t0 .. t0 + nsub - 1 with subsets order[t % M],
// images from buffer par0; state: the 4-int barrier state (zeroed by the launch sequence; state[3] != 0
// afterwards when a barrier wait gave up).
hipError_t launch_batch_persistent(const SliceDev *tab, int ns, int nwg_fp, int nwg_bp, const int *order, int M,
                                   long long t0, long long nsub, int par0, const BatchUpdate &u, int *state,
                                   int blocks, int dtype, hipStream_t s);
int persistent_blocks_per_cu(int dtype);
int forward_workgroups(const GeomDev &G, int nv, int fp_waves, bool split);   // per-launch workgroup count
// Whether the residual projection of nv views (of nviews) splits each block's lines over two workgroups:
// it can (float32, both planes fit the residual block) and its launch alone would underfill the device.
bool forward_split(const GeomDev &G, int nv, int nviews, int dtype);
bool split_eligible(const GeomDev &G, int nv, int nviews, int dtype);
bool launch_underfills(int forward_wgs);   // fewer than two workgroups per CU
int update_workgroups(const GeomDev &G);

hipError_t launch_transpose(const float *x, float *xT, int nx, int ny, hipStream_t s);
// FBP-like image of sinogram y into x (flat detector); q is an [nviews][nb] scratch sinogram.
hipError_t launch_fbp(const ct_geom *g, const void *y, int ytype, float *q, const double2 *cs, float *x, hipStream_t s);
// out = max(in, 0) (or 0), float32; outc (if non-NULL) and outT: its copy and transpose in ctype.
hipError_t launch_clip_copy(const float *in, float *out, void *outc, void *outT, int nx, int ny, int zero, int ctype,
                            hipStream_t s);
hipError_t launch_scale(float *x, size_t n, float a, hipStream_t s);
hipError_t launch_fill(float *x, size_t n, float a, hipStream_t s);
hipError_t launch_kappa(const float *bw, const float *b1, float *kappa, size_t n, hipStream_t s);
// dst = (float) src for n elements of ctype src
hipError_t launch_to_float(const void *src, int ctype, float *dst, size_t n, hipStream_t s);
hipError_t launch_add_counter(int *c, int add, hipStream_t s);
hipError_t launch_set_counter(int *c, int value, hipStream_t s);
// Learned start (ct_unet.hip): x = mu_water * max(network(FBP(y) / mu_water), 0).
ct_status unet_input(ct_geom *g, const void *y, double factor, float *x_in, hipStream_t s);
ct_status learned_start(ct_geom *g, const ct_unet *u, const void *y, double mu_water, float *x, float *a, float *b,
                        hipStream_t s);
// FP64 reductions (ct_reduce.hip) into the handle's reduction buffer Workspace::red: the trace region at
// kRedTrace, the cost region at kRedCost, kRedSize doubles in all.
constexpr int kTraceOut = 4;
constexpr int kCostOut = 3;
constexpr size_t kRedTrace = 0, kRedCost = 1152, kRedSize = 2048;
// out[0] = sum over the pixels within radius (all when radius <= 0) of (x - ref)^2, out[1] = their count,
// out[2] = number of pixels where x, g or h is not finite, out[3] = sum over all pixels of (x - ref)^2 (ref may be
// NULL: then only out[2] is meaningful). out is followed by 4 * 256 doubles of scratch.
hipError_t launch_trace_reduce(const float *x, const float *ref, const float *gv, const float *h, int nx, int ny,
                               float dx, float dy, float radius, double *out, hipStream_t s);
// out[0] = 1/2 sum w (p - y)^2 over nsino samples (p float32, y and w in dtype), out[1] = R(x) (four directions,
// kappa_j kappa_n per pair when kappa != NULL), out[2] = out[0] + out[1]; followed by 2 * 256 doubles of scratch.
hipError_t launch_cost_reduce(const float *p, const void *y, const void *w, int dtype, size_t nsino, const float *x,
                              const float *kappa, int nx, int ny, int kind, double delta, double beta, double *out,
                              hipStream_t s);

}  // namespace ct
