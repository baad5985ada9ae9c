/*
 * ct.h -- C ABI of libctrlalm: relaxed OS-LALM (OS-RLALM) for 2-D fan-beam PWLS X-ray CT on AMD gfx950.
 *
 * The library solves the penalized weighted-least-squares problem of Nien & Fessler, "Relaxed linearized
 * algorithms for faster X-ray CT image reconstruction" (Section III, eq. ct_problem):
 *
 *     x_hat = argmin_{x in Omega}  1/2 || y - A x ||_W^2 + R(x),       Omega = { x >= 0 }
 *
 * with the edge-preserving regularizer of eq. def_reg (four directions, eight neighbours), by
 * Algorithm 1 ("proposed (over-)relaxed OS-LALM", Section III-A) with the alpha-dependent continuation
 * rho_k(alpha) of eq. dec_rho (Section III-B). A is a matched distance-driven fan-beam projector (the
 * paper cites but does not define its projector); A' is its exact transpose up to summation order.
 *
 * Conventions shared by every entry point:
 *   - Images are float32, [ny][nx] row-major. Pixel (i, j) is centred at
 *     x_j = (j - (nx-1)/2) dx, y_i = (i - (ny-1)/2) dy  (mm); values are attenuation in mm^-1.
 *   - Sinograms are [view][bin], acquisition order. View v has angle beta0 + span * v / nviews, the
 *     source sits at -dso (cos b, sin b); bin k spans detector coordinates
 *     [(k - nb/2 + u_offset) du, (k + 1 - nb/2 + u_offset) du] along (-sin b, cos b).
 *   - Subset m of M is the interleaved view set { v : v mod M == m } (nviews % M == 0 is required);
 *     its sinogram block is [nviews/M][nb] in ascending view order. subset = -1 means all views.
 *   - Every data pointer is a DEVICE pointer owned by the caller (e.g. a torch tensor's data_ptr()).
 *     `stream` is a hipStream_t (NULL = the null stream). Calls are stream-ordered and asynchronous
 *     unless stated otherwise.
 *   - Every call returns a ct_status; no exception crosses the ABI. On an argument error nothing is
 *     launched and outputs are untouched. ct_last_error() returns a thread-local message for the last
 *     non-OK status.
 */
#ifndef CTRLALM_CT_H
#define CTRLALM_CT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CT_OK = 0,
    CT_ERR_INVALID_ARG = 1,
    CT_ERR_OOM = 2,
    CT_ERR_HIP = 3,
    CT_ERR_UNSUPPORTED = 4,
    CT_ERR_DIVERGED = 5
} ct_status;

typedef enum { CT_DET_FLAT = 0, CT_DET_ARC = 1 } ct_detector;

/*
 * Storage type of the solver's sinogram inputs y and w, of its residual block M w (A_m x - y) and of the
 * image copies its forward projector reads. Sums are float32 in every mode, and the image state x, g, h
 * and D_L stay float32; 16-bit values are rounded to nearest even on store. CT_BF16 keeps float32's
 * range. CT_F16 overflows above 65504: w and the residual must stay below that; scaling w and beta by
 * the same power of two leaves every iterate unchanged (the x-step's numerator and denominator both
 * scale), which is how a caller brings large count-based weights into range.
 */
typedef enum { CT_F32 = 0, CT_F16 = 1, CT_BF16 = 2 } ct_dtype;

typedef struct {
    int nx, ny;          /* image size (pixels), each in [1, 4096]                                  */
    double dx, dy;       /* pixel size (mm), > 0                                                     */
    int nb;              /* detector bins, in [1, 8192]                                              */
    double du;           /* bin width at the detector (mm), > 0                                      */
    double u_offset;     /* detector offset in bins (0 = centred)                                    */
    int det;             /* ct_detector: flat, or arc centred on the source                          */
    int nviews;          /* projection views, >= 1                                                   */
    double beta0, span;  /* first view angle and angular span (rad); views at beta0 + span v / nviews */
    double dso, dsd;     /* source-isocentre and source-detector distances (mm), dsd > dso > 0      */
    int nsubsets;        /* M >= 1, nviews % M == 0                                                  */
    int storage;         /* ct_dtype: solver storage of y, w, residual and projector image copies    */
} ct_geom_desc;

typedef struct ct_geom ct_geom; /* opaque: device geometry tables + solver workspace */

/*
 * Build the per-view geometry tables (FP64 on the host, stored FP32 on the current device) and the
 * subset tables, and the back-projection's bin window of every (view, 16 x 16 pixel tile) pair
 * (8 bytes each: 7.9 MB for 512^2 pixels and 984 views; not built past 256 MiB, where the kernel derives
 * the windows itself). The handle owns them until ct_geom_destroy. The solver workspace inside the handle
 * is allocated on first use; solves on one handle must not overlap in time.
 * Errors: CT_ERR_INVALID_ARG for an inconsistent descriptor (sizes, distances, nviews % M), CT_ERR_OOM,
 * CT_ERR_HIP.
 */
ct_status ct_geom_create(const ct_geom_desc *desc, ct_geom **out);
void ct_geom_destroy(ct_geom *g);

/*
 * p = A_m x : distance-driven forward projection of the float32 image x ([ny][nx]) for subset m
 * (p is [nviews/M][nb]) or for all views when subset == -1 (p is [nviews][nb]). p is overwritten.
 * Projection is the operation inside the subset gradient of Algorithm 1 (Section III-A).
 */
ct_status ct_forward(const ct_geom *g, int subset, const float *x, float *p, void *stream);

/*
 * ct_forward for callers that cannot allocate device memory (code under stream or graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same result as ct_forward, bit for bit, but the
 * transposed image copy the projector reads lives in a fixed scratch array of the library on each GPU
 * (16 MiB: images of at most 4 Mi pixels; larger images are CT_ERR_INVALID_ARG, nothing launched) instead
 * of the handle's workspace. The call allocates nothing (no hipMalloc, no library allocation); the
 * geometry's device must be current. Every call on one GPU shares that GPU's array: calls that overlap in
 * time on one GPU (other streams, other threads) race on it and must be ordered by the caller.
 */
ct_status ct_forward_noalloc(const ct_geom *g, int subset, const float *x, float *p, void *stream);

/*
 * x = A_m' r : matched distance-driven back-projection (gather form, no atomics) of the float32
 * sinogram block r for subset m ([nviews/M][nb]) or all views (subset == -1, [nviews][nb]).
 * x ([ny][nx]) is overwritten.
 */
ct_status ct_back(const ct_geom *g, int subset, const float *r, float *x, void *stream);

/*
 * x = FBP-like image of the sinogram y ([nviews][nb], storage type), [ny][nx] float32, overwritten: per view a
 * cosine pre-weight on the detector magnified to the isocentre, the spatial Ram-Lak filter, then
 * pixel-driven back-projection with linear interpolation and the fan weight (dso / L)^2, clipped at zero.
 * Algorithm 1 starts from an FBP image; this is its plain, unwindowed form. Flat detector only
 * (CT_ERR_UNSUPPORTED otherwise). Uses the handle's workspace: do not overlap with a solve on the handle.
 */
ct_status ct_fbp(const ct_geom *g, const void *y, float *x, void *stream);

/* Warm-start network (ct_unet.h). */
typedef struct ct_unet ct_unet;

/* Subset processing order (the paper leaves it open). */
typedef enum { CT_ORDER_SEQUENTIAL = 0, CT_ORDER_BITREV = 1 } ct_subset_order;

typedef struct {
    double alpha;        /* relaxation, 1 <= alpha < 2; alpha = 1 is unrelaxed OS-LALM              */
    int niters;          /* outer iterations; each is M subiterations (one full projection pair)     */
    int rho_mode;        /* 0: continuation rho_k(alpha) with k the subiteration count, 1: fixed    */
    double rho_fixed;    /* rho when rho_mode == 1, > 0                                              */
    int potential;       /* 0: hyperbola d^2 (sqrt(1 + (t/d)^2) - 1), 1: Fair d^2 (|t/d| - log(1+|t/d|)),
                            2: q-GGMRF (p = 2, q = 1.2) t^2 / (2 (1 + |t/d|^0.8))                     */
    double delta, beta;  /* potential scale (mm^-1) and regularization strength; beta_i = beta/|s_i| */
    int huber;           /* 1: Huber curvature for D_R (the paper's choice), 0: maximum curvature   */
    int algorithm;       /* 1: Algorithm 1 (proposed relaxation), 2: Algorithm 2 (simple relaxation) */
    int subset_order;    /* ct_subset_order                                                          */
    int kappa;           /* 0: kappa = 1; 1: certainty weights kappa_j = sqrt(A'w / A'1)             */
    int start;           /* 0: x holds x0 on entry; 1: zero image; 2: FBP-like image (ct_fbp);
                            3: learned start mu_water * max(unet(FBP(y) / mu_water), 0)              */
    int init_full;       /* 0: initial gradient from the last subset (Algorithm 1 as written);
                            1: full gradient                                                         */
    double dl_scale;     /* multiplies D_L (1 = the majorizer diag{A'WA1})                            */
    const float *x_ref;  /* optional device reference image for the trace (NULL = none)              */
    double mu_water;     /* HU scale of the trace: HU = 1000 mu / mu_water (air = 0)                  */
    double fov_radius;   /* trace RMSD region: pixel centres within this radius (mm); <= 0: image    */
    int use_graph;       /* 1: replay one captured hipGraph per iteration; 0: plain launches          */
    int time_kernels;    /* 1 (ct_rlalm_solve only): after the solve, replay the last subiteration's
                            projection kernel and update kernel 50 times each, back to back between
                            one hipEvent pair per kernel (the result is already in x; only solve-owned
                            workspace is rewritten); read with ct_rlalm_kernel_times                  */
    const ct_unet *unet; /* network of start == 3 (its max sizes must cover the image; ny, nx
                            multiples of 8); NULL otherwise                                           */
    int forward_split;   /* at least two subsets: split each forward block's lines over two workgroups,
                            whose two float32 residual planes (in every storage mode) the update adds
                            (-1: when the launch would hold fewer than two workgroups per CU, counting
                            all slices of a batched launch; 0: never; 1: always). The same setting gives
                            the same bits in single and batched solves; other values are
                            CT_ERR_INVALID_ARG                                                        */
    double diverge_factor; /* traced solves: the cost Psi of a traced iteration counts as grown when it
                            exceeds diverge_factor times the lowest Psi traced so far (> 1)           */
    int diverge_window;  /* traced solves: CT_ERR_DIVERGED after this many consecutive grown rows
                            (0: cost growth is never an error; non-finite values still are)          */
} ct_rlalm_params;

/* Fill p with the defaults: alpha 1.999, 20 iterations, continuation, hyperbola delta 1e-4 beta 1024,
   Huber curvature, Algorithm 1, sequential order, kappa off, start 0, last-subset init, D_L scale 1,
   no trace reference, mu_water 0.02, whole image, graph on, forward split -1, divergence when the
   traced cost stays above twice its lowest value for 3 traced iterations in a row. */
void ct_rlalm_params_default(ct_rlalm_params *p);

typedef struct {
    int iter;            /* outer iteration count after which the row was taken                      */
    double seconds;      /* host wall time since the solve call started (synchronised)               */
    double rmsd_hu;      /* RMSD to x_ref in HU over the trace region (FP64 reduction on the device;
                            NaN without x_ref)                                                       */
    double rho;          /* rho of the last subiteration of that iteration                           */
    int finite;          /* 1 when x, g and h were all finite                                        */
    double rmsd_hu_all;  /* RMSD to x_ref in HU over the whole image (NaN without x_ref)              */
    double cost;         /* Psi(x) = 1/2 ||y - A x||_W^2 + R(x) of the iterate, as ct_cost computes it */
} ct_trace_row;

/*
 * Whole solve (Algorithm 1 or 2): D_L = diag{A'WA1} (Section III-A), optional certainty weights,
 * initialisation on the last subset, then niters * M subiterations with rho_k(alpha).
 * y, w: [nviews][nb] in the geometry's storage type. x: float32 [ny][nx]; on entry x0 (start == 0),
 * on exit x^(niters).
 * trace == NULL: the call is asynchronous (stream-ordered; it does not wait for the device). The
 *   finiteness of the final x, g and h is reduced on the device; ct_rlalm_status reports it.
 * trace != NULL: niters rows; after every iteration the call waits for the device and takes the row
 *   (RMSDs, and the cost Psi by an all-view projection and FP64 reductions). It returns
 *   CT_ERR_DIVERGED when a row is not finite, or when the cost stays above diverge_factor times its
 *   lowest traced value for diverge_window consecutive rows; x then holds the last traced iterate that
 *   was finite, and the rows after the one that stopped the solve have iter == 0.
 */
ct_status ct_rlalm_solve(ct_geom *g, const ct_rlalm_params *p, const void *y, const void *w, float *x,
                         ct_trace_row *trace, void *stream);

/*
 * Waits for the last untraced ct_rlalm_solve made on this handle and returns CT_ERR_DIVERGED when its
 * final x, g or h held a non-finite value, CT_OK otherwise (also when no such solve was made).
 */
ct_status ct_rlalm_status(ct_geom *g);

/*
 * PWLS cost of eq. ct_problem (Section III): out[0] = 1/2 sum w (A x - y)^2 over all views, out[1] = R(x)
 * of eq. def_reg with p's potential, delta and beta (four directions, beta / ||s|| per direction; when
 * kappa != NULL each pair term also carries kappa_j kappa_n), out[2] = out[0] + out[1]. A x is the
 * float32 all-view projection; the sums and the potential are FP64 on the device, in a fixed order
 * (deterministic). x, kappa: float32 [ny][nx]; y, w: [nviews][nb] in the storage type; out: DEVICE
 * pointer to 3 doubles. Asynchronous; uses the handle's workspace (do not overlap with a solve on it).
 */
ct_status ct_cost(ct_geom *g, const ct_rlalm_params *p, const void *y, const void *w, const float *x,
                  const float *kappa, double *out, void *stream);

/*
 * Batched solve of n independent slices (2-D scans of possibly different sizes), the arithmetic per slice
 * that of ct_rlalm_solve (Algorithm 1 with rho_k(alpha)). Two launch forms:
 *   lockstep: at every subiteration one forward-projection launch and one fused update launch cover all
 *     slices (a 1-D grid whose workgroups look up their slice); each outer iteration is replayed from a
 *     captured hipGraph;
 *   persistent: one captured hipGraph holds every slice's initialisation and ONE persistent launch that
 *     runs all niters * M subiterations: its resident workgroups take the forward work items of every
 *     slice, then the update tiles, with a grid-wide barrier after each phase (every barrier wait is
 *     bounded; if the grid was not fully resident the call returns CT_ERR_HIP instead of hanging).
 *   g[i]: a distinct handle per slice; all share nsubsets (M) and storage. y[i], w[i]: that slice's
 *     sinograms in the storage type; x[i]: its float32 image (x0 on entry when p->start == 0, result
 *     on exit). p applies to every slice; trace and time_kernels are not available here (CT_ERR_UNSUPPORTED).
 *   autotune: 0 = lockstep with the default shape (16-wave projection workgroups, slices in the given
 *     order; with n == 1 the result equals ct_rlalm_solve bit for bit); 1 = time the candidates on this
 *     set of slice shapes -- lockstep with 8 or 16 waves per projection workgroup, each with the forward
 *     split never and always (when p->forward_split is -1), persistent with 1, 2 or 4 resident workgroups
 *     per CU, each with the slices in the given order or largest first -- and keep
 *     the fastest, cached per process and on disk (a text file per GPU architecture and shape set under
 *     $CTRLALM_TUNE_DIR, else $XDG_CACHE_HOME/ctrlalm/tune, else ~/.cache/ctrlalm/tune); 2 = persistent,
 *     its candidates (1, 2 or 4 workgroups per CU, either slice order) timed on this batch and the fastest
 *     kept (not cached). The slice order never changes a result; the forward workgroup's wave count changes
 *     the projection's summation order (the persistent form uses 8). Persistent launches pay two grid
 *     barriers per subiteration, each with an agent-scope release and acquire per workgroup (a write-back
 *     and an invalidation of its XCD's L2): on large batches lockstep is usually faster.
 *   chosen: if non-NULL, receives the launch shape used.
 * Waits for the device at the end. Returns CT_ERR_DIVERGED (message names the slice) if any slice ends
 * non-finite.
 */
typedef struct {
    int fp_waves;          /* waves per forward-projection workgroup (8 or 16)                       */
    int largest_first;     /* 1: slices ordered by decreasing work in the batched grids              */
    double ms_subiteration;/* timed cost of one batched subiteration (tuned shapes; else 0)           */
    int persistent;        /* 1: the persistent single-launch form                                   */
    int blocks_per_cu;     /* persistent form: resident workgroups per CU                            */
    int forward_split;     /* lockstep forward launch: -1 automatic, 0 never, 1 always split each     */
                           /* block's lines over two workgroups (a solve's own forward_split wins)     */
} ct_batch_config;
ct_status ct_rlalm_solve_batched(ct_geom *const *g, int n, const ct_rlalm_params *p, const void *const *y,
                                 const void *const *w, float *const *x, int autotune, ct_batch_config *chosen,
                                 void *stream);

/*
 * Low-level state interface (checkpoint / resume). The state after t subiterations is (x, g, h, t);
 * rho and the subset follow from t. dl and kappa are the solve constants.
 *
 * ct_rlalm_prepare: dl = dl_scale * A'(w .* A 1) over all views; kappa (if non-NULL and p->kappa)
 *   = sqrt(A'w / A'1). Both [ny][nx] float32, caller-owned.
 * ct_rlalm_init: x = max(x, 0); zeta = g = M grad L_{M-1}(x) (or the full gradient), h = D_L x - zeta
 *   (Algorithm 1) or h = zeta (Algorithm 2). This is the t = 0 state.
 * ct_rlalm_iterate: advance the state by nsub subiterations starting at subiteration t0.
 */
ct_status ct_rlalm_prepare(ct_geom *g, const ct_rlalm_params *p, const void *w, float *dl, float *kappa,
                           void *stream);
ct_status ct_rlalm_init(ct_geom *g, const ct_rlalm_params *p, const void *y, const void *w, const float *dl,
                        float *x, float *gv, float *h, void *stream);
ct_status ct_rlalm_iterate(ct_geom *g, const ct_rlalm_params *p, const void *y, const void *w, const float *dl,
                           const float *kappa, float *x, float *gv, float *h, long long t0, long long nsub,
                           void *stream);

/* Kernel timing of the last ct_rlalm_solve made with time_kernels = 1 on this handle: n_* back-to-back
   launches and their total event-measured duration (ms). The forward kernel is the subset projection
   with its residual epilogue; the update kernel is the fused back-projection / relaxed update.
   Returns CT_ERR_INVALID_ARG if no timed solve has been made. */
typedef struct {
    long long n_forward, n_update;
    double ms_forward, ms_update;
} ct_kernel_times;
ct_status ct_rlalm_kernel_times(const ct_geom *g, ct_kernel_times *out);

/* Thread-local message describing the last non-OK status of a call made on this thread. */
const char *ct_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CTRLALM_CT_H */
