/*
 * ct_helix.h -- C ABI of libctrlalm, 3-D part: helical cone-beam PWLS reconstruction by relaxed OS-LALM.
 *
 * The paper's own setting is 3-D helical CT (Section III: the regularizer of eq. def_reg over 13 directions,
 * i.e. all 26 neighbours of a voxel; Section IV: helical scans). The problem is that of ct.h,
 *     x_hat = argmin_{x >= 0} 1/2 || y - A x ||_W^2 + R(x),
 * now over a volume, with A a separable distance-driven helical cone-beam projector (the paper cites but does
 * not define its projector) and the solver of Algorithm 1 with rho_k(alpha) (eq. dec_rho).
 *
 * Scanner: view v at angle b = beta0 + 2 pi v / views_per_turn, source S = (-dso cos b, -dso sin b,
 * z0 + feed v / views_per_turn). A flat detector panel moves with the source at distance dsd along
 * d = (cos b, sin b, 0); its point at coordinates (u, w) is S + dsd d + u e + w z_hat, e = (-sin b, cos b, 0),
 * with bin boundaries u_k = (k - nb/2 + u_offset) du and row boundaries w_r = (r - nr/2 + w_offset) dw.
 *
 * Projector: each view sweeps voxel planes y = y_i (|sin b| >= |cos b|, decided in FP64) or x = x_j. In a
 * plane, voxel column q and bin k overlap by the fan-beam distance-driven footprint f_t (overlap of the
 * column with the bin's two boundary rays, over the footprint's width); row r and voxel kz of the column
 * overlap by f_a, the overlap of the voxel with the row's height interval at the column centre's depth,
 * over that interval's height. Weight = (plane spacing / |cos theta_k|) sqrt(1 + w_c^2 / (dsd^2 + u_c^2))
 * f_t f_a: the length of the cell's central ray between neighbouring planes, times both footprints.
 *
 * Layouts: volumes float32 [nz][ny][nx] (x fastest); voxel (kz, i, j) is centred at
 * ((j - (nx-1)/2) dx, (i - (ny-1)/2) dy, zc + (kz - (nz-1)/2) dz). Sinograms float32 [view][row][bin].
 * Subset m of M: views v with v mod M == m, block [nviews/M][nr][nb]. All data pointers are DEVICE
 * pointers owned by the caller; stream is a hipStream_t. Errors as in ct.h (ct_last_error()).
 */
#ifndef CTRLALM_CT_HELIX_H
#define CTRLALM_CT_HELIX_H

#include "ct.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny, nz;         /* voxels: nx, ny in [1, 4096], nz in [1, 2048]                             */
    double dx, dy, dz;      /* voxel size (mm), > 0                                                     */
    double zc;              /* z of the volume centre (mm)                                              */
    int nb;                 /* detector channels, in [1, 8192]                                          */
    double du, u_offset;    /* channel width at the detector (mm) > 0; offset in channels               */
    int nr;                 /* detector rows, in [1, 1024]                                              */
    double dw, w_offset;    /* row height at the detector (mm) > 0; offset in rows                      */
    int nviews;             /* views in all, >= 1                                                       */
    int views_per_turn;     /* views per 2 pi, >= 1                                                     */
    double beta0;           /* angle of view 0 (rad)                                                    */
    double z0, feed;        /* source height at view 0 (mm); table feed per turn (mm, signed)           */
    double dso, dsd;        /* source-isocentre and source-detector distances (mm), dsd > dso > 0      */
    int nsubsets;           /* M >= 1, nviews % M == 0                                                  */
} ct_helix_desc;

typedef struct ct_helix ct_helix;   /* opaque: device tables + solver workspace                           */

/* Builds the tables (FP64 on the host, FP32 on the current device). CT_ERR_INVALID_ARG for an
   inconsistent descriptor (sizes, distances, nviews % M, a volume reaching the source circle),
   CT_ERR_OOM, CT_ERR_HIP. */
ct_status ct_helix_create(const ct_helix_desc *desc, ct_helix **out);
void ct_helix_destroy(ct_helix *h);

/* p = A_m x (subset m, p is [nviews/M][nr][nb]) or A x (subset -1, p is [nviews][nr][nb]); p overwritten.
   Asynchronous. Uses the handle's workspace (a transposed copy of x): calls on one handle are ordered
   on their streams by the caller. */
ct_status ct_helix_forward(ct_helix *h, int subset, const float *x, float *p, void *stream);

/* x = A_m' r (gather form, no atomics), r as p above; x [nz][ny][nx] overwritten. Asynchronous. */
ct_status ct_helix_back(ct_helix *h, int subset, const float *r, float *x, void *stream);

/*
 * Whole solve by Algorithm 1 (eq. relaxed_lal_iter_quad with rho_k(alpha)): D_L = dl_scale A'(w .* A 1),
 * initialisation on the last subset of the order (or the full gradient), niters * M subiterations, with
 * the 26-neighbour regularizer of p->potential, delta, beta (beta / ||s|| per offset of length 1, sqrt 2,
 * sqrt 3) and its Huber curvature (or maximum curvature). y, w: [nviews][nr][nb] float32; x: x0 on entry
 * when p->start == 0 (p->start == 1: zero), x^(niters) on exit.
 * Supported: p->algorithm 1, p->kappa 0, p->start 0 or 1, no trace; other values are CT_ERR_UNSUPPORTED.
 * The call waits for the device at the end and returns CT_ERR_DIVERGED when x, g or h holds a non-finite
 * value (x then holds the last iterate).
 */
ct_status ct_helix_solve(ct_helix *h, const ct_rlalm_params *p, const float *y, const float *w, float *x,
                         void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CTRLALM_CT_HELIX_H */
