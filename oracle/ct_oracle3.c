/*
 * FP64 CPU oracle for 3-D helical cone-beam PWLS reconstruction by relaxed OS-LALM.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the HIP path's 3-D solver is
 * checked against. Only the test suite and the benchmark's CPU leg may load it. It shares no code,
 * header, table or constant generator with the HIP library (nor with the 2-D oracle, whose conventions
 * it restates).
 *
 * Problem and method (Nien & Fessler, "Relaxed linearized algorithms for faster X-ray CT image
 * reconstruction"):
 *   - PWLS  min_{x>=0} 1/2 ||y - A x||_W^2 + R(x)                          (Section III, eq. ct_problem)
 *   - R(x) = sum_i beta_i sum_n phi([C_i x]_n) over 13 directions, i.e. all 26 neighbours of a voxel,
 *     the paper's 3-D setting (eq. def_reg and the text after it); beta_i = beta / ||s_i|| with the
 *     offset length in voxel units (1, sqrt 2, sqrt 3), kappa = 1
 *   - D_L = diag{A' W A 1}, Huber curvature D_R                            (Section III-A)
 *   - the relaxed OS-LALM iteration with rho_k(alpha)                       (Algorithm 1; eq. dec_rho)
 *
 * Scanner: a helical source S_v = (-dso cos b_v, -dso sin b_v, z0 + feed v / V) with b_v = beta0 + 2 pi v / V
 * (V views per turn) and a flat detector panel at distance dsd from the source, perpendicular to the
 * central direction d_v = (cos b_v, sin b_v, 0), moving with the source: the point at detector
 * coordinates (u, w) is S_v + dsd d_v + u e_v + w z_hat with e_v = (-sin b_v, cos b_v, 0). Bin boundaries
 * u_k = (k - nb/2 + u_offset) du, row boundaries w_l = (l - nr/2 + w_offset) dw.
 *
 * Projector (the paper cites but does not define its projector): separable distance-driven. A view
 * sweeps voxel planes y = y_i ("row sweep", |sin b| >= |cos b| - 1e-12 decided in FP64) or x = x_j;
 * within a plane, voxel column (line, q) and detector cell (row l, bin k) interact with weight
 *     a = s_k sec phi_{k,l} * f_t(k, q) * f_a(l, kappa)
 *   f_t = |[q, q+1] cap [b_k, b_{k+1}]| / |b_{k+1} - b_k|: b_k is where the plane meets the transaxial
 *         boundary ray of u_k (the 2-D fan-beam distance-driven footprint, in voxel units along the line)
 *   f_a = |[kappa, kappa+1] cap [z_l, z_{l+1}]| / (z_{l+1} - z_l): z_l is the height, in voxel units, at
 *         which the ray towards row boundary w_l passes the voxel column's centre depth
 *         ell = (c - S)·d_v (column centre c), i.e. S_z + w_l ell / dsd (the axial footprint uses the
 *         magnification at the column centre)
 *   s_k = plane spacing / |cos theta_k|, theta_k between the plane normal and the transaxial ray through
 *         the bin centre; sec phi_{k,l} = sqrt(1 + w_c^2 / (dsd^2 + u_c^2)) at the cell centre (u_c, w_c):
 *         s_k sec phi is the length of the cell's central ray between two neighbouring planes.
 * The forward projector merges sorted boundary lists (transaxial, then axial per column); the
 * brute-force evaluator below computes every weight from the definition on its own, for the tests.
 *
 * Layouts: volume [nz][ny][nx] (x fastest), voxel (kz, i, j) centred at ((j - (nx-1)/2) dx,
 * (i - (ny-1)/2) dy, zc + (kz - (nz-1)/2) dz); sinogram [view][row][bin].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define H3_PI 3.14159265358979323846

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz, zc;
    int nb;
    double du, u_offset;
    int nr;
    double dw, w_offset;
    int nviews, views_per_turn;
    double beta0, z0, feed;
    double dso, dsd;
} h3_geom;

typedef struct {
    double alpha;
    int niters, nsubsets;
    int rho_mode;
    double rho_fixed;
    int potential;
    double delta, beta;
    int huber;
    int algorithm;
    int init_full;
    double dl_scale;
    int subset_order;
    int kappa;   /* unused in 3-D (kappa = 1) */
} h3_params;

/* ------------------------------------------------------------------------------------------------ */
/* Geometry of one view                                                                              */
/* ------------------------------------------------------------------------------------------------ */

typedef struct {
    double c, s;          /* cos b, sin b */
    double sx, sy, sz;    /* source */
    int row_sweep;
    int nl, nq;           /* planes swept, voxel columns per plane line */
    double *px, *py;      /* transaxial detector boundary points, nb + 1 */
    double *scale;        /* s_k, nb */
    double *secphi;       /* [nr][nb] */
} h3_view;

static double u_bound(const h3_geom *g, double k) { return (k - 0.5 * g->nb + g->u_offset) * g->du; }
static double w_bound(const h3_geom *g, double l) { return (l - 0.5 * g->nr + g->w_offset) * g->dw; }

static void h3_view_init(const h3_geom *g, int v, h3_view *o)
{
    const double beta = g->beta0 + 2.0 * H3_PI * (double)v / (double)g->views_per_turn;
    o->c = cos(beta);
    o->s = sin(beta);
    o->sx = -g->dso * o->c;
    o->sy = -g->dso * o->s;
    o->sz = g->z0 + g->feed * (double)v / (double)g->views_per_turn;
    o->row_sweep = fabs(o->s) >= fabs(o->c) - 1e-12;
    o->nl = o->row_sweep ? g->ny : g->nx;
    o->nq = o->row_sweep ? g->nx : g->ny;
    o->px = (double *)malloc(sizeof(double) * (g->nb + 1));
    o->py = (double *)malloc(sizeof(double) * (g->nb + 1));
    o->scale = (double *)malloc(sizeof(double) * g->nb);
    o->secphi = (double *)malloc(sizeof(double) * g->nb * g->nr);
    const double off = g->dsd - g->dso;
    for (int k = 0; k <= g->nb; ++k) {
        const double u = u_bound(g, k);
        o->px[k] = off * o->c - u * o->s;
        o->py[k] = off * o->s + u * o->c;
    }
    for (int k = 0; k < g->nb; ++k) {
        const double uc = u_bound(g, k + 0.5);
        const double rx = off * o->c - uc * o->s - o->sx, ry = off * o->s + uc * o->c - o->sy;
        const double len = sqrt(rx * rx + ry * ry);
        o->scale[k] = o->row_sweep ? g->dy * len / fabs(ry) : g->dx * len / fabs(rx);
        for (int l = 0; l < g->nr; ++l) {
            const double wc = w_bound(g, l + 0.5);
            o->secphi[(size_t)l * g->nb + k] = sqrt(1.0 + wc * wc / (g->dsd * g->dsd + uc * uc));
        }
    }
}

static void h3_view_free(h3_view *o)
{
    free(o->px); free(o->py); free(o->scale); free(o->secphi);
}

/* Transaxial boundary positions b[k], k = 0..nb, on plane line l, in voxel units along the line. */
static void h3_line_bounds(const h3_geom *g, const h3_view *o, int l, double *b)
{
    if (o->row_sweep) {
        const double yl = ((double)l - 0.5 * (g->ny - 1)) * g->dy;
        for (int k = 0; k <= g->nb; ++k) {
            const double X = o->sx + (yl - o->sy) * (o->px[k] - o->sx) / (o->py[k] - o->sy);
            b[k] = X / g->dx + 0.5 * g->nx;
        }
    } else {
        const double xl = ((double)l - 0.5 * (g->nx - 1)) * g->dx;
        for (int k = 0; k <= g->nb; ++k) {
            const double Y = o->sy + (xl - o->sx) * (o->py[k] - o->sy) / (o->px[k] - o->sx);
            b[k] = Y / g->dy + 0.5 * g->ny;
        }
    }
}

/* Axial row boundaries z[l], l = 0..nr, in voxel units (voxel kz spans [kz, kz+1]) at column (i, j). */
static void h3_column_rows(const h3_geom *g, const h3_view *o, int i, int j, double *z)
{
    const double xc = ((double)j - 0.5 * (g->nx - 1)) * g->dx;
    const double yc = ((double)i - 0.5 * (g->ny - 1)) * g->dy;
    const double ell = (xc - o->sx) * o->c + (yc - o->sy) * o->s;
    const double zlo = g->zc - 0.5 * g->nz * g->dz;
    for (int l = 0; l <= g->nr; ++l) z[l] = (o->sz + w_bound(g, l) * ell / g->dsd - zlo) / g->dz;
}

/* Transaxial pairs of one line: (bin k, voxel column q, f_t * s_k) for every nonzero overlap, found by
   the sequential merge of the ascending bin intervals with the voxel edges 0..nq. Returns the count. */
static int h3_line_pairs(const h3_geom *g, const h3_view *o, const double *b, int *pk, int *pq, double *pw)
{
    const int nb = g->nb, nq = o->nq;
    const int inc = b[nb] > b[0];
    int n = 0, kk = 0;
#define BIN_OF(kk) (inc ? (kk) : nb - 1 - (kk))
#define LO_OF(kk) (inc ? b[(kk)] : b[nb - (kk)])
#define HI_OF(kk) (inc ? b[(kk) + 1] : b[nb - 1 - (kk)])
    while (kk < nb && HI_OF(kk) <= 0.0) ++kk;
    if (kk >= nb) return 0;
    int q = (int)floor(LO_OF(kk));
    if (q < 0) q = 0;
    while (kk < nb && q < nq) {
        const double lo = LO_OF(kk), hi = HI_OF(kk);
        const double a0 = lo > (double)q ? lo : (double)q;
        const double a1 = hi < (double)(q + 1) ? hi : (double)(q + 1);
        if (a1 > a0 && hi > lo) {
            const int k = BIN_OF(kk);
            pk[n] = k;
            pq[n] = q;
            pw[n] = o->scale[k] * (a1 - a0) / (hi - lo);
            ++n;
        }
        if (hi < (double)(q + 1)) ++kk; else ++q;
    }
#undef BIN_OF
#undef LO_OF
#undef HI_OF
    return n;
}

/* Axial pairs of one column: (row l, voxel kz, f_a) by the merge of the ascending row intervals z[l]
   with the voxel edges 0..nz. Returns the count. */
static int h3_column_pairs(const h3_geom *g, const double *z, int *pl, int *pz, double *pa)
{
    const int nr = g->nr, nz = g->nz;
    int n = 0, l = 0;
    while (l < nr && z[l + 1] <= 0.0) ++l;
    if (l >= nr) return 0;
    int kz = (int)floor(z[l]);
    if (kz < 0) kz = 0;
    while (l < nr && kz < nz) {
        const double lo = z[l], hi = z[l + 1];
        const double a0 = lo > (double)kz ? lo : (double)kz;
        const double a1 = hi < (double)(kz + 1) ? hi : (double)(kz + 1);
        if (a1 > a0) {
            pl[n] = l;
            pz[n] = kz;
            pa[n] = (a1 - a0) / (hi - lo);
            ++n;
        }
        if (hi < (double)(kz + 1)) ++l; else ++kz;
    }
    return n;
}

static inline size_t vox(const h3_geom *g, int kz, int i, int j) { return ((size_t)kz * g->ny + i) * g->nx + j; }

/* One view's contribution on one line: mode 0 forward (p[l][k] += a x), mode 1 back (x += a r[l][k]). */
static void h3_line(const h3_geom *g, const h3_view *o, int line, int mode, const double *x_in, double *p_out,
                    const double *r_in, double *x_out, double *b, int *pk, int *pq, double *pw, double *z, int *pl,
                    int *pz, double *pa)
{
    h3_line_bounds(g, o, line, b);
    const int nt = h3_line_pairs(g, o, b, pk, pq, pw);
    for (int t = 0; t < nt; ++t) {
        const int k = pk[t], q = pq[t];
        const int i = o->row_sweep ? line : q, j = o->row_sweep ? q : line;
        h3_column_rows(g, o, i, j, z);
        const int na = h3_column_pairs(g, z, pl, pz, pa);
        for (int a = 0; a < na; ++a) {
            const size_t cell = (size_t)pl[a] * g->nb + k;
            const double wgt = pw[t] * o->secphi[cell] * pa[a];
            const size_t vi = vox(g, pz[a], i, j);
            if (mode == 0) p_out[cell] += wgt * x_in[vi];
            else x_out[vi] += wgt * r_in[cell];
        }
    }
}

typedef struct {
    double *b, *pw, *z, *pa;
    int *pk, *pq, *pl, *pz;
} h3_scratch;

static void scratch_init(const h3_geom *g, h3_scratch *s)
{
    const int npair = 2 * (g->nb + (g->nx > g->ny ? g->nx : g->ny)) + 4;
    const int nax = 2 * (g->nr + g->nz) + 4;
    s->b = (double *)malloc(sizeof(double) * (g->nb + 1));
    s->pw = (double *)malloc(sizeof(double) * npair);
    s->pk = (int *)malloc(sizeof(int) * npair);
    s->pq = (int *)malloc(sizeof(int) * npair);
    s->z = (double *)malloc(sizeof(double) * (g->nr + 1));
    s->pa = (double *)malloc(sizeof(double) * nax);
    s->pl = (int *)malloc(sizeof(int) * nax);
    s->pz = (int *)malloc(sizeof(int) * nax);
}

static void scratch_free(h3_scratch *s)
{
    free(s->b); free(s->pw); free(s->pk); free(s->pq); free(s->z); free(s->pa); free(s->pl); free(s->pz);
}

/* p[iv][nr][nb] = (A x) for views[iv]. */
void h3_forward(const h3_geom *g, const int *views, int nv, const double *x, double *p)
{
    const size_t cells = (size_t)g->nr * g->nb;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int iv = 0; iv < nv; ++iv) {
        h3_view o;
        h3_view_init(g, views[iv], &o);
        h3_scratch s;
        scratch_init(g, &s);
        double *pv = p + (size_t)iv * cells;
        memset(pv, 0, sizeof(double) * cells);
        for (int line = 0; line < o.nl; ++line)
            h3_line(g, &o, line, 0, x, pv, NULL, NULL, s.b, s.pk, s.pq, s.pw, s.z, s.pl, s.pz, s.pa);
        scratch_free(&s);
        h3_view_free(&o);
    }
}

/* x = A' r over views[iv] (x overwritten); r is [nv][nr][nb]. Row-sweep views run in parallel over planes
   y = y_i, column-sweep views over planes x = x_j: a line writes only its own voxels. */
void h3_back(const h3_geom *g, const int *views, int nv, const double *r, double *x)
{
    const size_t nvox = (size_t)g->nx * g->ny * g->nz, cells = (size_t)g->nr * g->nb;
    memset(x, 0, sizeof(double) * nvox);
    h3_view *os = (h3_view *)malloc(sizeof(h3_view) * (nv > 0 ? nv : 1));
    for (int iv = 0; iv < nv; ++iv) h3_view_init(g, views[iv], &os[iv]);
    for (int pass = 0; pass < 2; ++pass) {
        const int nl = pass == 0 ? g->ny : g->nx;
        #pragma omp parallel for schedule(dynamic, 1)
        for (int line = 0; line < nl; ++line) {
            h3_scratch s;
            scratch_init(g, &s);
            for (int iv = 0; iv < nv; ++iv) {
                if (os[iv].row_sweep != (pass == 0)) continue;
                h3_line(g, &os[iv], line, 1, NULL, NULL, r + (size_t)iv * cells, x, s.b, s.pk, s.pq, s.pw, s.z,
                        s.pl, s.pz, s.pa);
            }
            scratch_free(&s);
        }
    }
    for (int iv = 0; iv < nv; ++iv) h3_view_free(&os[iv]);
    free(os);
}

/*
 * Brute force, for the tests: every weight of view v as a dense [nr*nb][nz*ny*nx] matrix, each entry
 * evaluated from the definition on its own (the ray-plane crossing by its ray parameter, interval
 * overlaps by min / max), without the merges.
 */
void h3_weights_dense(const h3_geom *g, int v, double *out)
{
    const double beta = g->beta0 + 2.0 * H3_PI * (double)v / (double)g->views_per_turn;
    const double c = cos(beta), s = sin(beta);
    const double S[3] = {-g->dso * c, -g->dso * s, g->z0 + g->feed * (double)v / (double)g->views_per_turn};
    const int row = fabs(s) >= fabs(c) - 1e-12;
    const double zlo = g->zc - 0.5 * g->nz * g->dz;
    const size_t nvox = (size_t)g->nx * g->ny * g->nz;
    for (int l = 0; l < g->nr; ++l)
        for (int k = 0; k < g->nb; ++k) {
            double *rowp = out + ((size_t)l * g->nb + k) * nvox;
            /* central ray of the cell */
            const double uc = u_bound(g, k + 0.5), wc = w_bound(g, l + 0.5);
            const double C[3] = {S[0] + g->dsd * c - uc * s, S[1] + g->dsd * s + uc * c, S[2] + wc};
            const double R[3] = {C[0] - S[0], C[1] - S[1], C[2] - S[2]};
            const double rlen = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
            /* length of the central ray between two neighbouring planes */
            const double seg = row ? g->dy * rlen / fabs(R[1]) : g->dx * rlen / fabs(R[0]);
            for (int kz = 0; kz < g->nz; ++kz)
                for (int i = 0; i < g->ny; ++i)
                    for (int j = 0; j < g->nx; ++j) {
                        const double xc = ((double)j - 0.5 * (g->nx - 1)) * g->dx;
                        const double yc = ((double)i - 0.5 * (g->ny - 1)) * g->dy;
                        /* transaxial: the two boundary rays of bin k crossing the voxel's plane */
                        double bb[2];
                        for (int e = 0; e < 2; ++e) {
                            const double u = u_bound(g, k + e);
                            const double P[2] = {S[0] + g->dsd * c - u * s, S[1] + g->dsd * s + u * c};
                            if (row) {
                                const double t = (yc - S[1]) / (P[1] - S[1]);
                                bb[e] = (S[0] + t * (P[0] - S[0])) / g->dx + 0.5 * g->nx;
                            } else {
                                const double t = (xc - S[0]) / (P[0] - S[0]);
                                bb[e] = (S[1] + t * (P[1] - S[1])) / g->dy + 0.5 * g->ny;
                            }
                        }
                        const double q0 = row ? (double)j : (double)i;
                        const double blo = fmin(bb[0], bb[1]), bhi = fmax(bb[0], bb[1]);
                        const double ot = fmin(bhi, q0 + 1.0) - fmax(blo, q0);
                        if (!(ot > 0.0) || !(bhi > blo)) continue;
                        /* axial: rows l, l+1 boundaries at the column centre's depth */
                        const double ell = (xc - S[0]) * c + (yc - S[1]) * s;
                        const double za = (S[2] + w_bound(g, l) * ell / g->dsd - zlo) / g->dz;
                        const double zb = (S[2] + w_bound(g, l + 1) * ell / g->dsd - zlo) / g->dz;
                        const double oa = fmin(zb, kz + 1.0) - fmax(za, (double)kz);
                        if (!(oa > 0.0)) continue;
                        rowp[((size_t)kz * g->ny + i) * g->nx + j] = seg * (ot / (bhi - blo)) * (oa / (zb - za));
                    }
        }
}

int h3_row_sweep(const h3_geom *g, int v)
{
    const double beta = g->beta0 + 2.0 * H3_PI * (double)v / (double)g->views_per_turn;
    return fabs(sin(beta)) >= fabs(cos(beta)) - 1e-12;
}

/* ------------------------------------------------------------------------------------------------ */
/* Regularizer: 13 directions (all 26 neighbours)                                                    */
/* ------------------------------------------------------------------------------------------------ */

/* offsets (dz, di, dj), the first nonzero component positive: one per neighbour pair */
static const int D13[13][3] = {{0, 0, 1}, {0, 1, 0}, {1, 0, 0}, {0, 1, 1}, {0, 1, -1}, {1, 0, 1}, {1, 0, -1},
                               {1, 1, 0}, {1, -1, 0}, {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};

static double dir_norm(int d) { return sqrt((double)(D13[d][0] * D13[d][0] + D13[d][1] * D13[d][1] + D13[d][2] * D13[d][2])); }

#define QGG_Q 1.2
static double pot(int kind, double d, double t)
{
    const double z = t / d;
    if (kind == 0) return d * d * (sqrt(1.0 + z * z) - 1.0);
    const double a = fabs(z);
    if (kind == 1) return d * d * (a - log1p(a));
    return 0.5 * t * t / (1.0 + pow(a, 2.0 - QGG_Q));
}
static double wpot(int kind, double d, double t)
{
    const double z = t / d;
    if (kind == 0) return 1.0 / sqrt(1.0 + z * z);
    if (kind == 1) return 1.0 / (1.0 + fabs(z));
    const double s = pow(fabs(z), 2.0 - QGG_Q);
    return (2.0 + QGG_Q * s) / (2.0 * (1.0 + s) * (1.0 + s));
}

static int inside(const h3_geom *g, int kz, int i, int j)
{
    return kz >= 0 && kz < g->nz && i >= 0 && i < g->ny && j >= 0 && j < g->nx;
}

double h3_reg_cost(const h3_geom *g, const double *x, int kind, double delta, double beta)
{
    double total = 0.0;
    for (int d = 0; d < 13; ++d) {
        double acc = 0.0;
        for (int kz = 0; kz < g->nz; ++kz)
            for (int i = 0; i < g->ny; ++i)
                for (int j = 0; j < g->nx; ++j) {
                    const int k2 = kz + D13[d][0], i2 = i + D13[d][1], j2 = j + D13[d][2];
                    if (!inside(g, k2, i2, j2)) continue;
                    acc += pot(kind, delta, x[vox(g, kz, i, j)] - x[vox(g, k2, i2, j2)]);
                }
        total += beta / dir_norm(d) * acc;
    }
    return total;
}

/* grad = nabla R(x); dr = 2 sum_i beta_i omega(t) over both neighbours of each direction (omega = 1 with
   huber == 0: the maximum curvature). */
void h3_reg_grad(const h3_geom *g, const double *x, int kind, double delta, double beta, int huber, double *grad,
                 double *dr)
{
    #pragma omp parallel for schedule(static)
    for (int kz = 0; kz < g->nz; ++kz)
        for (int i = 0; i < g->ny; ++i)
            for (int j = 0; j < g->nx; ++j) {
                const double xc = x[vox(g, kz, i, j)];
                double gs = 0.0, ds = 0.0;
                for (int d = 0; d < 13; ++d) {
                    const double bd = beta / dir_norm(d);
                    for (int sg = -1; sg <= 1; sg += 2) {
                        const int k2 = kz + sg * D13[d][0], i2 = i + sg * D13[d][1], j2 = j + sg * D13[d][2];
                        if (!inside(g, k2, i2, j2)) continue;
                        const double t = xc - x[vox(g, k2, i2, j2)];
                        const double om = wpot(kind, delta, t);
                        gs += bd * om * t;
                        ds += bd * 2.0 * (huber ? om : 1.0);
                    }
                }
                grad[vox(g, kz, i, j)] = gs;
                if (dr) dr[vox(g, kz, i, j)] = ds;
            }
}

/* ------------------------------------------------------------------------------------------------ */
/* Cost, D_L, subsets, the relaxed OS-LALM iteration                                                 */
/* ------------------------------------------------------------------------------------------------ */

static int subset_views(int nviews, int M, int m, int *views)
{
    int n = 0;
    for (int v = m; v < nviews; v += M) views[n++] = v;
    return n;
}

double h3_cost(const h3_geom *g, const double *y, const double *w, const double *x, int kind, double delta,
               double beta)
{
    const int nv = g->nviews;
    const size_t ns = (size_t)nv * g->nr * g->nb;
    int *views = (int *)malloc(sizeof(int) * nv);
    for (int v = 0; v < nv; ++v) views[v] = v;
    double *p = (double *)malloc(sizeof(double) * ns);
    h3_forward(g, views, nv, x, p);
    double data = 0.0;
    for (size_t n = 0; n < ns; ++n) data += 0.5 * w[n] * (p[n] - y[n]) * (p[n] - y[n]);
    free(p); free(views);
    return data + h3_reg_cost(g, x, kind, delta, beta);
}

void h3_dl(const h3_geom *g, const double *w, double *dl)
{
    const int nv = g->nviews;
    const size_t nvox = (size_t)g->nx * g->ny * g->nz, ns = (size_t)nv * g->nr * g->nb;
    int *views = (int *)malloc(sizeof(int) * nv);
    for (int v = 0; v < nv; ++v) views[v] = v;
    double *one = (double *)malloc(sizeof(double) * nvox);
    double *p = (double *)malloc(sizeof(double) * ns);
    for (size_t n = 0; n < nvox; ++n) one[n] = 1.0;
    h3_forward(g, views, nv, one, p);
    for (size_t n = 0; n < ns; ++n) p[n] *= w[n];
    h3_back(g, views, nv, p, dl);
    free(one); free(p); free(views);
}

double h3_rho(long long k, double alpha)
{
    if (k == 0) return 1.0;
    const double a = H3_PI / (alpha * (double)(k + 1));
    return a * sqrt(1.0 - 0.25 * a * a);
}

/* subset processing order: sequential, or bit-reversed (the permutation of 0..M-1 by the bit reversal of
   the next power of two, keeping the values below M) */
static void order_table(int M, int kind, int *ord)
{
    if (kind == 0) {
        for (int m = 0; m < M; ++m) ord[m] = m;
        return;
    }
    int bits = 0;
    while ((1 << bits) < M) ++bits;
    int n = 0;
    for (int r = 0; r < (1 << bits); ++r) {
        int v = 0;
        for (int b = 0; b < bits; ++b)
            if (r & (1 << b)) v |= 1 << (bits - 1 - b);
        if (v < M) ord[n++] = v;
    }
}

/* zeta = M A_m' W_m (A_m x - y_m) over the listed views. */
static void subset_grad(const h3_geom *g, const int *views, int nv, const double *y, const double *w,
                        const double *x, double scale, double *p, double *zeta)
{
    const size_t cells = (size_t)g->nr * g->nb;
    h3_forward(g, views, nv, x, p);
    for (int iv = 0; iv < nv; ++iv) {
        const size_t base = (size_t)views[iv] * cells;
        for (size_t c = 0; c < cells; ++c) {
            double *pc = p + (size_t)iv * cells + c;
            *pc = scale * w[base + c] * (*pc - y[base + c]);
        }
    }
    h3_back(g, views, nv, p, zeta);
}

/* Initial state from x (clipped): zeta on the last subset of the order (or all views), g = zeta,
   h = D_L x - zeta. */
void h3_rlalm_init(const h3_geom *g, const h3_params *pp, const double *y, const double *w, const double *dl,
                   double *x, double *gv, double *h)
{
    const size_t nvox = (size_t)g->nx * g->ny * g->nz;
    const int M = pp->nsubsets;
    int *ord = (int *)malloc(sizeof(int) * M);
    order_table(M, pp->subset_order, ord);
    int *views = (int *)malloc(sizeof(int) * g->nviews);
    double *p = (double *)malloc(sizeof(double) * (size_t)g->nviews * g->nr * g->nb);
    for (size_t n = 0; n < nvox; ++n) x[n] = x[n] > 0.0 ? x[n] : 0.0;
    int nv;
    double sc;
    if (pp->init_full) {
        nv = g->nviews;
        for (int v = 0; v < nv; ++v) views[v] = v;
        sc = 1.0;
    } else {
        nv = subset_views(g->nviews, M, ord[M - 1], views);
        sc = (double)M;
    }
    subset_grad(g, views, nv, y, w, x, sc, p, gv);
    for (size_t n = 0; n < nvox; ++n) h[n] = dl[n] * x[n] - gv[n];
    free(ord); free(views); free(p);
}

/*
 * Subiterations t0 .. t0 + nsub - 1 of the proposed relaxation as a transition of the state (x, g, h):
 *   gamma = (rho - 1) g + rho h;  x+ = [(rho D_L + D_R)^-1 (gamma + D_R x - grad R(x))]_+
 *   zeta = M grad L_m(x+);  g+ = rho/(rho+1) (alpha zeta + (1 - alpha) g) + g/(rho+1);
 *   h+ = alpha (D_L x+ - zeta) + (1 - alpha) h
 * with rho = rho_t (eq. dec_rho, t the subiteration count) or fixed, m the subset of subiteration t.
 */
void h3_rlalm_iterate(const h3_geom *g, const h3_params *pp, const double *y, const double *w, const double *dl,
                      double *x, double *gv, double *h, long long t0, long long nsub)
{
    const size_t nvox = (size_t)g->nx * g->ny * g->nz;
    const int M = pp->nsubsets;
    int *ord = (int *)malloc(sizeof(int) * M);
    order_table(M, pp->subset_order, ord);
    int *views = (int *)malloc(sizeof(int) * (g->nviews / M + 1));
    double *p = (double *)malloc(sizeof(double) * ((size_t)g->nviews / M + 1) * g->nr * g->nb);
    double *zeta = (double *)malloc(sizeof(double) * nvox);
    double *gr = (double *)malloc(sizeof(double) * nvox);
    double *dr = (double *)malloc(sizeof(double) * nvox);
    const double alpha = pp->alpha;
    for (long long t = t0; t < t0 + nsub; ++t) {
        const double rho = pp->rho_mode == 0 ? h3_rho(t, alpha) : pp->rho_fixed;
        h3_reg_grad(g, x, pp->potential, pp->delta, pp->beta, pp->huber, gr, dr);
        for (size_t n = 0; n < nvox; ++n) {
            const double gamma = (rho - 1.0) * gv[n] + rho * h[n];
            const double curv = rho * dl[n] + dr[n];
            const double xn = curv > 0.0 ? (gamma + dr[n] * x[n] - gr[n]) / curv : x[n];
            x[n] = xn > 0.0 ? xn : 0.0;
        }
        const int nv = subset_views(g->nviews, M, ord[t % M], views);
        subset_grad(g, views, nv, y, w, x, (double)M, p, zeta);
        for (size_t n = 0; n < nvox; ++n) {
            const double z = zeta[n], go = gv[n];
            gv[n] = rho / (rho + 1.0) * (alpha * z + (1.0 - alpha) * go) + go / (rho + 1.0);
            h[n] = alpha * (dl[n] * x[n] - z) + (1.0 - alpha) * h[n];
        }
    }
    free(ord); free(views); free(p); free(zeta); free(gr); free(dr);
}

/* Whole solve: D_L (times dl_scale), initialisation, niters * M subiterations. x: x0 in, x^(K) out. */
void h3_rlalm_solve(const h3_geom *g, const h3_params *pp, const double *y, const double *w, double *x,
                    double *dl)
{
    const size_t nvox = (size_t)g->nx * g->ny * g->nz;
    h3_dl(g, w, dl);
    for (size_t n = 0; n < nvox; ++n) dl[n] *= pp->dl_scale;
    double *gv = (double *)malloc(sizeof(double) * nvox);
    double *h = (double *)malloc(sizeof(double) * nvox);
    h3_rlalm_init(g, pp, y, w, dl, x, gv, h);
    h3_rlalm_iterate(g, pp, y, w, dl, x, gv, h, 0, (long long)pp->niters * pp->nsubsets);
    free(gv); free(h);
}
