/*
 * FP64 CPU oracle for relaxed OS-LALM (OS-RLALM) PWLS fan-beam CT reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously-correct reference that the HIP
 * path is checked against. Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it. It shares no code, header, table or constant generator with the HIP library.
 *
 * Everything is computed in double precision, following the paper (Nien & Fessler, "Relaxed linearized
 * algorithms for faster X-ray CT image reconstruction"):
 *   - PWLS problem  min_{x>=0} 1/2 ||y - A x||_W^2 + R(x)                (Section III, eq. ct_problem)
 *   - regularizer   R(x) = sum_i beta_i sum_n phi([C_i x]_n)            (Section III, eq. def_reg; kappa = 1)
 *   - D_L = diag{A' W A 1}                                               (Section III-A, diagonal majorizer)
 *   - Huber curvature D_R of R at the current x                          (Section III-A)
 *   - the proposed relaxed OS-LALM (Algorithm 1) as a state transition written from eq.
 *     relaxed_lal_iter_quad, and the simple relaxation (Algorithm 2)
 *   - the alpha-dependent continuation rho_k(alpha)                      (Section III-B, eq. dec_rho)
 *   - reference solution x* by FGM with gradient-based adaptive restart  (Section IV-A, footnote reference)
 *
 * The paper cites, but does not define, its projector. The operator here is the distance-driven
 * fan-beam projector, computed by the classic sequential merge of sorted pixel edges and detector-bin
 * boundaries along each image line:
 *   a_{(v,k),(l,q)} = (Delta_l / |cos theta_{v,k}|) * |pixel q  intersect  [b_k(l), b_{k+1}(l)]|
 *                                                  / |b_{k+1}(l) - b_k(l)|
 * where the image "lines" l are rows for views whose central ray is within 45 degrees of the y axis
 * ("row sweep", decided in FP64 as |sin beta| >= |cos beta| - 1e-12) and columns otherwise, b_k(l) is
 * the point where the ray from the source through detector boundary k crosses line l (in pixel units
 * along the line), and theta_{v,k} is the angle between the line normal and the ray through the centre
 * of bin k.
 *
 * Parity status: every function here is pinned by CPU tests (brute force, closed forms, invariants);
 * the OS-RLALM iterates themselves have no closed form and are pinned through those invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

typedef struct {
    int nx, ny;
    double dx, dy;
    int nb;
    double du, u_offset;
    int det; /* 0 = flat, 1 = arc */
    int nviews;
    double beta0, span;
    double dso, dsd;
} or_geom;

/* ------------------------------------------------------------------------------------------------ */
/* Geometry                                                                                          */
/* ------------------------------------------------------------------------------------------------ */

typedef struct {
    double sx, sy;      /* source */
    double dxv, dyv;    /* central direction d */
    double ex, ey;      /* detector axis e */
    int row_sweep;
} or_view;

static void view_of(const or_geom *g, int v, or_view *o)
{
    double beta = g->beta0 + g->span * (double)v / (double)g->nviews;
    double c = cos(beta), s = sin(beta);
    o->dxv = c; o->dyv = s;
    o->ex = -s; o->ey = c;
    o->sx = -g->dso * c; o->sy = -g->dso * s;
    o->row_sweep = fabs(s) >= fabs(c) - 1e-12;
}

/* Detector point at detector coordinate u (mm). */
static void det_point(const or_geom *g, const or_view *o, double u, double *px, double *py)
{
    if (g->det == 0) {
        double off = g->dsd - g->dso;
        *px = off * o->dxv + u * o->ex;
        *py = off * o->dyv + u * o->ey;
    } else {
        double gam = u / g->dsd;
        *px = o->sx + g->dsd * (cos(gam) * o->dxv + sin(gam) * o->ex);
        *py = o->sy + g->dsd * (cos(gam) * o->dyv + sin(gam) * o->ey);
    }
}

static double bin_boundary_u(const or_geom *g, int k) { return ((double)k - 0.5 * g->nb + g->u_offset) * g->du; }

int or_row_sweep(const or_geom *g, int v)
{
    or_view o;
    view_of(g, v, &o);
    return o.row_sweep;
}

/*
 * Per (view, line): positions b[k], k = 0..nb, of the boundary rays on line l in pixel units along the
 * line (pixel q spans [q, q+1]), and the per-bin scale Delta_l / |cos theta_k|.
 */
typedef struct {
    int nl, nq;          /* number of lines, pixels per line */
    double *px, *py;     /* detector boundary points, nb+1 */
    double *scale;       /* nb */
    or_view o;
} view_tab;

static void view_tab_init(const or_geom *g, int v, view_tab *t)
{
    view_of(g, v, &t->o);
    t->nl = t->o.row_sweep ? g->ny : g->nx;
    t->nq = t->o.row_sweep ? g->nx : g->ny;
    t->px = (double *)malloc(sizeof(double) * (g->nb + 1));
    t->py = (double *)malloc(sizeof(double) * (g->nb + 1));
    t->scale = (double *)malloc(sizeof(double) * g->nb);
    for (int k = 0; k <= g->nb; ++k) det_point(g, &t->o, bin_boundary_u(g, k), &t->px[k], &t->py[k]);
    for (int k = 0; k < g->nb; ++k) {
        double cx, cy;
        det_point(g, &t->o, 0.5 * (bin_boundary_u(g, k) + bin_boundary_u(g, k + 1)), &cx, &cy);
        double rx = cx - t->o.sx, ry = cy - t->o.sy;
        double len = sqrt(rx * rx + ry * ry);
        /* theta: angle between the ray and the line normal (y axis for rows, x axis for columns) */
        t->scale[k] = t->o.row_sweep ? g->dy * len / fabs(ry) : g->dx * len / fabs(rx);
    }
}

static void view_tab_free(view_tab *t)
{
    free(t->px); free(t->py); free(t->scale);
}

/* Boundary positions on line l (pixel units along the line, pixel q spans [q, q+1]). */
static void line_boundaries(const or_geom *g, const view_tab *t, int l, double *b)
{
    const or_view *o = &t->o;
    if (o->row_sweep) {
        double yl = ((double)l - 0.5 * (g->ny - 1)) * g->dy;
        for (int k = 0; k <= g->nb; ++k) {
            double X = o->sx + (yl - o->sy) * (t->px[k] - o->sx) / (t->py[k] - o->sy);
            b[k] = X / g->dx + 0.5 * g->nx;
        }
    } else {
        double xl = ((double)l - 0.5 * (g->nx - 1)) * g->dx;
        for (int k = 0; k <= g->nb; ++k) {
            double Y = o->sy + (xl - o->sx) * (t->py[k] - o->sy) / (t->px[k] - o->sx);
            b[k] = Y / g->dy + 0.5 * g->ny;
        }
    }
}

/* index of image element (line l, pixel q) in the [ny][nx] row-major image */
static inline size_t img_index(const or_geom *g, const view_tab *t, int l, int q)
{
    return t->o.row_sweep ? (size_t)l * g->nx + q : (size_t)q * g->nx + l;
}

/*
 * Sequential merge of the ascending detector-bin intervals with the pixel edges 0, 1, ..., nq along
 * one line. Calls back once per nonzero overlap with (bin k, pixel q, weight a).
 * mode 0: forward (p[k] += a * img), mode 1: back (img += a * r[k]).
 */
static void merge_line(const or_geom *g, const view_tab *t, int l, const double *b, int mode,
                       const double *img_in, double *p_out, const double *r_in, double *img_out)
{
    int nb = g->nb, nq = t->nq;
    int inc = b[nb] > b[0];
    int kk = 0;
    /* ascending order position kk -> bin index k and its interval [lo, hi] */
#define BIN_OF(kk) (inc ? (kk) : nb - 1 - (kk))
#define LO_OF(kk) (inc ? b[(kk)] : b[nb - (kk)])
#define HI_OF(kk) (inc ? b[(kk) + 1] : b[nb - 1 - (kk)])
    while (kk < nb && HI_OF(kk) <= 0.0) ++kk;
    if (kk >= nb) return;
    int q = (int)floor(LO_OF(kk));
    if (q < 0) q = 0;
    while (kk < nb && q < nq) {
        double lo = LO_OF(kk), hi = HI_OF(kk);
        double a0 = lo > (double)q ? lo : (double)q;
        double a1 = hi < (double)(q + 1) ? hi : (double)(q + 1);
        if (a1 > a0 && hi > lo) {
            int k = BIN_OF(kk);
            double a = t->scale[k] * (a1 - a0) / (hi - lo);
            size_t idx = img_index(g, t, l, q);
            if (mode == 0) p_out[k] += a * img_in[idx];
            else img_out[idx] += a * r_in[k];
        }
        if (hi < (double)(q + 1)) ++kk; else ++q;
    }
#undef BIN_OF
#undef LO_OF
#undef HI_OF
}

/* p[iv][k] = (A x) for views[iv], iv = 0..nv-1. */
void or_forward(const or_geom *g, const int *views, int nv, const double *x, double *p)
{
    #pragma omp parallel for schedule(dynamic, 1) if ((long)nv * g->nb * (g->nx + g->ny) > 2000000L)
    for (int iv = 0; iv < nv; ++iv) {
        view_tab t;
        view_tab_init(g, views[iv], &t);
        double *b = (double *)malloc(sizeof(double) * (g->nb + 1));
        double *pv = p + (size_t)iv * g->nb;
        memset(pv, 0, sizeof(double) * g->nb);
        for (int l = 0; l < t.nl; ++l) {
            line_boundaries(g, &t, l, b);
            merge_line(g, &t, l, b, 0, x, pv, NULL, NULL);
        }
        free(b);
        view_tab_free(&t);
    }
}

/* x = A' r over views[iv] (x overwritten). r is [nv][nb]. */
void or_back(const or_geom *g, const int *views, int nv, const double *r, double *x)
{
    size_t npix = (size_t)g->nx * g->ny;
    memset(x, 0, sizeof(double) * npix);
    view_tab *tabs = (view_tab *)malloc(sizeof(view_tab) * (nv > 0 ? nv : 1));
    for (int iv = 0; iv < nv; ++iv) view_tab_init(g, views[iv], &tabs[iv]);
    /* pass 0: row-sweep views, parallel over rows; pass 1: column-sweep views, parallel over columns.
       Each line writes only its own pixels, so there are no write conflicts. */
    for (int pass = 0; pass < 2; ++pass) {
        int nl = pass == 0 ? g->ny : g->nx;
        #pragma omp parallel for schedule(dynamic, 4) if ((long)nv * g->nb * (g->nx + g->ny) > 2000000L)
        for (int l = 0; l < nl; ++l) {
            double *b = (double *)malloc(sizeof(double) * (g->nb + 1));
            for (int iv = 0; iv < nv; ++iv) {
                if (tabs[iv].o.row_sweep != (pass == 0)) continue;
                line_boundaries(g, &tabs[iv], l, b);
                merge_line(g, &tabs[iv], l, b, 1, NULL, NULL, r + (size_t)iv * g->nb, x);
            }
            free(b);
        }
    }
    for (int iv = 0; iv < nv; ++iv) view_tab_free(&tabs[iv]);
    free(tabs);
}

/* Per-bin scale Delta/|cos theta| and sweep mode (for tests). scale is [nb]. */
void or_view_scale(const or_geom *g, int v, double *scale, int *row_sweep)
{
    view_tab t;
    view_tab_init(g, v, &t);
    memcpy(scale, t.scale, sizeof(double) * g->nb);
    *row_sweep = t.o.row_sweep;
    view_tab_free(&t);
}

/* Boundary positions b[k] (k = 0..nb) of view v on line l (for tests). */
void or_line_boundaries(const or_geom *g, int v, int l, double *b)
{
    view_tab t;
    view_tab_init(g, v, &t);
    line_boundaries(g, &t, l, b);
    view_tab_free(&t);
}

/* ------------------------------------------------------------------------------------------------ */
/* Regularizer: R(x) = sum_i beta_i sum_n phi([C_i x]_n)                                             */
/* Four directions (0,1), (1,0), (1,1), (1,-1) in (row, col) offsets, beta_i = beta / ||s_i||,       */
/* kappa = 1, a difference exists only when both pixels are inside the image.                        */
/* potential 0 = hyperbola delta^2 (sqrt(1 + (t/delta)^2) - 1), 1 = Fair delta^2 (|t/d| - log(1+|t/d|)), */
/* 2 = q-GGMRF with p = 2, q = 1.2 (the q-generalized Gaussian MRF the paper's chest-scan experiment    */
/* cites, in its published form): |t|^2 / (2 (1 + |t/d|^(p-q))), t^2/2 near 0 like the other two.       */
/* ------------------------------------------------------------------------------------------------ */

static const int DIR_DI[4] = {0, 1, 1, 1};
static const int DIR_DJ[4] = {1, 0, 1, -1};

#define QGG_Q 1.2

static double pot(int kind, double d, double t)
{
    double z = t / d;
    if (kind == 0) return d * d * (sqrt(1.0 + z * z) - 1.0);
    double a = fabs(z);
    if (kind == 1) return d * d * (a - log1p(a));
    return 0.5 * t * t / (1.0 + pow(a, 2.0 - QGG_Q));
}

/* Huber curvature phi'(t)/t (its limit 1 at t = 0). For the q-GGMRF, with s = |t/d|^(2-q):
   phi'(t) = t (2 + q s) / (2 (1 + s)^2). */
static double wpot(int kind, double d, double t)
{
    double z = t / d;
    if (kind == 0) return 1.0 / sqrt(1.0 + z * z);
    if (kind == 1) return 1.0 / (1.0 + fabs(z));
    double s = pow(fabs(z), 2.0 - QGG_Q);
    return (2.0 + QGG_Q * s) / (2.0 * (1.0 + s) * (1.0 + s));
}

static double dpot(int kind, double d, double t)
{
    double z = t / d;
    if (kind == 0) return t / sqrt(1.0 + z * z);
    if (kind == 1) return t / (1.0 + fabs(z));
    return t * wpot(kind, d, t);
}

static double dir_beta(double beta, int i) { return i < 2 ? beta : beta / sqrt(2.0); }

double or_reg_cost_k(int nx, int ny, const double *x, int kind, double delta, double beta, const double *kap);
double or_reg_cost(int nx, int ny, const double *x, int kind, double delta, double beta)
{
    return or_reg_cost_k(nx, ny, x, kind, delta, beta, NULL);
}

/* R(x) with certainty weights: each pair term is multiplied by kappa_j kappa_n (kap NULL: kappa = 1). */
double or_reg_cost_k(int nx, int ny, const double *x, int kind, double delta, double beta, const double *kap)
{
    double total = 0.0;
    for (int d = 0; d < 4; ++d) {
        double bd = dir_beta(beta, d), acc = 0.0;
        for (int i = 0; i < ny; ++i)
            for (int j = 0; j < nx; ++j) {
                int i2 = i + DIR_DI[d], j2 = j + DIR_DJ[d];
                if (i2 < 0 || i2 >= ny || j2 < 0 || j2 >= nx) continue;
                double kk = kap ? kap[(size_t)i * nx + j] * kap[(size_t)i2 * nx + j2] : 1.0;
                acc += kk * pot(kind, delta, x[(size_t)i * nx + j] - x[(size_t)i2 * nx + j2]);
            }
        total += bd * acc;
    }
    return total;
}

/*
 * grad = nabla R(x); dr = Huber-curvature diagonal majorizer: for each pair term with difference t,
 * each of its two pixels receives |c| * ||c||_1 * omega(t) = 2 omega(t) times beta_i (SQS by convexity).
 * When huber == 0, omega is replaced by its maximum 1 (the fixed maximum-curvature majorizer).
 */
void or_reg_grad_k(int nx, int ny, const double *x, int kind, double delta, double beta, int huber,
                   const double *kap, double *grad, double *dr);
void or_reg_grad(int nx, int ny, const double *x, int kind, double delta, double beta, int huber,
                 double *grad, double *dr)
{
    or_reg_grad_k(nx, ny, x, kind, delta, beta, huber, NULL, grad, dr);
}

void or_reg_grad_k(int nx, int ny, const double *x, int kind, double delta, double beta, int huber,
                   const double *kap, double *grad, double *dr)
{
    #pragma omp parallel for schedule(static) if ((long)nx * ny > 65536L)
    for (int i = 0; i < ny; ++i)
        for (int j = 0; j < nx; ++j) {
            double gsum = 0.0, dsum = 0.0, xc = x[(size_t)i * nx + j];
            for (int d = 0; d < 4; ++d) {
                double bd = dir_beta(beta, d);
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    int i2 = i + sgn * DIR_DI[d], j2 = j + sgn * DIR_DJ[d];
                    if (i2 < 0 || i2 >= ny || j2 < 0 || j2 >= nx) continue;
                    double t = xc - x[(size_t)i2 * nx + j2];
                    double kk = kap ? kap[(size_t)i * nx + j] * kap[(size_t)i2 * nx + j2] : 1.0;
                    gsum += kk * bd * dpot(kind, delta, t);
                    dsum += kk * bd * 2.0 * (huber ? wpot(kind, delta, t) : 1.0);
                }
            }
            grad[(size_t)i * nx + j] = gsum;
            if (dr) dr[(size_t)i * nx + j] = dsum;
        }
}

/* ------------------------------------------------------------------------------------------------ */
/* Cost, D_L, subsets                                                                                */
/* ------------------------------------------------------------------------------------------------ */

/* Interleaved subset m of M: views v with v mod M == m, ascending. Returns the count. */
int or_subset_views(int nviews, int M, int m, int *views)
{
    int n = 0;
    for (int v = m; v < nviews; v += M) views[n++] = v;
    return n;
}

/* Psi(x) = 1/2 sum w (A x - y)^2 + R(x), over all views */
double or_cost(const or_geom *g, const double *y, const double *w, const double *x, int kind, double delta,
               double beta)
{
    int nv = g->nviews;
    int *views = (int *)malloc(sizeof(int) * nv);
    for (int v = 0; v < nv; ++v) views[v] = v;
    double *p = (double *)malloc(sizeof(double) * (size_t)nv * g->nb);
    or_forward(g, views, nv, x, p);
    double data = 0.0;
    for (size_t i = 0; i < (size_t)nv * g->nb; ++i) {
        double r = p[i] - y[i];
        data += 0.5 * w[i] * r * r;
    }
    free(p); free(views);
    return data + or_reg_cost(g->nx, g->ny, x, kind, delta, beta);
}

/* D_L = A' (w .* (A 1)) over all views (the diagonal majorizer of A' W A). */
void or_dl(const or_geom *g, const double *w, double *dl)
{
    int nv = g->nviews;
    size_t npix = (size_t)g->nx * g->ny;
    int *views = (int *)malloc(sizeof(int) * nv);
    for (int v = 0; v < nv; ++v) views[v] = v;
    double *ones = (double *)malloc(sizeof(double) * npix);
    for (size_t i = 0; i < npix; ++i) ones[i] = 1.0;
    double *p = (double *)malloc(sizeof(double) * (size_t)nv * g->nb);
    or_forward(g, views, nv, ones, p);
    for (size_t i = 0; i < (size_t)nv * g->nb; ++i) p[i] *= w[i];
    or_back(g, views, nv, p, dl);
    free(p); free(ones); free(views);
}

/*
 * zeta = scale * A_m' (w_m .* (A_m x - y_m)) for the listed views (y, w are full [nviews][nb] arrays).
 * Work buffers p must hold nv*nb doubles.
 */
static void subset_grad(const or_geom *g, const int *views, int nv, const double *y, const double *w,
                        const double *x, double scale, double *p, double *zeta)
{
    or_forward(g, views, nv, x, p);
    for (int iv = 0; iv < nv; ++iv) {
        size_t off = (size_t)views[iv] * g->nb;
        double *pv = p + (size_t)iv * g->nb;
        for (int k = 0; k < g->nb; ++k) pv[k] = scale * w[off + k] * (pv[k] - y[off + k]);
    }
    or_back(g, views, nv, p, zeta);
}

/* Full data-term gradient A' W (A x - y). */
void or_data_grad(const or_geom *g, const double *y, const double *w, const double *x, double *grad)
{
    int nv = g->nviews;
    int *views = (int *)malloc(sizeof(int) * nv);
    for (int v = 0; v < nv; ++v) views[v] = v;
    double *p = (double *)malloc(sizeof(double) * (size_t)nv * g->nb);
    subset_grad(g, views, nv, y, w, x, 1.0, p, grad);
    free(p); free(views);
}

/* ------------------------------------------------------------------------------------------------ */
/* Continuation sequence rho_k(alpha) (Section III-B, eq. dec_rho): 1 at k = 0, else                */
/* pi/(alpha (k+1)) sqrt(1 - (pi/(2 alpha (k+1)))^2). k counts subiterations.                        */
/* ------------------------------------------------------------------------------------------------ */

double or_rho(long long k, double alpha)
{
    if (k == 0) return 1.0;
    double a = OR_PI / (alpha * (double)(k + 1));
    double b = OR_PI / (2.0 * alpha * (double)(k + 1));
    return a * sqrt(1.0 - b * b);
}

/* ------------------------------------------------------------------------------------------------ */
/* Algorithm 1 (proposed relaxed OS-LALM) and Algorithm 2 (simple relaxation)                        */
/* ------------------------------------------------------------------------------------------------ */

typedef struct {
    double alpha;
    int niters;         /* outer iterations, each of M subiterations */
    int nsubsets;       /* M */
    int rho_mode;       /* 0 continuation, 1 fixed */
    double rho_fixed;
    int potential;      /* 0 hyperbola, 1 Fair, 2 q-GGMRF */
    double delta, beta;
    int huber;          /* 1 Huber curvature D_R (the paper's choice), 0 maximum curvature */
    int algorithm;      /* 1 proposed (with h), 2 simple */
    int init_full;      /* 0: initial gradient from the last subset (as written), 1: full gradient */
    double dl_scale;    /* multiplies D_L (1 = the majorizer; < 1 violates it) */
    int subset_order;   /* 0: subsets m = 0, 1, ..., M-1; 1: bit-reversed order */
    int kappa;          /* 0: kappa = 1; 1: certainty weights kappa_j = sqrt([A'w]_j / [A'1]_j) */
} or_params;

/* Position i of the subset order: identity, or the bit reversal of 0..P-1 (P the next power of two
   >= M) with the values >= M dropped. */
static void subset_order_table(int M, int kind, int *order)
{
    if (kind == 0) { for (int m = 0; m < M; ++m) order[m] = m; return; }
    int P = 1, bits = 0, n = 0;
    while (P < M) { P <<= 1; ++bits; }
    for (int i = 0; i < P; ++i) {
        int r = 0;
        for (int b = 0; b < bits; ++b) if (i & (1 << b)) r |= 1 << (bits - 1 - b);
        if (r < M) order[n++] = r;
    }
}

void or_subset_order(int M, int kind, int *order) { subset_order_table(M, kind, order); }

/* kappa_j = sqrt([A' w]_j / [A' 1]_j) over all views (0 where no ray meets the pixel) */
void or_kappa(const or_geom *g, const double *w, double *kap)
{
    int nv = g->nviews;
    size_t npix = (size_t)g->nx * g->ny, nsino = (size_t)nv * g->nb;
    int *views = (int *)malloc(sizeof(int) * nv);
    for (int v = 0; v < nv; ++v) views[v] = v;
    double *ones = (double *)malloc(sizeof(double) * nsino);
    double *b1 = (double *)malloc(sizeof(double) * npix);
    for (size_t i = 0; i < nsino; ++i) ones[i] = 1.0;
    or_back(g, views, nv, w, kap);
    or_back(g, views, nv, ones, b1);
    for (size_t j = 0; j < npix; ++j) kap[j] = b1[j] > 0.0 ? sqrt(kap[j] > 0.0 ? kap[j] / b1[j] : 0.0) : 0.0;
    free(views); free(ones); free(b1);
}

/*
 * One subiteration as a state transition (x, g, h) at subiteration t -> the state at t + 1, written from
 * the quadratic-loss form of the proposed relaxed linearized AL iteration (eq. relaxed_lal_iter_quad)
 * under the substitution A <- W^(1/2) A, y <- W^(1/2) y (eq. ct_substitution), with phi the indicator of
 * Omega, psi = R majorized by its Huber-curvature quadratic Q_R(.; x) (Section III-A), D_A = D_L, the
 * subset gradient M grad L_m in place of grad L (ordered subsets, m the subset of subiteration t), and
 * rho = rho_t (eq. dec_rho; t counts subiterations):
 *   gamma = (rho - 1) g + rho h
 *   x+    = argmin_{x in Omega} Q_R(x; x_old) + 1/2 || x - (rho D_L)^-1 gamma ||^2_{rho D_L}
 *         = [ (rho D_L + D_R)^-1 (gamma + D_R x_old - grad R(x_old)) ]_+     (separable, clipped)
 *   zeta  = M grad L_m(x+)
 *   g+    = rho/(rho+1) (alpha zeta + (1 - alpha) g) + g/(rho+1)
 *   h+    = alpha (D_L x+ - zeta) + (1 - alpha) h
 * The simple relaxation (the paper's second OS algorithm, Algorithm 2) has no h recursion; its x-step
 * linearizes at the last subset gradient, gamma = rho (D_L x_old - zeta_old) + (rho - 1) g, and the h
 * slot holds that last zeta.
 */
typedef struct {
    const or_geom *g;
    const or_params *pp;
    const double *y, *w, *dl, *kap;
    int M, nvm;
    int *order, *views;
    double *p, *zeta, *gr, *dr;
} or_machine;

static void transition(const or_machine *mc, long long t, double *x, double *gv, double *h)
{
    const or_params *pp = mc->pp;
    const size_t npix = (size_t)mc->g->nx * mc->g->ny;
    const double rho = pp->rho_mode == 0 ? or_rho(t, pp->alpha) : pp->rho_fixed;
    const double alpha = pp->alpha;
    /* majorizer of R at the current image: grad R(x_old) and the Huber curvature D_R(x_old) */
    or_reg_grad_k(mc->g->nx, mc->g->ny, x, pp->potential, pp->delta, pp->beta, pp->huber, mc->kap, mc->gr, mc->dr);
    for (size_t j = 0; j < npix; ++j) {
        const double gamma = pp->algorithm == 1 ? (rho - 1.0) * gv[j] + rho * h[j]
                                                : rho * (mc->dl[j] * x[j] - h[j]) + (rho - 1.0) * gv[j];
        const double curv = rho * mc->dl[j] + mc->dr[j];
        const double xn = curv > 0.0 ? (gamma + mc->dr[j] * x[j] - mc->gr[j]) / curv : x[j];
        x[j] = xn > 0.0 ? xn : 0.0;
    }
    const int nv = or_subset_views(mc->g->nviews, mc->M, mc->order[t % mc->M], mc->views);
    subset_grad(mc->g, mc->views, nv, mc->y, mc->w, x, (double)mc->M, mc->p, mc->zeta);
    for (size_t j = 0; j < npix; ++j) {
        const double z = mc->zeta[j], gold = gv[j];
        gv[j] = rho / (rho + 1.0) * (alpha * z + (1.0 - alpha) * gold) + gold / (rho + 1.0);
        h[j] = pp->algorithm == 1 ? alpha * (mc->dl[j] * x[j] - z) + (1.0 - alpha) * h[j] : z;
    }
}

/* Runs the transitions t0 .. t0+nsub-1 on the state (x, g, h); optionally records the RMSD (HU, over mask)
   to xref after every trace_every whole iterations. */
static void rlalm_subiters(const or_geom *g, const or_params *pp, const double *y, const double *w,
                           const double *dl, const double *kap, double *x, double *gv, double *h, long long t0,
                           long long nsub, double *rmsd_ref_out, const double *xref, const unsigned char *mask,
                           double mu_w, int trace_every)
{
    or_machine mc;
    const size_t npix = (size_t)g->nx * g->ny;
    mc.g = g; mc.pp = pp; mc.y = y; mc.w = w; mc.dl = dl; mc.kap = kap;
    mc.M = pp->nsubsets;
    mc.nvm = g->nviews / mc.M;
    mc.order = (int *)malloc(sizeof(int) * mc.M);
    subset_order_table(mc.M, pp->subset_order, mc.order);
    mc.views = (int *)malloc(sizeof(int) * (mc.nvm + 1));
    mc.p = (double *)malloc(sizeof(double) * (size_t)(mc.nvm + 1) * g->nb);
    mc.zeta = (double *)malloc(sizeof(double) * npix);
    mc.gr = (double *)malloc(sizeof(double) * npix);
    mc.dr = (double *)malloc(sizeof(double) * npix);
    for (long long t = t0; t < t0 + nsub; ++t) {
        transition(&mc, t, x, gv, h);
        if (rmsd_ref_out && trace_every > 0 && ((t + 1) % ((long long)mc.M * trace_every)) == 0) {
            long long it = (t + 1) / ((long long)mc.M * trace_every) - 1;
            double acc = 0.0; size_t cnt = 0;
            for (size_t j = 0; j < npix; ++j)
                if (!mask || mask[j]) { double d = x[j] - xref[j]; acc += d * d; ++cnt; }
            rmsd_ref_out[it] = cnt ? 1000.0 / mu_w * sqrt(acc / (double)cnt) : 0.0;
        }
    }
    free(mc.views); free(mc.p); free(mc.zeta); free(mc.gr); free(mc.dr); free(mc.order);
}

/*
 * Initialisation (Algorithm 1, first line): x clipped to the constraint set, then
 * zeta = g = M grad L_M(x) on the last subset (or the full gradient when init_full), h = D_L x - zeta.
 * For Algorithm 2, h holds zeta (it is only read as zeta there).
 */
void or_rlalm_init(const or_geom *g, const or_params *pp, const double *y, const double *w, const double *dl,
                   double *x, double *gv, double *h)
{
    int M = pp->nsubsets;
    size_t npix = (size_t)g->nx * g->ny;
    for (size_t j = 0; j < npix; ++j) x[j] = x[j] > 0.0 ? x[j] : 0.0;
    double *zeta = (double *)malloc(sizeof(double) * npix);
    if (pp->init_full) {
        or_data_grad(g, y, w, x, zeta);
    } else {
        int nvm = g->nviews / M;
        int *views = (int *)malloc(sizeof(int) * (nvm + 1));
        double *p = (double *)malloc(sizeof(double) * (size_t)(nvm + 1) * g->nb);
        int *order = (int *)malloc(sizeof(int) * M);
        subset_order_table(M, pp->subset_order, order);
        int nv = or_subset_views(g->nviews, M, order[M - 1], views);
        subset_grad(g, views, nv, y, w, x, (double)M, p, zeta);
        free(views); free(p); free(order);
    }
    for (size_t j = 0; j < npix; ++j) {
        gv[j] = zeta[j];
        h[j] = pp->algorithm == 1 ? dl[j] * x[j] - zeta[j] : zeta[j];
    }
    free(zeta);
}

/* Advance the state (x, g, h) by nsub subiterations starting at subiteration index t0.
   kap: certainty weights (used only when pp->kappa; may be NULL otherwise). */
void or_rlalm_iterate(const or_geom *g, const or_params *pp, const double *y, const double *w, const double *dl,
                      const double *kap, double *x, double *gv, double *h, long long t0, long long nsub)
{
    rlalm_subiters(g, pp, y, w, dl, pp->kappa ? kap : NULL, x, gv, h, t0, nsub, NULL, NULL, NULL, 0.0, 0);
}

/*
 * Whole solve: D_L (scaled by dl_scale), init, niters*M subiterations. x: in x0, out x^(K).
 * Optional trace: rmsd_hu[k] (k = 0..niters-1) of x after iteration k+1 against xref over mask.
 */
void or_rlalm_solve(const or_geom *g, const or_params *pp, const double *y, const double *w, double *x,
                    double *dl_out, const double *xref, const unsigned char *mask, double mu_w, double *rmsd_hu)
{
    size_t npix = (size_t)g->nx * g->ny;
    double *dl = dl_out ? dl_out : (double *)malloc(sizeof(double) * npix);
    double *gv = (double *)malloc(sizeof(double) * npix);
    double *h = (double *)malloc(sizeof(double) * npix);
    double *kap = NULL;
    or_dl(g, w, dl);
    for (size_t j = 0; j < npix; ++j) dl[j] *= pp->dl_scale;
    if (pp->kappa) {
        kap = (double *)malloc(sizeof(double) * npix);
        or_kappa(g, w, kap);
    }
    or_rlalm_init(g, pp, y, w, dl, x, gv, h);
    rlalm_subiters(g, pp, y, w, dl, kap, x, gv, h, 0, (long long)pp->niters * pp->nsubsets, rmsd_hu, xref, mask, mu_w,
                   rmsd_hu ? 1 : 0);
    if (!dl_out) free(dl);
    free(gv); free(h); free(kap);
}

/* ------------------------------------------------------------------------------------------------ */
/* Reference solution x*: projected FGM with gradient-based adaptive restart, diagonal preconditioner */
/* (D_L + D_R^max)^-1 (a fixed majorizer of the Hessian, so every step is a majorize-minimize step).  */
/* Stops after maxit or when both the step change and the projected-gradient residual are small.      */
/* Returns the number of iterations run.                                                              */
/* ------------------------------------------------------------------------------------------------ */

int or_xstar(const or_geom *g, const double *y, const double *w, int kind, double delta, double beta, double *x,
             int maxit, double step_tol, double kkt_tol, double *kkt_out)
{
    size_t npix = (size_t)g->nx * g->ny;
    double *dl = (double *)malloc(sizeof(double) * npix);
    double *pre = (double *)malloc(sizeof(double) * npix);
    double *gr = (double *)malloc(sizeof(double) * npix);
    double *grr = (double *)malloc(sizeof(double) * npix);
    double *dmax = (double *)malloc(sizeof(double) * npix);
    double *z = (double *)malloc(sizeof(double) * npix);
    double *xo = (double *)malloc(sizeof(double) * npix);
    double *x100 = (double *)malloc(sizeof(double) * npix);
    or_dl(g, w, dl);
    /* maximum-curvature regularizer majorizer (omega = 1) */
    or_reg_grad(g->nx, g->ny, x, kind, delta, beta, 0, grr, dmax);
    for (size_t j = 0; j < npix; ++j) {
        double d = dl[j] + dmax[j];
        pre[j] = d > 0.0 ? 1.0 / d : 0.0;
        x[j] = x[j] > 0.0 ? x[j] : 0.0;
        z[j] = x[j];
        x100[j] = x[j];
    }
    /* normaliser for the KKT residual: gradient norm at x = 0 */
    double *zero = (double *)calloc(npix, sizeof(double));
    or_data_grad(g, y, w, zero, gr);
    double g0 = 0.0;
    for (size_t j = 0; j < npix; ++j) g0 += gr[j] * gr[j];
    g0 = sqrt(g0);
    free(zero);
    double tk = 1.0, kkt = INFINITY;
    int it;
    for (it = 0; it < maxit; ++it) {
        or_data_grad(g, y, w, z, gr);
        or_reg_grad(g->nx, g->ny, z, kind, delta, beta, 1, grr, NULL);
        double dot = 0.0;
        for (size_t j = 0; j < npix; ++j) {
            double gz = gr[j] + grr[j];
            xo[j] = x[j];
            double xn = z[j] - pre[j] * gz;
            x[j] = xn > 0.0 ? xn : 0.0;
            dot += gz * (x[j] - xo[j]);
        }
        double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tk * tk));
        if (dot > 0.0) { /* gradient restart */
            tn = 1.0;
            for (size_t j = 0; j < npix; ++j) z[j] = x[j];
        } else {
            double mom = (tk - 1.0) / tn;
            for (size_t j = 0; j < npix; ++j) z[j] = x[j] + mom * (x[j] - xo[j]);
        }
        tk = tn;
        if ((it + 1) % 100 == 0) {
            /* KKT residual of the constrained problem at x: || min(x, grad Psi(x)) || / ||grad L(0)|| */
            or_data_grad(g, y, w, x, gr);
            or_reg_grad(g->nx, g->ny, x, kind, delta, beta, 1, grr, NULL);
            double acc = 0.0, chg = 0.0;
            for (size_t j = 0; j < npix; ++j) {
                double gg = gr[j] + grr[j];
                double m = x[j] < gg ? x[j] : gg;
                acc += m * m;
                double d = x[j] - x100[j];
                chg += d * d;
                x100[j] = x[j];
            }
            kkt = g0 > 0.0 ? sqrt(acc) / g0 : sqrt(acc);
            double chg_rms = sqrt(chg / (double)npix);
            if (chg_rms < step_tol && kkt < kkt_tol) { ++it; break; }
        }
    }
    if (kkt_out) *kkt_out = kkt;
    free(dl); free(pre); free(gr); free(grr); free(dmax); free(z); free(xo); free(x100);
    return it;
}

/* ------------------------------------------------------------------------------------------------ */
/* FBP-like start: ramp-filtered, fan-weighted, pixel-driven back-projection (flat detector).        */
/* Per view: cosine pre-weight dsd/sqrt(dsd^2 + u^2) on data magnified to the isocentre, spatial     */
/* Ram-Lak filter, then linear-interpolated pixel-driven back-projection with distance weight        */
/* (dso / L)^2, where L is the source-to-pixel distance along the central ray. Clipped at 0.         */
/* ------------------------------------------------------------------------------------------------ */

void or_fbp(const or_geom *g, const double *y, double *x)
{
    int nb = g->nb;
    double dui = g->du * g->dso / g->dsd; /* bin width magnified to the isocentre */
    size_t npix = (size_t)g->nx * g->ny;
    memset(x, 0, sizeof(double) * npix);
    double *q = (double *)malloc(sizeof(double) * (size_t)g->nviews * nb);
    /* Ram-Lak kernel on the isocentre grid: h[0] = 1/(4 d^2), h[n odd] = -1/(pi n d)^2, else 0 */
    for (int v = 0; v < g->nviews; ++v) {
        double *qv = q + (size_t)v * nb;
        const double *yv = y + (size_t)v * nb;
        for (int k = 0; k < nb; ++k) {
            double acc = 0.0;
            for (int k2 = 0; k2 < nb; ++k2) {
                int n = k - k2;
                double hk;
                if (n == 0) hk = 1.0 / (4.0 * dui * dui);
                else if (n & 1) hk = -1.0 / ((OR_PI * n * dui) * (OR_PI * n * dui));
                else hk = 0.0;
                double u2 = ((double)k2 + 0.5 - 0.5 * nb + g->u_offset) * dui;
                double cw = g->dso / sqrt(g->dso * g->dso + u2 * u2);
                acc += hk * cw * yv[k2];
            }
            qv[k] = acc * dui;
        }
    }
    double dbeta = g->span / (double)g->nviews;
    /* full scan: each ray is measured twice, hence the 1/2 */
    double fac = 0.5 * dbeta;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < g->ny; ++i)
        for (int j = 0; j < g->nx; ++j) {
            double px = ((double)j - 0.5 * (g->nx - 1)) * g->dx;
            double py = ((double)i - 0.5 * (g->ny - 1)) * g->dy;
            double acc = 0.0;
            for (int v = 0; v < g->nviews; ++v) {
                double beta = g->beta0 + g->span * (double)v / (double)g->nviews;
                double c = cos(beta), s = sin(beta);
                double L = g->dso + px * c + py * s;      /* distance source->pixel along d */
                double t = -px * s + py * c;              /* along e */
                double u_iso = g->dso * t / L;            /* magnified to isocentre */
                double kf = u_iso / dui + 0.5 * nb - g->u_offset - 0.5;
                int k0 = (int)floor(kf);
                double f = kf - k0;
                if (k0 < 0 || k0 + 1 >= nb) continue;
                const double *qv = q + (size_t)v * nb;
                double val = (1.0 - f) * qv[k0] + f * qv[k0 + 1];
                acc += val * (g->dso / L) * (g->dso / L);
            }
            double xv = fac * acc;
            x[(size_t)i * g->nx + j] = xv > 0.0 ? xv : 0.0;
        }
    free(q);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP regions that follow (timing legs). Results do not depend on it: every parallel loop
   writes disjoint outputs and none reduces across threads. */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
