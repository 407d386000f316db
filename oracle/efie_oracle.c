/*
 * efie_oracle.c -- CPU FP64 reference ("oracle") for the isogeometric EFIE
 * Galerkin operator and its interpolation-based fast multipole compression.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source with
 * the HIP library: geometry is evaluated by the Cox-de Boor recursion (not Bezier
 * extraction), the glued spline basis is evaluated directly (no superspace, no
 * transformation matrix), far-field blocks are formed literally as the K_1^(a,b)
 * and K_2 matrices, and cluster moments are integrated directly on every level
 * (no transfer matrices).
 *
 * Paper map (Doelz, Kurz, Schoeps, Wolf, "Isogeometric boundary elements in
 * electromagnetism: rigorous analysis, fast methods, and examples"):
 *   - B-spline recursion ........................ Sec. 3.1, Definition (B-Splines)
 *   - NURBS patch map F_j ....................... Sec. 3.1, eq. (def::geom)
 *   - Piola pull-back, surface divergence ....... Sec. 3.2 (iota_1, iota_2)
 *   - div-conforming space S^1 .................. Sec. 3.2 (spline complex)
 *   - Helmholtz kernel .......................... Sec. 2.2, eq. (eq:HelmholtzGreen)
 *   - Galerkin matrix ........................... Sec. 3.2, eq. (eq:MSLtested),
 *                                                 pulled back per Sec. 4.1, eq. (eq:Vkh)
 *   - localized kernel, interpolation, K_1, K_2,
 *     moment matrices M, M^d ..................... Sec. 4.2 (eq:lockernel, eq:twomatrices,
 *                                                 eq:FMMlr)
 *   - potential (representation formula) ........ Sec. 2.2, eq. (eq:ESLP)
 *
 * Everything is in patch-parameter coordinates u in [0,1]^2 of each patch; with
 * the Piola map, phi dsigma = dF phi_hat du and div_G phi dsigma = div phi_hat du,
 * so the surface measure tau cancels from both bilinear-form terms.
 *
 * Element-pair quadrature (the paper cites standard BEM rules without fixing one):
 *   disjoint pairs  : tensor Gauss-Legendre, g points per parameter direction;
 *   identical pairs : relative-coordinate split per direction (w = |x_k - y_k|),
 *                     Duffy split of the (w1,w2) square into two triangles;
 *   common edge     : relative split along the edge, Duffy split of the
 *                     (distance-to-edge, distance-to-edge, w) cube into 3 pyramids;
 *   common vertex   : Duffy split of the 4-cube into 4 pyramids at the vertex;
 * each sub-rule is a tensor Gauss rule with gs points in each of its 4 variables.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define MAXDEG 4          /* max discretisation degree p */
#define MAXQ 16           /* max interpolation degree q */
#define MAXLEV 10         /* max cluster-tree level */
#define MAXLOC 40         /* max local glued functions on one element: 2 p (p+1), p <= 4 */
#define MAXG 24           /* max Gauss points per direction */

/* ------------------------------------------------------------------------- */
/* problem description                                                       */
/* ------------------------------------------------------------------------- */
typedef struct {
    int pu, pv, nu, nv;
    const double *ku, *kv;     /* knot vectors (copied) */
    const double *ctrl;        /* [nv][nu][4] (x,y,z,w) */
    int exact;                 /* 1: exact sphere map b(u,v)/|b(u,v)| instead of the NURBS */
    double V[4][3];            /* b = bilinear interpolation of these cube vertices (corners 00, 10, 01, 11) */
} patch_t;

typedef struct {
    int P;
    patch_t *pat;
    double *store;             /* owns the copied knots and control points */
    int p, m, n;               /* discretisation degree, level, n = 2^m elements per direction */
    int N;                     /* glued unknowns */
    int nb;                    /* n + p : padded 1-D index range of the DOF table */
    int32_t *dof;              /* [P][2][nb][nb] global index (i2 major, i1 minor), -1 = none */
    int8_t *sgn;               /* same layout, +-1 */
    double *kd, *kd1;          /* uniform p-open knot vectors: degree p (n+2p+1), degree p-1 (n+2p-1) */
    double kappa;
    int g, gs;                 /* regular / singular Gauss orders */
    int kernel;                /* 0 Helmholtz, 1 polynomial test kernel */
    int scalar;                /* 1: scalar single layer (patchwise tensor B-splines of degree p,
                                  A_ij = int int G phi_j phi_i, Sec. 4.2), 0: the EFIE */
    double gx[MAXG], gw[MAXG], sx[MAXG], sw[MAXG];
    double scale;              /* geometry size for vertex matching */
    int nthreads;
} ctx_t;

static int nloc(const void *cv)
{
    const ctx_t *c = (const ctx_t *)cv;
    return c->scalar ? (c->p + 1) * (c->p + 1) : 2 * c->p * (c->p + 1);
}
static double dcoef(const void *cv)
{
    const ctx_t *c = (const ctx_t *)cv;
    return c->scalar ? 1.0 : -1.0 / (c->kappa * c->kappa);
}

/* ------------------------------------------------------------------------- */
/* Gauss-Legendre rule on [0,1] by Newton iteration on the Legendre recurrence */
/* ------------------------------------------------------------------------- */
int or_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1 || n > 64) return -1;
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {   /* recompute derivative at the converged root */
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        /* map from [-1,1] to [0,1]; ascending order */
        x[n - 1 - i] = 0.5 * (1.0 + z);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);   /* = 2/((1-z^2)P'^2) / 2 */
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* B-splines: the recursion of Definition (B-Splines), all functions at once  */
/* ------------------------------------------------------------------------- */
/* knots: nk entries, degree p -> nk-p-1 functions.  val/der sized nk-p-1.
 * Half-open indicator intervals; at the right end point the last non-empty
 * interval is taken closed so that the basis is a partition of unity on [0,1]. */
static void bspline_all(int p, const double *knots, int nk, double x, double *val, double *der)
{
    double tab[2][512];
    int nint = nk - 1;
    int last = -1;
    for (int j = 0; j < nint; ++j) if (knots[j] < knots[j + 1]) last = j;
    for (int j = 0; j < nint; ++j) {
        int in = (knots[j] <= x && x < knots[j + 1]);
        if (j == last && x >= knots[j + 1]) in = 1;
        tab[0][j] = in ? 1.0 : 0.0;
    }
    double *prev = tab[0], *cur = tab[1];
    double lower[512];
    for (int k = 1; k <= p; ++k) {
        int nf = nk - k - 1;
        for (int j = 0; j < nf; ++j) {
            double a = 0.0, b = 0.0;
            double d1 = knots[j + k] - knots[j], d2 = knots[j + k + 1] - knots[j + 1];
            if (d1 > 0.0) a = (x - knots[j]) / d1 * prev[j];
            if (d2 > 0.0) b = (knots[j + k + 1] - x) / d2 * prev[j + 1];
            cur[j] = a + b;
        }
        if (k == p) memcpy(lower, prev, sizeof(double) * (nk - k));
        double *t = prev; prev = cur; cur = t;
    }
    int nf = nk - p - 1;
    for (int j = 0; j < nf; ++j) val[j] = prev[j];
    if (der) {
        if (p == 0) { for (int j = 0; j < nf; ++j) der[j] = 0.0; return; }
        for (int j = 0; j < nf; ++j) {
            double a = 0.0, b = 0.0;
            double d1 = knots[j + p] - knots[j], d2 = knots[j + p + 1] - knots[j + 1];
            if (d1 > 0.0) a = p / d1 * lower[j];
            if (d2 > 0.0) b = p / d2 * lower[j + 1];
            der[j] = a - b;
        }
    }
}

/* The p+1 B-splines b_{span-p..span} that are nonzero on the knot span
 * [knots[span], knots[span+1]), evaluated as the polynomial piece of that span
 * (the same recursion with the degree-0 indicator fixed to that span).  Used for
 * element-local evaluation, so points on an element boundary take the element's
 * own piece. */
static void bspline_piece(int p, const double *knots, int span, double x, double *val, double *der)
{
    double tab[MAXDEG + 2][MAXDEG + 2];
    tab[0][0] = 1.0;
    for (int k = 1; k <= p; ++k) {
        for (int i = 0; i <= k; ++i) {
            int j = span - k + i;
            double a = 0.0, b = 0.0;
            if (i >= 1) {                     /* b_j^{k-1} */
                double d1 = knots[j + k] - knots[j];
                if (d1 > 0.0) a = (x - knots[j]) / d1 * tab[k - 1][i - 1];
            }
            if (i <= k - 1) {                 /* b_{j+1}^{k-1} */
                double d2 = knots[j + k + 1] - knots[j + 1];
                if (d2 > 0.0) b = (knots[j + k + 1] - x) / d2 * tab[k - 1][i];
            }
            tab[k][i] = a + b;
        }
    }
    for (int i = 0; i <= p; ++i) val[i] = tab[p][i];
    if (der) {
        for (int i = 0; i <= p; ++i) {
            if (p == 0) { der[i] = 0.0; continue; }
            int j = span - p + i;
            double a = 0.0, b = 0.0;
            if (i >= 1) {
                double d1 = knots[j + p] - knots[j];
                if (d1 > 0.0) a = p / d1 * tab[p - 1][i - 1];
            }
            if (i <= p - 1) {
                double d2 = knots[j + p + 1] - knots[j + 1];
                if (d2 > 0.0) b = p / d2 * tab[p - 1][i];
            }
            der[i] = a - b;
        }
    }
}

/* exported for the pins */
int or_bspline_eval(int p, const double *knots, int nk, int npts, const double *x, double *val, double *der)
{
    int nf = nk - p - 1;
    if (nk > 500 || p < 0 || nf < 1) return -1;
    for (int i = 0; i < npts; ++i)
        bspline_all(p, knots, nk, x[i], val + (size_t)i * nf, der ? der + (size_t)i * nf : NULL);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* NURBS patch map F_j and its parameter derivatives                          */
/* ------------------------------------------------------------------------- */
static void patch_eval(const patch_t *pt, double u, double v, double F[3], double Fu[3], double Fv[3])
{
    if (pt->exact) {
        /* radial projection of the bilinear cube face onto the unit sphere:
         * F = b / |b|, dF = (db - F (F . db)) / |b| */
        double b[3], bu_[3], bv_[3];
        for (int k = 0; k < 3; ++k) {
            b[k] = (1 - u) * (1 - v) * pt->V[0][k] + u * (1 - v) * pt->V[1][k] + (1 - u) * v * pt->V[2][k] +
                   u * v * pt->V[3][k];
            bu_[k] = -(1 - v) * pt->V[0][k] + (1 - v) * pt->V[1][k] - v * pt->V[2][k] + v * pt->V[3][k];
            bv_[k] = -(1 - u) * pt->V[0][k] - u * pt->V[1][k] + (1 - u) * pt->V[2][k] + u * pt->V[3][k];
        }
        const double nb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        for (int k = 0; k < 3; ++k) F[k] = b[k] / nb;
        const double fu = F[0] * bu_[0] + F[1] * bu_[1] + F[2] * bu_[2];
        const double fv = F[0] * bv_[0] + F[1] * bv_[1] + F[2] * bv_[2];
        for (int k = 0; k < 3; ++k) {
            if (Fu) Fu[k] = (bu_[k] - F[k] * fu) / nb;
            if (Fv) Fv[k] = (bv_[k] - F[k] * fv) / nb;
        }
        return;
    }
    double bu[512], du[512], bv[512], dv[512];
    bspline_all(pt->pu, pt->ku, pt->nu + pt->pu + 1, u, bu, du);
    bspline_all(pt->pv, pt->kv, pt->nv + pt->pv + 1, v, bv, dv);
    double A[4] = {0, 0, 0, 0}, Au[4] = {0, 0, 0, 0}, Av[4] = {0, 0, 0, 0};
    for (int j2 = 0; j2 < pt->nv; ++j2) {
        if (bv[j2] == 0.0 && dv[j2] == 0.0) continue;
        for (int j1 = 0; j1 < pt->nu; ++j1) {
            if (bu[j1] == 0.0 && du[j1] == 0.0) continue;
            const double *c = pt->ctrl + ((size_t)j2 * pt->nu + j1) * 4;
            double w = c[3];
            double B = bu[j1] * bv[j2], Bu = du[j1] * bv[j2], Bv = bu[j1] * dv[j2];
            for (int k = 0; k < 3; ++k) {
                A[k] += B * w * c[k]; Au[k] += Bu * w * c[k]; Av[k] += Bv * w * c[k];
            }
            A[3] += B * w; Au[3] += Bu * w; Av[3] += Bv * w;
        }
    }
    for (int k = 0; k < 3; ++k) {
        double f = A[k] / A[3];
        F[k] = f;
        if (Fu) Fu[k] = (Au[k] - f * Au[3]) / A[3];
        if (Fv) Fv[k] = (Av[k] - f * Av[3]) / A[3];
    }
}

/* ------------------------------------------------------------------------- */
/* context                                                                    */
/* ------------------------------------------------------------------------- */
void *or_create(int P, const int32_t *deg, const int32_t *nctrl, const double *knots, const double *ctrl,
                int p, int m, int N, const int32_t *dof, const int8_t *sgn,
                double kappa, int g, int gs, int kernel)
{
    if (P < 1 || p < 1 || p > MAXDEG || m < 0 || m > 12 || g < 1 || g > MAXG || gs < 1 || gs > MAXG)
        return NULL;
    ctx_t *c = (ctx_t *)calloc(1, sizeof(ctx_t));
    c->P = P; c->p = p; c->m = m; c->n = 1 << m; c->N = N; c->nb = c->n + p;
    c->kappa = kappa; c->g = g; c->gs = gs; c->kernel = kernel;
    size_t nkn = 0, nct = 0;
    for (int j = 0; j < P; ++j) {
        nkn += (size_t)(nctrl[2 * j] + deg[2 * j] + 1) + (nctrl[2 * j + 1] + deg[2 * j + 1] + 1);
        nct += (size_t)nctrl[2 * j] * nctrl[2 * j + 1] * 4;
    }
    c->store = (double *)malloc(sizeof(double) * (nkn + nct));
    memcpy(c->store, knots, sizeof(double) * nkn);
    memcpy(c->store + nkn, ctrl, sizeof(double) * nct);
    c->pat = (patch_t *)calloc(P, sizeof(patch_t));
    size_t ok = 0, oc = nkn;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int j = 0; j < P; ++j) {
        patch_t *pt = &c->pat[j];
        pt->pu = deg[2 * j]; pt->pv = deg[2 * j + 1];
        pt->nu = nctrl[2 * j]; pt->nv = nctrl[2 * j + 1];
        pt->ku = c->store + ok; ok += pt->nu + pt->pu + 1;
        pt->kv = c->store + ok; ok += pt->nv + pt->pv + 1;
        pt->ctrl = c->store + oc; oc += (size_t)pt->nu * pt->nv * 4;
        for (int i = 0; i < pt->nu * pt->nv; ++i)
            for (int k = 0; k < 3; ++k) {
                double x = pt->ctrl[4 * i + k];
                if (x < lo[k]) lo[k] = x;
                if (x > hi[k]) hi[k] = x;
            }
    }
    c->scale = fmax(hi[0] - lo[0], fmax(hi[1] - lo[1], hi[2] - lo[2]));
    size_t nd = (size_t)P * 2 * c->nb * c->nb;
    c->dof = (int32_t *)malloc(sizeof(int32_t) * nd);
    c->sgn = (int8_t *)malloc(nd);
    memcpy(c->dof, dof, sizeof(int32_t) * nd);
    memcpy(c->sgn, sgn, nd);
    int n = c->n;
    c->kd = (double *)malloc(sizeof(double) * (n + 2 * p + 1));
    c->kd1 = (double *)malloc(sizeof(double) * (n + 2 * p - 1));
    for (int i = 0; i <= p; ++i) { c->kd[i] = 0.0; c->kd[n + p + i] = 1.0; }
    for (int i = 1; i < n; ++i) c->kd[p + i] = (double)i / n;
    for (int i = 0; i < p; ++i) { c->kd1[i] = 0.0; c->kd1[n + p - 1 + i] = 1.0; }
    for (int i = 1; i < n; ++i) c->kd1[p - 1 + i] = (double)i / n;
    or_gauss_legendre(g, c->gx, c->gw);
    or_gauss_legendre(gs, c->sx, c->sw);
#ifdef _OPENMP
    c->nthreads = omp_get_max_threads();
#else
    c->nthreads = 1;
#endif
    return c;
}

void or_destroy(void *h)
{
    ctx_t *c = (ctx_t *)h;
    if (!c) return;
    free(c->store); free(c->pat); free(c->dof); free(c->sgn); free(c->kd); free(c->kd1); free(c);
}

/* Replace every patch map by the exact unit sphere: each patch's corners (from its
 * NURBS map, on the unit sphere) are scaled onto the circumscribed cube, and the
 * bilinear face through them is projected radially.  For the six-patch cube-sphere
 * this is the analytic cube-sphere map, with the same corners and orientation. */
int or_set_scalar(void *h)
{
    ((ctx_t *)h)->scalar = 1;
    return 0;
}

int or_set_exact_sphere(void *h)
{
    ctx_t *c = (ctx_t *)h;
    if (!c) return -1;
    static const double cu[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
    for (int j = 0; j < c->P; ++j) {
        patch_t *pt = &c->pat[j];
        for (int k = 0; k < 4; ++k) {
            double F[3];
            patch_eval(pt, cu[k][0], cu[k][1], F, NULL, NULL);
            const double a = fmax(fabs(F[0]), fmax(fabs(F[1]), fabs(F[2])));
            for (int d = 0; d < 3; ++d) pt->V[k][d] = F[d] / a;
        }
        pt->exact = 1;
    }
    return 0;
}

int or_geom_eval(void *h, int j, int npts, const double *uv, double *out /* [npts][9] F,Fu,Fv */)
{
    ctx_t *c = (ctx_t *)h;
    if (j < 0 || j >= c->P) return -1;
    for (int i = 0; i < npts; ++i)
        patch_eval(&c->pat[j], uv[2 * i], uv[2 * i + 1], out + 9 * i, out + 9 * i + 3, out + 9 * i + 6);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* local glued basis on one element                                          */
/* ------------------------------------------------------------------------- */
/* Local function order on element (e1,e2): component 0 (u-flux, degree (p,p-1)):
 * i2 = e2..e2+p-1 (major), i1 = e1..e1+p (minor); then component 1 (degree (p-1,p)):
 * i2 = e2..e2+p, i1 = e1..e1+p-1. */


typedef struct {
    int nl;
    int idx[MAXLOC];
    double sg[MAXLOC];
    int comp[MAXLOC];
} locmap_t;

static void local_map(const ctx_t *c, int j, int e1, int e2, locmap_t *L)
{
    int p = c->p, nb = c->nb, k = 0;
    if (c->scalar) {   /* tensor B-splines b_{e1+t1}(u) b_{e2+t2}(v), t2 major */
        for (int t2 = 0; t2 <= p; ++t2)
            for (int t1 = 0; t1 <= p; ++t1) {
                size_t o = (((size_t)j * 2) * nb + (e2 + t2)) * nb + (e1 + t1);
                L->idx[k] = c->dof[o];
                L->sg[k] = 1.0;
                L->comp[k] = 0;
                ++k;
            }
        L->nl = k;
        return;
    }
    for (int a = 0; a < 2; ++a) {
        int r1 = (a == 0) ? p + 1 : p, r2 = (a == 0) ? p : p + 1;
        for (int t2 = 0; t2 < r2; ++t2)
            for (int t1 = 0; t1 < r1; ++t1) {
                size_t o = (((size_t)j * 2 + a) * nb + (e2 + t2)) * nb + (e1 + t1);
                L->idx[k] = c->dof[o];
                L->sg[k] = (double)c->sgn[o];
                L->comp[k] = a;
                ++k;
            }
    }
    L->nl = k;
}

/* Values at patch point (u,v) on element (e1,e2) of patch j:
 *   Phi[l][0..2] = phi_hat_l^a * d_aF   (Cartesian Piola field times tau)
 *   D[l]         = div phi_hat_l        (patch-parameter divergence)
 * without the gluing sign; also returns F (point) if X != NULL. */
typedef struct {
    double X[3];
    double Phi[MAXLOC][3];
    double D[MAXLOC];
} pointval_t;

static void element_pieces(const ctx_t *c, int e1, int e2, double u, double v, double *bpu, double *dpu,
                           double *bqu, double *dqu, double *bpv, double *dpv, double *bqv, double *dqv)
{
    int p = c->p;
    /* element e spans knot interval e+p of the degree-p vector and e+p-1 of the degree-(p-1) one */
    bspline_piece(p, c->kd, e1 + p, u, bpu, dpu);
    bspline_piece(p - 1, c->kd1, e1 + p - 1, u, bqu, dqu);
    bspline_piece(p, c->kd, e2 + p, v, bpv, dpv);
    bspline_piece(p - 1, c->kd1, e2 + p - 1, v, bqv, dqv);
}

static void point_values(const ctx_t *c, int j, int e1, int e2, double u, double v, pointval_t *pv)
{
    int p = c->p;
    double Fu[3], Fv[3];
    patch_eval(&c->pat[j], u, v, pv->X, Fu, Fv);
    double bpu[MAXDEG + 1], dpu[MAXDEG + 1], bqu[MAXDEG + 1], dqu[MAXDEG + 1];
    double bpv[MAXDEG + 1], dpv[MAXDEG + 1], bqv[MAXDEG + 1], dqv[MAXDEG + 1];
    element_pieces(c, e1, e2, u, v, bpu, dpu, bqu, dqu, bpv, dpv, bqv, dqv);
    int k = 0;
    if (c->scalar) {   /* value times the surface element |d_uF x d_vF| in D, no field part */
        double nx = Fu[1] * Fv[2] - Fu[2] * Fv[1], ny = Fu[2] * Fv[0] - Fu[0] * Fv[2], nz = Fu[0] * Fv[1] - Fu[1] * Fv[0];
        double J = sqrt(nx * nx + ny * ny + nz * nz);
        for (int t2 = 0; t2 <= p; ++t2)
            for (int t1 = 0; t1 <= p; ++t1) {
                pv->Phi[k][0] = pv->Phi[k][1] = pv->Phi[k][2] = 0.0;
                pv->D[k] = bpu[t1] * bpv[t2] * J;
                ++k;
            }
        return;
    }
    for (int t2 = 0; t2 < p; ++t2)            /* component 0: b^p(u) b^{p-1}(v) */
        for (int t1 = 0; t1 <= p; ++t1) {
            double val = bpu[t1] * bqv[t2];
            double div = dpu[t1] * bqv[t2];
            for (int d = 0; d < 3; ++d) pv->Phi[k][d] = val * Fu[d];
            pv->D[k] = div;
            ++k;
        }
    for (int t2 = 0; t2 <= p; ++t2)           /* component 1: b^{p-1}(u) b^p(v) */
        for (int t1 = 0; t1 < p; ++t1) {
            double val = bqu[t1] * bpv[t2];
            double div = bqu[t1] * dpv[t2];
            for (int d = 0; d < 3; ++d) pv->Phi[k][d] = val * Fv[d];
            pv->D[k] = div;
            ++k;
        }
}

/* the discrete field x_h = sum_i x_i phi_i at patch points: parameter components
 * (phi_hat^1, phi_hat^2) and the divergence, for the flux-continuity pin */
int or_field_param(void *h, const double *xin, int j, int npts, const double *uv, double *out /* [npts][3] cplx */)
{
    ctx_t *c = (ctx_t *)h;
    const cplx *x = (const cplx *)xin;
    cplx *o = (cplx *)out;
    int p = c->p, n = c->n;
    for (int i = 0; i < npts; ++i) {
        double u = uv[2 * i], v = uv[2 * i + 1];
        int e1 = (int)floor(u * n), e2 = (int)floor(v * n);
        if (e1 >= n) e1 = n - 1;
        if (e2 >= n) e2 = n - 1;
        if (e1 < 0) e1 = 0;
        if (e2 < 0) e2 = 0;
        locmap_t L;
        local_map(c, j, e1, e2, &L);
        double bpu[MAXDEG + 1], dpu[MAXDEG + 1], bqu[MAXDEG + 1], dqu[MAXDEG + 1];
        double bpv[MAXDEG + 1], dpv[MAXDEG + 1], bqv[MAXDEG + 1], dqv[MAXDEG + 1];
        element_pieces(c, e1, e2, u, v, bpu, dpu, bqu, dqu, bpv, dpv, bqv, dqv);
        cplx a0 = 0, a1 = 0, dv = 0;
        int k = 0;
        for (int t2 = 0; t2 < p; ++t2)
            for (int t1 = 0; t1 <= p; ++t1, ++k) {
                cplx cf = L.sg[k] * x[L.idx[k]];
                a0 += cf * bpu[t1] * bqv[t2]; dv += cf * dpu[t1] * bqv[t2];
            }
        for (int t2 = 0; t2 <= p; ++t2)
            for (int t1 = 0; t1 < p; ++t1, ++k) {
                cplx cf = L.sg[k] * x[L.idx[k]];
                a1 += cf * bqu[t1] * bpv[t2]; dv += cf * bqu[t1] * dpv[t2];
            }
        o[3 * i] = a0; o[3 * i + 1] = a1; o[3 * i + 2] = dv;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* kernels                                                                    */
/* ------------------------------------------------------------------------- */
/* Helmholtz fundamental solution e^{i k r}/(4 pi r) (eq:HelmholtzGreen), or the
 * polynomial test kernel used to pin the far-field algebra: on affine patches it
 * is a polynomial of degree <= 4 in every parameter variable, so degree >= 4
 * interpolation reproduces it exactly; or 1/(4 pi r) (kernel 2, pins of the
 * singular rules). */
static cplx kernel_eval(const ctx_t *c, const double *x, const double *y)
{
    double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (c->kernel == 1) {
        double xy = x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
        double t = x[0] * y[1] - 0.3 * x[2] * y[2];
        return (1.0 + 0.5 * xy + 0.25 * r2 + t * t) + I * (0.2 - 0.1 * xy + 0.3 * r2 * r2);
    }
    double r = sqrt(r2);
    if (c->kernel == 2) return 1.0 / (4.0 * M_PI * r);
    return cexp(I * c->kappa * r) / (4.0 * M_PI * r);
}

/* ------------------------------------------------------------------------- */
/* element-pair quadrature                                                    */
/* ------------------------------------------------------------------------- */
typedef struct { double o[2], a1[2], a2[2]; } frame_t;   /* local = o + s1 a1 + s2 a2 */

static const double CORNER[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};

static void element_corners(const ctx_t *c, int j, int e1, int e2, double X[4][3])
{
    double h = 1.0 / c->n;
    for (int k = 0; k < 4; ++k)
        patch_eval(&c->pat[j], (e1 + CORNER[k][0]) * h, (e2 + CORNER[k][1]) * h, X[k], NULL, NULL);
}

/* shared corners: returns count; pairs (ti, si) of test/trial corner indices */
static int shared_corners(const ctx_t *c, double A[4][3], double B[4][3], int ti[4], int si[4])
{
    double tol = 1e-9 * c->scale;
    int ns = 0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            double d = fabs(A[a][0] - B[b][0]) + fabs(A[a][1] - B[b][1]) + fabs(A[a][2] - B[b][2]);
            if (d <= tol) { ti[ns] = a; si[ns] = b; ++ns; }
        }
    return ns;
}

/* the corner of the unit square adjacent to corner a that is not b */
static int other_neighbour(int a, int b)
{
    int n1 = (a + 1) & 3, n2 = (a + 3) & 3;
    return (n1 == b) ? n2 : n1;
}

static void frame_from(int o, int e2c, int e1c, frame_t *f)
{
    f->o[0] = CORNER[o][0]; f->o[1] = CORNER[o][1];
    f->a1[0] = CORNER[e1c][0] - CORNER[o][0]; f->a1[1] = CORNER[e1c][1] - CORNER[o][1];
    f->a2[0] = CORNER[e2c][0] - CORNER[o][0]; f->a2[1] = CORNER[e2c][1] - CORNER[o][1];
}

/* One element pair: B[l][l'] (nl x nl, unsigned local functions) of
 *   int_e int_e' k(F(u)-F(u')) [ Phi_l(u).Phi_l'(u') - kappa^-2 D_l(u) D_l'(u') ] du du'
 * which is eq:Vkh summed over (alpha,beta) for the glued functions' pieces on e, e'. */
typedef struct {
    int j, e1, e2;
} elem_t;

/* integrand accumulation at one point pair */
static void accum_point(const ctx_t *c, const pointval_t *A, const pointval_t *B, double w, int nl, cplx *blk)
{
    cplx kv = kernel_eval(c, A->X, B->X) * w;
    double cd = dcoef(c);
    for (int l = 0; l < nl; ++l) {
        for (int lp = 0; lp < nl; ++lp) {
            double g = A->Phi[l][0] * B->Phi[lp][0] + A->Phi[l][1] * B->Phi[lp][1] + A->Phi[l][2] * B->Phi[lp][2]
                       + cd * A->D[l] * B->D[lp];
            blk[l * nl + lp] += kv * g;
        }
    }
}

/* regular tensor rule, factorised over the test points:
 *   B = sum_q w_q sum_c Psi_l^c(q) ( sum_q' w_q' k(q,q') Psi_l'^c(q') ) */
static void pair_regular(const ctx_t *c, const pointval_t *TA, const pointval_t *TB, int nq, const double *wq,
                         int nl, cplx *blk)
{
    double cd = dcoef(c);
    cplx Z[MAXLOC][4];
    for (int q = 0; q < nq; ++q) {
        for (int l = 0; l < nl; ++l) Z[l][0] = Z[l][1] = Z[l][2] = Z[l][3] = 0.0;
        for (int qp = 0; qp < nq; ++qp) {
            cplx kv = kernel_eval(c, TA[q].X, TB[qp].X) * wq[qp];
            for (int l = 0; l < nl; ++l) {
                Z[l][0] += kv * TB[qp].Phi[l][0];
                Z[l][1] += kv * TB[qp].Phi[l][1];
                Z[l][2] += kv * TB[qp].Phi[l][2];
                Z[l][3] += kv * TB[qp].D[l];
            }
        }
        for (int l = 0; l < nl; ++l)
            for (int lp = 0; lp < nl; ++lp)
                blk[l * nl + lp] += wq[q] * (TA[q].Phi[l][0] * Z[lp][0] + TA[q].Phi[l][1] * Z[lp][1] +
                                             TA[q].Phi[l][2] * Z[lp][2] + cd * TA[q].D[l] * Z[lp][3]);
    }
}

/* element Gauss data for the regular rule */
static void element_gauss(const ctx_t *c, int j, int e1, int e2, pointval_t *T, double *wq)
{
    double h = 1.0 / c->n;
    int g = c->g, q = 0;
    for (int b = 0; b < g; ++b)
        for (int a = 0; a < g; ++a, ++q) {
            point_values(c, j, e1, e2, (e1 + c->gx[a]) * h, (e2 + c->gx[b]) * h, &T[q]);
            wq[q] = c->gw[a] * c->gw[b] * h * h;
        }
}

static void map_local(const frame_t *f, double s1, double s2, double *l)
{
    l[0] = f->o[0] + s1 * f->a1[0] + s2 * f->a2[0];
    l[1] = f->o[1] + s1 * f->a1[1] + s2 * f->a2[1];
}

/* evaluate a singular sub-rule point given canonical local coordinates */
static void sing_point(const ctx_t *c, const elem_t *E, const elem_t *Ep, const frame_t *fA, const frame_t *fB,
                       double s1, double s2, double t1, double t2, double w, int nl, cplx *blk)
{
    double h = 1.0 / c->n, la[2], lb[2];
    pointval_t A, B;
    map_local(fA, s1, s2, la);
    map_local(fB, t1, t2, lb);
    point_values(c, E->j, E->e1, E->e2, (E->e1 + la[0]) * h, (E->e2 + la[1]) * h, &A);
    point_values(c, Ep->j, Ep->e1, Ep->e2, (Ep->e1 + lb[0]) * h, (Ep->e2 + lb[1]) * h, &B);
    accum_point(c, &A, &B, w * h * h * h * h, nl, blk);
}

/* identical elements */
static void pair_identical(const ctx_t *c, const elem_t *E, int nl, cplx *blk)
{
    frame_t id = {{0, 0}, {1, 0}, {0, 1}};
    int gs = c->gs;
    const double *x = c->sx, *wg = c->sw;
    for (int tri = 0; tri < 2; ++tri)
        for (int sg1 = 0; sg1 < 2; ++sg1)
            for (int sg2 = 0; sg2 < 2; ++sg2)
                for (int a = 0; a < gs; ++a)
                    for (int b = 0; b < gs; ++b)
                        for (int cc = 0; cc < gs; ++cc)
                            for (int d = 0; d < gs; ++d) {
                                double xi = x[a], eta = x[b], t1 = x[cc], t2 = x[d];
                                double w1 = tri == 0 ? xi : xi * eta;
                                double w2 = tri == 0 ? xi * eta : xi;
                                double s1, s2, r1, r2;
                                if (sg1 == 0) { s1 = (1 - w1) * t1; r1 = s1 + w1; }
                                else { r1 = (1 - w1) * t1; s1 = r1 + w1; }
                                if (sg2 == 0) { s2 = (1 - w2) * t2; r2 = s2 + w2; }
                                else { r2 = (1 - w2) * t2; s2 = r2 + w2; }
                                double wt = wg[a] * wg[b] * wg[cc] * wg[d] * xi * (1 - w1) * (1 - w2);
                                sing_point(c, E, E, &id, &id, s1, s2, r1, r2, wt, nl, blk);
                            }
}

/* common edge; frames put the edge at s1 = 0 / t1 = 0 with matching s2 = t2 */
static void pair_edge(const ctx_t *c, const elem_t *E, const elem_t *Ep, const frame_t *fA, const frame_t *fB,
                      int nl, cplx *blk)
{
    int gs = c->gs;
    const double *x = c->sx, *wg = c->sw;
    for (int pyr = 0; pyr < 3; ++pyr)
        for (int sg = 0; sg < 2; ++sg)
            for (int a = 0; a < gs; ++a)
                for (int b = 0; b < gs; ++b)
                    for (int cc = 0; cc < gs; ++cc)
                        for (int d = 0; d < gs; ++d) {
                            double xi = x[a], e1 = x[b], e2 = x[cc], t = x[d];
                            double A, B, W;     /* distance of test / trial point to the edge, |s2 - t2| */
                            if (pyr == 0) { A = xi; B = xi * e1; W = xi * e2; }
                            else if (pyr == 1) { B = xi; A = xi * e1; W = xi * e2; }
                            else { W = xi; A = xi * e1; B = xi * e2; }
                            double s2, t2;
                            if (sg == 0) { s2 = (1 - W) * t; t2 = s2 + W; }
                            else { t2 = (1 - W) * t; s2 = t2 + W; }
                            double wt = wg[a] * wg[b] * wg[cc] * wg[d] * xi * xi * (1 - W);
                            sing_point(c, E, Ep, fA, fB, A, s2, B, t2, wt, nl, blk);
                        }
}

/* common vertex; frames put the vertex at the origin of both elements */
static void pair_vertex(const ctx_t *c, const elem_t *E, const elem_t *Ep, const frame_t *fA, const frame_t *fB,
                        int nl, cplx *blk)
{
    int gs = c->gs;
    const double *x = c->sx, *wg = c->sw;
    for (int pyr = 0; pyr < 4; ++pyr)
        for (int a = 0; a < gs; ++a)
            for (int b = 0; b < gs; ++b)
                for (int cc = 0; cc < gs; ++cc)
                    for (int d = 0; d < gs; ++d) {
                        double xi = x[a], z[4], rest[3] = {xi * x[b], xi * x[cc], xi * x[d]};
                        int k = 0;
                        for (int i = 0; i < 4; ++i) z[i] = (i == pyr) ? xi : rest[k++];
                        double wt = wg[a] * wg[b] * wg[cc] * wg[d] * xi * xi * xi;
                        sing_point(c, E, Ep, fA, fB, z[0], z[1], z[2], z[3], wt, nl, blk);
                    }
}

/* classify and integrate one element pair; TA/TB/wq: Gauss data of the two elements */
static void element_pair(const ctx_t *c, const elem_t *E, const elem_t *Ep, const pointval_t *TA,
                         const pointval_t *TB, const double *wq, double CA[4][3], double CB[4][3], cplx *blk)
{
    int nl = nloc(c);
    memset(blk, 0, sizeof(cplx) * nl * nl);
    int ti[4], si[4];
    int ns = shared_corners(c, CA, CB, ti, si);
    if (ns == 0) {
        pair_regular(c, TA, TB, c->g * c->g, wq, nl, blk);
    } else if (ns == 4) {
        pair_identical(c, E, nl, blk);
    } else if (ns == 2 && (((ti[0] - ti[1]) & 3) != 2) && (((si[0] - si[1]) & 3) != 2)) {
        frame_t fA, fB;
        /* test: origin at shared corner ti[0], a2 towards ti[1], a1 to the other neighbour */
        frame_from(ti[0], ti[1], other_neighbour(ti[0], ti[1]), &fA);
        frame_from(si[0], si[1], other_neighbour(si[0], si[1]), &fB);
        pair_edge(c, E, Ep, &fA, &fB, nl, blk);
    } else if (ns == 1) {
        frame_t fA, fB;
        frame_from(ti[0], (ti[0] + 3) & 3, (ti[0] + 1) & 3, &fA);
        frame_from(si[0], (si[0] + 3) & 3, (si[0] + 1) & 3, &fB);
        pair_vertex(c, E, Ep, &fA, &fB, nl, blk);
    } else {
        /* 3 shared corners cannot happen for a valid conforming mesh */
        pair_regular(c, TA, TB, c->g * c->g, wq, nl, blk);
    }
}

/* exported: one element-pair block (for pins); blk is nl*nl complex (re,im) */
int or_element_pair(void *h, int j, int e1, int e2, int jp, int f1, int f2, double *blk_out)
{
    ctx_t *c = (ctx_t *)h;
    int ng = c->g * c->g, nl = nloc(c);
    pointval_t *TA = (pointval_t *)malloc(sizeof(pointval_t) * ng);
    pointval_t *TB = (pointval_t *)malloc(sizeof(pointval_t) * ng);
    double *wq = (double *)malloc(sizeof(double) * ng);
    elem_t E = {j, e1, e2}, Ep = {jp, f1, f2};
    element_gauss(c, j, e1, e2, TA, wq);
    element_gauss(c, jp, f1, f2, TB, wq);
    double CA[4][3], CB[4][3];
    element_corners(c, j, e1, e2, CA);
    element_corners(c, jp, f1, f2, CB);
    cplx *blk = (cplx *)malloc(sizeof(cplx) * nl * nl);
    element_pair(c, &E, &Ep, TA, TB, wq, CA, CB, blk);
    memcpy(blk_out, blk, sizeof(cplx) * nl * nl);
    free(blk); free(TA); free(TB); free(wq);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* per-element cache of Gauss data and corners                               */
/* ------------------------------------------------------------------------- */
typedef struct {
    int E;
    pointval_t *T;   /* [E][g*g] */
    double *w;       /* [g*g] weights (same for all elements) */
    double (*C)[4][3];
} ecache_t;

static void ecache_build(const ctx_t *c, ecache_t *ec, const uint8_t *need)
{
    int n = c->n, ng = c->g * c->g;
    ec->E = c->P * n * n;
    ec->T = (pointval_t *)malloc(sizeof(pointval_t) * (size_t)ec->E * ng);
    ec->w = (double *)malloc(sizeof(double) * ng);
    ec->C = malloc(sizeof(double[4][3]) * ec->E);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < ec->E; ++e) {
        int j = e / (n * n), r = e % (n * n), e2 = r / n, e1 = r % n;
        element_corners(c, j, e1, e2, ec->C[e]);
        if (need && !need[e]) continue;
        double wq[MAXG * MAXG];
        element_gauss(c, j, e1, e2, ec->T + (size_t)e * ng, wq);
    }
    /* weights are element independent */
    {
        double h = 1.0 / c->n;
        int q = 0;
        for (int b = 0; b < c->g; ++b)
            for (int a = 0; a < c->g; ++a, ++q) ec->w[q] = c->gw[a] * c->gw[b] * h * h;
    }
}

static void ecache_free(ecache_t *ec) { free(ec->T); free(ec->w); free(ec->C); }

/* ------------------------------------------------------------------------- */
/* dense operator                                                             */
/* ------------------------------------------------------------------------- */
/* A_ij for all i,j (eq:MSLtested with the element rule), row-major N x N complex */
int or_dense_matrix(void *h, double *Aout)
{
    ctx_t *c = (ctx_t *)h;
    int n = c->n, E = c->P * n * n, nl = nloc(c), ng = c->g * c->g;
    ecache_t ec;
    ecache_build(c, &ec, NULL);
    cplx *A = (cplx *)Aout;
    memset(A, 0, sizeof(cplx) * (size_t)c->N * c->N);
#pragma omp parallel
    {
        cplx *blk = (cplx *)malloc(sizeof(cplx) * nl * nl);
#pragma omp for schedule(dynamic, 1)
        for (int e = 0; e < E; ++e) {
            elem_t Ee = {e / (n * n), (e % (n * n)) % n, (e % (n * n)) / n};
            locmap_t La;
            local_map(c, Ee.j, Ee.e1, Ee.e2, &La);
            for (int f = 0; f < E; ++f) {
                elem_t Ef = {f / (n * n), (f % (n * n)) % n, (f % (n * n)) / n};
                locmap_t Lb;
                local_map(c, Ef.j, Ef.e1, Ef.e2, &Lb);
                element_pair(c, &Ee, &Ef, ec.T + (size_t)e * ng, ec.T + (size_t)f * ng, ec.w, ec.C[e], ec.C[f], blk);
                for (int l = 0; l < nl; ++l)
                    for (int lp = 0; lp < nl; ++lp) {
                        cplx v = La.sg[l] * Lb.sg[lp] * blk[l * nl + lp];
                        double *dst = (double *)&A[(size_t)La.idx[l] * c->N + Lb.idx[lp]];
#pragma omp atomic
                        dst[0] += creal(v);
#pragma omp atomic
                        dst[1] += cimag(v);
                    }
            }
        }
        free(blk);
    }
    ecache_free(&ec);
    return 0;
}

/* y = A x restricted to test elements with tmask[e] != 0 (all if tmask == NULL);
 * only rows whose full support is masked are complete. */
int or_dense_apply(void *h, const double *xin, double *yout, const uint8_t *tmask)
{
    ctx_t *c = (ctx_t *)h;
    int n = c->n, E = c->P * n * n, nl = nloc(c), ng = c->g * c->g;
    const cplx *x = (const cplx *)xin;
    ecache_t ec;
    ecache_build(c, &ec, NULL);
    int nt = c->nthreads;
    cplx *ybuf = (cplx *)calloc((size_t)nt * c->N, sizeof(cplx));
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cplx *yl = ybuf + (size_t)tid * c->N;
        cplx *blk = (cplx *)malloc(sizeof(cplx) * nl * nl);
#pragma omp for schedule(static)
        for (int e = 0; e < E; ++e) {
            if (tmask && !tmask[e]) continue;
            elem_t Ee = {e / (n * n), (e % (n * n)) % n, (e % (n * n)) / n};
            locmap_t La;
            local_map(c, Ee.j, Ee.e1, Ee.e2, &La);
            for (int f = 0; f < E; ++f) {
                elem_t Ef = {f / (n * n), (f % (n * n)) % n, (f % (n * n)) / n};
                locmap_t Lb;
                local_map(c, Ef.j, Ef.e1, Ef.e2, &Lb);
                element_pair(c, &Ee, &Ef, ec.T + (size_t)e * ng, ec.T + (size_t)f * ng, ec.w, ec.C[e], ec.C[f], blk);
                for (int l = 0; l < nl; ++l) {
                    cplx s = 0;
                    for (int lp = 0; lp < nl; ++lp) s += Lb.sg[lp] * blk[l * nl + lp] * x[Lb.idx[lp]];
                    yl[La.idx[l]] += La.sg[l] * s;
                }
            }
        }
        free(blk);
    }
    cplx *y = (cplx *)yout;
    for (int i = 0; i < c->N; ++i) {
        cplx s = 0;
        for (int t = 0; t < nt; ++t) s += ybuf[(size_t)t * c->N + i];
        y[i] = s;
    }
    free(ybuf);
    ecache_free(&ec);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* right-hand side  f_i = - int_Gamma e_inc . phi_i dsigma                   */
/* ------------------------------------------------------------------------- */
/* kind 0: plane wave  pol * exp(i kappa dir.x)         (par = dir[3], pol re[3], pol im[3])
 * kind 1: Hertz dipole field DP_{x0} with moment p0     (par = x0[3], p0[3])
 * (Sec. 5.2, Definition (Hertz-Dipole)) */
static void field_eval(const ctx_t *c, int kind, const double *par, const double *x, cplx E[3])
{
    double k = c->kappa;
    if (kind == 0) {
        double ph = k * (par[0] * x[0] + par[1] * x[1] + par[2] * x[2]);
        cplx e = cexp(I * ph);
        for (int d = 0; d < 3; ++d) E[d] = (par[3 + d] + I * par[6 + d]) * e;
    } else {
        double rv[3] = {x[0] - par[0], x[1] - par[1], x[2] - par[2]};
        double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
        double nn[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
        const double *p0 = par + 3;
        /* (n x p0) x n = p0 - n (n.p0) */
        double np = nn[0] * p0[0] + nn[1] * p0[1] + nn[2] * p0[2];
        cplx e = cexp(I * k * r);
        for (int d = 0; d < 3; ++d) {
            double t1 = p0[d] - nn[d] * np;
            double t2 = 3.0 * nn[d] * np - p0[d];
            E[d] = e * (k * k / r * t1 + (1.0 / (r * r * r) - I * k / (r * r)) * t2);
        }
    }
}

/* scalar Dirichlet data g for the single layer (V w = g):
 * kind 2: point source G(x - x0) = e^{i kappa r} / (4 pi r)   (par = x0[3])
 * kind 3: plane wave exp(i kappa dir.x)                       (par = dir[3])
 * kind 4: the constant 1 */
static cplx scalar_field(const ctx_t *c, int kind, const double *par, const double *x)
{
    if (kind == 2) {
        double rv[3] = {x[0] - par[0], x[1] - par[1], x[2] - par[2]};
        double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
        return cexp(I * c->kappa * r) / (4.0 * M_PI * r);
    }
    if (kind == 3) return cexp(I * c->kappa * (par[0] * x[0] + par[1] * x[1] + par[2] * x[2]));
    return 1.0;
}

int or_rhs(void *h, int kind, const double *par, double *fout)
{
    ctx_t *c = (ctx_t *)h;
    int n = c->n, E = c->P * n * n, nl = nloc(c), ng = c->g * c->g;
    cplx *f = (cplx *)fout;
    memset(f, 0, sizeof(cplx) * c->N);
    for (int e = 0; e < E; ++e) {   /* serial: small */
        int j = e / (n * n), r = e % (n * n), e1 = r % n, e2 = r / n;
        locmap_t L;
        local_map(c, j, e1, e2, &L);
        pointval_t T;
        double h1 = 1.0 / n;
        for (int b = 0; b < c->g; ++b)
            for (int a = 0; a < c->g; ++a) {
                point_values(c, j, e1, e2, (e1 + c->gx[a]) * h1, (e2 + c->gx[b]) * h1, &T);
                double w = c->gw[a] * c->gw[b] * h1 * h1;
                if (c->scalar) {   /* f_i = int g phi_i dsigma (the surface element is in D) */
                    cplx g = scalar_field(c, kind, par, T.X);
                    for (int l = 0; l < nl; ++l) f[L.idx[l]] += w * g * T.D[l];
                    continue;
                }
                cplx Ein[3];
                field_eval(c, kind, par, T.X, Ein);
                for (int l = 0; l < nl; ++l)
                    f[L.idx[l]] -= L.sg[l] * w * (Ein[0] * T.Phi[l][0] + Ein[1] * T.Phi[l][1] + Ein[2] * T.Phi[l][2]);
            }
    }
    (void)ng;
    return 0;
}

int or_field(void *h, int kind, const double *par, int npts, const double *x, double *Eout)
{
    ctx_t *c = (ctx_t *)h;
    for (int i = 0; i < npts; ++i) field_eval(c, kind, par, x + 3 * i, (cplx *)Eout + 3 * i);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* potential  e_s(x) = int G(x-y) w(y) + kappa^-2 grad_x int G(x-y) div w(y)  */
/* (eq:ESLP), g x g Gauss per element, points away from Gamma                 */
/* ------------------------------------------------------------------------- */
int or_potential(void *h, const double *win, int npts, const double *x, double *Eout)
{
    ctx_t *c = (ctx_t *)h;
    int n = c->n, E = c->P * n * n, nl = nloc(c);
    const cplx *w = (const cplx *)win;
    cplx *out = (cplx *)Eout;
    double k = c->kappa, h1 = 1.0 / n;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < npts; ++i) {
        cplx acc[3] = {0, 0, 0};
        const double *xp = x + 3 * i;
        pointval_t T;
        for (int e = 0; e < E; ++e) {
            int j = e / (n * n), r = e % (n * n), e1 = r % n, e2 = r / n;
            locmap_t L;
            local_map(c, j, e1, e2, &L);
            for (int b = 0; b < c->g; ++b)
                for (int a = 0; a < c->g; ++a) {
                    point_values(c, j, e1, e2, (e1 + c->gx[a]) * h1, (e2 + c->gx[b]) * h1, &T);
                    double wt = c->gw[a] * c->gw[b] * h1 * h1;
                    cplx W[3] = {0, 0, 0}, dv = 0;
                    for (int l = 0; l < nl; ++l) {
                        cplx cf = L.sg[l] * w[L.idx[l]];
                        W[0] += cf * T.Phi[l][0]; W[1] += cf * T.Phi[l][1]; W[2] += cf * T.Phi[l][2];
                        dv += cf * T.D[l];
                    }
                    double rv[3] = {xp[0] - T.X[0], xp[1] - T.X[1], xp[2] - T.X[2]};
                    double rr = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
                    cplx G = cexp(I * k * rr) / (4.0 * M_PI * rr);
                    if (c->scalar) {   /* u(x) = int G(x - y) w(y) dsigma: value in acc[0] */
                        acc[0] += wt * G * dv;
                        continue;
                    }
                    cplx dG = G * (I * k * rr - 1.0) / (rr * rr);     /* grad_x G = (x-y) dG */
                    for (int d = 0; d < 3; ++d) acc[d] += wt * (G * W[d] + dG * rv[d] * dv / (k * k));
                }
        }
        out[3 * i] = acc[0]; out[3 * i + 1] = acc[1]; out[3 * i + 2] = acc[2];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* the interpolation-based FMM, literal form (Sec. 4.2)                       */
/* ------------------------------------------------------------------------- */
/* Chebyshev points of the first kind on [0,1] and Lagrange polynomials by the
 * product formula. */
static void cheb_nodes(int q, double *x)
{
    for (int m = 0; m <= q; ++m) x[m] = 0.5 * (1.0 + cos((2.0 * m + 1.0) * M_PI / (2.0 * q + 2.0)));
}

static void lagrange_all(int q, const double *xn, double s, double *L)
{
    for (int m = 0; m <= q; ++m) {
        double v = 1.0;
        for (int k = 0; k <= q; ++k)
            if (k != m) v *= (s - xn[k]) / (xn[m] - xn[k]);
        L[m] = v;
    }
}

int or_lagrange(int q, int npts, const double *s, double *L)
{
    double xn[MAXQ + 1];
    if (q < 1 || q > MAXQ) return -1;
    cheb_nodes(q, xn);
    for (int i = 0; i < npts; ++i) lagrange_all(q, xn, s[i], L + (size_t)i * (q + 1));
    return 0;
}

/* |d_uF x d_vF| from a node record (F, d_uF, d_vF) */
static double surf_elem(const double *g9)
{
    const double *Fu = g9 + 3, *Fv = g9 + 6;
    double nx = Fu[1] * Fv[2] - Fu[2] * Fv[1], ny = Fu[2] * Fv[0] - Fu[0] * Fv[2], nz = Fu[0] * Fv[1] - Fu[1] * Fv[0];
    return sqrt(nx * nx + ny * ny + nz * nz);
}

/* cluster id (patch j, level l, k1, k2) -> offset within level: j*4^l + k2*2^l + k1 */
typedef struct {
    int j, lvl, k1, k2;
} clu_t;

static clu_t clu_of(int lvl, int id)
{
    clu_t r;
    int s = 1 << lvl;
    r.lvl = lvl; r.j = id / (s * s);
    int o = id % (s * s);
    r.k2 = o / s; r.k1 = o % s;
    return r;
}

/*
 * y = A_q x  (or rows of it) with
 *   near : element-pair quadrature over all element pairs of the near leaf
 *          cluster pairs (tgt_near[i], src_near[i]) on level L
 *   far  : for every admissible pair (lvl, tgt, src): the blocks
 *            K_1^(a,b)[m,m'] = G(x_m,x'_m') <d_aF(x_m), d_bF(x'_m')>,
 *            K_2[m,m']       = -kappa^-2 G(x_m,x'_m')
 *          applied to the cluster moments of x:
 *            s^b[m'] = int_{src} L_m' x_h^b du',  d[m'] = int_{src} L_m' div x_h du'
 *          and tested with the cluster moments of the test functions (eq:FMMlr).
 * Cluster moments are integrated directly on every level (non-nested).
 * tmask: optional per-element mask of test elements to evaluate (rows touched only
 * by masked elements are complete).
 */
/* qlev[l]: interpolation degree of the clusters of level l = 0..L (the same degree on
 * every level is the method of Sec. 4.2; a degree per level is the variable-order form,
 * each level's moments and node geometry taken directly with its own degree) */
int or_fmm_apply(void *h, const int32_t *qlev, int L, int nfar, const int32_t *far_lvl, const int32_t *far_tgt,
                 const int32_t *far_src, int nnear, const int32_t *near_tgt, const int32_t *near_src,
                 const double *xin, double *yout, const uint8_t *tmask)
{
    ctx_t *c = (ctx_t *)h;
    if (!qlev || L < 0 || L > c->m) return -1;
    int qmax = 0;
    for (int l = 0; l <= L; ++l) {
        if (qlev[l] < 1 || qlev[l] > MAXQ) return -1;
        if (qlev[l] > qmax) qmax = qlev[l];
    }
    int n = c->n, E = c->P * n * n, nl = nloc(c), ng = c->g * c->g, p = c->p;
    /* per-cluster storage with the largest node count; level l uses its first Q_l */
    int Q = (qmax + 1) * (qmax + 1);
    double hh = 1.0 / n, ik2 = 1.0 / (c->kappa * c->kappa);
    const cplx *x = (const cplx *)xin;
    cplx *y = (cplx *)yout;
    memset(y, 0, sizeof(cplx) * c->N);
    double xnl[MAXLEV + 1][MAXQ + 1];
    for (int l = 0; l <= L; ++l) cheb_nodes(qlev[l], xnl[l]);

    /* Gauss rule exact for degree qmax + p per direction (moment integrals) */
    int nm = (qmax + p + 2) / 2 + 1;
    double mx[MAXG], mw[MAXG];
    or_gauss_legendre(nm, mx, mw);
    int nmq = nm * nm;

    /* x_h^a, div x_h at the moment points of every element, and the test-function
     * values (unsigned) at the same points */
    cplx *xv = (cplx *)malloc(sizeof(cplx) * (size_t)E * nmq * 3);
    double *tv = (double *)malloc(sizeof(double) * (size_t)E * nmq * nl * 2);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < E; ++e) {
        int j = e / (n * n), r = e % (n * n), e1 = r % n, e2 = r / n;
        locmap_t Lm;
        local_map(c, j, e1, e2, &Lm);
        double bpu[MAXDEG + 1], dpu[MAXDEG + 1], bqu[MAXDEG + 1], dqu[MAXDEG + 1];
        double bpv[MAXDEG + 1], dpv[MAXDEG + 1], bqv[MAXDEG + 1], dqv[MAXDEG + 1];
        for (int b = 0; b < nm; ++b)
            for (int a = 0; a < nm; ++a) {
                int g = b * nm + a;
                double u = (e1 + mx[a]) * hh, v = (e2 + mx[b]) * hh;
                element_pieces(c, e1, e2, u, v, bpu, dpu, bqu, dqu, bpv, dpv, bqv, dqv);
                cplx x0 = 0, x1 = 0, dv = 0;
                int k = 0;
                if (c->scalar) {   /* the parameter-space function x_h (no surface element) */
                    for (int t2 = 0; t2 <= p; ++t2)
                        for (int t1 = 0; t1 <= p; ++t1, ++k) {
                            double val = bpu[t1] * bpv[t2];
                            tv[(((size_t)e * nmq + g) * nl + k) * 2] = 0.0;
                            tv[(((size_t)e * nmq + g) * nl + k) * 2 + 1] = val;
                            dv += x[Lm.idx[k]] * val;
                        }
                    xv[((size_t)e * nmq + g) * 3 + 0] = 0;
                    xv[((size_t)e * nmq + g) * 3 + 1] = 0;
                    xv[((size_t)e * nmq + g) * 3 + 2] = dv;
                    continue;
                }
                for (int t2 = 0; t2 < p; ++t2)
                    for (int t1 = 0; t1 <= p; ++t1, ++k) {
                        double val = bpu[t1] * bqv[t2], dd = dpu[t1] * bqv[t2];
                        tv[(((size_t)e * nmq + g) * nl + k) * 2] = val;
                        tv[(((size_t)e * nmq + g) * nl + k) * 2 + 1] = dd;
                        cplx cf = Lm.sg[k] * x[Lm.idx[k]];
                        x0 += cf * val; dv += cf * dd;
                    }
                for (int t2 = 0; t2 <= p; ++t2)
                    for (int t1 = 0; t1 < p; ++t1, ++k) {
                        double val = bqu[t1] * bpv[t2], dd = bqu[t1] * dpv[t2];
                        tv[(((size_t)e * nmq + g) * nl + k) * 2] = val;
                        tv[(((size_t)e * nmq + g) * nl + k) * 2 + 1] = dd;
                        cplx cf = Lm.sg[k] * x[Lm.idx[k]];
                        x1 += cf * val; dv += cf * dd;
                    }
                xv[((size_t)e * nmq + g) * 3 + 0] = x0;
                xv[((size_t)e * nmq + g) * 3 + 1] = x1;
                xv[((size_t)e * nmq + g) * 3 + 2] = dv;
            }
    }

    /* per level: cluster moments (s^1, s^2, d) and node geometry */
    int nlev = L + 1;
    size_t *lvoff = (size_t *)malloc(sizeof(size_t) * (nlev + 1));
    lvoff[0] = 0;
    for (int l = 0; l < nlev; ++l) lvoff[l + 1] = lvoff[l] + (size_t)c->P * (1u << (2 * l));
    size_t NC = lvoff[nlev];
    cplx *mom = (cplx *)calloc(NC * Q * 3, sizeof(cplx));
    cplx *loc = (cplx *)calloc(NC * Q * 3, sizeof(cplx));   /* t^1, t^2, t^d */
    double *geo = (double *)malloc(sizeof(double) * NC * Q * 9);
    for (int l = 0; l < nlev; ++l) {
        int s = 1 << l, sub = n / s;   /* elements per cluster side */
        double H = 1.0 / s;
        long ncl = (long)c->P * s * s;
        const int q = qlev[l], Q1 = q + 1;
        const double *xn = xnl[l];
#pragma omp parallel for schedule(dynamic, 4)
        for (long id = 0; id < ncl; ++id) {
            clu_t cl = clu_of(l, (int)id);
            cplx *M = mom + (lvoff[l] + id) * Q * 3;
            double *Gm = geo + (lvoff[l] + id) * Q * 9;
            for (int m2 = 0; m2 < Q1; ++m2)
                for (int m1 = 0; m1 < Q1; ++m1) {
                    double *o = Gm + (m2 * Q1 + m1) * 9;
                    patch_eval(&c->pat[cl.j], (cl.k1 + xn[m1]) * H, (cl.k2 + xn[m2]) * H, o, o + 3, o + 6);
                }
            double La[MAXQ + 1], Lb[MAXQ + 1];
            for (int f2 = 0; f2 < sub; ++f2)
                for (int f1 = 0; f1 < sub; ++f1) {
                    int e1 = cl.k1 * sub + f1, e2 = cl.k2 * sub + f2;
                    int e = (cl.j * n + e2) * n + e1;
                    for (int b = 0; b < nm; ++b)
                        for (int a = 0; a < nm; ++a) {
                            int g = b * nm + a;
                            double u = (e1 + mx[a]) * hh, v = (e2 + mx[b]) * hh;
                            double w = mw[a] * mw[b] * hh * hh;
                            lagrange_all(q, xn, (u - cl.k1 * H) / H, La);
                            lagrange_all(q, xn, (v - cl.k2 * H) / H, Lb);
                            const cplx *xe = xv + ((size_t)e * nmq + g) * 3;
                            for (int m2 = 0; m2 < Q1; ++m2)
                                for (int m1 = 0; m1 < Q1; ++m1) {
                                    double Lw = La[m1] * Lb[m2] * w;
                                    cplx *Mm = M + (m2 * Q1 + m1) * 3;
                                    Mm[0] += Lw * xe[0]; Mm[1] += Lw * xe[1]; Mm[2] += Lw * xe[2];
                                }
                        }
                }
        }
    }

    /* which clusters are needed as targets */
    uint8_t *tneed = (uint8_t *)calloc(NC, 1);
    for (int e = 0; e < E; ++e) {
        if (tmask && !tmask[e]) continue;
        int j = e / (n * n), r = e % (n * n), e1 = r % n, e2 = r / n;
        for (int l = 0; l < nlev; ++l) {
            int s = 1 << l, sub = n / s;
            tneed[lvoff[l] + (size_t)j * s * s + (e2 / sub) * s + (e1 / sub)] = 1;
        }
    }

    /* far field: literal K_1^(a,b), K_2 per admissible block; grouped by target */
#pragma omp parallel
    {
        cplx *K = (cplx *)malloc(sizeof(cplx) * Q);
#pragma omp for schedule(dynamic, 8)
        for (int f = 0; f < nfar; ++f) {
            int l = far_lvl[f];
            size_t ti = lvoff[l] + far_tgt[f], si = lvoff[l] + far_src[f];
            if (!tneed[ti]) continue;
            const int Ql = (qlev[l] + 1) * (qlev[l] + 1);   /* nodes of this level */
            const double *Gt = geo + ti * Q * 9, *Gs = geo + si * Q * 9;
            const cplx *Ms = mom + si * Q * 3;
            cplx *tl = (cplx *)malloc(sizeof(cplx) * Q * 3);
            memset(tl, 0, sizeof(cplx) * Q * 3);
            for (int mt = 0; mt < Ql; ++mt) {
                const double *xt = Gt + mt * 9;
                for (int ms = 0; ms < Ql; ++ms) K[ms] = kernel_eval(c, xt, Gs + ms * 9);
                if (c->scalar) {
                    /* scalar localized kernel G(x_m, x'_m') |J(x_m)| |J'(x'_m')| on the moments */
                    double Jt = surf_elem(xt);
                    cplx s = 0;
                    for (int ms = 0; ms < Ql; ++ms) s += K[ms] * surf_elem(Gs + ms * 9) * Ms[ms * 3 + 2];
                    tl[mt * 3 + 2] += Jt * s;
                    continue;
                }
                for (int a = 0; a < 2; ++a) {
                    const double *da = xt + 3 + 3 * a;
                    cplx s = 0;
                    for (int b = 0; b < 2; ++b)
                        for (int ms = 0; ms < Ql; ++ms) {
                            const double *db = Gs + ms * 9 + 3 + 3 * b;
                            cplx K1 = K[ms] * (da[0] * db[0] + da[1] * db[1] + da[2] * db[2]);
                            s += K1 * Ms[ms * 3 + b];
                        }
                    tl[mt * 3 + a] += s;
                }
                cplx s = 0;
                for (int ms = 0; ms < Ql; ++ms) s += -ik2 * K[ms] * Ms[ms * 3 + 2];
                tl[mt * 3 + 2] += s;
            }
            cplx *dst = loc + ti * Q * 3;
            for (int k = 0; k < Q * 3; ++k) {
                double *d = (double *)&dst[k];
#pragma omp atomic
                d[0] += creal(tl[k]);
#pragma omp atomic
                d[1] += cimag(tl[k]);
            }
            free(tl);
        }
        free(K);
    }

    /* test side of the far field and the near field, per test element */
    int nt = c->nthreads;
    cplx *ybuf = (cplx *)calloc((size_t)nt * c->N, sizeof(cplx));
    /* near pairs grouped by target leaf cluster */
    size_t nleaf = lvoff[L + 1] - lvoff[L];
    int *cnt = (int *)calloc(nleaf + 1, sizeof(int));
    for (int i = 0; i < nnear; ++i) cnt[near_tgt[i] + 1]++;
    for (size_t i = 0; i < nleaf; ++i) cnt[i + 1] += cnt[i];
    int *lst = (int *)malloc(sizeof(int) * (nnear > 0 ? nnear : 1));
    int *fill = (int *)calloc(nleaf, sizeof(int));
    for (int i = 0; i < nnear; ++i) lst[cnt[near_tgt[i]] + fill[near_tgt[i]]++] = near_src[i];

    /* Gauss data of all elements that take part in a near pair of a needed leaf */
    uint8_t *eneed = (uint8_t *)calloc(E, 1);
    {
        int s = 1 << L, sub = n / s;
        for (int e = 0; e < E; ++e) {
            if (tmask && !tmask[e]) continue;
            int j = e / (n * n), r = e % (n * n), e1 = r % n, e2 = r / n;
            int lt = j * s * s + (e2 / sub) * s + (e1 / sub);
            eneed[e] = 1;
            for (int k = cnt[lt]; k < cnt[lt + 1]; ++k) {
                clu_t cs = clu_of(L, lst[k]);
                for (int f2 = 0; f2 < sub; ++f2)
                    for (int f1 = 0; f1 < sub; ++f1)
                        eneed[(cs.j * n + cs.k2 * sub + f2) * n + cs.k1 * sub + f1] = 1;
            }
        }
    }
    ecache_t ec;
    ecache_build(c, &ec, eneed);

#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cplx *yl = ybuf + (size_t)tid * c->N;
        cplx *blk = (cplx *)malloc(sizeof(cplx) * nl * nl);
        double La[MAXQ + 1], Lb[MAXQ + 1];
#pragma omp for schedule(static)
        for (int e = 0; e < E; ++e) {
            if (tmask && !tmask[e]) continue;
            int j = e / (n * n), r = e % (n * n), e1 = r % n, e2 = r / n;
            elem_t Ee = {j, e1, e2};
            locmap_t La_;
            local_map(c, j, e1, e2, &La_);
            cplx ye[MAXLOC];
            for (int l = 0; l < nl; ++l) ye[l] = 0;
            /* far: y_l += int_e [ phi_l^a t^a + div phi_l t^d ] over all ancestor levels */
            for (int l = 0; l < nlev; ++l) {
                int s = 1 << l, sub = n / s;
                double H = 1.0 / s;
                int k1 = e1 / sub, k2 = e2 / sub;
                const int q = qlev[l], Q1 = q + 1;
                const double *xn = xnl[l];
                const cplx *T = loc + (lvoff[l] + (size_t)j * s * s + k2 * s + k1) * Q * 3;
                for (int b = 0; b < nm; ++b)
                    for (int a = 0; a < nm; ++a) {
                        int g = b * nm + a;
                        double u = (e1 + mx[a]) * hh, v = (e2 + mx[b]) * hh;
                        double w = mw[a] * mw[b] * hh * hh;
                        lagrange_all(q, xn, (u - k1 * H) / H, La);
                        lagrange_all(q, xn, (v - k2 * H) / H, Lb);
                        cplx t1 = 0, t2 = 0, td = 0;
                        for (int m2 = 0; m2 < Q1; ++m2)
                            for (int m1 = 0; m1 < Q1; ++m1) {
                                double Lw = La[m1] * Lb[m2];
                                const cplx *Tm = T + (m2 * Q1 + m1) * 3;
                                t1 += Lw * Tm[0]; t2 += Lw * Tm[1]; td += Lw * Tm[2];
                            }
                        const double *tvp = tv + ((size_t)e * nmq + g) * nl * 2;
                        for (int k = 0; k < nl; ++k) {
                            cplx ta = (k < p * (p + 1)) ? t1 : t2;
                            ye[k] += w * (tvp[2 * k] * ta + tvp[2 * k + 1] * td);
                        }
                    }
            }
            /* near: all element pairs of the near leaf pairs of e's leaf cluster */
            {
                int s = 1 << L, sub = n / s;
                int lt = j * s * s + (e2 / sub) * s + (e1 / sub);
                for (int k = cnt[lt]; k < cnt[lt + 1]; ++k) {
                    clu_t cs = clu_of(L, lst[k]);
                    for (int f2 = 0; f2 < sub; ++f2)
                        for (int f1 = 0; f1 < sub; ++f1) {
                            int fe1 = cs.k1 * sub + f1, fe2 = cs.k2 * sub + f2;
                            int f = (cs.j * n + fe2) * n + fe1;
                            elem_t Ef = {cs.j, fe1, fe2};
                            locmap_t Lb_;
                            local_map(c, cs.j, fe1, fe2, &Lb_);
                            element_pair(c, &Ee, &Ef, ec.T + (size_t)e * ng, ec.T + (size_t)f * ng, ec.w,
                                         ec.C[e], ec.C[f], blk);
                            for (int l = 0; l < nl; ++l) {
                                cplx sacc = 0;
                                for (int lp = 0; lp < nl; ++lp) sacc += Lb_.sg[lp] * blk[l * nl + lp] * x[Lb_.idx[lp]];
                                ye[l] += sacc;
                            }
                        }
                }
            }
            for (int l = 0; l < nl; ++l) yl[La_.idx[l]] += La_.sg[l] * ye[l];
        }
        free(blk);
    }
    for (int i = 0; i < c->N; ++i) {
        cplx s = 0;
        for (int t = 0; t < nt; ++t) s += ybuf[(size_t)t * c->N + i];
        y[i] = s;
    }
    free(ybuf); free(cnt); free(lst); free(fill); free(eneed); free(tneed);
    ecache_free(&ec);
    free(xv); free(tv); free(lvoff); free(mom); free(loc); free(geo);
    return 0;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* int_Gamma div_Gamma phi_i dsigma = int div phi_hat_i du for every glued unknown
 * (zero for every unknown of a closed surface: the normal flux is continuous) */
int or_div_integrals(void *h, double *out)
{
    ctx_t *c = (ctx_t *)h;
    int n = c->n, E = c->P * n * n, nl = nloc(c);
    double hh = 1.0 / n;
    memset(out, 0, sizeof(double) * c->N);
    for (int e = 0; e < E; ++e) {
        int j = e / (n * n), r = e % (n * n), e1 = r % n, e2 = r / n;
        locmap_t L;
        local_map(c, j, e1, e2, &L);
        pointval_t T;
        for (int b = 0; b < c->g; ++b)
            for (int a = 0; a < c->g; ++a) {
                point_values(c, j, e1, e2, (e1 + c->gx[a]) * hh, (e2 + c->gx[b]) * hh, &T);
                double w = c->gw[a] * c->gw[b] * hh * hh;
                for (int l = 0; l < nl; ++l) out[L.idx[l]] += L.sg[l] * w * T.D[l];
            }
    }
    return 0;
}
