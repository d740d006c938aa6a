/*
 * oracle.c -- serial FP64 CPU reference for the sparse-grid isogeometric
 * method of Beck, Sangalli & Tamellini ("A sparse-grid isogeometric solver").
 *
 * TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only callers.  Shares no code with the
 * GPU library.
 *
 * What it computes, in the paper's order:
 *   - open knot vectors of the dyadic level sequence (Sec. 3, univariate
 *     sequence Xi_alpha with 2^alpha elements), optionally graded with the
 *     radical map of Sec. 4.4;
 *   - B-splines by the Cox-de Boor recursion, eq. (Bsp), with 0/0 = 0;
 *   - the geometry map F of eq. (F-B-splines), rational (NURBS) when weights
 *     are given;
 *   - the Galerkin system of Problem 1 (generalised to -div(a grad u) = f)
 *     on the isoparametric space of eq. (spline_space_phys), assembled by an
 *     element loop with p+1 Gauss-Legendre points per direction, solved by a
 *     direct (profile Cholesky) factorisation as in Sec. 4.1, followed by one
 *     FP64 refinement step;
 *   - the combination technique, eq. (TD-combi-tec):
 *       u_J = sum_{J-d+1 <= |b| <= J} (-1)^(J-|b|) binom(d-1, J-|b|) u_b.
 *
 * Readings where the paper is silent:
 *   - levels start at lmin (default 0); the combination index is w - d*lmin;
 *   - evaluation at the last knot uses the last non-empty interval;
 *   - discrete basis phi_j = B_j / W (W the NURBS weight function of F);
 *   - nonhomogeneous Dirichlet data: corner values interpolated, the other
 *     boundary coefficients by an edge-wise L2 projection (2D only).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXP 8
#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1]: Newton iteration on P_n                     */
/* ------------------------------------------------------------------------ */
/* P_n(z) and P_{n-1}(z) by the three-term recurrence
 * (k+1) P_{k+1} = (2k+1) z P_k - k P_{k-1}. */
static void legendre(int n, double z, double* pn, double* pnm1) {
    double p0 = 1.0, p1 = z;
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *pnm1 = p0;
}

int orc_gauss_legendre(int n, double* x, double* w) {
    if (n < 1 || n > 64) return -1;
    for (int i = 0; i < n; ++i) {
        double z = cos(PI * (i + 0.75) / (n + 0.5)), pn, pm, dp;
        for (int it = 0; it < 100; ++it) {
            legendre(n, z, &pn, &pm);
            dp = n * (z * pn - pm) / (z * z - 1.0);   /* P_n'(z) */
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        legendre(n, z, &pn, &pm);
        dp = n * (z * pn - pm) / (z * z - 1.0);
        x[n - 1 - i] = z;                             /* ascending nodes */
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
    return n;
}

/* ------------------------------------------------------------------------ */
/* knot vectors                                                              */
/* ------------------------------------------------------------------------ */
/* Breakpoint map t -> xi.  RADICAL is the two-sided map of Sec. 4.4 (the
 * printed fraction t^g / (1/2^(g-1)) equals 2^(g-1) t^g, continuous at 1/2);
 * TOWARD0 / TOWARD1 grade toward one end only. */
double orc_grade(int gkind, double gamma, double t) {
    switch (gkind) {
        case ORC_GRADE_RADICAL:
            if (t <= 0.5) return pow(2.0, gamma - 1.0) * pow(t, gamma);
            return 1.0 - pow(2.0, gamma - 1.0) * pow(1.0 - t, gamma);
        case ORC_GRADE_TOWARD0:
            return pow(t, gamma);
        case ORC_GRADE_TOWARD1:
            return 1.0 - pow(1.0 - t, gamma);
        default:
            return t;
    }
}

/* Open knot vector of level l: 2^l elements, end multiplicity p+1, interior
 * multiplicity p-r (so C^r at interior breakpoints, Sec. 2.2). */
int orc_num_knots(int p, int r, int level) {
    if (p < 1 || r < 0 || r >= p || level < 0) return -1;
    return 2 * (p + 1) + ((1 << level) - 1) * (p - r);
}

int orc_make_knots(int p, int r, int level, int gkind, double gamma, double* out) {
    int nk = orc_num_knots(p, r, level);
    if (nk < 0) return -1;
    int ne = 1 << level, k = 0;
    for (int i = 0; i <= p; ++i) out[k++] = 0.0;
    for (int e = 1; e < ne; ++e) {
        double z = orc_grade(gkind, gamma, (double)e / ne);
        for (int m = 0; m < p - r; ++m) out[k++] = z;
    }
    for (int i = 0; i <= p; ++i) out[k++] = 1.0;
    return k;
}

/* ------------------------------------------------------------------------ */
/* Cox-de Boor, eq. (Bsp)                                                    */
/* ------------------------------------------------------------------------ */
/* Interval index s with knots[s] <= x < knots[s+1]; at the right end the last
 * non-empty interval is used (reading for xi = 1). */
int orc_find_span(int p, int nknots, const double* U, double x) {
    int n = nknots - p - 1;            /* number of basis functions */
    if (x >= U[n]) {
        int s = n - 1;
        while (s > p && U[s] == U[s + 1]) --s;
        return s;
    }
    if (x <= U[p]) return p;
    int lo = p, hi = n;                /* U[lo] <= x < U[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (x < U[mid]) hi = mid; else lo = mid;
    }
    return lo;
}

static double ratio(double num, double den) { return den == 0.0 ? 0.0 : num / den; }

/* Values N[a] = B_{s-p+a,p}(x) and derivatives dN[a], a = 0..p, by running the
 * recursion of eq. (Bsp) from degree 0 on the indices that can be non-zero on
 * interval s.  Tab[k][i] holds B_{s-k+i,k}. */
static void basis_local(int p, const double* U, int s, double x, double* N, double* dN) {
    double T[MAXP + 1][MAXP + 2];
    T[0][0] = 1.0;
    for (int k = 1; k <= p; ++k) {
        for (int i = 0; i <= k; ++i) {
            int j = s - k + i;        /* global index of B_{j,k} */
            double left = 0.0, right = 0.0;
            if (i >= 1)               /* B_{j,k-1} = T[k-1][i-1] */
                left = ratio(x - U[j], U[j + k] - U[j]) * T[k - 1][i - 1];
            if (i <= k - 1)           /* B_{j+1,k-1} = T[k-1][i] */
                right = ratio(U[j + k + 1] - x, U[j + k + 1] - U[j + 1]) * T[k - 1][i];
            T[k][i] = left + right;
        }
    }
    for (int a = 0; a <= p; ++a) N[a] = T[p][a];
    if (!dN) return;
    /* B'_{j,p} = p/(U_{j+p}-U_j) B_{j,p-1} - p/(U_{j+p+1}-U_{j+1}) B_{j+1,p-1} */
    for (int a = 0; a <= p; ++a) {
        int j = s - p + a;
        double d = 0.0;
        if (p >= 1) {
            if (a >= 1) d += ratio((double)p, U[j + p] - U[j]) * T[p - 1][a - 1];
            if (a <= p - 1) d -= ratio((double)p, U[j + p + 1] - U[j + 1]) * T[p - 1][a];
        }
        dN[a] = d;
    }
}

int orc_basis_all(int p, int nknots, const double* U, double x, double* vals, double* ders) {
    int n = nknots - p - 1;
    if (n < 1 || p > MAXP) return -1;
    int s = orc_find_span(p, nknots, U, x);
    double N[MAXP + 1], dN[MAXP + 1];
    basis_local(p, U, s, x, N, dN);
    for (int i = 0; i < n; ++i) { vals[i] = 0.0; if (ders) ders[i] = 0.0; }
    for (int a = 0; a <= p; ++a) {
        vals[s - p + a] = N[a];
        if (ders) ders[s - p + a] = dN[a];
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* geometry map F (eq. F-B-splines), rational when weights are present       */
/* ------------------------------------------------------------------------ */
void orc_geometry(const orc_problem* pb, int patch, const double* xi, double* x, double* jac,
                  double* wfun, double* dwfun) {
    const orc_patch* P = &pb->patches[patch];
    int d = pb->dim;
    int n[3] = {1, 1, 1}, s[3] = {0, 0, 0};
    double N[3][MAXP + 1], dN[3][MAXP + 1];
    for (int k = 0; k < d; ++k) {
        int pg = P->degree[k];
        n[k] = P->nknots[k] - pg - 1;
        s[k] = orc_find_span(pg, P->nknots[k], P->knots[k], xi[k]);
        basis_local(pg, P->knots[k], s[k], xi[k], N[k], dN[k]);
    }
    for (int k = d; k < 3; ++k) { N[k][0] = 1.0; dN[k][0] = 0.0; }
    /* homogeneous sums: X_c = sum w P_c B, W = sum w B and their derivatives */
    double Xh[3] = {0, 0, 0}, dXh[3][3] = {{0}}, Wh = 0.0, dWh[3] = {0, 0, 0};
    int pg0 = P->degree[0], pg1 = d > 1 ? P->degree[1] : 0, pg2 = d > 2 ? P->degree[2] : 0;
    for (int c = 0; c <= pg2; ++c)
        for (int b = 0; b <= pg1; ++b)
            for (int a = 0; a <= pg0; ++a) {
                int j0 = s[0] - pg0 + a;
                int j1 = d > 1 ? s[1] - pg1 + b : 0;
                int j2 = d > 2 ? s[2] - pg2 + c : 0;
                int64_t idx = j0 + (int64_t)n[0] * (j1 + (int64_t)n[1] * j2);
                double wt = P->weights ? P->weights[idx] : 1.0;
                double bv[3] = {N[0][a], N[1][b], N[2][c]};
                double bd[3] = {dN[0][a], dN[1][b], dN[2][c]};
                double B = bv[0] * bv[1] * bv[2];
                double dB[3];
                dB[0] = bd[0] * bv[1] * bv[2];
                dB[1] = bv[0] * bd[1] * bv[2];
                dB[2] = bv[0] * bv[1] * bd[2];
                Wh += wt * B;
                for (int k = 0; k < d; ++k) dWh[k] += wt * dB[k];
                for (int cc = 0; cc < d; ++cc) {
                    double pc = P->ctrl[idx * d + cc];
                    Xh[cc] += wt * pc * B;
                    for (int k = 0; k < d; ++k) dXh[cc][k] += wt * pc * dB[k];
                }
            }
    for (int cc = 0; cc < d; ++cc) {
        x[cc] = Xh[cc] / Wh;
        if (jac)
            for (int k = 0; k < d; ++k) jac[cc * d + k] = (dXh[cc][k] - x[cc] * dWh[k]) / Wh;
    }
    if (wfun) *wfun = Wh;
    if (dwfun)
        for (int k = 0; k < d; ++k) dwfun[k] = dWh[k];
}

/* ------------------------------------------------------------------------ */
/* fields                                                                     */
/* ------------------------------------------------------------------------ */
static void sincos_coef(const double* prm, const double* x, double* a, double* da) {
    double amp = prm[0], sh = prm[1];
    double sx = sin(2 * PI * (x[0] + sh)), cx = cos(2 * PI * (x[0] + sh));
    double sy = sin(2 * PI * x[1]), cy = cos(2 * PI * x[1]);
    *a = 1.0 + amp * sx * cy;
    da[0] = 2 * PI * amp * cx * cy;
    da[1] = -2 * PI * amp * sx * sy;
    da[2] = 0.0;
}

/* u = P(s) x y^2 with s = x^2 + y^2 and P(s) = -(s-1)(s-4) (Sec. 4.2) */
static void annulus_u(const double* x, double* u, double* g, double* lap) {
    double X = x[0], Y = x[1], s = X * X + Y * Y;
    double P = -(s - 1.0) * (s - 4.0), dP = -2.0 * s + 5.0, ddP = -2.0;
    *u = P * X * Y * Y;
    g[0] = Y * Y * (2.0 * X * X * dP + P);
    g[1] = 2.0 * X * Y * (Y * Y * dP + P);
    /* u_xx = y^2 (6 x P' + 4 x^3 P''), u_yy = 2x (5 y^2 P' + 2 y^4 P'' + P) */
    double uxx = Y * Y * (6.0 * X * dP + 4.0 * X * X * X * ddP);
    double uyy = 2.0 * X * (5.0 * Y * Y * dP + 2.0 * Y * Y * Y * Y * ddP + P);
    *lap = uxx + uyy;
}

static void poly_u(int dim, const double* x, double* u, double* g, double* lap) {
    double q[3], dq[3];
    for (int k = 0; k < dim; ++k) { q[k] = x[k] * (1.0 - x[k]); dq[k] = 1.0 - 2.0 * x[k]; }
    double prod = 1.0;
    for (int k = 0; k < dim; ++k) prod *= q[k];
    *u = prod;
    double L = 0.0;
    for (int k = 0; k < dim; ++k) {
        double rest = 1.0;
        for (int j = 0; j < dim; ++j) if (j != k) rest *= q[j];
        g[k] = dq[k] * rest;
        L += -2.0 * rest;
    }
    *lap = L;
}

static double grid3d(const orc_field* fld, const double* x) {
    double v = 0.0;
    int i[3];
    double t[3];
    for (int k = 0; k < 3; ++k) {
        int n = fld->n[k];
        double s = x[k] * (n - 1);
        int ii = (int)floor(s);
        if (ii < 0) ii = 0;
        if (ii > n - 2) ii = n - 2;
        i[k] = ii;
        t[k] = s - ii;
    }
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                double wt = (a ? t[0] : 1 - t[0]) * (b ? t[1] : 1 - t[1]) * (c ? t[2] : 1 - t[2]);
                int64_t idx = (i[0] + a) + (int64_t)fld->n[0] * ((i[1] + b) + (int64_t)fld->n[1] * (i[2] + c));
                v += wt * fld->data[idx];
            }
    return v;
}

static void corner_u(const double* x, double* u, double* g) {
    double r = sqrt(x[0] * x[0] + x[1] * x[1]);
    double th = atan2(x[1], x[0]);
    if (th < 0) th += 2 * PI;
    if (r == 0.0) { *u = 0.0; if (g) { g[0] = g[1] = 0.0; } return; }
    double r23 = pow(r, 2.0 / 3.0);
    *u = r23 * sin(2.0 * th / 3.0);
    if (g) {
        double dr = (2.0 / 3.0) * r23 / r * sin(2.0 * th / 3.0);
        double dt = (2.0 / 3.0) * r23 / r * cos(2.0 * th / 3.0);
        g[0] = dr * cos(th) - dt * sin(th);
        g[1] = dr * sin(th) + dt * cos(th);
    }
}

double orc_field_value(const orc_field* fld, int dim, const double* x) {
    double u, g[3] = {0, 0, 0}, lap, a, da[3];
    switch (fld->kind) {
        case ORC_FLD_CONST:
            return fld->prm[0];
        case ORC_FLD_SINPROD: {
            double v = fld->prm[0];
            for (int k = 0; k < dim; ++k) v *= sin(PI * x[k]);
            return v;
        }
        case ORC_FLD_SINCOS:
            sincos_coef(fld->prm, x, &a, da);
            return a;
        case ORC_FLD_ANNULUS_RHS:
            annulus_u(x, &u, g, &lap);
            sincos_coef(fld->prm, x, &a, da);
            return -(a * lap + da[0] * g[0] + da[1] * g[1]);
        case ORC_FLD_POLY_RHS:
            poly_u(dim, x, &u, g, &lap);
            sincos_coef(fld->prm, x, &a, da);
            return -(a * lap + da[0] * g[0] + da[1] * g[1]);
        case ORC_FLD_GRID3D:
            return grid3d(fld, x);
        case ORC_FLD_CORNER:
            corner_u(x, &u, NULL);
            return u;
        case ORC_FLD_AFFINE: {
            double v = fld->prm[0];
            for (int k = 0; k < dim; ++k) v += fld->prm[1 + k] * x[k];
            return v;
        }
        default:
            return NAN;
    }
}

void orc_exact_value(const orc_field* fld, int dim, const double* x, double* u, double* grad) {
    double g[3] = {0, 0, 0}, lap;
    switch (fld->kind) {
        case ORC_EX_ANNULUS_U: {
            double z = dim == 3 ? sin(PI * x[2]) : 1.0;
            annulus_u(x, u, g, &lap);
            if (dim == 3) {
                g[2] = *u * PI * cos(PI * x[2]);
                g[0] *= z;
                g[1] *= z;
                *u *= z;
            }
            break;
        }
        case ORC_EX_SINPROD_U: {
            double v = fld->prm[0];
            for (int k = 0; k < dim; ++k) v *= sin(PI * x[k]);
            *u = v;
            for (int k = 0; k < dim; ++k) {
                double t = fld->prm[0] * PI * cos(PI * x[k]);
                for (int j = 0; j < dim; ++j) if (j != k) t *= sin(PI * x[j]);
                g[k] = t;
            }
            break;
        }
        case ORC_EX_POLY_U:
            poly_u(dim, x, u, g, &lap);
            break;
        case ORC_FLD_CORNER:
            corner_u(x, u, g);
            break;
        case ORC_FLD_AFFINE:
            *u = orc_field_value(fld, dim, x);
            for (int k = 0; k < dim; ++k) g[k] = fld->prm[1 + k];
            break;
        default:
            *u = NAN;
    }
    if (grad)
        for (int k = 0; k < dim; ++k) grad[k] = g[k];
}

/* ------------------------------------------------------------------------ */
/* combination technique, eq. (TD-combi-tec)                                 */
/* ------------------------------------------------------------------------ */
static double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double v = 1.0;
    for (int i = 1; i <= k; ++i) v = v * (n - k + i) / i;
    return v;
}

/* First line of eq. (TD-combi-tec) read with the sum over b restored:
 * c_b = sum over k in {0,1}^d with |b+k| <= J of (-1)^|k|, J = w - d*lmin and
 * b the shifted level.  Used by the tests to pin the binomial form below. */
double orc_comb_coef_sum(int dim, int w, int lmin, const int* levels) {
    int J = w - dim * lmin, nb = 0;
    for (int k = 0; k < dim; ++k) nb += levels[k] - lmin;
    double c = 0.0;
    for (int mask = 0; mask < (1 << dim); ++mask) {
        int nk = 0;
        for (int k = 0; k < dim; ++k) nk += (mask >> k) & 1;
        if (nb + nk <= J) c += (nk % 2) ? -1.0 : 1.0;
    }
    return c;
}

/* Components in lexicographic order (level 1 slowest), second line of
 * eq. (TD-combi-tec): J-d+1 <= |b| <= J, c_b = (-1)^(J-|b|) binom(d-1, J-|b|). */
int orc_components(const orc_problem* pb, int* levels, double* coef, int cap) {
    int d = pb->dim, J = pb->w - d * pb->lmin, cnt = 0;
    if (J < 0) return 0;
    int b[3] = {0, 0, 0};
    int lim1 = d > 1 ? J : 0, lim2 = d > 2 ? J : 0;
    for (b[0] = 0; b[0] <= J; ++b[0])
        for (b[1] = 0; b[1] <= lim1; ++b[1])
            for (b[2] = 0; b[2] <= lim2; ++b[2]) {
                int s = b[0] + b[1] + b[2];
                if (s > J || s < J - d + 1) continue;
                if (cnt < cap) {
                    for (int k = 0; k < d; ++k) levels[cnt * d + k] = b[k] + pb->lmin;
                    int j = J - s;
                    coef[cnt] = ((j % 2) ? -1.0 : 1.0) * binom(d - 1, j);
                }
                ++cnt;
            }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* discrete space of one component grid (all patches)                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int dim, npatch, p;
    int n[3];                         /* basis functions per direction (same on every patch) */
    int nk[3];
    double* knots[ORC_MAX_PATCH][3];
    int64_t nloc;                     /* basis functions per patch */
    int64_t* map;                     /* [npatch*nloc] -> dof >= 0, or -(1+dirichlet id) */
    int64_t ndof, ndir;
    double* gval;                     /* Dirichlet values [ndir] */
} space_t;

static void space_free(space_t* S) {
    for (int pt = 0; pt < S->npatch; ++pt)
        for (int k = 0; k < S->dim; ++k) free(S->knots[pt][k]);
    free(S->map);
    free(S->gval);
}

static int64_t uf_find(int64_t* par, int64_t i) {
    while (par[i] != i) { par[i] = par[par[i]]; i = par[i]; }
    return i;
}

/* side s of a patch: 0 xi1=0, 1 xi1=1, 2 xi2=0, 3 xi2=1, 4 xi3=0, 5 xi3=1 */
static int on_side(const space_t* S, const int* j, int side) {
    int k = side / 2;
    return (side % 2) ? j[k] == S->n[k] - 1 : j[k] == 0;
}

static int build_space(const orc_problem* pb, const int* levels, int keep_boundary, space_t* S) {
    memset(S, 0, sizeof(*S));
    S->dim = pb->dim;
    S->npatch = pb->npatch;
    S->p = pb->p;
    int d = pb->dim;
    for (int k = 0; k < 3; ++k) S->n[k] = 1;
    for (int pt = 0; pt < pb->npatch; ++pt)
        for (int k = 0; k < d; ++k) {
            int nk = orc_num_knots(pb->p, pb->r, levels[k]);
            if (nk < 0) return -1;
            S->nk[k] = nk;
            S->n[k] = nk - pb->p - 1;
            S->knots[pt][k] = (double*)malloc(sizeof(double) * nk);
            orc_make_knots(pb->p, pb->r, levels[k], pb->gkind[pt][k], pb->gamma[pt][k],
                           S->knots[pt][k]);
        }
    S->nloc = (int64_t)S->n[0] * S->n[1] * S->n[2];
    int64_t tot = S->nloc * pb->npatch;
    int64_t* par = (int64_t*)malloc(sizeof(int64_t) * tot);
    char* dir = (char*)calloc(tot, 1);
    for (int64_t i = 0; i < tot; ++i) par[i] = i;
    /* interface sides glue matching basis functions (conforming, same orientation) */
    for (int f = 0; f < pb->ninterface; ++f) {
        const orc_interface* I = &pb->interfaces[f];
        int ka = I->side_a / 2, kb = I->side_b / 2;
        int ta[2], tb[2], nt = 0, mt = 0;   /* tangential directions, increasing */
        for (int k = 0; k < d; ++k) {
            if (k != ka) ta[nt++] = k;
            if (k != kb) tb[mt++] = k;
        }
        for (int64_t li = 0; li < S->nloc; ++li) {
            int j[3] = {(int)(li % S->n[0]), (int)((li / S->n[0]) % S->n[1]),
                        (int)(li / ((int64_t)S->n[0] * S->n[1]))};
            if (!on_side(S, j, I->side_a)) continue;
            int jb[3] = {0, 0, 0};
            jb[kb] = (I->side_b % 2) ? S->n[kb] - 1 : 0;
            for (int t = 0; t < nt; ++t) jb[tb[t]] = j[ta[t]];
            int64_t lb = jb[0] + (int64_t)S->n[0] * (jb[1] + (int64_t)S->n[1] * jb[2]);
            int64_t ra = uf_find(par, I->patch_a * S->nloc + li);
            int64_t rb = uf_find(par, I->patch_b * S->nloc + lb);
            if (ra != rb) par[ra < rb ? rb : ra] = ra < rb ? ra : rb;
        }
    }
    /* Dirichlet: every side that is not an interface side */
    if (!keep_boundary) {
        for (int pt = 0; pt < pb->npatch; ++pt)
            for (int side = 0; side < 2 * d; ++side) {
                int is_if = 0;
                for (int f = 0; f < pb->ninterface; ++f) {
                    const orc_interface* I = &pb->interfaces[f];
                    if ((I->patch_a == pt && I->side_a == side) ||
                        (I->patch_b == pt && I->side_b == side)) is_if = 1;
                }
                if (is_if) continue;
                for (int64_t li = 0; li < S->nloc; ++li) {
                    int j[3] = {(int)(li % S->n[0]), (int)((li / S->n[0]) % S->n[1]),
                                (int)(li / ((int64_t)S->n[0] * S->n[1]))};
                    if (on_side(S, j, side)) dir[uf_find(par, pt * S->nloc + li)] = 1;
                }
            }
    }
    /* numbering: single patch in the order with the shortest direction fastest
     * (narrow profile); several patches patch by patch */
    S->map = (int64_t*)malloc(sizeof(int64_t) * tot);
    int64_t* cls = (int64_t*)malloc(sizeof(int64_t) * tot);
    const int64_t unset = INT64_MIN;
    for (int64_t i = 0; i < tot; ++i) cls[i] = unset;
    int ord[3] = {0, 1, 2};
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b)
            if (S->n[ord[b]] < S->n[ord[a]]) { int t = ord[a]; ord[a] = ord[b]; ord[b] = t; }
    int64_t ndof = 0, ndir = 0;
    for (int pt = 0; pt < pb->npatch; ++pt) {
        int j[3];
        int lim[3] = {S->n[ord[0]], d > 1 ? S->n[ord[1]] : 1, d > 2 ? S->n[ord[2]] : 1};
        for (int c = 0; c < lim[2]; ++c)
            for (int b = 0; b < lim[1]; ++b)
                for (int a = 0; a < lim[0]; ++a) {
                    j[0] = j[1] = j[2] = 0;
                    j[ord[0]] = a;
                    if (d > 1) j[ord[1]] = b;
                    if (d > 2) j[ord[2]] = c;
                    int64_t li = j[0] + (int64_t)S->n[0] * (j[1] + (int64_t)S->n[1] * j[2]);
                    int64_t root = uf_find(par, pt * S->nloc + li);
                    if (cls[root] == unset) cls[root] = dir[root] ? -(1 + ndir++) : ndof++;
                    S->map[pt * S->nloc + li] = cls[root];
                }
    }
    S->ndof = ndof;
    S->ndir = ndir;
    S->gval = (double*)calloc(ndir > 0 ? ndir : 1, sizeof(double));
    free(cls);
    free(par);
    free(dir);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* nonhomogeneous Dirichlet lifting (2D): corners interpolate g, each edge   */
/* L2-projects g on its trace space with the corners fixed                   */
/* ------------------------------------------------------------------------ */
static int dense_spd_solve(int n, double* A, double* b);

static int lift_dirichlet(const orc_problem* pb, space_t* S) {
    if (pb->g.kind == ORC_FLD_NONE || S->ndir == 0) return 0;
    if (pb->dim != 2) return -1;
    int p = pb->p, nq = pb->nq > 0 ? pb->nq : p + 1;
    double gx[64], gw[64];
    orc_gauss_legendre(nq, gx, gw);
    for (int pt = 0; pt < pb->npatch; ++pt) {
        if (pb->patches[pt].weights) return -1;
        for (int side = 0; side < 4; ++side) {
            int k = side / 2;             /* fixed direction */
            int t = 1 - k;                /* running direction */
            int jfix = (side % 2) ? S->n[k] - 1 : 0;
            int n = S->n[t];
            /* is this side Dirichlet? (all its basis functions lifted) */
            int64_t l0 = (k == 0) ? jfix + (int64_t)S->n[0] * 1 : 1 + (int64_t)S->n[0] * jfix;
            if (n < 3 || S->map[pt * S->nloc + l0] >= 0) continue;
            const double* U = S->knots[pt][t];
            /* corners: interpolation (open knots are interpolatory at the ends) */
            double cval[2];
            for (int e = 0; e < 2; ++e) {
                double xi[2];
                xi[k] = (double)(side % 2);
                xi[t] = (double)e;
                double x[2];
                orc_geometry(pb, pt, xi, x, NULL, NULL, NULL);
                cval[e] = orc_field_value(&pb->g, 2, x);
            }
            int m = n - 2;
            double* M = (double*)calloc((size_t)m * m, sizeof(double));
            double* rhs = (double*)calloc(m, sizeof(double));
            for (int i = p; i < S->nk[t] - p - 1; ++i) {
                if (U[i + 1] <= U[i]) continue;
                double h = U[i + 1] - U[i];
                for (int q = 0; q < nq; ++q) {
                    double s = U[i] + 0.5 * h * (gx[q] + 1.0);
                    double N[MAXP + 1];
                    basis_local(p, U, i, s, N, NULL);
                    double xi[2], x[2], jac[4];
                    xi[k] = (double)(side % 2);
                    xi[t] = s;
                    orc_geometry(pb, pt, xi, x, jac, NULL, NULL);
                    double ds = sqrt(jac[0 * 2 + t] * jac[0 * 2 + t] + jac[1 * 2 + t] * jac[1 * 2 + t]);
                    double wq = 0.5 * h * gw[q] * ds;
                    double gv = orc_field_value(&pb->g, 2, x);
                    for (int a = 0; a <= p; ++a) {
                        int ia = i - p + a;
                        if (ia == 0 || ia == n - 1) continue;
                        double corr = 0.0;
                        for (int b = 0; b <= p; ++b) {
                            int ib = i - p + b;
                            double mab = N[a] * N[b] * wq;
                            if (ib == 0) corr += mab * cval[0];
                            else if (ib == n - 1) corr += mab * cval[1];
                            else M[(ia - 1) * m + (ib - 1)] += mab;
                        }
                        rhs[ia - 1] += gv * N[a] * wq - corr;
                    }
                }
            }
            if (dense_spd_solve(m, M, rhs) != 0) { free(M); free(rhs); return -1; }
            for (int jt = 0; jt < n; ++jt) {
                int j[3] = {0, 0, 0};
                j[k] = jfix;
                j[t] = jt;
                int64_t li = j[0] + (int64_t)S->n[0] * j[1];
                int64_t mp = S->map[pt * S->nloc + li];
                if (mp >= 0) continue;
                double v = jt == 0 ? cval[0] : (jt == n - 1 ? cval[1] : rhs[jt - 1]);
                S->gval[-mp - 1] = v;
            }
            free(M);
            free(rhs);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* profile (skyline) symmetric storage and Cholesky                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int64_t* first;   /* first stored column of row i */
    int64_t* off;     /* start of row i in val */
    double* val;
} sky_t;

static double* sky_at(sky_t* A, int64_t i, int64_t j) {  /* i >= j */
    return &A->val[A->off[i] + (j - A->first[i])];
}

static void sky_free(sky_t* A) { free(A->first); free(A->off); free(A->val); }

static int sky_cholesky(sky_t* A) {
    for (int64_t i = 0; i < A->n; ++i) {
        int64_t fi = A->first[i];
        double* Li = &A->val[A->off[i] - fi];
        for (int64_t j = fi; j <= i; ++j) {
            int64_t fj = A->first[j];
            double* Lj = &A->val[A->off[j] - fj];
            int64_t k0 = fi > fj ? fi : fj;
            double s = Li[j];
            for (int64_t k = k0; k < j; ++k) s -= Li[k] * Lj[k];
            if (j < i) {
                Li[j] = s / Lj[j];
            } else {
                if (!(s > 0.0)) return -1;
                Li[i] = sqrt(s);
            }
        }
    }
    return 0;
}

static void sky_solve(const sky_t* L, double* x) {
    for (int64_t i = 0; i < L->n; ++i) {
        const double* Li = &L->val[L->off[i] - L->first[i]];
        double s = x[i];
        for (int64_t k = L->first[i]; k < i; ++k) s -= Li[k] * x[k];
        x[i] = s / Li[i];
    }
    for (int64_t i = L->n - 1; i >= 0; --i) {
        const double* Li = &L->val[L->off[i] - L->first[i]];
        x[i] /= Li[i];
        for (int64_t k = L->first[i]; k < i; ++k) x[k] -= Li[k] * x[i];
    }
}

/* y = b - A x with A symmetric in profile storage, extended-precision sums */
static void sky_residual(const sky_t* A, const double* b, const double* x, double* r) {
    long double* acc = (long double*)malloc(sizeof(long double) * A->n);
    for (int64_t i = 0; i < A->n; ++i) acc[i] = b[i];
    for (int64_t i = 0; i < A->n; ++i) {
        const double* Ai = &A->val[A->off[i] - A->first[i]];
        for (int64_t k = A->first[i]; k < i; ++k) {
            acc[i] -= (long double)Ai[k] * x[k];
            acc[k] -= (long double)Ai[k] * x[i];
        }
        acc[i] -= (long double)Ai[i] * x[i];
    }
    for (int64_t i = 0; i < A->n; ++i) r[i] = (double)acc[i];
    free(acc);
}

static int dense_spd_solve(int n, double* A, double* b) {
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0)) return -1;
        A[j * n + j] = sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / A[j * n + j];
        }
    }
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= A[i * n + k] * b[k];
        b[i] = s / A[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= A[k * n + i] * b[k];
        b[i] = s / A[i * n + i];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* element-loop assembly of the Galerkin system                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int mode;              /* 0: profile, 1: dense */
    int mass;
    sky_t* sky;
    double* dense;
    double* b;
    int64_t n;
} sink_t;

static void add_entry(sink_t* K, int64_t i, int64_t j, double v) {
    if (K->mode == 1) { K->dense[i * K->n + j] += v; return; }
    if (i >= j) *sky_at(K->sky, i, j) += v;
}

/* Loops over every element of every patch; at each Gauss point evaluates the
 * (p+1)^d local basis functions phi = B/W, their physical gradients
 * DF^{-T} grad(B/W), a(F(xi)), f(F(xi)) and accumulates
 *   A_ij += a grad phi_i . grad phi_j |det DF| w,  b_i += f phi_i |det DF| w
 * (or the mass matrix), lifting Dirichlet values into b.  With K == NULL only
 * the profile (first coupled column of each row) is recorded. */
static int assemble(const orc_problem* pb, const space_t* S, sink_t* K, int64_t* first) {
    int d = pb->dim, p = pb->p, nq = pb->nq > 0 ? pb->nq : p + 1;
    int nl = 1;
    for (int k = 0; k < d; ++k) nl *= (p + 1);
    double gx[64], gw[64];
    orc_gauss_legendre(nq, gx, gw);
    int nqd = 1;
    for (int k = 0; k < d; ++k) nqd *= nq;
    int64_t* gidx = (int64_t*)malloc(sizeof(int64_t) * nl);
    double* phi = (double*)malloc(sizeof(double) * nl);
    double* dphi = (double*)malloc(sizeof(double) * nl * 3);
    double* Aloc = (double*)malloc(sizeof(double) * nl * nl);
    double* bloc = (double*)malloc(sizeof(double) * nl);
    int E[3] = {1, 1, 1};
    for (int pt = 0; pt < pb->npatch; ++pt) {
        /* element k-ranges: non-empty knot intervals */
        int* espan[3];
        for (int k = 0; k < 3; ++k) {
            espan[k] = (int*)malloc(sizeof(int) * (k < d ? S->nk[k] : 1));
            E[k] = 0;
            if (k >= d) { espan[k][0] = 0; E[k] = 1; continue; }
            const double* U = S->knots[pt][k];
            for (int i = p; i < S->nk[k] - p - 1; ++i)
                if (U[i + 1] > U[i]) espan[k][E[k]++] = i;
        }
        for (int e2 = 0; e2 < E[2]; ++e2)
            for (int e1 = 0; e1 < E[1]; ++e1)
                for (int e0 = 0; e0 < E[0]; ++e0) {
                    int s[3] = {espan[0][e0], espan[1][e1], espan[2][e2]};
                    /* local -> global */
                    for (int l = 0; l < nl; ++l) {
                        int a[3] = {l % (p + 1), (l / (p + 1)) % (p + 1), l / ((p + 1) * (p + 1))};
                        int j[3] = {0, 0, 0};
                        for (int k = 0; k < d; ++k) j[k] = s[k] - p + a[k];
                        int64_t li = j[0] + (int64_t)S->n[0] * (j[1] + (int64_t)S->n[1] * j[2]);
                        gidx[l] = S->map[pt * S->nloc + li];
                    }
                    if (!K) {
                        int64_t mn = -1;
                        for (int l = 0; l < nl; ++l)
                            if (gidx[l] >= 0 && (mn < 0 || gidx[l] < mn)) mn = gidx[l];
                        for (int l = 0; l < nl; ++l)
                            if (gidx[l] >= 0 && first[gidx[l]] > mn) first[gidx[l]] = mn;
                        continue;
                    }
                    memset(Aloc, 0, sizeof(double) * nl * nl);
                    memset(bloc, 0, sizeof(double) * nl);
                    for (int qq = 0; qq < nqd; ++qq) {
                        int qi[3] = {qq % nq, (qq / nq) % nq, qq / (nq * nq)};
                        double xi[3] = {0, 0, 0}, wq = 1.0;
                        double N[3][MAXP + 1], dN[3][MAXP + 1];
                        for (int k = 0; k < d; ++k) {
                            const double* U = S->knots[pt][k];
                            double lo = U[s[k]], hi = U[s[k] + 1];
                            xi[k] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * gx[qi[k]];
                            wq *= 0.5 * (hi - lo) * gw[qi[k]];
                            basis_local(p, U, s[k], xi[k], N[k], dN[k]);
                        }
                        for (int k = d; k < 3; ++k) { N[k][0] = 1.0; dN[k][0] = 0.0; }
                        double x[3], jac[9], W, dW[3];
                        orc_geometry(pb, pt, xi, x, jac, &W, dW);
                        /* inverse Jacobian and determinant */
                        double det, inv[9];
                        if (d == 1) {
                            det = jac[0];
                            inv[0] = 1.0 / jac[0];
                        } else if (d == 2) {
                            det = jac[0] * jac[3] - jac[1] * jac[2];
                            inv[0] = jac[3] / det; inv[1] = -jac[1] / det;
                            inv[2] = -jac[2] / det; inv[3] = jac[0] / det;
                        } else {
                            const double* J = jac;
                            det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                                  J[2] * (J[3] * J[7] - J[4] * J[6]);
                            inv[0] = (J[4] * J[8] - J[5] * J[7]) / det;
                            inv[1] = (J[2] * J[7] - J[1] * J[8]) / det;
                            inv[2] = (J[1] * J[5] - J[2] * J[4]) / det;
                            inv[3] = (J[5] * J[6] - J[3] * J[8]) / det;
                            inv[4] = (J[0] * J[8] - J[2] * J[6]) / det;
                            inv[5] = (J[2] * J[3] - J[0] * J[5]) / det;
                            inv[6] = (J[3] * J[7] - J[4] * J[6]) / det;
                            inv[7] = (J[1] * J[6] - J[0] * J[7]) / det;
                            inv[8] = (J[0] * J[4] - J[1] * J[3]) / det;
                        }
                        if (!(det > 0.0)) goto fail;
                        double dv = det * wq;
                        double av = K->mass ? 1.0 : orc_field_value(&pb->a, d, x);
                        double fv = orc_field_value(&pb->f, d, x);
                        for (int l = 0; l < nl; ++l) {
                            int a[3] = {l % (p + 1), (l / (p + 1)) % (p + 1), l / ((p + 1) * (p + 1))};
                            double B = N[0][a[0]] * N[1][a[1]] * N[2][a[2]];
                            double dB[3] = {dN[0][a[0]] * N[1][a[1]] * N[2][a[2]],
                                            N[0][a[0]] * dN[1][a[1]] * N[2][a[2]],
                                            N[0][a[0]] * N[1][a[1]] * dN[2][a[2]]};
                            phi[l] = B / W;
                            double gp[3];
                            for (int k = 0; k < d; ++k) gp[k] = (dB[k] * W - B * dW[k]) / (W * W);
                            /* physical gradient: DF^{-T} grad_xi */
                            for (int c = 0; c < d; ++c) {
                                double t = 0.0;
                                for (int k = 0; k < d; ++k) t += inv[k * d + c] * gp[k];
                                dphi[l * 3 + c] = t;
                            }
                        }
                        for (int i = 0; i < nl; ++i) {
                            bloc[i] += fv * phi[i] * dv;
                            for (int j = 0; j < nl; ++j) {
                                double v;
                                if (K->mass) {
                                    v = phi[i] * phi[j];
                                } else {
                                    v = 0.0;
                                    for (int c = 0; c < d; ++c) v += dphi[i * 3 + c] * dphi[j * 3 + c];
                                    v *= av;
                                }
                                Aloc[i * nl + j] += v * dv;
                            }
                        }
                    }
                    for (int i = 0; i < nl; ++i) {
                        if (gidx[i] < 0) continue;
                        K->b[gidx[i]] += bloc[i];
                        for (int j = 0; j < nl; ++j) {
                            if (gidx[j] >= 0) add_entry(K, gidx[i], gidx[j], Aloc[i * nl + j]);
                            else K->b[gidx[i]] -= Aloc[i * nl + j] * S->gval[-gidx[j] - 1];
                        }
                    }
                }
        for (int k = 0; k < 3; ++k) free(espan[k]);
        continue;
    fail:
        for (int k = 0; k < 3; ++k) free(espan[k]);
        free(gidx); free(phi); free(dphi); free(Aloc); free(bloc);
        return -1;
    }
    free(gidx); free(phi); free(dphi); free(Aloc); free(bloc);
    return 0;
}

int64_t orc_ndof(const orc_problem* pb, const int* levels) {
    space_t S;
    if (build_space(pb, levels, 0, &S)) return -1;
    int64_t n = S.ndof;
    space_free(&S);
    return n;
}

/* Dense system (tests): rows/cols in the oracle's internal DOF order. */
int64_t orc_assemble_dense(const orc_problem* pb, const int* levels, int flags, double* A,
                           double* b, int64_t cap) {
    space_t S;
    if (build_space(pb, levels, flags & ORC_WITH_BOUNDARY, &S)) return -1;
    int64_t n = S.ndof;
    if (n > cap) { space_free(&S); return n; }
    if (!(flags & ORC_WITH_BOUNDARY) && lift_dirichlet(pb, &S)) { space_free(&S); return -2; }
    memset(A, 0, sizeof(double) * n * n);
    memset(b, 0, sizeof(double) * n);
    sink_t K = {1, (flags & ORC_MASS) ? 1 : 0, NULL, A, b, n};
    int rc = assemble(pb, &S, &K, NULL);
    space_free(&S);
    return rc ? -3 : n;
}

/* Full per-patch coefficient arrays (all basis functions, direction 1
 * fastest, Dirichlet values included) from the internal DOF vector. */
static void scatter_full(const space_t* S, const double* u, double* coef) {
    for (int pt = 0; pt < S->npatch; ++pt)
        for (int64_t li = 0; li < S->nloc; ++li) {
            int64_t m = S->map[pt * S->nloc + li];
            coef[pt * S->nloc + li] = m >= 0 ? u[m] : S->gval[-m - 1];
        }
}

/* Solve one component: assembly, profile Cholesky, one refinement step.
 * coef receives npatch * prod(n_k) values.  info (optional, 3 values):
 * relative residual before / after refinement, number of unknowns. */
int64_t orc_solve(const orc_problem* pb, const int* levels, double* coef, double* info) {
    space_t S;
    if (build_space(pb, levels, 0, &S)) return -1;
    if (lift_dirichlet(pb, &S)) { space_free(&S); return -2; }
    int64_t n = S.ndof;
    sky_t A = {n, NULL, NULL, NULL};
    A.first = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    A.off = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    for (int64_t i = 0; i < n; ++i) A.first[i] = i;
    assemble(pb, &S, NULL, A.first);
    int64_t tot = 0;
    for (int64_t i = 0; i < n; ++i) { A.off[i] = tot; tot += i - A.first[i] + 1; }
    A.val = (double*)calloc(tot > 0 ? tot : 1, sizeof(double));
    double* b = (double*)calloc(n > 0 ? n : 1, sizeof(double));
    sink_t K = {0, 0, &A, NULL, b, n};
    if (assemble(pb, &S, &K, NULL)) { sky_free(&A); free(b); space_free(&S); return -3; }
    sky_t L = A;
    L.first = A.first;
    L.off = A.off;
    L.val = (double*)malloc(sizeof(double) * (tot > 0 ? tot : 1));
    memcpy(L.val, A.val, sizeof(double) * tot);
    if (sky_cholesky(&L)) { free(L.val); sky_free(&A); free(b); space_free(&S); return -4; }
    double* x = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
    double* r = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
    memcpy(x, b, sizeof(double) * n);
    sky_solve(&L, x);
    double bn = 0.0, r0 = 0.0, r1 = 0.0;
    for (int64_t i = 0; i < n; ++i) bn += b[i] * b[i];
    sky_residual(&A, b, x, r);
    for (int64_t i = 0; i < n; ++i) r0 += r[i] * r[i];
    sky_solve(&L, r);
    for (int64_t i = 0; i < n; ++i) x[i] += r[i];
    sky_residual(&A, b, x, r);
    for (int64_t i = 0; i < n; ++i) r1 += r[i] * r[i];
    if (info) {
        info[0] = bn > 0 ? sqrt(r0 / bn) : 0.0;
        info[1] = bn > 0 ? sqrt(r1 / bn) : 0.0;
        info[2] = (double)n;
    }
    scatter_full(&S, x, coef);
    free(x); free(r); free(b); free(L.val); sky_free(&A);
    int64_t nfull = S.nloc * S.npatch;
    space_free(&S);
    return nfull;
}

/* ------------------------------------------------------------------------ */
/* evaluation and combination                                                */
/* ------------------------------------------------------------------------ */
/* u(xi) = sum_j c_j B_j(xi) / W(xi); grad (optional) is the physical gradient. */
static void eval_one(const orc_problem* pb, const space_t* S, const double* coef, int pt,
                     const double* xi, double* u, double* grad) {
    int d = pb->dim, p = pb->p;
    double N[3][MAXP + 1], dN[3][MAXP + 1];
    int s[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) {
        s[k] = orc_find_span(p, S->nk[k], S->knots[pt][k], xi[k]);
        basis_local(p, S->knots[pt][k], s[k], xi[k], N[k], dN[k]);
    }
    for (int k = d; k < 3; ++k) { N[k][0] = 1.0; dN[k][0] = 0.0; }
    double v = 0.0, dv[3] = {0, 0, 0};
    int lim1 = d > 1 ? p : 0, lim2 = d > 2 ? p : 0;
    for (int c = 0; c <= lim2; ++c)
        for (int b = 0; b <= lim1; ++b)
            for (int a = 0; a <= p; ++a) {
                int j0 = s[0] - p + a, j1 = d > 1 ? s[1] - p + b : 0, j2 = d > 2 ? s[2] - p + c : 0;
                double cf = coef[pt * S->nloc + j0 + (int64_t)S->n[0] * (j1 + (int64_t)S->n[1] * j2)];
                v += cf * N[0][a] * N[1][b] * N[2][c];
                dv[0] += cf * dN[0][a] * N[1][b] * N[2][c];
                dv[1] += cf * N[0][a] * dN[1][b] * N[2][c];
                dv[2] += cf * N[0][a] * N[1][b] * dN[2][c];
            }
    double x[3], jac[9], W, dW[3];
    orc_geometry(pb, pt, xi, x, jac, &W, dW);
    *u = v / W;
    if (!grad) return;
    double gp[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) gp[k] = (dv[k] * W - v * dW[k]) / (W * W);
    /* solve DF^T g = gp */
    if (d == 1) {
        grad[0] = gp[0] / jac[0];
    } else if (d == 2) {
        double det = jac[0] * jac[3] - jac[1] * jac[2];
        grad[0] = (jac[3] * gp[0] - jac[2] * gp[1]) / det;
        grad[1] = (-jac[1] * gp[0] + jac[0] * gp[1]) / det;
    } else {
        double A[9], bb[3] = {gp[0], gp[1], gp[2]};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A[i * 3 + j] = jac[j * 3 + i];
        /* Gaussian elimination with partial pivoting */
        for (int c = 0; c < 3; ++c) {
            int piv = c;
            for (int i = c + 1; i < 3; ++i) if (fabs(A[i * 3 + c]) > fabs(A[piv * 3 + c])) piv = i;
            for (int j = 0; j < 3; ++j) { double t = A[c * 3 + j]; A[c * 3 + j] = A[piv * 3 + j]; A[piv * 3 + j] = t; }
            double t = bb[c]; bb[c] = bb[piv]; bb[piv] = t;
            for (int i = c + 1; i < 3; ++i) {
                double f = A[i * 3 + c] / A[c * 3 + c];
                for (int j = c; j < 3; ++j) A[i * 3 + j] -= f * A[c * 3 + j];
                bb[i] -= f * bb[c];
            }
        }
        for (int i = 2; i >= 0; --i) {
            double t = bb[i];
            for (int j = i + 1; j < 3; ++j) t -= A[i * 3 + j] * grad[j];
            grad[i] = t / A[i * 3 + i];
        }
    }
}

int orc_eval(const orc_problem* pb, const int* levels, const double* coef, int64_t npts,
             const double* xi, const int* patch, double* u, double* grad) {
    space_t S;
    if (build_space(pb, levels, 0, &S)) return -1;
    int d = pb->dim;
    for (int64_t i = 0; i < npts; ++i)
        eval_one(pb, &S, coef, patch ? patch[i] : 0, xi + i * d, &u[i], grad ? grad + i * d : NULL);
    space_free(&S);
    return 0;
}

int64_t orc_sg_solve_all(const orc_problem* pb, double* coefs, int64_t cap) {
    int nc = orc_components(pb, NULL, NULL, 0);
    int* lv = (int*)malloc(sizeof(int) * 3 * (nc > 0 ? nc : 1));
    double* cc = (double*)malloc(sizeof(double) * (nc > 0 ? nc : 1));
    orc_components(pb, lv, cc, nc);
    int64_t off = 0;
    for (int c = 0; c < nc; ++c) {
        space_t S;
        if (build_space(pb, lv + c * pb->dim, 1, &S)) { off = -1; break; }
        int64_t need = S.nloc * S.npatch;
        space_free(&S);
        if (off + need > cap) { off = -2; break; }
        if (orc_solve(pb, lv + c * pb->dim, coefs + off, NULL) < 0) { off = -3; break; }
        off += need;
    }
    free(lv);
    free(cc);
    return off;
}

/* u_sg(xi) = sum_i c_i u_i(xi), accumulated in the lexicographic component order. */
int orc_sg_eval(const orc_problem* pb, const double* coefs, int64_t npts, const double* xi,
                const int* patch, double* u, double* grad) {
    int d = pb->dim;
    int nc = orc_components(pb, NULL, NULL, 0);
    int* lv = (int*)malloc(sizeof(int) * 3 * (nc > 0 ? nc : 1));
    double* cc = (double*)malloc(sizeof(double) * (nc > 0 ? nc : 1));
    orc_components(pb, lv, cc, nc);
    for (int64_t i = 0; i < npts; ++i) {
        u[i] = 0.0;
        if (grad) for (int k = 0; k < d; ++k) grad[i * d + k] = 0.0;
    }
    int64_t off = 0;
    for (int c = 0; c < nc; ++c) {
        space_t S;
        build_space(pb, lv + c * d, 0, &S);
        for (int64_t i = 0; i < npts; ++i) {
            double v, g[3];
            eval_one(pb, &S, coefs + off, patch ? patch[i] : 0, xi + i * d, &v, grad ? g : NULL);
            u[i] += cc[c] * v;
            if (grad) for (int k = 0; k < d; ++k) grad[i * d + k] += cc[c] * g[k];
        }
        off += S.nloc * S.npatch;
        space_free(&S);
    }
    free(lv);
    free(cc);
    return nc;
}

/* L2 and H1-seminorm errors against the exact solution, by (p+3)-point Gauss
 * quadrature on a uniform parametric reference mesh of nref^d cells per patch.
 * With levels == NULL the sparse-grid combination is measured, otherwise the
 * single tensor solution coef of that grid.  out = {L2 err, H1 semi err,
 * L2 norm of u, H1 semi norm of u}. */
static int errors_impl(const orc_problem* pb, const int* levels, const double* coef, int nref,
                       double* out) {
    int d = pb->dim, nq = pb->p + 3;
    double gx[64], gw[64];
    orc_gauss_legendre(nq, gx, gw);
    double e0 = 0, e1 = 0, n0 = 0, n1 = 0;
    int ncell = 1, nqd = 1;
    for (int k = 0; k < d; ++k) { ncell *= nref; nqd *= nq; }
    int64_t npts = (int64_t)ncell * nqd;
    double* xi = (double*)malloc(sizeof(double) * npts * d);
    double* wt = (double*)malloc(sizeof(double) * npts);
    int* pid = (int*)malloc(sizeof(int) * npts);
    double* u = (double*)malloc(sizeof(double) * npts);
    double* g = (double*)malloc(sizeof(double) * npts * d);
    for (int pt = 0; pt < pb->npatch; ++pt) {
        int64_t m = 0;
        for (int c = 0; c < ncell; ++c) {
            int ci[3] = {c % nref, (c / nref) % nref, c / (nref * nref)};
            for (int q = 0; q < nqd; ++q) {
                int qi[3] = {q % nq, (q / nq) % nq, q / (nq * nq)};
                double w = 1.0;
                for (int k = 0; k < d; ++k) {
                    xi[m * d + k] = (ci[k] + 0.5 * (gx[qi[k]] + 1.0)) / nref;
                    w *= 0.5 * gw[qi[k]] / nref;
                }
                wt[m] = w;
                pid[m] = pt;
                ++m;
            }
        }
        if (levels) orc_eval(pb, levels, coef, npts, xi, pid, u, g);
        else orc_sg_eval(pb, coef, npts, xi, pid, u, g);
        for (int64_t i = 0; i < npts; ++i) {
            double x[3], jac[9];
            orc_geometry(pb, pt, xi + i * d, x, jac, NULL, NULL);
            double det = d == 1 ? jac[0] : d == 2 ? jac[0] * jac[3] - jac[1] * jac[2]
                : jac[0] * (jac[4] * jac[8] - jac[5] * jac[7]) - jac[1] * (jac[3] * jac[8] - jac[5] * jac[6]) +
                  jac[2] * (jac[3] * jac[7] - jac[4] * jac[6]);
            double ue, ge[3];
            orc_exact_value(&pb->exact, d, x, &ue, ge);
            double w = wt[i] * fabs(det);
            e0 += w * (u[i] - ue) * (u[i] - ue);
            n0 += w * ue * ue;
            for (int k = 0; k < d; ++k) {
                e1 += w * (g[i * d + k] - ge[k]) * (g[i * d + k] - ge[k]);
                n1 += w * ge[k] * ge[k];
            }
        }
    }
    out[0] = sqrt(e0);
    out[1] = sqrt(e1);
    out[2] = sqrt(n0);
    out[3] = sqrt(n1);
    free(xi); free(wt); free(pid); free(u); free(g);
    return 0;
}

int orc_sg_errors(const orc_problem* pb, const double* coefs, int nref, double* out) {
    return errors_impl(pb, NULL, coefs, nref, out);
}

int orc_full_errors(const orc_problem* pb, const int* levels, const double* coef, int nref,
                    double* out) {
    return errors_impl(pb, levels, coef, nref, out);
}
