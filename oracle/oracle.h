/*
 * oracle.h -- serial FP64 CPU reference for the sparse-grid isogeometric
 * method (Beck, Sangalli & Tamellini, "A sparse-grid isogeometric solver").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library: both are written independently from the paper.
 *
 * Parity pins for every function are in tests/test_oracle_*.py.
 */
#ifndef SG_ORACLE_H
#define SG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_PATCH 4

/* one NURBS patch of the geometry map F (Sec. 2.2, "verbatim for NURBS") */
typedef struct {
    int degree[3];
    int nknots[3];
    const double* knots[3];
    const double* ctrl;     /* [n_d]...[n_1][dim], direction 1 fastest */
    const double* weights;  /* [n_d]...[n_1] or NULL (polynomial map)  */
} orc_patch;

/* analytic or sampled field (right-hand side, coefficient, Dirichlet data) */
enum {
    ORC_FLD_NONE = -1,
    ORC_FLD_CONST = 0,
    ORC_FLD_SINPROD = 1,
    ORC_FLD_SINCOS = 2,
    ORC_FLD_ANNULUS_RHS = 3,
    ORC_FLD_POLY_RHS = 4,
    ORC_FLD_GRID3D = 5,
    ORC_FLD_CORNER = 6,
    ORC_FLD_AFFINE = 7,
    /* exact solutions (error norms only) */
    ORC_EX_ANNULUS_U = 100,
    ORC_EX_SINPROD_U = 101,
    ORC_EX_POLY_U = 102
};

typedef struct {
    int kind;
    double prm[4];
    const double* data;   /* GRID3D samples, x fastest */
    int n[3];             /* GRID3D vertex counts */
} orc_field;

/* interface between two patches: side = 0 (xi1=0), 1 (xi1=1), 2 (xi2=0), 3 (xi2=1) */
typedef struct {
    int patch_a, side_a, patch_b, side_b;
} orc_interface;

enum { ORC_GRADE_UNIFORM = 0, ORC_GRADE_RADICAL = 1, ORC_GRADE_TOWARD0 = 2, ORC_GRADE_TOWARD1 = 3 };

typedef struct {
    int dim;
    int npatch;
    const orc_patch* patches;
    int ninterface;
    const orc_interface* interfaces;
    int p, r, w, lmin;
    int nq;                              /* Gauss points per direction; 0 => p+1 */
    int gkind[ORC_MAX_PATCH][3];         /* knot grading per patch and direction */
    double gamma[ORC_MAX_PATCH][3];
    orc_field f, a, g;                   /* g.kind == ORC_FLD_NONE => homogeneous Dirichlet */
    orc_field exact;
} orc_problem;

/* flags for orc_assemble_dense */
#define ORC_WITH_BOUNDARY 1   /* keep every basis function (no Dirichlet elimination) */
#define ORC_MASS 2            /* assemble the mass matrix instead of the stiffness */

int orc_gauss_legendre(int n, double* x, double* w);
int orc_num_knots(int p, int r, int level);
int orc_make_knots(int p, int r, int level, int gkind, double gamma, double* out);
double orc_grade(int gkind, double gamma, double t);
int orc_find_span(int p, int nknots, const double* knots, double x);
int orc_basis_all(int p, int nknots, const double* knots, double x, double* vals, double* ders);

void orc_geometry(const orc_problem* pb, int patch, const double* xi, double* x, double* jac,
                  double* wfun, double* dwfun);
double orc_field_value(const orc_field* fld, int dim, const double* x);
void orc_exact_value(const orc_field* fld, int dim, const double* x, double* u, double* grad);

int orc_components(const orc_problem* pb, int* levels, double* coef, int cap);
double orc_comb_coef_sum(int dim, int w, int lmin, const int* levels);
int64_t orc_ndof(const orc_problem* pb, const int* levels);
int64_t orc_assemble_dense(const orc_problem* pb, const int* levels, int flags, double* A,
                           double* b, int64_t cap);
int64_t orc_solve(const orc_problem* pb, const int* levels, double* coef, double* info);
int orc_eval(const orc_problem* pb, const int* levels, const double* coef, int64_t npts,
             const double* xi, const int* patch, double* u, double* grad);
int64_t orc_sg_solve_all(const orc_problem* pb, double* coefs, int64_t cap);
int orc_sg_eval(const orc_problem* pb, const double* coefs, int64_t npts, const double* xi,
                const int* patch, double* u, double* grad);
int orc_sg_errors(const orc_problem* pb, const double* coefs, int nref, double* out);
int orc_full_errors(const orc_problem* pb, const int* levels, const double* coef, int nref,
                    double* out);

#ifdef __cplusplus
}
#endif
#endif
