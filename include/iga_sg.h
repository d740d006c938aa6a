/*
 * iga_sg.h -- C interface of the MI355X sparse-grid isogeometric solver.
 *
 * The library solves, on one AMD GPU, every component problem of the
 * sparse-grid combination technique for a second-order elliptic problem
 *
 *     -div(a grad u) = f  in Omega = F([0,1]^d),   u = g on the boundary,
 *
 * (Problem 1 of Beck, Sangalli & Tamellini, "A sparse-grid isogeometric
 * solver", generalised to a variable coefficient a and Dirichlet data g),
 * discretised on the isoparametric spline spaces of Sec. 2.2 over the
 * anisotropic tensor grids of Sec. 3, and combines the component solutions
 * with the coefficients of eq. (TD-combi-tec).
 *
 * Call order:  iga_sg_plan_create -> iga_sg_workspace_bytes -> iga_sg_bind
 *              -> iga_sg_assemble -> iga_sg_solve -> iga_sg_combine / _eval
 *              -> iga_sg_destroy.
 * A call made out of order returns IGA_ERR_STATE.
 *
 * Memory: the plan owns host-side tables only.  Every device buffer the
 * library uses lies inside one caller-allocated workspace bound with
 * iga_sg_bind; the library never allocates device memory.  Pointer arguments
 * whose name ends in _dev are device pointers, _host are host pointers; they
 * are borrowed for the duration of the call.  All device work is enqueued on
 * the stream given to iga_sg_bind and is asynchronous unless stated.
 *
 * Errors: every call returns an iga_status; on failure iga_sg_last_error()
 * returns a message (thread-local).  No exception crosses this interface.
 * A plan must not be used from two threads at once; distinct plans may.
 */
#ifndef IGA_SG_H
#define IGA_SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct iga_sg_plan_s* iga_sg_plan;

typedef enum {
    IGA_OK = 0,
    IGA_ERR_INVALID_ARG = 1,   /* bad sizes, null pointers, unsupported combination */
    IGA_ERR_GEOMETRY = 2,      /* non-open knots, non-positive Jacobian, bad patch data */
    IGA_ERR_OUT_OF_MEMORY = 3, /* workspace too small */
    IGA_ERR_DEVICE = 4,        /* a HIP call failed */
    IGA_ERR_NOT_CONVERGED = 5, /* some component reached maxit (see the report) */
    IGA_ERR_BREAKDOWN = 6,     /* some component hit p'Ap <= 0 or a non-finite value */
    IGA_ERR_STATE = 7          /* call order violated */
} iga_status;

/* Knot grading of the solution knot vectors (Sec. 4.4): breakpoint i of
 * level l is g(i / 2^l).  RADICAL is the paper's two-sided map
 * g(t) = 2^(gamma-1) t^gamma for t <= 1/2 and 1 - 2^(gamma-1) (1-t)^gamma
 * otherwise; TOWARD0 / TOWARD1 grade toward one end: t^gamma, 1-(1-t)^gamma. */
enum { IGA_GRADE_UNIFORM = 0, IGA_GRADE_RADICAL = 1, IGA_GRADE_TOWARD0 = 2, IGA_GRADE_TOWARD1 = 3 };

/* One NURBS patch of the geometry map F, eq. (F-B-splines) ("verbatim for
 * NURBS", Sec. 2.2).  Host pointers, copied by iga_sg_plan_create.
 * ctrl: [n_d]...[n_1][dim] control points, direction 1 fastest;
 * weights: [n_d]...[n_1] or NULL for a polynomial map. */
typedef struct {
    int degree[3];
    int nknots[3];
    const double* knots_host[3];
    const double* ctrl_host;
    const double* weights_host;
    int grading[3];      /* IGA_GRADE_* of the solution knots, per direction */
    double gamma[3];     /* grading exponent (1 = uniform) */
} iga_patch;

/* Conforming C^0 interface: side s of a patch is 0 (xi_1=0), 1 (xi_1=1),
 * 2 (xi_2=0), 3 (xi_2=1), 4 (xi_3=0), 5 (xi_3=1). */
typedef struct {
    int patch_a, side_a, patch_b, side_b;
} iga_interface;

typedef struct {
    int dim;                         /* 2 or 3 */
    int npatch;                      /* >= 1 */
    const iga_patch* patches;
    int ninterface;
    const iga_interface* interfaces;
} iga_geometry;

/* Discretisation (Sec. 2.2 and Sec. 3): degree p in every direction,
 * interior continuity C^r (0 <= r < p), sparse-grid level w, minimum level
 * lmin per direction (components have levels i >= lmin with
 * w-d+1 <= |i| <= w), Gauss points per direction nq (0 => p+1).
 * nsamples (0 or 1 => one) problems that differ only in their field data
 * (coefficient samples) are planned, assembled and solved together: every
 * component grid exists once per sample, and "instance" s * ncomp + c names
 * component c of sample s in the calls below that take a component index. */
typedef struct {
    int p, r, w, lmin, nq;
    int nsamples;
    /* launch shape (0 => library default): unknowns per operator tile in 2D
     * (default 128) and in 3D (default 256), and the number of
     * fast-diagonalisation tasks of a solve below which 2D long directions
     * are kept in one block when LDS allows (default 256, the MI355X CU
     * count); the autotuner (tune.py) searches these */
    int op_tile, op_tile3, fd_tasks;
    /* nonzero: instead of the combination technique, the single full
     * tensor-product grid with level w in every direction (standard IGA at the
     * finest level of the sparse grid, the paper's comparison in Sec. 4);
     * combination coefficient 1, lmin ignored */
    int full;
    /* nindex > 0: instead of the sparse-grid set of level w, the combination
     * over the caller's downward-closed index set I of nindex multi-indices
     * (index_host [nindex][dim], absolute levels 0..24, host, copied): the
     * first line of eq. (TD-combi-tec) with its outer sum over I,
     * c_b = sum over z in {0,1}^dim with b + z in I of (-1)^|z|; multi-indices
     * with c_b = 0 get no grid.  A set that is not downward closed, or one
     * given together with full, returns IGA_ERR_INVALID_ARG. */
    const int* index_host;
    int nindex;
    /* nonzero with nindex > 0: every multi-index of the set gets a grid, also
     * those with c_b = 0 (their coefficient stays 0 in the combination), so
     * that the details of iga_sg_detail_norms can be formed */
    int keep_all;
} iga_sg_disc;

/* Fields (right-hand side f, coefficient a, Dirichlet data g). */
enum {
    IGA_FIELD_NONE = -1,
    IGA_FIELD_CONST = 0,        /* prm[0] */
    IGA_FIELD_SINPROD = 1,      /* prm[0] * prod_k sin(pi x_k) */
    IGA_FIELD_SINCOS = 2,       /* 1 + prm[0] sin(2 pi (x + prm[1])) cos(2 pi y) */
    IGA_FIELD_ANNULUS_RHS = 3,  /* -div(a grad u), u = -(x^2+y^2-1)(x^2+y^2-4) x y^2,
                                   a = SINCOS(prm[0], prm[1]) */
    IGA_FIELD_POLY_RHS = 4,     /* -div(a grad u), u = prod x_k (1-x_k), a = SINCOS(prm) */
    IGA_FIELD_GRID3D = 5,       /* trilinear interpolation on the vertex grid m/(n-1) of
                                   [0,1]^3; data_dev [n3][n2][n1], x fastest */
    IGA_FIELD_CORNER = 6,       /* r^(2/3) sin(2 theta/3), theta in [0, 2 pi) */
    IGA_FIELD_AFFINE = 7,       /* prm[0] + prm[1] x + prm[2] y + prm[3] z */
    IGA_FIELD_QP_SAMPLES = 8    /* values given at the Gauss points: data_dev [nqp_total] in the
                                   order of iga_sg_quad_points (every Gauss point of every grid of
                                   every sample); for f and a only; with a coefficient of this kind
                                   the learned preconditioner's log a input is 0 */
};

typedef struct {
    int kind;
    double prm[4];
    const double* data_dev;  /* GRID3D only; device memory */
    int n[3];
    int64_t sample_stride;   /* GRID3D in a plan of several samples: sample s reads
                                data_dev + s * sample_stride (0 => one field for all) */
} iga_field;

/* Precision of the inner solver (the outer refinement is always FP64). */
enum {
    IGA_PREC_FP64 = 0,    /* plain FD-preconditioned CG in FP64 */
    IGA_PREC_FP32 = 1,    /* FP32 operator and FP32 FD factors inside FP64 refinement */
    IGA_PREC_BF16FD = 2   /* FP32 operator, BF16 FD factors (FP32 accumulation), FP64 refinement */
};

typedef struct {
    int precision;     /* IGA_PREC_* */
    int batched;       /* 1: every grid in one persistent launch; 0: one grid per launch */
    double tol;        /* stop when r.P^-1 r <= tol^2 b.P^-1 b for the FP64 residual r = b - A x */
    double tol_inner;  /* inner relative tolerance (same norm) of each refinement step (mixed modes) */
    int maxit;         /* CG iterations per (inner) solve */
    int max_refine;    /* refinement steps (mixed modes); ignored for FP64 */
    int workgroups;    /* persistent launch width; 0 => library choice */
    int timing;        /* 1: fill report.kernel_ms with HIP-event times (synchronises);
                          2: also trace the phases of the persistent solve (report.phase_us) */
    int continue_cg;   /* refinement steps of the mixed modes: 0 restarts CG from the new FP64
                          residual (classic iterative refinement); 1 replaces the recursive
                          residual by the FP64 one and continues CG with its search direction */
    int precond;       /* 0: fast diagonalisation; 1: learned correction on top of it inside
                          flexible CG (3D plans, network attached by iga_sg_set_network); the
                          FP64 residual of every (re)start and the convergence test keep the
                          plain preconditioner */
    int learned_iters; /* precond 1: the correction acts on the residuals of the first
                          learned_iters - 1 iterations of each (inner) solve, plain fast
                          diagonalisation after them; 0 = on every iteration */
    int plain_fd;      /* 0: the fast-diagonalisation preconditioner with diagonal scaling,
                          z = S P^-1 S r, S = diag(sqrt(P_ii / A_ii)) (S P S has the
                          diagonal of A); 1: the unscaled pencil, z = P^-1 r */
    int schedule;      /* task schedule of the batched solve: 1 round robin over the launch's
                          tasks; 2 round robin over per-sweep lists that hold only the tasks
                          of grids still iterating (1 and 2: one cooperative launch whose
                          phases are separated by grid-wide barriers; the same results bit for
                          bit); 3 whole grid per workgroup: one workgroup runs the complete
                          refinement + CG of a grid and takes the next grid from a counter,
                          largest first (no grid-wide barrier); 0 library choice: 3 when every
                          grid has one fast-diagonalisation block and at most four operator
                          tiles, else 1 when each workgroup has at most one task per phase,
                          else 2.  Schedule 3 follows the same iteration per grid; its
                          reductions may group differently (rounding).  4 whole-device
                          kernels: the single grid of a full tensor plan (disc.full, one
                          patch, one sample) with its vectors in device memory, each CG step
                          a launch over the device (operator tiles, the preconditioner's mode
                          products as FP64 matrix-core GEMMs, elementwise updates with
                          fixed-order sums); FP64 only (a mixed request runs FP64, reported),
                          precond 0, plain_fd 0.  A full grid whose preconditioner vectors do
                          not fit the LDS of one workgroup is always solved this way (the
                          standard-IGA comparison of Sec. 4.2 at the paper's sizes); CG on
                          the recursive residual, the FP64 residual b - A x replacing it when
                          the test passes (at most max_refine restarts). */
} iga_sg_solve_opts;

/* Per-instance results (component c of sample s at s * ncomp + c); arrays
 * are caller-owned host buffers of length ncomp * nsamples (any may be NULL).  status: 0 converged, 5 maxit, 6 breakdown.
 * relres: ||b - A x||_2 / ||b||_2 of the last FP64 residual;
 * prelres: sqrt(r.P^-1 r / b.P^-1 b), the quantity the stopping test uses
 * (P the fast-diagonalisation preconditioner; about the relative
 * energy-norm error), which does not suffer the kappa*eps rounding floor of
 * the plain residual on strongly anisotropic grids. */
typedef struct {
    int ncomp;
    int* iters;
    int* refinements;
    double* relres;
    double* prelres;
    int* status;
    int total_iters;       /* sum of CG iterations over components */
    int sweeps;            /* iterations of the persistent loop (timing = 2) */
    double kernel_ms[4];   /* [1]: solve launch(es) in ms (timing >= 1) */
    int precision;         /* inner precision the solve ran with (IGA_PREC_*): a mixed mode is
                              declined (FP64 instead) when the plan's 1D eigenvalue ratio
                              max lambda / min lambda exceeds 1e7, where FP32 factors cannot
                              represent the pencil (strongly graded knots) */
    double lam_ratio;      /* that ratio, the largest over the plan's 1D tables */
    double phase_us[6];    /* timing = 2: mean wall time of the operator, update/forward and
                              backward phases per sweep (barrier included), then the mean
                              longest busy time of any workgroup in each phase */
} iga_sg_report;

/* Build a plan: index set and combination coefficients (eq. TD-combi-tec),
 * knot vectors per level (Sec. 3; grading Sec. 4.4), Gauss rules, 1D
 * stiffness/mass matrices and their generalised eigen-decompositions for the
 * fast-diagonalisation preconditioner, task lists.  Host only; no GPU call.
 * Errors: IGA_ERR_INVALID_ARG for unsupported sizes or combinations, among
 * them a component grid without interior unknowns (degree 1 at level 0:
 * raise lmin); IGA_ERR_GEOMETRY for bad patch data or a failed 1D
 * eigen-decomposition. */
iga_status iga_sg_plan_create(const iga_geometry* geom, const iga_sg_disc* disc, iga_sg_plan* out);

/* Bytes of device workspace the plan needs (256-byte aligned sub-buffers). */
iga_status iga_sg_workspace_bytes(iga_sg_plan plan, size_t* bytes);

/* Variant of iga_sg_bind for callers that cannot allocate device memory
 * (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc): the workspace is an array inside the library, one per device
 * (128 MiB, 256-byte aligned), held from the device's first static binding
 * until the process ends.  The call uploads the plan tables and computes the
 * basis tables as iga_sg_bind does (synchronising the stream) and allocates
 * nothing: no hipMalloc, no hipFree, no allocating library call.  Inputs
 * (fields, points) and outputs stay caller buffers.
 * The array of a device serves one plan at a time: a later
 * iga_sg_bind_static on the same device takes it over, and every call on a
 * plan bound before then returns IGA_ERR_STATE (rebind it).  The array keeps
 * the last binding's contents; everything a call reads is written by the
 * binding or by the call itself.  Calls of two plans that overlap on one
 * device race and are not supported.
 * Errors: IGA_ERR_OUT_OF_MEMORY when iga_sg_workspace_bytes exceeds 128 MiB
 * (nothing is touched), IGA_ERR_DEVICE when the array's address cannot be
 * obtained or an upload fails. */
iga_status iga_sg_bind_static(iga_sg_plan plan, void* stream);

/* Task counts of a batched solve (operator tiles; fast-diagonalisation tasks
 * with FP64 factors and with FP32/BF16 factors) and the LDS bytes a solve
 * workgroup takes (lds_bytes: with the learned preconditioner's activations
 * in 3D; lds_plain_bytes: a solve without it).  Any pointer may be NULL.
 * Host only. */
iga_status iga_sg_plan_stats(iga_sg_plan plan, int* op_tasks, int* fd_tasks_fp64, int* fd_tasks_lowp,
                             size_t* lds_bytes, size_t* lds_plain_bytes);

/* Bind a device workspace of at least iga_sg_workspace_bytes bytes and a HIP
 * stream (hipStream_t, NULL = default).  Uploads the plan tables and computes
 * the basis tables on the device; synchronises the stream before returning. */
iga_status iga_sg_bind(iga_sg_plan plan, void* workspace_dev, size_t bytes, void* stream);

/* Component list: levels_host [n][dim], ndof_host [n] (interior unknowns of
 * one sample), coef_host [n] (combination coefficients c_i).  Any pointer may
 * be NULL. */
iga_status iga_sg_components(iga_sg_plan plan, int* n, int* levels_host, int64_t* ndof_host,
                             double* coef_host);

/* Assemble every component system: per Gauss point the geometry map, its
 * Jacobian, a, f and the operator coefficients a w |det DF| DF^-1 DF^-T
 * (Sec. 2.2, Galerkin form of Problem 1), then the load vectors and the
 * diagonal of each operator (for the preconditioner's scaling), both summed
 * element by element.  f and a are required (analytic, GRID3D in 3D, or
 * QP_SAMPLES).  g: NULL or IGA_FIELD_NONE for homogeneous Dirichlet data;
 * otherwise an analytic field on a two-dimensional plan with polynomial maps
 * (Problem 1 with u = g on the boundary): the lift u_D interpolates g at the
 * patch corners and is the L2 projection (arc length) of g on each Dirichlet
 * side's trace space with the corners fixed; the load is corrected by
 * -a(u_D, phi) and u_D enters iga_sg_combine / iga_sg_eval /
 * iga_sg_coeffs_full.  Other data returns IGA_ERR_INVALID_ARG.  Enqueued
 * on the plan's stream; a non-positive det DF at a Gauss point sets a flag
 * that the next iga_sg_solve with a report returns as IGA_ERR_GEOMETRY. */
iga_status iga_sg_assemble(iga_sg_plan plan, const iga_field* f, const iga_field* a,
                           const iga_field* g);

/* Solve every component system with fast-diagonalisation preconditioned CG
 * (FP64, or mixed precision inside FP64 iterative refinement).  report may
 * be NULL.  Returns IGA_ERR_NOT_CONVERGED / IGA_ERR_BREAKDOWN if any
 * component failed; the other components are still solved. */
iga_status iga_sg_solve(iga_sg_plan plan, const iga_sg_solve_opts* opts, iga_sg_report* report);

/* u_dev[s * n + i] = sum_c coef_c u_{s,c}(xi_i), eq. (TD-combi-tec), for every
 * sample s (u_dev holds nsamples * n values), accumulated in FP64 in
 * component order.  xi_dev [n][dim] parametric points in [0,1]^dim,
 * patch_dev [n] patch ids or NULL (patch 0).  grad_dev (NULL: not computed)
 * receives the physical gradient of the same sum, [nsamples][n][dim]:
 * grad_x u = DF^-T grad_xi u (the discrete functions are B / W on the
 * geometry map F of eq. (F-B-splines), so grad_xi (v / W) =
 * (grad_xi v - (v / W) grad_xi W) / W), FP64 (the H1 errors of Sec. 4). */
iga_status iga_sg_combine(iga_sg_plan plan, const double* xi_dev, const int* patch_dev, int64_t n,
                          double* u_dev, double* grad_dev);

/* u_dev[i] = u_comp(xi_i) (and grad_dev [n][dim] its physical gradient, or
 * NULL) for one component instance (s * ncomp + c). */
iga_status iga_sg_eval(iga_sg_plan plan, int comp, const double* xi_dev, const int* patch_dev,
                       int64_t n, double* u_dev, double* grad_dev);

/* Copy the interior coefficients of component comp (lexicographic, direction
 * 1 fastest) to out_dev. */
iga_status iga_sg_coeffs(iga_sg_plan plan, int comp, double* out_dev);

/* Kernel-level hooks (tests, training data): y = A_comp x (which = 0 FP64
 * operator, 1 FP32 operator), y = P^-1 x (which = 2 FP64, 3 FP32, 4 BF16 fast
 * diagonalisation), y = b - A x (which = 5, FP64) or y = S P^-1 S x (which = 6,
 * FP64, the diagonally scaled preconditioner of iga_sg_solve_opts.plain_fd = 0,
 * S from the last iga_sg_assemble); x_dev, y_dev hold the component's interior
 * unknowns. */
iga_status iga_sg_apply(iga_sg_plan plan, int comp, int which, const double* x_dev, double* y_dev);

/* Full coefficient arrays of component comp (after iga_sg_solve): for each
 * patch in turn, every basis function of its grid ([n_d]..[n_1], direction 1
 * fastest, basis B / W of Sec. 2.2), the unknowns at their functions and the
 * Dirichlet lift's values (or 0) at the boundary functions; the function
 * u_comp on that patch is sum_j out_dev[j] B_j / W.  Parity hook. */
iga_status iga_sg_coeffs_full(iga_sg_plan plan, int comp, double* out_dev);

/* Load vector of component comp (after iga_sg_assemble) to out_dev. */
iga_status iga_sg_rhs(iga_sg_plan plan, int comp, double* out_dev);

/* Replace the load vector of component comp (after iga_sg_assemble, before
 * iga_sg_solve) by b_dev (device, the component's interior unknowns in the
 * layout of iga_sg_rhs): a caller's own right-hand side, or a fault forced
 * from the host (a non-finite entry ends that component with status 6 and
 * leaves the others untouched). */
iga_status iga_sg_set_rhs(iga_sg_plan plan, int comp, const double* b_dev);

/* Host copies of the 1D generalised eigen-decomposition K U = M U diag(lam),
 * U^T M U = I, of direction dir and level lev of patch 0: U_host [n][n]
 * (row i = basis function i, column k = eigenvector k), lam_host [n],
 * n = interior basis functions.  Any output may be NULL; *n receives n. */
iga_status iga_sg_fd_factor(iga_sg_plan plan, int dir, int lev, int* n, double* U_host,
                            double* lam_host);

/* Host copy of the 1D interior stiffness and mass of direction dir, level
 * lev (dense [n][n]). */
iga_status iga_sg_matrices_1d(iga_sg_plan plan, int dir, int lev, int* n, double* K_host,
                              double* M_host);

/* One step as a HIP graph: iga_sg_graph_capture records iga_sg_assemble(f,
 * a, no Dirichlet data) followed by iga_sg_solve(opts, no report) on the
 * plan's stream into a graph (the persistent solve as a cooperative kernel
 * node, so all its workgroups are resident as in the direct launch) and
 * instantiates it; iga_sg_graph_launch replays it on the plan's stream.  A
 * replay computes exactly what the two calls compute.  The fields' device
 * data must stay valid and unchanged in place for as long as the graph is
 * replayed (their values may change between replays).  opts.timing must be 0,
 * and the plan must be bound to a created stream (the legacy default stream
 * cannot be captured: IGA_ERR_STATE).
 * The instantiated graph (runtime-owned resources) is released by the next
 * capture, by iga_sg_bind (the graph records the workspace's addresses), by
 * iga_sg_set_network with another network, or by iga_sg_destroy; a launch
 * after such a release returns IGA_ERR_STATE.  Errors: IGA_ERR_STATE before iga_sg_bind or
 * a launch before a capture; the errors of iga_sg_assemble / iga_sg_solve;
 * IGA_ERR_DEVICE when the runtime cannot build the graph (the stream is left
 * out of capture mode either way). */
iga_status iga_sg_graph_capture(iga_sg_plan plan, const iga_field* f, const iga_field* a,
                                const iga_sg_solve_opts* opts);
iga_status iga_sg_graph_launch(iga_sg_plan plan);

/* The sparse-grid combination as a preconditioner of the full tensor
 * problem (the outlook of Sec. 5; eq. TD-combi-tec).  full: a full tensor
 * plan (disc.full, one patch, one sample, level w); sg: a plan of the same
 * geometry, degree, regularity and grading whose component levels are at
 * most w (a sparse grid, or a caller's index set), so that every component
 * space is nested in the full space.  Both bound to the same stream and
 * assembled with the same data (homogeneous Dirichlet).  Flexible CG on the
 * full problem with the two-level preconditioner
 *     z = y + S P^-1 S (r - A y),   y = sum_i c_i P_i A_i^-1 P_i^T r,
 * P_i the tensor product of the 1D prolongations from the component's levels
 * to w (interior unknowns), A_i the component's own Galerkin matrix (its
 * assembly), A_i^-1 applied by iga_sg_solve(sg, inner) (batched, to
 * inner->tol), S P^-1 S the full grid's scaled fast diagonalisation.  The
 * combination term alone does not act on the error outside the sparse-grid
 * space, hence the second level.  coarse_every = k > 0: the two-level
 * preconditioner on the first direction of each (re)start and on
 * iterations k, 2k, ...; the fast diagonalisation alone on the others;
 * coarse_every = 0: on the first direction only.  The stopping test and
 * restarts are those of schedule 4 (outer->tol, maxit, max_refine; the
 * solve runs in FP64).  report (nullable; one instance): iters = outer
 * iterations, sweeps = CG iterations of all inner solves.  The solution is
 * the full plan's (iga_sg_coeffs / iga_sg_combine of full); the sparse-grid
 * plan's load vector and solution are overwritten (assemble it again to
 * restore them).  Synchronises the stream once per outer iteration.
 * Errors: IGA_ERR_INVALID_ARG (plans that do not nest, other streams, bad
 * options), IGA_ERR_STATE (not assembled), the errors of iga_sg_solve. */
iga_status iga_sg_solve_twolevel(iga_sg_plan full, iga_sg_plan sg, const iga_sg_solve_opts* outer,
                                 const iga_sg_solve_opts* inner, int coarse_every, iga_sg_report* report);

/* Details of the combination technique (Sec. 3; the profits of the
 * knapsack choice, Sec. 4.2): for every grid b of a plan built from a
 * downward-closed index set with keep_all,
 *     norms_dev[b] = ( sum_q wq_dev[q] Delta_b(x_q)^2 )^(1/2),
 *     Delta_b = sum over z in {0,1}^d of (-1)^|z| u_(b-z)   (u of a negative
 *               level is 0),
 * with u_b the grid's solution (lift included) at the parametric points
 * xi_dev [n][dim] (device, FP64) and the caller's quadrature weights wq_dev
 * [n] (device, including |det DF|).  vals_dev: caller-owned device scratch of
 * ngrid * n doubles (the grid values, [grid][point], left there).  norms_dev:
 * [ngrid] device, grid order of iga_sg_components.  One patch, one sample.
 * Sums in a fixed order (reproducible).  Errors: IGA_ERR_INVALID_ARG (a plan
 * without keep_all, several patches or samples, null pointers),
 * IGA_ERR_STATE before iga_sg_solve. */
iga_status iga_sg_detail_norms(iga_sg_plan plan, const double* xi_dev, const double* wq_dev, int64_t n,
                               double* vals_dev, double* norms_dev);

/* The Gauss points of the plan, for fields sampled there (IGA_FIELD_QP_SAMPLES:
 * a random coefficient drawn at the quadrature points, data of another
 * code): xq_dev [nqp_total][dim] (device, FP64) receives the physical point
 * F(xi_q) of every Gauss point (the p+1-point rules per element of Sec. 4.1,
 * grid after grid in iga_sg_components order, sample after sample, within a
 * grid direction 1 fastest), wq_dev [nqp_total] (device, nullable) the
 * weight w_q |det DF(xi_q)|.  *nq_host receives nqp_total; with cap <
 * nqp_total (or xq_dev NULL) only the count is returned.  Asynchronous on the
 * plan's stream.  Errors: IGA_ERR_STATE before iga_sg_bind. */
iga_status iga_sg_quad_points(iga_sg_plan plan, double* xq_dev, double* wq_dev, int64_t cap, int64_t* nq_host);

/* Test hook: the 1D prolongation of a full tensor plan from level lev to the
 * plan's level w in direction dir (0-based), interior unknowns: T_host
 * [nf][nc] row-major (coarse function j = sum_i T[i][j] fine function i),
 * nf, nc set (T_host may be NULL to query the sizes). */
iga_status iga_sg_prolongation(iga_sg_plan plan, int dir, int lev, int* nf, int* nc, double* T_host);

void iga_sg_destroy(iga_sg_plan plan);
const char* iga_sg_last_error(void);
/* Library version string. */
const char* iga_sg_version(void);

#ifdef __cplusplus
}
#endif
#endif
