/*
 * lbs.h -- C-ABI of liblbs, a gfx950 (MI355X) solver for the Dirichlet
 * problem of the Laplace-Beltrami operator on the unit sphere with islands.
 *
 * Method (Kropinski & Nigam, "Fast integral equation methods for the
 * Laplace-Beltrami equation on the sphere"): the sphere minus M islands is
 * mapped to the plane by stereographic projection (Section 3); the solution
 * is a double-layer potential plus one log source per island
 * (Section 4.1, eq. eqn:u_multi), whose density and strengths solve the
 * Nystrom system of eq. matrix_eqns (Section 5):
 *
 *     [ I + K   E ] [ sigma ]   [ 2 g ]
 *     [   F     D ] [   A   ] = [  0  ]
 *
 * The system is solved by GMRES on the left-preconditioned form of
 * eq. matrix_eqns_c, and every product with I + K is evaluated by a 2D
 * Coulomb fast multipole method in the stereographic plane (Section 5).
 *
 * Conventions shared by every call:
 *  - Array arguments are DEVICE pointers unless the name ends in _host.
 *    Doubles are IEEE binary64.  Work is enqueued on `stream` (a
 *    hipStream_t passed as void*, NULL = the default stream) and the call
 *    returns without synchronizing unless stated otherwise.
 *  - Node order ("API order") is curve-major: island 0's nodes in
 *    parameter order t_j = 2 pi j / N_0, j = 0..N_0-1, then island 1, ...
 *    (Section 5, the vector sigma after eq. matrix_eqns).
 *  - Multi-right-hand-side arrays are column-major: column r of an
 *    (n x nrhs) array starts at offset r * n.
 *  - Ownership: inputs are borrowed for the duration of the call; outputs
 *    are caller-allocated.  A handle owns its device memory and must be
 *    used from one host thread at a time, with one stream at a time.
 *  - Errors: every call returns an lbs_status; nothing throws across the
 *    ABI.  On error, outputs are undefined (except where stated) and
 *    lbs_last_error() describes the failure.
 */
#ifndef LBS_H
#define LBS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbs_ctx *lbs_handle;

typedef enum {
  LBS_OK = 0,
  LBS_ERR_INVALID_ARG = 1,    /* bad pointer, size or option             */
  LBS_ERR_GEOMETRY = 2,       /* overlapping caps, pole inside or too    */
                              /* close to an island, non-finite input,   */
                              /* radius out of (0, pi/2)                 */
  LBS_ERR_NO_CONVERGENCE = 3, /* iteration limit reached; last iterate   */
                              /* and info are still written              */
  LBS_ERR_NOT_FINITE = 4,     /* NaN or Inf in the data                  */
  LBS_ERR_OUT_OF_MEMORY = 5,
  LBS_ERR_HIP = 6,            /* a HIP runtime call failed               */
  LBS_ERR_UNSUPPORTED = 7     /* valid request the library does not serve */
} lbs_status;

/* One island (Section 1.3): a simply connected cap-like region bounded by a
 * smooth curve.  Its boundary is the set of points at geodesic distance
 * r(t) from `center` in direction cos t e1 + sin t e2, e2 = e1 x center,
 * with r(t) = r0 (1 + sum_{n=1..8} coef[n-1] cos nt + coef[7+n] sin nt).
 * `center` is also the island's log-source point c_k (eq. eqn:u_multi).
 * center and e1 must be unit vectors with e1 . center = 0 (to 1e-10). */
typedef struct {
  double center[3];
  double e1[3];
  double r0;
  double coef[16];
} lbs_island;

enum { LBS_FP64 = 0, LBS_MIXED = 1 };            /* precision            */
enum { LBS_OP_IPLUSK = 0,  /* y = (I + K) sigma            (x, y: N)      */
       LBS_OP_K = 1,       /* y = K sigma                  (x, y: N)      */
       LBS_OP_SYSTEM = 2,  /* [y_s; y_a] = A [sigma; A]    (x, y: N + M)  */
       LBS_OP_PRECOND = 3, /* [y_s; y_a] = P^-1 A [sigma; A] (N + M)      */
       LBS_OP_IPLUSK_T = 4 /* y = (I + K)^T x, the transpose of the       */
                           /* Nystrom matrix of eq. disc_sphere (x, y: N) */
};
enum { LBS_MATVEC_FMM = 0, LBS_MATVEC_DIRECT = 1 }; /* far-field method   */

typedef struct {
  int32_t p64;       /* FP64 expansion terms (default 30)                  */
  int32_t p32;       /* FP32 expansion terms (default 16)                  */
  int32_t leaf_max;  /* max nodes per quadtree leaf (default 48)           */
  int32_t restart;   /* GMRES restart length (default 50, Section 6)       */
  int32_t max_iter;  /* GMRES iteration cap per solve (default 400)        */
  int32_t max_outer; /* mixed precision: refinement steps cap (default 8)  */
  double inner_tol;  /* mixed precision: inner GMRES tolerance (1e-5)      */
  int32_t matvec;    /* LBS_MATVEC_FMM (default) or LBS_MATVEC_DIRECT      */
  int32_t graphs;    /* 1 (default): every GMRES iteration (operator,      */
                     /* orthogonalisation, Givens update) is captured once */
                     /* per iteration index as a HIP graph on an internal  */
                     /* stream and replayed on the caller's stream; 0:     */
                     /* launched kernel by kernel.  Ignored while stage    */
                     /* timing is enabled.                                 */
  int32_t precond;   /* 1 (default): GMRES on the left-preconditioned      */
                     /* system P^-1 A of eq. matrix_eqns_c (block          */
                     /* preconditioner P = [[I, E], [F, D]] through its    */
                     /* Schur complement); 0: GMRES on A itself (eq.       */
                     /* matrix_eqns), whose condition number grows with N  */
                     /* (Section 6, Example 1, Table 1).  lbs_solve only.  */
  int32_t close_eval;/* 1 (default): lbs_eval replaces the trapezoidal     */
                     /* Cauchy sum of an island by the compensated rule    */
                     /* for exterior Cauchy integrals at targets in the    */
                     /* island's close zone (the cap of angular radius     */
                     /* max node distance from the centre + 8 node         */
                     /* spacings), accurate at any distance from the       */
                     /* curve; 0: the trapezoidal rule of eq. disc_sphere  */
                     /* everywhere.  lbs_eval_T / lbs_shape_vjp cover the  */
                     /* trapezoidal rule only and reject close targets     */
                     /* while it is 1.                                     */
  int32_t gpu_tree;  /* 1 (default): single-geometry handles build their  */
                     /* quadtrees and lists (set-up and evaluation plans)  */
                     /* with HIP kernels; 0: with host threads.  Batch     */
                     /* handles always use the host builder.  Both give    */
                     /* the same tree (lbs_compare_trees).                 */
  int32_t eval_tree; /* 0 (default): lbs_eval places each target in the   */
                     /* deepest box of the handle's own quadtree that      */
                     /* holds it and sums the box's local expansion, the   */
                     /* multipoles and nodes of its colleagues' subtrees   */
                     /* and the coarser adjacent leaves; lbs_eval_T and    */
                     /* lbs_shape_vjp apply the transpose of that sum (no  */
                     /* tree per target set); 1: these build a quadtree    */
                     /* over the nodes and the targets per target set.     */
                     /* Both are the FMM of Section 5 at the same order.   */
  int32_t m2l_groups;/* work-groups of the persistent FP32 M2L launch     */
                     /* (0 = the default 1024; else 64 .. 8192): the      */
                     /* launch shape lbs_autotune also tunes               */
  double schur_tol;  /* set-up forms each S_g^-1 (eq. matrix_eqns_c) by   */
                     /* Gauss-Jordan elimination in the natural order and  */
                     /* accepts it when the componentwise backward error   */
                     /* of S_g^-1 x for a fixed probe x is <= schur_tol    */
                     /* (default 1e-12), else redoes every block with      */
                     /* partial pivoting; <= 0: partial pivoting only.     */
                     /* lbs_schur_info reports which was used.             */
} lbs_options;

typedef struct {
  int32_t iters;          /* total GMRES iterations (all restarts, inner)  */
  int32_t outer_steps;    /* refinement steps (mixed precision), else 0    */
  double rel_resid;       /* final relative residual of the system GMRES   */
                          /* ran on, FP64 operator, worst system:          */
                          /* |P^-1 (b - A x)| / |P^-1 b| (precond = 1) or  */
                          /* |b - A x| / |b| (precond = 0)                 */
  double ms_solve;        /* wall time of the call                         */
  int32_t fp64_matvecs;   /* FMM applications in FP64                      */
  int32_t fp32_matvecs;   /* FMM applications with the FP32 far field      */
  double true_rel_resid;  /* |b - A x| / |b| of eq. matrix_eqns, b =       */
                          /* [2 g; 0], FP64 operator, worst system         */
} lbs_solve_info;

/* Fill *opt with the defaults listed above. */
void lbs_default_options(lbs_options *opt_host);

/* Build a solver for the boundary curves of `n_islands` islands
 * (Section 1.3) discretized with nodes_per_curve_host[k] >= 8 equispaced
 * nodes each (Section 5).  Computes the nodes and their stereographic
 * images (Section 3), the quadtree and interaction lists of the FMM, the
 * Schur complement S = D - F E of the block preconditioner and its inverse
 * (eq. matrix_eqns_c).  Synchronous.  opt_host may be NULL (defaults).
 * The north pole must lie outside every island's bounding cap (the cap of
 * radius max r(t) about the centre) and bounding caps must be disjoint;
 * both problems are rotation invariant, so callers rotate the sphere to
 * meet this.  Returns LBS_ERR_GEOMETRY otherwise. */
lbs_status lbs_setup(const lbs_island *islands_host, int32_t n_islands,
                     const int32_t *nodes_per_curve_host,
                     const lbs_options *opt_host, void *stream,
                     lbs_handle *out_host);

/* Set-up from sampled curves: the caller gives every node of every curve
 * with its first and second derivatives with respect to the curve's own
 * parameter t, at t_j = 2 pi j / N_k, j = 0..N_k-1 (x_host, xt_host,
 * xtt_host: N x 3 each, row-major, curve-major as the API order), and a
 * point inside each curve (centers_host: M x 3 unit vectors; it is the
 * island's log source c_k of eq. eqn:u_multi).  The trapezoidal rule of
 * eq. disc_sphere then runs over that parameter, as Section 6, Example 2
 * does with coastlines resampled at points equally spaced in arclength
 * (lbs_resample_curve_host).  Nodes must be unit vectors (to 1e-9) in the
 * open hemisphere about their centre, each curve must wind once about its
 * centre, and bounding caps (largest node distance from the centre plus
 * the largest chord between neighbouring nodes) follow the rules of
 * lbs_setup.  Everything else is as lbs_setup; the handle has no shape
 * coefficients (lbs_shape_vjp returns LBS_ERR_UNSUPPORTED).  Synchronous;
 * the host arrays are read during the call only. */
lbs_status lbs_setup_sampled(const double *x_host, const double *xt_host,
                             const double *xtt_host,
                             const double *centers_host, int32_t n_islands,
                             const int32_t *nodes_per_curve_host,
                             const lbs_options *opt_host, void *stream,
                             lbs_handle *out_host);

/* Host-only (no GPU needed): n_out points equally spaced in arclength on
 * the closed curve through the n_in >= 8 samples x_host (n_in x 3 unit
 * vectors at equispaced values of some parameter), starting at the first
 * sample, with x, x_t, x_tt for the parameter t = 2 pi s / L (x_out,
 * xt_out, xtt_out: n_out x 3, caller-allocated) and the length L.  The
 * curve is the trigonometric interpolant, with the modes |k| <= n_modes
 * (0: all below n_in / 2; fewer smooth the data), of the samples'
 * stereographic images from the antipode of center_host, a unit vector
 * inside the curve (Section 6, Example 2 smooths and resamples coastlines
 * this way before eq. disc_sphere).  LBS_ERR_GEOMETRY for a sample that is
 * not finite or lies opposite the centre. */
lbs_status lbs_resample_curve_host(int32_t n_in, const double *x_host,
                                   const double *center_host, int32_t n_modes,
                                   int32_t n_out, double *x_out_host,
                                   double *xt_out_host, double *xtt_out_host,
                                   double *length_host);

/* Batch of n_geoms independent geometries in one handle (one FMM forest;
 * every FMM stage is launched once for all geometries and right-hand
 * sides).  islands_host and nodes_per_curve_host are concatenated
 * geometry-major; geometry g owns islands_per_geom_host[g] islands.  Node,
 * island and data arrays of every later call are geometry-major as well
 * (API order inside a geometry); each (geometry, right-hand side) pair is
 * its own system, solved by GMRES in lockstep with its own Hessenberg
 * matrix and tolerance.  Validation as lbs_setup, per geometry.  The
 * direct matvec mode is not available for batches.  Synchronous. */
lbs_status lbs_setup_batch(int32_t n_geoms,
                           const int32_t *islands_per_geom_host,
                           const lbs_island *islands_host,
                           const int32_t *nodes_per_curve_host,
                           const lbs_options *opt_host, void *stream,
                           lbs_handle *out_host);

/* Geometry count and the node and island offsets of each geometry
 * (node_offsets_host: n_geoms + 1 entries, island_offsets_host: same);
 * either array may be NULL. */
lbs_status lbs_batch_info(lbs_handle h, int32_t *n_geoms_host,
                          int64_t *node_offsets_host,
                          int32_t *island_offsets_host);

/* Total node count N and island count M of a handle. */
lbs_status lbs_sizes(lbs_handle h, int64_t *n_nodes_host,
                     int32_t *n_islands_host);

/* Node positions on the sphere, API order, xyz: device (N x 3) row-major.
 * Use them to build Dirichlet data g. */
lbs_status lbs_nodes(lbs_handle h, double *xyz, void *stream);

/* Apply an operator of the discrete system (eq. matrix_eqns) to nrhs
 * vectors.  op is one of LBS_OP_*; precision LBS_FP64 evaluates the far
 * field with p64 terms in FP64, LBS_MIXED with p32 terms in FP32 (FP32
 * near field on differences of FP64 coordinates rounded to FP32); the
 * log-source and constraint rows are always FP64.  x and y are device
 * (n x nrhs), n = N or N + M by op. */
lbs_status lbs_matvec(lbs_handle h, int32_t op, int32_t precision,
                      int32_t nrhs, const double *x, double *y,
                      void *stream);

/* lbs_matvec for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same operators and kernels (op LBS_OP_IPLUSK, K, SYSTEM
 * or PRECOND; LBS_OP_IPLUSK_T returns LBS_ERR_UNSUPPORTED), with every
 * buffer beyond x and y (FMM strengths and expansions, partial sums,
 * completion counters, reduction space) in one static device array of
 * 128 MiB per GPU, which each GPU the library runs on holds until the
 * process ends.  An application that needs more (about 62 MB for one FP64
 * column at 1,024,000 nodes, 21 MB mixed) returns LBS_ERR_UNSUPPORTED.
 * The call allocates nothing.  Every call on a GPU shares that GPU's
 * array and leaves its contents behind: calls that overlap on one GPU (on
 * different streams or host threads) race. */
lbs_status lbs_matvec_noalloc(lbs_handle h, int32_t op, int32_t precision,
                              int32_t nrhs, const double *x, double *y,
                              void *stream);

/* Solve the system for Dirichlet data g (device, N x nrhs, API order):
 * GMRES(restart) on P^-1 A [sigma; A] = P^-1 [2g; 0] from x0 = 0 until the
 * preconditioned relative residual is <= tol (Section 5, Section 6); with
 * opt.precond = 0, GMRES on A [sigma; A] = [2g; 0] until its relative
 * residual is <= tol.
 * precision LBS_FP64: every matvec in FP64.  LBS_MIXED: iterative
 * refinement, outer residual with the FP64 operator, inner GMRES with the
 * FP32 far field to opt.inner_tol.  Writes sigma (N x nrhs) and the
 * log-source strengths A (M x nrhs); info_host may be NULL.  Synchronizes
 * `stream` once per GMRES iteration (an 8-byte residual read). */
lbs_status lbs_solve(lbs_handle h, int32_t precision, int32_t nrhs,
                     const double *g, double tol, double *sigma, double *A,
                     lbs_solve_info *info_host, void *stream);

/* Evaluate psi = W sigma + sum_m A_m G(x, c_m) (eq. eqn:u_multi) at
 * n_targets sphere points xyz_targets (device, T x 3 row-major) for nrhs
 * density/strength columns; u is device (T x nrhs).  Targets must lie in
 * the domain (outside every island; a target on a node is not supported);
 * the north pole is allowed.  The double layer is summed by the
 * trapezoidal rule of eq. disc_sphere, except at targets in an island's
 * close zone while opt.close_eval = 1, where that island's Cauchy sum is
 * taken by the compensated rule (Ioakimidis, Papadakis and Perdios 1991;
 * Helsing and Ojala 2008): v(z) = sum_j V_j a_j / (sum_j a_j - 2 pi i s_k),
 * a_j = h xi'_j / (xi_j - z), V the exterior boundary values of the Cauchy
 * integral.  Synchronous (builds a target tree and the close pairs on the
 * host; both are kept for the next call with the same targets). */
lbs_status lbs_eval(lbs_handle h, int32_t nrhs, const double *sigma,
                    const double *A, int64_t n_targets,
                    const double *xyz_targets, double *u, void *stream);

/* lbs_eval for a batch handle: targets [offsets[g], offsets[g+1]) belong to
 * geometry g (target_offsets_host: n_geoms + 1 host entries, offsets[0] = 0);
 * u is (offsets[n_geoms] x nrhs). */
lbs_status lbs_eval_batch(lbs_handle h, int32_t nrhs, const double *sigma,
                          const double *A,
                          const int64_t *target_offsets_host,
                          const double *xyz_targets, double *u, void *stream);

/* ----------------------------------------------------------- point vortices
 * Section 6, Example 2 places point vortices of strengths Gamma_j at points
 * v_j of the domain and decomposes the stream function as
 *   psi = psi* + sum_j Gamma_j G(x, v_j),
 * G the generalized fundamental solution (Section 1.1, eq.
 * eqn:greens_func), where psi* solves the Dirichlet problem with the data
 * g - sum_j Gamma_j G(x, v_j).  The flow is lbs_vortex_data -> lbs_solve ->
 * lbs_eval -> lbs_vortex_field.  The vortex sums are direct (FP64,
 * O(points x vortices)).  xyz_vortices: device (n_vortices x 3) unit
 * vectors; gamma: device (n_vortices x nrhs), one column of strengths per
 * right-hand side.  Single-geometry handles. */

/* g_star (N x nrhs) = g - sum_j Gamma_j G(x_i, v_j) at the nodes (g and
 * g_star may be the same array). */
lbs_status lbs_vortex_data(lbs_handle h, int32_t nrhs, const double *g,
                           int32_t n_vortices, const double *xyz_vortices,
                           const double *gamma, double *g_star, void *stream);

/* u (n_targets x nrhs) += sum_j Gamma_j G(x_t, v_j) at sphere targets
 * xyz_targets (n_targets x 3); a target on a vortex gives Inf. */
lbs_status lbs_vortex_field(lbs_handle h, int32_t nrhs, int32_t n_vortices,
                            const double *xyz_vortices, const double *gamma,
                            int64_t n_targets, const double *xyz_targets,
                            double *u, void *stream);

/* ---------------------------------------------------------------- adjoint
 * Derivatives of a scalar L(u) of the solution u = T x at targets, where
 * x = [sigma; A] solves the system of eqs. matrix_eqns with right-hand side
 * [2 g; 0] and T is the evaluation of eq. eqn:u_multi (Sections 4.1, 5):
 *   lambda = A^-T T^T w,  w = dL/du,
 *   dL/dg = 2 lambda_sigma,
 *   dL/dbeta = w^T (dT/dbeta) x - lambda^T (dA/dbeta) x,
 * beta = the 16 radius coefficients (a_1..a_8, b_1..b_8) of every island,
 * which move the nodes and with them xi, xi', xi'' (Section 3) in the
 * kernel, the log-source rows and the evaluation.  The node data g is a
 * vector held fixed when beta moves.  FP64 with the FMM of p64 terms
 * (lbs_solve_T also mixed).  Single-geometry handles (LBS_ERR_UNSUPPORTED otherwise, except
 * lbs_solve_T, which takes batch handles).  Device pointers, column-major
 * as in lbs_solve; calls are stream-ordered on `stream` and return after it
 * has drained. */

/* T^T w: gs (N x nrhs) = the double-layer part of the transposed
 * evaluation, ga (M x nrhs) = its log-source part, for target weights w
 * (n_targets x nrhs) at xyz_targets (n_targets x 3, as in lbs_eval; targets
 * at the north pole carry no Cauchy part).  n_targets = 0 gives zeros. */
lbs_status lbs_eval_T(lbs_handle h, int32_t nrhs, const double *w,
                      int64_t n_targets, const double *xyz_targets,
                      double *gs, double *ga, void *stream);

/* Solve A^T [lam_s; lam_a] = [rhs_s; rhs_a] (rhs_s, lam_s: N x nrhs;
 * rhs_a, lam_a: M x nrhs; rhs_a may be NULL for zeros) by GMRES with the
 * transposed block preconditioner on the right, to the relative residual
 * tol of the unpreconditioned transposed system, per system.  precision:
 * LBS_FP64, or LBS_MIXED (GMRES on the FP32 transposed FMM inside FP64
 * refinement, as in lbs_solve).  info as in lbs_solve (fp64_matvecs /
 * fp32_matvecs count transposed operator applications).
 * LBS_ERR_NO_CONVERGENCE when max_iter is reached; the iterate is still
 * written. */
lbs_status lbs_solve_T(lbs_handle h, int32_t precision, int32_t nrhs,
                       const double *rhs_s, const double *rhs_a, double tol,
                       double *lam_s, double *lam_a, lbs_solve_info *info_host,
                       void *stream);

/* dcoef (M x 16, island-major, coefficient order of lbs_island.coef) =
 * w^T (dT/dbeta) x - lambda^T (dA/dbeta) x for one solution (sigma: N,
 * A: M), the adjoint density lam_s (N; lambda's island part does not enter
 * because the constraint rows do not depend on the shape) and target
 * weights w (n_targets) at xyz_targets. */
lbs_status lbs_shape_vjp(lbs_handle h, const double *sigma, const double *A,
                         const double *lam_s, int64_t n_targets,
                         const double *xyz_targets, const double *w,
                         double *dcoef, void *stream);

/* Change the expansion orders of a handle (p64 in 20, 24, 30, 36, 40, 48;
 * p32 in 12, 16, 20, 24) without rebuilding its quadtree.  Drops the
 * cached evaluation plans and captured GMRES iterations.  Synchronous. */
lbs_status lbs_set_orders(lbs_handle h, int32_t p64, int32_t p32,
                          void *stream);

/* One measured setting of lbs_autotune: leaf size, the order that was
 * varied (p32 for a mixed application, p64 for an FP64 one, the other 0),
 * milliseconds per (I + K) application and its relative error
 * max|y - y_ref| / max|y_ref| against an FP64 order-48 reference. */
typedef struct {
  int32_t leaf_max, p32, p64, m2l_groups;
  double ms, err;
} lbs_tune_entry;

/* Autotuner of the FMM schedule for one geometry (arguments as lbs_setup):
 * for leaf sizes 24, 32, 48, 64, 96, 128 and orders p32 in 12..24 and p64
 * in 20..36 it times (I + K) on a fixed pseudo-random density and returns
 * in *best_host the base options (defaults if NULL) with the leaf size and
 * p32 of the fastest mixed application whose error is <= tol_mixed, and the
 * p64 of the fastest FP64 application on that leaf size with error
 * <= tol_fp64.  Every measured setting is written to entries_host (up to
 * max_entries; n_entries_host receives the count; both may be NULL).
 * LBS_ERR_UNSUPPORTED when no setting meets a tolerance.  Then, on the
 * chosen leaf size and p32, it times the FP32 M2L launch at 512, 1024 and
 * 2048 work-groups (entries with p32 set and m2l_groups nonzero) and keeps
 * the fastest in best_host->m2l_groups.  Synchronous; builds and destroys
 * one handle per leaf size and per launch shape. */
lbs_status lbs_autotune(const lbs_island *islands_host, int32_t n_islands,
                        const int32_t *nodes_per_curve_host,
                        const lbs_options *base_host, double tol_mixed,
                        double tol_fp64, void *stream, lbs_options *best_host,
                        lbs_tune_entry *entries_host, int32_t max_entries,
                        int32_t *n_entries_host);

/* lbs_autotune with an on-disk cache (for the callers that tune the same
 * geometry again, e.g. every run of a service): cache_path names a text
 * file of one line per tuned problem, keyed by a 64-bit FNV-1a hash of the
 * islands, the node counts, the base options, both tolerances, the device
 * (architecture name and compute-unit count) and the library build.  A hit
 * returns the stored best options and entries without touching the GPU; a
 * miss tunes and appends a line (a line that cannot be written only costs
 * the next call a new tuning).  *hit_host (may be NULL) tells which.
 * Concurrent writers append whole lines. */
lbs_status lbs_autotune_cached(const lbs_island *islands_host, int32_t n_islands,
                               const int32_t *nodes_per_curve_host,
                               const lbs_options *base_host, double tol_mixed,
                               double tol_fp64, void *stream, const char *cache_path,
                               lbs_options *best_host, lbs_tune_entry *entries_host,
                               int32_t max_entries, int32_t *n_entries_host,
                               int32_t *hit_host);

/* Per-stage GPU timing of operator applications.  With enable != 0 every
 * stage of every later lbs_matvec / lbs_solve call is bracketed by a pair
 * of HIP events recorded on the call's stream; lbs_stage_times waits for
 * them, returns the accumulated milliseconds and interval counts per stage
 * (n >= LBS_NSTAGES entries, indexed by LBS_STAGE_*) and resets them. */
enum { LBS_STAGE_STRENGTHS = 0, /* p_j = -i q_j sigma_j, tree order       */
       LBS_STAGE_UPWARD = 1,    /* leaf multipoles + M2M, all levels       */
       LBS_STAGE_L2L = 2,       /* L2L, all levels                         */
       LBS_STAGE_M2L = 3,       /* V-list M2L, all boxes                   */
       LBS_STAGE_P2L = 4,       /* X-list P2L, all boxes                   */
       LBS_STAGE_LEAF = 5,      /* L2P + W-list M2P + U-list P2P + row     */
                                /* assembly                                */
       LBS_STAGE_GAMMA = 6,     /* correction-term reduction               */
       LBS_STAGE_LOGSRC = 7,    /* log-source product E z                  */
       LBS_STAGE_CONSTRAINT = 8,/* F y and the Schur-complement solve      */
       LBS_NSTAGES = 9 };
lbs_status lbs_stage_timing(lbs_handle h, int32_t enable);
lbs_status lbs_stage_times(lbs_handle h, double *ms_host,
                           int64_t *launches_host, int32_t n);

/* Host-only step of the mixed-precision refinement of lbs_solve and
 * lbs_solve_T (no GPU needed): from the squared FP64 residual norms rn2 and
 * right-hand-side norms bn2 of S systems, the inner GMRES tolerance of each
 * system (itol: rn for a system with rn <= tol bn, which the inner solve
 * then skips; else max(inner_tol rn, tol bn / 2)) and *all_converged = 1
 * when every system meets tol.  LBS_ERR_NOT_FINITE when a norm is NaN, Inf
 * or negative: such a system is never taken as converged. */
lbs_status lbs_refine_tolerances_host(int32_t S, const double *rn2_host,
                                      const double *bn2_host, double tol,
                                      double inner_tol, double *itol_host,
                                      int32_t *all_converged_host);

/* Release a handle and its device memory.  NULL is accepted. */
lbs_status lbs_destroy(lbs_handle h);

/* Message for the last non-OK status returned on this host thread. */
const char *lbs_last_error(void);

/* Quadtree statistics of a handle: depth, boxes, leaves and the pair counts
 * of the four interaction lists (U: near-field leaf pairs, V: same-level
 * M2L pairs, W: multipole-to-target, X: source-to-local). */
typedef struct {
  int32_t levels, boxes, leaves, reserved;
  int64_t u_pairs, v_pairs, w_pairs, x_pairs;
  int64_t p2p_interactions; /* source-target point pairs of the U lists   */
  int64_t m2p_evals;        /* (W box, target point) multipole evaluations*/
  int64_t p2l_evals;        /* (X source point, box) local contributions  */
} lbs_tree_stats;
lbs_status lbs_tree_info(lbs_handle h, lbs_tree_stats *stats_host);

/* Host-only check of the quadtree builder (no GPU needed): builds the tree
 * for n planar points (x_host, y_host) with leaves of at most leaf_max
 * points and verifies that every ordered point pair (i, j), i != j, is
 * covered exactly once by the U, V, W and X lists.  *bad_pairs_host gets
 * the number of pairs covered zero or several times; stats_host may be
 * NULL.  O(n^2): for small n. */
lbs_status lbs_check_tree_host(const double *x_host, const double *y_host,
                               int64_t n, int32_t leaf_max,
                               int64_t *bad_pairs_host,
                               lbs_tree_stats *stats_host);

/* How set-up formed the Schur-complement inverses (eq. matrix_eqns_c):
 * *pivoted_host = 0 by Gauss-Jordan elimination in the natural order, 1 by
 * partial pivoting (options.schur_tol <= 0, or the natural order failed its
 * check); *omega_host = the probe backward error measured for the natural
 * order (largest over the geometries), -1 when it was not tried.  Either
 * pointer may be NULL.  Host only. */
lbs_status lbs_schur_info(lbs_handle h, int32_t *pivoted_host, double *omega_host);

/* Check of the Schur-complement inverse of the preconditioner (eq.
 * matrix_eqns_c): rebuilds every geometry's block S_g and returns in
 * *err_host the largest |S_g (S_g^-1 e_j) - e_j| over ncols unit vectors
 * e_j spread evenly over each block's columns (the GPU inverse from the
 * blocked Gauss-Jordan elimination of set-up).  Synchronous. */
lbs_status lbs_schur_residual(lbs_handle h, int32_t ncols, double *err_host,
                              void *stream);

/* Host-only check of the upward (M2M) and downward (L2L) pass programs (no
 * GPU needed): builds the tree of n planar points as lbs_check_tree_host
 * does, cuts its work boxes into components of at most cap LDS expansion
 * slots (16 .. 1024) and runs both programs on the host with scalar
 * stand-ins for the expansions (a multipole holds its box's source count, a
 * local its box's level).  *bad_host gets the number of wrong or
 * out-of-order results; rounds_host (may be NULL) the launches of the
 * upward and the downward pass. */
lbs_status lbs_check_passes_host(const double *x_host, const double *y_host,
                                 int64_t n, int32_t leaf_max, int32_t cap,
                                 int64_t *bad_host, int32_t *rounds_host);

/* Check of the GPU quadtree builder (needs a GPU): builds the tree and the
 * U, V, W, X lists for n device points (x, y) (and nt device targets
 * (tx, ty), or nt = 0 for targets = sources) with HIP kernels and with the
 * host builder, and sets *mismatches_host to the number of differing
 * entries over every box field, list and permutation (0: identical) and
 * *levels_host (may be NULL) to the depth.  Synchronous. */
lbs_status lbs_compare_trees(const double *x, const double *y, int64_t n,
                             const double *tx, const double *ty, int64_t nt,
                             int32_t leaf_max, int64_t *mismatches_host,
                             int32_t *levels_host, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LBS_H */
