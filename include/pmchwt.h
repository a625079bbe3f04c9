/*
 * pmchwt.h -- C ABI of the MI355X (gfx950) library for the Calderon-preconditioned
 * PMCHWT boundary element method of Kleanthous, Betcke, Hewett,
 * Escapil-Inchauspe, Jerez-Hanckes and Baran, "Accelerated Calderon
 * preconditioning for Maxwell transmission problems".
 *
 * The library assembles the Galerkin matrices of the electric (S) and magnetic
 * (C) boundary integral operators (Section 2) on Rao-Wilton-Glisson functions
 * of the primal mesh and on Buffa-Christiansen functions of the barycentric
 * mesh (Section 3.2), builds the multi-particle PMCHWT operator A and one of
 * the preconditioners I, A, D, D^i, D^e, S^i, S^e (Section 3.1), optionally
 * restricted to near-field interactions (the cutoff chi of Section 3.3), and
 * solves  M_P^-1 P M_A^-1 A x = M_P^-1 P M_A^-1 b  with restarted GMRES
 * (Section 3.2, Section 4).  Every step runs in HIP kernels on one GPU; the
 * host only builds mesh topology and index tables.
 *
 * Conventions
 *  - All functions return 0 (PMCHWT_OK) or a negative pmchwt_status; the
 *    message of the last failure is returned by pmchwt_last_error(ctx).
 *  - Input arrays are host memory owned by the caller and copied during the
 *    call.  Output arrays are caller-allocated host memory of the stated
 *    size.  All device memory is allocated and owned by the context and freed
 *    by pmchwt_destroy.
 *  - A context is not thread safe; use one per host thread.
 *  - Meshes: vertices double[nv*3] (x,y,z), triangles int32[nt*3] indexing
 *    them, counter-clockwise seen from the exterior medium (the normal n_m of
 *    Section 2 points outwards), closed, 2-manifold, no degenerate triangles.
 *  - Edges of a scatterer are numbered in lexicographic order of their
 *    (lower vertex, higher vertex) index pair.  T+ of an edge is the triangle
 *    that traverses it from its lower to its higher vertex.  RWG functions are
 *    in unit-flux form, (x - p+)/(2 A+) on T+ and -(x - p-)/(2 A-) on T-
 *    (the paper fixes no normalisation; physical outputs do not depend on it).
 *    BC function e is the Buffa-Christiansen function attached to edge e,
 *    oriented from its lower to its higher vertex.
 *  - Unknowns are scatterer-major: scatterer m holds [x_D (E_m); x_N (E_m)],
 *    the RWG coefficients of the scaled traces u^s_m = [gamma_D E^s;
 *    k_e gamma_N E^s] of Section 2 (mu = 1).
 *  - Complex numbers cross the ABI interleaved as pmchwt_complex.
 *  - Wavenumbers: k_m = k_e sqrt(eps_m) (principal root), mu = 1.
 */
#ifndef PMCHWT_H
#define PMCHWT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pmchwt_ctx pmchwt_ctx;

typedef struct {
  double re, im;
} pmchwt_complex;

typedef enum {
  PMCHWT_OK = 0,
  PMCHWT_ERR_INVALID_ARG = -1,   /* bad pointer, size, option or index */
  PMCHWT_ERR_INVALID_MESH = -2,  /* open, non-manifold, mis-oriented or degenerate mesh */
  PMCHWT_ERR_OUT_OF_MEMORY = -3, /* device allocation failed */
  PMCHWT_ERR_DEVICE = -4,        /* a HIP or rocSOLVER call failed */
  PMCHWT_ERR_NOT_CONVERGED = -5, /* GMRES hit max_iter; outputs hold the last iterate */
  PMCHWT_ERR_OVER_BUDGET = -6,   /* request larger than the server's HBM budget */
  PMCHWT_ERR_CANCELLED = -7,     /* server request cancelled */
  PMCHWT_ERR_STATE = -8,         /* call out of order (e.g. solve before assemble) */
  PMCHWT_PENDING = 1,            /* server request waiting for admission */
  PMCHWT_RUNNING = 2             /* server request admitted, not finished */
} pmchwt_status;

/* Preconditioning operator P (Section 3.1; cost per iteration in Table 1). */
typedef enum {
  PMCHWT_P_I = 0,     /* no preconditioner: GMRES on A itself                     */
  PMCHWT_P_A = 1,     /* P = A (classical Calderon)                               */
  PMCHWT_P_D = 2,     /* block diagonal of A: A^e_m + A^i_m per scatterer          */
  PMCHWT_P_D_INT = 3, /* A^i_m per scatterer                                      */
  PMCHWT_P_D_EXT = 4, /* A^e_m per scatterer                                      */
  PMCHWT_P_S_INT = 5, /* [[0, S^i_m/k_m], [-k_m S^i_m, 0]] per scatterer           */
  PMCHWT_P_S_EXT = 6  /* [[0, S^e_m/k_e], [-k_e S^e_m, 0]] per scatterer           */
} pmchwt_precond;

typedef enum { PMCHWT_FP64 = 0, PMCHWT_MIXED = 1 } pmchwt_precision;
typedef enum { PMCHWT_OP_S = 0, PMCHWT_OP_C = 1 } pmchwt_opkind;
typedef enum { PMCHWT_EXT = 0, PMCHWT_INT = 1 } pmchwt_medium;
typedef enum { PMCHWT_RWG = 0, PMCHWT_BC = 1 } pmchwt_space;

/* Quadrature and compression parameters of one operator family (the
 * bi-parametric parameters (chi, q) of Section 3.3).
 *   q_near, q_medium, q_far : orders 1..4 of the symmetric triangle rules
 *       (1, 3, 4, 6 points per triangle) for disjoint pairs with relative
 *       distance |c1 - c2| / max(diam) < 2, in [2, 4), >= 4.
 *   n_singular : Gauss-Legendre points per coordinate of the Sauter-Schwab
 *       rules for identical / shared-edge / shared-vertex pairs
 *       (paper's q_singular = 6 <-> 4, q_singular = 1 <-> 1), 1..8.
 *   chi : near-field cutoff, absolute length; an entry (i, j) of P is kept iff
 *       the bounding boxes of the supports of functions i and j are at most
 *       chi apart; chi < 0 means infinity.  Ignored for A (always dense).
 *   precision : PMCHWT_FP64, or PMCHWT_MIXED.  For A: disjoint pairs and
 *       operator storage in FP32, singular pairs in FP64.  For P: MIXED
 *       integrates the near-field BC entries in FP32 (pair classification in
 *       FP64, entries stored in FP64) and stores the inverted mass matrices
 *       M_A^-1 and M_A^-T in FP32.  All of this only perturbs the
 *       preconditioner, not the system that is solved.
 *   mass_method : how P's products apply M_A^-1 and M_A^-T (Section 3.2).
 *       0 = sparse inverse (FP32 values): row i of the inverse on the
 *       columns within mass_hops steps of M_A's sparsity graph, by a
 *       Chebyshev iteration on the spectrum interval [0.3, 1.05] (entries
 *       within about 1e-7 of the row maximum at 8 steps); an FP64 preconditioner refines
 *       each product once against the FP64 M_A (error squared).  A dense
 *       inverse replaces it if a row's column set exceeds 1024 or a column of
 *       M_A holds more than 24 entries.  1 = dense Gauss-Jordan inverse (rank
 *       updates on the matrix cores).  2 = dense inverse, MIXED by a
 *       Chebyshev iteration on the sparse M_A stopped at
 *       ||I - X M_A||_F / sqrt(n) <= 1e-6 (Gauss-Jordan if it does not get
 *       there), FP64 by Gauss-Jordan.  Dense inverses are read through a
 *       truncated CSR copy (entries below 2^-27 (MIXED) or 2^-52 (FP64, kept
 *       if under 40% dense) of their row's largest dropped) by products with
 *       fewer than 16 right-hand sides.  Zero-initialised structs get 0.
 *   operator_form : for A of a single scatterer, how products with one or
 *       two right-hand sides read it.  0 = automatic (symmetric tiles from
 *       4096 edges on), 1 = full rows, 2 = symmetric tiles: the upper
 *       128 x 128 tiles of the combined matrices (half the bytes; the
 *       operators are complex symmetric except where the singular rules
 *       give X_rc != X_cr, which a sparse correction restores exactly).
 *       Ignored for P and for several scatterers; 0 when zero-initialised.
 *   mass_hops : radius (steps of M_A's sparsity graph) of the column set of
 *       each row of the sparse inverse (mass_method 0), 1..8, with hops + 6
 *       Chebyshev steps.  0 = default: 8 for an FP64 preconditioner (entries
 *       within about 1e-7 of the row maximum, squared by the refinement), 6
 *       for MIXED (about 1e-6: the FP32 preconditioner only approximates P~,
 *       here to about 2e-5; GMRES needs the same iterations for radii 3..8
 *       on the benchmark sphere, and the smaller rows cut the bytes each
 *       product reads by about 1.7x).  Ignored for A.                        */
typedef struct {
  int32_t q_near, q_medium, q_far;
  int32_t n_singular;
  double chi;
  int32_t precision;
  int32_t mass_method;
  int32_t operator_form;
  int32_t mass_hops;
} pmchwt_assembly_opts;

/* Restarted GMRES (Section 4: tol 1e-5, restart 200).
 *   tol      : relative residual of the preconditioned system
 *   restart  : rho, Krylov vectors per cycle (1..1024)
 *   max_iter : total iteration cap
 *   ir_max   : outer iterative-refinement steps with an FP64 residual
 *              b - A x (0 = none).  With an A assembled in MIXED precision
 *              and ir_max > 0 the solve targets the FP64 system: the right-
 *              hand side's interior product and every residual use the
 *              matrix-free FP64 product of pmchwt_apply (which = 2, 3), and
 *              GMRES on the FP32 operators solves the correction equations,
 *              each right-hand side only as far as brings its FP64
 *              residual to half of tol (and at least by the factor tol). */
typedef struct {
  double tol;
  int32_t restart;
  int32_t max_iter;
  int32_t ir_max;
} pmchwt_solver_opts;

typedef struct {
  int32_t iterations;        /* total GMRES iterations R over all refinement steps     */
  int32_t converged;         /* 1 if every right-hand side met tol                      */
  int64_t matvecs;           /* boundary-operator applications, Table 1's unit          */
  double rel_residual;       /* worst final preconditioned relative residual            */
  int32_t ir_steps;          /* refinement steps performed                              */
  int32_t restarts;          /* completed GMRES cycles                                  */
  double ms_solve;           /* device time of the solve phase                          */
} pmchwt_solve_stats;

/* Per-phase device timings (HIP events on the context's stream) and the
 * algorithmic work of the last assemble / solve, for roofline reporting.     */
typedef struct {
  double ms_assemble_A;      /* regular + singular + scatter kernels of A               */
  double ms_assemble_regular;/* regular-pair kernel (pass 1) alone, sum over launches    */
  double ms_regular_combine; /* slot-row combination (pass 2) of the regular pairs      */
  double ms_assemble_singular;
  double ms_assemble_P;      /* near-field BC kernel                                    */
  double ms_mass;            /* mass and Gram matrices and their inverses               */
  int64_t regular_pairs;     /* ordered disjoint triangle pairs integrated, per k       */
  int64_t regular_point_pairs;
  int64_t singular_pairs;
  int64_t singular_point_pairs;
  int64_t bary_pairs;        /* barycentric triangle pairs integrated for P             */
  int64_t nnz_P;             /* stored entries per BC operator                          */
  int32_t regular_launches;  /* launches of the regular-pair kernel                     */
  int32_t n_wavenumbers;     /* wavenumbers per regular pair in the A kernels           */
  double recompute;          /* trial triangles integrated per test triangle / F        */
  double wall_setup;         /* host wall time of assemble: topology and uploads        */
  double wall_A;             /* ... assembly of A (host tables + kernels)               */
  double wall_P;             /* ... preconditioner (near-field pattern + kernel)        */
  double wall_mass;          /* ... mass / Gram matrices and the mass inverse           */
  double ms_matvec_total;    /* dense operator application kernels during the solve,
                                summed over the timed launches (matvec_timed: one
                                product in eight is timed, and every matrix-core
                                product)                                          */
  int64_t matvec_launches;
  int64_t matvec_bytes;      /* algorithmic operator bytes read by all those launches  */
  double ms_mfma_total;      /* many-RHS operator products on the matrix cores          */
  int64_t mfma_launches;
  int64_t mfma_flops;        /* real flops of those GEMMs (8 per complex MAC)           */
  int32_t mass_iterations;   /* Chebyshev steps of the last FP32 mass-matrix inverse
                                (0: Gauss-Jordan, always the case for FP64)          */
  double mass_residual;      /* ||I - X M_A||_F / sqrt(n) at its last check          */
  int64_t lookahead_discarded; /* Arnoldi steps queued ahead of a convergence and
                                  dropped (their operator products are not counted
                                  in the solve's matvecs)                            */
  double ms_matvec_reduce;   /* symmetric-tile products: the partial-sum and
                                correction kernel of the timed launches
                                (ms_matvec_total counts the tile kernel alone)    */
  int64_t matvec_timed;      /* GEMV launches whose time is in ms_matvec_total       */
  double ms_free_apply;      /* matrix-free FP64 products of a MIXED solve with
                                refinement: the FP64 right-hand side and the
                                refinement residuals                             */
  int64_t free_launches;
  double wall_tables_A;      /* host wall time of the geometry tables of A built by this
                                assemble (classification kernels with their scans and
                                read-backs, host layout work); 0 when reused          */
  double wall_tables_P;      /* ... of P: near-field pattern and dual-cell pair tables  */
  double wall_dual;          /* host wall time of the barycentric refinement and the
                                upload of its dual-cell tables (first assemble of a
                                geometry)                                             */
  double ms_fp64_copy;       /* device time of the FP64 copy of A that a MIXED solve
                                with refinement and 4 or more right-hand sides
                                assembles for its residuals (once per assemble)       */
} pmchwt_profile;

/* Version string of the library. */
const char *pmchwt_version(void);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * run all work on, or NULL for a stream owned by the context.               */
int pmchwt_create(pmchwt_ctx **out, int device, void *hip_stream);

/* Add scatterer Gamma_m with relative permittivity eps_r (mu_r = 1).
 * Validates the mesh (closed, consistently oriented, no zero-area
 * triangle); on failure returns PMCHWT_ERR_INVALID_MESH.                    */
int pmchwt_add_scatterer(pmchwt_ctx *ctx, const double *verts, int32_t nv, const int32_t *tris,
                         int32_t nt, pmchwt_complex eps_r, int32_t *scatterer_id_out);

/* Exterior wavenumber k_e > 0 (Section 2). */
int pmchwt_set_wavenumber(pmchwt_ctx *ctx, double k_ext);

/* Number of scatterers, edges E_m of scatterer m, total unknowns 2 sum E_m. */
int pmchwt_sizes(const pmchwt_ctx *ctx, int32_t *n_scatterers, int64_t *n_unknowns);
int pmchwt_num_edges(const pmchwt_ctx *ctx, int32_t m, int32_t *E_out);

/* Assemble A (RWG x RWG: S^e, C^e on all scatterers at k_e, S^i_m, C^i_m at
 * k_m), the BC operators the chosen preconditioner needs (near-field cutoff
 * P->chi), the mixed mass matrices M_A = <bc_j, rwg_i> (Section 3.2) and
 * their inverses, and the RWG Gram matrices used by the right-hand side.
 * Re-assembling replaces all previous operators.                              */
int pmchwt_assemble(pmchwt_ctx *ctx, const pmchwt_assembly_opts *A, const pmchwt_assembly_opts *P,
                    pmchwt_precond kind);

/* Copy one assembled Galerkin block to host.  op: S or C; medium: EXT (k_e)
 * or INT (k_m, only m == l); space: RWG (operators of A) or BC (operators of
 * P, zero outside the near field; only operators the preconditioner uses).
 * Block (m, l) has rows = functions of scatterer m, columns = of scatterer l;
 * out is row-major E_m x E_l with leading dimension ld >= E_l.              */
int pmchwt_get_block(pmchwt_ctx *ctx, pmchwt_opkind op, pmchwt_medium medium, pmchwt_space space,
                     int32_t m, int32_t l, pmchwt_complex *out, int64_t ld);

/* Same operators, n individual entries (rows[i], cols[i]) of block (m, l).  */
int pmchwt_get_entries(pmchwt_ctx *ctx, pmchwt_opkind op, pmchwt_medium medium, pmchwt_space space,
                       int32_t m, int32_t l, int64_t n, const int32_t *rows, const int32_t *cols,
                       pmchwt_complex *out);

/* Mixed mass matrix M_A of scatterer m, row-major E_m x E_m (rows RWG i,
 * columns BC j), real.                                                        */
int pmchwt_get_mass(pmchwt_ctx *ctx, int32_t m, double *out);

/* Galerkin right-hand side b_i = <(I/2 - D^i) u^inc, rwg_i> (Section 3.2) for
 * nrhs plane waves E^inc = p exp(i k_e d.x): dirs double[nrhs*3] unit, pols
 * pmchwt_complex[nrhs*3] with p.d = 0.  b_out[nrhs * N], N = unknowns.
 * The incident traces enter the identity term exactly and D^i through their
 * L2 projection onto RWG.                                                     */
int pmchwt_rhs(pmchwt_ctx *ctx, const double *dirs, const pmchwt_complex *pols, int32_t nrhs,
               pmchwt_complex *b_out);

/* y = Op x for nrhs vectors of length N.  which = 0: A, 1: the preconditioned
 * product M_P^-1 P M_A^-1 A (A alone for P = I), 2: A and 3: A^i (the
 * interior blocks of Section 2) with every entry integrated again in FP64 and
 * applied without storing it (the product of the FP64 Galerkin matrix also
 * when A is stored in FP32; it refines MIXED solves).                        */
int pmchwt_apply(pmchwt_ctx *ctx, int32_t which, const pmchwt_complex *x, int32_t nrhs,
                 pmchwt_complex *y);

/* Device-pointer forms (for callers whose vectors already live on the GPU,
 * e.g. torch tensors).  x_dev, y_dev, currents_dev, obs_dev and F_dev are
 * device pointers of the same sizes and layouts as the host arrays of the
 * plain forms (complex interleaved, scatterer-major [D_m ; N_m] per right-hand
 * side; obs_dev double[nobs*3]; F_dev nrhs*nobs*3), owned by the caller,
 * allocated through the HIP runtime this library runs on (the process's
 * libamdhip64) and not checked beyond null.  hip_stream is the caller's
 * hipStream_t of that runtime (NULL:
 * none): the context's work waits for what the caller enqueued on it before
 * the call, and the caller's later work on it waits for the outputs.
 * pmchwt_apply_device and pmchwt_far_field_device only enqueue (they return
 * before the outputs are written); pmchwt_solve_device takes its plane waves
 * from host memory, returns when the solve is done and writes the currents
 * to currents_dev.  Errors as for the plain forms.                          */
int pmchwt_apply_device(pmchwt_ctx *ctx, int32_t which, const pmchwt_complex *x_dev, int32_t nrhs,
                        pmchwt_complex *y_dev, void *hip_stream);
int pmchwt_solve_device(pmchwt_ctx *ctx, const double *dirs, const pmchwt_complex *pols, int32_t nrhs,
                        const pmchwt_solver_opts *opts, pmchwt_complex *currents_dev,
                        pmchwt_solve_stats *stats, void *hip_stream);
int pmchwt_far_field_device(pmchwt_ctx *ctx, const pmchwt_complex *currents_dev, int32_t nrhs,
                            const double *obs_dev, int32_t nobs, pmchwt_complex *F_dev, void *hip_stream);

/* Solve for the scattered traces of nrhs incident plane waves (see
 * pmchwt_rhs) with GMRES on the preconditioned system.  currents_out[nrhs*N].
 * Returns PMCHWT_ERR_NOT_CONVERGED (outputs still written) if max_iter is
 * reached before tol.  stats may be NULL.                                     */
int pmchwt_solve(pmchwt_ctx *ctx, const double *dirs, const pmchwt_complex *pols, int32_t nrhs,
                 const pmchwt_solver_opts *opts, pmchwt_complex *currents_out,
                 pmchwt_solve_stats *stats);

/* Far-field pattern F with E^s ~ exp(i k_e r)/r F(xhat) (Stratton-Chu,
 * Section 2) at nobs unit directions obs double[nobs*3], for nrhs current
 * vectors: F_out[nrhs * nobs * 3].                                            */
int pmchwt_far_field(pmchwt_ctx *ctx, const pmchwt_complex *currents, int32_t nrhs,
                     const double *obs, int32_t nobs, pmchwt_complex *F_out);

/* Total electric field at npts points (the Stratton-Chu representation of
 * Section 2 with the solved traces; the field maps of Section 5).  Outside
 * every scatterer E = E^inc + E^s, E^s = -sum_m [H^e(gamma_D E^s) +
 * E^e(gamma_N E^s)] at k_e; inside scatterer m the interior field
 * H^i_m(gamma_D E^i) + E^i_m(gamma_N E^i) at k_m, whose traces are the
 * solved ones plus the L2 projection of the incident traces onto RWG (the
 * transmission conditions).  currents[nrhs * N] as pmchwt_solve returned them
 * for the plane waves dirs / pols (same conventions); points double[npts*3];
 * E_out[nrhs * npts * 3] (point-major per right-hand side); region_out
 * int32[npts] or NULL: -1 outside, m inside scatterer m (decided by the solid
 * angle each closed surface subtends).  The surface integrals use the 6-point
 * rule on every triangle: accurate at points farther from the surface than
 * about one triangle size.  Errors: STATE before pmchwt_assemble,
 * INVALID_ARG.                                                                */
int pmchwt_near_field(pmchwt_ctx *ctx, const pmchwt_complex *currents, int32_t nrhs, const double *dirs,
                      const pmchwt_complex *pols, const double *points, int32_t npts, pmchwt_complex *E_out,
                      int32_t *region_out);

/* pmchwt_far_field without any device allocation, for callers that cannot
 * allocate device memory while they run (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, layout and
 * result as pmchwt_far_field (host arrays, copied during the call).  Every
 * device buffer it needs (currents, directions, quadrature points, weighted
 * currents, partial sums, F) lives in one static device array of 64 MiB per GPU,
 * held from the first pmchwt_create on that GPU until the process ends; the
 * call makes no hipMalloc, hipFree or other allocating device call.  Needs the
 * geometry on the device: call pmchwt_assemble first (else PMCHWT_ERR_STATE).
 * Sizes whose buffers exceed the 64 MiB return PMCHWT_ERR_INVALID_ARG (at the
 * 5120-triangle sphere: up to 15 right-hand sides with the 8192-direction
 * cross-section grid).  All calls on one GPU share the array: calls that
 * overlap on one GPU (several host threads or streams) race and must not be
 * issued.  The partial sums may be split into fewer segments than in
 * pmchwt_far_field, so results agree to rounding.                           */
int pmchwt_far_field_noalloc(pmchwt_ctx *ctx, const pmchwt_complex *currents, int32_t nrhs,
                             const double *obs, int32_t nobs, pmchwt_complex *F_out);

/* Extinction (optical theorem, (4 pi / k_e) Im(p* . F(d))) and scattering
 * (integral of |F|^2 over the sphere, 64 Gauss-Legendre nodes in cos(theta)
 * x 128 uniform nodes in phi) cross sections for nrhs solutions.            */
int pmchwt_cross_sections(pmchwt_ctx *ctx, const pmchwt_complex *currents, int32_t nrhs,
                          const double *dirs, const pmchwt_complex *pols, double *sigma_ext,
                          double *sigma_sca);

/* Host-only view of the Buffa-Christiansen construction (Section 3.2; no GPU
 * and no context needed).  For a mesh (same conventions as
 * pmchwt_add_scatterer) every BC function e restricted to a barycentric
 * child c = 6 t + j of its support is an RT0 field  alpha x - w.  Writes
 * `count` records: ids[2q] = e, ids[2q+1] = c, vals[4q..4q+3] =
 * (alpha, wx, wy, wz).  Pass ids = vals = NULL to query count first; on the
 * second call *count must hold the capacity.                                */
int pmchwt_bc_fields(const double *verts, int32_t nv, const int32_t *tris, int32_t nt, int64_t *count,
                     int32_t *ids, double *vals);

/* Timings and work counters of the last assemble and solve. */
int pmchwt_get_profile(const pmchwt_ctx *ctx, pmchwt_profile *out);

/* Message of the last failing call on ctx ("" if none).  Owned by ctx. */
const char *pmchwt_last_error(const pmchwt_ctx *ctx);

/* Free every device and host resource of ctx.  NULL is allowed. */
void pmchwt_destroy(pmchwt_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Serving: a request loop on one GPU with continuous batching.
 *
 * Callers that submit many independent scattering problems (different
 * meshes, sizes, wavenumbers, incident fields) and want them solved while
 * others are still running.  A server owns two host threads:
 *  - an admission thread takes requests in submission order.  It admits one
 *    when the summed device-memory estimate of the live requests plus its own
 *    stays within hbm_budget_bytes and fewer than max_live are live.  It then
 *    assembles the request on its own context and stream (the same work as
 *    pmchwt_assemble and the right-hand side of pmchwt_solve).
 *  - an engine thread advances every live request by one Krylov step per round.
 *    The operator products of all live requests with fewer than 16
 *    right-hand sides go out in grouped launches (one kernel carries the
 *    products of many requests); the rest of each step runs on the request's
 *    stream, so the requests' work overlaps on the device.
 * Assemblies of newly admitted requests overlap with the rounds.  A request's
 * arithmetic does not depend on what else is live: its results are the same
 * alone and in any mix.  Finished requests release their device memory
 * before the next admission.
 * The server functions are thread safe.
 * ------------------------------------------------------------------------- */
typedef struct pmchwt_server pmchwt_server;

typedef struct {
  size_t hbm_budget_bytes; /* admission limit on the summed device estimates   */
  int32_t max_live;        /* requests admitted at once, 1..256                 */
} pmchwt_server_opts;

/* One scattering problem: the arguments of pmchwt_add_scatterer (per
 * scatterer), pmchwt_set_wavenumber, pmchwt_assemble and pmchwt_solve.  All
 * arrays are copied during pmchwt_server_submit.                               */
typedef struct {
  int32_t n_scatterers;
  const double *const *verts;   /* [n_scatterers] -> double[nv[m]*3]            */
  const int32_t *nv;
  const int32_t *const *tris;   /* [n_scatterers] -> int32[nt[m]*3]             */
  const int32_t *nt;
  const pmchwt_complex *eps_r;  /* [n_scatterers]                               */
  double k_ext;
  int32_t nrhs;
  const double *dirs;           /* nrhs*3 unit                                  */
  const pmchwt_complex *pols;   /* nrhs*3, p.d = 0                              */
  pmchwt_assembly_opts opts_A, opts_P;
  int32_t precond;              /* pmchwt_precond                               */
  pmchwt_solver_opts solver;
} pmchwt_request;

typedef struct {
  int32_t status;          /* PMCHWT_PENDING, PMCHWT_RUNNING, PMCHWT_OK or an error
                              (PMCHWT_ERR_NOT_CONVERGED: results still written) */
  int32_t nrhs;
  int64_t n_unknowns;      /* N = 2 sum_m E_m                                    */
  int64_t device_bytes;    /* admission estimate                                 */
  double ms_queued;        /* submission -> admission                            */
  double ms_total;         /* submission -> results ready                        */
  pmchwt_solve_stats stats;
} pmchwt_result;

typedef struct {
  int64_t submitted, completed, failed, live, pending;
  int64_t rounds;           /* engine rounds                                      */
  int64_t max_live_seen;    /* most requests live in one round                    */
  int64_t grouped_launches; /* grouped operator launches                          */
  int64_t grouped_jobs;     /* products carried by them                           */
  int64_t bytes_in_use;     /* estimates of the live requests                     */
} pmchwt_server_stats;

/* Start a server on `device`.  Errors: INVALID_ARG, DEVICE, OUT_OF_MEMORY. */
int pmchwt_server_create(pmchwt_server **out, int device, const pmchwt_server_opts *opts);
/* Queue a request; *ticket identifies it.  Errors: INVALID_ARG (bad sizes or
 * options), INVALID_MESH (detected before admission), OVER_BUDGET (the
 * estimate alone exceeds the budget).                                         */
int pmchwt_server_submit(pmchwt_server *s, const pmchwt_request *req, uint64_t *ticket);
/* Current state of a request (res->status is PENDING, RUNNING, OK or an
 * error).  Returns INVALID_ARG for an unknown ticket.                         */
int pmchwt_server_poll(pmchwt_server *s, uint64_t ticket, pmchwt_result *res);
/* Block until the request has finished or timeout_ms (< 0: no limit) passed;
 * returns PMCHWT_OK when finished (res->status tells how), PMCHWT_RUNNING on
 * timeout.                                                                    */
int pmchwt_server_wait(pmchwt_server *s, uint64_t ticket, double timeout_ms, pmchwt_result *res);
/* Copy the results of a finished request and forget it: currents[nrhs * N]
 * (layout of pmchwt_solve), sigma_ext[nrhs], sigma_sca[nrhs]; any pointer may
 * be NULL.  Errors: INVALID_ARG (unknown ticket), STATE (not finished).       */
int pmchwt_server_fetch(pmchwt_server *s, uint64_t ticket, pmchwt_complex *currents, double *sigma_ext,
                        double *sigma_sca);
/* Cancel a pending or running request (its status becomes CANCELLED). */
int pmchwt_server_cancel(pmchwt_server *s, uint64_t ticket);
int pmchwt_server_get_stats(pmchwt_server *s, pmchwt_server_stats *out);
/* Finish the live requests' current round, cancel the rest, join the threads
 * and free everything.                                                        */
void pmchwt_server_destroy(pmchwt_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PMCHWT_H */
