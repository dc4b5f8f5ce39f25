/*
 * bemcap.h -- C ABI of the MI355X (gfx950) library for the P0 Galerkin
 * boundary element computation of the electrostatic capacity of a
 * polyhedron (Betcke, Haberl, Praetorius: "Adaptive boundary element methods
 * for the computation of the electrostatic capacity on complex polyhedra").
 *
 * Problem (Section 1.4, eqs. "laplace_integral" and "cap"; Section 2.7,
 * eq. "cap:ell"; the primal P0 Galerkin system of Appendix A,
 * eq. "discreteform:residual"):
 *
 *   V[i][j] = (1/4pi) int_{T_i} int_{T_j} 1/|x - y| dy dx,
 *   b[i]    = |T_i|,     V sigma = b,     Cap = (1/4pi) sum_i sigma_i |T_i|.
 *
 * The paper's own discretisation (Algorithm 1, step (i); Section 2.6) is
 * provided too: the Galerkin system on the dual mesh, built from V on the
 * barycentric refinement and solved with the hypersingular operator as
 * preconditioner (bc_dual_*).
 *
 * Conventions shared by every call
 *   - All functions are extern "C" and reentrant, and keep no state between
 *     calls: everything a later call needs lives in caller-owned buffers.
 *   - The library never allocates device memory: the caller passes device
 *     buffers (inputs, outputs and a workspace whose size the matching
 *     *_bytes function returns) and owns all of them.
 *   - "d_" pointers are device pointers, "h_" pointers host pointers.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *     enqueued on it; calls marked ASYNC return before the work finishes and
 *     their device outputs are valid after the stream is synchronised.
 *   - Argument, size and workspace errors are returned synchronously as a
 *     negative bc_status and nothing is enqueued.  Outcomes of device work
 *     (no convergence, breakdown) are written to the device result struct.
 *   - Meshes: vertices are M x 3 float64 row-major (x, y, z); triangles are
 *     N x 3 int32 row-major vertex indices.  The surface must be a closed,
 *     conforming, welded triangulation into plane triangles (Section 2.1);
 *     bc_mesh_check verifies this on the host.
 *   - Dense matrices are row-major N x ld with ld = bc_matrix_ld(N) (N rounded
 *     up to a multiple of 64); columns N..ld-1 are written as zeros.
 */
#ifndef BEMCAP_H
#define BEMCAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *bc_stream; /* a hipStream_t */

typedef enum bc_status {
  BC_OK = 0,
  BC_EINVAL = -1,      /* bad argument, size or option */
  BC_EMESH = -2,       /* mesh fails the validity check */
  BC_ENOMEM = -3,      /* workspace smaller than required */
  BC_EDEVICE = -4,     /* HIP runtime error (launch, copy, device query) */
  BC_ENOCONV = -5,     /* iteration limits reached before the tolerance */
  BC_EBREAKDOWN = -6,  /* p^T V p <= 0: the matrix is not positive definite */
  BC_ETIMEOUT = -7,    /* a cross-workgroup barrier exceeded its spin limit */
  BC_RUNNING = 1       /* batched solve: system not finished yet */
} bc_status;

typedef enum bc_precision {
  BC_FP64 = 0,  /* FP64 matrix, FP64 Krylov iterations */
  BC_MIXED = 1, /* FP32 matrix (far field computed in FP32, touching and
                   near pairs computed in FP64 and kept as an FP64 sparse
                   correction), FP32 CG with FP32 accumulation inside FP64
                   iterative refinement of the residual b - V sigma */
  BC_F32_F64 = 2 /* bc_matvec only: the FP32 matrix of a BC_MIXED assembly
                   applied to FP64 vectors with FP64 sums (the dense part
                   of the mixed dual system's products) */
} bc_precision;

/* ------------------------------------------------------------------------ */
/* Version, status text, sizes                                              */
/* ------------------------------------------------------------------------ */

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int32_t bc_version(void);

/* Static text for a status code; never NULL. */
const char *bc_status_string(int32_t status);

/* Leading dimension of a dense N x N matrix: N rounded up to 64. */
int64_t bc_matrix_ld(int64_t N);

/* Bytes of the dense matrix: N * ld * (8 for BC_FP64, 4 for BC_MIXED). */
size_t bc_matrix_bytes(int64_t N, int32_t precision);

/* ------------------------------------------------------------------------ */
/* Mesh validation (host)                                                   */
/* ------------------------------------------------------------------------ */

/* Section 2.1: a conforming triangulation of a closed polyhedral surface into
 * plane triangles.  Rejects (BC_EMESH): N < 4 or M < 4, non-finite
 * coordinates, indices outside [0, M), a triangle repeating a vertex, zero
 * area, duplicate (unwelded) vertex coordinates, unused vertices, and edges
 * not shared by exactly two triangles.  On failure *h_bad_index (if not NULL)
 * receives the offending triangle or vertex index (-1 if none applies).
 * Host memory only; no device work. */
int32_t bc_mesh_check(const double *h_verts, int64_t M, const int32_t *h_tris,
                      int64_t N, int64_t *h_bad_index);

/* ------------------------------------------------------------------------ */
/* Assembly: geometry, pair classification, dense V                        */
/* ------------------------------------------------------------------------ */

typedef struct bc_assembly_opts {
  int32_t far_order;  /* collapsed Gauss rule with far_order^2 points per
                         triangle for pairs sharing no vertex; 1..4, default 4 */
  int32_t ss_order;   /* Gauss points per coordinate of the 4-D singular
                         rules (coincident 6, edge 4, vertex 2 subdomains);
                         1..8, default 4 */
  int32_t precision;  /* bc_precision */
  int32_t far_low;    /* far_order 4: 1 integrates pairs of 64-element
                         blocks whose bounding boxes are far apart with
                         Radon's 7-point rule of degree 5 on each triangle
                         (49 instead of 256 point pairs): BC_MIXED from 8
                         largest element diameters, where its relative error
                         is at most 6e-10, below the FP32 rounding of the
                         stored entry (6e-8); BC_FP64 from 32 diameters,
                         where it is at most 1.4e-13.  0: one far rule
                         everywhere.  Ignored for far_order < 4.  The tile
                         lists it uses are built by bc_prepare, so
                         bc_prepare must have run on the mesh workspace (with
                         the same options) before bc_assemble. */
  double near_factor; /* BC_MIXED: pairs sharing no vertex with
                         |c_i - c_j|^2 < near_factor^2 max(diam_i, diam_j)^2
                         are computed in FP64 and corrected exactly; 0 = none.
                         Must be 0 for BC_FP64. */
  /* Orders of the singular rules chosen per touching pair (0 = off; all
   * zero gives ss_order everywhere).  ss_order is then the coincident
   * pairs' order. */
  int32_t ss_order_edge;   /* edge-adjacent pairs; 0: ss_order; 0..8 */
  int32_t ss_order_vertex; /* vertex-adjacent pairs; 0: ss_order; 0..8 */
  int32_t ss_order_sliver; /* > 0: at least this order for every touching
                              pair with an element whose diam^2 exceeds
                              sliver_ratio |T|.  The rules lose accuracy on
                              thin elements: the coincident integral of a
                              triangle with angles (10, 85, 85) degrees
                              (diam^2/|T| = 11.5) is off by 2.4e-3 at order
                              4 and 2.7e-5 at order 8; with angles
                              (10, 10, 160) (22.7) by 8.7e-2 and 1.6e-2.
                              0..8 */
  int32_t reserved;        /* must be 0 */
  double sliver_ratio;     /* > 0 when ss_order_sliver > 0 */
} bc_assembly_opts;

/* Sparse pattern produced by bc_prepare: every ordered pair (i, j) that
 * shares a vertex with, or is near, element i.  Counts of unordered pairs
 * (i <= j) by class are reported as well. */
typedef struct bc_pattern_info {
  int64_t nnz;          /* ordered entries of the pattern (both (i,j),(j,i)) */
  int64_t n_coincident; /* = N */
  int64_t n_edge;       /* unordered edge-adjacent pairs */
  int64_t n_vertex;     /* unordered pairs sharing exactly one vertex */
  int64_t n_near;       /* unordered near pairs (BC_MIXED) */
} bc_pattern_info;

/* Workspace for the mesh tables (geometry, quadrature points of the 4 x 4
 * rule and the distant tiles' 7-point rule, row pointers of the pattern, and the far-field tile lists:
 * the 64 x 64 element tiles of the upper block triangle by class, near or
 * diagonal / separated / at least 8 element diameters apart).  Depends on
 * N only. */
size_t bc_mesh_workspace_bytes(int64_t N);

/* Workspace for the pattern itself (row pointers, and column, class and row
 * of each entry, plus the FP64 correction values for BC_MIXED). */
size_t bc_pattern_bytes(int64_t N, int64_t nnz, int32_t precision);

/* Element geometry, pair classification (Section 2.1: pairs are told apart
 * by shared vertex indices of the conforming mesh) and the far-field tile
 * lists.  For BC_MIXED it also measures the mean relative error of the FP32
 * hardware inverse square root (a fixed computation on fixed inputs), which
 * the FP32 far field divides out of every entry.  Fills d_mesh_ws and
 * writes the pattern sizes to *h_info.  SYNCHRONOUS (waits for `stream`),
 * because the caller needs nnz to size the pattern buffer.  d_verts, d_tris
 * must stay unchanged until bc_assemble and bc_zz_indicators have run. */
int32_t bc_prepare(const double *d_verts, int64_t M, const int32_t *d_tris,
                   int64_t N, const bc_assembly_opts *opts, void *d_mesh_ws,
                   size_t mesh_ws_bytes, bc_pattern_info *h_info,
                   bc_stream stream);

/* Dense Galerkin matrix (Appendix A, eq. "discreteform:residual"; kernel of
 * eq. "strongform").  Pairs sharing no vertex use the collapsed Gauss rule
 * (FP64 for BC_FP64, FP32 with FP64-formed centroid differences for
 * BC_MIXED, Radon's 7-point rule on distant tiles with opts->far_low); touching pairs use the Sauter-Schwab-type rules in FP64; in
 * BC_MIXED near pairs are recomputed in FP64 too and d_pattern receives the
 * FP64 correction V64 - (double)(float)V64 of every pattern entry.  Only
 * i <= j is integrated; V[j][i] = V[i][j] exactly.  d_V: N x ld, double
 * (BC_FP64) or float (BC_MIXED).  opts must equal those given to bc_prepare.
 * ASYNC. */
int32_t bc_assemble(const double *d_verts, int64_t M, const int32_t *d_tris,
                    int64_t N, const bc_assembly_opts *opts,
                    const void *d_mesh_ws, size_t mesh_ws_bytes,
                    void *d_pattern, size_t pattern_bytes, int64_t nnz,
                    void *d_V, bc_stream stream);

/* Element areas |T_i| (the load vector b) from the mesh workspace, FP64,
 * length N.  ASYNC. */
int32_t bc_areas(const void *d_mesh_ws, int64_t N, double *d_area,
                 bc_stream stream);

/* ------------------------------------------------------------------------ */
/* Solve and capacity                                                       */
/* ------------------------------------------------------------------------ */

typedef struct bc_solve_opts {
  double rtol;        /* stop when ||b - A sigma||_2 <= rtol ||b||_2, with the
                         residual formed in FP64 (A = V, plus the FP64
                         correction in BC_MIXED); default 1e-12 (FP64) */
  double inner_rtol;  /* each inner CG run stops at ||r_k|| <= inner_rtol
                         ||r_0||; default 1e-13 (FP64), 1e-5 (BC_MIXED) */
  int32_t max_iter;   /* cap on CG iterations (matrix products) in total */
  int32_t max_outer;  /* cap on FP64 residual evaluations */
  int32_t jacobi;     /* 1: diagonal (Jacobi) preconditioning */
  int32_t x0_given;   /* 1: start from the caller's sigma; 0: from zero */
  double cap_rtol;    /* 0: off.  > 0: also stop once the capacity's
                         algebraic error is estimated below cap_rtol
                         (relative).  The capacity is reported as
                         (1/4pi) J(sigma), J(x) = 2 b^T x - x^T A x
                         = b^T x + x^T r with r = b - A x the last FP64
                         residual; for symmetric positive definite A it falls
                         short of the exact discrete capacity by exactly
                         (1/4pi) ||sigma* - sigma||_A^2 (the algebraic form of
                         Section 2.7's Proposition: the capacity error is the
                         squared energy error), so the capacity converges
                         twice as fast as the residual.  Each inner CG run
                         estimates that error from its steps: the sum of its
                         last four terms alpha_j gamma_j is the drop of the
                         squared energy error over those steps, a lower
                         bound on the error four steps back and above the
                         current error once that error halves over four
                         steps (Hestenes and Stiefel); the run stops once
                         the estimate is below 0.3 cap_rtol J; the
                         following FP64 residual step stops the solve once
                         it is below cap_rtol J.  Independently, the solve
                         also stops once ||sigma|| ||r|| <= cap_rtol
                         |b^T sigma|, a first-order bound that needs no CG
                         run (a converged initial guess).  Must be finite
                         and < 1. */
  int32_t spin_limit; /* 0: default (2^22 polls of about 64 clocks each).
                         > 0: bound on the polls of every cross-workgroup
                         wait of the solver; a wait that exceeds it ends the
                         solve with BC_ETIMEOUT (every workgroup leaves its
                         loop, nothing hangs).  A small value forces that
                         path, for tests of failure handling.  Must be
                         >= 0. */
  int32_t reserved;   /* must be 0 */
} bc_solve_opts;

/* Device-side result, written when a system finishes. */
typedef struct bc_result {
  double cap;          /* (1/4pi) (b^T sigma + sigma^T r), b = |T|, r the
                          last FP64 residual: (1/4pi) sum_i sigma_i |T_i| at
                          the exact discrete solution, and below it by
                          (1/4pi) ||sigma* - sigma||_A^2 otherwise (see
                          bc_solve_opts.cap_rtol); FP64, fixed-order sums */
  double rel_residual; /* ||b - A sigma|| / ||b|| at the last FP64 residual */
  int32_t iters;       /* CG iterations (matrix products with V) */
  int32_t outer;       /* FP64 residual evaluations */
  int32_t status;      /* BC_OK, BC_ENOCONV, BC_EBREAKDOWN, BC_ETIMEOUT, or
                          BC_RUNNING while a chunked batch is unfinished */
  int32_t precision;
  double cap_bound;    /* estimate of Cap's relative algebraic error: with
                          cap_rtol > 0 after a CG run, the last run's
                          estimate of ||sigma* - sigma||_A^2 / J(sigma);
                          otherwise ||sigma|| ||b - A sigma|| / |b^T sigma|,
                          a first-order bound (see bc_solve_opts.cap_rtol);
                          0 if not finished */
} bc_result;

/* Workspace of one system's solver state.  Depends on N and precision. */
size_t bc_solve_workspace_bytes(int64_t N, int32_t precision);

/* Number of workgroups the solver gives a system of size N.  It depends on N
 * only, so a system's arithmetic (row bands, reduction order) is the same
 * alone and inside any batch. */
int32_t bc_solve_workgroups(int64_t N);

/* Krylov solve of V sigma = b (Section 2.5, Remark (ii): CG applies since V
 * is symmetric positive definite) with b = |T| read from d_area, followed by
 * the capacity reduction (eq. "cap:ell").  One persistent cooperative
 * launch: CG in the Chronopoulos-Gear form (one matrix product and two
 * cross-workgroup barriers per iteration), restarted from FP64 residuals.
 * d_V, d_pattern as produced by bc_assemble (d_pattern may be NULL and
 * nnz 0 for BC_FP64).  d_sigma (FP64, length N) is the initial guess if
 * opts->x0_given and receives the solution.  d_result: one bc_result.
 * ASYNC. */
int32_t bc_solve(const void *d_V, int64_t N, int32_t precision,
                 const void *d_pattern, int64_t nnz, const double *d_area,
                 double *d_sigma, const bc_solve_opts *opts, void *d_ws,
                 size_t ws_bytes, bc_result *d_result, bc_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bc_solve
 * with the solver workspace in a 96 MiB device array instead of a caller
 * buffer, enough for any N up to 32000 in either precision; larger systems
 * return BC_ENOMEM (use bc_solve).  Same kernels, arithmetic and results as
 * bc_solve.  Exported by the companion library libbemcap_static.so (link
 * -lbemcap_static -lbemcap), which holds the array, so that only processes
 * that load it pay for it.  Allocates nothing: each GPU that runs the
 * companion library holds its own copy of the array until the process ends,
 * and the first call on a device looks up that copy's address.  Every call on one GPU shares the
 * array, so calls that overlap on one GPU (other streams, other threads)
 * race; the caller serialises them.  ASYNC. */
int32_t bc_solve_static(const void *d_V, int64_t N, int32_t precision,
                        const void *d_pattern, int64_t nnz,
                        const double *d_area, double *d_sigma,
                        const bc_solve_opts *opts, bc_result *d_result,
                        bc_stream stream);

/* One system of a batched solve (all pointers device pointers). */
typedef struct bc_system {
  const void *V;        /* N x ld matrix of `precision` */
  const void *pattern;  /* bc_assemble pattern (NULL allowed for BC_FP64) */
  const double *area;   /* b = |T| */
  double *sigma;        /* initial guess / solution */
  void *ws;             /* bc_solve_workspace_bytes(N, precision) bytes */
  bc_result *result;    /* device result */
  int64_t N;
  int64_t nnz;
  int32_t precision;
  int32_t start;        /* 1: (re)initialise this system's state; 0: resume */
  int32_t iter_budget;  /* > 0: this system's bound on matrix products in
                           this launch (overrides the call's iter_budget) */
  int32_t reserved;     /* must be 0 */
} bc_system;

/* Bytes of device scratch for the descriptors of a batch of n_sys systems. */
size_t bc_batch_scratch_bytes(int32_t n_sys);

/* Batched persistent solve: every system gets bc_solve_workgroups(N)
 * workgroups of one cooperative launch and runs the same state machine as
 * bc_solve.  iter_budget > 0 (or a system's own iter_budget > 0) bounds the
 * matrix products a system may do in this launch (continuous batching:
 * unfinished systems report BC_RUNNING and resume, bitwise identically, in
 * a later call with start = 0); iter_budget <= 0 runs every system without
 * a bound of its own to completion.  All
 * systems must share one precision.  The total workgroup count must not
 * exceed bc_solve_capacity().  h_sys is copied to d_scratch.  ASYNC. */
int32_t bc_solve_batched(int32_t n_sys, const bc_system *h_sys,
                         const bc_solve_opts *opts, int32_t iter_budget,
                         void *d_scratch, size_t scratch_bytes,
                         bc_stream stream);

/* Workgroups one cooperative solver launch may use on the current device. */
int32_t bc_solve_capacity(int32_t precision);

/* Capacity (1/4pi) sum_i sigma_i |T_i| in FP64 with a fixed summation order
 * (eq. "cap:ell"), written to *d_cap.  ASYNC. */
int32_t bc_capacity(const double *d_sigma, const double *d_area, int64_t N,
                    double *d_cap, bc_stream stream);

/* ------------------------------------------------------------------------ */
/* ZZ-type error indicators                                                 */
/* ------------------------------------------------------------------------ */

/* eta(T)^2 = h_T ||sigma_T - I sigma||^2_{L2(T)} (eq. "zz:T", Section 2.4)
 * for the P0 density sigma: I sigma is the S^1 function whose value at a
 * vertex is the area-weighted mean of sigma over the elements containing it
 * (increasing element order), and the L2 norm is evaluated in closed form.
 * h_mode 0: h_T = diam(T) (eq. "zz:T"); 1: h_T = |T|^(1/2).  Needs the mesh
 * workspace and pattern from bc_prepare / bc_assemble.  d_eta2: FP64,
 * length N.  ASYNC. */
int32_t bc_zz_indicators(const int32_t *d_tris, int64_t N,
                         const void *d_mesh_ws, const void *d_pattern,
                         int64_t nnz, const double *d_sigma, int32_t h_mode,
                         double *d_eta2, bc_stream stream);

/* ------------------------------------------------------------------------ */
/* Weighted-residual error estimator                                        */
/* ------------------------------------------------------------------------ */

/* Device scratch of bc_residual_indicators: per element 3 partial moments
 * per column chunk (the chunk count depends on N only) and 3 moments per
 * pattern entry.  0 for N < 1 or nnz < N. */
size_t bc_residual_workspace_bytes(int64_t N, int64_t nnz);

/* mu(T)^2 = diam(T) ||grad_G (1 - V Phi)||^2_{L2(T)} (Appendix A, eq.
 * "residual:indicator") for the P0 density Phi = d_sigma, with the
 * residual evaluated in the discontinuous piecewise linears (as the paper's
 * remark on the estimator's cost describes): on each element the L2
 * projection of 1 - V Phi onto the linear functions, whose surface gradient
 * is constant.  It needs the first moments m_k(T) = <V Phi, lambda_k>_T
 * (lambda_k the barycentric coordinate of the k-th input vertex of T),
 * computed in FP64 without storing a matrix: the collapsed Gauss rule of
 * opts->far_order on both triangles for pairs sharing no vertex, the
 * singular rules of opts->ss_order for touching pairs; O(N^2) point pairs
 * like the assembly (all ordered pairs).  Then
 * mu(T)^2 = 36 diam(T) |sum_k m_k (P_{k+2} - P_{k+1})|^2 / |T|^3.
 * d_mesh_ws, d_pattern, nnz and opts as given to bc_prepare / bc_assemble
 * (either precision: near entries of a mixed pattern take the regular rule
 * here).  d_mu2: N FP64; d_moments: NULL or N x 3 FP64 (m_k per element).
 * Fixed summation order.  ASYNC. */
int32_t bc_residual_indicators(const double *d_verts, const int32_t *d_tris,
                               int64_t N, const bc_assembly_opts *opts,
                               const void *d_mesh_ws, const void *d_pattern,
                               int64_t nnz, const double *d_sigma,
                               double *d_mu2, double *d_moments, void *d_ws,
                               size_t ws_bytes, bc_stream stream);

/* ------------------------------------------------------------------------ */
/* Standalone product with a stored matrix                                  */
/* ------------------------------------------------------------------------ */

/* Device scratch for bc_matvec with nrhs vectors (x padded to the leading
 * dimension, partial sums of the symmetric product: about 2% of the FP32
 * matrix per vector).  0 for an unsupported combination. */
size_t bc_matvec_workspace_bytes(int64_t N, int32_t precision, int32_t nrhs);

/* Y = V X for a matrix from bc_assemble (row-major N x bc_matrix_ld(N); only
 * the diagonal 128 x 128 blocks and the entries right of them are read,
 * V being symmetric).  X and Y hold nrhs vectors of N entries one after the
 * other; all of them share one pass over V.  BC_FP64: V, X, Y are FP64,
 * nrhs 1 or 3; BC_MIXED: FP32 (products accumulated in FP32), nrhs 1;
 * BC_F32_F64: FP32 V, FP64 X and Y (FP64 sums), nrhs 1 or 3.  The FP64
 * correction of a mixed matrix's touching and near entries is not applied.
 * Fixed summation order: the result depends on N (and nrhs) only.  d_x and
 * d_y must not overlap.  BC_EINVAL for other nrhs.  ASYNC. */
int32_t bc_matvec(const void *d_V, int64_t N, int32_t precision, int32_t nrhs,
                  const void *d_x, void *d_y, void *d_ws, size_t ws_bytes,
                  bc_stream stream);

/* ------------------------------------------------------------------------ */
/* Dual-mesh system with operator preconditioning (Algorithm 1, step (i);   */
/* Section 2.6, eq. "laplace_precond_discrete")                             */
/* ------------------------------------------------------------------------ */

/* The unknowns are the coefficients x_j of the dual-cell indicators, one per
 * vertex of the primal mesh (N triangles, M vertices).  The caller assembles
 * V_bary (FP64, bc_prepare + bc_assemble) on the barycentric refinement whose
 * son 6t + s of triangle t = (v0, v1, v2) is, in this order,
 * (v0, m01, c), (m01, v1, c), (v1, m12, c), (m12, v2, c), (v2, m20, c),
 * (m20, v0, c)   (c the centre of gravity, m the edge midpoints),
 * and passes the vertex-to-triangle incidence of the primal mesh as CSR:
 * d_iptr[M + 1], and for each entry the triangle d_itri[] and the vertex's
 * corner 0..2 in it d_icor[], triangles in increasing order per vertex. */
typedef struct {
  double rtol;           /* stop when the preconditioned residual of GMRES
                            has dropped by rtol, e.g. 1e-12 */
  double inexact_lambda; /* > 0: also stop at the first step k with
                            ||x_k - x_{k-1}||_V <= lambda eta(x_k), the energy
                            norm of the last update against the ZZ estimator
                            of the current iterate (Section 2.5, Remark (i),
                            lambda ~ 1e-3); 0: off */
  int32_t max_iter;      /* GMRES steps, <= restart */
  int32_t restart;       /* Krylov basis size the workspace was sized for */
  int32_t jacobi_sweeps; /* sweeps approximating M^{-1} (a fixed linear
                            operator; the solution does not depend on it) */
  int32_t h_mode;        /* mesh size of eta in the inexact stop: 0 diam(T),
                            1 |T|^(1/2) */
} bc_dual_opts;

typedef struct {
  double cap;            /* (1/4pi) sum_j x_j |T_j^dual|   (eq. "cap:ell") */
  double rel_residual;   /* last preconditioned relative residual */
  double energy_step;    /* ||x_k - x_{k-1}||_V of the last step (inexact
                            stop only, else 0) */
  double eta;            /* eta(x_k) = (sum_T eta_T^2)^(1/2) of the returned
                            iterate (inexact stop only, else 0) */
  int32_t iters;         /* GMRES steps (two passes over V_bary each: the
                            three curl components, then V_dual) */
  int32_t status;        /* BC_OK or BC_ENOCONV */
  int32_t stop;          /* 1 residual tolerance, 2 inexact-solve criterion,
                            3 exact invariant subspace, 0 step limit */
  int32_t reserved;
} bc_dual_result;

/* Device scratch for the dual system: per-triangle geometry and curls,
 * dual areas, mass matrix diagonal, the Krylov basis (restart + 1 vectors of
 * length M) and two more bases of restart vectors (the preconditioned basis
 * vectors and V_dual applied to them), vectors on the barycentric mesh and
 * the product's scratch. */
size_t bc_dual_workspace_bytes(int64_t N, int64_t M, int32_t restart);

/* Per triangle: area, diameter, surface curls of the hat functions
 * curl_G phi_a = (P_{a+1} - P_{a+2}) / (2|T|); per vertex: the dual area
 * |T_j^dual| = <phi_j, 1> = sum |T|/3 and the mass matrix diagonal
 * sum 11|T|/54.  d_verts: M x 3 FP64; d_tris: N x 3 int32.  ASYNC. */
int32_t bc_dual_setup(const double *d_verts, int64_t M, const int32_t *d_tris,
                      int64_t N, const int32_t *d_iptr, const int32_t *d_itri,
                      void *d_ws, size_t ws_bytes, int32_t restart,
                      bc_stream stream);

/* Preconditioned GMRES for V_dual x = f (V_dual = P^T V_bary P, f_j =
 * |T_j^dual|) with the hypersingular operator D_reg = sum_m Q_m^T V_bary Q_m
 * + a a^T as right and the inverse mass matrix as left preconditioner
 * (Section 2.6).  Writes x (M entries, FP64) to d_x and the capacity,
 * iteration count and status to *h_result.  x is formed as the combination
 * of the preconditioned basis vectors M^{-1} D_reg z_i, kept during the
 * iteration, which also gives every iterate's energy-norm update for the
 * inexact stop without further products.  precision BC_FP64: d_Vbary is
 * the FP64 matrix (d_pattern unused); BC_MIXED: d_Vbary is the FP32 matrix
 * of a mixed bc_assemble and d_pattern / nnz its pattern, whose FP64
 * corrections of the touching and near entries are added to every product;
 * products are formed with FP64 vectors and sums, so GMRES solves
 * (V32 + C64) exactly and the capacity differs from the FP64 one by the
 * solution-weighted rounding of the stored far field only.  Host-driven:
 * SYNCHRONOUS (waits for `stream` a few times per GMRES step).  Errors: BC_EINVAL for bad
 * options or sizes, BC_ENOMEM for a short workspace. */
int32_t bc_dual_solve(const void *d_Vbary, int32_t precision,
                      const void *d_pattern, int64_t nnz,
                      const int32_t *d_tris, int64_t N, int64_t M,
                      const int32_t *d_iptr, const int32_t *d_itri,
                      const int32_t *d_icor, void *d_ws, size_t ws_bytes,
                      const bc_dual_opts *opts, double *d_x,
                      bc_dual_result *h_result, bc_stream stream);

/* eta(T)^2 = h_T ||Phi - I Phi||^2_{L2(T)} (eq. "zz:T") for the dual
 * solution Phi = sum_j x_j chi_j^dual, I Phi = sum_j x_j phi_j, in closed
 * form on the six barycentric sons of each triangle.  h_mode 0: diam(T);
 * 1: |T|^(1/2).  Needs bc_dual_setup's workspace.  d_eta2: N FP64.  ASYNC. */
int32_t bc_dual_zz(const void *d_ws, size_t ws_bytes, const int32_t *d_tris,
                   int64_t N, int64_t M, int32_t restart, const double *d_x,
                   int32_t h_mode, double *d_eta2, bc_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* BEMCAP_H */
