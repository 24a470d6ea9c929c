/*
 * stokes_ifmm.h - C ABI of the MI355X library for the completed double-layer
 * Stokes boundary-integral system of a pipe filled with circular pores, its
 * block-diagonal and inverse-FMM preconditioners, and flexible GMRES.
 *
 * The problem (Coulier, Quaife, Darve, "An efficient preconditioner for the
 * fast simulation of a 2D Stokes flow in porous media", Section 2): find the
 * density sigma on the wall Gamma_0 and the pore boundaries Gamma_k such that
 * the Nystrom-discretised boundary-integral operator A maps sigma to the
 * prescribed boundary velocity f (equation "f = A sigma", Section 2.2).  The
 * operator used here is the double layer of Section 2.1 with its null space
 * removed: a Stokeslet and a rotlet at every pore centre, with three
 * constraint rows per pore, and a rank-one flux term on the wall.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array pointers are DEVICE pointers unless marked (host).  All floating
 *   point is IEEE FP64 unless stated.  The caller allocates and owns every
 *   array it passes; the library never frees caller memory.  Opaque handles
 *   are allocated by the library and released by the matching *_destroy.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Work is stream-ordered.  Entry points that return numbers to the host
 *   (gmres_solve) synchronise that stream before returning.
 * - Return value: 0 = OK; 1 = SBIE_NOT_CONVERGED (a warning: outputs hold
 *   the best iterate); negative = error, with a message available from
 *   sbie_last_error() on the calling thread.  No C++ exception crosses the
 *   ABI.
 *
 * Unknown vector layout (length n = 2*Nn + 3*M):
 *   [ sigma_x[0..Nn) | sigma_y[0..Nn) | (lambda_x, lambda_y, mu)_k, k=0..M-1 ]
 * Node order: pores 0..M-1 (consecutive nodes each), then the wall.
 *
 * The operator, row by row (r = x_i - x_j, rho = |r|, t_i = (-ny_i, nx_i)):
 *   node rows:  -1/2 sigma_i
 *               + sum_{j != i} w_j (1/pi) (r.n_j) r r^T / rho^4 sigma_j
 *               + w_i kappa_i / (2 pi) t_i t_i^T sigma_i
 *               + [i on wall] n_i / |Gamma_0| sum_{j on wall} w_j n_j.sigma_j
 *               + sum_k [ S(x_i - c_k) lambda_k + r_k R(x_i - c_k) mu_k ]
 *     with S(q) = (-log|q| I + q q^T/|q|^2)/(4 pi)   (Stokeslet)
 *          R(q) = (q_y, -q_x)/(4 pi |q|^2)            (rotlet)
 *   pore rows:  lambda_k row: sum_{j in k} w_j sigma_j / (2 pi r_k) - lambda_k
 *               mu_k row:     sum_{j in k} w_j (x_j - c_k)_perp . sigma_j
 *                                        / (2 pi r_k^2) - mu_k
 */
#ifndef STOKES_IFMM_H
#define STOKES_IFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  SBIE_OK = 0,
  SBIE_NOT_CONVERGED = 1,
  SBIE_INVALID_ARGUMENT = -1,
  SBIE_INVALID_GEOMETRY = -2,
  SBIE_OUT_OF_MEMORY = -3,
  SBIE_HIP_ERROR = -4,
  SBIE_BREAKDOWN = -5,
  SBIE_UNSUPPORTED = -6
};

/* Discretised boundary (Section 2.2: nodes are the quadrature points of the
 * trapezoid rule on every closed curve).
 *   n_nodes      Nn = sum of nodes over the pores and the wall.
 *   n_pores      M (may be 0).
 *   curve_off    (host) M+2 offsets; nodes of pore k are
 *                [curve_off[k], curve_off[k+1]); the wall is curve M.
 *   curve_off_dev  the same M+2 offsets in device memory.
 *   x, y         node positions.
 *   nx, ny       unit normal pointing OUT of the fluid (away from the pipe
 *                interior on the wall, towards the centre on a pore).
 *   w            trapezoid weight |x'(t)| 2 pi / N_curve (arclength weight).
 *   kappa        curvature vector dotted with n: +1/r on a pore, minus the
 *                curvature on the convex wall.
 *   cx, cy       pore centres (where the Stokeslet and rotlet sit), length M.
 *   radius       pore radii, length M.
 * All device arrays are FP64 and are only read. */
typedef struct {
  int64_t n_nodes;
  int32_t n_pores;
  int32_t reserved;
  const int64_t *curve_off;
  const int64_t *curve_off_dev;
  const double *x, *y;
  const double *nx, *ny;
  const double *w;
  const double *kappa;
  const double *cx, *cy;
  const double *radius;
} sbie_geom;

/* Message describing the last failure on the calling thread ("" if none). */
const char *sbie_last_error(void);

/* Checks that a geometry describes what the operator assumes (Section 2:
 * a closed outer wall enclosing disjoint circular pores; Section 2.2:
 * distinct trapezoid nodes on every curve), on the device:
 *   - every node: finite data, weight > 0, |n| = 1 (to 1e-8);
 *   - every pore node at distance radius[k] from (cx[k], cy[k]) (to 1e-8
 *     relative in the squared distance);
 *   - no node repeated on its own curve;
 *   - pores pairwise disjoint (centre distance > sum of radii), finite
 *     centres, radius > 0;
 *   - every pore centre inside the wall polygon and every wall node
 *     outside every pore disc (skipped when there is no wall).
 * Synchronises the stream.  Returns SBIE_OK or SBIE_INVALID_GEOMETRY (the
 * message names every violated condition); SBIE_INVALID_ARGUMENT for a bad
 * descriptor.  gmres_solve, bd_factor, ifmm_factor and the batched solver
 * entry points run the same checks before any other work; the matvec and
 * the assembly do not (they are the inner products of a solve). */
int sbie_validate_geometry(const sbie_geom *g, void *stream);

/* Entries A[rows, cols] of the operator above (Section 2.2, equation
 * "f = A sigma"), for arbitrary global row and column indices.
 *   rows   device int64[nr], each in [0, n).
 *   cols   device int64[nc], each in [0, n).
 *   out    device FP64, column-major nr x nc with leading dimension ld >= nr.
 * Errors: SBIE_INVALID_ARGUMENT for null pointers, nr/nc < 0 or ld < nr.
 * Indices are not range-checked on the device: out-of-range indices are the
 * caller's error (undefined result, never an out-of-bounds write to out). */
int stokes_bie_assemble(const sbie_geom *g, const int64_t *rows, int64_t nr,
                        const int64_t *cols, int64_t nc, double *out,
                        int64_t ld, void *stream);

/* y = A x (mode SBIE_MV_FULL), or only the principal-value double-layer sum
 * with its smooth diagonal limit, sum_{j != i} w_j D(x_i, x_j, n_j) sigma_j
 * + w_i kappa_i/(2 pi) t t^T sigma_i, in the node rows and zero in the pore
 * rows (mode SBIE_MV_DLP_ONLY).  Section 2.1 (double-layer kernel), Section
 * 2.2 (discretisation).  Mode SBIE_MV_FULL_ACCURATE computes the same y = A x
 * with compensated (two-sum) accumulation of every sum, for residuals that
 * must resolve much less than the rounding of the plain sums when the
 * density is far larger than the data; it costs about 1.5 matvecs.
 * x and y are device FP64 of length n and must not
 * overlap.  Direct O(Nn^2) evaluation; scratch memory comes from the
 * stream-ordered allocator and is released before return. */
enum { SBIE_MV_FULL = 0, SBIE_MV_DLP_ONLY = 1, SBIE_MV_FULL_ACCURATE = 2 };
int stokes_dlp_matvec(const sbie_geom *g, const double *x, double *y, int mode,
                      void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * y = A x as stokes_dlp_matvec (same modes, kernels and results up to the
 * rounding order of a different source-chunk count), with no allocation of
 * any kind.  Its scratch (source records, two scalars, partial sums) is a
 * fixed 64 MiB device array of the library, one per GPU, held until the
 * process ends.  The caller passes x and y as for stokes_dlp_matvec.
 * Limit: 8 Nn + 8 (M + 1) + 8 + (c + ceil(M / 64)) * k * Nn doubles must fit
 * in 64 MiB with at least c = 1 source chunk, where k = 2 (SBIE_MV_FULL,
 * SBIE_MV_DLP_ONLY) or 4 (SBIE_MV_FULL_ACCURATE); the source-chunk count is
 * lowered to fit.  Larger problems return SBIE_INVALID_ARGUMENT before any
 * launch (without pores: above 0.84 M nodes plain, 0.70 M accurate).  Every
 * call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (different streams or threads) race and must be serialised by the
 * caller.  Nothing in the array needs to start at zero: every call writes
 * what it reads. */
int stokes_dlp_matvec_noalloc(const sbie_geom *g, const double *x, double *y, int mode,
                              void *stream);

/* Velocity at points of the fluid from a solved density: the trapezoid rule
 * of Section 2.2 (equation "stokesSLP_discretized", here for the completed
 * double-layer representation),
 *   u(p) = sum_j w_j D(p, x_j, n_j) sigma_j
 *          + sum_k [ S(p - c_k) lambda_k + r_k R(p - c_k) mu_k ],
 * with no jump, diagonal limit or wall term (p is off the boundary).
 *   sigma     device FP64, length n (the unknown vector of gmres_solve).
 *   px, py    device FP64, np target points.
 *   ux, uy    device FP64, np outputs.
 *   uref_x, uref_y, err  optional (all three or none): err[i] = | |u(p_i)|
 *             - |uref_i| | / |uref_i|, the relative error of the velocity
 *             magnitude used to assess solutions (Section 4.1.1).
 * Accuracy: spectral once a point is farther than about sqrt(h) from the
 * boundary, h the local node spacing (Section 2.2); closer points get the
 * plain rule (no near-singular correction), and a point on a node gets no
 * contribution from that node.  Target points must be distinct.
 * np = 0 returns SBIE_OK.  Errors: SBIE_INVALID_ARGUMENT for null pointers
 * or np < 0.  Scratch memory comes from the stream-ordered allocator. */
int stokes_velocity(const sbie_geom *g, const double *sigma, const double *px, const double *py,
                    int64_t np, double *ux, double *uy, const double *uref_x, const double *uref_y,
                    double *err, void *stream);

/* Launch shape of the matvec's pair kernel (chosen by the autotuner):
 * targets_per_thread in {1, 2, 4, 8}; source_chunks >= 1 splits the source
 * loop across that many workgroups per target tile (0 = automatic). */
int stokes_dlp_matvec_set_shape(int targets_per_thread, int source_chunks);
/* Symmetric evaluation of the plain products' pair sum: the contributions of
 * node j to node i and of node i to node j share r, rho^2 and 1/rho^4, so
 * every unordered pair of nodes is evaluated once for both (superblocks of
 * 4 x 4 tiles of 256 nodes; per-superblock partial sums added in a fixed
 * order, so the result does not depend on the schedule).  mode 0 = never;
 * 1 = from 16,384 nodes up to 131,072 nodes (the default; its partial sums
 * take about nn^2 / 64 bytes); 2 = always up to 131,072 nodes.  Compensated
 * products and an explicit source-chunk count always use the chunked pair
 * kernel. */
int stokes_dlp_matvec_set_symmetric(int mode);
/* The launch plan stokes_dlp_matvec would use for this geometry and mode
 * (host outputs): symmetric evaluation (1) or chunked kernel (0), source
 * chunks (1 for the symmetric evaluation), targets per thread. */
int stokes_dlp_matvec_describe_plan(const sbie_geom *g, int mode, int32_t *symmetric, int32_t *chunks,
                                    int32_t *targets_per_thread);
/* Schedule of the batched products' pair stage (stokes_dlp_matvec_batched,
 * gmres_solve_batched): 1 = persistent grid with a device work queue (the
 * default), 0 = one workgroup per item.  Both give identical results. */
int stokes_dlp_matvec_batched_set_schedule(int persistent);

/* Kernel timing of the matvec's pair kernel (the dominant kernel): while
 * enabled, every launch of it is bracketed by HIP events recorded on the
 * stream it is launched on.  sbie_kernel_time synchronises those events,
 * returns the summed duration in milliseconds and the launch count, and
 * clears the record.  Not thread-safe; meant for benchmarks. */
int sbie_kernel_timing(int enable);
int sbie_kernel_time(double *total_ms, int64_t *launches);

/* Block-diagonal preconditioner (Section 4.1.1): one block per pore (its
 * nodes and its three constraint unknowns) and one block for the wall; each
 * block is assembled and inverted exactly.  bd_solve computes x = P^{-1} b
 * (device FP64 length n; x and b must not overlap). */
typedef struct sbie_bd sbie_bd;
int bd_factor(const sbie_geom *g, sbie_bd **out, void *stream);
int bd_solve(const sbie_bd *bd, const double *b, double *x, void *stream);
int bd_destroy(sbie_bd *bd);

/* Inverse fast multipole method (Section 3): an approximate factorisation of
 * the H^2 representation A ~ S + U A_coarse V^T (Section 3.1) built from
 * Chebyshev interpolation with a rank-revealing reduction, eliminated level
 * by level on the extended sparse system (Section 3.2) with fill-ins between
 * well-separated boxes compressed to tolerance eps and redirected through
 * the low-rank bases (Section 3.3).
 *   eps          relative truncation tolerance on singular values.
 *   cheb_n       Chebyshev nodes per direction for the initial bases.
 *   leaf_target  mean number of boundary nodes per non-empty leaf.
 *   max_depth    cap on the quadtree depth (0 = automatic).
 *   precision    0 = FP64 factor and apply; 1 = FP32 factor and apply;
 *                2 = FP64 factor stored a second time in FP32: ifmm_solve
 *                reads only that copy, widening each entry to FP64 (vectors
 *                and arithmetic stay FP64), so it moves half the bytes.
 *   compress     inputs of the two Gaussian-sketch products of the fill-in
 *                recompression (far fill-in blocks times a Gaussian matrix,
 *                and wide candidate sets times a Gaussian matrix, whose
 *                results only have to span the fill-ins' column spaces):
 *                0 = the factor's precision; 1 = rounded to FP16, 2 = rounded
 *                to BF16, both multiplied on the matrix cores with FP32
 *                accumulation.  The rounding perturbs each (norm-scaled)
 *                block by about the format's unit roundoff (FP16 4.9e-4,
 *                BF16 3.9e-3), which bounds the compression error from below:
 *                suited to eps >= 1e-3 (FP16) and eps >= 1e-2 (BF16).
 *                Every other product of the factorisation stays in the
 *                factor's precision.
 *   reserved     must be 0.
 * ifmm_solve computes x ~ A^{-1} b (device FP64, length n).
 * Errors: SBIE_UNSUPPORTED if a pore is larger than a leaf box allows;
 * SBIE_BREAKDOWN on a singular pivot. */
typedef struct {
  double eps;
  int32_t cheb_n;
  int32_t leaf_target;
  int32_t max_depth;
  int32_t precision;
  int32_t compress;
  int32_t reserved;
} ifmm_params;
typedef struct ifmm_handle ifmm_handle;
int ifmm_factor(const sbie_geom *g, const ifmm_params *p, ifmm_handle **out,
                void *stream);
int ifmm_solve(const ifmm_handle *h, const double *b, double *x, void *stream);
int ifmm_destroy(ifmm_handle *h);
/* Statistics of a factorisation (host): levels, leaves, max rank, factor
 * bytes and factor time in seconds; the algorithmic flops of its dense
 * products (2 m n k per product) and inverses (2 n^3 per Gauss-Jordan
 * inverse), summed from the operations it issued (the sketched pivoted
 * Gram-Schmidt, copies and norms are not counted); gemm_low_flops is the
 * part of gemm_flops run with FP16 or BF16 inputs. */
typedef struct {
  int32_t levels;
  int32_t leaves;
  int32_t max_rank;
  int32_t reserved;
  int64_t factor_bytes;
  double factor_seconds;
  double gemm_flops;
  double inverse_flops;
  double gemm_low_flops;
} ifmm_stats;
int ifmm_get_stats(const ifmm_handle *h, ifmm_stats *s);

/* Flexible GMRES with right preconditioning (Section 4 uses GMRES with a
 * preconditioner; here the preconditioner is applied on the right and the
 * stopping test is the true residual ||f - A sigma|| <= tol ||f||).
 * Arnoldi uses classical Gram-Schmidt applied twice, in FP64.
 *   f        device FP64 length n (right-hand side).
 *   sigma    device FP64 length n; the initial guess when use_x0 != 0, and
 *            the solution on return.
 *   pc       0 = none, 1 = block-diagonal (bd must be set), 2 = IFMM (ifmm
 *            must be set).
 *   res_hist (host, optional) max_iter + 2 doubles: relative residual per
 *            iteration.
 *   fmm      (optional) a fast-multipole plan of the same geometry: the
 *            Arnoldi products then use it (stokes_dlp_matvec_fmm), while
 *            every true residual keeps the direct compensated product, so
 *            the stopping test is the same as without it.  NULL = direct.
 * Returns SBIE_OK, SBIE_NOT_CONVERGED (sigma = best iterate) or an error. */
typedef struct sbie_fmm sbie_fmm;
typedef struct {
  double tol;
  int32_t max_iter;
  int32_t restart;
  int32_t pc;
  int32_t use_x0;
  const sbie_bd *bd;
  const ifmm_handle *ifmm;
  double *res_hist;
  const sbie_fmm *fmm;
} gmres_params;
typedef struct {
  int32_t iters;
  int32_t status;
  double rel_res_true;
  double rel_res_pc;
  double t_precond_s;
  double t_matvec_s;
  double t_arnoldi_s;
  double t_total_s;
} gmres_result;
int gmres_solve(const sbie_geom *g, const double *f, double *sigma,
                const gmres_params *p, gmres_result *res, void *stream);

/* ------------------------------------------------------------------------
 * Fast multipole evaluation of the double-layer pair sum (Section 2.2: the
 * matrix-vector products of GMRES can be computed by a fast multipole
 * method in O(N) work).  Black-box FMM with Chebyshev interpolation (the
 * far-field approximation of Section 3.1's H^2 operators): a quadtree on
 * the bounding square of the nodes (non-empty boxes only), uniform or
 * adaptive, with cheb_n x cheb_n tensor Chebyshev grids per box carrying
 * the multipole tensors of the sources and the local velocities.  Lists:
 * V (children of the parent's neighbours that do not touch the box:
 * multipole to local), U (leaves touching a leaf: direct sum), and on an
 * adaptive tree W (boxes smaller than a leaf that do not touch it but whose
 * parents do: multipole evaluated at the leaf's nodes) and X (the inverse
 * of W: a larger leaf's sources into the box's local expansion).  Only the
 * pair sum sum_{j != i} w_j (1/pi) (r.n_j) r r^T / rho^4 sigma_j changes;
 * every other term of the operator is evaluated as in stokes_dlp_matvec.
 * The error is that of the interpolation: it falls geometrically with
 * cheb_n, about a factor 4.5 per order (relative to the largest entry of
 * the product on the pipes of the tests: 2.6e-5 at 6, 1.3e-7 at 10, 3e-10
 * at 14, 1.2e-11 at 16); a quadtree of depth 0 or 1 has no far field and
 * gives the direct sum.
 *   cheb_n       Chebyshev nodes per direction: 4, 6, ..., 16.
 *   leaf_target  uniform tree with max_depth = 0: the shallowest depth whose
 *                non-empty leaves hold at most this many nodes on average;
 *                adaptive tree: every box holding more nodes than this is
 *                split (0 = 64).
 *   max_depth    uniform: the quadtree depth (0 = from leaf_target);
 *                adaptive: the deepest level allowed (0 = 20); at most 20.
 *   adaptive     0 = uniform depth, 1 = adaptive.
 * fmm_plan builds the tree and its lists on the host from the node
 * positions (read once from the device; synchronises) and keeps a copy of
 * the geometry descriptor: the geometry's arrays must outlive the plan, and
 * the plan must be rebuilt when the nodes move.  Calls that use one plan
 * must be ordered (one stream): they share its device buffers. */
typedef struct {
  int32_t cheb_n;
  int32_t leaf_target;
  int32_t max_depth;
  int32_t adaptive;
} fmm_params;
int fmm_plan(const sbie_geom *g, const fmm_params *p, sbie_fmm **out, void *stream);
/* y = A x as stokes_dlp_matvec with the pair sum from the plan; modes
 * SBIE_MV_FULL and SBIE_MV_DLP_ONLY (SBIE_MV_FULL_ACCURATE: SBIE_UNSUPPORTED). */
int stokes_dlp_matvec_fmm(const sbie_fmm *plan, const double *x, double *y, int mode,
                          void *stream);
/* Shape of a plan (host): depth (deepest level), non-empty leaves, boxes
 * over all levels, the shallowest leaf level, box pairs in the V lists,
 * node pairs summed directly (U lists), (leaf, box) pairs in the W lists and
 * (box, leaf) pairs in the X lists. */
typedef struct {
  int32_t depth;
  int32_t leaves;
  int32_t boxes;
  int32_t min_leaf_level;
  int64_t m2l_box_pairs;
  int64_t near_node_pairs;
  int64_t m2p_box_pairs;
  int64_t p2l_box_pairs;
} fmm_stats;
int fmm_get_stats(const sbie_fmm *plan, fmm_stats *s);
int fmm_destroy(sbie_fmm *plan);

/* ------------------------------------------------------------------------
 * The single-layer (first-kind) formulation the paper's experiments use
 * (Section 2.1, equations "stokesSLP" and "stokesBIE"; Section 2.2, the
 * corrected trapezoid rule).  Unknowns: [sigma_x (Nn) | sigma_y (Nn)], length
 * 2 Nn, no completion.  Row i:
 *   (A sigma)_i = sum_{j != i} w_j (1 + gamma_ij) G(x_i - x_j) sigma_j / (4 pi),
 *   G(r) = -log|r| I + r r^T / |r|^2,
 * where gamma_ij = gamma_d when j is on the curve of i at periodic index
 * distance d = 1..6 and 0 otherwise (the six-point-per-side rule for the
 * logarithmic singularity; the weights are derived from the error expansion
 * of the punctured trapezoid rule and returned by stokes_slp_weights).  Every
 * curve needs more than 12 nodes (SBIE_UNSUPPORTED otherwise).  The single
 * layer of the normal density of any closed curve vanishes on the whole
 * boundary, so the matrix has M + 1 singular values that go to zero with the
 * rule's error: the density is determined only up to those directions, the
 * velocity in the fluid is not affected.
 * ------------------------------------------------------------------------ */
/* gamma_1..gamma_6 (host array of 6 doubles). */
int stokes_slp_weights(double *gamma);
/* y = A sigma (device FP64, length 2 Nn, no overlap); mode SBIE_MV_FULL or
 * SBIE_MV_FULL_ACCURATE (compensated sums).  Direct O(Nn^2) evaluation. */
int stokes_slp_matvec(const sbie_geom *g, const double *x, double *y, int mode, void *stream);
/* Entries A[rows, cols] (indices in [0, 2 Nn), column-major, ld >= nr). */
int stokes_slp_assemble(const sbie_geom *g, const int64_t *rows, int64_t nr, const int64_t *cols,
                        int64_t nc, double *out, int64_t ld, void *stream);
/* Block-diagonal preconditioner of the single-layer matrix: one exactly
 * inverted block per curve (Section 4.1.1).  Applied with bd_solve; freed
 * with bd_destroy. */
int bd_factor_slp(const sbie_geom *g, sbie_bd **out, void *stream);
/* FGMRES on the single-layer system, as gmres_solve (f, sigma of length
 * 2 Nn); pc = 0 or 1 (a handle from bd_factor_slp); pc = 2 returns
 * SBIE_UNSUPPORTED (the IFMM here is built for the double layer). */
int gmres_solve_slp(const sbie_geom *g, const double *f, double *sigma,
                    const gmres_params *p, gmres_result *res, void *stream);
/* Velocity in the fluid from a single-layer density by the plain trapezoid
 * rule (equation "stokesSLP_discretized"), arguments as stokes_velocity. */
int stokes_slp_velocity(const sbie_geom *g, const double *sigma, const double *px, const double *py,
                        int64_t np, double *ux, double *uy, const double *uref_x, const double *uref_y,
                        double *err, void *stream);

/* ------------------------------------------------------------------------
 * Batches of independent geometries.
 * ------------------------------------------------------------------------ */
/* y_b = A_b x_b for every member b (geoms: host array of `count`
 * descriptors; x, y: host arrays of device pointers).  Every stage of the
 * product is one launch for the whole batch; the pair stage is by default a
 * persistent grid (as many workgroups as the device holds at once) whose
 * workgroups draw (member, target tile, source chunk) items from a device
 * work queue until it is empty.  Same modes and results as
 * stokes_dlp_matvec with the same launch shape.  Synchronises the stream. */
int stokes_dlp_matvec_batched(const sbie_geom *geoms, int32_t count, const double *const *x,
                              double *const *y, int mode, void *stream);

/* Per-member preconditioner of a batched solve (pc as in gmres_params). */
typedef struct {
  int32_t pc;
  int32_t use_x0;
  const sbie_bd *bd;
  const ifmm_handle *ifmm;
} gmres_member;

/* The FGMRES of gmres_solve for every member, advanced in lockstep: one
 * batched matvec and one set of batched Gram-Schmidt launches per step for
 * all members still iterating, one host copy of all Hessenberg columns per
 * step; preconditioners applied member by member.  f, sigma: host arrays of
 * device pointers.  restart <= 0 means unrestarted.  results[b] as for
 * gmres_solve, except that t_total_s is the whole batch's time, t_arnoldi_s
 * the time of all lockstep steps (preconditioners, products and
 * Gram-Schmidt together) and t_matvec_s = t_precond_s = 0.  Returns
 * SBIE_NOT_CONVERGED when any member did not converge (see results). */
int gmres_solve_batched(const sbie_geom *geoms, int32_t count, const double *const *f,
                        double *const *sigma, const gmres_member *members, double tol,
                        int32_t max_iter, int32_t restart, gmres_result *results, void *stream);

/* IFMM factorisations of every member (out: host array of `count` handles),
 * run concurrently by `workers` host threads, each on a stream of its own
 * (the factorisation is latency bound: small launches with host
 * synchronisation between elimination phases, so several members overlap on
 * the device).  On error every handle created is destroyed and out[] is set
 * to NULL.  Synchronises. */
int ifmm_factor_batched(const sbie_geom *geoms, int32_t count, const ifmm_params *params,
                        ifmm_handle **out, int32_t workers);

/* ------------------------------------------------------------------------
 * Learned warm start (not part of the paper: an initial guess for GMRES,
 * which stays the judge of the solution).  A per-pore multilayer perceptron
 * (FP32, exact-erf GELU between layers, none after the last) maps 64
 * geometry features of a pore to 64 Fourier coefficients of the density on
 * that pore.  Activations are column-major (width x batch).
 * ------------------------------------------------------------------------ */
typedef struct sbie_mlp sbie_mlp;
/* widths (host): nlayers + 1 layer widths.  Weights are He-normal from a
 * counter-based generator seeded by `seed`; biases zero. */
int mlp_create(int nlayers, const int32_t *widths, uint64_t seed, sbie_mlp **out,
               void *stream);
int mlp_destroy(sbie_mlp *net);
int mlp_num_params(const sbie_mlp *net, int64_t *count);
/* Parameters as one FP32 device array: for each layer, W (out x in,
 * column-major) then b (out). */
int mlp_get_params(const sbie_mlp *net, float *dst, void *stream);
int mlp_set_params(sbie_mlp *net, const float *src, void *stream);
/* Y (out x batch) = network(X (in x batch)). */
int mlp_forward(sbie_mlp *net, const float *X, int32_t batch, float *Y, void *stream);
/* Mean squared error against the standardised T and its gradient (kept for mlp_adam_step and
 * copied to grad when non-null; device, num_params floats); *loss (host,
 * optional) receives the loss; synchronises when loss is requested. */
int mlp_loss_grad(sbie_mlp *net, const float *X, const float *T, int32_t batch,
                  float *grad, double *loss, void *stream);
/* Standardisation (device FP32 arrays): the network sees
 * (x - in_mean) * in_scale and predicts targets standardised as
 * (t - out_mean) / out_std; mlp_forward returns de-standardised outputs and
 * mlp_loss_grad's loss is the MSE of the standardised targets.  Defaults are
 * the identity.  mlp_fit_scaling sets them from the mean and standard
 * deviation of every row of X and T (a row with zero spread keeps scale 1). */
int mlp_set_scaling(sbie_mlp *net, const float *in_mean, const float *in_scale,
                    const float *out_mean, const float *out_std, void *stream);
int mlp_get_scaling(const sbie_mlp *net, float *in_mean, float *in_scale, float *out_mean,
                    float *out_std, void *stream);
int mlp_fit_scaling(sbie_mlp *net, const float *X, const float *T, int32_t batch, void *stream);
/* One Adam step with bias correction using the last gradient. */
int mlp_adam_step(sbie_mlp *net, float lr, float beta1, float beta2, float eps,
                  void *stream);
/* Features of every pore (64 x M floats, device): radius; offsets and radii
 * of the 16 nearest pores (ties by index, zero padded); the inflow profile
 * k (H^2 - y_c^2) with k = 1/H^2 for the channel [y_lo, y_hi] and its slope at
 * the centre height; the distances to the two walls; zeros to 64. */
int warmstart_features(const sbie_geom *g, double y_lo, double y_hi, float *feats,
                       void *stream);
/* Fourier coefficients of a density on every pore (64 x M floats): per
 * velocity component a_0, a_1..a_15, b_1..b_15, a_16 with angles measured at
 * the pore centre (discrete Fourier transform of the nodal values). */
int warmstart_labels(const sbie_geom *g, const double *sigma, float *coeffs, void *stream);
/* Initial guess x0 (device FP64, length n): the Fourier series on every pore,
 * the given wall density (2 * N_ext values: x then y components; NULL = 0) on
 * the wall, and lambda, mu from the constraint functionals of x0. */
int warmstart_assemble(const sbie_geom *g, const float *coeffs, const double *wall_sigma,
                       double *x0, void *stream);

/* Improve an initial guess x0 (device FP64, length n) in place with two
 * steps that cannot raise the residual of the second: (1) solve the wall rows
 * exactly for the wall density with every other unknown held fixed,
 * x0_wall += A_ww^{-1} (f - A x0)_wall, where wall_bd is the block-diagonal
 * preconditioner of the same pipe without pores (its one block is A_ww, which
 * depends only on the wall); (2) scale x0 by alpha = <f, A x0> / <A x0, A x0>,
 * the minimiser of ||f - alpha A x0||.  *alpha (host, optional) receives the
 * factor; synchronises when it is requested.  Two matrix-vector products. */
int warmstart_refine(const sbie_geom *g, const sbie_bd *wall_bd, const double *f, double *x0,
                     double *alpha, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* STOKES_IFMM_H */
