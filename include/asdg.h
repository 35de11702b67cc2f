/*
 * asdg.h -- C ABI of the MI355X two-level additive Schwarz PCG library for
 * symmetric interior penalty DG (SIPG) discretisations of
 *     -div(rho grad u) = f in (0,1)^2,  u = 0 on the boundary,
 * on conforming polygonal meshes.
 *
 * Method (Antonietti, Houston, Pennesi, Suli, arXiv:1903.11357):
 *   - SIPG bilinear form, Sec. 2 eq. (Ah) with the weighted-average lifting
 *     of eq. (lifting), omega = rho^-/(rho^+ + rho^-), penalty eq. (Sigma)
 *     sigma_F = C_sigma <rho>_F p^2 / <h>_F (harmonic averages, h = cell
 *     diameter), space V_h of eq. (Vh) (total degree p >= 1);
 *   - additive Schwarz operator P_ad = sum_{i=0}^{N} P_i of Sec. 3 with exact
 *     local solvers on non-overlapping subdomains (unions of fine cells) and
 *     a coarse space V_0 of degree q (1 <= q <= p) on a coarse mesh that is
 *     either nested (agglomerates) or independent (non-nested), coupled by the
 *     L2 prolongation R_0^T of eq. (R0T) and the Galerkin operator of
 *     eq. (A0);
 *   - conjugate gradients preconditioned by P_ad from a zero initial guess,
 *     stopped on the Euclidean norm of the relative residual (Sec. 7).
 *
 * Conventions shared by every entry point
 *   - Status: every call returns ASDG_OK (0) or a negative asdg_status; a
 *     message is then available from asdg_last_error(). No exception or
 *     signal crosses the ABI.
 *   - Host pointers are read only during the call; the library copies what
 *     it keeps. Device pointers are hipMalloc'd (or torch) device memory on
 *     the current HIP device and must stay valid until the stream work that
 *     uses them has finished.
 *   - Device memory is owned by the caller: asdg_plan() reports four byte
 *     counts, the caller allocates them and hands them over with asdg_bind().
 *     The library never allocates device memory itself.
 *   - Streams are passed as void* holding a hipStream_t (NULL = default
 *     stream). All device work of a call is enqueued on that stream.
 *   - Vector layout: x[c * n_p + k] for cell c in the caller's cell order and
 *     basis index k; the basis on a cell with bounding box [x0,x1]x[y0,y1] is
 *     sqrt((2i+1)(2j+1)/(dx dy)) L_i(2(x-xc)/dx) L_j(2(y-yc)/dy), i+j <= p,
 *     ordered by degree d = i+j, then by j = 0..d (Legendre L_k).
 *   - A handle is not thread safe; distinct handles are independent.
 */
#ifndef ASDG_H
#define ASDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ASDG_OK = 0,
  ASDG_EINVAL = -1,      /* invalid argument, mesh or partition            */
  ASDG_ENOMEM = -2,      /* bound buffer smaller than asdg_plan() reported */
  ASDG_ENOTSPD = -3,     /* Cholesky pivot <= 0 or NaN (failed_subdomain)  */
  ASDG_ENOCONV = -4,     /* max_iter reached; x and stats still written    */
  ASDG_EBREAKDOWN = -5,  /* p.Ap <= 0 or NaN inside PCG                    */
  ASDG_EHIP = -6,        /* a HIP runtime call failed                      */
  ASDG_ESTATE = -7       /* call out of order (e.g. solve before factor)   */
} asdg_status;

typedef enum {
  ASDG_FP64 = 0,        /* local factors and sweeps in FP64                 */
  ASDG_FP32_LOCAL = 1   /* local factors/sweeps in FP32 (MFMA FP32 accumulate);
                           outer PCG, dot products, coarse solve in FP64     */
} asdg_precision;

typedef struct asdg_problem asdg_problem;

/* Conforming polygon mesh of the unit square: cell c has the vertices
 * cell_vertices[cell_ptr[c] .. cell_ptr[c+1]-1] in counter-clockwise order;
 * neighbouring cells share vertex ids (no hanging nodes). Cells must be
 * convex when used as a non-nested coarse mesh. */
typedef struct {
  int32_t n_vertices;
  const double* xy;              /* [n_vertices][2]                         */
  int32_t n_cells;
  const int32_t* cell_ptr;       /* [n_cells + 1]                           */
  const int32_t* cell_vertices;  /* [cell_ptr[n_cells]]                     */
} asdg_mesh;

/* Conforming tetrahedral mesh (the 3D case of Sec. 2): cell c has the
 * vertices tets[4c .. 4c+3]; neighbouring cells share vertex ids and whole
 * triangular faces; unmatched faces must lie on the bounding box of the
 * vertices (a box-shaped domain). Any vertex order. */
typedef struct {
  int32_t n_vertices;
  const double* xyz;     /* [n_vertices][3]                                 */
  int32_t n_cells;
  const int32_t* tets;   /* [n_cells][4]                                    */
} asdg_tet_mesh;

/* Vectorised right-hand side: out[k] = f(xy[2k], xy[2k+1]) for k < n
 * (tetrahedral meshes: f(xyz[3k], xyz[3k+1], xyz[3k+2])). */
typedef void (*asdg_field_fn)(int64_t n, const double* xy, double* out, void* user);

/* A ready-made asdg_field_fn for a load given as a double sine series on
 * the unit square (Sec. 2 takes any f in L^2(Omega)):
 *   f(x, y) = sum_{k=1..kx} sum_{l=1..ky} coef[(k-1) ky + (l-1)] sin(k pi x) sin(l pi y).
 * Pass asdg_field_sine_series as f and a pointer to an asdg_sine_series as
 * f_user of asdg_assemble; evaluated natively on the assembly's host
 * threads. coef is read only during the call. kx < 1, ky < 1 or a NULL
 * coef give NaN loads (asdg_field_fn has no error channel). */
typedef struct {
  int32_t kx, ky;      /* frequencies per direction                          */
  const double* coef;  /* [kx][ky] row-major                                 */
} asdg_sine_series;
void asdg_field_sine_series(int64_t n, const double* xy, double* out, void* user);

typedef struct {
  double rtol;          /* stop when ||r_k||_2 <= rtol * ||b||_2 (Sec. 7: 1e-8) */
  int32_t max_iter;     /* >= 1                                            */
  int32_t check_every;  /* iterations per captured graph replay (>= 1)     */
  int32_t use_graph;    /* 1: replay a captured hipGraph, 0: eager launches */
  int32_t time_kernels; /* 1: time every local-solve launch with HIP events
                           on the launch stream (forces eager launches)    */
} asdg_pcg_opts;

typedef struct {
  int32_t iterations;      /* CG iterations taken                          */
  int32_t converged;       /* 1 if ||r|| <= rtol ||b||                     */
  double rel_res;          /* recursive ||r_k|| / ||b||                    */
  double lambda_min;       /* Lanczos extreme eigenvalue estimates of      */
  double lambda_max;       /*   P^{-1} A from the CG coefficients          */
  double t_solve_ms;       /* wall time of the solve on the stream         */
  double t_local_ms;       /* summed local-solve kernel time (time_kernels) */
  int32_t n_local;         /* number of timed local-solve launches         */
  int32_t failed_subdomain;/* ENOTSPD: subdomain index, -1 = coarse        */
  double true_rel_res;     /* ||b - A x_k|| / ||b|| of the returned iterate,
                              computed on the device after the loop (one
                              operator apply and a fixed-order sum; 0 when
                              b = 0). Sec. 7 stops on the recursive
                              residual; this reports the true one beside it */
  double t_assemble_ms;    /* host wall time of the last asdg_assemble(_tet) */
  double t_factor_ms;      /* wall time of the last asdg_factor (synchronous) */
  double t_coarse_ms;      /* coarse setup: host transfer and Galerkin A_0 in
                              asdg_plan + the last asdg_setup_coarse        */
  /* the PCG time itself is t_solve_ms */
} asdg_pcg_stats;

/* Handle lifetime. asdg_destroy(NULL) is a no-op. */
asdg_status asdg_create(asdg_problem** out);
void asdg_destroy(asdg_problem* pb);
const char* asdg_last_error(const asdg_problem* pb);

/* Host-side SIPG assembly (Sec. 2, eqs. (Ah), (lifting), (Sigma)).
 * fine:      the fine mesh T_h.
 * p:         polynomial degree, 1 <= p <= 9 (Sec. 7 reaches p = 9 in Example 5;
 *            operator kernels of one wave per n_p DoFs up to p = 3, one thread per
 *            DoF above).
 * c_sigma:   penalty constant C_sigma > 0 (the paper's experiments use 10).
 * rho:       [n_cells] cell-wise constant coefficient, > 0 (Remark 2.1).
 * subdomain: [n_cells] subdomain id of each cell in 0..n_sub-1, every id used
 *            (the partition T_Hcal of Sec. 3 into unions of fine cells).
 * f, f_user: right-hand side, integrated with the cell quadrature.
 * Errors: EINVAL for p or c_sigma out of range, non-positive rho, a
 * clockwise or degenerate cell, an edge shared by more than two cells or an
 * unmatched edge inside the square, or an unused subdomain id. */
asdg_status asdg_assemble(asdg_problem* pb, const asdg_mesh* fine, int32_t p, double c_sigma,
                          const double* rho, const int32_t* subdomain, asdg_field_fn f,
                          void* f_user);

/* Host-side SIPG assembly on a tetrahedral mesh (Sec. 2 for d = 3: the
 * same flux form and penalty, triangular faces, h = cell diameter, n_p =
 * (p+1)(p+2)(p+3)/6). p: 1 <= p <= 3; other arguments as asdg_assemble. The
 * coarse space of such a problem must be given by coarse_of_cell (nested
 * agglomerates of the tetrahedra) in asdg_plan.
 * Errors: EINVAL for p or c_sigma out of range, non-positive rho, a
 * degenerate tetrahedron, a face shared by more than two cells or an
 * unmatched face inside the domain, or an unused subdomain id. */
asdg_status asdg_assemble_tet(asdg_problem* pb, const asdg_tet_mesh* fine, int32_t p, double c_sigma,
                              const double* rho, const int32_t* subdomain, asdg_field_fn f,
                              void* f_user);

/* Coarse space choice and device footprint (Sec. 3, V_0, eqs. (R0T), (A0)).
 * precision:      local factor precision.
 * q:              coarse degree, 1 <= q <= p (for p >= 5: q = 1 or q = p; other
 *                 values EINVAL); q = 0 disables the coarse level
 *                 (one-level method).
 * coarse_of_cell: [n_cells] nested coarse partition (coarse cell id of each
 *                 fine cell), or NULL when coarse_mesh is given.
 * coarse_mesh:    independent convex coarse mesh (non-nested case), or NULL.
 * bytes[4]:       out: sizes of the operator, factor, coarse and scratch
 *                 buffers the caller must allocate for asdg_bind().
 * The coarse transfer (L2 projection, exact convex clipping when non-nested)
 * and the Galerkin A_0 = P_0^T A P_0 are formed here on the host. */
asdg_status asdg_plan(asdg_problem* pb, asdg_precision precision, int32_t q,
                      const int32_t* coarse_of_cell, const asdg_mesh* coarse_mesh,
                      size_t bytes[4]);

/* Hands over caller-owned device buffers (sizes >= bytes[] from asdg_plan,
 * 256-byte aligned) and uploads the operator and coarse data on stream.
 * Errors: ENOMEM if a size is too small, EHIP on copy failure. */
asdg_status asdg_bind(asdg_problem* pb, void* const d_buf[4], const size_t sizes[4],
                      void* stream);

/* Forms every A_i = R_i A R_i^T (principal submatrix, Sec. 3 local solvers)
 * in tile-packed form and Cholesky-factorises all of them in one persistent
 * launch (MFMA). Synchronises the stream to read the status word.
 * Errors: ENOTSPD with failed_subdomain() = index. */
asdg_status asdg_factor(asdg_problem* pb, void* stream);

/* Uploads A_0 and factorises it in FP64 on the device (eq. (A0)).
 * Errors: ENOTSPD (coarse), ESTATE before asdg_bind(). */
asdg_status asdg_setup_coarse(asdg_problem* pb, void* stream);

/* Preconditioned CG (Sec. 7 protocol, x_0 = 0).
 * d_b:  [n] device right-hand side in caller layout, or NULL for the
 *       assembled load vector.
 * d_x:  [n] device output, caller layout.
 * opts: NULL = {1e-8, 20000, 16, 1, 0}.
 * stats: optional output.
 * Errors: ENOCONV (x written), EBREAKDOWN, ESTATE if not factored. */
asdg_status asdg_pcg_solve(asdg_problem* pb, const double* d_b, double* d_x,
                           const asdg_pcg_opts* opts, asdg_pcg_stats* stats, void* stream);

/* Non-blocking form of asdg_pcg_solve for request loops that keep several
 * solves in flight on different streams (each handle is one solve).
 *   asdg_pcg_begin:  enqueues x = 0, r = b, z = P^{-1} r, p = z on stream
 *                    (d_b as in asdg_pcg_solve) and an asynchronous copy of
 *                    the iteration state; returns at once.
 *   asdg_pcg_step:   enqueues one chunk of opts->check_every iterations (a
 *                    captured hipGraph) and the state copy; no-op once the
 *                    solve is done. Call only after asdg_pcg_poll reported
 *                    the previous chunk done (else ESTATE).
 *   asdg_pcg_poll:   never blocks; chunk_done = 1 once the last enqueued
 *                    chunk has finished, then solve_done = 1 if the solve
 *                    stopped (converged, max_iter or breakdown) and
 *                    iterations = iterations so far.
 *   asdg_pcg_finish: after solve_done, writes x (caller layout) and the
 *                    statistics (with the true residual against the d_b
 *                    given to asdg_pcg_begin, which must therefore stay
 *                    valid until this call returns); synchronises the
 *                    stream; returns the solve's status (OK, ENOCONV,
 *                    EBREAKDOWN).
 * The state copy goes to a small pinned host buffer owned by the handle. */
asdg_status asdg_pcg_begin(asdg_problem* pb, const double* d_b, const asdg_pcg_opts* opts, void* stream);
asdg_status asdg_pcg_step(asdg_problem* pb, void* stream);
asdg_status asdg_pcg_poll(asdg_problem* pb, int32_t* chunk_done, int32_t* solve_done, int32_t* iterations);
asdg_status asdg_pcg_finish(asdg_problem* pb, double* d_x, asdg_pcg_stats* stats, void* stream);

/* Single applications of hot-path steps on device vectors in caller layout,
 * for verification and benchmarking (what = ASDG_APPLY_*):
 *   OPERATOR: out = A in                       (SIPG operator, eq. (Ah))
 *   LOCAL:    out = sum_i R_i^T A_i^{-1} R_i in (local solvers, Sec. 3)
 *   COARSE:   out = P_0 A_0^{-1} P_0^T in       (coarse correction, Sec. 3)
 *   PRECOND:  out = LOCAL + COARSE              (the preconditioner)  */
enum { ASDG_APPLY_OPERATOR = 0, ASDG_APPLY_LOCAL = 1, ASDG_APPLY_COARSE = 2,
       ASDG_APPLY_PRECOND = 3 };
asdg_status asdg_apply(asdg_problem* pb, int32_t what, const double* d_in, double* d_out,
                       void* stream);

/* For callers that cannot allocate device memory or synchronise (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): out = A in (the ASDG_APPLY_OPERATOR step of asdg_apply, same
 * kernels and results) with its staging vectors in a static device array of
 * the library instead of the handle's bound scratch buffer, which it leaves
 * untouched, so it may run while a non-blocking solve of the same handle is
 * in flight. Calls no hipMalloc/hipFree and does not synchronise: the work
 * is only enqueued on `stream`. The array holds 2 * 1572864 doubles (24 MiB)
 * per GPU, for problems of at most 1572864 DoFs (EINVAL above that), kept
 * until the process ends and shared by every call on that GPU: calls that
 * overlap on one GPU (different streams, handles or threads) race, so order
 * them (one stream, or events). d_in, d_out: [n] device vectors in caller
 * layout. Errors: EINVAL (null vector, size), ESTATE (before asdg_bind),
 * EHIP. */
asdg_status asdg_apply_operator_static(asdg_problem* pb, const double* d_in, double* d_out, void* stream);

/* Problem sizes: info[0] = n_cells, [1] = n_p, [2] = n (DoFs), [3] = n_sub,
 * [4] = n0 (coarse DoFs), [5] = nnz blocks of A, [6] = max subdomain DoFs,
 * [7] = tile edge of the local factors (64 or 32, ASDG_TUNE_TILE; the
 * coarse factor's tiles are always 64). */
asdg_status asdg_info(const asdg_problem* pb, int64_t info[8]);

/* Host copies for verification, caller layout:
 *   asdg_export_rhs:      b [n]
 *   asdg_export_operator: A as COO triplets of its blocks; rows/cols/vals
 *                         have room for nnzb * n_p^2 entries (info[5]).
 *   asdg_export_coarse:   A_0 dense row-major [n0 * n0] (host-formed). */
asdg_status asdg_export_rhs(const asdg_problem* pb, double* b);
asdg_status asdg_export_operator(const asdg_problem* pb, int64_t* rows, int64_t* cols,
                                 double* vals);
asdg_status asdg_export_coarse(const asdg_problem* pb, double* a0);

/* Raw copy of the factor tiles of local subdomain `sub` (or the coarse
 * factor for sub = -1) into host memory `out`: nb(nb+1)/2 row-major
 * TILE x TILE tiles in packed lower order, diagonal tiles holding
 * inv(L_bb), elements of the factor precision (8 bytes in FP64 mode, 4 in
 * FP32-local mode; always 8 for the coarse factor). `out_bytes` must cover
 * them. For verification of asdg_factor/asdg_setup_coarse. */
asdg_status asdg_export_factor_tiles(asdg_problem* pb, int32_t sub, void* out, size_t out_bytes);

/* Launch-shape tuning (autotuner hook): what = ASDG_TUNE_*; value 0 restores
 * the default. CHOL_WG_PER_CU / TRSV_WG_PER_CU: persistent work-groups per
 * compute unit of the factorisation and triangular-sweep launches;
 * CHOL_GRID: total work-groups of the factorisation launch.
 * LOCAL_INVERSE (set before asdg_plan): 1 = apply the exact local solvers
 * through explicit inverses A_i^{-1} = L_i^{-T} L_i^{-1} formed after the
 * Cholesky factorisation (one pass over a packed symmetric matrix per
 * solve instead of two triangular sweeps; the factor buffer doubles); the
 * factor tiles then hold the lower tiles of A_i^{-1}. 0 = triangular sweeps.
 * SMALL_OFF (set before asdg_plan): by default, when every subdomain has at
 * most 64 DoFs (e.g. one element per subdomain, the setting of Sec. 7's
 * experiments), each A_i^{-1} is formed whole on the device (n_i x n_i,
 * row-major, factor precision) and applied inside the prolongation kernel;
 * asdg_export_factor_tiles then returns that n_i x n_i inverse. 1 = use the
 * tile path for such subdomains too.
 * NO_PRECOND (study aid, any time before a solve): 1 = asdg_pcg_solve runs
 * plain CG (identity preconditioner), so the Lanczos estimate in the stats
 * is K(A_h) rather than K(P_ad); asdg_apply is unaffected.
 * INV_WG_PER_CU: persistent work-groups per compute unit of the formation
 * of the explicit inverses. SYMV_WAVES: tiles (waves) per work-group of
 * the packed-inverse apply, 1, 2, 4 or 8 (others: EINVAL; default 4).
 * TASK_CHUNK:
 * queue order of the factorisation and inverse-formation tasks (tile tasks,
 * and the block-column tasks of INVERSE_SCHEDULE 2), 0 = all subdomains interleaved
 * (longest remaining path first), c > 0 = groups of c consecutive
 * subdomains one after the other (a smaller working set);
 * after asdg_bind it takes effect at the next asdg_factor. HOST_THREADS:
 * at most this many host threads for asdg_assemble / asdg_assemble_tet /
 * asdg_plan on this handle (0 = hardware threads, at most 16), for callers
 * that already run several handles' setup in parallel. COARSE_PACKED (set
 * before asdg_plan): storage of the explicit coarse inverse A_0^{-1} (used
 * for n0 <= 8192): 0 = packed lower tiles from n0 >= 4096 on, dense below
 * (default); 1 = always packed; 2 = always dense. The packed form is
 * applied by tiles (half the bytes), the dense one by one product.
 * FACTOR_SCHEDULE: how the local Cholesky factorisation is spread over
 * work-groups: 1 = one task per tile (a dependency-ordered queue with flag
 * waits: one subdomain can occupy many work-groups); 2 = one work-group per
 * subdomain (no waits; for many subdomains of similar size); 0 = automatic
 * (2 when the largest subdomain's factorisation is at most one and a half
 * times an even share of the whole over the device's work-groups).
 * INVERSE_SCHEDULE: the same choice for the formation of X = L^{-1}:
 * 1 = one task per tile, 2 = one work-group per block column of X (no
 * waits); 0 = automatic (2 when the largest column's products are at most
 * twice an even share). No launch shape or schedule changes the
 * arithmetic: results are identical for every setting.
 * TILE (set before asdg_plan): edge of the packed tiles of the local
 * Cholesky factors with the triangular sweeps (Sec. 3 local solvers):
 * 64 or 32 rows; 0 = automatic: 64, with the factor, scratch and task
 * buffers planned large enough for both edges, so that asdg_autotune
 * (FACTOR | LOCAL) can time both and keep the faster. 32-row tiles pad
 * each subdomain's ragged last tile row less, at the cost of four times
 * the tiles and twice the sweep steps. The edge changes the blocking of
 * the factorisation, so results of the two edges agree to rounding, not
 * bitwise. Explicit local inverses and the coarse factor always use 64
 * (LOCAL_INVERSE with TILE 32: EINVAL at asdg_plan). */
enum { ASDG_TUNE_CHOL_WG_PER_CU = 0, ASDG_TUNE_TRSV_WG_PER_CU = 1, ASDG_TUNE_CHOL_GRID = 2,
       ASDG_TUNE_TRACE = 3, ASDG_TUNE_LOCAL_INVERSE = 4, ASDG_TUNE_SMALL_OFF = 5, ASDG_TUNE_NO_PRECOND = 6,
       ASDG_TUNE_INV_WG_PER_CU = 7, ASDG_TUNE_SYMV_WAVES = 8, ASDG_TUNE_TASK_CHUNK = 9,
       ASDG_TUNE_HOST_THREADS = 10, ASDG_TUNE_COARSE_PACKED = 11, ASDG_TUNE_FACTOR_SCHEDULE = 12,
       ASDG_TUNE_INVERSE_SCHEDULE = 13, ASDG_TUNE_TILE = 14 };
asdg_status asdg_set_tuning(asdg_problem* pb, int32_t what, int32_t value);

/* Launch shapes chosen by asdg_autotune and the best times measured. */
typedef struct {
  int32_t chol_wg_per_cu, inv_wg_per_cu, trsv_wg_per_cu, symv_waves, task_chunk;
  double factor_ms; /* asdg_factor with the chosen shapes (0 if not tuned) */
  double local_ms;  /* one batched local solve with the chosen shape (0 if not tuned) */
  int32_t candidates; /* configurations timed */
  int32_t from_cache; /* 1: shapes taken from the process's tuning cache, nothing timed */
  int32_t factor_schedule; /* ASDG_TUNE_FACTOR_SCHEDULE in effect (1 or 2; 0 with whole small inverses) */
  int32_t inverse_schedule; /* ASDG_TUNE_INVERSE_SCHEDULE in effect (1 or 2; 0 without tiled explicit inverses) */
  int32_t tile; /* tile edge of the local factors in effect (64 or 32) */
} asdg_tune_report;

/* Own launch-shape autotuner (the batched factorisation and local-solve
 * launches of Sec. 3's local solvers): times every candidate on this
 * problem with HIP events on `stream` (one run when it takes more than
 * 20 ms, else the median of 3 to 15 runs filling about 20 ms) and keeps the
 * fastest, through the same
 * settings as asdg_set_tuning.
 * FACTOR | LOCAL with the automatic tile edge (ASDG_TUNE_TILE 0, triangular
 * sweeps): first the tile edge of the local factors, 64 or 32, by the time
 * of one batched local solve (the step repeated every iteration; each edge
 * factorised once with default shapes); then the shapes below for that edge.
 * ASDG_AUTOTUNE_FACTOR (after asdg_bind): the Cholesky schedule
 * (FACTOR_SCHEDULE 1, 2), with explicit inverses the schedule of
 * X = L^{-1} (INVERSE_SCHEDULE 1, 2), work-groups per compute unit of
 * the Cholesky launch (1, 2 with 64-row tiles; 4, 8 with 32-row tiles), the task order
 * (TASK_CHUNK 0, and 64 when there are more than 64 subdomains) and, with explicit inverses,
 * work-groups per compute unit of the inverse formation (1-4 FP32, 1-2
 * FP64); runs asdg_factor up to 15 times per candidate and leaves the
 * problem factorised. ASDG_AUTOTUNE_LOCAL (after
 * asdg_factor, or together with FACTOR): waves per work-group of the packed
 * apply (1, 2, 4, 8) or work-groups per compute unit of the triangular
 * sweeps (1-4); overwrites the solver's internal vectors (not the factors
 * or the coarse level). Problems whose subdomains all have at most 64 DoFs
 * (whole small inverses) have no such launches: nothing is timed. Results
 * of later solves are identical for every choice. rep may be NULL.
 * Results of a FACTOR | LOCAL run are kept in a process-wide cache keyed
 * by device architecture, precision, local-solve representation and size
 * class (subdomain count to a power of two, largest and mean tile rows per
 * subdomain, in 64-row units). With ASDG_AUTOTUNE_REUSE and a cache hit
 * nothing is timed: the cached shapes are applied (with FACTOR also the
 * cached tile edge, when the plan has room for both, and asdg_factor run
 * once) and rep->from_cache is 1.
 * Errors: EINVAL (flags), ESTATE (stage, or a solve in progress), EHIP,
 * and those of asdg_factor. */
enum { ASDG_AUTOTUNE_FACTOR = 1, ASDG_AUTOTUNE_LOCAL = 2, ASDG_AUTOTUNE_REUSE = 4 };
asdg_status asdg_autotune(asdg_problem* pb, int32_t what, void* stream, asdg_tune_report* rep);

/* The tuning cache as text, one line per size class (key, then Cholesky,
 * inverse-formation and sweep work-groups per CU, packed-apply waves,
 * task-order chunk, best factorisation and local-solve ms, Cholesky and
 * inverse-formation schedules, tile edge; lines of older files without the
 * last one to three fields load with automatic schedules and 64-row
 * tiles). save writes
 * the whole cache (EINVAL if the file cannot be written); load adds the
 * entries of a file written by save (n_entries: how many; EINVAL and
 * nothing added if it cannot be read or a line is malformed). Both are
 * safe to call from any thread. */
asdg_status asdg_tune_cache_save(const char* path);
asdg_status asdg_tune_cache_load(const char* path, int32_t* n_entries);

/* Task trace of the last batched local solve launched while
 * ASDG_TUNE_TRACE = 1 (profiling aid). tasks: [n][4] int32 (subdomain,
 * direction 0 = forward / 1 = backward, tile row, 0) in queue order; times:
 * [n][3] wall-clock ticks per task (dequeued, waits done, finished);
 * clock_mhz: tick rate. With tasks/times NULL only n_tasks (and the clock)
 * are returned. */
asdg_status asdg_export_trace(asdg_problem* pb, int32_t* tasks, uint64_t* times, int64_t max_tasks,
                              int64_t* n_tasks, double* clock_mhz);

/* Local-solver representation chosen by asdg_plan: ASDG_LOCAL_SWEEPS (tile
 * Cholesky factors, two triangular sweeps), ASDG_LOCAL_INVERSE (packed tile
 * inverses, one symmetric pass), ASDG_LOCAL_SMALL (whole inverses of
 * subdomains of at most 64 DoFs, applied inside the prolongation);
 * -1 before asdg_plan or for a NULL handle. */
enum { ASDG_LOCAL_SWEEPS = 0, ASDG_LOCAL_INVERSE = 1, ASDG_LOCAL_SMALL = 2 };
int32_t asdg_local_mode(const asdg_problem* pb);

/* Subdomain index of the last ENOTSPD failure (-1 = coarse, -2 = none). */
int32_t asdg_failed_subdomain(const asdg_problem* pb);

#ifdef __cplusplus
}
#endif

#endif /* ASDG_H */
