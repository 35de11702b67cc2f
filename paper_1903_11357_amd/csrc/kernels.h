// Launchers of the gfx950 kernels (internal to libasdg).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace asdg {

constexpr int TILE = 64;            // tile edge of the coarse factor and the explicit inverses (local sweeps: 64 or 32)
constexpr int MAXG = 8192;          // max work-groups of a kernel that reduces over the grid
constexpr int HIST = 65536;         // recorded CG coefficients (Lanczos estimate)

// Deterministic grid-wide sum: per-work-group partials, then the last
// work-group to finish adds them in index order (see grid_sum()).
constexpr int RGROUP = 64;  // work-groups per first-level arrival counter
struct Reduction {
  double partial[MAXG];             // one per work-group
  double gpartial[MAXG / RGROUP];   // one per group of RGROUP work-groups
  uint32_t gcounter[MAXG / RGROUP]; // arrivals per group; re-armed by the group's last
  uint32_t counter;                 // arrivals of group sums; re-armed by the last
  uint32_t pad;
  double result;
};
enum { RED_PQ = 0, RED_RR = 1, RED_RZ = 2, RED_BB = 3, N_RED = 4 };

// Device-resident PCG state (lives in the scratch buffer).
struct DevState {
  double bb;        // ||b||^2
  double tol2;      // rtol^2 ||b||^2
  double rr;        // last ||r||^2
  double trr;       // ||b - A x||^2 at exit (true residual, after the loop)
  int32_t it;       // completed iterations
  int32_t done;     // 1 once the loop must stop
  int32_t status;   // 0 running, 1 converged, 2 max_iter, 3 breakdown, 4 spin timeout
  int32_t max_iter;
  int32_t q_local;  // work queue counter of the local triangular solves
  int32_t q_coarse; // work queue counter of the coarse triangular solves
  int32_t q_chol;   // work queue counter of the factorisation
  int32_t chol_fail;// smallest failing subdomain (0x7fffffff = none)
  int32_t abort;    // set when a bounded wait expired
  int32_t pad;
};

// Per-subdomain descriptor of a tile-packed lower-triangular factor.
struct SubDesc {
  int32_t dof0;   // first (internal) DoF of the subdomain
  int32_t n;      // DoFs
  int32_t nb;     // tile rows = ceil(n / tile edge)
  int32_t tile0;  // index of tile (0,0); tile (b,j) is tile0 + b(b+1)/2 + j
};

// Vector / operator kernels (kern_vec.hip). `red` points at the N_RED
// reduction slots; kernels that reduce write red[RED_*].result.
hipError_t launch_spmv(int np, int32_t n_cells, const int32_t* row_ptr, const int32_t* col,
                       const double* blocks, const double* p, double* q, Reduction* red,
                       const DevState* st, hipStream_t s);
hipError_t launch_permute_in(int np, int32_t n_cells, const int32_t* perm, const double* src,
                             double* r, double* x, void* yl, void* zl, int local_f32,
                             Reduction* red, DevState* st, double rtol, int max_iter, hipStream_t s);
hipError_t launch_unpermute_out(int np, int32_t n_cells, const int32_t* perm, const double* x,
                                double* dst, hipStream_t s);
// st->trr = ||b - Ax||^2 with b in caller order (src, permuted on the fly)
// and Ax in internal order (ax); deterministic grid sum through `red`.
hipError_t launch_true_residual(int np, int32_t n_cells, const int32_t* perm, const double* src,
                                const double* ax, Reduction* red, DevState* st, hipStream_t s);
// Work-groups (= partials of the dot product each produces) of the operator
// apply and of the grid-stride vector kernels, for n DoFs.
int spmv_parts(int64_t n);
int vec_parts(int64_t n);
int prolong_parts(int64_t n);
hipError_t launch_update_xr(int64_t n, DevState* st, Reduction* red, int n_pq, const double* rz2,
                            double* alpha_hist, const double* p, const double* q, double* x, double* r, void* yl,
                            void* zl, int local_f32, hipStream_t s);
// r0 = P_0^T r with each coarse cell's entries split over `splits` work-
// groups: out holds `splits` partial vectors of n0 (splits = 1: r0).
hipError_t launch_restrict(int np, int nq, int32_t n_coarse, int splits, const int32_t* tptr,
                           const int32_t* tcell, const int32_t* tblk, const double* P, const double* r,
                           double* out, double* y0, double* z0, const DevState* st, hipStream_t s);
// Per-tile partial vectors of the packed symmetric local apply, summed per
// DoF by the prolongation kernel (in place of a local solution vector).
struct LocalParts {
  const int32_t* cell_sub;  // subdomain of each cell
  const SubDesc* subs;
  const void* part;  // 2*TILE entries per stored tile (rows, then columns); small: the inverses
  int small;         // 1: z_loc = A_i^{-1} r_i from whole small inverses (launch_small_inverse);
                     // 2: z = r (identity preconditioner; the coarse part is skipped too);
                     // 3: z_loc given as an FP64 vector in `part`
};
// n_pq > 0: a PCG iteration; work-group 0 sums n_pq partials of p.Ap and
// n_rr of ||r||^2, counts the iteration and takes the stopping decision.
hipError_t launch_prolong(int np, int nq, int32_t n_cells, const int32_t* pptr, const int32_t* pcol,
                          const double* P, const double* z0, const void* zl, const LocalParts* lp,
                          int local_f32, const double* r, double* z, Reduction* red, DevState* st,
                          int n_pq, int n_rr, hipStream_t s);
hipError_t launch_update_p(int64_t n, DevState* st, const Reduction* red, int n_rz, double* rz2,
                           double* beta_hist, const double* z, double* p, int init, hipStream_t s);
hipError_t launch_fill_i32(int32_t* dst, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_reset_queues(DevState* st, hipStream_t s);

// Local-factor formation and batched Cholesky (kern_chol.hip).
// tile: edge of the packed tiles, 64 or 32 (hipErrorInvalidValue otherwise).
hipError_t launch_gather_tiles(int np, int tile, int32_t n_tiles, const int4* tile_meta, const SubDesc* subs,
                               const int32_t* row_ptr, const int32_t* col, const double* blocks,
                               void* tiles, int f32, hipStream_t s);
// per_sub = 0: tasks (subdomain, j, b, -) of every tile, dependency-ordered;
// per_sub = 1: tasks (subdomain, -, -, -), one work-group per subdomain.
// Work-groups of four waves (tile 64) or one wave (tile 32).
hipError_t launch_cholesky(int f32, int tile, int per_sub, int32_t n_tasks, const int4* tasks, const SubDesc* subs,
                           void* tiles, int32_t* flags, DevState* st, int32_t* queue, int grid, hipStream_t s);

// Explicit local inverses (kern_inv.hip) and their packed symmetric apply
// (kern_symv.hip).
// cols = 0: tasks (subdomain, j, b, -) of every tile of X = L^{-1}, dependency-
// ordered; cols = 1: tasks (subdomain, j, -, -), one block column each.
hipError_t launch_inverse(int f32, int cols, int32_t n_tasks, const int4* tasks, int32_t n_tiles, const int4* meta,
                          const SubDesc* subs, void* L, void* X, int32_t* flags, DevState* st, int32_t* queue,
                          int grid_lower, int grid_gram, hipStream_t s);
// Phase 1 of the packed symmetric apply: per stored tile (b, j), the row
// sums S_bj r_j and the column sums S_bj^T r_b (diagonal tiles: row sums of
// the lower triangle with the diagonal, column sums of the strict lower
// triangle); summed per DoF by launch_prolong with LocalParts. meta[t] = (subdomain, b, j, rows of tile
// row b inside the subdomain). waves: tiles (waves) per work-group, 1, 2, 4 or 8 (hipErrorInvalidValue
// otherwise).
hipError_t launch_symv_tiles(int f32, int waves, int32_t n_tiles, const int4* meta, const SubDesc* subs, const void* S,
                             const double* r, void* part, const DevState* st, hipStream_t s);
// Per-DoF sums of the FP64 tile partials of one packed symmetric matrix of
// order n (nb tile rows), in the fixed order of the local prolongation
// (the packed coarse inverse).
hipError_t launch_tile_partials_sum(int32_t n, int32_t nb, const double* part, double* out, const DevState* st,
                                    hipStream_t s);
// out[i] = sum_s in[s n + i] (the restriction's split partial vectors).
hipError_t launch_sum_splits(int32_t n, int splits, const double* in, double* out, const DevState* st, hipStream_t s);

// Subdomains of at most 64 DoFs: A_i^{-1} whole (n_i x n_i row-major) at
// word offset subs[i].tile0, formed by one wave per subdomain (max_n =
// largest n_i, sizes the LDS).
hipError_t launch_small_inverse(int f32, int32_t n_sub, int np, int max_n, const SubDesc* subs, const int32_t* row_ptr,
                                const int32_t* col, const double* blocks, void* S, DevState* st, hipStream_t s);

// Coarse level with an explicit inverse: expand the packed lower tiles of
// A_0^{-1} to a dense row-major matrix; y = D x, one wave per row.
hipError_t launch_expand_sym(int32_t n0, const double* S, double* D, hipStream_t s);
hipError_t launch_dense_mv(int32_t n, int splits, const double* D, const double* xp, double* y, const DevState* st,
                           hipStream_t s);

// Batched forward/backward triangular sweeps (kern_trsv.hip) over packed
// tiles of edge `tile` (64 or 32).
// trace (optional): per task, wall-clock at dequeue, end of waits, end.
hipError_t launch_trsv(int f32, int tile, int32_t n_tasks, const int4* tasks, const SubDesc* subs,
                       const void* tiles, const double* r, void* y, void* z, DevState* st,
                       int32_t* queue, int grid, uint64_t* trace, hipStream_t s);

}  // namespace asdg
