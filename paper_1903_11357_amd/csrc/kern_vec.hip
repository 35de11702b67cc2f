// Operator apply, PCG vector updates, coarse restriction/prolongation.
//
// Block-sparse SIPG operator (Sec. 2, eq. (Ah)): one thread per output DoF
// (cell, a); blocks are stored row-major, so the thread streams row a of
// each block of its block row (n_p contiguous doubles) against the n_p
// contiguous entries of the neighbour's p; the n_p threads of a cell read
// one contiguous block together. Every DoF is independent, so the launch has
// n threads of memory-level parallelism instead of one dependent chain per
// block row.
//
// PCG (Sec. 7): every dot product is deterministic. The producing kernel
// stores one partial per work-group; the kernel that needs the value sums
// the partials itself, every work-group in the same fixed order (no
// floating-point atomics, no arrival counters, bitwise-repeatable solves).
// Work-group 0 of the prolongation, the last kernel of the preconditioner,
// takes the stopping decision and counts the iteration, so an iteration
// needs no separate control kernel.
#include "kern_common.h"

namespace asdg {

namespace {

constexpr int VEC_GRID = 1024;      // work-groups of the grid-stride vector kernels
constexpr int SPMV_GRID = 2048;     // work-groups of the operator apply
constexpr int PROLONG_GRID = 4096;  // prolongation (+ local partial sums): one DoF per thread up to 1M DoFs

int grid_for(int64_t n, int cap) {
  int64_t g = (n + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

template <int NP>
__global__ __launch_bounds__(256) void k_spmv(int32_t N, const int32_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col,
                                              const double* __restrict__ blocks,
                                              const double* __restrict__ p, double* __restrict__ q,
                                              Reduction* red, const DevState* st) {
  __shared__ double scratch[4];
  if (st && st->done) return;
  const int64_t n = (int64_t)N * NP;
  double dot = 0.0;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    const int cell = (int)(d / NP);
    const int a = (int)(d - (int64_t)cell * NP);
    const int k0 = row_ptr[cell], k1 = row_ptr[cell + 1];
    double acc = 0.0;
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
      const double* B = blocks + ((size_t)k * NP + a) * NP;  // row a of block k
      const double* pv = p + (size_t)col[k] * NP;
#pragma unroll
      for (int b = 0; b < NP; ++b) acc += B[b] * pv[b];
    }
    q[d] = acc;
    dot += p[d] * acc;
  }
  if (red) partial_store(dot, red + RED_PQ, scratch);
}

// Even n_p (2D p = 2, 3; tetrahedra p = 1, 2, 3): the lanes of a wave in
// groups of n_p per cell (64 / n_p cells per wave, the remaining lanes
// idle). Lane a of a cell reads the 16-byte pieces a + n_p i (i < n_p / 2)
// of each n_p x n_p block, so the group's loads cover contiguous 16 n_p
// bytes; those pieces are rows rho + 2i (rho = 2a / n_p) at columns
// c = 2 (a mod n_p/2), c + 1, and only p[c], p[c+1] of the neighbour are
// needed. Each lane keeps n_p / 2 partial row sums over all blocks of the
// row; the n_p / 2 lanes sharing a row parity add them (LDS, fixed order).
// Column indices are fetched U at a time ahead of the block and p loads.
template <int NP>
__global__ __launch_bounds__(256) void k_spmv_even(int32_t N, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ blocks,
                                                   const double* __restrict__ p, double* __restrict__ q,
                                                   Reduction* red, const DevState* st) {
  static_assert(NP % 2 == 0 && NP <= 64, "even block size");
  constexpr int H = NP / 2, CPW = 64 / NP, U = NP <= 10 ? 4 : 2;
  __shared__ double scratch[4];
  __shared__ double s_part[4][CPW * NP * H];
  if (st && st->done) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ci = lane / NP, a = lane - ci * NP;
  const int cp = 2 * (a % H);
  const int ngroups = (N + CPW - 1) / CPW;
  double* sp = s_part[w];
  double dot = 0.0;
  for (int g = blockIdx.x * 4 + w; g < ngroups; g += gridDim.x * 4) {
    const int cell = g * CPW + ci;
    const bool on = ci < CPW && cell < N;
    double acc[H];
#pragma unroll
    for (int i = 0; i < H; ++i) acc[i] = 0.0;
    if (on) {
      const int k0 = row_ptr[cell], k1 = row_ptr[cell + 1];
      for (int kb = k0; kb < k1; kb += U) {
        int cc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cc[u] = kb + u < k1 ? col[kb + u] : -1;
        double2 pv[U], bb[U][H];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (cc[u] >= 0) {
            pv[u] = *reinterpret_cast<const double2*>(p + (size_t)cc[u] * NP + cp);
            const double2* B = reinterpret_cast<const double2*>(blocks + (size_t)(kb + u) * NP * NP) + a;
#pragma unroll
            for (int i = 0; i < H; ++i) bb[u][i] = B[NP * i];
          } else {
            pv[u] = make_double2(0.0, 0.0);
#pragma unroll
            for (int i = 0; i < H; ++i) bb[u][i] = make_double2(0.0, 0.0);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int i = 0; i < H; ++i) acc[i] += bb[u][i].x * pv[u].x + bb[u][i].y * pv[u].y;
      }
#pragma unroll
      for (int i = 0; i < H; ++i) sp[(ci * NP + a) * H + i] = acc[i];
    }
    wave_sync();
    if (on) {
      // row a = (a & 1) + 2 (a >> 1): sum over the lanes of that parity
      const int rr = a & 1, ii = a >> 1;
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < H; ++m) v += sp[(ci * NP + rr * H + m) * H + ii];
      const int64_t d = (int64_t)cell * NP + a;
      q[d] = v;
      dot += p[d] * v;
    }
    wave_sync();
  }
  if (red) partial_store(dot, red + RED_PQ, scratch);
}

// r = permuted b, x = 0 (x optional), triangular-sweep outputs = sentinel
// (yl, zl optional); with `st`, ||b||^2 and the initial PCG state.
template <typename T>
__global__ __launch_bounds__(256) void k_permute_in(int np, int32_t N, const int32_t* __restrict__ perm,
                                                    const double* __restrict__ src, double* __restrict__ r,
                                                    double* __restrict__ x, T* __restrict__ yl,
                                                    T* __restrict__ zl, Reduction* red, DevState* st,
                                                    double rtol, int max_iter) {
  __shared__ double scratch[4];
  const int64_t n = (int64_t)N * np;
  double acc = 0.0;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = d / np;
    const int a = (int)(d - cell * np);
    const double v = src[(int64_t)perm[cell] * np + a];
    r[d] = v;
    if (x) x[d] = 0.0;
    if (yl) {
      yl[d] = sentinel<T>();
      zl[d] = sentinel<T>();
    }
    acc += v * v;
  }
  if (!st) return;
  double bb;
  if (grid_sum(acc, red + RED_BB, scratch, bb) && threadIdx.x == 0) {
    st->bb = bb;
    st->tol2 = rtol * rtol * bb;
    st->rr = bb;
    st->it = 0;
    st->max_iter = max_iter;
    st->q_local = 0;
    st->q_coarse = 0;
    st->abort = 0;
    if (bb == 0.0) {
      st->done = 1;
      st->status = 1;
    } else if (!(bb == bb)) {
      st->done = 1;
      st->status = 3;
    } else {
      st->done = 0;
      st->status = 0;
    }
  }
}

__global__ __launch_bounds__(256) void k_unpermute(int np, int32_t N, const int32_t* __restrict__ perm,
                                                   const double* __restrict__ x, double* __restrict__ dst) {
  const int64_t n = (int64_t)N * np;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = d / np;
    const int a = (int)(d - cell * np);
    dst[(int64_t)perm[cell] * np + a] = x[d];
  }
}

// ||b - Ax||^2 (the true residual of the final iterate, Sec. 7 reports the
// relative residual): b read through the permutation, Ax from the operator
// apply of x in internal order; fixed-order grid sum into st->trr.
__global__ __launch_bounds__(256) void k_true_residual(int np, int32_t N, const int32_t* __restrict__ perm,
                                                       const double* __restrict__ src, const double* __restrict__ ax,
                                                       Reduction* red, DevState* st) {
  __shared__ double scratch[4];
  const int64_t n = (int64_t)N * np;
  double acc = 0.0;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = d / np;
    const int a = (int)(d - cell * np);
    const double e = src[(int64_t)perm[cell] * np + a] - ax[d];
    acc += e * e;
  }
  double tot;
  if (grid_sum(acc, red, scratch, tot) && threadIdx.x == 0) st->trr = tot;
}

// alpha = (r.z)/(p.Ap) with p.Ap summed from the operator apply's partials;
// x += alpha p; r -= alpha Ap; partials of ||r||^2. On breakdown (p.Ap not
// positive) x and r are left unchanged; the stopping decision after the
// preconditioner reports it. Work-group 0 records alpha and re-arms the
// work queues of the triangular sweeps.
template <typename T>
__global__ __launch_bounds__(256) void k_update_xr(int64_t n, DevState* st, Reduction* red, int n_pq,
                                                   const double* __restrict__ rz2, double* __restrict__ alpha_hist,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   T* __restrict__ yl, T* __restrict__ zl) {
  __shared__ double scratch[4];
  if (st->done) return;
  // the operands of this thread's first KX elements are loaded before the
  // reduction, so their latency overlaps it
  constexpr int KX = 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, d0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double xv[KX], pv[KX], rv0[KX], qv[KX];
#pragma unroll
  for (int u = 0; u < KX; ++u) {
    const int64_t d = d0 + u * stride;
    if (d < n) {
      xv[u] = x[d];
      pv[u] = p[d];
      rv0[u] = r[d];
      qv[u] = q[d];
    }
  }
  const double pq = partials_sum(red + RED_PQ, n_pq, scratch);
  const int it = st->it;
  const double alpha = pq > 0.0 ? rz2[it & 1] / pq : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (it < HIST) alpha_hist[it] = alpha;
    st->q_local = 0;
    st->q_coarse = 0;
  }
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < KX; ++u) {
    const int64_t d = d0 + u * stride;
    if (d < n) {
      x[d] = xv[u] + alpha * pv[u];
      const double rv = rv0[u] - alpha * qv[u];
      r[d] = rv;
      acc += rv * rv;
      if (yl) {  // re-arm the sweep dataflow vectors
        yl[d] = sentinel<T>();
        zl[d] = sentinel<T>();
      }
    }
  }
  for (int64_t d = d0 + KX * stride; d < n; d += stride) {
    x[d] += alpha * p[d];
    const double rv = r[d] - alpha * q[d];
    r[d] = rv;
    acc += rv * rv;
    if (yl) {
      yl[d] = sentinel<T>();
      zl[d] = sentinel<T>();
    }
  }
  partial_store(acc, red + RED_RR, scratch);
}

// r0 = P_0^T r. The (entry, fine row a) pairs of coarse cell J's transposed
// list are split over `splits` work-groups (blockIdx.x = J * splits + s,
// threads stride the pairs: consecutive threads read consecutive rows of a
// P block and consecutive entries of r); work-group (J, s) writes its NQ
// fixed-order sums to out[(s n_coarse + J) NQ + c].
// With one split that is r0 itself; otherwise the coarse solve adds the
// splits (launch_dense_mv). y0/z0 (optional): re-armed sweep sentinels.
template <int NP, int NQ>
__global__ __launch_bounds__(256) void k_restrict(int32_t n_coarse, int splits, const int32_t* __restrict__ tptr,
                                                  const int32_t* __restrict__ tcell,
                                                  const int32_t* __restrict__ tblk, const double* __restrict__ P,
                                                  const double* __restrict__ r, double* __restrict__ out,
                                                  double* __restrict__ y0, double* __restrict__ z0,
                                                  const DevState* st) {
  __shared__ double scratch[4];
  if (st && st->done) return;
  const int J = blockIdx.x / splits, sp = blockIdx.x - J * splits;
  double acc[NQ];
#pragma unroll
  for (int c = 0; c < NQ; ++c) acc[c] = 0.0;
  const int k0 = tptr[J], pairs = (tptr[J + 1] - k0) * NP;
#pragma unroll 4
  for (int i = sp * blockDim.x + threadIdx.x; i < pairs; i += splits * blockDim.x) {
    const int kk = i / NP, a = i - kk * NP;
    const int k = k0 + kk;
    const double v = r[(size_t)tcell[k] * NP + a];
    const double* Pr = P + ((size_t)tblk[k] * NP + a) * NQ;
#pragma unroll
    for (int c = 0; c < NQ; ++c) acc[c] += Pr[c] * v;
  }
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const double sum = block_sum(acc[c], scratch);
    if (threadIdx.x == 0) {
      out[((size_t)sp * n_coarse + J) * NQ + c] = sum;
      if (y0) {
        y0[J * NQ + c] = sentinel_f64();
        z0[J * NQ + c] = sentinel_f64();
      }
    }
  }
}

// z = z_loc + P_0 z0 (either part optional), and r.z. The local part is
// (L = 0) a vector zl; (L = 1) the sum, in a fixed order, of the packed
// symmetric apply's per-tile partial vectors for the DoF's row:
//   z_loc[d] = sum_{j<=b} part(b,j).rows[rho] + sum_{j>=b} part(j,b).cols[rho]
// with d = dof0 + 64 b + rho in its subdomain; or (L = 2) row `loc` of a
// small subdomain's whole inverse times r_i (n_i <= 64 terms, FP64 sums);
// or (L = 3) r itself (identity preconditioner, no coarse part); or (L = 4)
// an FP64 vector zd computed before (the small-subdomain solves run as a
// launch of their own beside the coarse correction).
//
// With `red`, partials of r.z. With n_pq > 0 (a PCG iteration), work-group 0
// also sums the partials of p.Ap and ||r||^2 left by the operator apply and
// the residual update, counts the iteration and takes the stopping decision
// (abort > breakdown > converged > iteration limit). No other work-group of
// this launch reads the fields it writes.
template <int NP, int NQ, typename T, int L>
__global__ __launch_bounds__(256) void k_prolong(int32_t N, const int32_t* __restrict__ pptr,
                                                 const int32_t* __restrict__ pcol, const double* __restrict__ P,
                                                 const double* __restrict__ z0, const T* __restrict__ zl,
                                                 const int32_t* __restrict__ cell_sub,
                                                 const SubDesc* __restrict__ subs, const T* __restrict__ part,
                                                 const double* __restrict__ zd, const double* __restrict__ r,
                                                 double* __restrict__ z, Reduction* red, DevState* st, int n_pq,
                                                 int n_rr) {
  __shared__ double scratch[4];
  if (st && st->done) return;
  if (n_pq > 0 && blockIdx.x == 0) {
    const double pq = partials_sum(red + RED_PQ, n_pq, scratch);
    const double rr = partials_sum(red + RED_RR, n_rr, scratch);
    if (threadIdx.x == 0) {
      const int it1 = st->it + 1;
      st->it = it1;
      st->rr = rr;
      if (st->abort) {
        st->status = 4;
        st->done = 1;
      } else if (!(pq > 0.0) || !(rr == rr)) {
        st->status = 3;
        st->done = 1;
      } else if (rr <= st->tol2) {
        st->status = 1;
        st->done = 1;
      } else if (it1 >= st->max_iter) {
        st->status = 2;
        st->done = 1;
      }
    }
  }
  const int64_t n = (int64_t)N * NP;
  double acc = 0.0;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = d / NP;
    const int a = (int)(d - cell * NP);
    double v = 0.0;
    if (L == 3) {
      v = r[d];  // identity preconditioner (plain CG)
    } else if (L == 4) {
      v = zd[d];
    } else if (L == 2) {
      const SubDesc sd = subs[cell_sub[cell]];
      const int loc = (int)(d - sd.dof0);
      const T* Srow = part + sd.tile0 + (size_t)loc * sd.n;
      const double* ri = r + sd.dof0;
#pragma unroll 8
      for (int b = 0; b < sd.n; ++b) v += (double)Srow[b] * ri[b];
    } else if (L == 1) {
      const SubDesc sd = subs[cell_sub[cell]];
      const int loc = (int)(d - sd.dof0);
      const int b = loc / TILE, rho = loc - b * TILE;
      const T* pr = part + (size_t)(sd.tile0 + b * (b + 1) / 2) * 2 * TILE + rho;
      // (unrolled so the independent loads are in flight together; the sums stay in order)
#pragma unroll 8
      for (int j = 0; j <= b; ++j) v += (double)pr[(size_t)j * 2 * TILE];
      v += (double)pr[(size_t)b * 2 * TILE + TILE];  // strictly lower part of the diagonal tile, transposed
#pragma unroll 8
      for (int j = b + 1; j < sd.nb; ++j)
        v += (double)part[(size_t)(sd.tile0 + j * (j + 1) / 2 + b) * 2 * TILE + TILE + rho];
    } else if (zl) {
      v = (double)zl[d];
    }
    if (pptr) {
      for (int e = pptr[cell]; e < pptr[cell + 1]; ++e) {
        const double* Pb = P + (size_t)e * NP * NQ + a * NQ;
        const double* zc = z0 + (size_t)pcol[e] * NQ;
#pragma unroll
        for (int c = 0; c < NQ; ++c) v += Pb[c] * zc[c];
      }
    }
    z[d] = v;
    acc += r[d] * v;
  }
  if (red) partial_store(acc, red + RED_RZ, scratch);
}

// beta = (r.z)_new / (r.z)_old; p = z + beta p (init: p = z).
__global__ __launch_bounds__(256) void k_update_p(int64_t n, DevState* st, const Reduction* red, int n_rz,
                                                  double* __restrict__ rz2, double* __restrict__ beta_hist,
                                                  const double* __restrict__ z, double* __restrict__ p, int init) {
  __shared__ double scratch[4];
  if (st->done) return;
  // this thread's first KP elements of z and p are loaded before the reduction
  constexpr int KP = 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, d0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double zv[KP], pv[KP];
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    const int64_t d = d0 + u * stride;
    if (d < n) {
      zv[u] = z[d];
      pv[u] = init ? 0.0 : p[d];
    }
  }
  const double rz_new = partials_sum(red + RED_RZ, n_rz, scratch);
  if (init) {
    if (blockIdx.x == 0 && threadIdx.x == 0) rz2[0] = rz_new;
#pragma unroll
    for (int u = 0; u < KP; ++u) {
      const int64_t d = d0 + u * stride;
      if (d < n) p[d] = zv[u];
    }
    for (int64_t d = d0 + KP * stride; d < n; d += stride) p[d] = z[d];
    return;
  }
  const int it = st->it;
  const double beta = rz_new / rz2[(it - 1) & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    rz2[it & 1] = rz_new;
    if (it - 1 < HIST) beta_hist[it - 1] = beta;
  }
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    const int64_t d = d0 + u * stride;
    if (d < n) p[d] = zv[u] + beta * pv[u];
  }
  for (int64_t d = d0 + KP * stride; d < n; d += stride) p[d] = z[d] + beta * p[d];
}

__global__ void k_fill_i32(int32_t* dst, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

__global__ void k_reset_queues(DevState* st) {
  if (threadIdx.x == 0) {
    st->q_local = 0;
    st->q_coarse = 0;
    st->q_chol = 0;
    st->chol_fail = 0x7fffffff;
    st->abort = 0;
    st->done = 0;
    st->status = 0;
  }
}

}  // namespace

int spmv_parts(int64_t n) { return grid_for(n, SPMV_GRID); }
int vec_parts(int64_t n) { return grid_for(n, VEC_GRID); }
int prolong_parts(int64_t n) { return grid_for(n, PROLONG_GRID); }

hipError_t launch_spmv(int np, int32_t N, const int32_t* row_ptr, const int32_t* col, const double* blocks,
                       const double* p, double* q, Reduction* red, const DevState* st, hipStream_t s) {
  dim3 g(spmv_parts((int64_t)N * np)), b(256);
  switch (np) {
    case 3: hipLaunchKernelGGL(k_spmv<3>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    case 6: hipLaunchKernelGGL(k_spmv_even<6>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    case 10: hipLaunchKernelGGL(k_spmv_even<10>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    case 15: hipLaunchKernelGGL(k_spmv<15>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    // tetrahedra: p = 1, 3 (p = 2 shares n_p = 10 with p = 3 in 2D)
    case 4: hipLaunchKernelGGL(k_spmv_even<4>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    case 20: hipLaunchKernelGGL(k_spmv_even<20>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    // 2D p = 5..9 (the condition-number studies of high degree): one thread per DoF
    case 21: hipLaunchKernelGGL(k_spmv<21>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    case 28: hipLaunchKernelGGL(k_spmv<28>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    case 36: hipLaunchKernelGGL(k_spmv<36>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    case 45: hipLaunchKernelGGL(k_spmv<45>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    case 55: hipLaunchKernelGGL(k_spmv<55>, g, b, 0, s, N, row_ptr, col, blocks, p, q, red, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_permute_in(int np, int32_t N, const int32_t* perm, const double* src, double* r, double* x,
                             void* yl, void* zl, int local_f32, Reduction* red, DevState* st, double rtol,
                             int max_iter, hipStream_t s) {
  dim3 g(grid_for((int64_t)N * np, VEC_GRID)), b(256);
  if (local_f32)
    hipLaunchKernelGGL(k_permute_in<float>, g, b, 0, s, np, N, perm, src, r, x, (float*)yl, (float*)zl, red, st,
                       rtol, max_iter);
  else
    hipLaunchKernelGGL(k_permute_in<double>, g, b, 0, s, np, N, perm, src, r, x, (double*)yl, (double*)zl, red, st,
                       rtol, max_iter);
  return hipGetLastError();
}

hipError_t launch_unpermute_out(int np, int32_t N, const int32_t* perm, const double* x, double* dst,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute, dim3(grid_for((int64_t)N * np, VEC_GRID)), dim3(256), 0, s, np, N, perm, x, dst);
  return hipGetLastError();
}

hipError_t launch_true_residual(int np, int32_t N, const int32_t* perm, const double* src, const double* ax,
                                Reduction* red, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_true_residual, dim3(grid_for((int64_t)N * np, VEC_GRID)), dim3(256), 0, s, np, N, perm, src,
                     ax, red, st);
  return hipGetLastError();
}

hipError_t launch_update_xr(int64_t n, DevState* st, Reduction* red, int n_pq, const double* rz2,
                            double* alpha_hist, const double* p, const double* q, double* x, double* r, void* yl,
                            void* zl, int local_f32, hipStream_t s) {
  dim3 g(vec_parts(n)), b(256);
  if (local_f32)
    hipLaunchKernelGGL(k_update_xr<float>, g, b, 0, s, n, st, red, n_pq, rz2, alpha_hist, p, q, x, r, (float*)yl,
                       (float*)zl);
  else
    hipLaunchKernelGGL(k_update_xr<double>, g, b, 0, s, n, st, red, n_pq, rz2, alpha_hist, p, q, x, r,
                       (double*)yl, (double*)zl);
  return hipGetLastError();
}

template <int NP, int NQ>
static void restrict_t(int32_t nc, int splits, const int32_t* tptr, const int32_t* tcell, const int32_t* tblk,
                       const double* P, const double* r, double* out, double* y0, double* z0, const DevState* st,
                       hipStream_t s) {
  hipLaunchKernelGGL((k_restrict<NP, NQ>), dim3(nc * splits), dim3(256), 0, s, nc, splits, tptr, tcell, tblk, P, r,
                     out, y0, z0, st);
}

#define ASDG_PQ_SWITCH(NPV, NQV, CALL) \
  if (np == NPV && nq == NQV) {        \
    CALL;                              \
    return hipGetLastError();          \
  }

hipError_t launch_restrict(int np, int nq, int32_t nc, int splits, const int32_t* tptr, const int32_t* tcell,
                           const int32_t* tblk, const double* P, const double* r, double* out, double* y0, double* z0,
                           const DevState* st, hipStream_t s) {
  if (splits < 1 || (int64_t)nc * splits > 0x7fffffff) return hipErrorInvalidValue;
#define R_(A, B) ASDG_PQ_SWITCH(A, B, (restrict_t<A, B>(nc, splits, tptr, tcell, tblk, P, r, out, y0, z0, st, s)))
  R_(3, 3) R_(6, 3) R_(6, 6) R_(10, 3) R_(10, 6) R_(10, 10) R_(15, 3) R_(15, 6) R_(15, 10) R_(15, 15)
  R_(4, 4) R_(10, 4) R_(20, 4) R_(20, 10) R_(20, 20)
  R_(21, 3) R_(21, 21) R_(28, 3) R_(28, 28) R_(36, 3) R_(36, 36) R_(45, 3) R_(45, 45) R_(55, 3) R_(55, 55)
#undef R_
  return hipErrorInvalidValue;
}

template <int NP, int NQ, typename T>
static void prolong_tt(int32_t N, const int32_t* pptr, const int32_t* pcol, const double* P, const double* z0,
                       const void* zl, const LocalParts* lp, const double* r, double* z, Reduction* red,
                       DevState* st, int n_pq, int n_rr, hipStream_t s) {
  dim3 g(prolong_parts((int64_t)N * NP)), b(256);
  if (lp && lp->small == 3)
    hipLaunchKernelGGL((k_prolong<NP, NQ, T, 4>), g, b, 0, s, N, pptr, pcol, P, z0, nullptr, nullptr, nullptr,
                       nullptr, (const double*)lp->part, r, z, red, st, n_pq, n_rr);
  else if (lp && lp->small == 2)
    hipLaunchKernelGGL((k_prolong<NP, NQ, T, 3>), g, b, 0, s, N, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr, nullptr, r, z, red, st, n_pq, n_rr);
  else if (lp && lp->small)
    hipLaunchKernelGGL((k_prolong<NP, NQ, T, 2>), g, b, 0, s, N, pptr, pcol, P, z0, nullptr, lp->cell_sub, lp->subs,
                       (const T*)lp->part, nullptr, r, z, red, st, n_pq, n_rr);
  else if (lp)
    hipLaunchKernelGGL((k_prolong<NP, NQ, T, 1>), g, b, 0, s, N, pptr, pcol, P, z0, nullptr, lp->cell_sub, lp->subs,
                       (const T*)lp->part, nullptr, r, z, red, st, n_pq, n_rr);
  else
    hipLaunchKernelGGL((k_prolong<NP, NQ, T, 0>), g, b, 0, s, N, pptr, pcol, P, z0, (const T*)zl, nullptr, nullptr,
                       nullptr, nullptr, r, z, red, st, n_pq, n_rr);
}

template <int NP, int NQ>
static void prolong_t(int32_t N, const int32_t* pptr, const int32_t* pcol, const double* P, const double* z0,
                      const void* zl, const LocalParts* lp, int f32, const double* r, double* z, Reduction* red,
                      DevState* st, int n_pq, int n_rr, hipStream_t s) {
  if (f32)
    prolong_tt<NP, NQ, float>(N, pptr, pcol, P, z0, zl, lp, r, z, red, st, n_pq, n_rr, s);
  else
    prolong_tt<NP, NQ, double>(N, pptr, pcol, P, z0, zl, lp, r, z, red, st, n_pq, n_rr, s);
}

hipError_t launch_prolong(int np, int nq, int32_t N, const int32_t* pptr, const int32_t* pcol, const double* P,
                          const double* z0, const void* zl, const LocalParts* lp, int f32, const double* r, double* z,
                          Reduction* red, DevState* st, int n_pq, int n_rr, hipStream_t s) {
  if (!pptr) nq = (np == 4 || np == 20) ? 4 : 3;  // no coarse level: any instantiation, the loop is skipped
  if (n_pq > 0 && (!red || !st)) return hipErrorInvalidValue;
#define P_(A, B) \
  ASDG_PQ_SWITCH(A, B, (prolong_t<A, B>(N, pptr, pcol, P, z0, zl, lp, f32, r, z, red, st, n_pq, n_rr, s)))
  P_(3, 3) P_(6, 3) P_(6, 6) P_(10, 3) P_(10, 6) P_(10, 10) P_(15, 3) P_(15, 6) P_(15, 10) P_(15, 15)
  P_(4, 4) P_(10, 4) P_(20, 4) P_(20, 10) P_(20, 20)
  P_(21, 3) P_(21, 21) P_(28, 3) P_(28, 28) P_(36, 3) P_(36, 36) P_(45, 3) P_(45, 45) P_(55, 3) P_(55, 55)
#undef P_
  return hipErrorInvalidValue;
}

hipError_t launch_update_p(int64_t n, DevState* st, const Reduction* red, int n_rz, double* rz2, double* beta_hist,
                           const double* z, double* p, int init, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p, dim3(vec_parts(n)), dim3(256), 0, s, n, st, red, n_rz, rz2, beta_hist, z, p, init);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* dst, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 4096)), dim3(256), 0, s, dst, n, v);
  return hipGetLastError();
}

hipError_t launch_reset_queues(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

}  // namespace asdg
