// Operator apply, PCG vector updates, coarse restriction/prolongation.
//
// Block-sparse SIPG operator (Sec. 2, eq. (Ah)): one wavefront per block row;
// the row's blocks are read as one dense n_p x (nnz_row * n_p) panel stored
// column-major, so a load instruction of the wave covers 64/n_p consecutive
// columns = one contiguous run of memory. Partial sums of the 64/n_p column
// groups are combined with cross-lane reads.
//
// PCG (Sec. 7): every reduction is two-stage and deterministic (fixed
// per-work-group order, then a fixed-order sum of the NPART partials that
// each consumer work-group recomputes redundantly), so no floating-point
// atomics are used and repeated solves are bitwise identical.
#include "kern_common.h"

namespace asdg {

namespace {

template <int NP>
__global__ __launch_bounds__(256) void k_spmv(int32_t N, const int32_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col,
                                              const double* __restrict__ blocks,
                                              const double* __restrict__ p, double* __restrict__ q,
                                              double* __restrict__ part, const DevState* st) {
  __shared__ double scratch[4];
  if (st && st->done) return;
  constexpr int G = 64 / NP;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane / NP, rr = lane - g * NP;
  const bool active = g < G;
  double dot = 0.0;
  const int total_waves = gridDim.x * 4;
  for (int row = blockIdx.x * 4 + w; row < N; row += total_waves) {
    const int k0 = row_ptr[row], k1 = row_ptr[row + 1];
    const int ncol = (k1 - k0) * NP;
    const double* Bp = blocks + (size_t)k0 * NP * NP;
    double acc = 0.0;
    if (active) {
      for (int c = g; c < ncol; c += G) {
        const int blk = c / NP, cc = c - blk * NP;
        acc += Bp[(size_t)c * NP + rr] * p[(size_t)col[k0 + blk] * NP + cc];
      }
    }
    double s = acc;
#pragma unroll
    for (int gg = 1; gg < G; ++gg) s += __shfl(acc, gg * NP + rr, 64);
    if (g == 0) {
      q[(size_t)row * NP + rr] = s;
      dot += p[(size_t)row * NP + rr] * s;
    }
  }
  dot = block_sum(dot, scratch);
  if (part && threadIdx.x == 0) part[blockIdx.x] = dot;
}

template <typename T>
__global__ __launch_bounds__(256) void k_permute_in(int np, int32_t N, const int32_t* __restrict__ perm,
                                                    const double* __restrict__ src, double* __restrict__ r,
                                                    double* __restrict__ x, T* __restrict__ yl,
                                                    T* __restrict__ zl, double* __restrict__ part) {
  __shared__ double scratch[4];
  const int64_t n = (int64_t)N * np;
  double acc = 0.0;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = d / np;
    const int a = (int)(d - cell * np);
    const double v = src[(int64_t)perm[cell] * np + a];
    r[d] = v;
    if (x) x[d] = 0.0;
    yl[d] = sentinel<T>();
    zl[d] = sentinel<T>();
    acc += v * v;
  }
  acc = block_sum(acc, scratch);
  if (part && threadIdx.x == 0) part[blockIdx.x] = acc;
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

__global__ __launch_bounds__(256) void k_init_check(DevState* st, const double* __restrict__ part_bb,
                                                    double rtol, int max_iter) {
  __shared__ double scratch[4];
  const double bb = reduce_partials(part_bb, scratch);
  if (threadIdx.x == 0) {
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

template <typename T>
__global__ __launch_bounds__(256) void k_update_xr(int64_t n, DevState* st, const double* __restrict__ part_pq,
                                                   const double* __restrict__ rz2, double* __restrict__ alpha_hist,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   T* __restrict__ yl, T* __restrict__ zl,
                                                   double* __restrict__ part_rr) {
  __shared__ double scratch[4];
  if (st->done) return;
  const double pq = reduce_partials(part_pq, scratch);
  const int it = st->it;
  const double alpha = rz2[it & 1] / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0 && it < HIST) alpha_hist[it] = alpha;
  double acc = 0.0;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    x[d] += alpha * p[d];
    const double rv = r[d] - alpha * q[d];
    r[d] = rv;
    acc += rv * rv;
    yl[d] = sentinel<T>();
    zl[d] = sentinel<T>();
  }
  acc = block_sum(acc, scratch);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_check(DevState* st, const double* __restrict__ part_rr,
                                               const double* __restrict__ part_pq) {
  __shared__ double scratch[4];
  if (st->done) return;
  const double rr = reduce_partials(part_rr, scratch);
  const double pq = reduce_partials(part_pq, scratch);
  if (threadIdx.x == 0) {
    const int it = st->it + 1;
    st->it = it;
    st->rr = rr;
    st->q_local = 0;
    st->q_coarse = 0;
    if (st->abort) {
      st->status = 4;
      st->done = 1;
    } else if (!(pq > 0.0) || !(rr == rr)) {
      st->status = 3;
      st->done = 1;
    } else if (rr <= st->tol2) {
      st->status = 1;
      st->done = 1;
    } else if (it >= st->max_iter) {
      st->status = 2;
      st->done = 1;
    }
  }
}

// r0 = P_0^T r: one work-group per coarse cell, entries in fixed order.
template <int NP, int NQ>
__global__ __launch_bounds__(256) void k_restrict(const int32_t* __restrict__ tptr, const int32_t* __restrict__ tcell,
                                                  const int32_t* __restrict__ tblk, const double* __restrict__ P,
                                                  const double* __restrict__ r, double* __restrict__ r0,
                                                  double* __restrict__ y0, double* __restrict__ z0,
                                                  const DevState* st) {
  __shared__ double scratch[4];
  if (st && st->done) return;
  const int J = blockIdx.x;
  double acc[NQ];
#pragma unroll
  for (int c = 0; c < NQ; ++c) acc[c] = 0.0;
  for (int k = tptr[J] + threadIdx.x; k < tptr[J + 1]; k += blockDim.x) {
    const int cell = tcell[k];
    const double* Pb = P + (size_t)tblk[k] * NP * NQ;
    const double* rv = r + (size_t)cell * NP;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      const double v = rv[a];
#pragma unroll
      for (int c = 0; c < NQ; ++c) acc[c] += Pb[a * NQ + c] * v;
    }
  }
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const double s = block_sum(acc[c], scratch);
    if (threadIdx.x == 0) {
      r0[J * NQ + c] = s;
      y0[J * NQ + c] = sentinel_f64();
      z0[J * NQ + c] = sentinel_f64();
    }
  }
}

// z = z_loc + P_0 z0 (coarse part optional), partial sums of r.z.
template <int NP, int NQ, typename T>
__global__ __launch_bounds__(256) void k_prolong(int32_t N, const int32_t* __restrict__ pptr,
                                                 const int32_t* __restrict__ pcol, const double* __restrict__ P,
                                                 const double* __restrict__ z0, const T* __restrict__ zl,
                                                 const double* __restrict__ r, double* __restrict__ z,
                                                 double* __restrict__ part, const DevState* st) {
  __shared__ double scratch[4];
  if (st && st->done) return;
  const int64_t n = (int64_t)N * NP;
  double acc = 0.0;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = d / NP;
    const int a = (int)(d - cell * NP);
    double v = zl ? (double)zl[d] : 0.0;
    if (pptr) {
      for (int e = pptr[cell]; e < pptr[cell + 1]; ++e) {
        const double* Pb = P + (size_t)e * NP * NQ + a * NQ;
        const double* zc = z0 + (size_t)pcol[e] * NQ;
#pragma unroll
        for (int c = 0; c < NQ; ++c) v += Pb[c] * zc[c];
      }
    }
    z[d] = v;
    if (part) acc += r[d] * v;
  }
  if (part) {
    acc = block_sum(acc, scratch);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
  }
}

__global__ __launch_bounds__(256) void k_update_p(int64_t n, DevState* st, const double* __restrict__ part_rz,
                                                  double* __restrict__ rz2, double* __restrict__ beta_hist,
                                                  const double* __restrict__ z, double* __restrict__ p, int init) {
  __shared__ double scratch[4];
  if (st->done) return;
  const double rz_new = reduce_partials(part_rz, scratch);
  if (init) {
    if (blockIdx.x == 0 && threadIdx.x == 0) rz2[0] = rz_new;
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x)
      p[d] = z[d];
    return;
  }
  const int it = st->it;
  const double beta = rz_new / rz2[(it - 1) & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    rz2[it & 1] = rz_new;
    if (it - 1 < HIST) beta_hist[it - 1] = beta;
  }
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x)
    p[d] = z[d] + beta * p[d];
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

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, NPART));
}

}  // namespace

hipError_t launch_spmv(int np, int32_t N, const int32_t* row_ptr, const int32_t* col, const double* blocks,
                       const double* p, double* q, double* part, const DevState* st, hipStream_t s) {
  dim3 g(NPART), b(256);
  switch (np) {
    case 3: hipLaunchKernelGGL(k_spmv<3>, g, b, 0, s, N, row_ptr, col, blocks, p, q, part, st); break;
    case 6: hipLaunchKernelGGL(k_spmv<6>, g, b, 0, s, N, row_ptr, col, blocks, p, q, part, st); break;
    case 10: hipLaunchKernelGGL(k_spmv<10>, g, b, 0, s, N, row_ptr, col, blocks, p, q, part, st); break;
    case 15: hipLaunchKernelGGL(k_spmv<15>, g, b, 0, s, N, row_ptr, col, blocks, p, q, part, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_permute_in(int np, int32_t N, const int32_t* perm, const double* src, double* r, double* x,
                             void* yl, void* zl, int local_f32, double* part_bb, hipStream_t s) {
  dim3 g(NPART), b(256);
  if (local_f32)
    hipLaunchKernelGGL(k_permute_in<float>, g, b, 0, s, np, N, perm, src, r, x, (float*)yl, (float*)zl, part_bb);
  else
    hipLaunchKernelGGL(k_permute_in<double>, g, b, 0, s, np, N, perm, src, r, x, (double*)yl, (double*)zl, part_bb);
  return hipGetLastError();
}

hipError_t launch_unpermute_out(int np, int32_t N, const int32_t* perm, const double* x, double* dst,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute, dim3(grid_for((int64_t)N * np)), dim3(256), 0, s, np, N, perm, x, dst);
  return hipGetLastError();
}

hipError_t launch_init_check(DevState* st, const double* part_bb, double rtol, int max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_init_check, dim3(1), dim3(256), 0, s, st, part_bb, rtol, max_iter);
  return hipGetLastError();
}

hipError_t launch_update_xr(int64_t n, DevState* st, const double* part_pq, const double* rz_hist,
                            double* alpha_hist, const double* p, const double* q, double* x, double* r, void* yl,
                            void* zl, int local_f32, double* part_rr, hipStream_t s) {
  dim3 g(NPART), b(256);
  if (local_f32)
    hipLaunchKernelGGL(k_update_xr<float>, g, b, 0, s, n, st, part_pq, rz_hist, alpha_hist, p, q, x, r,
                       (float*)yl, (float*)zl, part_rr);
  else
    hipLaunchKernelGGL(k_update_xr<double>, g, b, 0, s, n, st, part_pq, rz_hist, alpha_hist, p, q, x, r,
                       (double*)yl, (double*)zl, part_rr);
  return hipGetLastError();
}

hipError_t launch_check(DevState* st, const double* part_rr, const double* part_pq, hipStream_t s) {
  hipLaunchKernelGGL(k_check, dim3(1), dim3(256), 0, s, st, part_rr, part_pq);
  return hipGetLastError();
}

template <int NP, int NQ>
static void restrict_t(int32_t nc, const int32_t* tptr, const int32_t* tcell, const int32_t* tblk, const double* P,
                       const double* r, double* r0, double* y0, double* z0, const DevState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_restrict<NP, NQ>), dim3(nc), dim3(256), 0, s, tptr, tcell, tblk, P, r, r0, y0, z0, st);
}

#define ASDG_PQ_SWITCH(NPV, NQV, CALL) \
  if (np == NPV && nq == NQV) {        \
    CALL;                              \
    return hipGetLastError();          \
  }

hipError_t launch_restrict(int np, int nq, int32_t nc, const int32_t* tptr, const int32_t* tcell, const int32_t* tblk,
                           const double* P, const double* r, double* r0, double* y0, double* z0, const DevState* st,
                           hipStream_t s) {
#define R_(A, B) ASDG_PQ_SWITCH(A, B, (restrict_t<A, B>(nc, tptr, tcell, tblk, P, r, r0, y0, z0, st, s)))
  R_(3, 3) R_(6, 3) R_(6, 6) R_(10, 3) R_(10, 6) R_(10, 10) R_(15, 3) R_(15, 6) R_(15, 10) R_(15, 15)
#undef R_
  return hipErrorInvalidValue;
}

template <int NP, int NQ>
static void prolong_t(int32_t N, const int32_t* pptr, const int32_t* pcol, const double* P, const double* z0,
                      const void* zl, int f32, const double* r, double* z, double* part, const DevState* st,
                      hipStream_t s) {
  dim3 g(NPART), b(256);
  if (f32)
    hipLaunchKernelGGL((k_prolong<NP, NQ, float>), g, b, 0, s, N, pptr, pcol, P, z0, (const float*)zl, r, z, part, st);
  else
    hipLaunchKernelGGL((k_prolong<NP, NQ, double>), g, b, 0, s, N, pptr, pcol, P, z0, (const double*)zl, r, z, part,
                       st);
}

hipError_t launch_prolong(int np, int nq, int32_t N, const int32_t* pptr, const int32_t* pcol, const double* P,
                          const double* z0, const void* zl, int f32, const double* r, double* z, double* part,
                          const DevState* st, hipStream_t s) {
  if (!pptr) nq = 3;  // no coarse level: any instantiation, the loop is skipped
#define P_(A, B) ASDG_PQ_SWITCH(A, B, (prolong_t<A, B>(N, pptr, pcol, P, z0, zl, f32, r, z, part, st, s)))
  P_(3, 3) P_(6, 3) P_(6, 6) P_(10, 3) P_(10, 6) P_(10, 10) P_(15, 3) P_(15, 6) P_(15, 10) P_(15, 15)
#undef P_
  return hipErrorInvalidValue;
}

hipError_t launch_update_p(int64_t n, DevState* st, const double* part_rz, double* rz2, double* beta_hist,
                           const double* z, double* p, int init, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p, dim3(NPART), dim3(256), 0, s, n, st, part_rz, rz2, beta_hist, z, p, init);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* dst, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, dst, n, v);
  return hipGetLastError();
}

hipError_t launch_reset_queues(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

}  // namespace asdg
