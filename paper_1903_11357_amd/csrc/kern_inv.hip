// Formation of the explicit local inverses S_i = A_i^{-1} = L_i^{-T} L_i^{-1}
// (the exact local solvers of Sec. 3, applied by kern_symv.hip), the whole
// inverses of small subdomains, and the dense coarse inverse.
//
// Setup, after the tile Cholesky (diagonal tiles hold D_b = inv(L_bb)):
//   X = L^{-1}:  X_bb = D_b,  X_bj = -D_b sum_{k=j}^{b-1} L_bk X_kj  (b > j)
//     tasks ordered by their longest path to the end, one persistent
//     launch, per-tile flags (MFMA);
//   S = X^T X:   S_bj = sum_{k=b}^{nb-1} X_kb^T X_kj  (b >= j), independent
//     tiles (MFMA), written over the factor tiles.
#include "kern_mfma.h"

namespace asdg {

namespace {

using namespace mfma;

constexpr size_t TT = (size_t)TILE * TILE;

// ---------------------------------------------------------------- X = L^{-1}
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 2) void k_inv_lower(int32_t n_tasks, const int4* __restrict__ tasks,
                                                   const SubDesc* __restrict__ subs, const T* __restrict__ L,
                                                   T* X, int32_t* flags, DevState* st, int32_t* queue) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);
  T* Bs = As + TILE * LDA;
  __shared__ int s_task;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R0 = 32 * (wave >> 1), C0 = 32 * (wave & 1);
  for (;;) {
    if (tid == 0) s_task = load_agent(&st->abort) ? n_tasks : atomicAdd(queue, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= n_tasks) break;
    const int4 td = tasks[t];  // x: subdomain, y: column j, z: row b
    const SubDesc sd = subs[td.x];
    const int j = td.y, b = td.z;
    const T* Lb = L + (size_t)sd.tile0 * TT;
    T* Xb = X + (size_t)sd.tile0 * TT;
    int32_t* fl = flags + sd.tile0;
    T* out = Xb + (size_t)(b * (b + 1) / 2 + j) * TT;
    if (b == j) {
      // X_bb = D_b
      TileRegs<T> d;
      d.load(Lb + (size_t)(b * (b + 1) / 2 + b) * TT);
      d.store_coherent(out);
    } else {
      Quad<T> acc;
      acc.zero();
      // operands of step k + 1 are loaded into registers during the MFMA work of step k
      TileRegs<T> gl, gx;
      wait_flag(fl + j * (j + 1) / 2 + j, st);
      gl.load(Lb + (size_t)(b * (b + 1) / 2 + j) * TT);
      gx.load_coherent(Xb + (size_t)(j * (j + 1) / 2 + j) * TT);
      for (int k = j; k < b; ++k) {
        gl.put(As);    // L_bk
        gx.put_t(Bs);  // Bs[c][m] = X_kj[m][c]
        // the barrier of the wait also makes the tiles just written visible to all waves
        if (k + 1 < b) {
          wait_flag(fl + (k + 1) * (k + 2) / 2 + j, st);
          gl.load(Lb + (size_t)(b * (b + 1) / 2 + k + 1) * TT);
          gx.load_coherent(Xb + (size_t)((k + 1) * (k + 2) / 2 + j) * TT);
        } else {
          __syncthreads();
          gl.load(Lb + (size_t)(b * (b + 1) / 2 + b) * TT);  // D_b, for the last product
        }
        acc.mma(As, Bs, R0, C0, lane, T(1));
        __syncthreads();
      }
      // X_bj = -D_b acc: Bs[c][m] = acc[m][c], As = D_b
#pragma unroll
      for (int e = 0; e < 16; ++e) Bs[(C0 + Quad<T>::col(e, lane)) * LDA + R0 + Quad<T>::row(e, lane)] = acc.get(e);
      gl.put(As);
      __syncthreads();
      acc.zero();
      acc.mma(As, Bs, R0, C0, lane, T(-1));
#pragma unroll
      for (int e = 0; e < 16; ++e)
        store_agent(out + (R0 + Quad<T>::row(e, lane)) * TILE + C0 + Quad<T>::col(e, lane), acc.get(e));
    }
    wait_own_stores();
    __syncthreads();
    if (tid == 0) store_agent(fl + b * (b + 1) / 2 + j, 1);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- X = L^{-1}, column tasks
// The same products in the same order as k_inv_lower, scheduled by block
// column: task (i, j) computes column j of X_i top to bottom in one
// work-group, X_jj = D_j, then for b = j+1 .. nb-1
//   acc = sum_{k=j}^{b-1} L_bk X_kj,   X_bj = -D_b acc.
// Every X_kj a task reads was written by the same work-group earlier in the
// task (visible after the barrier that ends its row), so there are no flags,
// no waits and no device-coherent loads; columns are independent and queued
// longest first. The operands of the next product (and D_b) are loaded into
// registers during the current MFMA work, across row boundaries.
// Results are bitwise those of k_inv_lower.
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 3 : 2) void k_inv_cols(int32_t n_tasks, const int4* __restrict__ tasks,
                                                  const SubDesc* __restrict__ subs, const T* __restrict__ L, T* X,
                                                  DevState* st, int32_t* queue) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);
  T* Bs = As + TILE * LDA;
  __shared__ int s_task;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R0 = 32 * (wave >> 1), C0 = 32 * (wave & 1);
  for (;;) {
    if (tid == 0) s_task = atomicAdd(queue, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= n_tasks) break;
    const int4 td = tasks[t];  // x: subdomain, y: column j
    const SubDesc sd = subs[td.x];
    const int j = td.y, nb = sd.nb;
    const T* Lb = L + (size_t)sd.tile0 * TT;
    T* Xb = X + (size_t)sd.tile0 * TT;
    const T* Dj = Lb + (size_t)(j * (j + 1) / 2 + j) * TT;
    TileRegs<T> gl, gx;
    gx.load(Dj);  // X_jj = D_j: the operand of every row's first product
    gx.store(Xb + (size_t)(j * (j + 1) / 2 + j) * TT);
    if (j + 1 >= nb) {
      __syncthreads();
      continue;
    }
    gl.load(Lb + (size_t)((j + 1) * (j + 2) / 2 + j) * TT);
    for (int b = j + 1; b < nb; ++b) {
      const size_t rb = (size_t)b * (b + 1) / 2;
      Quad<T> acc;
      acc.zero();
      for (int k = j; k < b; ++k) {
        gl.put(As);    // L_bk
        gx.put_t(Bs);  // Bs[c][m] = X_kj[m][c]
        __syncthreads();
        // operands of the next product (b, k + 1); after the row's last one,
        // D_b for the row end and the next row's first L tile (b + 1, j)
        if (k + 1 < b) {
          gl.load(Lb + (rb + k + 1) * TT);
          gx.load(Xb + (size_t)((k + 1) * (k + 2) / 2 + j) * TT);
        } else {
          if (b + 1 < nb) gl.load(Lb + ((size_t)(b + 1) * (b + 2) / 2 + j) * TT);
          gx.load(Lb + (rb + b) * TT);
        }
        acc.mma(As, Bs, R0, C0, lane, T(1));
        __syncthreads();
      }
      // X_bj = -D_b acc: Bs[c][m] = acc[m][c], As = D_b
#pragma unroll
      for (int e = 0; e < 16; ++e) Bs[(C0 + Quad<T>::col(e, lane)) * LDA + R0 + Quad<T>::row(e, lane)] = acc.get(e);
      gx.put(As);
      __syncthreads();
      if (b + 1 < nb) gx.load(Dj);  // the next row's first X operand
      acc.zero();
      acc.mma(As, Bs, R0, C0, lane, T(-1));
      T* out = Xb + (rb + j) * TT;
#pragma unroll
      for (int e = 0; e < 16; ++e) out[(R0 + Quad<T>::row(e, lane)) * TILE + C0 + Quad<T>::col(e, lane)] = acc.get(e);
      // the row's tile is complete and visible to the whole work-group
      // before a later row loads it (and before As/Bs are overwritten)
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- S = X^T X
template <typename T>
__global__ __launch_bounds__(256) void k_inv_gram(int32_t n_tiles, const int4* __restrict__ meta,
                                                  const SubDesc* __restrict__ subs, const T* __restrict__ X,
                                                  T* __restrict__ S) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);
  T* Bs = As + TILE * LDA;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R0 = 32 * (wave >> 1), C0 = 32 * (wave & 1);
  for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int4 m = meta[t];  // x: subdomain, y: row b, z: column j
    const SubDesc sd = subs[m.x];
    const int b = m.y, j = m.z;
    const T* Xb = X + (size_t)sd.tile0 * TT;
    Quad<T> acc;
    acc.zero();
    TileRegs<T> ga, gb;
    ga.load(Xb + (size_t)(b * (b + 1) / 2 + b) * TT);
    gb.load(Xb + (size_t)(b * (b + 1) / 2 + j) * TT);
    for (int k = b; k < sd.nb; ++k) {
      ga.put_t(As);  // As[r][m] = X_kb[m][r]
      gb.put_t(Bs);  // Bs[c][m] = X_kj[m][c]
      __syncthreads();
      if (k + 1 < sd.nb) {
        ga.load(Xb + (size_t)((k + 1) * (k + 2) / 2 + b) * TT);
        gb.load(Xb + (size_t)((k + 1) * (k + 2) / 2 + j) * TT);
      }
      acc.mma(As, Bs, R0, C0, lane, T(1));
      __syncthreads();
    }
    T* out = S + (size_t)t * TT;
#pragma unroll
    for (int e = 0; e < 16; ++e) out[(R0 + Quad<T>::row(e, lane)) * TILE + C0 + Quad<T>::col(e, lane)] = acc.get(e);
  }
}

// ---------------------------------------------------------------- small subdomains
// Subdomains of at most 64 DoFs (the case of one element per subdomain):
// one wave per subdomain gathers A_i from the block rows into LDS (FP64),
// factors it A_i = L L^T, forms X = L^{-1} row by row (lane = column) and
// writes A_i^{-1} = X^T X whole (n_i x n_i row-major, at word offset
// sd.tile0). Entry (i, j) and (j, i) add the same products in the same
// order, so the stored inverse is exactly symmetric. A non-positive pivot
// reports the subdomain through st->chol_fail (smallest index wins).
template <typename T>
__global__ __launch_bounds__(64) void k_small_inverse(int32_t n_sub, int np, int ld, const SubDesc* __restrict__ subs,
                                                      const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ blocks, T* __restrict__ S,
                                                      DevState* st) {
  extern __shared__ double sm[];
  const int isub = blockIdx.x, lane = threadIdx.x;
  const SubDesc sd = subs[isub];
  const int n = sd.n, c0 = sd.dof0 / np, nc = n / np;
  double* A = sm;           // [n][ld]
  double* X = sm + n * ld;  // [n][ld]
  for (int e = lane; e < n * ld; e += 64) A[e] = 0.0;
  wave_sync();
  for (int cc = 0; cc < nc; ++cc) {
    const int c = c0 + cc;
    for (int k = row_ptr[c]; k < row_ptr[c + 1]; ++k) {
      const int cj = col[k] - c0;
      if (cj < 0 || cj >= nc) continue;  // coupling to another subdomain
      for (int e = lane; e < np * np; e += 64) {
        const int a = e / np, b = e - a * np;
        A[(cc * np + a) * ld + cj * np + b] = blocks[(size_t)k * np * np + e];
      }
    }
  }
  wave_sync();
  for (int k = 0; k < n; ++k) {
    const double d = A[k * ld + k];
    if (!(d > 0.0)) {
      if (lane == 0) atomicMin(&st->chol_fail, isub);
      return;  // d is the same for every lane: the whole wave leaves
    }
    const double lkk = sqrt(d);
    wave_sync();
    if (lane == k) A[k * ld + k] = lkk;
    else if (lane > k && lane < n) A[lane * ld + k] /= lkk;
    wave_sync();
    if (lane > k && lane < n) {
      const double lik = A[lane * ld + k];
      for (int j = k + 1; j <= lane; ++j) A[lane * ld + j] -= lik * A[j * ld + k];
    }
    wave_sync();
  }
  // X = L^{-1}: lane j owns column j; X_ij = (delta_ij - sum_{k=j}^{i-1} L_ik X_kj) / L_ii
  for (int i = 0; i < n; ++i) {
    if (lane <= i) {
      double acc = lane == i ? 1.0 : 0.0;
      for (int k = lane; k < i; ++k) acc -= A[i * ld + k] * X[k * ld + lane];
      X[i * ld + lane] = acc / A[i * ld + i];
    }
  }
  wave_sync();
  if (lane < n) {
    T* Si = S + sd.tile0 + (size_t)lane * n;
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int k = max(lane, j); k < n; ++k) acc += X[k * ld + lane] * X[k * ld + j];
      Si[j] = (T)acc;
    }
  }
}

// ---------------------------------------------------------------- coarse
// Dense symmetric A_0^{-1} (row-major n0 x n0) from its packed lower tiles
// (single "subdomain" at tile 0; diagonal tiles stored whole).
__global__ __launch_bounds__(256) void k_expand_sym(int32_t n0, const double* __restrict__ S,
                                                    double* __restrict__ D) {
  const int64_t nn = (int64_t)n0 * n0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n0), j = (int)(e - (int64_t)i * n0);
    const int bi = i / TILE, bj = j / TILE, ri = i - bi * TILE, rj = j - bj * TILE;
    D[e] = bi >= bj ? S[(size_t)(bi * (bi + 1) / 2 + bj) * TT + ri * TILE + rj]
                    : S[(size_t)(bj * (bj + 1) / 2 + bi) * TT + rj * TILE + ri];
  }
}

// y = D x for a dense row-major n x n matrix, x given as `splits` partial
// vectors (x = sum_s xp[s n + i], added in order of s into LDS by every
// work-group). One wave per row; each lane strides the row by 64 (coalesced
// 512-byte loads, eight in flight); fixed-order wave sum.
__global__ __launch_bounds__(256) void k_dense_mv(int32_t n, int splits, const double* __restrict__ D,
                                                  const double* __restrict__ xp, double* __restrict__ y,
                                                  const DevState* st) {
  extern __shared__ double xs[];
  if (st && st->done) return;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  // the row's first KD entries per lane are loaded before the prologue
  constexpr int KD = 8;
  const double* Dr = D + (size_t)(row < n ? row : 0) * n;
  double dv[KD];
#pragma unroll
  for (int u = 0; u < KD; ++u) {
    const int j = lane + 64 * u;
    dv[u] = j < n ? Dr[j] : 0.0;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = 0.0;
    for (int sp = 0; sp < splits; ++sp) v += xp[(size_t)sp * n + i];
    xs[i] = v;
  }
  __syncthreads();
  if (row >= n) return;
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < KD; ++u) {
    const int j = lane + 64 * u;
    if (j < n) acc += dv[u] * xs[j];
  }
#pragma unroll 8
  for (int j = lane + 64 * KD; j < n; j += 64) acc += Dr[j] * xs[j];
  acc = warp_sum(acc);
  if (lane == 0) y[row] = acc;
}

template <typename K>
hipError_t big_lds(K kernel, size_t sh) {
  if (sh <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
}

}  // namespace

hipError_t launch_inverse(int f32, int cols, int32_t n_tasks, const int4* tasks, int32_t n_tiles, const int4* meta,
                          const SubDesc* subs, void* L, void* X, int32_t* flags, DevState* st, int32_t* queue,
                          int grid_lower, int grid_gram, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  hipError_t e;
  if (f32) {
    const size_t sh = 2 * TILE * LDA * sizeof(float);
    if (cols)
      hipLaunchKernelGGL(k_inv_cols<float>, dim3(grid_lower), dim3(256), sh, s, n_tasks, tasks, subs, (const float*)L,
                         (float*)X, st, queue);
    else
      hipLaunchKernelGGL(k_inv_lower<float>, dim3(grid_lower), dim3(256), sh, s, n_tasks, tasks, subs,
                         (const float*)L, (float*)X, flags, st, queue);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_inv_gram<float>, dim3(grid_gram), dim3(256), sh, s, n_tiles, meta, subs, (const float*)X,
                       (float*)L);
  } else {
    const size_t sh = 2 * TILE * LDA * sizeof(double);
    if ((e = big_lds(k_inv_lower<double>, sh)) != hipSuccess) return e;
    if ((e = big_lds(k_inv_cols<double>, sh)) != hipSuccess) return e;
    if ((e = big_lds(k_inv_gram<double>, sh)) != hipSuccess) return e;
    if (cols)
      hipLaunchKernelGGL(k_inv_cols<double>, dim3(grid_lower), dim3(256), sh, s, n_tasks, tasks, subs,
                         (const double*)L, (double*)X, st, queue);
    else
      hipLaunchKernelGGL(k_inv_lower<double>, dim3(grid_lower), dim3(256), sh, s, n_tasks, tasks, subs,
                         (const double*)L, (double*)X, flags, st, queue);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_inv_gram<double>, dim3(grid_gram), dim3(256), sh, s, n_tiles, meta, subs,
                       (const double*)X, (double*)L);
  }
  return hipGetLastError();
}

hipError_t launch_small_inverse(int f32, int32_t n_sub, int np, int max_n, const SubDesc* subs, const int32_t* row_ptr,
                                const int32_t* col, const double* blocks, void* S, DevState* st, hipStream_t s) {
  if (n_sub <= 0) return hipSuccess;
  if (max_n < 1 || max_n > TILE) return hipErrorInvalidValue;
  const int ld = max_n + 1;
  const size_t sh = 2 * (size_t)max_n * ld * sizeof(double);
  hipError_t e;
  if (f32) {
    if ((e = big_lds(k_small_inverse<float>, sh)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_small_inverse<float>, dim3(n_sub), dim3(64), sh, s, n_sub, np, ld, subs, row_ptr, col, blocks,
                       (float*)S, st);
  } else {
    if ((e = big_lds(k_small_inverse<double>, sh)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_small_inverse<double>, dim3(n_sub), dim3(64), sh, s, n_sub, np, ld, subs, row_ptr, col,
                       blocks, (double*)S, st);
  }
  return hipGetLastError();
}

hipError_t launch_expand_sym(int32_t n0, const double* S, double* D, hipStream_t s) {
  if (n0 <= 0) return hipSuccess;
  const int64_t nn = (int64_t)n0 * n0;
  const int g = (int)std::max<int64_t>(1, std::min<int64_t>((nn + 255) / 256, 8192));
  hipLaunchKernelGGL(k_expand_sym, dim3(g), dim3(256), 0, s, n0, S, D);
  return hipGetLastError();
}

hipError_t launch_dense_mv(int32_t n, int splits, const double* D, const double* xp, double* y, const DevState* st,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (splits < 1 || (size_t)n * 8 > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dense_mv, dim3((n + 3) / 4), dim3(256), (size_t)n * 8, s, n, splits, D, xp, y, st);
  return hipGetLastError();
}

}  // namespace asdg
