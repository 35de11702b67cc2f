// Local matrices A_i = R_i A R_i^T (principal submatrices, Sec. 3) in
// tile-packed form and their batched Cholesky factorisation in one
// persistent launch.
//
// Left-looking tile algorithm. Task (i, j, b), b >= j, owns tile (b, j) of
// subdomain i:
//   S = A_bj - sum_{k<j} L_bk L_jk^T                      (MFMA)
//   b == j: L_jj = chol(S) in LDS, store inv(L_jj) in the diagonal slot
//   b >  j: L_bj = S inv(L_jj)^T                           (MFMA)
// and raises the tile's flag. Tasks are dequeued from an atomic counter in
// a host order where every dependency precedes its consumer (the host
// sorts them by their longest path to the end of the factorisation); a
// task waits (bounded) only on flags of tasks already dequeued by running
// work-groups. Producers write tiles with device-coherent stores and raise
// the flag only after those stores have completed; consumers read tiles
// produced in the same launch with device-coherent loads, so no cache
// write-back or invalidation is needed. The operands of update k + 1 are
// loaded into registers while the MFMA work of update k runs.
//
// MFMA tiles: tile edge TB = 64 (four waves per work-group) or 32 (one
// wave); each wave owns a 32x32 quadrant. FP32: v_mfma_f32_32x32x2f32; FP64:
// 2x2 v_mfma_f64_16x16x4f64. Both edges run the same algorithm; a smaller
// edge pads less of each subdomain's ragged last tile row.
#include "kern_mfma.h"

namespace asdg {

namespace {

using namespace mfma;

// One task (b, j) of subdomain `sub` (tiles at `base`, flags at `fl`).
// OWN = false: the tile-task schedule, where the tiles it reads were written
// by other work-groups of the launch (flag waits, device-coherent loads and
// stores, the tile's flag raised at the end). OWN = true: the subdomain
// schedule, where one work-group runs all tasks of its subdomain in column
// order, so every tile it reads it wrote itself earlier (plain loads and
// stores, ordered by the barrier that ends each task). The arithmetic is the
// same in both.
template <typename T, int TB, bool OWN>
__device__ __forceinline__ void chol_tile(int sub, int j, int b, T* base, int32_t* fl, DevState* st, T* As, T* Bs,
                                          int& s_fail) {
  using SH = Shape<TB>;
  constexpr size_t TT = (size_t)TB * TB;
  constexpr int LD = SH::LD, NT = SH::THREADS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R0 = SH::r0(wave), C0 = SH::c0(wave);
  T* Cg = base + (size_t)(b * (b + 1) / 2 + j) * TT;
  const int rb = b * (b + 1) / 2, rj = j * (j + 1) / 2;  // first tiles of block rows b and j

  Quad<T> acc;
#pragma unroll
  for (int e = 0; e < 16; ++e)
    acc.set(e, Cg[(R0 + Quad<T>::row(e, lane)) * TB + C0 + Quad<T>::col(e, lane)]);

  TileRegs<T, TB> ga, gb;
  if (j > 0) {
    if (OWN) {
      ga.load(base + (size_t)rb * TT);
      gb.load(base + (size_t)rj * TT);
    } else {
      wait_flags(fl + rb, fl + rj, st);
      ga.load_coherent(base + (size_t)rb * TT);
      gb.load_coherent(base + (size_t)rj * TT);
    }
  }
  for (int k = 0; k < j; ++k) {
    ga.put(As);
    gb.put(Bs);
    // the barrier (of the wait) also makes the tiles just written visible to all waves
    if (k + 1 < j) {
      if (OWN) {
        __syncthreads();
        ga.load(base + (size_t)(rb + k + 1) * TT);
        gb.load(base + (size_t)(rj + k + 1) * TT);
      } else {
        wait_flags(fl + rb + k + 1, fl + rj + k + 1, st);
        ga.load_coherent(base + (size_t)(rb + k + 1) * TT);
        gb.load_coherent(base + (size_t)(rj + k + 1) * TT);
      }
    } else {
      __syncthreads();
    }
    acc.template mma<TB>(As, Bs, R0, C0, lane, T(-1));
    __syncthreads();
  }

  if (b == j) {
    // S -> LDS, unblocked Cholesky of the lower triangle
#pragma unroll
    for (int e = 0; e < 16; ++e) As[(R0 + Quad<T>::row(e, lane)) * LD + C0 + Quad<T>::col(e, lane)] = acc.get(e);
    if (tid == 0) s_fail = 0;
    __syncthreads();
    for (int kk = 0; kk < TB; ++kk) {
      if (tid == 0) {
        T d = As[kk * LD + kk];
        if (!(d > T(0))) {
          s_fail = 1;
          d = T(1);
        }
        As[kk * LD + kk] = sqrt(d);
      }
      __syncthreads();
      if (tid > kk && tid < TB) As[tid * LD + kk] /= As[kk * LD + kk];
      __syncthreads();
      // trailing update of the lower triangle: thread (ii, jj) pairs with jj <= ii
      const int m = TB - kk - 1;
      for (int e = tid; e < m * m; e += NT) {
        const int ii = kk + 1 + e / m, jj = kk + 1 + e % m;
        if (jj <= ii) As[ii * LD + jj] -= As[ii * LD + kk] * As[jj * LD + kk];
      }
      __syncthreads();
    }
    if (s_fail && tid == 0) atomicMin(&st->chol_fail, sub);
    // inverse of the lower-triangular L_jj, one column per thread
    if (tid < TB) {
      const int c = tid;
      for (int ii = 0; ii < TB; ++ii) {
        T v;
        if (ii < c) {
          v = T(0);
        } else if (ii == c) {
          v = T(1) / As[c * LD + c];
        } else {
          T s = T(0);
          for (int m2 = c; m2 < ii; ++m2) s += As[ii * LD + m2] * Bs[m2 * LD + c];
          v = -s / As[ii * LD + ii];
        }
        Bs[ii * LD + c] = v;
      }
    }
    __syncthreads();
    for (int e = tid; e < TB * TB; e += NT) {
      if (OWN)
        Cg[e] = Bs[(e / TB) * LD + (e % TB)];
      else
        store_agent(Cg + e, Bs[(e / TB) * LD + (e % TB)]);
    }
  } else {
    // L_bj = S inv(L_jj)^T
    if (OWN) {
      gb.load(base + (size_t)(rj + j) * TT);
    } else {
      wait_flag(fl + rj + j, st);
      gb.load_coherent(base + (size_t)(rj + j) * TT);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) As[(R0 + Quad<T>::row(e, lane)) * LD + C0 + Quad<T>::col(e, lane)] = acc.get(e);
    gb.put(Bs);
    __syncthreads();
    acc.zero();
    acc.template mma<TB>(As, Bs, R0, C0, lane, T(1));
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      T* o = Cg + (R0 + Quad<T>::row(e, lane)) * TB + C0 + Quad<T>::col(e, lane);
      if (OWN)
        *o = acc.get(e);
      else
        store_agent(o, acc.get(e));
    }
  }
  if (!OWN) {
    wait_own_stores();
    __syncthreads();
    if (tid == 0) store_agent(fl + rb + j, 1);
  }
  __syncthreads();
}

// Tile-task schedule: one task per tile of every subdomain, from a queue
// ordered by longest remaining path (see the file comment).
template <typename T, int TB>
__global__ __launch_bounds__(Shape<TB>::THREADS, 2) void k_cholesky(int32_t n_tasks, const int4* __restrict__ tasks,
                                                                  const SubDesc* __restrict__ subs, T* tiles,
                                                                  int32_t* flags, DevState* st, int32_t* queue) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);
  T* Bs = As + TB * Shape<TB>::LD;
  __shared__ int s_task;
  __shared__ int s_fail;
  constexpr size_t TT = (size_t)TB * TB;
  const int tid = threadIdx.x;
  for (;;) {
    // after a failed wait every work-group stops taking tasks
    if (tid == 0) s_task = load_agent(&st->abort) ? n_tasks : atomicAdd(queue, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= n_tasks) break;
    const int4 td = tasks[t];  // x: subdomain, y: column j, z: row b
    const SubDesc sd = subs[td.x];
    chol_tile<T, TB, false>(td.x, td.y, td.z, tiles + (size_t)sd.tile0 * TT, flags + sd.tile0, st, As, Bs, s_fail);
  }
}

// Subdomain schedule: one work-group factorises a whole subdomain, column by
// column (tasks (j, j), (j, j+1), ..., (j, nb-1), then column j + 1); the
// subdomains come from a queue ordered largest first. No flags and no waits:
// for many subdomains of similar size (as many as the work-groups that fit
// on the device, or more), every work-group stays busy on its own data.
template <typename T, int TB>
__global__ __launch_bounds__(Shape<TB>::THREADS, 2) void k_cholesky_subs(int32_t n_tasks,
                                                                       const int4* __restrict__ tasks,
                                                                       const SubDesc* __restrict__ subs, T* tiles,
                                                                       DevState* st, int32_t* queue) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* As = reinterpret_cast<T*>(smem_raw);
  T* Bs = As + TB * Shape<TB>::LD;
  __shared__ int s_task;
  __shared__ int s_fail;
  constexpr size_t TT = (size_t)TB * TB;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) s_task = atomicAdd(queue, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= n_tasks) break;
    const int i = tasks[t].x;
    const SubDesc sd = subs[i];
    T* base = tiles + (size_t)sd.tile0 * TT;
    for (int j = 0; j < sd.nb; ++j)
      for (int b = j; b < sd.nb; ++b) chol_tile<T, TB, true>(i, j, b, base, nullptr, st, As, Bs, s_fail);
  }
}

// Tile-packed A_i from the BSR operator (identity on the padding).
template <typename T, int TB>
__global__ __launch_bounds__(256) void k_gather(int np, int64_t n_elems, const int4* __restrict__ meta,
                                                const SubDesc* __restrict__ subs, const int32_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ col, const double* __restrict__ blocks,
                                                T* __restrict__ tiles) {
  constexpr int64_t TT = (int64_t)TB * TB;
  for (int64_t E = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; E < n_elems; E += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = E / TT;
    const int e = (int)(E - t * TT);
    const int4 m = meta[t];  // x: subdomain, y: b, z: j
    const SubDesc sd = subs[m.x];
    const int gr = m.y * TB + e / TB, gc = m.z * TB + e % TB;
    double v;
    if (gr >= sd.n || gc >= sd.n) {
      v = (gr == gc) ? 1.0 : 0.0;
    } else {
      const int R = sd.dof0 + gr, C = sd.dof0 + gc;
      const int cr = R / np, a = R - cr * np, cc = C / np, bb = C - cc * np;
      v = 0.0;
      for (int k = row_ptr[cr]; k < row_ptr[cr + 1]; ++k) {
        if (col[k] == cc) {
          v = blocks[(size_t)k * np * np + a * np + bb];  // row-major blocks
          break;
        }
      }
    }
    tiles[E] = (T)v;
  }
}

template <typename T, int TB>
hipError_t cholesky_tb(int per_sub, int32_t n_tasks, const int4* tasks, const SubDesc* subs, void* tiles,
                       int32_t* flags, DevState* st, int32_t* queue, int grid, hipStream_t s) {
  const size_t sh = 2 * TB * Shape<TB>::LD * sizeof(T);
  // set once per process and instantiation (function-local statics are
  // initialised once even when several host threads factorise at once)
  static const hipError_t attr =
      hipFuncSetAttribute((const void*)k_cholesky<T, TB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  static const hipError_t attr_s =
      hipFuncSetAttribute((const void*)k_cholesky_subs<T, TB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (attr != hipSuccess) return attr;
  if (attr_s != hipSuccess) return attr_s;
  if (per_sub)
    hipLaunchKernelGGL((k_cholesky_subs<T, TB>), dim3(grid), dim3(Shape<TB>::THREADS), sh, s, n_tasks, tasks, subs,
                       (T*)tiles, st, queue);
  else
    hipLaunchKernelGGL((k_cholesky<T, TB>), dim3(grid), dim3(Shape<TB>::THREADS), sh, s, n_tasks, tasks, subs,
                       (T*)tiles, flags, st, queue);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gather_tiles(int np, int tile, int32_t n_tiles, const int4* meta, const SubDesc* subs,
                               const int32_t* row_ptr, const int32_t* col, const double* blocks, void* tiles, int f32,
                               hipStream_t s) {
  if (tile != 32 && tile != 64) return hipErrorInvalidValue;
  const int64_t n = (int64_t)n_tiles * tile * tile;
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
  if (f32) {
    if (tile == 64)
      hipLaunchKernelGGL((k_gather<float, 64>), dim3(grid), dim3(256), 0, s, np, n, meta, subs, row_ptr, col, blocks,
                         (float*)tiles);
    else
      hipLaunchKernelGGL((k_gather<float, 32>), dim3(grid), dim3(256), 0, s, np, n, meta, subs, row_ptr, col, blocks,
                         (float*)tiles);
  } else {
    if (tile == 64)
      hipLaunchKernelGGL((k_gather<double, 64>), dim3(grid), dim3(256), 0, s, np, n, meta, subs, row_ptr, col,
                         blocks, (double*)tiles);
    else
      hipLaunchKernelGGL((k_gather<double, 32>), dim3(grid), dim3(256), 0, s, np, n, meta, subs, row_ptr, col,
                         blocks, (double*)tiles);
  }
  return hipGetLastError();
}

hipError_t launch_cholesky(int f32, int tile, int per_sub, int32_t n_tasks, const int4* tasks, const SubDesc* subs,
                           void* tiles, int32_t* flags, DevState* st, int32_t* queue, int grid, hipStream_t s) {
  if (tile != 32 && tile != 64) return hipErrorInvalidValue;
  if (n_tasks <= 0) return hipSuccess;
  if (f32)
    return tile == 64 ? cholesky_tb<float, 64>(per_sub, n_tasks, tasks, subs, tiles, flags, st, queue, grid, s)
                      : cholesky_tb<float, 32>(per_sub, n_tasks, tasks, subs, tiles, flags, st, queue, grid, s);
  return tile == 64 ? cholesky_tb<double, 64>(per_sub, n_tasks, tasks, subs, tiles, flags, st, queue, grid, s)
                    : cholesky_tb<double, 32>(per_sub, n_tasks, tasks, subs, tiles, flags, st, queue, grid, s);
}

}  // namespace asdg
