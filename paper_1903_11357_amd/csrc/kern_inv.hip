// Explicit local inverses S_i = A_i^{-1} = L_i^{-T} L_i^{-1} and their
// application z_i = S_i r_i (exact local solvers of Sec. 3 applied as one
// packed symmetric matrix-vector product per subdomain).
//
// Setup, after the tile Cholesky (diagonal tiles hold D_b = inv(L_bb)):
//   X = L^{-1}:  X_bb = D_b,  X_bj = -D_b sum_{k=j}^{b-1} L_bk X_kj  (b > j)
//     tasks ordered by their longest path to the end, one persistent
//     launch, per-tile flags (MFMA);
//   S = X^T X:   S_bj = sum_{k=b}^{nb-1} X_kb^T X_kj  (b >= j), independent
//     tiles (MFMA), written over the factor tiles.
// Apply: every lower tile S_bj (b > j) is read once and contributes S_bj r_j
// to block row b and S_bj^T r_b to block row j; the diagonal tiles
// contribute S_bb r_b. Phase 1 writes these 64-vectors per tile, phase 2
// adds them per DoF in a fixed order (deterministic, no atomics). No
// sequential chain: every tile is independent.
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
  extern __shared__ unsigned char smem_raw[];
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

// ---------------------------------------------------------------- S = X^T X
template <typename T>
__global__ __launch_bounds__(256) void k_inv_gram(int32_t n_tiles, const int4* __restrict__ meta,
                                                  const SubDesc* __restrict__ subs, const T* __restrict__ X,
                                                  T* __restrict__ S) {
  extern __shared__ unsigned char smem_raw[];
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

// ---------------------------------------------------------------- apply
// One wave per stored tile S_bj. Lane l = 16 r0 + c4 holds rows r0 + 4k
// (k < 16), columns 4 c4 .. 4 c4 + 3 of the tile: every load instruction of
// the wave reads four whole 256-byte rows. The 64 row sums (S_bj r_j) and the
// 64 column sums (S_bj^T r_b) are finished by butterfly reduce-scatters over
// lane bits 0-3 and 4-5, so each lane ends with one row sum (row r0 + 4 c4)
// and one column sum (column 4 c4 + r0): no LDS reduction, no barrier.
// The FP32 tiles are streamed with non-temporal loads (they are read once
// per application); for FP64 plain loads measured faster.
template <typename T>
struct TileRow;
template <>
struct TileRow<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static void load(const float* p, float (&o)[4]) {
    const v4 v = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
  __device__ static void lds4(const float* p, float (&o)[4]) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};
template <>
struct TileRow<double> {
  __device__ static void load(const double* p, double (&o)[4]) {
    const double2 u = reinterpret_cast<const double2*>(p)[0], v = reinterpret_cast<const double2*>(p)[1];
    o[0] = u.x;
    o[1] = u.y;
    o[2] = v.x;
    o[3] = v.y;
  }
  __device__ static void lds4(const double* p, double (&o)[4]) { load(p, o); }
};

// Phase 1: part[t] = (S_bj r_j, S_bj^T r_b) for tile t = (b, j); the second
// half is written only for off-diagonal tiles (diagonal tiles are stored
// whole). Entries of r beyond the subdomain's n are taken as zero.
// WPB waves (tiles) per work-group, a launch-shape choice of the autotuner.
template <typename T, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_symv_tiles(int32_t n_tiles, const int4* __restrict__ meta,
                                                         const SubDesc* __restrict__ subs, const T* __restrict__ S,
                                                         const double* __restrict__ r, T* __restrict__ part,
                                                         const DevState* st) {
  __shared__ __align__(16) T s_r[WPB][2 * TILE];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = blockIdx.x * WPB + w;
  if ((st && st->done) || t >= n_tiles) return;
  const int c4 = lane & 15, r0 = lane >> 4;
  T a[16][4];
  const T* base = S + (size_t)t * TT + r0 * TILE + 4 * c4;
#pragma unroll
  for (int k = 0; k < 16; ++k) TileRow<T>::load(base + 4 * TILE * k, a[k]);
  const int4 m = meta[t];
  const SubDesc sd = subs[m.x];
  const int b = m.y, j = m.z;
  const int gj = j * TILE + lane, gb = b * TILE + lane;
  T* sr = s_r[w];
  sr[lane] = gj < sd.n ? (T)r[sd.dof0 + gj] : T(0);
  // r_b stored so that rows r0 + 4k (k = 0..15) are contiguous at 16 r0
  sr[TILE + (lane & 3) * 16 + (lane >> 2)] = gb < sd.n ? (T)r[sd.dof0 + gb] : T(0);
  wave_sync();
  T rj[4], rb[16];
  TileRow<T>::lds4(sr + 4 * c4, rj);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T v[4];
    TileRow<T>::lds4(sr + TILE + 16 * r0 + 4 * q, v);
#pragma unroll
    for (int e = 0; e < 4; ++e) rb[4 * q + e] = v[e];
  }
  T ra[16], ca[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    ra[k] = a[k][0] * rj[0] + a[k][1] * rj[1] + a[k][2] * rj[2] + a[k][3] * rj[3];
#pragma unroll
    for (int c = 0; c < 4; ++c) ca[c] += a[k][c] * rb[k];
  }
#pragma unroll
  for (int h = 8; h >= 1; h >>= 1) {
    const bool hi = lane & h;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const T send = hi ? ra[i] : ra[i + h];
      const T keep = hi ? ra[i + h] : ra[i];
      ra[i] = keep + __shfl_xor(send, h, 64);
    }
  }
#pragma unroll
  for (int h = 2; h >= 1; h >>= 1) {
    const bool hi = lane & (16 * h);
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const T send = hi ? ca[i] : ca[i + h];
      const T keep = hi ? ca[i + h] : ca[i];
      ca[i] = keep + __shfl_xor(send, 16 * h, 64);
    }
  }
  T* pt = part + (size_t)t * 2 * TILE;
  pt[r0 + 4 * c4] = ra[0];
  if (j < b) pt[TILE + 4 * c4 + r0] = ca[0];
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
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = 0.0;
    for (int sp = 0; sp < splits; ++sp) v += xp[(size_t)sp * n + i];
    xs[i] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* Dr = D + (size_t)row * n;
  double acc = 0.0;
#pragma unroll 8
  for (int j = lane; j < n; j += 64) acc += Dr[j] * xs[j];
  acc = warp_sum(acc);
  if (lane == 0) y[row] = acc;
}

template <typename K>
hipError_t big_lds(K kernel, size_t sh) {
  if (sh <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
}

}  // namespace

hipError_t launch_inverse(int f32, int32_t n_tasks, const int4* tasks, int32_t n_tiles, const int4* meta,
                          const SubDesc* subs, void* L, void* X, int32_t* flags, DevState* st, int32_t* queue,
                          int grid_lower, int grid_gram, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  hipError_t e;
  if (f32) {
    const size_t sh = 2 * TILE * LDA * sizeof(float);
    hipLaunchKernelGGL(k_inv_lower<float>, dim3(grid_lower), dim3(256), sh, s, n_tasks, tasks, subs,
                       (const float*)L, (float*)X, flags, st, queue);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_inv_gram<float>, dim3(grid_gram), dim3(256), sh, s, n_tiles, meta, subs, (const float*)X,
                       (float*)L);
  } else {
    const size_t sh = 2 * TILE * LDA * sizeof(double);
    if ((e = big_lds(k_inv_lower<double>, sh)) != hipSuccess) return e;
    if ((e = big_lds(k_inv_gram<double>, sh)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_inv_lower<double>, dim3(grid_lower), dim3(256), sh, s, n_tasks, tasks, subs,
                       (const double*)L, (double*)X, flags, st, queue);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_inv_gram<double>, dim3(grid_gram), dim3(256), sh, s, n_tiles, meta, subs,
                       (const double*)X, (double*)L);
  }
  return hipGetLastError();
}

template <int WPB>
static void symv_tiles_wpb(int f32, int32_t n_tiles, const int4* meta, const SubDesc* subs, const void* S,
                           const double* r, void* part, const DevState* st, hipStream_t s) {
  const dim3 g((n_tiles + WPB - 1) / WPB), bl(64 * WPB);
  if (f32)
    hipLaunchKernelGGL((k_symv_tiles<float, WPB>), g, bl, 0, s, n_tiles, meta, subs, (const float*)S, r,
                       (float*)part, st);
  else
    hipLaunchKernelGGL((k_symv_tiles<double, WPB>), g, bl, 0, s, n_tiles, meta, subs, (const double*)S, r,
                       (double*)part, st);
}

hipError_t launch_symv_tiles(int f32, int waves, int32_t n_tiles, const int4* meta, const SubDesc* subs, const void* S,
                             const double* r, void* part, const DevState* st, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (waves) {
    case 1: symv_tiles_wpb<1>(f32, n_tiles, meta, subs, S, r, part, st, s); break;
    case 2: symv_tiles_wpb<2>(f32, n_tiles, meta, subs, S, r, part, st, s); break;
    case 4: symv_tiles_wpb<4>(f32, n_tiles, meta, subs, S, r, part, st, s); break;
    case 8: symv_tiles_wpb<8>(f32, n_tiles, meta, subs, S, r, part, st, s); break;
    default: return hipErrorInvalidValue;
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
