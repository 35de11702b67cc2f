// Explicit local inverses S_i = A_i^{-1} = L_i^{-T} L_i^{-1} and their
// application z_i = S_i r_i (exact local solvers of Sec. 3 applied as one
// packed symmetric matrix-vector product per subdomain).
//
// Setup, after the tile Cholesky (diagonal tiles hold D_b = inv(L_bb)):
//   X = L^{-1}:  X_bb = D_b,  X_bj = -D_b sum_{k=j}^{b-1} L_bk X_kj  (b > j)
//     tasks in row order, one persistent launch, per-tile flags (MFMA);
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
__global__ __launch_bounds__(256) void k_inv_lower(int32_t n_tasks, const int4* __restrict__ tasks,
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
      const T* D = Lb + (size_t)(b * (b + 1) / 2 + b) * TT;
      for (int e = tid; e < TILE * TILE; e += blockDim.x) store_agent(out + e, D[e]);
    } else {
      Quad<T> acc;
      acc.zero();
      for (int k = j; k < b; ++k) {
        wait_flag(fl + k * (k + 1) / 2 + j, st);
        tile_to_lds(Lb + (size_t)(b * (b + 1) / 2 + k) * TT, As, false);    // L_bk
        tile_to_lds_t(Xb + (size_t)(k * (k + 1) / 2 + j) * TT, Bs, true);  // Bs[c][m] = X_kj[m][c]
        __syncthreads();
        acc.mma(As, Bs, R0, C0, lane, T(1));
        __syncthreads();
      }
      // X_bj = -D_b acc: Bs[c][m] = acc[m][c], As = D_b
#pragma unroll
      for (int e = 0; e < 16; ++e) Bs[(C0 + Quad<T>::col(e, lane)) * LDA + R0 + Quad<T>::row(e, lane)] = acc.get(e);
      tile_to_lds(Lb + (size_t)(b * (b + 1) / 2 + b) * TT, As, false);
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
    for (int k = b; k < sd.nb; ++k) {
      tile_to_lds_t(Xb + (size_t)(k * (k + 1) / 2 + b) * TT, As, false);  // As[r][m] = X_kb[m][r]
      tile_to_lds_t(Xb + (size_t)(k * (k + 1) / 2 + j) * TT, Bs, false);  // Bs[c][m] = X_kj[m][c]
      __syncthreads();
      acc.mma(As, Bs, R0, C0, lane, T(1));
      __syncthreads();
    }
    T* out = S + (size_t)t * TT;
#pragma unroll
    for (int e = 0; e < 16; ++e) out[(R0 + Quad<T>::row(e, lane)) * TILE + C0 + Quad<T>::col(e, lane)] = acc.get(e);
  }
}

// ---------------------------------------------------------------- apply
template <typename T>
struct V16;
template <>
struct V16<float> {
  using V = float4;
  static constexpr int N = 4;
  __device__ static float at(const V& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
};
template <>
struct V16<double> {
  using V = double2;
  static constexpr int N = 2;
  __device__ static double at(const V& v, int i) { return i == 0 ? v.x : v.y; }
};

// Phase 1: UNROLL consecutive tiles per work-group; part[t] = (S_bj r_j, S_bj^T r_b).
template <typename T, int UNROLL>
__global__ __launch_bounds__(256) void k_symv_tiles(int32_t n_tiles, const int4* __restrict__ meta,
                                                    const SubDesc* __restrict__ subs, const T* __restrict__ S,
                                                    const double* __restrict__ r, T* __restrict__ part,
                                                    const DevState* st) {
  using VT = V16<T>;
  using V = typename VT::V;
  constexpr int VEC = VT::N;
  constexpr int LPR = TILE / VEC;
  constexpr int RPP = 256 / LPR;
  constexpr int PASSES = TILE / RPP;
  __shared__ T s_red[UNROLL][4][TILE];
  if (st && st->done) return;
  const int tid = threadIdx.x;
  const int lc = tid % LPR, r0 = tid / LPR;
  const int lane = tid & 63, wave = tid >> 6;
  const int t0 = blockIdx.x * UNROLL;
  V tv[UNROLL][PASSES];
  int4 mt[UNROLL];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    const int t = min(t0 + u, n_tiles - 1);
    mt[u] = meta[t];
#pragma unroll
    for (int k = 0; k < PASSES; ++k) tv[u][k] = *(const V*)(S + (size_t)t * TT + (r0 + RPP * k) * TILE + lc * VEC);
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    const SubDesc sd = subs[mt[u].x];
    const int b = mt[u].y, j = mt[u].z;
    const bool valid = t0 + u < n_tiles;
    // rows: S_bj r_j
    T rj[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const int gc = j * TILE + lc * VEC + v;
      rj[v] = gc < sd.n ? (T)r[sd.dof0 + gc] : T(0);
    }
    T accu[PASSES];
#pragma unroll
    for (int k = 0; k < PASSES; ++k) {
      T a = T(0);
#pragma unroll
      for (int v = 0; v < VEC; ++v) a += VT::at(tv[u][k], v) * rj[v];
      accu[k] = a;
    }
#pragma unroll
    for (int k = 0; k < PASSES; ++k)
#pragma unroll
      for (int o = LPR / 2; o >= 1; o >>= 1) accu[k] += __shfl_xor(accu[k], o, 64);
    if (valid && lc == 0) {
#pragma unroll
      for (int k = 0; k < PASSES; ++k) part[(size_t)(t0 + u) * 2 * TILE + r0 + RPP * k] = accu[k];
    }
    // columns: S_bj^T r_b (off-diagonal tiles only)
    if (j < b) {
      T accv[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) accv[v] = T(0);
#pragma unroll
      for (int k = 0; k < PASSES; ++k) {
        const int gr = b * TILE + r0 + RPP * k;
        const T rb = gr < sd.n ? (T)r[sd.dof0 + gr] : T(0);
#pragma unroll
        for (int v = 0; v < VEC; ++v) accv[v] += VT::at(tv[u][k], v) * rb;
      }
#pragma unroll
      for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int o = LPR; o < 64; o <<= 1) accv[v] += __shfl_xor(accv[v], o, 64);
      if (lane < LPR) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) s_red[u][wave][lc * VEC + v] = accv[v];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    if (t0 + u < n_tiles && mt[u].z < mt[u].y && tid < TILE)
      part[(size_t)(t0 + u) * 2 * TILE + TILE + tid] = s_red[u][0][tid] + s_red[u][1][tid] + s_red[u][2][tid] + s_red[u][3][tid];
  }
}

// Phase 2: z[d] = sum_{j<=b} part(b,j).rows[rho] + sum_{j>b} part(j,b).cols[rho].
template <typename T>
__global__ __launch_bounds__(256) void k_symv_gather(int np, int32_t N, const int32_t* __restrict__ cell_sub,
                                                     const SubDesc* __restrict__ subs, const T* __restrict__ part,
                                                     T* __restrict__ z, const DevState* st) {
  if (st && st->done) return;
  const int64_t n = (int64_t)N * np;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    const SubDesc sd = subs[cell_sub[d / np]];
    const int loc = (int)(d - sd.dof0);
    const int b = loc / TILE, rho = loc - b * TILE;
    double s = 0.0;
    const T* pb = part + (size_t)(sd.tile0 + b * (b + 1) / 2) * 2 * TILE + rho;
    for (int j = 0; j <= b; ++j) s += (double)pb[(size_t)j * 2 * TILE];
    for (int j = b + 1; j < sd.nb; ++j)
      s += (double)part[(size_t)(sd.tile0 + j * (j + 1) / 2 + b) * 2 * TILE + TILE + rho];
    z[d] = (T)s;
  }
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

hipError_t launch_symv(int f32, int np, int32_t N, int32_t n_tiles, const int4* meta, const SubDesc* subs,
                       const int32_t* cell_sub, const void* S, const double* r, void* part, void* z,
                       const DevState* st, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  const int64_t n = (int64_t)N * np;
  const int g2 = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  if (f32) {
    constexpr int U = 4;
    hipLaunchKernelGGL((k_symv_tiles<float, U>), dim3((n_tiles + U - 1) / U), dim3(256), 0, s, n_tiles, meta, subs,
                       (const float*)S, r, (float*)part, st);
    hipLaunchKernelGGL(k_symv_gather<float>, dim3(g2), dim3(256), 0, s, np, N, cell_sub, subs, (const float*)part,
                       (float*)z, st);
  } else {
    constexpr int U = 2;
    hipLaunchKernelGGL((k_symv_tiles<double, U>), dim3((n_tiles + U - 1) / U), dim3(256), 0, s, n_tiles, meta,
                       subs, (const double*)S, r, (double*)part, st);
    hipLaunchKernelGGL(k_symv_gather<double>, dim3(g2), dim3(256), 0, s, np, N, cell_sub, subs,
                       (const double*)part, (double*)z, st);
  }
  return hipGetLastError();
}

}  // namespace asdg
