// Batched triangular sweeps z_i = L_i^{-T} L_i^{-1} r_i for every subdomain
// (exact local solvers of Sec. 3 applied in parallel) in one persistent
// launch.
//
// Each factor is stored as packed lower-triangular TILE x TILE tiles,
// row-major inside a tile; the diagonal tiles hold inv(L_bb) (formed during
// the factorisation), so every step of a sweep is a tile GEMV.
//
// Work decomposition: a task is one tile row of one sweep of one subdomain:
//   forward  (i, b): y_b = inv(L_bb) (r_b - sum_{j<b} L_bj y_j)
//   backward (i, b): z_b = inv(L_bb)^T (y_b - sum_{j>b} L_jb^T z_j)
// Work-groups take tasks from an atomic counter in a host-sorted order in
// which every dependency precedes its consumer, so a task only ever waits
// for tasks already held by running work-groups (no co-residency
// assumption). The dependency "value written" is carried by the values
// themselves: y and z are pre-filled with a NaN sentinel and written with
// device-coherent stores; consumers poll the values they need with
// device-coherent loads. Every wait is bounded (see kern_common.h).
#include "kern_common.h"

namespace asdg {

namespace {

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using V = float4;
  static constexpr int N = 4;
  __device__ static float at(const V& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
};
template <>
struct Vec16<double> {
  using V = double2;
  static constexpr int N = 2;
  __device__ static double at(const V& v, int i) { return i == 0 ? v.x : v.y; }
};

template <typename T>
__device__ __forceinline__ T wait_value(const T* p, DevState* st) {
  T v = load_agent(p);
  if (!is_sentinel(v)) return v;
  for (int64_t budget = WAIT_BUDGET; budget > 0; --budget) {
    __builtin_amdgcn_s_sleep(1);
    v = load_agent(p);
    if (!is_sentinel(v)) return v;
    if ((budget & 255) == 0 && load_agent(&st->abort)) return T(0);
  }
  store_agent(&st->abort, 1);
  return T(0);
}

constexpr int UNROLL = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_trsv(int32_t n_tasks, const int4* __restrict__ tasks,
                                              const SubDesc* __restrict__ subs, const T* __restrict__ tiles,
                                              const double* __restrict__ r, T* y, T* z, DevState* st,
                                              int32_t* queue) {
  using VT = Vec16<T>;
  using V = typename VT::V;
  constexpr int VEC = VT::N;
  constexpr int LPR = TILE / VEC;     // lanes covering one tile row
  constexpr int RPP = 256 / LPR;      // tile rows per pass of the work-group
  constexpr int PASSES = TILE / RPP;  // passes per tile
  constexpr size_t TT = (size_t)TILE * TILE;
  __shared__ int s_task;
  __shared__ T s_vec[TILE];
  __shared__ T s_red[4][TILE];
  if (st->done) return;
  const int tid = threadIdx.x;
  const int lc = tid % LPR, r0 = tid / LPR;
  const int lane = tid & 63, wave = tid >> 6;

  for (;;) {
    if (tid == 0) s_task = atomicAdd(queue, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= n_tasks) break;
    const int4 td = tasks[t];
    const SubDesc sd = subs[td.x];
    const int b = td.z;
    const int n = sd.n;
    const T* base = tiles + (size_t)sd.tile0 * TT;
    const T* D = base + (size_t)(b * (b + 1) / 2 + b) * TT;

    if (td.y == 0) {
      // ---------------- forward: row tiles (b, 0..b-1), then inv(L_bb)
      T acc[PASSES];
#pragma unroll
      for (int k = 0; k < PASSES; ++k) acc[k] = T(0);
      const T* rowbase = base + (size_t)(b * (b + 1) / 2) * TT;
      const T* yv = y + sd.dof0 + lc * VEC;
      int j = 0;
      for (; j + UNROLL <= b; j += UNROLL) {
        V tv[UNROLL][PASSES];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
          for (int k = 0; k < PASSES; ++k)
            tv[u][k] = *(const V*)(rowbase + (size_t)(j + u) * TT + (r0 + RPP * k) * TILE + lc * VEC);
        T xv[UNROLL][VEC];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
          for (int v = 0; v < VEC; ++v) xv[u][v] = wait_value(yv + (j + u) * TILE + v, st);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
          for (int k = 0; k < PASSES; ++k)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[k] += VT::at(tv[u][k], v) * xv[u][v];
      }
      for (; j < b; ++j) {
        V tv[PASSES];
#pragma unroll
        for (int k = 0; k < PASSES; ++k)
          tv[k] = *(const V*)(rowbase + (size_t)j * TT + (r0 + RPP * k) * TILE + lc * VEC);
        T xv[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) xv[v] = wait_value(yv + j * TILE + v, st);
#pragma unroll
        for (int k = 0; k < PASSES; ++k)
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[k] += VT::at(tv[k], v) * xv[v];
      }
#pragma unroll
      for (int k = 0; k < PASSES; ++k)
#pragma unroll
        for (int o = LPR / 2; o >= 1; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
      if (lc == 0) {
#pragma unroll
        for (int k = 0; k < PASSES; ++k) {
          const int row = r0 + RPP * k;
          const int gi = b * TILE + row;
          const T rv = gi < n ? (T)r[sd.dof0 + gi] : T(0);
          s_vec[row] = rv - acc[k];
        }
      }
      __syncthreads();
      T sv[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) sv[v] = s_vec[lc * VEC + v];
#pragma unroll
      for (int k = 0; k < PASSES; ++k) {
        const V dv = *(const V*)(D + (r0 + RPP * k) * TILE + lc * VEC);
        T a = T(0);
#pragma unroll
        for (int v = 0; v < VEC; ++v) a += VT::at(dv, v) * sv[v];
        acc[k] = a;
      }
#pragma unroll
      for (int k = 0; k < PASSES; ++k)
#pragma unroll
        for (int o = LPR / 2; o >= 1; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
      if (lc == 0) {
#pragma unroll
        for (int k = 0; k < PASSES; ++k) {
          const int gi = b * TILE + r0 + RPP * k;
          if (gi < n) store_agent(y + sd.dof0 + gi, acc[k]);
        }
      }
      __syncthreads();
    } else {
      // ---------------- backward: column tiles (b+1..nb-1, b)^T, then inv(L_bb)^T
      T acc[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] = T(0);
      const int nb = sd.nb;
      int j = b + 1;
      for (; j + UNROLL <= nb; j += UNROLL) {
        V tv[UNROLL][PASSES];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const T* tile = base + (size_t)((j + u) * (j + u + 1) / 2 + b) * TT;
#pragma unroll
          for (int k = 0; k < PASSES; ++k) tv[u][k] = *(const V*)(tile + (r0 + RPP * k) * TILE + lc * VEC);
        }
        T zv[UNROLL][PASSES];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
          for (int k = 0; k < PASSES; ++k) {
            const int gi = (j + u) * TILE + r0 + RPP * k;
            zv[u][k] = gi < n ? wait_value(z + sd.dof0 + gi, st) : T(0);
          }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
          for (int k = 0; k < PASSES; ++k)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] += VT::at(tv[u][k], v) * zv[u][k];
      }
      for (; j < nb; ++j) {
        const T* tile = base + (size_t)(j * (j + 1) / 2 + b) * TT;
        V tv[PASSES];
#pragma unroll
        for (int k = 0; k < PASSES; ++k) tv[k] = *(const V*)(tile + (r0 + RPP * k) * TILE + lc * VEC);
        T zv[PASSES];
#pragma unroll
        for (int k = 0; k < PASSES; ++k) {
          const int gi = j * TILE + r0 + RPP * k;
          zv[k] = gi < n ? wait_value(z + sd.dof0 + gi, st) : T(0);
        }
#pragma unroll
        for (int k = 0; k < PASSES; ++k)
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[v] += VT::at(tv[k], v) * zv[k];
      }
      // combine the RPP row groups: in-wave, then across the 4 waves
#pragma unroll
      for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int o = LPR; o < 64; o <<= 1) acc[v] += __shfl_xor(acc[v], o, 64);
      if (lane < LPR) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) s_red[wave][lc * VEC + v] = acc[v];
      }
      __syncthreads();
      if (tid < TILE) {
        const T u = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
        const int gi = b * TILE + tid;
        const T yv = gi < n ? wait_value(y + sd.dof0 + gi, st) : T(0);
        s_vec[tid] = yv - u;
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] = T(0);
#pragma unroll
      for (int k = 0; k < PASSES; ++k) {
        const V dv = *(const V*)(D + (r0 + RPP * k) * TILE + lc * VEC);
        const T s = s_vec[r0 + RPP * k];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] += VT::at(dv, v) * s;
      }
#pragma unroll
      for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int o = LPR; o < 64; o <<= 1) acc[v] += __shfl_xor(acc[v], o, 64);
      if (lane < LPR) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) s_red[wave][lc * VEC + v] = acc[v];
      }
      __syncthreads();
      if (tid < TILE) {
        const T u = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
        const int gi = b * TILE + tid;
        if (gi < n) store_agent(z + sd.dof0 + gi, u);
      }
      __syncthreads();
    }
  }
}

}  // namespace

hipError_t launch_trsv(int f32, int32_t n_tasks, const int4* tasks, const SubDesc* subs, const void* tiles,
                       const double* r, void* y, void* z, DevState* st, int32_t* queue, int grid,
                       hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_trsv<float>, dim3(grid), dim3(256), 0, s, n_tasks, tasks, subs, (const float*)tiles, r,
                       (float*)y, (float*)z, st, queue);
  else
    hipLaunchKernelGGL(k_trsv<double>, dim3(grid), dim3(256), 0, s, n_tasks, tasks, subs, (const double*)tiles, r,
                       (double*)y, (double*)z, st, queue);
  return hipGetLastError();
}

}  // namespace asdg
