// Batched triangular sweeps z_i = L_i^{-T} L_i^{-1} r_i for every subdomain
// (exact local solvers of Sec. 3 applied in parallel) in one persistent
// launch.
//
// Each factor is stored as packed lower-triangular TB x TB tiles (TB = 64
// or 32), row-major inside a tile; the diagonal tiles hold inv(L_bb) (formed during
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
// device-coherent loads (one per thread per chunk of tiles, shared through
// LDS). Every wait is bounded (see kern_common.h).
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

// One thread waits for `p` (the value a producer wrote last, or one of the
// values it wrote together); the barrier then releases the work-group, whose
// threads read their own values with wait_value (almost always at once).
// Keeps the polling traffic of a waiting work-group to a single thread.
template <typename T>
__device__ __forceinline__ void wait_group(const T* p, DevState* st) {
  if (threadIdx.x == 0 && p) (void)wait_value(p, st);
  __syncthreads();
}

template <typename T, int UNROLL, int TB>
__global__ __launch_bounds__(256) void k_trsv(int32_t n_tasks, const int4* __restrict__ tasks,
                                              const SubDesc* __restrict__ subs, const T* __restrict__ tiles,
                                              const double* __restrict__ r, T* y, T* z, DevState* st,
                                              int32_t* queue, uint64_t* trace) {
  using VT = Vec16<T>;
  using V = typename VT::V;
  constexpr int VEC = VT::N;
  constexpr int LPR = TB / VEC;     // lanes covering one tile row
  constexpr int RPP = 256 / LPR;      // tile rows per pass of the work-group
  constexpr int PASSES = TB / RPP;  // passes per tile
  constexpr size_t TT = (size_t)TB * TB;
  __shared__ int s_task;
  __shared__ T s_vec[TB];
  __shared__ T s_red[4][TB];
  __shared__ T s_x[2][UNROLL * TB];  // staged y (forward) or z (backward) values, double-buffered
  static_assert(UNROLL * TB <= 256, "one staged value per thread");
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
    if (trace && tid == 0) trace[3 * (size_t)t] = wall_clock64();
    const int4 td = tasks[t];
    const SubDesc sd = subs[td.x];
    const int b = td.z;
    const int n = sd.n;
    const T* base = tiles + (size_t)sd.tile0 * TT;
    const T* D = base + (size_t)(b * (b + 1) / 2 + b) * TT;
    // the diagonal inverse and the right-hand side are needed last: fetch them first
    V dv[PASSES];
#pragma unroll
    for (int k = 0; k < PASSES; ++k) dv[k] = *(const V*)(D + (r0 + RPP * k) * TB + lc * VEC);
    T rhs[PASSES];  // forward: r rows of this tile row (lanes lc == 0)
#pragma unroll
    for (int k = 0; k < PASSES; ++k) {
      const int gi = b * TB + r0 + RPP * k;
      rhs[k] = (td.y == 0 && lc == 0 && gi < n) ? (T)r[sd.dof0 + gi] : T(0);
    }

    if (td.y == 0) {
      // ---------------- forward: row tiles (b, 0..b-1), then inv(L_bb)
      T acc[PASSES];
#pragma unroll
      for (int k = 0; k < PASSES; ++k) acc[k] = T(0);
      const T* rowbase = base + (size_t)(b * (b + 1) / 2) * TT;
      const T* yv0 = y + sd.dof0;
      int buf = 0;
      for (int j = 0; j < b; j += UNROLL, buf ^= 1) {
        V tv[UNROLL][PASSES];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const bool ok = j + u < b;
#pragma unroll
          for (int k = 0; k < PASSES; ++k)
            tv[u][k] = ok ? *(const V*)(rowbase + (size_t)(j + u) * TT + (r0 + RPP * k) * TB + lc * VEC) : V{};
        }
        // the chunk's y values: one poller for the latest tile, then one
        // device-coherent load per thread, shared via LDS
        const int jl = min(j + UNROLL, b) - 1;
        wait_group(yv0 + jl * TB + TB - 1, st);
        if (tid < UNROLL * TB) {
          const int jt = j + tid / TB;
          s_x[buf][tid] = jt < b ? wait_value(yv0 + jt * TB + (tid % TB), st) : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
          for (int k = 0; k < PASSES; ++k)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[k] += VT::at(tv[u][k], v) * s_x[buf][u * TB + lc * VEC + v];
      }
      if (trace && tid == 0) trace[3 * (size_t)t + 1] = wall_clock64();
#pragma unroll
      for (int k = 0; k < PASSES; ++k)
#pragma unroll
        for (int o = LPR / 2; o >= 1; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
      if (lc == 0) {
#pragma unroll
        for (int k = 0; k < PASSES; ++k) {
          s_vec[r0 + RPP * k] = rhs[k] - acc[k];
        }
      }
      __syncthreads();
      T sv[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) sv[v] = s_vec[lc * VEC + v];
#pragma unroll
      for (int k = 0; k < PASSES; ++k) {
        T a = T(0);
#pragma unroll
        for (int v = 0; v < VEC; ++v) a += VT::at(dv[k], v) * sv[v];
        acc[k] = a;
      }
#pragma unroll
      for (int k = 0; k < PASSES; ++k)
#pragma unroll
        for (int o = LPR / 2; o >= 1; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
      if (lc == 0) {
#pragma unroll
        for (int k = 0; k < PASSES; ++k) {
          const int gi = b * TB + r0 + RPP * k;
          if (gi < n) store_agent(y + sd.dof0 + gi, acc[k]);
        }
      }
      if (trace && tid == 0) trace[3 * (size_t)t + 2] = wall_clock64();
      __syncthreads();
    } else {
      // ---------------- backward: column tiles (b+1..nb-1, b)^T, then inv(L_bb)^T
      T acc[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] = T(0);
      const int nb = sd.nb;
      // oldest tiles first: z_{b+1} (produced last) is needed in the last chunk
      int buf = 0;
      for (int jhi = nb - 1; jhi > b; jhi -= UNROLL, buf ^= 1) {
        const int jlo = max(jhi - UNROLL + 1, b + 1);  // chunk = tiles jlo..jhi
        V tv[UNROLL][PASSES];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int jj = jlo + u;
          const bool ok = jj <= jhi;
          const T* tile = base + (size_t)(jj * (jj + 1) / 2 + b) * TT;
#pragma unroll
          for (int k = 0; k < PASSES; ++k) tv[u][k] = ok ? *(const V*)(tile + (r0 + RPP * k) * TB + lc * VEC) : V{};
        }
        // tile jlo was finished last among the chunk's tiles
        wait_group(z + sd.dof0 + jlo * TB, st);
        if (tid < UNROLL * TB) {
          const int gi = jlo * TB + tid;
          s_x[buf][tid] = (gi < (jhi + 1) * TB && gi < n) ? wait_value(z + sd.dof0 + gi, st) : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
          for (int k = 0; k < PASSES; ++k) {
            const T zk = s_x[buf][u * TB + r0 + RPP * k];
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] += VT::at(tv[u][k], v) * zk;
          }
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
      if (tid < TB) {
        const T u = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
        const int gi = b * TB + tid;
        const T yv = gi < n ? wait_value(y + sd.dof0 + gi, st) : T(0);
        s_vec[tid] = yv - u;
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] = T(0);
#pragma unroll
      for (int k = 0; k < PASSES; ++k) {
        const T s = s_vec[r0 + RPP * k];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] += VT::at(dv[k], v) * s;
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
      if (tid < TB) {
        const T u = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
        const int gi = b * TB + tid;
        if (gi < n) store_agent(z + sd.dof0 + gi, u);
      }
      if (trace && tid == 0) trace[3 * (size_t)t + 2] = wall_clock64();
      __syncthreads();
    }
  }
}

}  // namespace

hipError_t launch_trsv(int f32, int tile, int32_t n_tasks, const int4* tasks, const SubDesc* subs,
                       const void* tiles, const double* r, void* y, void* z, DevState* st, int32_t* queue, int grid,
                       uint64_t* trace, hipStream_t s) {
  if (tile != 32 && tile != 64) return hipErrorInvalidValue;
  if (n_tasks <= 0) return hipSuccess;
  if (f32) {
    if (tile == 64)
      hipLaunchKernelGGL((k_trsv<float, 4, 64>), dim3(grid), dim3(256), 0, s, n_tasks, tasks, subs,
                         (const float*)tiles, r, (float*)y, (float*)z, st, queue, trace);
    else
      hipLaunchKernelGGL((k_trsv<float, 8, 32>), dim3(grid), dim3(256), 0, s, n_tasks, tasks, subs,
                         (const float*)tiles, r, (float*)y, (float*)z, st, queue, trace);
  } else {
    if (tile == 64)
      hipLaunchKernelGGL((k_trsv<double, 2, 64>), dim3(grid), dim3(256), 0, s, n_tasks, tasks, subs,
                         (const double*)tiles, r, (double*)y, (double*)z, st, queue, trace);
    else
      hipLaunchKernelGGL((k_trsv<double, 4, 32>), dim3(grid), dim3(256), 0, s, n_tasks, tasks, subs,
                         (const double*)tiles, r, (double*)y, (double*)z, st, queue, trace);
  }
  return hipGetLastError();
}

}  // namespace asdg
