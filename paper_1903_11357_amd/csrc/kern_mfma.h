// MFMA tile helpers shared by the factorisation kernels (gfx950, wave64).
// A work-group owns one TB x TB tile (TB = 64 or 32) with one wave per 32x32
// quadrant: four waves for TB = 64 (wave w at rows 32*(w/2), columns
// 32*(w%2)), a single wave for TB = 32.
#pragma once

#include "kern_common.h"

namespace asdg {
namespace mfma {

constexpr int LDA = TILE + 1;  // padded LDS row (bank spread for column reads)

// Work-group shape for a TB x TB tile: one wave per 32x32 quadrant.
template <int TB>
struct Shape {
  static_assert(TB == 32 || TB == 64, "tile edge 32 or 64");
  static constexpr int LD = TB + 1;                 // padded LDS row
  static constexpr int QPR = TB / 32;               // quadrants per tile row
  static constexpr int THREADS = 64 * QPR * QPR;    // one wave per quadrant
  __device__ static int r0(int wave) { return 32 * (wave / QPR); }
  __device__ static int c0(int wave) { return 32 * (wave % QPR); }
};

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Per-lane accumulator of a wave's 32x32 quadrant, 16 values per lane.
template <typename T>
struct Quad;

template <>
struct Quad<float> {
  f32x16 c;
  __device__ void zero() {
#pragma unroll
    for (int e = 0; e < 16; ++e) c[e] = 0.0f;
  }
  // v_mfma_f32_32x32x2f32 result: register e of lane l holds D[8(e/4) + 4(l/32) + e%4][l%32]
  __device__ static int row(int e, int lane) { return 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3); }
  __device__ static int col(int e, int lane) { return lane & 31; }
  __device__ float get(int e) const { return c[e]; }
  __device__ void set(int e, float v) { c[e] = v; }
  // c += sign * A[R0.., :] * B[C0.., :]^T with A, B in LDS (row-major, row
  // pitch TB + 1, TB columns)
  template <int TB = TILE>
  __device__ void mma(const float* A, const float* B, int R0, int C0, int lane, float sign) {
    constexpr int LD = TB + 1;
    const float* a = A + (R0 + (lane & 31)) * LD + (lane >> 5);
    const float* b = B + (C0 + (lane & 31)) * LD + (lane >> 5);
#pragma unroll 8
    for (int k0 = 0; k0 < TB; k0 += 2) c = __builtin_amdgcn_mfma_f32_32x32x2f32(sign * a[k0], b[k0], c, 0, 0, 0);
  }
};

template <>
struct Quad<double> {
  f64x4 c[4];
  __device__ void zero() {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int v = 0; v < 4; ++v) c[s][v] = 0.0;
  }
  // v_mfma_f64_16x16x4f64 result: register v of lane l holds D[4v + l/16][l%16]
  __device__ static int row(int e, int lane) { return 16 * ((e >> 2) >> 1) + 4 * (e & 3) + (lane >> 4); }
  __device__ static int col(int e, int lane) { return 16 * ((e >> 2) & 1) + (lane & 15); }
  __device__ double get(int e) const { return c[e >> 2][e & 3]; }
  __device__ void set(int e, double v) { c[e >> 2][e & 3] = v; }
  template <int TB = TILE>
  __device__ void mma(const double* A, const double* B, int R0, int C0, int lane, double sign) {
    constexpr int LD = TB + 1;
    const double* a0 = A + (R0 + (lane & 15)) * LD + (lane >> 4);
    const double* a1 = a0 + 16 * LD;
    const double* b0 = B + (C0 + (lane & 15)) * LD + (lane >> 4);
    const double* b1 = b0 + 16 * LD;
#pragma unroll 4
    for (int k0 = 0; k0 < TB; k0 += 4) {
      const double x0 = sign * a0[k0], x1 = sign * a1[k0];
      const double y0 = b0[k0], y1 = b1[k0];
      c[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, c[0], 0, 0, 0);
      c[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, c[1], 0, 0, 0);
      c[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, c[2], 0, 0, 0);
      c[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, c[3], 0, 0, 0);
    }
  }
};

// Thread 0 waits (bounded) until both flags are raised; one barrier.
__device__ __forceinline__ void wait_flags(const int32_t* f0, const int32_t* f1, DevState* st) {
  if (threadIdx.x == 0) {
    int ok = load_agent(f0) != 0 && load_agent(f1) != 0;
    for (int64_t budget = WAIT_BUDGET; !ok && budget > 0; --budget) {
      __builtin_amdgcn_s_sleep(2);
      ok = load_agent(f0) != 0 && load_agent(f1) != 0;
      if (!ok && (budget & 255) == 0 && load_agent(&st->abort)) break;
    }
    if (!ok) store_agent(&st->abort, 1);
  }
  __syncthreads();
}

__device__ __forceinline__ void wait_flag(const int32_t* f, DevState* st) {
  if (threadIdx.x == 0) {
    int ok = load_agent(f) != 0;
    for (int64_t budget = WAIT_BUDGET; !ok && budget > 0; --budget) {
      __builtin_amdgcn_s_sleep(2);
      ok = load_agent(f) != 0;
      if (!ok && (budget & 255) == 0 && load_agent(&st->abort)) break;
    }
    if (!ok) store_agent(&st->abort, 1);
  }
  __syncthreads();
}

// A tile (global, row-major TB x TB) held in registers by the NT threads of
// a work-group: thread t keeps elements t + NT i, i < TB * TB / NT (16 for
// both tile shapes). Loading the next operands into registers before the
// MFMA work on the current ones overlaps global latency with compute.
template <typename T, int TB = TILE, int NT = Shape<TB>::THREADS>
struct TileRegs {
  static constexpr int N = TB * TB / NT;
  static constexpr int LD = TB + 1;
  T v[N];
  __device__ void load(const T* g) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = g[threadIdx.x + NT * i];
  }
  __device__ void load_coherent(const T* g) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = load_agent(g + threadIdx.x + NT * i);
  }
  __device__ void store(T* g) const {
#pragma unroll
    for (int i = 0; i < N; ++i) g[threadIdx.x + NT * i] = v[i];
  }
  __device__ void store_coherent(T* g) const {
#pragma unroll
    for (int i = 0; i < N; ++i) store_agent(g + threadIdx.x + NT * i, v[i]);
  }
  // s[r][c] = g[r][c]
  __device__ void put(T* s) const {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int e = threadIdx.x + NT * i;
      s[(e / TB) * LD + (e % TB)] = v[i];
    }
  }
  // s[c][r] = g[r][c]
  __device__ void put_t(T* s) const {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int e = threadIdx.x + NT * i;
      s[(e % TB) * LD + (e / TB)] = v[i];
    }
  }
};

}  // namespace mfma
}  // namespace asdg
