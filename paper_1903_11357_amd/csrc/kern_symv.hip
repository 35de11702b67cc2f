// Application of the explicit local inverses S_i = A_i^{-1} (the exact
// local solvers of Sec. 3 applied as one packed symmetric matrix-vector
// product per subdomain): z_i = S_i r_i.
//
// Every lower tile S_bj (b > j) is read once and contributes S_bj r_j to
// block row b and S_bj^T r_b to block row j. The diagonal tiles are stored
// whole but read only on and below the diagonal: with L_b that lower part,
// S_bb r_b = L_b r_b + (L_b - diag)^T r_b, again a row-sum and a column-sum
// vector. This kernel writes these 64-vectors per tile; the prolongation
// kernel adds them per DoF in a fixed order (deterministic, no atomics). No
// sequential chain: every tile is independent.
#include <algorithm>

#include "kern_common.h"

namespace asdg {

namespace {

constexpr size_t TT = (size_t)TILE * TILE;

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
// whole). Entries of r beyond the subdomain's n are taken as zero. meta[t].w
// is the number of rows of tile row b inside the subdomain: the padding rows
// of a ragged last tile row (zero, and identity on the diagonal, with r zero
// there) contribute nothing to the sums that are read and are not loaded.
// WPB waves (tiles) per work-group, a launch-shape choice of the autotuner.
//
// The two precisions take the load forms measured fastest for them. FP32:
// the tile index is made wave-uniform, so its meta data and subdomain
// descriptor come through scalar loads; the 16 row pieces are loaded without
// branches and the loads of r are issued right behind them, so no wave
// waits for its tile before fetching r. A piece that is not read (see below)
// is loaded from the tile's first piece instead, which lane 0 reads in the
// same instruction: no extra memory traffic; at most 96 registers, so five
// waves fit per SIMD. FP64 (twice the registers per piece): one branch per
// row piece, and r after the tile (a third wave per SIMD would spill).
template <typename T, int WPB>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1))) void k_symv_tiles(int32_t n_tiles, const int4* __restrict__ meta,
                                                         const SubDesc* __restrict__ subs, const T* __restrict__ S,
                                                         const double* __restrict__ r, T* __restrict__ part,
                                                         const DevState* st) {
  constexpr bool F32 = sizeof(T) == 4;
  __shared__ __align__(16) T s_r[WPB][2 * TILE];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = F32 ? __builtin_amdgcn_readfirstlane(blockIdx.x * WPB + w) : blockIdx.x * WPB + w;
  if ((st && st->done) || t >= n_tiles) return;
  const int c4 = lane & 15, r0 = lane >> 4;
  const int4 m = meta[t];
  const int b = m.y, j = m.z;
  const bool diag = j == b;
  // diagonal tiles: rows r0 + 4k are read only in the 16-byte pieces that
  // reach the diagonal (column offset 4 c4 - 4k <= r0); nor are rows beyond
  // the subdomain. Where such a piece holds other values (FP32), they never
  // reach a sum that is read: the masks below drop the diagonal tiles' upper
  // pieces, r is zero beyond the subdomain, and the row sums of padding rows
  // are not read.
  const int cut = diag ? 4 * c4 - r0 : -64;
  const int rows = m.w - r0;  // row r0 + 4k is inside the subdomain when 4k < rows
  T a[16][4];
  const T* tile = S + (size_t)t * TT;
  const int off = r0 * TILE + 4 * c4;
  if (F32) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      TileRow<T>::load(tile + (cut <= 4 * k && 4 * k < rows ? off + 4 * TILE * k : 0), a[k]);
    __builtin_amdgcn_sched_barrier(0);  // all tile loads issue before the loads of r wait for the descriptor
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (cut <= 4 * k && 4 * k < rows) {
        TileRow<T>::load(tile + off + 4 * TILE * k, a[k]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) a[k][e] = T(0);
      }
    }
  }
  const SubDesc sd = subs[m.x];
  const int gj = j * TILE + lane, gb = b * TILE + lane;
  T* sr = s_r[w];
  T vj, vb;
  if (F32) {
    // indices clamped into the subdomain: no branch around the loads
    const double rjv = r[sd.dof0 + min(gj, sd.n - 1)], rbv = r[sd.dof0 + min(gb, sd.n - 1)];
    vj = gj < sd.n ? (T)rjv : T(0);
    vb = gb < sd.n ? (T)rbv : T(0);
  } else {
    vj = gj < sd.n ? (T)r[sd.dof0 + gj] : T(0);
    vb = gb < sd.n ? (T)r[sd.dof0 + gb] : T(0);
  }
  sr[lane] = vj;
  // r_b stored so that rows r0 + 4k (k = 0..15) are contiguous at 16 r0
  sr[TILE + (lane & 3) * 16 + (lane >> 2)] = vb;
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
  // diagonal tiles: row sums over columns c <= r, column sums over rows
  // r > c (with cut + e = c - r for the element (r, c) = (r0 + 4k, 4 c4 + e))
  T ra[16], ca[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    T lo[4], sl[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      lo[e] = cut + e <= 4 * k ? a[k][e] : T(0);
      sl[e] = cut + e < 4 * k ? a[k][e] : T(0);
    }
    ra[k] = lo[0] * rj[0] + lo[1] * rj[1] + lo[2] * rj[2] + lo[3] * rj[3];
#pragma unroll
    for (int c = 0; c < 4; ++c) ca[c] += sl[c] * rb[k];
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
  pt[TILE + 4 * c4 + r0] = ca[0];
}

// Per-DoF sums of the tile partials of one packed symmetric matrix of
// order n with nb tile rows (tile (b, j) at b(b+1)/2 + j), in the same fixed
// order as the local solves' prolongation: row sums of tiles (b, 0..b), the
// diagonal tile's column sums, then column sums of tiles (b+1..nb-1, b).
__global__ __launch_bounds__(256) void k_tile_partials_sum(int32_t n, int32_t nb, const double* __restrict__ part,
                                                           double* __restrict__ out, const DevState* st) {
  if (st && st->done) return;
  for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < n; d += gridDim.x * blockDim.x) {
    const int b = d / TILE, rho = d - b * TILE;
    const double* pr = part + (size_t)(b * (b + 1) / 2) * 2 * TILE + rho;
    double v = 0.0;
#pragma unroll 8
    for (int j = 0; j <= b; ++j) v += pr[(size_t)j * 2 * TILE];
    v += pr[(size_t)b * 2 * TILE + TILE];
#pragma unroll 8
    for (int j = b + 1; j < nb; ++j) v += part[(size_t)(j * (j + 1) / 2 + b) * 2 * TILE + TILE + rho];
    out[d] = v;
  }
}

// out[i] = sum over s < splits of in[s n + i], in order of s.
__global__ __launch_bounds__(256) void k_sum_splits(int32_t n, int splits, const double* __restrict__ in,
                                                    double* __restrict__ out, const DevState* st) {
  if (st && st->done) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int s = 0; s < splits; ++s) v += in[(size_t)s * n + i];
    out[i] = v;
  }
}

}  // namespace

hipError_t launch_tile_partials_sum(int32_t n, int32_t nb, const double* part, double* out, const DevState* st,
                                    hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if ((int64_t)nb * TILE < n) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_tile_partials_sum, dim3(grid), dim3(256), 0, s, n, nb, part, out, st);
  return hipGetLastError();
}

hipError_t launch_sum_splits(int32_t n, int splits, const double* in, double* out, const DevState* st, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (splits < 1) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_sum_splits, dim3(grid), dim3(256), 0, s, n, splits, in, out, st);
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

}  // namespace asdg
