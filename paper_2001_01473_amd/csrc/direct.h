// Direct (one time step per launch) stencil kernels for gfx950.
//
// The temporally blocked kernels keep 2r accumulator planes per fused level in
// registers; for the largest stencils (the 125-point box in float64, radius 3
// and 4 in 3D, box radius 3 and 4 in 2D) that state does not fit a lane.
// These kernels cover them: a workgroup stages its output tile plus an r-wide
// margin in LDS, and every thread sums its cells' terms straight from LDS in
// the canonical (d0, d1[, d2]) order with the same accumulation policy as
// the blocked kernels -- so where both exist, they give the same bits.  Each
// launch is one time step: HBM traffic is one read and one write per cell and
// step (AN5D's b_T = 1), the tile margins are re-read from L2.
//
// Tiles: 2D 64 columns x 16 rows, 3D 64 (32 for radius >= 3) columns x 8
// rows x 4 planes; 256 threads, one column each, stacked along the rows.  The
// staged tile stays within 64 KiB of LDS for every supported radius.
#pragma once

#include "kcommon.h"

namespace s5d {

constexpr int kDirectY2 = 16, kDirectY3 = 8, kDirectZ3 = 4;

template <int NDIM, int R>
constexpr int direct_dx() {
  return NDIM == 3 && R >= 3 ? 32 : 64;
}

// Geometry of one direct launch (one grid, one step).
struct DirectArgs {
  const void* src;
  void* dst;
  const void* coef;  // device array of the stencil's coefficients, canonical order, working type
  int32_t I0, I1, I2;
  int32_t n0, n1, n2;  // tiles along each axis (2D: n2 = 1)
};

// Box stencils: each thread owns XB consecutive cells along the last axis in
// NPR (plane, row) pairs.  Row by row in canonical order it reads the XB + 2r
// staged values the row contributes once and feeds all 2r+1 terms of its XB
// cells from registers (each cell still sums in (d0, d1, d2) order), so LDS
// reads per term fall from 1 to (XB + 2r) / (XB (2r+1)).
template <typename T, int ACC, int NDIM, int R>
__device__ __forceinline__ void direct_box_cells(const DirectArgs& a, const T* tile, const T* __restrict__ c,
                                                 T* __restrict__ dst, int oz, int oy, int ox, int PZ, int PY,
                                                 int PX) {
  (void)a;
  constexpr int DX = direct_dx<NDIM, R>();
  constexpr int DY = NDIM == 2 ? kDirectY2 : kDirectY3;
  constexpr int DZ = NDIM == 2 ? 1 : kDirectZ3;
  constexpr int SX = DX + 2 * R, SY = DY + 2 * R;
  constexpr int XB = 4;
  constexpr int TXN = DX / XB;        // threads along the last axis
  constexpr int TYN = 256 / TXN;      // threads over the (plane, row) pairs
  constexpr int NPR = DZ * DY / TYN;  // (plane, row) pairs per thread
  static_assert(DX % XB == 0 && (DZ * DY) % TYN == 0 && NPR >= 1, "direct tile does not split evenly");
  constexpr int E = 2 * R + 1;
  const int tx = threadIdx.x % TXN, tyz = threadIdx.x / TXN;
  Accum<T, ACC> acc[NPR][XB];
  constexpr int NROWS = NDIM == 3 ? E * E : E;
  // rows one at a time (a runtime loop keeps one segment per pair live); the
  // first term of every cell is the first column of row 0
#pragma unroll 1
  for (int row = 0; row < NROWS; ++row) {
    const int D0 = NDIM == 3 ? row / E : 0, D1 = NDIM == 3 ? row % E : row;
    const T* __restrict__ crow = c + row * E;
    sfor<NPR>([&](auto P) S5D_INL {
      const int pr = tyz + TYN * P;
      const int z = NDIM == 3 ? pr / DY : 0, y = NDIM == 3 ? pr % DY : pr;
      const int base = NDIM == 3 ? ((z + D0) * SY + y + D1) * SX + XB * tx : (y + D1) * SX + XB * tx;
      T seg[XB + 2 * R];
      sfor<XB + 2 * R>([&](auto X) S5D_INL { seg[X] = tile[base + X]; });
      sfor<E>([&](auto D2) S5D_INL {
        const T ck = crow[D2];
        sfor<XB>([&](auto J) S5D_INL {
          if (D2 == 0 && row == 0)
            acc[P][J].first(ck, seg[J + D2]);
          else
            acc[P][J].add(ck, seg[J + D2]);
        });
      });
    });
  }
#pragma unroll
  for (int P = 0; P < NPR; ++P) {
    const int pr = tyz + TYN * P;
    const int z = NDIM == 3 ? pr / DY : 0, y = NDIM == 3 ? pr % DY : pr;
    const int gz = oz + R + z, gy = oy + R + y;
    const bool row_in = gy < PY - R && (NDIM == 2 || gz < PZ - R);
#pragma unroll
    for (int J = 0; J < XB; ++J) {
      const int gx = ox + R + XB * tx + J;
      if (row_in && gx < PX - R)
        dst[(static_cast<int64_t>(NDIM == 3 ? gz : 0) * PY + gy) * PX + gx] = acc[P][J].value();
    }
  }
}

// Star stencils (few terms, mostly one per row): one column per thread, RY
// rows per plane; consecutive threads read consecutive LDS words.
template <typename T, int ACC, int NDIM, int R>
__device__ __forceinline__ void direct_star_cells(const DirectArgs& a, const T* tile, const T* __restrict__ c,
                                                  T* __restrict__ dst, int oz, int oy, int ox, int PZ, int PY,
                                                  int PX) {
  (void)a;
  constexpr int DX = direct_dx<NDIM, R>();
  constexpr int DY = NDIM == 2 ? kDirectY2 : kDirectY3;
  constexpr int DZ = NDIM == 2 ? 1 : kDirectZ3;
  constexpr int SX = DX + 2 * R, SY = DY + 2 * R;
  constexpr int TY = 256 / DX;  // threads stacked along the rows
  constexpr int RY = DY / TY;   // rows (per plane) per thread
  const int tx = threadIdx.x % DX, ty = threadIdx.x / DX;
  Accum<T, ACC> acc[DZ][RY];
  // cell (z, j) of this thread: tile plane z + R, row ty + TY j + R, column tx + R
  auto at = [&](int z, int j, int d0, int d1, int d2) S5D_INL -> T {
    if constexpr (NDIM == 3)
      return tile[((z + R + d0) * SY + ty + TY * j + R + d1) * SX + tx + R + d2];
    else
      return tile[(ty + TY * j + R + d0) * SX + tx + R + d1];
  };
  int k = 0;
  bool first = true;
  auto term = [&](int d0, int d1, int d2) S5D_INL {
    const T ck = c[k++];
#pragma unroll
    for (int z = 0; z < DZ; ++z)
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        if (first)
          acc[z][j].first(ck, at(z, j, d0, d1, d2));
        else
          acc[z][j].add(ck, at(z, j, d0, d1, d2));
      }
    first = false;
  };
  // canonical order of the star's offsets
  if constexpr (NDIM == 3) {
    for (int d = -R; d < 0; ++d) term(d, 0, 0);
    for (int d = -R; d < 0; ++d) term(0, d, 0);
    for (int d = -R; d <= R; ++d) term(0, 0, d);
    for (int d = 1; d <= R; ++d) term(0, d, 0);
    for (int d = 1; d <= R; ++d) term(d, 0, 0);
  } else {
    for (int d = -R; d < 0; ++d) term(d, 0, 0);
    for (int d = -R; d <= R; ++d) term(0, d, 0);
    for (int d = 1; d <= R; ++d) term(d, 0, 0);
  }
  const int gx = ox + R + tx;
#pragma unroll
  for (int z = 0; z < DZ; ++z)
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const int gz = oz + R + z, gy = oy + R + ty + TY * j;
      const bool in = gx < PX - R && gy < PY - R && (NDIM == 2 || gz < PZ - R);
      if (in) dst[(static_cast<int64_t>(NDIM == 3 ? gz : 0) * PY + gy) * PX + gx] = acc[z][j].value();
    }
}

template <typename T, int ACC, int NDIM, int R, bool BOX>
__device__ __forceinline__ void direct_block(const DirectArgs& a, int lb, T* tile) {
  constexpr int DX = direct_dx<NDIM, R>();
  constexpr int DY = NDIM == 2 ? kDirectY2 : kDirectY3;
  constexpr int DZ = NDIM == 2 ? 1 : kDirectZ3;
  constexpr int SX = DX + 2 * R, SY = DY + 2 * R, SZ = NDIM == 2 ? 1 : DZ + 2 * R;
  static_assert(SX * SY * SZ * sizeof(T) <= 65536, "staged tile exceeds 64 KiB");
  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);
  const T* __restrict__ c = static_cast<const T*>(a.coef);

  // tile origin in padded coordinates (= first output cell - R)
  const int t2 = lb % a.n2, t1 = (lb / a.n2) % a.n1, t0 = lb / (a.n2 * a.n1);
  const int P0 = a.I0 + 2 * R, P1 = a.I1 + 2 * R;
  const int P2 = NDIM == 3 ? a.I2 + 2 * R : 1;
  // 2D: axes (0, 1) are the tile's (Y, X); 3D: (0, 1, 2) are (Z, Y, X)
  const int oz = NDIM == 3 ? t0 * DZ : 0;
  const int oy = NDIM == 3 ? t1 * DY : t0 * DY;
  const int ox = NDIM == 3 ? t2 * DX : t1 * DX;
  const int PY = NDIM == 3 ? P1 : P0, PX = NDIM == 3 ? P2 : P1;
  const int PZ = NDIM == 3 ? P0 : 1;

  for (int i = threadIdx.x; i < SZ * SY * SX; i += 256) {
    const int z = i / (SY * SX), y = (i / SX) % SY, x = i % SX;
    const int gz = oz + z, gy = oy + y, gx = ox + x;
    T v = T(0);
    if (gz < PZ && gy < PY && gx < PX) v = src[(static_cast<int64_t>(gz) * PY + gy) * PX + gx];
    tile[i] = v;
  }
  __syncthreads();

  if constexpr (BOX)
    direct_box_cells<T, ACC, NDIM, R>(a, tile, c, dst, oz, oy, ox, PZ, PY, PX);
  else
    direct_star_cells<T, ACC, NDIM, R>(a, tile, c, dst, oz, oy, ox, PZ, PY, PX);
}

template <typename T, int ACC, int NDIM, int R, bool BOX>
constexpr int direct_tile_elems() {
  constexpr int DY = NDIM == 2 ? kDirectY2 : kDirectY3;
  return (direct_dx<NDIM, R>() + 2 * R) * (DY + 2 * R) * (NDIM == 2 ? 1 : kDirectZ3 + 2 * R);
}

template <typename T, int ACC, int NDIM, int R, bool BOX>
__global__ __launch_bounds__(256) void direct_kernel(DirectArgs a) {
  __shared__ T tile[direct_tile_elems<T, ACC, NDIM, R, BOX>()];
  direct_block<T, ACC, NDIM, R, BOX>(a, xcd_logical_block(blockIdx.x, gridDim.x), tile);
}

template <typename T, int ACC, int NDIM, int R, bool BOX>
__global__ __launch_bounds__(256) void direct_batch_kernel(const DirectArgs* __restrict__ items,
                                                           const BlockMap* __restrict__ map) {
  __shared__ T tile[direct_tile_elems<T, ACC, NDIM, R, BOX>()];
  const BlockMap m = map[xcd_logical_block(blockIdx.x, gridDim.x)];
  const DirectArgs a = items[__builtin_amdgcn_readfirstlane(m.item)];
  direct_block<T, ACC, NDIM, R, BOX>(a, __builtin_amdgcn_readfirstlane(m.block), tile);
}

template <int NDIM, int R>
int64_t direct_args(DirectArgs& a, const void* src, void* dst, const void* coef, int I0, int I1, int I2) {
  a.src = src;
  a.dst = dst;
  a.coef = coef;
  a.I0 = I0;
  a.I1 = I1;
  a.I2 = NDIM == 3 ? I2 : 1;
  constexpr int DX = direct_dx<NDIM, R>();
  if constexpr (NDIM == 3) {
    a.n0 = (I0 + kDirectZ3 - 1) / kDirectZ3;
    a.n1 = (I1 + kDirectY3 - 1) / kDirectY3;
    a.n2 = (I2 + DX - 1) / DX;
  } else {
    a.n0 = (I0 + kDirectY2 - 1) / kDirectY2;
    a.n1 = (I1 + DX - 1) / DX;
    a.n2 = 1;
  }
  const int64_t nblk = static_cast<int64_t>(a.n0) * a.n1 * a.n2;
  return nblk > INT32_MAX ? 0 : nblk;
}

template <typename T, int ACC, int R, bool BOX>
hipError_t launch_direct2d(const Round2D& rd) {
  DirectArgs a;
  const int64_t nblk = direct_args<2, R>(a, rd.src, rd.dst, rd.dcoef, rd.I0, rd.I1, 1);
  if (nblk == 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((direct_kernel<T, ACC, 2, R, BOX>), dim3(static_cast<unsigned>(nblk)), dim3(256), 0, rd.stream,
                     a);
  return hipGetLastError();
}

template <typename T, int ACC, int R, bool BOX>
hipError_t launch_direct3d(const Round3D& rd) {
  DirectArgs a;
  const int64_t nblk = direct_args<3, R>(a, rd.src, rd.dst, rd.dcoef, rd.I0, rd.I1, rd.I2);
  if (nblk == 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((direct_kernel<T, ACC, 3, R, BOX>), dim3(static_cast<unsigned>(nblk)), dim3(256), 0, rd.stream,
                     a);
  return hipGetLastError();
}

template <int R>
int fill_direct2d(void* item, const Round2D& rd) {
  DirectArgs a;
  const int64_t nblk = direct_args<2, R>(a, rd.src, rd.dst, rd.dcoef, rd.I0, rd.I1, 1);
  __builtin_memcpy(item, &a, sizeof(a));
  return static_cast<int>(nblk);
}

template <int R>
int fill_direct3d(void* item, const Round3D& rd) {
  DirectArgs a;
  const int64_t nblk = direct_args<3, R>(a, rd.src, rd.dst, rd.dcoef, rd.I0, rd.I1, rd.I2);
  __builtin_memcpy(item, &a, sizeof(a));
  return static_cast<int>(nblk);
}

template <typename T, int ACC, int NDIM, int R, bool BOX>
hipError_t launch_direct_batch(const void* items, const BlockMap* map, int nblocks, hipStream_t stream) {
  hipLaunchKernelGGL((direct_batch_kernel<T, ACC, NDIM, R, BOX>), dim3(nblocks), dim3(256), 0, stream,
                     static_cast<const DirectArgs*>(items), map);
  return hipGetLastError();
}

template <typename T, int ACC, int NDIM, int R, bool BOX>
int occupancy_direct() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, direct_kernel<T, ACC, NDIM, R, BOX>, 256, 0) != hipSuccess)
    return 0;
  return nb;
}

}  // namespace s5d
