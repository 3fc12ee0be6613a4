// Direct 3D kernel for star stencils and the 27-point box: one time step per
// launch, streaming whole rows.
//
// Every wave64 computes one segment of 64 x CPL cells (one 16-byte vector per
// lane) of M consecutive interior rows (plane p, rows i0 .. i0 + M - 1) of
// the axis-2 extent; waves are numbered segment-fastest, then row group, then
// plane, and workgroups run in plain dispatch order, so at any moment the
// machine streams one window of consecutive rows and the rows a cell shares
// with its neighbours are re-read from the caches.  For each stencil row
// (p + d0, i + d1) a lane loads its vector straight from global memory, once
// for all the wave's rows that use it.  The centre rows of a star take their
// r neighbours on either side from the adjacent lanes (DPP; the wave's edge
// lanes from two wave-uniform loads); box rows load them per lane.  Each cell
// sums its terms in the canonical (d0, d1, d2) order with the same
// accumulation policy as the blocked kernels, so the results have the same
// bits.  Stores are non-temporal.  No LDS, no barrier: waves are independent.
#pragma once

#include "kcommon.h"

namespace s5d {

struct Stream3DArgs {
  const void* src;
  void* dst;
  const void* coef;  // device array of the coefficients, canonical order, working type
  int32_t I0, I1, I2;
  int32_t nws;       // wave segments per row
  int32_t ngr;       // groups of rows per plane (M rows each)
  int64_t nwaves;    // I0 * ngr * nws
};

constexpr int kStream3DThreads = 512;

// Rows per wave: a wave's M consecutive rows share the loads of their
// planes' rows (stars: M + 2r row loads of plane p and 2r M of the other
// planes instead of (4r + 1) M; boxes: (2r + 1)(M + 2r) instead of
// (2r + 1)^2 M).  Measured at 512^3 against 1, 2, 3, 4 and 8 rows: for stars
// 4 at radius 1 and 4, 2 at radius 2 and 3 (float32, float64 and compensated
// alike; 3 rows misalign with the workgroups, 8 spill); 4 for the 27-point
// box.
template <typename T, int R, bool BOX>
constexpr int stream3d_rows() {
  if constexpr (BOX) return 4;
  return R == 2 || R == 3 ? 2 : 4;
}

template <typename T, int ACC, int R, bool BOX>
__device__ __forceinline__ void stream3d_wave(const Stream3DArgs& a, int64_t gw) {
  constexpr int CPL = 16 / static_cast<int>(sizeof(T));
  constexpr int E = 2 * R + 1;
  constexpr int M = stream3d_rows<T, R, BOX>();
  constexpr bool DPPH = !BOX && R <= CPL;  // a lane shift reaches one neighbouring lane only
  const int P1 = a.I1 + 2 * R, P2 = a.I2 + 2 * R;
  const int ws = static_cast<int>(gw % a.nws);
  const int64_t rg = gw / a.nws;
  const int i0 = R + static_cast<int>(rg % a.ngr) * M;  // first interior row of this wave
  const int p = R + static_cast<int>(rg / a.ngr);       // interior plane
  const int lane = threadIdx.x & 63;
  const int wc0 = R + ws * 64 * CPL;  // first column of this wave (uniform)
  const int c0 = wc0 + lane * CPL;    // first column of this lane
  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);
  const T* __restrict__ c = static_cast<const T*>(a.coef);

  // the lane's cells of row (pp, ii) and, if `full`, their r neighbours on
  // each side; columns beyond the padded row read 0 (they feed no stored
  // cell), rows beyond it read the last row (they feed no stored row)
  auto load_row = [&](T (&x)[CPL + 2 * R], int pp, int ii, bool full) S5D_INL {
    const T* rp = src + (static_cast<int64_t>(pp) * P1 + min(ii, P1 - 1)) * P2;
    if (DPPH || !full) {
      if (c0 + CPL <= P2) {
        const LaneVec<T, CPL> v = *reinterpret_cast<const LaneVec<T, CPL>*>(rp + c0);
        sfor<CPL>([&](auto K) S5D_INL { x[R + K] = v.v[K]; });
      } else {
        sfor<CPL>([&](auto K) S5D_INL { x[R + K] = c0 + K < P2 ? rp[c0 + K] : T(0); });
      }
      if (full) {
        sfor<R>([&](auto J) S5D_INL {
          x[J] = lane_from_lower(x[CPL + J]);
          x[R + CPL + J] = lane_from_upper(x[R + J]);
        });
        sfor<R>([&](auto J) S5D_INL {
          const int lc = wc0 - R + J, rc = wc0 + 64 * CPL + J;
          const T lft = rp[lc < P2 ? lc : P2 - 1];
          const T rgt = rp[rc < P2 ? rc : P2 - 1];
          x[J] = lane == 0 ? lft : x[J];
          x[R + CPL + J] = lane == 63 ? (rc < P2 ? rgt : T(0)) : x[R + CPL + J];
        });
      }
    } else if (c0 + CPL + R <= P2) {
      const LaneVec<T, CPL> v = *reinterpret_cast<const LaneVec<T, CPL>*>(rp + c0);
      sfor<CPL>([&](auto K) S5D_INL { x[R + K] = v.v[K]; });
      sfor<R>([&](auto J) S5D_INL {
        x[J] = rp[c0 - R + J];
        x[R + CPL + J] = rp[c0 + CPL + J];
      });
    } else {
      sfor<CPL + 2 * R>([&](auto X) S5D_INL {
        const int col = c0 - R + X;
        x[X] = col < P2 ? rp[col] : T(0);
      });
    }
  };

  // rows i0 .. i0 + M - 1 of plane p; each cell sums (d0 < 0), then the
  // rows of its plane in d1 order (the centre row with its d2 terms), then
  // (d0 > 0)
  Accum<T, ACC> acc[M][CPL];
  if constexpr (BOX) {
    // planes p - R .. p + R, each with the rows i0 - R + Q of that plane
    sfor<E>([&](auto D0) S5D_INL {
      sfor<M + 2 * R>([&](auto Q) S5D_INL {
        T x[CPL + 2 * R];
        load_row(x, p - R + D0, i0 - R + Q, true);
        sfor<M>([&](auto MI) S5D_INL {
          constexpr int d1 = Q - MI - R;
          if constexpr (d1 >= -R && d1 <= R) {
            sfor<E>([&](auto D2) S5D_INL {
              const T ck = c[(D0 * E + d1 + R) * E + D2];
              sfor<CPL>([&](auto K) S5D_INL {
                if constexpr (D0 == 0 && d1 == -R && D2 == 0) acc[MI][K].first(ck, x[K + D2]);
                else acc[MI][K].add(ck, x[K + D2]);
              });
            });
          }
        });
      });
    });
  } else {
  sfor<R>([&](auto J) S5D_INL {  // (d0, 0, 0), d0 < 0
    sfor<M>([&](auto MI) S5D_INL {
      T x[CPL + 2 * R];
      load_row(x, p - R + J, i0 + MI, false);
      sfor<CPL>([&](auto K) S5D_INL {
        if constexpr (J == 0) acc[MI][K].first(c[J], x[R + K]);
        else acc[MI][K].add(c[J], x[R + K]);
      });
    });
  });
  sfor<M + 2 * R>([&](auto Q) S5D_INL {  // plane p, rows i0 - R + Q
    constexpr int mc = Q - R;             // the wave's row whose centre row this is
    T x[CPL + 2 * R];
    load_row(x, p, i0 - R + Q, mc >= 0 && mc < M);
    sfor<M>([&](auto MI) S5D_INL {
      constexpr int d1 = Q - MI - R;
      if constexpr (d1 < 0 && d1 >= -R) {
        sfor<CPL>([&](auto K) S5D_INL { acc[MI][K].add(c[R + (d1 + R)], x[R + K]); });
      } else if constexpr (d1 == 0) {
        sfor<E>([&](auto D2) S5D_INL {
          sfor<CPL>([&](auto K) S5D_INL { acc[MI][K].add(c[2 * R + D2], x[K + D2]); });
        });
      } else if constexpr (d1 > 0 && d1 <= R) {
        sfor<CPL>([&](auto K) S5D_INL { acc[MI][K].add(c[4 * R + d1], x[R + K]); });
      }
    });
  });
  sfor<R>([&](auto J) S5D_INL {  // (d0, 0, 0), d0 > 0
    sfor<M>([&](auto MI) S5D_INL {
      T x[CPL + 2 * R];
      load_row(x, p + 1 + J, i0 + MI, false);
      sfor<CPL>([&](auto K) S5D_INL { acc[MI][K].add(c[5 * R + 1 + J], x[R + K]); });
    });
  });
  }

  sfor<M>([&](auto MI) S5D_INL {
    if (i0 + MI < a.I1 + R) {
      T out[CPL];
      sfor<CPL>([&](auto K) S5D_INL { out[K] = acc[MI][K].value(); });
      T* wp = dst + (static_cast<int64_t>(p) * P1 + i0 + MI) * P2;
      if (c0 + CPL <= a.I2 + R) {
        using VT = T __attribute__((ext_vector_type(CPL), aligned(sizeof(T))));  // element-aligned address
        VT v;
        sfor<CPL>([&](auto K) S5D_INL { v[+K] = out[K]; });
        __builtin_nontemporal_store(v, reinterpret_cast<VT*>(wp + c0));
      } else {
        sfor<CPL>([&](auto K) S5D_INL {
          if (c0 + K < a.I2 + R) wp[c0 + K] = out[K];
        });
      }
    }
  });
}

// Workgroup lb: waves lb * 8 .. lb * 8 + 7 of the grid (those past the last
// one return at once).
template <typename T, int ACC, int R, bool BOX>
__device__ __forceinline__ void stream3d_block(const Stream3DArgs& a, int lb) {
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int64_t gw = static_cast<int64_t>(lb) * (kStream3DThreads / 64) + w;
  if (gw >= a.nwaves) return;
  stream3d_wave<T, ACC, R, BOX>(a, gw);
}

template <typename T, int ACC, int R, bool BOX>
__global__ __launch_bounds__(kStream3DThreads) void stream3d_kernel(Stream3DArgs a) {
  stream3d_block<T, ACC, R, BOX>(a, blockIdx.x);
}

template <typename T, int ACC, int R, bool BOX>
__global__ __launch_bounds__(kStream3DThreads) void stream3d_batch_kernel(const Stream3DArgs* __restrict__ items,
                                                                          const BlockMap* __restrict__ map) {
  const BlockMap m = map[xcd_logical_block(blockIdx.x, gridDim.x)];
  const Stream3DArgs a = uniform_copy(items[__builtin_amdgcn_readfirstlane(m.item)]);
  stream3d_block<T, ACC, R, BOX>(a, __builtin_amdgcn_readfirstlane(m.block));
}

template <typename T, int R, bool BOX>
int64_t stream3d_args(Stream3DArgs& a, const Round3D& rd) {
  constexpr int CPL = 16 / static_cast<int>(sizeof(T));
  a.src = rd.src;
  a.dst = rd.dst;
  a.coef = rd.dcoef;
  a.I0 = rd.I0;
  a.I1 = rd.I1;
  a.I2 = rd.I2;
  a.nws = (rd.I2 + 64 * CPL - 1) / (64 * CPL);
  a.ngr = (rd.I1 + stream3d_rows<T, R, BOX>() - 1) / stream3d_rows<T, R, BOX>();
  a.nwaves = static_cast<int64_t>(rd.I0) * a.ngr * a.nws;
  const int64_t nblk = (a.nwaves + kStream3DThreads / 64 - 1) / (kStream3DThreads / 64);
  return nblk > INT32_MAX ? 0 : nblk;
}

template <typename T, int ACC, int R, bool BOX>
hipError_t launch_stream3d(const Round3D& rd) {
  Stream3DArgs a;
  const int64_t nblk = stream3d_args<T, R, BOX>(a, rd);
  if (nblk == 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((stream3d_kernel<T, ACC, R, BOX>), dim3(static_cast<unsigned>(nblk)), dim3(kStream3DThreads), 0,
                     rd.stream, a);
  return hipGetLastError();
}

template <typename T, int R, bool BOX>
int fill_stream3d(void* item, const Round3D& rd) {
  Stream3DArgs a;
  const int64_t nblk = stream3d_args<T, R, BOX>(a, rd);
  __builtin_memcpy(item, &a, sizeof(a));
  return static_cast<int>(nblk);
}

template <typename T, int ACC, int R, bool BOX>
hipError_t launch_stream3d_batch(const void* items, const BlockMap* map, int nblocks, hipStream_t stream) {
  hipLaunchKernelGGL((stream3d_batch_kernel<T, ACC, R, BOX>), dim3(nblocks), dim3(kStream3DThreads), 0, stream,
                     static_cast<const Stream3DArgs*>(items), map);
  return hipGetLastError();
}

template <typename T, int ACC, int R, bool BOX>
int occupancy_stream3d() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stream3d_kernel<T, ACC, R, BOX>, kStream3DThreads, 0) !=
      hipSuccess)
    return 0;
  return nb;
}

}  // namespace s5d
