// Direct 2D kernel: one time step per launch, streaming whole rows.
//
// Workgroup (row group g, segment s) computes the cells of the M interior
// rows p0 .. p0 + M - 1 (p0 = R + g*M) in columns [R + s*SEG, R + (s+1)*SEG),
// SEG = kStreamThreads x CPL cells.  Each thread reads its CPL cells and the
// r cells on either side from the M + 2r rows p0 - r .. p0 + M - 1 + r
// straight from global memory, once for all its M rows, and sums every cell's
// terms in the canonical (d0, d1) order, with the same accumulation policy as
// the blocked kernels -- so both give the same bits.  Workgroups run in plain
// dispatch order: at any moment the whole machine works on one window of
// consecutive rows, which the memory system streams like a plain copy; the
// rows shared with the neighbouring groups are served by the caches
// (measured on MI355X: 12 % faster than giving each XCD its own contiguous
// band of rows).  Star stencils take the in-row neighbours of the centre row
// from the neighbouring lanes (DPP); the wave's two edge lanes take theirs
// from two wave-uniform loads, so no lane diverges.  Results are written with
// non-temporal stores (they are not read again in this launch).  No LDS, no
// barrier.
#pragma once

#include "kcommon.h"

namespace s5d {

struct Stream2DArgs {
  const void* src;
  void* dst;
  const void* coef;  // device array of the coefficients, canonical order, working type
  int32_t I0, I1;
  int32_t nseg;      // segments per row
  int32_t ngr;       // groups of M rows along axis 0
};

constexpr int kStreamThreads = 512;  // threads per workgroup (measured best of 128..1024)

template <typename T>
constexpr int stream2d_cpl() {
  return 16 / static_cast<int>(sizeof(T));  // one 16-byte vector per thread
}

// Rows per thread: a thread's M consecutive rows share the loads of the
// M + 2r stencil rows (instead of 2r + 1 each).  Measured at 16384^2 against
// 1, 2, 4 and 8 rows: 2 for plain radius-1 stencils, 4 for the others
// (float32 and float64 alike).
template <int ACC, int R>
constexpr int stream2d_rows() {
  return ACC == 0 && R == 1 ? 2 : 4;
}

template <typename T, int ACC, int R, bool BOX>
__device__ __forceinline__ void stream2d_block(const Stream2DArgs& a, int lb) {
  constexpr int CPL = stream2d_cpl<T>();
  constexpr int SEG = kStreamThreads * CPL;
  constexpr int E = 2 * R + 1;
  const int P1 = a.I1 + 2 * R;
  constexpr int M = stream2d_rows<ACC, R>();
  const int p0 = R + (lb / a.nseg) * M;     // first interior row of this workgroup
  const int seg = lb - (lb / a.nseg) * a.nseg;
  const int c0 = R + seg * SEG + static_cast<int>(threadIdx.x) * CPL;  // first column of this thread
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int wc0 = R + seg * SEG + wave * 64 * CPL;                      // first column of this wave
  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);
  const T* __restrict__ c = static_cast<const T*>(a.coef);
  // the thread's cells and their r neighbours on each side, per stencil row;
  // columns beyond the padded row read 0 (they feed no stored cell)
  constexpr bool DPPH = !BOX && R <= CPL;  // a lane shift reaches one neighbouring lane only
  // rows beyond the padded grid read its last row (they feed no stored row)
  auto load_row = [&](T (&x)[CPL + 2 * R], int row, bool full) S5D_INL {
    const T* rp = src + static_cast<int64_t>(min(row, a.I0 + 2 * R - 1)) * P1;
    if constexpr (DPPH) {
      // own cells (a vector, or cell by cell at the row end); then, with
      // every lane active, the neighbours from the adjacent lanes
      if (c0 + CPL <= P1) {
        const LaneVec<T, CPL> v = *reinterpret_cast<const LaneVec<T, CPL>*>(rp + c0);
        sfor<CPL>([&](auto K) S5D_INL { x[R + K] = v.v[K]; });
      } else {
        sfor<CPL>([&](auto K) S5D_INL { x[R + K] = c0 + K < P1 ? rp[c0 + K] : T(0); });
      }
      if (full) {
        sfor<R>([&](auto J) S5D_INL {
          x[J] = lane_from_lower(x[CPL + J]);
          x[R + CPL + J] = lane_from_upper(x[R + J]);
        });
        // the wave's edge lanes: wave-uniform loads (clamped into the row
        // for a wave past its end, whose cells are not stored)
        const int lane = threadIdx.x & 63;
        sfor<R>([&](auto J) S5D_INL {
          const int lc = wc0 - R + J, rc = wc0 + 64 * CPL + J;
          const T lft = rp[lc < P1 ? lc : P1 - 1];
          const T rgt = rp[rc < P1 ? rc : P1 - 1];
          x[J] = lane == 0 ? lft : x[J];
          x[R + CPL + J] = lane == 63 ? (rc < P1 ? rgt : T(0)) : x[R + CPL + J];
        });
      }
    } else if (c0 + CPL + R <= P1) {
      const LaneVec<T, CPL> v = *reinterpret_cast<const LaneVec<T, CPL>*>(rp + c0);
      sfor<CPL>([&](auto K) S5D_INL { x[R + K] = v.v[K]; });
      if (full)
        sfor<R>([&](auto J) S5D_INL {
          x[J] = rp[c0 - R + J];
          x[R + CPL + J] = rp[c0 + CPL + J];
        });
    } else {
      sfor<CPL + 2 * R>([&](auto X) S5D_INL {
        const int col = c0 - R + X;
        x[X] = (col < P1 && (full || (X >= R && X < R + CPL))) ? rp[col] : T(0);
      });
    }
  };
  // rows p0 .. p0 + M - 1: stencil row Q = p0 - R + Q serves row m as its
  // d0 = Q - m - R, so every cell still sums its rows in d0 order
  Accum<T, ACC> acc[M][CPL];
  sfor<M + 2 * R>([&](auto Q) S5D_INL {
    constexpr int mc = Q - R;  // the row whose centre row this is
    T x[CPL + 2 * R];
    load_row(x, p0 - R + Q, BOX || (mc >= 0 && mc < M));
    sfor<M>([&](auto MI) S5D_INL {
      constexpr int d0 = Q - MI - R;
      if constexpr (d0 >= -R && d0 <= R) {
        if constexpr (BOX) {
          sfor<E>([&](auto D1) S5D_INL {
            const T ck = c[(d0 + R) * E + decltype(D1)::value];
            sfor<CPL>([&](auto K) S5D_INL {
              if constexpr (d0 == -R && decltype(D1)::value == 0)
                acc[MI][K].first(ck, x[K + D1]);
              else
                acc[MI][K].add(ck, x[K + D1]);
            });
          });
        } else if constexpr (d0 != 0) {
          const T ck = c[d0 < 0 ? d0 + R : 3 * R + d0];
          sfor<CPL>([&](auto K) S5D_INL {
            if constexpr (d0 == -R)
              acc[MI][K].first(ck, x[R + K]);
            else
              acc[MI][K].add(ck, x[R + K]);
          });
        } else {
          sfor<E>([&](auto D1) S5D_INL {
            const T ck = c[R + decltype(D1)::value];
            sfor<CPL>([&](auto K) S5D_INL { acc[MI][K].add(ck, x[K + D1]); });
          });
        }
      }
    });
  });
  sfor<M>([&](auto MI) S5D_INL {
    if (p0 + MI < a.I0 + R) {
      T out[CPL];
      sfor<CPL>([&](auto K) S5D_INL { out[K] = acc[MI][K].value(); });
      T* wp = dst + static_cast<int64_t>(p0 + MI) * P1;
      if (c0 + CPL <= a.I1 + R) {
        using VT = T __attribute__((ext_vector_type(CPL), aligned(sizeof(T))));  // element-aligned address
        VT v;
        sfor<CPL>([&](auto K) S5D_INL { v[+K] = out[K]; });
        __builtin_nontemporal_store(v, reinterpret_cast<VT*>(wp + c0));
      } else {
        sfor<CPL>([&](auto K) S5D_INL {
          if (c0 + K < a.I1 + R) wp[c0 + K] = out[K];
        });
      }
    }
  });
}

template <typename T, int ACC, int R, bool BOX>
__global__ __launch_bounds__(kStreamThreads) void stream2d_kernel(Stream2DArgs a) {
  stream2d_block<T, ACC, R, BOX>(a, blockIdx.x);
}

template <typename T, int ACC, int R, bool BOX>
__global__ __launch_bounds__(kStreamThreads) void stream2d_batch_kernel(const Stream2DArgs* __restrict__ items,
                                                             const BlockMap* __restrict__ map) {
  const BlockMap m = map[xcd_logical_block(blockIdx.x, gridDim.x)];
  const Stream2DArgs a = items[__builtin_amdgcn_readfirstlane(m.item)];
  stream2d_block<T, ACC, R, BOX>(a, __builtin_amdgcn_readfirstlane(m.block));
}

template <typename T, int ACC, int R>
int64_t stream2d_args(Stream2DArgs& a, const Round2D& rd) {
  constexpr int SEG = kStreamThreads * stream2d_cpl<T>();
  a.src = rd.src;
  a.dst = rd.dst;
  a.coef = rd.dcoef;
  a.I0 = rd.I0;
  a.I1 = rd.I1;
  a.nseg = (rd.I1 + SEG - 1) / SEG;
  a.ngr = (rd.I0 + stream2d_rows<ACC, R>() - 1) / stream2d_rows<ACC, R>();
  const int64_t nblk = static_cast<int64_t>(a.ngr) * a.nseg;
  return nblk > INT32_MAX ? 0 : nblk;
}

template <typename T, int ACC, int R, bool BOX>
hipError_t launch_stream2d(const Round2D& rd) {
  Stream2DArgs a;
  const int64_t nblk = stream2d_args<T, ACC, R>(a, rd);
  if (nblk == 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((stream2d_kernel<T, ACC, R, BOX>), dim3(static_cast<unsigned>(nblk)), dim3(kStreamThreads), 0, rd.stream,
                     a);
  return hipGetLastError();
}

template <typename T, int ACC, int R>
int fill_stream2d(void* item, const Round2D& rd) {
  Stream2DArgs a;
  const int64_t nblk = stream2d_args<T, ACC, R>(a, rd);
  __builtin_memcpy(item, &a, sizeof(a));
  return static_cast<int>(nblk);
}

template <typename T, int ACC, int R, bool BOX>
hipError_t launch_stream2d_batch(const void* items, const BlockMap* map, int nblocks, hipStream_t stream) {
  hipLaunchKernelGGL((stream2d_batch_kernel<T, ACC, R, BOX>), dim3(nblocks), dim3(kStreamThreads), 0, stream,
                     static_cast<const Stream2DArgs*>(items), map);
  return hipGetLastError();
}

template <typename T, int ACC, int R, bool BOX>
int occupancy_stream2d() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stream2d_kernel<T, ACC, R, BOX>, kStreamThreads, 0) != hipSuccess)
    return 0;
  return nb;
}

}  // namespace s5d
