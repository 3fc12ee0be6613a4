// 2D temporally blocked stencil sweep for gfx950 (device code + launcher).
//
// Method (AN5D "Execution Model" and "Optimizations"): a tile of the plane
// normal to the streaming axis (axis 0) walks along axis 0 and carries BT
// computational streams, one per fused time level.  Level T updates the row
// that lies T*R rows behind the row just loaded, so each row is read from HBM
// once and written once per BT time steps.  The tile overlaps its neighbours
// by BT*R columns on each side; the valid width shrinks by 2R per level and
// only the compute region of level BT is stored.  The axis-0 extent is cut
// into stream blocks of `chunk` rows (h_SN, "Division of Streaming
// Dimension"), each of which starts BT*R rows early to warm up the levels.
//
// MI355X mapping (differs from the paper's CUDA design):
//  * one wave64 is one tile; lane l owns CPL consecutive columns, so the tile
//    is 64*CPL columns wide and needs no shared memory and no barrier: the
//    in-plane neighbours that live in another lane come from DPP whole-wave
//    shifts (wave_shr:1 / wave_shl:1).  Lanes at the tile edge receive
//    meaningless values, which only ever reach the overlap region that the
//    shrinking valid width discards.
//  * per level a window of 2R+1 rows lives in VGPRs with fixed roles ("Register
//    Allocation"): the stream loop is unrolled by a multiple of 2R+1 so every
//    window slot is a compile-time register and no value is ever shifted.
//  * star stencils exchange only the centre row across lanes ("diagonal-access
//    free"); box stencils exchange each row once when it enters the window and
//    keep the 2R neighbour values beside it.
//  * rows are prefetched PF = (2R+1)*PFK steps ahead into staging registers
//    (PFK = 0 loads each row in place, for stencils whose window is large).
//  * boundary cells (the fixed halo of width R) are passed through unchanged at
//    every level ("halo overwrite" in the paper); only waves whose tile or stream
//    block touches the boundary run that code path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "s5d_internal.h"

namespace s5d {

template <int N>
using ic = std::integral_constant<int, N>;

template <typename F, int... Is>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(ic<Is>{}), ...);
}
// Compile-time loop: f(ic<0>{}), ..., f(ic<N-1>{}).
template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int pmod(int a, int m) { return ((a % m) + m) % m; }

// DPP whole-wavefront shifts by one lane.  wave_shr:1 (0x138) hands lane l
// the value of lane l-1; wave_shl:1 (0x130) hands lane l the value of lane
// l+1.  The lane without a source receives 0.
__device__ __forceinline__ int lane_from_lower_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ int lane_from_upper_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, false);
}

__device__ __forceinline__ float lane_from_lower(float v) {
  return __int_as_float(lane_from_lower_i32(__float_as_int(v)));
}
__device__ __forceinline__ float lane_from_upper(float v) {
  return __int_as_float(lane_from_upper_i32(__float_as_int(v)));
}
__device__ __forceinline__ double lane_from_lower(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_from_lower_i32(static_cast<int>(b));
  const int hi = lane_from_lower_i32(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double lane_from_upper(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_from_upper_i32(static_cast<int>(b));
  const int hi = lane_from_upper_i32(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<unsigned int>(lo));
}

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
// that consecutive logical blocks (neighbouring tiles, which share BT*R
// overlap columns) run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_logical_block(int b, int nblk) {
  const int q = nblk >> 3, rem = nblk & 7, x = b & 7, i = b >> 3;
  return x < rem ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

template <typename T, int R, bool BOX, int BT, int CPL, int PFK, bool EDGE>
__device__ __forceinline__ void sweep2d_body(const Sweep2DArgs& a, const CoefPack<T, npts(2, R, BOX)>& cf,
                                             int lane, int tile, int chunk) {
  constexpr int U = 2 * R + 1;        // window rows per level
  constexpr int W = 64 * CPL;         // tile width (columns)
  constexpr int C = W - 2 * BT * R;   // compute-region width
  constexpr int PF = U * PFK;         // prefetch distance in steps (0: load in place)
  constexpr int NS = PF > 0 ? PF : U; // steps per unrolled iteration
  constexpr int NX = BOX ? 2 * R : 1; // cached lane-exchange values per window row

  const int I0 = a.I0, I1 = a.I1;
  const int P0 = I0 + 2 * R, P1 = I1 + 2 * R;
  const int c_first = R + tile * C;      // first compute column
  const int col0 = c_first - BT * R;     // first column of the tile
  const int row_a = R + chunk * a.chunk; // first output row of this stream block
  const int row_b = min(row_a + a.chunk, I0 + R);

  int ldcol[CPL];
  bool st[CPL], hcol[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    const int col = col0 + lane * CPL + k;
    ldcol[k] = min(max(col, 0), P1 - 1);
    st[k] = col >= c_first && col < c_first + C && col < I1 + R;
    hcol[k] = col < R || col >= I1 + R;
  }

  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);

  T win[BT][U][CPL];
  T ext[BT][U][NX];
  T stage[PF > 0 ? PF : 1][CPL];
  sfor<BT>([&](auto L) {
    sfor<U>([&](auto S) {
      sfor<CPL>([&](auto K) { win[L][S][K] = T(0); });
      sfor<NX>([&](auto K) { ext[L][S][K] = T(0); });
    });
  });

  auto load_row = [&](T (&v)[CPL], int row) {
    const T* rp = src + static_cast<int64_t>(min(row, P0 - 1)) * P1;
    sfor<CPL>([&](auto K) { v[K] = rp[ldcol[K]]; });
  };
  // Neighbour values of a row held by the adjacent lanes: x[0..R-1] are the
  // last R cells of lane l-1, x[R..2R-1] the first R cells of lane l+1.
  auto exchange = [&](const T (&v)[CPL], T (&x)[NX]) {
    if constexpr (BOX) {
      sfor<R>([&](auto J) {
        x[J] = lane_from_lower(v[CPL - R + J]);
        x[R + J] = lane_from_upper(v[J]);
      });
    }
  };

  const int s_lo = max(0, row_a - BT * R);
  const int s0 = s_lo - s_lo % U;       // step phases line up with window slots
  const int s_end = row_b + BT * R;     // level BT stores row row_b-1 at step s_end-1
  const int niter = (s_end - s0 + NS - 1) / NS;

  if constexpr (PF > 0) sfor<PF>([&](auto J) { load_row(stage[J], s0 + J); });

  for (int it = 0; it < niter; ++it) {
    const int sb = s0 + it * NS;
    sfor<NS>([&](auto PH) {
      constexpr int ph = PH;
      const int s = sb + ph;
      constexpr int sl0 = ph % U;
      if constexpr (PF > 0) {
        sfor<CPL>([&](auto K) { win[0][sl0][K] = stage[ph][K]; });
        load_row(stage[ph], s + PF);
      } else {
        load_row(win[0][sl0], s);
      }
      exchange(win[0][sl0], ext[0][sl0]);

      sfor<BT>([&](auto LI) {
        constexpr int lv = LI + 1;            // level computed here
        constexpr int base = ph - lv * R;     // its output row is s - lv*R
        const T(&w)[U][CPL] = win[lv - 1];
        const T(&x)[U][NX] = ext[lv - 1];
        constexpr int cs = pmod(base, U);     // slot of the centre row
        T out[CPL];

        if constexpr (!BOX) {
          // centre row extended by R cells of each neighbouring lane
          T E[CPL + 2 * R];
          sfor<R>([&](auto J) {
            E[J] = lane_from_lower(w[cs][CPL - R + J]);
            E[R + CPL + J] = lane_from_upper(w[cs][J]);
          });
          sfor<CPL>([&](auto K) { E[R + K] = w[cs][K]; });
          sfor<CPL>([&](auto K) {
            // canonical order: (-R,0)..(-1,0), (0,-R)..(0,R), (1,0)..(R,0)
            T acc = cf.c[0] * w[pmod(base - R, U)][K];
            sfor<R - 1>([&](auto D) {
              acc = fmadd(cf.c[1 + D], w[pmod(base - R + 1 + D, U)][K], acc);
            });
            sfor<2 * R + 1>([&](auto D) { acc = fmadd(cf.c[R + D], E[K + D], acc); });
            sfor<R>([&](auto D) {
              acc = fmadd(cf.c[3 * R + 1 + D], w[pmod(base + 1 + D, U)][K], acc);
            });
            out[K] = acc;
          });
        } else {
          // canonical order: d0 = -R..R outer, d1 = -R..R inner
          sfor<CPL>([&](auto K) {
            T acc;
            sfor<2 * R + 1>([&](auto D0) {
              constexpr int sl = pmod(base - R + D0, U);
              sfor<2 * R + 1>([&](auto D1) {
                constexpr int m = K + D1;     // index into [left R | own CPL | right R]
                T v;
                if constexpr (m < R) {
                  v = x[sl][m];
                } else if constexpr (m < R + CPL) {
                  v = w[sl][m - R];
                } else {
                  v = x[sl][m - CPL];
                }
                constexpr int ci = D0 * (2 * R + 1) + D1;
                if constexpr (ci == 0) {
                  acc = cf.c[0] * v;
                } else {
                  acc = fmadd(cf.c[ci], v, acc);
                }
              });
            });
            out[K] = acc;
          });
        }

        if constexpr (EDGE) {
          // fixed boundary: rows 0..R-1 and I0+R.., columns 0..R-1 and I1+R..
          const int q = s - lv * R;
          if (q < R || q >= I0 + R) {
            sfor<CPL>([&](auto K) { out[K] = w[cs][K]; });
          } else {
            sfor<CPL>([&](auto K) { out[K] = hcol[K] ? w[cs][K] : out[K]; });
          }
        }

        if constexpr (lv < BT) {
          sfor<CPL>([&](auto K) { win[lv][cs][K] = out[K]; });
          exchange(win[lv][cs], ext[lv][cs]);
        } else {
          const int q = s - BT * R;
          if (q >= row_a && q < row_b) {
            T* rp = dst + static_cast<int64_t>(q) * P1;
            sfor<CPL>([&](auto K) {
              if (st[K]) rp[ldcol[K]] = out[K];
            });
          }
        }
      });
    });
  }
}

template <typename T, int R, bool BOX, int BT, int CPL, int PFK>
__global__ __launch_bounds__(64 * kWavesPerBlock) void sweep2d_kernel(Sweep2DArgs a,
                                                                    CoefPack<T, npts(2, R, BOX)> cf) {
  constexpr int W = 64 * CPL;
  constexpr int C = W - 2 * BT * R;
  static_assert(R <= CPL, "the lane exchange reaches one neighbouring lane only");
  static_assert(C >= 1, "tile narrower than its overlap");
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wid = lb * kWavesPerBlock + wib;
  if (wid >= a.nwaves) return;
  const int lane = threadIdx.x & 63;
  const int tile = wid % a.ntiles;
  const int chunk = wid / a.ntiles;

  const int P1 = a.I1 + 2 * R;
  const int col0 = R + tile * C - BT * R;
  const int row_a = R + chunk * a.chunk;
  const int row_b = min(row_a + a.chunk, a.I0 + R);
  const bool edge = col0 < 0 || col0 + W > P1 || row_a - (BT - 1) * R < R ||
                    row_b + (BT - 1) * R > a.I0 + R;
  if (edge)
    sweep2d_body<T, R, BOX, BT, CPL, PFK, true>(a, cf, lane, tile, chunk);
  else
    sweep2d_body<T, R, BOX, BT, CPL, PFK, false>(a, cf, lane, tile, chunk);
}

template <typename T, int R, bool BOX, int BT, int CPL, int PFK>
hipError_t launch_sweep2d(const Round2D& rd) {
  constexpr int NP = npts(2, R, BOX);
  constexpr int C = 64 * CPL - 2 * BT * R;
  CoefPack<T, NP> cf;
  for (int k = 0; k < NP; ++k) cf.c[k] = static_cast<T>(rd.coeffs[k]);
  Sweep2DArgs a;
  a.src = rd.src;
  a.dst = rd.dst;
  a.I0 = rd.I0;
  a.I1 = rd.I1;
  a.chunk = rd.chunk;
  a.ntiles = (rd.I1 + C - 1) / C;
  const int nchunks = (rd.I0 + rd.chunk - 1) / rd.chunk;
  a.nwaves = a.ntiles * nchunks;
  a.pad = 0;
  const int nblk = (a.nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((sweep2d_kernel<T, R, BOX, BT, CPL, PFK>), dim3(nblk), dim3(64 * kWavesPerBlock), 0,
                     rd.stream, a, cf);
  return hipGetLastError();
}

template <typename T, int R, bool BOX, int BT, int CPL, int PFK>
int occupancy_sweep2d() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep2d_kernel<T, R, BOX, BT, CPL, PFK>,
                                                   64 * kWavesPerBlock, 0) != hipSuccess)
    return 0;
  return nb;
}

template <typename T, int R, bool BOX, int BT, int CPL, int PFK>
Kernel2D make_kernel2d() {
  return Kernel2D{&launch_sweep2d<T, R, BOX, BT, CPL, PFK>, &occupancy_sweep2d<T, R, BOX, BT, CPL, PFK>, CPL, BT,
                  64 * CPL};
}

}  // namespace s5d
