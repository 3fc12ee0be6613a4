// 2D temporally blocked sweep for stencils that are not a fixed weighted sum
// of the neighbours (device code + launcher): gradient2d, whose update is
// non-linear in the cell values (AN5D Table 3), and stencils whose weights
// differ from cell to cell (multi-array input).
//
// Method (AN5D "Execution Model", the case Table 1 calls "Otherwise": a cell
// can only be computed once all 2R+1 rows it reads are present, so partial
// sums do not apply): as in the associative sweep, a tile streams along axis
// 0 and carries BT fused time levels; level L emits the row L*R rows behind
// the row just loaded, the tile overlaps its neighbours by BT*R columns and
// only its compute region is stored.  Each level keeps a window of the last
// 2R+1 rows it received, in fixed register slots (row p in slot p mod 2R+1;
// the stream loop is unrolled by a multiple of 2R+1), and computes its output
// row from the full window when the newest row arrives.
//
// MI355X mapping: one wave64 is one tile and lane l owns CPL consecutive
// columns, so every row of a window is a register tuple per lane; in-row
// neighbours in another lane come from DPP whole-wave shifts.  The paper
// keeps the 1+2R rows of the "Otherwise" case in shared memory; here they
// never leave the registers and the tile needs no LDS except the EDGE waves'
// stash of boundary columns (as in the associative sweep).
//
// Operations (OP):
//  OP_GRADIENT (star, R = 1): out = cc*f + 1/sqrt(c0 + sum_n (f - f_n)^2)
//    over the four axis neighbours in canonical order (-1,0), (0,-1), (0,1),
//    (1,0); every operation is rounded on its own (no contraction), so the
//    result is the IEEE evaluation of that expression in that order.
//  OP_VARCOEF: out = sum_k C[k][o] * A[o + o_k] in canonical offset order, one
//    fused multiply-add per term after the first product; C is n arrays of
//    the interior's extents (weight k of all cells first), read through
//    per-row buffer descriptors (rows and columns outside the interior read
//    0, and those outputs are replaced by the fixed boundary or discarded).
#pragma once

#include "sweep2d.h"  // EdgeStash, blocks2d and the shared helpers

namespace s5d {

enum { OP_GRADIENT = 0, OP_VARCOEF = 1 };

// Coefficients of a window sweep: (cc, c0) for gradient2d; none for the
// variable-coefficient sweep (its weights come from the field array).
template <typename T, int OP>
struct WinCoef {
  T c[OP == OP_GRADIENT ? 2 : 1];
};

struct SweepW2DArgs {
  Sweep2DArgs a;
  const void* fields;  // OP_VARCOEF: n_points arrays of I0 x I1 weights
};

template <typename T, int OP, int R, bool BOX, int BT, int CPL, int NR, bool EDGE>
__device__ __forceinline__ void sweepw2d_body(const SweepW2DArgs& wa, const WinCoef<T, OP>& cf, int lane,
                                              int tile, int row_a, int row_b, EdgeStash<T, R, BT, CPL>* stash) {
  constexpr int NWIN = 2 * R + 1;     // rows in a level's window
  constexpr int NS = lcm_i(NWIN, NR); // steps per unrolled iteration
  constexpr int W = 64 * CPL;
  constexpr int LO = overlap_left(BT, R, sizeof(T));
  constexpr int C = compute_width(W, BT, R, sizeof(T));
  constexpr bool WHOLE = LO % CPL == 0 && C % CPL == 0;
  constexpr int MCOL = BT * R + 1;
  constexpr int XL = CPL + 2 * R;
  constexpr int NP = npts(2, R, BOX);
  constexpr uint32_t WB = sizeof(T);
  static_assert(OP != OP_GRADIENT || (R == 1 && !BOX), "gradient2d is the radius-1 star");

  const Sweep2DArgs& a = wa.a;
  const int I0 = a.I0, I1 = a.I1;
  const int P0 = I0 + 2 * R, P1 = I1 + 2 * R;
  const int c_first = R + tile * C;
  const int col0 = c_first - LO;
  const int colL = col0 + lane * CPL;

  uint32_t soff[CPL];
  bool full = true;
  sfor<CPL>([&](auto K) S5D_INL {
    const int col = colL + K;
    const bool st = col >= c_first && col < c_first + C && col < I1 + R;
    full = full && st;
    soff[K] = st ? static_cast<uint32_t>(col) * WB : kOutOfRange;
  });
  const uint32_t vstore = full ? static_cast<uint32_t>(colL) * WB : kOutOfRange;
  if (full) sfor<CPL>([&](auto K) S5D_INL { soff[K] = kOutOfRange; });
  uint32_t loff[CPL];
  bool hcol[CPL];
  int hl = -1;
  if constexpr (EDGE) {
    bool left = false, right = false;
    sfor<CPL>([&](auto K) S5D_INL {
      const int col = colL + K;
      loff[K] = (col >= 0 && col < P1) ? static_cast<uint32_t>(col) * WB : kOutOfRange;
      const bool l = col >= 0 && col < R, r = col >= I1 + R && col < P1;
      hcol[K] = l || r;
      left |= l;
      right |= r;
    });
    const int lL = (0 - col0) / CPL;
    const int lR = (I1 + R - col0) / CPL;
    if (left) hl = lane - lL;
    else if (right) hl = 2 + lane - lR;
  }
  // weight-field columns: interior column col - R of each row
  uint32_t foff[CPL];
  if constexpr (OP == OP_VARCOEF)
    sfor<CPL>([&](auto K) S5D_INL {
      const int col = colL + K;
      foff[K] = (col >= R && col < I1 + R) ? static_cast<uint32_t>(col - R) * WB : kOutOfRange;
    });

  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);
  const T* __restrict__ fld = static_cast<const T*>(wa.fields);

  auto load_row = [&](T (&v)[CPL], int row) S5D_INL {
    if constexpr (EDGE) {
      const auto rs = make_rsrc(src + static_cast<int64_t>(min(row, P0)) * P1,
                                row < P0 ? static_cast<uint32_t>(P1) * WB : 0u);
      sfor<CPL>([&](auto K) S5D_INL { buf_load(v[K], rs, loff[K]); });
    } else {
      const T* rp = src + static_cast<int64_t>(min(row, P0 - 1)) * P1 + colL;
      const LaneVec<T, CPL> lv = *reinterpret_cast<const LaneVec<T, CPL>*>(rp);
      sfor<CPL>([&](auto K) S5D_INL { v[K] = lv.v[K]; });
    }
  };

  using RowV = T __attribute__((ext_vector_type(CPL)));
  RowV ringv[NR];
  T win[BT][NWIN][CPL];
  sfor<BT>([&](auto L) S5D_INL {
    sfor<NWIN>([&](auto S) S5D_INL { sfor<CPL>([&](auto K) S5D_INL { win[L][S][K] = T(0); }); });
  });

  const int s_lo = max(0, row_a - BT * R);
  const int s0 = s_lo - s_lo % NS;
  const int s_end = row_b + BT * R;
  const int niter = (s_end - s0 + NS - 1) / NS;

  auto load_vec = [&](RowV& v, int row) S5D_INL {
    T t[CPL];
    load_row(t, row);
    sfor<CPL>([&](auto K) S5D_INL { v[+K] = t[K]; });
  };
  sfor<NR - 1>([&](auto J) S5D_INL {
    load_vec(ringv[J], s0 + J);
    __builtin_amdgcn_sched_barrier(0);
  });

  // one output cell of a level from its window; o is the output row
  auto extend = [&](const T (&row)[CPL], T (&E)[XL]) S5D_INL {
    sfor<CPL>([&](auto K) S5D_INL { E[R + K] = row[K]; });
    sfor<R>([&](auto J) S5D_INL {
      E[J] = lane_from_lower(row[CPL - R + J]);
      E[R + CPL + J] = lane_from_upper(row[J]);
    });
  };

  auto iteration = [&](const int sb) S5D_INL {
    sfor<NS>([&](auto PH) S5D_INL {
      const int s = sb + PH;
      load_vec(ringv[pmod(PH - 1, NR)], s + NR - 1);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (EDGE) {
        if (hl >= 0) sfor<CPL>([&](auto K) S5D_INL { stash->cols[s % MCOL][hl][K] = ringv[PH % NR][+K]; });
      }
      T cur[CPL];
      sfor<CPL>([&](auto K) S5D_INL { cur[K] = ringv[PH % NR][+K]; });

      sfor<BT>([&](auto LI) S5D_INL {
        constexpr int lv = LI + 1;                          // level receiving row p = s - (lv-1)*R
        constexpr int pw = pmod(PH - (lv - 1) * R, NWIN);   // window slot of p
        T(&wn)[NWIN][CPL] = win[LI];
        sfor<CPL>([&](auto K) S5D_INL { wn[pw][K] = cur[K]; });
        const int o = s - lv * R;  // output row of this level
        // window slot of row o + d0
#define S5D_WSLOT(d0) pmod(pw - R + (d0), NWIN)

        T out[CPL];
        if constexpr (OP == OP_GRADIENT) {
          T E[XL];
          extend(wn[S5D_WSLOT(0)], E);
          constexpr int s_up = S5D_WSLOT(-1), s_dn = S5D_WSLOT(1);
          sfor<CPL>([&](auto K) S5D_INL {
#pragma clang fp contract(off)
            const T f = E[R + K];
            T s2 = cf.c[1];
            T d = f - wn[s_up][K];
            s2 = s2 + d * d;
            d = f - E[R + K - 1];
            s2 = s2 + d * d;
            d = f - E[R + K + 1];
            s2 = s2 + d * d;
            d = f - wn[s_dn][K];
            s2 = s2 + d * d;
            const T root = ieee_sqrt(s2);
            const T q = T(1) / root;
            out[K] = cf.c[0] * f + q;
          });
        } else {
          // the weights of output row o: NP rows of the field (row o - R of
          // the interior), every lane loading its CPL columns
          const bool orow = o >= R && o < I0 + R;
          T wgt[NP][CPL];
          sfor<NP>([&](auto KI) S5D_INL {
            const auto rs = make_rsrc(fld + (static_cast<int64_t>(KI) * I0 + (orow ? o - R : 0)) * I1,
                                      orow ? static_cast<uint32_t>(I1) * WB : 0u);
            sfor<CPL>([&](auto K) S5D_INL { buf_load(wgt[KI][K], rs, foff[K]); });
          });
          T E[2 * R + 1][XL];
          sfor<2 * R + 1>([&](auto D) S5D_INL {
            if constexpr (BOX || D == R) extend(wn[S5D_WSLOT(D - R)], E[D]);
          });
          sfor<CPL>([&](auto K) S5D_INL {
            T acc = T(0);
            sfor<2 * R + 1>([&](auto D0) S5D_INL {
              sfor<2 * R + 1>([&](auto D1) S5D_INL {
                constexpr int d0 = D0 - R, d1 = D1 - R;
                if constexpr (BOX || d0 == 0 || d1 == 0) {
                  // canonical index of offset (d0, d1)
                  constexpr int ki = BOX ? D0 * (2 * R + 1) + D1
                                         : (d0 < 0 ? D0 : (d0 > 0 ? 3 * R + d0 : R + D1));
                  T x;
                  if constexpr (BOX || d0 == 0) x = E[D0][K + D1];
                  else x = wn[S5D_WSLOT(d0)][K];
                  if constexpr (ki == 0) acc = wgt[0][K] * x;
                  else acc = fmadd(wgt[ki][K], x, acc);
                }
              });
            });
            out[K] = acc;
          });
        }
#undef S5D_WSLOT

        if constexpr (EDGE && lv < BT) {
          if (o < R || o >= I0 + R) {
            if (o >= 0 && o < P0) load_row(out, o);
          } else {
            const LaneVec<T, CPL> hv = *reinterpret_cast<const LaneVec<T, CPL>*>(
                stash->cols[o % MCOL][hl < 0 ? 0 : hl]);
            sfor<CPL>([&](auto K) S5D_INL { out[K] = hcol[K] ? hv.v[K] : out[K]; });
          }
        }

        if constexpr (lv < BT) {
          sfor<CPL>([&](auto K) S5D_INL { cur[K] = out[K]; });
        } else {
          const bool keep = o >= row_a && o < row_b;
          const auto rs = make_rsrc(dst + static_cast<int64_t>(keep ? o : row_a) * P1,
                                    keep ? static_cast<uint32_t>(P1) * WB : 0u);
          buf_store_lane(out, rs, vstore);
          if constexpr (EDGE || !WHOLE) sfor<CPL>([&](auto K) S5D_INL { buf_store(out[K], rs, soff[K]); });
        }
      });
    });
  };
  iteration(s0);
  for (int it = 1; it < niter; ++it) iteration(s0 + it * NS);
}

template <typename T, int OP, int R, bool BOX, int BT, int CPL, int NR>
__global__ __launch_bounds__(64 * kWavesPerBlock) void sweepw2d_kernel(SweepW2DArgs wa, WinCoef<T, OP> cf) {
  __shared__ EdgeStash<T, R, BT, CPL> stash[kWavesPerBlock];
  constexpr int W = 64 * CPL;
  constexpr int LO = overlap_left(BT, R, sizeof(T));
  constexpr int C = compute_width(W, BT, R, sizeof(T));
  static_assert(R <= CPL, "the lane exchange reaches one neighbouring lane only");
  static_assert(C >= 1, "tile narrower than its overlap");
  const Sweep2DArgs& a = wa.a;
  const int lb = blockIdx.x;
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = a.g.nb;
  const int x = lb % nb;
  const int wid = (lb / nb) * kWavesPerBlock + wib;
  if (wid >= a.nwaves) return;
  const int lane = threadIdx.x & 63;
  const int tile = wid % a.ntiles;
  int row_a, row_b;
  band_rows2d(a.g, R, a.I0, x, wid / a.ntiles, row_a, row_b);
  if (row_b <= row_a) return;
  const int P1 = a.I1 + 2 * R;
  const int col0 = R + tile * C - LO;
  const bool edge = col0 < 0 || col0 + W > P1 || row_a - (BT - 1) * R < R || row_b + (BT - 1) * R > a.I0 + R;
  if (edge)
    sweepw2d_body<T, OP, R, BOX, BT, CPL, NR, true>(wa, cf, lane, tile, row_a, row_b, &stash[wib]);
  else
    sweepw2d_body<T, OP, R, BOX, BT, CPL, NR, false>(wa, cf, lane, tile, row_a, row_b, &stash[wib]);
}

template <typename T, int OP, int R, bool BOX, int BT, int CPL, int NR>
hipError_t launch_sweepw2d(const Round2D& rd) {
  constexpr int C = compute_width(64 * CPL, BT, R, sizeof(T));
  SweepW2DArgs wa;
  Sweep2DArgs& a = wa.a;
  a.src = rd.src;
  a.dst = rd.dst;
  a.I0 = rd.I0;
  a.I1 = rd.I1;
  a.g = make_bands2d(rd.I0, rd.chunk);
  a.ntiles = (rd.I1 + C - 1) / C;
  const int64_t nw = static_cast<int64_t>(a.ntiles) * (a.g.n1 + a.g.n2);
  a.nwaves = nw > INT32_MAX / kXcds ? 0 : static_cast<int32_t>(nw);
  if (a.nwaves == 0) return hipErrorInvalidConfiguration;
  wa.fields = rd.fields;
  if (OP == OP_VARCOEF && !rd.fields) return hipErrorInvalidValue;
  WinCoef<T, OP> cf;
  if constexpr (OP == OP_GRADIENT) {
    cf.c[0] = static_cast<T>(rd.coeffs[0]);
    cf.c[1] = static_cast<T>(rd.coeffs[1]);
  } else {
    cf.c[0] = T(0);
  }
  const int nblk = blocks2d(a);
  hipLaunchKernelGGL((sweepw2d_kernel<T, OP, R, BOX, BT, CPL, NR>), dim3(nblk), dim3(64 * kWavesPerBlock), 0,
                     rd.stream, wa, cf);
  return hipGetLastError();
}

template <typename T, int OP, int R, bool BOX, int BT, int CPL, int NR>
int occupancy_sweepw2d() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweepw2d_kernel<T, OP, R, BOX, BT, CPL, NR>,
                                                   64 * kWavesPerBlock, 0) != hipSuccess)
    return 0;
  return nb;
}

// Window kernels have no batched entry point: batches and servers reject
// their plans.
template <typename T, int OP, int R, bool BOX, int BT, int CPL, int NR>
Kernel2D make_kernelw2d() {
  return Kernel2D{&launch_sweepw2d<T, OP, R, BOX, BT, CPL, NR>,
                  &occupancy_sweepw2d<T, OP, R, BOX, BT, CPL, NR>,
                  CPL,
                  BT,
                  64 * CPL,
                  nullptr,
                  nullptr,
                  0};
}

}  // namespace s5d
