// 3D temporally blocked stencil sweep for gfx950 (device code + launcher).
//
// Method (AN5D "Execution Model", "Optimizations", "Division of Streaming
// Dimension"): a tile of the plane normal to the streaming axis 0 walks along
// axis 0 carrying BT fused time levels; level T emits the plane T*R planes
// behind the plane just loaded.  The tile overlaps its neighbours by BT*R
// cells on every side of both in-plane axes; only its compute region is
// stored.  Axis 0 is cut into stream blocks of `chunk` planes.
//
// MI355X mapping:
//  * one workgroup of NW waves is one tile of B1 = NW*M rows (axis 1) by
//    B2 = 64*CPL columns (axis 2); wave w holds rows w*M .. w*M+M-1 and lane
//    l holds CPL consecutive columns of each of them, all in registers;
//  * axis-2 neighbours that live in another lane come from DPP whole-wave
//    shifts (as in the 2D kernel); axis-1 neighbours that live in another
//    wave come from a double-buffered LDS exchange of the R edge rows of each
//    wave: one barrier per level and step, as the paper's double-buffered
//    shared memory;
//  * partial sums along axis 0: an arriving plane is pushed into the 2R+1
//    output planes it feeds, so a level holds 2R accumulator planes; each
//    output is summed in canonical (d0, d1, d2) order;
//  * the boundary (width R on every face) keeps its values: every level also
//    keeps its last R arriving planes (a fixed-slot delay line), and in tiles
//    or stream blocks that touch the boundary the emitted value of a boundary
//    cell is taken from there -- it is the value that cell had one level
//    earlier, which by induction is its original value.
#pragma once

#include "kcommon.h"

namespace s5d {

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int M, int NW, int NR, bool EDGE>
__device__ __forceinline__ void sweep3d_body(const Sweep3DArgs& a, const CoefPack<T, ncoef(3, R, BOX, EXPR)>& cf,
                                             int w, int lane, int t1, int t2, int chunk,
                                             T (*xbuf)[NW][2 * R][64 * CPL]) {
  static_assert(R <= M, "an edge-row exchange reaches one neighbouring wave only");
  constexpr int NA = 2 * R;          // pending output planes per level
  constexpr int NS = lcm_i(NA, NR);  // steps per unrolled iteration
  constexpr int B1 = NW * M;         // tile rows (axis 1)
  constexpr int B2 = 64 * CPL;       // tile columns (axis 2)
  constexpr int C1 = B1 - 2 * BT * R;
  constexpr int LO2 = overlap_left(BT, R, sizeof(T));  // column overlap on the left
  constexpr int C2 = compute_width(B2, BT, R, sizeof(T));
  constexpr bool WHOLE = LO2 % CPL == 0 && C2 % CPL == 0;  // compute columns are whole lanes
  constexpr int XR = M + 2 * R;      // extended rows: R from wave w-1 | own M | R from wave w+1
  constexpr int XL = CPL + 2 * R;    // extended columns
  constexpr uint32_t WB = sizeof(T);
  using RowV = T __attribute__((ext_vector_type(CPL)));

  const int I0 = a.I0, I1 = a.I1, I2 = a.I2;
  const int P0 = I0 + 2 * R, P1 = I1 + 2 * R, P2 = I2 + 2 * R;
  const int r_first = R + t1 * C1, c_first = R + t2 * C2;
  const int row0 = r_first - BT * R + w * M;  // first row held by this wave
  const int colL = c_first - LO2 + lane * CPL;
  const int pl_a = R + chunk * a.chunk;        // output planes of this stream block
  const int pl_b = min(pl_a + a.chunk, I0 + R);

  // per-row store validity (wave-uniform) and per-cell column masks
  bool row_st[M], row_hal[M];
  sfor<M>([&](auto MI) S5D_INL {
    const int i = row0 + MI;
    row_st[MI] = i >= r_first && i < r_first + C1 && i < I1 + R;
    row_hal[MI] = i < R || i >= I1 + R;
  });
  uint32_t soff[CPL], loff[CPL];
  bool hcol[CPL];
  bool full = true;
  sfor<CPL>([&](auto K) S5D_INL {
    const int col = colL + K;
    const bool st = col >= c_first && col < c_first + C2 && col < I2 + R;
    full = full && st;
    soff[K] = st ? static_cast<uint32_t>(col) * WB : kOutOfRange;
    loff[K] = (col >= 0 && col < P2) ? static_cast<uint32_t>(col) * WB : kOutOfRange;
    hcol[K] = col < R || col >= I2 + R;
  });
  const uint32_t vstore = full ? static_cast<uint32_t>(colL) * WB : kOutOfRange;
  if (full) sfor<CPL>([&](auto K) S5D_INL { soff[K] = kOutOfRange; });

  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);

  auto row_ptr = [&](const T* base, int p, int i) S5D_INL {
    return base + (static_cast<int64_t>(p) * P1 + i) * P2;
  };
  auto load_plane = [&](RowV (&v)[M], int p) S5D_INL {
    sfor<M>([&](auto MI) S5D_INL {
      const int i = row0 + MI;
      if constexpr (EDGE) {
        const bool in = p < P0 && i >= 0 && i < P1;
        const auto rs = make_rsrc(row_ptr(src, in ? p : 0, in ? i : 0), in ? static_cast<uint32_t>(P2) * WB : 0u);
        sfor<CPL>([&](auto K) S5D_INL {
          T t;
          buf_load(t, rs, loff[K]);
          v[MI][+K] = t;
        });
      } else {
        const LaneVec<T, CPL> lv = *reinterpret_cast<const LaneVec<T, CPL>*>(row_ptr(src, min(p, P0 - 1), i) + colL);
        sfor<CPL>([&](auto K) S5D_INL { v[MI][+K] = lv.v[K]; });
      }
    });
  };

  // Folded lane shifts (float32 stars): the centre row's axis-2 terms that
  // read a neighbouring lane take it through the FMA's DPP operand, with the
  // coefficient in a VGPR.
  constexpr bool FOLD = ACC == 0 && std::is_same_v<T, float> && !BOX;
  T cv[2 * R + 1];
  if constexpr (FOLD)
    sfor<2 * R + 1>([&](auto D2) S5D_INL {
      if constexpr (decltype(D2)::value != R) cv[D2] = to_vgpr(cf.c[2 * R + D2]);
    });
  // the same for the 27-point box: every row's axis-2 terms at d2 = -1, +1
  constexpr bool FOLDB = ACC == 0 && std::is_same_v<T, float> && BOX && R == 1;
  T cvb[FOLDB ? 27 : 1];
  if constexpr (FOLDB)
    sfor<27>([&](auto CI) S5D_INL {
      if constexpr (decltype(CI)::value % 3 != 1) cvb[CI] = to_vgpr(cf.c[CI]);
    });

  // Only levels below BT pass values on: the last level is stored, and the
  // boundary is never stored, so it needs no pass-through.
  constexpr int NCEN = BT > 1 ? BT - 1 : 1;
  Accum<T, ACC> acc[BT][NA][M][CPL];
  T cen[NCEN][R][M][CPL];  // last R arriving planes of levels 1..BT-1 (boundary pass-through)
  RowV ring[NR][M];
  sfor<BT>([&](auto L) S5D_INL {
    sfor<NA>([&](auto S) S5D_INL {
      sfor<M>([&](auto MI) S5D_INL { sfor<CPL>([&](auto K) S5D_INL { acc[L][S][MI][K].zero(); }); });
    });
    if constexpr (EDGE && L < NCEN)
      sfor<R>([&](auto S) S5D_INL {
        sfor<M>([&](auto MI) S5D_INL { sfor<CPL>([&](auto K) S5D_INL { cen[L][S][MI][K] = T(0); }); });
      });
  });

  const int s_lo = max(0, pl_a - BT * R);
  const int s0 = s_lo - s_lo % NS;
  const int s_end = pl_b + BT * R;
  const int niter = (s_end - s0 + NS - 1) / NS;

  sfor<NR - 1>([&](auto J) S5D_INL {
    load_plane(ring[J], s0 + J);
    __builtin_amdgcn_sched_barrier(0);
  });

  auto iteration = [&](const int sb) S5D_INL {
    sfor<NS>([&](auto PH) S5D_INL {
      const int s = sb + PH;
      load_plane(ring[pmod(PH - 1, NR)], s + NR - 1);
      __builtin_amdgcn_sched_barrier(0);
      T cur[M][CPL];
      sfor<M>([&](auto MI) S5D_INL { sfor<CPL>([&](auto K) S5D_INL { cur[MI][K] = ring[PH % NR][MI][+K]; }); });

      sfor<BT>([&](auto LI) S5D_INL {
        constexpr int lv = LI + 1;                       // level receiving plane p = s-(lv-1)*R
        constexpr int pm = pmod(PH - (lv - 1) * R, NA);  // p mod 2R
        constexpr int so = pmod(pm + R, NA);             // slot of planes p-R and p+R
        constexpr int par = (PH * BT + LI) & 1;          // exchange buffer (NS*BT is even)
        constexpr int cs = PH % R;                       // delay-line slot of planes p and p-R
        Accum<T, ACC>(&A)[NA][M][CPL] = acc[LI];

        // axis-1 exchange: publish the R first and R last rows, read the
        // neighbouring waves' ones (the tile's outer waves read their own:
        // those rows lie in the overlap that the valid region discards)
        sfor<R>([&](auto J) S5D_INL {
          sfor<CPL>([&](auto K) S5D_INL {
            xbuf[par][w][J][lane * CPL + K] = cur[J][K];
            xbuf[par][w][R + J][lane * CPL + K] = cur[M - R + J][K];
          });
        });
        __syncthreads();
        const int wu = w > 0 ? w - 1 : w, wd = w + 1 < NW ? w + 1 : w;
        T X[XR][XL];  // extended plane around this wave's rows
        sfor<R>([&](auto J) S5D_INL {
          const LaneVec<T, CPL> up = *reinterpret_cast<const LaneVec<T, CPL>*>(&xbuf[par][wu][R + J][lane * CPL]);
          const LaneVec<T, CPL> dn = *reinterpret_cast<const LaneVec<T, CPL>*>(&xbuf[par][wd][J][lane * CPL]);
          sfor<CPL>([&](auto K) S5D_INL {
            X[J][R + K] = up.v[K];
            X[R + M + J][R + K] = dn.v[K];
          });
        });
        sfor<M>([&](auto MI) S5D_INL { sfor<CPL>([&](auto K) S5D_INL { X[R + MI][R + K] = cur[MI][K]; }); });
        // axis-2 extension: all rows for box stencils, own rows for star ones
        sfor<XR>([&](auto XI) S5D_INL {
          if constexpr (BOX || (XI >= R && XI < R + M)) {
            sfor<R>([&](auto J) S5D_INL {
              X[XI][J] = lane_from_lower(X[XI][CPL + J]);
              X[XI][R + CPL + J] = lane_from_upper(X[XI][R + J]);
            });
          }
        });

        // contribution of the arriving plane to the output d0 planes before it
        auto add_plane = [&](auto D0, Accum<T, ACC>& acc_k, auto MI, auto K, auto FIRST) S5D_INL {
          constexpr int d0 = D0;
          constexpr bool first = FIRST;
          if constexpr (BOX) {
            sfor<2 * R + 1>([&](auto D1) S5D_INL {
              sfor<2 * R + 1>([&](auto D2) S5D_INL {
                constexpr int ci = ((d0 + R) * (2 * R + 1) + D1) * (2 * R + 1) + D2;
                constexpr int e = decltype(K)::value + decltype(D2)::value;  // extended column
                constexpr bool lead = first && D1 == 0 && D2 == 0;
                if constexpr (FOLDB && (e < R || e >= R + CPL)) {
                  constexpr bool shr = e < R;
                  constexpr int src = shr ? CPL - R + e : e - R - CPL;
                  if constexpr (lead) acc_k.s = mul_dpp<shr>(X[MI + D1][R + src], cvb[ci]);
                  else acc_k.s = fma_dpp<shr>(acc_k.s, X[MI + D1][R + src], cvb[ci]);
                } else {
                  const T v = X[MI + D1][K + D2];
                  if constexpr (lead) acc_k.first(cf.c[ci], v);
                  else acc_k.add(cf.c[ci], v);
                }
              });
            });
          } else if constexpr (d0 != 0) {
            // (d0,0,0): indices 0..R-1 before the centre plane, 5R+1.. after
            constexpr int ci = d0 < 0 ? d0 + R : 5 * R + d0;
            if constexpr (first) acc_k.first(cf.c[ci], X[R + MI][R + K]);
            else acc_k.add(cf.c[ci], X[R + MI][R + K]);
          } else {
            // centre plane: (0,d1,0) d1<0, then (0,0,d2), then (0,d1,0) d1>0
            sfor<R>([&](auto J) S5D_INL { acc_k.add(cf.c[R + J], X[MI + J][R + K]); });
            sfor<2 * R + 1>([&](auto D2) S5D_INL {
              constexpr int e = decltype(K)::value + decltype(D2)::value;  // extended column
              if constexpr (FOLD && (e < R || e >= R + CPL)) {
                constexpr bool shr = e < R;  // from lane l-1, else lane l+1
                constexpr int src = shr ? CPL - R + e : e - R - CPL;
                acc_k.s = fma_dpp<shr>(acc_k.s, X[R + MI][R + src], cv[D2]);
              } else {
                acc_k.add(cf.c[2 * R + D2], X[R + MI][K + D2]);
              }
            });
            sfor<R>([&](auto J) S5D_INL { acc_k.add(cf.c[4 * R + 1 + J], X[R + MI + 1 + J][R + K]); });
          }
        };

        T out[M][CPL];
        sfor<M>([&](auto MI) S5D_INL {
          sfor<CPL>([&](auto K) S5D_INL {
            Accum<T, ACC> v = A[so][MI][K];
            add_plane(ic<R>{}, v, MI, K, std::false_type{});
            out[MI][K] = finish<EXPR>(v.value(), cf);
          });
        });
        sfor<M>([&](auto MI) S5D_INL {
          sfor<CPL>([&](auto K) S5D_INL { add_plane(ic<-R>{}, A[so][MI][K], MI, K, std::true_type{}); });
        });
        sfor<2 * R - 1>([&](auto J) S5D_INL {
          constexpr int d0 = -R + 1 + J;
          constexpr int sl = pmod(pm - d0, NA);
          sfor<M>([&](auto MI) S5D_INL {
            sfor<CPL>([&](auto K) S5D_INL { add_plane(ic<d0>{}, A[sl][MI][K], MI, K, std::false_type{}); });
          });
        });

        if constexpr (EDGE && lv < BT) {
          // output o = p - R: boundary cells take the value plane o had when it
          // arrived here (R steps ago); then the slot records plane p
          const int o = s - lv * R;
          const bool pl_hal = o < R || o >= I0 + R;
          sfor<M>([&](auto MI) S5D_INL {
            const bool rh = pl_hal || row_hal[MI];
            sfor<CPL>([&](auto K) S5D_INL {
              out[MI][K] = (rh || hcol[K]) ? cen[LI][cs][MI][K] : out[MI][K];
              cen[LI][cs][MI][K] = cur[MI][K];
            });
          });
        }

        if constexpr (lv < BT) {
          sfor<M>([&](auto MI) S5D_INL { sfor<CPL>([&](auto K) S5D_INL { cur[MI][K] = out[MI][K]; }); });
        } else {
          const int o = s - BT * R;
          const bool keep_pl = o >= pl_a && o < pl_b;
          sfor<M>([&](auto MI) S5D_INL {
            const bool keep = keep_pl && row_st[MI];
            const auto rs = make_rsrc(row_ptr(dst, keep ? o : pl_a, keep ? row0 + MI : r_first),
                                      keep ? static_cast<uint32_t>(P2) * WB : 0u);
            buf_store_lane(out[MI], rs, vstore);
            // lanes straddling the compute region's edge store cell by cell
            if constexpr (EDGE || !WHOLE) sfor<CPL>([&](auto K) S5D_INL { buf_store(out[MI][K], rs, soff[K]); });
          });
        }
      });
    });
  };
  iteration(s0);
  for (int it = 1; it < niter; ++it) iteration(s0 + it * NS);
}

// Workgroup lb of one grid's launch: one (tile, stream block) pair.
template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int M, int NW, int NR>
__device__ __forceinline__ void sweep3d_block(const Sweep3DArgs& a, const CoefPack<T, ncoef(3, R, BOX, EXPR)>& cf, int lb,
                                              T (&xbuf)[2][NW][2 * R][64 * CPL]) {
  constexpr int B1 = NW * M, B2 = 64 * CPL;
  constexpr int C1 = B1 - 2 * BT * R, C2 = compute_width(B2, BT, R, sizeof(T));
  static_assert(R <= CPL, "the lane exchange reaches one neighbouring lane only");
  static_assert(C1 >= 1 && C2 >= 1, "tile narrower than its overlap");
  const int t2 = lb % a.nt2;
  const int t1 = (lb / a.nt2) % a.nt1;
  const int chunk = lb / (a.nt2 * a.nt1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;

  const int P1 = a.I1 + 2 * R, P2 = a.I2 + 2 * R;
  const int row0 = R + t1 * C1 - BT * R, col0 = R + t2 * C2 - overlap_left(BT, R, sizeof(T));
  const int pl_a = R + chunk * a.chunk;
  const int pl_b = min(pl_a + a.chunk, a.I0 + R);
  const bool edge = row0 < 0 || row0 + B1 > P1 || col0 < 0 || col0 + B2 > P2 ||
                    pl_a - (BT - 1) * R < R || pl_b + (BT - 1) * R > a.I0 + R;
  if (edge)
    sweep3d_body<T, ACC, EXPR, R, BOX, BT, CPL, M, NW, NR, true>(a, cf, w, lane, t1, t2, chunk, xbuf);
  else
    sweep3d_body<T, ACC, EXPR, R, BOX, BT, CPL, M, NW, NR, false>(a, cf, w, lane, t1, t2, chunk, xbuf);
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int M, int NW, int NR>
__global__ __launch_bounds__(64 * NW) void sweep3d_kernel(Sweep3DArgs a, CoefPack<T, ncoef(3, R, BOX, EXPR)> cf) {
  __shared__ T xbuf[2][NW][2 * R][64 * CPL];
  sweep3d_block<T, ACC, EXPR, R, BOX, BT, CPL, M, NW, NR>(a, cf, xcd_logical_block(blockIdx.x, gridDim.x), xbuf);
}

// One grid of a batched launch: its geometry and coefficients.
template <typename T, int NP>
struct alignas(16) Item3D {
  Sweep3DArgs a;
  CoefPack<T, NP> cf;
};

// Batched launch: workgroup b runs workgroup map[b].block of grid map[b].item.
template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int M, int NW, int NR>
__global__ __launch_bounds__(64 * NW) void sweep3d_batch_kernel(const Item3D<T, ncoef(3, R, BOX, EXPR)>* __restrict__ items,
                                                              const BlockMap* __restrict__ map) {
  __shared__ T xbuf[2][NW][2 * R][64 * CPL];
  const BlockMap m = map[xcd_logical_block(blockIdx.x, gridDim.x)];
  const Item3D<T, ncoef(3, R, BOX, EXPR)>& it = items[__builtin_amdgcn_readfirstlane(m.item)];
  const Sweep3DArgs a = it.a;
  const CoefPack<T, ncoef(3, R, BOX, EXPR)> cf = it.cf;
  sweep3d_block<T, ACC, EXPR, R, BOX, BT, CPL, M, NW, NR>(a, cf, __builtin_amdgcn_readfirstlane(m.block), xbuf);
}

// Geometry of one grid's launch; returns its workgroup count (0 if it does
// not fit a 32-bit grid).
template <typename T, int EXPR, int R, bool BOX, int BT, int CPL, int M, int NW>
int64_t make_args3d(const Round3D& rd, Sweep3DArgs& a, CoefPack<T, ncoef(3, R, BOX, EXPR)>& cf) {
  constexpr int NP = ncoef(3, R, BOX, EXPR);  // the divisor c0 last for EXPR_DIV
  constexpr int C1 = NW * M - 2 * BT * R, C2 = compute_width(64 * CPL, BT, R, sizeof(T));
  for (int k = 0; k < NP; ++k) cf.c[k] = static_cast<T>(rd.coeffs[k]);
  a.src = rd.src;
  a.dst = rd.dst;
  a.I0 = rd.I0;
  a.I1 = rd.I1;
  a.I2 = rd.I2;
  a.chunk = rd.chunk;
  a.nt1 = (rd.I1 + C1 - 1) / C1;
  a.nt2 = (rd.I2 + C2 - 1) / C2;
  const int nchunks = (rd.I0 + rd.chunk - 1) / rd.chunk;
  const int64_t nblk = static_cast<int64_t>(a.nt1) * a.nt2 * nchunks;
  return nblk > INT32_MAX ? 0 : nblk;
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int M, int NW, int NR>
hipError_t launch_sweep3d(const Round3D& rd) {
  Sweep3DArgs a;
  CoefPack<T, ncoef(3, R, BOX, EXPR)> cf;
  const int64_t nblk = make_args3d<T, EXPR, R, BOX, BT, CPL, M, NW>(rd, a, cf);
  if (nblk == 0) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((sweep3d_kernel<T, ACC, EXPR, R, BOX, BT, CPL, M, NW, NR>), dim3(static_cast<unsigned>(nblk)),
                     dim3(64 * NW), 0, rd.stream, a, cf);
  return hipGetLastError();
}

template <typename T, int EXPR, int R, bool BOX, int BT, int CPL, int M, int NW>
int fill_item3d(void* item, const Round3D& rd) {
  Item3D<T, ncoef(3, R, BOX, EXPR)> it;
  const int64_t nblk = make_args3d<T, EXPR, R, BOX, BT, CPL, M, NW>(rd, it.a, it.cf);
  __builtin_memcpy(item, &it, sizeof(it));
  return static_cast<int>(nblk);
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int M, int NW, int NR>
hipError_t launch_batch3d(const void* items, const BlockMap* map, int nblocks, hipStream_t stream) {
  hipLaunchKernelGGL((sweep3d_batch_kernel<T, ACC, EXPR, R, BOX, BT, CPL, M, NW, NR>), dim3(nblocks), dim3(64 * NW), 0,
                     stream, static_cast<const Item3D<T, ncoef(3, R, BOX, EXPR)>*>(items), map);
  return hipGetLastError();
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int M, int NW, int NR>
int occupancy_sweep3d() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep3d_kernel<T, ACC, EXPR, R, BOX, BT, CPL, M, NW, NR>, 64 * NW,
                                                   0) != hipSuccess)
    return 0;
  return nb;
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int M, int NW, int NR>
Kernel3D make_kernel3d() {
  return Kernel3D{&launch_sweep3d<T, ACC, EXPR, R, BOX, BT, CPL, M, NW, NR>,
                  &occupancy_sweep3d<T, ACC, EXPR, R, BOX, BT, CPL, M, NW, NR>,
                  CPL,
                  M,
                  NW,
                  BT,
                  &fill_item3d<T, EXPR, R, BOX, BT, CPL, M, NW>,
                  &launch_batch3d<T, ACC, EXPR, R, BOX, BT, CPL, M, NW, NR>,
                  static_cast<int>(sizeof(Item3D<T, ncoef(3, R, BOX, EXPR)>))};
}

}  // namespace s5d
