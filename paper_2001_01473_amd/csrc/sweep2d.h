// 2D temporally blocked stencil sweep for gfx950 (device code + launcher).
//
// Method (AN5D "Execution Model" and "Optimizations"): a tile of the plane
// normal to the streaming axis (axis 0) walks along axis 0 and carries BT
// computational streams, one per fused time level.  Level T emits the row
// that lies T*R rows behind the row just loaded, so each row is read from HBM
// once and written once per BT time steps.  The tile overlaps its neighbours
// by BT*R columns on each side; the valid width shrinks by 2R per level and
// only the compute region of level BT is stored.  The axis-0 extent is cut
// into stream blocks ("Division of Streaming Dimension"), each of which
// starts BT*R rows early to warm up the levels; blocks are h_SN rows long
// except for a tail of half-length blocks at the end of each XCD's band of
// rows (Bands2D).
//
// MI355X mapping (differs from the paper's CUDA design):
//  * one wave64 is one tile; lane l owns CPL consecutive columns, so the tile
//    is 64*CPL columns wide and needs no shared memory and no barrier: the
//    in-plane neighbours that live in another lane come from DPP whole-wave
//    shifts (wave_shr:1 / wave_shl:1).  Lanes at the tile edge receive
//    meaningless values, which only ever reach the overlap region that the
//    shrinking valid width discards.  For plain float32 stars and 3x3 boxes
//    the shift is folded into the term's FMA (fma_dpp), with the coefficient
//    in a VGPR.
//  * partial sums ("associative" stencils in the paper): a row arriving at
//    level T is pushed at once into the 2R+1 output rows it contributes to,
//    so a level holds only 2R pending accumulator rows and the arriving row is
//    dead after its pushes.  Output row o receives its contributions in the
//    order its source rows arrive, o-R first, so each output is summed in the
//    canonical offset order: (d0, d1) lexicographic, d0 outermost.  The
//    accumulator slot of row o is o mod 2R; the stream loop is unrolled by a
//    multiple of 2R, so every slot is a fixed register ("Register Allocation":
//    no value is ever shifted between registers).
//  * loaded rows sit in a ring of NR register rows (one vector register tuple
//    each; the stream loop is unrolled by lcm(2R, NR)); at step s the slot
//    consumed at step s-1 receives row s+NR-1, so NR-1 rows are in flight.  The first unrolled iteration is peeled so the
//    loop is entered with the same loads and stores outstanding as at its back
//    edge, which lets the compiler wait on exactly the oldest ring row.
//  * fixed boundary (width R on every face): cells of the boundary keep their
//    value at every level (the paper overwrites them with the original value).
//    Only waves whose tile or stream block touches the boundary (EDGE) do this:
//    boundary rows are re-read from the source buffer (never written, and
//    L2-resident since level 0 has just read them); the boundary-column cells
//    of the last BT*R+1 rows are stashed in LDS when level 0 loads them.  EDGE waves read through buffer descriptors, so columns and rows
//    outside the grid read as 0 without a branch; interior waves read whole
//    lane vectors.  Stores go through per-row buffer descriptors: lanes whose
//    cells all lie in the compute region store one vector, the lanes at its
//    edge store cell by cell, and out-of-range offsets turn the unused path
//    and the masked cells into no-ops without a branch.
#pragma once

#include "kcommon.h"

namespace s5d {

// Per-wave LDS stash of the boundary-column cells of the last BT*R+1 rows,
// used by EDGE waves only: lane vectors of the (at most 4) lanes that hold
// boundary columns.
template <typename T, int R, int BT, int CPL>
struct alignas(16) EdgeStash {
  T cols[BT * R + 1][4][CPL];
};

// Coefficients (canonical order) of the in-row terms that read a neighbouring
// lane: the centre row's off-centre points of a star, every column but the
// centre one of a box.
template <int R, bool BOX>
constexpr bool folded_coef2d(int ci) {
  return BOX ? ci % (2 * R + 1) != R : (ci >= R && ci <= 3 * R && ci != 2 * R);
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int NR, bool EDGE>
__device__ __forceinline__ void sweep2d_body(const Sweep2DArgs& a, const CoefPack<T, ncoef(2, R, BOX, EXPR)>& cf,
                                             int lane, int tile, int row_a, int row_b,
                                             EdgeStash<T, R, BT, CPL>* stash) {
  constexpr int NA = 2 * R;         // pending output rows per level
  constexpr int NS = lcm_i(NA, NR); // steps per unrolled iteration (NR: rows in the load ring)
  constexpr int W = 64 * CPL;       // tile width (columns)
  constexpr int LO = overlap_left(BT, R, sizeof(T));  // overlap columns on the left
  constexpr int C = compute_width(W, BT, R, sizeof(T)); // compute-region width
  // the compute region is whole lanes when it starts and ends on lane edges
  constexpr bool WHOLE = LO % CPL == 0 && C % CPL == 0;
  constexpr int MCOL = BT * R + 1;  // rows kept in the boundary-column stash
  constexpr int XL = CPL + 2 * R;   // extended row: R cells of lane-1 | own CPL | R cells of lane+1
  constexpr uint32_t WB = sizeof(T);

  const int I0 = a.I0, I1 = a.I1;
  const int P0 = I0 + 2 * R, P1 = I1 + 2 * R;
  const int c_first = R + tile * C;      // first compute column
  const int col0 = c_first - LO;         // first column of the tile
  const int colL = col0 + lane * CPL;    // first column owned by this lane

  // Stores: a lane whose CPL cells all lie in the compute region writes them
  // as one vector (vstore); a lane that straddles its edge writes cell by cell
  // (soff).  When the region is whole lanes, only a tile that reaches the
  // grid's last column (an EDGE wave) has such a lane.  Out-of-range offsets
  // make the unused path a no-op.
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
  int hl = -1;  // index of this lane in the boundary-column stash
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
    const int lL = (0 - col0) / CPL;       // lane holding column 0 (col0 <= 0 when present)
    const int lR = (I1 + R - col0) / CPL;  // lane holding column I1+R
    if (left) hl = lane - lL;
    else if (right) hl = 2 + lane - lR;
  }

  const T* __restrict__ src = static_cast<const T*>(a.src);
  T* __restrict__ dst = static_cast<T*>(a.dst);

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

  // Folded lane shifts: the coefficients of in-row terms that read a
  // neighbouring lane live in VGPRs.
  constexpr int NP = npts(2, R, BOX);
  constexpr bool FOLD = ACC == 0 && std::is_same_v<T, float> && (!BOX || R == 1);
  T cv[NP];
  if constexpr (FOLD)
    sfor<NP>([&](auto I) S5D_INL {
      if constexpr (folded_coef2d<R, BOX>(I)) cv[I] = to_vgpr(cf.c[I]);
    });

  Accum<T, ACC> acc[BT][NA][CPL];
  using RowV = T __attribute__((ext_vector_type(CPL)));
  RowV ringv[NR];
  sfor<BT>([&](auto L) S5D_INL { sfor<NA>([&](auto S) S5D_INL { sfor<CPL>([&](auto K) S5D_INL { acc[L][S][K].zero(); }); }); });

  const int s_lo = max(0, row_a - BT * R);
  const int s0 = s_lo - s_lo % NS;    // step phases line up with accumulator slots
  const int s_end = row_b + BT * R;   // level BT emits row row_b-1 at step s_end-1
  const int niter = (s_end - s0 + NS - 1) / NS;

  auto load_vec = [&](RowV& v, int row) S5D_INL {
    T t[CPL];
    load_row(t, row);
    sfor<CPL>([&](auto K) S5D_INL { v[+K] = t[K]; });
  };
  sfor<NR - 1>([&](auto J) S5D_INL {
    load_vec(ringv[J], s0 + J);
    __builtin_amdgcn_sched_barrier(0);  // keep ring order: the loop waits on the oldest load
  });

  auto iteration = [&](const int sb) S5D_INL {
    sfor<NS>([&](auto PH) S5D_INL {
      const int s = sb + PH;
      // the slot consumed at the previous step is free: request row s+NR-1 into it
      load_vec(ringv[pmod(PH - 1, NR)], s + NR - 1);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (EDGE) {
        // level 0 holds original values: stash the boundary columns of row s
        if (hl >= 0) sfor<CPL>([&](auto K) S5D_INL { stash->cols[s % MCOL][hl][K] = ringv[PH % NR][+K]; });
      }
      T cur[CPL];
      sfor<CPL>([&](auto K) S5D_INL { cur[K] = ringv[PH % NR][+K]; });

      sfor<BT>([&](auto LI) S5D_INL {
        constexpr int lv = LI + 1;                       // level receiving row p = s-(lv-1)*R
        constexpr int pm = pmod(PH - (lv - 1) * R, NA);  // p mod 2R
        constexpr int so = pmod(pm + R, NA);             // slot of rows p-R and p+R
        Accum<T, ACC>(&A)[NA][CPL] = acc[LI];

        T E[XL];
        sfor<CPL>([&](auto K) S5D_INL { E[R + K] = cur[K]; });
        sfor<R>([&](auto J) S5D_INL {
          E[J] = lane_from_lower(cur[CPL - R + J]);
          E[R + CPL + J] = lane_from_upper(cur[J]);
        });

        // one in-row term: coefficient ci times extended-row cell e
        auto term = [&](Accum<T, ACC>& acc_k, auto CI, auto EI, auto FIRST) S5D_INL {
          constexpr int ci = CI, e = EI;
          constexpr bool first = FIRST;
          if constexpr (FOLD && (e < R || e >= R + CPL)) {
            constexpr bool shr = e < R;  // from lane l-1, else lane l+1
            constexpr int src = shr ? CPL - R + e : e - R - CPL;
            if constexpr (first) acc_k.s = mul_dpp<shr>(cur[src], cv[ci]);
            else acc_k.s = fma_dpp<shr>(acc_k.s, cur[src], cv[ci]);
          } else if constexpr (first) {
            acc_k.first(cf.c[ci], E[e]);
          } else {
            acc_k.add(cf.c[ci], E[e]);
          }
        };
        // contribution of the arriving row to the output d0 rows before it
        auto add_row = [&](auto D0, Accum<T, ACC>& acc_k, auto K, auto FIRST) S5D_INL {
          constexpr int d0 = D0;
          constexpr bool first = FIRST;
          if constexpr (BOX) {
            sfor<2 * R + 1>([&](auto D1) S5D_INL {
              term(acc_k, ic<(d0 + R) * (2 * R + 1) + D1>{}, ic<K + D1>{},
                   std::integral_constant<bool, first && D1 == 0>{});
            });
          } else if constexpr (d0 != 0) {
            constexpr int ci = d0 < 0 ? d0 + R : 3 * R + d0;
            if constexpr (first) acc_k.first(cf.c[ci], cur[K]);
            else acc_k.add(cf.c[ci], cur[K]);
          } else {
            sfor<2 * R + 1>([&](auto D1) S5D_INL { term(acc_k, ic<R + D1>{}, ic<K + D1>{}, std::false_type{}); });
          }
        };

        // 1. output p-R receives its last contribution (d0 = +R) and leaves
        T out[CPL];
        sfor<CPL>([&](auto K) S5D_INL {
          Accum<T, ACC> v = A[so][K];
          add_row(ic<R>{}, v, K, std::false_type{});
          out[K] = finish<EXPR>(v.value(), cf);
        });
        // 2. output p+R starts in the freed slot (d0 = -R)
        sfor<CPL>([&](auto K) S5D_INL { add_row(ic<-R>{}, A[so][K], K, std::true_type{}); });
        // 3. outputs p+R-1 .. p-R+1 (d0 = -R+1 .. R-1)
        sfor<2 * R - 1>([&](auto J) S5D_INL {
          constexpr int d0 = -R + 1 + J;
          constexpr int sl = pmod(pm - d0, NA);
          sfor<CPL>([&](auto K) S5D_INL { add_row(ic<d0>{}, A[sl][K], K, std::false_type{}); });
        });


        if constexpr (EDGE && lv < BT) {
          // the last level is only stored, and boundary cells are never stored
          const int o = s - lv * R;
          if (o < R || o >= I0 + R) {
            // boundary row: never written, so the source buffer still holds it
            if (o >= 0 && o < P0) load_row(out, o);
          } else {
            // every lane reads a stash slot (its own, or slot 0 if it holds no
            // boundary column, where hcol is all false): no divergent branch
            const LaneVec<T, CPL> hv = *reinterpret_cast<const LaneVec<T, CPL>*>(
                stash->cols[o % MCOL][hl < 0 ? 0 : hl]);
            sfor<CPL>([&](auto K) S5D_INL { out[K] = hcol[K] ? hv.v[K] : out[K]; });
          }
        }

        if constexpr (lv < BT) {
          sfor<CPL>([&](auto K) S5D_INL { cur[K] = out[K]; });
        } else {
          // rows outside the stream block get an empty descriptor: no branch,
          // so the whole unrolled iteration stays one basic block
          const int o = s - BT * R;
          const bool keep = o >= row_a && o < row_b;
          const auto rs = make_rsrc(dst + static_cast<int64_t>(keep ? o : row_a) * P1,
                                    keep ? static_cast<uint32_t>(P1) * WB : 0u);
          buf_store_lane(out, rs, vstore);
          if constexpr (EDGE || !WHOLE) sfor<CPL>([&](auto K) S5D_INL { buf_store(out[K], rs, soff[K]); });
        }
      });
    });
  };
  // The first iteration is peeled so that the loop is entered with the same
  // memory operations in flight as at its back edge: the wait on the oldest
  // ring row then counts every younger load and store.
  iteration(s0);
  for (int it = 1; it < niter; ++it) iteration(s0 + it * NS);
}

// Workgroup lb of one grid's launch: kWavesPerBlock waves, one tile each, of
// band lb % nb (with 8 bands, the XCD the workgroup runs on in a launch of
// its own).
template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int NR>
__device__ __forceinline__ void sweep2d_block(const Sweep2DArgs& a, const CoefPack<T, ncoef(2, R, BOX, EXPR)>& cf, int lb,
                                              EdgeStash<T, R, BT, CPL>* stash) {
  constexpr int W = 64 * CPL;
  constexpr int LO = overlap_left(BT, R, sizeof(T));
  constexpr int C = compute_width(W, BT, R, sizeof(T));
  static_assert(R <= CPL, "the lane exchange reaches one neighbouring lane only");
  static_assert(C >= 1, "tile narrower than its overlap");
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = a.g.nb;
  const int x = lb % nb;
  const int wid = (lb / nb) * kWavesPerBlock + wib;  // wave within the band
  if (wid >= a.nwaves) return;
  const int lane = threadIdx.x & 63;
  const int tile = wid % a.ntiles;
  int row_a, row_b;
  band_rows2d(a.g, R, a.I0, x, wid / a.ntiles, row_a, row_b);
  if (row_b <= row_a) return;

  const int P1 = a.I1 + 2 * R;
  const int col0 = R + tile * C - LO;
  const bool edge = col0 < 0 || col0 + W > P1 || row_a - (BT - 1) * R < R ||
                    row_b + (BT - 1) * R > a.I0 + R;
  if (edge)
    sweep2d_body<T, ACC, EXPR, R, BOX, BT, CPL, NR, true>(a, cf, lane, tile, row_a, row_b, &stash[wib]);
  else
    sweep2d_body<T, ACC, EXPR, R, BOX, BT, CPL, NR, false>(a, cf, lane, tile, row_a, row_b, &stash[wib]);
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int NR>
__global__ __launch_bounds__(64 * kWavesPerBlock) void sweep2d_kernel(Sweep2DArgs a,
                                                                    CoefPack<T, ncoef(2, R, BOX, EXPR)> cf) {
  __shared__ EdgeStash<T, R, BT, CPL> stash[kWavesPerBlock];
  sweep2d_block<T, ACC, EXPR, R, BOX, BT, CPL, NR>(a, cf, blockIdx.x, stash);
}

// One grid of a batched launch: its geometry and coefficients.
template <typename T, int NP>
struct alignas(16) Item2D {
  Sweep2DArgs a;
  CoefPack<T, NP> cf;
};

// Batched launch: workgroup b runs workgroup map[b].block of grid map[b].item.
// Item and map are read once per wave with scalar loads (uniform addresses)
// and copied into registers before the sweep starts.
template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int NR>
__global__ __launch_bounds__(64 * kWavesPerBlock) void sweep2d_batch_kernel(
    const Item2D<T, ncoef(2, R, BOX, EXPR)>* __restrict__ items, const BlockMap* __restrict__ map) {
  __shared__ EdgeStash<T, R, BT, CPL> stash[kWavesPerBlock];
  const BlockMap m = map[xcd_logical_block(blockIdx.x, gridDim.x)];
  const Item2D<T, ncoef(2, R, BOX, EXPR)>& it = items[__builtin_amdgcn_readfirstlane(m.item)];
  const Sweep2DArgs a = uniform_copy(it.a);
  const CoefPack<T, ncoef(2, R, BOX, EXPR)> cf = uniform_copy(it.cf);
  sweep2d_block<T, ACC, EXPR, R, BOX, BT, CPL, NR>(a, cf, __builtin_amdgcn_readfirstlane(m.block), stash);
}

template <typename T, int EXPR, int R, bool BOX, int BT, int CPL>
Sweep2DArgs make_args2d(const Round2D& rd, CoefPack<T, ncoef(2, R, BOX, EXPR)>& cf) {
  constexpr int NP = ncoef(2, R, BOX, EXPR);  // the divisor c0 last for EXPR_DIV
  constexpr int C = compute_width(64 * CPL, BT, R, sizeof(T));
  for (int k = 0; k < NP; ++k) cf.c[k] = static_cast<T>(rd.coeffs[k]);
  Sweep2DArgs a;
  a.src = rd.src;
  a.dst = rd.dst;
  a.I0 = rd.I0;
  a.I1 = rd.I1;
  a.g = make_bands2d(rd.I0, rd.chunk);
  a.ntiles = (rd.I1 + C - 1) / C;
  const int64_t nw = static_cast<int64_t>(a.ntiles) * (a.g.n1 + a.g.n2);
  a.nwaves = nw > INT32_MAX / kXcds ? 0 : static_cast<int32_t>(nw);
  return a;
}

// Workgroups of a launch: nb bands of ceil(nwaves / kWavesPerBlock).
inline int blocks2d(const Sweep2DArgs& a) {
  return a.g.nb * ((a.nwaves + kWavesPerBlock - 1) / kWavesPerBlock);
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int NR>
hipError_t launch_sweep2d(const Round2D& rd) {
  CoefPack<T, ncoef(2, R, BOX, EXPR)> cf;
  const Sweep2DArgs a = make_args2d<T, EXPR, R, BOX, BT, CPL>(rd, cf);
  if (a.nwaves == 0) return hipErrorInvalidConfiguration;
  const int nblk = blocks2d(a);
  hipLaunchKernelGGL((sweep2d_kernel<T, ACC, EXPR, R, BOX, BT, CPL, NR>), dim3(nblk), dim3(64 * kWavesPerBlock), 0,
                     rd.stream, a, cf);
  return hipGetLastError();
}

template <typename T, int EXPR, int R, bool BOX, int BT, int CPL>
int fill_item2d(void* item, const Round2D& rd) {
  Item2D<T, ncoef(2, R, BOX, EXPR)> it;
  it.a = make_args2d<T, EXPR, R, BOX, BT, CPL>(rd, it.cf);
  __builtin_memcpy(item, &it, sizeof(it));
  return blocks2d(it.a);
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int NR>
hipError_t launch_batch2d(const void* items, const BlockMap* map, int nblocks, hipStream_t stream) {
  hipLaunchKernelGGL((sweep2d_batch_kernel<T, ACC, EXPR, R, BOX, BT, CPL, NR>), dim3(nblocks),
                     dim3(64 * kWavesPerBlock), 0, stream,
                     static_cast<const Item2D<T, ncoef(2, R, BOX, EXPR)>*>(items), map);
  return hipGetLastError();
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int NR>
int occupancy_sweep2d() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep2d_kernel<T, ACC, EXPR, R, BOX, BT, CPL, NR>,
                                                   64 * kWavesPerBlock, 0) != hipSuccess)
    return 0;
  return nb;
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int BT, int CPL, int NR>
Kernel2D make_kernel2d() {
  return Kernel2D{&launch_sweep2d<T, ACC, EXPR, R, BOX, BT, CPL, NR>,
                  &occupancy_sweep2d<T, ACC, EXPR, R, BOX, BT, CPL, NR>,
                  CPL,
                  BT,
                  64 * CPL,
                  &fill_item2d<T, EXPR, R, BOX, BT, CPL>,
                  &launch_batch2d<T, ACC, EXPR, R, BOX, BT, CPL, NR>,
                  static_cast<int>(sizeof(Item2D<T, ncoef(2, R, BOX, EXPR)>))};
}

}  // namespace s5d
