// Persistent batched execution of the 2D blocked sweep (device code +
// launcher): every round of every grid of a stencil family in ONE launch.
//
// A family is one element type, accumulation, expression, shape, radius and
// tile width (cells per lane); its kernel holds the blocked sweep of each
// compiled depth b_T of the family and picks one per round, so grids of
// different depths and the shorter tail rounds of a schedule share the
// launch.  The launch has at most as many workgroups as fit on the device at
// once.  Each workgroup repeatedly takes the next ticket of a device queue
// (persist_schedule.h: items ordered by round index, then grid, then the
// workgroup of that round's own launch), waits until its grid's completion
// counter shows that the grid's previous rounds have finished, runs the
// workgroup of the round exactly as the round's own launch would run it
// (sweep2d_block: same tiles, stream blocks and arithmetic, so the same
// bits), and then counts its waves as done.  Grids therefore move from round
// to round on their own, without a device-wide barrier between round indices.
//
// Memory ordering: every wave makes its stores visible device-wide (an
// agent-scope release, which writes the XCD's L2 back) before it counts
// itself done; once the waiting thread has read the counter it issues an
// agent-scope acquire fence (which invalidates the stale cache lines of its CU
// and XCD), and the workgroup barrier after it orders every wave's loads of
// the round after that.
//
// The wait is bounded: after `wait_limit` polls without progress the
// workgroup records status 1 in the control block and leaves; every other
// workgroup stops at its next ticket.  The host reads the status after the
// launch (s5d_batch_status).  A correct schedule never waits long: an item
// only depends on items with smaller tickets, all of which are held by
// running workgroups.
#pragma once

#include "persist2d.h"
#include "sweep2d.h"

namespace s5d {

// One round of one grid: the geometry and coefficients its own launch would
// get, its depth and its place in the completion counters.
template <typename T, int NP>
struct alignas(16) PRound2D {
  Sweep2DArgs a;
  CoefPack<T, NP> cf;
  int32_t grid;  // completion counter
  int32_t need;  // waves of the grid done before this round may start
  int32_t bt;    // fused depth
  int32_t pad;
};

template <int BT, int NR>
struct Depth {
  static constexpr int bt = BT, nr = NR;
};

template <typename T, int R, int CPL, typename D, typename... DS>
constexpr size_t max_stash_bytes() {
  constexpr size_t s = sizeof(EdgeStash<T, R, D::bt, CPL>);
  if constexpr (sizeof...(DS) == 0) return s;
  else return s > max_stash_bytes<T, R, CPL, DS...>() ? s : max_stash_bytes<T, R, CPL, DS...>();
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int CPL, typename D, typename... DS>
__device__ __forceinline__ void persist_block2d(int bt, const Sweep2DArgs& a,
                                                const CoefPack<T, ncoef(2, R, BOX, EXPR)>& cf, int lb,
                                                unsigned char* stash) {
  if (bt == D::bt) {
    sweep2d_block<T, ACC, EXPR, R, BOX, D::bt, CPL, D::nr>(a, cf, lb,
                                                           reinterpret_cast<EdgeStash<T, R, D::bt, CPL>*>(stash));
  } else if constexpr (sizeof...(DS) > 0) {
    persist_block2d<T, ACC, EXPR, R, BOX, CPL, DS...>(bt, a, cf, lb, stash);
  }
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int CPL, int WPE, typename... DS>
__global__ __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(WPE))) void sweep2d_persist_kernel(
    const PRound2D<T, ncoef(2, R, BOX, EXPR)>* __restrict__ rounds, const PersistItem* __restrict__ items,
    int32_t n_items, int32_t* __restrict__ ctl, int64_t wait_limit) {
  constexpr size_t SB = max_stash_bytes<T, R, CPL, DS...>();
  __shared__ __attribute__((aligned(16))) unsigned char stash[kWavesPerBlock * SB];
  __shared__ int32_t s_ticket, s_ok;
  int32_t* done = ctl + kPersistCtl;
  for (;;) {
    if (threadIdx.x == 0) {
      const int32_t t = __hip_atomic_fetch_add(&ctl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int32_t ok = __hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
      if (ok && t < n_items) {
        const PRound2D<T, ncoef(2, R, BOX, EXPR)>& rd = rounds[items[t].round];
        const int32_t g = rd.grid, need = rd.need;
        int64_t polls = 0;
        while (__hip_atomic_load(&done[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (polls++ >= wait_limit ||
              __hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            __hip_atomic_store(&ctl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(8);
        }
        // one acquire once the counter is reached (polling does not need one)
        if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      s_ticket = t;
      s_ok = ok;
    }
    __syncthreads();
    const int32_t t = s_ticket, ok = s_ok;
    __syncthreads();  // thread 0 rewrites both only after every wave has read them
    if (t >= n_items || !ok) break;
    const PersistItem it = items[t];
    const int32_t ri = __builtin_amdgcn_readfirstlane(it.round);
    const int32_t lb = __builtin_amdgcn_readfirstlane(it.block);
    const Sweep2DArgs a = uniform_copy(rounds[ri].a);
    const CoefPack<T, ncoef(2, R, BOX, EXPR)> cf = uniform_copy(rounds[ri].cf);
    const int32_t bt = __builtin_amdgcn_readfirstlane(rounds[ri].bt);
    const int32_t g = __builtin_amdgcn_readfirstlane(rounds[ri].grid);
    persist_block2d<T, ACC, EXPR, R, BOX, CPL, DS...>(bt, a, cf, lb, stash);
    // publish this wave's stores, then count the wave (waves that had no
    // tile in this workgroup count too)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_add(&done[g], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T, int EXPR, int R, bool BOX, int CPL, typename D, typename... DS>
int fill_persist_round2d_at(void* out, const Round2D& rd, int bt, int grid, int need) {
  if (bt == D::bt) {
    PRound2D<T, ncoef(2, R, BOX, EXPR)> pr;
    pr.a = make_args2d<T, EXPR, R, BOX, D::bt, CPL>(rd, pr.cf);
    pr.grid = grid;
    pr.need = need;
    pr.bt = bt;
    pr.pad = 0;
    __builtin_memcpy(out, &pr, sizeof(pr));
    return pr.a.nwaves == 0 ? 0 : blocks2d(pr.a);
  }
  if constexpr (sizeof...(DS) > 0) return fill_persist_round2d_at<T, EXPR, R, BOX, CPL, DS...>(out, rd, bt, grid, need);
  return -1;
}

template <typename T, int EXPR, int R, bool BOX, int CPL, typename... DS>
int fill_persist_round2d(void* out, const Round2D& rd, int bt, int grid, int need) {
  return fill_persist_round2d_at<T, EXPR, R, BOX, CPL, DS...>(out, rd, bt, grid, need);
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int CPL, int WPE, typename... DS>
hipError_t launch_persist2d(const void* rounds, const PersistItem* items, int32_t n_items, int32_t* ctl,
                            int64_t wait_limit, int nblocks, hipStream_t stream) {
  hipLaunchKernelGGL((sweep2d_persist_kernel<T, ACC, EXPR, R, BOX, CPL, WPE, DS...>), dim3(nblocks),
                     dim3(64 * kWavesPerBlock), 0, stream,
                     static_cast<const PRound2D<T, ncoef(2, R, BOX, EXPR)>*>(rounds), items, n_items, ctl,
                     wait_limit);
  return hipGetLastError();
}

template <typename T, int ACC, int EXPR, int R, bool BOX, int CPL, int WPE, typename... DS>
int occupancy_persist2d() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep2d_persist_kernel<T, ACC, EXPR, R, BOX, CPL, WPE, DS...>,
                                                   64 * kWavesPerBlock, 0) != hipSuccess)
    return 0;
  return nb;
}

// WPE: waves per SIMD the kernel's registers must allow (the occupancy of the
// family's deepest depth in a launch of its own).
template <typename T, int ACC, int EXPR, int R, bool BOX, int CPL, int WPE, typename... DS>
Persist2D make_persist2d() {
  return Persist2D{&launch_persist2d<T, ACC, EXPR, R, BOX, CPL, WPE, DS...>,
                   &occupancy_persist2d<T, ACC, EXPR, R, BOX, CPL, WPE, DS...>,
                   &fill_persist_round2d<T, EXPR, R, BOX, CPL, DS...>,
                   static_cast<int>(sizeof(PRound2D<T, ncoef(2, R, BOX, EXPR)>))};
}

}  // namespace s5d
