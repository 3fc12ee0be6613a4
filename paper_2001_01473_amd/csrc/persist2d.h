// Persistent batched 2D launches (sweepp2d.h): one kernel per stencil family
// (kind, expression, shape, radius, cells per lane) holding the depths
// 1..max_bt of the family; the work list comes from persist_schedule.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "persist_schedule.h"
#include "s5d_internal.h"

namespace s5d {

using LaunchPersistFn = hipError_t (*)(const void* rounds, const PersistItem* items, int32_t n_items, int32_t* ctl,
                                       int64_t wait_limit, int nblocks, hipStream_t stream);
// Write the round-table entry of one round (depth bt) into `out`; returns the
// round's workgroups, 0 if it does not fit a launch, -1 if the family has no
// kernel of that depth.
using FillPersistFn = int (*)(void* out, const Round2D& rd, int bt, int grid, int need);

struct Persist2D {
  LaunchPersistFn launch;
  Occupancy2DFn occupancy;  // resident workgroups per CU
  FillPersistFn fill_round;
  int round_bytes;
};

struct EntryP2D {
  int dtype, expr, box, r, cpl;
  int max_bt;  // depths 1..max_bt
  Persist2D (*make)();
};
extern const EntryP2D kRegistryP2D[];
extern const int kRegistryP2DSize;

// Set n int32 values at p to v with a kernel (no memset node, so the call may
// be captured in a HIP graph and replayed).
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t stream);

// Control block of one persistent launch: [0] next ticket, [1] status (0 ok,
// 1 a dependency wait ran out), then one completion counter per grid.
constexpr int kPersistCtl = 4;

}  // namespace s5d
