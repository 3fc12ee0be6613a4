// Grouped launches of many grids' rounds (batch.cpp), shared by the batch
// executor and the server.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "host.h"

namespace s5d {

// One round of one grid: bt fused steps of `plan` from src into dst.
struct RoundItem {
  const s5d_plan* plan;
  int bt;
  const void* src;
  void* dst;
  int chunk;  // stream-block length for this launch (0: the plan's)
};

// One batched launch: the kernel variant, and the byte offsets of its items
// and of its workgroup map inside the device table.
struct GroupLaunch {
  LaunchBatchFn fn;
  size_t items_off;
  size_t map_off;
  int nblocks;
};

// Lay out the items and workgroup maps of one round step in `blob` (host
// copy of the device table), one GroupLaunch per kernel variant.
s5d_status build_step(const std::vector<RoundItem>& items, std::vector<unsigned char>& blob,
                      std::vector<GroupLaunch>& out);

// Streams a step's launches spread over: the caller's stream plus up to
// kMaxSideStreams side streams that fork from it and join back into it.
constexpr int kMaxSideStreams = 3;
struct StepStreams {
  int n_side = 0;
  hipStream_t side[kMaxSideStreams] = {nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxSideStreams] = {nullptr, nullptr, nullptr};
  // create n_side non-blocking side streams and their events (n_side <= kMaxSideStreams)
  hipError_t create(int n_side);
  void destroy();
};

// Enqueue the launches of a step whose table was uploaded to `dev`.  With
// side streams, a step of several launches (kernel variants, which touch
// different grids) forks: launch j goes to stream j mod (1 + n_side), so the
// variants overlap on the device, and the step joins back into `stream`
// before the next one.
hipError_t enqueue_step(const std::vector<GroupLaunch>& launches, const unsigned char* dev, hipStream_t stream,
                        const StepStreams* ss = nullptr);

// EINVAL if any two [begin, end) byte ranges overlap.
s5d_status check_disjoint(const std::vector<std::pair<uintptr_t, uintptr_t>>& ranges);

}  // namespace s5d
