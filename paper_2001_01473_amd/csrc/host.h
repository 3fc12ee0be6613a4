// Host-side internals shared by the C ABI translation units: the plan
// object, error reporting and the round schedule.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "persist2d.h"
#include "s5d_internal.h"
#include "stencil5d.h"

struct s5d_plan {
  s5d_desc d;
  std::vector<double> coeffs;
  s5d_tuning tun;
  int64_t padded[3];
  int64_t bytes;
  int elem;
  int kind;                  // kernel kind: KIND_F32, KIND_F64 or KIND_F32_COMP
  int expr = 0;              // S5D_EXPR_*
  bool direct = false;       // direct kernels (one step per launch) instead of blocked ones
  bool chunk_auto = false;   // stream_chunk was chosen by the library (not asked for)
  int64_t slots = 0;         // 2D: resident waves of the plan's variant on the whole device
  s5d::Kernel2D by_bt[16];   // 2D: index bt -> kernel for a round of bt steps (same tile)
  s5d::Kernel3D by_bt3[16];  // 3D: likewise
  // device copy of the coefficients in the working type (direct kernels);
  // shared by copies of the plan, freed with the last of them
  std::shared_ptr<void> dcoef;
};

namespace s5d {

// Record a detail string for s5d_last_error() on this thread; returns st.
s5d_status fail(s5d_status st, const std::string& msg);
s5d_status device_fail(hipError_t e, const char* what);
void clear_error();

// The fused depth of every round of a plan's sweep, in launch order (empty
// for T = 0).  Round k reads buffer k % 2 and writes buffer (k + 1) % 2; the
// number of rounds has the parity of T, so the result is in buffer T % 2.
std::vector<int> plan_rounds(const s5d_plan* p);

// Launch one round of bt fused steps of plan p from src into dst (fields:
// the per-cell weights of a variable-coefficient plan, else null).
hipError_t launch_round(const s5d_plan* p, int bt, const void* src, void* dst, hipStream_t stream,
                        const void* fields = nullptr);

// The batched-launch hooks of the kernel that runs a round of bt steps of p.
struct BatchHooks {
  LaunchBatchFn launch;  // identifies the kernel variant
  int item_bytes;
};
BatchHooks batch_hooks(const s5d_plan* p, int bt);
// Write p's batch item for a round into `item`; returns its workgroups.
int fill_round_item(const s5d_plan* p, int bt, const void* src, void* dst, void* item, int chunk = 0);

// Write the persistent-launch round table entry of one round of p (depth bt,
// family kernel k) into `out`; returns the round's workgroups (0: too large,
// -1: the family has no kernel of that depth).
int fill_persist_round(const s5d_plan* p, const Persist2D& k, int bt, const void* src, void* dst, void* out,
                       int chunk, int grid, int need);

// Stream-block length for a grid that shares each launch with others and
// gets about `share` (0 < share <= 1) of the machine's workgroup slots: the
// library's chooser run for that many slots.  The plan's own length when the
// caller chose it, or for direct kernels.
int shared_chunk(const s5d_plan* p, int bt, double share);

// Copy the fixed boundary of buf0 into buf1 (before the first round).
hipError_t launch_boundary_copy(const s5d_plan* p, const void* buf0, void* buf1, hipStream_t stream);

// Check a (buf0, buf1) pair against a plan: non-null, aligned, disjoint.
s5d_status check_buffers(const s5d_plan* p, const void* buf0, const void* buf1);

// Performance model of a plan's whole sweep (tune.cpp).
s5d_status model_plan(const s5d_plan* p, s5d_model* out);

// The autotuned blocking cached for this descriptor's stencil, dtype,
// accumulation and extent bucket, if any.
bool tune_cache_lookup(const s5d_desc& d, s5d_tuning* tun);

// Load the autotuner's shipped choices once per process: the file named by
// S5D_TUNING_FILE (empty: none), else tuning_gfx950.txt beside the library.
void load_default_tuning();

}  // namespace s5d
