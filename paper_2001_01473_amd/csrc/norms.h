// Error and norm reductions in float64 (norms.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s5d {

// First-pass workgroups for n elements (at most kNormMaxParts); each leaves
// five float64 partials in the workspace.
constexpr int kNormMaxParts = 2048;
int error_norms_parts(int64_t n);

// Device address of this device's norm scratch (kNormMaxParts x 5 doubles),
// resolved once per device with hipGetSymbolAddress; the calling thread's
// current device is the one meant.
hipError_t error_norms_scratch(double** out);
int64_t error_norms_scratch_bytes();

hipError_t launch_error_norms(const void* got, int got_f64, const void* ref, int ref_f64, int64_t n, double* out,
                              double* partial, int nparts, hipStream_t stream);

}  // namespace s5d
