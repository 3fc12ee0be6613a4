// Error and norm reductions between a computed grid and a reference grid, in
// float64 on the GPU.
//
// For n elements g (float32 or float64) and o (float32 or float64) the two
// launches below produce, with d = |g - o| formed in float64:
//   [0] max d                      [1] max |o|
//   [2] max d / |o|  (d where o = 0)
//   [3] sqrt(sum d^2 / n)          [4] sqrt(sum o^2 / n)
// Maxima propagate NaN, so a NaN anywhere in g or o shows in [0], [2], [3].
//
// The first launch gives each workgroup a fixed, strided share of the
// elements and writes its five partials to the workspace; the second, a single
// workgroup, folds the partials in a fixed order.  For a given n the
// result therefore does not depend on scheduling and repeats bit for bit.  The
// work is bound by HBM bandwidth: each element is read once with 16-byte
// loads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "norms.h"

namespace s5d {
namespace {

constexpr int kNormThreads = 256;
constexpr int kNormVals = 5;

__device__ __forceinline__ double nanmax(double m, double x) { return (x > m || x != x) ? x : m; }

struct NormAcc {
  double mabs = 0.0, mref = 0.0, mrel = 0.0, sse = 0.0, ssr = 0.0;
  __device__ __forceinline__ void add(double g, double o) {
    const double d = __builtin_fabs(g - o);
    const double ao = __builtin_fabs(o);
    mabs = nanmax(mabs, d);
    mref = nanmax(mref, ao);
    mrel = nanmax(mrel, ao != 0.0 ? d / ao : d);
    sse = __builtin_fma(d, d, sse);
    ssr = __builtin_fma(ao, ao, ssr);
  }
  __device__ __forceinline__ void merge(const NormAcc& b) {
    mabs = nanmax(mabs, b.mabs);
    mref = nanmax(mref, b.mref);
    mrel = nanmax(mrel, b.mrel);
    sse += b.sse;
    ssr += b.ssr;
  }
};

// Reduce the five values over the workgroup; the result is valid in thread 0.
__device__ NormAcc block_reduce(NormAcc a) {
  __shared__ double part[kNormThreads / 64][kNormVals];
  for (int off = 32; off >= 1; off >>= 1) {
    NormAcc b;
    b.mabs = __shfl_xor(a.mabs, off, 64);
    b.mref = __shfl_xor(a.mref, off, 64);
    b.mrel = __shfl_xor(a.mrel, off, 64);
    b.sse = __shfl_xor(a.sse, off, 64);
    b.ssr = __shfl_xor(a.ssr, off, 64);
    a.merge(b);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[w][0] = a.mabs;
    part[w][1] = a.mref;
    part[w][2] = a.mrel;
    part[w][3] = a.sse;
    part[w][4] = a.ssr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kNormThreads / 64; ++i) {
      NormAcc b;
      b.mabs = part[i][0];
      b.mref = part[i][1];
      b.mrel = part[i][2];
      b.sse = part[i][3];
      b.ssr = part[i][4];
      a.merge(b);
    }
  }
  return a;
}

template <typename E>
__device__ __forceinline__ void load4(const E* p, int64_t v, double (&x)[4]) {
  if constexpr (sizeof(E) == 4) {
    const float4 q = reinterpret_cast<const float4*>(p)[v];
    x[0] = q.x;
    x[1] = q.y;
    x[2] = q.z;
    x[3] = q.w;
  } else {
    const double2 a = reinterpret_cast<const double2*>(p)[2 * v];
    const double2 b = reinterpret_cast<const double2*>(p)[2 * v + 1];
    x[0] = a.x;
    x[1] = a.y;
    x[2] = b.x;
    x[3] = b.y;
  }
}

// Pass 1: workgroup b takes the 4-element vectors b*T + t, b*T + t + B*T, ...
// (T threads, B workgroups) and the scalar tail n - 4*(n/4) goes to
// workgroup 0.  Both pointers are 16-byte aligned (checked by the host).
template <typename G, typename O>
__global__ void __launch_bounds__(kNormThreads) norms_partial_kernel(const G* __restrict__ g,
                                                                   const O* __restrict__ o, int64_t n,
                                                                   double* __restrict__ partial) {
  NormAcc a;
  const int64_t nv = n >> 2;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kNormThreads;
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * kNormThreads + threadIdx.x; v < nv; v += stride) {
    double xg[4], xo[4];
    load4(g, v, xg);
    load4(o, v, xo);
#pragma unroll
    for (int k = 0; k < 4; ++k) a.add(xg[k], xo[k]);
  }
  if (blockIdx.x == 0) {
    const int64_t i = (nv << 2) + threadIdx.x;
    if (i < n) a.add(static_cast<double>(g[i]), static_cast<double>(o[i]));
  }
  a = block_reduce(a);
  if (threadIdx.x == 0) {
    double* p = partial + static_cast<int64_t>(blockIdx.x) * kNormVals;
    p[0] = a.mabs;
    p[1] = a.mref;
    p[2] = a.mrel;
    p[3] = a.sse;
    p[4] = a.ssr;
  }
}

// Pass 2: one workgroup; thread t folds partials t, t + T, ... in order, then
// the workgroup tree.  Writes every output, so `out` needs no clearing.
__global__ void __launch_bounds__(kNormThreads) norms_final_kernel(const double* __restrict__ partial,
                                                                 int nparts, int64_t n,
                                                                 double* __restrict__ out) {
  NormAcc a;
  for (int i = threadIdx.x; i < nparts; i += kNormThreads) {
    NormAcc b;
    const double* p = partial + static_cast<int64_t>(i) * kNormVals;
    b.mabs = p[0];
    b.mref = p[1];
    b.mrel = p[2];
    b.sse = p[3];
    b.ssr = p[4];
    a.merge(b);
  }
  a = block_reduce(a);
  if (threadIdx.x == 0) {
    const double inv = n > 0 ? 1.0 / static_cast<double>(n) : 0.0;
    out[0] = a.mabs;
    out[1] = a.mref;
    out[2] = a.mrel;
    out[3] = __builtin_sqrt(a.sse * inv);
    out[4] = __builtin_sqrt(a.ssr * inv);
  }
}

template <typename G, typename O>
hipError_t launch_norms_typed(const void* g, const void* o, int64_t n, double* out, double* partial, int nparts,
                              hipStream_t stream) {
  if (n > 0)
    hipLaunchKernelGGL((norms_partial_kernel<G, O>), dim3(nparts), dim3(kNormThreads), 0, stream,
                       static_cast<const G*>(g), static_cast<const O*>(o), n, partial);
  else
    nparts = 0;
  hipLaunchKernelGGL(norms_final_kernel, dim3(1), dim3(kNormThreads), 0, stream, partial, nparts, n, out);
  return hipGetLastError();
}

}  // namespace

// Scratch of the allocation-free entry point: room for the first-pass partials
// of one call at the largest launch (kNormMaxParts workgroups x five values,
// 80 KiB).  Each device holds its own copy for the life of the process.  In
// host code this name is only a stand-in for the symbol, never a device
// address: kernels get the address that hipGetSymbolAddress returns.
static __device__ __align__(256) double scratch[kNormMaxParts * kNormVals];

hipError_t error_norms_scratch(double** out) {
  // one resolved address per device, looked up with that device current
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = static_cast<double*>(p);
  }
  *out = addr[dev];
  return hipSuccess;
}

int64_t error_norms_scratch_bytes() { return static_cast<int64_t>(sizeof(scratch)); }

int error_norms_parts(int64_t n) {
  // at least four 4-element vectors per thread, and at most kNormMaxParts
  // workgroups (8 per CU)
  const int64_t per = static_cast<int64_t>(kNormThreads) * 4 * 4;
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > kNormMaxParts) b = kNormMaxParts;
  return static_cast<int>(b);
}

hipError_t launch_error_norms(const void* got, int got_f64, const void* ref, int ref_f64, int64_t n, double* out,
                              double* partial, int nparts, hipStream_t stream) {
  if (!got_f64 && !ref_f64) return launch_norms_typed<float, float>(got, ref, n, out, partial, nparts, stream);
  if (!got_f64 && ref_f64) return launch_norms_typed<float, double>(got, ref, n, out, partial, nparts, stream);
  if (got_f64 && !ref_f64) return launch_norms_typed<double, float>(got, ref, n, out, partial, nparts, stream);
  return launch_norms_typed<double, double>(got, ref, n, out, partial, nparts, stream);
}

}  // namespace s5d
