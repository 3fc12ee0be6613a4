// Boundary copy: the fixed halo of width r on every face of a padded grid.
//
// The double-buffered loop never writes the boundary, so both buffers must
// carry the same boundary values (AN5D Fig. 4: only interior indices are
// assigned).  The library receives the initial state in buffer 0 and fills the
// boundary of buffer 1 with this kernel before the first round.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "persist2d.h"
#include "s5d_internal.h"

namespace s5d {
namespace {

// Halo cells are enumerated without touching the interior:
//   A: both axis-0 slabs      2*r0 x P1 x P2
//   B: both axis-1 slabs      (P0-2*r0) x 2*r1 x P2
//   C: both axis-2 slabs      (P0-2*r0) x (P1-2*r1) x 2*r2
// (2D grids use P2 = 1, r2 = 0, so part C is empty.)  Cells t0, t0+stride,
// ... of that enumeration are copied.
template <typename E>
__device__ __forceinline__ void copy_halo_cells(const E* __restrict__ src, E* __restrict__ dst, int64_t P0,
                                                int64_t P1, int64_t P2, int64_t r0, int64_t r1, int64_t r2,
                                                int64_t t0, int64_t stride) {
  const int64_t nA = 2 * r0 * P1 * P2;
  const int64_t I0 = P0 - 2 * r0;
  const int64_t nB = I0 * 2 * r1 * P2;
  const int64_t nC = I0 * (P1 - 2 * r1) * 2 * r2;
  const int64_t total = nA + nB + nC;
  for (int64_t t = t0; t < total; t += stride) {
    int64_t i0, i1, i2;
    if (t < nA) {
      i0 = t / (P1 * P2);
      const int64_t rem = t - i0 * P1 * P2;
      i1 = rem / P2;
      i2 = rem - i1 * P2;
      if (i0 >= r0) i0 += P0 - 2 * r0;
    } else if (t < nA + nB) {
      const int64_t u = t - nA;
      i0 = u / (2 * r1 * P2);
      const int64_t rem = u - i0 * 2 * r1 * P2;
      i1 = rem / P2;
      i2 = rem - i1 * P2;
      i0 += r0;
      if (i1 >= r1) i1 += P1 - 2 * r1;
    } else {
      const int64_t u = t - nA - nB;
      const int64_t J1 = P1 - 2 * r1;
      i0 = u / (J1 * 2 * r2);
      const int64_t rem = u - i0 * J1 * 2 * r2;
      i1 = rem / (2 * r2);
      i2 = rem - i1 * 2 * r2;
      i0 += r0;
      i1 += r1;
      if (i2 >= r2) i2 += P2 - 2 * r2;
    }
    const int64_t p = (i0 * P1 + i1) * P2 + i2;
    dst[p] = src[p];
  }
}

template <typename E>
__global__ void halo_copy_kernel(const E* __restrict__ src, E* __restrict__ dst, int64_t P0, int64_t P1,
                                 int64_t P2, int64_t r0, int64_t r1, int64_t r2) {
  copy_halo_cells(src, dst, P0, P1, P2, r0, r1, r2, static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x,
                  static_cast<int64_t>(gridDim.x) * blockDim.x);
}

// Many grids at once: blockIdx.y selects the grid (a wave-uniform branch on
// its element size), blockIdx.x strides over its halo cells.
__global__ void halo_copy_batch_kernel(const HaloItem* __restrict__ items) {
  const HaloItem& h = items[blockIdx.y];
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t r2 = h.P2 > 1 ? h.r : 0;
  if (h.elem == 4)
    copy_halo_cells(static_cast<const uint32_t*>(h.src), static_cast<uint32_t*>(h.dst), h.P0, h.P1, h.P2, h.r,
                    h.r, r2, t0, stride);
  else
    copy_halo_cells(static_cast<const uint64_t*>(h.src), static_cast<uint64_t*>(h.dst), h.P0, h.P1, h.P2, h.r,
                    h.r, r2, t0, stride);
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

}  // namespace

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int threads = 256;
  int64_t blocks = (n + threads - 1) / threads;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_halo_copy(const void* src, void* dst, int elem_bytes, int ndim, const int64_t* padded, int r,
                            hipStream_t stream) {
  const int64_t P0 = padded[0], P1 = padded[1], P2 = ndim == 3 ? padded[2] : 1;
  const int64_t r2 = ndim == 3 ? r : 0;
  const int64_t total = P0 * P1 * P2 - (P0 - 2 * r) * (P1 - 2 * r) * (P2 - 2 * r2);
  if (total <= 0) return hipSuccess;
  const int threads = 256;
  int64_t blocks = (total + threads - 1) / threads;
  if (blocks > 4096) blocks = 4096;
  if (elem_bytes == 4) {
    hipLaunchKernelGGL(halo_copy_kernel<uint32_t>, dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, stream,
                       static_cast<const uint32_t*>(src), static_cast<uint32_t*>(dst), P0, P1, P2,
                       static_cast<int64_t>(r), static_cast<int64_t>(r), r2);
  } else {
    hipLaunchKernelGGL(halo_copy_kernel<uint64_t>, dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, stream,
                       static_cast<const uint64_t*>(src), static_cast<uint64_t*>(dst), P0, P1, P2,
                       static_cast<int64_t>(r), static_cast<int64_t>(r), r2);
  }
  return hipGetLastError();
}

int64_t halo_cells(int ndim, const int64_t* padded, int r) {
  const int64_t P0 = padded[0], P1 = padded[1], P2 = ndim == 3 ? padded[2] : 1;
  const int64_t r2 = ndim == 3 ? r : 0;
  return P0 * P1 * P2 - (P0 - 2 * r) * (P1 - 2 * r) * (P2 - 2 * r2);
}

hipError_t launch_halo_copy_batch(const HaloItem* items, int n, int64_t max_cells, hipStream_t stream) {
  if (n <= 0 || max_cells <= 0) return hipSuccess;
  if (n > 65535) return hipErrorInvalidValue;
  const int threads = 256;
  int64_t bx = (max_cells + threads - 1) / threads;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(halo_copy_batch_kernel, dim3(static_cast<unsigned>(bx), static_cast<unsigned>(n)),
                     dim3(threads), 0, stream, items);
  return hipGetLastError();
}

}  // namespace s5d
