// Internal interfaces shared by the host scheduler and the kernel units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s5d {

// Stencil points: star 2*r*d + 1, box (2r+1)^d (AN5D Table 3).
constexpr int npts(int ndim, int r, bool box) {
  return box ? (ndim == 2 ? (2 * r + 1) * (2 * r + 1) : (2 * r + 1) * (2 * r + 1) * (2 * r + 1))
             : 2 * r * ndim + 1;
}

// Columns of overlap on the left and right of a tile (the last axis): at
// least bt*r each (the valid width shrinks by r per side and level), chosen so
// that the tile's first column and the compute width are multiples of
// 16 bytes / elem: with the tile at column R + t*C - left, every tile then
// starts on the same 16-byte phase of its row, 0 when the row pitch is a
// multiple of 16 bytes, so the lanes' vector loads are aligned.
constexpr int overlap_left(int bt, int r, int elem) {
  int x = bt * r;
  while ((x - r) % (16 / elem) != 0) ++x;
  return x;
}
constexpr int overlap_right(int bt, int r, int elem) {
  int y = bt * r;
  while ((overlap_left(bt, r, elem) + y) % (16 / elem) != 0) ++y;
  return y;
}
// Compute-region width of a tile of w columns.
constexpr int compute_width(int w, int bt, int r, int elem) {
  return w - overlap_left(bt, r, elem) - overlap_right(bt, r, elem);
}

// Coefficients travel by value in the kernel arguments, so they are loaded
// into scalar registers once per wave and feed every FMA as an SGPR operand.
template <typename T, int N>
struct CoefPack {
  T c[N];
};

// Everything one launch of a 2D round needs besides the coefficients.
struct Round2D {
  const void* src;
  void* dst;
  int32_t I0, I1;   // interior extents (axis 0 streams)
  int32_t chunk;    // h_SN: output rows per stream block
  const double* coeffs;  // host, canonical order
  const void* dcoef;     // device copy in the working type (direct kernels)
  hipStream_t stream;
};

// Geometry of one 2D launch, derived on the host.
struct Sweep2DArgs {
  const void* src;
  void* dst;
  int32_t I0, I1;
  int32_t ntiles;   // tiles across axis 1
  int32_t nwaves;   // ntiles * stream blocks
  int32_t chunk;    // h_SN
  int32_t pad;
};

using Launch2DFn = hipError_t (*)(const Round2D&);
using Occupancy2DFn = int (*)();   // resident workgroups per CU (0 if unknown)

// Batched launches: one launch runs a round of many grids that share a kernel
// variant.  The host writes one item per grid (its launch geometry and its
// coefficients in the variant's layout, item_bytes each) and one BlockMap
// entry per workgroup of the launch: which item, and which workgroup of that
// grid's own launch it stands for.
struct BlockMap {
  int32_t item;
  int32_t block;
};
using FillItem2DFn = int (*)(void* item, const Round2D& rd);  // returns the grid's workgroups
using LaunchBatchFn = hipError_t (*)(const void* items, const BlockMap* map, int nblocks, hipStream_t stream);

struct Kernel2D {
  Launch2DFn launch;
  Occupancy2DFn occupancy;
  int cpl;       // cells per lane
  int bt;        // fused time steps
  int tile;      // 64 * cpl
  FillItem2DFn fill_item;
  LaunchBatchFn launch_batch;
  int item_bytes;
};

// One compiled 2D kernel variant.  The build enumerates the variants (one
// object file each) and writes the table kRegistry2D.
// Kernel kinds: the element type and the accumulation policy of a variant.
enum { KIND_F32 = 0, KIND_F64 = 1, KIND_F32_COMP = 2 };

struct Entry2D {
  int dtype;   // kernel kind: KIND_F32, KIND_F64 or KIND_F32_COMP
  int box;     // 0 = star, 1 = box
  int r;
  int cpl;
  int bt;
  Kernel2D (*make)();
};
extern const Entry2D kRegistry2D[];
extern const int kRegistry2DSize;

// Everything one launch of a 3D round needs besides the coefficients.
struct Round3D {
  const void* src;
  void* dst;
  int32_t I0, I1, I2;  // interior extents (axis 0 streams)
  int32_t chunk;       // h_SN: output planes per stream block
  const double* coeffs;  // host, canonical order
  const void* dcoef;     // device copy in the working type (direct kernels)
  hipStream_t stream;
};

struct Sweep3DArgs {
  const void* src;
  void* dst;
  int32_t I0, I1, I2;
  int32_t nt1, nt2;  // tiles along axes 1 and 2
  int32_t chunk;
};

using Launch3DFn = hipError_t (*)(const Round3D&);
using FillItem3DFn = int (*)(void* item, const Round3D& rd);

struct Kernel3D {
  Launch3DFn launch;
  Occupancy2DFn occupancy;  // resident workgroups per CU
  int cpl;                  // cells per lane along axis 2
  int m;                    // rows per wave along axis 1
  int nw;                   // waves per workgroup (tile rows = nw * m)
  int bt;
  FillItem3DFn fill_item;
  LaunchBatchFn launch_batch;
  int item_bytes;
};

struct Entry3D {
  int dtype;  // kernel kind, as for Entry2D
  int box, r, cpl, m, nw, bt;
  Kernel3D (*make)();
};
extern const Entry3D kRegistry3D[];
extern const int kRegistry3DSize;

// Direct (one step per launch) kernels: the variant for a kernel kind,
// dimensionality, radius (1..4) and shape (direct.hip).  As for the blocked
// kernels, bt is 1 and tile fields describe the staged tile.
Kernel2D direct_kernel2d(int kind, int r, bool box);
Kernel3D direct_kernel3d(int kind, int r, bool box);

// Copy the boundary cells (width r on every face) of a padded grid.
hipError_t launch_halo_copy(const void* src, void* dst, int elem_bytes, int ndim,
                            const int64_t* padded, int r, hipStream_t stream);

constexpr int kWavesPerBlock = 4;

}  // namespace s5d
