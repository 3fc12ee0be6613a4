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

// Expressions of the blocked kernels: the plain weighted sum, or the weighted
// sum divided by one constant c0 (AN5D Table 3: j2d5pt, j2d9pt, j2d9pt-gol,
// j3d27pt), which travels after the weights.
enum { EXPR_LINEAR = 0, EXPR_DIV = 1, EXPR_GRADIENT = 2, EXPR_VARCOEF = 3 };
constexpr int ncoef(int ndim, int r, bool box, int expr) {
  return npts(ndim, r, box) + (expr == EXPR_DIV ? 1 : 0);
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
  const void* fields = nullptr;  // per-cell weights (variable-coefficient sweeps)
};

// Stream blocks of a 2D launch, laid out for the XCDs.  Workgroups are
// dispatched round-robin over the kXcds XCDs.  The rows are cut into nb bands
// (nb = 8, or fewer when a band would not hold one block of h_SN rows: 4, 2,
// 1) of hb = ceil(I0 / nb) rows; workgroup b works on band b % nb, so with
// nb = 8 band x runs on XCD x, and walks its blocks in the order b / nb.  A
// band is cut into n1 blocks of h1 rows followed by n2 blocks of h2 rows: when
// the band holds more than two blocks of h1 rows, its last rows go in blocks
// of h2 = h1 / 2 (h1 >= 32), so each XCD runs its long blocks first and ends
// on short ones, which shortens the tail of the launch; otherwise every block
// is h1 rows (h2 = h1, the last one possibly shorter).  Neighbouring tiles of
// a block row run on one XCD and share its L2.
constexpr int kXcds = 8;

struct Bands2D {
  int32_t nb;      // bands
  int32_t hb;      // rows per band
  int32_t h1, n1;  // long blocks: rows, count
  int32_t h2, n2;  // short blocks: rows, count
};

__host__ __device__ inline Bands2D make_bands2d(int I0, int chunk) {
  Bands2D g;
  const int h = chunk < 1 ? 1 : chunk;
  g.nb = kXcds;
  while (g.nb > 1 && (I0 + g.nb - 1) / g.nb < h) g.nb /= 2;
  g.hb = (I0 + g.nb - 1) / g.nb;
  g.h1 = h < g.hb ? h : g.hb;
  if (g.h1 < 1) g.h1 = 1;
  const int nfull = g.hb / g.h1;
  if (nfull > 2 && g.h1 >= 32) {
    g.n1 = nfull - 2;
    g.h2 = g.h1 / 2;
  } else {
    g.n1 = 0;
    g.h2 = g.h1;
  }
  g.n2 = (g.hb - g.n1 * g.h1 + g.h2 - 1) / g.h2;
  return g;
}

// Output rows [a, b) of block c of band x (empty when b <= a).  The fields
// are read into values first: a conditional over two fields of the struct
// would select between their addresses, and a struct indexed that way
// cannot stay in registers.
__host__ __device__ inline void band_rows2d(const Bands2D& g, int R, int I0, int x, int c, int& a, int& b) {
  const int hb = g.hb, h1 = g.h1, n1 = g.n1, h2 = g.h2;
  const int band0 = R + x * hb;
  const int band1 = band0 + hb < I0 + R ? band0 + hb : I0 + R;
  const bool lng = c < n1;
  a = lng ? band0 + c * h1 : band0 + n1 * h1 + (c - n1) * h2;
  const int e = a + (lng ? h1 : h2);
  b = e < band1 ? e : band1;
}

// Geometry of one 2D launch, derived on the host.
struct Sweep2DArgs {
  const void* src;
  void* dst;
  int32_t I0, I1;
  int32_t ntiles;   // tiles across axis 1
  int32_t nwaves;   // waves per band: ntiles * (n1 + n2)
  Bands2D g;        // stream blocks (h_SN = g.h1)
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
  int expr;    // EXPR_LINEAR or EXPR_DIV (window kernels: EXPR_GRADIENT, EXPR_VARCOEF)
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
  int expr;   // EXPR_LINEAR or EXPR_DIV
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

// The boundary copies of many grids in one launch: a device table of n items
// (at most 65535); max_cells = the largest halo_cells() among them.
struct HaloItem {
  const void* src;
  void* dst;
  int64_t P0, P1, P2;  // padded extents (P2 = 1 for 2D grids)
  int32_t r;           // boundary width
  int32_t elem;        // bytes per cell: 4 or 8
};
int64_t halo_cells(int ndim, const int64_t* padded, int r);
hipError_t launch_halo_copy_batch(const HaloItem* items, int n, int64_t max_cells, hipStream_t stream);

constexpr int kWavesPerBlock = 4;

}  // namespace s5d
