// Instantiations of the direct (one step per launch) kernels: every kernel
// kind, radius 1..4 and shape, in 2D and 3D.
#include "direct.h"
#include "stream2d.h"
#include "stream3d.h"

namespace s5d {
namespace {

// 2D: the row-streaming kernel (stream2d.h), except for float64 box
// stencils of radius 3 and 4, whose row-streaming threads need too many
// registers and lose to the LDS-staged tiles (measured on MI355X at 16384^2:
// 185 vs 191 GCell/s for radius 3, 104 vs 162 for radius 4; in float32 row
// streaming wins, 435 vs 271 and 327 vs 236); 3D: the row-streaming kernel
// (stream3d.h) for star stencils and the 27-point box (at 512^3: 473 vs 235
// GCell/s float32, 217 vs 138 float64), the LDS-staged tiles for larger boxes,
// whose row-streaming waves hold too many rows in registers (box3d2r float32
// 122 vs 127, float64 11 vs 70).
template <typename T, int ACC, int R, bool BOX>
Kernel2D make2d() {
  if constexpr (BOX && R >= 3 && std::is_same_v<T, double>)
    return Kernel2D{&launch_direct2d<T, ACC, R, BOX>,
                    &occupancy_direct<T, ACC, 2, R, BOX>,
                    0,
                    1,
                    direct_dx<2, R>(),
                    &fill_direct2d<R>,
                    &launch_direct_batch<T, ACC, 2, R, BOX>,
                    static_cast<int>(sizeof(DirectArgs))};
  else
    return Kernel2D{&launch_stream2d<T, ACC, R, BOX>,
                    &occupancy_stream2d<T, ACC, R, BOX>,
                    0,
                    1,
                    kStreamThreads * stream2d_cpl<T>(),
                    &fill_stream2d<T, ACC, R>,
                    &launch_stream2d_batch<T, ACC, R, BOX>,
                    static_cast<int>(sizeof(Stream2DArgs))};
}

template <typename T, int ACC, int R, bool BOX>
Kernel3D make3d() {
  if constexpr (!BOX || R == 1)
    return Kernel3D{&launch_stream3d<T, ACC, R, BOX>,
                    &occupancy_stream3d<T, ACC, R, BOX>,
                    0,
                    1,
                    kStream3DThreads / 64,
                    1,
                    &fill_stream3d<T, R, BOX>,
                    &launch_stream3d_batch<T, ACC, R, BOX>,
                    static_cast<int>(sizeof(Stream3DArgs))};
  else
    return Kernel3D{&launch_direct3d<T, ACC, R, BOX>,
                    &occupancy_direct<T, ACC, 3, R, BOX>,
                    0,
                    kDirectY3,
                    1,
                    1,
                    &fill_direct3d<R>,
                    &launch_direct_batch<T, ACC, 3, R, BOX>,
                    static_cast<int>(sizeof(DirectArgs))};
}

template <typename T, int ACC>
Kernel2D pick2d(int r, bool box) {
  switch (r * 2 + box) {
    case 2: return make2d<T, ACC, 1, false>();
    case 3: return make2d<T, ACC, 1, true>();
    case 4: return make2d<T, ACC, 2, false>();
    case 5: return make2d<T, ACC, 2, true>();
    case 6: return make2d<T, ACC, 3, false>();
    case 7: return make2d<T, ACC, 3, true>();
    case 8: return make2d<T, ACC, 4, false>();
    case 9: return make2d<T, ACC, 4, true>();
    default: return Kernel2D{};
  }
}

template <typename T, int ACC>
Kernel3D pick3d(int r, bool box) {
  switch (r * 2 + box) {
    case 2: return make3d<T, ACC, 1, false>();
    case 3: return make3d<T, ACC, 1, true>();
    case 4: return make3d<T, ACC, 2, false>();
    case 5: return make3d<T, ACC, 2, true>();
    case 6: return make3d<T, ACC, 3, false>();
    case 7: return make3d<T, ACC, 3, true>();
    case 8: return make3d<T, ACC, 4, false>();
    case 9: return make3d<T, ACC, 4, true>();
    default: return Kernel3D{};
  }
}

}  // namespace

Kernel2D direct_kernel2d(int kind, int r, bool box) {
  if (kind == KIND_F32) return pick2d<float, 0>(r, box);
  if (kind == KIND_F64) return pick2d<double, 0>(r, box);
  if (kind == KIND_F32_COMP) return pick2d<float, 1>(r, box);
  return Kernel2D{};
}

Kernel3D direct_kernel3d(int kind, int r, bool box) {
  if (kind == KIND_F32) return pick3d<float, 0>(r, box);
  if (kind == KIND_F64) return pick3d<double, 0>(r, box);
  if (kind == KIND_F32_COMP) return pick3d<float, 1>(r, box);
  return Kernel3D{};
}

}  // namespace s5d
