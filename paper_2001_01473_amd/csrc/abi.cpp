// C ABI of libstencil5d.so: descriptor validation, blocking choice and the
// round scheduler (AN5D "Host Code": repeated launches of b_T fused steps, the
// last rounds shortened so the result lands where the modulo double buffer
// of the C program leaves it).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "host.h"
#include "norms.h"

using s5d::Entry2D;
using s5d::Entry3D;
using s5d::Kernel2D;
using s5d::Kernel3D;
using s5d::KIND_F32;
using s5d::KIND_F32_COMP;
using s5d::KIND_F64;

namespace {

thread_local std::string g_last_error;

}  // namespace

namespace s5d {

s5d_status fail(s5d_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

s5d_status device_fail(hipError_t e, const char* what) {
  return fail(S5D_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

}  // namespace s5d

using s5d::device_fail;
using s5d::fail;

namespace {

// Largest radius with kernels, per dimensionality and shape.
// (radius 1..4 for every shape: the direct kernels cover what no blocked
// variant does)
int max_radius(int ndim, int shape) {
  (void)ndim;
  (void)shape;
  return 4;
}

const Entry3D* find3d(int kind, int expr, int box, int r, int cpl, int m, int nw, int bt) {
  for (int i = 0; i < s5d::kRegistry3DSize; ++i) {
    const Entry3D& e = s5d::kRegistry3D[i];
    if (e.dtype == kind && e.expr == expr && e.box == box && e.r == r && e.cpl == cpl && e.m == m && e.nw == nw &&
        e.bt == bt)
      return &e;
  }
  return nullptr;
}

// 3D defaults: depth and rows per wave (tile family: 2 rows per wave is the
// 16-wave tile, 4 the 8-wave one), the best pair measured on MI355X at 512^3,
// T = 1000, and a floor on the stream-block length where
// the measured optimum lies above the chooser's pick (the float32 27-point
// box: 64 planes, 620 GCell/s against 566 at the chooser's 19).  Compensated
// accumulation is bound by arithmetic from the first level on.
struct Default3D {
  int bt, m;
  int hmin = 0;  // stream-block floor (planes), for extents of at least 4 * hmin
};
Default3D default_tuning3(int kind, int box, int r, int expr = 0) {
  if (expr == s5d::EXPR_DIV) return kind == KIND_F64 ? Default3D{2, 2} : Default3D{2, 4};
  if (kind == KIND_F32_COMP) return {1, 2};
  if (kind == KIND_F64) {
    if (r == 1) return box ? Default3D{2, 4} : Default3D{3, 2};
    return box ? Default3D{1, 2} : Default3D{2, 2};
  }
  if (r == 1) return box ? Default3D{2, 4, 64} : Default3D{3, 2};
  return box ? Default3D{1, 4} : Default3D{2, 4};
}
int default_bt3(int kind, int box, int r, int expr) { return default_tuning3(kind, box, r, expr).bt; }

// Stencils whose direct kernel measured faster than every blocked variant
// on MI355X.  3D at 512^3: the 125-point float32 box, the compensated
// 27-point box, and the compensated stars (row streaming: 501 vs 433 GCell/s
// for the 7-point star, 309 vs 194 for the 13-point one).  2D at 16384^2:
// every compensated stencil but the 5-point star (row streaming against the
// best blocked depth: star r = 2..4 487 / 360 / 289 vs 450 / 294 / 229,
// box r = 1, 2 562 / 250 vs 417 / 181; the 5-point star keeps b_T = 3, 843
// vs 697).
bool prefer_direct(int kind, int ndim, int box, int r) {
  if (ndim == 2) return kind == KIND_F32_COMP && (box || r >= 2);
  if (ndim != 3) return false;
  if (!box) return kind == KIND_F32_COMP && r <= 2;
  return (kind == KIND_F32 && r == 2) || (kind == KIND_F32_COMP && r == 1);
}

// Is any blocked variant compiled for this stencil?
bool has_blocked(int kind, int expr, int ndim, int box, int r) {
  if (ndim == 2) {
    for (int i = 0; i < s5d::kRegistry2DSize; ++i) {
      const Entry2D& e = s5d::kRegistry2D[i];
      if (e.dtype == kind && e.expr == expr && e.box == box && e.r == r) return true;
    }
    return false;
  }
  for (int i = 0; i < s5d::kRegistry3DSize; ++i) {
    const Entry3D& e = s5d::kRegistry3D[i];
    if (e.dtype == kind && e.expr == expr && e.box == box && e.r == r) return true;
  }
  return false;
}

const Entry2D* find2d(int kind, int expr, int box, int r, int cpl, int bt) {
  for (int i = 0; i < s5d::kRegistry2DSize; ++i) {
    const Entry2D& e = s5d::kRegistry2D[i];
    if (e.dtype == kind && e.expr == expr && e.box == box && e.r == r && e.cpl == cpl && e.bt == bt) return &e;
  }
  return nullptr;
}

int max_bt2d(int kind, int expr, int box, int r, int cpl) {
  int best = 0;
  for (int i = 0; i < s5d::kRegistry2DSize; ++i) {
    const Entry2D& e = s5d::kRegistry2D[i];
    if (e.dtype == kind && e.expr == expr && e.box == box && e.r == r && e.cpl == cpl) best = std::max(best, e.bt);
  }
  return best;
}

// Defaults when the caller leaves b_T and the cells per lane to the library:
// the best pair the autotuner measured on MI355X at 16384^2, per (kind, shape,
// radius).  Low-order stencils take deep temporal blocking (AN5D "Scaling
// Performance"); high-order and box stencils shallower, where the per-level
// work and the register window grow.
struct Default2D {
  int bt, cpl;
};
Default2D default_tuning(int kind, int box, int r, int expr = 0) {
  // expression stencils: the division costs an IEEE quotient per cell and
  // level, gradient2d a square root and a quotient (bound by arithmetic from
  // b_T = 2 on), per-cell weights n extra loads per cell and level; one tile
  // width each (4 float32 / 2 float64 cells per lane)
  if (expr == s5d::EXPR_GRADIENT || expr == s5d::EXPR_VARCOEF) return {2, kind == KIND_F64 ? 2 : 4};
  if (expr == s5d::EXPR_DIV) {
    const int c = kind == KIND_F64 ? 2 : 4;
    if (box) return {kind == KIND_F64 ? 6 : 5, c};
    return {r == 1 ? 8 : 5, c};
  }
  static const Default2D f32_star[4] = {{10, 4}, {7, 4}, {5, 4}, {3, 4}};
  static const Default2D f32_box[4] = {{7, 4}, {3, 4}, {2, 4}, {1, 4}};
  static const Default2D f64_star[4] = {{10, 2}, {6, 2}, {3, 4}, {2, 4}};
  static const Default2D f64_box[4] = {{9, 2}, {4, 2}, {2, 4}, {2, 4}};
  static const Default2D comp_star[4] = {{3, 4}, {3, 4}, {1, 4}, {1, 4}};
  static const Default2D comp_box[4] = {{3, 4}, {1, 4}, {1, 4}, {1, 4}};
  const int i = std::min(std::max(r, 1), 4) - 1;  // radius 1..4 (larger radii have no kernels)
  if (kind == KIND_F32) return box ? f32_box[i] : f32_star[i];
  if (kind == KIND_F32_COMP) return box ? comp_box[i] : comp_star[i];
  return box ? f64_box[i] : f64_star[i];
}
int default_bt(int kind, int box, int r, int expr) { return default_tuning(kind, box, r, expr).bt; }

struct DeviceInfo {
  int cus = 256;
  bool ok = false;
};

DeviceInfo query_device() {
  DeviceInfo d;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return d;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
    d.cus = cus;
    d.ok = true;
  } else {
    (void)hipGetLastError();
  }
  return d;
}

// Stream-block length h_SN (AN5D "Division of Streaming Dimension" and the
// SM efficiency of its "Performance Model"): a block of h rows costs
// h + 2*b_T*r row-steps (the warm-up and drain of the fused levels); the
// launch takes the blocks' total work spread over `slots` resident units plus
// a tail of about kTail block durations, as the last blocks finish unevenly
// (measured on MI355X: many short blocks beat one wave of long ones).
// Minimise  max(blocks / slots, 1) * (h + 2 b_T r) + kTail * (h + 2 b_T r).
constexpr double kTail = 0.75;

int choose_chunk(int64_t I0, int64_t ntiles, int64_t slots, int bt, int r) {
  const int64_t hmin = std::max<int64_t>(8, static_cast<int64_t>(bt) * r);
  int64_t best_h = I0;
  double best_cost = 1e300;
  const int64_t max_nch = std::max<int64_t>(1, I0 / hmin);
  for (int64_t nch = 1; nch <= max_nch && nch <= 65536; ++nch) {
    const int64_t h = (I0 + nch - 1) / nch;
    const int64_t blocks = ntiles * ((I0 + h - 1) / h);
    const double per = static_cast<double>(h + 2LL * bt * r);
    const double cost = std::max(static_cast<double>(blocks) / static_cast<double>(slots), 1.0) * per + kTail * per;
    if (cost < best_cost * (1.0 - 1e-9)) {
      best_cost = cost;
      best_h = h;
    }
  }
  return static_cast<int>(std::min<int64_t>(best_h, INT32_MAX));
}

// A whole sweep as (n_full rounds of bt) followed by up to three shorter
// rounds; the total round count has the parity of T, so the result lands in
// buffer T % 2 (AN5D "Host Code").
struct RoundSchedule {
  int64_t n_full = 0;
  int bt = 1;
  int tail[3] = {0, 0, 0};
  int n_tail = 0;
  int64_t total() const { return n_full + n_tail; }
};

RoundSchedule schedule_rounds(int64_t T, int bt) {
  RoundSchedule s;
  s.bt = bt;
  if (T <= 0) return s;
  const int64_t n = (T + bt - 1) / bt;
  const int last = static_cast<int>(T - (n - 1) * bt);
  if ((n % 2) == (T % 2)) {
    if (last == bt) {
      s.n_full = n;
    } else {
      s.n_full = n - 1;
      s.tail[s.n_tail++] = last;
    }
  } else if (last >= 2) {
    s.n_full = n - 1;
    s.tail[s.n_tail++] = last - 1;
    s.tail[s.n_tail++] = 1;
  } else {
    // last == 1 and n >= 2 (n == 1 would mean T == 1, which matches parity);
    // a mismatch needs bt >= 2, so the round before can give up one step.
    s.n_full = n - 2;
    s.tail[s.n_tail++] = bt - 1;
    s.tail[s.n_tail++] = 1;
    s.tail[s.n_tail++] = 1;
  }
  return s;
}

}  // namespace

namespace {

// Direct kernels: one step per launch; the device coefficient table is made
// here (the only device allocation of a plan).
s5d_status plan_direct(s5d_plan* p, const s5d_tuning& req, int box, int r) {
  if (req.bt > 1 || req.cells_per_lane > 0 || req.rows_per_wave > 0 || req.tile0 > 0 || req.tile1 > 0 ||
      req.stream_chunk > 0)
    return fail(S5D_EINVAL, "direct kernels take no blocking parameters");
  if (p->d.ndim == 2) {
    p->by_bt[1] = s5d::direct_kernel2d(p->kind, r, box != 0);
    if (!p->by_bt[1].launch) return fail(S5D_EUNSUPPORTED, "no direct 2D kernel for this stencil");
    p->tun.tile0 = p->by_bt[1].tile;
  } else {
    p->by_bt3[1] = s5d::direct_kernel3d(p->kind, r, box != 0);
    if (!p->by_bt3[1].launch) return fail(S5D_EUNSUPPORTED, "no direct 3D kernel for this stencil");
    p->tun.tile0 = p->by_bt3[1].m;
  }
  p->direct = true;
  p->tun.bt = 1;
  p->tun.kernel = S5D_KERNEL_DIRECT;
  const size_t n = p->coeffs.size();
  std::vector<unsigned char> host(n * static_cast<size_t>(p->elem));
  for (size_t k = 0; k < n; ++k) {
    if (p->elem == 4) {
      const float v = static_cast<float>(p->coeffs[k]);
      std::memcpy(host.data() + 4 * k, &v, 4);
    } else {
      std::memcpy(host.data() + 8 * k, &p->coeffs[k], 8);
    }
  }
  void* dev = nullptr;
  hipError_t e = hipMalloc(&dev, host.size());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return device_fail(e, "hipMalloc of the coefficient table");
  }
  p->dcoef = std::shared_ptr<void>(dev, [](void* q) { (void)hipFree(q); });
  e = hipMemcpy(dev, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return device_fail(e, "upload of the coefficient table");
  return S5D_OK;
}

s5d_status plan_2d(s5d_plan* p, const s5d_tuning& req, int box, int r) {
  const s5d_desc& d = p->d;
  int cpl = req.cells_per_lane;
  if (req.tile0 > 0) {
    if (req.tile0 % 64 != 0) return fail(S5D_EINVAL, "tile0 must be a multiple of 64 (one wave64 per tile)");
    if (cpl > 0 && cpl * 64 != req.tile0) return fail(S5D_EINVAL, "tile0 != 64 * cells_per_lane");
    cpl = req.tile0 / 64;
  }
  if (req.tile1 > 0 || req.rows_per_wave > 0) return fail(S5D_EINVAL, "tile1 and rows_per_wave are 3D fields");
  int bt = req.bt;
  const int ex = p->expr;
  if (cpl == 0) {
    // the default tile width, if it is built to the requested (or default) depth
    const int c = default_tuning(p->kind, box, r, ex).cpl;
    if (max_bt2d(p->kind, ex, box, r, c) >= (bt > 0 ? bt : default_bt(p->kind, box, r, ex))) cpl = c;
  }
  if (cpl == 0) {
    // widest tile that still reaches the requested (or default) depth
    const int want = bt > 0 ? bt : default_bt(p->kind, box, r, ex);
    int best_cpl = 0, best_bt = 0;
    for (int c : {4, 2, 8}) {
      const int mb = std::min(want, max_bt2d(p->kind, ex, box, r, c));
      if (mb > best_bt) {
        best_bt = mb;
        best_cpl = c;
      }
    }
    if (best_cpl == 0) return fail(S5D_EUNSUPPORTED, "no kernel variant for this stencil");
    cpl = best_cpl;
  }
  const int bt_cap = max_bt2d(p->kind, ex, box, r, cpl);
  if (bt_cap == 0) return fail(S5D_EUNSUPPORTED, "no kernel with cells_per_lane=" + std::to_string(cpl));
  if (bt == 0) bt = std::min(default_bt(p->kind, box, r, ex), bt_cap);
  if (bt > bt_cap)
    return fail(S5D_EUNSUPPORTED, "bt=" + std::to_string(bt) + " exceeds the deepest kernel built for this stencil (" +
                                      std::to_string(bt_cap) + ")");
  if (d.steps > 0 && bt > d.steps) bt = static_cast<int>(d.steps);
  for (int b = 1; b <= bt; ++b) {
    const Entry2D* e = find2d(p->kind, ex, box, r, cpl, b);
    if (!e) return fail(S5D_EUNSUPPORTED, "kernel variant missing for bt=" + std::to_string(b));
    p->by_bt[b] = e->make();
  }
  int chunk = req.stream_chunk;
  {
    const DeviceInfo dev = query_device();
    int occ = dev.ok ? p->by_bt[bt].occupancy() : 0;
    if (occ <= 0) occ = 2;
    p->slots = static_cast<int64_t>(dev.cus) * occ * s5d::kWavesPerBlock;
  }
  if (chunk == 0) {
    const int64_t C = s5d::compute_width(64 * cpl, bt, r, p->elem);
    const int64_t ntiles = (d.interior[1] + C - 1) / C;
    chunk = choose_chunk(d.interior[0], ntiles, p->slots, bt, r);
    p->chunk_auto = true;
  }
  if (chunk < 1) return fail(S5D_EINVAL, "stream_chunk must be >= 1");
  p->tun.bt = bt;
  p->tun.tile0 = 64 * cpl;
  p->tun.stream_chunk = chunk;
  p->tun.cells_per_lane = cpl;
  return S5D_OK;
}

s5d_status plan_3d(s5d_plan* p, const s5d_tuning& req, int box, int r) {
  const s5d_desc& d = p->d;
  // tile shape: the (cells per lane, rows per wave, waves) family built for
  // this stencil; explicit fields must match one of them
  const Entry3D* fam = nullptr;
  int bt_cap = 0;
  // without an explicit shape, the default family if it is built
  int want_m = req.rows_per_wave;
  const int ex = p->expr;
  if (want_m == 0 && req.cells_per_lane == 0 && req.tile0 == 0 && req.tile1 == 0) {
    const int m = default_tuning3(p->kind, box, r, ex).m;
    for (int i = 0; i < s5d::kRegistry3DSize && want_m == 0; ++i) {
      const Entry3D& e = s5d::kRegistry3D[i];
      if (e.dtype == p->kind && e.expr == ex && e.box == box && e.r == r && e.m == m) want_m = m;
    }
  }
  for (int i = 0; i < s5d::kRegistry3DSize; ++i) {
    const Entry3D& e = s5d::kRegistry3D[i];
    if (e.dtype != p->kind || e.expr != ex || e.box != box || e.r != r) continue;
    if (req.cells_per_lane > 0 && e.cpl != req.cells_per_lane) continue;
    if (want_m > 0 && e.m != want_m) continue;
    if (req.tile0 > 0 && e.m * e.nw != req.tile0) continue;
    if (req.tile1 > 0 && 64 * e.cpl != req.tile1) continue;
    if (!fam || (e.cpl == fam->cpl && e.m == fam->m && e.nw == fam->nw)) {
      fam = &e;
      bt_cap = std::max(bt_cap, e.bt);
    }
  }
  if (!fam) return fail(S5D_EUNSUPPORTED, "no 3D kernel for this stencil and tile shape");
  int bt = req.bt > 0 ? req.bt : std::min(default_bt3(p->kind, box, r, ex), bt_cap);
  if (bt > bt_cap)
    return fail(S5D_EUNSUPPORTED, "bt=" + std::to_string(bt) + " exceeds the deepest 3D kernel built (" +
                                      std::to_string(bt_cap) + ")");
  if (d.steps > 0 && bt > d.steps) bt = static_cast<int>(d.steps);
  for (int b = 1; b <= bt; ++b) {
    const Entry3D* e = find3d(p->kind, ex, box, r, fam->cpl, fam->m, fam->nw, b);
    if (!e) return fail(S5D_EUNSUPPORTED, "3D kernel variant missing for bt=" + std::to_string(b));
    p->by_bt3[b] = e->make();
  }
  const int B1 = fam->m * fam->nw, B2 = 64 * fam->cpl;
  int chunk = req.stream_chunk;
  if (chunk == 0) {
    const DeviceInfo dev = query_device();
    int occ = dev.ok ? p->by_bt3[bt].occupancy() : 0;
    if (occ <= 0) occ = 1;
    const int64_t C1 = B1 - 2LL * bt * r, C2 = s5d::compute_width(B2, bt, r, p->elem);
    const int64_t ntiles = ((d.interior[1] + C1 - 1) / C1) * ((d.interior[2] + C2 - 1) / C2);
    const int64_t slots = static_cast<int64_t>(dev.cus) * occ;  // resident workgroups
    chunk = choose_chunk(d.interior[0], ntiles, slots, bt, r);
    const Default3D def = default_tuning3(p->kind, box, r, ex);
    if (def.hmin > 0 && bt == def.bt && fam->m == def.m && d.interior[0] >= 4LL * def.hmin)
      chunk = std::max(chunk, def.hmin);
  }
  if (chunk < 1) return fail(S5D_EINVAL, "stream_chunk must be >= 1");
  p->tun.bt = bt;
  p->tun.tile0 = B1;
  p->tun.tile1 = B2;
  p->tun.stream_chunk = chunk;
  p->tun.cells_per_lane = fam->cpl;
  p->tun.rows_per_wave = fam->m;
  return S5D_OK;
}

}  // namespace

namespace s5d {

std::vector<int> plan_rounds(const s5d_plan* p) {
  const RoundSchedule rs = schedule_rounds(p->d.steps, p->tun.bt);
  std::vector<int> out;
  out.reserve(static_cast<size_t>(rs.total()));
  for (int64_t i = 0; i < rs.n_full; ++i) out.push_back(rs.bt);
  for (int i = 0; i < rs.n_tail; ++i) out.push_back(rs.tail[i]);
  return out;
}

namespace {
Round2D round2d(const s5d_plan* p, const void* src, void* dst, hipStream_t stream, const void* fields = nullptr) {
  Round2D rd;
  rd.fields = fields;
  rd.dcoef = p->dcoef.get();
  rd.src = src;
  rd.dst = dst;
  rd.I0 = static_cast<int32_t>(p->d.interior[0]);
  rd.I1 = static_cast<int32_t>(p->d.interior[1]);
  rd.chunk = p->tun.stream_chunk;
  rd.coeffs = p->coeffs.data();
  rd.stream = stream;
  return rd;
}
Round3D round3d(const s5d_plan* p, const void* src, void* dst, hipStream_t stream) {
  Round3D rd;
  rd.dcoef = p->dcoef.get();
  rd.src = src;
  rd.dst = dst;
  rd.I0 = static_cast<int32_t>(p->d.interior[0]);
  rd.I1 = static_cast<int32_t>(p->d.interior[1]);
  rd.I2 = static_cast<int32_t>(p->d.interior[2]);
  rd.chunk = p->tun.stream_chunk;
  rd.coeffs = p->coeffs.data();
  rd.stream = stream;
  return rd;
}
}  // namespace

hipError_t launch_round(const s5d_plan* p, int bt, const void* src, void* dst, hipStream_t stream,
                        const void* fields) {
  if (p->d.ndim == 3) return p->by_bt3[bt].launch(round3d(p, src, dst, stream));
  return p->by_bt[bt].launch(round2d(p, src, dst, stream, fields));
}

BatchHooks batch_hooks(const s5d_plan* p, int bt) {
  if (p->d.ndim == 3) return BatchHooks{p->by_bt3[bt].launch_batch, p->by_bt3[bt].item_bytes};
  return BatchHooks{p->by_bt[bt].launch_batch, p->by_bt[bt].item_bytes};
}

int fill_round_item(const s5d_plan* p, int bt, const void* src, void* dst, void* item, int chunk) {
  if (p->d.ndim == 3) {
    Round3D rd = round3d(p, src, dst, nullptr);
    if (chunk > 0) rd.chunk = chunk;
    return p->by_bt3[bt].fill_item(item, rd);
  }
  Round2D rd = round2d(p, src, dst, nullptr);
  if (chunk > 0) rd.chunk = chunk;
  return p->by_bt[bt].fill_item(item, rd);
}

int fill_persist_round(const s5d_plan* p, const Persist2D& k, int bt, const void* src, void* dst, void* out,
                       int chunk, int grid, int need) {
  Round2D rd = round2d(p, src, dst, nullptr);
  if (chunk > 0) rd.chunk = chunk;
  return k.fill_round(out, rd, bt, grid, need);
}

int shared_chunk(const s5d_plan* p, int bt, double share) {
  if (p->direct || !p->chunk_auto || p->d.ndim != 2 || bt < 1 || p->slots <= 0) return p->tun.stream_chunk;
  const int r = p->d.radius;
  const int64_t C = s5d::compute_width(64 * p->tun.cells_per_lane, bt, r, p->elem);
  const int64_t ntiles = (p->d.interior[1] + C - 1) / C;
  const double all = static_cast<double>(p->slots);  // the plan's own variant (depth p->tun.bt)
  const int64_t slots = std::max<int64_t>(1, static_cast<int64_t>(all * std::min(1.0, std::max(share, 0.0))));
  return choose_chunk(p->d.interior[0], ntiles, slots, bt, r);
}

hipError_t launch_boundary_copy(const s5d_plan* p, const void* buf0, void* buf1, hipStream_t stream) {
  return launch_halo_copy(buf0, buf1, p->elem, p->d.ndim, p->padded, p->d.radius, stream);
}

s5d_status check_buffers(const s5d_plan* p, const void* buf0, const void* buf1) {
  if (!buf0 || !buf1) return fail(S5D_EINVAL, "buffer pointer is NULL");
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(buf0), a1 = reinterpret_cast<uintptr_t>(buf1);
  const uintptr_t nb = static_cast<uintptr_t>(p->bytes);
  if (a0 < a1 + nb && a1 < a0 + nb) return fail(S5D_EINVAL, "buffers overlap");
  if (a0 % p->elem != 0 || a1 % p->elem != 0) return fail(S5D_EINVAL, "buffers not aligned to the element size");
  return S5D_OK;
}

}  // namespace s5d

extern "C" {

const char* s5d_status_string(s5d_status status) {
  switch (status) {
    case S5D_OK: return "S5D_OK";
    case S5D_EINVAL: return "S5D_EINVAL";
    case S5D_EUNSUPPORTED: return "S5D_EUNSUPPORTED";
    case S5D_ENOMEM: return "S5D_ENOMEM";
    case S5D_EDEVICE: return "S5D_EDEVICE";
    case S5D_EBUDGET: return "S5D_EBUDGET";
    case S5D_ECANCELED: return "S5D_ECANCELED";
    case S5D_ETIMEDOUT: return "S5D_ETIMEDOUT";
    default: return "S5D_UNKNOWN";
  }
}

const char* s5d_last_error(void) { return g_last_error.c_str(); }

s5d_status s5d_plan_create(const s5d_desc* desc, const s5d_tuning* tuning, s5d_plan** out) {
  g_last_error.clear();
  if (!out) return fail(S5D_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(S5D_EINVAL, "desc is NULL");
  if (desc->struct_size < sizeof(s5d_desc)) return fail(S5D_EINVAL, "desc->struct_size too small");
  const s5d_desc& d = *desc;
  if (d.ndim != 2 && d.ndim != 3) return fail(S5D_EINVAL, "ndim must be 2 or 3");
  if (d.radius < 1) return fail(S5D_EINVAL, "radius must be >= 1");
  if (d.shape != S5D_STAR && d.shape != S5D_BOX) return fail(S5D_EINVAL, "shape must be S5D_STAR or S5D_BOX");
  if (d.dtype != S5D_F32 && d.dtype != S5D_F64) return fail(S5D_EINVAL, "dtype must be S5D_F32 or S5D_F64");
  if (d.accum != S5D_ACC_PLAIN && d.accum != S5D_ACC_COMPENSATED)
    return fail(S5D_EINVAL, "accum must be S5D_ACC_PLAIN or S5D_ACC_COMPENSATED");
  if (d.accum == S5D_ACC_COMPENSATED && d.dtype != S5D_F32)
    return fail(S5D_EINVAL, "compensated accumulation is defined for float32 grids only");
  if (d.steps < 0) return fail(S5D_EINVAL, "steps must be >= 0");
  if (d.radius > 64) return fail(S5D_EINVAL, "radius out of range");
  if (d.expr < S5D_EXPR_LINEAR || d.expr > S5D_EXPR_VARCOEF)
    return fail(S5D_EINVAL, "expr must be one of S5D_EXPR_LINEAR, _DIV, _GRADIENT, _VARCOEF");
  if (d.reserved != 0) return fail(S5D_EINVAL, "desc->reserved must be 0");
  if (d.expr != S5D_EXPR_LINEAR && d.accum != S5D_ACC_PLAIN)
    return fail(S5D_EUNSUPPORTED, "compensated accumulation is built for the linear stencils only");
  if (d.expr == S5D_EXPR_GRADIENT && (d.ndim != 2 || d.radius != 1 || d.shape != S5D_STAR))
    return fail(S5D_EINVAL, "gradient2d is the 2D star of radius 1");
  int64_t n_points = d.shape == S5D_BOX ? 1 : 2LL * d.radius * d.ndim + 1;
  if (d.shape == S5D_BOX)
    for (int a = 0; a < d.ndim; ++a) n_points *= 2LL * d.radius + 1;
  const int64_t n_expected = d.expr == S5D_EXPR_LINEAR ? n_points
                             : d.expr == S5D_EXPR_DIV  ? n_points + 1
                             : d.expr == S5D_EXPR_GRADIENT ? 2
                                                           : 0;
  if (d.n_coeffs != n_expected)
    return fail(S5D_EINVAL, "n_coeffs is " + std::to_string(d.n_coeffs) + ", the stencil and expression take " +
                                std::to_string(n_expected));
  if (n_expected > 0 && !d.coeffs) return fail(S5D_EINVAL, "coeffs is NULL");
  if (d.expr == S5D_EXPR_DIV && d.coeffs[n_expected - 1] == 0.0) return fail(S5D_EINVAL, "the divisor c0 is 0");
  for (int64_t k = 0; k < d.n_coeffs; ++k)
    if (!std::isfinite(d.coeffs[k])) return fail(S5D_EINVAL, "coefficient " + std::to_string(k) + " is not finite");
  int64_t total = 1;
  int64_t padded[3] = {1, 1, 1};
  for (int a = 0; a < d.ndim; ++a) {
    if (d.interior[a] < 1) return fail(S5D_EINVAL, "interior extents must be >= 1");
    if (d.interior[a] > (1LL << 30)) return fail(S5D_EINVAL, "interior extent too large");
    padded[a] = d.interior[a] + 2LL * d.radius;
    total *= padded[a];
    if (total > (1LL << 31) - 1) return fail(S5D_EUNSUPPORTED, "padded grid exceeds 2^31-1 cells");
  }

  // kernels address one padded row through a buffer descriptor whose range
  // is a 32-bit byte count
  if (padded[d.ndim - 1] * (d.dtype == S5D_F32 ? 4 : 8) >= (1LL << 31))
    return fail(S5D_EUNSUPPORTED, "padded row exceeds 2^31 bytes");

  s5d_tuning req;
  std::memset(&req, 0, sizeof(req));
  if (tuning) {
    if (tuning->struct_size < sizeof(s5d_tuning)) return fail(S5D_EINVAL, "tuning->struct_size too small");
    req = *tuning;
    if (req.bt < 0 || req.tile0 < 0 || req.tile1 < 0 || req.stream_chunk < 0 || req.cells_per_lane < 0 ||
        req.waves_per_eu < 0)
      return fail(S5D_EINVAL, "tuning fields must be >= 0");
    if (req.kernel != S5D_KERNEL_AUTO && req.kernel != S5D_KERNEL_BLOCKED && req.kernel != S5D_KERNEL_DIRECT)
      return fail(S5D_EINVAL, "kernel must be S5D_KERNEL_AUTO, _BLOCKED or _DIRECT");
    if (req.bt > 15) return fail(S5D_EINVAL, "bt must be <= 15");
    if (req.waves_per_eu != 0) return fail(S5D_EINVAL, "waves_per_eu is reserved and must be 0");
  }

  if (d.radius > max_radius(d.ndim, d.shape))
    return fail(S5D_EUNSUPPORTED, "no kernel for this dimensionality/shape/radius");

  const int box = d.shape == S5D_BOX ? 1 : 0;
  const int r = d.radius;
  s5d_plan* p = new (std::nothrow) s5d_plan;
  if (!p) return fail(S5D_ENOMEM, "plan allocation failed");
  p->d = d;
  p->expr = d.expr;
  try {
    if (d.n_coeffs > 0) p->coeffs.assign(d.coeffs, d.coeffs + d.n_coeffs);
  } catch (...) {
    delete p;
    return fail(S5D_ENOMEM, "coefficient copy failed");
  }
  p->d.coeffs = nullptr;
  for (int a = 0; a < 3; ++a) p->padded[a] = padded[a];
  p->elem = d.dtype == S5D_F32 ? 4 : 8;
  p->kind = d.accum == S5D_ACC_COMPENSATED ? KIND_F32_COMP : d.dtype == S5D_F32 ? KIND_F32 : KIND_F64;
  p->bytes = total * p->elem;
  auto reset = [&]() {
    for (int b = 0; b < 16; ++b) {
      p->by_bt[b] = Kernel2D{};
      p->by_bt3[b] = Kernel3D{};
    }
    p->direct = false;
    p->chunk_auto = false;
    p->slots = 0;
    p->dcoef.reset();
    std::memset(&p->tun, 0, sizeof(p->tun));
    p->tun.struct_size = sizeof(s5d_tuning);
  };
  reset();
  // without a tuning, an autotuned choice for this stencil and extent bucket
  // is taken if one is cached and still valid; else the library's defaults
  s5d_tuning cached;
  s5d_status st = S5D_EINVAL;
  s5d::load_default_tuning();
  if (!tuning && s5d::tune_cache_lookup(d, &cached)) {
    st = d.ndim == 2 ? plan_2d(p, cached, box, r) : plan_3d(p, cached, box, r);
    if (st != S5D_OK) {
      g_last_error.clear();
      reset();
    } else {
      // the library chose it (through the tuner), not the caller: batches and
      // servers may still size the stream blocks for a grid's share
      p->chunk_auto = true;
    }
  }
  const bool no_blocking = req.bt <= 1 && req.cells_per_lane == 0 && req.rows_per_wave == 0 && req.tile0 == 0 &&
                           req.tile1 == 0 && req.stream_chunk == 0;
  // b_T = 1 asked for: the row-streaming direct kernel (2D stars and boxes of
  // radius <= 2, the 3D 7-point star and 27-point box; plain or compensated
  // accumulation) is faster than the blocked kernel at depth 1 (compensated
  // at 16384^2: star2d1r 697 vs 539 GCell/s, box2d1r 562 vs 389)
  const bool linear = d.expr == S5D_EXPR_LINEAR;
  if (!linear && req.kernel == S5D_KERNEL_DIRECT)
    return fail(S5D_EUNSUPPORTED, "expression stencils run on the blocked kernels only");
  const bool stream_bt1 = linear && req.kernel == S5D_KERNEL_AUTO && no_blocking && req.bt == 1 &&
                          ((d.ndim == 2 && (!box || r <= 2)) || (d.ndim == 3 && r == 1));
  if (st != S5D_OK) {
    if (req.kernel == S5D_KERNEL_DIRECT || stream_bt1 ||
        (linear && req.kernel == S5D_KERNEL_AUTO && no_blocking && req.bt == 0 &&
         prefer_direct(p->kind, d.ndim, box, r))) {
      st = plan_direct(p, req, box, r);
    } else {
      st = d.ndim == 2 ? plan_2d(p, req, box, r) : plan_3d(p, req, box, r);
      // no blocked variant for this stencil: the direct kernels, unless the
      // caller asked for blocking or gave blocking parameters
      if (st == S5D_EUNSUPPORTED && linear && req.kernel == S5D_KERNEL_AUTO && no_blocking &&
          !has_blocked(p->kind, 0, d.ndim, box, r)) {
        g_last_error.clear();
        reset();
        st = plan_direct(p, req, box, r);
      }
    }
  }
  if (st == S5D_OK) p->tun.kernel = p->direct ? S5D_KERNEL_DIRECT : S5D_KERNEL_BLOCKED;
  if (st != S5D_OK) {
    delete p;
    return st;
  }
  *out = p;
  return S5D_OK;
}

void s5d_plan_destroy(s5d_plan* plan) { delete plan; }

s5d_status s5d_plan_query(const s5d_plan* plan, s5d_tuning* chosen, int64_t* bytes_per_buffer) {
  if (!plan) return fail(S5D_EINVAL, "plan is NULL");
  if (chosen) {
    if (chosen->struct_size != 0 && chosen->struct_size < sizeof(s5d_tuning))
      return fail(S5D_EINVAL, "chosen->struct_size too small");
    *chosen = plan->tun;
  }
  if (bytes_per_buffer) *bytes_per_buffer = plan->bytes;
  return S5D_OK;
}

s5d_status s5d_run(const s5d_plan* plan, void* buf0, void* buf1, void* stream, int32_t* result_index) {
  g_last_error.clear();
  if (plan && plan->expr == S5D_EXPR_VARCOEF)
    return fail(S5D_EINVAL, "a plan with per-cell weights runs through s5d_run_fields");
  return s5d_run_fields(plan, buf0, buf1, nullptr, stream, result_index);
}

s5d_status s5d_run_fields(const s5d_plan* plan, void* buf0, void* buf1, const void* fields, void* stream,
                          int32_t* result_index) {
  g_last_error.clear();
  if (!plan) return fail(S5D_EINVAL, "plan is NULL");
  if ((plan->expr == S5D_EXPR_VARCOEF) != (fields != nullptr))
    return fail(S5D_EINVAL, plan->expr == S5D_EXPR_VARCOEF ? "fields is NULL" : "fields given for a plan without per-cell weights");
  if (fields && (reinterpret_cast<uintptr_t>(fields) % plan->elem) != 0)
    return fail(S5D_EINVAL, "fields not aligned to the element size");
  const s5d_status bst = s5d::check_buffers(plan, buf0, buf1);
  if (bst != S5D_OK) return bst;
  const int64_t T = plan->d.steps;
  if (result_index) *result_index = static_cast<int32_t>(T % 2);
  if (T == 0) return S5D_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  hipError_t e = s5d::launch_boundary_copy(plan, buf0, buf1, st);
  if (e != hipSuccess) return device_fail(e, "boundary copy launch");
  void* bufs[2] = {buf0, buf1};
  const std::vector<int> rounds = s5d::plan_rounds(plan);
  for (size_t k = 0; k < rounds.size(); ++k) {
    e = s5d::launch_round(plan, rounds[k], bufs[k % 2], bufs[(k + 1) % 2], st, fields);
    if (e != hipSuccess) return device_fail(e, "sweep launch");
  }
  return S5D_OK;
}

int64_t s5d_error_norms_workspace_bytes(int64_t n) {
  if (n < 0) return -1;
  return static_cast<int64_t>(s5d::error_norms_parts(n)) * 5 * static_cast<int64_t>(sizeof(double));
}

s5d_status s5d_error_norms(const void* got, int32_t got_dtype, const void* ref, int32_t ref_dtype, int64_t n,
                           double* out, void* workspace, int64_t workspace_bytes, void* stream) {
  g_last_error.clear();
  if (n < 0) return fail(S5D_EINVAL, "n must be >= 0");
  if ((got_dtype != S5D_F32 && got_dtype != S5D_F64) || (ref_dtype != S5D_F32 && ref_dtype != S5D_F64))
    return fail(S5D_EINVAL, "dtypes must be S5D_F32 or S5D_F64");
  if (!out || !workspace) return fail(S5D_EINVAL, "out and workspace must not be NULL");
  if (n > 0 && (!got || !ref)) return fail(S5D_EINVAL, "got and ref must not be NULL");
  if ((n > 0 && ((reinterpret_cast<uintptr_t>(got) | reinterpret_cast<uintptr_t>(ref)) & 15)) ||
      ((reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(workspace)) & 7))
    return fail(S5D_EINVAL, "got and ref must be 16-byte aligned, out and workspace 8-byte aligned");
  if (workspace_bytes < s5d_error_norms_workspace_bytes(n))
    return fail(S5D_EINVAL, "workspace smaller than s5d_error_norms_workspace_bytes(n)");
  const uintptr_t o0 = reinterpret_cast<uintptr_t>(out), w0 = reinterpret_cast<uintptr_t>(workspace);
  if (o0 < w0 + static_cast<uintptr_t>(workspace_bytes) && w0 < o0 + S5D_NORMS_COUNT * sizeof(double))
    return fail(S5D_EINVAL, "out overlaps the workspace");
  const hipError_t e = s5d::launch_error_norms(got, got_dtype == S5D_F64, ref, ref_dtype == S5D_F64, n, out,
                                               static_cast<double*>(workspace), s5d::error_norms_parts(n),
                                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "error-norm launch");
  return S5D_OK;
}

s5d_status s5d_error_norms_noalloc(const void* got, int32_t got_dtype, const void* ref, int32_t ref_dtype,
                                   int64_t n, double* out, void* stream) {
  g_last_error.clear();
  if (n < 0) return fail(S5D_EINVAL, "n must be >= 0");
  if ((got_dtype != S5D_F32 && got_dtype != S5D_F64) || (ref_dtype != S5D_F32 && ref_dtype != S5D_F64))
    return fail(S5D_EINVAL, "dtypes must be S5D_F32 or S5D_F64");
  if (!out) return fail(S5D_EINVAL, "out must not be NULL");
  if (n > 0 && (!got || !ref)) return fail(S5D_EINVAL, "got and ref must not be NULL");
  if ((n > 0 && ((reinterpret_cast<uintptr_t>(got) | reinterpret_cast<uintptr_t>(ref)) & 15)) ||
      (reinterpret_cast<uintptr_t>(out) & 7))
    return fail(S5D_EINVAL, "got and ref must be 16-byte aligned, out 8-byte aligned");
  const int64_t need = s5d_error_norms_workspace_bytes(n);
  if (need > s5d::error_norms_scratch_bytes())
    return fail(S5D_EINVAL, "n needs " + std::to_string(need) + " bytes of partials, more than the " +
                                std::to_string(s5d::error_norms_scratch_bytes()) + "-byte scratch");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (stream) {
    hipDevice_t sdev = -1;
    e = hipStreamGetDevice(static_cast<hipStream_t>(stream), &sdev);
    if (e != hipSuccess) return device_fail(e, "hipStreamGetDevice");
    if (sdev != dev) return fail(S5D_EINVAL, "stream belongs to another device than the current one");
  }
  double* scratch = nullptr;
  e = s5d::error_norms_scratch(&scratch);
  if (e != hipSuccess) return device_fail(e, "address of the norm scratch");
  e = s5d::launch_error_norms(got, got_dtype == S5D_F64, ref, ref_dtype == S5D_F64, n, out, scratch,
                              s5d::error_norms_parts(n), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "error-norm launch");
  return S5D_OK;
}

}  // extern "C"
