// Performance model and autotuner for the blocking parameters.
//
// The model follows AN5D's "Performance Model": count what every thread does
// per launch -- computation, global (HBM) traffic, shared-memory (LDS)
// traffic -- divide each total by the device's rate for it, take the largest
// as the launch time and divide by the workgroup-slot efficiency.  What is
// counted is re-derived for these kernels: a wave64 holds a tile of 64*CPL
// columns (2D) or a workgroup holds NW*M rows by 64*CPL columns (3D); every
// lane computes every fused level (there are no idle threads to discount);
// lanes outside the grid move no data; LDS carries only the 3D edge-row
// exchange.  The tuner enumerates the compiled variants and a set of stream
// block lengths, ranks them by the model, measures the best few on the GPU and
// caches the winner per (stencil, dtype, accumulation, extent bucket).
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "host.h"

namespace s5d {
namespace {

// Device rates.  VALU lane-operations per clock per CU: 64 in float32 and in
// float64.  The kernels are built without packed float32 instructions, and
// unpacked float32 FMAs issue at the float64 rate: 64 lanes per clock per CU
// (78.6e12 flop/s at 256 CUs and 2.4 GHz; MI355X's published 157.3 TFLOP/s
// float32 peak counts packed operations).  HBM: the practical streaming rate
// (a plain device copy sustains about 6 TB/s of the 8 TB/s peak).  LDS: 128
// bytes per clock per CU.
struct Rates {
  double valu, hbm, lds;  // valu: lane-operations per second
  int cus;
};

Rates device_rates() {
  Rates r{256 * 64 * 2.4e9, 6.0e12, 256 * 128 * 2.4e9, 256};
  int dev = 0, cus = 0, khz = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
    double clock = 2.4e9;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev) == hipSuccess && khz > 0)
      clock = khz * 1e3;
    r.cus = cus;
    r.valu = cus * 64.0 * clock;
    r.lds = cus * 128.0 * clock;
  }
  (void)hipGetLastError();
  return r;
}

// VALU lane-operations per cell per fused level.
double ops_per_cell(const s5d_plan* p, int cpl) {
  const int r = p->d.radius, nd = p->d.ndim;
  const bool box = p->d.shape == S5D_BOX;
  const int n = static_cast<int>(p->expr == EXPR_LINEAR ? p->coeffs.size()
                                                         : (box ? (nd == 2 ? (2 * r + 1) * (2 * r + 1)
                                                                           : (2 * r + 1) * (2 * r + 1) * (2 * r + 1))
                                                                : 2 * r * nd + 1));
  const int words = p->elem / 4;
  // terms: one FMA each, or the compensated sequence (two products split
  // exactly, a two-sum and two adds: nine operations) plus its final add
  double ops = p->kind == KIND_F32_COMP ? 9.0 * (n - 1) + 3.0 : static_cast<double>(n);
  // expressions: an IEEE quotient (about 10 float32 / 16 float64 operations);
  // gradient2d: 4 differences, 4 squares, 4 sums, a square root and a
  // quotient (about 12 + 20 / 12 + 36) replacing the weighted sum; per-cell
  // weights: one extra load per term (counted with the loads below)
  const bool f64 = p->elem == 8;
  if (p->expr == EXPR_DIV) ops = static_cast<double>(n - 1) + (f64 ? 16.0 : 10.0);
  if (p->expr == EXPR_GRADIENT) ops = f64 ? 48.0 : 32.0;
  if (p->expr == EXPR_VARCOEF) ops = static_cast<double>(n) * 1.5;
  // lane exchange: R cells from each neighbouring lane for every row that
  // needs in-row neighbours (one row for a star, 2r+1 rows or planes x rows
  // for a box), by 32-bit DPP moves -- except in the 2D plain float32 star
  // and 3x3 box kernels, which fold the shift into the FMA
  const int rows_ext = box ? (nd == 2 ? 2 * r + 1 : (2 * r + 1) * (2 * r + 1)) : (nd == 2 ? 1 : 1);
  const bool folded = nd == 2 && p->kind == KIND_F32 && (!box || r == 1);
  if (!folded) ops += static_cast<double>(rows_ext) * 2.0 * r * words / cpl;
  ops += 0.5;  // loads, stores, ring bookkeeping, per cell
  return ops;
}

// Tail of a launch in workgroup durations (as in the stream-block chooser).
constexpr double kTail = 0.75;

// Rows [a, b) clipped to [0, n).
int64_t clip(int64_t a, int64_t b, int64_t n) { return std::max<int64_t>(0, std::min(b, n) - std::max<int64_t>(a, 0)); }

struct RoundModel {
  double ops = 0, gm = 0, lds = 0;
  int64_t wgs = 0;
  int wg_per_cu = 2;
};

RoundModel model_round2d(const s5d_plan* p, int bt) {
  RoundModel m;
  const int r = p->d.radius, cpl = p->tun.cells_per_lane, W = 64 * cpl;
  const int LO = overlap_left(bt, r, p->elem), C = compute_width(W, bt, r, p->elem);
  const int64_t I0 = p->d.interior[0], I1 = p->d.interior[1], P0 = I0 + 2 * r, P1 = I1 + 2 * r;
  const int64_t h = p->tun.stream_chunk, w = p->elem;
  const Bands2D g = make_bands2d(static_cast<int>(I0), static_cast<int>(h));
  const int64_t ntiles = (I1 + C - 1) / C;
  int64_t cols_read = 0, cols_written = 0;
  for (int64_t t = 0; t < ntiles; ++t) {
    const int64_t c0 = r + t * C;
    cols_read += clip(c0 - LO, c0 - LO + W, P1);
    cols_written += std::min<int64_t>(C, I1 - t * C);
  }
  double rows_read = 0, rows_comp = 0;
  int64_t blocks = 0;  // non-empty stream blocks
  for (int x = 0; x < g.nb; ++x)
    for (int c = 0; c < g.n1 + g.n2; ++c) {
      int a = 0, b = 0;
      band_rows2d(g, r, static_cast<int>(I0), x, c, a, b);
      if (b <= a) continue;
      ++blocks;
      rows_read += clip(a - static_cast<int64_t>(bt) * r, b + static_cast<int64_t>(bt) * r, P0);
      for (int T = 1; T <= bt; ++T) rows_comp += static_cast<double>(b - a) + 2.0 * (bt - T) * r;
    }
  m.gm = (rows_read * cols_read + static_cast<double>(I0) * cols_written) * w;
  if (p->expr == EXPR_VARCOEF) {
    // the weights of every cell, once per round from HBM (the levels re-read
    // them from the caches)
    const int n = p->d.shape == S5D_BOX ? (2 * r + 1) * (2 * r + 1) : 4 * r + 1;
    m.gm += static_cast<double>(n) * static_cast<double>(I0) * static_cast<double>(I1) * w;
  }
  m.ops = rows_comp * W * ntiles * ops_per_cell(p, cpl);
  m.wgs = (ntiles * blocks + kWavesPerBlock - 1) / kWavesPerBlock;
  const int occ = p->by_bt[bt].occupancy ? p->by_bt[bt].occupancy() : 0;
  m.wg_per_cu = occ > 0 ? occ : 2;
  return m;
}

// Direct kernels: one step per launch; HBM moves each cell once in and once
// out (the tile margins come from L2), LDS takes the staged tile once and one
// read per term and cell.
RoundModel model_round_direct(const s5d_plan* p) {
  RoundModel m;
  const int nd = p->d.ndim, r = p->d.radius;
  const int64_t w = p->elem;
  double cells = 1, staged = 1;
  int64_t tiles = 1;
  // 2D: one row of 512 x (16 bytes / w) cells per workgroup, no LDS (box
  // radius 3-4: LDS tiles of 16 x 64); 3D stars: about 8 rows of 64 x (16
  // bytes / w) cells per workgroup (one per wave), no LDS; 3D boxes: LDS
  // tiles of 4 x 8 x (64, or 32 for r >= 3) cells
  const bool lds2 = p->d.shape == S5D_BOX && r >= 3;
  const bool lds3 = p->d.shape == S5D_BOX;
  const int dims2[2] = {lds2 ? 16 : 1, lds2 ? 64 : 512 * 16 / static_cast<int>(w)};
  const int dims3[3] = {lds3 ? 4 : 1, lds3 ? 8 : 8, lds3 ? (r >= 3 ? 32 : 64) : 64 * 16 / static_cast<int>(w)};
  for (int a = 0; a < nd; ++a) {
    const int64_t I = p->d.interior[a];
    const int D = nd == 2 ? dims2[a] : dims3[a];
    const int64_t n = (I + D - 1) / D;
    tiles *= n;
    cells *= static_cast<double>(I);
    staged *= static_cast<double>(D + 2 * r);
  }
  const double n_terms = static_cast<double>(p->coeffs.size());
  m.gm = 2.0 * cells * w;
  const double ops_term = p->kind == KIND_F32_COMP ? 9.0 : 1.0;
  const bool uses_lds = (nd == 3 && lds3) || (nd == 2 && lds2);
  m.ops = cells * (n_terms * ops_term + 2.0) + (uses_lds ? static_cast<double>(tiles) * staged * 2.0 : 0.0);
  m.lds = uses_lds ? cells * n_terms * w + static_cast<double>(tiles) * staged * w : 0.0;
  m.wgs = tiles;
  const Kernel2D& k2 = p->by_bt[1];
  const Kernel3D& k3 = p->by_bt3[1];
  const int occ = nd == 2 ? (k2.occupancy ? k2.occupancy() : 0) : (k3.occupancy ? k3.occupancy() : 0);
  m.wg_per_cu = occ > 0 ? occ : 2;
  return m;
}

RoundModel model_round3d(const s5d_plan* p, int bt) {
  RoundModel m;
  const Kernel3D& k = p->by_bt3[bt];
  const int r = p->d.radius, cpl = k.cpl, B1 = k.nw * k.m, B2 = 64 * cpl;
  const int LO2 = overlap_left(bt, r, p->elem);
  const int C1 = B1 - 2 * bt * r, C2 = compute_width(B2, bt, r, p->elem);
  const int64_t I0 = p->d.interior[0], I1 = p->d.interior[1], I2 = p->d.interior[2];
  const int64_t P0 = I0 + 2 * r, P1 = I1 + 2 * r, P2 = I2 + 2 * r;
  const int64_t h = p->tun.stream_chunk, w = p->elem;
  const int64_t nt1 = (I1 + C1 - 1) / C1, nt2 = (I2 + C2 - 1) / C2, nch = (I0 + h - 1) / h;
  double rows_read = 0, rows_written = 0, cols_read = 0, cols_written = 0;
  for (int64_t t = 0; t < nt1; ++t) {
    const int64_t a = r + t * C1 - static_cast<int64_t>(bt) * r;
    rows_read += clip(a, a + B1, P1);
    rows_written += std::min<int64_t>(C1, I1 - t * C1);
  }
  for (int64_t t = 0; t < nt2; ++t) {
    const int64_t a = r + t * C2 - LO2;
    cols_read += clip(a, a + B2, P2);
    cols_written += std::min<int64_t>(C2, I2 - t * C2);
  }
  double planes_read = 0, planes_comp = 0;
  for (int64_t c = 0; c < nch; ++c) {
    const int64_t a = r + c * h, b = std::min<int64_t>(a + h, I0 + r);
    planes_read += clip(a - static_cast<int64_t>(bt) * r, b + static_cast<int64_t>(bt) * r, P0);
    for (int T = 1; T <= bt; ++T) planes_comp += static_cast<double>(b - a) + 2.0 * (bt - T) * r;
  }
  m.gm = (planes_read * rows_read * cols_read + static_cast<double>(I0) * rows_written * cols_written) * w;
  const double cells_comp = planes_comp * static_cast<double>(B1) * B2 * nt1 * nt2;
  m.ops = cells_comp * ops_per_cell(p, cpl);
  // each wave writes and reads its 2r edge rows per level and plane
  m.lds = planes_comp * nt1 * nt2 * k.nw * 2.0 * (2.0 * r * B2 * w);
  m.wgs = nt1 * nt2 * nch;
  const int occ = k.occupancy ? k.occupancy() : 0;
  m.wg_per_cu = occ > 0 ? occ : 1;
  return m;
}

}  // namespace

s5d_status model_plan(const s5d_plan* p, s5d_model* out) {
  const Rates rt = device_rates();
  double t_alu = 0, t_hbm = 0, t_lds = 0, total = 0, ops = 0, bytes = 0, eff_main = 1;
  int64_t wgs_main = 0;
  const std::vector<int> rounds = plan_rounds(p);
  std::map<int, RoundModel> cache;
  for (size_t k = 0; k < rounds.size(); ++k) {
    const int bt = rounds[k];
    auto it = cache.find(bt);
    if (it == cache.end())
      it = cache
               .emplace(bt, p->direct ? model_round_direct(p)
                                      : (p->d.ndim == 3 ? model_round3d(p, bt) : model_round2d(p, bt)))
               .first;
    const RoundModel& m = it->second;
    const double valu = rt.valu;  // float32 (unpacked) and float64 issue at one rate
    const double ta = m.ops / valu, tg = m.gm / rt.hbm, tl = m.lds / rt.lds;
    // slot efficiency: with fewer workgroups than resident slots the machine
    // is part idle; otherwise the last workgroups finish unevenly, a tail of
    // about kTail workgroup durations (one workgroup lasts body * slots / wgs)
    const double slots = static_cast<double>(rt.cus) * m.wg_per_cu;
    const double frac = slots / static_cast<double>(std::max<int64_t>(m.wgs, 1));
    const double fill = 1.0 / (std::max(1.0, frac) + kTail * std::min(1.0, frac));
    total += std::max(ta, std::max(tg, tl)) / fill;
    t_alu += ta;
    t_hbm += tg;
    t_lds += tl;
    ops += m.ops;
    bytes += m.gm;
    if (k == 0) {
      eff_main = fill;
      wgs_main = m.wgs;
    }
  }
  out->seconds = total;
  out->t_alu = t_alu;
  out->t_hbm = t_hbm;
  out->t_lds = t_lds;
  out->bound = (t_alu >= t_hbm && t_alu >= t_lds) ? 0 : (t_hbm >= t_lds ? 1 : 2);
  out->eff_cu = eff_main;
  out->hbm_bytes = bytes;
  out->valu_ops = ops;
  out->workgroups = wgs_main;
  return S5D_OK;
}

// ---------------------------------------------------------------------------
// Tuning cache, keyed by stencil, dtype, accumulation and the power-of-two
// bucket of every extent.
namespace {

using Key = std::tuple<int, int, int, int, int, int, int, int, int>;

Key key_of(const s5d_desc& d) {
  auto bucket = [](int64_t x) { return x <= 1 ? 0 : static_cast<int>(std::ceil(std::log2(static_cast<double>(x)))); };
  return Key{d.ndim, d.shape, d.radius, d.dtype, d.accum, d.expr, bucket(d.interior[0]), bucket(d.interior[1]),
             d.ndim == 3 ? bucket(d.interior[2]) : 0};
}

// The winner's stream-block length was measured for one set of extents: it is
// kept for exactly those, while other extents of the same bucket have it
// chosen again for their own size (stream_chunk = 0).
struct CacheEntry {
  s5d_tuning tun;
  double sec_per_step;
  int64_t interior[3];
};

std::mutex g_cache_mu;
std::map<Key, CacheEntry> g_cache;

}  // namespace

void load_default_tuning() {
  static std::once_flag once;
  std::call_once(once, [] {
    std::string path;
    if (const char* env = std::getenv("S5D_TUNING_FILE")) {
      path = env;  // an empty value disables the file
    } else {
      Dl_info info;
      if (dladdr(reinterpret_cast<void*>(&load_default_tuning), &info) && info.dli_fname) {
        const std::string so = info.dli_fname;
        const size_t slash = so.rfind('/');
        path = (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tuning_gfx950.txt";
      }
    }
    if (path.empty()) return;
    if (FILE* f = std::fopen(path.c_str(), "r")) {
      std::fclose(f);
      // a malformed file leaves the library's own defaults in place
      (void)s5d_tune_cache_load(path.c_str());
      clear_error();
    }
  });
}

bool tune_cache_lookup(const s5d_desc& d, s5d_tuning* tun) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(key_of(d));
  if (it == g_cache.end()) return false;
  *tun = it->second.tun;
  bool same = true;
  for (int a = 0; a < d.ndim; ++a) same = same && it->second.interior[a] == d.interior[a];
  if (!same) tun->stream_chunk = 0;
  return true;
}

}  // namespace s5d

using s5d::device_fail;
using s5d::fail;

namespace {

struct Candidate {
  s5d_tuning tun;
  double model = 0, measured = -1;
};

// Time one candidate: a sweep of two full rounds (2*b_T steps) on scratch
// buffers, after one warm-up; returns seconds per time step.
s5d_status measure(const s5d_desc& d, const s5d_tuning& tun, void* b0, void* b1, const void* fields, hipStream_t st,
                   int reps, double* sec_per_step) {
  s5d_desc dd = d;
  dd.steps = 2LL * tun.bt;
  s5d_plan* p = nullptr;
  s5d_status rc = s5d_plan_create(&dd, &tun, &p);
  if (rc != S5D_OK) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) rc = s5d_run_fields(p, b0, b1, fields, st, nullptr);
  if (e == hipSuccess && rc == S5D_OK) e = hipEventRecord(e0, st);
  for (int i = 0; e == hipSuccess && rc == S5D_OK && i < reps; ++i) rc = s5d_run_fields(p, b0, b1, fields, st, nullptr);
  if (e == hipSuccess && rc == S5D_OK) e = hipEventRecord(e1, st);
  if (e == hipSuccess && rc == S5D_OK) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess && rc == S5D_OK) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  s5d_plan_destroy(p);
  if (rc != S5D_OK) return rc;
  if (e != hipSuccess) return device_fail(e, "autotune timing");
  *sec_per_step = ms * 1e-3 / reps / static_cast<double>(dd.steps);
  return S5D_OK;
}

}  // namespace

extern "C" {

s5d_status s5d_plan_model(const s5d_plan* plan, s5d_model* out) {
  s5d::clear_error();
  if (!plan || !out) return fail(S5D_EINVAL, "plan and out must not be NULL");
  if (out->struct_size < sizeof(s5d_model)) return fail(S5D_EINVAL, "out->struct_size too small");
  return s5d::model_plan(plan, out);
}

s5d_status s5d_autotune(const s5d_desc* desc, int32_t top_k, void* stream, s5d_tuning* best,
                        s5d_tune_report* report) {
  s5d::clear_error();
  if (!desc || !best) return fail(S5D_EINVAL, "desc and best must not be NULL");
  if (top_k < 0) return fail(S5D_EINVAL, "top_k must be >= 0");
  if (report && report->struct_size < sizeof(s5d_tune_report))
    return fail(S5D_EINVAL, "report->struct_size too small");
  // the library's own choice first: it validates the descriptor and is the
  // baseline the tuner must match
  s5d_plan* base = nullptr;
  s5d_status rc = s5d_plan_create(desc, nullptr, &base);
  if (rc != S5D_OK) return rc;
  const int64_t bytes = base->bytes;
  s5d_tuning base_tun;
  std::memset(&base_tun, 0, sizeof(base_tun));
  base_tun.struct_size = sizeof(s5d_tuning);
  (void)s5d_plan_query(base, &base_tun, nullptr);
  const bool base_direct = base->direct;
  s5d_plan_destroy(base);
  if (base_direct) {
    // a direct kernel has no blocking parameters: nothing to choose
    *best = base_tun;
    if (report) {
      report->n_candidates = 1;
      report->n_measured = 0;
      report->model_best_seconds = 0;
      report->best_seconds_per_step = -1;
      report->default_seconds_per_step = -1;
    }
    return S5D_OK;
  }

  // enumerate: every compiled depth and tile family, a ladder of stream
  // block lengths plus the library's own choice (stream_chunk = 0)
  const int kind = desc->accum == S5D_ACC_COMPENSATED ? s5d::KIND_F32_COMP : desc->dtype;
  const int box = desc->shape == S5D_BOX ? 1 : 0;
  std::vector<std::tuple<int, int, int>> fams;  // (cpl, rows_per_wave, bt)
  if (desc->ndim == 2) {
    for (int i = 0; i < s5d::kRegistry2DSize; ++i) {
      const s5d::Entry2D& e = s5d::kRegistry2D[i];
      if (e.dtype == kind && e.expr == desc->expr && e.box == box && e.r == desc->radius)
        fams.emplace_back(e.cpl, 0, e.bt);
    }
  } else {
    for (int i = 0; i < s5d::kRegistry3DSize; ++i) {
      const s5d::Entry3D& e = s5d::kRegistry3D[i];
      if (e.dtype == kind && e.expr == desc->expr && e.box == box && e.r == desc->radius)
        fams.emplace_back(e.cpl, e.m, e.bt);
    }
  }
  const int64_t I0 = desc->interior[0];
  std::vector<int> chunks{0};
  for (int64_t h = 32; h < I0; h *= 2) chunks.push_back(static_cast<int>(h));
  chunks.push_back(static_cast<int>(std::min<int64_t>(I0, INT32_MAX)));
  std::vector<Candidate> cands;
  for (const auto& f : fams) {
    if (desc->steps > 0 && std::get<2>(f) > desc->steps) continue;
    for (int h : chunks) {
      Candidate c;
      std::memset(&c.tun, 0, sizeof(c.tun));
      c.tun.struct_size = sizeof(s5d_tuning);
      c.tun.bt = std::get<2>(f);
      c.tun.cells_per_lane = std::get<0>(f);
      c.tun.rows_per_wave = std::get<1>(f);
      c.tun.stream_chunk = h;
      s5d_plan* p = nullptr;
      if (s5d_plan_create(desc, &c.tun, &p) != S5D_OK) continue;  // e.g. a missing shallower depth
      s5d_model m;
      m.struct_size = sizeof(m);
      s5d::model_plan(p, &m);
      (void)s5d_plan_query(p, &c.tun, nullptr);
      s5d_plan_destroy(p);
      c.model = m.seconds;
      cands.push_back(c);
    }
  }
  s5d::clear_error();
  if (cands.empty()) return fail(S5D_EUNSUPPORTED, "no kernel variant for this stencil");
  std::stable_sort(cands.begin(), cands.end(), [](const Candidate& a, const Candidate& b) { return a.model < b.model; });
  // drop duplicates (the library's choice may coincide with a ladder entry)
  std::vector<Candidate> uniq;
  for (const Candidate& c : cands) {
    bool dup = false;
    for (const Candidate& u : uniq)
      dup = dup || (u.tun.bt == c.tun.bt && u.tun.cells_per_lane == c.tun.cells_per_lane &&
                    u.tun.rows_per_wave == c.tun.rows_per_wave && u.tun.stream_chunk == c.tun.stream_chunk);
    if (!dup) uniq.push_back(c);
  }
  cands.swap(uniq);

  Candidate* win = &cands[0];
  bool base_won = false;
  double base_measured = -1;
  int n_measured = 0;
  if (top_k > 0 && desc->steps > 0) {
    void* b0 = nullptr;
    void* b1 = nullptr;
    void* fl = nullptr;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMalloc(&b0, static_cast<size_t>(bytes));
    if (e == hipSuccess) e = hipMalloc(&b1, static_cast<size_t>(bytes));
    if (e == hipSuccess) e = hipMemsetAsync(b0, 0, static_cast<size_t>(bytes), st);  // timing does not depend on values
    if (e == hipSuccess && desc->expr == S5D_EXPR_VARCOEF) {
      // per-cell weights for the timing runs (values do not matter either)
      const int64_t np = box ? (desc->ndim == 2 ? 1LL : (2LL * desc->radius + 1)) * (2LL * desc->radius + 1) *
                                   (2LL * desc->radius + 1)
                             : 2LL * desc->radius * desc->ndim + 1;
      const int64_t fb = np * desc->interior[0] * desc->interior[1] * (desc->dtype == S5D_F64 ? 8 : 4);
      e = hipMalloc(&fl, static_cast<size_t>(fb));
      if (e == hipSuccess) e = hipMemsetAsync(fl, 0, static_cast<size_t>(fb), st);
    }
    if (e != hipSuccess) {
      if (b0) (void)hipFree(b0);
      if (b1) (void)hipFree(b1);
      if (fl) (void)hipFree(fl);
      return device_fail(e, "autotune scratch buffers");
    }
    const int reps = 3;
    double best_t = 1e300;
    for (size_t i = 0; i < cands.size() && static_cast<int>(i) < top_k; ++i) {
      rc = measure(*desc, cands[i].tun, b0, b1, fl, st, reps, &cands[i].measured);
      if (rc != S5D_OK) break;
      ++n_measured;
      if (cands[i].measured < best_t) {
        best_t = cands[i].measured;
        win = &cands[i];
      }
    }
    if (rc == S5D_OK) rc = measure(*desc, base_tun, b0, b1, fl, st, reps, &base_measured);
    (void)hipStreamSynchronize(st);
    (void)hipFree(b0);
    (void)hipFree(b1);
    if (fl) (void)hipFree(fl);
    if (rc != S5D_OK) return rc;
    if (base_measured > 0 && base_measured < best_t) {
      // the library's own choice stays if no candidate beats it
      cands.push_back(Candidate{base_tun, 0.0, base_measured});
      win = &cands.back();
      base_won = true;
    }
  }
  *best = win->tun;
  if (!base_won) {
    // (the library's own choice needs no entry: plans without one get it)
    std::lock_guard<std::mutex> lk(s5d::g_cache_mu);
    s5d::g_cache[s5d::key_of(*desc)] =
        s5d::CacheEntry{win->tun, win->measured, {desc->interior[0], desc->interior[1], desc->interior[2]}};
  }
  if (report) {
    report->n_candidates = static_cast<int32_t>(cands.size());
    report->n_measured = n_measured;
    report->model_best_seconds = cands[0].model;
    report->best_seconds_per_step = win->measured;
    report->default_seconds_per_step = base_measured;
  }
  return S5D_OK;
}

s5d_status s5d_tune_cache_save(const char* path) {
  s5d::clear_error();
  if (!path) return fail(S5D_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(S5D_EINVAL, std::string("cannot open ") + path);
  std::lock_guard<std::mutex> lk(s5d::g_cache_mu);
  std::fprintf(f, "# stencil5d tuning cache v2: ndim shape radius dtype accum expr b0 b1 b2 : bt tile0 tile1 "
                  "stream_chunk cells_per_lane rows_per_wave : seconds_per_step : interior0 interior1 "
                  "interior2 (the extents stream_chunk was measured for)\n");
  for (const auto& kv : s5d::g_cache) {
    const auto& k = kv.first;
    const s5d_tuning& t = kv.second.tun;
    const int64_t* in = kv.second.interior;
    std::fprintf(f, "%d %d %d %d %d %d %d %d %d : %d %d %d %d %d %d : %.9g : %lld %lld %lld\n", std::get<0>(k),
                 std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k),
                 std::get<7>(k), std::get<8>(k), t.bt, t.tile0, t.tile1, t.stream_chunk, t.cells_per_lane, t.rows_per_wave,
                 kv.second.sec_per_step, static_cast<long long>(in[0]), static_cast<long long>(in[1]),
                 static_cast<long long>(in[2]));
  }
  const bool ok = std::fclose(f) == 0;
  return ok ? S5D_OK : fail(S5D_EINVAL, std::string("write failed: ") + path);
}

s5d_status s5d_tune_cache_load(const char* path) {
  s5d::clear_error();
  if (!path) return fail(S5D_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(S5D_EINVAL, std::string("cannot open ") + path);
  char line[512];
  std::map<s5d::Key, s5d::CacheEntry> loaded;
  bool bad = false;
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int k[9], t[6];
    double sec = 0;
    long long in[3] = {0, 0, 0};
    if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d : %d %d %d %d %d %d : %lf : %lld %lld %lld", &k[0], &k[1],
                    &k[2], &k[3], &k[4], &k[5], &k[6], &k[7], &k[8], &t[0], &t[1], &t[2], &t[3], &t[4], &t[5], &sec,
                    &in[0], &in[1], &in[2]) != 19) {
      bad = true;
      break;
    }
    s5d_tuning tun;
    std::memset(&tun, 0, sizeof(tun));
    tun.struct_size = sizeof(tun);
    tun.bt = t[0];
    tun.tile0 = t[1];
    tun.tile1 = t[2];
    tun.stream_chunk = t[3];
    tun.cells_per_lane = t[4];
    tun.rows_per_wave = t[5];
    loaded[s5d::Key{k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7], k[8]}] =
        s5d::CacheEntry{tun, sec, {static_cast<int64_t>(in[0]), static_cast<int64_t>(in[1]), static_cast<int64_t>(in[2])}};
  }
  std::fclose(f);
  if (bad) return fail(S5D_EINVAL, std::string("malformed tuning cache: ") + path);
  std::lock_guard<std::mutex> lk(s5d::g_cache_mu);
  for (const auto& kv : loaded) s5d::g_cache[kv.first] = kv.second;
  return S5D_OK;
}

void s5d_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(s5d::g_cache_mu);
  s5d::g_cache.clear();
}

}  // extern "C"
