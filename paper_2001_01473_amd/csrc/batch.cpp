// Batched execution of many independent sweeps.
//
// Every grid keeps the round schedule its own plan gives it (the same rounds,
// fused depths and buffer order as s5d_run), so a batched result is bit for
// bit the result the grid gets alone.  What changes is how rounds reach the
// GPU: at round index k, the k-th rounds of all grids that run the same kernel
// variant go into ONE launch, whose workgroups are mapped to (grid, workgroup
// of that grid's own launch) by a table built here.  Small grids, which alone
// cannot fill 256 CUs, then share launches with the others, and the launch
// count drops from the sum of all grids' rounds to about one per round index
// and variant.  The whole sequence can be captured once into a HIP graph and
// replayed with one graph launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "batch.h"
#include "host.h"

namespace s5d {

namespace {
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
}  // namespace

s5d_status build_step(const std::vector<RoundItem>& items, std::vector<unsigned char>& blob,
                      std::vector<GroupLaunch>& out) {
  // group by kernel variant, in order of first appearance
  std::vector<LaunchBatchFn> order;
  std::map<LaunchBatchFn, std::vector<size_t>> groups;
  for (size_t i = 0; i < items.size(); ++i) {
    const BatchHooks h = batch_hooks(items[i].plan, items[i].bt);
    if (!h.launch) return fail(S5D_EUNSUPPORTED, "kernel variant without a batched entry point");
    auto it = groups.find(h.launch);
    if (it == groups.end()) {
      order.push_back(h.launch);
      groups[h.launch] = {i};
    } else {
      it->second.push_back(i);
    }
  }
  std::vector<unsigned char> scratch;
  for (LaunchBatchFn fn : order) {
    const std::vector<size_t>& members = groups[fn];
    const int item_bytes = batch_hooks(items[members[0]].plan, items[members[0]].bt).item_bytes;
    GroupLaunch g;
    g.fn = fn;
    g.items_off = align_up(blob.size(), 256);
    blob.resize(g.items_off + members.size() * static_cast<size_t>(item_bytes));
    std::vector<int> nblk(members.size());
    for (size_t j = 0; j < members.size(); ++j) {
      const RoundItem& ri = items[members[j]];
      // write through an aligned temporary: blob may reallocate below
      scratch.assign(static_cast<size_t>(item_bytes) + 16, 0);
      void* tmp = reinterpret_cast<void*>(align_up(reinterpret_cast<uintptr_t>(scratch.data()), 16));
      nblk[j] = fill_round_item(ri.plan, ri.bt, ri.src, ri.dst, tmp, ri.chunk);
      if (nblk[j] <= 0) return fail(S5D_EUNSUPPORTED, "grid too large for one launch");
      std::memcpy(blob.data() + g.items_off + j * static_cast<size_t>(item_bytes), tmp,
                  static_cast<size_t>(item_bytes));
    }
    // the largest grids first: their workgroups start first, the small grids
    // fill the tail of the launch
    std::vector<size_t> by_size(members.size());
    for (size_t j = 0; j < by_size.size(); ++j) by_size[j] = j;
    std::stable_sort(by_size.begin(), by_size.end(), [&](size_t a, size_t b) { return nblk[a] > nblk[b]; });
    int64_t total = 0;
    for (int b : nblk) total += b;
    if (total > INT32_MAX) return fail(S5D_EUNSUPPORTED, "batched launch exceeds 2^31 workgroups");
    g.map_off = align_up(blob.size(), 256);
    g.nblocks = static_cast<int>(total);
    blob.resize(g.map_off + static_cast<size_t>(total) * sizeof(BlockMap));
    BlockMap* map = reinterpret_cast<BlockMap*>(blob.data() + g.map_off);
    int64_t pos = 0;
    for (size_t j : by_size)
      for (int b = 0; b < nblk[j]; ++b) map[pos++] = BlockMap{static_cast<int32_t>(j), b};
    out.push_back(g);
  }
  return S5D_OK;
}

hipError_t StepStreams::create(int n) {
  n_side = 0;
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e != hipSuccess) {
    fork = nullptr;
    return e;
  }
  for (int i = 0; i < n && i < kMaxSideStreams; ++i) {
    e = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
    if (e != hipSuccess) {
      side[i] = nullptr;
      return e;
    }
    e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      join[i] = nullptr;
      return e;
    }
    n_side = i + 1;
  }
  return hipSuccess;
}

void StepStreams::destroy() {
  for (int i = 0; i < kMaxSideStreams; ++i) {
    if (side[i]) (void)hipStreamSynchronize(side[i]);
    if (side[i]) (void)hipStreamDestroy(side[i]);
    if (join[i]) (void)hipEventDestroy(join[i]);
    side[i] = nullptr;
    join[i] = nullptr;
  }
  if (fork) (void)hipEventDestroy(fork);
  fork = nullptr;
  n_side = 0;
}

hipError_t enqueue_step(const std::vector<GroupLaunch>& launches, const unsigned char* dev, hipStream_t stream,
                        const StepStreams* ss) {
  const int nside = (ss && ss->fork && launches.size() >= 2)
                        ? std::min<int>(ss->n_side, static_cast<int>(launches.size()) - 1)
                        : 0;
  hipError_t e = hipSuccess;
  if (nside > 0) {
    if ((e = hipEventRecord(ss->fork, stream)) != hipSuccess) return e;
    for (int i = 0; i < nside; ++i)
      if ((e = hipStreamWaitEvent(ss->side[i], ss->fork, 0)) != hipSuccess) return e;
  }
  for (size_t j = 0; j < launches.size(); ++j) {
    const GroupLaunch& g = launches[j];
    const int q = nside > 0 ? static_cast<int>(j % static_cast<size_t>(nside + 1)) : 0;
    e = g.fn(dev + g.items_off, reinterpret_cast<const BlockMap*>(dev + g.map_off), g.nblocks,
             q == 0 ? stream : ss->side[q - 1]);
    if (e != hipSuccess) return e;
  }
  for (int i = 0; i < nside; ++i) {
    if ((e = hipEventRecord(ss->join[i], ss->side[i])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(stream, ss->join[i], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

s5d_status check_disjoint(const std::vector<std::pair<uintptr_t, uintptr_t>>& ranges) {
  std::vector<std::pair<uintptr_t, uintptr_t>> r = ranges;
  std::sort(r.begin(), r.end());
  for (size_t i = 1; i < r.size(); ++i)
    if (r[i].first < r[i - 1].second) return fail(S5D_EINVAL, "buffers of different grids overlap");
  return S5D_OK;
}

}  // namespace s5d

namespace s5d {
namespace {
// Persistent mode: one launch per stencil family, over its round table and
// work items (byte offsets into the device blob) and its control block.
struct FamilyLaunch {
  Persist2D k;
  size_t rounds_off = 0, items_off = 0, ctl_off = 0;
  int32_t n_items = 0;
  int nblocks = 0;
};
constexpr int64_t kDefaultWaitLimit = int64_t{1} << 24;
// Shortest stream block of a library-chosen length in a persistent launch:
// the queue balances the load by itself, and every work item pays an
// agent-scope release and acquire, so fewer, longer blocks win (measured on
// MI355X, 64-grid mix: 1117 GCell/s at the shared-launch lengths, 1356 with
// this floor, 1335 at 512, 1007 at 1024).
constexpr int kPersistMinChunk = 256;
}  // namespace
}  // namespace s5d

struct s5d_batch {
  // boundary copies of every grid with work: one launch over a device table
  // of HaloItems at byte offset halo_off of the device blob
  int32_t n_halo = 0;
  int64_t halo_max_cells = 0;
  size_t halo_off = 0;
  std::vector<std::vector<s5d::GroupLaunch>> steps;
  std::vector<int32_t> result_index;
  // device coefficient tables of the plans (direct kernels read them through
  // the batch items); held here because plans may be destroyed after creation
  std::vector<std::shared_ptr<void>> coef_tables;
  unsigned char* dev = nullptr;
  int device = 0;
  s5d::StepStreams ss;  // side streams for steps of several kernel variants
  bool graph = false;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  // persistent mode: the family launches and their control blocks (one
  // contiguous int32 range of the blob, cleared before every run)
  bool persistent = false;
  std::vector<s5d::FamilyLaunch> families;
  size_t ctl_off = 0;
  int64_t ctl_ints = 0;
  int64_t wait_limit = s5d::kDefaultWaitLimit;
};

namespace {

hipError_t enqueue_batch(const s5d_batch* b, hipStream_t st) {
  constexpr int kMaxHaloItems = 65535;  // grid y-dimension of the boundary-copy launch
  const s5d::HaloItem* halo = reinterpret_cast<const s5d::HaloItem*>(b->dev + b->halo_off);
  if (b->persistent && b->ctl_ints > 0) {
    const hipError_t e =
        s5d::launch_fill_i32(reinterpret_cast<int32_t*>(b->dev + b->ctl_off), b->ctl_ints, 0, st);
    if (e != hipSuccess) return e;
  }
  for (int32_t i = 0; i < b->n_halo; i += kMaxHaloItems) {
    const hipError_t e = s5d::launch_halo_copy_batch(halo + i, std::min(kMaxHaloItems, b->n_halo - i),
                                                     b->halo_max_cells, st);
    if (e != hipSuccess) return e;
  }
  if (b->persistent) {
    // families touch different grids: fork them over the side streams
    const int nf = static_cast<int>(b->families.size());
    const int nside = (b->ss.fork && nf >= 2) ? std::min(b->ss.n_side, nf - 1) : 0;
    hipError_t e = hipSuccess;
    if (nside > 0) {
      if ((e = hipEventRecord(b->ss.fork, st)) != hipSuccess) return e;
      for (int i = 0; i < nside; ++i)
        if ((e = hipStreamWaitEvent(b->ss.side[i], b->ss.fork, 0)) != hipSuccess) return e;
    }
    for (int j = 0; j < nf; ++j) {
      const s5d::FamilyLaunch& f = b->families[j];
      const int q = nside > 0 ? j % (nside + 1) : 0;
      e = f.k.launch(b->dev + f.rounds_off, reinterpret_cast<const s5d::PersistItem*>(b->dev + f.items_off),
                     f.n_items, reinterpret_cast<int32_t*>(b->dev + f.ctl_off), b->wait_limit, f.nblocks,
                     q == 0 ? st : b->ss.side[q - 1]);
      if (e != hipSuccess) return e;
    }
    for (int i = 0; i < nside; ++i) {
      if ((e = hipEventRecord(b->ss.join[i], b->ss.side[i])) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(st, b->ss.join[i], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  for (const auto& step : b->steps) {
    const hipError_t e = s5d::enqueue_step(step, b->dev, st, &b->ss);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void release(s5d_batch* b) {
  if (!b) return;
  if (b->exec || b->dev) (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  b->ss.destroy();
  if (b->dev) (void)hipFree(b->dev);
  (void)hipGetLastError();
  delete b;
}

}  // namespace

namespace s5d {

// Persistent mode: group the grids by stencil family, lay out each family's
// round table, work items and control block in `blob`, and size its launch.
s5d_status build_persistent(s5d_batch* b, const s5d_plan* const* plans, void* const* buf0, void* const* buf1,
                            int32_t n, const std::vector<std::vector<int>>& rounds, const std::vector<int>& chunks,
                            const std::vector<double>& work, std::vector<unsigned char>& blob) {
  // family of every grid with work
  std::vector<int> fam(static_cast<size_t>(n), -1);
  for (int32_t g = 0; g < n; ++g) {
    if (rounds[g].empty()) continue;
    const s5d_plan* p = plans[g];
    const int box = p->d.shape == S5D_BOX ? 1 : 0;
    if (p->d.ndim != 2 || p->direct)
      return fail(S5D_EUNSUPPORTED, "grid " + std::to_string(g) + ": persistent batches run 2D blocked plans only");
    const int bt_max = *std::max_element(rounds[g].begin(), rounds[g].end());
    for (int i = 0; i < kRegistryP2DSize; ++i) {
      const EntryP2D& e = kRegistryP2D[i];
      if (e.dtype == p->kind && e.expr == p->expr && e.box == box && e.r == p->d.radius &&
          e.cpl == p->tun.cells_per_lane && bt_max <= e.max_bt) {
        fam[g] = i;
        break;
      }
    }
    if (fam[g] < 0)
      return fail(S5D_EUNSUPPORTED, "grid " + std::to_string(g) + ": no persistent kernel for this stencil, "
                                    "cells per lane and depth");
  }
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
    (void)hipGetLastError();
    cus = 256;
  }
  double total_work = 0;
  for (int32_t g = 0; g < n; ++g)
    if (fam[g] >= 0) total_work += work[g];
  std::vector<unsigned char> tmp;
  std::vector<size_t> ctl_offs;  // control blocks are laid out after every table
  std::vector<int64_t> ctl_sizes;
  for (int fi = 0; fi < kRegistryP2DSize; ++fi) {
    std::vector<int32_t> members;
    double fwork = 0;
    for (int32_t g = 0; g < n; ++g)
      if (fam[g] == fi) {
        members.push_back(g);
        fwork += work[g];
      }
    if (members.empty()) continue;
    FamilyLaunch f;
    f.k = kRegistryP2D[fi].make();
    const size_t rb = static_cast<size_t>(f.k.round_bytes);
    tmp.assign(rb + 16, 0);
    void* scratch = reinterpret_cast<void*>(align_up(reinterpret_cast<uintptr_t>(tmp.data()), 16));
    // workgroups of every round of every member (need is not known yet)
    std::vector<std::vector<int32_t>> blocks(members.size());
    std::vector<int> pchunk(static_cast<size_t>(n), 0);
    for (int32_t g : members) pchunk[g] = plans[g]->chunk_auto ? std::max(chunks[g], kPersistMinChunk) : chunks[g];
    for (size_t j = 0; j < members.size(); ++j) {
      const int32_t g = members[j];
      void* bufs[2] = {buf0[g], buf1[g]};
      for (size_t k = 0; k < rounds[g].size(); ++k) {
        const int nb = fill_persist_round(plans[g], f.k, rounds[g][k], bufs[k % 2], bufs[(k + 1) % 2], scratch,
                                          pchunk[g], 0, 0);
        if (nb <= 0) return fail(S5D_EUNSUPPORTED, "grid " + std::to_string(g) + ": round does not fit a launch");
        blocks[j].push_back(nb);
      }
    }
    std::vector<PersistRound> prounds;
    std::vector<PersistItem> items;
    if (!persist_schedule(blocks, kWavesPerBlock, prounds, items))
      return fail(S5D_EUNSUPPORTED, "persistent work list exceeds 2^31 items");
    f.rounds_off = align_up(blob.size(), 256);
    blob.resize(f.rounds_off + prounds.size() * rb);
    for (size_t i = 0; i < prounds.size(); ++i) {
      const PersistRound& pr = prounds[i];
      const int32_t g = members[pr.grid];
      void* bufs[2] = {buf0[g], buf1[g]};
      const int k = pr.round;
      fill_persist_round(plans[g], f.k, rounds[g][k], bufs[k % 2], bufs[(k + 1) % 2], scratch, pchunk[g], pr.grid,
                         pr.need);
      std::memcpy(blob.data() + f.rounds_off + i * rb, scratch, rb);
    }
    f.items_off = align_up(blob.size(), 256);
    blob.resize(f.items_off + items.size() * sizeof(PersistItem));
    std::memcpy(blob.data() + f.items_off, items.data(), items.size() * sizeof(PersistItem));
    f.n_items = static_cast<int32_t>(items.size());
    // resident workgroups, shared with the other families by their work
    int occ = f.k.occupancy ? f.k.occupancy() : 0;
    if (occ <= 0) occ = 1;
    const double share = total_work > 0 ? fwork / total_work : 1.0;
    const int64_t slots = static_cast<int64_t>(cus) * occ;
    f.nblocks = static_cast<int>(std::max<int64_t>(
        1, std::min<int64_t>(f.n_items, static_cast<int64_t>(std::ceil(static_cast<double>(slots) * share)))));
    ctl_sizes.push_back(kPersistCtl + static_cast<int64_t>(members.size()));
    b->families.push_back(f);
  }
  // one contiguous control range for all families (cleared by one launch)
  b->ctl_off = align_up(blob.size(), 256);
  size_t off = b->ctl_off;
  for (size_t j = 0; j < b->families.size(); ++j) {
    b->families[j].ctl_off = off;
    off += static_cast<size_t>(ctl_sizes[j]) * sizeof(int32_t);
  }
  b->ctl_ints = static_cast<int64_t>((off - b->ctl_off) / sizeof(int32_t));
  blob.resize(off, 0);
  return S5D_OK;
}

}  // namespace s5d

using s5d::device_fail;
using s5d::fail;

extern "C" {

s5d_status s5d_batch_create(const s5d_plan* const* plans, void* const* buf0, void* const* buf1, int32_t n,
                            int32_t flags, s5d_batch** out) {
  s5d::clear_error();
  if (!out) return fail(S5D_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 0) return fail(S5D_EINVAL, "n must be >= 0");
  if (n > 0 && (!plans || !buf0 || !buf1)) return fail(S5D_EINVAL, "plans, buf0 and buf1 must not be NULL");
  if (flags & ~(S5D_BATCH_GRAPH | S5D_BATCH_PERSISTENT)) return fail(S5D_EINVAL, "unknown flags");
  std::vector<std::pair<uintptr_t, uintptr_t>> ranges;
  for (int32_t g = 0; g < n; ++g) {
    if (!plans[g]) return fail(S5D_EINVAL, "plans[" + std::to_string(g) + "] is NULL");
    const s5d_status st = s5d::check_buffers(plans[g], buf0[g], buf1[g]);
    if (st != S5D_OK) return fail(st, "grid " + std::to_string(g) + ": " + s5d_last_error());
    for (void* p : {buf0[g], buf1[g]}) {
      const uintptr_t a = reinterpret_cast<uintptr_t>(p);
      ranges.emplace_back(a, a + static_cast<uintptr_t>(plans[g]->bytes));
    }
  }
  const s5d_status dst = s5d::check_disjoint(ranges);
  if (dst != S5D_OK) return dst;

  s5d_batch* b = new (std::nothrow) s5d_batch;
  if (!b) return fail(S5D_ENOMEM, "batch allocation failed");
  b->graph = (flags & S5D_BATCH_GRAPH) != 0;
  b->persistent = (flags & S5D_BATCH_PERSISTENT) != 0;
  std::vector<std::vector<int>> rounds(static_cast<size_t>(n));
  size_t kmax = 0;
  try {
    std::vector<s5d::HaloItem> halos;
    b->result_index.resize(static_cast<size_t>(n));
    for (int32_t g = 0; g < n; ++g) {
      const s5d_plan* p = plans[g];
      b->result_index[g] = static_cast<int32_t>(p->d.steps % 2);
      if (p->dcoef) b->coef_tables.push_back(p->dcoef);
      rounds[g] = s5d::plan_rounds(p);
      kmax = std::max(kmax, rounds[g].size());
      if (!rounds[g].empty()) {
        s5d::HaloItem h;
        h.src = buf0[g];
        h.dst = buf1[g];
        h.P0 = p->padded[0];
        h.P1 = p->padded[1];
        h.P2 = p->d.ndim == 3 ? p->padded[2] : 1;
        h.r = p->d.radius;
        h.elem = p->elem;
        halos.push_back(h);
        b->halo_max_cells = std::max(b->halo_max_cells, s5d::halo_cells(p->d.ndim, p->padded, p->d.radius));
      }
    }
    b->n_halo = static_cast<int32_t>(halos.size());
    // Each grid shares the machine with all the others (launches of different
    // kernel variants overlap on two streams): its stream blocks are chosen
    // for its fraction of the batch's cell-updates, which gives the small
    // grids fewer, longer blocks than they would take alone.  The block
    // length does not change any result bit.
    std::vector<int> chunks(static_cast<size_t>(n), 0);
    std::vector<double> work(static_cast<size_t>(n), 0.0);
    double total_work = 0;
    for (int32_t g = 0; g < n; ++g) {
      if (rounds[g].empty()) continue;
      work[g] = static_cast<double>(plans[g]->d.steps) * static_cast<double>(plans[g]->bytes / plans[g]->elem);
      total_work += work[g];
    }
    for (int32_t g = 0; g < n; ++g)
      if (!rounds[g].empty() && total_work > 0)
        chunks[g] = s5d::shared_chunk(plans[g], plans[g]->tun.bt, work[g] / total_work);
    std::vector<unsigned char> blob;
    if (!halos.empty()) {
      b->halo_off = 0;
      blob.resize(halos.size() * sizeof(s5d::HaloItem));
      std::memcpy(blob.data(), halos.data(), blob.size());
    }
    if (b->persistent) {
      const s5d_status st = s5d::build_persistent(b, plans, buf0, buf1, n, rounds, chunks, work, blob);
      if (st != S5D_OK) {
        release(b);
        return st;
      }
      kmax = 0;  // no per-round-index steps
    }
    b->steps.resize(kmax);
    for (size_t k = 0; k < kmax; ++k) {
      std::vector<s5d::RoundItem> items;
      for (int32_t g = 0; g < n; ++g) {
        if (k >= rounds[g].size()) continue;
        void* bufs[2] = {buf0[g], buf1[g]};
        items.push_back(s5d::RoundItem{plans[g], rounds[g][k], bufs[k % 2], bufs[(k + 1) % 2], chunks[g]});
      }
      const s5d_status st = s5d::build_step(items, blob, b->steps[k]);
      if (st != S5D_OK) {
        release(b);
        return st;
      }
    }
    if (!blob.empty()) {
      if (hipGetDevice(&b->device) != hipSuccess) {
        release(b);
        return device_fail(hipGetLastError(), "hipGetDevice");
      }
      hipError_t e = hipMalloc(reinterpret_cast<void**>(&b->dev), blob.size());
      if (e != hipSuccess) {
        b->dev = nullptr;
        release(b);
        return device_fail(e, "hipMalloc of the batch tables");
      }
      e = hipMemcpy(b->dev, blob.data(), blob.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        release(b);
        return device_fail(e, "upload of the batch tables");
      }
      size_t widest = std::max<size_t>(1, b->families.size());
      for (const auto& step : b->steps) widest = std::max(widest, step.size());
      if (widest >= 2) {
        e = b->ss.create(static_cast<int>(std::min<size_t>(widest - 1, s5d::kMaxSideStreams)));
        if (e != hipSuccess) {
          release(b);
          return device_fail(e, "side streams of the batch");
        }
      }
    }
  } catch (const std::bad_alloc&) {
    release(b);
    return fail(S5D_ENOMEM, "host allocation failed");
  }
  *out = b;
  return S5D_OK;
}

s5d_status s5d_batch_run(s5d_batch* batch, void* stream, int32_t* result_index) {
  s5d::clear_error();
  if (!batch) return fail(S5D_EINVAL, "batch is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  if (result_index)
    for (size_t g = 0; g < batch->result_index.size(); ++g) result_index[g] = batch->result_index[g];
  if (batch->n_halo == 0) return S5D_OK;
  if (!batch->graph) {
    const hipError_t e = enqueue_batch(batch, st);
    return e == hipSuccess ? S5D_OK : device_fail(e, "batched launch");
  }
  if (!batch->exec) {
    // capture once on a private stream; the executable graph then runs on
    // any stream of the device
    hipError_t e = hipStreamCreateWithFlags(&batch->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      batch->capture_stream = nullptr;
      return device_fail(e, "capture stream");
    }
    e = hipStreamBeginCapture(batch->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return device_fail(e, "hipStreamBeginCapture");
    const hipError_t le = enqueue_batch(batch, batch->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(batch->capture_stream, &graph);
    if (le != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return device_fail(le != hipSuccess ? le : e, "graph capture");
    }
    e = hipGraphInstantiate(&batch->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      batch->exec = nullptr;
      return device_fail(e, "hipGraphInstantiate");
    }
  }
  const hipError_t e = hipGraphLaunch(batch->exec, st);
  return e == hipSuccess ? S5D_OK : device_fail(e, "hipGraphLaunch");
}

s5d_status s5d_batch_query(const s5d_batch* batch, int32_t* n_launches, int32_t* n_round_steps) {
  s5d::clear_error();
  if (!batch) return fail(S5D_EINVAL, "batch is NULL");
  int32_t nl = (batch->n_halo + 65534) / 65535;
  if (batch->persistent && batch->ctl_ints > 0) nl += 1 + static_cast<int32_t>(batch->families.size());
  for (const auto& s : batch->steps) nl += static_cast<int32_t>(s.size());
  if (n_launches) *n_launches = nl;
  if (n_round_steps) *n_round_steps = static_cast<int32_t>(batch->steps.size());
  return S5D_OK;
}

s5d_status s5d_batch_persistent_info(const s5d_batch* batch, int32_t* n_launches, int64_t* workgroups,
                                     int64_t* items) {
  s5d::clear_error();
  if (!batch) return fail(S5D_EINVAL, "batch is NULL");
  int64_t wg = 0, it = 0;
  for (const s5d::FamilyLaunch& f : batch->families) {
    wg += f.nblocks;
    it += f.n_items;
  }
  if (n_launches) *n_launches = static_cast<int32_t>(batch->families.size());
  if (workgroups) *workgroups = wg;
  if (items) *items = it;
  return S5D_OK;
}

s5d_status s5d_batch_status(s5d_batch* batch, void* stream) {
  s5d::clear_error();
  if (!batch) return fail(S5D_EINVAL, "batch is NULL");
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "hipStreamSynchronize");
  for (const s5d::FamilyLaunch& f : batch->families) {
    int32_t ctl[2] = {0, 0};
    e = hipMemcpy(ctl, batch->dev + f.ctl_off, sizeof(ctl), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(e, "reading the persistent launch status");
    if (ctl[1] != 0) return fail(S5D_ETIMEDOUT, "a workgroup's wait for its grid's previous round ran out");
  }
  return S5D_OK;
}

s5d_status s5d_batch_set_wait_limit(s5d_batch* batch, int64_t polls) {
  s5d::clear_error();
  if (!batch) return fail(S5D_EINVAL, "batch is NULL");
  if (polls < 0) return fail(S5D_EINVAL, "polls must be >= 0");
  batch->wait_limit = polls;
  if (batch->exec) {
    // the limit is a kernel argument of the captured launches: capture again
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(batch->exec);
    batch->exec = nullptr;
  }
  return S5D_OK;
}

void s5d_batch_destroy(s5d_batch* batch) { release(batch); }

s5d_status s5d_run_batch(const s5d_plan* const* plans, void* const* buf0, void* const* buf1, int32_t n,
                         void* stream, int32_t* result_index) {
  s5d_batch* b = nullptr;
  s5d_status st = s5d_batch_create(plans, buf0, buf1, n, 0, &b);
  if (st != S5D_OK) return st;
  st = s5d_batch_run(b, stream, result_index);
  const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  release(b);
  if (st != S5D_OK) return st;
  return e == hipSuccess ? S5D_OK : device_fail(e, "hipStreamSynchronize");
}

}  // extern "C"
