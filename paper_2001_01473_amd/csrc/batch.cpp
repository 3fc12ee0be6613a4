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
#include <cstring>
#include <map>
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

hipError_t enqueue_step(const std::vector<GroupLaunch>& launches, const unsigned char* dev, hipStream_t stream,
                        hipStream_t side, hipEvent_t fork, hipEvent_t join) {
  const bool split = side && fork && join && launches.size() >= 2;
  hipError_t e = hipSuccess;
  if (split) {
    if ((e = hipEventRecord(fork, stream)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(side, fork, 0)) != hipSuccess) return e;
  }
  for (size_t j = 0; j < launches.size(); ++j) {
    const GroupLaunch& g = launches[j];
    e = g.fn(dev + g.items_off, reinterpret_cast<const BlockMap*>(dev + g.map_off), g.nblocks,
             split && j % 2 == 1 ? side : stream);
    if (e != hipSuccess) return e;
  }
  if (split) {
    if ((e = hipEventRecord(join, side)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(stream, join, 0)) != hipSuccess) return e;
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

struct s5d_batch {
  struct Boundary {
    const void* src;
    void* dst;
    int elem, ndim, r;
    int64_t padded[3];
  };
  std::vector<Boundary> boundaries;
  std::vector<std::vector<s5d::GroupLaunch>> steps;
  std::vector<int32_t> result_index;
  unsigned char* dev = nullptr;
  int device = 0;
  hipStream_t side = nullptr;  // second stream for steps of several kernel variants
  hipEvent_t fork = nullptr, join = nullptr;
  bool graph = false;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

hipError_t enqueue_batch(const s5d_batch* b, hipStream_t st) {
  for (const s5d_batch::Boundary& h : b->boundaries) {
    const hipError_t e = s5d::launch_halo_copy(h.src, h.dst, h.elem, h.ndim, h.padded, h.r, st);
    if (e != hipSuccess) return e;
  }
  for (const auto& step : b->steps) {
    const hipError_t e = s5d::enqueue_step(step, b->dev, st, b->side, b->fork, b->join);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void release(s5d_batch* b) {
  if (!b) return;
  if (b->exec || b->dev) (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->dev) (void)hipFree(b->dev);
  (void)hipGetLastError();
  delete b;
}

}  // namespace

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
  if (flags & ~S5D_BATCH_GRAPH) return fail(S5D_EINVAL, "unknown flags");
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
  std::vector<std::vector<int>> rounds(static_cast<size_t>(n));
  size_t kmax = 0;
  try {
    b->result_index.resize(static_cast<size_t>(n));
    for (int32_t g = 0; g < n; ++g) {
      const s5d_plan* p = plans[g];
      b->result_index[g] = static_cast<int32_t>(p->d.steps % 2);
      rounds[g] = s5d::plan_rounds(p);
      kmax = std::max(kmax, rounds[g].size());
      if (!rounds[g].empty()) {
        s5d_batch::Boundary h{buf0[g], buf1[g], p->elem, p->d.ndim, p->d.radius, {0, 0, 0}};
        for (int a = 0; a < 3; ++a) h.padded[a] = p->padded[a];
        b->boundaries.push_back(h);
      }
    }
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
      bool multi = false;
      for (const auto& step : b->steps) multi = multi || step.size() >= 2;
      if (multi) {
        e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
        if (e != hipSuccess) {
          release(b);
          return device_fail(e, "side stream of the batch");
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
  if (batch->boundaries.empty()) return S5D_OK;
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
  int32_t nl = static_cast<int32_t>(batch->boundaries.size());
  for (const auto& s : batch->steps) nl += static_cast<int32_t>(s.size());
  if (n_launches) *n_launches = nl;
  if (n_round_steps) *n_round_steps = static_cast<int32_t>(batch->steps.size());
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
