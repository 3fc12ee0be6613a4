// Serving loop: continuous batching of independent sweep requests.
//
// Requests (a plan and an initial grid) queue in arrival order.  Each tick
//  1. admits queued requests in FIFO order while their two device buffers fit
//     the HBM budget (stream-ordered allocation, initial copy, boundary copy);
//  2. advances EVERY running request by one round of its own schedule (the
//     rounds s5d_run would give it, so every result is bit-identical to the
//     request run alone), all of them in one batched launch per kernel
//     variant, through a device table uploaded from pinned staging;
//  3. records an event; requests whose last round is in this tick complete
//     when it fires, and their completion time is read from the GPU clock.
// New arrivals therefore join at round boundaries, and grids stay resident in
// HBM from admission to completion.  At most kSlots ticks are in flight: the
// host prepares the next tick while the GPU runs the previous ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <new>
#include <unordered_map>
#include <vector>

#include "batch.h"
#include "host.h"

namespace {

constexpr int kSlots = 3;
// With few requests running, a tick enqueues several rounds of each so that
// it holds about this many launches (the host's per-tick work is then spread
// over more GPU work); at most kMaxRoundsPerTick.
constexpr int kTargetLaunches = 8;
constexpr int kMaxRoundsPerTick = 16;

struct Request {
  int64_t id = 0;
  s5d_plan plan;
  const void* init = nullptr;
  hipEvent_t init_ev = nullptr;  // recorded after the copy of init; null once that copy is known done
  bool keep = false;
  bool cancel = false;           // cancellation asked for while running
  int32_t state = S5D_REQ_QUEUED;
  s5d_status status = S5D_OK;    // why a FAILED request failed
  double t_arrival = 0, t_admit = -1, t_done = -1;
  std::vector<int> rounds;
  size_t next = 0;
  void* buf[2] = {nullptr, nullptr};
  int64_t bytes2 = 0;  // both buffers
  int64_t updates = 0;
};

double cells_of(const Request* r) { return static_cast<double>(r->plan.bytes / r->plan.elem); }

struct Slot {
  unsigned char* host = nullptr;  // pinned staging
  unsigned char* dev = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

struct Finishing {
  hipEvent_t ev;
  std::vector<Request*> reqs;
};

}  // namespace

struct s5d_server {
  s5d_server_config cfg;
  hipStream_t stream = nullptr;
  s5d::StepStreams ss;  // side streams: launches of different kernel variants overlap
  hipEvent_t base = nullptr;
  std::chrono::steady_clock::time_point t0;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  std::deque<Request*> queue;
  std::vector<Request*> running;
  std::deque<Finishing> finishing;
  std::vector<hipEvent_t> event_pool;
  Slot slots[kSlots];
  int64_t next_id = 1;
  int64_t used = 0, peak = 0;
  int64_t ticks = 0, launches = 0, done = 0, failed = 0, updates_done = 0;
  int64_t admissions = 0, work_ticks = 0;  // counters of the fault-injection knobs
  double first_arrival = -1, last_done = -1;
  std::vector<double> latencies;
};

using s5d::device_fail;
using s5d::fail;

namespace {

double host_now(const s5d_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

s5d_status take_event(s5d_server* s, hipEvent_t* ev) {
  if (!s->event_pool.empty()) {
    *ev = s->event_pool.back();
    s->event_pool.pop_back();
    return S5D_OK;
  }
  const hipError_t e = hipEventCreate(ev);
  return e == hipSuccess ? S5D_OK : device_fail(e, "hipEventCreate");
}

void release_buffers(s5d_server* s, Request* r) {
  bool held = false;
  for (void*& b : r->buf) {
    if (b) (void)hipFreeAsync(b, s->stream);  // stream-ordered: after the request's last use
    held = held || b;
    b = nullptr;
  }
  if (held) s->used -= r->bytes2;
}

// Has the copy out of the request's init been completed on the device?
// (Returns the event to the pool once it has.)
bool init_released(const s5d_server* cs, Request* r) {
  if (!r->init_ev) return true;
  const hipError_t q = hipEventQuery(r->init_ev);
  if (q == hipErrorNotReady) return false;
  (void)hipGetLastError();
  const_cast<s5d_server*>(cs)->event_pool.push_back(r->init_ev);
  r->init_ev = nullptr;
  return true;
}

// A request that will not run (any more): FAILED, memory returned.
void fail_request(s5d_server* s, Request* r, s5d_status why) {
  release_buffers(s, r);
  r->state = S5D_REQ_FAILED;
  r->status = why;
  r->init = nullptr;
  ++s->failed;
}

// Move requests whose completion event has fired to DONE.
s5d_status retire(s5d_server* s) {
  while (!s->finishing.empty()) {
    Finishing& f = s->finishing.front();
    const hipError_t q = hipEventQuery(f.ev);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) return device_fail(q, "hipEventQuery");
    float ms = 0.f;
    const hipError_t e = hipEventElapsedTime(&ms, s->base, f.ev);
    const double t = e == hipSuccess ? ms * 1e-3 : host_now(s);
    for (Request* r : f.reqs) {
      r->t_done = t;
      r->state = S5D_REQ_DONE;
      ++s->done;
      s->updates_done += r->updates;
      s->latencies.push_back(t - r->t_arrival);
      s->last_done = std::max(s->last_done, t);
    }
    s->event_pool.push_back(f.ev);
    s->finishing.pop_front();
  }
  return S5D_OK;
}

// Mark `reqs` as finishing once the work enqueued so far completes; results
// that are not kept give their memory back (stream-ordered).
s5d_status record_finish(s5d_server* s, const std::vector<Request*>& reqs) {
  hipEvent_t ev = nullptr;
  const s5d_status st = take_event(s, &ev);
  if (st != S5D_OK) return st;
  const hipError_t e = hipEventRecord(ev, s->stream);
  if (e != hipSuccess) {
    s->event_pool.push_back(ev);
    return device_fail(e, "hipEventRecord");
  }
  for (Request* r : reqs)
    if (!r->keep) release_buffers(s, r);
  s->finishing.push_back(Finishing{ev, reqs});
  return S5D_OK;
}

// Allocate the request's buffers, copy its initial grid in, copy the
// boundary into the second buffer.  On failure nothing stays allocated and
// the request is left for the caller to fail.
s5d_status admit(s5d_server* s, Request* r) {
  const int64_t nb = r->plan.bytes;
  if (s->cfg.fail_admit_every > 0 && (++s->admissions % s->cfg.fail_admit_every) == 0)
    return fail(S5D_EDEVICE, "injected admission failure (fail_admit_every)");
  for (int i = 0; i < 2; ++i) {
    const hipError_t e = hipMallocAsync(&r->buf[i], static_cast<size_t>(nb), s->stream);
    if (e != hipSuccess) {
      r->buf[i] = nullptr;
      if (i == 1) {
        (void)hipFreeAsync(r->buf[0], s->stream);
        r->buf[0] = nullptr;
      }
      (void)hipGetLastError();
      return device_fail(e, "hipMallocAsync");
    }
  }
  s->used += r->bytes2;  // release_buffers gives it back from here on
  hipError_t e = hipMemcpyAsync(r->buf[0], r->init, static_cast<size_t>(nb), hipMemcpyDefault, s->stream);
  if (e != hipSuccess) return device_fail(e, "initial copy");
  // init may be dropped by the caller only once this copy has run
  hipEvent_t ev = nullptr;
  s5d_status st = take_event(s, &ev);
  if (st != S5D_OK) return st;
  e = hipEventRecord(ev, s->stream);
  if (e != hipSuccess) {
    s->event_pool.push_back(ev);
    return device_fail(e, "hipEventRecord");
  }
  r->init_ev = ev;
  r->init = nullptr;
  r->rounds = s5d::plan_rounds(&r->plan);
  if (!r->rounds.empty()) {
    e = s5d::launch_boundary_copy(&r->plan, r->buf[0], r->buf[1], s->stream);
    if (e != hipSuccess) return device_fail(e, "boundary copy launch");
  }
  r->state = S5D_REQ_RUNNING;
  r->t_admit = host_now(s);
  return S5D_OK;
}

s5d_status grow_slot(Slot& sl, size_t need) {
  if (need <= sl.cap) return S5D_OK;
  size_t cap = std::max<size_t>(need, 2 * sl.cap);
  cap = std::max<size_t>(cap, 1 << 16);
  if (sl.pending) (void)hipEventSynchronize(sl.ev);
  sl.pending = false;
  if (sl.host) (void)hipHostFree(sl.host);
  if (sl.dev) (void)hipFree(sl.dev);
  sl.host = nullptr;
  sl.dev = nullptr;
  sl.cap = 0;
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&sl.host), cap, hipHostMallocDefault);
  if (e != hipSuccess) {
    sl.host = nullptr;
    return device_fail(e, "hipHostMalloc of the tick table");
  }
  e = hipMalloc(reinterpret_cast<void**>(&sl.dev), cap);
  if (e != hipSuccess) {
    sl.dev = nullptr;
    return device_fail(e, "hipMalloc of the tick table");
  }
  sl.cap = cap;
  return S5D_OK;
}

void destroy_server(s5d_server* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (auto& kv : s->reqs) {
    for (void* b : kv.second->buf)
      if (b) (void)hipFreeAsync(b, s->stream);
    if (kv.second->init_ev) (void)hipEventDestroy(kv.second->init_ev);
  }
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (Slot& sl : s->slots) {
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.dev) (void)hipFree(sl.dev);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  }
  for (Finishing& f : s->finishing) (void)hipEventDestroy(f.ev);
  for (hipEvent_t ev : s->event_pool) (void)hipEventDestroy(ev);
  if (s->base) (void)hipEventDestroy(s->base);
  s->ss.destroy();
  if (s->stream) (void)hipStreamDestroy(s->stream);
  (void)hipGetLastError();
  delete s;
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  // nearest rank
  size_t k = static_cast<size_t>(std::ceil(q * static_cast<double>(v.size())));
  k = std::min(std::max<size_t>(k, 1), v.size());
  return v[k - 1];
}

// Can every round of this plan go into a batched launch?  (Checked at
// submission, so that a tick never meets a request it cannot launch.)
s5d_status check_batchable(const s5d_plan* p) {
  const std::vector<int> rounds = s5d::plan_rounds(p);
  std::vector<int> seen;
  static char dummy[2][16];
  for (int bt : rounds) {
    if (std::find(seen.begin(), seen.end(), bt) != seen.end()) continue;
    seen.push_back(bt);
    const s5d::BatchHooks h = s5d::batch_hooks(p, bt);
    if (!h.launch || h.item_bytes <= 0) return fail(S5D_EUNSUPPORTED, "kernel variant without a batched entry point");
    std::vector<unsigned char> item(static_cast<size_t>(h.item_bytes) + 16);
    void* tmp = reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(item.data()) + 15) & ~uintptr_t(15));
    if (s5d::fill_round_item(p, bt, dummy[0], dummy[1], tmp) <= 0)
      return fail(S5D_EUNSUPPORTED, "grid too large for one batched launch");
  }
  return S5D_OK;
}

}  // namespace

extern "C" {

s5d_status s5d_server_create(const s5d_server_config* config, s5d_server** out) {
  s5d::clear_error();
  if (!out) return fail(S5D_EINVAL, "out is NULL");
  *out = nullptr;
  if (!config) return fail(S5D_EINVAL, "config is NULL");
  if (config->struct_size < sizeof(s5d_server_config)) return fail(S5D_EINVAL, "config->struct_size too small");
  if (config->hbm_budget_bytes <= 0) return fail(S5D_EINVAL, "hbm_budget_bytes must be > 0");
  if (config->max_running < 0) return fail(S5D_EINVAL, "max_running must be >= 0");
  if (config->rounds_per_tick < 0 || config->rounds_per_tick > 1024)
    return fail(S5D_EINVAL, "rounds_per_tick must be in 0..1024");
  if (config->n_streams < 0 || config->n_streams > 1 + s5d::kMaxSideStreams)
    return fail(S5D_EINVAL, "n_streams must be in 0..4");
  if (config->fail_admit_every < 0 || config->fail_tick_every < 0)
    return fail(S5D_EINVAL, "fault-injection periods must be >= 0");
  s5d_server* s = new (std::nothrow) s5d_server;
  if (!s) return fail(S5D_ENOMEM, "server allocation failed");
  s->cfg = *config;
  if (s->cfg.n_streams == 0) s->cfg.n_streams = 1 + s5d::kMaxSideStreams;
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    s->stream = nullptr;
    destroy_server(s);
    return device_fail(e, "server stream");
  }
  e = s->ss.create(s->cfg.n_streams - 1);
  if (e != hipSuccess) {
    destroy_server(s);
    return device_fail(e, "server side streams");
  }
  for (Slot& sl : s->slots) {
    e = hipEventCreate(&sl.ev);
    if (e != hipSuccess) {
      sl.ev = nullptr;
      destroy_server(s);
      return device_fail(e, "hipEventCreate");
    }
  }
  e = hipEventCreate(&s->base);
  if (e == hipSuccess) e = hipEventRecord(s->base, s->stream);
  if (e == hipSuccess) e = hipEventSynchronize(s->base);
  if (e != hipSuccess) {
    destroy_server(s);
    return device_fail(e, "server clock");
  }
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return S5D_OK;
}

void s5d_server_destroy(s5d_server* server) { destroy_server(server); }

s5d_status s5d_server_now(const s5d_server* server, double* seconds) {
  if (!server || !seconds) return fail(S5D_EINVAL, "server and seconds must not be NULL");
  *seconds = host_now(server);
  return S5D_OK;
}

s5d_status s5d_server_submit(s5d_server* s, const s5d_plan* plan, const void* init, double arrival,
                             int32_t keep_result, int64_t* id) {
  s5d::clear_error();
  if (!s || !plan || !init) return fail(S5D_EINVAL, "server, plan and init must not be NULL");
  const int64_t bytes2 = 2 * plan->bytes;
  if (bytes2 > s->cfg.hbm_budget_bytes) return fail(S5D_EBUDGET, "request larger than the HBM budget");
  const s5d_status bst = check_batchable(plan);
  if (bst != S5D_OK) return bst;
  std::unique_ptr<Request> r(new (std::nothrow) Request);
  if (!r) return fail(S5D_ENOMEM, "request allocation failed");
  try {
    r->plan = *plan;
  } catch (...) {
    return fail(S5D_ENOMEM, "plan copy failed");
  }
  r->id = s->next_id++;
  r->init = init;
  r->keep = keep_result != 0;
  r->t_arrival = arrival >= 0 ? arrival : host_now(s);
  r->bytes2 = bytes2;
  r->updates = plan->d.steps * plan->d.interior[0] * plan->d.interior[1] *
               (plan->d.ndim == 3 ? plan->d.interior[2] : 1);
  if (s->first_arrival < 0 || r->t_arrival < s->first_arrival) s->first_arrival = r->t_arrival;
  Request* raw = r.get();
  s->reqs[raw->id] = std::move(r);
  s->queue.push_back(raw);
  if (id) *id = raw->id;
  return S5D_OK;
}

s5d_status s5d_server_cancel(s5d_server* s, int64_t id) {
  s5d::clear_error();
  if (!s) return fail(S5D_EINVAL, "server is NULL");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(S5D_EINVAL, "unknown request id");
  Request* r = it->second.get();
  if (r->state == S5D_REQ_QUEUED) {
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), r), s->queue.end());
    fail_request(s, r, S5D_ECANCELED);
  } else if (r->state == S5D_REQ_RUNNING) {
    // leaves at the start of the next tick, before any further round of it
    r->cancel = true;
  }
  return S5D_OK;
}

s5d_status s5d_server_tick(s5d_server* s, int32_t* n_running, int32_t* n_queued) {
  s5d::clear_error();
  if (!s) return fail(S5D_EINVAL, "server is NULL");
  s5d_status st = retire(s);
  if (st != S5D_OK) return st;
  // cancelled requests leave before this tick's rounds; their buffers are
  // freed after the work already enqueued for them
  {
    std::vector<Request*> still;
    for (Request* r : s->running) {
      if (r->cancel)
        fail_request(s, r, S5D_ECANCELED);
      else
        still.push_back(r);
    }
    s->running.swap(still);
  }
  // 1. admission, FIFO under the budget; a request whose admission fails is
  // FAILED and the queue moves on
  std::vector<Request*> fin;
  while (!s->queue.empty()) {
    Request* r = s->queue.front();
    if (s->cfg.max_running > 0 && static_cast<int64_t>(s->running.size()) >= s->cfg.max_running) break;
    if (s->used + r->bytes2 > s->cfg.hbm_budget_bytes) break;
    s->queue.pop_front();
    st = admit(s, r);
    if (st != S5D_OK) {
      fail_request(s, r, st);
      continue;
    }
    s->peak = std::max(s->peak, s->used);
    if (r->rounds.empty())
      fin.push_back(r);  // zero steps: the result is the initial grid
    else
      s->running.push_back(r);
  }
  // requests of zero steps finish at admission
  if (!fin.empty()) {
    st = record_finish(s, fin);
    if (st != S5D_OK) {
      for (Request* r : fin) fail_request(s, r, st);
      return st;
    }
    fin.clear();
  }
  // 2. one round (or a few, while few requests run) of every running request.
  // The tick is planned on copies of the requests' round indices, which are
  // committed only for rounds whose launches were enqueued.
  if (!s->running.empty()) {
    const int n = static_cast<int>(s->running.size());
    const int K = s->cfg.rounds_per_tick > 0
                      ? s->cfg.rounds_per_tick
                      : std::min(kMaxRoundsPerTick, std::max(1, (kTargetLaunches + n - 1) / n));
    std::vector<Request*> act = s->running;
    std::vector<size_t> nx(act.size());
    for (size_t i = 0; i < act.size(); ++i) nx[i] = act[i]->next;
    std::vector<unsigned char> blob;
    std::vector<std::vector<s5d::GroupLaunch>> steps;
    std::vector<std::vector<size_t>> in_step;   // indices into act of the requests of step j
    std::vector<std::vector<Request*>> fin_after;  // requests whose last round is in step j
    try {
      for (int j = 0; j < K; ++j) {
        // as in a batch: each request's stream blocks are chosen for its share
        // of the step (its fraction of the step's cell-updates; the launches
        // of a step overlap on several streams); results do not depend on the
        // block length
        double step_work = 0;
        for (size_t i = 0; i < act.size(); ++i)
          if (nx[i] < act[i]->rounds.size()) step_work += static_cast<double>(act[i]->rounds[nx[i]]) * cells_of(act[i]);
        if (step_work <= 0) break;
        std::vector<s5d::RoundItem> items;
        in_step.emplace_back();
        fin_after.emplace_back();
        for (size_t i = 0; i < act.size(); ++i) {
          Request* r = act[i];
          if (nx[i] >= r->rounds.size()) continue;
          const size_t k = nx[i]++;
          const int bt = r->rounds[k];
          const int chunk = s5d::shared_chunk(&r->plan, bt, bt * cells_of(r) / step_work);
          items.push_back(s5d::RoundItem{&r->plan, bt, r->buf[k % 2], r->buf[(k + 1) % 2], chunk});
          in_step.back().push_back(i);
          if (nx[i] == r->rounds.size()) fin_after.back().push_back(r);
        }
        steps.emplace_back();
        st = s5d::build_step(items, blob, steps.back());
        if (st != S5D_OK) return st;  // nothing enqueued, nothing committed
      }
    } catch (const std::bad_alloc&) {
      return fail(S5D_ENOMEM, "host allocation failed while planning a tick");
    }
    Slot& sl = s->slots[s->ticks % kSlots];
    if (sl.pending) {
      const hipError_t e = hipEventSynchronize(sl.ev);  // paces the host: at most kSlots ticks in flight
      if (e != hipSuccess) return device_fail(e, "hipEventSynchronize");
      sl.pending = false;
    }
    st = grow_slot(sl, blob.size());
    if (st != S5D_OK) return st;
    std::memcpy(sl.host, blob.data(), blob.size());
    hipError_t e = hipMemcpyAsync(sl.dev, sl.host, blob.size(), hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return device_fail(e, "tick table upload");
    // the staging slot is busy from here on, whatever happens below
    (void)hipEventRecord(sl.ev, s->stream);
    sl.pending = true;
    ++s->ticks;
    const bool inject = s->cfg.fail_tick_every > 0 && (++s->work_ticks % s->cfg.fail_tick_every) == 0;
    size_t j_bad = steps.size();  // first step whose launches did not all go out
    s5d_status bad = S5D_OK;
    for (size_t j = 0; j < steps.size(); ++j) {
      if (inject && j + 1 == steps.size()) {
        bad = fail(S5D_EDEVICE, "injected launch failure (fail_tick_every)");
        j_bad = j;
        break;
      }
      e = s5d::enqueue_step(steps[j], sl.dev, s->stream, &s->ss);
      if (e != hipSuccess) {
        bad = device_fail(e, "tick launch");
        j_bad = j;
        break;
      }
      s->launches += static_cast<int64_t>(steps[j].size());
      // requests whose last round is in step j complete when it does (a
      // request that ends here has no round in a later step, so a failure
      // further on cannot touch it)
      if (!fin_after[j].empty()) {
        const s5d_status fst = record_finish(s, fin_after[j]);
        if (fst != S5D_OK) {
          for (Request* r : fin_after[j]) fail_request(s, r, fst);
          bad = fst;
        }
      }
    }
    if (j_bad == 0) return bad;  // nothing of this tick was enqueued: no round index moves
    // commit the round indices of the launched steps; a request with a round
    // in a step that was not (wholly) launched is FAILED
    std::vector<char> hit(act.size(), 0);
    for (size_t j = j_bad; j < steps.size(); ++j)
      for (size_t i : in_step[j]) hit[i] = 1;
    std::vector<Request*> still;
    for (size_t i = 0; i < act.size(); ++i) {
      Request* r = act[i];
      if (r->state != S5D_REQ_RUNNING) continue;  // failed above
      if (hit[i]) {
        fail_request(s, r, bad);
        continue;
      }
      r->next = nx[i];
      if (r->next < r->rounds.size()) still.push_back(r);
    }
    s->running.swap(still);
    if (bad != S5D_OK) return bad;
  }
  if (n_running) *n_running = static_cast<int32_t>(s->running.size());
  if (n_queued) *n_queued = static_cast<int32_t>(s->queue.size());
  return S5D_OK;
}

s5d_status s5d_server_sync(s5d_server* s) {
  s5d::clear_error();
  if (!s) return fail(S5D_EINVAL, "server is NULL");
  const hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return device_fail(e, "hipStreamSynchronize");
  return retire(s);
}

s5d_status s5d_server_request(const s5d_server* s, int64_t id, s5d_request_info* info) {
  s5d::clear_error();
  if (!s || !info) return fail(S5D_EINVAL, "server and info must not be NULL");
  if (info->struct_size < sizeof(s5d_request_info)) return fail(S5D_EINVAL, "info->struct_size too small");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(S5D_EINVAL, "unknown request id");
  Request* r = it->second.get();
  info->state = r->state;
  info->status = r->status;
  info->result_index = static_cast<int32_t>(r->plan.d.steps % 2);
  info->updates = r->updates;
  info->t_arrival = r->t_arrival;
  info->t_admit = r->t_admit;
  info->t_done = r->t_done;
  info->rounds_done = static_cast<int64_t>(r->next);
  info->init_in_use = (r->state == S5D_REQ_QUEUED || !init_released(s, r)) ? 1 : 0;
  return S5D_OK;
}

s5d_status s5d_server_fetch(s5d_server* s, int64_t id, void* dst) {
  s5d::clear_error();
  if (!s || !dst) return fail(S5D_EINVAL, "server and dst must not be NULL");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(S5D_EINVAL, "unknown request id");
  Request* r = it->second.get();
  if (r->state != S5D_REQ_DONE || !r->keep || !r->buf[0])
    return fail(S5D_EINVAL, "request is not finished or its result was not kept");
  const int64_t T = r->plan.d.steps;
  hipError_t e =
      hipMemcpyAsync(dst, r->buf[T % 2], static_cast<size_t>(r->plan.bytes), hipMemcpyDefault, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return device_fail(e, "result copy");
  release_buffers(s, r);
  r->state = S5D_REQ_RELEASED;
  return S5D_OK;
}

s5d_status s5d_server_get_stats(const s5d_server* s, s5d_server_stats* out) {
  s5d::clear_error();
  if (!s || !out) return fail(S5D_EINVAL, "server and out must not be NULL");
  if (out->struct_size < sizeof(s5d_server_stats)) return fail(S5D_EINVAL, "out->struct_size too small");
  out->submitted = static_cast<int64_t>(s->reqs.size());
  out->queued = static_cast<int64_t>(s->queue.size());
  out->running = static_cast<int64_t>(s->running.size());
  out->done = s->done;
  out->failed = s->failed;
  out->bytes_in_use = s->used;
  out->bytes_peak = s->peak;
  out->ticks = s->ticks;
  out->launches = s->launches;
  out->updates_done = s->updates_done;
  out->latency_p50 = percentile(s->latencies, 0.50);
  out->latency_p99 = percentile(s->latencies, 0.99);
  out->makespan = (s->done > 0 && s->first_arrival >= 0) ? s->last_done - s->first_arrival : 0.0;
  return S5D_OK;
}

}  // extern "C"
