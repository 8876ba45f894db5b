// Amplitude server: continuous admission of sliced-network requests.
//
// Requests (a tensor network, its path and sliced bonds; Sections II.A-II.B)
// are queued by rn_server_submit.  A worker thread admits them whenever a
// slot (a HIP stream) is free and the request's footprint -- its tensors plus
// the network workspace the planner reports -- fits the HBM budget, either
// in arrival order or smallest first (planned flops) with an aging bound: a
// request overtaken max_overtakes times goes next, and while it does not fit
// the free memory nothing else is admitted.  While younger requests wait,
// aged ones hold at most all but one slot (with two or more slots), so a
// burst of large aged requests cannot shut out the small ones behind them.  Admitted requests copy their
// tensors into a device arena,
// where they stay until the request completes, and run concurrently on
// their slot streams, so a request arriving while others are on the GPU
// starts as soon as memory and a slot free up.  Completion is detected with
// events; latency = completion time - submit time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "rn_internal.hpp"

namespace rn {
namespace {

using Clock = std::chrono::steady_clock;

struct FreeList {
  std::vector<std::pair<size_t, size_t>> blocks;  // (offset, size), sorted, merged
  explicit FreeList(size_t total = 0) {
    if (total) blocks.push_back({0, total});
  }
  bool alloc(size_t size, size_t* off) {
    size = (size + 255) & ~size_t(255);
    for (size_t i = 0; i < blocks.size(); ++i) {
      if (blocks[i].second >= size) {
        *off = blocks[i].first;
        blocks[i].first += size;
        blocks[i].second -= size;
        if (blocks[i].second == 0) blocks.erase(blocks.begin() + i);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t size) {
    size = (size + 255) & ~size_t(255);
    blocks.push_back({off, size});
    std::sort(blocks.begin(), blocks.end());
    std::vector<std::pair<size_t, size_t>> m;
    for (auto& b : blocks) {
      if (!m.empty() && m.back().first + m.back().second == b.first)
        m.back().second += b.second;
      else
        m.push_back(b);
    }
    blocks = m;
  }
};

struct Request {
  uint64_t ticket = 0;
  rn_mode mode = RN_FP64;
  int32_t nt = 0, nsteps = 0, nsliced = 0;
  std::vector<rn_tensor> desc;
  std::vector<std::vector<char>> data;
  std::vector<std::vector<int32_t>> labels;
  std::vector<int32_t> path, sliced;
  size_t ws_bytes = 0, tensor_bytes = 0, footprint = 0;
  double flops = 0;    // planned useful flops (admission order)
  int overtaken = 0;   // later requests admitted before this one
  bool aged = false;   // admitted after being overtaken max_overtakes times
  NetOpts opts;  // batched-slice count fitted to the budget at submission
  std::shared_ptr<void> plan;  // made at submission, run by the worker
  Clock::time_point t_submit, t_start, t_done;
  size_t arena_off = 0;
  int slot = -1;
  hipEvent_t done_ev = nullptr;
};

}  // namespace
}  // namespace rn

struct rn_server {
  rn_handle h = nullptr;
  size_t budget = 0;
  int max_active = 4;
  char* arena = nullptr;
  rn::FreeList free;
  size_t in_use = 0;
  std::vector<hipStream_t> streams;
  std::vector<bool> slot_busy;
  double* amp_host = nullptr;  // pinned, 2 doubles per slot
  std::mutex mu;
  std::condition_variable cv;
  std::deque<rn::Request*> queue;
  std::vector<rn::Request*> active;
  std::map<uint64_t, rn_result> results;
  uint64_t next_ticket = 1;
  int64_t completed = 0;
  int policy = 1;           // 0 arrival order, 1 smallest first with aging
  int max_overtakes = 8;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  bool stop = false;
  std::thread worker;
};

namespace rn {
namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

void finish(rn_server* S, Request* r, int32_t status, const double amp[2]) {
  rn_result res{};
  res.status = status;
  if (amp) {
    res.amp[0] = amp[0];
    res.amp[1] = amp[1];
  }
  auto sec = [](Clock::duration d) { return std::chrono::duration<double>(d).count(); };
  res.latency_s = sec(r->t_done - r->t_submit);
  res.queue_s = status == RN_OK ? sec(r->t_start - r->t_submit) : 0.0;
  res.run_s = status == RN_OK ? sec(r->t_done - r->t_start) : 0.0;
  res.footprint_bytes = (double)r->footprint;
  res.start_s = status == RN_OK ? sec(r->t_start - S->t0) : 0.0;
  res.done_s = sec(r->t_done - S->t0);
  S->results[r->ticket] = res;
  if (r->done_ev) hipEventDestroy(r->done_ev);
  delete r;
}

// Admit r on a free slot: copy tensors into the arena and enqueue the
// network contraction.  Worker thread only, without S->mu held.
int32_t start(rn_server* S, Request* r, int slot) {
  hipStream_t s = S->streams[slot];
  char* base = S->arena + r->arena_off;
  size_t off = 0;
  std::vector<rn_tensor> dev = r->desc;
  hipError_t e = hipSuccess;
  for (int i = 0; i < r->nt && e == hipSuccess; ++i) {
    dev[i].data = base + off;
    e = hipMemcpyAsync(base + off, r->data[i].data(), r->data[i].size(), hipMemcpyHostToDevice,
                       s);
    off += al256(r->data[i].size());
  }
  if (e != hipSuccess) return RN_ERR_HIP;
  double* amp_dev = reinterpret_cast<double*>(base + off);
  off += 256;
  void* ws = base + off;
  std::vector<const int32_t*> lab(r->nt);
  for (int i = 0; i < r->nt; ++i) lab[i] = r->labels[i].data();
  rn_status st = network_run_planned(S->h, r->plan, r->nt, dev.data(), lab.data(), r->nsteps,
                                     r->path.data(), r->nsliced, r->sliced.data(), r->mode, ws,
                                     r->ws_bytes, s, amp_dev, nullptr);
  if (st != RN_OK) return st;
  if (hipMemcpyAsync(S->amp_host + 2 * slot, amp_dev, 2 * sizeof(double), hipMemcpyDeviceToHost,
                     s) != hipSuccess)
    return RN_ERR_HIP;
  if (hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming) != hipSuccess)
    return RN_ERR_HIP;
  if (hipEventRecord(r->done_ev, s) != hipSuccess) return RN_ERR_HIP;
  return RN_OK;
}

void worker_loop(rn_server* S) {
  hipSetDevice(S->h->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool progress = false;
    // Retire finished requests.
    for (size_t i = 0; i < S->active.size();) {
      Request* r = S->active[i];
      const hipError_t q = hipEventQuery(r->done_ev);
      if (q != hipErrorNotReady) {
        // Done, or the stream failed: either way the request leaves.
        r->t_done = Clock::now();
        double amp[2] = {S->amp_host[2 * r->slot], S->amp_host[2 * r->slot + 1]};
        S->slot_busy[r->slot] = false;
        S->free.release(r->arena_off, r->footprint);
        S->in_use -= r->footprint;
        S->active.erase(S->active.begin() + i);
        ++S->completed;
        finish(S, r, q == hipSuccess ? RN_OK : RN_ERR_HIP, q == hipSuccess ? amp : nullptr);
        progress = true;
      } else {
        ++i;
      }
    }
    // Admit while a slot and memory are free.
    for (;;) {
      // Requests that can never fit the budget complete with RN_ERR_OOM.
      for (size_t qi = 0; qi < S->queue.size();) {
        Request* r = S->queue[qi];
        if (r->footprint > S->budget) {
          S->queue.erase(S->queue.begin() + qi);
          r->t_done = Clock::now();
          finish(S, r, RN_ERR_OOM, nullptr);
          progress = true;
        } else {
          ++qi;
        }
      }
      if (S->queue.empty()) break;
      int slot = -1;
      for (int q = 0; q < (int)S->slot_busy.size(); ++q)
        if (!S->slot_busy[q]) {
          slot = q;
          break;
        }
      if (slot < 0) break;
      // Candidates in admission order: arrival order; or an aged request
      // first, then smallest planned flops (ties: arrival).
      std::vector<size_t> cand(S->queue.size());
      for (size_t qi = 0; qi < cand.size(); ++qi) cand[qi] = qi;
      if (S->policy == 1) {
        std::stable_sort(cand.begin(), cand.end(), [&](size_t a, size_t b) {
          const Request* ra = S->queue[a];
          const Request* rb = S->queue[b];
          const bool aa = ra->overtaken >= S->max_overtakes;
          const bool ab = rb->overtaken >= S->max_overtakes;
          if (aa != ab) return aa;
          if (aa) return ra->ticket < rb->ticket;
          if (ra->flops != rb->flops) return ra->flops < rb->flops;
          return ra->ticket < rb->ticket;
        });
      }
      int aged_running = 0;
      for (const Request* a : S->active) aged_running += a->aged ? 1 : 0;
      bool young_waiting = false;
      for (const Request* q : S->queue) young_waiting |= q->overtaken < S->max_overtakes;
      const bool aged_room =
          S->max_active < 2 || !young_waiting || aged_running < S->max_active - 1;
      size_t pick = SIZE_MAX, off = 0;
      for (size_t c : cand) {
        Request* r = S->queue[c];
        const bool aged = S->policy == 1 && r->overtaken >= S->max_overtakes;
        if (aged && !aged_room) continue;  // all but one slot hold aged requests
        if (S->free.alloc(r->footprint, &off)) {
          pick = c;
          break;
        }
        // Arrival order, or an aged request: wait for memory, admit nothing
        // past it.
        if (S->policy == 0 || aged) break;
      }
      if (pick == SIZE_MAX) break;
      Request* r = S->queue[pick];
      r->aged = S->policy == 1 && r->overtaken >= S->max_overtakes;
      for (Request* q : S->queue)
        if (q->ticket < r->ticket) ++q->overtaken;
      S->queue.erase(S->queue.begin() + pick);
      r->arena_off = off;
      r->slot = slot;
      r->t_start = Clock::now();
      S->slot_busy[slot] = true;
      S->in_use += r->footprint;
      // Enqueueing a network takes host time: let submitters and pollers in.
      lk.unlock();
      int32_t st = start(S, r, slot);
      lk.lock();
      if (st != RN_OK) {
        // The slot stream may hold part of the request: drain it first.
        hipStreamSynchronize(S->streams[slot]);
        S->slot_busy[slot] = false;
        S->free.release(off, r->footprint);
        S->in_use -= r->footprint;
        r->t_done = Clock::now();
        finish(S, r, st, nullptr);
      } else {
        S->active.push_back(r);
      }
      progress = true;
    }
    if (progress) S->cv.notify_all();
    if (S->stop && S->queue.empty() && S->active.empty()) break;
    if (S->active.empty())
      S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
    else
      S->cv.wait_for(lk, std::chrono::microseconds(50));
  }
}

}  // namespace
}  // namespace rn

using namespace rn;

extern "C" {

rn_status rn_server_create(int device, size_t hbm_budget, int32_t max_active,
                           rn_server_t* srv) {
  if (!srv) return fail(RN_ERR_INVALID, "null server pointer");
  if (hbm_budget < 4096 || max_active < 1 || max_active > 16)
    return fail(RN_ERR_INVALID, "budget below 4 KiB or max_active outside 1..16");
  rn_server* S = new rn_server();
  rn_status st = rn_create(&S->h, device);
  if (st != RN_OK) {
    delete S;
    return st;
  }
  S->h->graphs_enabled = false;  // every request is a new network
  S->budget = hbm_budget & ~size_t(255);
  S->max_active = max_active;
  hipError_t e = hipMalloc(&S->arena, S->budget);
  if (e == hipSuccess) e = hipHostMalloc(&S->amp_host, sizeof(double) * 2 * max_active,
                                         hipHostMallocDefault);
  for (int i = 0; i < max_active && e == hipSuccess; ++i) {
    hipStream_t s;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) S->streams.push_back(s);
  }
  if (e != hipSuccess) {
    std::string msg = std::string("server resources: ") + hipGetErrorString(e);
    for (auto s : S->streams) hipStreamDestroy(s);
    if (S->amp_host) hipHostFree(S->amp_host);
    if (S->arena) hipFree(S->arena);
    rn_destroy(S->h);
    delete S;
    return fail(RN_ERR_HIP, msg);
  }
  S->free = FreeList(S->budget);
  S->slot_busy.assign(max_active, false);
  S->worker = std::thread(worker_loop, S);
  *srv = S;
  return RN_OK;
}

rn_status rn_server_submit(rn_server_t S, int32_t nt, const rn_tensor* T,
                           const int32_t* const* labels, int32_t nsteps, const int32_t* path,
                           int32_t nsliced, const int32_t* sliced, rn_mode mode,
                           uint64_t* ticket) {
  if (!S || !ticket) return fail(RN_ERR_INVALID, "null argument");
  auto t0 = Clock::now();
  if (nt < 1 || !T || !labels) return fail(RN_ERR_INVALID, "empty network");
  const size_t es = mode == RN_FP64 ? 16 : 8;
  size_t tensor_bytes = 0;
  for (int i = 0; i < nt; ++i) {
    if (T[i].rank < 0 || T[i].rank > 40) return fail(RN_ERR_INVALID, "tensor rank out of range");
    tensor_bytes += al256(es << T[i].rank);
  }
  // Admission granularity: a request whose workspace would not fit the
  // budget beside its tensors runs with fewer sliced bonds batched per pass
  // (more passes, less memory); only one that does not fit even with a
  // single slice per pass is refused at admission.
  NetOpts o;
  const size_t fixed = tensor_bytes + 256;
  o.footprint = S->budget > fixed ? (int64_t)(S->budget - fixed) : 1;
  size_t ws = 0;
  double flops = 0;
  int bb = 0;
  std::shared_ptr<void> plan;
  rn_status st = network_plan_keep(nt, T, labels, nsteps, path, nsliced, sliced, mode, o, &plan,
                                   &ws, &flops, &bb);
  if (st == RN_ERR_OOM) {
    o = NetOpts{};
    st = network_plan_keep(nt, T, labels, nsteps, path, nsliced, sliced, mode, o, &plan, &ws,
                           &flops, &bb);
  }
  if (st != RN_OK) return st;
  o.batch_bits = bb;
  o.footprint = 0;
  Request* r = new Request();
  r->opts = o;
  r->plan = std::move(plan);
  r->mode = mode;
  r->nt = nt;
  r->nsteps = nsteps;
  r->nsliced = nsliced;
  r->desc.assign(T, T + nt);
  for (int i = 0; i < nt; ++i) {
    size_t n = es << T[i].rank;
    r->data.emplace_back(static_cast<const char*>(T[i].data),
                         static_cast<const char*>(T[i].data) + n);
    r->labels.emplace_back(labels[i], labels[i] + T[i].rank);
    r->tensor_bytes += al256(n);
  }
  r->path.assign(path, path + 2 * nsteps);
  r->sliced.assign(sliced, sliced + nsliced);
  r->ws_bytes = ws;
  r->flops = flops;
  r->footprint = r->tensor_bytes + 256 + al256(ws);
  r->t_submit = t0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->queue.push_back(r);
  }
  S->cv.notify_all();
  return RN_OK;
}

rn_status rn_server_set_admission(rn_server_t S, int32_t policy, int32_t max_overtakes) {
  if (!S) return fail(RN_ERR_INVALID, "null server");
  if (policy < 0 || policy > 1 || max_overtakes < 0)
    return fail(RN_ERR_INVALID, "policy is 0 or 1, max_overtakes >= 0");
  std::lock_guard<std::mutex> lk(S->mu);
  S->policy = policy;
  S->max_overtakes = max_overtakes;
  return RN_OK;
}

rn_status rn_server_poll(rn_server_t S, uint64_t ticket, int32_t* done, rn_result* res) {
  if (!S || !done) return fail(RN_ERR_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->results.find(ticket);
  *done = it != S->results.end();
  if (*done && res) *res = it->second;
  return RN_OK;
}

rn_status rn_server_wait(rn_server_t S, uint64_t ticket, rn_result* res) {
  if (!S) return fail(RN_ERR_INVALID, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  if (ticket == 0 || ticket >= S->next_ticket) return fail(RN_ERR_INVALID, "unknown ticket");
  S->cv.wait(lk, [&] { return S->results.count(ticket) > 0; });
  if (res) *res = S->results[ticket];
  return RN_OK;
}

rn_status rn_server_stats(rn_server_t S, int64_t* queued, int64_t* active, int64_t* completed,
                          size_t* bytes_in_use) {
  if (!S) return fail(RN_ERR_INVALID, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  if (queued) *queued = (int64_t)S->queue.size();
  if (active) *active = (int64_t)S->active.size();
  if (completed) *completed = S->completed;
  if (bytes_in_use) *bytes_in_use = S->in_use;
  return RN_OK;
}

rn_status rn_server_destroy(rn_server_t S) {
  if (!S) return RN_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  S->worker.join();
  for (auto s : S->streams) {
    hipStreamSynchronize(s);
    hipStreamDestroy(s);
  }
  hipHostFree(S->amp_host);
  hipFree(S->arena);
  rn_destroy(S->h);
  delete S;
  return RN_OK;
}

}  // extern "C"
