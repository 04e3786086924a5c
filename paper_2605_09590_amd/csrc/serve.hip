// Serving loop: noise-map requests against many operators on one GPU.
//
// Requests (an operator description, a probe range and a caller-owned FP64
// accumulator) queue in arrival order.  A request is admitted when a slot is
// free and its peak device bytes fit beside the resident operators of the
// admitted ones inside the server's HBM budget; the budget is one device
// allocation carved by a first-fit arena, so the loop itself never calls
// hipMalloc / hipFree.  Each slot owns a HIP stream (default priority).  The
// worker thread keeps up to `depth` probe tiles in flight per admitted
// request, round robin over the slots, retires tiles by event, and frees a
// finished request's operator at once, so the next queued request can enter
// while the others keep running (tile-granular continuous batching).
//
// A request's result depends only on its own description and probe range:
// its tiles are the same probe_tile-sized pieces of [0, nprobes) as a direct
// pico_noise_map call would make, accumulated in order on its own stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "arena.h"
#include "pico.h"
#include "runtime.h"

namespace pico {
pico_status_t set_error(pico_status_t st, const std::string& msg);
pico_status_t estimate_bytes(const pico_op_desc_t* d, size_t* resident, size_t* peak);
pico_status_t init_in_arena(const pico_op_desc_t* d, void* stream, DeviceArena* arena, pico_op_t* out);
}  // namespace pico

namespace {

struct Request {
  pico_request_info_t info{};
  pico_op_desc_t desc{};
  std::vector<double> psi;
  uint64_t seed = 0;
  int32_t dist = 0;
  pico_accum_t acc{};
  size_t peak = 0, resident = 0, reserved = 0;
  pico_op_t op = nullptr;
  int slot = -1;
  int64_t issued = 0;
  std::deque<hipEvent_t> inflight;
};

using Clock = std::chrono::steady_clock;

}  // namespace

struct pico_server_s {
  pico::DeviceArena arena;
  pico::DevAllocator base_by;       // allocator that made arena.base
  int device = 0;
  int max_slots = 1, depth = 2;
  std::vector<hipStream_t> streams;
  std::vector<bool> slot_busy;
  std::vector<hipEvent_t> ev_pool;
  Clock::time_point t0 = Clock::now();

  std::mutex mu;
  std::condition_variable cv;       // wakes the worker (submit, stop)
  std::condition_variable idle_cv;  // wakes waiters when a request finishes
  std::deque<std::unique_ptr<Request>> queue;   // guarded by mu
  std::deque<pico_request_info_t> done;         // guarded by mu
  int64_t pending = 0;                          // queued + admitted, guarded by mu
  uint64_t next_id = 1;                         // guarded by mu
  bool stop = false;                            // guarded by mu

  // worker-only state
  std::vector<std::unique_ptr<Request>> active;
  size_t reserved = 0;
  bool blocked = false;   // an admission failed on fragmentation: wait for a completion
  std::thread worker;

  double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }

  hipEvent_t take_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }

  void finish(Request& r) {
    r.info.t_done_ms = now_ms();
    if (r.op) pico_destroy(r.op);   // every tile has retired: releases to the arena only
    r.op = nullptr;
    reserved -= r.reserved;
    if (r.slot >= 0) slot_busy[r.slot] = false;
    blocked = false;
    std::lock_guard<std::mutex> lk(mu);
    done.push_back(r.info);
    --pending;
    idle_cv.notify_all();
  }

  static void fail_request(Request& r, pico_status_t st) {
    r.info.status = st;
    const char* msg = pico_last_error();   // the worker's own (thread-local) message
    std::snprintf(r.info.error, sizeof(r.info.error), "%s", msg ? msg : "");
  }

  int free_slot() const {
    for (int i = 0; i < max_slots; ++i)
      if (!slot_busy[i]) return i;
    return -1;
  }

  // returns true when something changed
  bool retire() {
    bool progress = false;
    for (size_t i = 0; i < active.size();) {
      Request& r = *active[i];
      while (!r.inflight.empty()) {
        const hipError_t q = hipEventQuery(r.inflight.front());
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess && r.info.status == PICO_OK) r.info.status = PICO_EDEVICE;
        ev_pool.push_back(r.inflight.front());
        r.inflight.pop_front();
        progress = true;
      }
      const bool over = r.issued == r.info.probes || r.info.status != PICO_OK;
      if (over && r.inflight.empty()) {
        finish(r);
        active.erase(active.begin() + i);
        progress = true;
      } else {
        ++i;
      }
    }
    return progress;
  }

  bool admit() {
    bool progress = false;
    for (;;) {
      std::unique_ptr<Request> r;
      const int slot = free_slot();
      {
        std::lock_guard<std::mutex> lk(mu);
        if (queue.empty() || slot < 0 || blocked) return progress;
        if (reserved + queue.front()->peak > arena.book.capacity()) return progress;
        r = std::move(queue.front());
        queue.pop_front();
      }
      r->slot = slot;
      r->reserved = r->peak;
      reserved += r->reserved;
      slot_busy[slot] = true;
      r->info.t_admit_ms = now_ms();
      const pico_status_t st = pico::init_in_arena(&r->desc, streams[slot], &arena, &r->op);
      progress = true;
      if (st == PICO_ENOMEM && !active.empty()) {
        // the arena is fragmented: retry once a running request has finished
        reserved -= r->reserved;
        slot_busy[slot] = false;
        blocked = true;
        std::lock_guard<std::mutex> lk(mu);
        queue.push_front(std::move(r));
        return progress;
      }
      if (st != PICO_OK) {
        fail_request(*r, st);
        r->op = nullptr;
        finish(*r);
        continue;
      }
      uint64_t res = 0;
      (void)pico_op_bytes(r->op, &res, nullptr);
      reserved -= r->reserved;
      r->reserved = res;
      reserved += res;
      active.push_back(std::move(r));
    }
  }

  bool issue() {
    bool progress = false;
    for (auto& rp : active) {
      Request& r = *rp;
      const int64_t tile = r.desc.probe_tile;
      while (r.info.status == PICO_OK && (int)r.inflight.size() < depth && r.issued < r.info.probes) {
        const int64_t k = std::min<int64_t>(tile, r.info.probes - r.issued);
        const pico_status_t st =
            pico_noise_map(r.op, r.seed, r.info.first_probe + r.issued, k, r.dist, &r.acc, nullptr,
                           streams[r.slot]);
        if (st != PICO_OK) {
          fail_request(r, st);
          break;
        }
        hipEvent_t e = take_event();
        if (!e || hipEventRecord(e, streams[r.slot]) != hipSuccess) {
          if (e) ev_pool.push_back(e);
          (void)hipStreamSynchronize(streams[r.slot]);   // no event: retire this tile synchronously
        } else {
          r.inflight.push_back(e);
        }
        r.issued += k;
        progress = true;
      }
    }
    return progress;
  }

  void run() {
    (void)hipSetDevice(device);
    for (;;) {
      bool progress = retire();
      progress |= admit();
      progress |= issue();
      std::unique_lock<std::mutex> lk(mu);
      if (stop && queue.empty() && active.empty()) break;
      if (!progress) {
        // outstanding tiles: poll again shortly; otherwise sleep until a submit
        if (!active.empty()) cv.wait_for(lk, std::chrono::microseconds(50));
        else cv.wait(lk, [&] { return stop || (!queue.empty() && !blocked); });
      }
    }
  }
};

extern "C" {

pico_status_t pico_server_create(uint64_t hbm_budget, int32_t max_slots, int32_t tiles_in_flight,
                                 pico_server_t* out) {
  if (!out) return pico::set_error(PICO_EINVAL, "NULL output handle");
  *out = nullptr;
  if (hbm_budget < pico::OffsetArena::kAlign) return pico::set_error(PICO_EINVAL, "hbm_budget too small");
  if (max_slots < 1 || max_slots > 64) return pico::set_error(PICO_EINVAL, "max_slots must be in 1..64");
  if (tiles_in_flight < 1 || tiles_in_flight > 64)
    return pico::set_error(PICO_EINVAL, "tiles_in_flight must be in 1..64");
  auto srv = std::make_unique<pico_server_s>();
  srv->max_slots = max_slots;
  srv->depth = tiles_in_flight;
  if (hipGetDevice(&srv->device) != hipSuccess) return pico::set_error(PICO_EDEVICE, "no current device");
  srv->arena.book.reset(hbm_budget);
  void* base = nullptr;
  hipError_t e = pico::dev_alloc(&base, srv->arena.book.capacity(), &srv->base_by);
  if (e != hipSuccess)
    return pico::set_error(e == hipErrorOutOfMemory ? PICO_ENOMEM : PICO_EDEVICE,
                           std::string("server budget: ") + hipGetErrorString(e));
  srv->arena.base = static_cast<char*>(base);
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t s = nullptr;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) {
      for (hipStream_t t : srv->streams) (void)hipStreamDestroy(t);
      pico::dev_free(base, srv->base_by);
      return pico::set_error(PICO_EDEVICE, std::string("stream: ") + hipGetErrorString(e));
    }
    srv->streams.push_back(s);
  }
  srv->slot_busy.assign(max_slots, false);
  pico_server_s* raw = srv.get();
  srv->worker = std::thread([raw] { raw->run(); });
  *out = srv.release();
  return PICO_OK;
}

pico_status_t pico_server_submit(pico_server_t srv, const pico_op_desc_t* d, uint64_t seed,
                                 int64_t first_probe, int64_t nprobes, int32_t dist,
                                 const pico_accum_t* acc, uint64_t* req_id) {
  if (!srv || !d || !acc || !acc->sum) return pico::set_error(PICO_EINVAL, "NULL server, descriptor or accumulator");
  if (nprobes < 1 || first_probe < 0) return pico::set_error(PICO_EINVAL, "nprobes must be >= 1, first_probe >= 0");
  if (dist < 0 || dist > 3) return pico::set_error(PICO_EINVAL, "unknown probe family");
  size_t resident = 0, peak = 0;
  if (pico_status_t st = pico::estimate_bytes(d, &resident, &peak)) return st;
  if (peak > srv->arena.book.capacity())
    return pico::set_error(PICO_ENOMEM, "request needs " + std::to_string(peak) +
                                            " device bytes, more than the server budget");
  auto r = std::make_unique<Request>();
  r->desc = *d;
  if (d->psi) {
    r->psi.assign(d->psi, d->psi + 2 * (size_t)d->ncoils * d->ncoils);
    r->desc.psi = r->psi.data();
  }
  r->seed = seed;
  r->dist = dist;
  r->acc = *acc;
  r->peak = peak;
  r->resident = resident;
  r->info.first_probe = first_probe;
  r->info.probes = nprobes;
  r->info.status = PICO_OK;
  r->info.bytes_peak = peak;
  r->info.bytes_resident = resident;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return pico::set_error(PICO_EINVAL, "server is shutting down");
    r->info.id = srv->next_id++;
    r->info.t_submit_ms = srv->now_ms();
    if (req_id) *req_id = r->info.id;
    srv->queue.push_back(std::move(r));
    ++srv->pending;
  }
  srv->cv.notify_one();
  return PICO_OK;
}

pico_status_t pico_server_poll(pico_server_t srv, pico_request_info_t* out, int32_t max, int32_t* n) {
  if (!srv || !n || (max > 0 && !out)) return pico::set_error(PICO_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  int32_t k = 0;
  while (k < max && !srv->done.empty()) {
    out[k++] = srv->done.front();
    srv->done.pop_front();
  }
  *n = k;
  return PICO_OK;
}

pico_status_t pico_server_wait_idle(pico_server_t srv, double timeout_s) {
  if (!srv) return pico::set_error(PICO_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(srv->mu);
  const auto pred = [&] { return srv->pending == 0; };
  if (timeout_s < 0) {
    srv->idle_cv.wait(lk, pred);
    return PICO_OK;
  }
  if (!srv->idle_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
    return pico::set_error(PICO_ENOTCONV, "requests still pending after the timeout");
  return PICO_OK;
}

pico_status_t pico_server_usage(pico_server_t srv, uint64_t* budget, uint64_t* arena_used,
                                int32_t* queued, int32_t* active) {
  if (!srv) return pico::set_error(PICO_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (budget) *budget = srv->arena.book.capacity();
  if (arena_used) {
    std::lock_guard<std::mutex> la(srv->arena.mu);
    *arena_used = srv->arena.book.used();
  }
  if (queued) *queued = (int32_t)srv->queue.size();
  if (active) *active = (int32_t)(srv->pending - (int64_t)srv->queue.size());
  return PICO_OK;
}

void pico_server_destroy(pico_server_t srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  if (srv->worker.joinable()) srv->worker.join();   // serves what was submitted, then exits
  for (hipEvent_t e : srv->ev_pool) (void)hipEventDestroy(e);
  for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
  pico::dev_free(srv->arena.base, srv->base_by);
  delete srv;
}

}  // extern "C"
