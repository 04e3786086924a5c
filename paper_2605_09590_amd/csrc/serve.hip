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
// finished request's slot at once, so the next queued request can enter
// while the others keep running (tile-granular continuous batching).
// Finished operators stay resident in the budget, keyed by the content of
// their description (scalar fields, psi, and a hash of the device arrays the
// caller passed), and a later request with the same key takes an idle one
// instead of running pico_init; idle operators are evicted least recently
// used when a new one needs their bytes.  A request may leave probe_tile at
// 0: its tile shape then comes from the autotuner's cache file
// (pico_server_set_tuning), else from a size rule.
//
// A request's result depends only on its own description and probe range:
// its tiles are the same probe_tile-sized pieces of [0, nprobes) as a direct
// pico_noise_map call would make, accumulated in order on its own stream (a
// reused operator holds no state from its previous request that its tiles
// read).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
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
bool tune_lookup(const std::string& path, const pico_op_desc_t* d, pico_tune_t* out);
}  // namespace pico

namespace {

constexpr int kHashBlocks = 256;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {   // SplitMix64 finaliser (Steele et al. 2014)
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// XOR over 32-bit words w_i of mix64(i * phi + w_i): order independent, so the
// blocks reduce in any order; part[blockIdx.x] gets each block's share
__global__ void k_hash_words(const uint8_t* __restrict__ data, uint64_t bytes, uint64_t* __restrict__ part) {
  __shared__ uint64_t red[256];
  const uint64_t words = (bytes + 3) / 4;
  uint64_t h = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t w = 0;
    if (4 * i + 4 <= bytes) {
      w = reinterpret_cast<const uint32_t*>(data)[i];
    } else {
      for (uint64_t b = 4 * i; b < bytes; ++b) w |= (uint32_t)data[b] << (8 * (b - 4 * i));
    }
    h ^= mix64(i * 0x9e3779b97f4a7c15ull + w);
  }
  red[threadIdx.x] = h;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] ^= red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

uint64_t mix_host(uint64_t h, uint64_t v) {
  uint64_t z = h ^ (v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2));
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

struct CachedOp {
  uint64_t key = 0;
  pico_op_t op = nullptr;
  size_t resident = 0;
  bool busy = false;
  uint64_t used = 0;
};

struct Request {
  pico_request_info_t info{};
  pico_op_desc_t desc{};
  std::vector<double> psi;
  uint64_t seed = 0;
  int32_t dist = 0;
  pico_accum_t acc{};
  size_t peak = 0, resident = 0, reserved = 0;
  pico_op_t op = nullptr;
  CachedOp* cached = nullptr;   // the resident operator the request runs on
  bool keyed = false;
  uint64_t key = 0;             // content key of the description
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

  std::string tune_path;                        // guarded by mu
  int64_t hits = 0, misses = 0;                 // guarded by mu
  int32_t n_cached = 0;                         // guarded by mu
  uint64_t cached_bytes = 0;                    // guarded by mu

  // worker-only state
  std::vector<std::unique_ptr<Request>> active;
  std::vector<std::unique_ptr<CachedOp>> cache;   // resident operators, busy or idle
  uint64_t clock = 0;
  uint64_t* hash_part = nullptr;                  // [kHashBlocks] in the arena
  size_t reserved = 0;   // resident bytes of every cached operator + peaks of operators being built
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

  void publish_cache_stats() {
    size_t b = 0;
    for (auto& c : cache) b += c->resident;
    std::lock_guard<std::mutex> lk(mu);
    n_cached = (int32_t)cache.size();
    cached_bytes = b;
  }

  void drop(CachedOp* c) {
    pico_destroy(c->op);   // every tile has retired: releases to the arena only
    reserved -= c->resident;
    cache.erase(std::find_if(cache.begin(), cache.end(), [&](const auto& p) { return p.get() == c; }));
  }

  // frees the least recently used idle operator; false if none is idle
  bool evict_one() {
    CachedOp* lru = nullptr;
    for (auto& c : cache)
      if (!c->busy && (!lru || c->used < lru->used)) lru = c.get();
    if (!lru) return false;
    drop(lru);
    return true;
  }

  void finish(Request& r) {
    r.info.t_done_ms = now_ms();
    if (r.cached) {
      if (r.info.status == PICO_OK) {
        r.cached->busy = false;          // stays resident for the next request with its key
        r.cached->used = ++clock;
      } else {
        drop(r.cached);
      }
    } else if (r.op) {
      pico_destroy(r.op);
      reserved -= r.reserved;
    } else {
      reserved -= r.reserved;
    }
    r.cached = nullptr;
    r.op = nullptr;
    publish_cache_stats();
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

  // content key of a description: its scalar fields and psi, and the hashes
  // of the device arrays it points to (read on the slot's stream)
  bool content_key(const pico_op_desc_t& d, hipStream_t st, uint64_t* out) {
    uint64_t h = 0x5049434f;   // "PICO"
    const int32_t ints[] = {d.ny, d.nx, d.ncoils, d.sampling, d.cg_iters, d.power_iters, d.probe_tile, d.recon,
                            d.fista_iters, d.wavelet_levels, d.kb_width, d.normal_form, d.tv_inner_iters,
                            d.storage, d.graph, d.noncart_normal};
    for (int32_t v : ints) h = mix_host(h, (uint64_t)(uint32_t)v);
    const double dbl[] = {d.lambda, d.cg_tol, d.power_margin, d.cs_lambda, d.oversamp};
    for (double v : dbl) {
      uint64_t u;
      std::memcpy(&u, &v, 8);
      h = mix_host(h, u);
    }
    h = mix_host(h, (uint64_t)d.nsamples);
    const size_t n = (size_t)d.ny * d.nx;
    if (d.psi)
      for (size_t i = 0; i < 2 * (size_t)d.ncoils * d.ncoils; ++i) {
        uint64_t u;
        std::memcpy(&u, &d.psi[i], 8);
        h = mix_host(h, u);
      }
    struct Arr {
      const void* p;
      uint64_t bytes;
    } arrs[] = {{d.maps, (uint64_t)d.ncoils * n * 8},
                {d.mask, d.sampling == PICO_CART_1D ? (uint64_t)d.ny : d.sampling == PICO_CART_2D ? (uint64_t)n : 0},
                {d.traj, d.sampling == PICO_NONCART ? (uint64_t)d.nsamples * 8 : 0},
                {d.kdata, d.recon != PICO_CGSENSE ? (uint64_t)d.ncoils * n * 8 : 0}};
    std::vector<uint64_t> part(kHashBlocks);
    for (const Arr& a : arrs) {
      h = mix_host(h, a.p && a.bytes ? a.bytes : 0);
      if (!a.p || !a.bytes) continue;
      hipLaunchKernelGGL(k_hash_words, dim3(kHashBlocks), dim3(256), 0, st, static_cast<const uint8_t*>(a.p),
                         a.bytes, hash_part);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(part.data(), hash_part, kHashBlocks * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return false;
      uint64_t x = 0;
      for (uint64_t v : part) x ^= v;
      h = mix_host(h, x);
    }
    *out = h;
    return true;
  }

  bool admit() {
    bool progress = false;
    for (;;) {
      Request* f = nullptr;
      const int slot = free_slot();
      {
        std::lock_guard<std::mutex> lk(mu);
        if (queue.empty() || slot < 0 || blocked) return progress;
        f = queue.front().get();   // only this thread pops, so f stays valid
      }
      if (!f->keyed) {
        if (!content_key(f->desc, streams[slot], &f->key)) {
          f->key = 0;   // hashing failed: build a fresh operator, never shared
          f->info.op_reused = 0;
        }
        f->keyed = true;
      }
      CachedOp* hit = nullptr;
      if (f->key)
        for (auto& c : cache)
          if (!c->busy && c->key == f->key) hit = c.get();
      if (!hit) {
        // make room among the idle resident operators, oldest first
        while (reserved + f->peak > arena.book.capacity() && evict_one()) progress = true;
        if (reserved + f->peak > arena.book.capacity()) {
          publish_cache_stats();
          return progress;
        }
      }
      std::unique_ptr<Request> r;
      {
        std::lock_guard<std::mutex> lk(mu);
        r = std::move(queue.front());
        queue.pop_front();
        if (hit) ++hits;
        else ++misses;
      }
      r->slot = slot;
      slot_busy[slot] = true;
      r->info.t_admit_ms = now_ms();
      progress = true;
      if (hit) {
        hit->busy = true;
        hit->used = ++clock;
        r->cached = hit;
        r->op = hit->op;
        r->info.op_reused = 1;
        active.push_back(std::move(r));
        continue;
      }
      r->reserved = r->peak;
      reserved += r->reserved;
      pico_status_t st = pico::init_in_arena(&r->desc, streams[slot], &arena, &r->op);
      while (st == PICO_ENOMEM && evict_one()) {   // fragmented: free idle operators and retry
        st = pico::init_in_arena(&r->desc, streams[slot], &arena, &r->op);
      }
      if (st == PICO_ENOMEM && !active.empty()) {
        // still fragmented: retry once a running request has finished
        reserved -= r->reserved;
        r->reserved = 0;
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
      r->reserved = 0;
      reserved += res;
      auto c = std::make_unique<CachedOp>();
      c->key = r->key;
      c->op = r->op;
      c->resident = res;
      c->busy = true;
      c->used = ++clock;
      r->cached = c.get();
      if (r->key) {
        cache.push_back(std::move(c));
      } else {   // unkeyed: not shared; destroyed when it finishes
        r->cached = nullptr;
        r->reserved = res;
        reserved -= res;
        reserved += r->reserved;
      }
      publish_cache_stats();
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
  srv->hash_part = static_cast<uint64_t*>(srv->arena.alloc(kHashBlocks * sizeof(uint64_t)));
  if (!srv->hash_part) {
    pico::dev_free(base, srv->base_by);
    return pico::set_error(PICO_EINVAL, "hbm_budget too small");
  }
  srv->reserved = pico::OffsetArena::round_up(kHashBlocks * sizeof(uint64_t));
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
  pico_op_desc_t dd = *d;
  if (dd.probe_tile == 0) {
    // tile shape from the autotuner's cache, else about 2^23 voxels per tile
    // (power of two in 16..256), never much more than the request's probes
    std::string path;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      path = srv->tune_path;
    }
    pico_tune_t t{};
    if (pico::tune_lookup(path, &dd, &t)) {
      dd.probe_tile = t.probe_tile;
      dd.normal_form = t.normal_form;
      dd.graph = t.graph;
    } else {
      const int64_t n = (int64_t)std::max(dd.ny, 1) * std::max(dd.nx, 1);
      int K = 16;
      while (K < 256 && (int64_t)K * 2 * n <= ((int64_t)1 << 23)) K *= 2;
      while (K > 16 && K / 2 >= nprobes) K /= 2;
      dd.probe_tile = K;
      dd.graph = 1;
    }
  }
  d = &dd;
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
  r->info.probe_tile = d->probe_tile;
  r->info.op_reused = 0;
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

pico_status_t pico_server_set_tuning(pico_server_t srv, const char* cache_path) {
  if (!srv) return pico::set_error(PICO_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->tune_path = cache_path ? cache_path : "";
  return PICO_OK;
}

pico_status_t pico_server_cache_stats(pico_server_t srv, int32_t* resident_ops, uint64_t* resident_bytes,
                                      int64_t* hits, int64_t* misses) {
  if (!srv) return pico::set_error(PICO_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (resident_ops) *resident_ops = srv->n_cached;
  if (resident_bytes) *resident_bytes = srv->cached_bytes;
  if (hits) *hits = srv->hits;
  if (misses) *misses = srv->misses;
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
  for (auto& c : srv->cache) pico_destroy(c->op);
  srv->cache.clear();
  for (hipEvent_t e : srv->ev_pool) (void)hipEventDestroy(e);
  for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
  pico::dev_free(srv->arena.base, srv->base_by);
  delete srv;
}

}  // extern "C"
