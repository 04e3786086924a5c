// Tile-shape autotuner: for one operator description, times the candidate
// probe tiles (right-hand sides per batched CG / tangent batch), the
// phase-encode normal-operator forms (column FFTs, dense blocks on the FP32
// or split-FP16 matrix cores) and direct launches against graph replay on a
// short noise-map run, keeps the fastest, and records it in a text cache keyed
// by the shape of the problem, so later calls (and the serving loop, for
// requests that leave probe_tile at 0) take the measured choice without timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "arena.h"
#include "pico.h"
#include "runtime.h"

namespace pico {
pico_status_t set_error(pico_status_t st, const std::string& msg);
pico_status_t estimate_bytes(const pico_op_desc_t* d, size_t* resident, size_t* peak);

// Shape key: everything the cost depends on, coil counts in buckets of 8 and
// non-Cartesian sample counts in buckets of 4096.
std::string tune_key(const pico_op_desc_t* d) {
  const bool cs = d->recon != PICO_CGSENSE;
  const long ns = d->sampling == PICO_NONCART ? (long)((d->nsamples + 4095) / 4096) : 0;
  char buf[256];
  std::snprintf(buf, sizeof buf, "s%d_r%d_%dx%d_c%d_it%d_tikh%d_st%d_T%d_in%d_lv%d_m%ld_g%d", d->sampling, d->recon,
                d->ny, d->nx, (d->ncoils + 7) / 8 * 8, cs ? 0 : d->cg_iters, (!cs && d->lambda > 0.0) ? 1 : 0,
                d->storage, cs ? d->fista_iters : 0, d->recon == PICO_CS_FISTA_TV ? d->tv_inner_iters : 0,
                d->recon == PICO_CS_FISTA_L1WAV ? d->wavelet_levels : 0, ns,
                d->sampling == PICO_NONCART ? d->noncart_normal : 0);
  return buf;
}

namespace {

std::mutex g_tune_mu;

bool read_cache(const std::string& path, std::map<std::string, pico_tune_t>& out) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    std::string key;
    pico_tune_t t{};
    if (is >> key >> t.probe_tile >> t.normal_form >> t.graph >> t.probes_per_s) out[key] = t;
  }
  return true;
}

bool write_cache(const std::string& path, const std::map<std::string, pico_tune_t>& m) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return false;
    f << "# libpico tile tuning: key probe_tile normal_form graph probes_per_s\n";
    for (const auto& kv : m)
      f << kv.first << ' ' << kv.second.probe_tile << ' ' << kv.second.normal_form << ' ' << kv.second.graph << ' '
        << kv.second.probes_per_s << '\n';
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

// probes per second of one candidate: a warm-up tile, then tiles until at
// least 2 and 20 ms of device time
pico_status_t time_candidate(const pico_op_desc_t* d, hipStream_t s, double* rate) {
  pico_op_t op = nullptr;
  if (pico_status_t st = pico_init(d, s, &op)) return st;
  const size_t n = (size_t)d->ny * d->nx;
  void* buf = nullptr;
  DevAllocator by;
  hipError_t e = dev_alloc(&buf, OffsetArena::round_up(3 * n * sizeof(double)), &by);
  if (e != hipSuccess) {
    pico_destroy(op);
    return set_error(PICO_ENOMEM, "autotune accumulators");
  }
  double* acc3 = static_cast<double*>(buf);
  pico_accum_t acc{acc3, acc3 + n, acc3 + 2 * n, 0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  pico_status_t st = PICO_OK;
  int64_t probes = 0;
  float ms = 0.0f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    st = set_error(PICO_EDEVICE, "autotune events");
  } else if ((st = pico_noise_map(op, 1, 0, d->probe_tile, 0, &acc, nullptr, s)) == PICO_OK) {
    const int64_t K = d->probe_tile;
    int tiles = 0;
    (void)hipEventRecord(e0, s);
    for (;;) {
      if ((st = pico_noise_map(op, 1, (tiles + 1) * K, K, 0, &acc, nullptr, s)) != PICO_OK) break;
      ++tiles;
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) {
        st = set_error(PICO_EDEVICE, "autotune timing");
        break;
      }
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (tiles >= 2 && ms >= 20.0f) break;
    }
    probes = (int64_t)tiles * K;
  }
  (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  dev_free(buf, by);
  pico_destroy(op);
  if (st == PICO_OK) *rate = ms > 0.0f ? probes / (ms * 1e-3) : 0.0;
  return st;
}

}  // namespace

// Cached choice for desc (false if none), for the serving loop
bool tune_lookup(const std::string& path, const pico_op_desc_t* d, pico_tune_t* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::map<std::string, pico_tune_t> m;
  if (path.empty() || !read_cache(path, m)) return false;
  auto it = m.find(tune_key(d));
  if (it == m.end()) return false;
  *out = it->second;
  out->from_cache = 1;
  return true;
}

}  // namespace pico

extern "C" {

pico_status_t pico_autotune(const pico_op_desc_t* desc, uint64_t max_bytes, const char* cache_path, void* stream,
                            pico_tune_t* out) {
  if (!desc || !out) return pico::set_error(PICO_EINVAL, "NULL descriptor or output");
  const std::string path = cache_path ? cache_path : "";
  if (pico::tune_lookup(path, desc, out)) return PICO_OK;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int> forms = {desc->normal_form};
  if (desc->sampling == PICO_CART_1D && desc->recon == PICO_CGSENSE) {
    forms = {1};
    if (pico::gram_supported(desc->ny)) {
      forms.push_back(2);
      forms.push_back(3);
    }
  }
  pico_tune_t best{};
  bool any = false;
  std::string why;
  pico_op_desc_t d = *desc;
  for (int form : forms) {
    double form_best = 0.0;
    for (int K : {16, 32, 64, 128, 256, 512}) {
      d.probe_tile = K;
      d.normal_form = form;
      d.graph = 1;
      size_t res = 0, peak = 0;
      if (pico_status_t st = pico::estimate_bytes(&d, &res, &peak)) return st;
      if (max_bytes && peak > max_bytes) continue;
      double rate = 0.0;
      const pico_status_t st = pico::time_candidate(&d, s, &rate);
      if (st == PICO_ENOMEM) {
        why = pico_last_error();
        continue;
      }
      if (st != PICO_OK) return st;
      if (!any || rate > best.probes_per_s) best = {K, form, 1, rate, 0};
      any = true;
      // larger tiles only pay while the device is not yet full: stop this
      // form once doubling the tile gains less than 3 %
      if (rate < 1.03 * form_best) break;
      form_best = std::max(form_best, rate);
    }
  }
  if (!any) return pico::set_error(PICO_ENOMEM, "no probe tile fits the byte limit" + (why.empty() ? "" : ": " + why));
  // graph replay against direct launches at the chosen shape
  d.probe_tile = best.probe_tile;
  d.normal_form = best.normal_form;
  d.graph = 0;
  double direct = 0.0;
  if (pico::time_candidate(&d, s, &direct) == PICO_OK && direct > best.probes_per_s) {
    best.graph = 0;
    best.probes_per_s = direct;
  }
  *out = best;
  if (!path.empty()) {
    std::lock_guard<std::mutex> lk(pico::g_tune_mu);
    std::map<std::string, pico_tune_t> m;
    pico::read_cache(path, m);
    m[pico::tune_key(desc)] = best;
    if (!pico::write_cache(path, m)) return pico::set_error(PICO_EINVAL, "cannot write the tuning cache " + path);
  }
  return PICO_OK;
}

}  // extern "C"
