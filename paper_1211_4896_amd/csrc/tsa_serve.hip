// Request serving over resident cubes: admission by scratch budget,
// continuous batching of region requests, full-cube requests on their own
// stream, event-polled retirement (include/tsa_serve.h).
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tsa_serve.h"
#include "tsa_internal.hpp"

namespace tsa {
size_t batch_ws_bytes(const tsa_cube* cube, int32_t nbins, int32_t nq);
int run_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                     tsa_result* d_results, uint64_t* d_hists, const tsa_tune* tune, void* d_ws, size_t ws_bytes,
                     tsa_stream_t stream);
}  // namespace tsa

using namespace tsa;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Item {
  tsa_request req;
  tsa_response resp;
  int64_t replay_index;  // >= 0: response goes to the replay output array
  size_t cost;
};

struct CubeRec {
  tsa_cube cube;
  float lo, hi;
  bool range_ok;
  size_t full_ws;
};

struct RegionLane {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  tsa_region* d_regions = nullptr;
  tsa_result* d_results = nullptr;
  uint64_t* d_hists = nullptr;
  tsa_region* h_regions = nullptr;
  tsa_result* h_results = nullptr;
  uint64_t* h_hists = nullptr;
  std::vector<Item*> items;
  bool busy = false;
};

struct FullLane {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  tsa_result* d_result = nullptr;
  uint64_t* d_counts = nullptr;
  uint64_t* d_outl = nullptr;
  tsa_result* h_result = nullptr;
  uint64_t* h_counts = nullptr;
  std::vector<Item*> items;  // every request the current shared scan answers
  bool has_hist = false;
  bool busy = false;
};

}  // namespace

struct tsa_server {
  tsa_server_config cfg;
  int device = 0;
  std::vector<CubeRec> cubes;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Item*> arrivals;            // guarded by mu
  std::deque<Item*> done;                // guarded by mu
  uint64_t submitted = 0, finished = 0;  // guarded by mu
  tsa_response* replay_out = nullptr;    // guarded by mu
  // scheduler-thread state
  std::deque<Item*> pend_region, pend_full, adm_region, adm_full;
  std::vector<RegionLane> rl;
  FullLane fl;
  size_t region_cost = 0;
  size_t budget_used = 0;
  std::atomic<size_t> budget_peak{0};
  int admitted = 0;
  std::atomic<bool> stop{false};
  std::thread th;
  // counters
  uint64_t n_batches = 0, n_batch_items = 0, n_full = 0, n_scans = 0, max_batch_seen = 0, n_admit_waits = 0;
  double busy_region_s = 0, busy_full_s = 0;
};

namespace {

void fail_item(tsa_server* s, Item* it, int status) {
  it->resp.status = status;
  it->resp.t_done = now_s();
}

void finish_item(tsa_server* s, Item* it) {
  std::lock_guard<std::mutex> g(s->mu);
  if (it->replay_index >= 0 && s->replay_out) {
    s->replay_out[it->replay_index] = it->resp;
    delete it;
  } else {
    s->done.push_back(it);
  }
  s->finished++;
  s->cv.notify_all();
}

tsa_result nan_result() {
  tsa_result r;
  r.count = r.nan_count = 0;
  r.mean = r.m2 = r.std = r.min = r.max = r.median = __builtin_nan("");
  r.status = TSA_OK;
  r.flags = 0;
  return r;
}

void release(tsa_server* s, Item* it) {
  s->budget_used -= it->cost;
  s->admitted--;
}

// retire finished lanes; returns true if anything finished
bool retire(tsa_server* s) {
  bool did = false;
  for (RegionLane& L : s->rl) {
    if (!L.busy || hipEventQuery(L.ev) != hipSuccess) continue;
    const double t = now_s();
    const int nb = s->cfg.region_nbins;
    for (size_t i = 0; i < L.items.size(); ++i) {
      Item* it = L.items[i];
      it->resp.result = L.h_results[i];
      it->resp.status = L.h_results[i].status;
      if (it->req.h_hist) memcpy(it->req.h_hist, L.h_hists + i * (size_t)nb, sizeof(uint64_t) * nb);
      it->resp.t_done = t;
      release(s, it);
      finish_item(s, it);
    }
    L.items.clear();
    L.busy = false;
    did = true;
  }
  if (s->fl.busy && hipEventQuery(s->fl.ev) == hipSuccess) {
    const double t = now_s();
    uint64_t tot = 0;
    if (s->fl.has_hist)
      for (int b = 0; b < s->cfg.full_nbins; ++b) tot += s->fl.h_counts[b];
    for (Item* it : s->fl.items) {
      const CubeRec& c = s->cubes[it->req.cube];
      tsa_result r = nan_result();
      r.status = s->fl.h_result->status;
      if (it->req.kind == TSA_REQ_FULL_MEDIAN) {
        r.count = s->fl.h_result->count;
        r.nan_count = s->fl.h_result->nan_count;
        r.median = s->fl.h_result->median;
      } else {
        r.count = tot;
        r.min = c.lo;
        r.max = c.hi;
        if (it->req.h_hist) memcpy(it->req.h_hist, s->fl.h_counts, sizeof(uint64_t) * s->cfg.full_nbins);
      }
      it->resp.result = r;
      it->resp.status = r.status;
      it->resp.t_done = t;
      release(s, it);
      finish_item(s, it);
    }
    s->fl.items.clear();
    s->fl.busy = false;
    did = true;
  }
  return did;
}

size_t item_cost(tsa_server* s, const Item* it) {
  if (it->req.kind == TSA_REQ_REGION) return s->region_cost;
  return s->cubes[it->req.cube].full_ws + sizeof(uint64_t) * (size_t)s->cfg.full_nbins;
}

// arrivals -> pending -> admitted (FIFO per class, while slots and scratch allow)
bool admit(tsa_server* s) {
  bool did = false;
  {
    std::lock_guard<std::mutex> g(s->mu);
    while (!s->arrivals.empty()) {
      Item* it = s->arrivals.front();
      s->arrivals.pop_front();
      (it->req.kind == TSA_REQ_REGION ? s->pend_region : s->pend_full).push_back(it);
      did = true;
    }
  }
  const size_t cap = s->cfg.scratch_bytes;
  for (int round = 0; round < 2; ++round) {
    std::deque<Item*>& P = round == 0 ? s->pend_full : s->pend_region;
    std::deque<Item*>& A = round == 0 ? s->adm_full : s->adm_region;
    while (!P.empty()) {
      Item* it = P.front();
      const size_t c = item_cost(s, it);
      if (s->admitted >= s->cfg.max_admitted || (cap && s->budget_used + c > cap)) {
        s->n_admit_waits++;
        break;
      }
      P.pop_front();
      it->cost = c;
      s->budget_used += c;
      if (s->budget_used > s->budget_peak.load()) s->budget_peak.store(s->budget_used);
      s->admitted++;
      it->resp.t_admit = now_s();
      A.push_back(it);
      did = true;
    }
  }
  return did;
}

bool launch(tsa_server* s) {
  bool did = false;
  for (RegionLane& L : s->rl) {
    if (L.busy || s->adm_region.empty()) continue;
    // one cube per batch: the cube of the oldest admitted request
    const int32_t cube = s->adm_region.front()->req.cube;
    std::deque<Item*> keep;
    while (!s->adm_region.empty() && (int)L.items.size() < s->cfg.max_batch) {
      Item* it = s->adm_region.front();
      s->adm_region.pop_front();
      if (it->req.cube == cube)
        L.items.push_back(it);
      else
        keep.push_back(it);
    }
    while (!keep.empty()) {
      s->adm_region.push_front(keep.back());
      keep.pop_back();
    }
    const int nq = (int)L.items.size();
    // pad to a power of two with empty boxes (rejected at once by the planner),
    // so each lane replays a handful of captured launch graphs
    int nq_pad = 1;
    while (nq_pad < nq) nq_pad <<= 1;
    if (nq_pad > s->cfg.max_batch) nq_pad = s->cfg.max_batch;
    const double t = now_s();
    for (int i = 0; i < nq; ++i) {
      L.h_regions[i] = L.items[i]->req.region;
      L.items[i]->resp.t_launch = t;
    }
    for (int i = nq; i < nq_pad; ++i) L.h_regions[i] = tsa_region{0, 0, 0, 0, 0, 0};
    const CubeRec& c = s->cubes[cube];
    int st = hipMemcpyAsync(L.d_regions, L.h_regions, sizeof(tsa_region) * nq_pad, hipMemcpyHostToDevice,
                            L.stream) == hipSuccess
                 ? TSA_OK
                 : TSA_EDEVICE;
    if (st == TSA_OK)
      st = run_region_batch(&c.cube, L.d_regions, nq_pad, s->cfg.region_nbins, L.d_results, L.d_hists, nullptr,
                            L.d_ws, L.ws_bytes, (tsa_stream_t)L.stream);
    if (st == TSA_OK &&
        (hipMemcpyAsync(L.h_results, L.d_results, sizeof(tsa_result) * nq, hipMemcpyDeviceToHost, L.stream) !=
             hipSuccess ||
         hipMemcpyAsync(L.h_hists, L.d_hists, sizeof(uint64_t) * (size_t)nq * s->cfg.region_nbins,
                        hipMemcpyDeviceToHost, L.stream) != hipSuccess ||
         hipEventRecord(L.ev, L.stream) != hipSuccess))
      st = TSA_EDEVICE;
    if (st != TSA_OK) {
      for (Item* it : L.items) {
        fail_item(s, it, st);
        release(s, it);
        finish_item(s, it);
      }
      L.items.clear();
      continue;
    }
    L.busy = true;
    s->n_batches++;
    s->n_batch_items += (uint64_t)nq;
    if ((uint64_t)nq > s->max_batch_seen) s->max_batch_seen = (uint64_t)nq;
    did = true;
  }
  if (!s->fl.busy && !s->adm_full.empty()) {
    // one shared scan answers every admitted full-cube request on the cube of
    // the oldest one: histogram requests share one pass, median requests the
    // two radix passes, and both kinds together the fused two-pass trio
    const int32_t cube = s->adm_full.front()->req.cube;
    std::deque<Item*> keep;
    bool any_hist = false, any_median = false;
    while (!s->adm_full.empty()) {
      Item* it = s->adm_full.front();
      s->adm_full.pop_front();
      if (it->req.cube == cube) {
        s->fl.items.push_back(it);
        any_hist |= it->req.kind == TSA_REQ_FULL_HIST;
        any_median |= it->req.kind == TSA_REQ_FULL_MEDIAN;
      } else {
        keep.push_back(it);
      }
    }
    while (!keep.empty()) {
      s->adm_full.push_front(keep.back());
      keep.pop_back();
    }
    const CubeRec& c = s->cubes[cube];
    const double t = now_s();
    for (Item* it : s->fl.items) it->resp.t_launch = t;
    const tsa_stream_t fs = (tsa_stream_t)s->fl.stream;
    int st = TSA_OK;
    if (any_hist && !c.range_ok) st = TSA_EINVAL;
    const size_t fused_lds = ((size_t)s->cfg.full_nbins + 64 + 4096) * 4;
    if (st == TSA_OK && any_hist && any_median && fused_lds <= 65536) {
      st = run_stats(&c.cube, nullptr, s->cfg.full_nbins, s->fl.d_result, s->fl.d_counts, s->fl.d_outl, s->fl.d_ws,
                     s->fl.ws_bytes, fs);
    } else {
      if (st == TSA_OK && any_hist)
        st = run_histogram(&c.cube, nullptr, c.lo, c.hi, s->cfg.full_nbins, s->fl.d_counts, s->fl.d_outl,
                           s->fl.d_ws, s->fl.ws_bytes, fs);
      if (st == TSA_OK && any_median)
        st = run_median(&c.cube, nullptr, s->fl.d_result, s->fl.d_ws, s->fl.ws_bytes, fs);
    }
    if (st == TSA_OK && !any_median) {
      tsa_result ok = nan_result();
      *s->fl.h_result = ok;  // only histograms: no device result to copy
    }
    if (st == TSA_OK && any_median &&
        hipMemcpyAsync(s->fl.h_result, s->fl.d_result, sizeof(tsa_result), hipMemcpyDeviceToHost, s->fl.stream) !=
            hipSuccess)
      st = TSA_EDEVICE;
    if (st == TSA_OK && any_hist &&
        hipMemcpyAsync(s->fl.h_counts, s->fl.d_counts, sizeof(uint64_t) * s->cfg.full_nbins, hipMemcpyDeviceToHost,
                       s->fl.stream) != hipSuccess)
      st = TSA_EDEVICE;
    if (st == TSA_OK && hipEventRecord(s->fl.ev, s->fl.stream) != hipSuccess) st = TSA_EDEVICE;
    if (st != TSA_OK) {
      for (Item* it : s->fl.items) {
        it->resp.result = nan_result();
        it->resp.result.status = st;
        fail_item(s, it, st);
        release(s, it);
        finish_item(s, it);
      }
      s->fl.items.clear();
    } else {
      s->fl.has_hist = any_hist;
      s->fl.busy = true;
      s->n_full += s->fl.items.size();
      s->n_scans++;
    }
    did = true;
  }
  return did;
}

void scheduler(tsa_server* s) {
  (void)hipSetDevice(s->device);
  int idle = 0;
  for (;;) {
    bool did = retire(s);
    did |= admit(s);
    did |= launch(s);
    if (s->stop.load()) {
      bool busy = s->fl.busy;
      for (RegionLane& L : s->rl) busy |= L.busy;
      std::lock_guard<std::mutex> g(s->mu);
      if (!busy && s->arrivals.empty() && s->pend_region.empty() && s->pend_full.empty() && s->adm_region.empty() &&
          s->adm_full.empty())
        break;
    }
    if (did) {
      idle = 0;
    } else if (++idle > 64) {
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    } else {
      std::this_thread::yield();
    }
  }
}

void free_lanes(tsa_server* s) {
  for (RegionLane& L : s->rl) {
    if (L.stream) (void)hipStreamDestroy(L.stream);
    if (L.ev) (void)hipEventDestroy(L.ev);
    (void)hipFree(L.d_ws);
    (void)hipFree(L.d_regions);
    (void)hipFree(L.d_results);
    (void)hipFree(L.d_hists);
    (void)hipHostFree(L.h_regions);
    (void)hipHostFree(L.h_results);
    (void)hipHostFree(L.h_hists);
  }
  FullLane& F = s->fl;
  if (F.stream) (void)hipStreamDestroy(F.stream);
  if (F.ev) (void)hipEventDestroy(F.ev);
  (void)hipFree(F.d_ws);
  (void)hipFree(F.d_result);
  (void)hipFree(F.d_counts);
  (void)hipFree(F.d_outl);
  (void)hipHostFree(F.h_result);
  (void)hipHostFree(F.h_counts);
}

}  // namespace

extern "C" {

double tsa_server_now(void) { return now_s(); }

int tsa_server_create(const tsa_server_config* cfg, tsa_server** out) {
  if (!cfg || !out) return TSA_EINVAL;
  if (cfg->max_batch < 1 || cfg->max_batch > 4096 || cfg->region_lanes < 1 || cfg->region_lanes > 4 ||
      cfg->max_admitted < 1 || cfg->region_nbins < 1 || cfg->region_nbins > 4096 || cfg->full_nbins < 1 ||
      cfg->full_nbins > 65536 || cfg->reserved != 0)
    return TSA_EINVAL;
  DevInfo dev;
  int st = device_info(&dev);
  if (st) return st;
  tsa_server* s = new tsa_server();
  s->cfg = *cfg;
  (void)hipGetDevice(&s->device);
  // a valid cube descriptor for the layout query (the batch layout depends on nq only)
  tsa_cube probe = {(const void*)256, TSA_F32, 0, 4, 1, 1};
  const size_t bws = batch_ws_bytes(&probe, cfg->region_nbins, cfg->max_batch);
  s->region_cost = bws / (size_t)cfg->max_batch + sizeof(tsa_result) + sizeof(tsa_region) +
                   sizeof(uint64_t) * (size_t)cfg->region_nbins;
  s->rl.resize(cfg->region_lanes);
  bool ok = bws > 0;
  for (RegionLane& L : s->rl) {
    const size_t nq = (size_t)cfg->max_batch, nb = (size_t)cfg->region_nbins;
    ok = ok && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc(&L.d_ws, bws) == hipSuccess;
    L.ws_bytes = bws;
    ok = ok && hipMalloc((void**)&L.d_regions, sizeof(tsa_region) * nq) == hipSuccess;
    ok = ok && hipMalloc((void**)&L.d_results, sizeof(tsa_result) * nq) == hipSuccess;
    ok = ok && hipMalloc((void**)&L.d_hists, sizeof(uint64_t) * nq * nb) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&L.h_regions, sizeof(tsa_region) * nq, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&L.h_results, sizeof(tsa_result) * nq, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&L.h_hists, sizeof(uint64_t) * nq * nb, hipHostMallocDefault) == hipSuccess;
  }
  FullLane& F = s->fl;
  ok = ok && hipStreamCreateWithFlags(&F.stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&F.ev, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipMalloc((void**)&F.d_result, sizeof(tsa_result)) == hipSuccess;
  ok = ok && hipMalloc((void**)&F.d_counts, sizeof(uint64_t) * cfg->full_nbins) == hipSuccess;
  ok = ok && hipMalloc((void**)&F.d_outl, 2 * sizeof(uint64_t)) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&F.h_result, sizeof(tsa_result), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&F.h_counts, sizeof(uint64_t) * cfg->full_nbins, hipHostMallocDefault) ==
                 hipSuccess;
  if (!ok) {
    free_lanes(s);
    delete s;
    return TSA_EDEVICE;
  }
  s->th = std::thread(scheduler, s);
  *out = s;
  return TSA_OK;
}

int tsa_server_add_cube(tsa_server* s, const tsa_cube* cube, int32_t* id) {
  if (!s || !cube || !id) return TSA_EINVAL;
  int st = check_cube(cube);
  if (st) return st;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->submitted != s->finished) return TSA_EBUSY;  // add cubes while idle
  // min/max now, as the data "loads"
  const size_t ws = tsa_workspace_bytes(TSA_OP_MOMENTS, cube, nullptr, 0, 0);
  const size_t full_ws = tsa_workspace_bytes(TSA_OP_MEDIAN, cube, nullptr, 0, 0);
  const size_t hws = tsa_workspace_bytes(TSA_OP_HISTOGRAM, cube, nullptr, s->cfg.full_nbins, 0);
  size_t need = ws > full_ws ? ws : full_ws;
  if (hws > need) need = hws;
  FullLane& F = s->fl;
  if (need > F.ws_bytes) {
    (void)hipStreamSynchronize(F.stream);
    (void)hipFree(F.d_ws);
    F.d_ws = nullptr;
    if (hipMalloc(&F.d_ws, need) != hipSuccess) {
      F.ws_bytes = 0;
      return TSA_EDEVICE;
    }
    F.ws_bytes = need;
  }
  st = run_moments(cube, nullptr, F.d_result, F.d_ws, F.ws_bytes, (tsa_stream_t)F.stream);
  if (st) return st;
  tsa_result r;
  if (hipMemcpyAsync(&r, F.d_result, sizeof(r), hipMemcpyDeviceToHost, F.stream) != hipSuccess ||
      hipStreamSynchronize(F.stream) != hipSuccess)
    return TSA_EDEVICE;
  CubeRec c;
  c.cube = *cube;
  c.lo = (float)r.min;
  c.hi = (float)r.max;
  c.range_ok = r.count > 0 && std::isfinite(c.lo) && std::isfinite(c.hi) && std::isfinite(c.hi - c.lo);
  c.full_ws = full_ws > hws ? full_ws : hws;
  s->cubes.push_back(c);
  *id = (int32_t)s->cubes.size() - 1;
  return TSA_OK;
}

static int submit_item(tsa_server* s, const tsa_request* r, int64_t replay_index) {
  if (!s || !r) return TSA_EINVAL;
  if (r->kind < TSA_REQ_REGION || r->kind > TSA_REQ_FULL_MEDIAN) return TSA_EINVAL;
  Item* it = new Item();
  it->req = *r;
  it->replay_index = replay_index;
  it->cost = 0;
  it->resp.tag = r->tag;
  it->resp.kind = r->kind;
  it->resp.status = TSA_OK;
  it->resp.result = nan_result();
  it->resp.t_submit = now_s();
  it->resp.t_admit = it->resp.t_launch = it->resp.t_done = 0.0;
  std::lock_guard<std::mutex> g(s->mu);
  if (r->cube < 0 || r->cube >= (int32_t)s->cubes.size()) {
    delete it;
    return TSA_EINVAL;
  }
  // a request costing more than the whole budget could never be admitted and
  // would hold up every later request of its class
  if (s->cfg.scratch_bytes && item_cost(s, it) > s->cfg.scratch_bytes) {
    delete it;
    return TSA_ENOMEM;
  }
  if (s->arrivals.size() >= (1u << 20)) {
    delete it;
    return TSA_EBUSY;
  }
  s->arrivals.push_back(it);
  s->submitted++;
  return TSA_OK;
}

int tsa_server_submit(tsa_server* s, const tsa_request* r) { return submit_item(s, r, -1); }

int tsa_server_poll(tsa_server* s, tsa_response* out, int32_t cap) {
  if (!s || (!out && cap > 0)) return TSA_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  int n = 0;
  while (n < cap && !s->done.empty()) {
    Item* it = s->done.front();
    s->done.pop_front();
    out[n++] = it->resp;
    delete it;
  }
  return n;
}

int tsa_server_drain(tsa_server* s, double timeout_s) {
  if (!s) return TSA_EINVAL;
  std::unique_lock<std::mutex> g(s->mu);
  auto pred = [s] { return s->finished == s->submitted; };
  if (timeout_s <= 0) {
    s->cv.wait(g, pred);
    return TSA_OK;
  }
  return s->cv.wait_for(g, std::chrono::duration<double>(timeout_s), pred) ? TSA_OK : TSA_EBUSY;
}

int tsa_server_replay(tsa_server* s, const tsa_request* reqs, const double* t_arrival, int32_t n,
                      tsa_response* out) {
  if (!s || n < 0 || (n > 0 && (!reqs || !t_arrival || !out))) return TSA_EINVAL;
  {
    std::unique_lock<std::mutex> g(s->mu);
    s->cv.wait(g, [s] { return s->finished == s->submitted; });
    s->replay_out = out;
  }
  const double t0 = now_s();
  for (int32_t i = 0; i < n; ++i) {
    const double due = t0 + t_arrival[i];
    for (;;) {
      const double left = due - now_s();
      if (left <= 0) break;
      if (left > 200e-6)
        std::this_thread::sleep_for(std::chrono::duration<double>(left - 150e-6));
      else
        std::this_thread::yield();
    }
    const int st = submit_item(s, &reqs[i], i);
    if (st) {
      out[i].tag = reqs[i].tag;
      out[i].status = st;
      out[i].kind = reqs[i].kind;
    }
  }
  std::unique_lock<std::mutex> g(s->mu);
  s->cv.wait(g, [s] { return s->finished == s->submitted; });
  s->replay_out = nullptr;
  return TSA_OK;
}

int tsa_server_stats(tsa_server* s, char* buf, size_t len) {
  if (!s || !buf) return TSA_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  char tmp[768];
  const int n = snprintf(tmp, sizeof(tmp),
                         "{\"batches\": %llu, \"batched_requests\": %llu, \"max_batch\": %llu, \"full_requests\": "
                         "%llu, \"full_scans\": %llu, \"admission_waits\": %llu, \"submitted\": %llu, "
                         "\"finished\": %llu, \"scratch_bytes\": %llu, \"budget_peak\": %llu, "
                         "\"region_cost\": %llu}",
                         (unsigned long long)s->n_batches, (unsigned long long)s->n_batch_items,
                         (unsigned long long)s->max_batch_seen, (unsigned long long)s->n_full,
                         (unsigned long long)s->n_scans,
                         (unsigned long long)s->n_admit_waits, (unsigned long long)s->submitted,
                         (unsigned long long)s->finished, (unsigned long long)s->cfg.scratch_bytes,
                         (unsigned long long)s->budget_peak.load(), (unsigned long long)s->region_cost);
  if (n < 0 || (size_t)n + 1 > len) return TSA_ENOMEM;
  memcpy(buf, tmp, (size_t)n + 1);
  return n;
}

int tsa_server_destroy(tsa_server* s) {
  if (!s) return TSA_EINVAL;
  s->stop.store(true);
  if (s->th.joinable()) s->th.join();
  free_lanes(s);
  for (Item* it : s->done) delete it;
  delete s;
  return TSA_OK;
}

}  // extern "C"
