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
#include "tsa_sched.hpp"

namespace tsa {
size_t batch_ws_bytes(const tsa_cube* cube, int32_t nbins, int32_t nq);
int run_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                     tsa_result* d_results, uint64_t* d_hists, const tsa_tune* tune, void* d_ws, size_t ws_bytes,
                     tsa_stream_t stream);
}  // namespace tsa

using namespace tsa;

namespace {

using sched::Job;

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
  // results then histograms in one allocation (and its pinned mirror), so one
  // copy brings a batch's answers back
  void* d_out = nullptr;
  void* h_out = nullptr;
  size_t hist_off = 0;  // bytes from the start to the histograms
  tsa_result* d_results = nullptr;
  uint64_t* d_hists = nullptr;
  tsa_region* h_regions = nullptr;
  tsa_result* h_results = nullptr;
  uint64_t* h_hists = nullptr;
  std::vector<Job*> jobs;
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
  std::vector<Job*> jobs;  // every request the current shared scan answers
  int32_t cube = 0;
  bool has_hist = false;
};

// The scheduler's executor on one GPU: region batches on their own streams,
// full-cube scans on another; completion found by polling events.
class GpuExecutor final : public sched::Executor {
 public:
  explicit GpuExecutor(const tsa_server_config& cfg) : cfg_(cfg) {}
  ~GpuExecutor() override { free_all(); }

  int init() {
    DevInfo dev;
    int st = device_info(&dev);
    if (st) return st;
    // a valid cube descriptor for the layout query (the batch layout depends on nq only)
    tsa_cube probe = {(const void*)256, TSA_F32, 0, 4, 1, 1};
    const size_t bws = batch_ws_bytes(&probe, cfg_.region_nbins, cfg_.max_batch);
    if (!bws) return TSA_EINVAL;
    region_cost_ = bws / (size_t)cfg_.max_batch + sizeof(tsa_result) + sizeof(tsa_region) +
                   sizeof(uint64_t) * (size_t)cfg_.region_nbins;
    rl_.resize(cfg_.region_lanes);
    bool ok = true;
    for (RegionLane& L : rl_) {
      const size_t nq = (size_t)cfg_.max_batch, nb = (size_t)cfg_.region_nbins;
      ok = ok && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
      ok = ok && hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) == hipSuccess;
      ok = ok && hipMalloc(&L.d_ws, bws) == hipSuccess;
      L.ws_bytes = bws;
      L.hist_off = (sizeof(tsa_result) * nq + 255) & ~(size_t)255;
      const size_t out_bytes = L.hist_off + sizeof(uint64_t) * nq * nb;
      ok = ok && hipMalloc((void**)&L.d_regions, sizeof(tsa_region) * nq) == hipSuccess;
      ok = ok && hipMalloc(&L.d_out, out_bytes) == hipSuccess;
      ok = ok && hipHostMalloc((void**)&L.h_regions, sizeof(tsa_region) * nq, hipHostMallocDefault) == hipSuccess;
      ok = ok && hipHostMalloc(&L.h_out, out_bytes, hipHostMallocDefault) == hipSuccess;
      if (ok) {
        L.d_results = (tsa_result*)L.d_out;
        L.d_hists = (uint64_t*)((char*)L.d_out + L.hist_off);
        L.h_results = (tsa_result*)L.h_out;
        L.h_hists = (uint64_t*)((char*)L.h_out + L.hist_off);
      }
    }
    FullLane& F = fl_;
    ok = ok && hipStreamCreateWithFlags(&F.stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&F.ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc((void**)&F.d_result, sizeof(tsa_result)) == hipSuccess;
    ok = ok && hipMalloc((void**)&F.d_counts, sizeof(uint64_t) * cfg_.full_nbins) == hipSuccess;
    ok = ok && hipMalloc((void**)&F.d_outl, 2 * sizeof(uint64_t)) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&F.h_result, sizeof(tsa_result), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&F.h_counts, sizeof(uint64_t) * cfg_.full_nbins, hipHostMallocDefault) ==
                   hipSuccess;
    return ok ? TSA_OK : TSA_EDEVICE;
  }

  // Registers a resident cube and finds its min/max now, as the data loads.
  // The caller makes sure no request is in flight.
  int add_cube(const tsa_cube* cube, int32_t* id) {
    const size_t ws = tsa_workspace_bytes(TSA_OP_MOMENTS, cube, nullptr, 0, 0);
    const size_t full_ws = tsa_workspace_bytes(TSA_OP_MEDIAN, cube, nullptr, 0, 0);
    const size_t hws = tsa_workspace_bytes(TSA_OP_HISTOGRAM, cube, nullptr, cfg_.full_nbins, 0);
    size_t need = ws > full_ws ? ws : full_ws;
    if (hws > need) need = hws;
    FullLane& F = fl_;
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
    int st = run_moments(cube, nullptr, F.d_result, F.d_ws, F.ws_bytes, (tsa_stream_t)F.stream);
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
    std::lock_guard<std::mutex> g(cubes_mu_);
    cubes_.push_back(c);
    *id = (int32_t)cubes_.size() - 1;
    return TSA_OK;
  }

  int lanes() const override { return cfg_.region_lanes; }
  int32_t cubes() const override {
    std::lock_guard<std::mutex> g(cubes_mu_);
    return (int32_t)cubes_.size();
  }
  size_t region_cost() const override { return region_cost_; }
  size_t full_cost(int32_t cube) const override {
    std::lock_guard<std::mutex> g(cubes_mu_);
    return cubes_[cube].full_ws + sizeof(uint64_t) * (size_t)cfg_.full_nbins;
  }

  int start_region(int lane, int32_t cube, Job* const* jobs, int nq) override {
    RegionLane& L = rl_[lane];
    // pad to a power of two with empty boxes (rejected at once by the planner),
    // so each lane replays a handful of captured launch graphs
    int nq_pad = 1;
    while (nq_pad < nq) nq_pad <<= 1;
    if (nq_pad > cfg_.max_batch) nq_pad = cfg_.max_batch;
    for (int i = 0; i < nq; ++i) L.h_regions[i] = jobs[i]->req.region;
    for (int i = nq; i < nq_pad; ++i) L.h_regions[i] = tsa_region{0, 0, 0, 0, 0, 0};
    const CubeRec c = cube_rec(cube);
    int st = hipMemcpyAsync(L.d_regions, L.h_regions, sizeof(tsa_region) * nq_pad, hipMemcpyHostToDevice,
                            L.stream) == hipSuccess
                 ? TSA_OK
                 : TSA_EDEVICE;
    if (st == TSA_OK)
      st = run_region_batch(&c.cube, L.d_regions, nq_pad, cfg_.region_nbins, L.d_results, L.d_hists, nullptr,
                            L.d_ws, L.ws_bytes, (tsa_stream_t)L.stream);
    // one copy: the results (and the unused slots past nq) and the nq histograms
    if (st == TSA_OK &&
        (hipMemcpyAsync(L.h_out, L.d_out, L.hist_off + sizeof(uint64_t) * (size_t)nq * cfg_.region_nbins,
                        hipMemcpyDeviceToHost, L.stream) != hipSuccess ||
         hipEventRecord(L.ev, L.stream) != hipSuccess))
      st = TSA_EDEVICE;
    if (st == TSA_OK) L.jobs.assign(jobs, jobs + nq);
    return st;
  }

  bool region_finished(int lane) override {
    RegionLane& L = rl_[lane];
    if (hipEventQuery(L.ev) != hipSuccess) return false;
    const int nb = cfg_.region_nbins;
    for (size_t i = 0; i < L.jobs.size(); ++i) {
      Job* j = L.jobs[i];
      j->resp.result = L.h_results[i];
      j->resp.status = L.h_results[i].status;
      if (j->req.h_hist) memcpy(j->req.h_hist, L.h_hists + i * (size_t)nb, sizeof(uint64_t) * nb);
    }
    L.jobs.clear();
    return true;
  }

  // One scan answers every job: histogram requests share one pass, median
  // requests the radix passes, both kinds together the fused two-pass trio.
  int start_full(int32_t cube, Job* const* jobs, int n) override {
    FullLane& F = fl_;
    bool any_hist = false, any_median = false;
    for (int i = 0; i < n; ++i) {
      any_hist |= jobs[i]->req.kind == TSA_REQ_FULL_HIST;
      any_median |= jobs[i]->req.kind == TSA_REQ_FULL_MEDIAN;
    }
    const CubeRec c = cube_rec(cube);
    const tsa_stream_t fs = (tsa_stream_t)F.stream;
    int st = TSA_OK;
    if (any_hist && !c.range_ok) st = TSA_EINVAL;
    const size_t fused_lds = ((size_t)cfg_.full_nbins + 64 + 4096) * 4;
    const int64_t chunk = (int64_t)cfg_.full_chunk_kvoxels << 10;
    const int64_t volume = c.cube.nx * c.cube.ny * c.cube.nz;
    if (chunk > 0 && chunk < volume) {  // each pass in z-slab launches of at most `chunk` voxels
      if (st == TSA_OK && any_hist)
        st = run_histogram_chunked(&c.cube, c.lo, c.hi, cfg_.full_nbins, F.d_counts, F.d_outl, F.d_ws, F.ws_bytes,
                                   fs, chunk);
      if (st == TSA_OK && any_median) st = run_median_chunked(&c.cube, F.d_result, F.d_ws, F.ws_bytes, fs, chunk);
    } else if (st == TSA_OK && any_hist && any_median && fused_lds <= 65536) {
      st = run_stats(&c.cube, nullptr, cfg_.full_nbins, F.d_result, F.d_counts, F.d_outl, F.d_ws, F.ws_bytes, fs);
    } else {
      if (st == TSA_OK && any_hist)
        st = run_histogram(&c.cube, nullptr, c.lo, c.hi, cfg_.full_nbins, F.d_counts, F.d_outl, F.d_ws,
                           F.ws_bytes, fs);
      if (st == TSA_OK && any_median)
        st = run_median(&c.cube, nullptr, F.d_result, F.d_ws, F.ws_bytes, fs);
    }
    if (st == TSA_OK && !any_median) *F.h_result = sched::nan_result();  // only histograms: no device result
    if (st == TSA_OK && any_median &&
        hipMemcpyAsync(F.h_result, F.d_result, sizeof(tsa_result), hipMemcpyDeviceToHost, F.stream) !=
            hipSuccess)
      st = TSA_EDEVICE;
    if (st == TSA_OK && any_hist &&
        hipMemcpyAsync(F.h_counts, F.d_counts, sizeof(uint64_t) * cfg_.full_nbins, hipMemcpyDeviceToHost,
                       F.stream) != hipSuccess)
      st = TSA_EDEVICE;
    if (st == TSA_OK && hipEventRecord(F.ev, F.stream) != hipSuccess) st = TSA_EDEVICE;
    if (st == TSA_OK) {
      F.jobs.assign(jobs, jobs + n);
      F.cube = cube;
      F.has_hist = any_hist;
    }
    return st;
  }

  bool full_finished() override {
    FullLane& F = fl_;
    if (hipEventQuery(F.ev) != hipSuccess) return false;
    uint64_t tot = 0;
    if (F.has_hist)
      for (int b = 0; b < cfg_.full_nbins; ++b) tot += F.h_counts[b];
    const CubeRec c = cube_rec(F.cube);
    for (Job* j : F.jobs) {
      tsa_result r = sched::nan_result();
      r.status = F.h_result->status;
      if (j->req.kind == TSA_REQ_FULL_MEDIAN) {
        r.count = F.h_result->count;
        r.nan_count = F.h_result->nan_count;
        r.median = F.h_result->median;
      } else {
        r.count = tot;
        r.min = c.lo;
        r.max = c.hi;
        if (j->req.h_hist) memcpy(j->req.h_hist, F.h_counts, sizeof(uint64_t) * cfg_.full_nbins);
      }
      j->resp.result = r;
      j->resp.status = r.status;
    }
    F.jobs.clear();
    return true;
  }

 private:
  CubeRec cube_rec(int32_t cube) const {
    std::lock_guard<std::mutex> g(cubes_mu_);
    return cubes_[cube];
  }

  void free_all() {
    for (RegionLane& L : rl_) {
      if (L.stream) (void)hipStreamDestroy(L.stream);
      if (L.ev) (void)hipEventDestroy(L.ev);
      (void)hipFree(L.d_ws);
      (void)hipFree(L.d_regions);
      (void)hipFree(L.d_out);
      (void)hipHostFree(L.h_regions);
      (void)hipHostFree(L.h_out);
    }
    FullLane& F = fl_;
    if (F.stream) (void)hipStreamDestroy(F.stream);
    if (F.ev) (void)hipEventDestroy(F.ev);
    (void)hipFree(F.d_ws);
    (void)hipFree(F.d_result);
    (void)hipFree(F.d_counts);
    (void)hipFree(F.d_outl);
    (void)hipHostFree(F.h_result);
    (void)hipHostFree(F.h_counts);
  }

  const tsa_server_config cfg_;
  size_t region_cost_ = 0;
  std::vector<RegionLane> rl_;
  FullLane fl_;
  mutable std::mutex cubes_mu_;
  std::vector<CubeRec> cubes_;  // guarded by cubes_mu_
};

}  // namespace

// The server handle: the GPU executor and the scheduler driving it.
struct tsa_server {
  tsa_server_config cfg;
  int device = 0;
  GpuExecutor ex;
  sched::Scheduler sch;
  explicit tsa_server(const tsa_server_config& c) : cfg(c), ex(c), sch(c, &ex) {}
};

extern "C" {

double tsa_server_now(void) { return sched::now_s(); }

int tsa_server_create(const tsa_server_config* cfg, tsa_server** out) {
  if (!cfg || !out) return TSA_EINVAL;
  if (cfg->max_batch < 1 || cfg->max_batch > 4096 || cfg->region_lanes < 1 || cfg->region_lanes > 4 ||
      cfg->max_admitted < 1 || cfg->region_nbins < 1 || cfg->region_nbins > 4096 || cfg->full_nbins < 1 ||
      cfg->full_nbins > 65536 || cfg->full_chunk_kvoxels < 0)
    return TSA_EINVAL;
  tsa_server* s = new tsa_server(*cfg);
  (void)hipGetDevice(&s->device);
  const int st = s->ex.init();
  if (st) {
    delete s;
    return st;
  }
  const int device = s->device;
  s->sch.start([device] { (void)hipSetDevice(device); });
  *out = s;
  return TSA_OK;
}

int tsa_server_add_cube(tsa_server* s, const tsa_cube* cube, int32_t* id) {
  if (!s || !cube || !id) return TSA_EINVAL;
  int st = check_cube(cube);
  if (st) return st;
  std::lock_guard<std::mutex> g(s->sch.lock());
  if (!s->sch.idle_locked()) return TSA_EBUSY;  // add cubes while idle
  return s->ex.add_cube(cube, id);
}

int tsa_server_submit(tsa_server* s, const tsa_request* r) {
  if (!s || !r) return TSA_EINVAL;
  return s->sch.submit(r, -1);
}

int tsa_server_poll(tsa_server* s, tsa_response* out, int32_t cap) {
  if (!s || (!out && cap > 0)) return TSA_EINVAL;
  return s->sch.poll(out, cap);
}

int tsa_server_drain(tsa_server* s, double timeout_s) {
  if (!s) return TSA_EINVAL;
  return s->sch.drain(timeout_s);
}

int tsa_server_replay(tsa_server* s, const tsa_request* reqs, const double* t_arrival, int32_t n,
                      tsa_response* out) {
  if (!s || n < 0 || (n > 0 && (!reqs || !t_arrival || !out))) return TSA_EINVAL;
  return s->sch.replay(reqs, t_arrival, n, out);
}

int tsa_server_stats(tsa_server* s, char* buf, size_t len) {
  if (!s || !buf) return TSA_EINVAL;
  return s->sch.stats(buf, len);
}

int tsa_server_destroy(tsa_server* s) {
  if (!s) return TSA_EINVAL;
  s->sch.stop();
  delete s;
  return TSA_OK;
}

}  // extern "C"
