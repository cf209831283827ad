// The serving scheduler (include/tsa_serve.h), independent of the device:
// admission by slots and a scratch budget, FIFO per request class, continuous
// batching of region requests into lanes, one shared full-cube scan at a
// time, retirement by polling.  It drives an Executor -- the HIP one in
// tsa_serve.hip, or a CPU fake with controllable delays in the tests -- from
// one thread of its own.  Plain C++17 (no HIP), so the tests build it with a
// host compiler, also under ThreadSanitizer.
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/tsa_serve.h"

namespace tsa {
namespace sched {

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

inline tsa_result nan_result() {
  tsa_result r;
  r.count = r.nan_count = 0;
  r.mean = r.m2 = r.std = r.min = r.max = r.median = __builtin_nan("");
  r.status = TSA_OK;
  r.flags = 0;
  return r;
}

// One request on its way through the scheduler.
struct Job {
  tsa_request req;
  tsa_response resp;
  int64_t replay_index;  // >= 0: the response goes to the replay output array
  size_t cost;           // scratch held while admitted
};

// What the scheduler drives.  Calls come from the scheduler thread only,
// except cubes() and the cost queries, which submit() also makes.
class Executor {
 public:
  virtual ~Executor() = default;
  virtual int lanes() const = 0;                       // region batches in flight at once
  virtual int32_t cubes() const = 0;                   // registered cubes (ids 0 .. cubes()-1)
  virtual size_t region_cost() const = 0;              // scratch of one region request
  virtual size_t full_cost(int32_t cube) const = 0;    // scratch of one full-cube request
  // Starts the batch jobs[0..n) (every job on `cube`) on `lane`; TSA_OK or an
  // error, in which case nothing runs.
  virtual int start_region(int lane, int32_t cube, Job* const* jobs, int n) = 0;
  // True once the lane's batch has finished; each job's result, status and
  // histogram are then filled in.
  virtual bool region_finished(int lane) = 0;
  // Starts one scan of `cube` answering every full-cube job in jobs[0..n).
  virtual int start_full(int32_t cube, Job* const* jobs, int n) = 0;
  // True once the scan has finished, its jobs filled in.
  virtual bool full_finished() = 0;
};

class Scheduler {
 public:
  Scheduler(const tsa_server_config& cfg, Executor* ex) : cfg_(cfg), ex_(ex), lanes_(ex->lanes()) {}
  ~Scheduler() { stop(); }

  // Starts the scheduler thread; on_start runs first on it (e.g. to select
  // the device the executor works on).
  void start(std::function<void()> on_start = {}) {
    th_ = std::thread([this, on_start] {
      if (on_start) on_start();
      loop();
    });
  }

  // Finishes every queued and in-flight job, then ends the thread.
  void stop() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_.store(true);
    }
    arrive_cv_.notify_all();
    if (th_.joinable()) th_.join();
    std::lock_guard<std::mutex> g(mu_);
    for (Job* j : done_) delete j;
    done_.clear();
  }

  // Queues a request (any thread).  TSA_EINVAL: bad kind or cube id;
  // TSA_ENOMEM: it costs more than the whole scratch budget (it could never
  // be admitted and would hold up its class); TSA_EBUSY: 2^20 waiting.
  int submit(const tsa_request* r, int64_t replay_index) {
    if (!r || r->kind < TSA_REQ_REGION || r->kind > TSA_REQ_FULL_MEDIAN) return TSA_EINVAL;
    if (r->cube < 0 || r->cube >= ex_->cubes()) return TSA_EINVAL;
    const size_t cost = r->kind == TSA_REQ_REGION ? ex_->region_cost() : ex_->full_cost(r->cube);
    if (cfg_.scratch_bytes && cost > cfg_.scratch_bytes) return TSA_ENOMEM;
    Job* j = new Job();
    j->req = *r;
    j->replay_index = replay_index;
    j->cost = cost;
    j->resp.tag = r->tag;
    j->resp.kind = r->kind;
    j->resp.status = TSA_OK;
    j->resp.result = nan_result();
    j->resp.t_submit = now_s();
    j->resp.t_admit = j->resp.t_launch = j->resp.t_done = 0.0;
    std::lock_guard<std::mutex> g(mu_);
    if (arrivals_.size() >= (1u << 20)) {
      delete j;
      return TSA_EBUSY;
    }
    arrivals_.push_back(j);
    submitted_++;
    arrive_cv_.notify_one();  // wakes a scheduler waiting with nothing in flight
    return TSA_OK;
  }

  int poll(tsa_response* out, int32_t cap) {
    std::lock_guard<std::mutex> g(mu_);
    int n = 0;
    while (n < cap && !done_.empty()) {
      Job* j = done_.front();
      done_.pop_front();
      out[n++] = j->resp;
      delete j;
    }
    return n;
  }

  // Waits until every submitted request has finished (timeout_s <= 0: no limit).
  int drain(double timeout_s) {
    std::unique_lock<std::mutex> g(mu_);
    auto all = [this] { return finished_ == submitted_; };
    if (timeout_s <= 0) {
      cv_.wait(g, all);
      return TSA_OK;
    }
    return cv_.wait_for(g, std::chrono::duration<double>(timeout_s), all) ? TSA_OK : TSA_EBUSY;
  }

  // True while nothing is queued or in flight (the caller holds lock()).
  bool idle_locked() const { return finished_ == submitted_; }
  std::mutex& lock() { return mu_; }

  int replay(const tsa_request* reqs, const double* t_arrival, int32_t n, tsa_response* out) {
    {
      std::unique_lock<std::mutex> g(mu_);
      cv_.wait(g, [this] { return finished_ == submitted_; });
      replay_out_ = out;
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
      const int st = submit(&reqs[i], i);
      if (st) {
        out[i].tag = reqs[i].tag;
        out[i].status = st;
        out[i].kind = reqs[i].kind;
      }
    }
    std::unique_lock<std::mutex> g(mu_);
    cv_.wait(g, [this] { return finished_ == submitted_; });
    replay_out_ = nullptr;
    return TSA_OK;
  }

  int stats(char* buf, size_t len) {
    char tmp[768];
    int n;
    {
      std::lock_guard<std::mutex> g(mu_);
      n = snprintf(tmp, sizeof(tmp),
                   "{\"batches\": %llu, \"batched_requests\": %llu, \"max_batch\": %llu, \"full_requests\": "
                   "%llu, \"full_scans\": %llu, \"admission_waits\": %llu, \"submitted\": %llu, "
                   "\"finished\": %llu, \"scratch_bytes\": %llu, \"budget_peak\": %llu, "
                   "\"region_cost\": %llu, \"admitted_peak\": %llu}",
                   (unsigned long long)n_batches_.load(), (unsigned long long)n_batch_items_.load(),
                   (unsigned long long)max_batch_seen_.load(), (unsigned long long)n_full_.load(),
                   (unsigned long long)n_scans_.load(), (unsigned long long)n_admit_waits_.load(),
                   (unsigned long long)submitted_, (unsigned long long)finished_,
                   (unsigned long long)cfg_.scratch_bytes, (unsigned long long)budget_peak_.load(),
                   (unsigned long long)ex_->region_cost(), (unsigned long long)admitted_peak_.load());
    }
    if (n < 0 || (size_t)n + 1 > len) return TSA_ENOMEM;
    memcpy(buf, tmp, (size_t)n + 1);
    return n;
  }

 private:
  struct Lane {
    std::vector<Job*> jobs;
    bool busy = false;
  };

  void finish(Job* j) {
    std::lock_guard<std::mutex> g(mu_);
    if (j->replay_index >= 0 && replay_out_) {
      replay_out_[j->replay_index] = j->resp;
      delete j;
    } else {
      done_.push_back(j);
    }
    finished_++;
    cv_.notify_all();
  }

  void release(Job* j) {
    budget_used_ -= j->cost;
    admitted_--;
  }

  void fail(Job* j, int st) {
    j->resp.result = nan_result();
    j->resp.result.status = st;
    j->resp.status = st;
    j->resp.t_done = now_s();
    release(j);
    finish(j);
  }

  // finished lanes and scans -> done
  bool retire() {
    bool did = false;
    for (int l = 0; l < lanes_; ++l) {
      Lane& L = rl_[l];
      if (!L.busy || !ex_->region_finished(l)) continue;
      const double t = now_s();
      for (Job* j : L.jobs) {
        j->resp.t_done = t;
        release(j);
        finish(j);
      }
      L.jobs.clear();
      L.busy = false;
      did = true;
    }
    if (full_.busy && ex_->full_finished()) {
      const double t = now_s();
      for (Job* j : full_.jobs) {
        j->resp.t_done = t;
        release(j);
        finish(j);
      }
      full_.jobs.clear();
      full_.busy = false;
      did = true;
    }
    return did;
  }

  // arrivals -> pending -> admitted (FIFO per class, while slots and scratch allow)
  bool admit() {
    bool did = false;
    {
      std::lock_guard<std::mutex> g(mu_);
      while (!arrivals_.empty()) {
        Job* j = arrivals_.front();
        arrivals_.pop_front();
        (j->req.kind == TSA_REQ_REGION ? pend_region_ : pend_full_).push_back(j);
        did = true;
      }
    }
    const size_t cap = cfg_.scratch_bytes;
    for (int round = 0; round < 2; ++round) {
      std::deque<Job*>& P = round == 0 ? pend_full_ : pend_region_;
      std::deque<Job*>& A = round == 0 ? adm_full_ : adm_region_;
      while (!P.empty()) {
        Job* j = P.front();
        if (admitted_ >= cfg_.max_admitted || (cap && budget_used_ + j->cost > cap)) {
          n_admit_waits_++;
          break;
        }
        P.pop_front();
        budget_used_ += j->cost;
        if (budget_used_ > budget_peak_.load()) budget_peak_.store(budget_used_);
        admitted_++;
        if ((uint64_t)admitted_ > admitted_peak_.load()) admitted_peak_.store((uint64_t)admitted_);
        j->resp.t_admit = now_s();
        A.push_back(j);
        did = true;
      }
    }
    return did;
  }

  // Takes from q every job on the cube of its oldest one (up to max), keeping
  // the others in their order.
  static void take_cube(std::deque<Job*>& q, size_t max, std::vector<Job*>& out) {
    const int32_t cube = q.front()->req.cube;
    std::deque<Job*> keep;
    while (!q.empty() && out.size() < max) {
      Job* j = q.front();
      q.pop_front();
      if (j->req.cube == cube)
        out.push_back(j);
      else
        keep.push_back(j);
    }
    while (!keep.empty()) {
      q.push_front(keep.back());
      keep.pop_back();
    }
  }

  bool launch() {
    bool did = false;
    for (int l = 0; l < lanes_; ++l) {
      Lane& L = rl_[l];
      if (L.busy || adm_region_.empty()) continue;
      take_cube(adm_region_, (size_t)cfg_.max_batch, L.jobs);
      const double t = now_s();
      for (Job* j : L.jobs) j->resp.t_launch = t;
      const int st = ex_->start_region(l, L.jobs.front()->req.cube, L.jobs.data(), (int)L.jobs.size());
      if (st != TSA_OK) {
        for (Job* j : L.jobs) fail(j, st);
        L.jobs.clear();
        continue;
      }
      L.busy = true;
      n_batches_++;
      n_batch_items_ += L.jobs.size();
      if (L.jobs.size() > max_batch_seen_.load()) max_batch_seen_.store(L.jobs.size());
      did = true;
    }
    if (!full_.busy && !adm_full_.empty()) {
      // one shared scan answers every admitted full-cube request on the cube
      // of the oldest one
      take_cube(adm_full_, (size_t)-1, full_.jobs);
      const double t = now_s();
      for (Job* j : full_.jobs) j->resp.t_launch = t;
      const int st = ex_->start_full(full_.jobs.front()->req.cube, full_.jobs.data(), (int)full_.jobs.size());
      if (st != TSA_OK) {
        for (Job* j : full_.jobs) fail(j, st);
        full_.jobs.clear();
      } else {
        full_.busy = true;
        n_full_ += full_.jobs.size();
        n_scans_++;
      }
      did = true;
    }
    return did;
  }

  void loop() {
    rl_.resize((size_t)lanes_);
    int idle = 0;
    for (;;) {
      bool did = retire();
      did |= admit();
      did |= launch();
      if (stop_.load()) {
        bool busy = full_.busy;
        for (const Lane& L : rl_) busy |= L.busy;
        std::lock_guard<std::mutex> g(mu_);
        if (!busy && arrivals_.empty() && pend_region_.empty() && pend_full_.empty() && adm_region_.empty() &&
            adm_full_.empty())
          break;
      }
      // Work in flight: poll its events without sleeping (a sleep here is added
      // to every request's latency).  Nothing in flight and nothing to start:
      // wait for an arrival (or stop), with a timeout as a safety net.
      if (did) {
        idle = 0;
        continue;
      }
      bool busy = full_.busy;
      for (const Lane& L : rl_) busy |= L.busy;
      if (busy || ++idle <= 64) {
        std::this_thread::yield();
      } else {
        std::unique_lock<std::mutex> g(mu_);
        arrive_cv_.wait_for(g, std::chrono::milliseconds(1), [this] { return !arrivals_.empty() || stop_.load(); });
      }
    }
  }

  const tsa_server_config cfg_;
  Executor* const ex_;
  const int lanes_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::condition_variable arrive_cv_;  // new arrivals and stop, for a scheduler with nothing in flight
  std::deque<Job*> arrivals_;            // guarded by mu_
  std::deque<Job*> done_;                // guarded by mu_
  uint64_t submitted_ = 0, finished_ = 0;  // guarded by mu_
  tsa_response* replay_out_ = nullptr;   // guarded by mu_
  // scheduler-thread state
  std::deque<Job*> pend_region_, pend_full_, adm_region_, adm_full_;
  std::vector<Lane> rl_;
  Lane full_;
  size_t budget_used_ = 0;
  int admitted_ = 0;
  std::atomic<bool> stop_{false};
  std::thread th_;
  // counters, read by stats() from other threads
  std::atomic<uint64_t> n_batches_{0}, n_batch_items_{0}, n_full_{0}, n_scans_{0}, max_batch_seen_{0},
      n_admit_waits_{0}, budget_peak_{0}, admitted_peak_{0};
};

}  // namespace sched
}  // namespace tsa
