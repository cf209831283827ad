// The serving scheduler (paper_1211_4896_amd/csrc/tsa_sched.hpp) on the CPU,
// driving a fake executor whose region batches and full-cube scans take
// controllable times and whose launches can be made to fail.  Checks FIFO
// order per class, batching by cube, admission by slots and by scratch
// budget, shared full-cube scans, drain timeouts, launch failures, replay,
// and many submitting threads (built under ThreadSanitizer by the test that
// runs this program as well).  Prints "all ok" and exits 0 when every check
// holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <thread>
#include <vector>

#include "../../paper_1211_4896_amd/csrc/tsa_sched.hpp"

using tsa::sched::Executor;
using tsa::sched::Job;
using tsa::sched::now_s;
using tsa::sched::Scheduler;

static int g_fail = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                      \
    }                                                                \
  } while (0)

// Region results: count = 2 * tag; full-cube results: count = 3 * tag.
class FakeExecutor final : public Executor {
 public:
  FakeExecutor(int lanes, int ncubes, size_t region_cost, size_t full_cost)
      : lanes_(lanes), ncubes_(ncubes), region_cost_(region_cost), full_cost_(full_cost), lane_(lanes) {}

  int lanes() const override { return lanes_; }
  int32_t cubes() const override { return ncubes_; }
  size_t region_cost() const override { return region_cost_; }
  size_t full_cost(int32_t) const override { return full_cost_; }

  int start_region(int lane, int32_t cube, Job* const* jobs, int n) override {
    std::lock_guard<std::mutex> g(mu);
    if (fail_region_launches > 0) {
      --fail_region_launches;
      return TSA_EDEVICE;
    }
    std::vector<uint64_t> tags;
    for (int i = 0; i < n; ++i) {
      if (jobs[i]->req.cube != cube || jobs[i]->req.kind != TSA_REQ_REGION) mixed = true;
      tags.push_back(jobs[i]->req.tag);
    }
    region_batches.push_back(tags);
    lane_[lane].jobs.assign(jobs, jobs + n);
    lane_[lane].end = now_s() + region_s;
    inflight += n;
    if (inflight > max_inflight) max_inflight = inflight;
    return TSA_OK;
  }

  bool region_finished(int lane) override {
    std::lock_guard<std::mutex> g(mu);
    Lane& L = lane_[lane];
    if (now_s() < L.end) return false;
    for (Job* j : L.jobs) {
      j->resp.result.count = 2 * j->req.tag;
      j->resp.result.status = TSA_OK;
      j->resp.status = TSA_OK;
    }
    inflight -= (int)L.jobs.size();
    L.jobs.clear();
    return true;
  }

  int start_full(int32_t cube, Job* const* jobs, int n) override {
    std::lock_guard<std::mutex> g(mu);
    std::vector<uint64_t> tags;
    for (int i = 0; i < n; ++i) {
      if (jobs[i]->req.cube != cube || jobs[i]->req.kind == TSA_REQ_REGION) mixed = true;
      tags.push_back(jobs[i]->req.tag);
    }
    full_scans.push_back(tags);
    full_.jobs.assign(jobs, jobs + n);
    full_.end = now_s() + full_s;
    inflight += n;
    if (inflight > max_inflight) max_inflight = inflight;
    return TSA_OK;
  }

  bool full_finished() override {
    std::lock_guard<std::mutex> g(mu);
    if (now_s() < full_.end) return false;
    for (Job* j : full_.jobs) {
      j->resp.result.count = 3 * j->req.tag;
      j->resp.status = TSA_OK;
    }
    inflight -= (int)full_.jobs.size();
    full_.jobs.clear();
    return true;
  }

  // set before the scheduler starts or read after it drained
  std::mutex mu;
  double region_s = 0.002, full_s = 0.005;
  int fail_region_launches = 0;
  std::vector<std::vector<uint64_t>> region_batches, full_scans;
  int inflight = 0, max_inflight = 0;
  bool mixed = false;

 private:
  struct Lane {
    std::vector<Job*> jobs;
    double end = 0;
  };
  const int lanes_;
  const int32_t ncubes_;
  const size_t region_cost_, full_cost_;
  std::vector<Lane> lane_;
  Lane full_;
};

static tsa_server_config config(int max_batch, int lanes, int max_admitted, size_t scratch) {
  tsa_server_config c;
  c.max_batch = max_batch;
  c.region_lanes = lanes;
  c.max_admitted = max_admitted;
  c.region_nbins = 16;
  c.full_nbins = 16;
  c.full_chunk_kvoxels = 0;
  c.scratch_bytes = scratch;
  return c;
}

static tsa_request region(int32_t cube, uint64_t tag) {
  tsa_request r;
  memset(&r, 0, sizeof(r));
  r.cube = cube;
  r.kind = TSA_REQ_REGION;
  r.region = tsa_region{0, 0, 0, 1, 1, 1};
  r.tag = tag;
  return r;
}

static tsa_request full(int32_t cube, int kind, uint64_t tag) {
  tsa_request r;
  memset(&r, 0, sizeof(r));
  r.cube = cube;
  r.kind = kind;
  r.tag = tag;
  return r;
}

static std::vector<tsa_response> poll_all(Scheduler& s, size_t n) {
  std::vector<tsa_response> out(n + 8);
  const int got = s.poll(out.data(), (int32_t)out.size());
  out.resize(got < 0 ? 0 : (size_t)got);
  return out;
}

static long stat_of(Scheduler& s, const char* key) {
  char buf[1024];
  if (s.stats(buf, sizeof(buf)) < 0) return -1;
  const char* p = strstr(buf, key);
  if (!p) return -1;
  p = strchr(p, ':');
  return p ? atol(p + 1) : -1;
}

// Region requests of one cube go out in submission order, at most max_batch
// per launch; responses carry their own results.
static void test_fifo_and_batches() {
  FakeExecutor ex(1, 1, 100, 1000);
  ex.region_s = 0.003;
  Scheduler s(config(4, 1, 1000, 0), &ex);
  s.start();
  for (uint64_t i = 0; i < 10; ++i) {
    tsa_request r = region(0, i);
    CHECK(s.submit(&r, -1) == TSA_OK);
  }
  CHECK(s.drain(5.0) == TSA_OK);
  const auto resp = poll_all(s, 10);
  CHECK(resp.size() == 10);
  for (const auto& r : resp) {
    CHECK(r.status == TSA_OK);
    CHECK(r.result.count == 2 * r.tag);
    CHECK(r.t_submit <= r.t_admit && r.t_admit <= r.t_launch && r.t_launch <= r.t_done);
  }
  std::vector<uint64_t> order;
  for (const auto& b : ex.region_batches) {
    CHECK(b.size() >= 1 && b.size() <= 4);
    order.insert(order.end(), b.begin(), b.end());
  }
  CHECK(order.size() == 10);
  for (size_t i = 0; i < order.size(); ++i) CHECK(order[i] == i);
  CHECK(ex.region_batches.size() >= 3);  // 10 requests, 4 a batch
  s.stop();
}

// A batch holds one cube: the cube of the oldest admitted request; the
// others keep their order for later batches.
static void test_batches_by_cube() {
  FakeExecutor ex(1, 2, 100, 1000);
  ex.region_s = 0.02;
  Scheduler s(config(64, 1, 1000, 0), &ex);
  s.start();
  tsa_request r0 = region(1, 100);
  CHECK(s.submit(&r0, -1) == TSA_OK);  // occupies the lane
  std::this_thread::sleep_for(std::chrono::milliseconds(5));
  for (uint64_t i = 0; i < 12; ++i) {
    tsa_request r = region((int32_t)(i % 2), i);
    CHECK(s.submit(&r, -1) == TSA_OK);
  }
  CHECK(s.drain(5.0) == TSA_OK);
  CHECK(!ex.mixed);
  CHECK(ex.region_batches.size() == 3);
  if (ex.region_batches.size() == 3) {
    CHECK(ex.region_batches[0] == std::vector<uint64_t>({100}));
    CHECK(ex.region_batches[1] == std::vector<uint64_t>({0, 2, 4, 6, 8, 10}));  // cube 0: oldest waiting
    CHECK(ex.region_batches[2] == std::vector<uint64_t>({1, 3, 5, 7, 9, 11}));
  }
  CHECK(poll_all(s, 13).size() == 13);
  s.stop();
}

// No more than max_admitted requests hold scratch at once.
static void test_slot_admission() {
  FakeExecutor ex(4, 1, 100, 1000);
  ex.region_s = 0.004;
  Scheduler s(config(1, 4, 3, 0), &ex);
  s.start();
  for (uint64_t i = 0; i < 12; ++i) {
    tsa_request r = region(0, i);
    CHECK(s.submit(&r, -1) == TSA_OK);
  }
  CHECK(s.drain(5.0) == TSA_OK);
  CHECK(ex.max_inflight <= 3);
  CHECK(ex.max_inflight == 3);
  CHECK(stat_of(s, "\"admitted_peak\"") == 3);
  CHECK(stat_of(s, "\"admission_waits\"") > 0);
  CHECK(poll_all(s, 12).size() == 12);
  s.stop();
}

// The scratch budget limits what is admitted; a request costing more than the
// whole budget is refused at submission; the budget is returned as requests
// finish.
static void test_budget_admission() {
  FakeExecutor ex(4, 1, 100, 1000);
  ex.region_s = 0.004;
  Scheduler s(config(1, 4, 1000, 250), &ex);  // room for two region requests
  s.start();
  for (uint64_t i = 0; i < 10; ++i) {
    tsa_request r = region(0, i);
    CHECK(s.submit(&r, -1) == TSA_OK);
  }
  tsa_request big = full(0, TSA_REQ_FULL_MEDIAN, 99);
  CHECK(s.submit(&big, -1) == TSA_ENOMEM);
  CHECK(s.drain(5.0) == TSA_OK);
  CHECK(ex.max_inflight == 2);
  CHECK(stat_of(s, "\"budget_peak\"") == 200);
  CHECK(stat_of(s, "\"submitted\"") == 10);
  CHECK(poll_all(s, 10).size() == 10);
  s.stop();
}

// Full-cube requests admitted while a scan runs are answered together by the
// next scan of the oldest one's cube; every request exactly once.
static void test_shared_full_scans() {
  FakeExecutor ex(1, 2, 100, 1000);
  ex.full_s = 0.02;
  Scheduler s(config(8, 1, 1000, 0), &ex);
  s.start();
  tsa_request first = full(0, TSA_REQ_FULL_HIST, 0);
  CHECK(s.submit(&first, -1) == TSA_OK);
  std::this_thread::sleep_for(std::chrono::milliseconds(5));
  const int32_t cubes[] = {1, 0, 1, 0, 0};
  for (uint64_t i = 0; i < 5; ++i) {
    tsa_request r = full(cubes[i], i % 2 ? TSA_REQ_FULL_MEDIAN : TSA_REQ_FULL_HIST, i + 1);
    CHECK(s.submit(&r, -1) == TSA_OK);
  }
  CHECK(s.drain(5.0) == TSA_OK);
  CHECK(!ex.mixed);
  CHECK(ex.full_scans.size() == 3);
  if (ex.full_scans.size() == 3) {
    CHECK(ex.full_scans[0] == std::vector<uint64_t>({0}));
    CHECK(ex.full_scans[1] == std::vector<uint64_t>({1, 3}));     // cube 1, oldest waiting
    CHECK(ex.full_scans[2] == std::vector<uint64_t>({2, 4, 5}));  // cube 0
  }
  const auto resp = poll_all(s, 6);
  CHECK(resp.size() == 6);
  std::set<uint64_t> seen;
  for (const auto& r : resp) {
    CHECK(r.result.count == 3 * r.tag);
    seen.insert(r.tag);
  }
  CHECK(seen.size() == 6);
  CHECK(stat_of(s, "\"full_scans\"") == 3);
  s.stop();
}

// drain() with a timeout gives up while work is in flight and returns TSA_OK
// once it is done.
static void test_drain_timeout() {
  FakeExecutor ex(1, 1, 100, 1000);
  ex.region_s = 0.15;
  Scheduler s(config(8, 1, 1000, 0), &ex);
  s.start();
  tsa_request r = region(0, 7);
  CHECK(s.submit(&r, -1) == TSA_OK);
  const double t0 = now_s();
  CHECK(s.drain(0.02) == TSA_EBUSY);
  CHECK(now_s() - t0 < 0.14);
  CHECK(s.drain(0.0) == TSA_OK);
  const auto resp = poll_all(s, 1);
  CHECK(resp.size() == 1 && resp[0].result.count == 14);
  s.stop();
}

// A launch that fails reports its error in every request of that batch and
// returns their scratch; later batches run.
static void test_launch_failure() {
  FakeExecutor ex(1, 1, 100, 1000);
  ex.fail_region_launches = 1;
  Scheduler s(config(4, 1, 2, 0), &ex);
  s.start();
  for (uint64_t i = 0; i < 6; ++i) {
    tsa_request r = region(0, i);
    CHECK(s.submit(&r, -1) == TSA_OK);
  }
  CHECK(s.drain(5.0) == TSA_OK);
  const auto resp = poll_all(s, 6);
  CHECK(resp.size() == 6);
  int failed = 0;
  for (const auto& r : resp) {
    if (r.status == TSA_EDEVICE)
      ++failed;
    else
      CHECK(r.status == TSA_OK && r.result.count == 2 * r.tag);
  }
  CHECK(failed >= 1 && failed <= 2);  // the first batch: what was admitted (2 slots)
  s.stop();
}

static void test_bad_requests() {
  FakeExecutor ex(1, 2, 100, 1000);
  Scheduler s(config(4, 1, 10, 0), &ex);
  s.start();
  tsa_request r = region(2, 0);  // no cube 2
  CHECK(s.submit(&r, -1) == TSA_EINVAL);
  r = region(-1, 0);
  CHECK(s.submit(&r, -1) == TSA_EINVAL);
  r = region(0, 0);
  r.kind = 7;
  CHECK(s.submit(&r, -1) == TSA_EINVAL);
  CHECK(s.submit(nullptr, -1) == TSA_EINVAL);
  CHECK(s.drain(1.0) == TSA_OK);
  s.stop();
}

// Open-loop replay: every response lands in its request's slot.
static void test_replay() {
  FakeExecutor ex(2, 2, 100, 1000);
  ex.region_s = 0.001;
  ex.full_s = 0.003;
  Scheduler s(config(16, 2, 64, 0), &ex);
  s.start();
  const int n = 200;
  std::vector<tsa_request> reqs;
  std::vector<double> t;
  for (int i = 0; i < n; ++i) {
    reqs.push_back(i % 10 == 3 ? full(i % 2, TSA_REQ_FULL_MEDIAN, (uint64_t)i) : region(i % 2, (uint64_t)i));
    t.push_back(i * 0.0002);
  }
  std::vector<tsa_response> out((size_t)n);
  CHECK(s.replay(reqs.data(), t.data(), n, out.data()) == TSA_OK);
  for (int i = 0; i < n; ++i) {
    CHECK(out[i].tag == (uint64_t)i);
    CHECK(out[i].status == TSA_OK);
    CHECK(out[i].result.count == (i % 10 == 3 ? 3u : 2u) * (uint64_t)i);
  }
  CHECK(poll_all(s, 1).empty());  // replayed responses are not polled
  s.stop();
}

// Many submitting and polling threads at once.
static void test_many_threads() {
  FakeExecutor ex(3, 3, 100, 1000);
  ex.region_s = 0.0005;
  ex.full_s = 0.002;
  Scheduler s(config(32, 3, 128, 40000), &ex);
  s.start();
  const int T = 4, per = 400;
  std::vector<std::thread> th;
  for (int k = 0; k < T; ++k)
    th.emplace_back([&s, k] {
      for (int i = 0; i < per; ++i) {
        const uint64_t tag = (uint64_t)(k * per + i);
        tsa_request r = (i % 17 == 5) ? full(i % 3, TSA_REQ_FULL_HIST, tag) : region(i % 3, tag);
        while (s.submit(&r, -1) == TSA_EBUSY) std::this_thread::yield();
      }
    });
  std::vector<tsa_response> got;
  std::thread poller([&s, &got] {
    std::vector<tsa_response> buf(64);
    while (got.size() < (size_t)(T * per)) {
      const int n = s.poll(buf.data(), (int32_t)buf.size());
      for (int i = 0; i < n; ++i) got.push_back(buf[i]);
      if (n == 0) std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
  });
  for (auto& t : th) t.join();
  CHECK(s.drain(20.0) == TSA_OK);
  poller.join();
  CHECK(got.size() == (size_t)(T * per));
  std::set<uint64_t> tags;
  for (const auto& r : got) {
    tags.insert(r.tag);
    const bool is_full = ((r.tag % per) % 17) == 5;
    CHECK(r.result.count == (is_full ? 3u : 2u) * r.tag);
  }
  CHECK(tags.size() == (size_t)(T * per));
  CHECK(!ex.mixed);
  CHECK(stat_of(s, "\"budget_peak\"") <= 40000);
  s.stop();
}

int main() {
  test_fifo_and_batches();
  test_batches_by_cube();
  test_slot_admission();
  test_budget_admission();
  test_shared_full_scans();
  test_drain_timeout();
  test_launch_failure();
  test_bad_requests();
  test_replay();
  test_many_threads();
  if (g_fail) {
    fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  printf("all ok\n");
  return 0;
}
