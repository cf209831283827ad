// Optional per-kernel timing with HIP events on the launch stream, and a
// plain copy kernel used to calibrate hardware byte counters.
//
// When tracing is on, every library launch is bracketed by two events
// recorded on the stream it is launched on; tsa_trace_read() waits for the
// last one and reports, per kernel name, the number of launches and the
// total / min / max elapsed milliseconds.
#include <mutex>
#include <string>
#include <vector>

#include "tsa_internal.hpp"

namespace tsa {

namespace {
struct Rec {
  const char* name;
  hipEvent_t a, b;
};
struct TraceState {
  std::mutex mu;
  bool on = false;
  size_t cap = 0;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> recs;
  const char* cur = nullptr;
  hipEvent_t cur_a = nullptr;
};
TraceState& T() {
  static TraceState t;
  return t;
}
}  // namespace

bool trace_active() { return T().on; }

void trace_begin(const char* name, hipStream_t s) {
  TraceState& t = T();
  if (!t.on) return;
  std::lock_guard<std::mutex> g(t.mu);
  if (t.used + 2 > t.pool.size()) {
    t.cur = nullptr;
    return;
  }
  t.cur = name;
  t.cur_a = t.pool[t.used++];
  hipEventRecord(t.cur_a, s);
}

void trace_end(hipStream_t s) {
  TraceState& t = T();
  if (!t.on) return;
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.cur) return;
  hipEvent_t b = t.pool[t.used++];
  hipEventRecord(b, s);
  t.recs.push_back({t.cur, t.cur_a, b});
  t.cur = nullptr;
}

}  // namespace tsa

using namespace tsa;

extern "C" {

// Start (on != 0, room for `cap` launches) or stop tracing.  Clears records.
int tsa_trace_enable(int32_t on, int32_t cap) {
  TraceState& t = T();
  std::lock_guard<std::mutex> g(t.mu);
  t.recs.clear();
  t.used = 0;
  t.cur = nullptr;
  if (!on) {
    t.on = false;
    return TSA_OK;
  }
  if (cap < 1) cap = 1;
  const size_t want = 2 * (size_t)cap;
  while (t.pool.size() < want) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return TSA_EDEVICE;
    t.pool.push_back(e);
  }
  t.on = true;
  return TSA_OK;
}

// JSON object {"kernel": [launches, total_ms, min_ms, max_ms], ...}; waits
// for the recorded events.  Returns the length written, or a negative status.
int tsa_trace_read(char* buf, size_t len) {
  TraceState& t = T();
  std::lock_guard<std::mutex> g(t.mu);
  struct Agg {
    std::string name;
    int n = 0;
    double tot = 0, mn = 1e30, mx = 0;
  };
  std::vector<Agg> aggs;
  for (const Rec& r : t.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return TSA_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return TSA_EDEVICE;
    Agg* a = nullptr;
    for (Agg& x : aggs)
      if (x.name == r.name) a = &x;
    if (!a) {
      aggs.push_back(Agg{});
      a = &aggs.back();
      a->name = r.name;
    }
    a->n++;
    a->tot += ms;
    a->mn = ms < a->mn ? ms : a->mn;
    a->mx = ms > a->mx ? ms : a->mx;
  }
  std::string s = "{";
  char tmp[256];
  for (size_t i = 0; i < aggs.size(); ++i) {
    snprintf(tmp, sizeof(tmp), "%s\"%s\": [%d, %.6f, %.6f, %.6f]", i ? ", " : "", aggs[i].name.c_str(), aggs[i].n,
             aggs[i].tot, aggs[i].mn, aggs[i].mx);
    s += tmp;
  }
  s += "}";
  if (!buf || len < s.size() + 1) return TSA_ENOMEM;
  memcpy(buf, s.c_str(), s.size() + 1);
  return (int)s.size();
}

}  // extern "C"

namespace tsa {
// Read-only bandwidth probe: the statistics passes' load pattern with the
// least possible work per element.
__global__ __launch_bounds__(512) void k_read_probe(const uint4* __restrict__ src, uint64_t n,
                                                    uint32_t* __restrict__ sink) {
  __shared__ uint32_t red[8];
  constexpr int U = 4;
  const uint64_t chunk = (uint64_t)blockDim.x * U, stride = chunk * gridDim.x;
  uint32_t acc = 0;
  for (uint64_t cb = (uint64_t)blockIdx.x * chunk; cb < n; cb += stride) {
    uint4 r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = cb + (uint64_t)u * blockDim.x + threadIdx.x;
      r[u] = i < n ? load16<true>(src + i) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= r[u].x ^ r[u].y ^ r[u].z ^ r[u].w;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc ^= (uint32_t)__shfl_xor(acc, o);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t x = 0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) x ^= red[w];
    sink[blockIdx.x] = x;
  }
}

__global__ void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
}  // namespace tsa

extern "C" {
// Plain device copy of `bytes` (a multiple of 16, 16-byte aligned pointers):
// the reference workload for scaling FETCH_SIZE / WRITE_SIZE counters.
int tsa_internal_copy(void* dst, const void* src, size_t bytes, tsa_stream_t stream) {
  if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16) return TSA_EINVAL;
  const uint64_t n = bytes / 16;
  hipStream_t s = (hipStream_t)stream;
  trace_begin("copy", s);
  hipLaunchKernelGGL(k_copy16, dim3(2048), dim3(512), 0, s, (const uint4*)src, (uint4*)dst, n);
  trace_end(s);
  return hipGetLastError() == hipSuccess ? TSA_OK : TSA_EDEVICE;
}

int32_t tsa_internal_probe_blocks(void) {
  DevInfo dev;
  if (device_info(&dev) != TSA_OK) return 0;
  return dev.cus * 2;
}

int tsa_internal_read_probe(const void* src, size_t bytes, uint32_t* d_sink, tsa_stream_t stream) {
  if (!src || !d_sink || bytes % 16 || (uintptr_t)src % 16) return TSA_EINVAL;
  const int32_t blocks = tsa_internal_probe_blocks();
  if (blocks < 1) return TSA_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  trace_begin("read_probe", s);
  hipLaunchKernelGGL(k_read_probe, dim3(blocks), dim3(512), 0, s, (const uint4*)src, (uint64_t)(bytes / 16), d_sink);
  trace_end(s);
  return hipGetLastError() == hipSuccess ? TSA_OK : TSA_EDEVICE;
}
}  // extern "C"
