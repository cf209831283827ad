// Autotuner of the batched region queries: times a grid of launch choices on
// the caller's own batch and remembers the fastest per shape class.
#include <map>
#include <mutex>
#include <string>

#include "tsa_internal.hpp"

extern "C" int tsa_tune_load(const char* path);

namespace tsa {
size_t batch_ws_bytes(const tsa_cube* cube, int32_t nbins, int32_t nq);
int run_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                     tsa_result* d_results, uint64_t* d_hists, const tsa_tune* tune, void* d_ws, size_t ws_bytes,
                     tsa_stream_t stream);

namespace {
std::mutex g_mu;
std::map<std::string, tsa_tune>& table() {
  static std::map<std::string, tsa_tune> t;
  return t;
}
int log2_bucket(uint32_t v) {
  int b = 0;
  while ((1u << (b + 1)) <= v && b < 31) ++b;
  return b;
}
}  // namespace

// Shape class of a batch: device architecture, dtype, bin count, log2 of nq.
std::string tune_key(const tsa_cube* cube, int32_t nbins, int32_t nq) {
  int dev = 0;
  hipDeviceProp_t p;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) arch = p.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  char buf[160];
  snprintf(buf, sizeof(buf), "%s|%s|nbins=%d|nq2=%d", arch.c_str(), cube->dtype == TSA_F32 ? "f32" : "i16", nbins,
           log2_bucket((uint32_t)nq));
  return buf;
}

bool tune_lookup(const tsa_cube* cube, int32_t nbins, int32_t nq, tsa_tune* out) {
  static std::once_flag once;
  std::call_once(once, [] {
    if (const char* path = getenv("TSA_TUNE_CACHE")) (void)tsa_tune_load(path);
  });
  const std::string k = tune_key(cube, nbins, nq);
  std::lock_guard<std::mutex> g(g_mu);
  auto it = table().find(k);
  if (it == table().end()) return false;
  *out = it->second;
  return true;
}

}  // namespace tsa

using namespace tsa;

extern "C" {

int tsa_tune_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                          tsa_result* d_results, uint64_t* d_hists, void* d_ws, size_t ws_bytes, tsa_stream_t stream,
                          int32_t reps, tsa_tune* best, float* best_ms) {
  if (!best || reps < 1) return TSA_EINVAL;
  int st = check_cube(cube);
  if (st) return st;
  if (ws_bytes < batch_ws_bytes(cube, nbins, nq)) return TSA_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return TSA_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return TSA_EDEVICE;
  }
  // coordinate search: tile size x blocks per CU, then the LDS replicas of
  // each histogram bin at the best of those, then the candidate cap
  float bms = 1e30f;
  const int32_t cm = (int32_t)kBatchCandMax;
  tsa_tune bt = {0, 256, 4, cm, 0};
  auto trial = [&](const tsa_tune& t) -> int {
    int r = run_region_batch(cube, d_regions, nq, nbins, d_results, d_hists, &t, d_ws, ws_bytes, stream);  // warm
    if (r) return r;
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < reps && r == TSA_OK; ++i)
      r = run_region_batch(cube, d_regions, nq, nbins, d_results, d_hists, &t, d_ws, ws_bytes, stream);
    (void)hipEventRecord(e1, s);
    if (r) return r;
    if (hipEventSynchronize(e1) != hipSuccess) return TSA_EDEVICE;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)reps;
    if (ms < bms) {
      bms = ms;
      bt = t;
    }
    return TSA_OK;
  };
  const int32_t tiles[] = {0, 65536, 262144, 1048576};
  const int32_t bpcs[] = {2, 4, 6, 8};
  for (int32_t tv : tiles)
    for (int32_t bpc : bpcs)
      if (!st) st = trial(tsa_tune{tv, 256, bpc, cm, 0});
  const int32_t reps_of_bin[] = {1, 2, 4, 8};
  const tsa_tune b1 = bt;
  for (int32_t r : reps_of_bin)
    if (!st) st = trial(tsa_tune{b1.tile_voxels, 256, b1.blocks_per_cu, cm, r});
  const int32_t caps[] = {65536, 262144, 4 << 20};  // 1M was measured with every choice above
  const tsa_tune b2 = bt;
  for (int32_t c : caps)
    if (!st) st = trial(tsa_tune{b2.tile_voxels, 256, b2.blocks_per_cu, c, b2.replicas});
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  *best = bt;
  if (best_ms) *best_ms = bms;
  std::lock_guard<std::mutex> g(g_mu);
  table()[tune_key(cube, nbins, nq)] = bt;
  return TSA_OK;
}

int tsa_tune_save(const char* path) {
  if (!path) return TSA_EINVAL;
  std::lock_guard<std::mutex> g(g_mu);
  FILE* f = fopen(path, "w");
  if (!f) return TSA_EINVAL;
  fprintf(f, "{");
  bool first = true;
  for (auto& kv : table()) {
    fprintf(f, "%s\n  \"%s\": [%d, %d, %d, %d, %d]", first ? "" : ",", kv.first.c_str(), kv.second.tile_voxels,
            kv.second.block_threads, kv.second.blocks_per_cu, kv.second.cand_max, kv.second.replicas);
    first = false;
  }
  fprintf(f, "\n}\n");
  fclose(f);
  return TSA_OK;
}

int tsa_tune_load(const char* path) {
  if (!path) return TSA_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return TSA_EINVAL;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, n);
  fclose(f);
  // entries: "key": [tile_voxels, block_threads, blocks_per_cu, cand_max(, replicas)]
  int loaded = 0;
  size_t pos = 0;
  std::lock_guard<std::mutex> g(g_mu);
  for (;;) {
    const size_t q0 = txt.find('"', pos);
    if (q0 == std::string::npos) break;
    const size_t q1 = txt.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const size_t lb = txt.find('[', q1), rb = txt.find(']', q1);
    if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
    tsa_tune t;
    t.replicas = 0;  // entries written before the replica count was tuned hold four numbers
    const int got = sscanf(txt.c_str() + lb + 1, "%d , %d , %d , %d , %d", &t.tile_voxels, &t.block_threads,
                           &t.blocks_per_cu, &t.cand_max, &t.replicas);
    if (got == 4 || got == 5) {
      table()[txt.substr(q0 + 1, q1 - q0 - 1)] = t;
      ++loaded;
    }
    pos = rb + 1;
  }
  return loaded;
}

}  // extern "C"
