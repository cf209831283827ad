// The C ABI (include/tsa.h): argument checks and dispatch.
#include "tsa_internal.hpp"

namespace tsa {
size_t batch_ws_bytes(const tsa_cube* cube, int32_t nbins, int32_t nq);
int run_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                     tsa_result* d_results, uint64_t* d_hists, const tsa_tune* tune, void* d_ws, size_t ws_bytes,
                     tsa_stream_t stream);
}  // namespace tsa

using namespace tsa;

extern "C" {

size_t tsa_workspace_bytes(int32_t op, const tsa_cube* cube, const tsa_region* region, int32_t nbins, int32_t nq) {
  if (check_cube(cube) != TSA_OK) return 0;
  if (op == TSA_OP_REGION_BATCH) {
    if (nq < 1 || nq > (1 << 20) || nbins < 1 || nbins > 4096) return 0;
    return batch_ws_bytes(cube, nbins, nq);
  }
  if (op < TSA_OP_MOMENTS || op > TSA_OP_MAD || op == TSA_OP_REGION_BATCH) return 0;
  if ((op == TSA_OP_HISTOGRAM || op == TSA_OP_STATS) && (nbins < 1 || nbins > 65536)) return 0;
  tsa_region b;
  if (region_box(cube, region, &b) != TSA_OK) return 0;
  const int64_t volume = (b.x1 - b.x0) * (b.y1 - b.y0) * (b.z1 - b.z0);
  return single_ws_bytes(volume);
}

int tsa_moments(const tsa_cube* cube, const tsa_region* region, tsa_result* d_out, void* d_ws, size_t ws_bytes,
                tsa_stream_t stream) {
  return run_moments(cube, region, d_out, d_ws, ws_bytes, stream);
}

int tsa_histogram(const tsa_cube* cube, const tsa_region* region, float lo, float hi, int32_t nbins,
                  uint64_t* d_counts, uint64_t* d_outliers, void* d_ws, size_t ws_bytes, tsa_stream_t stream) {
  return run_histogram(cube, region, lo, hi, nbins, d_counts, d_outliers, d_ws, ws_bytes, stream);
}

int tsa_median(const tsa_cube* cube, const tsa_region* region, tsa_result* d_out, void* d_ws, size_t ws_bytes,
               tsa_stream_t stream) {
  return run_median(cube, region, d_out, d_ws, ws_bytes, stream);
}

int tsa_stats(const tsa_cube* cube, const tsa_region* region, int32_t nbins, tsa_result* d_out, uint64_t* d_counts,
              uint64_t* d_outliers, void* d_ws, size_t ws_bytes, tsa_stream_t stream) {
  return run_stats(cube, region, nbins, d_out, d_counts, d_outliers, d_ws, ws_bytes, stream);
}

int tsa_stats_static(const tsa_cube* cube, const tsa_region* region, int32_t nbins, tsa_result* d_out,
                     uint64_t* d_counts, uint64_t* d_outliers, tsa_stream_t stream) {
  return run_stats_static(cube, region, nbins, d_out, d_counts, d_outliers, stream);
}

size_t tsa_stats_static_scratch_bytes(void) { return stats_static_scratch_bytes(); }

int64_t tsa_stats_static_candidate_keys(void) { return stats_static_cand_keys(); }

int tsa_quantile(const tsa_cube* cube, const tsa_region* region, double q, int32_t digits, double* d_out,
                 void* d_ws, size_t ws_bytes, tsa_stream_t stream) {
  return run_quantile(cube, region, q, digits, d_out, d_ws, ws_bytes, stream);
}

int tsa_mad(const tsa_cube* cube, const tsa_region* region, double* d_out, void* d_ws, size_t ws_bytes,
            tsa_stream_t stream) {
  return run_mad(cube, region, d_out, d_ws, ws_bytes, stream);
}

int tsa_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                     tsa_result* d_results, uint64_t* d_hists, const tsa_tune* tune, void* d_ws, size_t ws_bytes,
                     tsa_stream_t stream) {
  return run_region_batch(cube, d_regions, nq, nbins, d_results, d_hists, tune, d_ws, ws_bytes, stream);
}

const char* tsa_status_string(int32_t status) {
  switch (status) {
    case TSA_OK:
      return "ok";
    case TSA_EINVAL:
      return "invalid argument";
    case TSA_ENOMEM:
      return "workspace too small";
    case TSA_EDEVICE:
      return "device error";
    case TSA_ENOTSUP:
      return "not supported";
    case TSA_EBUSY:
      return "busy";
    default:
      return "unknown status";
  }
}

const char* tsa_version(void) { return "tsa 0.1.0 (gfx950)"; }

// Host-side check of the invariant-divisor division used by the row walker.
uint32_t tsa_internal_magic_div(uint32_t n, uint32_t d) {
  if (d == 0) return 0;
  const Magic g = make_magic(d);
  const uint32_t t = (uint32_t)(((uint64_t)n * g.m) >> 32);
  return (t + ((n - t) >> g.s1)) >> g.s2;
}

}  // extern "C"
