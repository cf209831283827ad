// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/tsa.h"
#include "../../include/tsa_trace.h"
#include "tsa_device.hpp"
#include "tsa_ops.hpp"
#include "tsa_walk.hpp"

namespace tsa {

constexpr int kUnroll = 4;            // 16-byte loads in flight per lane
constexpr uint32_t kTileUnits = 8192; // vectors per rows tile (single-region calls)
constexpr int kMaxBlocks = 8192;      // upper bound of a pass grid (moment partial slots)
// The fused passes add their per-block counts into kHistCopies copies of a
// histogram (block b into copy b % kHistCopies), summed by the next one-block
// kernel: a thousand blocks ending together otherwise queue on the same
// counters.  Pass B's copies hold up to kCopyBinsMax bins (more bins take the
// wide passes, which count into the output directly).
constexpr int kHistCopies = 8;
constexpr uint32_t kCopyBinsMax = 12288;
// region batch: largest first-digit bucket whose keys a box copies out (larger ones
// take a third pass over the box); the epilogue scans the copy with one block
constexpr uint32_t kBatchCandMax = 1u << 20;
// tsa_stats_static: bytes of its fixed per-device scratch array
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;

struct Tuning {
  int block = 512;     // threads per block of the streaming passes
  int bpc = 0;         // blocks per compute unit (0: each call's own default)
  bool nt = true;      // non-temporal 16-byte loads
  int rep_shift = -1;  // log2 LDS replicas (-1: by bin count)
};

struct DevInfo {
  int cus;
  size_t lds_per_block;
};

int device_info(DevInfo* out);

// Launch tracing (tsa_trace_enable / tsa_trace_read): no-ops unless enabled.
bool trace_active();
void trace_begin(const char* name, hipStream_t s);
void trace_end(hipStream_t s);
#define TSA_TRACED(NAME, S, ...) \
  do {                           \
    ::tsa::trace_begin(NAME, S); \
    __VA_ARGS__;                 \
    ::tsa::trace_end(S);         \
  } while (0)
// Launch sequences captured once into HIP graphs and replayed, keyed by every
// argument of the call (unused slots zero).  TSA_GRAPH=0 disables them.
struct GraphKey {
  uintptr_t v[24];
};
bool graphs_enabled();
// Replays the graph cached under key on s, or captures enqueue(ctx, stream)
// on a private stream first; returns the capture's or the launch's status.
int graph_run(const GraphKey& key, hipStream_t s, int (*enqueue)(void* ctx, hipStream_t), void* ctx);

Magic make_magic(uint32_t d);
int check_cube(const tsa_cube* c);
int region_box(const tsa_cube* c, const tsa_region* r, tsa_region* b);
int make_geom(const tsa_cube* c, const tsa_region& b, uint32_t tile_units, Geom* g, bool* vec, int64_t* volume);
size_t single_ws_bytes(int64_t volume);

int run_moments(const tsa_cube* cube, const tsa_region* region, tsa_result* d_out, void* d_ws, size_t ws_bytes,
                tsa_stream_t stream);
int run_histogram(const tsa_cube* cube, const tsa_region* region, float lo, float hi, int32_t nbins,
                  uint64_t* d_counts, uint64_t* d_outliers, void* d_ws, size_t ws_bytes, tsa_stream_t stream);
int run_histogram_wide(const tsa_cube* cube, const Geom& g, bool vec, int grid, int block, float lo, float hi,
                       float scale, int32_t nbins, uint64_t* d_counts, uint64_t* d_outl, hipStream_t s);
int run_median(const tsa_cube* cube, const tsa_region* region, tsa_result* d_out, void* d_ws, size_t ws_bytes,
               tsa_stream_t stream);
int run_quantile(const tsa_cube* cube, const tsa_region* region, double q, int32_t digits, double* d_out,
                 void* d_ws, size_t ws_bytes, tsa_stream_t stream);
int run_mad(const tsa_cube* cube, const tsa_region* region, double* d_out, void* d_ws, size_t ws_bytes,
            tsa_stream_t stream);
int run_stats(const tsa_cube* cube, const tsa_region* region, int32_t nbins, tsa_result* d_out, uint64_t* d_counts,
              uint64_t* d_outliers, void* d_ws, size_t ws_bytes, tsa_stream_t stream);
int run_histogram_chunked(const tsa_cube* cube, float lo, float hi, int32_t nbins, uint64_t* d_counts,
                          uint64_t* d_outliers, void* d_ws, size_t ws_bytes, tsa_stream_t stream,
                          int64_t chunk_voxels);
int run_median_chunked(const tsa_cube* cube, tsa_result* d_out, void* d_ws, size_t ws_bytes, tsa_stream_t stream,
                       int64_t chunk_voxels);
int run_stats_static(const tsa_cube* cube, const tsa_region* region, int32_t nbins, tsa_result* d_out,
                     uint64_t* d_counts, uint64_t* d_outliers, tsa_stream_t stream);
size_t stats_static_scratch_bytes();
int64_t stats_static_cand_keys();

}  // namespace tsa
