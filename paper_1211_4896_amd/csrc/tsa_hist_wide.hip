// Histograms with more bins than 32-bit LDS counters can hold (up to 65536).
//
// Counters are 16-bit halves of LDS words, so 65536 bins take 128 KB.  A
// block flushes its non-zero counters to the global uint64 bins and clears
// them after at most 65535 - 16 elements, so no half can overflow into its
// neighbour.  When the device grants less LDS than the bins need, the bins are
// covered in several passes of contiguous bin ranges.
#include <math.h>

#include "tsa_internal.hpp"

namespace tsa {

template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_hist16(Geom g, float lo, float hi, float scale, int32_t nbins, int32_t b0,
                                                 int32_t nb, uint32_t epoch, uint64_t* __restrict__ counts,
                                                 uint64_t* __restrict__ outl, int count_out) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t osm[32];
  lds_zero(lds, ((uint32_t)nb + 1u) >> 1);
  __syncthreads();
  Hist16Acc h{lds, lo, hi, scale, nbins - 1, b0, nb, counts, epoch, 0u, count_out != 0, 0u, 0u};
  walk<DT, VEC, kUnroll, NT>(g, h);
  h.flush();
  if (count_out) block_add_outliers(h.below, h.above, outl, osm);
}

template <int DT, bool VEC, bool NT>
static int launch_hist16(const Geom& g, int grid, int block, size_t lds, float lo, float hi, float scale,
                         int32_t nbins, int32_t b0, int32_t nb, uint32_t epoch, uint64_t* counts, uint64_t* outl,
                         int count_out, hipStream_t s) {
  if (lds > 65536) {
    if (hipFuncSetAttribute((const void*)k_hist16<DT, VEC, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
      return TSA_EDEVICE;
  }
  TSA_TRACED("hist16", s,
             hipLaunchKernelGGL((k_hist16<DT, VEC, NT>), dim3(grid), dim3(block), lds, s, g, lo, hi, scale, nbins,
                                b0, nb, epoch, counts, outl, count_out));
  return hipGetLastError() == hipSuccess ? TSA_OK : TSA_EDEVICE;
}

int run_histogram_wide(const tsa_cube* cube, const Geom& g, bool vec, int grid, int block, float lo, float hi,
                       float scale, int32_t nbins, uint64_t* d_counts, uint64_t* d_outl, hipStream_t s) {
  DevInfo dev;
  int st = device_info(&dev);
  if (st) return st;
  size_t budget = dev.lds_per_block;
  if (budget > 163840) budget = 163840;
  budget -= 512;  // static LDS of the kernel
  const int32_t per_pass = (int32_t)((budget / 4) * 2);  // 16-bit counters
  const int epv = vec ? (cube->dtype == TSA_F32 ? 4 : 8) : 1;
  const int64_t per_chunk = (int64_t)block * kUnroll * epv;
  int64_t ep = (65535 - 16) / per_chunk;
  if (ep < 1) return TSA_ENOTSUP;
  const uint32_t epoch = (uint32_t)ep;
  const bool nt = true;
  for (int32_t b0 = 0; b0 < nbins; b0 += per_pass) {
    const int32_t nb = (nbins - b0) < per_pass ? (nbins - b0) : per_pass;
    const size_t lds = (size_t)((nb + 1) / 2) * 4;
    const int co = b0 == 0;
    if (cube->dtype == TSA_F32) {
      st = vec ? launch_hist16<0, true, true>(g, grid, block, lds, lo, hi, scale, nbins, b0, nb, epoch, d_counts,
                                              d_outl, co, s)
               : launch_hist16<0, false, false>(g, grid, block, lds, lo, hi, scale, nbins, b0, nb, epoch, d_counts,
                                                d_outl, co, s);
    } else {
      st = vec ? launch_hist16<1, true, true>(g, grid, block, lds, lo, hi, scale, nbins, b0, nb, epoch, d_counts,
                                              d_outl, co, s)
               : launch_hist16<1, false, false>(g, grid, block, lds, lo, hi, scale, nbins, b0, nb, epoch, d_counts,
                                                d_outl, co, s);
    }
    (void)nt;
    if (st) return st;
  }
  return TSA_OK;
}

}  // namespace tsa
