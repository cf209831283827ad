// Whole-cube and single-region kernels: moments, histogram, radix-select
// median, and the fused two-pass trio.
#include <math.h>

#include <mutex>
#include <vector>

#include "tsa_internal.hpp"

namespace tsa {

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Several disjoint ranges filled by one launch: on a small cube the gaps
// between dependent launches, not the bytes, set the time of the clears.
struct FillRange {
  uint32_t* p;
  uint64_t n;
  uint32_t v, pad;
};
constexpr int kMaxFills = 6;
struct FillSet {
  FillRange r[kMaxFills];
  int count, pad;
};
__global__ void k_fill_set(FillSet f) {
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < f.count; ++k)
    for (uint64_t i = i0; i < f.r[k].n; i += stride) f.r[k].p[i] = f.r[k].v;
}

// ---------------------------------------------------------------------------
// moments pass: one Partial per block
// ---------------------------------------------------------------------------
// float32 lanes sum about a shift of their own and the partials hold
// (n, mean, M2); int16 partials hold exact integer sums.
template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_moments(Geom g, Partial* __restrict__ parts) {
  __shared__ MomShared sm;
  if constexpr (DT == 0) {
    ShiftMomAcc acc;
    walk<DT, VEC, kUnroll, NT>(g, acc);
    block_store_centered(acc, sm, parts + blockIdx.x);
  } else {
    MomAcc<DT> acc;
    walk<DT, VEC, kUnroll, NT>(g, acc);
    block_store_partial(acc, sm, parts + blockIdx.x);
  }
}

// ---------------------------------------------------------------------------
// fixed-range histogram pass (Section 4.1)
// ---------------------------------------------------------------------------
template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_hist(Geom g, float lo, float hi, float scale, int32_t nbins,
                                               uint32_t rshift, uint64_t* __restrict__ counts,
                                               uint64_t* __restrict__ outl) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t osm[32];
  lds_zero(lds, ((uint32_t)nbins << rshift) + kTrash);
  __syncthreads();
  HistAcc h{lds, lo, hi, scale, nbins - 1, rshift, threadIdx.x & ((1u << rshift) - 1u)};
  walk<DT, VEC, kUnroll, NT>(g, h);
  __syncthreads();
  lds_flush(lds, (uint32_t)nbins, rshift, counts);
  block_add_outliers(h.below, h.above, outl, osm);
}

// ---------------------------------------------------------------------------
// histograms of more bins than one LDS copy holds (the standalone call)
// ---------------------------------------------------------------------------
// Where the window of kWinBins 32-bit LDS counters goes: one block bins a
// sample of 64 voxels per lane spread evenly over the region (the stated
// formula), counts them per group of nbins/256 bins, and writes the first bin
// of the run of groups that holds the most samples.  Only the placement
// depends on the sample; k_hist_win counts every voxel exactly wherever the
// window is.
constexpr int kPlaceThreads = 1024, kPlacePerLane = 64;

template <int DT>
__global__ __launch_bounds__(kPlaceThreads) void k_hist_place(const void* base, int64_t nx, int64_t ny, tsa_region b,
                                                              float lo, float hi, float scale, int32_t nbins,
                                                              int32_t* __restrict__ w0_out) {
  using T = typename Ty<DT>::T;
  __shared__ uint32_t coarse[256];
  uint32_t gshift = 0;  // bins per group: 2^gshift, at most 256 groups
  while (((uint32_t)(nbins - 1) >> gshift) >= 256u) ++gshift;
  for (int i = threadIdx.x; i < 256; i += blockDim.x) coarse[i] = 0u;
  __syncthreads();
  const int64_t lx = b.x1 - b.x0, ly = b.y1 - b.y0, lz = b.z1 - b.z0;
  const uint64_t vol = (uint64_t)lx * (uint64_t)ly * (uint64_t)lz;
  const uint64_t ns = (uint64_t)kPlaceThreads * kPlacePerLane;
  for (int k = 0; k < kPlacePerLane; ++k) {
    const uint64_t s = (uint64_t)k * kPlaceThreads + threadIdx.x;
    const uint64_t i = (uint64_t)(((unsigned __int128)s * vol) / ns);  // < vol
    const int64_t x = (int64_t)(i % (uint64_t)lx), r = (int64_t)(i / (uint64_t)lx);
    const int64_t y = r % ly, z = r / ly;
    const float v = (float)((const T*)base)[(b.z0 + z) * nx * ny + (b.y0 + y) * nx + (b.x0 + x)];
    if (v >= lo && v <= hi) {
      const int32_t bin = min(max((int32_t)((v - lo) * scale), 0), nbins - 1);
      atomicAdd(&coarse[(uint32_t)bin >> gshift], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int32_t ngroups = (int32_t)(((uint32_t)(nbins - 1) >> gshift) + 1);
    const int32_t wg = min((int32_t)(kWinBins >> gshift), ngroups);  // groups the window spans
    uint32_t run = 0;
    for (int32_t g = 0; g < wg; ++g) run += coarse[g];
    uint32_t best = run;
    int32_t best_g = 0;
    for (int32_t g = 1; g + wg <= ngroups; ++g) {
      run += coarse[g + wg - 1];
      run -= coarse[g - 1];
      if (run > best) {
        best = run;
        best_g = g;
      }
    }
    int32_t w0 = best_g << gshift;
    if (w0 > nbins - (int32_t)kWinBins) w0 = max(nbins - (int32_t)kWinBins, 0);
    *w0_out = w0;
  }
}

template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_hist_win(Geom g, float lo, float hi, float scale, int32_t nbins,
                                                   const int32_t* __restrict__ w0p, uint64_t* __restrict__ counts,
                                                   uint64_t* __restrict__ outl) {
  extern __shared__ uint32_t lds[];  // kWinBins window counters
  __shared__ uint32_t osm[32];
  const int32_t w0 = *w0p;
  lds_zero(lds, kWinBins);
  __syncthreads();
  HistWinOutAcc h{lds, lo, hi, scale, nbins - 1, w0, counts};
  walk<DT, VEC, kUnroll, NT>(g, h);
  __syncthreads();
  const uint32_t nw = (uint32_t)min((int32_t)kWinBins, nbins - w0);
  for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) {
    const uint32_t c = lds[i];
    if (c) atomicAdd((unsigned long long*)(counts + w0 + i), (unsigned long long)c);
  }
  block_add_outliers(h.below, h.above, outl, osm);
}

// ---------------------------------------------------------------------------
// radix selection: level passes over the cube
// ---------------------------------------------------------------------------
template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_level1(Geom g, uint32_t rshift, uint64_t* __restrict__ hist1) {
  extern __shared__ uint32_t lds[];
  lds_zero(lds, ((uint32_t)kBins1 << rshift) + kTrash);
  __syncthreads();
  Digit1Acc<DT> d{lds, rshift, threadIdx.x & ((1u << rshift) - 1u)};
  walk<DT, VEC, kUnroll, NT>(g, d);
  __syncthreads();
  lds_flush(lds, kBins1, rshift, hist1);
}

template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_level2(Geom g, SelState* __restrict__ st, uint64_t* __restrict__ hist2,
                                                 uint32_t* __restrict__ cand) {
  __shared__ uint32_t lds[kBins2];
  __shared__ CandShared cs;
  if (st->done) return;
  lds_zero(lds, kBins2);
  __syncthreads();
  Level2Acc<DT> a{lds, st->prefix >> kShift1, st->compact != 0, cand_sink(cs, cand, &st->ncand, st->cand_cap)};
  walk<DT, VEC, kUnroll, NT>(g, a);
  a.finish();
  __syncthreads();
  lds_flush(lds, kBins2, 0, hist2);
}

// Level 3 reads the candidate list when level 2 made one, else the cube.
// first = 0: one more slab of a scan cut into slabs (the candidates, when
// there are any, were counted with the first).
template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_level3(Geom g, SelState* __restrict__ st, uint64_t* __restrict__ hist3,
                                                 const uint32_t* __restrict__ cand, int first) {
  __shared__ uint32_t lds[kBins3];
  if (st->done || (st->compact && !first)) return;
  lds_zero(lds, kBins3);
  __syncthreads();
  const uint32_t p2 = st->prefix >> kShift2;
  if (st->compact) {
    const uint32_t n = min(st->ncand, st->cand_cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
      const uint32_t key = cand[i];
      if ((key >> kShift2) == p2) lds_inc(lds, key & 0xFFu);
    }
  } else {
    Level3Acc<DT> a{lds, p2};
    walk<DT, VEC, kUnroll, NT>(g, a);
  }
  __syncthreads();
  lds_flush(lds, kBins3, 0, hist3);
}

// ---------------------------------------------------------------------------
// one-block epilogues: moments merge and digit selection
// ---------------------------------------------------------------------------

TSA_DEV double value_of_key(uint32_t k, int dtype) {
  return dtype == 0 ? (double)__uint_as_float(f32bits_of_key(k)) : (double)i16_of_key(k);
}

struct MergeShared {
  double n[1024], m[1024], q[1024];
  uint32_t kmin[1024], kmax[1024];
  int first;
};

// Whole block: merge np partials in a fixed order (each thread a strided
// sequence, then a pairwise tree) and write the moments fields of *out.
// Returns (in every thread) the global count and min/max keys.
// centered: the partials hold (mean about ref, M2) (k_moments' float32
// lanes); they are merged about one reference, the ref of the first partial
// with a finite mean, which the mean gets back at the end.
TSA_DEV void merge_moments(const Partial* __restrict__ parts, int np, int dtype, uint64_t volume, tsa_result* out,
                           MergeShared& sm, uint64_t& n_out, uint32_t& kmin_out, uint32_t& kmax_out,
                           bool centered = false) {
  const int t = threadIdx.x, bs = blockDim.x;
  double ref0 = 0.0;
  if (centered) {
    if (t == 0) sm.first = np;
    __syncthreads();
    for (int i = t; i < np; i += bs) {
      const Partial& p = parts[i];
      if (p.n && __builtin_isfinite(p.s)) {
        atomicMin(&sm.first, i);
        break;
      }
    }
    __syncthreads();
    if (sm.first < np) ref0 = parts[sm.first].ref;
  }
  double n = 0.0, m = 0.0, q = 0.0;
  uint32_t mn = 0xFFFFFFFFu, mx = 0u;
  for (int i = t; i < np; i += bs) {
    const Partial p = parts[i];
    double pn, pm, pq;
    partial_stats(p, dtype, pn, pm, pq, centered, ref0);
    chan_merge(n, m, q, pn, pm, pq);
    if (p.n) {
      mn = min(mn, p.kmin);
      mx = max(mx, p.kmax);
    }
  }
  sm.n[t] = n;
  sm.m[t] = m;
  sm.q[t] = q;
  sm.kmin[t] = mn;
  sm.kmax[t] = mx;
  __syncthreads();
  for (int s = bs / 2; s > 0; s >>= 1) {
    if (t < s) {
      double a = sm.n[t], b = sm.m[t], c = sm.q[t];
      chan_merge(a, b, c, sm.n[t + s], sm.m[t + s], sm.q[t + s]);
      sm.n[t] = a;
      sm.m[t] = b;
      sm.q[t] = c;
      sm.kmin[t] = min(sm.kmin[t], sm.kmin[t + s]);
      sm.kmax[t] = max(sm.kmax[t], sm.kmax[t + s]);
    }
    __syncthreads();
  }
  const double N = sm.n[0];
  const uint64_t cnt = (uint64_t)N;
  n_out = cnt;
  kmin_out = sm.kmin[0];
  kmax_out = sm.kmax[0];
  if (t == 0) {
    out->count = cnt;
    out->nan_count = volume - cnt;
    out->status = TSA_OK;
    if (cnt == 0) {
      out->mean = out->m2 = out->std = out->min = out->max = __builtin_nan("");
    } else {
      const double vmin = value_of_key(sm.kmin[0], dtype), vmax = value_of_key(sm.kmax[0], dtype);
      out->min = vmin;
      out->max = vmax;
      if (sm.kmin[0] == sm.kmax[0]) {  // every valid voxel holds the same value
        out->mean = vmin;
        out->m2 = 0.0;
        out->std = 0.0;
      } else {
        const double m2 = sm.q[0] < 0.0 ? 0.0 : sm.q[0];  // NaN (infinite values) stays
        out->mean = ref0 + sm.m[0];
        out->m2 = m2;
        out->std = sqrt(m2 / N);
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(1024) void k_moments_merge(const Partial* __restrict__ parts, int np, int dtype,
                                                        uint64_t volume, tsa_result* out) {
  __shared__ MergeShared sm;
  uint64_t n;
  uint32_t a, b;
  merge_moments(parts, np, dtype, volume, out, sm, n, a, b, dtype == 0);
}

struct SelectShared {
  uint64_t wsum[16];
  uint32_t found;
};

// Whole block: choose the digit of the current level from its histogram.
// Level 1 also fixes n and the rank k = floor((n-1)/2) of the lower median.
// When the key is complete, writes the median (and, if write_counts, the
// count fields) to *out.
// With qout != NULL the finished selection goes to qout[0..2] = (value, width of
// the bucket it came from (0 when all digits were selected), count) instead of
// out->median.  st->rank_mode / q / levels select the rank and an early stop.
TSA_DEV void select_level(int level, const uint64_t* __restrict__ hist, SelState* st, int dtype, uint64_t volume,
                          tsa_result* out, bool write_counts, SelectShared& sm, double* qout = nullptr) {
  if (st->done) return;
  const int nb = level == 3 ? kBins3 : kBins1;
  const int shift = level == 1 ? kShift1 : level == 2 ? kShift2 : 0;
  const int t = threadIdx.x, bs = blockDim.x;
  const int per = (nb + bs - 1) / bs;
  const int b0 = t * per;
  uint64_t local = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) local += hist[b0 + i];
  // block exclusive scan of `local`
  const int lane = t % kWave, w = t / kWave;
  uint64_t inc = local;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) sm.wsum[w] = inc;
  if (t == 0) sm.found = 0;
  __syncthreads();
  uint64_t base = inc - local, total = 0;
  for (int i = 0; i < bs / kWave; ++i) {
    if (i < w) base += sm.wsum[i];
    total += sm.wsum[i];
  }
  uint64_t n = level == 1 ? total : st->n;
  if (level == 1 && n == 0) {
    __syncthreads();
    if (t == 0) {
      st->n = 0;
      st->done = 1;
      if (qout) {
        qout[0] = qout[1] = __builtin_nan("");
        qout[2] = 0.0;
      }
      out->median = __builtin_nan("");
      if (write_counts) {
        out->count = 0;
        out->nan_count = volume;
        out->status = TSA_OK;
      }
    }
    return;
  }
  uint64_t k = st->k;
  if (level == 1) {
    if (st->rank_mode) {
      const double kk = floor(st->q * (double)(n - 1));
      k = kk <= 0.0 ? 0 : kk >= (double)(n - 1) ? n - 1 : (uint64_t)kk;
    } else {
      k = (n - 1) / 2;
    }
  }
  __syncthreads();  // every thread has read st before it changes
  if (local > 0 && k >= base && k < base + local) {
    uint64_t cum = base;
    int d = b0;
    for (int i = 0; i < per; ++i) {
      const uint64_t h = (b0 + i < nb) ? hist[b0 + i] : 0;
      if (k < cum + h) {
        d = b0 + i;
        break;
      }
      cum += h;
    }
    const uint64_t bucket = hist[d];
    const uint32_t prefix = (level == 1 ? 0u : st->prefix) | ((uint32_t)d << shift);
    st->n = n;
    st->k = k - cum;
    st->bucket_n = bucket;
    st->prefix = prefix;
    st->level = level;
    if (level == 1) st->compact = bucket <= st->cand_cap ? 1u : 0u;
    const bool exact = level == 3 || (dtype == 1 && level == 2);
    const bool complete = exact || (st->levels >= 1 && (uint32_t)level >= st->levels);
    if (complete) {
      st->done = 1;
      st->result_key = prefix;
      if (qout) {
        // the bucket [prefix, prefix | rest] holds the rank: its smallest value
        // and its width bound the early answer
        uint32_t rest = level == 1 ? 0x000FFFFFu : level == 2 ? 0xFFu : 0u;
        if (dtype == 1) rest &= 0xFFFF0000u;
        double lo = value_of_key(prefix, dtype), hi = value_of_key(prefix | rest, dtype);
        if (lo != lo) lo = -__builtin_inf();
        if (hi != hi) hi = __builtin_inf();
        qout[0] = lo;
        qout[1] = exact ? 0.0 : hi - lo;
        qout[2] = (double)n;
      }
      out->median = value_of_key(prefix, dtype);
      if (write_counts) {
        out->count = n;
        out->nan_count = volume - n;
        out->status = TSA_OK;
      }
    }
    sm.found = 1;
  }
  __syncthreads();
  if (t == 0 && !sm.found) {  // inconsistent histogram: never expected
    st->done = 1;
    out->median = __builtin_nan("");
    out->status = TSA_EDEVICE;
  }
}

__global__ __launch_bounds__(1024) void k_select(int level, const uint64_t* __restrict__ hist, SelState* st,
                                                 int dtype, uint64_t volume, tsa_result* out, int write_counts,
                                                 double* qout) {
  __shared__ SelectShared sm;
  select_level(level, hist, st, dtype, volume, out, write_counts != 0, sm, qout);
}

// ---------------------------------------------------------------------------
// median absolute deviation: the radix passes over d = |x - m|
// ---------------------------------------------------------------------------
template <int DT>
TSA_DEV void median_of_state(const SelState* med, float& mf, int32_t& mi) {
  const uint32_t k = med->result_key;
  mf = __uint_as_float(f32bits_of_key(k));
  mi = i16_of_key(k);
}

template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_mlevel1(Geom g, uint32_t rshift, const SelState* __restrict__ med,
                                                  uint64_t* __restrict__ hist1) {
  extern __shared__ uint32_t lds[];
  if (!med->done || med->n == 0) return;
  lds_zero(lds, ((uint32_t)kBins1 << rshift) + kTrash);
  __syncthreads();
  float mf;
  int32_t mi;
  median_of_state<DT>(med, mf, mi);
  AbsDev<DT, Digit1Acc<0>> a{Digit1Acc<0>{lds, rshift, threadIdx.x & ((1u << rshift) - 1u)}, mf, mi};
  walk<DT, VEC, kUnroll, NT>(g, a);
  __syncthreads();
  lds_flush(lds, kBins1, rshift, hist1);
}

template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_mlevel2(Geom g, const SelState* __restrict__ med, SelState* __restrict__ st,
                                                  uint64_t* __restrict__ hist2, uint32_t* __restrict__ cand) {
  __shared__ uint32_t lds[kBins2];
  __shared__ CandShared cs;
  if (st->done) return;
  lds_zero(lds, kBins2);
  __syncthreads();
  float mf;
  int32_t mi;
  median_of_state<DT>(med, mf, mi);
  AbsDev<DT, Level2Acc<0>> a{
      Level2Acc<0>{lds, st->prefix >> kShift1, st->compact != 0, cand_sink(cs, cand, &st->ncand, st->cand_cap)}, mf,
      mi};
  walk<DT, VEC, kUnroll, NT>(g, a);
  a.inner.finish();
  __syncthreads();
  lds_flush(lds, kBins2, 0, hist2);
}

template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_mlevel3(Geom g, const SelState* __restrict__ med, SelState* __restrict__ st,
                                                  uint64_t* __restrict__ hist3, const uint32_t* __restrict__ cand) {
  __shared__ uint32_t lds[kBins3];
  if (st->done) return;
  lds_zero(lds, kBins3);
  __syncthreads();
  const uint32_t p2 = st->prefix >> kShift2;
  if (st->compact) {
    const uint32_t n = min(st->ncand, st->cand_cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
      const uint32_t key = cand[i];
      if ((key >> kShift2) == p2) lds_inc(lds, key & 0xFFu);
    }
  } else {
    float mf;
    int32_t mi;
    median_of_state<DT>(med, mf, mi);
    AbsDev<DT, Level3Acc<0>> a{Level3Acc<0>{lds, p2}, mf, mi};
    walk<DT, VEC, kUnroll, NT>(g, a);
  }
  __syncthreads();
  lds_flush(lds, kBins3, 0, hist3);
}

// out[0..2] = (median, MAD, count); NaN, NaN, 0 without a valid voxel.
__global__ void k_mad_finish(const SelState* __restrict__ med, const SelState* __restrict__ st, int dtype,
                             double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (med->n == 0 || !med->done || !st->done) {
    out[0] = out[1] = __builtin_nan("");
    out[2] = (double)med->n;
    return;
  }
  out[0] = value_of_key(med->result_key, dtype);
  out[1] = (double)__uint_as_float(f32bits_of_key(st->result_key));
  out[2] = (double)med->n;
}

// ---------------------------------------------------------------------------
// fused trio: pass A (moments + digit 1), mid (merge + select 1 + range),
// pass B (histogram over [min, max] + level 2)
// ---------------------------------------------------------------------------
template <int DT>
struct PassA {
  MomAcc<DT, false> mom;  // the count is the digit histogram's total
  Digit1Acc<DT> d1;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    mom(raw, in);
    d1(raw, in);
  }
  TSA_DEV void chunk() {}
};

template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_pass_a(Geom g, uint32_t rshift, Partial* __restrict__ parts,
                                                 uint64_t* __restrict__ hist1, uint64_t* __restrict__ hcopy,
                                                 uint32_t hcopy_n) {
  extern __shared__ uint32_t lds[];
  __shared__ MomShared sm;
  // pass B's histogram copies start at zero (cleared here, not by a launch of their own)
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < hcopy_n; i += gridDim.x * blockDim.x) hcopy[i] = 0ull;
  lds_zero(lds, ((uint32_t)kBins1 << rshift) + kTrash);
  __syncthreads();
  PassA<DT> a{MomAcc<DT, false>{}, Digit1Acc<DT>{lds, rshift, threadIdx.x & ((1u << rshift) - 1u)}};
  walk<DT, VEC, kUnroll, NT>(g, a);
  // every valid value incremented one first-digit counter: the block's count
  // is their total (each lane adds a strided share; the partial sums them)
  __syncthreads();
  uint32_t c = 0;
  for (uint32_t i = threadIdx.x; i < ((uint32_t)kBins1 << rshift); i += blockDim.x) c += lds[i];
  a.mom.cnt = c;
  block_store_partial(a.mom, sm, parts + blockIdx.x);
  __syncthreads();
  lds_flush(lds, kBins1, rshift, hist1 + (size_t)(blockIdx.x % kHistCopies) * kBins1);
}

__global__ __launch_bounds__(1024) void k_mid(const Partial* __restrict__ parts, int np, int dtype, uint64_t volume,
                                              int32_t nbins, uint64_t* __restrict__ hist1, SelState* st,
                                              tsa_result* out) {
  __shared__ MergeShared msm;
  __shared__ SelectShared ssm;
  // pass A's blocks added into kHistCopies copies of the first-digit counts: summed into the first
  static_assert(kBins1 % 1024 == 0, "k_mid runs as one block of 1024 threads, four bins a thread");
  uint64_t c[kBins1 / 1024];
#pragma unroll
  for (int j = 0; j < kBins1 / 1024; ++j) {  // every load issued before the first add
    const uint32_t b = threadIdx.x + 1024u * j;
    c[j] = hist1[b];
#pragma unroll
    for (int k = 1; k < kHistCopies; ++k) c[j] += hist1[(size_t)k * kBins1 + b];
  }
#pragma unroll
  for (int j = 0; j < kBins1 / 1024; ++j) hist1[threadIdx.x + 1024u * j] = c[j];
  __syncthreads();
  uint64_t n;
  uint32_t kmin, kmax;
  merge_moments(parts, np, dtype, volume, out, msm, n, kmin, kmax);
  if (threadIdx.x == 0) {
    uint32_t ok = 0;
    float lo = 0.f, hi = 0.f, scale = 0.f;
    if (n > 0) {
      lo = (float)value_of_key(kmin, dtype);
      hi = (float)value_of_key(kmax, dtype);
      if (isfinite(lo) && isfinite(hi)) {
        if (lo == hi) {
          ok = 1;
        } else {
          const float width = hi - lo;
          if (isfinite(width)) {
            scale = (float)nbins / width;
            ok = (isfinite(scale) && scale != 0.0f) ? 1u : 0u;
          }
        }
      }
    }
    st->hist_ok = ok;
    st->lo = lo;
    st->hi = hi;
    st->scale = scale;
    // pass B recomputes M2 about c = fl32(mean) when the values differ (float32 cubes)
    const double mean = out->mean;
    const bool von = dtype == 0 && n > 0 && kmin != kmax && isfinite(mean) &&
                     one_pass_m2_at_risk(mean, out->m2 / (double)n);
    st->shift = von ? (float)mean : 0.0f;
    st->var_on = von ? 1u : 0u;
    out->flags = ok ? 0 : TSA_FLAG_HIST_SKIPPED;
    out->median = __builtin_nan("");
  }
  __syncthreads();
  select_level(1, hist1, st, dtype, volume, out, false, ssm);
  __syncthreads();
  if (threadIdx.x == 0) {
    // many bins: pass B counts the kWinBins bins around the median's first-digit
    // bucket in LDS (where noise-dominated cubes put nearly every value)
    int32_t w0 = 0;
    if (st->hist_ok && nbins > (int32_t)kWinBins) {
      double bm = ((double)(float)value_of_key(st->prefix, dtype) - (double)st->lo) * (double)st->scale;
      if (!(bm >= 0.0)) bm = 0.0;
      if (bm > (double)(nbins - 1)) bm = (double)(nbins - 1);
      w0 = (int32_t)bm - (int32_t)(kWinBins / 2);
      if (w0 > nbins - (int32_t)kWinBins) w0 = nbins - (int32_t)kWinBins;
      if (w0 < 0) w0 = 0;
    }
    st->win0 = w0;
  }
}

template <int DT>
struct PassB {
  HistOwnAcc h;
  Level2Acc<DT> l2;
  VarAcc var;
  bool hist_on, var_on;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    if (hist_on) h(raw, in);
    l2(raw, in);
    if constexpr (DT == 0) {
      if (var_on) var(raw, in);
    }
  }
  TSA_DEV void chunk() {}
};

template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_pass_b(Geom g, int32_t nbins, uint32_t rshift, uint32_t stage,
                                                 SelState* __restrict__ st,
                                                 uint64_t* __restrict__ counts, uint64_t* __restrict__ outl,
                                                 uint64_t* __restrict__ hist2, uint32_t* __restrict__ cand,
                                                 Partial* __restrict__ parts2) {
  // dynamic LDS: [nbins << rshift] histogram, [kBins2] level-2 digits, then the
  // candidate staging of the block's waves
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t osm[32];
  __shared__ MomShared sm;
  const uint32_t hsize = ((uint32_t)nbins << rshift) + kTrash;
  uint32_t* l2 = lds + hsize;
  const bool hist_on = st->hist_ok != 0;
  const bool sel_on = st->done == 0;
  const bool var_on = DT == 0 && st->var_on != 0;
  if (!hist_on && !sel_on && !var_on) return;
  lds_zero(lds, hsize + kBins2);
  const CandSink sink = cand_sink_lds(l2 + kBins2, stage, cand, &st->ncand, st->cand_cap);
  __syncthreads();
  PassB<DT> b{HistOwnAcc{lds, st->lo, st->scale, nbins - 1, rshift, threadIdx.x & ((1u << rshift) - 1u)},
              Level2Acc<DT>{l2, sel_on ? (st->prefix >> kShift1) : 0xFFFFFFFFu, sel_on && st->compact != 0, sink},
              VarAcc{st->shift}, hist_on, var_on};
  walk<DT, VEC, kUnroll, NT>(g, b);
  b.l2.finish();
  __syncthreads();
  // into one of kHistCopies copies (counts holds them nbins apart), summed by k_var_finish
  if (hist_on) lds_flush(lds, (uint32_t)nbins, rshift, counts + (size_t)(blockIdx.x % kHistCopies) * (uint32_t)nbins);
  if (sel_on) lds_flush(l2, kBins2, 0, hist2);
  // values lie in their own [min, max]: the outlier counters keep their zeros

  if (var_on) block_store_var(b.var, sm, parts2 + blockIdx.x);
}

// Pass B with a window of kWinBins 32-bit LDS counters (more bins than fit):
// one 1024-lane block per compute unit; values outside the window go straight
// to the global bins.
template <int DT>
struct PassBWin {
  HistWinAcc h;
  Level2Acc<DT> l2;
  VarAcc var;
  bool hist_on, var_on;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    if (hist_on) h(raw, in);
    l2(raw, in);
    if constexpr (DT == 0) {
      if (var_on) var(raw, in);
    }
  }
  TSA_DEV void chunk() {}
};

template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_pass_bwin(Geom g, int32_t nbins, SelState* __restrict__ st,
                                                    uint64_t* __restrict__ counts, uint64_t* __restrict__ hist2,
                                                    uint32_t* __restrict__ cand, Partial* __restrict__ parts2) {
  // dynamic LDS: [kWinBins] window counters, [kBins2] level-2 digits, candidate staging
  extern __shared__ uint32_t lds[];
  __shared__ MomShared sm;
  uint32_t* l2 = lds + kWinBins;
  const bool hist_on = st->hist_ok != 0;
  const bool sel_on = st->done == 0;
  const bool var_on = DT == 0 && st->var_on != 0;
  if (!hist_on && !sel_on && !var_on) return;
  lds_zero(lds, kWinBins + kBins2);
  const CandSink sink = cand_sink_lds(l2 + kBins2, kWaveStage, cand, &st->ncand, st->cand_cap);
  __syncthreads();
  const int32_t w0 = st->win0;
  PassBWin<DT> b{HistWinAcc{lds, st->lo, st->scale, nbins - 1, w0, counts},
                 Level2Acc<DT>{l2, sel_on ? (st->prefix >> kShift1) : 0xFFFFFFFFu, sel_on && st->compact != 0, sink},
                 VarAcc{st->shift}, hist_on, var_on};
  walk<DT, VEC, kUnroll, NT>(g, b);
  b.l2.finish();
  __syncthreads();
  if (hist_on) {
    const uint32_t nw = (uint32_t)min((int32_t)kWinBins, nbins - w0);
    for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) {
      const uint32_t c = lds[i];
      if (c) atomicAdd((unsigned long long*)(counts + w0 + i), (unsigned long long)c);
    }
  }
  if (sel_on) lds_flush(l2, kBins2, 0, hist2);
  if (var_on) block_store_var(b.var, sm, parts2 + blockIdx.x);
}

// Pass B with 16-bit histogram counters (nbins too large for 32-bit LDS
// counters): the histogram flushes its counters every `epoch` chunks.
template <int DT>
struct PassB16 {
  Hist16Acc h;
  Level2Acc<DT> l2;
  VarAcc var;
  bool hist_on, var_on;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    if (hist_on) h(raw, in);
    l2(raw, in);
    if constexpr (DT == 0) {
      if (var_on) var(raw, in);
    }
  }
  TSA_DEV void chunk() {
    if (hist_on) h.chunk();
  }
};

template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(1024) void k_pass_b16(Geom g, int32_t nbins, uint32_t epoch, SelState* __restrict__ st,
                                                   uint64_t* __restrict__ counts, uint64_t* __restrict__ outl,
                                                   uint64_t* __restrict__ hist2, uint32_t* __restrict__ cand,
                                                   Partial* __restrict__ parts2) {
  extern __shared__ uint32_t lds[];  // [(nbins+1)/2] 16-bit counter pairs, then [kBins2] level-2 digits
  __shared__ uint32_t osm[32];
  __shared__ MomShared sm;
  __shared__ CandShared cs;
  const uint32_t hwords = ((uint32_t)nbins + 1u) >> 1;
  uint32_t* l2 = lds + hwords;
  const bool hist_on = st->hist_ok != 0;
  const bool sel_on = st->done == 0;
  const bool var_on = DT == 0 && st->var_on != 0;
  if (!hist_on && !sel_on && !var_on) return;
  lds_zero(lds, hwords + kBins2);
  __syncthreads();
  PassB16<DT> b{Hist16Acc{lds, st->lo, st->hi, st->scale, nbins - 1, 0, nbins, counts, epoch, 0u, true, 0u, 0u},
                Level2Acc<DT>{l2, sel_on ? (st->prefix >> kShift1) : 0xFFFFFFFFu, sel_on && st->compact != 0,
                              cand_sink(cs, cand, &st->ncand, st->cand_cap)},
                VarAcc{st->shift}, hist_on, var_on};
  walk<DT, VEC, kUnroll, NT>(g, b);
  b.l2.finish();
  if (hist_on) b.h.flush();
  __syncthreads();
  if (sel_on) lds_flush(l2, kBins2, 0, hist2);
  if (hist_on) block_add_outliers(b.h.below, b.h.above, outl, osm);
  if (var_on) block_store_var(b.var, sm, parts2 + blockIdx.x);
}

// M2 about the shift c: M2 = sum (x-c)^2 - n (mean - c)^2, block partials
// added in a fixed order (strided per thread, then a pairwise tree).
__global__ __launch_bounds__(1024) void k_var_finish(const Partial* __restrict__ parts2, int np,
                                                     const SelState* __restrict__ st, tsa_result* out,
                                                     const uint64_t* __restrict__ hcopy, int32_t nbins,
                                                     uint64_t* __restrict__ counts) {
  __shared__ double sq[1024];
  if (hcopy) {  // the histogram from pass B's kHistCopies copies
    for (uint32_t b = threadIdx.x; b < (uint32_t)nbins; b += blockDim.x) {
      uint64_t c = 0;
#pragma unroll
      for (int k = 0; k < kHistCopies; ++k) c += hcopy[(size_t)k * (uint32_t)nbins + b];
      counts[b] = c;
    }
  }
  if (!st->var_on) return;
  const int t = threadIdx.x, bs = blockDim.x;
  double q = 0.0;
  for (int i = t; i < np; i += bs) q += parts2[i].q;
  sq[t] = q;
  __syncthreads();
  for (int s2 = bs / 2; s2 > 0; s2 >>= 1) {
    if (t < s2) sq[t] += sq[t + s2];
    __syncthreads();
  }
  if (t == 0) {
    const double n = (double)out->count;
    const double dm = out->mean - (double)st->shift;
    double m2 = sq[0] - n * dm * dm;
    if (m2 < 0.0) m2 = 0.0;  // rounding below zero; NaN (infinite values) stays
    out->m2 = m2;
    out->std = sqrt(m2 / n);
  }
}

// ---------------------------------------------------------------------------
// host side: argument checks, geometry, workspace layout, launches
// ---------------------------------------------------------------------------

static const Tuning& tuning() {
  static Tuning t = [] {
    Tuning x;
    if (const char* s = getenv("TSA_BLOCK")) x.block = atoi(s);
    if (const char* s = getenv("TSA_BPC")) x.bpc = atoi(s);
    if (const char* s = getenv("TSA_NT")) x.nt = atoi(s) != 0;
    if (const char* s = getenv("TSA_REP")) x.rep_shift = atoi(s);
    if (x.block != 256 && x.block != 512 && x.block != 1024) x.block = 512;
    if (x.bpc < 1 || x.bpc > 16) x.bpc = 0;
    if (x.rep_shift < 0 || x.rep_shift > 3) x.rep_shift = -1;
    return x;
  }();
  return t;
}

int device_info(DevInfo* out) {
  static DevInfo cache[64];
  static bool have[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return TSA_EDEVICE;
  if (!have[dev]) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return TSA_EDEVICE;
    if (strncmp(p.gcnArchName, "gfx950", 6) != 0) return TSA_ENOTSUP;
    cache[dev].cus = p.multiProcessorCount;
    cache[dev].lds_per_block = p.sharedMemPerBlock;
    have[dev] = true;
  }
  *out = cache[dev];
  return TSA_OK;
}

Magic make_magic(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < (uint64_t)d) ++l;
  Magic g;
  g.m = (uint32_t)((((1ull << 32) * ((1ull << l) - (uint64_t)d)) / (uint64_t)d) + 1ull);
  g.s1 = l ? 1u : 0u;
  g.s2 = l ? l - 1u : 0u;
  return g;
}

int check_cube(const tsa_cube* c) {
  if (!c || !c->data) return TSA_EINVAL;
  if (c->dtype != TSA_F32 && c->dtype != TSA_I16) return TSA_ENOTSUP;
  if (c->reserved != 0) return TSA_EINVAL;
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) return TSA_EINVAL;
  if (c->nx > (1ll << 31) || c->ny > (1ll << 31) || c->nz > (1ll << 31)) return TSA_EINVAL;
  const double n = (double)c->nx * (double)c->ny * (double)c->nz;
  if (n > (double)(1ll << 46)) return TSA_EINVAL;
  return TSA_OK;
}

int region_box(const tsa_cube* c, const tsa_region* r, tsa_region* b) {
  if (!r) {
    b->x0 = b->y0 = b->z0 = 0;
    b->x1 = c->nx;
    b->y1 = c->ny;
    b->z1 = c->nz;
    return TSA_OK;
  }
  if (r->x0 < 0 || r->y0 < 0 || r->z0 < 0 || r->x1 > c->nx || r->y1 > c->ny || r->z1 > c->nz) return TSA_EINVAL;
  if (r->x0 >= r->x1 || r->y0 >= r->y1 || r->z0 >= r->z1) return TSA_EINVAL;
  *b = *r;
  return TSA_OK;
}

// Build the walk geometry of box b; tile_units = target vectors per rows tile.
int make_geom(const tsa_cube* c, const tsa_region& b, uint32_t tile_units, Geom* g, bool* vec, int64_t* volume) {
  const int64_t esz = c->dtype == TSA_F32 ? 4 : 2;
  const int64_t epv = 16 / esz;
  const int64_t lx = b.x1 - b.x0, ly = b.y1 - b.y0, lz = b.z1 - b.z0;
  *volume = lx * ly * lz;
  memset(g, 0, sizeof(*g));
  g->base = c->data;
  const bool aligned = ((uintptr_t)c->data % 16) == 0;
  const int64_t e0 = b.x0 + c->nx * (b.y0 + c->ny * b.z0);
  const bool contig = (lx == c->nx && (ly == c->ny || lz == 1)) || (ly == 1 && lz == 1);
  if (contig) {
    g->mode = 0;
    const int64_t e1 = e0 + *volume;
    *vec = aligned;
    if (aligned) {
      int64_t v0 = (e0 + epv - 1) / epv, v1 = e1 / epv;
      if (v0 >= v1) {
        g->v0 = g->v1 = 0;
        g->h0 = e0;
        g->h1 = e1;
        g->t0 = g->t1 = 0;
      } else {
        g->v0 = v0;
        g->v1 = v1;
        g->h0 = e0;
        g->h1 = v0 * epv;
        g->t0 = v1 * epv;
        g->t1 = e1;
      }
    } else {
      g->v0 = e0;
      g->v1 = e1;
    }
    return TSA_OK;
  }
  g->mode = 1;
  if ((uint64_t)ly * (uint64_t)lz > 0xFFFFFFFFull) return TSA_EINVAL;
  g->nrows = (uint32_t)(ly * lz);
  g->ly = (uint32_t)ly;
  *vec = aligned && (c->nx % epv) == 0;
  if (*vec) {
    const int64_t c0 = b.x0 / epv, c1 = (b.x1 + epv - 1) / epv;
    g->v_origin = (b.x0 / epv) + (c->nx / epv) * (b.y0 + c->ny * b.z0);
    g->v_ystride = c->nx / epv;
    g->v_zstride = (c->nx / epv) * c->ny;
    g->vpr = (uint32_t)(c1 - c0);
    g->head_skip = (uint32_t)(b.x0 % epv);
    g->last_valid = (uint32_t)(b.x1 - (c1 - 1) * epv);
  } else {
    g->v_origin = e0;
    g->v_ystride = c->nx;
    g->v_zstride = c->nx * c->ny;
    g->vpr = (uint32_t)lx;
    g->head_skip = 0;
    g->last_valid = 1;
  }
  uint32_t rpt = tile_units / g->vpr;
  if (rpt < 1) rpt = 1;
  while ((uint64_t)rpt * g->vpr > (1ull << 30) && rpt > 1) rpt >>= 1;
  g->rpt = rpt;
  g->ntiles = (g->nrows + rpt - 1) / rpt;
  g->ly_m = make_magic(g->ly);
  g->vpr_m = make_magic(g->vpr);
  return TSA_OK;
}

// Blocks for a pass over geometry g.
static int pass_grid(const Geom& g, bool vec, int block, int maxblocks) {
  int64_t want;
  if (g.mode == 0)
    want = vec ? (g.v1 - g.v0 + (int64_t)block * kUnroll - 1) / ((int64_t)block * kUnroll)
               : (g.v1 - g.v0 + block - 1) / block;
  else
    want = g.ntiles;
  if (want < 1) want = 1;
  if (want > maxblocks) want = maxblocks;
  return (int)want;
}

// Workspace layout of the single-region calls.
struct WsLayout {
  size_t partials, partials2, hist1, hist2, hist3, state, state2, result, outl, hcopy, cand, total;
  uint32_t cand_cap;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// cand_limit: most candidate keys the layout may hold (the fixed scratch of
// tsa_stats_static); a median bucket above the capacity takes a third pass.
static WsLayout ws_layout(int64_t volume, int64_t cand_limit = INT64_MAX) {
  WsLayout L;
  size_t o = 0;
  L.partials = o;
  o = align256(o + sizeof(Partial) * kMaxBlocks);
  L.partials2 = o;
  o = align256(o + sizeof(Partial) * kMaxBlocks);
  L.hist1 = o;
  o = align256(o + 8 * (size_t)kBins1 * kHistCopies);
  L.hist2 = o;
  o = align256(o + 8 * kBins2);
  L.hist3 = o;
  o = align256(o + 8 * kBins3);
  L.state = o;
  o = align256(o + sizeof(SelState));
  L.state2 = o;
  o = align256(o + sizeof(SelState));
  L.result = o;
  o = align256(o + sizeof(tsa_result));
  L.outl = o;
  o = align256(o + 16);
  L.hcopy = o;
  o = align256(o + 8 * (size_t)kHistCopies * kCopyBinsMax);
  int64_t cap = volume / 64;
  if (cap < 65536) cap = 65536;
  if (cap > (1ll << 26)) cap = 1ll << 26;
  if (cap > volume) cap = volume;
  if (cap > cand_limit) cap = cand_limit;
  L.cand_cap = (uint32_t)cap;
  L.cand = o;
  o = align256(o + 4 * (size_t)cap);
  L.total = o;
  return L;
}

size_t single_ws_bytes(int64_t volume) { return ws_layout(volume).total; }

static int launch_ok() { return hipGetLastError() == hipSuccess ? TSA_OK : TSA_EDEVICE; }

static void fill32(void* p, size_t words, uint32_t v, hipStream_t s) {
  if (words == 0) return;
  int blocks = (int)((words + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  TSA_TRACED("fill", s, hipLaunchKernelGGL(k_fill32, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, (uint64_t)words, v));
}

// One launch for up to kMaxFills disjoint (words, value) ranges.
static void fill_set(std::initializer_list<FillRange> ranges, hipStream_t s) {
  FillSet f{};
  uint64_t most = 0;
  for (const FillRange& r : ranges) {
    if (r.n == 0) continue;
    f.r[f.count++] = r;  // callers pass at most kMaxFills
    if (r.n > most) most = r.n;
  }
  if (f.count == 0) return;
  int blocks = (int)((most + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  TSA_TRACED("fill", s, hipLaunchKernelGGL(k_fill_set, dim3(blocks), dim3(256), 0, s, f));
}

#define TSA_DISPATCH(DTV, VECV, NTV, EXPR)                              \
  do {                                                                  \
    if ((DTV) == 0 && (VECV) && (NTV)) {                                \
      constexpr int DT = 0;                                             \
      constexpr bool VEC = true, NT = true;                             \
      EXPR;                                                             \
    } else if ((DTV) == 0 && (VECV) && !(NTV)) {                        \
      constexpr int DT = 0;                                             \
      constexpr bool VEC = true, NT = false;                            \
      EXPR;                                                             \
    } else if ((DTV) == 0 && !(VECV)) {                                 \
      constexpr int DT = 0;                                             \
      constexpr bool VEC = false, NT = false;                           \
      EXPR;                                                             \
    } else if ((DTV) == 1 && (VECV) && (NTV)) {                         \
      constexpr int DT = 1;                                             \
      constexpr bool VEC = true, NT = true;                             \
      EXPR;                                                             \
    } else if ((DTV) == 1 && (VECV) && !(NTV)) {                        \
      constexpr int DT = 1;                                             \
      constexpr bool VEC = true, NT = false;                            \
      EXPR;                                                             \
    } else {                                                            \
      constexpr int DT = 1;                                             \
      constexpr bool VEC = false, NT = false;                           \
      EXPR;                                                             \
    }                                                                   \
  } while (0)

// Common preparation of a single-region call.
struct Prep {
  DevInfo dev;
  tsa_region box;
  Geom g;
  bool vec;
  int64_t volume;
  WsLayout L;
  char* ws;
  hipStream_t s;
  int block, grid, bpc;
};

// Blocks per compute unit by call (measured on the 1024x1024x1280 float32
// cube): the fused trio and the moments gain from a third block per CU, the
// histogram and the radix passes lose.
constexpr int kBpcStats = 3, kBpcMoments = 3, kBpcHist = 2, kBpcSelect = 2;

static int prepare(const tsa_cube* cube, const tsa_region* region, void* d_ws, size_t ws_bytes,
                   tsa_stream_t stream, Prep* P, int bpc_default, int64_t cand_limit = INT64_MAX) {
  int st = check_cube(cube);
  if (st) return st;
  if ((st = region_box(cube, region, &P->box))) return st;
  if ((st = device_info(&P->dev))) return st;
  if ((st = make_geom(cube, P->box, kTileUnits, &P->g, &P->vec, &P->volume))) return st;
  P->L = ws_layout(P->volume, cand_limit);
  if (!d_ws || ws_bytes < P->L.total) return TSA_ENOMEM;
  P->ws = (char*)d_ws;
  P->s = (hipStream_t)stream;
  const Tuning& T = tuning();
  P->block = T.block;
  P->bpc = T.bpc ? T.bpc : bpc_default;
  int maxb = P->dev.cus * P->bpc;
  if (maxb > kMaxBlocks) maxb = kMaxBlocks;
  P->grid = pass_grid(P->g, P->vec, P->block, maxb);
  return TSA_OK;
}

static uint32_t rep_shift_for(int nbins, size_t lds_budget) {
  const Tuning& T = tuning();
  uint32_t r = 0;
  if (T.rep_shift >= 0)
    r = (uint32_t)T.rep_shift;
  else
    r = nbins <= 1024 ? 2u : nbins <= 4096 ? 1u : 0u;
  while (r > 0 && ((size_t)nbins << r) * 4 > lds_budget) --r;
  return r;
}

// Zero the level histograms and the selection state, set the capacity, and
// clear the caller's output counters (d_counts: nbins u64, outl: 2 u64; null
// for none), all in one launch.
static void reset_select(const Prep& P, uint64_t* d_counts = nullptr, int32_t nbins = 0, uint64_t* outl = nullptr) {
  char* lo = P.ws + P.L.hist1;
  char* cap = P.ws + P.L.state + offsetof(SelState, cand_cap);
  char* hi = P.ws + P.L.state + sizeof(SelState);
  static_assert(offsetof(SelState, cand_cap) % 4 == 0, "word-aligned capacity");
  fill_set({FillRange{(uint32_t*)lo, (uint64_t)(cap - lo) / 4, 0u, 0u},
            FillRange{(uint32_t*)cap, 1u, P.L.cand_cap, 0u},
            FillRange{(uint32_t*)(cap + 4), (uint64_t)(hi - cap - 4) / 4, 0u, 0u},
            FillRange{(uint32_t*)d_counts, d_counts ? (uint64_t)nbins * 2 : 0u, 0u, 0u},
            FillRange{(uint32_t*)outl, outl ? 4u : 0u, 0u, 0u}},
           P.s);
}

template <int DT, bool VEC, bool NT>
static int launch_pass_b16(const Prep& P, int block, int grid, size_t lds, int32_t nbins, uint32_t epoch,
                           SelState* stp, uint64_t* d_counts, uint64_t* outl, uint64_t* h2, uint32_t* cand,
                           Partial* parts2) {
  if (lds > 65536 && hipFuncSetAttribute((const void*)k_pass_b16<DT, VEC, NT>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return TSA_EDEVICE;
  TSA_TRACED("pass_b16", P.s,
             hipLaunchKernelGGL((k_pass_b16<DT, VEC, NT>), dim3(grid), dim3(block), lds, P.s, P.g, nbins, epoch, stp,
                                d_counts, outl, h2, cand, parts2));
  return TSA_OK;
}

template <int DT, bool VEC, bool NT>
static int launch_pass_bwin(const Prep& P, int block, int grid, size_t lds, int32_t nbins, SelState* stp,
                            uint64_t* d_counts, uint64_t* h2, uint32_t* cand, Partial* parts2) {
  if (hipFuncSetAttribute((const void*)k_pass_bwin<DT, VEC, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return TSA_EDEVICE;
  TSA_TRACED("pass_bwin", P.s,
             hipLaunchKernelGGL((k_pass_bwin<DT, VEC, NT>), dim3(grid), dim3(block), lds, P.s, P.g, nbins, stp,
                                d_counts, h2, cand, parts2));
  return TSA_OK;
}

template <int DT, bool VEC, bool NT>
static int launch_hist_win(const Prep& P, int grid, size_t lds, float lo, float hi, float scale, int32_t nbins,
                           const int32_t* w0p, uint64_t* d_counts, uint64_t* outl) {
  if (hipFuncSetAttribute((const void*)k_hist_win<DT, VEC, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return TSA_EDEVICE;
  TSA_TRACED("hist_win", P.s,
             hipLaunchKernelGGL((k_hist_win<DT, VEC, NT>), dim3(grid), dim3(1024), lds, P.s, P.g, lo, hi, scale,
                                nbins, w0p, d_counts, outl));
  return TSA_OK;
}

int run_moments(const tsa_cube* cube, const tsa_region* region, tsa_result* d_out, void* d_ws, size_t ws_bytes,
                tsa_stream_t stream) {
  if (!d_out) return TSA_EINVAL;
  Prep P;
  int st = prepare(cube, region, d_ws, ws_bytes, stream, &P, kBpcMoments);
  if (st) return st;
  Partial* parts = (Partial*)(P.ws + P.L.partials);
  TSA_TRACED("moments", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_moments<DT, VEC, NT>), dim3(P.grid), dim3(P.block), 0, P.s, P.g, parts)));
  TSA_TRACED("moments_merge", P.s,
             hipLaunchKernelGGL(k_moments_merge, dim3(1), dim3(1024), 0, P.s, parts, P.grid, cube->dtype,
                                (uint64_t)P.volume, d_out));
  return launch_ok();
}

int run_histogram(const tsa_cube* cube, const tsa_region* region, float lo, float hi, int32_t nbins,
                  uint64_t* d_counts, uint64_t* d_outliers, void* d_ws, size_t ws_bytes, tsa_stream_t stream) {
  if (!d_counts) return TSA_EINVAL;
  if (nbins < 1 || nbins > 65536) return TSA_EINVAL;
  if (!isfinite(lo) || !isfinite(hi) || lo > hi) return TSA_EINVAL;
  float scale = 0.0f;
  if (lo < hi) {
    volatile float width = hi - lo;
    if (!isfinite(width)) return TSA_EINVAL;
    volatile float sc = (float)nbins / width;
    if (!isfinite(sc) || sc == 0.0f) return TSA_EINVAL;
    scale = sc;
  }
  Prep P;
  int st = prepare(cube, region, d_ws, ws_bytes, stream, &P, kBpcHist);
  if (st) return st;
  uint64_t* outl = d_outliers ? d_outliers : (uint64_t*)(P.ws + P.L.outl);
  fill_set({FillRange{(uint32_t*)d_counts, (uint64_t)nbins * 2, 0u, 0u}, FillRange{(uint32_t*)outl, 4u, 0u, 0u}},
           P.s);
  const size_t budget = P.dev.lds_per_block < 65536 ? P.dev.lds_per_block : 65536;
  const uint32_t rs = rep_shift_for(nbins, budget);
  const size_t lds = (((size_t)nbins << rs) + kTrash) * 4;
  if (lds <= budget) {
    TSA_TRACED("hist", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                   hipLaunchKernelGGL((k_hist<DT, VEC, NT>), dim3(P.grid), dim3(P.block), lds, P.s, P.g, lo, hi, scale,
                                      nbins, rs, d_counts, outl)));
    return launch_ok();
  }
  // a window of 32-bit counters where a sample of the region puts most values,
  // one 1024-lane block per compute unit; else 16-bit counters in epochs
  const size_t lds_win = (size_t)kWinBins * 4;
  if (lds_win + 1024 <= P.dev.lds_per_block) {
    int32_t* w0p = (int32_t*)(P.ws + P.L.state + offsetof(SelState, win0));
    if (cube->dtype == TSA_F32)
      TSA_TRACED("hist_place", P.s,
                 hipLaunchKernelGGL(k_hist_place<0>, dim3(1), dim3(kPlaceThreads), 0, P.s, cube->data, cube->nx,
                                    cube->ny, P.box, lo, hi, scale, nbins, w0p));
    else
      TSA_TRACED("hist_place", P.s,
                 hipLaunchKernelGGL(k_hist_place<1>, dim3(1), dim3(kPlaceThreads), 0, P.s, cube->data, cube->nx,
                                    cube->ny, P.box, lo, hi, scale, nbins, w0p));
    int grid = P.dev.cus;
    if (grid > P.grid) grid = P.grid;
    int stw = TSA_OK;
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 stw = (launch_hist_win<DT, VEC, NT>(P, grid, lds_win, lo, hi, scale, nbins, w0p, d_counts, outl)));
    if (stw) return stw;
    return launch_ok();
  }
  return run_histogram_wide(cube, P.g, P.vec, P.grid, P.block, lo, hi, scale, nbins, d_counts, outl, P.s);
}

static int launch_median_tail(const tsa_cube* cube, const Prep& P, tsa_result* d_out, bool write_counts,
                              double* qout = nullptr) {
  SelState* stp = (SelState*)(P.ws + P.L.state);
  uint64_t* h2 = (uint64_t*)(P.ws + P.L.hist2);
  uint64_t* h3 = (uint64_t*)(P.ws + P.L.hist3);
  uint32_t* cand = (uint32_t*)(P.ws + P.L.cand);
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 2, (const uint64_t*)h2, stp, cube->dtype,
                                (uint64_t)P.volume, d_out, (int)write_counts, qout));
  TSA_TRACED("level3", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_level3<DT, VEC, NT>), dim3(P.grid), dim3(P.block), 0, P.s, P.g, stp, h3,
                                    (const uint32_t*)cand, 1)));
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 3, (const uint64_t*)h3, stp, cube->dtype,
                                (uint64_t)P.volume, d_out, (int)write_counts, qout));
  return launch_ok();
}

int run_median(const tsa_cube* cube, const tsa_region* region, tsa_result* d_out, void* d_ws, size_t ws_bytes,
               tsa_stream_t stream) {
  if (!d_out) return TSA_EINVAL;
  Prep P;
  int st = prepare(cube, region, d_ws, ws_bytes, stream, &P, kBpcSelect);
  if (st) return st;
  reset_select(P);
  SelState* stp = (SelState*)(P.ws + P.L.state);
  uint64_t* h1 = (uint64_t*)(P.ws + P.L.hist1);
  uint64_t* h2 = (uint64_t*)(P.ws + P.L.hist2);
  uint32_t* cand = (uint32_t*)(P.ws + P.L.cand);
  const uint32_t rs = rep_shift_for(kBins1, 32768);
  TSA_TRACED("level1", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_level1<DT, VEC, NT>), dim3(P.grid), dim3(P.block), (((size_t)kBins1 << rs) + kTrash) * 4,
                                    P.s, P.g, rs, h1)));
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 1, (const uint64_t*)h1, stp, cube->dtype,
                                (uint64_t)P.volume, d_out, 1, (double*)nullptr));
  TSA_TRACED("level2", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_level2<DT, VEC, NT>), dim3(P.grid), dim3(P.block), 0, P.s, P.g, stp, h2, cand)));
  return launch_median_tail(cube, P, d_out, true);
}

// ---------------------------------------------------------------------------
// Whole-cube scans cut into z-slabs of at most chunk_voxels voxels: every
// pass over the data goes out as one launch per slab, so a device shared
// with other streams (the serving loop's region batches) can start their
// work between two launches of a long scan.  The same kernels accumulate
// their counters across the slabs, so the results are the same as one
// launch per pass gives.
// ---------------------------------------------------------------------------
struct Slab {
  Geom g;
  bool vec;
  int grid;
};

static int slabs_of(const tsa_cube* cube, int64_t chunk_voxels, const Prep& P, std::vector<Slab>* out) {
  const int64_t plane = cube->nx * cube->ny;
  int64_t planes = chunk_voxels / plane;
  if (planes < 1) planes = 1;
  int maxb = P.dev.cus * P.bpc;
  if (maxb > kMaxBlocks) maxb = kMaxBlocks;
  for (int64_t z0 = 0; z0 < cube->nz; z0 += planes) {
    const tsa_region b{0, 0, z0, cube->nx, cube->ny, z0 + planes < cube->nz ? z0 + planes : cube->nz};
    Slab sl;
    int64_t vol = 0;
    const int st = make_geom(cube, b, kTileUnits, &sl.g, &sl.vec, &vol);
    if (st) return st;
    sl.grid = pass_grid(sl.g, sl.vec, P.block, maxb);
    out->push_back(sl);
  }
  return TSA_OK;
}

int run_histogram_chunked(const tsa_cube* cube, float lo, float hi, int32_t nbins, uint64_t* d_counts,
                          uint64_t* d_outliers, void* d_ws, size_t ws_bytes, tsa_stream_t stream,
                          int64_t chunk_voxels) {
  if (!d_counts || chunk_voxels < 1) return TSA_EINVAL;
  if (nbins < 1 || nbins > 65536) return TSA_EINVAL;
  if (!isfinite(lo) || !isfinite(hi) || lo > hi) return TSA_EINVAL;
  float scale = 0.0f;
  if (lo < hi) {
    volatile float width = hi - lo;
    if (!isfinite(width)) return TSA_EINVAL;
    volatile float sc = (float)nbins / width;
    if (!isfinite(sc) || sc == 0.0f) return TSA_EINVAL;
    scale = sc;
  }
  Prep P;
  int st = prepare(cube, nullptr, d_ws, ws_bytes, stream, &P, kBpcHist);
  if (st) return st;
  std::vector<Slab> slabs;
  if ((st = slabs_of(cube, chunk_voxels, P, &slabs))) return st;
  uint64_t* outl = d_outliers ? d_outliers : (uint64_t*)(P.ws + P.L.outl);
  fill_set({FillRange{(uint32_t*)d_counts, (uint64_t)nbins * 2, 0u, 0u}, FillRange{(uint32_t*)outl, 4u, 0u, 0u}},
           P.s);
  const size_t budget = P.dev.lds_per_block < 65536 ? P.dev.lds_per_block : 65536;
  const uint32_t rs = rep_shift_for(nbins, budget);
  const size_t lds = (((size_t)nbins << rs) + kTrash) * 4;
  for (const Slab& sl : slabs) {
    if (lds <= budget) {
      TSA_TRACED("hist", P.s,
        TSA_DISPATCH(cube->dtype, sl.vec, tuning().nt,
                     hipLaunchKernelGGL((k_hist<DT, VEC, NT>), dim3(sl.grid), dim3(P.block), lds, P.s, sl.g, lo, hi,
                                        scale, nbins, rs, d_counts, outl)));
    } else if ((st = run_histogram_wide(cube, sl.g, sl.vec, sl.grid, P.block, lo, hi, scale, nbins, d_counts, outl,
                                        P.s))) {
      return st;
    }
  }
  return launch_ok();
}

int run_median_chunked(const tsa_cube* cube, tsa_result* d_out, void* d_ws, size_t ws_bytes, tsa_stream_t stream,
                       int64_t chunk_voxels) {
  if (!d_out || chunk_voxels < 1) return TSA_EINVAL;
  Prep P;
  int st = prepare(cube, nullptr, d_ws, ws_bytes, stream, &P, kBpcSelect);
  if (st) return st;
  std::vector<Slab> slabs;
  if ((st = slabs_of(cube, chunk_voxels, P, &slabs))) return st;
  reset_select(P);
  SelState* stp = (SelState*)(P.ws + P.L.state);
  uint64_t* h1 = (uint64_t*)(P.ws + P.L.hist1);
  uint64_t* h2 = (uint64_t*)(P.ws + P.L.hist2);
  uint64_t* h3 = (uint64_t*)(P.ws + P.L.hist3);
  uint32_t* cand = (uint32_t*)(P.ws + P.L.cand);
  const uint32_t rs = rep_shift_for(kBins1, 32768);
  for (const Slab& sl : slabs)
    TSA_TRACED("level1", P.s,
      TSA_DISPATCH(cube->dtype, sl.vec, tuning().nt,
                   hipLaunchKernelGGL((k_level1<DT, VEC, NT>), dim3(sl.grid), dim3(P.block),
                                      (((size_t)kBins1 << rs) + kTrash) * 4, P.s, sl.g, rs, h1)));
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 1, (const uint64_t*)h1, stp, cube->dtype,
                                (uint64_t)P.volume, d_out, 1, (double*)nullptr));
  for (const Slab& sl : slabs)
    TSA_TRACED("level2", P.s,
      TSA_DISPATCH(cube->dtype, sl.vec, tuning().nt,
                   hipLaunchKernelGGL((k_level2<DT, VEC, NT>), dim3(sl.grid), dim3(P.block), 0, P.s, sl.g, stp, h2,
                                      cand)));
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 2, (const uint64_t*)h2, stp, cube->dtype,
                                (uint64_t)P.volume, d_out, 1, (double*)nullptr));
  for (size_t i = 0; i < slabs.size(); ++i)
    TSA_TRACED("level3", P.s,
      TSA_DISPATCH(cube->dtype, slabs[i].vec, tuning().nt,
                   hipLaunchKernelGGL((k_level3<DT, VEC, NT>), dim3(slabs[i].grid), dim3(P.block), 0, P.s,
                                      slabs[i].g, stp, h3, (const uint32_t*)cand, i == 0 ? 1 : 0)));
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 3, (const uint64_t*)h3, stp, cube->dtype,
                                (uint64_t)P.volume, d_out, 1, (double*)nullptr));
  return launch_ok();
}

static int enqueue_stats(const tsa_cube* cube, const tsa_region* region, int32_t nbins, tsa_result* d_out,
                         uint64_t* d_counts, uint64_t* d_outliers, void* d_ws, size_t ws_bytes, tsa_stream_t stream,
                         int64_t cand_limit = INT64_MAX);

namespace {
struct StatsCall {
  const tsa_cube* cube;
  const tsa_region* region;
  int32_t nbins;
  tsa_result* d_out;
  uint64_t* d_counts;
  uint64_t* d_outliers;
  void* d_ws;
  size_t ws_bytes;
};
int enqueue_stats_call(void* ctx, hipStream_t s) {
  const StatsCall& c = *(const StatsCall*)ctx;
  return enqueue_stats(c.cube, c.region, c.nbins, c.d_out, c.d_counts, c.d_outliers, c.d_ws, c.ws_bytes, s);
}
}  // namespace

// The fused trio's launches go out as one replayed graph (keyed by every
// argument, the box's corners included), so the GPU does not wait on the host
// between its short kernels; traced calls launch directly.
int run_stats(const tsa_cube* cube, const tsa_region* region, int32_t nbins, tsa_result* d_out, uint64_t* d_counts,
              uint64_t* d_outliers, void* d_ws, size_t ws_bytes, tsa_stream_t stream) {
  // argument errors, tracing, and more bins than one LDS histogram holds (the
  // wide passes set kernel attributes at launch) take the direct launch
  int dev = 0;
  if (check_cube(cube) != TSA_OK || !d_out || !d_counts || nbins < 1 || nbins > 8192 || !d_ws ||
      !graphs_enabled() || trace_active() || hipGetDevice(&dev) != hipSuccess)
    return enqueue_stats(cube, region, nbins, d_out, d_counts, d_outliers, d_ws, ws_bytes, stream);
  GraphKey key;
  memset(&key, 0, sizeof(key));
  key.v[0] = 2;  // tsa_stats
  key.v[1] = (uintptr_t)cube->data;
  key.v[2] = (uintptr_t)cube->dtype;
  key.v[3] = (uintptr_t)cube->nx;
  key.v[4] = (uintptr_t)cube->ny;
  key.v[5] = (uintptr_t)cube->nz;
  key.v[6] = (uintptr_t)nbins;
  key.v[7] = (uintptr_t)d_out;
  key.v[8] = (uintptr_t)d_counts;
  key.v[9] = (uintptr_t)d_outliers;
  key.v[10] = (uintptr_t)d_ws;
  key.v[11] = (uintptr_t)ws_bytes;
  key.v[12] = (uintptr_t)dev;
  if (region) {
    key.v[13] = 1;
    key.v[14] = (uintptr_t)region->x0;
    key.v[15] = (uintptr_t)region->y0;
    key.v[16] = (uintptr_t)region->z0;
    key.v[17] = (uintptr_t)region->x1;
    key.v[18] = (uintptr_t)region->y1;
    key.v[19] = (uintptr_t)region->z1;
  }
  StatsCall c{cube, region, nbins, d_out, d_counts, d_outliers, d_ws, ws_bytes};
  return graph_run(key, (hipStream_t)stream, enqueue_stats_call, &c);
}

// ---------------------------------------------------------------------------
// tsa_stats_static: the fused trio on a fixed scratch array of the library's
// own, for callers that cannot allocate device memory.  The host never uses
// the array's name as an address: each device's copy is looked up once with
// hipGetSymbolAddress (with that device current) and that pointer is what
// the kernels get.  Every call on a device shares its copy; calls that
// overlap on one device race.  Each call clears what has to start at zero
// (selection state, level histograms, counts and outliers) with fill kernels.
// ---------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::once_flag g_scratch_once[kMaxScratchDevices];
void* g_scratch_ptr[kMaxScratchDevices];
int g_scratch_status[kMaxScratchDevices];
}  // namespace

static int static_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return TSA_EDEVICE;
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
    g_scratch_status[dev] = (e == hipSuccess && p) ? TSA_OK : TSA_EDEVICE;
  });
  *out = g_scratch_ptr[dev];
  return g_scratch_status[dev];
}

// Candidate keys the fixed scratch holds beside everything else of the call.
static int64_t static_cand_limit() {
  const size_t fixed = ws_layout(0, 0).total;
  return (int64_t)((kStaticScratchBytes - fixed) / 4) & ~(int64_t)63;
}

int run_stats_static(const tsa_cube* cube, const tsa_region* region, int32_t nbins, tsa_result* d_out,
                     uint64_t* d_counts, uint64_t* d_outliers, tsa_stream_t stream) {
  void* ws = nullptr;
  const int st = static_scratch(&ws);
  if (st) return st;
  // launched directly: a graph would be instantiated, and instantiation may allocate
  return enqueue_stats(cube, region, nbins, d_out, d_counts, d_outliers, ws, kStaticScratchBytes, stream,
                       static_cand_limit());
}

size_t stats_static_scratch_bytes() { return kStaticScratchBytes; }
int64_t stats_static_cand_keys() { return static_cand_limit(); }

static int enqueue_stats(const tsa_cube* cube, const tsa_region* region, int32_t nbins, tsa_result* d_out,
                         uint64_t* d_counts, uint64_t* d_outliers, void* d_ws, size_t ws_bytes, tsa_stream_t stream,
                         int64_t cand_limit) {
  if (!d_out || !d_counts) return TSA_EINVAL;
  if (nbins < 1 || nbins > 65536) return TSA_EINVAL;
  Prep P;
  int st = prepare(cube, region, d_ws, ws_bytes, stream, &P, kBpcStats, cand_limit);
  if (st) return st;
  const size_t budget = P.dev.lds_per_block < 65536 ? P.dev.lds_per_block : 65536;
  const size_t cand_small = (size_t)(P.block / kWave) * kWaveStage * 4;  // pass B's candidate staging
  const bool wide = ((size_t)nbins + kTrash + kBins2) * 4 + cand_small > budget;
  // 16-bit counters: (nbins+1)/2 words + level-2 digits, plus ~10 KB of static LDS
  const size_t lds16 = ((((size_t)nbins + 1) / 2) + kBins2) * 4;
  if (wide && lds16 + 10240 > P.dev.lds_per_block) return TSA_ENOTSUP;
  uint64_t* outl = d_outliers ? d_outliers : (uint64_t*)(P.ws + P.L.outl);
  reset_select(P, d_counts, nbins, outl);
  Partial* parts = (Partial*)(P.ws + P.L.partials);
  SelState* stp = (SelState*)(P.ws + P.L.state);
  uint64_t* h1 = (uint64_t*)(P.ws + P.L.hist1);
  uint64_t* h2 = (uint64_t*)(P.ws + P.L.hist2);
  uint32_t* cand = (uint32_t*)(P.ws + P.L.cand);
  uint64_t* hcopy = (uint64_t*)(P.ws + P.L.hcopy);
  if (!wide && nbins > (int32_t)kCopyBinsMax) return TSA_ENOTSUP;  // cannot happen: the LDS bounds nbins first
  const uint32_t rs1 = rep_shift_for(kBins1, 32768);
  TSA_TRACED("pass_a", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_pass_a<DT, VEC, NT>), dim3(P.grid), dim3(P.block), (((size_t)kBins1 << rs1) + kTrash) * 4,
                                    P.s, P.g, rs1, parts, h1, hcopy, wide ? 0u : (uint32_t)kHistCopies * (uint32_t)nbins)));
  TSA_TRACED("mid", P.s,
             hipLaunchKernelGGL(k_mid, dim3(1), dim3(1024), 0, P.s, (const Partial*)parts, P.grid, cube->dtype,
                                (uint64_t)P.volume, nbins, h1, stp, d_out));
  Partial* parts2 = (Partial*)(P.ws + P.L.partials2);
  int np2 = P.grid;
  if (!wide) {
    // replicas only as far as bpc blocks of pass B still share a compute unit
    // (its static LDS: candidate staging, moment reduction, outliers)
    const size_t per_block = P.dev.lds_per_block / (size_t)P.bpc;
    // (and within the 64 KB a launch takes without raising its LDS limit)
    const size_t cap_b = per_block < budget ? per_block : budget;
    auto fixed_of = [&](size_t cb) { return sizeof(MomShared) + 32 * 4 + cb + (kBins2 + kTrash) * 4 + 1024; };  // + slack
    // the deep candidate stage when one replica of every bin still fits beside it
    uint32_t stage = kWaveStageBig;
    size_t cand_b = (size_t)(P.block / kWave) * stage * 4;
    if (fixed_of(cand_b) + ((size_t)nbins + kTrash) * 4 > cap_b) {
      stage = kWaveStage;
      cand_b = cand_small;
    }
    const size_t fixed_b = fixed_of(cand_b);
    const size_t budget_b = cap_b > fixed_b ? cap_b - fixed_b : 0;
    uint32_t rsb = rep_shift_for(nbins, budget_b);
    const size_t ldsb = (((size_t)nbins << rsb) + kTrash + kBins2) * 4 + cand_b;
    TSA_TRACED("pass_b", P.s,
      TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                   hipLaunchKernelGGL((k_pass_b<DT, VEC, NT>), dim3(P.grid), dim3(P.block), ldsb, P.s, P.g, nbins,
                                      rsb, stage, stp, hcopy, outl, h2, cand, parts2)));
  } else {
    // one 1024-thread block per compute unit: a window of 32-bit counters when
    // the device grants the LDS, else 16-bit counters flushed in epochs
    const int blk = 1024;
    int grid = P.dev.cus;
    if (grid > P.grid) grid = P.grid;
    np2 = grid;
    const size_t lds_win = ((size_t)kWinBins + kBins2 + (blk / kWave) * kWaveStage) * 4;
    if (lds_win + sizeof(MomShared) + 1024 <= P.dev.lds_per_block) {
      int stw = TSA_OK;
      TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                   stw = (launch_pass_bwin<DT, VEC, NT>(P, blk, grid, lds_win, nbins, stp, d_counts, h2, cand,
                                                        parts2)));
      if (stw) return stw;
      TSA_TRACED("var_finish", P.s,
                 hipLaunchKernelGGL(k_var_finish, dim3(1), dim3(1024), 0, P.s, (const Partial*)parts2, np2,
                                    (const SelState*)stp, d_out, (const uint64_t*)nullptr, nbins, d_counts));
      return launch_median_tail(cube, P, d_out, false);
    }
    const int epv = P.vec ? (cube->dtype == TSA_F32 ? 4 : 8) : 1;
    const int64_t ep = (65535 - 16) / ((int64_t)blk * kUnroll * epv);
    if (ep < 1) return TSA_ENOTSUP;
    int st2 = TSA_OK;
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 st2 = (launch_pass_b16<DT, VEC, NT>(P, blk, grid, lds16, nbins, (uint32_t)ep, stp, d_counts, outl,
                                                     h2, cand, parts2)));
    if (st2) return st2;
  }
  TSA_TRACED("var_finish", P.s,
             hipLaunchKernelGGL(k_var_finish, dim3(1), dim3(1024), 0, P.s, (const Partial*)parts2, np2,
                                (const SelState*)stp, d_out, wide ? (const uint64_t*)nullptr : (const uint64_t*)hcopy,
                                nbins, d_counts));
  return launch_median_tail(cube, P, d_out, false);
}


__global__ void k_init_rank(SelState* st, double q, uint32_t mode, uint32_t levels) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->q = q;
    st->rank_mode = mode;
    st->levels = levels;
  }
}

int run_quantile(const tsa_cube* cube, const tsa_region* region, double q, int32_t digits, double* d_out,
                 void* d_ws, size_t ws_bytes, tsa_stream_t stream) {
  if (!d_out || !(q >= 0.0 && q <= 1.0) || digits < 1 || digits > 3) return TSA_EINVAL;
  Prep P;
  int st = prepare(cube, region, d_ws, ws_bytes, stream, &P, kBpcSelect);
  if (st) return st;
  reset_select(P);
  SelState* stp = (SelState*)(P.ws + P.L.state);
  tsa_result* scratch = (tsa_result*)(P.ws + P.L.result);
  uint64_t* h1 = (uint64_t*)(P.ws + P.L.hist1);
  uint64_t* h2 = (uint64_t*)(P.ws + P.L.hist2);
  uint32_t* cand = (uint32_t*)(P.ws + P.L.cand);
  TSA_TRACED("init", P.s, hipLaunchKernelGGL(k_init_rank, dim3(1), dim3(64), 0, P.s, stp, q, 1u, (uint32_t)digits));
  const uint32_t rs = rep_shift_for(kBins1, 32768);
  TSA_TRACED("level1", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_level1<DT, VEC, NT>), dim3(P.grid), dim3(P.block),
                                    (((size_t)kBins1 << rs) + kTrash) * 4, P.s, P.g, rs, h1)));
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 1, (const uint64_t*)h1, stp, cube->dtype,
                                (uint64_t)P.volume, scratch, 0, d_out));
  TSA_TRACED("level2", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_level2<DT, VEC, NT>), dim3(P.grid), dim3(P.block), 0, P.s, P.g, stp, h2,
                                    cand)));
  return launch_median_tail(cube, P, scratch, false, d_out);
}

int run_mad(const tsa_cube* cube, const tsa_region* region, double* d_out, void* d_ws, size_t ws_bytes,
            tsa_stream_t stream) {
  if (!d_out) return TSA_EINVAL;
  Prep P;
  int st = prepare(cube, region, d_ws, ws_bytes, stream, &P, kBpcSelect);
  if (st) return st;
  reset_select(P);
  SelState* med = (SelState*)(P.ws + P.L.state);
  SelState* sb = (SelState*)(P.ws + P.L.state2);
  tsa_result* scratch = (tsa_result*)(P.ws + P.L.result);
  uint64_t* h1 = (uint64_t*)(P.ws + P.L.hist1);
  uint64_t* h2 = (uint64_t*)(P.ws + P.L.hist2);
  uint64_t* h3 = (uint64_t*)(P.ws + P.L.hist3);
  uint32_t* cand = (uint32_t*)(P.ws + P.L.cand);
  {
    char* b = (char*)sb;
    const size_t c = offsetof(SelState, cand_cap);
    fill_set({FillRange{(uint32_t*)b, c / 4, 0u, 0u}, FillRange{(uint32_t*)(b + c), 1u, P.L.cand_cap, 0u},
              FillRange{(uint32_t*)(b + c + 4), (sizeof(SelState) - c - 4) / 4, 0u, 0u}},
             P.s);
  }
  // 1. the lower median m
  const uint32_t rs = rep_shift_for(kBins1, 32768);
  TSA_TRACED("level1", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_level1<DT, VEC, NT>), dim3(P.grid), dim3(P.block),
                                    (((size_t)kBins1 << rs) + kTrash) * 4, P.s, P.g, rs, h1)));
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 1, (const uint64_t*)h1, med, cube->dtype,
                                (uint64_t)P.volume, scratch, 0, (double*)nullptr));
  TSA_TRACED("level2", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_level2<DT, VEC, NT>), dim3(P.grid), dim3(P.block), 0, P.s, P.g, med, h2,
                                    cand)));
  st = launch_median_tail(cube, P, scratch, false);
  if (st) return st;
  // 2. the lower median of |x - m| (float keys whatever the cube's type)
  fill32(h1, (P.L.state - P.L.hist1) / 4, 0u, P.s);
  TSA_TRACED("mad_level1", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_mlevel1<DT, VEC, NT>), dim3(P.grid), dim3(P.block),
                                    (((size_t)kBins1 << rs) + kTrash) * 4, P.s, P.g, rs, (const SelState*)med, h1)));
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 1, (const uint64_t*)h1, sb, 0,
                                (uint64_t)P.volume, scratch, 0, (double*)nullptr));
  TSA_TRACED("mad_level2", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_mlevel2<DT, VEC, NT>), dim3(P.grid), dim3(P.block), 0, P.s, P.g,
                                    (const SelState*)med, sb, h2, cand)));
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 2, (const uint64_t*)h2, sb, 0,
                                (uint64_t)P.volume, scratch, 0, (double*)nullptr));
  TSA_TRACED("mad_level3", P.s,
    TSA_DISPATCH(cube->dtype, P.vec, tuning().nt,
                 hipLaunchKernelGGL((k_mlevel3<DT, VEC, NT>), dim3(P.grid), dim3(P.block), 0, P.s, P.g,
                                    (const SelState*)med, sb, h3, (const uint32_t*)cand)));
  TSA_TRACED("select", P.s,
             hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, P.s, 3, (const uint64_t*)h3, sb, 0,
                                (uint64_t)P.volume, scratch, 0, (double*)nullptr));
  TSA_TRACED("mad_finish", P.s,
             hipLaunchKernelGGL(k_mad_finish, dim3(1), dim3(64), 0, P.s, (const SelState*)med, (const SelState*)sb,
                                cube->dtype, d_out));
  return launch_ok();
}

}  // namespace tsa
