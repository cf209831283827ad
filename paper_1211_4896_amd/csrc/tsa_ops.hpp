// Per-element accumulators and block-level epilogues shared by the kernels.
#pragma once

#include <climits>

#include "tsa_device.hpp"

#ifndef TSA_BRANCHLESS
#define TSA_BRANCHLESS 0
#endif
#ifndef TSA_BALLOT_COUNT
#define TSA_BALLOT_COUNT 0
#endif

namespace tsa {

// ---- validity and key of one element ---------------------------------------
template <int DT>
struct Elt;
template <>
struct Elt<0> {
  TSA_DEV static bool valid(float x, bool in) { return in && (x == x); }
  TSA_DEV static uint32_t key(float x) { return key_f32(__float_as_uint(x)); }
  TSA_DEV static float val(float x) { return x; }
};
template <>
struct Elt<1> {
  TSA_DEV static bool valid(int16_t, bool in) { return in; }
  TSA_DEV static uint32_t key(int16_t x) { return key_i16(x); }
  TSA_DEV static float val(int16_t x) { return (float)x; }
};

// ---- moments (Section 4.2): count, min/max keys, sum and sum of squares -------
// NaN and masked lanes add 0.  COUNT = false: the caller supplies the count (a
// pass that also builds the first-digit histogram of the valid values has it
// as the histogram's total).
template <int DT, bool COUNT = true>
struct MomAcc;

// float32: per-lane running sums in double.  Each value and its square are
// exact in double (a float32 square needs 48 significand bits and lies in
// [2^-298, 2^256]), so every step rounds once, with relative error 2^-53.
// gfx950 issues double adds and fused multiply-adds at the single-precision
// rate, which makes this both cheaper and more accurate than float pairs
// carrying their rounding errors (TwoSum and FMA splits).
template <bool COUNT>
struct MomAcc<0, COUNT> {
  double s = 0.0, q = 0.0;
  uint32_t kmin = 0xFFFFFFFFu, kmax = 0u, cnt = 0u;
  TSA_DEV void operator()(float x, bool in) {
    const bool ok = Elt<0>::valid(x, in);
    const double v = (double)(ok ? x : 0.0f);
    s += v;
    q = __builtin_fma(v, v, q);
    const uint32_t k = Elt<0>::key(x);
    kmin = min(kmin, ok ? k : 0xFFFFFFFFu);
    kmax = max(kmax, ok ? k : 0u);
    if constexpr (COUNT) {
#if TSA_BALLOT_COUNT
      cnt += (uint32_t)__popcll(__ballot(ok));  // wave total, kept uniform (scalar unit)
#else
      cnt += ok ? 1u : 0u;
#endif
    }
  }
  TSA_DEV void chunk() {}
};

// int16: exact integer sums (|x| <= 32768, x^2 <= 2^30).
template <bool COUNT>
struct MomAcc<1, COUNT> {
  int64_t s = 0;
  uint64_t q = 0;
  uint32_t kmin = 0xFFFFFFFFu, kmax = 0u, cnt = 0u;
  TSA_DEV void operator()(int16_t x, bool in) {
    const int32_t v = in ? (int32_t)x : 0;
    s += v;
    q += (uint32_t)(v * v);
    const uint32_t k = key_i16(x);
    kmin = min(kmin, in ? k : 0xFFFFFFFFu);
    kmax = max(kmax, in ? k : 0u);
    if constexpr (COUNT) cnt += in ? 1u : 0u;
  }
  TSA_DEV void chunk() {}
};

// Chan et al.'s pairwise update of (n, mean, M2) (the O(1) combine of
// Section 4.2's partial sums).  A partial whose mean is infinite (it holds
// infinities) makes the merged mean the sum of the two means (+inf, -inf, or
// NaN when both signs occur) and the spread undefined (NaN).
TSA_DEV void chan_merge(double& na, double& ma, double& qa, double nb, double mb, double qb) {
  if (nb == 0.0) return;
  if (na == 0.0) {
    na = nb;
    ma = mb;
    qa = qb;
    return;
  }
  const double n = na + nb;
  if (!__builtin_isfinite(ma) || !__builtin_isfinite(mb)) {
    ma = ma + mb;
    qa = __builtin_nan("");
    na = n;
    return;
  }
  const double d = mb - ma;
  ma = ma + d * (nb / n);
  qa = qa + qb + d * d * (na * nb / n);
  na = n;
}

// (n, mean, M2) of one block partial, in double.  centered: the partial holds
// M2 and its mean about p.ref (tsa_moments' shifted lanes), returned here as
// the mean about ref0; else float32 partials hold the sums S and Q, int16
// partials exact integer sums.
TSA_DEV void partial_stats(const Partial& p, int dtype, double& n, double& m, double& q, bool centered = false,
                           double ref0 = 0.0) {
  n = (double)p.n;
  if (p.n == 0) {
    m = q = 0.0;
    return;
  }
  if (dtype == 0) {
    if (centered) {
      m = p.s + (p.ref - ref0);  // ref - ref0: two float32 values, exact in double
      q = p.q;
    } else {
      m = p.s / n;
      q = p.q - p.s * m;
    }
  } else {
    // exact n*Q - S^2 in 128-bit integers, then one rounding to double
    const __int128 num = (__int128)p.qi * (__int128)p.n - (__int128)p.si * (__int128)p.si;
    const int64_t hi = (int64_t)(num >> 64);
    const uint64_t lo = (uint64_t)num;
    m = (double)p.si / n;
    q = ((double)hi * 18446744073709551616.0 + (double)lo) / n;
  }
}

// float32, one pass, for the moments alone: every lane subtracts a shift c,
// its first finite valid value, before summing, and keeps sum (x - c) and
// sum (x - c)^2 in double.  x - c is exact in double (or within 2^-53 when
// the exponents lie more than 29 apart), so the lane's
// M2 = sum (x-c)^2 - (sum (x-c))^2 / n loses only the digits that
// (mean - c)^2 / var costs, where c is one of the lane's own values, instead
// of the (mean / std)^2 that unshifted sums of x and x^2 lose.  Infinities
// seen before the first finite value add +-inf either way (c stays 0 until
// then), so the shift is the same for every finite value of the lane.
struct ShiftMomAcc {
  double c = 0.0, s = 0.0, q = 0.0;
  uint32_t kmin = 0xFFFFFFFFu, kmax = 0u, cnt = 0u;
  bool have = false;
  TSA_DEV void operator()(float x, bool in) {
    const bool ok = Elt<0>::valid(x, in);
    const double v = (double)x;
    const bool take = !have && ok && __builtin_isfinite(x);
    c = take ? v : c;
    have = have || take;
    const double d = ok ? v - c : 0.0;
    s += d;
    q = __builtin_fma(d, d, q);
    const uint32_t k = Elt<0>::key(x);
    kmin = min(kmin, ok ? k : 0xFFFFFFFFu);
    kmax = max(kmax, ok ? k : 0u);
    cnt += ok ? 1u : 0u;
  }
  TSA_DEV void chunk() {}
};

// Reduce a block's lanes (fixed order) and store one Partial.
struct alignas(16) MomShared {
  double s[16], q[16], ref[16];
  int64_t si[16];
  uint64_t qi[16];
  uint32_t kmin[16], kmax[16];
  uint64_t cnt[16];
};

TSA_DEV double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);  // a + b == b + a: every lane ends equal
  return v;
}

template <bool COUNT>
TSA_DEV void block_store_partial(MomAcc<0, COUNT>& a, MomShared& sm, Partial* out) {
  const double s = wave_sum_f64(a.s), q = wave_sum_f64(a.q);
  const uint32_t kmin = wave_min_u32(a.kmin), kmax = wave_max_u32(a.kmax);
#if TSA_BALLOT_COUNT
  const uint64_t cnt = a.cnt;  // already the wave's total
#else
  const uint64_t cnt = wave_sum_u64(a.cnt);
#endif
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) {
    sm.s[w] = s;
    sm.q[w] = q;
    sm.kmin[w] = kmin;
    sm.kmax[w] = kmax;
    sm.cnt[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
    double bs = sm.s[0], bq = sm.q[0];
    uint32_t mn = sm.kmin[0], mx = sm.kmax[0];
    uint64_t n = sm.cnt[0];
    for (int i = 1; i < nw; ++i) {
      bs += sm.s[i];
      bq += sm.q[i];
      mn = min(mn, sm.kmin[i]);
      mx = max(mx, sm.kmax[i]);
      n += sm.cnt[i];
    }
    Partial p;
    p.n = n;
    p.kmin = mn;
    p.kmax = mx;
    p.s = bs;
    p.q = bq;
    p.si = 0;
    p.qi = 0;
    *out = p;
  }
}

template <bool COUNT>
TSA_DEV void block_store_partial(MomAcc<1, COUNT>& a, MomShared& sm, Partial* out) {
  const int64_t s = wave_sum_i64(a.s);
  const uint64_t q = wave_sum_u64(a.q);
  const uint32_t kmin = wave_min_u32(a.kmin), kmax = wave_max_u32(a.kmax);
  const uint64_t cnt = wave_sum_u64(a.cnt);
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) {
    sm.si[w] = s;
    sm.qi[w] = q;
    sm.kmin[w] = kmin;
    sm.kmax[w] = kmax;
    sm.cnt[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
    Partial p;
    p.n = 0;
    p.si = 0;
    p.qi = 0;
    p.kmin = 0xFFFFFFFFu;
    p.kmax = 0u;
    for (int i = 0; i < nw; ++i) {
      p.si += sm.si[i];
      p.qi += sm.qi[i];
      p.kmin = min(p.kmin, sm.kmin[i]);
      p.kmax = max(p.kmax, sm.kmax[i]);
      p.n += sm.cnt[i];
    }
    p.s = p.q = 0.0;
    *out = p;
  }
}

// Lanes of ShiftMomAcc: each lane's (n, mean, M2), then Chan merges down a
// fixed tree (lane i takes lane i + o, o = 32 .. 1), the block's waves in
// order.  Means are carried about one reference value, the shift of the
// wave's (then the block's) first lane that has one, so the differences of
// means the merge forms are exact to the spread's scale, not the mean's:
// with mean/std = 1e7 a mean rounded to its own ulp would already cost 1e-9
// of the spread.  The Partial holds (n, mean about ref, M2, ref) ("centered")
// and the key extremes.
TSA_DEV void block_store_centered(ShiftMomAcc& a, MomShared& sm, Partial* out) {
  const uint64_t have = __ballot(a.have);
  const double ref_w = have ? __shfl(a.c, __builtin_ctzll(have)) : 0.0;
  double n = (double)a.cnt, m = 0.0, m2 = 0.0;
  if (a.cnt) {
    const double r = a.s / n;
    m = (a.c - ref_w) + r;  // a.c - ref_w: two float32 values (or 0), exact in double
    m2 = a.q - a.s * r;
    if (m2 < 0.0) m2 = 0.0;  // rounding below zero; NaN (infinite values) stays
  }
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const double nb = __shfl_down(n, o), mb = __shfl_down(m, o), qb = __shfl_down(m2, o);
    if (lane < o) chan_merge(n, m, m2, nb, mb, qb);
  }
  const uint32_t kmin = wave_min_u32(a.kmin), kmax = wave_max_u32(a.kmax);
  if (lane == 0) {
    sm.s[w] = m;
    sm.q[w] = m2;
    sm.ref[w] = have ? ref_w : __builtin_nan("");  // NaN: no finite value in the wave
    sm.cnt[w] = (uint64_t)n;
    sm.kmin[w] = kmin;
    sm.kmax[w] = kmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
    double ref = 0.0;
    for (int i = nw - 1; i >= 0; --i)
      if (sm.ref[i] == sm.ref[i]) ref = sm.ref[i];
    double bn = 0.0, bm = 0.0, bq = 0.0;
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
    for (int i = 0; i < nw; ++i) {
      // a wave without a finite value has a non-finite mean whatever its shift
      const double sh = sm.ref[i] == sm.ref[i] ? sm.ref[i] - ref : 0.0;
      chan_merge(bn, bm, bq, (double)sm.cnt[i], sm.s[i] + sh, sm.q[i]);
      mn = min(mn, sm.kmin[i]);
      mx = max(mx, sm.kmax[i]);
    }
    Partial p;
    p.n = (uint64_t)bn;
    p.kmin = mn;
    p.kmax = mx;
    p.s = bm;
    p.q = bq;
    p.ref = ref;
    p.qi = 0;
    *out = p;
  }
}

// ---- second moment about a shift (two-pass form, fused path) ----------------
// sum (x - c)^2 in double: the difference of two float32 values is formed in
// double (exact unless their exponents lie more than 29 apart, then within
// 2^-53), so the squares carry no cancellation however large the mean is
// against the spread, and they stay inside [2^-298, 2^258].
struct VarAcc {
  float c;
  double q = 0.0;
  TSA_DEV void operator()(float x, bool in) {
    const bool ok = in && (x == x);
    const double d = (double)(ok ? x : c) - (double)c;  // masked lanes: d = 0
    q = __builtin_fma(d, d, q);
  }
  TSA_DEV void chunk() {}
};

TSA_DEV void block_store_var(VarAcc& a, MomShared& sm, Partial* out) {
  const double q = wave_sum_f64(a.q);
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) sm.q[w] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
    double bq = sm.q[0];
    for (int i = 1; i < nw; ++i) bq += sm.q[i];
    Partial p;
    p.n = 0;
    p.kmin = p.kmax = 0;
    p.s = 0.0;
    p.q = bq;
    p.si = 0;
    p.qi = 0;
    *out = p;
  }
}

// ---- |x - m| as the element (median absolute deviation) ----------------------
// Feeds an accumulator written for float elements with d = |x - m|: one IEEE
// single-precision subtraction for float32 cubes, exact for int16 cubes (the
// integer difference is at most 65535, exact in float).  A value equal to m
// deviates by +0, also when both are the same infinity (where the IEEE
// difference would be NaN), so every non-NaN voxel has a deviation.  NaN
// stays NaN.
template <int DT, class Inner>
struct AbsDev {
  Inner inner;
  float mf;
  int32_t mi;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    float d;
    if constexpr (DT == 0)
      d = ((float)raw == mf) ? 0.0f : fabsf((float)raw - mf);
    else
      d = (float)abs((int32_t)raw - mi);
    inner(d, in);
  }
  TSA_DEV void chunk() { inner.chunk(); }
};

// ---- LDS-privatised counters -------------------------------------------------
// Every LDS counter array is followed by kTrash spare words (one per lane of a
// wave) that branch-free increments of invalid lanes may hit; they are never read.
constexpr uint32_t kTrash = 64;

// Bin b, replica r lives at lds[(b << rshift) + r]; a lane uses replica
// (lane & (R-1)) so lanes of one wave that hit the same bin mostly touch
// different words.
TSA_DEV void lds_inc(uint32_t* lds, uint32_t idx) {
  __hip_atomic_fetch_add(lds + idx, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Increment for the lanes where m holds, rare across the wave: the wave skips
// the LDS instruction entirely when no lane needs it (an exec-masked LDS
// instruction with no active lane still takes an issue slot).
TSA_DEV void lds_inc_rare(uint32_t* lds, bool m, uint32_t idx) {
  if (__ballot(m) != 0ull) {
    if (m) lds_inc(lds, idx);
  }
}

TSA_DEV void lds_zero(uint32_t* lds, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) lds[i] = 0u;
}

// Sum the replicas of each bin and add the non-zero ones to global counters.
TSA_DEV void lds_flush(const uint32_t* lds, uint32_t nbins, uint32_t rshift, uint64_t* g) {
  const uint32_t R = 1u << rshift;
  for (uint32_t b = threadIdx.x; b < nbins; b += blockDim.x) {
    uint32_t c = 0;
    for (uint32_t r = 0; r < R; ++r) c += lds[(b << rshift) + r];
    if (c) atomicAdd((unsigned long long*)(g + b), (unsigned long long)c);
  }
}

// ---- histogram (Section 4.1) ---------------------------------------------------
struct HistAcc {
  uint32_t* lds;
  float lo, hi, scale;
  int32_t nbm1;
  uint32_t rshift, rep;
  uint32_t below = 0, above = 0;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    const float v = (float)raw;  // exact for int16
    below += (in && v < lo) ? 1u : 0u;
    above += (in && v > hi) ? 1u : 0u;
#if TSA_BRANCHLESS
    const float d = v - lo;
    const float t = d * scale;  // lo == hi: scale == 0 and t == 0
    const int32_t b = min(max((int32_t)t, 0), nbm1);
    // out-of-range and NaN lanes count into spare words past the bins
    const uint32_t idx = (in && v >= lo && v <= hi) ? ((uint32_t)b << rshift) + rep
                                                    : ((uint32_t)(nbm1 + 1) << rshift) + (threadIdx.x & 63u);
    lds_inc(lds, idx);
#else
    if (in && v >= lo && v <= hi) {  // NaN fails both tests
      const float d = v - lo;
      const float t = d * scale;  // lo == hi: scale == 0 and t == 0
      const int32_t b = min(max((int32_t)t, 0), nbm1);
      lds_inc(lds, ((uint32_t)b << rshift) + rep);
    }
#endif
  }
  TSA_DEV void chunk() {}
};

// Histogram over the values' own [min, max] (lo and hi are the extremes of the
// same values, both finite): every valid value is in range, so only NaN needs a
// test, (v - lo) * scale is never negative, and there are no outliers.  Gives
// the same bins as HistAcc for such a range.
struct HistOwnAcc {
  uint32_t* lds;
  float lo, scale;
  int32_t nbm1;
  uint32_t rshift, rep;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    const float v = (float)raw;  // exact for int16
    if (in && v == v) {
      const float t = (v - lo) * scale;  // lo == hi: scale == 0 and t == 0
      const int32_t b = min((int32_t)t, nbm1);
      lds_inc(lds, ((uint32_t)b << rshift) + rep);
    }
  }
  TSA_DEV void chunk() {}
};

// Histogram over the values' own [min, max] with more bins than LDS holds as
// 32-bit counters: a window of kWinBins bins [w0, w0 + kWinBins) is counted in
// LDS, bins outside it directly in the global counters (exact for any data;
// fast when the window holds most values).  Same bins as HistOwnAcc.
constexpr uint32_t kWinBins = 32768;
struct HistWinAcc {
  uint32_t* lds;
  float lo, scale;
  int32_t nbm1, w0;
  uint64_t* counts;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    const float v = (float)raw;  // exact for int16
    if (in && v == v) {
      const float t = (v - lo) * scale;
      const int32_t b = min((int32_t)t, nbm1);
      const uint32_t rel = (uint32_t)(b - w0);
      if (rel < kWinBins)
        lds_inc(lds, rel);
      else
        atomicAdd((unsigned long long*)(counts + b), 1ull);
    }
  }
  TSA_DEV void chunk() {}
};

// HistWinAcc for a caller's range [lo, hi]: values below lo and above hi are
// counted apart (as HistAcc counts them), in-range values in the window
// [w0, w0 + kWinBins) go to the LDS counters, the other in-range values to
// the global bins.
struct HistWinOutAcc {
  uint32_t* lds;
  float lo, hi, scale;
  int32_t nbm1, w0;
  uint64_t* counts;
  uint32_t below = 0, above = 0;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    const float v = (float)raw;  // exact for int16
    below += (in && v < lo) ? 1u : 0u;
    above += (in && v > hi) ? 1u : 0u;
    if (in && v >= lo && v <= hi) {  // NaN fails both tests
      const float t = (v - lo) * scale;  // lo == hi: scale == 0 and t == 0
      const int32_t b = min(max((int32_t)t, 0), nbm1);
      const uint32_t rel = (uint32_t)(b - w0);
      if (rel < kWinBins)
        lds_inc(lds, rel);
      else
        atomicAdd((unsigned long long*)(counts + b), 1ull);
    }
  }
  TSA_DEV void chunk() {}
};

// ---- histogram with 16-bit LDS counters (up to 65536 bins) ---------------------
// Bins [b0, b0+nb) live as 16-bit halves of LDS words; every `epoch` calls of
// chunk() the block adds its non-zero counters to the global uint64 bins and
// clears them, so no half can carry into its neighbour (the caller bounds the
// elements per epoch by 65535).
struct Hist16Acc {
  uint32_t* lds;
  float lo, hi, scale;
  int32_t nbm1, b0, nb;
  uint64_t* counts;
  uint32_t epoch, chunks;
  bool count_out;
  uint32_t below, above;

  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    const float v = (float)raw;
    if (count_out) {
      below += (in && v < lo) ? 1u : 0u;
      above += (in && v > hi) ? 1u : 0u;
    }
    if (in && v >= lo && v <= hi) {
      const float d = v - lo;
      const float t = d * scale;
      const int32_t b = min(max((int32_t)t, 0), nbm1);
      const uint32_t rel = (uint32_t)(b - b0);
      if (rel < (uint32_t)nb)
        __hip_atomic_fetch_add(lds + (rel >> 1), 1u << ((rel & 1u) * 16u), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  TSA_DEV void flush() {
    __syncthreads();
    const uint32_t words = ((uint32_t)nb + 1u) >> 1;
    for (uint32_t w = threadIdx.x; w < words; w += blockDim.x) {
      const uint32_t x = lds[w];
      if (x) {
        const uint32_t c0 = x & 0xFFFFu, c1 = x >> 16;
        if (c0) atomicAdd((unsigned long long*)(counts + b0 + 2 * w), (unsigned long long)c0);
        if (c1) atomicAdd((unsigned long long*)(counts + b0 + 2 * w + 1), (unsigned long long)c1);
        lds[w] = 0u;
      }
    }
    __syncthreads();
  }
  TSA_DEV void chunk() {
    if (++chunks == epoch) {
      chunks = 0;
      flush();
    }
  }
};

TSA_DEV void block_add_outliers(uint32_t below, uint32_t above, uint64_t* g, uint32_t* sm) {
  below = wave_sum_u32(below);
  above = wave_sum_u32(above);
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) {
    sm[2 * w] = below;
    sm[2 * w + 1] = above;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t b = 0, a = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
      b += sm[2 * i];
      a += sm[2 * i + 1];
    }
    if (b) atomicAdd((unsigned long long*)g, (unsigned long long)b);
    if (a) atomicAdd((unsigned long long*)(g + 1), (unsigned long long)a);
  }
}

// ---- digit selection and moment merges (whole block / one thread) -----------
// Block-wide choice of the digit holding rank k in a histogram of nb bins
// (u32 counts).  Returns false when k is not inside the histogram.  SH provides
// wsum[blockDim.x / 64], found, sel_digit, sel_cum and sel_bucket in LDS.
template <class SH>
TSA_DEV bool block_select_u32(const uint32_t* hist, int nb, uint64_t k, SH& sh, uint32_t* digit,
                              uint64_t* cum_before, uint64_t* bucket) {
  const int t = threadIdx.x, bs = blockDim.x;
  const int per = (nb + bs - 1) / bs;
  const int b0 = t * per;
  uint64_t local = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) local += hist[b0 + i];
  const int lane = t % kWave, w = t / kWave;
  uint64_t inc = local;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) sh.wsum[w] = inc;
  if (t == 0) sh.found = 0;
  __syncthreads();
  uint64_t base = inc - local;
  for (int i = 0; i < w; ++i) base += sh.wsum[i];
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
    sh.sel_digit = (uint32_t)d;
    sh.sel_cum = cum;
    sh.sel_bucket = hist[d];
    sh.found = 1;
  }
  __syncthreads();
  const bool found = sh.found != 0;
  *digit = sh.sel_digit;
  *cum_before = sh.sel_cum;
  *bucket = sh.sel_bucket;
  __syncthreads();
  return found;
}

// Wave-wide inclusive prefix sum of 32-bit values: Hillis-Steele steps of 1,
// 2, 4 and 8 lanes inside each row of 16 (DPP row shifts; a lane with no
// source adds 0), then lane 15 of rows 0 and 2 added to rows 1 and 3, then
// lane 31 added to rows 2 and 3 (DPP row broadcasts).
TSA_DEV uint32_t wave_scan_incl_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

// block_select_u32 for histograms whose total fits in 32 bits (a mini-map
// cell): 32-bit DPP scans instead of 64-bit shuffles, and every wave total
// read at once.  SH provides wsum32[16] (16-byte aligned), found, sel_digit, sel_cum32 and
// sel_bucket32 in LDS; blockDim.x is at most 1024.
template <class SH>
TSA_DEV bool block_select_small(const uint32_t* hist, int nb, uint32_t k, SH& sh, uint32_t* digit,
                                uint32_t* cum_before, uint32_t* bucket) {
  const int t = threadIdx.x, bs = blockDim.x;
  const int per = (nb + bs - 1) / bs;
  const int b0 = t * per;
  uint32_t local = 0;
  if ((per & (per - 1)) == 0) {  // a power of two: each run read from an offset rotated by t / 8,
    // so lanes whose runs start in the same bank read different banks (8 a run: none shared)
    for (int i = 0; i < per; ++i) {
      const int j = b0 + ((i + (t >> 3)) & (per - 1));
      if (j < nb) local += hist[j];
    }
  } else {
    for (int i = 0; i < per; ++i)
      if (b0 + i < nb) local += hist[b0 + i];
  }
  const int lane = t % kWave, w = t / kWave;
  const uint32_t inc = wave_scan_incl_u32(local);
  if (lane == kWave - 1) sh.wsum32[w] = inc;
  if (t == 0) sh.found = 0;
  __syncthreads();
  uint32_t base = inc - local;
  const uint4* ws4 = reinterpret_cast<const uint4*>(sh.wsum32);  // 16-byte aligned in SH
#pragma unroll
  for (int i = 0; i < 4; ++i) {  // waves below this one, four totals a read
    const uint4 v = ws4[i];
    base += (4 * i < w ? v.x : 0u) + (4 * i + 1 < w ? v.y : 0u) + (4 * i + 2 < w ? v.z : 0u) +
            (4 * i + 3 < w ? v.w : 0u);
  }
  if (local > 0 && k >= base && k - base < local) {
    uint32_t cum = base;
    int d = b0;
    for (int i = 0; i < per; ++i) {
      const uint32_t h = (b0 + i < nb) ? hist[b0 + i] : 0u;
      if (k - cum < h) {
        d = b0 + i;
        break;
      }
      cum += h;
    }
    sh.sel_digit = (uint32_t)d;
    sh.sel_cum32 = cum;
    sh.sel_bucket32 = hist[d];
    sh.found = 1;
  }
  __syncthreads();
  const bool found = sh.found != 0;
  *digit = sh.sel_digit;
  *cum_before = sh.sel_cum32;
  *bucket = sh.sel_bucket32;
  __syncthreads();
  return found;
}

TSA_DEV double bvalue_of_key(uint32_t k, int dtype) {
  return dtype == 0 ? (double)__uint_as_float(f32bits_of_key(k)) : (double)i16_of_key(k);
}

// ---- radix digits of the key (Section 4.3 replaced by radix selection) --------
template <int DT>
struct Digit1Acc {  // top 12 key bits of every valid element
  uint32_t* lds;
  uint32_t rshift, rep;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
#if TSA_BRANCHLESS
    // invalid lanes count into spare words past the bins (one per lane)
    const uint32_t idx = Elt<DT>::valid(raw, in) ? ((Elt<DT>::key(raw) >> kShift1) << rshift) + rep
                                                   : ((uint32_t)kBins1 << rshift) + (threadIdx.x & 63u);
    lds_inc(lds, idx);
#else
    if (Elt<DT>::valid(raw, in)) lds_inc(lds, ((Elt<DT>::key(raw) >> kShift1) << rshift) + rep);
#endif
  }
  TSA_DEV void chunk() {}
};

// Candidate keys are staged per wave in LDS and copied to the global list in
// runs of up to kWaveStage keys, so the global counter sees one atomic per run
// instead of one per wave instruction.  Each wave owns its stage: no block
// barrier is needed, so the block's waves keep their loads in flight.  The
// walkers call every accumulator from all lanes at the same points, so the
// wave's fill count is an ordinary variable that every lane updates alike
// (kept in a register, no LDS round trip per append).
// A copy-out waits for its global atomic, so a deeper stage (fewer copy-outs)
// pays where the LDS allows it.
constexpr uint32_t kWaveStage = 128;     // staged keys per wave (default)
constexpr uint32_t kWaveStageBig = 512;  // where the LDS has room
constexpr int kMaxWaves = 16;

// Staging of a block of NW waves, S keys each.
template <int NW, uint32_t S = kWaveStage>
struct CandSharedN {
  uint32_t buf[NW][S];
};
using CandShared = CandSharedN<kMaxWaves>;

struct CandSink {
  uint32_t* buf;      // `stage` staged keys per wave
  uint32_t* list;     // global list
  uint32_t* counter;  // global fill counter
  uint32_t cap;       // global capacity
  uint32_t stage;     // keys per wave the stage holds
  uint32_t fill;      // keys this wave has staged (equal in every lane)
};

template <int NW, uint32_t S>
TSA_DEV CandSink cand_sink(CandSharedN<NW, S>& cs, uint32_t* list, uint32_t* counter, uint32_t cap) {
  return CandSink{&cs.buf[0][0], list, counter, cap, S, 0u};
}

// Staging carved from dynamic LDS: `stage` words per wave of the block.
TSA_DEV CandSink cand_sink_lds(uint32_t* base, uint32_t stage, uint32_t* list, uint32_t* counter, uint32_t cap) {
  return CandSink{base, list, counter, cap, stage, 0u};
}

// The wave copies its `fill` staged keys out (one global atomic).  Whole wave.
TSA_DEV void cand_copy_out(const CandSink& k, uint32_t fill) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  __builtin_amdgcn_wave_barrier();  // the staged writes of every lane come first
  uint32_t g = 0;
  if (lane == 0) g = atomicAdd(k.counter, fill);
  g = __builtin_amdgcn_readfirstlane(g);  // lane 0's result, without an LDS permute
  for (uint32_t i = lane; i < fill; i += kWave)
    if (g + i < k.cap) k.list[g + i] = k.buf[w * k.stage + i];
  __builtin_amdgcn_wave_barrier();  // and the reads finish before the stage is refilled
}

// Wave-aggregated append of the lanes whose flag is set (bal = their ballot).
// Kept inline: an out-of-line call costs the element loops more than its
// code size saves (measured on the fused pass B).
TSA_DEV void cand_append_slow(bool m, uint32_t key, uint64_t bal, CandSink& k) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const uint32_t n = (uint32_t)__popcll(bal);
  if (k.fill + n > k.stage) {
    cand_copy_out(k, k.fill);
    k.fill = 0;
  }
  const uint32_t off = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
  if (m) k.buf[w * k.stage + k.fill + off] = key;
  k.fill += n;
}

TSA_DEV void cand_append(bool m, uint32_t key, CandSink& k) {
  const uint64_t bal = __ballot(m);
  if (bal != 0) cand_append_slow(m, key, bal, k);
}

// Whole block (blockDim.x at most 1024): every wave's still-staged keys
// copied out under one global reservation for the block.  One same-address
// atomic per block instead of one per wave: when a thousand blocks end
// together (a small cube, one unit of work each) their waves' reservations
// queued on the one counter for tens of microseconds.
TSA_DEV void cand_finish_block(CandSink& k) {
  __shared__ uint32_t fill_w[16];
  __shared__ uint32_t base_b;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  if (lane == 0) fill_w[w] = k.fill;
  __syncthreads();  // also orders every lane's staged writes before the copy
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int i = 0; i < nw; ++i) tot += fill_w[i];
    base_b = tot ? atomicAdd(k.counter, tot) : 0u;
  }
  __syncthreads();
  uint32_t g = base_b;
  for (int i = 0; i < w; ++i) g += fill_w[i];
  for (uint32_t i = lane; i < k.fill; i += kWave)
    if (g + i < k.cap) k.list[g + i] = k.buf[w * k.stage + i];
  k.fill = 0;
  __syncthreads();  // fill_w and base_b read by every wave before a later call rewrites them
}

template <int DT>
struct Level2Acc {  // keys inside the level-1 bucket: next 12 bits, optional copy
  uint32_t* lds;
  uint32_t p1;
  bool compact;
  CandSink sink;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    const uint32_t key = Elt<DT>::key(raw);
    const bool m = Elt<DT>::valid(raw, in) && (key >> kShift1) == p1;
    const uint64_t bal = __ballot(m);
    if (bal != 0ull) {  // rare: most waves skip both the count and the copy
      if (m) lds_inc(lds, (key >> kShift2) & 0xFFFu);
      if (compact) cand_append_slow(m, key, bal, sink);
    }
  }
  TSA_DEV void chunk() {}
  // what every wave still holds, one reservation for the block (call with
  // every thread of the block; compact is the same across the block)
  TSA_DEV void finish() {
    if (compact) cand_finish_block(sink);
  }
};

template <int DT>
struct Level3Acc {  // keys inside the level-2 bucket: last 8 bits
  uint32_t* lds;
  uint32_t p2;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    const uint32_t key = Elt<DT>::key(raw);
    lds_inc_rare(lds, Elt<DT>::valid(raw, in) && (key >> kShift2) == p2, key & 0xFFu);
  }
  TSA_DEV void chunk() {}
};

}  // namespace tsa
