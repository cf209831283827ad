// Device-side building blocks for the cube-statistics kernels (gfx950).
//
// Everything here runs on CDNA4 wave64: 16-byte global loads, wave
// reductions by cross-lane shuffles, LDS-privatised counters, and
// order-preserving 32-bit keys for the median's radix selection.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define TSA_DEV __device__ __forceinline__

namespace tsa {

constexpr int kWave = 64;

// ---- radix digits of the 32-bit key: 12 + 12 + 8 bits --------------------
constexpr int kShift1 = 20, kShift2 = 8;
constexpr int kBins1 = 4096, kBins2 = 4096, kBins3 = 256;

// Whether the one-pass M2 = Q - S^2/n can miss the stated accuracy: its
// relative error grows with 1 + mean^2/var (cancellation), so past
// mean^2 > 9 var the second moment is recomputed about the mean.  Squares of
// float32 values lie in [2^-298, 2^256] and never leave the double range.
TSA_DEV bool one_pass_m2_at_risk(double mean, double var1) {
  return !(var1 > 0.0) || mean * mean > 9.0 * var1;
}

// ---- order-preserving keys -------------------------------------------------
// float32: flip all bits of negatives, set the sign bit of non-negatives, so
// unsigned key order is IEEE totalOrder (-0 < +0; NaN never reaches a key).
TSA_DEV uint32_t key_f32(uint32_t u) { return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u); }
TSA_DEV uint32_t f32bits_of_key(uint32_t k) { return (k & 0x80000000u) ? (k ^ 0x80000000u) : ~k; }
// int16: offset binary in the top 16 bits (the low 16 bits are zero).
TSA_DEV uint32_t key_i16(int32_t v) { return ((uint32_t)(v & 0xFFFF) ^ 0x8000u) << 16; }
TSA_DEV int32_t i16_of_key(uint32_t k) { return (int32_t)(int16_t)(uint16_t)((k >> 16) ^ 0x8000u); }

// ---- 32-bit division by an invariant divisor (multiply-high + shifts) ------
struct Magic {
  uint32_t m, s1, s2;
};
TSA_DEV uint32_t mdiv(uint32_t n, const Magic& g) {
  uint32_t t = __umulhi(n, g.m);
  return (t + ((n - t) >> g.s1)) >> g.s2;
}
// The constants of mdiv for divisor d >= 1, computed on the device.
TSA_DEV Magic dev_magic(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < (uint64_t)d) ++l;
  Magic g;
  g.m = (uint32_t)((((1ull << 32) * ((1ull << l) - (uint64_t)d)) / (uint64_t)d) + 1ull);
  g.s1 = l ? 1u : 0u;
  g.s2 = l ? l - 1u : 0u;
  return g;
}

// ---- element types ---------------------------------------------------------
template <int DT>
struct Ty;
template <>
struct Ty<0> {  // float32
  using T = float;
  static constexpr int EPV = 4;  // elements per 16-byte vector
  TSA_DEV static T get(const uint4& r, int e) {
    return __uint_as_float(e == 0 ? r.x : e == 1 ? r.y : e == 2 ? r.z : r.w);
  }
};
template <>
struct Ty<1> {  // int16
  using T = int16_t;
  static constexpr int EPV = 8;
  TSA_DEV static T get(const uint4& r, int e) {
    uint32_t w = (e >> 1) == 0 ? r.x : (e >> 1) == 1 ? r.y : (e >> 1) == 2 ? r.z : r.w;
    return (int16_t)((e & 1) ? (w >> 16) : (w & 0xFFFFu));
  }
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
TSA_DEV uint4 load16(const uint4* p) {
  const u32x4* q = (const u32x4*)p;
  u32x4 v;
  if constexpr (NT)
    v = __builtin_nontemporal_load(q);
  else
    v = *q;
  uint4 r;
  r.x = v.x;
  r.y = v.y;
  r.z = v.z;
  r.w = v.w;
  return r;
}

// ---- wave / block reductions -------------------------------------------------
TSA_DEV uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
TSA_DEV uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
TSA_DEV uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor(v, o));
  return v;
}
TSA_DEV uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o));
  return v;
}
TSA_DEV int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ---- per-block moment partial ------------------------------------------------
// float32 cubes: double sums s = sum x, q = sum x^2 (or of squared deviations);
// int16 cubes: exact integer sums si, qi.  Keys give min/max.
struct Partial {
  uint64_t n;
  uint32_t kmin, kmax;
  double s, q;  // float32: sums S and Q, or (centered) the mean about ref and M2
  union {
    int64_t si;  // int16: exact sum
    double ref;  // centered float32: the value the mean is taken about
  };
  uint64_t qi;  // int16: exact sum of squares
};
static_assert(sizeof(Partial) == 48, "partial layout");

// Median selection state kept in device workspace between kernels.
struct SelState {
  uint64_t n;         // valid voxels
  uint64_t k;         // rank still to find inside the current bucket
  uint64_t bucket_n;  // voxels in the current bucket
  uint32_t prefix;    // key bits fixed so far (top-aligned)
  uint32_t level;     // digits selected so far (0..3)
  uint32_t compact;   // 1: level 2 copies the bucket's keys to the candidate list
  uint32_t done;      // 1: result_key is final (or n == 0)
  uint32_t result_key;
  uint32_t ncand;     // candidates appended (atomic)
  uint32_t cand_cap;  // capacity of the candidate list
  uint32_t hist_ok;   // fused path: histogram range valid
  float lo, hi, scale;
  float shift;        // fused path: fl32(mean) that pass B subtracts before squaring
  uint32_t var_on;    // fused path: pass B recomputes M2 about `shift`
  uint32_t pad0;
  double q;           // rank_mode 1: the rank is floor(q (n - 1))
  uint32_t rank_mode; // 0: lower median, 1: quantile q
  uint32_t levels;    // digits to select before stopping (3 = exact)
  int32_t win0;       // fused path, many bins: first bin of the LDS window
  uint32_t pad;
};
static_assert(sizeof(SelState) == 104, "state layout");

}  // namespace tsa
