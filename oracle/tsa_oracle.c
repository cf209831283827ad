/*
 * CPU oracle for the cube statistics -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this.  It shares no code with the GPU library and is deliberately
 * plain and slow: one loop per definition, in the order the definition reads.
 *
 * Paper: Hassan, Fluke, Barnes & Kilborn, "Tera-scale astronomical data
 * analysis and visualization", MNRAS (arXiv 1211.4896).
 *
 * Conventions (the paper leaves these open; the readings are listed with the
 * design notes of the project):
 *   - a NaN voxel is the paper's NULL value and is left out of every statistic
 *     (Section 4, the NULL-handling challenge);
 *   - +-inf are ordinary values;
 *   - order is IEEE-754 totalOrder restricted to non-NaN values, so -0 < +0;
 *   - a region is a half-open box [x0,x1) x [y0,y1) x [z0,z1); each voxel in
 *     it is visited once (Section 4, overlap exclusion);
 *   - layout is dense, x fastest: index = x + nx*(y + ny*z).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_F32 = 0, OR_I16 = 1 };

typedef struct {
  uint64_t count;     /* non-NaN voxels */
  uint64_t nan_count; /* NaN voxels */
  double mean;        /* (1/n) sum x */
  double m2;          /* sum (x - mean)^2 */
  double std;         /* sqrt(m2 / n), population form */
  double min, max;    /* under totalOrder */
} oracle_moments_t;

/* ---- region walk -------------------------------------------------------- */

typedef struct {
  int64_t x0, y0, z0, x1, y1, z1;
} obox;

static int box_ok(int64_t nx, int64_t ny, int64_t nz, const int64_t* b, obox* o) {
  if (!b) {
    o->x0 = o->y0 = o->z0 = 0;
    o->x1 = nx; o->y1 = ny; o->z1 = nz;
    return 1;
  }
  o->x0 = b[0]; o->y0 = b[1]; o->z0 = b[2]; o->x1 = b[3]; o->y1 = b[4]; o->z1 = b[5];
  if (o->x0 < 0 || o->y0 < 0 || o->z0 < 0) return 0;
  if (o->x1 > nx || o->y1 > ny || o->z1 > nz) return 0;
  if (o->x0 >= o->x1 || o->y0 >= o->y1 || o->z0 >= o->z1) return 0;
  return 1;
}

static double load(const void* data, int dtype, int64_t i) {
  if (dtype == OR_F32) return (double)((const float*)data)[i];
  return (double)((const int16_t*)data)[i];
}

/* totalOrder "a before b" for non-NaN doubles holding float or int16 values */
static int tot_less(double a, double b) {
  if (a < b) return 1;
  if (a > b) return 0;
  return signbit(a) && !signbit(b); /* equal values: only -0 before +0 */
}

/* Neumaier's improved Kahan-Babuska summation: s + c carries the running sum */
static void nsum_add(double* s, double* c, double x) {
  double t = *s + x;
  if (fabs(*s) >= fabs(x))
    *c += (*s - t) + x;
  else
    *c += (x - t) + *s;
  *s = t;
}

/*
 * Global mean and standard deviation (Section 4.2): the sum, the sum of squares
 * and the count of the non-NULL voxels.  Here the sum is taken in double with
 * Neumaier compensation, and the spread uses the corrected two-pass form
 * M2 = sum (x-m)^2 - (sum (x-m))^2 / n with m the pass-1 mean, which is the
 * same quantity as sum x^2 - (sum x)^2 / n without its cancellation.
 * min/max (Section 4.1: known at load time) are taken in the same pass.
 * Infinities: the sum of values holding +inf is +inf, holding -inf is -inf,
 * holding both is undefined, so the mean is +inf, -inf or NaN and the spread
 * is undefined (NaN).  A region whose valid values are all the same value
 * (an infinity included) has mean = that value and M2 = std = 0.
 * Returns 0, or -1 for an invalid region or dtype.
 */
int oracle_moments(const void* data, int dtype, int64_t nx, int64_t ny, int64_t nz,
                   const int64_t* box, oracle_moments_t* out) {
  obox B;
  if ((dtype != OR_F32 && dtype != OR_I16) || !box_ok(nx, ny, nz, box, &B)) return -1;
  uint64_t n = 0, nn = 0, npinf = 0, nminf = 0;
  double s = 0.0, c = 0.0, mn = NAN, mx = NAN;
  for (int64_t z = B.z0; z < B.z1; ++z)
    for (int64_t y = B.y0; y < B.y1; ++y)
      for (int64_t x = B.x0; x < B.x1; ++x) {
        double v = load(data, dtype, x + nx * (y + ny * z));
        if (v != v) {
          ++nn;
          continue;
        }
        if (n == 0) {
          mn = v;
          mx = v;
        } else {
          if (tot_less(v, mn)) mn = v;
          if (tot_less(mx, v)) mx = v;
        }
        ++n;
        if (isinf(v)) {
          if (v > 0) ++npinf; else ++nminf;
          continue;
        }
        nsum_add(&s, &c, v);
      }
  out->count = n;
  out->nan_count = nn;
  out->min = mn;
  out->max = mx;
  if (n == 0) {
    out->mean = out->m2 = out->std = NAN;
    return 0;
  }
  if (!tot_less(mn, mx)) { /* every valid value is the same value */
    out->mean = mn;
    out->m2 = out->std = 0.0;
    return 0;
  }
  if (npinf || nminf) {
    out->mean = (npinf && nminf) ? NAN : (npinf ? INFINITY : -INFINITY);
    out->m2 = out->std = NAN;
    return 0;
  }
  double mean = (s + c) / (double)n;
  double d_s = 0.0, d_c = 0.0, q_s = 0.0, q_c = 0.0;
  for (int64_t z = B.z0; z < B.z1; ++z)
    for (int64_t y = B.y0; y < B.y1; ++y)
      for (int64_t x = B.x0; x < B.x1; ++x) {
        double v = load(data, dtype, x + nx * (y + ny * z));
        if (v != v) continue;
        double d = v - mean;
        nsum_add(&d_s, &d_c, d);
        nsum_add(&q_s, &q_c, d * d);
      }
  double sd = d_s + d_c;
  double m2 = (q_s + q_c) - sd * sd / (double)n;
  if (m2 < 0.0) m2 = 0.0;
  out->mean = mean;
  out->m2 = m2;
  out->std = sqrt(m2 / (double)n);
  return 0;
}

/*
 * Histogram scale, computed once in single precision:
 *   scale = (float)nbins / (hi - lo).
 * Returns 0 and writes *scale, or -1 when lo/hi/nbins are not acceptable
 * (non-finite bounds, lo > hi, nbins outside [1, 65536], or a non-finite or
 * zero scale when lo < hi).  lo == hi is accepted; its scale is unused.
 */
int oracle_hist_scale(float lo, float hi, int32_t nbins, float* scale) {
  if (nbins < 1 || nbins > 65536) return -1;
  if (!isfinite(lo) || !isfinite(hi) || lo > hi) return -1;
  if (lo == hi) {
    *scale = 0.0f;
    return 0;
  }
  volatile float width = hi - lo;
  if (!isfinite(width)) return -1;
  volatile float sc = (float)nbins / width;
  if (!isfinite(sc) || sc == 0.0f) return -1;
  *scale = sc;
  return 0;
}

/*
 * Fixed-range N-bin histogram (Section 4.1), one visit per voxel.  For a
 * non-NaN value v (int16 converted to float exactly):
 *   v < lo -> outliers[0];  v > hi -> outliers[1];
 *   otherwise t = (v - lo) * scale in single precision (two IEEE operations,
 *   no fused multiply-add), b = (int)t (truncation), b = min(b, nbins-1),
 *   counts[b] += 1.  When lo == hi every v == lo lands in bin 0.
 * counts[nbins] and outliers[2] are overwritten.  Returns 0 or -1.
 */
int oracle_histogram(const void* data, int dtype, int64_t nx, int64_t ny, int64_t nz,
                     const int64_t* box, float lo, float hi, int32_t nbins, uint64_t* counts,
                     uint64_t* outliers) {
  obox B;
  float scale;
  if ((dtype != OR_F32 && dtype != OR_I16) || !box_ok(nx, ny, nz, box, &B)) return -1;
  if (oracle_hist_scale(lo, hi, nbins, &scale) != 0) return -1;
  memset(counts, 0, sizeof(uint64_t) * (size_t)nbins);
  outliers[0] = outliers[1] = 0;
  for (int64_t z = B.z0; z < B.z1; ++z)
    for (int64_t y = B.y0; y < B.y1; ++y)
      for (int64_t x = B.x0; x < B.x1; ++x) {
        int64_t i = x + nx * (y + ny * z);
        float v = dtype == OR_F32 ? ((const float*)data)[i] : (float)((const int16_t*)data)[i];
        if (v != v) continue;
        if (v < lo) {
          outliers[0]++;
          continue;
        }
        if (v > hi) {
          outliers[1]++;
          continue;
        }
        int32_t b;
        if (lo == hi) {
          b = 0;
        } else {
          volatile float d = v - lo; /* volatile: one rounding per operation */
          volatile float t = d * scale;
          b = (int32_t)t;
          if (b > nbins - 1) b = nbins - 1;
        }
        counts[b]++;
      }
  return 0;
}

/* ---- Torben's method (Appendix A, Algorithm 1) --------------------------- */

/* The guess of one iteration: midpoint of the bracket in single precision. */
float oracle_torben_guess(float mn, float mx) {
  volatile float s = mn + mx;
  volatile float g = s / 2.0f;
  return g;
}

/*
 * Torben Mogensen's median (Section 4.3; Appendix A).  Each iteration visits
 * every value once and classifies it against the guess as less, greater or
 * equal, keeping the largest value below and the smallest above the guess;
 * the bracket [Min, Max] then moves to one of those two values.  The half
 * count is the integer (n + 1) / 2, which makes the result the lower median.
 * Values are float32 (int16 converted exactly); NaN is dropped before the
 * loop, since both comparisons are false for it and it would be counted as
 * equal.  The arithmetic is single precision as in the paper's table of a
 * sample run.
 *
 * trace (optional, may be NULL) receives per iteration: guess, Min, Max,
 * less, greater, equal as doubles, at most trace_cap rows.
 * Returns the iteration count (>= 1), 0 when there is no non-NaN value
 * (*median = NaN), or -1 when the iteration cap is hit.
 */
int oracle_torben(const void* data, int dtype, int64_t n_all, float* median, double* trace,
                  int trace_cap) {
  float* v = (float*)malloc(sizeof(float) * (size_t)(n_all > 0 ? n_all : 1));
  int64_t n = 0;
  for (int64_t i = 0; i < n_all; ++i) {
    float f = dtype == OR_F32 ? ((const float*)data)[i] : (float)((const int16_t*)data)[i];
    if (f == f) v[n++] = f;
  }
  if (n == 0) {
    free(v);
    *median = NAN;
    return 0;
  }
  float mn = v[0], mx = v[0];
  for (int64_t i = 1; i < n; ++i) {
    if (v[i] < mn) mn = v[i];
    if (v[i] > mx) mx = v[i];
  }
  const int64_t half = (n + 1) / 2; /* integer division */
  int64_t less = 0, greater = 0, equal = 0;
  float guess = mn, maxltguess = mn, mingtguess = mx;
  int it = 0;
  for (;;) {
    if (it >= 4096) {
      free(v);
      return -1;
    }
    guess = oracle_torben_guess(mn, mx);
    less = greater = equal = 0;
    maxltguess = mn;
    mingtguess = mx;
    for (int64_t i = 0; i < n; ++i) {
      if (v[i] < guess) {
        less++;
        if (v[i] > maxltguess) maxltguess = v[i];
      } else if (v[i] > guess) {
        greater++;
        if (v[i] < mingtguess) mingtguess = v[i];
      } else {
        equal++;
      }
    }
    if (trace && it < trace_cap) {
      double* r = trace + 6 * it;
      r[0] = guess; r[1] = mn; r[2] = mx;
      r[3] = (double)less; r[4] = (double)greater; r[5] = (double)equal;
    }
    ++it;
    if (less <= half && greater <= half) break;
    if (less > greater)
      mx = maxltguess;
    else
      mn = mingtguess;
  }
  if (less >= half)
    *median = maxltguess;
  else if (less + equal >= half)
    *median = guess;
  else
    *median = mingtguess;
  free(v);
  return it;
}

/* ---- lower median by sorting (small inputs) ------------------------------ */

static int cmp_total(const void* pa, const void* pb) {
  double a = *(const double*)pa, b = *(const double*)pb;
  if (tot_less(a, b)) return -1;
  if (tot_less(b, a)) return 1;
  return 0;
}

/*
 * Lower median by its definition: sort the non-NaN values of the region by
 * totalOrder and take the one at 0-based rank floor((n-1)/2).  O(n log n) via
 * qsort; meant for small inputs.  Writes NaN when n == 0.  Returns 0 or -1.
 */
int oracle_median_sort(const void* data, int dtype, int64_t nx, int64_t ny, int64_t nz,
                       const int64_t* box, double* median, uint64_t* count) {
  obox B;
  if ((dtype != OR_F32 && dtype != OR_I16) || !box_ok(nx, ny, nz, box, &B)) return -1;
  int64_t vol = (B.x1 - B.x0) * (B.y1 - B.y0) * (B.z1 - B.z0);
  double* v = (double*)malloc(sizeof(double) * (size_t)vol);
  int64_t n = 0;
  for (int64_t z = B.z0; z < B.z1; ++z)
    for (int64_t y = B.y0; y < B.y1; ++y)
      for (int64_t x = B.x0; x < B.x1; ++x) {
        double f = load(data, dtype, x + nx * (y + ny * z));
        if (f == f) v[n++] = f;
      }
  *count = (uint64_t)n;
  if (n == 0) {
    *median = NAN;
  } else {
    qsort(v, (size_t)n, sizeof(double), cmp_total);
    *median = v[(n - 1) / 2];
  }
  free(v);
  return 0;
}
