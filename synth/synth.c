/*
 * Seeded synthetic image cubes: the stand-in for the paper's HI survey cubes
 * (HIPASS and its replications, Table 2 of Section 5; the LMC cube of Table 1).
 *
 * This module only makes inputs. It holds none of the statistics' arithmetic,
 * and both the GPU path and the CPU oracle consume its output unchanged.
 *
 * Layout: dense, x fastest, index = x + nx*(y + ny*z)  (RA, Dec, frequency).
 *
 * Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: draw i of stream s is mix(key_s + (i+1)*gamma), with key_s derived
 * from the user seed and a fixed stream tag.  Every voxel's noise therefore
 * depends only on (seed, voxel index), so any z-chunking and any thread count
 * give the same bytes.
 *
 * Cube recipe (float32):
 *   1. noise: N(0,1) by the Box-Muller transform on draw pairs (2j, 2j+1) of
 *      the noise stream; voxel 2j takes the cosine branch, 2j+1 the sine one;
 *   2. sources: S 3-D Gaussians A*exp(-r^2/(2 sigma^2)) truncated at r <= 4
 *      sigma, added in source-index order, each addition done in double and
 *      rounded back to float;
 *   3. NULL voxels: axis-aligned slabs 1-4 voxels thick along a random axis,
 *      extents of at least a quarter of the cube in the other two, added until
 *      their summed volume reaches the requested NaN fraction (a slab that would
 *      overshoot it by more than 10% is redrawn).  NaN is written last.
 * Cube recipe (int16): value U[-32768, 32767] from the noise stream, plus
 * sources with integer-rounded amplitudes summed in int32, then saturated.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t tag) {
  return mix64(seed * GAMMA + tag * 0xD1B54A32D192ED03ull + 0x1234567ull);
}

static inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GAMMA); }

/* uniform in (0, 1] with 53 random bits */
static inline double unit_open0(uint64_t r) { return ((double)(r >> 11) + 1.0) * 0x1.0p-53; }
/* uniform in [0, 1) */
static inline double unit(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

enum { TAG_NOISE = 1, TAG_SRC = 2, TAG_NAN = 3 };

typedef struct {
  double cx, cy, cz, amp, sigma;
} source_t;

typedef struct {
  int64_t x0, y0, z0, x1, y1, z1;
} box_t;

typedef struct {
  int64_t nx, ny, nz;
  uint64_t seed;
  int64_t n_sources;
  double amp_lo, amp_hi;
  int amp_log; /* 0: uniform amplitude, 1: log-uniform */
  double sig_lo, sig_hi;
  double nan_frac;
  int dtype; /* 0 f32, 1 i16 */
} synth_cfg;

static void make_sources(const synth_cfg* c, source_t* s) {
  uint64_t key = stream_key(c->seed, TAG_SRC);
  for (int64_t i = 0; i < c->n_sources; ++i) {
    uint64_t b = (uint64_t)i * 5;
    s[i].cx = unit(draw(key, b + 0)) * (double)c->nx;
    s[i].cy = unit(draw(key, b + 1)) * (double)c->ny;
    s[i].cz = unit(draw(key, b + 2)) * (double)c->nz;
    double u = unit(draw(key, b + 3));
    if (c->amp_log)
      s[i].amp = exp(log(c->amp_lo) + u * (log(c->amp_hi) - log(c->amp_lo)));
    else
      s[i].amp = c->amp_lo + u * (c->amp_hi - c->amp_lo);
    s[i].sigma = c->sig_lo + unit(draw(key, b + 4)) * (c->sig_hi - c->sig_lo);
  }
}

static int64_t rand_range(uint64_t key, uint64_t* ctr, int64_t lo, int64_t hi) {
  /* integer uniform in [lo, hi] */
  uint64_t span = (uint64_t)(hi - lo + 1);
  uint64_t r = draw(key, (*ctr)++);
  return lo + (int64_t)(r % span);
}

/* Returns the number of slabs written to out (at most cap). */
static int64_t make_slabs(const synth_cfg* c, box_t* out, int64_t cap) {
  if (c->nan_frac <= 0.0) return 0;
  uint64_t key = stream_key(c->seed, TAG_NAN);
  uint64_t ctr = 0;
  double N = (double)c->nx * (double)c->ny * (double)c->nz;
  double target = c->nan_frac * N, vol = 0.0;
  int64_t dims[3] = {c->nx, c->ny, c->nz};
  int64_t k = 0, skipped = 0;
  while (vol < target && k < cap) {
    int axis = (int)rand_range(key, &ctr, 0, 2);
    int64_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      int64_t ext;
      if (a == axis) {
        int64_t t = rand_range(key, &ctr, 1, 4);
        ext = t < dims[a] ? t : dims[a];
      } else {
        int64_t mn = dims[a] / 4 > 0 ? dims[a] / 4 : 1;
        ext = rand_range(key, &ctr, mn, dims[a]);
      }
      int64_t o = rand_range(key, &ctr, 0, dims[a] - ext);
      lo[a] = o;
      hi[a] = o + ext;
    }
    double v = (double)(hi[0] - lo[0]) * (double)(hi[1] - lo[1]) * (double)(hi[2] - lo[2]);
    /* a slab that would overshoot the target by more than 10% is redrawn (bounded) */
    if (vol + v > 1.1 * target && skipped < 256) {
      ++skipped;
      continue;
    }
    out[k].x0 = lo[0]; out[k].y0 = lo[1]; out[k].z0 = lo[2];
    out[k].x1 = hi[0]; out[k].y1 = hi[1]; out[k].z1 = hi[2];
    vol += v;
    ++k;
  }
  return k;
}

typedef struct {
  const synth_cfg* c;
  const source_t* src;
  const box_t* slabs;
  int64_t nslabs;
  int64_t z0, z1;   /* slices this worker writes (global z) */
  int64_t zbase;    /* global z of out[0] */
  void* out;
  int64_t nan_count;
} job_t;

static void noise_f32(const synth_cfg* c, float* out, int64_t g0, int64_t g1) {
  /* global voxel indices [g0, g1) */
  uint64_t key = stream_key(c->seed, TAG_NOISE);
  int64_t i = g0;
  while (i < g1) {
    int64_t j = i >> 1;
    double u1 = unit_open0(draw(key, (uint64_t)(2 * j)));
    double u2 = unit(draw(key, (uint64_t)(2 * j + 1)));
    double r = sqrt(-2.0 * log(u1));
    double th = 6.283185307179586 * u2;
    if ((i & 1) == 0) {
      out[i - g0] = (float)(r * cos(th));
      if (i + 1 < g1) out[i + 1 - g0] = (float)(r * sin(th));
      i += 2;
    } else {
      out[i - g0] = (float)(r * sin(th));
      i += 1;
    }
  }
}

static void noise_i16(const synth_cfg* c, int32_t* out, int64_t g0, int64_t g1) {
  uint64_t key = stream_key(c->seed, TAG_NOISE);
  for (int64_t i = g0; i < g1; ++i) out[i - g0] = (int32_t)(draw(key, (uint64_t)i) % 65536u) - 32768;
}

static void* worker(void* arg) {
  job_t* J = (job_t*)arg;
  const synth_cfg* c = J->c;
  int64_t plane = c->nx * c->ny;
  int64_t nz = J->z1 - J->z0;
  if (nz <= 0) return NULL;
  int64_t g0 = J->z0 * plane, g1 = J->z1 * plane;
  int32_t* acc = NULL;
  float* f = NULL;
  if (c->dtype == 0) {
    f = (float*)J->out + (J->z0 - J->zbase) * plane;
    noise_f32(c, f, g0, g1);
  } else {
    acc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g1 - g0));
    noise_i16(c, acc, g0, g1);
  }
  /* sources, in index order */
  for (int64_t s = 0; s < c->n_sources; ++s) {
    const source_t* S = &J->src[s];
    double R = 4.0 * S->sigma;
    int64_t zlo = (int64_t)ceil(S->cz - R), zhi = (int64_t)floor(S->cz + R);
    if (zlo < J->z0) zlo = J->z0;
    if (zhi > J->z1 - 1) zhi = J->z1 - 1;
    if (zlo > zhi) continue;
    int64_t ylo = (int64_t)ceil(S->cy - R), yhi = (int64_t)floor(S->cy + R);
    int64_t xlo = (int64_t)ceil(S->cx - R), xhi = (int64_t)floor(S->cx + R);
    if (ylo < 0) ylo = 0;
    if (yhi > c->ny - 1) yhi = c->ny - 1;
    if (xlo < 0) xlo = 0;
    if (xhi > c->nx - 1) xhi = c->nx - 1;
    double inv2s2 = 1.0 / (2.0 * S->sigma * S->sigma);
    double amp_i = c->dtype == 1 ? nearbyint(S->amp) : S->amp;
    for (int64_t z = zlo; z <= zhi; ++z) {
      double dz = (double)z - S->cz;
      for (int64_t y = ylo; y <= yhi; ++y) {
        double dy = (double)y - S->cy;
        for (int64_t x = xlo; x <= xhi; ++x) {
          double dx = (double)x - S->cx;
          double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 > R * R) continue;
          double g = exp(-r2 * inv2s2);
          int64_t li = (z - J->z0) * plane + y * c->nx + x;
          if (c->dtype == 0)
            f[li] = (float)((double)f[li] + S->amp * g);
          else
            acc[li] += (int32_t)nearbyint(amp_i * g);
        }
      }
    }
  }
  if (c->dtype == 1) {
    int16_t* o = (int16_t*)J->out + (J->z0 - J->zbase) * plane;
    for (int64_t i = 0; i < g1 - g0; ++i) {
      int32_t v = acc[i];
      o[i] = (int16_t)(v > 32767 ? 32767 : (v < -32768 ? -32768 : v));
    }
    free(acc);
    return NULL;
  }
  /* NULL slabs, written last */
  int64_t cnt = 0;
  const float qnan = __builtin_nanf("");
  for (int64_t k = 0; k < J->nslabs; ++k) {
    const box_t* B = &J->slabs[k];
    int64_t za = B->z0 > J->z0 ? B->z0 : J->z0;
    int64_t zb = B->z1 < J->z1 ? B->z1 : J->z1;
    for (int64_t z = za; z < zb; ++z)
      for (int64_t y = B->y0; y < B->y1; ++y) {
        float* row = f + (z - J->z0) * plane + y * c->nx;
        for (int64_t x = B->x0; x < B->x1; ++x) row[x] = qnan;
      }
  }
  for (int64_t i = 0; i < g1 - g0; ++i) cnt += (f[i] != f[i]);
  J->nan_count = cnt;
  return NULL;
}

/*
 * Fill out[] with slices [z0, z1) of the cube described by the arguments.
 * out holds (z1-z0)*nx*ny elements of float (dtype 0) or int16 (dtype 1).
 * Returns the number of NaN voxels written, or -1 on bad arguments.
 */
int64_t synth_cube(int64_t nx, int64_t ny, int64_t nz, uint64_t seed, int64_t n_sources,
                   double amp_lo, double amp_hi, int amp_log, double sig_lo, double sig_hi,
                   double nan_frac, int dtype, int64_t z0, int64_t z1, void* out, int threads) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || z0 < 0 || z1 > nz || z0 > z1 || !out) return -1;
  if (dtype != 0 && dtype != 1) return -1;
  synth_cfg c = {nx, ny, nz, seed, n_sources, amp_lo, amp_hi, amp_log, sig_lo, sig_hi, nan_frac, dtype};
  source_t* src = (source_t*)malloc(sizeof(source_t) * (size_t)(n_sources > 0 ? n_sources : 1));
  make_sources(&c, src);
  int64_t cap = 1 << 22;
  box_t* slabs = (box_t*)malloc(sizeof(box_t) * (size_t)cap);
  int64_t nslabs = dtype == 0 ? make_slabs(&c, slabs, cap) : 0;
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  int64_t nzc = z1 - z0;
  if (threads > nzc) threads = (int)(nzc > 0 ? nzc : 1);
  pthread_t th[256];
  job_t jobs[256];
  for (int t = 0; t < threads; ++t) {
    jobs[t].c = &c;
    jobs[t].src = src;
    jobs[t].slabs = slabs;
    jobs[t].nslabs = nslabs;
    jobs[t].z0 = z0 + nzc * t / threads;
    jobs[t].z1 = z0 + nzc * (t + 1) / threads;
    jobs[t].zbase = z0;
    jobs[t].out = out;
    jobs[t].nan_count = 0;
  }
  for (int t = 1; t < threads; ++t) pthread_create(&th[t], NULL, worker, &jobs[t]);
  worker(&jobs[0]);
  for (int t = 1; t < threads; ++t) pthread_join(th[t], NULL);
  int64_t nan_count = 0;
  for (int t = 0; t < threads; ++t) nan_count += jobs[t].nan_count;
  free(src);
  free(slabs);
  return nan_count;
}
