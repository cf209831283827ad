// 3-D spectrum tool (Section 4.4): data profiles along arbitrary rays through
// the resident cube, sampled at a constant step with trilinear interpolation.
//
// One lane per sample; a block takes 256 consecutive samples of one ray, so
// the lanes of a wave read neighbouring voxels and the eight corner loads of
// successive samples hit the same cache lines.  Positions and weights are
// formed in double exactly as the header states, so the result does not
// depend on the launch shape.
#include <math.h>

#include "tsa_internal.hpp"

namespace tsa {
namespace {

constexpr int kSpecBlock = 256;

struct SpecArgs {
  const void* base;
  int64_t nx, ny, nz;
  const double* rays;  // nrays x (ox, oy, oz, sx, sy, sz)
  double* out;         // nrays x nsamples
  int64_t nsamples;
  int64_t blocks_per_ray;
};

// Lower corner, fraction and upper corner of coordinate p (inside [0, n-1]).
TSA_DEV void axis_cell(double p, int64_t n, int64_t& i0, double& f, int64_t& i1) {
  i0 = (int64_t)floor(p);
  if (n >= 2) {
    if (i0 > n - 2) i0 = n - 2;
  } else {
    i0 = 0;
  }
  f = p - (double)i0;
  i1 = i0 + 1 < n ? i0 + 1 : n - 1;
}

template <int DT>
TSA_DEV double voxel(const void* base, int64_t idx) {
  if constexpr (DT == 0)
    return (double)((const float*)base)[idx];
  else
    return (double)((const int16_t*)base)[idx];
}

template <int DT>
__global__ __launch_bounds__(kSpecBlock) void k_spectrum(SpecArgs a) {
  const int64_t ray = (int64_t)blockIdx.x / a.blocks_per_ray;
  const int64_t i = ((int64_t)blockIdx.x % a.blocks_per_ray) * kSpecBlock + threadIdx.x;
  if (i >= a.nsamples) return;
  const double* r = a.rays + 6 * ray;
  const double di = (double)i;
  const double px = r[0] + di * r[3];
  const double py = r[1] + di * r[4];
  const double pz = r[2] + di * r[5];
  double res = __builtin_nan("");
  if (px >= 0.0 && px <= (double)(a.nx - 1) && py >= 0.0 && py <= (double)(a.ny - 1) && pz >= 0.0 &&
      pz <= (double)(a.nz - 1)) {
    int64_t x0, x1, y0, y1, z0, z1;
    double fx, fy, fz;
    axis_cell(px, a.nx, x0, fx, x1);
    axis_cell(py, a.ny, y0, fy, y1);
    axis_cell(pz, a.nz, z0, fz, z1);
    const int64_t xs[2] = {x0, x1};
    const int64_t rows[4] = {(z0 * a.ny + y0) * a.nx, (z0 * a.ny + y1) * a.nx, (z1 * a.ny + y0) * a.nx,
                             (z1 * a.ny + y1) * a.nx};
    const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
    // Issue every corner load before the weighted sum (latency overlap).
    double v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = voxel<DT>(a.base, rows[c >> 1] + xs[c & 1]);
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double w = (wx[c & 1] * wy[(c >> 1) & 1]) * wz[c >> 2];
      if (w != 0.0) acc = acc + w * v[c];
    }
    res = acc;
  }
  a.out[ray * a.nsamples + i] = res;
}

}  // namespace

int run_spectrum(const tsa_cube* cube, const double* d_rays, int32_t nrays, int32_t nsamples, double* d_out,
                 tsa_stream_t stream) {
  int st = check_cube(cube);
  if (st) return st;
  if (nrays < 0 || nsamples < 0) return TSA_EINVAL;
  if (nrays == 0 || nsamples == 0) return TSA_OK;
  if (!d_rays || !d_out) return TSA_EINVAL;
  const int64_t bpr = ((int64_t)nsamples + kSpecBlock - 1) / kSpecBlock;
  const int64_t blocks = bpr * nrays;
  if (blocks > (int64_t)(1u << 31) / kSpecBlock) return TSA_EINVAL;  // grid limit
  hipStream_t s = (hipStream_t)stream;
  SpecArgs a;
  a.base = cube->data;
  a.nx = cube->nx;
  a.ny = cube->ny;
  a.nz = cube->nz;
  a.rays = d_rays;
  a.out = d_out;
  a.nsamples = nsamples;
  a.blocks_per_ray = bpr;
  if (cube->dtype == TSA_F32)
    TSA_TRACED("spectrum", s, hipLaunchKernelGGL(k_spectrum<0>, dim3((uint32_t)blocks), dim3(kSpecBlock), 0, s, a));
  else
    TSA_TRACED("spectrum", s, hipLaunchKernelGGL(k_spectrum<1>, dim3((uint32_t)blocks), dim3(kSpecBlock), 0, s, a));
  return hipGetLastError() == hipSuccess ? TSA_OK : TSA_EDEVICE;
}

}  // namespace tsa

extern "C" int tsa_spectrum(const tsa_cube* cube, const double* d_rays, int32_t nrays, int32_t nsamples,
                            double* d_out, tsa_stream_t stream) {
  return tsa::run_spectrum(cube, d_rays, nrays, nsamples, d_out, stream);
}
