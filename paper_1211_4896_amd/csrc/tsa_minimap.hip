// Statistical mini-map (Section 4.5): the cube cut into a regular grid of
// cells, each summarised by the statistics of a region query, and the local
// threshold built from it: per cell, how many voxels lie above the cell's
// mean + k standard deviations.
//
// The cell statistics are a region batch over the grid's boxes (planned on
// the device, so no box list crosses PCIe).  The threshold pass streams the
// cube once in row order: a block owns a band of rows that share one cell row
// (fixed y and z cell index) and a chunk of up to 4096 columns, so every lane
// keeps its columns' thresholds and counters in registers for the whole band
// and no per-voxel division or lookup is needed.
#include <math.h>

#include "tsa_internal.hpp"

namespace tsa {

size_t batch_ws_bytes(const tsa_cube* cube, int32_t nbins, int32_t nq);
int run_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                     tsa_result* d_results, uint64_t* d_hists, const tsa_tune* tune, void* d_ws, size_t ws_bytes,
                     tsa_stream_t stream);

namespace {

constexpr int kMaxCells = 65536;  // the region batch's query limit
constexpr int kSigBlock = 256;
constexpr int kSigPos = 4;                                // element groups per lane per row
constexpr int kSigEPL = 4;                                // elements per group
constexpr int kSigChunk = kSigBlock * kSigPos * kSigEPL;  // 4096 columns per block
constexpr int kSigRows = 128;                             // rows per block, at most
constexpr int kSigUnroll = 4;                             // rows loaded together

struct Grid {
  int64_t ncx, ncy, ncz, ncells;
};

int grid_of(const tsa_cube* cube, int32_t cx, int32_t cy, int32_t cz, Grid* g) {
  int st = check_cube(cube);
  if (st) return st;
  if (cx < 1 || cy < 1 || cz < 1) return TSA_EINVAL;
  g->ncx = (cube->nx + cx - 1) / cx;
  g->ncy = (cube->ny + cy - 1) / cy;
  g->ncz = (cube->nz + cz - 1) / cz;
  const double nc = (double)g->ncx * (double)g->ncy * (double)g->ncz;
  if (nc > kMaxCells) return TSA_EINVAL;
  g->ncells = g->ncx * g->ncy * g->ncz;
  // Every cell must stay below 2^32 voxels (the region batch's box limit).
  const double cell_vox = (double)(cx < cube->nx ? cx : cube->nx) * (double)(cy < cube->ny ? cy : cube->ny) *
                          (double)(cz < cube->nz ? cz : cube->nz);
  if (cell_vox >= 4294967296.0) return TSA_EINVAL;
  return TSA_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

__global__ void k_grid_plan(tsa_region* __restrict__ boxes, int64_t nx, int64_t ny, int64_t nz, int32_t cx,
                            int32_t cy, int32_t cz, int64_t ncx, int64_t ncy, int64_t ncells) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  const int64_t i = c % ncx, j = (c / ncx) % ncy, k = c / (ncx * ncy);
  tsa_region b;
  b.x0 = i * cx;
  b.y0 = j * cy;
  b.z0 = k * cz;
  b.x1 = min(b.x0 + (int64_t)cx, nx);
  b.y1 = min(b.y0 + (int64_t)cy, ny);
  b.z1 = min(b.z0 + (int64_t)cz, nz);
  boxes[c] = b;
}

struct SigArgs {
  const void* base;
  int64_t nx, ny, nz;
  int32_t cx, cy, cz, subs;
  int64_t ncx, ncy, nchunk;
  const tsa_result* cells;
  double k;
  uint64_t* above;
};

// The float threshold equivalent to "v > mean + k*std" for every float v:
// the largest float not above the double threshold (NaN when the cell has no
// valid voxel, so nothing counts).
TSA_DEV float cell_threshold(const tsa_result& r, double k) {
  if (r.count == 0) return __builtin_nanf("");
  const double prod = k * r.std;
  const double thr = r.mean + prod;
  if (isnan(thr)) return __builtin_nanf("");
  float f = (float)thr;
  if ((double)f > thr) f = nextafterf(f, -INFINITY);
  return f;
}

template <int DT>
TSA_DEV float elem(const void* row, int64_t x) {
  if constexpr (DT == 0)
    return ((const float*)row)[x];
  else
    return (float)((const int16_t*)row)[x];
}

// Column of element e (0..15) of lane t inside a chunk starting at xc0.
// Vector layout: group p of lane t is the 4 consecutive columns at
// 4*(t + 256 p); scalar layout: element e is column t + 256 e.
template <bool VEC>
TSA_DEV int64_t col_of(int64_t xc0, int t, int e) {
  if constexpr (VEC)
    return xc0 + 4 * (t + kSigBlock * (e >> 2)) + (e & 3);
  else
    return xc0 + t + kSigBlock * e;
}

template <int DT, bool VEC>
__global__ __launch_bounds__(kSigBlock) void k_sigma(SigArgs a) {
  __shared__ uint32_t cnt_lds[kSigChunk];
  const int t = threadIdx.x;
  uint64_t b = blockIdx.x;
  const int64_t sub = (int64_t)(b % (uint64_t)a.subs);
  b /= (uint64_t)a.subs;
  const int64_t xch = (int64_t)(b % (uint64_t)a.nchunk);
  b /= (uint64_t)a.nchunk;
  const int64_t cyi = (int64_t)(b % (uint64_t)a.ncy), czi = (int64_t)(b / (uint64_t)a.ncy);
  const int64_t y0 = cyi * a.cy, y1 = min(y0 + (int64_t)a.cy, a.ny);
  const int64_t z0 = czi * a.cz, z1 = min(z0 + (int64_t)a.cz, a.nz);
  const int64_t rows_y = y1 - y0, rows = rows_y * (z1 - z0);
  const int64_t r0 = sub * kSigRows;
  if (r0 >= rows) return;  // the same for the whole block, before any barrier
  const int64_t r1 = min(r0 + (int64_t)kSigRows, rows);
  const int64_t xc0 = xch * kSigChunk, xc1 = min(xc0 + (int64_t)kSigChunk, a.nx);
  const int64_t c_first = xc0 / a.cx;
  const int64_t ncl = (xc1 - 1) / a.cx - c_first + 1;
  const int64_t cell_row = a.ncx * (cyi + a.ncy * czi);

  for (int i = t; i < ncl; i += kSigBlock) cnt_lds[i] = 0u;

  float thr[kSigPos * kSigEPL];
  uint32_t cnt[kSigPos * kSigEPL];
#pragma unroll
  for (int e = 0; e < kSigPos * kSigEPL; ++e) {
    const int64_t x = col_of<VEC>(xc0, t, e);
    thr[e] = x < xc1 ? cell_threshold(a.cells[cell_row + x / a.cx], a.k) : __builtin_nanf("");
    cnt[e] = 0u;
  }
  __syncthreads();

  const size_t esz = DT == 0 ? 4 : 2;
  const char* base = (const char*)a.base;
  int64_t yy = r0 % rows_y, zz = r0 / rows_y;
  for (int64_t r = r0; r < r1; r += kSigUnroll) {
    const char* rowp[kSigUnroll];
    bool live[kSigUnroll];
#pragma unroll
    for (int u = 0; u < kSigUnroll; ++u) {
      live[u] = r + u < r1;
      rowp[u] = base + (size_t)(((z0 + zz) * a.ny + (y0 + yy)) * a.nx) * esz;
      if (++yy == rows_y) {
        yy = 0;
        ++zz;
      }
    }
    if constexpr (VEC) {
      // 16-byte (float32) or 8-byte (int16) groups of 4 elements.
      uint4 vf[kSigUnroll][kSigPos];
      uint2 vi[kSigUnroll][kSigPos];
#pragma unroll
      for (int u = 0; u < kSigUnroll; ++u)
#pragma unroll
        for (int p = 0; p < kSigPos; ++p) {
          const int64_t x = col_of<true>(xc0, t, 4 * p);
          if (live[u] && x < xc1) {
            if constexpr (DT == 0)
              vf[u][p] = load16<true>((const uint4*)(rowp[u] + (size_t)x * 4));
            else
              vi[u][p] = *(const uint2*)(rowp[u] + (size_t)x * 2);
          } else {
            // Rows past the band and columns past the chunk: a float32 NaN never
            // counts; int16 zeros are masked by `live` below (columns past the
            // chunk have a NaN threshold).
            vf[u][p] = make_uint4(0x7fc00000u, 0x7fc00000u, 0x7fc00000u, 0x7fc00000u);
            vi[u][p] = make_uint2(0u, 0u);
          }
        }
#pragma unroll
      for (int u = 0; u < kSigUnroll; ++u)
#pragma unroll
        for (int p = 0; p < kSigPos; ++p) {
          float v[4];
          if constexpr (DT == 0) {
            v[0] = __uint_as_float(vf[u][p].x);
            v[1] = __uint_as_float(vf[u][p].y);
            v[2] = __uint_as_float(vf[u][p].z);
            v[3] = __uint_as_float(vf[u][p].w);
          } else {
            v[0] = (float)(int16_t)(vi[u][p].x & 0xFFFFu);
            v[1] = (float)(int16_t)(vi[u][p].x >> 16);
            v[2] = (float)(int16_t)(vi[u][p].y & 0xFFFFu);
            v[3] = (float)(int16_t)(vi[u][p].y >> 16);
          }
          const bool ok = DT == 0 || live[u];  // int16 dead rows carry zeros: skip them
#pragma unroll
          for (int e = 0; e < 4; ++e) cnt[4 * p + e] += (ok && v[e] > thr[4 * p + e]) ? 1u : 0u;
        }
    } else {
      float v[kSigUnroll][kSigPos * kSigEPL];
#pragma unroll
      for (int u = 0; u < kSigUnroll; ++u)
#pragma unroll
        for (int e = 0; e < kSigPos * kSigEPL; ++e) {
          const int64_t x = col_of<false>(xc0, t, e);
          v[u][e] = (live[u] && x < xc1) ? elem<DT>(rowp[u], x) : __builtin_nanf("");
        }
#pragma unroll
      for (int u = 0; u < kSigUnroll; ++u)
#pragma unroll
        for (int e = 0; e < kSigPos * kSigEPL; ++e) cnt[e] += v[u][e] > thr[e] ? 1u : 0u;
    }
  }

#pragma unroll
  for (int e = 0; e < kSigPos * kSigEPL; ++e) {
    const int64_t x = col_of<VEC>(xc0, t, e);
    if (x < xc1 && cnt[e]) atomicAdd(&cnt_lds[x / a.cx - c_first], cnt[e]);
  }
  __syncthreads();
  for (int i = t; i < ncl; i += kSigBlock) {
    const uint32_t c = cnt_lds[i];
    if (c) atomicAdd((unsigned long long*)&a.above[cell_row + c_first + i], (unsigned long long)c);
  }
}

__global__ void k_zero64(uint64_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace

size_t minimap_ws_bytes(const tsa_cube* cube, int32_t cx, int32_t cy, int32_t cz, int32_t nbins) {
  Grid g;
  if (grid_of(cube, cx, cy, cz, &g) != TSA_OK) return 0;
  const size_t bw = batch_ws_bytes(cube, nbins, (int32_t)g.ncells);
  if (!bw) return 0;
  return align256(sizeof(tsa_region) * (size_t)g.ncells) + bw;
}

int run_minimap(const tsa_cube* cube, int32_t cx, int32_t cy, int32_t cz, int32_t nbins, tsa_result* d_cells,
                uint64_t* d_hists, void* d_ws, size_t ws_bytes, tsa_stream_t stream) {
  Grid g;
  int st = grid_of(cube, cx, cy, cz, &g);
  if (st) return st;
  if (!d_cells || !d_hists || nbins < 1 || nbins > 4096) return TSA_EINVAL;
  const size_t need = minimap_ws_bytes(cube, cx, cy, cz, nbins);
  if (!need) return TSA_EINVAL;
  if (!d_ws || ws_bytes < need) return TSA_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  tsa_region* boxes = (tsa_region*)d_ws;
  const size_t off = align256(sizeof(tsa_region) * (size_t)g.ncells);
  const int blocks = (int)((g.ncells + 255) / 256);
  TSA_TRACED("minimap_plan", s,
             hipLaunchKernelGGL(k_grid_plan, dim3(blocks), dim3(256), 0, s, boxes, cube->nx, cube->ny, cube->nz, cx,
                                cy, cz, g.ncx, g.ncy, g.ncells));
  if (hipGetLastError() != hipSuccess) return TSA_EDEVICE;
  return run_region_batch(cube, boxes, (int32_t)g.ncells, nbins, d_cells, d_hists, nullptr, (char*)d_ws + off,
                          ws_bytes - off, stream);
}

int run_sigma_count(const tsa_cube* cube, int32_t cx, int32_t cy, int32_t cz, const tsa_result* d_cells, double k,
                    uint64_t* d_above, tsa_stream_t stream) {
  Grid g;
  int st = grid_of(cube, cx, cy, cz, &g);
  if (st) return st;
  if (!d_cells || !d_above || !isfinite(k)) return TSA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  SigArgs a;
  a.base = cube->data;
  a.nx = cube->nx;
  a.ny = cube->ny;
  a.nz = cube->nz;
  a.cx = cx;
  a.cy = cy;
  a.cz = cz;
  a.ncx = g.ncx;
  a.ncy = g.ncy;
  a.nchunk = (cube->nx + kSigChunk - 1) / kSigChunk;
  const int64_t band_rows = (int64_t)(cy < cube->ny ? cy : cube->ny) * (int64_t)(cz < cube->nz ? cz : cube->nz);
  const int64_t subs = (band_rows + kSigRows - 1) / kSigRows;
  const double nblocks = (double)subs * (double)a.nchunk * (double)g.ncy * (double)g.ncz;
  if (nblocks > (double)(1 << 24)) return TSA_EINVAL;  // grid limit: too many thin cells
  a.subs = (int32_t)subs;
  a.cells = d_cells;
  a.k = k;
  a.above = d_above;
  const int zb = (int)((g.ncells + 255) / 256);
  TSA_TRACED("sigma_zero", s, hipLaunchKernelGGL(k_zero64, dim3(zb), dim3(256), 0, s, d_above, g.ncells));
  const uintptr_t group_align = cube->dtype == TSA_F32 ? 16 : 8;  // bytes of a 4-element group
  const bool vec = ((uintptr_t)cube->data % group_align) == 0 && (cube->nx % 4) == 0;
  const dim3 grid((uint32_t)nblocks);
  if (cube->dtype == TSA_F32) {
    if (vec)
      TSA_TRACED("sigma", s, hipLaunchKernelGGL((k_sigma<0, true>), grid, dim3(kSigBlock), 0, s, a));
    else
      TSA_TRACED("sigma", s, hipLaunchKernelGGL((k_sigma<0, false>), grid, dim3(kSigBlock), 0, s, a));
  } else {
    if (vec)
      TSA_TRACED("sigma", s, hipLaunchKernelGGL((k_sigma<1, true>), grid, dim3(kSigBlock), 0, s, a));
    else
      TSA_TRACED("sigma", s, hipLaunchKernelGGL((k_sigma<1, false>), grid, dim3(kSigBlock), 0, s, a));
  }
  return hipGetLastError() == hipSuccess ? TSA_OK : TSA_EDEVICE;
}

}  // namespace tsa

using namespace tsa;

extern "C" {

size_t tsa_minimap_workspace_bytes(const tsa_cube* cube, int32_t cell_x, int32_t cell_y, int32_t cell_z,
                                   int32_t nbins) {
  if (nbins < 1 || nbins > 4096) return 0;
  return minimap_ws_bytes(cube, cell_x, cell_y, cell_z, nbins);
}

int64_t tsa_minimap_cells(const tsa_cube* cube, int32_t cell_x, int32_t cell_y, int32_t cell_z) {
  Grid g;
  const int st = grid_of(cube, cell_x, cell_y, cell_z, &g);
  return st ? (int64_t)st : g.ncells;
}

int tsa_minimap(const tsa_cube* cube, int32_t cell_x, int32_t cell_y, int32_t cell_z, int32_t nbins,
                tsa_result* d_cells, uint64_t* d_hists, void* d_ws, size_t ws_bytes, tsa_stream_t stream) {
  return run_minimap(cube, cell_x, cell_y, cell_z, nbins, d_cells, d_hists, d_ws, ws_bytes, stream);
}

int tsa_sigma_count(const tsa_cube* cube, int32_t cell_x, int32_t cell_y, int32_t cell_z, const tsa_result* d_cells,
                    double k, uint64_t* d_above, tsa_stream_t stream) {
  return run_sigma_count(cube, cell_x, cell_y, cell_z, d_cells, k, d_above, stream);
}

}  // extern "C"
