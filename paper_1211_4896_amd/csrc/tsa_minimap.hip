// Statistical mini-map (Section 4.5): the cube cut into a regular grid of
// cells, each summarised by the statistics of a region query, and the local
// threshold built from it: per cell, how many voxels lie above the cell's
// mean + k standard deviations.
//
// Cells whose rows hold at most 768 voxels and whose 768 / w rows per lane
// cover the cell in 64 values (a 30x30x30 cell: 36) are answered by one
// 768-lane workgroup each, the cell read from HBM once into registers (up to
// 64 values per lane; at most 80 registers a lane up to 40 values, so two
// workgroups share a compute unit and one's loads and barriers overlap the
// other's counting):
// moments and the first key digit, then the histogram
// over the cell's own [min, max] with the first digit's bucket copied to LDS,
// and the median's last two digits (or, for a bucket of at most 64 keys, the
// ranks of its keys), all from registers, with only counters and that copy in LDS.  Larger cells go through
// the region batch over the grid's boxes (planned on the device, so no box
// list crosses PCIe).  The threshold pass streams the
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
constexpr int kSigEPL = 4;                   // elements per group
constexpr int kSigChunk = kSigBlock * 4 * kSigEPL;  // widest column chunk of a block (P = 4)
constexpr int kSigRows = 256;                // rows per block, at most

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

// TSA_MINIMAP_BATCH=1 sends every mini-map through the region batch (for
// comparing the two paths); otherwise cells of at most 32768 voxels use the
// register-resident k_mm_reg.
bool register_path_on() {
  static const bool on = [] {
    const char* e = getenv("TSA_MINIMAP_BATCH");
    return !(e && e[0] == '1');
  }();
  return on;
}

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

// P element groups of 4 per lane and row (chunk of 1024 P columns), U = 16 / P
// rows loaded together: 16 loads in flight per lane whatever the row width.
template <int DT, bool VEC, int P>
__global__ __launch_bounds__(kSigBlock) void k_sigma(SigArgs a) {
  constexpr int U = 16 / P;
  constexpr int64_t CH = (int64_t)kSigBlock * P * kSigEPL;
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
  const int64_t xc0 = xch * CH, xc1 = min(xc0 + CH, a.nx);
  const int64_t c_first = xc0 / a.cx;
  const int64_t ncl = (xc1 - 1) / a.cx - c_first + 1;
  const int64_t cell_row = a.ncx * (cyi + a.ncy * czi);

  for (int i = t; i < ncl; i += kSigBlock) cnt_lds[i] = 0u;

  float thr[P * kSigEPL];
  uint32_t cnt[P * kSigEPL];
#pragma unroll
  for (int e = 0; e < P * kSigEPL; ++e) {
    const int64_t x = col_of<VEC>(xc0, t, e);
    thr[e] = x < xc1 ? cell_threshold(a.cells[cell_row + x / a.cx], a.k) : __builtin_nanf("");
    cnt[e] = 0u;
  }
  __syncthreads();

  const size_t esz = DT == 0 ? 4 : 2;
  const char* base = (const char*)a.base;
  int64_t yy = r0 % rows_y, zz = r0 / rows_y;
  for (int64_t r = r0; r < r1; r += U) {
    const char* rowp[U];
    bool live[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      live[u] = r + u < r1;
      rowp[u] = base + (size_t)(((z0 + zz) * a.ny + (y0 + yy)) * a.nx) * esz;
      if (++yy == rows_y) {
        yy = 0;
        ++zz;
      }
    }
    if constexpr (VEC) {
      // 16-byte (float32) or 8-byte (int16) groups of 4 elements.
      uint4 vf[U][P];
      uint2 vi[U][P];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int p = 0; p < P; ++p) {
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
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int p = 0; p < P; ++p) {
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
      float v[U][P * kSigEPL];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < P * kSigEPL; ++e) {
          const int64_t x = col_of<false>(xc0, t, e);
          v[u][e] = (live[u] && x < xc1) ? elem<DT>(rowp[u], x) : __builtin_nanf("");
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < P * kSigEPL; ++e) cnt[e] += v[u][e] > thr[e] ? 1u : 0u;
    }
  }

#pragma unroll
  for (int e = 0; e < P * kSigEPL; ++e) {
    const int64_t x = col_of<VEC>(xc0, t, e);
    if (x < xc1 && cnt[e]) atomicAdd(&cnt_lds[x / a.cx - c_first], cnt[e]);
  }
  __syncthreads();
  for (int i = t; i < ncl; i += kSigBlock) {
    const uint32_t c = cnt_lds[i];
    if (c) atomicAdd((unsigned long long*)&a.above[cell_row + c_first + i], (unsigned long long)c);
  }
}

// ---- LDS-resident cells ----------------------------------------------------------
constexpr int kMMBlock = 768;

struct MMArgs {
  const void* base;
  int64_t nx, ny, nz;
  int32_t cx, cy, cz, nbins;
  int64_t ncx, ncy, ncells, per_xcd;
  uint32_t rshift, pad;
  Magic mx_full, mx_edge, my_full, my_edge;  // division by a cell's width / height (full or last cell)
  uint32_t ky_full, ky_edge;                 // ceil(2^32 / height) of a full / the last cell (0 for height 1)
  Magic m_ncx, m_ncy;                        // division by the grid's cells along x and y
  tsa_result* out;
  uint64_t* hists;
};

struct MMShared {
  MomShared mom;
  Partial part;
  alignas(16) uint32_t wsum32[16];
  uint32_t found, sel_digit, sel_cum32, sel_bucket32;
  // the cell's parameters, set by thread 0
  uint64_t cnt, k;
  uint32_t kmin, kmax, prefix, go;
  float lo, hi, scale, shift;
  uint32_t hist_ok, var_on;
  uint32_t status;
  uint32_t ncand;  // keys of the first-digit bucket copied to the candidate list
};

// Keys of the first-digit bucket a cell copies to LDS during the second sweep
// (when the bucket is no larger), so the last digit is counted over them
// instead of over every value again.
constexpr uint32_t kMMCand = 4096;
// A bucket of at most kMMRankMax keys is finished from the candidate list by
// counting ranks (no second-digit counters, no further block-wide scans).
constexpr uint32_t kMMRankMax = 64;

// LDS words by byte address.  The per-value increments add a shifted index to
// a base held in a register (one shift-and-add), and add a register holding 1:
// both values pass through an empty asm barrier so the compiler neither folds
// the base back into a constant it adds separately nor rebuilds the 1 before
// every increment.
typedef __attribute__((address_space(3))) uint32_t lds_word;
TSA_DEV uint32_t lds_byte_addr(uint32_t* p) { return (uint32_t)(uintptr_t)(lds_word*)p; }
TSA_DEV uint32_t in_register(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}
TSA_DEV uint32_t in_scalar_register(uint32_t v) {
  asm volatile("" : "+s"(v));
  return v;
}
TSA_DEV void lds_add_at(uint32_t byte_addr, uint32_t v) {
  __hip_atomic_fetch_add((lds_word*)(uintptr_t)byte_addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// A workgroup barrier that orders LDS only: this wave's LDS operations
// complete, then the barrier.  __syncthreads() also waits for every global
// load in flight, which right after the cell's loads would hold each wave
// until its last value arrived.
TSA_DEV void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Histogram words of a cell: nbins << rshift replicas and the trash words,
// rounded up to whole 16-byte groups.
__host__ __device__ inline uint32_t mm_hist_words(int32_t nbins, uint32_t rshift) {
  return ((((uint32_t)nbins << rshift) + kTrash) + 3u) & ~3u;
}
// Clears `words` (a multiple of 4) LDS words from a 16-byte aligned start, 16 bytes a store.
TSA_DEV void mm_zero(uint32_t* p, uint32_t words, int t) {
  uint4* q = reinterpret_cast<uint4*>(p);
  for (uint32_t i = (uint32_t)t; i < words / 4u; i += kMMBlock) q[i] = make_uint4(0u, 0u, 0u, 0u);
}

// One workgroup per cell, the cell held in registers (a 30^3 cell is 36
// values per lane), all loaded at once, and the LDS holds only counters.  The per-value work
// (moments, keys, digits, histogram: two LDS atomics a value) and the per-cell
// scans and barriers bound this kernel, not HBM.  Every value is held as float32: int16 converts exactly, its double
// sums stay exact (a cell's sums of squares stay below 2^53) and float keys
// order it the same way, and slots past the cell hold NaN, so no per-slot
// validity test is needed past the loads.  Block b works on cell (b % 8) * per_xcd + b / 8,
// so the cells one XCD (and its L2) sees are neighbours sharing cache lines at
// their x edges.
//
// Lanes take whole rows of the cell: lane t owns column t % w, and with
// R = 768 / w rows side by side it holds rows t / w, t / w + R, t / w + 2R,
// ... of the cell's h * d rows (row r is y = r % h, z = r / h).  Each value is
// one constant address step from the last, plus a plane carry when y wraps,
// in 32-bit offsets from the cell's corner.  Slots past the cell (and lanes
// past R whole rows) hold NaN and drop out at each step's NaN test.
// Up to 40 values a lane the kernel is held to 80 registers, so two
// workgroups (six waves a SIMD) share a compute unit.
template <int DT, int EPT>
__global__ __launch_bounds__(kMMBlock) __attribute__((amdgpu_waves_per_eu(EPT <= 40 ? 6 : 3))) void k_mm_reg(
    MMArgs a) {
  using T = typename Ty<DT>::T;
  // digit counters [kBins1 + kTrash] | histogram [(nbins << rshift) + kTrash] | candidates [kMMCand]
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ MMShared sh;
  const int t = threadIdx.x;
  const int64_t cell = (int64_t)(blockIdx.x % 8u) * a.per_xcd + blockIdx.x / 8u;
  if (cell >= a.ncells) return;  // the same for the whole block
  // the grid holds fewer than 2^31 cells (checked on the host): 32-bit
  // divisions by multiply-high, not 64-bit divisions in every wave
  const uint32_t c32 = (uint32_t)cell, row = mdiv(c32, a.m_ncx), ck32 = mdiv(row, a.m_ncy);
  const int64_t ci = c32 - row * (uint32_t)a.ncx, cj = row - ck32 * (uint32_t)a.ncy, ck = ck32;
  const int64_t x0 = ci * a.cx, y0 = cj * a.cy, z0 = ck * a.cz;
  const uint32_t w = (uint32_t)(min(x0 + (int64_t)a.cx, a.nx) - x0);
  const uint32_t h = (uint32_t)(min(y0 + (int64_t)a.cy, a.ny) - y0);
  const uint32_t dd = (uint32_t)(min(z0 + (int64_t)a.cz, a.nz) - z0);
  const uint32_t nvox = w * h * dd;
  uint32_t* dig = lds;
  uint32_t* hist = lds + kBins1 + kTrash;
  const uint32_t hwords = mm_hist_words(a.nbins, a.rshift);
  uint32_t* cand = hist + hwords;
  mm_zero(dig, kBins1 + kTrash + hwords, t);  // digit counters and histogram, adjacent

  // 1. every load of the lane in flight at once
  float x[EPT];
  // the cell's corner, made visibly uniform (scalar registers) for the loads' scalar base
  const uint64_t corner_v = (uint64_t)(uintptr_t)((const T*)a.base + (z0 * a.nx * a.ny + y0 * a.nx + x0));
  typedef const __attribute__((address_space(1))) char gchar;
  gchar* corner = (gchar*)(uintptr_t)(
      ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(corner_v >> 32)) << 32) |
      (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)corner_v));  // the builtin returns int: no sign extension
  const Magic mw = w == (uint32_t)a.cx ? a.mx_full : a.mx_edge;
  const Magic mh = h == (uint32_t)a.cy ? a.my_full : a.my_edge;
  const uint32_t kh = h == (uint32_t)a.cy ? a.ky_full : a.ky_edge;
  const uint32_t nx32 = (uint32_t)a.nx, plane32 = (uint32_t)(a.nx * a.ny);
  const uint32_t rows_side = (uint32_t)kMMBlock / w;  // w <= 768 (checked on the host)
  const uint32_t nrows = h * dd;
  {
    const uint32_t r0 = mdiv((uint32_t)t, mw);
    const uint32_t lx = (uint32_t)t - r0 * w;
    const uint32_t dz = mdiv(rows_side, mh), dy = rows_side - dz * h;  // rows_side = dz h + dy
    const uint32_t lz = mdiv(r0, mh);
    const uint32_t ly = r0 - lz * h;
    // byte offsets from the cell's corner: a cell spans fewer than 2^32 bytes
    // of the cube (checked on the host)
    constexpr uint32_t es = sizeof(T);
    uint32_t off = (lz * plane32 + ly * nx32 + lx) * es;
    const uint32_t step = (dz * plane32 + dy * nx32) * es;
    const uint32_t wrap = (plane32 - h * nx32) * es;  // y passing h: one more plane, h rows back
    // y as a 32-bit fraction of h (kh = ceil(2^32 / h)): adding dy carries out
    // of 32 bits exactly when y passes h, for the at most 64 * 768 rows of a
    // register cell (the error of the rounded step stays below one row)
    uint32_t yf = ly * kh;
    const uint32_t dyf = dy * kh;
    // slots holding a row of the cell: a prefix of the lane's slots
    const uint32_t nvalid = (r0 < rows_side && r0 < nrows) ? (nrows - r0 + rows_side - 1) / rows_side : 0u;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      if ((uint32_t)j < nvalid)  // slots past the cell never touch memory
        x[j] = (float)*(const __attribute__((address_space(1))) T*)(corner + off);
      else
        x[j] = __builtin_nanf("");
      uint32_t yn;
      const bool carry = __builtin_add_overflow(yf, dyf, &yn);
      yf = yn;
      off += step + (carry ? wrap : 0u);
    }
  }
  lds_barrier();  // counters cleared (the loads still in flight)
  // moments, min/max keys and the first key digit.  The per-value steps are
  // written out here rather than through the shared accumulators: every step
  // sits under the value's own NaN test, so no select is needed, and the
  // digit counters need no wave vote (a wave with no matching lane skips the
  // masked LDS increment by its exec mask).
  MomAcc<0, false> mom;  // the count is the first-digit histogram's total
  const uint32_t one = in_register(1u), dig_b = in_register(lds_byte_addr(dig));
  const uint32_t word_shift = in_scalar_register(2u);  // kept opaque: one shift-and-add per increment
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    {
      const float v = x[j];
      if (v == v) {
        const double d = (double)v;
        mom.s += d;
        mom.q = __builtin_fma(d, d, mom.q);
        const uint32_t k = key_f32(__float_as_uint(v));
        mom.kmin = min(mom.kmin, k);
        mom.kmax = max(mom.kmax, k);
        lds_add_at(dig_b + ((k >> kShift1) << word_shift), one);
      }
    }
  }
  __syncthreads();
  // The values' NaN tests are repeated in the later sweeps rather than kept:
  // an empty register barrier stops the compiler from holding 2 scalar
  // registers of lane mask per value across the phases (it spills them to
  // vector lanes, which costs more than the compare).
#pragma unroll
  for (int j = 0; j < EPT; ++j) asm volatile("" : "+v"(x[j]));
  {
    uint32_t c = 0;
    for (uint32_t i = t; i < kBins1; i += kMMBlock) c += dig[i];
    mom.cnt = c;
  }
  block_store_partial(mom, sh.mom, &sh.part);  // ends with thread 0 writing sh.part
  __syncthreads();
  tsa_result& R = a.out[cell];
  if (t == 0) {
    const Partial p = sh.part;
    double n, mean, m2;
    partial_stats(p, 0, n, mean, m2);
    R.count = p.n;
    R.nan_count = nvox - p.n;
    R.status = TSA_OK;
    R.flags = 0;
    sh.cnt = p.n;
    sh.go = 0;
    sh.hist_ok = 0;
    sh.var_on = 0;
    const double qnan = __builtin_nan("");
    if (p.n == 0) {
      R.mean = R.m2 = R.std = R.min = R.max = R.median = qnan;
      R.flags = TSA_FLAG_HIST_SKIPPED;
    } else {
      const double vmin = bvalue_of_key(p.kmin, 0), vmax = bvalue_of_key(p.kmax, 0);
      R.min = vmin;
      R.max = vmax;
      const float lo = (float)vmin, hi = (float)vmax;
      if (p.kmin == p.kmax) {  // constant cell
        R.mean = vmin;
        R.m2 = 0.0;
        R.std = 0.0;
        R.median = vmin;
        sh.hist_ok = isfinite(lo) ? 2u : 0u;  // 2: every value in bin 0
        if (!sh.hist_ok) R.flags = TSA_FLAG_HIST_SKIPPED;
      } else {
        if (m2 < 0.0) m2 = 0.0;  // rounding below zero; NaN (infinite values) stays
        R.mean = mean;
        R.m2 = m2;
        R.std = sqrt(m2 / n);
        sh.go = 1;
        sh.k = (p.n - 1) / 2;
        float scale = 0.f;
        if (isfinite(lo) && isfinite(hi)) {
          const float width = hi - lo;
          if (isfinite(width)) {
            scale = (float)a.nbins / width;
            sh.hist_ok = (isfinite(scale) && scale != 0.0f) ? 1u : 0u;
          }
        }
        if (!sh.hist_ok) R.flags = TSA_FLAG_HIST_SKIPPED;
        sh.lo = lo;
        sh.scale = scale;
        sh.var_on = (isfinite(mean) && one_pass_m2_at_risk(mean, m2 / n)) ? 1u : 0u;
        sh.shift = sh.var_on ? (float)mean : 0.0f;
      }
    }
  }
  __syncthreads();
  if (__builtin_amdgcn_readfirstlane(sh.go)) {
    // 2. first digit; histogram over [min, max] + second digit (+ M2 about the mean)
    uint32_t d1, d2, d3;
    uint32_t cum, bucket;  // a cell holds fewer than 2^32 voxels
    bool found = block_select_small(dig, kBins1, (uint32_t)sh.k, sh, &d1, &cum, &bucket);
    uint32_t k = (uint32_t)sh.k - cum;
    const bool compact = bucket <= kMMCand;     // the bucket's keys fit the candidate list
    const bool by_rank = bucket <= kMMRankMax;  // and are few enough to rank by counting
    mm_zero(dig, kBins2, t);
    if (t == 0) {
      sh.ncand = 0;
      sh.found = 0;
    }
    __syncthreads();
    // histogram over [min, max] (the formula of HistOwnAcc: b = min((int)((v -
    // lo) * scale), nbins - 1), replica lane % R of bin b) + the first digit's
    // bucket: copied to LDS, and its second digit counted unless it is small
    // enough to rank.  A cell without a histogram still counts (every index
    // clamped into the bins, never written out), so the sweep needs no switch.
    const float lo = sh.lo, scale = sh.scale;
    const uint32_t nbm1 = (uint32_t)a.nbins - 1u;
    const uint32_t rshift = a.rshift, rs2 = rshift + 2u;
    const uint32_t hrep_b = in_register(lds_byte_addr(hist) + (((uint32_t)t & ((1u << rshift) - 1u)) << 2));
    // the first digit's bucket as a float interval, to its non-NaN keys; the
    // test on floats admits both zeros at a zero end, the key then decides
    const uint32_t kb0 = max(d1 << kShift1, 0x007FFFFFu);
    const uint32_t kb1 = min((d1 << kShift1) | ((1u << kShift1) - 1u), 0xFF800000u);
    const float blo = __uint_as_float(f32bits_of_key(kb0)), bhi = __uint_as_float(f32bits_of_key(kb1));
    VarAcc var{sh.shift};
    // block-uniform switch, kept in a scalar register
    const bool var_on = __builtin_amdgcn_readfirstlane(sh.var_on) != 0;
#define TSA_MM_PASS2(VAR_STEP)                                                  \
  _Pragma("unroll") for (int j = 0; j < EPT; ++j) {                             \
    {                                                                           \
      const float v = x[j];                                                     \
      if (v == v) {                                                             \
        const float tb = (v - lo) * scale; /* lo == hi: scale 0, tb 0 */        \
        lds_add_at(hrep_b + (min((uint32_t)(int32_t)tb, nbm1) << rs2), one);    \
        if (v >= blo && v <= bhi) {                                             \
          const uint32_t k = key_f32(__float_as_uint(v));                       \
          if ((k >> kShift1) == d1) {                                           \
            if (!by_rank) lds_inc(dig, (k >> kShift2) & 0xFFFu);                \
            if (compact) {                                                      \
              const uint32_t slot = __hip_atomic_fetch_add(                     \
                  &sh.ncand, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);  \
              if (slot < kMMCand) cand[slot] = k;                               \
            }                                                                   \
          }                                                                     \
        }                                                                       \
        VAR_STEP;                                                               \
      }                                                                         \
    }                                                                           \
  }
    if (var_on)  // rare: the second moment about the mean in the same sweep
      TSA_MM_PASS2(var(v, true))
    else
      TSA_MM_PASS2((void)0)
#undef TSA_MM_PASS2
    if (var_on) block_store_var(var, sh.mom, &sh.part);
    __syncthreads();
    if (t == 0 && var_on) {
      const double n = (double)sh.cnt;
      const double dm = R.mean - (double)sh.shift;
      double m2 = sh.part.q - n * dm * dm;
      if (m2 < 0.0) m2 = 0.0;  // rounding below zero; NaN (infinite values) stays
      R.m2 = m2;
      R.std = sqrt(m2 / n);
    }
    const uint32_t ncand = min(sh.ncand, kMMCand);  // final: the sweep ended at a barrier
    if (by_rank) {
      // 2b. the bucket's keys are all in the list: candidate i's rank is the
      // number of keys below it plus the equal keys listed before it, so the
      // ranks are 0..n-1 once each and one thread holds rank k
      if ((uint32_t)t < ncand && ncand == bucket) {
        const uint32_t key_i = cand[t];
        const uint4* c4 = reinterpret_cast<const uint4*>(cand);  // 16-byte aligned
        uint32_t r = 0;
        for (uint32_t j = 0; j < ncand; j += 4) {  // every lane reads the same words
          const uint4 q = c4[j >> 2];
          const uint32_t kj[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
          for (uint32_t u = 0; u < 4; ++u)
            r += (j + u < ncand && (kj[u] < key_i || (kj[u] == key_i && j + u < (uint32_t)t))) ? 1u : 0u;
        }
        if (r == k) {
          sh.prefix = key_i;
          sh.found = 1;
        }
      }
      __syncthreads();
      if (t == 0) {
        if (found && sh.found)
          R.median = bvalue_of_key(sh.prefix, 0);
        else {
          R.median = __builtin_nan("");
          R.status = TSA_EDEVICE;
        }
      }
    } else {
      found = block_select_small(dig, kBins2, k, sh, &d2, &cum, &bucket) && found;
      k -= cum;
      const uint32_t prefix = (d1 << kShift1) | (d2 << kShift2);
      // 3. last 8 bits over the keys of the second-digit bucket
      mm_zero(dig, kBins3, t);
      __syncthreads();
      const uint32_t p2 = prefix >> kShift2;
      if (compact) {  // over the bucket's copied keys
        for (uint32_t i = t; i < ncand; i += kMMBlock) {
          const uint32_t key = cand[i];
          if ((key >> kShift2) == p2) lds_inc(dig, key & 0xFFu);
        }
      } else {  // over every value again
#pragma unroll
        for (int j = 0; j < EPT; ++j) asm volatile("" : "+v"(x[j]));
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const float v = x[j];
          if (v == v) {
            const uint32_t k = key_f32(__float_as_uint(v));
            if ((k >> kShift2) == p2) lds_inc(dig, k & 0xFFu);
          }
        }
      }
      __syncthreads();
      found = block_select_small(dig, kBins3, k, sh, &d3, &cum, &bucket) && found;
      if (t == 0) {
        if (found)
          R.median = bvalue_of_key(prefix | d3, 0);
        else {
          R.median = __builtin_nan("");
          R.status = TSA_EDEVICE;
        }
      }
    }
  }
  __syncthreads();
  // 4. the cell's histogram (every bin written).  G threads (a power of two,
  // at most 8) share a bin, each summing R / G of its replicas in an order
  // rotated by the bin so a wave's reads fall in different banks, and the G
  // partial sums meet by lane exchange.
  uint64_t* H = a.hists + cell * (int64_t)a.nbins;
  const uint32_t ok = sh.hist_ok, R1 = 1u << a.rshift, nb = (uint32_t)a.nbins;
  uint32_t lg = 0;  // log2 G
  while (lg < 3u && (1u << (lg + 1u)) <= R1 && (nb << (lg + 1u)) <= (uint32_t)kMMBlock) ++lg;
  const uint32_t G = 1u << lg, per = R1 >> lg;
  for (uint32_t base = 0; base < (nb << lg); base += kMMBlock) {  // the same trip count for every lane
    const uint32_t idx = base + (uint32_t)t, b = idx >> lg, part = idx & (G - 1u);
    uint32_t c = 0;
    if (ok == 1u && b < nb) {
      const uint32_t* hb = hist + (b << a.rshift) + part * per;
      for (uint32_t i = 0; i < per; ++i) c += hb[(i + b) & (per - 1u)];
    }
    for (uint32_t m = 1; m < G; m <<= 1) c += __shfl_xor(c, (int)m);
    if (b < nb && part == 0) H[b] = ok == 1u ? (uint64_t)c : (ok == 2u && b == 0) ? sh.cnt : 0ull;
  }
}

// ceil(2^32 / h) as a 32-bit y fraction step (h = 1 never wraps: 0)
uint32_t y_fraction(uint64_t h) { return h <= 1 ? 0u : (uint32_t)(((1ull << 32) + h - 1) / h); }

// Values per lane for a w x h x d cell (0: the register path does not hold
// it): rows of w voxels, 768 / w rows side by side.
int mm_ept(uint64_t w, uint64_t h, uint64_t d) {
  if (w > (uint64_t)kMMBlock) return 0;
  const uint64_t side = kMMBlock / w, need = (h * d + side - 1) / side;
  for (int e : {16, 32, 36, 40, 48, 64})
    if (need <= (uint64_t)e) return e;
  return 0;
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
  const uint64_t cxe = (uint64_t)(cx < cube->nx ? cx : cube->nx), cye = (uint64_t)(cy < cube->ny ? cy : cube->ny),
                 cze = (uint64_t)(cz < cube->nz ? cz : cube->nz);
  // 32-bit byte offsets inside a cell: its corner to its far corner
  const bool span32 = (double)cze * (double)cube->nx * (double)cube->ny * (cube->dtype == TSA_F32 ? 4.0 : 2.0) <
                      4294967296.0;
  const int ept = (span32 && g.ncells < (1ll << 31)) ? mm_ept(cxe, cye, cze) : 0;
  if (ept && register_path_on()) {
    // histogram replicas: up to 64 per bin within 4096 counters (64: one per
    // lane of a wave, so a wave's increments never share a word or a bank)
    uint32_t rshift = 0;
    while (rshift < 6 && ((uint32_t)nbins << (rshift + 1)) <= 4096u) ++rshift;
    const size_t lds = ((size_t)kBins1 + kTrash + mm_hist_words(nbins, rshift) + kMMCand) * 4;
    MMArgs m;
    m.base = cube->data;
    m.nx = cube->nx;
    m.ny = cube->ny;
    m.nz = cube->nz;
    m.cx = cx;
    m.cy = cy;
    m.cz = cz;
    m.nbins = nbins;
    m.ncx = g.ncx;
    m.ncy = g.ncy;
    m.ncells = g.ncells;
    m.per_xcd = (g.ncells + 7) / 8;
    m.rshift = rshift;
    m.pad = 0;
    const int64_t ex = cube->nx - (g.ncx - 1) * cx, ey = cube->ny - (g.ncy - 1) * cy;  // last cell's edges
    m.mx_full = make_magic((uint32_t)(cx < cube->nx ? cx : cube->nx));
    m.mx_edge = make_magic((uint32_t)ex);
    m.my_full = make_magic((uint32_t)(cy < cube->ny ? cy : cube->ny));
    m.my_edge = make_magic((uint32_t)ey);
    m.m_ncx = make_magic((uint32_t)g.ncx);
    m.m_ncy = make_magic((uint32_t)g.ncy);
    m.ky_full = y_fraction((uint64_t)(cy < cube->ny ? cy : cube->ny));
    m.ky_edge = y_fraction((uint64_t)ey);
    m.out = d_cells;
    m.hists = d_hists;
    const dim3 grid((uint32_t)(m.per_xcd * 8));
#define TSA_MM_LAUNCH(DTV, EPTV) \
  TSA_TRACED("minimap_cells", s, hipLaunchKernelGGL((k_mm_reg<DTV, EPTV>), grid, dim3(kMMBlock), lds, s, m))
#define TSA_MM_BY_EPT(DTV)         \
  do {                             \
    if (ept == 16)                 \
      TSA_MM_LAUNCH(DTV, 16);      \
    else if (ept == 32)            \
      TSA_MM_LAUNCH(DTV, 32);      \
    else if (ept == 36)            \
      TSA_MM_LAUNCH(DTV, 36);      \
    else if (ept == 40)            \
      TSA_MM_LAUNCH(DTV, 40);      \
    else if (ept == 48)            \
      TSA_MM_LAUNCH(DTV, 48);      \
    else                           \
      TSA_MM_LAUNCH(DTV, 64);      \
  } while (0)
    if (cube->dtype == TSA_F32)
      TSA_MM_BY_EPT(0);
    else
      TSA_MM_BY_EPT(1);
#undef TSA_MM_BY_EPT
#undef TSA_MM_LAUNCH
    return hipGetLastError() == hipSuccess ? TSA_OK : TSA_EDEVICE;
  }
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
  const int P = cube->nx <= 1024 ? 1 : cube->nx <= 2048 ? 2 : 4;
  const int64_t chunk = (int64_t)kSigBlock * P * kSigEPL;
  a.nchunk = (cube->nx + chunk - 1) / chunk;
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
#define TSA_SIGMA_LAUNCH(DTV, VECV, PV) \
  TSA_TRACED("sigma", s, hipLaunchKernelGGL((k_sigma<DTV, VECV, PV>), grid, dim3(kSigBlock), 0, s, a))
#define TSA_SIGMA_BY_P(DTV, VECV)      \
  do {                                 \
    if (P == 1)                        \
      TSA_SIGMA_LAUNCH(DTV, VECV, 1);  \
    else if (P == 2)                   \
      TSA_SIGMA_LAUNCH(DTV, VECV, 2);  \
    else                               \
      TSA_SIGMA_LAUNCH(DTV, VECV, 4);  \
  } while (0)
  if (cube->dtype == TSA_F32) {
    if (vec)
      TSA_SIGMA_BY_P(0, true);
    else
      TSA_SIGMA_BY_P(0, false);
  } else {
    if (vec)
      TSA_SIGMA_BY_P(1, true);
    else
      TSA_SIGMA_BY_P(1, false);
  }
#undef TSA_SIGMA_BY_P
#undef TSA_SIGMA_LAUNCH
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
