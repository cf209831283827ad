// Visiting the voxels of a cube or of a box inside it, 16 bytes per lane.
//
// Two shapes of work:
//  * contiguous: the box is one run of memory (whole cube, whole planes, one
//    row).  Blocks stride over 16-byte vectors; U vector loads are issued per
//    lane before any is consumed, so each CU keeps many bytes in flight.  The
//    few elements before the first and after the last aligned vector are
//    visited one by one by block 0.
//  * rows: a general box is ly*lz rows of lx elements.  Rows are grouped into
//    tiles; a block flattens its tile's (row, vector) pairs so that narrow
//    boxes still fill every lane.  Row starts share one alignment offset
//    (nx is a multiple of the vector width), so the first and last vector of
//    every row carry the same element masks.
#pragma once

#include "tsa_device.hpp"

namespace tsa {

struct Geom {
  const void* base;
  int32_t mode;  // 0 contiguous, 1 rows
  int32_t pad0;
  // contiguous: vectors [v0, v1) plus single elements [h0, h1) and [t0, t1)
  int64_t v0, v1, h0, h1, t0, t1;
  // rows: units are vectors (or elements on the scalar path)
  int64_t v_origin, v_ystride, v_zstride;
  uint32_t ly, nrows, vpr, rpt, ntiles;
  uint32_t head_skip, last_valid;
  uint32_t pad1;
  Magic ly_m, vpr_m;
};

// Rows [r0, r0 + nr) of a box (row r is y = r % ly, z = r / ly inside the
// box), flattened over (row, vector) so narrow rows still fill the lanes.
// Unit li (a vector, or an element on the scalar path) is column li % vpr of
// tile row li / vpr.  A lane finds its first U units with two divisions by
// invariant divisors, then steps every unit by bs*U units with constant
// increments and at most one carry per axis: no division and no 64-bit
// multiply inside the loop.
struct RowCursor {
  uint32_t j, ry, rz;  // column, y and z of the unit inside the box
  int64_t off;         // its index from the box origin, in units
};

// The elements of one 16-byte vector of a row: in_box masks the lanes before
// the box's first and past its last element when the vector is the first or
// last of its row (column j of vpr), and every element when ok is false.
template <int DT, class F>
TSA_DEV void visit_row_vec(const uint4& r, uint32_t j, uint32_t vpr, uint32_t head_skip, uint32_t last_valid,
                           bool ok, F& f) {
  using TT = Ty<DT>;
  const bool first = j == 0, last = j == vpr - 1;
#pragma unroll
  for (int e = 0; e < TT::EPV; ++e) {
    const bool in = ok && (!first || (uint32_t)e >= head_skip) && (!last || (uint32_t)e < last_valid);
    f(TT::get(r, e), in);
  }
}

template <int DT, bool VEC, int U, bool NT, class F>
TSA_DEV void walk_rows(const void* base, int64_t v_origin, int64_t v_ystride, int64_t v_zstride, uint32_t ly,
                       const Magic& ly_m, uint32_t vpr, const Magic& vpr_m, uint32_t head_skip, uint32_t last_valid,
                       uint32_t r0, uint32_t nr, F& f) {
  using TT = Ty<DT>;
  using T = typename TT::T;
  const uint32_t bs = blockDim.x;
  const uint32_t cnt = nr * vpr;
  if (cnt == 0) return;
  // the step of bs*U units as (rows, columns), the rows as (planes, y)
  const uint32_t step = bs * U;
  const uint32_t dq = mdiv(step, vpr_m), dr = step - dq * vpr;
  const uint32_t dqz = mdiv(dq, ly_m), dqy = dq - dqz * ly;
  const int64_t dstep = (int64_t)dqz * v_zstride + (int64_t)dqy * v_ystride + dr;
  RowCursor c[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t li = u * bs + threadIdx.x;
    const uint32_t lr = mdiv(li, vpr_m);
    c[u].j = li - lr * vpr;
    const uint32_t row = r0 + lr;
    c[u].rz = mdiv(row, ly_m);
    c[u].ry = row - c[u].rz * ly;
    c[u].off = (int64_t)c[u].rz * v_zstride + (int64_t)c[u].ry * v_ystride + c[u].j;
  }
  const uint4* vb = (const uint4*)base + v_origin;
  const T* sb = (const T*)base + v_origin;
  // full steps: every unit of the step lies in the tile, no per-unit test
  uint32_t li0 = 0;
  for (; li0 + step <= cnt; li0 += step) {
    if constexpr (VEC) {
      uint4 r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = load16<NT>(vb + c[u].off);
#pragma unroll
      for (int u = 0; u < U; ++u) visit_row_vec<DT>(r[u], c[u].j, vpr, head_skip, last_valid, true, f);
    } else {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = sb[c[u].off];
#pragma unroll
      for (int u = 0; u < U; ++u) f(v[u], true);
    }
    // advance every cursor by step units
#pragma unroll
    for (int u = 0; u < U; ++u) {
      RowCursor& k = c[u];
      k.j += dr;
      k.ry += dqy;
      k.rz += dqz;
      k.off += dstep;
      if (k.j >= vpr) {  // carry from the column into the row
        k.j -= vpr;
        k.ry += 1;
        k.off += v_ystride - (int64_t)vpr;
      }
      if (k.ry >= ly) {  // carry from y into z (ry < 2 ly here)
        k.ry -= ly;
        k.rz += 1;
        k.off += v_zstride - (int64_t)ly * v_ystride;
      }
    }
    f.chunk();
  }
  // the last, partial step: units past the tile load nothing and reach f
  // with in_box false, so every lane still calls f at the same points
  if (li0 < cnt) {
    if constexpr (VEC) {
      uint4 r[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ok[u] = li0 + u * bs + threadIdx.x < cnt;
        r[u] = make_uint4(0u, 0u, 0u, 0u);
        if (ok[u]) r[u] = load16<NT>(vb + c[u].off);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) visit_row_vec<DT>(r[u], c[u].j, vpr, head_skip, last_valid, ok[u], f);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = li0 + u * bs + threadIdx.x < cnt;
        T v = (T)0;
        if (ok) v = sb[c[u].off];
        f(v, ok);
      }
    }
    f.chunk();
  }
}

// f(T value, bool in_box) is called once per element slot; in_box is false
// for the masked lanes of the first/last vector of a row and for slots past
// the end of the work.  Every lane of the block calls f at the same points
// (never from divergent code), so f may use wave-wide operations that need
// every lane.  f.chunk() is called by every thread of the block at the same
// points, after at most blockDim.x * U vectors have been visited since the
// previous call, so it may synchronise the block.
template <int DT, bool VEC, int U, bool NT, class F>
TSA_DEV void walk(const Geom& g, F& f) {
  using TT = Ty<DT>;
  using T = typename TT::T;
  const T* sb = (const T*)g.base;
  const int64_t bs = blockDim.x;
  if (g.mode == 0) {
    if constexpr (VEC) {
      const uint4* vb = (const uint4*)g.base;
      const int64_t chunk = bs * U;
      const int64_t stride = chunk * gridDim.x;
      for (int64_t cb = g.v0 + (int64_t)blockIdx.x * chunk; cb < g.v1; cb += stride) {
        const int64_t i = cb + threadIdx.x;
        if (cb + chunk <= g.v1) {
          uint4 r[U];
#pragma unroll
          for (int u = 0; u < U; ++u) r[u] = load16<NT>(vb + i + u * bs);
#pragma unroll
          for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < TT::EPV; ++e) f(TT::get(r[u], e), true);
          }
        } else {  // the last, partial chunk of a block: lanes past the end see in_box false
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t j = i + u * bs;
            const bool ok = j < g.v1;
            uint4 r = make_uint4(0u, 0u, 0u, 0u);
            if (ok) r = load16<NT>(vb + j);
#pragma unroll
            for (int e = 0; e < TT::EPV; ++e) f(TT::get(r, e), ok);
          }
        }
        f.chunk();
      }
      if (blockIdx.x == 0) {
        for (int64_t e0 = g.h0; e0 < g.h1; e0 += bs) {
          const int64_t e = e0 + threadIdx.x;
          const bool ok = e < g.h1;
          T v = (T)0;
          if (ok) v = sb[e];
          f(v, ok);
        }
        for (int64_t e0 = g.t0; e0 < g.t1; e0 += bs) {
          const int64_t e = e0 + threadIdx.x;
          const bool ok = e < g.t1;
          T v = (T)0;
          if (ok) v = sb[e];
          f(v, ok);
        }
      }
    } else {
      const int64_t chunk = bs * U;
      const int64_t stride = chunk * gridDim.x;
      for (int64_t cb = g.v0 + (int64_t)blockIdx.x * chunk; cb < g.v1; cb += stride) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t j = cb + u * bs + threadIdx.x;
          const bool ok = j < g.v1;
          T v = (T)0;
          if (ok) v = sb[j];
          f(v, ok);
        }
        f.chunk();
      }
    }
    return;
  }
  // rows
  for (uint32_t t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
    const uint32_t r0 = t * g.rpt;
    walk_rows<DT, VEC, U, NT>(g.base, g.v_origin, g.v_ystride, g.v_zstride, g.ly, g.ly_m, g.vpr, g.vpr_m,
                              g.head_skip, g.last_valid, r0, min(g.rpt, g.nrows - r0), f);
  }
}

}  // namespace tsa
