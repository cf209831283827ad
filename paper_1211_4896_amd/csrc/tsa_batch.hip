// Batched region queries: thousands of sub-cube boxes, each getting moments,
// a histogram over its own [min, max] and its lower median, in ONE
// persistent kernel.
//
// Work items are tickets drawn from one device counter.  With T1 tiles in the
// whole batch (each box cut into row tiles), ticket t means
//   t in [0, T1)      phase 1: moments + first key digit of tile t
//   t in [T1, 2 T1)   phase 2: histogram + second key digit (+ candidate copy,
//                     + second moment about the mean) of tile t - T1
//   t in [2 T1, 3 T1) phase 3 (rare): last key digit of tile t - 2 T1
// The block that finishes the last tile of a box's phase runs that box's
// epilogue (merge, digit selection, next-phase set-up).  A box that is one
// tile ("solo") is finished whole by the block that draws its phase-1 ticket:
// both passes (and the rare third) back to back, its counters kept in that
// block's LDS, no other block involved and nothing to publish; its phase-2
// and phase-3 tickets are skipped.  A phase-2 tile waits
// for its box's phase-1 epilogue; a phase-3 tile skips at once unless phase 1
// left its box without a candidate copy, and then waits for the box's phase-2
// epilogue.  Tickets are handed out in increasing order, so every wait is on
// tiles already taken by running blocks that never wait on anything later:
// the kernel needs no co-resident grid and cannot deadlock.
// Every wait is bounded; a block that gives up raises an error word and the
// boxes left unfinished report TSA_EDEVICE.
#include <math.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "tsa_internal.hpp"

namespace tsa {

constexpr uint32_t kPoolPerQuery = 16384;   // candidate pool keys per query (shared by the batch)
constexpr int kBBlock = 256;
#ifndef TSA_BATCH_UNROLL
#define TSA_BATCH_UNROLL 4
#endif
constexpr int kBUnroll = TSA_BATCH_UNROLL;  // 16-byte loads in flight per lane in a tile walk
constexpr int kMaxQueries = 65536;
constexpr uint32_t kSpinLimit = 1u << 24;        // polls per wait, at most
constexpr uint64_t kWaitTicks = 100000000ull * 10;  // 10 s of the 100 MHz wall clock

struct QGeom {
  int64_t v_origin;
  uint64_t volume;
  uint32_t ly, nrows, vpr, rpt, ntiles, head_skip, last_valid, valid;
  uint32_t solo;  // one tile: the whole box in one block
  Magic ly_m, vpr_m;
};

struct QState {
  uint32_t done1, done2, done3;
  uint32_t p1_ready, p2_ready;
  uint32_t skip2, need3, compact, cand_base, cand_n, cand_fill;
  uint32_t prefix, hist_ok, var_on, finished;
  float lo, hi, scale, shift;
  uint64_t n, k;
};

struct BatchHdr {
  uint64_t T1;
  uint64_t ticket;
  // keys of the candidate pool handed out, or asked for past its end: a 64-bit
  // sum of at most 65536 buckets below 2^32 each never wraps
  uint64_t pool_top;
  uint32_t err;
  uint32_t nq, tile_units;  // tile_units: chosen on the device when the caller set none
};

// Reserves `bucket` keys of the shared candidate pool with one atomic add
// (a compare-and-swap loop costs microseconds per success when a thousand
// blocks contend).  Returns false, leaving the range to nobody, when the
// pool has no room; the counter then only grows past pool_keys.
TSA_DEV bool pool_reserve(BatchHdr* hdr, uint32_t bucket, uint32_t pool_keys, uint32_t* base) {
  const uint64_t b = atomicAdd((unsigned long long*)&hdr->pool_top, (unsigned long long)bucket);
  if (b + bucket > pool_keys) return false;
  *base = (uint32_t)b;
  return true;
}

struct BArgs {
  const void* base;
  int64_t nx, ny, nz;
  const tsa_region* regions;
  int32_t nq, nbins;
  uint32_t rshift, tile_units, max_tiles, cand_max, pool_keys;  // tile_units 0: chosen on the device
  uint32_t grid;  // persistent blocks
  uint32_t spin_limit;  // polls per wait, at most
  int32_t vec;
  tsa_result* results;
  uint64_t* hists;
  BatchHdr* hdr;
  QGeom* geom;
  QState* st;
  uint64_t* tile_base;
  uint32_t* tile_q;  // ticket (tile of the batch) -> query
  Partial* parts1;
  double* parts2;  // per tile: sum of squared deviations about the shift
  uint32_t* digits;
  uint32_t* pool;
};

// ---------------------------------------------------------------------------
// planning
// ---------------------------------------------------------------------------

// Tile size when the caller chose none: the batch's units (16-byte vectors,
// or elements on the scalar path) spread over about four tiles per persistent
// block, within [kAutoMinVoxels, kAutoMaxVoxels] voxels per tile: small
// batches cut their few boxes finely enough to fill the GPU, large ones keep
// the per-tile zeroing, flushing and counting rare.
constexpr uint32_t kAutoMinVoxels = 16384, kAutoMaxVoxels = 1u << 20;

template <int DT>
__global__ __launch_bounds__(1024) void k_bauto(BArgs a) {
  __shared__ uint64_t part[16];
  const int t = threadIdx.x;
  const int64_t epv = DT == 0 ? 4 : 8;
  uint64_t local = 0;
  for (int q = t; q < a.nq; q += blockDim.x) {
    const tsa_region r = a.regions[q];
    if (!(r.x0 >= 0 && r.y0 >= 0 && r.z0 >= 0 && r.x1 <= a.nx && r.y1 <= a.ny && r.z1 <= a.nz && r.x0 < r.x1 &&
          r.y0 < r.y1 && r.z0 < r.z1))
      continue;
    const uint64_t row = a.vec ? (uint64_t)((r.x1 + epv - 1) / epv - r.x0 / epv) : (uint64_t)(r.x1 - r.x0);
    local += row * (uint64_t)(r.y1 - r.y0) * (uint64_t)(r.z1 - r.z0);
  }
  local = wave_sum_u64(local);
  if (t % kWave == 0) part[t / kWave] = local;
  __syncthreads();
  if (t == 0) {
    uint64_t total = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) total += part[i];
    const uint64_t per_unit = a.vec ? (uint64_t)epv : 1u;  // voxels per unit
    const uint64_t lo = kAutoMinVoxels / per_unit, hi = kAutoMaxVoxels / per_unit;
    uint64_t tu = total / (4ull * a.grid);
    if (tu < lo) tu = lo;
    if (tu > hi) tu = hi;
    a.hdr->tile_units = (uint32_t)tu;
  }
}

template <int DT>
__global__ void k_bplan(BArgs a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.nq) return;
  const tsa_region r = a.regions[q];
  QGeom g;
  memset(&g, 0, sizeof(g));
  bool ok = r.x0 >= 0 && r.y0 >= 0 && r.z0 >= 0 && r.x1 <= a.nx && r.y1 <= a.ny && r.z1 <= a.nz && r.x0 < r.x1 &&
            r.y0 < r.y1 && r.z0 < r.z1;
  tsa_result res;
  res.count = 0;
  res.nan_count = 0;
  res.mean = res.m2 = res.std = res.min = res.max = res.median = __builtin_nan("");
  res.status = TSA_OK;
  res.flags = 0;
  if (ok) {
    const int64_t lx = r.x1 - r.x0, ly = r.y1 - r.y0, lz = r.z1 - r.z0;
    const uint64_t vol = (uint64_t)lx * (uint64_t)ly * (uint64_t)lz;
    const uint64_t nrows = (uint64_t)ly * (uint64_t)lz;
    ok = vol < (1ull << 32) && nrows < (1ull << 32);
    if (ok) {
      const int64_t epv = a.vec ? (DT == 0 ? 4 : 8) : 1;
      g.volume = vol;
      g.ly = (uint32_t)ly;
      g.nrows = (uint32_t)nrows;
      if (a.vec) {
        const int64_t c0 = r.x0 / epv, c1 = (r.x1 + epv - 1) / epv;
        g.v_origin = c0 + (a.nx / epv) * (r.y0 + a.ny * r.z0);
        g.vpr = (uint32_t)(c1 - c0);
        g.head_skip = (uint32_t)(r.x0 % epv);
        g.last_valid = (uint32_t)(r.x1 - (c1 - 1) * epv);
      } else {
        g.v_origin = r.x0 + a.nx * (r.y0 + a.ny * r.z0);
        g.vpr = (uint32_t)lx;
        g.head_skip = 0;
        g.last_valid = 1;
      }
      const uint32_t tu = a.tile_units ? a.tile_units : a.hdr->tile_units;
      uint64_t rpt = tu / g.vpr;
      if (rpt < 1) rpt = 1;
      uint64_t nt = (g.nrows + rpt - 1) / rpt;
      if (nt > a.max_tiles) {
        rpt = (g.nrows + a.max_tiles - 1) / a.max_tiles;
        nt = (g.nrows + rpt - 1) / rpt;
      }
      ok = rpt * g.vpr < (1ull << 31);
      g.rpt = (uint32_t)rpt;
      g.ntiles = ok ? (uint32_t)nt : 0u;
      g.ly_m = dev_magic(g.ly);
      g.vpr_m = dev_magic(g.vpr);
      g.valid = ok ? 1u : 0u;
      g.solo = (ok && nt == 1) ? 1u : 0u;
      res.nan_count = vol;  // until the moments say otherwise
    }
  }
  if (!ok) {
    g.valid = 0;
    g.ntiles = 0;
    res.status = TSA_EINVAL;
    res.flags = TSA_FLAG_BAD_REGION;
  }
  a.geom[q] = g;
  QState s;
  memset(&s, 0, sizeof(s));
  a.st[q] = s;
  a.results[q] = res;
}

// Exclusive scan of the tile counts (one block) and the batch header.
__global__ __launch_bounds__(1024) void k_bscan(BArgs a) {
  __shared__ uint64_t wsum[16];
  const int t = threadIdx.x, bs = blockDim.x;
  const int per = (a.nq + bs - 1) / bs;
  const int q0 = t * per;
  uint64_t local = 0;
  for (int i = 0; i < per; ++i)
    if (q0 + i < a.nq) local += a.geom[q0 + i].ntiles;
  const int lane = t % kWave, w = t / kWave;
  uint64_t inc = local;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  uint64_t base = inc - local, total = 0;
  for (int i = 0; i < bs / kWave; ++i) {
    if (i < w) base += wsum[i];
    total += wsum[i];
  }
  for (int i = 0; i < per; ++i) {
    if (q0 + i < a.nq) {
      const uint32_t nt = a.geom[q0 + i].ntiles;
      a.tile_base[q0 + i] = base;
      for (uint32_t k = 0; k < nt; ++k) a.tile_q[base + k] = (uint32_t)(q0 + i);
      base += nt;
    }
  }
  if (t == 0) {
    a.tile_base[a.nq] = total;
    a.hdr->T1 = total;
    a.hdr->nq = (uint32_t)a.nq;
  }
}

// ---------------------------------------------------------------------------
// block helpers of the persistent kernel
// ---------------------------------------------------------------------------
struct BShared {
  uint64_t t;
  uint32_t q, tile, last, flag;
  uint32_t cand_base, compact;
  Partial part;
  MomShared mom;
  alignas(16) uint32_t wsum32[16];
  uint32_t found, sel_digit, sel_cum32, sel_bucket32;
};

// The epilogues' per-thread merge arrays live in the dynamic LDS, past the
// words epilogue 2 counts into: a tile's counters are flushed before its
// block can run an epilogue, so the space is free then (this keeps the static
// LDS small and lets more blocks share a compute unit).
constexpr uint32_t kEpOffWords = 1024;
struct EpScratch {
  double* mn;
  double* mm;
  double* mq;
  uint32_t* kmin;
  uint32_t* kmax;
};
TSA_DEV EpScratch ep_scratch(uint32_t* lds) {
  double* d = (double*)(lds + kEpOffWords);
  uint32_t* u = (uint32_t*)(d + 3 * kBBlock);
  return EpScratch{d, d + kBBlock, d + 2 * kBBlock, u, u + kBBlock};
}
constexpr size_t kEpLdsBytes = (size_t)kEpOffWords * 4 + (3 * 8 + 2 * 4) * (size_t)kBBlock;

// Thread 0 waits until *p >= v (bounded by `limit` polls and kWaitTicks);
// result broadcast to the block.
TSA_DEV bool block_wait_ge(const uint32_t* p, uint32_t v, uint32_t* err, BShared& sh, uint32_t limit) {
  if (threadIdx.x == 0) {
    uint32_t ok = 0;
    const uint64_t t0 = wall_clock64();
    for (uint32_t it = 0; it < limit; ++it) {
      // relaxed polls, one acquire once the value is there (an agent-scope
      // acquire invalidates this XCD's L2)
      if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= v) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = 1;
        break;
      }
      if ((it & 255u) == 255u) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        if (wall_clock64() - t0 > kWaitTicks) break;
      }
      // back off after a few quick polls: hundreds of waiting blocks polling
      // one word at full rate slow down the loads of the blocks still working
      if (it < 16)
        __builtin_amdgcn_s_sleep(4);
      else
        __builtin_amdgcn_s_sleep(127);
    }
    if (!ok) atomicOr(err, 1u);
    sh.flag = ok;
  }
  __syncthreads();
  const bool ok = sh.flag != 0;
  __syncthreads();
  return ok;
}

// Every wave waits until its own global stores and atomics are acknowledged
// (s_waitcnt vmcnt(0)) before the barrier after which one thread publishes
// the block's work with an agent-scope release: a workgroup barrier alone
// does not wait for other waves' writes to reach the L2 that the release
// writes back.
TSA_DEV void block_writes_done() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt 0; expcnt and lgkmcnt not waited for
  __syncthreads();
}

// ---------------------------------------------------------------------------
// epilogues (whole block)
// ---------------------------------------------------------------------------
template <int DT>
TSA_DEV void epilogue1(const BArgs& a, uint32_t q, BShared& sh, uint32_t* lds) {
  const EpScratch ep = ep_scratch(lds);
  const QGeom& g = a.geom[q];
  QState& s = a.st[q];
  tsa_result& R = a.results[q];
  const int t = threadIdx.x, bs = blockDim.x;
  const uint64_t tb = a.tile_base[q];
  // fixed-order Chan merge of the tile partials
  double n = 0.0, m = 0.0, m2 = 0.0;
  uint32_t mn = 0xFFFFFFFFu, mx = 0u;
  for (uint32_t i = t; i < g.ntiles; i += bs) {
    const Partial p = a.parts1[tb + i];
    double pn, pm, pq;
    partial_stats(p, DT, pn, pm, pq);
    chan_merge(n, m, m2, pn, pm, pq);
    if (p.n) {
      mn = min(mn, p.kmin);
      mx = max(mx, p.kmax);
    }
  }
  ep.mn[t] = n;
  ep.mm[t] = m;
  ep.mq[t] = m2;
  ep.kmin[t] = mn;
  ep.kmax[t] = mx;
  __syncthreads();
  for (int s2 = bs / 2; s2 > 0; s2 >>= 1) {
    if (t < s2) {
      double x = ep.mn[t], y = ep.mm[t], z = ep.mq[t];
      chan_merge(x, y, z, ep.mn[t + s2], ep.mm[t + s2], ep.mq[t + s2]);
      ep.mn[t] = x;
      ep.mm[t] = y;
      ep.mq[t] = z;
      ep.kmin[t] = min(ep.kmin[t], ep.kmin[t + s2]);
      ep.kmax[t] = max(ep.kmax[t], ep.kmax[t + s2]);
    }
    __syncthreads();
  }
  const uint64_t cnt = (uint64_t)ep.mn[0];
  const double mean = ep.mm[0];
  const uint32_t kmin = ep.kmin[0], kmax = ep.kmax[0];
  const uint32_t* dig = a.digits + (size_t)q * kBins1;
  bool skip2 = false;
  if (t == 0) {
    R.count = cnt;
    R.nan_count = g.volume - cnt;
    s.n = cnt;
    if (cnt == 0) {
      R.flags |= TSA_FLAG_HIST_SKIPPED;
      s.finished = 1;
    } else {
      const double vmin = bvalue_of_key(kmin, DT), vmax = bvalue_of_key(kmax, DT);
      R.min = vmin;
      R.max = vmax;
      if (kmin == kmax) {
        R.mean = vmin;
        R.m2 = 0.0;
        R.std = 0.0;
        R.median = vmin;
        if (isfinite((float)vmin))
          a.hists[(size_t)q * a.nbins] = cnt;  // lo == hi: every value in bin 0
        else
          R.flags |= TSA_FLAG_HIST_SKIPPED;  // an infinite range has no bins
        s.finished = 1;
      } else {
        const double q2 = ep.mq[0] < 0.0 ? 0.0 : ep.mq[0];  // NaN (infinite values) stays
        R.mean = mean;
        R.m2 = q2;
        R.std = sqrt(q2 / (double)cnt);
      }
    }
  }
  skip2 = cnt == 0 || kmin == kmax;
  if (!skip2) {
    const uint32_t k = (uint32_t)((cnt - 1) / 2);  // a box holds fewer than 2^32 voxels
    uint32_t d, cum, bucket;
    const bool found = block_select_small(dig, kBins1, k, sh, &d, &cum, &bucket);
    // the first-digit counts become the second-digit counts: clear them
    for (int i = t; i < kBins1; i += bs) a.digits[(size_t)q * kBins1 + i] = 0u;
    if (t == 0) {
      if (!found) {
        R.status = TSA_EDEVICE;
        skip2 = true;
        s.finished = 1;
      } else {
        s.prefix = d << kShift1;
        s.k = k - cum;
        float lo = (float)bvalue_of_key(kmin, DT), hi = (float)bvalue_of_key(kmax, DT), scale = 0.f;
        uint32_t ok = 0;
        if (isfinite(lo) && isfinite(hi)) {
          const float width = hi - lo;
          if (isfinite(width)) {
            scale = (float)a.nbins / width;
            ok = (isfinite(scale) && scale != 0.0f) ? 1u : 0u;
          }
        }
        s.lo = lo;
        s.hi = hi;
        s.scale = scale;
        s.hist_ok = ok;
        if (!ok) R.flags |= TSA_FLAG_HIST_SKIPPED;
        s.var_on = (DT == 0 && isfinite(mean) && one_pass_m2_at_risk(mean, R.m2 / (double)cnt)) ? 1u : 0u;
        s.shift = s.var_on ? (float)mean : 0.0f;
        s.compact = 0;
        // int16 keys are complete after the second digit: no candidates needed.
        // A box that finds the pool full takes the third pass instead.
        uint32_t base = 0;
        if (DT == 0 && bucket <= a.cand_max && pool_reserve(a.hdr, bucket, a.pool_keys, &base)) {
          s.compact = 1;
          s.cand_base = base;
          s.cand_n = (uint32_t)bucket;
        }
      }
    }
  }
  block_writes_done();  // every thread's clearing of the digit counts precedes the release below
  if (t == 0) {
    s.skip2 = skip2 ? 1u : 0u;
    __hip_atomic_store(&s.p1_ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

template <int DT>
TSA_DEV void epilogue2(const BArgs& a, uint32_t q, BShared& sh, uint32_t* lds) {
  const QGeom& g = a.geom[q];
  QState& s = a.st[q];
  tsa_result& R = a.results[q];
  const int t = threadIdx.x, bs = blockDim.x;
  const EpScratch ep = ep_scratch(lds);
  if (!s.skip2) {
    const uint64_t n = s.n;
    if (DT == 0 && s.var_on) {
      const uint64_t tb = a.tile_base[q];
      double x = 0.0;
      for (uint32_t i = t; i < g.ntiles; i += bs) x += a.parts2[tb + i];
      ep.mm[t] = x;
      __syncthreads();
      for (int s2 = bs / 2; s2 > 0; s2 >>= 1) {
        if (t < s2) ep.mm[t] += ep.mm[t + s2];
        __syncthreads();
      }
      if (t == 0) {
        const double dm = R.mean - (double)s.shift;
        double m2 = ep.mm[0] - (double)n * dm * dm;
        if (m2 < 0.0) m2 = 0.0;  // rounding below zero; NaN (infinite values) stays
        R.m2 = m2;
        R.std = sqrt(m2 / (double)n);
      }
      __syncthreads();
    }
    uint32_t* dig = a.digits + (size_t)q * kBins1;
    uint32_t d, cum, bucket;
    bool found = block_select_small(dig, kBins2, (uint32_t)s.k, sh, &d, &cum, &bucket);
    const uint32_t prefix = s.prefix | (d << kShift2);
    const uint32_t k2 = (uint32_t)s.k - cum;
    if (!found) {
      if (t == 0) {
        R.status = TSA_EDEVICE;
        s.finished = 1;
      }
    } else if (DT == 1) {  // int16 keys have no bits below the second digit
      if (t == 0) {
        R.median = bvalue_of_key(prefix, DT);
        s.finished = 1;
      }
    } else if (s.compact) {
      // last 8 bits from the copied candidates
      for (int i = t; i < kBins3; i += bs) lds[i] = 0u;
      __syncthreads();
      const uint32_t* c = a.pool + s.cand_base;
      const uint32_t nc = min(s.cand_n, __hip_atomic_load(&s.cand_fill, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      const uint32_t p2 = prefix >> kShift2;
      for (uint32_t i = t; i < nc; i += bs) {
        const uint32_t key = c[i];
        if ((key >> kShift2) == p2) lds_inc(lds, key & 0xFFu);
      }
      __syncthreads();
      uint32_t d3, cum3, b3;
      found = block_select_small(lds, kBins3, k2, sh, &d3, &cum3, &b3);
      if (t == 0) {
        if (found)
          R.median = bvalue_of_key(prefix | d3, DT);
        else
          R.status = TSA_EDEVICE;
        s.finished = 1;
      }
    } else {
      for (int i = t; i < kBins3; i += bs) dig[i] = 0u;
      if (t == 0) {
        s.prefix = prefix;
        s.k = k2;
        s.need3 = 1;
        R.flags |= TSA_FLAG_PHASE3;
      }
    }
  }
  block_writes_done();  // every thread's clearing of the digit counts precedes the release below
  if (t == 0) {
    __hip_atomic_store(&s.p2_ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

template <int DT>
TSA_DEV void epilogue3(const BArgs& a, uint32_t q, BShared& sh) {
  QState& s = a.st[q];
  uint32_t d, cum, bucket;
  const bool found = block_select_small(a.digits + (size_t)q * kBins1, kBins3, (uint32_t)s.k, sh, &d, &cum, &bucket);
  if (threadIdx.x == 0) {
    if (found)
      a.results[q].median = bvalue_of_key(s.prefix | d, DT);
    else
      a.results[q].status = TSA_EDEVICE;
    s.finished = 1;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// per-tile accumulators
// ---------------------------------------------------------------------------
template <int DT>
struct BPass1 {
  MomAcc<DT, false> mom;  // the count is the digit histogram's total
  Digit1Acc<DT> d1;
  template <class T>
  TSA_DEV void operator()(T raw, bool in) {
    mom(raw, in);
    d1(raw, in);
  }
  TSA_DEV void chunk() {}
};

template <int DT>
struct BPass2 {
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

template <int DT, bool VEC, bool NT, class F>
TSA_DEV void walk_tile(const BArgs& a, const QGeom& g, uint32_t tile, F& f) {
  const uint32_t r0 = tile * g.rpt;
  const uint32_t nr = min(g.rpt, g.nrows - r0);
  const int64_t epv = VEC ? (DT == 0 ? 4 : 8) : 1;
  const int64_t ys = a.nx / epv, zs = (a.nx / epv) * a.ny;
  walk_rows<DT, VEC, kBUnroll, NT>(a.base, g.v_origin, ys, zs, g.ly, g.ly_m, g.vpr, g.vpr_m, g.head_skip,
                                   g.last_valid, r0, nr, f);
}

// ---------------------------------------------------------------------------
// a one-tile box, whole, in one block (phase-1 ticket of a solo box)
// ---------------------------------------------------------------------------
// The same steps and arithmetic as the tiled path -- the partial, the merge of
// one partial, the digit choices, the histogram formula, the candidate pool
// -- so the results are the same bits; only the counters stay in LDS between
// the passes instead of going through global memory and the epilogues.
template <int DT, bool VEC, bool NT, class CS>
TSA_DEV void solo_box(const BArgs& a, uint32_t q, BShared& sh, CS& cs, uint32_t* lds) {
  const QGeom& g = a.geom[q];
  QState& s = a.st[q];
  tsa_result& R = a.results[q];
  const int t = threadIdx.x;
  // pass 1: moments + first key digit
  lds_zero(lds, kBins1 + kTrash);
  __syncthreads();
  BPass1<DT> f{MomAcc<DT, false>{}, Digit1Acc<DT>{lds, 0u, 0u}};
  walk_tile<DT, VEC, NT>(a, g, 0u, f);
  __syncthreads();
  uint32_t c = 0;  // every valid value incremented one first-digit counter
  for (int b = t; b < kBins1; b += kBBlock) c += lds[b];
  f.mom.cnt = c;
  block_store_partial(f.mom, sh.mom, &sh.part);
  __syncthreads();
  const Partial p = sh.part;
  double n = 0.0, mean = 0.0, m2 = 0.0;
  partial_stats(p, DT, n, mean, m2);
  const uint64_t cnt = p.n;
  const uint32_t kmin = cnt ? p.kmin : 0xFFFFFFFFu, kmax = cnt ? p.kmax : 0u;
  const double vmin = bvalue_of_key(kmin, DT), vmax = bvalue_of_key(kmax, DT);
  if (t == 0) {
    R.count = cnt;
    R.nan_count = g.volume - cnt;
    s.n = cnt;
    if (cnt == 0) {
      R.flags |= TSA_FLAG_HIST_SKIPPED;
    } else {
      R.min = vmin;
      R.max = vmax;
      if (kmin == kmax) {
        R.mean = vmin;
        R.m2 = 0.0;
        R.std = 0.0;
        R.median = vmin;
        if (isfinite((float)vmin))
          a.hists[(size_t)q * a.nbins] = cnt;  // lo == hi: every value in bin 0
        else
          R.flags |= TSA_FLAG_HIST_SKIPPED;  // an infinite range has no bins
      } else {
        const double q2 = m2 < 0.0 ? 0.0 : m2;  // NaN (infinite values) stays
        R.mean = mean;
        R.m2 = q2;
        R.std = sqrt(q2 / (double)cnt);
      }
    }
  }
  if (cnt == 0 || kmin == kmax) {
    if (t == 0) s.finished = 1;
    return;
  }
  const uint32_t k = (uint32_t)((cnt - 1) / 2);  // a box holds fewer than 2^32 voxels
  uint32_t d, cum, bucket;
  if (!block_select_small(lds, kBins1, k, sh, &d, &cum, &bucket)) {
    if (t == 0) {
      R.status = TSA_EDEVICE;
      s.finished = 1;
    }
    return;
  }
  const uint32_t prefix = d << kShift1;
  const uint32_t k2 = k - cum;
  // the histogram's range and scale, the shift of the second moment (every
  // thread computes the same values)
  const float lo = (float)vmin, hi = (float)vmax;
  float scale = 0.f;
  bool hist_on = false;
  if (isfinite(lo) && isfinite(hi)) {
    const float width = hi - lo;
    if (isfinite(width)) {
      scale = (float)a.nbins / width;
      hist_on = isfinite(scale) && scale != 0.0f;
    }
  }
  const double q2 = m2 < 0.0 ? 0.0 : m2;
  const bool var_on = DT == 0 && isfinite(mean) && one_pass_m2_at_risk(mean, q2 / (double)cnt);
  const float shift = var_on ? (float)mean : 0.0f;
  if (t == 0) {
    if (!hist_on) R.flags |= TSA_FLAG_HIST_SKIPPED;
    // candidate pool reservation, as the tiled path makes it
    uint32_t base = 0;
    const uint32_t compact =
        (DT == 0 && bucket <= a.cand_max && pool_reserve(a.hdr, bucket, a.pool_keys, &base)) ? 1u : 0u;
    sh.compact = compact;
    sh.cand_base = base;
  }
  __syncthreads();
  const bool compact = sh.compact != 0;
  const uint32_t cand_base = sh.cand_base;
  // pass 2: histogram + second key digit (+ candidate copy, + second moment about the shift)
  const uint32_t hsize = ((uint32_t)a.nbins << a.rshift) + kTrash;
  uint32_t* l2 = lds + hsize;
  lds_zero(lds, hsize + kBins2);
  __syncthreads();
  BPass2<DT> f2{HistOwnAcc{lds, lo, scale, a.nbins - 1, a.rshift, (uint32_t)t & ((1u << a.rshift) - 1u)},
                Level2Acc<DT>{l2, prefix >> kShift1, compact, cand_sink(cs, a.pool + cand_base, &s.cand_fill, bucket)},
                VarAcc{shift}, hist_on, var_on};
  walk_tile<DT, VEC, NT>(a, g, 0u, f2);
  f2.l2.finish();
  __syncthreads();
  if (hist_on) lds_flush(lds, (uint32_t)a.nbins, a.rshift, a.hists + (size_t)q * a.nbins);
  if (var_on) {
    const double vq = wave_sum_f64(f2.var.q);
    const int w = t / kWave, lane = t % kWave;
    if (lane == 0) sh.mom.q[w] = vq;
    __syncthreads();
    if (t == 0) {
      double bq = sh.mom.q[0];
      for (int i = 1; i < kBBlock / kWave; ++i) bq += sh.mom.q[i];
      const double dm = R.mean - (double)shift;
      double v = bq - (double)cnt * dm * dm;
      if (v < 0.0) v = 0.0;  // rounding below zero; NaN (infinite values) stays
      R.m2 = v;
      R.std = sqrt(v / (double)cnt);
    }
  }
  uint32_t d2, cum2, b2;
  if (!block_select_small(l2, kBins2, k2, sh, &d2, &cum2, &b2)) {  // ends with a barrier
    if (t == 0) {
      R.status = TSA_EDEVICE;
      s.finished = 1;
    }
    return;
  }
  const uint32_t prefix2 = prefix | (d2 << kShift2);
  const uint32_t k3 = k2 - cum2;
  if (DT == 1) {  // int16 keys have no bits below the second digit
    if (t == 0) {
      R.median = bvalue_of_key(prefix2, DT);
      s.finished = 1;
    }
    return;
  }
  // last 8 bits: from the copied candidates, else a third pass over the box
  for (int i = t; i < kBins3; i += kBBlock) lds[i] = 0u;
  __syncthreads();
  if (compact) {
    const uint32_t* cl = a.pool + cand_base;
    const uint32_t nc = min(bucket, __hip_atomic_load(&s.cand_fill, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint32_t p2 = prefix2 >> kShift2;
    for (uint32_t i = t; i < nc; i += kBBlock) {
      const uint32_t key = cl[i];
      if ((key >> kShift2) == p2) lds_inc(lds, key & 0xFFu);
    }
  } else {
    Level3Acc<DT> f3{lds, prefix2 >> kShift2};
    walk_tile<DT, VEC, NT>(a, g, 0u, f3);
    if (t == 0) R.flags |= TSA_FLAG_PHASE3;
  }
  __syncthreads();
  uint32_t d3, cum3, b3;
  const bool found = block_select_small(lds, kBins3, k3, sh, &d3, &cum3, &b3);
  if (t == 0) {
    if (found)
      R.median = bvalue_of_key(prefix2 | d3, DT);
    else
      R.status = TSA_EDEVICE;
    s.finished = 1;
  }
}

// ---------------------------------------------------------------------------
// the persistent kernel
// ---------------------------------------------------------------------------
template <int DT, bool VEC, bool NT>
__global__ __launch_bounds__(kBBlock) void k_batch(BArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  __shared__ BShared sh;
  __shared__ CandSharedN<kBBlock / kWave> cs;
  const int t = threadIdx.x;
  const uint64_t T1 = a.hdr->T1;
  for (;;) {
    if (t == 0) sh.t = atomicAdd((unsigned long long*)&a.hdr->ticket, 1ull);
    __syncthreads();
    const uint64_t tk = sh.t;
    __syncthreads();
    int phase;
    uint64_t lt;
    if (tk < T1) {
      phase = 1;
      lt = tk;
    } else if (tk < 2 * T1) {
      phase = 2;
      lt = tk - T1;
    } else {
      phase = 3;
      lt = tk - 2 * T1;
      if (lt >= T1) return;  // every ticket handed out
    }
    // ticket -> (query, tile).  Tiles are taken box after box, so each box
    // finishes its phase early and its next-phase tiles seldom wait for it.
    if (t == 0) {
      const uint32_t qq = a.tile_q[lt];
      sh.q = qq;
      sh.tile = (uint32_t)(lt - a.tile_base[qq]);
    }
    __syncthreads();
    const uint32_t q = sh.q, tile = sh.tile;
    __syncthreads();
    const QGeom& g = a.geom[q];
    QState& s = a.st[q];

    if (g.solo) {  // uniform across the block (every thread read the same q)
      if (phase == 1) solo_box<DT, VEC, NT>(a, q, sh, cs, lds);
      __syncthreads();
      continue;  // its other tickets have nothing to do
    }
    if (phase == 1) {
      lds_zero(lds, kBins1 + kTrash);
      __syncthreads();
      BPass1<DT> f{MomAcc<DT, false>{}, Digit1Acc<DT>{lds, 0u, 0u}};
      walk_tile<DT, VEC, NT>(a, g, tile, f);
      __syncthreads();
      uint32_t c = 0;  // every valid value incremented one first-digit counter
      for (int b = t; b < kBins1; b += kBBlock) c += lds[b];
      f.mom.cnt = c;
      block_store_partial(f.mom, sh.mom, a.parts1 + a.tile_base[q] + tile);
      __syncthreads();
      uint32_t* dig = a.digits + (size_t)q * kBins1;
      for (int b = t; b < kBins1; b += kBBlock) {
        const uint32_t c = lds[b];
        if (c) atomicAdd(dig + b, c);
      }
    } else if (phase == 2) {
      if (!block_wait_ge(&s.p1_ready, 1u, &a.hdr->err, sh, a.spin_limit)) return;
      if (!s.skip2) {
        const uint32_t hsize = ((uint32_t)a.nbins << a.rshift) + kTrash;
        uint32_t* l2 = lds + hsize;
        lds_zero(lds, hsize + kBins2);
        __syncthreads();
        const bool hist_on = s.hist_ok != 0, var_on = DT == 0 && s.var_on != 0;
        BPass2<DT> f{HistOwnAcc{lds, s.lo, s.scale, a.nbins - 1, a.rshift, (uint32_t)t & ((1u << a.rshift) - 1u)},
                     Level2Acc<DT>{l2, s.prefix >> kShift1, s.compact != 0,
                                   cand_sink(cs, a.pool + s.cand_base, &s.cand_fill, s.cand_n)},
                     VarAcc{s.shift}, hist_on, var_on};
        walk_tile<DT, VEC, NT>(a, g, tile, f);
        f.l2.finish();
        __syncthreads();
        if (hist_on) lds_flush(lds, (uint32_t)a.nbins, a.rshift, a.hists + (size_t)q * a.nbins);
        uint32_t* dig = a.digits + (size_t)q * kBins1;
        for (int b = t; b < kBins2; b += kBBlock) {
          const uint32_t c = l2[b];
          if (c) atomicAdd(dig + b, c);
        }
        if (var_on) {
          __syncthreads();
          const double vq = wave_sum_f64(f.var.q);
          const int w = t / kWave, lane = t % kWave;
          if (lane == 0) sh.mom.q[w] = vq;
          __syncthreads();
          if (t == 0) {
            double bq = sh.mom.q[0];
            for (int i = 1; i < kBBlock / kWave; ++i) bq += sh.mom.q[i];
            a.parts2[a.tile_base[q] + tile] = bq;
          }
        }
      }
    } else {
      // only a box left without a candidate copy can need the last digit
      if (!block_wait_ge(&s.p1_ready, 1u, &a.hdr->err, sh, a.spin_limit)) return;
      if (t == 0) sh.flag = (DT == 0 && s.skip2 == 0 && s.compact == 0) ? 1u : 0u;
      __syncthreads();
      const bool may3 = sh.flag != 0;
      __syncthreads();
      if (!may3) continue;
      if (!block_wait_ge(&s.p2_ready, 1u, &a.hdr->err, sh, a.spin_limit)) return;
      if (t == 0) sh.flag = s.need3;
      __syncthreads();
      const bool need3 = sh.flag != 0;
      __syncthreads();
      if (!need3) continue;
      lds_zero(lds, kBins3);
      __syncthreads();
      Level3Acc<DT> f{lds, s.prefix >> kShift2};
      walk_tile<DT, VEC, NT>(a, g, tile, f);
      __syncthreads();
      uint32_t* dig = a.digits + (size_t)q * kBins1;
      for (int b = t; b < kBins3; b += kBBlock) {
        const uint32_t c = lds[b];
        if (c) atomicAdd(dig + b, c);
      }
    }
    // count the tile; the block finishing the last one runs the epilogue
    block_writes_done();
    if (t == 0) {
      // the release publishes this tile's partial and counters (the block's
      // writes precede it through the barrier above); only the block that
      // counts the last tile acquires, since only it reads the others' work.
      // Each agent-scope release writes back this XCD's L2 and each acquire
      // invalidates it, so a tile pays one of the first and none of the second.
      uint32_t* cnt = phase == 1 ? &s.done1 : phase == 2 ? &s.done2 : &s.done3;
      const uint32_t prev = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      sh.last = prev + 1 == g.ntiles ? 1u : 0u;
      if (sh.last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (sh.last) {
      if (phase == 1)
        epilogue1<DT>(a, q, sh, lds);
      else if (phase == 2)
        epilogue2<DT>(a, q, sh, lds);
      else
        epilogue3<DT>(a, q, sh);
    }
    __syncthreads();
  }
}

// Boxes left unfinished (a bounded wait gave up) report a device error.
__global__ void k_bfinal(BArgs a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.nq) return;
  if (a.geom[q].valid && !a.st[q].finished) a.results[q].status = TSA_EDEVICE;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct BLayout {
  size_t hdr, geom, st, tile_base, tile_q, parts1, parts2, digits, pool, total;
  uint32_t max_tiles, pool_keys;
};

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

static BLayout batch_layout(int32_t nq) {
  BLayout L;
  uint32_t mt = (1u << 20) / (uint32_t)nq;
  if (mt > 256) mt = 256;
  if (mt < 16) mt = 16;
  L.max_tiles = mt;
  size_t o = 0;
  L.hdr = o;
  o = al(o + sizeof(BatchHdr));
  L.geom = o;
  o = al(o + sizeof(QGeom) * (size_t)nq);
  L.st = o;
  o = al(o + sizeof(QState) * (size_t)nq);
  L.tile_base = o;
  o = al(o + 8 * ((size_t)nq + 1));
  L.tile_q = o;
  o = al(o + 4 * (size_t)nq * mt);
  L.parts1 = o;
  o = al(o + sizeof(Partial) * (size_t)nq * mt);
  L.parts2 = o;
  o = al(o + sizeof(double) * (size_t)nq * mt);
  L.digits = o;
  o = al(o + 4 * (size_t)kBins1 * nq);
  uint64_t pk = (uint64_t)kPoolPerQuery * (uint64_t)nq;
  if (pk < (1ull << 20)) pk = 1ull << 20;
  if (pk > (1ull << 28)) pk = 1ull << 28;
  L.pool_keys = (uint32_t)pk;
  L.pool = o;
  o = al(o + 4 * (size_t)pk);
  L.total = o;
  return L;
}

size_t batch_ws_bytes(const tsa_cube* cube, int32_t nbins, int32_t nq) {
  if (check_cube(cube) != TSA_OK || nq < 1 || nq > kMaxQueries || nbins < 1 || nbins > 4096) return 0;
  return batch_layout(nq).total;
}

static void bfill3(void* p0, size_t n0, void* p1, size_t n1, void* p2, size_t n2, hipStream_t s);

// launch choices of this thread's last enqueued batch (tsa_internal_batch_last_config)
struct BatchConfig {
  int32_t tile_units, bpc, replicas, cand_max;
  bool set;
};
static thread_local BatchConfig g_last_config = {0, 0, 0, 0, false};

// log2 of the LDS replicas per histogram bin of phase 2: the caller's choice
// (0: 4 up to 1024 bins, 2 up to 2048, else 1), reduced while the phase-2
// counters (replicated bins + second-digit bins) would not fit one launch's
// 64 KB or the block's share of the compute unit's LDS.
uint32_t batch_rep_shift(int32_t nbins, int replicas, size_t lds_per_cu, int bpc) {
  uint32_t r = replicas == 0 ? (nbins <= 1024 ? 2u : nbins <= 2048 ? 1u : 0u)
                             : (uint32_t)__builtin_ctz((unsigned)replicas);
  size_t cap = lds_per_cu / (size_t)(bpc > 0 ? bpc : 1);
  if (cap > 65536) cap = 65536;
  cap = cap > 4096 ? cap - 4096 : 0;  // the kernel's static LDS (about 3.2 KB)
  while (r > 0 && ((((size_t)nbins << r) + kTrash + kBins2) * 4) > cap) --r;
  return r;
}

static int enqueue_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                                tsa_result* d_results, uint64_t* d_hists, const tsa_tune* tune, void* d_ws,
                                size_t ws_bytes, hipStream_t s);
bool tune_lookup(const tsa_cube* cube, int32_t nbins, int32_t nq, tsa_tune* out);

// ---- graph cache -------------------------------------------------------------
// A launch sequence of one argument set (clears, plan, scan, persistent
// kernel, final check; or the passes of tsa_stats) is captured once into a HIP
// graph on a private stream and replayed on the caller's stream afterwards.
// Entries are keyed by every argument; the cache keeps the most recent
// kGraphCap of them.
namespace {
constexpr size_t kGraphCap = 256;
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
  uint64_t used;
};
struct GraphCache {
  std::mutex mu;
  std::vector<GraphEntry> entries;
  std::vector<GraphKey> seen;  // argument sets launched once, directly (most recent kSeenCap)
  uint64_t clock = 0;
};
constexpr size_t kSeenCap = 1024;
GraphCache& graphs() {
  static GraphCache g;
  return g;
}
bool same_key(const GraphKey& a, const GraphKey& b) { return memcmp(a.v, b.v, sizeof(a.v)) == 0; }
}  // namespace

// Polls per bounded wait when set (>= 0) by tsa_internal_batch_wait_limit;
// -1: kSpinLimit.  Calls made while it is set launch directly (no graph).
static std::atomic<int64_t> g_wait_polls{-1};

bool graphs_enabled() {
  static const bool on = [] {
    const char* e = getenv("TSA_GRAPH");
    return !(e && e[0] == '0');
  }();
  return on;
}

int graph_run(const GraphKey& key, hipStream_t s, int (*enqueue)(void* ctx, hipStream_t), void* ctx) {
  GraphCache& G = graphs();
  bool again = false;
  {
    std::lock_guard<std::mutex> g(G.mu);
    for (GraphEntry& e : G.entries) {
      if (same_key(e.key, key)) {
        e.used = ++G.clock;
        return hipGraphLaunch(e.exec, s) == hipSuccess ? TSA_OK : TSA_EDEVICE;
      }
    }
    // an argument set is captured the second time it comes: one-off calls
    // (fresh buffers every time) launch directly and cost no capture
    for (size_t i = 0; i < G.seen.size() && !again; ++i) again = same_key(G.seen[i], key);
    if (!again) {
      if (G.seen.size() >= kSeenCap) G.seen.erase(G.seen.begin());
      G.seen.push_back(key);
    }
  }
  if (!again) return enqueue(ctx, s);
  thread_local hipStream_t cap = nullptr;
  if (!cap && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return TSA_EDEVICE;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return TSA_EDEVICE;
  const int st = enqueue(ctx, cap);
  hipGraph_t graph = nullptr;
  const bool ended = hipStreamEndCapture(cap, &graph) == hipSuccess;
  if (st != TSA_OK || !ended || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return st != TSA_OK ? st : TSA_EDEVICE;
  }
  hipGraphExec_t exec = nullptr;
  const bool inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
  (void)hipGraphDestroy(graph);
  if (!inst) return TSA_EDEVICE;
  {
    std::lock_guard<std::mutex> g(G.mu);
    if (G.entries.size() >= kGraphCap) {
      size_t victim = 0;
      for (size_t i = 1; i < G.entries.size(); ++i)
        if (G.entries[i].used < G.entries[victim].used) victim = i;
      (void)hipGraphExecDestroy(G.entries[victim].exec);
      G.entries.erase(G.entries.begin() + victim);
    }
    G.entries.push_back(GraphEntry{key, exec, ++G.clock});
  }
  return hipGraphLaunch(exec, s) == hipSuccess ? TSA_OK : TSA_EDEVICE;
}

namespace {
struct BatchCall {
  const tsa_cube* cube;
  const tsa_region* d_regions;
  int32_t nq, nbins;
  tsa_result* d_results;
  uint64_t* d_hists;
  const tsa_tune* tune;
  void* d_ws;
  size_t ws_bytes;
};
int enqueue_batch_call(void* ctx, hipStream_t s) {
  const BatchCall& c = *(const BatchCall*)ctx;
  return enqueue_region_batch(c.cube, c.d_regions, c.nq, c.nbins, c.d_results, c.d_hists, c.tune, c.d_ws,
                              c.ws_bytes, s);
}
}  // namespace

int run_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                     tsa_result* d_results, uint64_t* d_hists, const tsa_tune* tune, void* d_ws, size_t ws_bytes,
                     tsa_stream_t stream) {
  int st = check_cube(cube);
  if (st) return st;
  if (!d_regions || !d_results || !d_hists || nq < 1 || nq > kMaxQueries || nbins < 1 || nbins > 4096)
    return TSA_EINVAL;
  if (!d_ws || ws_bytes < batch_layout(nq).total) return TSA_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  tsa_tune tuned;
  if (!tune && tune_lookup(cube, nbins, nq, &tuned)) tune = &tuned;
  if (!graphs_enabled() || trace_active() || g_wait_polls.load() >= 0)
    return enqueue_region_batch(cube, d_regions, nq, nbins, d_results, d_hists, tune, d_ws, ws_bytes, s);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TSA_EDEVICE;
  GraphKey key;
  memset(&key, 0, sizeof(key));
  key.v[0] = 1;  // the region batch
  key.v[1] = (uintptr_t)cube->data;
  key.v[2] = (uintptr_t)cube->dtype;
  key.v[3] = (uintptr_t)cube->nx;
  key.v[4] = (uintptr_t)cube->ny;
  key.v[5] = (uintptr_t)cube->nz;
  key.v[6] = (uintptr_t)d_regions;
  key.v[7] = (uintptr_t)nq;
  key.v[8] = (uintptr_t)nbins;
  key.v[9] = (uintptr_t)d_results;
  key.v[10] = (uintptr_t)d_hists;
  key.v[11] = (uintptr_t)d_ws;
  key.v[12] = (uintptr_t)ws_bytes;
  key.v[13] = (uintptr_t)dev;
  if (tune) {
    key.v[14] = ((uintptr_t)(uint32_t)tune->tile_voxels << 32) | (uint32_t)tune->block_threads;
    key.v[15] = ((uintptr_t)(uint32_t)tune->blocks_per_cu << 32) | (uint32_t)tune->cand_max;
    key.v[16] = 1;
    key.v[17] = (uintptr_t)(uint32_t)tune->replicas;
  }
  BatchCall c{cube, d_regions, nq, nbins, d_results, d_hists, tune, d_ws, ws_bytes};
  return graph_run(key, s, enqueue_batch_call, &c);
}

static int enqueue_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                                tsa_result* d_results, uint64_t* d_hists, const tsa_tune* tune, void* d_ws,
                                size_t ws_bytes, hipStream_t s) {
  int st = check_cube(cube);
  if (st) return st;
  if (!d_regions || !d_results || !d_hists || nq < 1 || nq > kMaxQueries || nbins < 1 || nbins > 4096)
    return TSA_EINVAL;
  const BLayout L = batch_layout(nq);
  if (!d_ws || ws_bytes < L.total) return TSA_ENOMEM;
  DevInfo dev;
  if ((st = device_info(&dev))) return st;
  uint32_t tile_units = 0, cand_max = kBatchCandMax;  // 0: chosen on the device from the batch's volume
  int bpc = 4;
  int replicas = 0;  // 0: by bin count
  if (tune) {
    if (tune->tile_voxels >= 1024) tile_units = (uint32_t)tune->tile_voxels / (cube->dtype == TSA_F32 ? 4 : 8);
    if (tune->blocks_per_cu >= 1 && tune->blocks_per_cu <= 16) bpc = tune->blocks_per_cu;
    if (tune->cand_max >= 0) cand_max = (uint32_t)tune->cand_max;
    if (tune->block_threads != 0 && tune->block_threads != kBBlock) return TSA_ENOTSUP;
    if (tune->replicas != 0 && tune->replicas != 1 && tune->replicas != 2 && tune->replicas != 4 &&
        tune->replicas != 8)
      return TSA_EINVAL;
    replicas = tune->replicas;
  }
  if (tile_units && tile_units < 256) tile_units = 256;
  const int epv = cube->dtype == TSA_F32 ? 4 : 8;
  const bool vec = ((uintptr_t)cube->data % 16) == 0 && (cube->nx % epv) == 0;
  if (!vec) tile_units *= (uint32_t)epv;  // scalar units are elements
  char* ws = (char*)d_ws;
  BArgs a;
  a.base = cube->data;
  a.nx = cube->nx;
  a.ny = cube->ny;
  a.nz = cube->nz;
  a.regions = d_regions;
  a.nq = nq;
  a.nbins = nbins;
  a.rshift = batch_rep_shift(nbins, replicas, dev.lds_per_block, bpc);
  g_last_config = BatchConfig{(int32_t)tile_units, bpc, 1 << a.rshift, (int32_t)cand_max, true};
  a.tile_units = tile_units;
  a.grid = (uint32_t)(dev.cus * bpc);
  {
    const int64_t polls = g_wait_polls.load();
    a.spin_limit = polls >= 0 ? (uint32_t)polls : kSpinLimit;
  }
  a.max_tiles = L.max_tiles;
  a.cand_max = cand_max;
  a.pool_keys = L.pool_keys;
  a.vec = vec ? 1 : 0;
  a.results = d_results;
  a.hists = d_hists;
  a.hdr = (BatchHdr*)(ws + L.hdr);
  a.geom = (QGeom*)(ws + L.geom);
  a.st = (QState*)(ws + L.st);
  a.tile_base = (uint64_t*)(ws + L.tile_base);
  a.tile_q = (uint32_t*)(ws + L.tile_q);
  a.parts1 = (Partial*)(ws + L.parts1);
  a.parts2 = (double*)(ws + L.parts2);
  a.digits = (uint32_t*)(ws + L.digits);
  a.pool = (uint32_t*)(ws + L.pool);
  const size_t lds1 = ((size_t)kBins1 + kTrash) * 4;
  const size_t lds2 = (((size_t)nbins << a.rshift) + kTrash + kBins2) * 4;
  size_t lds = lds1 > lds2 ? lds1 : lds2;
  if (lds < kEpLdsBytes) lds = kEpLdsBytes;
  bfill3(a.hdr, sizeof(BatchHdr) / 4, a.digits, (size_t)kBins1 * nq, d_hists, (size_t)nbins * nq * 2, s);
  const int pb = (nq + 255) / 256;
  if (!a.tile_units) {
    if (cube->dtype == TSA_F32)
      TSA_TRACED("batch_auto", s, hipLaunchKernelGGL(k_bauto<0>, dim3(1), dim3(1024), 0, s, a));
    else
      TSA_TRACED("batch_auto", s, hipLaunchKernelGGL(k_bauto<1>, dim3(1), dim3(1024), 0, s, a));
  }
  if (cube->dtype == TSA_F32)
    TSA_TRACED("batch_plan", s, hipLaunchKernelGGL(k_bplan<0>, dim3(pb), dim3(256), 0, s, a));
  else
    TSA_TRACED("batch_plan", s, hipLaunchKernelGGL(k_bplan<1>, dim3(pb), dim3(256), 0, s, a));
  TSA_TRACED("batch_scan", s, hipLaunchKernelGGL(k_bscan, dim3(1), dim3(1024), 0, s, a));
  const int grid = (int)a.grid;
  if (cube->dtype == TSA_F32) {
    if (vec)
      TSA_TRACED("batch", s, hipLaunchKernelGGL((k_batch<0, true, true>), dim3(grid), dim3(kBBlock), lds, s, a));
    else
      TSA_TRACED("batch", s, hipLaunchKernelGGL((k_batch<0, false, false>), dim3(grid), dim3(kBBlock), lds, s, a));
  } else {
    if (vec)
      TSA_TRACED("batch", s, hipLaunchKernelGGL((k_batch<1, true, true>), dim3(grid), dim3(kBBlock), lds, s, a));
    else
      TSA_TRACED("batch", s, hipLaunchKernelGGL((k_batch<1, false, false>), dim3(grid), dim3(kBBlock), lds, s, a));
  }
  TSA_TRACED("batch_final", s, hipLaunchKernelGGL(k_bfinal, dim3(pb), dim3(256), 0, s, a));
  return hipGetLastError() == hipSuccess ? TSA_OK : TSA_EDEVICE;
}

// The batch's clears (header, digit counters, output histograms) in one
// launch: a small batch's time is mostly the gaps between its launches.
struct BFill3 {
  uint32_t* p[3];
  uint64_t n[3];
};
__global__ void k_bfill32(BFill3 f) {
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    for (uint64_t i = i0; i < f.n[k]; i += stride) f.p[k][i] = 0u;
}

static void bfill3(void* p0, size_t n0, void* p1, size_t n1, void* p2, size_t n2, hipStream_t s) {
  const size_t most = n0 > n1 ? (n0 > n2 ? n0 : n2) : (n1 > n2 ? n1 : n2);
  if (!most) return;
  int blocks = (int)((most + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  const BFill3 f{{(uint32_t*)p0, (uint32_t*)p1, (uint32_t*)p2}, {n0, n1, n2}};
  TSA_TRACED("fill", s, hipLaunchKernelGGL(k_bfill32, dim3(blocks), dim3(256), 0, s, f));
}

}  // namespace tsa

extern "C" int tsa_internal_batch_last_config(int32_t* out) {
  if (!out) return TSA_EINVAL;
  const tsa::BatchConfig& c = tsa::g_last_config;
  if (!c.set) return TSA_ENOTSUP;
  out[0] = c.tile_units;
  out[1] = c.bpc;
  out[2] = c.replicas;
  out[3] = c.cand_max;
  return TSA_OK;
}

extern "C" int tsa_internal_batch_wait_limit(int32_t polls) {
  tsa::g_wait_polls.store(polls < 0 ? -1 : (int64_t)polls);
  return TSA_OK;
}
