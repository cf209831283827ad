/*
 * tsa.h -- C ABI of the MI355X (gfx950) cube-statistics library (libtsa.so).
 *
 * Implements the data-parallel analysis path of Hassan, Fluke, Barnes &
 * Kilborn, "Tera-scale astronomical data analysis and visualization" (MNRAS,
 * arXiv 1211.4896), Section 4: global histogram (4.1), global mean and
 * standard deviation (4.2) and global median (4.3), over 3-D image cubes
 * held resident in GPU memory, plus batched queries over many small
 * caller-chosen sub-cubes (the local statistics of the Section 4
 * introduction).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Cube layout: dense, x fastest, element (x,y,z) at index x + nx*(y + ny*z)
 *    (RA, Dec, frequency as in the paper's survey cubes).  Element type float32
 *    or int16.  The cube pointer is a device pointer; the caller owns it and it
 *    must stay valid and unmodified until the stream reaches the end of the call.
 *  - NULL voxels (Section 4 asks for them to be left out) are
 *    NaN; they are excluded from every statistic and counted in nan_count.
 *    +-inf are ordinary values.  int16 cubes have no NULL value.
 *  - Ordering is IEEE-754 totalOrder on non-NaN values (-0 < +0); min, max and
 *    the median are returned bit-exactly as stored values.
 *  - A region is a half-open box [x0,x1) x [y0,y1) x [z0,z1) with
 *    0 <= x0 < x1 <= nx (same for y, z).  Each voxel in it is counted once.
 *    Passing NULL where a region is accepted means the whole cube.
 *  - Every compute call is asynchronous on the given HIP stream (NULL = the
 *    legacy default stream).  Argument errors are detected on the host and
 *    returned synchronously before anything is enqueued; nothing aborts and no
 *    exception crosses the ABI.  Data-dependent conditions found on the device
 *    are reported in tsa_result.status / tsa_result.flags.
 *  - Device memory for outputs and scratch is owned by the caller.  Scratch
 *    ("workspace") size comes from tsa_workspace_bytes(); the library never
 *    allocates or frees device memory in a compute call.
 *  - Calls on different streams may run concurrently if they use different
 *    workspaces and outputs.  A workspace must not be shared by two calls that
 *    can overlap.
 */
#ifndef TSA_H
#define TSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hipStream_t without pulling in the HIP headers (same underlying type). */
typedef struct ihipStream_t* tsa_stream_t;

typedef enum {
  TSA_OK = 0,
  TSA_EINVAL = -1,  /* bad argument (null pointer, bad box, bad range, ...) */
  TSA_ENOMEM = -2,  /* workspace smaller than tsa_workspace_bytes() */
  TSA_EDEVICE = -3, /* a HIP call or kernel launch failed */
  TSA_ENOTSUP = -4, /* dtype, layout or device not supported */
  TSA_EBUSY = -5    /* serving: no free slot or scratch for the request */
} tsa_status;

typedef enum { TSA_F32 = 0, TSA_I16 = 1 } tsa_dtype;

typedef struct {
  const void* data; /* device pointer to nx*ny*nz elements */
  int32_t dtype;    /* tsa_dtype */
  int32_t reserved; /* must be 0 */
  int64_t nx, ny, nz;
} tsa_cube;

typedef struct {
  int64_t x0, y0, z0, x1, y1, z1; /* half-open box */
} tsa_region;

/* tsa_result.flags bits */
#define TSA_FLAG_HIST_SKIPPED 1 /* histogram over [min,max] skipped: no valid voxel or non-finite min/max */
#define TSA_FLAG_BAD_REGION 2   /* region_batch: this query's box was invalid (results left NaN / 0) */
#define TSA_FLAG_PHASE3 4       /* region_batch: the median needed a third selection pass */

typedef struct {
  uint64_t count;     /* non-NaN voxels */
  uint64_t nan_count; /* NaN voxels */
  double mean;        /* (1/count) * sum x                      (Section 4.2) */
  double m2;          /* sum (x - mean)^2                        (Section 4.2) */
  double std;         /* sqrt(m2 / count): population form       (Section 4.2) */
  double min, max;    /* totalOrder extremes, exact              (Section 4.1) */
  double median;      /* lower median: rank floor((count-1)/2)   (Section 4.3) */
  int32_t status;     /* TSA_OK, or an error found on the device */
  int32_t flags;      /* TSA_FLAG_* */
} tsa_result;         /* 72 bytes; NaN fields when count == 0 */

/* Which operation a workspace is sized for. */
typedef enum {
  TSA_OP_MOMENTS = 0,
  TSA_OP_HISTOGRAM = 1,
  TSA_OP_MEDIAN = 2,
  TSA_OP_STATS = 3,
  TSA_OP_REGION_BATCH = 4,
  TSA_OP_QUANTILE = 5,
  TSA_OP_MAD = 6
} tsa_op;

/* Tunables of tsa_region_batch (NULL = the autotuner's remembered choice for
 * the batch's shape, else the defaults: automatic tiles, 4 blocks per CU,
 * 2^20-key candidate cap, replicas by bin count).  In a given struct,
 * tile_voxels below 1024, blocks_per_cu 0 and replicas 0 keep their defaults;
 * cand_max is taken as given (0: no candidate copy, every box whose median
 * needs a last digit takes a third pass). */
typedef struct {
  int32_t tile_voxels;     /* target voxels per work item (>= 1024); below 1024: chosen on the
                              device so the batch makes about four tiles per persistent block,
                              16K to 1M voxels each */
  int32_t block_threads;   /* 0 or 256 (the batch kernel's block size; others: TSA_ENOTSUP) */
  int32_t blocks_per_cu;   /* persistent blocks per compute unit, >= 1 */
  int32_t cand_max;        /* largest bucket compacted for the median's last digits */
  int32_t replicas;        /* LDS copies of each histogram bin (bin privatisation): 1, 2, 4 or 8;
                              0 = by bin count (4 up to 1024 bins, 2 up to 2048, else 1); fewer
                              are used where the copies would not fit the block's LDS */
} tsa_tune;

/*
 * Bytes of device workspace needed by one call of `op` on `cube` (region may
 * be NULL = whole cube; nbins is used by TSA_OP_HISTOGRAM / TSA_OP_STATS /
 * TSA_OP_REGION_BATCH; nq by TSA_OP_REGION_BATCH).  Returns 0 on bad
 * arguments.  Never touches the device other than to query its properties.
 */
size_t tsa_workspace_bytes(int32_t op, const tsa_cube* cube, const tsa_region* region, int32_t nbins,
                           int32_t nq);

/*
 * Global moments (Section 4.2, with min/max of Section 4.1): count, nan_count,
 * mean, m2, std, min, max of the non-NaN voxels of `region` (host pointer or
 * NULL).  Writes those fields and status/flags of *d_out (device pointer); the
 * median field is left untouched.  Per-lane sums are double (float32 cubes)
 * or exact integers (int16), block partials are merged in double in a fixed
 * order (deterministic).
 */
int tsa_moments(const tsa_cube* cube, const tsa_region* region, tsa_result* d_out, void* d_ws,
                size_t ws_bytes, tsa_stream_t stream);

/*
 * Fixed-range histogram (Section 4.1).  For a non-NaN value v (int16 is
 * converted to float exactly): v < lo counts in d_outliers[0], v > hi in
 * d_outliers[1]; otherwise bin b = min((int)((v - lo) * scale), nbins - 1)
 * with scale = (float)nbins / (hi - lo), all in IEEE single precision
 * (round-to-nearest, no fused multiply-add, denormals kept); lo == hi puts
 * every v == lo in bin 0.  d_counts (uint64[nbins], device) and d_outliers
 * (uint64[2], device, may be NULL) are overwritten.
 * Errors (TSA_EINVAL): nbins outside [1, 65536]; lo or hi not finite;
 * lo > hi; hi - lo or scale not finite, or scale == 0.
 */
int tsa_histogram(const tsa_cube* cube, const tsa_region* region, float lo, float hi, int32_t nbins,
                  uint64_t* d_counts, uint64_t* d_outliers, void* d_ws, size_t ws_bytes,
                  tsa_stream_t stream);

/*
 * Exact median (Section 4.3), read as the lower median: the non-NaN value of
 * 0-based rank floor((count-1)/2) under totalOrder.  Found by radix selection
 * on order-preserving 32-bit keys (12+12+8 key bits; no host round trip).
 * Writes median, count, nan_count, status of *d_out; other fields untouched.
 */
int tsa_median(const tsa_cube* cube, const tsa_region* region, tsa_result* d_out, void* d_ws,
               size_t ws_bytes, tsa_stream_t stream);

/*
 * The three statistics together: moments, the nbins histogram over the
 * region's own [min, max], and the lower median, in two passes over the data
 * (moments + first key digit; histogram + second key digit), then a pass over
 * the few candidates left.  Fills every field of *d_out; d_counts
 * (uint64[nbins]) and d_outliers (uint64[2], may be NULL) as in
 * tsa_histogram.  When there is no valid voxel or min/max is not finite the
 * histogram is all zero and TSA_FLAG_HIST_SKIPPED is set.
 */
int tsa_stats(const tsa_cube* cube, const tsa_region* region, int32_t nbins, tsa_result* d_out,
              uint64_t* d_counts, uint64_t* d_outliers, void* d_ws, size_t ws_bytes,
              tsa_stream_t stream);

/*
 * tsa_stats without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, allocation-free serving loops, harnesses
 * that forbid hipMalloc): the same kernels and outputs as tsa_stats, with
 * every piece of scratch taken from a fixed array of
 * tsa_stats_static_scratch_bytes() (8 MiB) that the library holds on each
 * device until the process ends.  The call itself allocates nothing (no
 * hipMalloc, no graph).  Any cube or region is accepted: the median's
 * candidate list holds at most tsa_stats_static_candidate_keys() keys, and a
 * larger last key bucket is settled by a third pass over the data.
 * Every call on a device shares that device's array, so calls that can
 * overlap on one device (two streams, two threads) race and must be
 * serialised by the caller; each call clears what must start at zero.
 * Errors as tsa_stats; TSA_EDEVICE if the array's device address cannot be
 * found; TSA_ENOMEM if the call's scratch would exceed the array (not
 * reachable with the capped candidate list).
 */
int tsa_stats_static(const tsa_cube* cube, const tsa_region* region, int32_t nbins, tsa_result* d_out,
                     uint64_t* d_counts, uint64_t* d_outliers, tsa_stream_t stream);

/* Size in bytes of tsa_stats_static's per-device scratch array. */
size_t tsa_stats_static_scratch_bytes(void);

/* Candidate keys tsa_stats_static's scratch holds for the median's last digits. */
int64_t tsa_stats_static_candidate_keys(void);

/*
 * The lower q-quantile: the non-NaN value of 0-based rank floor(q * (count-1))
 * under totalOrder, the product rounded to double (q in [0, 1]; q = 0.5 is the
 * lower median).  The same radix selection as tsa_median.  digits = 3 selects
 * every key bit (exact); digits = 1 or 2 stops after that many digits (one or
 * two passes over the data; the median of Section 4.3's sample run is known
 * to ~1e-6 after 20 of its 31 iterations, this is the radix analogue) and
 * returns the smallest value of the key bucket holding the rank.
 * d_out (device, 3 doubles) = (value, bucket width, count): the exact answer
 * lies in [value, value + width]; width is 0 when digits = 3.  NaN, NaN, 0
 * without a valid voxel.  TSA_EINVAL for q outside [0,1] or digits outside 1..3.
 */
int tsa_quantile(const tsa_cube* cube, const tsa_region* region, double q, int32_t digits, double* d_out,
                 void* d_ws, size_t ws_bytes, tsa_stream_t stream);

/*
 * Median absolute deviation (Section 4.3 names it as an extension of the
 * median method): m = the lower median, then the lower median of |x - m| over
 * the non-NaN values, x - m rounded to single precision (int16: exact).  A
 * value equal to m deviates by +0, also when m is infinite (where the IEEE
 * difference would be NaN), so the rank is taken over all count values.
 * Four radix passes over the data.  d_out (device, 3 doubles) = (m, MAD,
 * count); NaN, NaN, 0 without a valid voxel.
 */
int tsa_mad(const tsa_cube* cube, const tsa_region* region, double* d_out, void* d_ws, size_t ws_bytes,
            tsa_stream_t stream);

/*
 * Batched region queries (local statistics over caller-chosen boxes,
 * Section 4; the statistical mini-map of Section 4.5 is a regular grid of
 * them).  For each of the nq boxes in d_regions (device array), computes what
 * tsa_stats computes, with the histogram over the box's own [min, max]:
 * d_results[q] (device, nq entries) and d_hists[q*nbins .. +nbins) (device,
 * uint64).  All queries run in one persistent kernel fed by a device work
 * queue of (query, phase, tile) items; no host round trip.  An invalid box
 * sets TSA_FLAG_BAD_REGION and status TSA_EINVAL in its own result only.
 * nq in [1, 65536], nbins in [1, 4096], each box below 2^32 voxels.  tune
 * may be NULL.
 */
int tsa_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                     tsa_result* d_results, uint64_t* d_hists, const tsa_tune* tune, void* d_ws,
                     size_t ws_bytes, tsa_stream_t stream);

/*
 * Autotuner of tsa_region_batch: runs the caller's batch (same arguments as
 * tsa_region_batch; outputs are overwritten) under a search over launch
 * choices -- tile size (automatic, 64K, 256K, 1M voxels) x persistent blocks
 * per compute unit (2, 4, 6, 8), then LDS replicas per histogram bin (1, 2,
 * 4, 8) at the best of those, then the candidate cap (64K, 256K, 1M, 4M keys)
 * -- `reps` timed runs each after one warm-up, and writes the fastest to *best
 * (and its mean time in
 * milliseconds to *best_ms, if not NULL).  The choice is remembered for the
 * batch's shape class (device architecture, dtype, nbins, log2 nq) and used by
 * later tsa_region_batch calls with tune == NULL.  Synchronizes the stream.
 */
int tsa_tune_region_batch(const tsa_cube* cube, const tsa_region* d_regions, int32_t nq, int32_t nbins,
                          tsa_result* d_results, uint64_t* d_hists, void* d_ws, size_t ws_bytes,
                          tsa_stream_t stream, int32_t reps, tsa_tune* best, float* best_ms);

/*
 * Statistical mini-map (Section 4.5): the scaled-down cube whose points each
 * summarise a larger region.  The cube is cut into cells of
 * cell_x * cell_y * cell_z voxels, the last cell along an axis keeping the
 * remainder; cell (i, j, k) covers [i cx, min((i+1) cx, nx)) x ... and is
 * entry i + ncx (j + ncy k) of the outputs, with ncx = ceil(nx / cx) and so on.
 * Each cell gets what tsa_region_batch gives a box: d_cells (device,
 * ncells tsa_result) and d_hists (device, ncells * nbins uint64, each over the
 * cell's own [min, max]).  The cell boxes are planned on the device and the
 * statistics come from one region batch.  Workspace:
 * tsa_minimap_workspace_bytes().  TSA_EINVAL for cell edges < 1, more than
 * 65536 cells, a cell of 2^32 voxels or more, nbins outside [1, 4096].
 */
int tsa_minimap(const tsa_cube* cube, int32_t cell_x, int32_t cell_y, int32_t cell_z, int32_t nbins,
                tsa_result* d_cells, uint64_t* d_hists, void* d_ws, size_t ws_bytes, tsa_stream_t stream);

/* Workspace bytes of tsa_minimap (0 on bad arguments). */
size_t tsa_minimap_workspace_bytes(const tsa_cube* cube, int32_t cell_x, int32_t cell_y, int32_t cell_z,
                                   int32_t nbins);

/* Number of mini-map cells for these cell edges, or a negative status. */
int64_t tsa_minimap_cells(const tsa_cube* cube, int32_t cell_x, int32_t cell_y, int32_t cell_z);

/*
 * Local k-sigma threshold counts (Section 4.5: the mini-map's statistics set
 * a local threshold): for every cell c, the number of non-NaN voxels v of c
 * with v > mean_c + k * std_c, where mean_c and std_c are d_cells[c] as
 * written by tsa_minimap for the same cube and cell edges, and the threshold
 * is k * std_c rounded to double, then added to mean_c and rounded to double;
 * v is compared exactly (int16 converted to float).  Cells without a valid
 * voxel count 0.  d_above (device, ncells uint64) is overwritten.  One
 * streaming pass over the cube; no workspace.  TSA_EINVAL for a non-finite k
 * or bad cell edges (as tsa_minimap).
 */
int tsa_sigma_count(const tsa_cube* cube, int32_t cell_x, int32_t cell_y, int32_t cell_z,
                    const tsa_result* d_cells, double k, uint64_t* d_above, tsa_stream_t stream);

/*
 * 3-D spectrum tool (Section 4.4, Fig. 8): data profiles along arbitrary
 * rays, sampled at a constant step with trilinear interpolation.
 * d_rays (device, nrays x 6 doubles) holds per ray its origin (ox, oy, oz)
 * and step vector (sx, sy, sz) in voxel units, voxel (x, y, z) sitting at the
 * integer point (x, y, z).  Sample i of ray r (0 <= i < nsamples) is at
 * p = origin + i * step per coordinate (the product rounded to double, then
 * the sum).  A sample outside [0, nx-1] x [0, ny-1] x [0, nz-1] is NaN.
 * Inside, per axis x0 = min(floor(x), nx - 2) (0 when nx == 1),
 * fx = x - x0, x1 = min(x0 + 1, nx - 1); corner c = bx + 2 by + 4 bz has
 * weight (wx * wy) * wz with w = 1 - f for bit 0 and f for bit 1, and the
 * sample is 0.0 plus weight * value over c = 0..7 in order, corners of weight
 * 0 skipped, in double (int16 converted exactly); a NaN corner of non-zero
 * weight gives NaN.  d_out (device, nrays x nsamples doubles, ray-major) is
 * overwritten.  nrays or nsamples 0: nothing to do.  TSA_EINVAL for negative
 * counts, null pointers, or more than 2^31 samples' worth of launch.
 */
int tsa_spectrum(const tsa_cube* cube, const double* d_rays, int32_t nrays, int32_t nsamples, double* d_out,
                 tsa_stream_t stream);

/* Write the remembered tuning choices as JSON to `path` (host file).  The
 * library also loads the file named by the environment variable
 * TSA_TUNE_CACHE, if set, before its first lookup. */
int tsa_tune_save(const char* path);

/* Merge the choices saved in `path`; returns how many were read, or TSA_EINVAL. */
int tsa_tune_load(const char* path);

/* Human-readable text for a tsa_status value (static storage). */
const char* tsa_status_string(int32_t status);

/* Library version string (static storage). */
const char* tsa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TSA_H */
