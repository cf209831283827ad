/*
 * tsa_serve.h -- request serving over cubes resident in GPU memory
 * (libtsa.so).
 *
 * The paper's framework answers analysis requests from remote clients against
 * cubes held in GPU memory, so that requests travel to where the data sits
 * instead of the data to the client (Sections 2 and 5); this is that service
 * on one GPU.  A server owns a scheduler thread that
 *   - keeps a registry of resident cubes (min/max computed when a cube is
 *     added, as Section 4.1 computes them while the data loads);
 *   - admits requests while a device-scratch budget and a slot limit allow;
 *   - batches the admitted region requests of one cube into tsa_region_batch
 *     launches on several streams, so a new batch starts while earlier ones
 *     run (continuous batching: requests arriving mid-flight join the next
 *     batch instead of waiting for the queue to drain);
 *   - runs full-cube histogram and median requests on a stream of their own,
 *     overlapping the region batches on the device; every full-cube request
 *     admitted for one cube is answered by one shared scan of that cube (one
 *     histogram pass, the radix passes, or the fused two-pass trio), its
 *     passes cut into z-slab launches of a voxel budget when one is set;
 *   - retires finished work by polling events and timestamps every stage.
 * Each request's result depends only on its own cube and box, never on what
 * else is in flight.
 *
 * Deployment: the server's streams (region_lanes + 1) overlap only if each
 * has a hardware queue of its own; HIP gives a process four by default, which
 * the caller's other streams share.  Start the process with
 * GPU_MAX_HW_QUEUES of at least region_lanes + 1 plus the caller's busy
 * streams (8 covers two lanes), or a region lane can wait behind a full-cube
 * scan queued ahead of it.
 */
#ifndef TSA_SERVE_H
#define TSA_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "tsa.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tsa_server tsa_server;

typedef struct {
  int32_t max_batch;      /* region requests per batch launch, 1..4096 */
  int32_t region_lanes;   /* region batches in flight at once (streams), 1..4 */
  int32_t max_admitted;   /* requests admitted (holding scratch) at once, >= 1 */
  int32_t region_nbins;   /* bins of a region request's histogram over its own [min,max], 1..4096 */
  int32_t full_nbins;     /* bins of a full-cube histogram over the cube's [min,max], 1..65536 */
  int32_t full_chunk_kvoxels; /* voxels (in units of 1024) per kernel launch of a full-cube scan's passes:
                                 each pass over a cube goes out as one launch per z-slab of at most that
                                 many voxels, so region batches can start between them; 0 = one launch
                                 per pass (the fused two-pass trio when both kinds share a scan) */
  size_t scratch_bytes;   /* admission budget of device scratch, bytes (0 = no limit beyond the slots) */
} tsa_server_config;

typedef enum {
  TSA_REQ_REGION = 0,      /* moments + histogram over own [min,max] + median of a box */
  TSA_REQ_FULL_HIST = 1,   /* full_nbins histogram of the whole cube over its [min,max] */
  TSA_REQ_FULL_MEDIAN = 2  /* lower median (and count) of the whole cube */
} tsa_req_kind;

typedef struct {
  int32_t cube;       /* id returned by tsa_server_add_cube */
  int32_t kind;       /* tsa_req_kind */
  tsa_region region;  /* TSA_REQ_REGION only */
  uint64_t* h_hist;   /* optional host buffer receiving the histogram (region_nbins or full_nbins entries) */
  uint64_t tag;       /* caller's identifier, echoed in the response */
} tsa_request;

typedef struct {
  uint64_t tag;
  tsa_result result;  /* fields the request kind defines; NaN/0 elsewhere */
  double t_submit;    /* tsa_server_now() seconds at submission */
  double t_admit;     /* ... when admitted (scratch reserved) */
  double t_launch;    /* ... when its work was enqueued on the GPU */
  double t_done;      /* ... when the scheduler saw it finished */
  int32_t kind;
  int32_t status;     /* TSA_OK, or the error of its launch */
} tsa_response;

/* Create a server on the current HIP device: allocates its device scratch
 * and pinned host staging once, starts the scheduler thread. */
int tsa_server_create(const tsa_server_config* cfg, tsa_server** out);

/* Register a resident cube (device memory owned by the caller, unchanged while
 * the server lives); computes its min/max now.  Writes the cube id. */
int tsa_server_add_cube(tsa_server* s, const tsa_cube* cube, int32_t* id);

/* Queue one request (thread-safe, non-blocking).  TSA_EINVAL for a bad
 * cube id / kind; TSA_EBUSY when more than 1<<20 requests are waiting. */
int tsa_server_submit(tsa_server* s, const tsa_request* r);

/* Copy up to cap finished responses (completion order) into out; returns the
 * number copied (>= 0) or a negative status. */
int tsa_server_poll(tsa_server* s, tsa_response* out, int32_t cap);

/* Wait until every submitted request has finished (timeout_s <= 0: forever).
 * TSA_OK, or TSA_EBUSY on timeout. */
int tsa_server_drain(tsa_server* s, double timeout_s);

/* Open-loop replay: submit reqs[i] at t_arrival[i] seconds after the call
 * starts (non-decreasing), wait for all, write their responses to out[i]
 * (request order).  Responses of these requests are not also returned by
 * tsa_server_poll. */
int tsa_server_replay(tsa_server* s, const tsa_request* reqs, const double* t_arrival, int32_t n,
                      tsa_response* out);

/* Scheduler counters as a JSON object (batches, batch sizes, admissions waited, ...). */
int tsa_server_stats(tsa_server* s, char* buf, size_t len);

/* Stop the scheduler (finishing in-flight work) and free everything. */
int tsa_server_destroy(tsa_server* s);

/* The server clock (monotonic seconds). */
double tsa_server_now(void);

#ifdef __cplusplus
}
#endif

#endif /* TSA_SERVE_H */
