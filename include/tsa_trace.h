/*
 * tsa_trace.h -- measurement support of libtsa.so (not part of the
 * statistics): per-kernel timing with HIP events, a plain copy kernel whose
 * byte counts calibrate hardware counters, and a read-only probe that
 * measures the HBM read bandwidth a streaming kernel can reach.
 */
#ifndef TSA_TRACE_H
#define TSA_TRACE_H

#include <stddef.h>
#include <stdint.h>

#include "tsa.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * on != 0: from now on every kernel the library launches is bracketed by two
 * HIP events recorded on its launch stream, for up to `cap` launches (later
 * launches are not recorded).  on == 0: stop.  Either way earlier records are
 * dropped.  Returns TSA_OK or TSA_EDEVICE (event creation failed).  Not meant
 * to be toggled while other threads launch library work.
 */
int tsa_trace_enable(int32_t on, int32_t cap);

/*
 * Waits for the recorded events and writes a JSON object
 * {"kernel name": [launches, total_ms, min_ms, max_ms], ...} into buf (host,
 * len bytes, NUL-terminated).  Returns the string length, TSA_ENOMEM if buf
 * is too small, or TSA_EDEVICE.
 */
int tsa_trace_read(char* buf, size_t len);

/*
 * Copies `bytes` (a multiple of 16) from src to dst (device pointers, 16-byte
 * aligned) with a plain streaming kernel, asynchronously on `stream`.
 * Returns TSA_EINVAL on bad arguments.
 */
int tsa_internal_copy(void* dst, const void* src, size_t bytes, tsa_stream_t stream);

/*
 * Reads `bytes` (a multiple of 16) from src (device, 16-byte aligned) with the
 * 16-byte non-temporal loads and the grid shape of the statistics passes
 * (512 lanes x 2 blocks per compute unit, four loads in flight per lane) and
 * XOR-folds every 32-bit word: one word per block to d_sink (device, at least
 * tsa_internal_probe_blocks() words).  The XOR of the d_sink words is the XOR
 * of the whole buffer.  Returns TSA_EINVAL on bad arguments.
 */
int tsa_internal_read_probe(const void* src, size_t bytes, uint32_t* d_sink, tsa_stream_t stream);

/* Number of sink words tsa_internal_read_probe writes on the current device. */
int32_t tsa_internal_probe_blocks(void);

/*
 * Testing support: caps every bounded wait of the region batch's persistent
 * kernel at `polls` polls (polls < 0: the default cap).  With 0 polls every
 * wait gives up at once, so a test drives the give-up path -- the waiting
 * block stops, the boxes left unfinished report TSA_EDEVICE -- while every
 * kernel still exits.  Batches launched while a cap is set bypass the launch
 * graph cache.  Process-wide; not meant to be changed while other threads
 * launch batches.  Returns TSA_OK.
 */
int tsa_internal_batch_wait_limit(int32_t polls);

/*
 * Testing support: the launch choices of the last region batch this thread
 * enqueued (a graph replay enqueues nothing): out[0] = tile units requested
 * (0: chosen on the device), out[1] = persistent blocks per compute unit,
 * out[2] = LDS replicas per histogram bin, out[3] = candidate cap.  out is a
 * host array of 4 ints.  Returns TSA_EINVAL for NULL, TSA_ENOTSUP before the
 * thread's first batch, else TSA_OK.
 */
int tsa_internal_batch_last_config(int32_t* out);

#ifdef __cplusplus
}
#endif

#endif /* TSA_TRACE_H */
