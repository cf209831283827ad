/*
 * tsa_trace.h -- measurement support of libtsa.so (not part of the
 * statistics): per-kernel timing with HIP events, and a plain copy kernel
 * whose byte counts calibrate hardware counters.
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

#ifdef __cplusplus
}
#endif

#endif /* TSA_TRACE_H */
