/*
 * lbch_diag.h — measurement helper of liblbch (not part of the method).
 *
 * A plain streaming copy, used to measure the practical HBM copy bandwidth
 * next to the step kernel and to calibrate the FETCH_SIZE / WRITE_SIZE
 * hardware counters against a kernel that moves a known number of bytes.
 */
#ifndef LBCH_DIAG_H
#define LBCH_DIAG_H

#include <stdint.h>

#include "lbch.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Copies `bytes` bytes from src to dst (both device pointers, 16-byte
 * aligned, non-overlapping; bytes a multiple of 16 and > 0) with one kernel
 * of 16-byte loads and stores, enqueued on hip_stream (NULL = null stream).
 * Does not synchronise.  Bad arguments -> LBCH_E_INVALID. */
lbch_status lbch_diag_copy(const void* src, void* dst, int64_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBCH_DIAG_H */
