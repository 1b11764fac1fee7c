/*
 * zolo_stats.h - per-kernel launch statistics of the Zolo-PD library.
 *
 * When enabled, every launch of the library's main kernels (the FP64 MFMA
 * GEMM, one entry per tile shape and transpose combination, the structured-QR
 * panel and the Cholesky diagonal-block kernels) is bracketed by HIP events on
 * the stream it runs on, and the library accumulates, per kernel, the number of
 * launches, the summed event time, the algorithmic floating-point work
 * (2 m n k per product, reduced for triangular operands and symmetric
 * outputs) and the algorithmic memory traffic (every operand read once and
 * the output written once: for a GEMM the used parts of A and B per batch,
 * Cin when beta != 0, and C; zero where a kernel does not model it).  These
 * give the measured rate of a kernel as work / time, the per-stage profile of
 * Table 7 of the paper at kernel granularity.
 * Statistics are process-wide (all handles); the calls and the recording are
 * serialised by one lock, so concurrent solves may record into them.
 */
#ifndef ZOLO_STATS_H
#define ZOLO_STATS_H

#ifdef __cplusplus
extern "C" {
#endif

/* Start (on != 0) or stop recording.  Returns 0. */
int zolo_stats_enable(int on);
/* Forget every recorded launch.  Returns 0. */
int zolo_stats_reset(void);
/* Waits for pending events, then reports entry `index` (0 <= index <
 * zolo_stats_count()): its kernel name (NUL-terminated, truncated to
 * name_len), launches, total milliseconds, total algorithmic flops and total
 * algorithmic bytes.  Any output pointer may be NULL.  Returns 0, or -1 for
 * an index out of range. */
int zolo_stats_get(int index, char* name, int name_len, long long* launches, double* ms, double* flops,
                   double* bytes);
/* Number of entries (kernels seen since the last reset). */
int zolo_stats_count(void);

#ifdef __cplusplus
}
#endif

#endif /* ZOLO_STATS_H */
