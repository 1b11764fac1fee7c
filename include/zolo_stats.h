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

/* GEMM tile autotuning.  The FP64 MFMA GEMM has several tile shapes whose
 * results are bit-identical (each output element sums the same products in
 * the same order), so which one runs changes speed only.  For each shape
 * class (device, transposes, triangular-operand flags, batch reduction,
 * whether beta != 0, and floor(log2) of m, n and k) the first six calls run
 * the three candidates twice each, in the order 0 1 2 2 1 0, on the caller's
 * own data, each timed by a pair of HIP events that the library reads only
 * once they have completed (it never waits on them).  Later calls of the
 * class use the candidate with the least time per flop, where one replaces
 * the fixed rule's tile only if it is more than 3% faster.  Split-K products
 * keep the fixed tile.  The choices are process-wide and serialised by one
 * lock.
 * Tuning is off by default (the fixed rule is as fast on the Zolo-PD
 * workloads, and which kernel runs then does not depend on timing noise):
 * zolo_autotune_enable(1) turns it on, zolo_autotune_enable(0) off again;
 * without a call the environment variable ZOLO_AUTOTUNE=1 turns it on.
 * Returns 0. */
int zolo_autotune_enable(int on);
/* Forget every choice made so far: the next calls of each class time the
 * candidates again.  Returns 0. */
int zolo_autotune_reset(void);

/* Destroys every HIP event the statistics and the autotuner hold (up to
 * 16384 for the statistics) after waiting for the pending ones; the recorded
 * figures are kept and recording can resume (events are created again on
 * demand).  Call it before the process ends, with no solve running, so that
 * no library-owned HIP object is left for the runtime's own teardown.
 * Returns 0. */
int zolo_release_events(void);

#ifdef __cplusplus
}
#endif

#endif /* ZOLO_STATS_H */
