/*
 * crf_bench.h -- measurement helper of the thermochemistry library (not part of the
 * computation): a throughput probe whose rates are the denominators of the roofline
 * fractions the benchmark reports for the VALU-bound kernels.
 */
#ifndef CRF_BENCH_H
#define CRF_BENCH_H

#include <stdint.h>

#include "crf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Enqueue one throughput probe on `stream`: `threads` threads (a multiple of 256, at
 * most 2^26) each run 8 independent chains of `iters` operations of one kind:
 *   0  e^x in FP64 by the library's own exponential (Cody-Waite reduction, degree-11
 *      polynomial), the one its FP64 rate constants use;
 *   1  e^x in FP64 by the device math library;
 *   2  e^x in FP32 (__expf, the hardware exponential), as the mixed mode uses;
 *   3  FP64 fused multiply-add;
 *   4  FP32 fused multiply-add.
 * out: DEVICE array of `threads` doubles (written; keeps the chains alive).  The caller
 * times the call (operations = threads x iters x 8).  CRF_E_ARG for other arguments,
 * CRF_E_DEVICE for a failed launch. */
crf_status crf_peak_rate(int kind, int64_t threads, int iters, double *out, crf_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* CRF_BENCH_H */
