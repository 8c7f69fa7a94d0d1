/*
 * snn_testing.h -- test support of libsnn: the raw values of the candidate
 * screen, for checking its rounding bound pair by pair.  Not part of the
 * search interface (include/snn.h); tests call it to verify, on adversarial
 * inputs, that every pair the normative rule accepts passes the screen.
 *
 * The screen (Section 4, eq. (ip2), evaluated on the matrix cores) compares
 * for a query q and a candidate j
 *     D[q][j] = fl_mfma( sum_k A[q][k] B[j][k] + C[q] )   with   H[j]
 * and passes the pair iff D >= H.  A and B are the operand rows the screen
 * multiplies (16-bit values: bf16 or fp16 bit patterns; fp32 for the fp32
 * screen), C the per-query start value and H the candidate's half squared
 * norm, all in the accumulator's units (scaled by 2^(2 scale_exp) for fp16).
 */
#ifndef SNN_TESTING_H_
#define SNN_TESTING_H_

#include "snn.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t precision; /* snn_precision of the screen: MIXED (bf16), FP16 or FP32 */
  int32_t terms;     /* 16-bit operand values per coordinate: 1, or 3 for the bf16 hi/lo split
                        (query rows [hi | hi | lo], candidate rows [hi | lo | hi] or [hi | lo]
                        with the third segment reusing hi when kb = 2 ka / 3) */
  int32_t ka;        /* values per query operand row (fp32 screen: [y, C_q, 0 ...]) */
  int32_t kb;        /* values per candidate operand row (fp32 screen: the centred row y, kb = d) */
  int32_t chain;     /* products per screen value (K of the bound) */
  int32_t scale_exp; /* FP16: operands are fp16(2^e y); 0 otherwise */
} snn_screen_layout;

/* The screen a query of this index with radius R and these options would
 * run (opts NULL: AUTO), and its operand row sizes; no device work.
 * Errors: SNN_EINVAL (NULL, bad R or options, a metric other than L2, or a
 * choice of the float64 path, which has no screen), SNN_ENOTSUP. */
snn_status snn_debug_screen_layout(snn_index_t idx, double R, const snn_options* opts, snn_screen_layout* layout);

/* Screen values of every (query, candidate) pair, computed with the same
 * operand loads and matrix-instruction chain as the query's screen kernel.
 *   Q: device, m x d (index dtype); 1 <= m.  n = the index's row count.
 *   D: device, m x n floats: D[q * n + j], q in the caller's query order, j in
 *      the index's score order (snn_index_view.perm maps j to the data row).
 *   H: device, n floats.   C: device, m floats.
 *   A: device, m x ka values (uint16, or float for FP32), caller's order.
 *   B: device, n x kb values (uint16, or float for FP32), score order.
 * The work runs on the index's stream; the call returns when it is done.
 * Errors: as snn_debug_screen_layout, and SNN_EINVAL for NULL buffers or
 * NaN/Inf in Q. */
snn_status snn_debug_screen(snn_index_t idx, const void* Q, int64_t m, double R, const snn_options* opts, float* D,
                            float* H, float* C, void* A, void* B, snn_screen_layout* layout);

#ifdef __cplusplus
}
#endif

#endif /* SNN_TESTING_H_ */
