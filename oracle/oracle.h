/*
 * Plain CPU oracle for the LightKernel persistent-thread dispatch path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls this
 * code; only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * do.  It shares no header, helper or constant with the HIP library.
 *
 * Every function is the plain definition of what a work item or the dispatch loop
 * computes, written as scalar loops in the order the definition states them.
 *
 * Sources:
 *   - the paper's model (Sec. 1; Sec. 2.3): the host hands a persistent worker a
 *     descriptor of the work plus references to its input and output data, and the
 *     worker executes it; work is placed on one cluster of cores (Sec. 1, Sec. 2.1);
 *   - Sec. 3: a stage triggers "one or multiple" clusters and waits for them;
 *   - the work-item bodies themselves are not defined by the paper (its only item is
 *     a compute-only loop, Sec. 3); they are the evaluation workloads' items:
 *     int32 affine map modulo 2^32 followed by an int64 sum, an int64 sum of int32,
 *     fp32 y = alpha*x + y with one fused multiply-add, and an fp32 copy;
 *   - Sec. 3: the paper's own work item is a compute-only loop of a given number of
 *     iterations that touches no memory; to the dispatch loop it is an item with no
 *     memory effect whose result is 0.
 */
#ifndef LK_ORACLE_H
#define LK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Work-item operation identifiers as the oracle numbers them (its own numbering). */
enum { ORC_NOP = 0, ORC_AFFINE_SUM_I32 = 1, ORC_SUM_I32_I64 = 2, ORC_SAXPY_F32 = 3, ORC_COPY_F32 = 4,
       ORC_SPIN = 5, ORC_AXPY_F32 = 7 };

/* y[i] = (a*x[i] + b) mod 2^32, read as two's complement; returns sum of (int64)y[i]. */
int64_t orc_affine_sum_i32(const int32_t *x, int32_t *y, uint64_t n, int32_t a, int32_t b);
/* returns sum of (int64)x[i]. */
int64_t orc_sum_i32_i64(const int32_t *x, uint64_t n);
/* y[i] = fmaf(alpha, x[i], y[i]): one binary32 fused multiply-add, round to nearest even. */
void orc_saxpy_f32(const float *x, float *y, uint64_t n, float alpha);
/* out[i] = fmaf(alpha, x[i], y[i]): the same single fused multiply-add with y read from
 * its own buffer and the result written to a third one. */
void orc_axpy_f32(const float *x, const float *y, float *out, uint64_t n, float alpha);
/* out[i] = in[i], bit for bit. */
void orc_copy_f32(const float *in, float *out, uint64_t n);
/* The paper's compute-only item (Sec. 3): `iters` loop iterations (iters >= 0) that read
 * and write no memory; what the loop computes is discarded, so the item's whole observable
 * effect is its result, 0.  Returns 0, or -1 for a negative count. */
int64_t orc_spin(int32_t iters);

/* Slice j of an n-element item split over k workers of one cluster:
 * m = ceil(n/k) rounded up to a multiple of 256; slice j = [min(n, j*m), min(n, (j+1)*m)). */
void orc_slice(uint64_t n, uint32_t k, uint32_t j, uint64_t *lo, uint64_t *hi);

/* One work item as the sequential specification sees it. */
typedef struct {
  uint32_t op;
  uint64_t n;
  int32_t a, b;  /* SPIN: a = iterations */
  float alpha;
  const void *in;
  void *out;
  const void *in2;  /* AXPY_F32: y */
} orc_item;

/* Execute one item over its whole range; returns its int64 result (0 for ops without one). */
int64_t orc_exec(const orc_item *it);
/* Execute one item split over a k-member cluster, slice by slice in member order, and
 * return the int64 sum of the member partials. */
int64_t orc_exec_cluster(const orc_item *it, uint32_t k);
/* Sequential specification of one mailbox: execute items[0..count) in submission order,
 * each exactly once; results[i] receives item i's int64 result. Returns 0, or -1 on an
 * unknown op or a SPIN item with a negative count (execution stops at that item). */
int orc_run_fifo(const orc_item *items, uint64_t count, int64_t *results);
/* One element of a SAXPY chain: y <- fmaf(alphas[k], x, y) for k = 0..count-1. */
float orc_saxpy_chain_elem(float x, float y, const float *alphas, uint64_t count);

#ifdef __cplusplus
}
#endif
#endif
