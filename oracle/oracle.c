/*
 * Plain CPU oracle for the LightKernel persistent-thread dispatch path.
 * TEST INFRASTRUCTURE ONLY: see oracle.h.  Built with -O2 -fno-fast-math
 * -ffp-contract=off so that every floating-point operation is the one written here.
 */
#include "oracle.h"
#include <math.h>
#include <string.h>

/* Work-item body "int32 affine then int64 sum": the product and the sum are taken
 * modulo 2^32 (unsigned wrap-around), and the 32-bit pattern is read as two's
 * complement.  The int64 sum cannot overflow for n < 2^32. */
int64_t orc_affine_sum_i32(const int32_t *x, int32_t *y, uint64_t n, int32_t a, int32_t b) {
  uint32_t ua = (uint32_t)a, ub = (uint32_t)b;
  int64_t s = 0;
  for (uint64_t i = 0; i < n; i++) {
    uint32_t u = ua * (uint32_t)x[i] + ub;
    int32_t v;
    memcpy(&v, &u, sizeof v);
    if (y) y[i] = v;
    s += (int64_t)v;
  }
  return s;
}

/* Work-item body "int64 reduce-sum" over int32 input. */
int64_t orc_sum_i32_i64(const int32_t *x, uint64_t n) {
  int64_t s = 0;
  for (uint64_t i = 0; i < n; i++) s += (int64_t)x[i];
  return s;
}

/* Work-item body "fp32 SAXPY", in place on y, one correctly rounded fma per element. */
void orc_saxpy_f32(const float *x, float *y, uint64_t n, float alpha) {
  for (uint64_t i = 0; i < n; i++) y[i] = fmaf(alpha, x[i], y[i]);
}

/* Work-item body "fp32 AXPY, out of place": as SAXPY, with y and the result apart. */
void orc_axpy_f32(const float *x, const float *y, float *out, uint64_t n, float alpha) {
  for (uint64_t i = 0; i < n; i++) out[i] = fmaf(alpha, x[i], y[i]);
}

/* Work-item body "fp32 copy". */
void orc_copy_f32(const float *in, float *out, uint64_t n) {
  for (uint64_t i = 0; i < n; i++) out[i] = in[i];
}

/* The paper's benchmark item (Sec. 3): a loop of `iters` iterations with no memory
 * traffic.  Its iterations leave no trace in memory and it returns no value, so as a
 * work item it has no memory effect and result 0. */
int64_t orc_spin(int32_t iters) { return iters < 0 ? -1 : 0; }

/* A stage that triggers several clusters' cores (Sec. 3) gives each member one
 * contiguous slice; slice lengths are rounded up to whole 256-element groups. */
void orc_slice(uint64_t n, uint32_t k, uint32_t j, uint64_t *lo, uint64_t *hi) {
  uint64_t m = 0;
  if (k > 0) {
    m = n / k + (n % k != 0);
    m = (m + 255) / 256 * 256;
  }
  uint64_t l = (uint64_t)j * m, h = l + m;
  if (k == 0 || j >= k) l = h = n;
  if (l > n) l = n;
  if (h > n) h = n;
  *lo = l;
  *hi = h;
}

static int64_t exec_range(const orc_item *it, uint64_t lo, uint64_t hi) {
  uint64_t len = hi - lo;
  switch (it->op) {
    case ORC_NOP:
      return 0;
    case ORC_AFFINE_SUM_I32:
      return orc_affine_sum_i32((const int32_t *)it->in + lo, (int32_t *)it->out + lo, len, it->a, it->b);
    case ORC_SUM_I32_I64:
      return orc_sum_i32_i64((const int32_t *)it->in + lo, len);
    case ORC_SAXPY_F32:
      orc_saxpy_f32((const float *)it->in + lo, (float *)it->out + lo, len, it->alpha);
      return 0;
    case ORC_COPY_F32:
      orc_copy_f32((const float *)it->in + lo, (float *)it->out + lo, len);
      return 0;
    case ORC_AXPY_F32:
      orc_axpy_f32((const float *)it->in + lo, (const float *)it->in2 + lo, (float *)it->out + lo, len, it->alpha);
      return 0;
    case ORC_SPIN:
      /* every member of a cluster runs the whole loop; the item touches none of its range */
      return 0;
    default:
      return 0;
  }
}

int64_t orc_exec(const orc_item *it) { return exec_range(it, 0, it->n); }

int64_t orc_exec_cluster(const orc_item *it, uint32_t k) {
  int64_t total = 0;
  for (uint32_t j = 0; j < k; j++) {
    uint64_t lo, hi;
    orc_slice(it->n, k, j, &lo, &hi);
    total += exec_range(it, lo, hi);
  }
  return total;
}

/* The dispatch loop's sequential specification for one mailbox (Sec. 1, Sec. 2.3):
 * descriptors are executed one after another in the order the host posted them,
 * each exactly once. */
int orc_run_fifo(const orc_item *items, uint64_t count, int64_t *results) {
  for (uint64_t i = 0; i < count; i++) {
    if (items[i].op > ORC_SPIN && items[i].op != ORC_AXPY_F32) return -1;
    if (items[i].op == ORC_SPIN && orc_spin(items[i].a) < 0) return -1;
    int64_t r = orc_exec(&items[i]);
    if (results) results[i] = r;
  }
  return 0;
}

float orc_saxpy_chain_elem(float x, float y, const float *alphas, uint64_t count) {
  for (uint64_t k = 0; k < count; k++) y = fmaf(alphas[k], x, y);
  return y;
}
