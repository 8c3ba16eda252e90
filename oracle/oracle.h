/*
 * oracle.h -- plain, slow, single-threaded CPU oracle for the parallel
 * reduction x0 (+) x1 (+) ... (+) x(n-1) of Jradi, do Nascimento and Martins,
 * "A Fast and Generic GPU-Based Parallel Reduction Implementation".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no header, constant, table or
 * helper with the GPU path: type and operator codes below are this file's own.
 *
 * Conventions
 *   dtype codes : 0 int32, 1 uint32, 2 float32, 3 float64, 4 float16, 5 bfloat16,
 *                 6 int64, 7 uint64
 *   op codes    : 0 sum, 1 product, 2 min, 3 max, 4 and, 5 or, 6 xor
 *   Every function takes host pointers, never allocates memory the caller must
 *   free, and returns 0 on success or a negative value for an unsupported
 *   (dtype, op) pair or a bad argument.
 */
#ifndef REDUCTION_ORACLE_H
#define REDUCTION_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Algorithm 1 (Summation) of Section 1.1 generalised to every operator of
 * Section 1.1 on 32-bit integers: left fold acc <- acc (+) x[i] starting from
 * the neutral element.  + and x wrap modulo 2^32; min/max compare as signed
 * when is_signed != 0, unsigned otherwise; and/or/xor act on the bits. */
int orc_fold_u32(const uint32_t* x, int64_t n, int op, int is_signed, uint32_t* out);

/* The same fold on 64-bit integers (+ and x wrap modulo 2^64; min/max signed
 * when is_signed != 0); and/or/xor also serve the bits of float64 data. */
int orc_fold_u64(const uint64_t* x, int64_t n, int op, int is_signed, uint64_t* out);

/* Bitwise and/or/xor left fold on 16-bit patterns (float16/bfloat16 bits). */
int orc_fold_u16(const uint16_t* x, int64_t n, int op, uint16_t* out);

/* Integer min (is_max = 0) or max of width-bit (32 or 64) values, signed or
 * unsigned, and the lowest index attaining it (-1 when n = 0). */
int orc_argext_int(const void* x, int64_t n, int width, int is_signed, int is_max, uint64_t* value,
                   int64_t* first);

/* Value of element i of a float array of the given dtype, as a double
 * (exact for every supported float dtype). */
double orc_load_float(const void* x, int64_t i, int dtype);

/* Exact sum of the stored values of a float array (dtype 2..5): a
 * fixed-point long accumulator holding every finite value exactly, rounded
 * once to double, round-to-nearest-even.  *abs_sum receives sum |x_i|,
 * computed the same exact way.  NaN inputs, or +inf together with -inf,
 * give NaN; otherwise an infinity gives that infinity. */
int orc_exact_sum(const void* x, int64_t n, int dtype, double* sum, double* abs_sum);

/* Product of the stored values of a float array as a left fold in
 * double-double arithmetic (error-free product by fma), rounded to double. */
int orc_prod(const void* x, int64_t n, int dtype, double* out);

/* Float min (is_max = 0) or max (is_max = 1) under IEEE 754-2019
 * minimum/maximum: any NaN makes the result NaN, and -0 < +0.  *first
 * receives the lowest index attaining the result (the first NaN if any),
 * or -1 when n = 0, in which case *out is +inf for min and -inf for max. */
int orc_minmax(const void* x, int64_t n, int dtype, int is_max, double* out, int64_t* first);

/* Segmented form: out[s] = (+) of x[offsets[s] .. offsets[s+1]).  Results are
 * written as double for float dtypes with op sum/prod/min/max (exact sum for
 * sum), and as uint64 bit patterns (zero-extended) for integer dtypes and for
 * bitwise ops on float dtypes.  out must hold nseg 8-byte entries. */
int orc_segmented(const void* x, const int64_t* offsets, int64_t nseg, int dtype, int op,
                  void* out);

/* Scan, the prefix form of the reduction: out[i] is the reduction of the
 * elements of i's run up to and including i (exclusive = 0), or of those
 * strictly before i (exclusive != 0; the neutral element at a run's first
 * position).  Position 0 and every position in heads[0..nheads) start a run
 * (heads nondecreasing, values outside [0, n) ignored): no heads gives the
 * plain scan, CSR segment offsets give the per-segment scan.  Results per
 * position follow orc_segmented: double (exact-then-rounded sums, double-double
 * products, exact min/max) for float data, uint64 bit patterns otherwise.
 * out must hold n 8-byte entries. */
int orc_scan(const void* x, int64_t n, int dtype, int op, int exclusive, const int64_t* heads,
             int64_t nheads, void* out);

/* Row-wise reduction of a float32 matrix [rows, cols] (row-major), op in
 * {sum, product, min, max}: y[r] as double (exact sum for sum), idx[r] the
 * lowest column attaining min/max (-1 otherwise), zeros[r] the number of
 * exact zeros in the row (product only, else 0). */
int orc_row_forward(const float* x, int64_t rows, int64_t cols, int op, double* y,
                    int64_t* idx, int64_t* zeros);

/* Gradient of the row-wise reduction with respect to x, given the upstream
 * gradient g[rows]:  sum -> g[r];  min/max -> g[r] at the lowest index
 * attaining the extreme, 0 elsewhere;  product -> g[r] times the product of
 * every other element of the row, formed from exclusive prefix and suffix
 * products in double-double (no division).  grad is [rows, cols] doubles. */
int orc_row_grad(const float* x, int64_t rows, int64_t cols, int op, const double* g,
                 double* grad);

/* Timing baseline, not a correctness source: Algorithm 1 (Summation) as a
 * left fold of a float32 array accumulated in double.  threads = 1 folds
 * x[0..n) in index order on the calling thread; threads = T > 1 splits x into
 * T contiguous chunks of near-equal size, folds each on its own thread and
 * adds the T partial sums in chunk order (a fixed order, so the result is
 * reproducible for a given T).  1 <= T <= 256; returns -4 if a thread cannot
 * be started. */
int orc_fold_sum_f32(const float* x, int64_t n, int threads, double* out);

#ifdef __cplusplus
}
#endif
#endif
