/*
 * oracle.c -- plain CPU oracle for the parallel reduction (TEST INFRASTRUCTURE).
 *
 * What it computes (Jradi, do Nascimento, Martins, arXiv 1710.07358):
 *   Section 1.1 defines the reduction of X = {x0..x(n-1)} as x0 (+) ... (+) x(n-1)
 *   for an associative combiner (+, x, and, or, xor, min, max, ...), and
 *   Algorithm 1 (Summation) states it as a left fold from the neutral element.
 *   The footnotes of Section 1.1 note that floating-point + is not associative
 *   (1.5 + 4^50 - 4^50 may give 0 or 1.5) and point to compensation or double
 *   precision as remedies.
 *
 * How it computes it (slow on purpose, obviously correct):
 *   - integer ops and bitwise ops: the left fold of Algorithm 1, verbatim;
 *   - float min/max: a left fold with IEEE 754-2019 minimum/maximum semantics;
 *   - float sum: the exact real sum of the stored values, held in a fixed-point
 *     long accumulator (units of 2^-1074), rounded once to double;
 *   - float product: a left fold in double-double arithmetic;
 *   - row-wise gradients: their definitions, with exclusive prefix/suffix
 *     products in double-double;
 *   - a timing baseline only: Algorithm 1's float32 left fold in double, on
 *     one thread or split into contiguous chunks over several threads.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * load this file.  It shares nothing with the GPU path.
 *
 * Build: gcc -O2 -fPIC -shared -pthread (no -ffast-math: the float code relies on
 * strict IEEE evaluation and on fma being exact-then-rounded).
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

enum { DT_I32 = 0, DT_U32 = 1, DT_F32 = 2, DT_F64 = 3, DT_F16 = 4, DT_BF16 = 5, DT_I64 = 6, DT_U64 = 7 };
enum { OP_SUM = 0, OP_PROD = 1, OP_MIN = 2, OP_MAX = 3, OP_AND = 4, OP_OR = 5, OP_XOR = 6 };

/* ------------------------------------------------------------------ */
/* Integer and bitwise folds (Algorithm 1 with the combiner swapped).   */
/* ------------------------------------------------------------------ */

int orc_fold_u32(const uint32_t* x, int64_t n, int op, int is_signed, uint32_t* out) {
    uint32_t acc;
    switch (op) { /* neutral elements */
    case OP_SUM: acc = 0u; break;
    case OP_PROD: acc = 1u; break;
    case OP_MIN: acc = is_signed ? (uint32_t)INT32_MAX : UINT32_MAX; break;
    case OP_MAX: acc = is_signed ? (uint32_t)INT32_MIN : 0u; break;
    case OP_AND: acc = UINT32_MAX; break;
    case OP_OR: acc = 0u; break;
    case OP_XOR: acc = 0u; break;
    default: return -1;
    }
    if (n < 0) return -2;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t v = x[i];
        switch (op) {
        case OP_SUM: acc = acc + v; break; /* unsigned: wraps mod 2^32 */
        case OP_PROD: acc = acc * v; break;
        case OP_MIN:
            if (is_signed) acc = ((int32_t)v < (int32_t)acc) ? v : acc;
            else acc = (v < acc) ? v : acc;
            break;
        case OP_MAX:
            if (is_signed) acc = ((int32_t)v > (int32_t)acc) ? v : acc;
            else acc = (v > acc) ? v : acc;
            break;
        case OP_AND: acc = acc & v; break;
        case OP_OR: acc = acc | v; break;
        case OP_XOR: acc = acc ^ v; break;
        }
    }
    *out = acc;
    return 0;
}

int orc_fold_u64(const uint64_t* x, int64_t n, int op, int is_signed, uint64_t* out) {
    uint64_t acc;
    switch (op) { /* neutral elements */
    case OP_SUM: acc = 0u; break;
    case OP_PROD: acc = 1u; break;
    case OP_MIN: acc = is_signed ? (uint64_t)INT64_MAX : UINT64_MAX; break;
    case OP_MAX: acc = is_signed ? (uint64_t)INT64_MIN : 0u; break;
    case OP_AND: acc = UINT64_MAX; break;
    case OP_OR: acc = 0u; break;
    case OP_XOR: acc = 0u; break;
    default: return -1;
    }
    if (n < 0) return -2;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t v = x[i];
        switch (op) {
        case OP_SUM: acc = acc + v; break; /* wraps mod 2^64 */
        case OP_PROD: acc = acc * v; break;
        case OP_MIN:
            if (is_signed) acc = ((int64_t)v < (int64_t)acc) ? v : acc;
            else acc = (v < acc) ? v : acc;
            break;
        case OP_MAX:
            if (is_signed) acc = ((int64_t)v > (int64_t)acc) ? v : acc;
            else acc = (v > acc) ? v : acc;
            break;
        case OP_AND: acc &= v; break;
        case OP_OR: acc |= v; break;
        case OP_XOR: acc ^= v; break;
        }
    }
    *out = acc;
    return 0;
}

/* Lowest index attaining the integer min (is_max = 0) or max of x, read as
 * width-bit (32 or 64) signed or unsigned integers; -1 when n = 0. */
int orc_argext_int(const void* x, int64_t n, int width, int is_signed, int is_max, uint64_t* value,
                   int64_t* first) {
    if (n < 0 || (width != 32 && width != 64)) return -2;
    int64_t at = -1;
    uint64_t best = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t v = width == 32 ? ((const uint32_t*)x)[i] : ((const uint64_t*)x)[i];
        int better;
        if (at < 0) better = 1;
        else if (is_signed && width == 32)
            better = is_max ? ((int32_t)v > (int32_t)best) : ((int32_t)v < (int32_t)best);
        else if (is_signed)
            better = is_max ? ((int64_t)v > (int64_t)best) : ((int64_t)v < (int64_t)best);
        else
            better = is_max ? (v > best) : (v < best);
        if (better) {
            best = v;
            at = i;
        }
    }
    *value = best;
    *first = at;
    return 0;
}

int orc_fold_u16(const uint16_t* x, int64_t n, int op, uint16_t* out) {
    uint16_t acc;
    if (op == OP_AND) acc = 0xFFFFu;
    else if (op == OP_OR || op == OP_XOR) acc = 0u;
    else return -1;
    if (n < 0) return -2;
    for (int64_t i = 0; i < n; ++i) {
        if (op == OP_AND) acc = (uint16_t)(acc & x[i]);
        else if (op == OP_OR) acc = (uint16_t)(acc | x[i]);
        else acc = (uint16_t)(acc ^ x[i]);
    }
    *out = acc;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Decoding stored float values to double (exact for every dtype).     */
/* ------------------------------------------------------------------ */

/* IEEE binary16: 1 sign, 5 exponent (bias 15), 10 fraction bits. */
static double decode_f16(uint16_t h) {
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 0x1F;
    int m = h & 0x3FF;
    double v;
    if (e == 0) v = ldexp((double)m, -24);                 /* subnormal: m * 2^-24 */
    else if (e == 31) v = (m == 0) ? INFINITY : NAN;
    else v = ldexp((double)(m | 0x400), e - 25);           /* 1.m * 2^(e-15) */
    return sign ? -v : v;
}

/* bfloat16 is the upper half of an IEEE binary32. */
static double decode_bf16(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

double orc_load_float(const void* x, int64_t i, int dtype) {
    switch (dtype) {
    case DT_F32: return (double)((const float*)x)[i];
    case DT_F64: return ((const double*)x)[i];
    case DT_F16: return decode_f16(((const uint16_t*)x)[i]);
    case DT_BF16: return decode_bf16(((const uint16_t*)x)[i]);
    case DT_I32: return (double)((const int32_t*)x)[i];
    case DT_U32: return (double)((const uint32_t*)x)[i];
    }
    return NAN;
}

static int is_float_dtype(int dt) { return dt == DT_F32 || dt == DT_F64 || dt == DT_F16 || dt == DT_BF16; }

/* ------------------------------------------------------------------ */
/* Exact summation: fixed-point long accumulator.                       */
/*                                                                      */
/* Every finite double is an integer multiple of 2^-1074 and smaller   */
/* than 2^1024, so the sum of up to 2^40 of them is an integer times    */
/* 2^-1074 of at most 1074+1024+40 bits.  The accumulator keeps that   */
/* integer in base-2^32 digits, each stored in an int64 so that carries */
/* can be propagated lazily.                                            */
/* ------------------------------------------------------------------ */

#define LA_DIGITS 72 /* 72 * 32 = 2304 bits > 2138 */

typedef struct {
    int64_t d[LA_DIGITS];
    int64_t pending; /* additions since the last carry propagation */
} longacc;

static void la_init(longacc* a) { memset(a, 0, sizeof *a); }

/* Propagate carries so every digit but the top one lies in [0, 2^32). */
static void la_normalize(longacc* a) {
    for (int i = 0; i < LA_DIGITS - 1; ++i) {
        int64_t carry = a->d[i] >> 32; /* arithmetic shift: floor division */
        a->d[i] -= carry * ((int64_t)1 << 32);
        a->d[i + 1] += carry;
    }
    a->pending = 0;
}

/* Add (negate ? -1 : +1) * mant * 2^(pos - 1074), with mant < 2^53, pos >= 0. */
static void la_add(longacc* a, uint64_t mant, int pos, int negate) {
    int digit = pos >> 5, shift = pos & 31;
    /* mant << shift spans at most 85 bits: split into three 32-bit pieces */
    uint64_t lo = (mant << shift) & 0xFFFFFFFFu;
    uint64_t mid = shift ? (mant >> (32 - shift)) & 0xFFFFFFFFu : (mant >> 32) & 0xFFFFFFFFu;
    uint64_t hi = shift ? (mant >> (64 - shift)) : 0u;
    if (negate) {
        a->d[digit] -= (int64_t)lo;
        a->d[digit + 1] -= (int64_t)mid;
        a->d[digit + 2] -= (int64_t)hi;
    } else {
        a->d[digit] += (int64_t)lo;
        a->d[digit + 1] += (int64_t)mid;
        a->d[digit + 2] += (int64_t)hi;
    }
    if (++a->pending >= ((int64_t)1 << 29)) la_normalize(a);
}

/* Add the finite double v exactly. */
static void la_add_double(longacc* a, double v, int force_positive) {
    if (v == 0.0) return;
    int negate = (v < 0.0) && !force_positive;
    double m = fabs(v);
    int e;
    double f = frexp(m, &e);             /* m = f * 2^e, f in [0.5, 1) */
    /* m = mant * 2^(e-53) with mant a 53-bit integer; shift so the exponent
       is at least -1074 (subnormals have fewer significant bits). */
    int exp2 = e - 53;
    uint64_t mant = (uint64_t)ldexp(f, 53); /* exact: f has <= 53 significant bits */
    if (exp2 < -1074) {
        int drop = -1074 - exp2;         /* these low bits are zero for a valid double */
        mant >>= drop;
        exp2 = -1074;
    }
    la_add(a, mant, exp2 + 1074, negate);
}

/* Round the accumulated integer times 2^-1074 to the nearest double, ties to
 * even.  Works digit by digit (base 2^32) so that rounding costs O(digits). */
static double la_round(longacc* a) {
    la_normalize(a);
    uint32_t mag[LA_DIGITS];
    int negative = a->d[LA_DIGITS - 1] < 0;
    /* two's complement magnitude across digits */
    if (negative) {
        uint64_t borrow = 1; /* -v = ~v + 1 */
        for (int i = 0; i < LA_DIGITS; ++i) {
            uint64_t inv = (~(uint64_t)(uint32_t)a->d[i]) & 0xFFFFFFFFu;
            uint64_t s = inv + borrow;
            mag[i] = (uint32_t)s;
            borrow = s >> 32;
        }
    } else {
        for (int i = 0; i < LA_DIGITS; ++i) mag[i] = (uint32_t)a->d[i];
    }
    int td = LA_DIGITS - 1;
    while (td >= 0 && mag[td] == 0) --td;
    if (td < 0) return 0.0;
    int tb = 31;
    while (!((mag[td] >> tb) & 1u)) --tb;
    const int top = td * 32 + tb; /* index of the leading one bit */
    /* the 96 bits below and including the leading digit, left-aligned */
    uint64_t hi = ((uint64_t)mag[td] << 32) | (td >= 1 ? mag[td - 1] : 0u);
    uint64_t lo3 = td >= 2 ? mag[td - 2] : 0u;
    int sticky_digits = 0;
    for (int i = td - 3; i >= 0 && !sticky_digits; --i) sticky_digits = mag[i] != 0;
    /* shift so the leading one sits at bit 63 of w (w holds 64 bits; rest -> below) */
    const int lead = 63 - (32 + tb);   /* bits to shift hi left */
    uint64_t w = lead ? (hi << lead) | (lo3 >> (32 - lead)) : hi;
    const uint64_t below = lead ? (lo3 << (32 + lead)) & 0xFFFFFFFFFFFFFFFFull : (lo3 << 32);
    double r;
    if (top < 53) {
        /* the whole value fits in 53 bits: exact */
        uint64_t m = w >> (63 - top);
        r = ldexp((double)m, -1074);
    } else {
        uint64_t t = w >> 11;                 /* 53 leading bits */
        int round_bit = (int)((w >> 10) & 1u);
        int sticky = ((w & 0x3FFu) != 0) || below != 0 || sticky_digits;
        if (round_bit && (sticky || (t & 1u))) ++t;
        int e = top - 52 - 1074;
        if (t == ((uint64_t)1 << 53)) { t >>= 1; ++e; }
        r = ldexp((double)t, e); /* overflows to inf exactly when it should */
    }
    return negative ? -r : r;
}

int orc_exact_sum(const void* x, int64_t n, int dtype, double* sum, double* abs_sum) {
    if (!is_float_dtype(dtype) || n < 0) return -1;
    static longacc acc, aacc; /* large; kept off the stack (oracle is single-threaded) */
    la_init(&acc);
    la_init(&aacc);
    int has_nan = 0, has_pinf = 0, has_ninf = 0;
    for (int64_t i = 0; i < n; ++i) {
        double v = orc_load_float(x, i, dtype);
        if (isnan(v)) { has_nan = 1; continue; }
        if (isinf(v)) { if (v > 0) has_pinf = 1; else has_ninf = 1; continue; }
        la_add_double(&acc, v, 0);
        la_add_double(&aacc, v, 1);
    }
    double s = la_round(&acc);
    double as = la_round(&aacc);
    if (has_nan || (has_pinf && has_ninf)) s = NAN;
    else if (has_pinf) s = INFINITY;
    else if (has_ninf) s = -INFINITY;
    if (has_nan) as = NAN;
    else if (has_pinf || has_ninf) as = INFINITY;
    if (sum) *sum = s;
    if (abs_sum) *abs_sum = as;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Double-double product fold.                                          */
/* ------------------------------------------------------------------ */

typedef struct { double hi, lo; } dd;

/* (hi + lo) * b with the exact product hi*b recovered by fma.
 *
 * A zero, infinite or NaN leading product is returned as it stands, with a
 * zero tail: it is then the IEEE product itself (the sign of a zero is the
 * exclusive-or of the factors' signs), and the error-free step, whose sum
 * p + e would turn -0 into +0 and inf - inf into NaN, does not apply. */
static dd dd_mul_double(dd a, double b) {
    double p = a.hi * b;
    if (p == 0.0 || !isfinite(p)) {
        dd z = { p, 0.0 };
        return z;
    }
    double e = fma(a.hi, b, -p); /* exact rounding error of a.hi*b */
    e = fma(a.lo, b, e);
    double s = p + e;
    double t = e - (s - p);
    dd r = { s, t };
    return r;
}

static dd dd_mul(dd a, dd b) {
    double p = a.hi * b.hi;
    if (p == 0.0 || !isfinite(p)) {
        dd z = { p, 0.0 };
        return z;
    }
    double e = fma(a.hi, b.hi, -p);
    e += a.hi * b.lo + a.lo * b.hi;
    double s = p + e;
    double t = e - (s - p);
    dd r = { s, t };
    return r;
}

/* The double nearest hi + lo.  A zero tail leaves hi untouched, so a signed
 * zero keeps its sign (-0 + +0 would round to +0). */
static double dd_value(dd a) { return a.lo == 0.0 ? a.hi : a.hi + a.lo; }

int orc_prod(const void* x, int64_t n, int dtype, double* out) {
    if (!is_float_dtype(dtype) || n < 0) return -1;
    dd acc = { 1.0, 0.0 };
    for (int64_t i = 0; i < n; ++i) acc = dd_mul_double(acc, orc_load_float(x, i, dtype));
    *out = dd_value(acc);
    return 0;
}

/* ------------------------------------------------------------------ */
/* IEEE 754-2019 minimum / maximum fold.                                */
/* ------------------------------------------------------------------ */

/* 1 when v should replace the current extreme cur (strictly better). */
static int strictly_better(double v, double cur, int is_max) {
    if (is_max) {
        if (v > cur) return 1;
        if (v == cur && v == 0.0 && signbit(cur) && !signbit(v)) return 1; /* +0 beats -0 */
    } else {
        if (v < cur) return 1;
        if (v == cur && v == 0.0 && !signbit(cur) && signbit(v)) return 1; /* -0 beats +0 */
    }
    return 0;
}

int orc_minmax(const void* x, int64_t n, int dtype, int is_max, double* out, int64_t* first) {
    if (!is_float_dtype(dtype) || n < 0) return -1;
    double acc = is_max ? -INFINITY : INFINITY;
    int64_t at = -1;
    for (int64_t i = 0; i < n; ++i) {
        double v = orc_load_float(x, i, dtype);
        if (at >= 0 && isnan(acc)) break; /* NaN is absorbing; keep the first one */
        if (isnan(v) || at < 0 || strictly_better(v, acc, is_max)) {
            acc = v;
            at = i;
        }
    }
    *out = acc;
    if (first) *first = at;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Segmented form.                                                      */
/* ------------------------------------------------------------------ */

int orc_segmented(const void* x, const int64_t* offsets, int64_t nseg, int dtype, int op,
                  void* out) {
    if (nseg < 0) return -2;
    size_t esz = (dtype == DT_F64 || dtype == DT_I64 || dtype == DT_U64) ? 8
               : (dtype == DT_F16 || dtype == DT_BF16) ? 2 : 4;
    int bitwise = (op == OP_AND || op == OP_OR || op == OP_XOR);
    for (int64_t s = 0; s < nseg; ++s) {
        int64_t b = offsets[s], e = offsets[s + 1];
        if (e < b) return -3;
        const void* p = (const char*)x + (size_t)b * esz;
        int64_t len = e - b;
        int rc;
        if (dtype == DT_I32 || dtype == DT_U32 || (bitwise && dtype == DT_F32)) {
            uint32_t r;
            rc = orc_fold_u32((const uint32_t*)p, len, op, dtype == DT_I32, &r);
            ((uint64_t*)out)[s] = r;
        } else if (dtype == DT_I64 || dtype == DT_U64 || (bitwise && dtype == DT_F64)) {
            uint64_t r;
            rc = orc_fold_u64((const uint64_t*)p, len, op, dtype == DT_I64, &r);
            ((uint64_t*)out)[s] = r;
        } else if (bitwise) {
            uint16_t r;
            rc = orc_fold_u16((const uint16_t*)p, len, op, &r);
            ((uint64_t*)out)[s] = r;
        } else if (op == OP_SUM) {
            rc = orc_exact_sum(p, len, dtype, &((double*)out)[s], 0);
        } else if (op == OP_PROD) {
            rc = orc_prod(p, len, dtype, &((double*)out)[s]);
        } else {
            rc = orc_minmax(p, len, dtype, op == OP_MAX, &((double*)out)[s], 0);
        }
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Scan (the prefix form of the reduction).                             */
/*                                                                      */
/* out[i] combines the elements of i's run up to and including i        */
/* (inclusive) or strictly before i (exclusive; the neutral element at  */
/* the first position of a run).  Position 0 and every position listed  */
/* in heads (nondecreasing; values outside [0, n) are ignored) start a  */
/* run, so a plain scan has no heads and a segmented scan over CSR      */
/* offsets passes the offsets.                                          */
/* ------------------------------------------------------------------ */

/* a (op) b on width-bit integers (signed comparison for min/max when is_signed). */
static uint64_t int_combine(uint64_t a, uint64_t b, int op, int width, int is_signed) {
    const uint64_t mask = width == 64 ? ~(uint64_t)0 : (((uint64_t)1 << width) - 1);
    uint64_t r;
    switch (op) {
    case OP_SUM: r = a + b; break;
    case OP_PROD: r = a * b; break;
    case OP_AND: r = a & b; break;
    case OP_OR: r = a | b; break;
    case OP_XOR: r = a ^ b; break;
    default: {
        int less;
        if (is_signed && width == 32) less = (int32_t)(uint32_t)a < (int32_t)(uint32_t)b;
        else if (is_signed && width == 64) less = (int64_t)a < (int64_t)b;
        else less = a < b;
        r = (op == OP_MIN) ? (less ? a : b) : (less ? b : a);
    }
    }
    return r & mask;
}

static uint64_t int_identity(int op, int width, int is_signed) {
    const uint64_t mask = width == 64 ? ~(uint64_t)0 : (((uint64_t)1 << width) - 1);
    const uint64_t sign = (uint64_t)1 << (width - 1);
    switch (op) {
    case OP_PROD: return 1u;
    case OP_AND: return mask;
    case OP_MIN: return is_signed ? sign - 1 : mask;
    case OP_MAX: return is_signed ? sign : 0u;
    default: return 0u; /* sum, or, xor */
    }
}

/* Running state of one run of a scan. */
typedef struct {
    int as_int, op, dtype, width, is_signed;
    uint64_t iacc;                    /* integer and bitwise ops */
    longacc* sum;                     /* float sum: exact */
    int sum_nan, sum_pinf, sum_ninf;
    dd prod;                          /* float product */
    double ext;                       /* float min/max */
} scan_state;

static void scan_restart(scan_state* st) {
    if (st->as_int) st->iacc = int_identity(st->op, st->width, st->is_signed);
    else if (st->op == OP_SUM) {
        la_init(st->sum);
        st->sum_nan = st->sum_pinf = st->sum_ninf = 0;
    } else if (st->op == OP_PROD) {
        st->prod.hi = 1.0;
        st->prod.lo = 0.0;
    } else st->ext = (st->op == OP_MAX) ? -INFINITY : INFINITY;
}

static void scan_fold(scan_state* st, const void* x, int64_t i) {
    if (st->as_int) {
        uint64_t v = st->width == 64 ? ((const uint64_t*)x)[i]
                   : st->width == 32 ? ((const uint32_t*)x)[i] : ((const uint16_t*)x)[i];
        st->iacc = int_combine(st->iacc, v, st->op, st->width, st->is_signed);
        return;
    }
    double v = orc_load_float(x, i, st->dtype);
    if (st->op == OP_SUM) {
        if (isnan(v)) st->sum_nan = 1;
        else if (isinf(v)) { if (v > 0) st->sum_pinf = 1; else st->sum_ninf = 1; }
        else la_add_double(st->sum, v, 0);
    } else if (st->op == OP_PROD) {
        st->prod = dd_mul_double(st->prod, v);
    } else if (!isnan(st->ext) && (isnan(v) || strictly_better(v, st->ext, st->op == OP_MAX))) {
        st->ext = v; /* a NaN, once in, stays */
    }
}

static void scan_emit(scan_state* st, void* out, int64_t i) {
    if (st->as_int) ((uint64_t*)out)[i] = st->iacc;
    else if (st->op == OP_SUM) {
        double r = la_round(st->sum);
        if (st->sum_nan || (st->sum_pinf && st->sum_ninf)) r = NAN;
        else if (st->sum_pinf) r = INFINITY;
        else if (st->sum_ninf) r = -INFINITY;
        ((double*)out)[i] = r;
    } else if (st->op == OP_PROD) ((double*)out)[i] = dd_value(st->prod);
    else ((double*)out)[i] = st->ext;
}

int orc_scan(const void* x, int64_t n, int dtype, int op, int exclusive, const int64_t* heads,
             int64_t nheads, void* out) {
    if (n < 0 || nheads < 0 || op < OP_SUM || op > OP_XOR || dtype < DT_I32 || dtype > DT_U64) return -2;
    for (int64_t h = 1; h < nheads; ++h)
        if (heads[h] < heads[h - 1]) return -3;
    static longacc acc; /* large; kept off the stack (oracle is single-threaded) */
    scan_state st;
    memset(&st, 0, sizeof st);
    st.op = op;
    st.dtype = dtype;
    st.as_int = !is_float_dtype(dtype) || op == OP_AND || op == OP_OR || op == OP_XOR;
    st.width = (dtype == DT_F64 || dtype == DT_I64 || dtype == DT_U64) ? 64
             : (dtype == DT_F16 || dtype == DT_BF16) ? 16 : 32;
    st.is_signed = (dtype == DT_I32 || dtype == DT_I64);
    st.sum = &acc;
    int64_t h = 0;
    for (int64_t i = 0; i < n; ++i) {
        int start = (i == 0);
        while (h < nheads && heads[h] <= i) start |= (heads[h++] == i);
        if (start) scan_restart(&st);
        if (exclusive) scan_emit(&st, out, i);
        scan_fold(&st, x, i);
        if (!exclusive) scan_emit(&st, out, i);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Row-wise forward and gradient.                                       */
/* ------------------------------------------------------------------ */

int orc_row_forward(const float* x, int64_t rows, int64_t cols, int op, double* y,
                    int64_t* idx, int64_t* zeros) {
    if (rows < 0 || cols < 0) return -2;
    for (int64_t r = 0; r < rows; ++r) {
        const float* row = x + r * cols;
        int rc = 0;
        if (idx) idx[r] = -1;
        if (zeros) zeros[r] = 0;
        if (op == OP_SUM) rc = orc_exact_sum(row, cols, DT_F32, &y[r], 0);
        else if (op == OP_PROD) {
            rc = orc_prod(row, cols, DT_F32, &y[r]);
            if (zeros) {
                int64_t z = 0;
                for (int64_t j = 0; j < cols; ++j) z += (row[j] == 0.0f);
                zeros[r] = z;
            }
        } else if (op == OP_MIN || op == OP_MAX) {
            int64_t at;
            rc = orc_minmax(row, cols, DT_F32, op == OP_MAX, &y[r], &at);
            if (idx) idx[r] = at;
        } else return -1;
        if (rc) return rc;
    }
    return 0;
}

int orc_row_grad(const float* x, int64_t rows, int64_t cols, int op, const double* g,
                 double* grad) {
    if (rows < 0 || cols < 0) return -2;
    for (int64_t r = 0; r < rows; ++r) {
        const float* row = x + r * cols;
        double* gr = grad + r * cols;
        if (op == OP_SUM) {
            /* d/dx_j of sum_i x_i is 1 for every j */
            for (int64_t j = 0; j < cols; ++j) gr[j] = g[r];
        } else if (op == OP_MIN || op == OP_MAX) {
            /* the extreme is x at the lowest attaining index; only that entry moves it */
            double v;
            int64_t at;
            int rc = orc_minmax(row, cols, DT_F32, op == OP_MAX, &v, &at);
            if (rc) return rc;
            for (int64_t j = 0; j < cols; ++j) gr[j] = (j == at) ? g[r] : 0.0;
        } else if (op == OP_PROD) {
            /* d/dx_j prod_i x_i = prod_{i<j} x_i * prod_{i>j} x_i: suffix products
               right to left into a scratch row, then a left-to-right walk that
               carries the prefix product. */
            static dd* suffix = 0;
            static int64_t cap = 0;
            if (cap < cols + 1) {
                dd* grown = (dd*)realloc(suffix, sizeof(dd) * (size_t)(cols + 1));
                if (!grown) return -4;
                suffix = grown;
                cap = cols + 1;
            }
            dd run = { 1.0, 0.0 };
            suffix[cols] = run;
            for (int64_t j = cols - 1; j >= 0; --j) {
                run = dd_mul_double(run, (double)row[j]);
                suffix[j] = run; /* product of x[j..cols) */
            }
            dd prefix = { 1.0, 0.0 }; /* product of x[0..j) */
            for (int64_t j = 0; j < cols; ++j) {
                dd t = dd_mul_double(dd_mul(prefix, suffix[j + 1]), g[r]);
                gr[j] = dd_value(t);
                prefix = dd_mul_double(prefix, (double)row[j]);
            }
        } else return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 as a CPU timing baseline (not a correctness source).     */
/* ------------------------------------------------------------------ */

/* One thread's share: the left fold of Algorithm 1 over x[lo..hi) of a
   float32 array, accumulated in double (Section 1.1's footnote names double
   precision as the simple remedy for float rounding). */
typedef struct {
    const float* x;
    int64_t lo, hi;
    double s;
} fold_part;

static void* fold_part_run(void* arg) {
    fold_part* p = (fold_part*)arg;
    double s = 0.0;
    for (int64_t i = p->lo; i < p->hi; ++i) s = s + (double)p->x[i];
    p->s = s;
    return 0;
}

int orc_fold_sum_f32(const float* x, int64_t n, int threads, double* out) {
    enum { MAX_THREADS = 256 };
    if (n < 0 || threads < 1 || threads > MAX_THREADS) return -2;
    fold_part part[MAX_THREADS];
    pthread_t tid[MAX_THREADS];
    for (int t = 0; t < threads; ++t) {
        part[t].x = x;
        part[t].lo = n / threads * t + (t < n % threads ? t : n % threads);
        part[t].hi = part[t].lo + n / threads + (t < n % threads ? 1 : 0);
        part[t].s = 0.0;
    }
    if (threads == 1) {
        fold_part_run(&part[0]);
        *out = part[0].s;
        return 0;
    }
    int started = 0;
    for (int t = 1; t < threads; ++t) {
        if (pthread_create(&tid[t], 0, fold_part_run, &part[t]) != 0) break;
        ++started;
    }
    fold_part_run(&part[0]);
    for (int t = 1; t <= started; ++t) pthread_join(tid[t], 0);
    if (started != threads - 1) return -4;
    double s = 0.0; /* the chunks' partial sums, folded in chunk order */
    for (int t = 0; t < threads; ++t) s = s + part[t].s;
    *out = s;
    return 0;
}
