/*
 * Plain C restatement of the oracle (TEST INFRASTRUCTURE ONLY): the per-rank
 * kernels of Table 3 and the execution model of Section 4, the same
 * definitions as the Python modules of this package, written out with no
 * blocking, vectorisation or reordering beyond what each definition states.
 * It is built into oracle/liboracle.so (gcc, no fast-math, no contraction of
 * a*b+c into one rounding); only tests/ and bench.py's CPU baseline load it.
 * It shares no code, header or constant with the GPU library.
 *
 * Exports (C-ABI, plain pointers and sizes):
 *   ref_vecadd_f32(a, b, c, n)            c[i] = fl32(a[i] + b[i])
 *   ref_vecmul_f32(a, b, c, n, iters)     c[i] = a[i] * b[i], iterated on c
 *   ref_bs_f64(S, K, T, r, sigma, call, put, n)  European call and put, binary64
 *   ref_sgemm_f64(A, B, C, n)             C = A B, n x n row-major, binary64 sums
 *   ref_sgemm_rows_f64(A, B, C, n, r0, rows)  rows r0 .. r0+rows-1 of the same
 *   model_eq1 .. model_eq11                closed forms of Section 4.1 / 4.2.3
 *   des_simulate(style, rules, n, t_in, t_comp, t_out)  discrete-event makespan
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* ------------------------------------------------------------ kernels */

/* Vector addition of Table 3: one correctly rounded binary32 addition per
 * element (x86-64 SSE arithmetic: round to nearest even, denormals kept). */
void ref_vecadd_f32(const float* a, const float* b, float* c, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i) c[i] = a[i] + b[i];
}

/* Vector multiplication of Table 3 (the model validation of Section 6): one
 * binary32 product per element, then `iters - 1` more products of the
 * running value by b[i]. */
void ref_vecmul_f32(const float* a, const float* b, float* c, uint64_t n, int iters) {
  for (uint64_t i = 0; i < n; ++i) {
    float v = a[i] * b[i];
    for (int t = 1; t < iters; ++t) v = v * b[i];
    c[i] = v;
  }
}

/* Standard normal distribution function N(x) = erfc(-x / sqrt 2) / 2. */
static double norm_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* European call and put without dividends (Black and Scholes 1973, the model
 * of the BlackScholes benchmark of Table 3), binary64 from binary32 inputs:
 *   d1 = (ln(S/K) + (r + sigma^2/2) T) / (sigma sqrt T),  d2 = d1 - sigma sqrt T
 *   call = S N(d1) - K e^{-rT} N(d2),  put = K e^{-rT} N(-d2) - S N(-d1);
 * where sigma sqrt T = 0 the price is its limit, the discounted intrinsic
 * value. */
void ref_bs_f64(const float* S, const float* K, const float* T, double r, double sigma, double* call, double* put,
                uint64_t n) {
  for (uint64_t i = 0; i < n; ++i) {
    const double s = S[i], k = K[i], t = T[i];
    const double vol = sigma * sqrt(t);
    const double dk = k * exp(-r * t);
    if (vol == 0.0) {
      call[i] = s - dk > 0.0 ? s - dk : 0.0;
      put[i] = dk - s > 0.0 ? dk - s : 0.0;
      continue;
    }
    const double d1 = (log(s / k) + (r + 0.5 * sigma * sigma) * t) / vol;
    const double d2 = d1 - vol;
    call[i] = s * norm_cdf(d1) - dk * norm_cdf(d2);
    put[i] = dk * norm_cdf(-d2) - s * norm_cdf(-d1);
  }
}

/* Single-precision matrix multiplication of Table 3, reference value:
 * C[i][j] = sum over k of A[i][k] B[k][j], products and sums in binary64, k
 * in increasing order; row-major n x n, no scaling, no transposes. */
void ref_sgemm_f64(const float* A, const float* B, double* C, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i)
    for (uint64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (uint64_t k = 0; k < n; ++k) s += (double)A[i * n + k] * (double)B[k * n + j];
      C[i * n + j] = s;
    }
}

/* The same for rows [row0, row0 + rows) of C only (written to C's first
 * `rows` rows): a bounded slice of a large product, for timing samples. */
void ref_sgemm_rows_f64(const float* A, const float* B, double* C, uint64_t n, uint64_t row0, uint64_t rows) {
  for (uint64_t i = row0; i < row0 + rows && i < n; ++i)
    for (uint64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (uint64_t k = 0; k < n; ++k) s += (double)A[i * n + k] * (double)B[k * n + j];
      C[(i - row0) * n + j] = s;
    }
}

/* ------------------------------------------------------------ execution model
 * Symbols of Table 2: n = N_process, t_init = T_init, t_ctx = T_ctx_switch,
 * t_in = T_data_in, t_comp = T_comp, t_out = T_data_out. */

static double dmax(double x, double y) { return x > y ? x : y; }
static double dmin(double x, double y) { return x < y ? x : y; }

/* Eq. 1: processes one after another, each with its own initialisation,
 * send, compute and retrieve, and a context switch between consecutive ones. */
double model_eq1(double n, double t_init, double t_ctx, double t_in, double t_comp, double t_out) {
  return n * (t_init + t_in + t_comp + t_out) + (n - 1.0) * t_ctx;
}
/* Eq. 2: compute-intensive kernels under PS-1. */
double model_eq2(double n, double t_in, double t_comp, double t_out) { return n * (t_in + t_out) + t_comp; }
/* Eq. 3: compute-intensive kernels under PS-2. */
double model_eq3(double n, double t_in, double t_comp, double t_out) { return t_in + n * t_comp + t_out; }
/* Eq. 4: I/O-intensive kernels under PS-1. */
double model_eq4(double n, double t_in, double t_comp, double t_out) { return n * (t_in + t_out) + t_comp; }
/* Eq. 5: I/O-intensive under PS-2 when t_out < t_in. */
double model_eq5(double n, double t_in, double t_comp, double t_out) { return n * t_in + t_comp + t_out; }
/* Eq. 6: I/O-intensive under PS-2 when t_out >= t_in. */
double model_eq6(double n, double t_in, double t_comp, double t_out) { return t_in + t_comp + n * t_out; }
/* Eq. 7: Eq. 5 and Eq. 6 in one expression. */
double model_eq7(double n, double t_in, double t_comp, double t_out) {
  return n * dmax(t_in, t_out) + t_comp + dmin(t_in, t_out);
}
/* Eq. 8: speedup of the virtualised compute-intensive case, Eq. 1 / Eq. 2. */
double model_eq8(double n, double t_init, double t_ctx, double t_in, double t_comp, double t_out) {
  return model_eq1(n, t_init, t_ctx, t_in, t_comp, t_out) / model_eq2(n, t_in, t_comp, t_out);
}
/* Eq. 9: speedup of the virtualised I/O-intensive case, Eq. 1 / Eq. 7. */
double model_eq9(double n, double t_init, double t_ctx, double t_in, double t_comp, double t_out) {
  return model_eq1(n, t_init, t_ctx, t_in, t_comp, t_out) / model_eq7(n, t_in, t_comp, t_out);
}
/* Eq. 10: the limit of Eq. 8 for many processes. */
double model_eq10(double t_init, double t_ctx, double t_in, double t_comp, double t_out) {
  return (t_init + t_in + t_comp + t_out + t_ctx) / (t_in + t_out);
}
/* Eq. 11: the limit of Eq. 9 for many processes. */
double model_eq11(double t_init, double t_ctx, double t_in, double t_comp, double t_out) {
  return (t_init + t_in + t_comp + t_out + t_ctx) / dmax(t_in, t_out);
}

/* Discrete-event schedule of the stream rules of Section 4.2.1 (the brute
 * force beside the closed forms): n streams, each with a send (t_in), a
 * kernel (t_comp) and a retrieve (t_out) in that order, enqueued in the
 * order of PS-1 (style 1: all sends, all kernels, all retrieves) or PS-2
 * (style 2: per stream send, kernel, retrieve).  Rules:
 *  1. an operation starts after the previous one of its stream has ended;
 *  2. sends are served one at a time, and so are retrieves, in enqueue
 *     order; a send and a retrieve may overlap;
 *  3. kernels never wait for one another except through 4 and 5;
 *  4. (rules 0, the single hardware queue) a retrieve waits until every
 *     kernel enqueued before it has ended;
 *  5. (rules 0) that wait holds back every kernel enqueued after the
 *     retrieve until it is satisfied.
 * rules 1 ("multiqueue") drops 4 and 5.  Every constraint refers to earlier
 * operations, so one pass in enqueue order gives every start time.  Returns
 * the time the last operation ends, or -1 for bad arguments. */
double des_simulate(int style, int rules, int n, double t_in, double t_comp, double t_out) {
  if (n < 1 || (style != 1 && style != 2) || (rules != 0 && rules != 1)) return -1.0;
  double* stream_end = (double*)calloc((size_t)n, sizeof(double));
  if (!stream_end) return -1.0;
  double send_free = 0.0, rtrv_free = 0.0, kernel_gate = 0.0, kernels_end = 0.0, last = 0.0;
  int kernels = 0;
  const int total = 3 * n;
  for (int q = 0; q < total; ++q) {
    int stream, kind; /* kind 0 send, 1 kernel, 2 retrieve */
    if (style == 1) {
      kind = q / n;
      stream = q % n;
    } else {
      stream = q / 3;
      kind = q % 3;
    }
    double start = stream_end[stream];
    double dur;
    if (kind == 0) {
      start = dmax(start, send_free);
      dur = t_in;
    } else if (kind == 1) {
      if (rules == 0) start = dmax(start, kernel_gate);
      dur = t_comp;
    } else {
      start = dmax(start, rtrv_free);
      if (rules == 0 && kernels > 0) {
        start = dmax(start, kernels_end);
        kernel_gate = dmax(kernel_gate, kernels_end);
      }
      dur = t_out;
    }
    const double end = start + dur;
    if (kind == 0) send_free = end;
    else if (kind == 2) rtrv_free = end;
    else {
      kernels_end = kernels ? dmax(kernels_end, end) : end;
      ++kernels;
    }
    stream_end[stream] = end;
    last = dmax(last, end);
  }
  free(stream_end);
  return last;
}
