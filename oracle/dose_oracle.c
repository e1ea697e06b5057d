/*
 * dose_oracle.c — CPU oracle for the dose product d = A x.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the GPU library
 * never links, calls or includes it, and it includes nothing from the library.
 *
 * Everything is computed from definitions, in FP64 where arithmetic happens:
 *
 *   - Value formats.  The paper stores the dose-deposition matrix in IEEE-754
 *     half precision (Sec. II-D, Sec. III).  Encoders below follow the IEEE-754
 *     binary16 / bfloat16 bit layouts and the OCP 8-bit E4M3 ("FN") layout:
 *     find the binade of |v|, scale |v| exactly by a power of two so that one
 *     quantum is 1, round to the nearest integer with ties to even, and
 *     assemble sign, biased exponent and significand.  Decoders evaluate the
 *     bit fields.  The E4M3 variant carries a per-row FP32 scale
 *     s_i = fl32(max_j |a_ij| / 448); its decoded entry is fl32(q_ij * s_i).
 *
 *   - Product.  Listing 1 of the paper computes, for every row i of a CSR
 *     matrix, y_i = sum over the row's stored entries k of data[k]*x[col[k]].
 *     The oracle evaluates exactly that sum, in ascending k, in FP64, starting
 *     from +0.  Every product of a decoded value (at most 24 significant bits)
 *     and an FP32 x is exact in FP64.
 *
 *   - Adjoint.  g_j = sum_i a_ij v_i, terms taken in ascending row order.
 *
 *   - Quadratic objective of plan optimisation (Sec. I: each optimisation
 *     iteration needs the dose, the objective and its gradient):
 *     f = sum_v w_v (d_v - p_v)^2 and the adjoint seed 2 w_v (d_v - p_v).
 *
 *   - Scenario dose and robust objective (Sec. I and II-A: the dose of several
 *     beams, possibly under several realisations of the uncertainties, is
 *     needed every iteration).  Each beam has its own deposition matrix over
 *     the shared dose grid, so the dose of one scenario is the sum of its
 *     beams' doses.  Over the scenarios' objectives f_s the robust forms are
 *     the worst case max_s f_s and the expectation sum_s pi_s f_s.  Their
 *     derivatives with respect to scenario s's objective are the weights c_s:
 *     pi_s (1/S without probabilities) for the expectation; for the worst
 *     case 1 for the first scenario attaining the maximum and 0 otherwise.
 *     The gradient seed of scenario s's dose is c_s times its own seed.
 *
 * Built with -O2 -fno-fast-math -ffp-contract=off so that the compiler keeps
 * every rounding as written.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* IEEE-754 binary16: 1 sign, 5 exponent (bias 15), 10 significand bits */
/* ------------------------------------------------------------------ */
uint16_t or_f16_encode(float v) {
  uint16_t sign = signbit(v) ? 0x8000u : 0u;
  if (isnan(v)) return 0x7E00u;
  if (isinf(v)) return sign | 0x7C00u;
  double a = fabs((double)v);
  if (a == 0.0) return sign;
  int e;
  frexp(a, &e);
  int E = e - 1; /* 2^E <= a < 2^(E+1) */
  if (E < -14) { /* below the normal range: one quantum is 2^-24 */
    double q = nearbyint(ldexp(a, 24));
    return (uint16_t)(sign | (uint16_t)q); /* q == 1024 is the smallest normal */
  }
  double q = nearbyint(ldexp(a, 10 - E)); /* 1024 <= q <= 2048 */
  if (q == 2048.0) {
    q = 1024.0;
    E += 1;
  }
  if (E > 15) return sign | 0x7C00u; /* rounds past 65504: infinity */
  return (uint16_t)(sign | (uint16_t)((E + 15) << 10) | (uint16_t)(q - 1024.0));
}

double or_f16_decode(uint16_t h) {
  int s = (h >> 15) & 1, E = (h >> 10) & 31, m = h & 1023;
  double mag;
  if (E == 31)
    mag = m ? NAN : INFINITY;
  else if (E == 0)
    mag = ldexp((double)m, -24);
  else
    mag = ldexp((double)(1024 + m), E - 25);
  return s ? -mag : mag;
}

/* ------------------------------------------------------------------ */
/* bfloat16: 1 sign, 8 exponent (bias 127), 7 significand bits          */
/* ------------------------------------------------------------------ */
uint16_t or_bf16_encode(float v) {
  uint16_t sign = signbit(v) ? 0x8000u : 0u;
  if (isnan(v)) return 0x7FC0u;
  if (isinf(v)) return sign | 0x7F80u;
  double a = fabs((double)v);
  if (a == 0.0) return sign;
  int e;
  frexp(a, &e);
  int E = e - 1;
  if (E < -126) { /* one quantum is 2^-133 */
    double q = nearbyint(ldexp(a, 133));
    return (uint16_t)(sign | (uint16_t)q);
  }
  double q = nearbyint(ldexp(a, 7 - E)); /* 128 <= q <= 256 */
  if (q == 256.0) {
    q = 128.0;
    E += 1;
  }
  if (E > 127) return sign | 0x7F80u;
  return (uint16_t)(sign | (uint16_t)((E + 127) << 7) | (uint16_t)(q - 128.0));
}

double or_bf16_decode(uint16_t b) {
  int s = (b >> 15) & 1, E = (b >> 7) & 255, m = b & 127;
  double mag;
  if (E == 255)
    mag = m ? NAN : INFINITY;
  else if (E == 0)
    mag = ldexp((double)m, -133);
  else
    mag = ldexp((double)(128 + m), E - 134);
  return s ? -mag : mag;
}

/* ------------------------------------------------------------------ */
/* OCP E4M3 (FN): 1 sign, 4 exponent (bias 7), 3 significand bits; no   */
/* infinities, S.1111.111 is NaN, largest finite 448.  Rounds to       */
/* nearest-even and saturates magnitudes above 448 to 448.             */
/* ------------------------------------------------------------------ */
uint8_t or_e4m3_encode_sat(float v) {
  uint8_t sign = signbit(v) ? 0x80u : 0u;
  if (isnan(v)) return 0x7Fu;
  double a = fabs((double)v);
  if (a == 0.0) return sign;
  if (isinf(v)) return sign | 0x7Eu;
  int e;
  frexp(a, &e);
  int E = e - 1;
  if (E < -6) { /* one quantum is 2^-9 */
    double q = nearbyint(ldexp(a, 9));
    return (uint8_t)(sign | (uint8_t)q); /* q == 8 is the smallest normal */
  }
  double q = nearbyint(ldexp(a, 3 - E)); /* 8 <= q <= 16 */
  if (q == 16.0) {
    q = 8.0;
    E += 1;
  }
  if (E > 8) return sign | 0x7Eu;
  unsigned code = (unsigned)((E + 7) << 3) | (unsigned)(q - 8.0);
  if (code > 0x7Eu) code = 0x7Eu;
  return (uint8_t)(sign | code);
}

double or_e4m3_decode(uint8_t c) {
  int s = (c >> 7) & 1, E = (c >> 3) & 15, m = c & 7;
  double mag;
  if (E == 15 && m == 7)
    mag = NAN;
  else if (E == 0)
    mag = ldexp((double)m, -9);
  else
    mag = ldexp((double)(8 + m), E - 10);
  return s ? -mag : mag;
}

/* Per-row scale of the E4M3 variant: fl32(amax / 448); 1 when that is 0
 * (an all-zero row, or amax so small that the quotient underflows). */
float or_e4m3_row_scale(const float* vals, int64_t n) {
  float amax = 0.0f;
  for (int64_t k = 0; k < n; ++k) {
    float a = fabsf(vals[k]);
    if (a > amax) amax = a;
  }
  float s = amax / 448.0f;
  return s == 0.0f ? 1.0f : s;
}

/* ------------------------------------------------------------------ */
/* Array helpers: encode and decode whole value streams.                */
/* ------------------------------------------------------------------ */
void or_f16_encode_n(const float* v, int64_t n, uint16_t* out) {
  for (int64_t k = 0; k < n; ++k) out[k] = or_f16_encode(v[k]);
}
void or_f16_decode_n(const uint16_t* h, int64_t n, double* out) {
  for (int64_t k = 0; k < n; ++k) out[k] = or_f16_decode(h[k]);
}
void or_bf16_encode_n(const float* v, int64_t n, uint16_t* out) {
  for (int64_t k = 0; k < n; ++k) out[k] = or_bf16_encode(v[k]);
}
void or_bf16_decode_n(const uint16_t* h, int64_t n, double* out) {
  for (int64_t k = 0; k < n; ++k) out[k] = or_bf16_decode(h[k]);
}
void or_e4m3_encode_n(const float* v, int64_t n, uint8_t* out) {
  for (int64_t k = 0; k < n; ++k) out[k] = or_e4m3_encode_sat(v[k]);
}
void or_e4m3_decode_n(const uint8_t* c, int64_t n, double* out) {
  for (int64_t k = 0; k < n; ++k) out[k] = or_e4m3_decode(c[k]);
}

/* Decoded matrix entries (as FP32, which holds every decoded value exactly)
 * for a CSR matrix whose FP32 source values are `vals`.
 * fmt: 1 = binary16, 2 = bfloat16, 3 = E4M3 with per-row scale, 4 = the FP32
 * values themselves (the paper's Single configuration, Sec. V).
 * For fmt 3, `scale_out` (n_rows entries) receives the row scales. */
int or_decode_matrix(int fmt, int64_t n_rows, const int64_t* row_ptr, const float* vals,
                     float* dec_out, float* scale_out) {
  for (int64_t i = 0; i < n_rows; ++i) {
    int64_t b = row_ptr[i], e = row_ptr[i + 1];
    if (fmt == 1) {
      for (int64_t k = b; k < e; ++k) dec_out[k] = (float)or_f16_decode(or_f16_encode(vals[k]));
    } else if (fmt == 2) {
      for (int64_t k = b; k < e; ++k) dec_out[k] = (float)or_bf16_decode(or_bf16_encode(vals[k]));
    } else if (fmt == 3) {
      float s = or_e4m3_row_scale(vals + b, e - b);
      if (scale_out) scale_out[i] = s;
      for (int64_t k = b; k < e; ++k) {
        float t = vals[k] / s;                               /* fl32(a / s) */
        float q = (float)or_e4m3_decode(or_e4m3_encode_sat(t)); /* exact in FP32 */
        dec_out[k] = q * s;                                  /* fl32(q * s) */
      }
    } else if (fmt == 4) {
      for (int64_t k = b; k < e; ++k) dec_out[k] = vals[k];
    } else {
      return -1;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* The product.                                                         */
/* ------------------------------------------------------------------ */
double or_row_dot(int64_t n, const int32_t* col, const float* dec, const float* x) {
  double acc = 0.0;
  for (int64_t k = 0; k < n; ++k) acc += (double)dec[k] * (double)x[col[k]];
  return acc;
}

void or_spmv(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const float* dec,
             const float* x, double* y) {
  for (int64_t i = 0; i < n_rows; ++i)
    y[i] = or_row_dot(row_ptr[i + 1] - row_ptr[i], col + row_ptr[i], dec + row_ptr[i], x);
}

/* The same product with the rows shared among threads (OpenMP; rows are
 * independent, so every y[i] is the same sum as in or_spmv).  Used to time
 * the oracle on all host cores; without OpenMP it is or_spmv. */
void or_spmv_rows_parallel(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const float* dec,
                           const float* x, double* y) {
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n_rows; ++i)
    y[i] = or_row_dot(row_ptr[i + 1] - row_ptr[i], col + row_ptr[i], dec + row_ptr[i], x);
}

/* Threads or_spmv_rows_parallel uses (1 without OpenMP). */
int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Same product for a multi-vector x stored [n_cols][n_rhs] -> y [n_rows][n_rhs]. */
void or_spmv_multi(int64_t n_rows, int32_t n_rhs, const int64_t* row_ptr, const int32_t* col,
                   const float* dec, const float* x, double* y) {
  for (int64_t i = 0; i < n_rows; ++i)
    for (int32_t r = 0; r < n_rhs; ++r) {
      double acc = 0.0;
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
        acc += (double)dec[k] * (double)x[(int64_t)col[k] * n_rhs + r];
      y[i * n_rhs + r] = acc;
    }
}

/* g = A^T v: for each column j, sum over rows i (ascending) of a_ij v_i. */
void or_spmv_T(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr, const int32_t* col,
               const float* dec, const float* v, double* g) {
  for (int64_t j = 0; j < n_cols; ++j) g[j] = 0.0;
  for (int64_t i = 0; i < n_rows; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
      g[col[k]] += (double)dec[k] * (double)v[i];
}

/* Transposed CSR of (row_ptr, col, dec): stable counting sort by column, so
 * the rows of A^T list their entries in ascending row of A. */
void or_transpose(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr, const int32_t* col,
                  const float* dec, int64_t* t_row_ptr, int32_t* t_col, float* t_dec) {
  for (int64_t j = 0; j <= n_cols; ++j) t_row_ptr[j] = 0;
  for (int64_t k = 0; k < row_ptr[n_rows]; ++k) t_row_ptr[col[k] + 1] += 1;
  for (int64_t j = 0; j < n_cols; ++j) t_row_ptr[j + 1] += t_row_ptr[j];
  /* next free slot of every row of A^T */
  for (int64_t i = 0; i < n_rows; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int64_t j = col[k];
      int64_t slot = t_row_ptr[j]++;
      t_col[slot] = (int32_t)i;
      t_dec[slot] = dec[k];
    }
  for (int64_t j = n_cols; j > 0; --j) t_row_ptr[j] = t_row_ptr[j - 1];
  t_row_ptr[0] = 0;
}

/* f = sum_v w_v (d_v - p_v)^2, ascending v, in FP64. */
double or_objective(int64_t n, const double* d, const float* p, const float* w) {
  double f = 0.0;
  for (int64_t v = 0; v < n; ++v) {
    double r = d[v] - (double)p[v];
    f += (double)w[v] * r * r;
  }
  return f;
}

/* Adjoint seed df/dd_v = 2 w_v (d_v - p_v), in FP64. */
void or_objective_seed(int64_t n, const double* d, const float* p, const float* w, double* out) {
  for (int64_t v = 0; v < n; ++v) out[v] = 2.0 * (double)w[v] * (d[v] - (double)p[v]);
}

/* sqrt(sum g_j^2), ascending j, in FP64. */
double or_norm2(int64_t n, const double* g) {
  double s = 0.0;
  for (int64_t j = 0; j < n; ++j) s += g[j] * g[j];
  return sqrt(s);
}

/* Dose of one scenario: d_v = sum_b part[b*n + v] over beams b ascending, in
 * FP64 (part holds the n-voxel dose of each beam, one after another). */
void or_beam_sum(int32_t n_beams, int64_t n, const double* part, double* d) {
  for (int64_t v = 0; v < n; ++v) {
    double s = 0.0;
    for (int32_t b = 0; b < n_beams; ++b) s += part[(int64_t)b * n + v];
    d[v] = s;
  }
}

/* Robust forms of the scenario objectives f_0..f_{S-1}: the worst case
 * max_s f_s with the first scenario attaining it, and the expectation
 * sum_s pi_s f_s in ascending s, or (sum_s f_s) / S when prob is NULL. */
void or_robust(int32_t n_scen, const double* f, const double* prob, double* worst, int64_t* arg,
               double* expected) {
  double w = f[0], e = 0.0;
  int64_t a = 0;
  for (int32_t s = 1; s < n_scen; ++s)
    if (f[s] > w) {
      w = f[s];
      a = s;
    }
  if (prob) {
    for (int32_t s = 0; s < n_scen; ++s) e += prob[s] * f[s];
  } else {
    for (int32_t s = 0; s < n_scen; ++s) e += f[s];
    e = e / (double)n_scen;
  }
  *worst = w;
  *arg = a;
  *expected = e;
}

/* Weights c_s of the robust forms (their derivatives with respect to f_s):
 * worst != 0: 1 for the first s attaining max f_s, else 0; worst == 0:
 * prob[s], or 1/n_scen without probabilities. */
void or_robust_weights(int32_t n_scen, const double* f, const double* prob, int32_t worst, double* c) {
  if (worst) {
    int32_t a = 0;
    for (int32_t s = 1; s < n_scen; ++s)
      if (f[s] > f[a]) a = s;
    for (int32_t s = 0; s < n_scen; ++s) c[s] = s == a ? 1.0 : 0.0;
  } else {
    for (int32_t s = 0; s < n_scen; ++s) c[s] = prob ? prob[s] : 1.0 / (double)n_scen;
  }
}

/* ------------------------------------------------------------------ */
/* SELL-C-sigma storage (Kreutzer et al., SIAM J. Sci. Comput. 36(5),   */
/* 2014), the SIMD-oriented sparse format the paper names as the next   */
/* one to investigate for dose matrices (Sec. II-C, Sec. VII).          */
/* ------------------------------------------------------------------ */
/* The layout: the rows are taken in consecutive windows of sigma rows (the
 * last window may be shorter); inside a window the rows are ordered by
 * descending length, rows of equal length keeping their ascending order.
 * The resulting sequence perm[0 .. n_rows) is cut into chunks of C
 * consecutive positions (the last chunk may hold fewer rows); a chunk's
 * width is the length of its longest row.  perm: n_rows entries;
 * width: ceil(n_rows / C) entries.  The sort is a plain insertion sort: slow
 * and obviously stable. */
void or_sell_layout(int64_t n_rows, const int64_t* row_ptr, int64_t C, int64_t sigma, int64_t* perm,
                    int64_t* width) {
  for (int64_t w0 = 0; w0 < n_rows; w0 += sigma) {
    int64_t w1 = w0 + sigma < n_rows ? w0 + sigma : n_rows;
    for (int64_t k = w0; k < w1; ++k) {
      int64_t r = k, len = row_ptr[r + 1] - row_ptr[r];
      int64_t q = k;
      /* move r before every earlier row of the window that is strictly shorter */
      while (q > w0 && row_ptr[perm[q - 1] + 1] - row_ptr[perm[q - 1]] < len) {
        perm[q] = perm[q - 1];
        --q;
      }
      perm[q] = r;
    }
  }
  for (int64_t c = 0; c * C < n_rows; ++c) {
    int64_t wmax = 0;
    for (int64_t i = c * C; i < (c + 1) * C && i < n_rows; ++i) {
      int64_t len = row_ptr[perm[i] + 1] - row_ptr[perm[i]];
      if (len > wmax) wmax = len;
    }
    width[c] = wmax;
  }
}

/* The packed SELL-C-sigma arrays: chunk c starts at off_c = C * (width_0 +
 * ... + width_(c-1)); entry j of the row at chunk position i (0 <= i < C)
 * sits at off_c + j * C + i (column-major inside the chunk).  Slots past a
 * row's length (and rows past n_rows in the last chunk) are padding: value
 * 0 and column -1.  val, col: C * sum(width) entries. */
void or_sell_pack(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const float* dec, int64_t C,
                  const int64_t* perm, const int64_t* width, float* sval, int32_t* scol) {
  int64_t off = 0;
  for (int64_t c = 0; c * C < n_rows; ++c) {
    for (int64_t j = 0; j < width[c]; ++j)
      for (int64_t i = 0; i < C; ++i) {
        int64_t slot = off + j * C + i, pos = c * C + i;
        sval[slot] = 0.0f;
        scol[slot] = -1;
        if (pos < n_rows) {
          int64_t r = perm[pos];
          if (j < row_ptr[r + 1] - row_ptr[r]) {
            sval[slot] = dec[row_ptr[r] + j];
            scol[slot] = col[row_ptr[r] + j];
          }
        }
      }
    off += C * width[c];
  }
}

/* y = A x over the packed arrays: the row at chunk position i gets the sum,
 * in ascending j, of its non-padding slots (FP64, from +0), stored at its
 * original index perm[c * C + i]. */
void or_sell_spmv(int64_t n_rows, int64_t C, const int64_t* perm, const int64_t* width, const float* sval,
                  const int32_t* scol, const float* x, double* y) {
  int64_t off = 0;
  for (int64_t c = 0; c * C < n_rows; ++c) {
    for (int64_t i = 0; i < C && c * C + i < n_rows; ++i) {
      double acc = 0.0;
      for (int64_t j = 0; j < width[c]; ++j) {
        int64_t slot = off + j * C + i;
        if (scol[slot] >= 0) acc += (double)sval[slot] * (double)x[scol[slot]];
      }
      y[perm[c * C + i]] = acc;
    }
    off += C * width[c];
  }
}

/* ------------------------------------------------------------------ */
/* Run-length column indices.  In a dose row the stored spots form a    */
/* few runs of consecutive columns (a pencil beam's spots along one     */
/* scanline), so the row's columns are described by (start, length)    */
/* pairs: the maximal runs c, c+1, ..., c+L-1 of consecutive columns,   */
/* in the row's order.  The paper notes that column indices are a       */
/* large part of the bytes moved (Sec. V); runs shrink them.            */
/* ------------------------------------------------------------------ */
/* run_ptr: n_rows + 1 offsets into start/len (run_ptr[0] = 0); start, len:
 * room for nnz runs.  Returns the number of runs. */
int64_t or_runs_encode(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, int64_t* run_ptr,
                       int32_t* start, int32_t* len) {
  int64_t n = 0;
  run_ptr[0] = 0;
  for (int64_t i = 0; i < n_rows; ++i) {
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      if (k > row_ptr[i] && col[k] == col[k - 1] + 1) {
        len[n - 1] += 1; /* continues the current run */
      } else {
        start[n] = col[k];
        len[n] = 1;
        ++n;
      }
    }
    run_ptr[i + 1] = n;
  }
  return n;
}

/* The columns the runs describe, row after row. */
void or_runs_decode(int64_t n_rows, const int64_t* run_ptr, const int32_t* start, const int32_t* len,
                    int32_t* col) {
  int64_t k = 0;
  for (int64_t i = 0; i < n_rows; ++i)
    for (int64_t r = run_ptr[i]; r < run_ptr[i + 1]; ++r)
      for (int32_t t = 0; t < len[r]; ++t) col[k++] = start[r] + t;
}
