/*
 * fh_oracle.c -- reference (oracle) generalized FrequencyHough, plain C, FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (libfh) shares no code, header, table generator or constant with it.
 *
 * What it computes (Miller et al., "A method to search for long duration
 * gravitational wave transients from isolated neutron stars using the
 * generalized FrequencyHough"):
 *
 *   - Sec. IV, Eq. (transform): a frequency f maps to x = f^(1-n); a signal
 *     following the power law of Sec. II (Eqs. diff_powlaws / powlaws) is the
 *     straight line x = x0 + (n-1) k (t - t0) in the (t - t0, x) plane.
 *   - Sec. IV: every peak of the time/frequency peakmap (Sec. III) therefore
 *     maps to a line in the (x0, k) plane,
 *        x0 = x - (n-1) k (t - t0);
 *     the Hough map is the histogram of these lines over an (x0, k) grid.
 *   - Sec. VI.C: the x0 grid is uniform with step dx0 = (n-1) df / f^n taken
 *     at the highest frequency f_max of the band (the smallest step), which
 *     starts at x0_min = f_max^(1-n).
 *
 * A peak occupies one frequency bin [f_j, f_j + df), df = 1/T_FFT.  Because x
 * decreases with f, the bin's image is the x-interval (X_{j+1}, X_j] with
 * X_j = f_j^(1-n); at row k_r and time T_i = t_i - t0 it is shifted by
 * -(n-1) k_r T_i.  In column units of the x0 grid,
 *
 *     u = A_j - C_r T_i,   A_j = (X_j - x0_min) / dx0,   C_r = (n-1) k_r / dx0,
 *
 * and the peak counts once in every column b with floor(u_lo) <= b <= floor(u_hi)
 * (u_lo from the bin's upper edge f_{j+1}, u_hi from its lower edge f_j),
 * clipped to [0, n_x0).
 *
 * Canonical floating point (fixed here so that any other implementation can
 * be compared bit for bit; every operation is one IEEE-754 binary64 operation
 * rounded to nearest, no contraction):
 *     df     = 1 / tfft
 *     f_j    = f_min + j * df                       (j = 0 .. n_f)
 *     X_j    = pow(f_j, 1 - n)
 *     x0_min = pow(f_max, 1 - n)                    (default)
 *     dx0    = ((n - 1) * df) * pow(f_max, -n)      (default)
 *     inv    = 1 / dx0
 *     A_j    = (X_j - x0_min) * inv
 *     C_r    = ((n - 1) * k_r) * inv
 *     T_i    = (i + 0.5) * tfft                     (FFT mid-time, t0 = start
 *                                                    of the first FFT) unless
 *                                                    explicit times are given
 *     u      = fma(-C_r, T_i, A)                    (single rounding)
 * and n_x0 defaults to ceil(N* - 1e-9) with the closed form
 *     N* = f_max ((f_max/f_min)^(n-1) - 1) / ((n-1) df),
 * the width of the transformed band [x0_min, f_min^(1-n)] in units of dx0.
 *
 * The accumulation here is deliberately the slow, direct one: for every
 * (row, peak) pair every covered cell is incremented.  The library reaches the
 * same integers through edge (+1/-1) updates and a prefix sum.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1

/* ---------------------------------------------------------------- grids -- */

/* Number of frequency bins of the band, or -1 if (f_max - f_min) * tfft is not
 * an integer to within 1e-9 (the peakmap's bins must tile the band). */
int orc_n_freq(double tfft, double f_min, double f_max) {
  double w = (f_max - f_min) * tfft;
  double r = floor(w + 0.5);
  if (!(fabs(w - r) <= 1e-9) || r < 1.0 || r > 2.0e9) return -1;
  return (int)r;
}

/* x = f^(1-n): the linearising change of coordinates (Sec. IV, Eq. transform). */
double orc_transform(double f, double n) { return pow(f, 1.0 - n); }

/* Default x0 grid of Sec. VI.C: start at f_max^(1-n), step (n-1) df f_max^(-n). */
void orc_x0_grid(double n, double tfft, double f_max, double* x0_min, double* dx0) {
  double df = 1.0 / tfft;
  *x0_min = pow(f_max, 1.0 - n);
  *dx0 = ((n - 1.0) * df) * pow(f_max, -n);
}

/* Columns needed to cover [f_max^(1-n), f_min^(1-n)] at the default step,
 * from the closed form (exact for rational band edges; the 1e-9 absorbs the
 * rounding of the closed form itself). */
int orc_n_x0(double n, double tfft, double f_min, double f_max) {
  double df = 1.0 / tfft;
  double nstar = f_max * (pow(f_max / f_min, n - 1.0) - 1.0) / ((n - 1.0) * df);
  double c = ceil(nstar - 1e-9);
  if (!(c >= 1.0) || c > 2.0e9) return -1;
  return (int)c;
}

/* The three tables of the canonical form.  A has n_f + 1 entries (bin edges),
 * C has n_k (rows), T has n_fft (times).  t may be NULL (FFT mid-times). */
void orc_tables(double n, double tfft, double f_min, int n_f, double x0_min, double dx0, int n_k,
                const double* k, int n_fft, const double* t, double* A, double* C, double* T) {
  double df = 1.0 / tfft;
  double inv = 1.0 / dx0;
  for (int j = 0; j <= n_f; ++j) {
    double fj = f_min + (double)j * df;
    double xj = pow(fj, 1.0 - n);
    A[j] = (xj - x0_min) * inv;
  }
  for (int r = 0; r < n_k; ++r) C[r] = ((n - 1.0) * k[r]) * inv;
  for (int i = 0; i < n_fft; ++i) T[i] = t ? t[i] : ((double)i + 0.5) * tfft;
}

/* ---------------------------------------------------------------- hough -- */

typedef struct {
  double n, tfft, f_min, f_max;
  int32_t n_fft;
  const double* t;  /* NULL: FFT mid-times */
  int32_t n_k;
  const double* k;
  double x0_min, dx0; /* dx0 == 0: defaults of Sec. VI.C */
  int32_t n_x0;       /* 0: closed-form default */
} orc_desc;

/* Resolve the grid of a description: fills n_f, x0_min, dx0, n_x0. */
int orc_resolve(const orc_desc* d, int* n_f, double* x0_min, double* dx0, int* n_x0) {
  *n_f = orc_n_freq(d->tfft, d->f_min, d->f_max);
  if (*n_f < 0) return ORC_EINVAL;
  if (d->dx0 != 0.0) {
    *x0_min = d->x0_min;
    *dx0 = d->dx0;
  } else {
    orc_x0_grid(d->n, d->tfft, d->f_max, x0_min, dx0);
  }
  *n_x0 = d->n_x0 > 0 ? d->n_x0 : orc_n_x0(d->n, d->tfft, d->f_min, d->f_max);
  if (*n_x0 <= 0) return ORC_EINVAL;
  return ORC_OK;
}

/*
 * Direct Hough map for the rows listed in `rows` (n_rows of them; rows == NULL
 * means all n_k rows in order).  out is int32 [n_rows][n_x0], row-major, x0
 * ascending.  Peaks are a CSR by FFT: FFT i owns bin[row_ptr[i] .. row_ptr[i+1]).
 * A bin index outside [0, n_f) is skipped and counted in *n_bad.  *n_pairs
 * (if not NULL) gets the number of (row, peak) pairs whose clipped interval
 * holds at least one column, the work the map really contains.
 */
int orc_hough_rows_pairs(const orc_desc* d, const int32_t* row_ptr, const int32_t* bin, const int32_t* rows,
                         int32_t n_rows, int32_t* out, int64_t* n_bad, int64_t* n_pairs) {
  int n_f, n_x0;
  double x0_min, dx0;
  if (orc_resolve(d, &n_f, &x0_min, &dx0, &n_x0) != ORC_OK) return ORC_EINVAL;
  double* A = (double*)malloc(sizeof(double) * (size_t)(n_f + 1));
  double* C = (double*)malloc(sizeof(double) * (size_t)(d->n_k > 0 ? d->n_k : 1));
  double* T = (double*)malloc(sizeof(double) * (size_t)(d->n_fft > 0 ? d->n_fft : 1));
  if (!A || !C || !T) {
    free(A); free(C); free(T);
    return ORC_EINVAL;
  }
  orc_tables(d->n, d->tfft, d->f_min, n_f, x0_min, dx0, d->n_k, d->k, d->n_fft, d->t, A, C, T);
  int nr = rows ? n_rows : d->n_k;
  memset(out, 0, sizeof(int32_t) * (size_t)nr * (size_t)n_x0);
  int64_t bad = 0, pairs = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad, pairs)
  for (int q = 0; q < nr; ++q) {
    int r = rows ? rows[q] : q;
    int32_t* h = out + (size_t)q * (size_t)n_x0;
    for (int i = 0; i < d->n_fft; ++i) {
      for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        int32_t j = bin[p];
        if (j < 0 || j >= n_f) {
          if (q == 0) ++bad;
          continue;
        }
        double u_lo = fma(-C[r], T[i], A[j + 1]); /* upper bin edge f_{j+1} */
        double u_hi = fma(-C[r], T[i], A[j]);     /* lower bin edge f_j */
        double b_lo = floor(u_lo);
        double b_hi = floor(u_hi);
        if (b_lo < 0.0) b_lo = 0.0;
        if (b_hi > (double)(n_x0 - 1)) b_hi = (double)(n_x0 - 1);
        pairs += b_lo <= b_hi;
        for (double b = b_lo; b <= b_hi; b += 1.0) h[(int64_t)b] += 1;
      }
    }
  }
  if (n_bad) *n_bad = bad;
  if (n_pairs) *n_pairs = pairs;
  free(A); free(C); free(T);
  return ORC_OK;
}

int orc_hough_rows(const orc_desc* d, const int32_t* row_ptr, const int32_t* bin, const int32_t* rows,
                   int32_t n_rows, int32_t* out, int64_t* n_bad) {
  return orc_hough_rows_pairs(d, row_ptr, bin, rows, n_rows, out, n_bad, NULL);
}

int orc_hough(const orc_desc* d, const int32_t* row_ptr, const int32_t* bin, int32_t* out, int64_t* n_bad) {
  return orc_hough_rows(d, row_ptr, bin, NULL, 0, out, n_bad);
}

/*
 * Rows of a map for checking large maps: the same direct counting as
 * orc_hough_rows_pairs, plus per-row totals, but each row stops early where
 * the definition says nothing more can land in the grid.  For n > 1 the
 * table A_j decreases with j (x = f^(1-n) falls as f grows) and, with k >= 0,
 * u = fma(-C_r, T_i, A_j) can only fall as j or T_i grows (rounding is
 * monotone).  So once a peak's u_hi is negative (its interval lies left of
 * column 0), every later peak of that FFT lies left too; and once the lowest
 * bin edge A_0 of an FFT is left of column 0, every later FFT is too.  These
 * exits need the bins of every FFT strictly ascending and times ascending;
 * when any FFT is not ascending, or n <= 1, the function takes every pair.
 * out (may be NULL) is int32 [n_rows][n_x0]; totals[q] = number of (peak,
 * cell) incidences of row rows[q] (the sum of its clipped interval widths);
 * pairs[q] = number of pairs with a non-empty clipped interval.
 */
int orc_rows_checked(const orc_desc* d, const int32_t* row_ptr, const int32_t* bin, const int32_t* rows,
                     int32_t n_rows, int32_t* out, int64_t* totals, int64_t* pairs_out) {
  int n_f, n_x0;
  double x0_min, dx0;
  if (orc_resolve(d, &n_f, &x0_min, &dx0, &n_x0) != ORC_OK) return ORC_EINVAL;
  double* A = (double*)malloc(sizeof(double) * (size_t)(n_f + 1));
  double* C = (double*)malloc(sizeof(double) * (size_t)(d->n_k > 0 ? d->n_k : 1));
  double* T = (double*)malloc(sizeof(double) * (size_t)(d->n_fft > 0 ? d->n_fft : 1));
  if (!A || !C || !T) {
    free(A); free(C); free(T);
    return ORC_EINVAL;
  }
  orc_tables(d->n, d->tfft, d->f_min, n_f, x0_min, dx0, d->n_k, d->k, d->n_fft, d->t, A, C, T);
  int exits = d->n > 1.0;
  for (int i = 0; i < d->n_fft && exits; ++i) {
    if (i > 0 && T[i] < T[i - 1]) exits = 0;
    for (int32_t p = row_ptr[i] + 1; p < row_ptr[i + 1]; ++p)
      if (bin[p] <= bin[p - 1]) exits = 0;
  }
  if (out) memset(out, 0, sizeof(int32_t) * (size_t)n_rows * (size_t)n_x0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int q = 0; q < n_rows; ++q) {
    const int r = rows[q];
    int32_t* h = out ? out + (size_t)q * (size_t)n_x0 : NULL;
    int64_t tot = 0, prs = 0;
    int row_exit = exits && C[r] >= 0.0;
    for (int i = 0; i < d->n_fft; ++i) {
      if (row_exit && fma(-C[r], T[i], A[0]) < 0.0) break; /* this FFT and all later ones left of the grid */
      for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        int32_t j = bin[p];
        if (j < 0 || j >= n_f) continue;
        double u_lo = fma(-C[r], T[i], A[j + 1]);
        double u_hi = fma(-C[r], T[i], A[j]);
        if (row_exit && u_hi < 0.0) break; /* this peak and the rest of its FFT left of the grid */
        double b_lo = floor(u_lo);
        double b_hi = floor(u_hi);
        if (b_lo < 0.0) b_lo = 0.0;
        if (b_hi > (double)(n_x0 - 1)) b_hi = (double)(n_x0 - 1);
        if (b_lo <= b_hi) {
          ++prs;
          tot += (int64_t)(b_hi - b_lo) + 1;
          if (h)
            for (double b = b_lo; b <= b_hi; b += 1.0) h[(int64_t)b] += 1;
        }
      }
    }
    totals[q] = tot;
    if (pairs_out) pairs_out[q] = prs;
  }
  free(A); free(C); free(T);
  return ORC_OK;
}

/* Per-pair clipped interval [b_lo, b_hi] of one (row, peak); returns its width
 * (0 if the image misses the grid).  Exposed for the tests' brute-force pins. */
int orc_pair_interval(const orc_desc* d, int32_t r, int32_t i, int32_t j, int32_t* b_lo_out, int32_t* b_hi_out) {
  int n_f, n_x0;
  double x0_min, dx0;
  if (orc_resolve(d, &n_f, &x0_min, &dx0, &n_x0) != ORC_OK) return -1;
  double df = 1.0 / d->tfft, inv = 1.0 / dx0;
  double a_lo = (pow(d->f_min + (double)(j + 1) * df, 1.0 - d->n) - x0_min) * inv;
  double a_hi = (pow(d->f_min + (double)j * df, 1.0 - d->n) - x0_min) * inv;
  double c = ((d->n - 1.0) * d->k[r]) * inv;
  double t = d->t ? d->t[i] : ((double)i + 0.5) * d->tfft;
  double b_lo = floor(fma(-c, t, a_lo));
  double b_hi = floor(fma(-c, t, a_hi));
  if (b_lo < 0.0) b_lo = 0.0;
  if (b_hi > (double)(n_x0 - 1)) b_hi = (double)(n_x0 - 1);
  *b_lo_out = (int32_t)(b_lo > 2e9 ? 2e9 : b_lo);
  *b_hi_out = (int32_t)(b_hi < -2e9 ? -2e9 : b_hi);
  return b_hi >= b_lo ? (int)(b_hi - b_lo + 1.0) : 0;
}

/* Threads the row loop of orc_hough_rows runs on (1 without OpenMP). */
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
