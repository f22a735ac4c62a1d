/*
 * sanitize_check.c -- runs the C oracle (fh_oracle.c, included) on small
 * seeded maps so that it can be built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py builds it with
 * gcc -fsanitize=address,undefined and runs it).  TEST INFRASTRUCTURE ONLY.
 *
 * Exercises every entry point of the oracle: the grid and tables, the direct
 * map with bad bins and explicit times, the row checker (whose rows must equal
 * the direct map's), the single-pair interval, and the n = 0 special case.
 * Exit status 0 when every comparison holds.
 */
#include "fh_oracle.c"

#include <stdio.h>

static uint64_t lcg = 0x9e3779b97f4a7c15ull;
static uint32_t next_u32(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(lcg >> 33);
}
static double next_unit(void) { return (double)next_u32() / 4294967296.0; }

static int run_case(double n, double tfft, double f_min, int n_f, int n_fft, int n_k, double k_max, int explicit_t) {
  const double f_max = f_min + n_f / tfft;
  double* k = malloc(sizeof(double) * (size_t)n_k);
  double* t = malloc(sizeof(double) * (size_t)n_fft);
  int32_t* row_ptr = malloc(sizeof(int32_t) * (size_t)(n_fft + 1));
  int32_t* bin = malloc(sizeof(int32_t) * (size_t)(n_fft * (n_f + 2)));
  for (int r = 0; r < n_k; ++r) k[r] = k_max * r / (n_k > 1 ? n_k - 1 : 1);
  double acc = 0;
  for (int i = 0; i < n_fft; ++i) {
    acc += 0.5 + 2.0 * next_unit();
    t[i] = acc;
  }
  int p = 0;
  row_ptr[0] = 0;
  for (int i = 0; i < n_fft; ++i) {
    if (i % 7 == 3) bin[p++] = -2; /* below the band */
    for (int j = 0; j < n_f; ++j)
      if (next_unit() < 0.15) bin[p++] = j;
    if (i % 11 == 5) bin[p++] = n_f + 4; /* above the band */
    row_ptr[i + 1] = p;
  }
  orc_desc d = {n, tfft, f_min, f_max, n_fft, explicit_t ? t : NULL, n_k, k, 0.0, 0.0, 0};
  int nf, nx;
  double x0m, dx;
  if (orc_resolve(&d, &nf, &x0m, &dx, &nx) != ORC_OK) return 1;
  int32_t* map = malloc(sizeof(int32_t) * (size_t)n_k * (size_t)nx);
  int32_t* map2 = malloc(sizeof(int32_t) * (size_t)n_k * (size_t)nx);
  int32_t* rows = malloc(sizeof(int32_t) * (size_t)n_k);
  int64_t* tot = malloc(sizeof(int64_t) * (size_t)n_k);
  int64_t* prs = malloc(sizeof(int64_t) * (size_t)n_k);
  int64_t bad = 0, pairs = 0;
  int fail = 0;
  for (int r = 0; r < n_k; ++r) rows[r] = n_k - 1 - r;
  if (orc_hough_rows_pairs(&d, row_ptr, bin, NULL, 0, map, &bad, &pairs) != ORC_OK) fail = 1;
  if (orc_rows_checked(&d, row_ptr, bin, rows, n_k, map2, tot, prs) != ORC_OK) fail = 1;
  int64_t all_pairs = 0;
  for (int q = 0; q < n_k && !fail; ++q) {
    int64_t s = 0;
    for (int b = 0; b < nx; ++b) {
      if (map2[(size_t)q * nx + b] != map[(size_t)rows[q] * nx + b]) fail = 1;
      s += map[(size_t)rows[q] * nx + b];
    }
    if (s != tot[q]) fail = 1;
    all_pairs += prs[q];
  }
  if (all_pairs != pairs) fail = 1;
  /* single pairs against the map's row 0 coverage of the first FFT's peaks */
  for (int q = row_ptr[0]; q < row_ptr[1] && !fail; ++q) {
    int32_t lo, hi;
    if (bin[q] < 0 || bin[q] >= nf) continue;
    int w = orc_pair_interval(&d, 0, 0, bin[q], &lo, &hi);
    if (w < 0 || (w > 0 && (lo < 0 || hi >= nx || hi - lo + 1 != w))) fail = 1;
  }
  free(k); free(t); free(row_ptr); free(bin); free(map); free(map2); free(rows); free(tot); free(prs);
  return fail;
}

int main(void) {
  int fail = 0;
  fail |= run_case(3.0, 2.0, 100.0, 48, 120, 12, 5e-9, 0);
  fail |= run_case(5.0, 4.0, 500.0, 64, 90, 9, 1e-13, 1);
  fail |= run_case(2.0, 1.0, 900.0, 32, 200, 17, 1e-7, 1);
  /* n = 0, the original FrequencyHough: x = f, an explicit grid descending in x0 */
  {
    double k[4] = {0.0, 0.01, 0.02, 0.03};
    int32_t row_ptr[4] = {0, 2, 3, 5};
    int32_t bin[5] = {1, 5, 2, 0, 7};
    orc_desc d = {0.0, 2.0, 100.0, 104.0, 3, NULL, 4, k, 104.0, -0.5, 10};
    int32_t map[40], map2[40];
    int32_t rows[4] = {0, 1, 2, 3};
    int64_t tot[4], prs[4], bad, pairs;
    fail |= orc_hough_rows_pairs(&d, row_ptr, bin, NULL, 0, map, &bad, &pairs) != ORC_OK;
    fail |= orc_rows_checked(&d, row_ptr, bin, rows, 4, map2, tot, prs) != ORC_OK;
    fail |= memcmp(map, map2, sizeof(map)) != 0;
  }
  printf("oracle sanitizer run: %s\n", fail ? "FAILED" : "ok");
  return fail;
}
