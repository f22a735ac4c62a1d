// Plan: validation of a map description, the host FP64 tables of the
// canonical index arithmetic, the tile shape, and the device workspace.
//
// Tables (Sec. IV, Eq. transform; Sec. VI.C for the x0 grid), each entry one
// binary64 operation at a time, rounded to nearest, no contraction:
//   df = 1/tfft,  A_j = (pow(f_min + j*df, 1-n) - x0_min) * (1/dx0)   j = 0..n_f
//   C_r = ((n-1)*k_r) * (1/dx0),  T_i = t_i or (i + 0.5)*tfft
// The device evaluates u = fma(-C_r, T_i, A_j) from these and nothing else.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "fh_internal.h"

namespace fh {

static bool is_finite(double x) { return std::isfinite(x); }

static int round_up(int x, int m) { return (x + m - 1) / m * m; }

int lds_bytes_for_shape(int n_f, int rows, int cols, int a_lds, int* pitch_out) {
  int pitch = round_up(cols + 1, 4);
  if (pitch_out) *pitch_out = pitch;
  long long b = (long long)rows * pitch * 4 + (long long)rows * 8 * 2 + (long long)rows * 4 * 2 + 256;
  if (a_lds) b += (long long)(n_f + 1) * 8;
  return b > (1LL << 30) ? (1 << 30) : (int)b;
}

MapArgs Plan::args(const fh_peaks& pk, int32_t* map) const {
  MapArgs a{};
  a.A = dA;
  a.C = dC;
  a.T = dT;
  a.J = dJ;
  a.rank = dRank;
  a.row_ptr = pk.row_ptr;
  a.bin = pk.bin;
  a.map = map;
  a.err = dErr;
  a.tfft = desc.tfft;
  a.t_uniform = t_uniform;
  a.n_peaks = (int32_t)pk.n_peaks;
  a.n_f = n_f;
  a.n_x0 = n_x0;
  a.n_k = desc.n_k;
  a.n_fft = desc.n_fft;
  a.n_words = n_words;
  a.n_J = n_J;
  a.rows = tile.rows;
  a.cols = tile.cols;
  a.mode = tile.mode;
  a.tiles_x = (n_x0 + tile.cols - 1) / tile.cols;
  a.tiles_y = (desc.n_k + tile.rows - 1) / tile.rows;
  a.tsplit = tile.tsplit;
  a.a_lds = (lds_bytes_for_shape(n_f, tile.rows, tile.cols, 1, nullptr) <= kLdsBudget) ? 1 : 0;
  a.lds_bytes = lds_bytes_for_shape(n_f, tile.rows, tile.cols, a.a_lds, &a.pitch);
  return a;
}

int64_t Plan::n_tiles() const {
  int64_t tx = (n_x0 + tile.cols - 1) / tile.cols;
  int64_t ty = (desc.n_k + tile.rows - 1) / tile.rows;
  return tx * ty * tile.tsplit;
}

// Automatic tile shape (the autotuner may override it through fh_tile_cfg).
static fh_tile_cfg auto_tile(const Plan& p) {
  fh_tile_cfg c{};
  const int nk = p.desc.n_k;
  if (p.n_x0 <= 6144 || p.n_J == 0) {
    c.mode = kModeWhole;
    c.threads = 256;
    c.cols = std::min(p.n_x0, 8192);
    int pitch = round_up(c.cols + 1, 4);
    int rows = (32 * 1024) / (pitch * 4);
    rows = std::max(1, std::min(rows, kMaxRowsPerTile));
    while (rows & (rows - 1)) rows &= rows - 1;  // power of two
    rows = std::min(rows, nk);
    // enough tiles to fill the chip: shrink the band, then split time
    int64_t tx = (p.n_x0 + c.cols - 1) / c.cols;
    while (rows > 4 && tx * ((nk + rows - 1) / rows) < 512) rows /= 2;
    c.rows = rows;
    int64_t tiles = tx * ((nk + rows - 1) / rows);
    int ts = 1;
    while (tiles * ts < 512 && ts < 64 && (int64_t)p.desc.n_fft / (ts * 2) >= 64) ts *= 2;
    c.tsplit = ts;
  } else {
    c.mode = kModeWindowed;
    c.threads = 512;
    c.rows = 1;
    c.cols = std::min(p.n_x0, 16384);
    c.tsplit = 1;
  }
  return c;
}

static fh_status validate_tile(const Plan& p, fh_tile_cfg* c) {
  if (c->mode != kModeWhole && c->mode != kModeWindowed) return FH_EINVAL;
  if (c->mode == kModeWindowed && p.n_J == 0) return FH_EINVAL;
  if (c->threads != 256 && c->threads != 512) return FH_EINVAL;
  if (c->rows < 1 || c->rows > kMaxRowsPerTile) return FH_EINVAL;
  if (c->cols < 1) return FH_EINVAL;
  if (c->cols > p.n_x0) c->cols = p.n_x0;
  if (c->rows > p.desc.n_k) c->rows = p.desc.n_k;
  if (c->tsplit < 1 || c->tsplit > p.desc.n_fft) return FH_EINVAL;
  if (lds_bytes_for_shape(p.n_f, c->rows, c->cols, 0, nullptr) > kLdsBudget) return FH_ERANGE;
  return FH_OK;
}

static void free_dev(Plan& p) {
  if (p.dA) (void)hipFree(p.dA);
  if (p.dC) (void)hipFree(p.dC);
  if (p.dT) (void)hipFree(p.dT);
  if (p.dJ) (void)hipFree(p.dJ);
  if (p.dRank) (void)hipFree(p.dRank);
  if (p.dErr) (void)hipFree(p.dErr);
  p.dA = p.dC = p.dT = nullptr;
  p.dJ = nullptr;
  p.dRank = nullptr;
  p.dErr = nullptr;
}

static void debug_report(const char* what, hipError_t e) {
  if (std::getenv("FH_DEBUG")) std::fprintf(stderr, "fh: %s failed: %s\n", what, hipGetErrorString(e));
}

template <typename T>
static fh_status upload(T** dst, const T* src, size_t n) {
  if (n == 0) n = 1;
  if (std::getenv("FH_FAKE_OOM")) return FH_ENOMEM;
  hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
  if (e != hipSuccess) {
    debug_report("hipMalloc", e);
    *dst = nullptr;
    return e == hipErrorOutOfMemory ? FH_ENOMEM : FH_EDEVICE;
  }
  if (src) {
    e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      debug_report("hipMemcpy", e);
      return FH_EDEVICE;
    }
  }
  return FH_OK;
}

}  // namespace fh

using namespace fh;

extern "C" fh_status fh_plan(const fh_map_desc* d, const fh_tile_cfg* cfg, fh_plan_t* out) {
  if (!d || !out) return FH_EINVAL;
  const double n = d->n, tfft = d->tfft, f_min = d->f_min, f_max = d->f_max;
  if (!is_finite(n) || !(n > 1.0)) return FH_EINVAL;
  if (!is_finite(tfft) || !(tfft > 0.0)) return FH_EINVAL;
  if (!is_finite(f_min) || !is_finite(f_max) || !(f_min > 0.0) || !(f_max > f_min)) return FH_EINVAL;
  const double w = (f_max - f_min) * tfft;
  const double wr = std::floor(w + 0.5);
  if (!(std::fabs(w - wr) <= 1e-9) || wr < 1.0) return FH_EINVAL;
  if (wr > (double)(1 << 24)) return FH_ERANGE;
  const int n_f = (int)wr;
  if (d->n_fft < 1 || d->n_k < 1 || !d->k) return FH_EINVAL;
  for (int r = 0; r < d->n_k; ++r) {
    if (!is_finite(d->k[r]) || d->k[r] < 0.0) return FH_EINVAL;
    if (r > 0 && d->k[r] < d->k[r - 1]) return FH_EINVAL;
  }
  if (d->t) {
    for (int i = 0; i < d->n_fft; ++i) {
      if (!is_finite(d->t[i])) return FH_EINVAL;
      if (i > 0 && d->t[i] < d->t[i - 1]) return FH_EINVAL;
    }
  }
  const double df = 1.0 / tfft;
  double x0_min, dx0;
  if (d->dx0 != 0.0) {
    if (!is_finite(d->dx0) || !(d->dx0 > 0.0) || !is_finite(d->x0_min)) return FH_EINVAL;
    x0_min = d->x0_min;
    dx0 = d->dx0;
  } else {
    x0_min = std::pow(f_max, 1.0 - n);
    dx0 = ((n - 1.0) * df) * std::pow(f_max, -n);
  }
  if (!is_finite(x0_min) || !is_finite(dx0) || !(dx0 > 0.0)) return FH_EINVAL;
  int64_t n_x0;
  if (d->n_x0 > 0) {
    n_x0 = d->n_x0;
  } else if (d->n_x0 == 0) {
    double nstar = f_max * (std::pow(f_max / f_min, n - 1.0) - 1.0) / ((n - 1.0) * df);
    double c = std::ceil(nstar - 1e-9);
    if (!is_finite(c) || c < 1.0) return FH_EINVAL;
    if (c >= 2147483647.0) return FH_ERANGE;
    n_x0 = (int64_t)c;
  } else {
    return FH_EINVAL;
  }
  if ((int64_t)d->n_k * n_x0 >= (1LL << 31)) return FH_ERANGE;

  Plan* pp = new (std::nothrow) Plan();
  if (!pp) return FH_ENOMEM;
  Plan& p = *pp;
  p.desc = *d;
  p.desc.t = nullptr;
  p.desc.k = nullptr;
  p.t_uniform = d->t ? 0 : 1;
  p.n_f = n_f;
  p.n_x0 = (int32_t)n_x0;
  p.x0_min = x0_min;
  p.dx0 = dx0;
  const double inv = 1.0 / dx0;
  try {
    p.A.resize(n_f + 1);
    p.C.resize(d->n_k);
    p.T.resize(d->n_fft);
  } catch (...) {
    delete pp;
    return FH_ENOMEM;
  }
  for (int j = 0; j <= n_f; ++j) p.A[j] = (std::pow(f_min + (double)j * df, 1.0 - n) - x0_min) * inv;
  for (int r = 0; r < d->n_k; ++r) p.C[r] = ((n - 1.0) * d->k[r]) * inv;
  for (int i = 0; i < d->n_fft; ++i) p.T[i] = d->t ? d->t[i] : ((double)i + 0.5) * tfft;
  for (int j = 0; j <= n_f; ++j)
    if (!is_finite(p.A[j]) || (j > 0 && p.A[j] > p.A[j - 1])) {
      delete pp;
      return FH_EINVAL;
    }
  for (int r = 0; r < d->n_k; ++r)
    if (!is_finite(p.C[r])) {
      delete pp;
      return FH_EINVAL;
    }
  // Column -> bin-edge table of the windowed mode: J[c] = last j with A_j >= c.
  const double a0 = std::max(p.A[0], 0.0);
  if (a0 + 2.0 <= (double)kMaxJTable) {
    p.n_J = (int32_t)std::ceil(a0) + 2;
    p.J.resize(p.n_J);
    int j = n_f;
    for (int c = 0; c < p.n_J; ++c) {
      while (j >= 0 && p.A[j] < (double)c) --j;
      p.J[c] = j;
    }
  }
  p.n_words = (n_f >> 5) + 1;
  fh_tile_cfg c = (cfg && cfg->mode != 0) ? *cfg : auto_tile(p);
  fh_status st = validate_tile(p, &c);
  if (st != FH_OK) {
    delete pp;
    return st;
  }
  p.tile = c;
  (void)hipGetDevice(&p.device);
  st = upload(&p.dA, p.A.data(), p.A.size());
  if (st == FH_OK) st = upload(&p.dC, p.C.data(), p.C.size());
  if (st == FH_OK) st = upload(&p.dT, p.T.data(), p.T.size());
  if (st == FH_OK && p.n_J > 0) st = upload(&p.dJ, p.J.data(), p.J.size());
  if (st == FH_OK && c.mode == kModeWindowed)
    st = upload<uint2>(&p.dRank, nullptr, (size_t)d->n_fft * (size_t)p.n_words);
  if (st == FH_OK) st = upload<unsigned long long>(&p.dErr, nullptr, 1);
  if (st == FH_OK && hipMemset(p.dErr, 0, sizeof(unsigned long long)) != hipSuccess) st = FH_EDEVICE;
  if (st != FH_OK) {
    free_dev(p);
    delete pp;
    return st;
  }
  *out = reinterpret_cast<fh_plan_t>(pp);
  return FH_OK;
}

extern "C" fh_status fh_plan_get_info(fh_plan_t h, fh_plan_info* out) {
  if (!h || !out) return FH_EINVAL;
  const Plan& p = reinterpret_cast<Plan&>(*h);
  out->n_f = p.n_f;
  out->n_x0 = p.n_x0;
  out->n_k = p.desc.n_k;
  out->n_fft = p.desc.n_fft;
  out->x0_min = p.x0_min;
  out->dx0 = p.dx0;
  out->tile = p.tile;
  out->n_tiles = p.n_tiles();
  int64_t ws = (int64_t)(p.A.size() + p.C.size() + p.T.size()) * 8 + (int64_t)p.J.size() * 4 + 8;
  if (p.dRank) ws += (int64_t)p.desc.n_fft * p.n_words * 8;
  out->workspace_bytes = ws;
  return FH_OK;
}

extern "C" fh_status fh_plan_tables(fh_plan_t h, double* A, double* C, double* T) {
  if (!h) return FH_EINVAL;
  const Plan& p = reinterpret_cast<Plan&>(*h);
  if (A) std::memcpy(A, p.A.data(), p.A.size() * 8);
  if (C) std::memcpy(C, p.C.data(), p.C.size() * 8);
  if (T) std::memcpy(T, p.T.data(), p.T.size() * 8);
  return FH_OK;
}

extern "C" void fh_plan_destroy(fh_plan_t h) {
  if (!h) return;
  Plan* p = reinterpret_cast<Plan*>(h);
  free_dev(*p);
  delete p;
}

extern "C" fh_status fh_hough(fh_plan_t h, const fh_peaks* pk, int32_t* map, void* stream) {
  if (!h || !pk || !map || !pk->row_ptr) return FH_EINVAL;
  if (pk->n_peaks < 0 || pk->n_peaks >= (1LL << 31)) return FH_EINVAL;
  if (pk->n_peaks > 0 && !pk->bin) return FH_EINVAL;
  const Plan& p = reinterpret_cast<Plan&>(*h);
  return launch_hough(p, *pk, map, (hipStream_t)stream);
}

extern "C" fh_status fh_device_errors(fh_plan_t h, void* stream, uint64_t* out) {
  if (!h || !out) return FH_EINVAL;
  const Plan& p = reinterpret_cast<Plan&>(*h);
  unsigned long long v = 0;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(&v, p.dErr, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess) return FH_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return FH_EDEVICE;
  *out = v;
  return FH_OK;
}

extern "C" const char* fh_status_str(fh_status s) {
  switch (s) {
    case FH_OK: return "ok";
    case FH_EINVAL: return "invalid argument";
    case FH_ENOMEM: return "out of memory";
    case FH_EDEVICE: return "device error";
    case FH_ERANGE: return "size out of range";
  }
  return "unknown status";
}

extern "C" const char* fh_version(void) { return "fh 0.1 gfx950"; }
