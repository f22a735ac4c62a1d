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

int lds_bytes_for_shape(int n_f, int rows, int cols, int a_lds, int threads, int* pitch_out, int wave_scratch) {
  int pitch = round_up(cols + 1, 4);
  if (pitch_out) *pitch_out = pitch;
  // [A][C rows][per-wave scratch][ia, ib rows][16 + 4 ints][64 discard ints][D rows x pitch, 16-aligned]
  long long b = (long long)rows * pitch * 4 + (long long)rows * 8 +
                (long long)(wave_scratch ? threads / 64 : 0) * kWaveScratchBytes + (long long)rows * 8 + 80 + 256 + 16;
  if (a_lds) b += (long long)(n_f + 2) * 8;
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
  // a single map's launch compiles only its own mode's pair loop
  const int wsc = tile.mode != kModeWindowed;
  a.a_lds = (lds_bytes_for_shape(n_f, tile.rows, tile.cols, 1, tile.threads, nullptr, wsc) <= kLdsBudget) ? 1 : 0;
  a.lds_bytes = lds_bytes_for_shape(n_f, tile.rows, tile.cols, a.a_lds, tile.threads, &a.pitch, wsc);
  return a;
}

int64_t Plan::n_tiles() const {
  int64_t tx = (n_x0 + tile.cols - 1) / tile.cols;
  int64_t ty = (desc.n_k + tile.rows - 1) / tile.rows;
  return tx * ty;
}

// Automatic tile shape (the autotuner may override it through fh_tile_cfg).
static fh_tile_cfg auto_tile(const Plan& p) {
  fh_tile_cfg c{};
  const int nk = p.desc.n_k;
  c.tsplit = 64;
  if (p.n_x0 <= 6144 || p.n_J == 0) {
    c.mode = kModeWhole;
    c.threads = 512;
    c.cols = std::min(p.n_x0, 8192);
    int pitch = round_up(c.cols + 1, 4);
    // about 28 KB of differential tile: three 512-thread work-groups share a CU
    // (40 KB allowed two; the batched maps run 20% faster this way)
    int rows = (28 * 1024) / (pitch * 4);
    rows = std::max(1, std::min(rows, kMaxRowsPerTile));
    while (rows & (rows - 1)) rows &= rows - 1;  // power of two
    c.rows = std::min(rows, nk);
  } else {
    c.mode = kModeWindowed;
    c.threads = 1024;
    c.rows = 1;
    // widest tile that leaves room for the A table in LDS
    int cols = 32768;
    while (cols > 1024 && lds_bytes_for_shape(p.n_f, 1, cols, 1, c.threads, nullptr) > kLdsBudget) cols -= 1024;
    int ntx = (p.n_x0 + cols - 1) / cols;
    c.cols = (p.n_x0 + ntx - 1) / ntx;
  }
  return c;
}

// FFT range [ia, ib) that can bring the band's image onto columns [c0, c1)
// at row shift C per second (host twin of the kernel's range, for costs).
static void host_fft_range(const Plan& p, double C, int c0, int c1, int* ia, int* ib) {
  const int nf = p.desc.n_fft;
  const double hi_s = p.A[0] - (double)c0 + 1.0;
  const double lo_s = p.A[p.n_f] - (double)c1 - 1.0;
  if (C == 0.0) {
    const bool ok = lo_s <= 0.0 && 0.0 <= hi_s;
    *ia = 0;
    *ib = ok ? nf : 0;
    return;
  }
  const double tl = lo_s / C, th = hi_s / C;
  *ia = (int)(std::lower_bound(p.T.begin(), p.T.end(), tl) - p.T.begin());
  *ib = (int)(std::upper_bound(p.T.begin(), p.T.end(), th) - p.T.begin());
  if (*ib < *ia) *ib = *ia;
}

// Relative cost model: one unit per (peak, row) pair handled, about 12.5
// peaks per 160 bins of noise peakmap (threshold 2.5), one unit per
// (row, FFT) item of the windowed mode.  In the whole-FFT mode every peak
// read also costs about kChunkPeakCost row steps for its chunk's set-up (its
// FFT, time, A edges and row bound): fitted to per-unit times of 2717 units
// on a 48-map batch, where the old weight of one made the tiles holding row
// k = 0 of long maps (every FFT read, few rows each) 2-3x underestimated.
static constexpr double kPeakDensity = 0.08;
static constexpr double kChunkPeakCost = 4.0;

static void build_profiles(Plan& p) {
  const int tx = (p.n_x0 + p.tile.cols - 1) / p.tile.cols;
  const int ty = (p.desc.n_k + p.tile.rows - 1) / p.tile.rows;
  p.prof.assign((size_t)tx * ty, TileProfile());
  p.total_cost = 0;
  std::vector<int> ia(p.tile.rows), ib(p.tile.rows);
  for (int rt = 0; rt < ty; ++rt) {
    const int r0 = rt * p.tile.rows, nrows = std::min(p.tile.rows, p.desc.n_k - r0);
    for (int ct = 0; ct < tx; ++ct) {
      const int c0 = ct * p.tile.cols, c1 = std::min(c0 + p.tile.cols, p.n_x0);
      TileProfile& pr = p.prof[(size_t)rt * tx + ct];
      int lo = p.desc.n_fft, hi = 0;
      for (int r = 0; r < nrows; ++r) {
        host_fft_range(p, p.C[r0 + r], c0, c1, &ia[r], &ib[r]);
        if (ia[r] < ib[r]) {
          lo = std::min(lo, ia[r]);
          hi = std::max(hi, ib[r]);
        }
      }
      if (p.tile.mode == kModeWhole && rt == 0 && ct == 0) {  // this tile also counts bad peaks
        lo = 0;
        hi = p.desc.n_fft;
      }
      if (hi < lo) hi = lo;
      pr.lo = lo;
      pr.hi = hi;
      pr.cum[0] = 0;
      for (int q = 0; q < kProfileSamples; ++q) {
        const int a = lo + (int)((int64_t)(hi - lo) * q / kProfileSamples);
        const int b = lo + (int)((int64_t)(hi - lo) * (q + 1) / kProfileSamples);
        double c = 0;
        if (b > a) {
          const int i = (a + b) / 2;
          if (p.tile.mode == kModeWhole) {
            int act = 0;
            for (int r = 0; r < nrows; ++r) act += (ia[r] <= i && i < ib[r]);
            c = kPeakDensity * p.n_f * (act + kChunkPeakCost);
          } else {
            for (int r = 0; r < nrows; ++r) {
              if (!(ia[r] <= i && i < ib[r])) continue;
              const double sh = p.C[r0 + r] * p.T[i];
              const double y0 = c0 + sh - 1.0, y1 = c1 + sh + 1.0;
              int jb = y0 < 0 ? p.n_f - 1 : (y0 >= p.n_J - 1 ? -1 : std::min(p.J[(int)y0], p.n_f - 1));
              int ja = y1 <= 0 ? 0 : (y1 >= p.n_J - 1 ? p.J[p.n_J - 1] : p.J[(int)std::ceil(y1)]);
              ja = std::max(ja, 0);
              c += 1.0 + kPeakDensity * std::max(0, jb - ja + 1);
            }
          }
          c *= (double)(b - a);
        }
        pr.cum[q + 1] = pr.cum[q] + (float)c;
      }
      p.total_cost += pr.cum[kProfileSamples];
    }
  }
}

void split_units(const Plan& p, int32_t mi, double target, std::vector<Unit>& units, std::vector<double>& cost,
                 std::vector<int4>& clears) {
  const int tx = (p.n_x0 + p.tile.cols - 1) / p.tile.cols;
  const int ty = (p.desc.n_k + p.tile.rows - 1) / p.tile.rows;
  for (int t = 0; t < tx * ty; ++t) {
    const TileProfile& pr = p.prof[t];
    const int rt = t / tx, ct = t % tx;
    const int nrows = std::min(p.tile.rows, p.desc.n_k - rt * p.tile.rows);
    const int W = std::min(p.tile.cols, p.n_x0 - ct * p.tile.cols);
    const double work = pr.cum[kProfileSamples];
    int pieces = (int)std::min<double>(p.tile.tsplit, std::max(1.0, std::floor(work / std::max(target, 1.0) + 0.5)));
    pieces = std::max(1, std::min(pieces, std::max(1, pr.hi - pr.lo)));
    const double store = 0.5 * nrows * W * (pieces > 1 ? 3.0 : 1.0);
    if (pieces == 1) {
      units.push_back(make_int4(mi, t, pr.lo, pr.hi));
      cost.push_back(work + store);
      continue;
    }
    clears.push_back(make_int4(mi, t, 0, 0));
    int prev = pr.lo;
    int q = 0;
    for (int k = 1; k <= pieces; ++k) {
      int cut;
      if (k == pieces) {
        cut = pr.hi;
      } else {
        const double want = work * k / pieces;
        while (q < kProfileSamples && pr.cum[q + 1] < want) ++q;
        const double seg = pr.cum[q + 1] - pr.cum[q];
        const double fr = seg > 0 ? (want - pr.cum[q]) / seg : 0.0;
        const int a = pr.lo + (int)((int64_t)(pr.hi - pr.lo) * q / kProfileSamples);
        const int b = pr.lo + (int)((int64_t)(pr.hi - pr.lo) * (q + 1) / kProfileSamples);
        cut = std::max(prev, std::min(pr.hi, a + (int)((b - a) * fr)));
      }
      if (cut > prev) {
        units.push_back(make_int4(mi | kUnitAtomic, t, prev, cut));
        cost.push_back(work / pieces + store / pieces);
      }
      prev = cut;
    }
  }
}

static fh_status validate_tile(const Plan& p, fh_tile_cfg* c) {
  if (c->mode != kModeWhole && c->mode != kModeWindowed) return FH_EINVAL;
  if (c->mode == kModeWindowed && p.n_J == 0) return FH_EINVAL;
  if (c->threads != 256 && c->threads != 512 && c->threads != 1024) return FH_EINVAL;
  if (c->rows < 1 || c->rows > kMaxRowsPerTile) return FH_EINVAL;
  if (c->cols < 1) return FH_EINVAL;
  if (c->cols > p.n_x0) c->cols = p.n_x0;
  if (c->rows > p.desc.n_k) c->rows = p.desc.n_k;
  if (c->tsplit < 1 || c->tsplit > 1024) return FH_EINVAL;
  if (lds_bytes_for_shape(p.n_f, c->rows, c->cols, 0, c->threads, nullptr) > kLdsBudget) return FH_ERANGE;
  return FH_OK;
}

static void free_dev(Plan& p) {
  if (p.sel_pending && p.ev_sel) (void)hipEventSynchronize(p.ev_sel);  // its copy still targets hSq
  if (p.dA) (void)hipFree(p.dA);
  if (p.dC) (void)hipFree(p.dC);
  if (p.dT) (void)hipFree(p.dT);
  if (p.dJ) (void)hipFree(p.dJ);
  if (p.dRank) (void)hipFree(p.dRank);
  if (p.dErr) (void)hipFree(p.dErr);
  if (p.dUnits) (void)hipFree(p.dUnits);
  if (p.dClears) (void)hipFree(p.dClears);
  if (p.dHead) (void)hipFree(p.dHead);
  if (p.dSel) (void)hipFree(p.dSel);
  p.dSel = nullptr;
  p.sel_words = 0;
  if (p.dProj) (void)hipFree(p.dProj);
  p.dProj = nullptr;
  p.proj_words = 0;
  if (p.hSq) (void)hipHostFree(p.hSq);
  p.hSq = nullptr;
  p.hsq_words = 0;
  if (p.ev_sel) (void)hipEventDestroy(p.ev_sel);
  p.ev_sel = nullptr;
  p.dUnits = nullptr;
  p.dClears = nullptr;
  p.dHead = nullptr;
  p.dA = p.dC = p.dT = nullptr;
  p.dJ = nullptr;
  p.dRank = nullptr;
  p.dErr = nullptr;
}

static void debug_report(const char* what, hipError_t e) {
  if (std::getenv("FH_DEBUG")) std::fprintf(stderr, "fh: %s failed: %s\n", what, hipGetErrorString(e));
}

fh_status device_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (std::getenv("FH_FAKE_OOM")) return FH_ENOMEM;
  const hipError_t e = hipMalloc(p, bytes ? bytes : 1);
  if (e != hipSuccess) {
    debug_report("hipMalloc", e);
    *p = nullptr;
    return e == hipErrorOutOfMemory ? FH_ENOMEM : FH_EDEVICE;
  }
  return FH_OK;
}

bool fake_device_error(const char* what) {
  const char* e = std::getenv("FH_FAKE_DEVICE_ERROR");
  return e && std::strcmp(e, what) == 0;
}

fh_status check_peaks(const fh_peaks* pk) {
  if (!pk || !pk->row_ptr) return FH_EINVAL;
  if (pk->n_peaks < 0 || pk->n_peaks >= (1LL << 31)) return FH_EINVAL;
  if (pk->n_peaks > 0 && !pk->bin) return FH_EINVAL;
  if ((reinterpret_cast<uintptr_t>(pk->bin) & 15) != 0) return FH_EINVAL;
  return FH_OK;
}

template <typename T>
static fh_status upload(T** dst, const T* src, size_t n) {
  if (n == 0) n = 1;
  void* v = nullptr;
  const fh_status st = device_alloc(&v, n * sizeof(T));
  *dst = static_cast<T*>(v);
  if (st != FH_OK) return st;
  if (src) {
    const hipError_t e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
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
    p.K.assign(d->k, d->k + d->n_k);
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
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p.device) == hipSuccess && cus > 0)
      p.n_cu = cus;
  }
  build_profiles(p);
  {
    int pitch;
    const int wsc = c.mode != kModeWindowed;
    const int a_lds = lds_bytes_for_shape(n_f, c.rows, c.cols, 1, c.threads, nullptr, wsc) <= kLdsBudget;
    const int lds = lds_bytes_for_shape(n_f, c.rows, c.cols, a_lds, c.threads, &pitch, wsc);
    const int resident = occupancy_grid(c.threads, lds, 1 << 30, c.mode);
    split_units(p, 0, p.total_cost / (4.0 * std::max(resident, 1)), p.units, p.unit_cost, p.clears);
    // longest first
    std::vector<size_t> order(p.units.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return p.unit_cost[x] > p.unit_cost[y]; });
    std::vector<Unit> u(order.size());
    std::vector<double> uc(order.size());
    for (size_t i = 0; i < order.size(); ++i) {
      u[i] = p.units[order[i]];
      uc[i] = p.unit_cost[order[i]];
    }
    p.units.swap(u);
    p.unit_cost.swap(uc);
    p.grid = std::max(1, std::min<int>(resident, (int)p.units.size()));
  }
  {
    // device A: the n_f + 1 bin edges and a pad entry +huge, read for a bad bin
    // (its interval is then empty)
    std::vector<double> a_pad(p.A);
    a_pad.push_back(1e300);
    st = upload(&p.dA, a_pad.data(), a_pad.size());
  }
  if (st == FH_OK) {
    // the row loop of the whole-FFT tiles reads C eight rows at a time
    std::vector<double> c_pad(p.C);
    c_pad.resize(p.C.size() + kCPad, 0.0);
    st = upload(&p.dC, c_pad.data(), c_pad.size());
  }
  if (st == FH_OK) st = upload(&p.dT, p.T.data(), p.T.size());
  if (st == FH_OK && p.n_J > 0) st = upload(&p.dJ, p.J.data(), p.J.size());
  if (st == FH_OK && c.mode == kModeWindowed)
    st = upload<uint2>(&p.dRank, nullptr, (size_t)d->n_fft * (size_t)p.n_words);
  if (st == FH_OK) st = upload<unsigned long long>(&p.dErr, nullptr, 1);
  if (st == FH_OK) st = upload<Unit>(&p.dUnits, p.units.data(), p.units.size());
  if (st == FH_OK) st = upload<int4>(&p.dClears, p.clears.data(), p.clears.size());
  if (st == FH_OK) st = upload<int32_t>(&p.dHead, nullptr, 1);
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

extern "C" fh_status fh_peaks_validate(const fh_peaks* pk) { return check_peaks(pk); }

extern "C" fh_status fh_hough(fh_plan_t h, const fh_peaks* pk, int32_t* map, void* stream) {
  if (!h || !map || check_peaks(pk) != FH_OK) return FH_EINVAL;
  const Plan& p = reinterpret_cast<Plan&>(*h);
  return launch_hough(p, *pk, map, (hipStream_t)stream);
}

extern "C" fh_status fh_plan_set_events(fh_plan_t h, void* start, void* stop) {
  if (!h || (!start) != (!stop)) return FH_EINVAL;
  Plan& p = reinterpret_cast<Plan&>(*h);
  p.ev_start = (hipEvent_t)start;
  p.ev_stop = (hipEvent_t)stop;
  return FH_OK;
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
