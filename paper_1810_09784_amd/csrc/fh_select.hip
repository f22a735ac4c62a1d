// Candidate selection on a Hough map (Sec. IV of the paper: squares over the
// (x0, k) plane, the best cell of each square and a second one a few k rows
// away, scored by the critical ratio CR = (y - mu) / sigma).
//
// The device reads the map once: one work-group per map row produces, for
// every column segment of the square grid, the exact int64 sum and sum of
// squares of the counts and the row's best cell (largest count, then
// smallest column).  The host adds the rows of each square, applies the
// row-major tie rule across rows and evaluates mu, sigma and CR in binary64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fh_internal.h"

namespace fh {

constexpr int kSelThreads = 256;

template <typename T>
using gsel = __attribute__((address_space(1))) T*;

__device__ __forceinline__ long long wave_sum_i64(long long x) {
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long y = __shfl_xor(x, o);
    x = y > x ? y : x;
  }
  return x;
}

// out[(r * sq_x0 + b) * 3 + {0, 1, 2}] = Sy, Sy2, (count << 32 | ~column)
__global__ void __launch_bounds__(kSelThreads) k_select_rows(const int32_t* map_, int n_x0, int col_lo, int col_hi,
                                                              int sq_x0, unsigned long long* out_) {
  const gsel<const int32_t> map = (gsel<const int32_t>)map_;
  const gsel<unsigned long long> out = (gsel<unsigned long long>)out_;
  __shared__ long long s_sy[kSelThreads / 64], s_sy2[kSelThreads / 64];
  __shared__ unsigned long long s_mx[kSelThreads / 64];
  const int r = blockIdx.x;
  const int W = col_hi - col_lo;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const gsel<const int32_t> row = map + (size_t)r * n_x0;
  for (int b = 0; b < sq_x0; ++b) {
    const int s0 = col_lo + (int)((long long)b * W / sq_x0);
    const int s1 = col_lo + (int)((long long)(b + 1) * W / sq_x0);
    long long sy = 0, sy2 = 0;
    unsigned long long mx = 0;
    for (int c = s0 + threadIdx.x; c < s1; c += kSelThreads) {
      const int y = row[c];
      sy += y;
      sy2 += (long long)y * y;
      const unsigned long long key = ((unsigned long long)(unsigned)y << 32) | (unsigned)(~(unsigned)c);
      mx = key > mx ? key : mx;
    }
    sy = wave_sum_i64(sy);
    sy2 = wave_sum_i64(sy2);
    mx = wave_max_u64(mx);
    if (lane == 0) {
      s_sy[wave] = sy;
      s_sy2[wave] = sy2;
      s_mx[wave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      long long a = 0, q = 0;
      unsigned long long m = 0;
      for (int w = 0; w < kSelThreads / 64; ++w) {
        a += s_sy[w];
        q += s_sy2[w];
        m = s_mx[w] > m ? s_mx[w] : m;
      }
      const size_t o = ((size_t)r * sq_x0 + b) * 3;
      out[o] = (unsigned long long)a;
      out[o + 1] = (unsigned long long)q;
      out[o + 2] = m;
    }
    __syncthreads();
  }
}

}  // namespace fh

using namespace fh;

extern "C" fh_status fh_select(fh_plan_t h, const int32_t* map, const fh_select_opts* o, fh_candidate* out, int32_t cap,
                               int32_t* n_out, void* stream) {
  if (!h || !map || !o || !n_out || cap < 0 || (cap > 0 && !out)) return FH_EINVAL;
  Plan& p = reinterpret_cast<Plan&>(*h);
  const int n_k = p.desc.n_k;
  const int col_lo = o->col_lo;
  const int col_hi = o->col_hi > 0 ? o->col_hi : p.n_x0;
  if (col_lo < 0 || col_hi > p.n_x0 || col_hi <= col_lo) return FH_EINVAL;
  const int W = col_hi - col_lo;
  if (o->sq_k < 1 || o->sq_k > n_k || o->sq_x0 < 1 || o->sq_x0 > std::min(W, kMaxSelectSegments)) return FH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int sq_x0 = o->sq_x0;
  hipLaunchKernelGGL(k_select_rows, dim3(n_k), dim3(kSelThreads), 0, s, map, p.n_x0, col_lo, col_hi, sq_x0,
                     (unsigned long long*)p.dSel);
  if (hipGetLastError() != hipSuccess) return FH_EDEVICE;
  std::vector<unsigned long long> rows((size_t)n_k * sq_x0 * 3);
  if (hipMemcpyAsync(rows.data(), p.dSel, rows.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FH_EDEVICE;
  int32_t total = 0;
  const double inv1n = 1.0 / (1.0 - p.desc.n);
  auto emit = [&](int r, int c, int y, int sq, int second, double mu, double sigma) {
    const double cr = ((double)y - mu) / sigma;
    if (!(cr >= o->cr_thr)) return;
    if (total < cap) {
      fh_candidate& e = out[total];
      std::memset(&e, 0, sizeof(e));
      e.row = r;
      e.col = c;
      e.count = y;
      e.square = sq;
      e.second = second;
      e.cr = cr;
      e.mu = mu;
      e.sigma = sigma;
      e.x0 = p.x0_min + ((double)c + 0.5) * p.dx0;
      e.k = p.K[r];
      e.f0 = std::pow(e.x0, inv1n);
      e.fdot0 = -e.k * std::pow(e.f0, p.desc.n);
    }
    ++total;
  };
  for (int a = 0; a < o->sq_k; ++a) {
    const int r0 = (int)((long long)a * n_k / o->sq_k), r1 = (int)((long long)(a + 1) * n_k / o->sq_k);
    for (int b = 0; b < sq_x0; ++b) {
      const int s0 = col_lo + (int)((long long)b * W / sq_x0), s1 = col_lo + (int)((long long)(b + 1) * W / sq_x0);
      const long long N = (long long)(r1 - r0) * (s1 - s0);
      if (N <= 0) continue;
      long long Sy = 0, Sy2 = 0;
      int best_r = -1, best_y = -1, best_c = -1;
      for (int r = r0; r < r1; ++r) {
        const unsigned long long* e = &rows[((size_t)r * sq_x0 + b) * 3];
        Sy += (long long)e[0];
        Sy2 += (long long)e[1];
        const int y = (int)(e[2] >> 32);
        if (y > best_y) {  // strictly greater: the smallest row wins ties
          best_y = y;
          best_r = r;
          best_c = (int)(~(unsigned)(e[2] & 0xffffffffu));
        }
      }
      const double mu = (double)Sy / (double)N;
      const double ex2 = (double)Sy2 / (double)N;
      const double var = ex2 - mu * mu;
      const double sigma = std::sqrt(var);
      if (!(sigma > 0.0)) continue;
      const int sq = a * sq_x0 + b;
      emit(best_r, best_c, best_y, sq, 0, mu, sigma);
      if (o->min_dk >= 1) {
        int r2 = -1, y2 = -1, c2 = -1;
        for (int r = r0; r < r1; ++r) {
          if (std::abs(r - best_r) < o->min_dk) continue;
          const unsigned long long* e = &rows[((size_t)r * sq_x0 + b) * 3];
          const int y = (int)(e[2] >> 32);
          if (y > y2) {
            y2 = y;
            r2 = r;
            c2 = (int)(~(unsigned)(e[2] & 0xffffffffu));
          }
        }
        if (r2 >= 0) emit(r2, c2, y2, sq, 1, mu, sigma);
      }
    }
  }
  *n_out = total;
  return FH_OK;
}
