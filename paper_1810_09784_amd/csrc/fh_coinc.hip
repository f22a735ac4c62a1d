// Coincidences of two candidate lists (Sec. IV): all pairs within max_d bins
// in (x0, k), segment by segment.  One thread per point of list a walks the b
// points of its segment; pairs go out through an atomic counter.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fh_internal.h"

namespace fh {

template <typename T>
using gco = __attribute__((address_space(1))) T*;

constexpr int kCoincThreads = 256;

__global__ void k_coinc_zero(int32_t* count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *(gco<int32_t>)count = 0;
}

// Grid over the points of a; each thread finds its segment by binary search
// over a_off (segments are contiguous in a).  A thread counts its pairs in a
// first pass; a wave prefix sum of the counts and one atomic per wave
// reserve the wave's output slots, and a second pass writes the pairs there.
// (One atomic per pair serialised on the counter: a list matched against
// itself has a pair for every point.)
__device__ __forceinline__ int wave_prefix(int x) {  // inclusive, over the 64 lanes
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

__global__ void __launch_bounds__(kCoincThreads)
    k_coinc(int n_seg, int na, const int32_t* a_off_, const fh_point* a_, int nb, const int32_t* b_off_,
            const fh_point* b_, const double* nm1_, const double* dt_, double max_d, int32_t* pairs_, double* dist_,
            int cap, int32_t* count_) {
  static_assert(kCoincThreads % 64 == 0, "whole wavefronts");
  const gco<const int32_t> a_off = (gco<const int32_t>)a_off_;
  const gco<const int32_t> b_off = (gco<const int32_t>)b_off_;
  const gco<const fh_point> a = (gco<const fh_point>)a_;
  const gco<const fh_point> b = (gco<const fh_point>)b_;
  const int ia = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const bool act = ia < na;  // every lane stays for the wave prefix sum
  int b0 = 0, b1 = 0;
  double pk = 0.0, pdx = 1.0, pdk = 1.0, xa = 0.0;
  if (act) {
    int lo = 0, hi = n_seg;  // last segment s with a_off[s] <= ia
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a_off[mid] <= ia) lo = mid; else hi = mid;
    }
    const int s = lo;
    pk = a[ia].k;
    pdx = a[ia].dx0;
    pdk = a[ia].dk;
    xa = a[ia].x0;
    if (nm1_ && dt_) {
      const double m = ((gco<const double>)nm1_)[s];
      const double t = ((gco<const double>)dt_)[s];
      xa = xa + (m * pk) * t;
    }
    b0 = max(b_off[s], 0);
    b1 = min(b_off[s + 1], nb);
  }
  auto dist = [&](int ib) {
    const double dx = (pdx + b[ib].dx0) * 0.5;
    const double dk = (pdk + b[ib].dk) * 0.5;
    const double u = (b[ib].x0 - xa) / dx;
    const double v = (b[ib].k - pk) / dk;
    return sqrt(u * u + v * v);
  };
  int n = 0;
  for (int ib = b0; ib < b1; ++ib) n += dist(ib) <= max_d;
  const int incl = wave_prefix(n);
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == 63) base = atomicAdd(count_, incl);  // the wave's total
  base = __shfl(base, 63, 64);
  int slot = base + incl - n;
  if (n == 0 || slot >= cap) return;
  for (int ib = b0; ib < b1 && slot < cap; ++ib) {
    const double d = dist(ib);
    if (d <= max_d) {
      ((gco<int32_t>)pairs_)[2 * (size_t)slot] = ia;
      ((gco<int32_t>)pairs_)[2 * (size_t)slot + 1] = ib;
      if (dist_) ((gco<double>)dist_)[slot] = d;
      ++slot;
    }
  }
}

}  // namespace fh

using namespace fh;

extern "C" fh_status fh_coincide(int32_t n_seg, int32_t na, const int32_t* a_off, const fh_point* a, int32_t nb,
                                 const int32_t* b_off, const fh_point* b, const double* nm1, const double* dt,
                                 double max_d, int32_t* pairs, double* dist, int32_t cap, int32_t* count,
                                 void* stream) {
  if (n_seg < 0 || na < 0 || nb < 0 || cap < 0 || !count || !std::isfinite(max_d) || max_d < 0.0) return FH_EINVAL;
  if (n_seg > 0 && (!a_off || !b_off)) return FH_EINVAL;
  if ((na > 0 && !a) || (nb > 0 && !b) || (cap > 0 && !pairs)) return FH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_coinc_zero, dim3(1), dim3(64), 0, s, count);
  if (hipGetLastError() != hipSuccess) return FH_EDEVICE;
  if (n_seg == 0 || na == 0) return FH_OK;
  const unsigned grid = (unsigned)((na + kCoincThreads - 1) / kCoincThreads);
  hipLaunchKernelGGL(k_coinc, dim3(grid), dim3(kCoincThreads), 0, s, n_seg, na, a_off, a, nb, b_off, b, nm1, dt,
                     max_d, pairs, dist, cap, count);
  return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE;
}
