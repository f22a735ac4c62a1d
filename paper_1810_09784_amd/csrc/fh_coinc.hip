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
// over a_off (segments are contiguous in a).
__global__ void __launch_bounds__(kCoincThreads)
    k_coinc(int n_seg, int na, const int32_t* a_off_, const fh_point* a_, int nb, const int32_t* b_off_,
            const fh_point* b_, const double* nm1_, const double* dt_, double max_d, int32_t* pairs_, double* dist_,
            int cap, int32_t* count_) {
  const gco<const int32_t> a_off = (gco<const int32_t>)a_off_;
  const gco<const int32_t> b_off = (gco<const int32_t>)b_off_;
  const gco<const fh_point> a = (gco<const fh_point>)a_;
  const gco<const fh_point> b = (gco<const fh_point>)b_;
  const int ia = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (ia >= na) return;
  int lo = 0, hi = n_seg;  // last segment s with a_off[s] <= ia
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a_off[mid] <= ia) lo = mid; else hi = mid;
  }
  const int s = lo;
  const double pk = a[ia].k, pdx = a[ia].dx0, pdk = a[ia].dk;
  double xa = a[ia].x0;
  if (nm1_ && dt_) {
    const double m = ((gco<const double>)nm1_)[s];
    const double t = ((gco<const double>)dt_)[s];
    xa = xa + (m * pk) * t;
  }
  const int b0 = max(b_off[s], 0), b1 = min(b_off[s + 1], nb);
  for (int ib = b0; ib < b1; ++ib) {
    const double dx = (pdx + b[ib].dx0) * 0.5;
    const double dk = (pdk + b[ib].dk) * 0.5;
    const double u = (b[ib].x0 - xa) / dx;
    const double v = (b[ib].k - pk) / dk;
    const double d = sqrt(u * u + v * v);
    if (d <= max_d) {
      const int slot = atomicAdd(count_, 1);
      if (slot < cap) {
        ((gco<int32_t>)pairs_)[2 * (size_t)slot] = ia;
        ((gco<int32_t>)pairs_)[2 * (size_t)slot + 1] = ib;
        if (dist_) ((gco<double>)dist_)[slot] = d;
      }
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
