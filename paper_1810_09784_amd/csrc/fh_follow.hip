// Follow-up projection (Sec. V on peakmaps): peaks moved by a candidate's
// power-law drift, histogrammed around the candidate's initial bin, and the
// critical ratio of that bin.  Work-groups per candidate split its FFTs;
// threads take FFTs, evaluate the drift once per FFT and add the FFT's moved
// peaks into an LDS histogram, which is added to the candidate's row.
//
// The drift bin b_i = floor((f(T_i) - f_min) tfft) is defined with the host C
// library's pow.  The device's pow may differ from it in the last bits, which
// can only matter where (f(T_i) - f_min) tfft lies within rounding distance of
// an integer.  The kernel flags a candidate when any of its FFTs does; the
// host then evaluates that candidate's drift table with std::pow and the
// candidate is projected again from the table.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <vector>

#include "fh_internal.h"

namespace fh {

template <typename T>
using gfo = __attribute__((address_space(1))) T*;

constexpr int kProjThreads = 256;
constexpr int kProjMaxW = 4096;

// Grid: (candidates, splits); thread t of block y takes FFTs y * threads + t,
// then every splits * threads, and the block adds its LDS histogram into the
// candidate's row of hist (cleared beforehand).
// shift_tab (host-evaluated drift b_i - b_0 of candidate c0, one per FFT):
// when set, the launch covers that one candidate and reads its drift from
// the table; otherwise every candidate evaluates its drift with the device's
// pow and sets flag[c] when some b_i is within rounding distance of a bin edge.
__global__ void __launch_bounds__(kProjThreads)
    k_project(const int32_t* row_ptr_, const int32_t* bin_, int n_peaks, int n_fft, int n_f, const double* T_,
              double n, double tfft, double f_min, const double* f0_, const double* k_, int w, int32_t* hist_,
              int32_t* flag_, const int32_t* shift_tab_, int c0) {
  extern __shared__ int hs[];
  const gfo<const int32_t> row_ptr = (gfo<const int32_t>)row_ptr_;
  const gfo<const int32_t> bin = (gfo<const int32_t>)bin_;
  const gfo<const double> T = (gfo<const double>)T_;
  const gfo<const int32_t> shift_tab = (gfo<const int32_t>)shift_tab_;
  const int c = c0 + (int)blockIdx.x;
  const int nb = 2 * w + 1;
  for (int x = threadIdx.x; x < nb; x += blockDim.x) hs[x] = 0;
  __syncthreads();
  const double f0 = ((gfo<const double>)f0_)[c];
  const double k = ((gfo<const double>)k_)[c];
  const double nm1 = n - 1.0;
  const double a = (k * nm1) * pow(f0, nm1);
  const double e = 1.0 / nm1;
  const double b0 = floor((f0 - f_min) * tfft);
  const int stride = (int)(gridDim.y * blockDim.x);
  bool near_edge = false;
  for (int i = (int)(blockIdx.y * blockDim.x + threadIdx.x); i < n_fft; i += stride) {
    double sh;
    if (shift_tab_) {
      sh = (double)shift_tab[i];
    } else {
      const double f = f0 / pow(1.0 + a * T[i], e);
      const double x = (f - f_min) * tfft;
      const double bi = floor(x);
      // this device pow and the host's agree to a few ulps of f; allow 2^-43 f tfft
      // (about 2^9 ulps) plus rounding of x itself
      const double margin = 0x1p-43 * fabs(f) * tfft + 0x1p-50 * fabs(x) + 0x1p-60;
      near_edge |= (x - bi < margin) || (bi + 1.0 - x < margin);
      // the drift in bins; |bi - b0| is below n_f + 1 whenever it matters
      sh = bi - b0;
    }
    // beyond these bounds no int32 bin can land within w of b0 (and the
    // conversions below stay defined)
    if (!(fabs(sh) < 2147483647.0) || !(fabs(b0) < 8.0e9)) continue;
    const int shift = (int)sh;
    const int lo = min(max(row_ptr[i], 0), n_peaks);
    const int hi = min(max(row_ptr[i + 1], lo), n_peaks);
    // the FFT's bins ascend: binary-search the first one that can land in
    // b0 - w .. b0 + w after the move, then walk until past the window
    const long long key_lo = (long long)shift + (long long)b0 - w, key_hi = key_lo + 2 * w;
    int u = lo, v = hi;
    while (u < v) {
      const int mid = (u + v) >> 1;
      if ((long long)bin[mid] < key_lo) u = mid + 1; else v = mid;
    }
    for (int p = u; p < hi; ++p) {
      const int j = bin[p];
      if ((long long)j > key_hi) break;
      if ((unsigned)j >= (unsigned)n_f) continue;
      const long long d = (long long)j - shift - (long long)b0;  // moved bin relative to b0
      if (d >= -w && d <= w) atomicAdd(&hs[(int)d + w], 1);
    }
  }
  if (near_edge) __hip_atomic_store((gfo<int32_t>)flag_ + c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  gfo<int32_t> out = (gfo<int32_t>)hist_ + (size_t)c * nb;
  for (int x = threadIdx.x; x < nb; x += blockDim.x)
    if (hs[x]) __hip_atomic_fetch_add(out + x, hs[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_project_clear(int32_t* hist, long long n) {
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x)
    ((gfo<int32_t>)hist)[x] = 0;
}

}  // namespace fh

using namespace fh;

extern "C" fh_status fh_project(fh_plan_t h, const fh_peaks* peaks, int32_t n_cand, const double* f0, const double* k,
                                int32_t w, int32_t guard, int32_t* hist, fh_projection* out, void* stream) {
  if (!h || !peaks || n_cand < 0 || w < 1 || w > kProjMaxW || guard < 0 || guard >= w) return FH_EINVAL;
  if (n_cand > 0 && (!f0 || !k || !hist || !out)) return FH_EINVAL;
  Plan& p = reinterpret_cast<Plan&>(*h);
  if (!peaks->row_ptr || peaks->n_peaks < 0 || peaks->n_peaks >= (1LL << 31) || (peaks->n_peaks > 0 && !peaks->bin))
    return FH_EINVAL;
  if (n_cand == 0) return FH_OK;
  hipStream_t s = (hipStream_t)stream;
  const int nb = 2 * w + 1;
  // plan scratch: a flag per candidate, then one candidate's drift table
  const size_t need = (size_t)n_cand + (size_t)p.desc.n_fft;
  if (need > p.proj_words) {
    if (p.dProj) (void)hipFree(p.dProj);
    p.dProj = nullptr;
    p.proj_words = 0;
    void* v = nullptr;
    const fh_status st = device_alloc(&v, need * sizeof(int32_t));
    if (st != FH_OK) return st;
    p.dProj = static_cast<int32_t*>(v);
    p.proj_words = need;
  }
  int32_t* d_flag = p.dProj;
  int32_t* d_tab = p.dProj + n_cand;
  // enough work-groups to fill the chip: the FFTs of each candidate are split
  const long long cells = (long long)n_cand * nb;
  hipLaunchKernelGGL(k_project_clear, dim3((unsigned)std::min<long long>(1024, (cells + 255) / 256)), dim3(256), 0, s,
                     hist, cells);
  hipLaunchKernelGGL(k_project_clear, dim3((unsigned)std::min<long long>(1024, (n_cand + 255) / 256)), dim3(256), 0, s,
                     d_flag, (long long)n_cand);
  const int splits = std::max(1, std::min(std::max(1, p.desc.n_fft / kProjThreads), 2048 / std::max(1, n_cand)));
  hipLaunchKernelGGL(k_project, dim3((unsigned)n_cand, (unsigned)splits), dim3(kProjThreads), nb * sizeof(int), s,
                     peaks->row_ptr,
                     peaks->bin, (int)peaks->n_peaks, p.desc.n_fft, p.n_f, p.dT, p.desc.n, p.desc.tfft, p.desc.f_min,
                     f0, k, (int)w, hist, d_flag, (const int32_t*)nullptr, 0);
  if (hipGetLastError() != hipSuccess) return FH_EDEVICE;
  std::vector<int32_t> hh((size_t)n_cand * nb), flags((size_t)n_cand);
  if (hipMemcpyAsync(flags.data(), d_flag, flags.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FH_EDEVICE;
  // candidates with a drift bin near an edge: the host's drift table, projected again
  std::vector<int32_t> tab;
  const double nm1 = p.desc.n - 1.0, e = 1.0 / nm1, tf = p.desc.tfft, fmin = p.desc.f_min;
  for (int c = 0; c < n_cand; ++c) {
    if (!flags[c]) continue;
    double fk[2];
    if (hipMemcpyAsync(&fk[0], f0 + c, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&fk[1], k + c, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return FH_EDEVICE;
    const double a = (fk[1] * nm1) * std::pow(fk[0], nm1);
    const double b0 = std::floor((fk[0] - fmin) * tf);
    tab.resize(p.desc.n_fft);
    for (int i = 0; i < p.desc.n_fft; ++i) {
      const double f = fk[0] / std::pow(1.0 + a * p.T[i], e);
      const double sh = std::floor((f - fmin) * tf) - b0;
      // beyond int32 no bin can land within w of b_0: any value past the band does
      tab[i] = std::fabs(sh) < 1e9 ? (int32_t)sh : (sh < 0 ? -1000000000 : 1000000000);
    }
    if (hipMemcpyAsync(d_tab, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess)
      return FH_EDEVICE;
    hipLaunchKernelGGL(k_project_clear, dim3((unsigned)std::min(1024, (nb + 255) / 256)), dim3(256), 0, s,
                       hist + (size_t)c * nb, (long long)nb);
    hipLaunchKernelGGL(k_project, dim3(1, (unsigned)splits), dim3(kProjThreads), nb * sizeof(int), s, peaks->row_ptr,
                       peaks->bin, (int)peaks->n_peaks, p.desc.n_fft, p.n_f, p.dT, p.desc.n, p.desc.tfft,
                       p.desc.f_min, f0, k, (int)w, hist, d_flag, (const int32_t*)d_tab, c);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return FH_EDEVICE;
  }
  if (hipMemcpyAsync(hh.data(), hist, hh.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FH_EDEVICE;
  for (int c = 0; c < n_cand; ++c) {
    const int32_t* y = &hh[(size_t)c * nb];
    long long S = 0, S2 = 0, N = 0;
    for (int x = 0; x < nb; ++x) {
      if (x >= w - guard && x <= w + guard) continue;
      S += y[x];
      S2 += (long long)y[x] * y[x];
      ++N;
    }
    fh_projection& o = out[c];
    std::memset(&o, 0, sizeof(o));
    o.y = y[w];
    o.host_drift = flags[c] ? 1 : 0;
    o.mu = (double)S / (double)N;
    const double ex2 = (double)S2 / (double)N;
    const double var = ex2 - o.mu * o.mu;
    o.sigma = std::sqrt(var);
    o.cr = o.sigma > 0.0 ? ((double)o.y - o.mu) / o.sigma : std::nan("");
  }
  return FH_OK;
}
