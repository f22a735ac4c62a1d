// Candidate selection on a Hough map (Sec. IV of the paper: squares over the
// (x0, k) plane, the best cell of each square and a second one a few k rows
// away, scored by the critical ratio CR = (y - mu) / sigma).
//
// Two passes on the device and a small finish on the host:
//  1. k_select_rows: one work-group per (map row, column segment of the square
//     grid) reads its part of the row once with 16-byte loads and writes the
//     exact int64 sum and sum of squares of the counts and the segment's best
//     cell (largest count, then smallest column);
//  2. k_select_squares: one work-group per square adds its rows' partials and
//     picks the best row (largest count, then smallest row) and the best row
//     at least min_dk rows away from it;
//  3. the host copies the per-square results (64 bytes each) and evaluates
//     mu, sigma and CR in binary64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "fh_internal.h"

namespace fh {

constexpr int kSelThreads = 256;
constexpr int kSelWaves = kSelThreads / 64;
constexpr int kSqWords = 6;  // per square: Sy, Sy2, key1, col1, key2, col2

template <typename T>
using gsel = __attribute__((address_space(1))) T*;
typedef int v4s __attribute__((ext_vector_type(4)));

// Order-preserving 32-bit image of a signed count, for packed (count, index) keys.
__device__ __forceinline__ unsigned long long biased(int y) { return (unsigned long long)((unsigned)y ^ 0x80000000u); }

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

// Sums and maximum over the work-group; the result is valid in thread 0.
__device__ __forceinline__ void block_reduce(long long& sy, long long& sy2, unsigned long long& key) {
  __shared__ long long s_sy[kSelWaves], s_sy2[kSelWaves];
  __shared__ unsigned long long s_key[kSelWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  sy = wave_sum_i64(sy);
  sy2 = wave_sum_i64(sy2);
  key = wave_max_u64(key);
  if (lane == 0) {
    s_sy[wave] = sy;
    s_sy2[wave] = sy2;
    s_key[wave] = key;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kSelWaves; ++w) {
      sy += s_sy[w];
      sy2 += s_sy2[w];
      key = s_key[w] > key ? s_key[w] : key;
    }
  }
}

struct SegAcc {
  long long sy = 0, sy2 = 0;
  int best = INT_MIN, col = -1;
  __device__ __forceinline__ void add(int y, int c) {  // columns arrive in ascending order per thread
    sy += y;
    sy2 += (long long)y * y;
    if (y > best || col < 0) {
      best = y;
      col = c;
    }
  }
};

// out[(r * sq_x0 + b) * 3 + {0, 1, 2}] = Sy, Sy2, (biased count << 32 | ~column)
// Grid: (n_k, sq_x0).  Segment b covers columns col_lo + floor(b W / sq_x0) ..
// col_lo + floor((b+1) W / sq_x0) - 1.
__global__ void __launch_bounds__(kSelThreads) k_select_rows(const int32_t* map_, int n_x0, int col_lo, int col_hi,
                                                              int sq_x0, unsigned long long* out_) {
  const gsel<const int32_t> map = (gsel<const int32_t>)map_;
  const int r = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  const int W = col_hi - col_lo;
  const int s0 = col_lo + (int)((long long)b * W / sq_x0);
  const int s1 = col_lo + (int)((long long)(b + 1) * W / sq_x0);
  const gsel<const int32_t> row = map + (size_t)r * n_x0;
  // columns [a0, a1) start on 16-byte boundaries
  const int head = (int)((4 - (((uintptr_t)(row + s0) >> 2) & 3)) & 3);
  const int a0 = min(s0 + head, s1);
  const int a1 = a0 + ((s1 - a0) & ~3);
  SegAcc acc;
  if (s0 + t < a0) acc.add(row[s0 + t], s0 + t);
  const gsel<const v4s> v = (gsel<const v4s>)(row + a0);
  const int nv = (a1 - a0) >> 2;
  int q = t;
  for (; q + 3 * kSelThreads < nv; q += 4 * kSelThreads) {
    v4s x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = v[q + u * kSelThreads];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = a0 + 4 * (q + u * kSelThreads);
      acc.add(x[u].x, c);
      acc.add(x[u].y, c + 1);
      acc.add(x[u].z, c + 2);
      acc.add(x[u].w, c + 3);
    }
  }
  for (; q < nv; q += kSelThreads) {
    const v4s x = v[q];
    const int c = a0 + 4 * q;
    acc.add(x.x, c);
    acc.add(x.y, c + 1);
    acc.add(x.z, c + 2);
    acc.add(x.w, c + 3);
  }
  if (a1 + t < s1) acc.add(row[a1 + t], a1 + t);
  unsigned long long key = acc.col >= 0 ? (biased(acc.best) << 32) | (unsigned)(~(unsigned)acc.col) : 0ull;
  long long sy = acc.sy, sy2 = acc.sy2;
  block_reduce(sy, sy2, key);
  if (t == 0) {
    gsel<unsigned long long> out = (gsel<unsigned long long>)out_ + ((size_t)r * sq_x0 + b) * 3;
    out[0] = (unsigned long long)sy;
    out[1] = (unsigned long long)sy2;
    out[2] = key;
  }
}

// Per square (a, b): rows floor(a n_k / sq_k) .. floor((a+1) n_k / sq_k) - 1.
// sq_out[(a * sq_x0 + b) * 6 + {0..5}] = Sy, Sy2, key1, col1, key2, col2 with
// key = biased count << 32 | ~row (0 = no such row).  Grid: (sq_k, sq_x0).
__device__ void square_body(const unsigned long long* rows_, int n_k, int sq_k, int sq_x0, int min_dk, int a, int b,
                            unsigned long long* sq_out_) {
  const gsel<const unsigned long long> rows = (gsel<const unsigned long long>)rows_;
  __shared__ int s_r1;
  const int t = threadIdx.x;
  const int r0 = (int)((long long)a * n_k / sq_k), r1 = (int)((long long)(a + 1) * n_k / sq_k);
  long long sy = 0, sy2 = 0;
  unsigned long long key = 0;
  for (int r = r0 + t; r < r1; r += kSelThreads) {
    const gsel<const unsigned long long> e = rows + ((size_t)r * sq_x0 + b) * 3;
    sy += (long long)e[0];
    sy2 += (long long)e[1];
    const unsigned long long k = (e[2] & 0xffffffff00000000ull) | (unsigned)(~(unsigned)r);
    key = k > key ? k : key;
  }
  block_reduce(sy, sy2, key);
  if (t == 0) s_r1 = key ? (int)~(unsigned)(key & 0xffffffffu) : -1;
  __syncthreads();
  const int best_r = s_r1;
  unsigned long long key2 = 0;
  if (min_dk >= 1 && best_r >= 0) {
    for (int r = r0 + t; r < r1; r += kSelThreads) {
      if (abs(r - best_r) < min_dk) continue;
      const unsigned long long k = (rows[((size_t)r * sq_x0 + b) * 3 + 2] & 0xffffffff00000000ull) |
                                   (unsigned)(~(unsigned)r);
      key2 = k > key2 ? k : key2;
    }
  }
  long long z0 = 0, z1 = 0;
  __syncthreads();  // block_reduce's LDS is reused
  block_reduce(z0, z1, key2);
  if (t == 0) {
    gsel<unsigned long long> o = (gsel<unsigned long long>)sq_out_ + ((size_t)a * sq_x0 + b) * kSqWords;
    auto col_of = [&](unsigned long long k) -> unsigned long long {
      if (!k) return ~0ull;
      const int r = (int)~(unsigned)(k & 0xffffffffu);
      return (unsigned long long)(~(unsigned)(rows[((size_t)r * sq_x0 + b) * 3 + 2] & 0xffffffffu));
    };
    o[0] = (unsigned long long)sy;
    o[1] = (unsigned long long)sy2;
    o[2] = key;
    o[3] = col_of(key);
    o[4] = key2;
    o[5] = col_of(key2);
  }
}

__global__ void __launch_bounds__(kSelThreads) k_select_squares(const unsigned long long* rows, int n_k, int sq_k,
                                                                 int sq_x0, int min_dk, unsigned long long* sq_out) {
  square_body(rows, n_k, sq_k, sq_x0, min_dk, blockIdx.x, blockIdx.y, sq_out);
}

// ------------------------------------------------------ batched selection --
// One map of a batched selection: its rows are global rows [row0, row0 +
// n_k) of the row partials, its squares global squares [sq0, sq0 + sq_k
// sq_x0) of the square results.
struct SelMap {
  const int32_t* map;
  int32_t n_k, n_x0, col_lo, col_hi;
  int32_t row0, sq0;
};

// The map holding global index g, for a table ascending in `first`.
template <typename F>
__device__ __forceinline__ int find_map(const SelMap* maps, int m, int g, F first) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(maps[mid]) <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Row pass over every map of the batch: one wavefront per (global row,
// column segment), sixteen per work-group.  The map of the work-group's
// first item is searched once and shared; a wavefront whose row lies in a
// later map searches for it.  Same sums, key and tie rule as k_select_rows.
constexpr int kBatchSelWaves = 16;

__global__ void __launch_bounds__(kBatchSelWaves * 64) k_select_rows_batch(const SelMap* __restrict__ maps, int m,
                                                                           long long n_items, int sq_x0,
                                                                           unsigned long long* rows_out_) {
  __shared__ int s_map;
  const int lane = threadIdx.x & 63;
  const long long item0 = (long long)blockIdx.x * kBatchSelWaves;
  if (threadIdx.x == 0)
    s_map = find_map(maps, m, (int)(item0 / sq_x0), [](const SelMap& x) { return x.row0; });
  __syncthreads();
  const long long item = item0 + (threadIdx.x >> 6);
  if (item >= n_items) return;  // uniform over the wavefront
  const int grow = (int)(item / sq_x0), b = (int)(item % sq_x0);
  int mi = s_map;
  if (grow >= maps[mi].row0 + maps[mi].n_k) mi = find_map(maps, m, grow, [](const SelMap& x) { return x.row0; });
  const SelMap M = maps[mi];
  const int r = grow - M.row0;
  const int W = M.col_hi - M.col_lo;
  const int s0 = M.col_lo + (int)((long long)b * W / sq_x0);
  const int s1 = M.col_lo + (int)((long long)(b + 1) * W / sq_x0);
  const gsel<const int32_t> row = (gsel<const int32_t>)M.map + (size_t)r * M.n_x0;
  SegAcc acc;
  for (int c = s0 + lane; c < s1; c += 64) acc.add(row[c], c);
  unsigned long long key = acc.col >= 0 ? (biased(acc.best) << 32) | (unsigned)(~(unsigned)acc.col) : 0ull;
  const long long sy = wave_sum_i64(acc.sy), sy2 = wave_sum_i64(acc.sy2);
  key = wave_max_u64(key);
  if (lane == 0) {
    gsel<unsigned long long> o = (gsel<unsigned long long>)rows_out_ + (size_t)item * 3;
    o[0] = (unsigned long long)sy;
    o[1] = (unsigned long long)sy2;
    o[2] = key;
  }
}

// Square reduction over every map of the batch: one work-group per global square.
__global__ void __launch_bounds__(kSelThreads) k_select_squares_batch(const SelMap* __restrict__ maps, int m, int sq_k,
                                                                     int sq_x0, int min_dk,
                                                                     const unsigned long long* rows,
                                                                     unsigned long long* sq_out) {
  const int g = blockIdx.x;
  const SelMap M = maps[find_map(maps, m, g, [](const SelMap& x) { return x.sq0; })];
  const int s = g - M.sq0;
  square_body(rows + (size_t)M.row0 * sq_x0 * 3, M.n_k, sq_k, sq_x0, min_dk, s / sq_x0, s % sq_x0,
              sq_out + (size_t)M.sq0 * kSqWords);
}

// Fused selection: its row partials carry the largest count of each (row,
// segment) but not its column.  For the best and the second row of every
// square, the first column of the row's segment holding that count (the
// selection's tie rule) is searched here, every load of a thread in flight
// at once.  Grid: (sq_k * sq_x0, 2).
constexpr int kColThreads = 1024;
constexpr int kColUnroll = 8;

__global__ void __launch_bounds__(kColThreads) k_select_cols(const int32_t* map_, int n_x0, int col_lo, int col_hi,
                                                              int sq_x0, unsigned long long* sq_out_) {
  __shared__ int s_first[kColThreads / 64];
  const int sqi = blockIdx.x, which = blockIdx.y, t = threadIdx.x;
  gsel<unsigned long long> o = (gsel<unsigned long long>)sq_out_ + (size_t)sqi * kSqWords;
  const unsigned long long key = o[2 + 2 * which];
  if (!key) return;  // uniform over the work-group
  const int y = (int)((unsigned)(key >> 32) ^ 0x80000000u);
  const int r = (int)~(unsigned)(key & 0xffffffffu);
  const int b = sqi % sq_x0;
  const int W = col_hi - col_lo;
  const int s0 = col_lo + (int)((long long)b * W / sq_x0);
  const int s1 = col_lo + (int)((long long)(b + 1) * W / sq_x0);
  const gsel<const int32_t> row = (gsel<const int32_t>)map_ + (size_t)r * n_x0;
  int first = INT_MAX;
  for (int c0 = s0; c0 < s1; c0 += kColThreads * kColUnroll) {
    int v[kColUnroll];
#pragma unroll
    for (int u = 0; u < kColUnroll; ++u) {
      const int c = c0 + u * kColThreads + t;
      v[u] = c < s1 ? row[c] : -1;
    }
#pragma unroll
    for (int u = kColUnroll - 1; u >= 0; --u)
      if (v[u] == y) first = min(first, c0 + u * kColThreads + t);
    if (__syncthreads_or(first != INT_MAX)) break;  // later columns are larger
  }
  for (int d = 32; d >= 1; d >>= 1) first = min(first, __shfl_xor(first, d));
  if ((t & 63) == 0) s_first[t >> 6] = first;
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kColThreads / 64; ++w) first = min(first, s_first[w]);
    o[3 + 2 * which] = (unsigned long long)(unsigned)first;
  }
}

}  // namespace fh

using namespace fh;

// Options checked against the plan; col_hi resolved.
static fh_status check_opts(const Plan& p, const fh_select_opts* o, fh_select_opts* r) {
  if (!o) return FH_EINVAL;
  *r = *o;
  r->col_hi = o->col_hi > 0 ? o->col_hi : p.n_x0;
  if (r->col_lo < 0 || r->col_hi > p.n_x0 || r->col_hi <= r->col_lo) return FH_EINVAL;
  const int W = r->col_hi - r->col_lo;
  if (r->sq_k < 1 || r->sq_k > p.desc.n_k || r->sq_x0 < 1 || r->sq_x0 > std::min(W, kMaxSelectSegments))
    return FH_EINVAL;
  return FH_OK;
}

// Selection scratch of the plan: row partials (3 n_k sq_x0 words), then the
// square results (kSqWords per square).  A pending fh_hough_select is waited
// for before the scratch is touched.
static fh_status sel_scratch(Plan& p, const fh_select_opts& o, unsigned long long** rows, unsigned long long** sq) {
  if (p.sel_pending && hipEventSynchronize(p.ev_sel) != hipSuccess) return FH_EDEVICE;
  const size_t row_words = (size_t)p.desc.n_k * o.sq_x0 * 3;
  const size_t need = row_words + (size_t)o.sq_k * o.sq_x0 * kSqWords;
  if (need > p.sel_words) {
    if (p.dSel) (void)hipFree(p.dSel);
    p.dSel = nullptr;
    p.sel_words = 0;
    void* v = nullptr;
    const fh_status st = device_alloc(&v, need * sizeof(unsigned long long));
    if (st != FH_OK) return st;
    p.dSel = static_cast<unsigned long long*>(v);
    p.sel_words = need;
  }
  *rows = p.dSel;
  *sq = p.dSel + row_words;
  return FH_OK;
}

// mu, sigma and CR of squares [s0, s1) from their exact sums (sq holds square
// s0 first), and their candidates: the first ones up to cap go to out,
// *total counts all of them.
static void emit_squares(const Plan& p, const fh_select_opts& o, const unsigned long long* sq, int s0, int s1,
                         fh_candidate* out, int32_t cap, int32_t* total_io, int n_rows = -1, int row_off = 0) {
  const int n_k = n_rows >= 0 ? n_rows : p.desc.n_k, sq_k = o.sq_k, sq_x0 = o.sq_x0;
  const int W = o.col_hi - o.col_lo;
  int32_t total = *total_io;
  const double inv1n = 1.0 / (1.0 - p.desc.n);
  auto emit = [&](unsigned long long key, unsigned long long col, int sqi, int second, double mu, double sigma) {
    const int y = (int)((unsigned)(key >> 32) ^ 0x80000000u);
    const int r = (int)~(unsigned)(key & 0xffffffffu) + row_off;
    const int c = (int)col;
    const double cr = ((double)y - mu) / sigma;
    if (!(cr >= o.cr_thr)) return;
    if (total < cap) {
      fh_candidate& e = out[total];
      std::memset(&e, 0, sizeof(e));
      e.row = r;
      e.col = c;
      e.count = y;
      e.square = sqi;
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
  (void)sq_k;
  for (int sqi = s0; sqi < s1; ++sqi) {
    const int a = sqi / sq_x0, b = sqi - a * sq_x0;
    const long long nr = (long long)(a + 1) * n_k / sq_k - (long long)a * n_k / sq_k;
    const long long nc = (long long)(b + 1) * W / sq_x0 - (long long)b * W / sq_x0;
    const long long N = nr * nc;
    const unsigned long long* e = &sq[(size_t)(sqi - s0) * kSqWords];
    if (N <= 0 || !e[2]) continue;
    const double mu = (double)(long long)e[0] / (double)N;
    const double ex2 = (double)(long long)e[1] / (double)N;
    const double var = ex2 - mu * mu;
    const double sigma = std::sqrt(var);
    if (!(sigma > 0.0)) continue;
    emit(e[2], e[3], sqi, 0, mu, sigma);
    if (e[4]) emit(e[4], e[5], sqi, 1, mu, sigma);
  }
  *total_io = total;
}

// All squares of a selection (square results of every square, in order).
static void emit_candidates(const Plan& p, const fh_select_opts& o, const unsigned long long* sq, fh_candidate* out,
                            int32_t cap, int32_t* n_out) {
  int32_t total = 0;
  emit_squares(p, o, sq, 0, o.sq_k * o.sq_x0, out, cap, &total);
  *n_out = total;
}

extern "C" fh_status fh_select(fh_plan_t h, const int32_t* map, const fh_select_opts* o, fh_candidate* out, int32_t cap,
                               int32_t* n_out, void* stream) {
  if (!h || !map || !o || !n_out || cap < 0 || (cap > 0 && !out)) return FH_EINVAL;
  Plan& p = reinterpret_cast<Plan&>(*h);
  fh_select_opts r;
  fh_status st = check_opts(p, o, &r);
  if (st != FH_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long *d_rows, *d_sq;
  st = sel_scratch(p, r, &d_rows, &d_sq);
  if (st != FH_OK) return st;
  hipLaunchKernelGGL(k_select_rows, dim3(p.desc.n_k, r.sq_x0), dim3(kSelThreads), 0, s, map, p.n_x0, r.col_lo,
                     r.col_hi, r.sq_x0, d_rows);
  hipLaunchKernelGGL(k_select_squares, dim3(r.sq_k, r.sq_x0), dim3(kSelThreads), 0, s, d_rows, p.desc.n_k, r.sq_k,
                     r.sq_x0, r.min_dk, d_sq);
  if (hipGetLastError() != hipSuccess) return FH_EDEVICE;
  std::vector<unsigned long long> sq((size_t)r.sq_k * r.sq_x0 * kSqWords);
  if (hipMemcpyAsync(sq.data(), d_sq, sq.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FH_EDEVICE;
  emit_candidates(p, r, sq.data(), out, cap, n_out);
  return FH_OK;
}

// ------------------------------------------- selection without allocation --
// fh_select_noalloc runs fh_select's kernels on a fixed scratch array instead
// of the plan's grown-on-demand buffer: the row partials, then the square
// results.  The array lives in the library's device image, one copy per GPU;
// its device address is looked up once per device (hipGetSymbolAddress) and
// only that address is handed to kernels and copies.  Both kernels write every
// word they later read, so nothing has to be cleared between calls.
constexpr size_t kNoAllocWords = size_t(1) << 19;  // 4 MiB of 64-bit words
static __device__ __align__(256) unsigned long long scratch[kNoAllocWords];
constexpr int kNoAllocDevices = 64;
constexpr int kNoAllocChunk = 256;  // squares per copy into the host finish
static unsigned long long* g_scratch_dev[kNoAllocDevices];
static std::mutex g_scratch_mu;

// Device address of this device's scratch array (current device).
static fh_status noalloc_scratch(unsigned long long** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return FH_EDEVICE;
  if (dev < 0 || dev >= kNoAllocDevices) return FH_ERANGE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FH_EDEVICE;
    g_scratch_dev[dev] = static_cast<unsigned long long*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return FH_OK;
}

extern "C" fh_status fh_select_noalloc(fh_plan_t h, const int32_t* map, const fh_select_opts* o, fh_candidate* out,
                                       int32_t cap, int32_t* n_out, void* stream) {
  if (!h || !map || !o || !n_out || cap < 0 || (cap > 0 && !out)) return FH_EINVAL;
  const Plan& p = reinterpret_cast<const Plan&>(*h);
  fh_select_opts r;
  fh_status st = check_opts(p, o, &r);
  if (st != FH_OK) return st;
  const size_t row_words = (size_t)p.desc.n_k * r.sq_x0 * 3;
  const size_t n_sq = (size_t)r.sq_k * r.sq_x0;
  if (row_words + n_sq * kSqWords > kNoAllocWords) return FH_ERANGE;
  unsigned long long* base = nullptr;
  st = noalloc_scratch(&base);
  if (st != FH_OK) return st;
  unsigned long long* d_rows = base;
  unsigned long long* d_sq = base + row_words;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_select_rows, dim3(p.desc.n_k, r.sq_x0), dim3(kSelThreads), 0, s, map, p.n_x0, r.col_lo,
                     r.col_hi, r.sq_x0, d_rows);
  hipLaunchKernelGGL(k_select_squares, dim3(r.sq_k, r.sq_x0), dim3(kSelThreads), 0, s, d_rows, p.desc.n_k, r.sq_k,
                     r.sq_x0, r.min_dk, d_sq);
  if (hipGetLastError() != hipSuccess) return FH_EDEVICE;
  // the host finish in chunks of squares through a buffer on the stack
  unsigned long long buf[kNoAllocChunk * kSqWords];
  int32_t total = 0;
  for (size_t s0 = 0; s0 < n_sq; s0 += kNoAllocChunk) {
    const size_t s1 = std::min(n_sq, s0 + kNoAllocChunk);
    if (hipMemcpyAsync(buf, d_sq + s0 * kSqWords, (s1 - s0) * kSqWords * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return FH_EDEVICE;
    emit_squares(p, r, buf, (int)s0, (int)s1, out, cap, &total);
  }
  *n_out = total;
  return FH_OK;
}

extern "C" fh_status fh_hough_select(fh_plan_t h, const fh_peaks* pk, int32_t* map, const fh_select_opts* o,
                                     void* stream) {
  if (!h || !map || !o || check_peaks(pk) != FH_OK) return FH_EINVAL;
  Plan& p = reinterpret_cast<Plan&>(*h);
  fh_select_opts r;
  fh_status st = check_opts(p, o, &r);
  if (st != FH_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long *d_rows, *d_sq;
  st = sel_scratch(p, r, &d_rows, &d_sq);
  if (st != FH_OK) return st;
  const size_t sq_words = (size_t)r.sq_k * r.sq_x0 * kSqWords;
  if (sq_words > p.hsq_words) {
    if (p.hSq) (void)hipHostFree(p.hSq);
    p.hSq = nullptr;
    p.hsq_words = 0;
    const hipError_t e = hipHostMalloc((void**)&p.hSq, sq_words * sizeof(unsigned long long), hipHostMallocDefault);
    if (e != hipSuccess) {
      p.hSq = nullptr;
      return e == hipErrorOutOfMemory ? FH_ENOMEM : FH_EDEVICE;
    }
    p.hsq_words = sq_words;
  }
  if (!p.ev_sel && hipEventCreateWithFlags(&p.ev_sel, hipEventDisableTiming) != hipSuccess) {
    p.ev_sel = nullptr;
    return FH_EDEVICE;
  }
  p.sel_pending = 0;
  const SelArgs sa{d_rows, r.sq_x0, r.col_lo, r.col_hi};
  st = launch_hough(p, *pk, map, s, &sa);
  if (st != FH_OK) return st;
  hipLaunchKernelGGL(k_select_squares, dim3(r.sq_k, r.sq_x0), dim3(kSelThreads), 0, s, d_rows, p.desc.n_k, r.sq_k,
                     r.sq_x0, r.min_dk, d_sq);
  hipLaunchKernelGGL(k_select_cols, dim3(r.sq_k * r.sq_x0, 2), dim3(kColThreads), 0, s, map, p.n_x0, r.col_lo, r.col_hi,
                     r.sq_x0, d_sq);
  if (hipGetLastError() != hipSuccess) return FH_EDEVICE;
  if (hipMemcpyAsync(p.hSq, d_sq, sq_words * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipEventRecord(p.ev_sel, s) != hipSuccess)
    return FH_EDEVICE;
  p.sel_opts = r;
  p.sel_pending = 1;
  return FH_OK;
}

extern "C" fh_status fh_select_results(fh_plan_t h, fh_candidate* out, int32_t cap, int32_t* n_out) {
  if (!h || !n_out || cap < 0 || (cap > 0 && !out)) return FH_EINVAL;
  Plan& p = reinterpret_cast<Plan&>(*h);
  if (!p.sel_pending) return FH_EINVAL;
  if (hipEventSynchronize(p.ev_sel) != hipSuccess) return FH_EDEVICE;
  emit_candidates(p, p.sel_opts, p.hSq, out, cap, n_out);
  p.sel_pending = 0;
  return FH_OK;
}

// ------------------------------------------------- selection in tiles --
// The selection of Sec. IV inside given 64 x 64 tiles of maps (the re-check
// of the tiles a proposer picks): each tile's rectangle, intersected with the
// analysed columns, is a small map of its own with sq_k x sq_x0 squares and
// square-local statistics.  All rectangles go through the batched row pass
// and square reduction in one launch each.
namespace {

struct Rect {
  const Plan* p;
  const int32_t* map;
  int32_t r0, n_rows, c0, c1;
};

constexpr int kTile = 64;

// The rectangle of tile t of a map of plan p, within the analysed columns of
// o; false if it holds no analysed column.
bool tile_rect(const Plan& p, const int32_t* map, const fh_select_opts& r, int t, Rect* out) {
  const int tb = (p.n_x0 + kTile - 1) / kTile;
  const int a = t / tb, b = t - a * tb;
  const int r0 = a * kTile, c0 = std::max(b * kTile, r.col_lo), c1 = std::min(b * kTile + kTile, std::min(p.n_x0, r.col_hi));
  if (r0 >= p.desc.n_k || c0 >= c1) return false;
  *out = Rect{&p, map + (size_t)r0 * p.n_x0, r0, std::min(kTile, p.desc.n_k - r0), c0, c1};
  return true;
}

fh_status select_rects(const std::vector<Rect>& rects, const std::vector<int32_t>& owner, int32_t n_owners,
                       const fh_select_opts& o, unsigned long long** scratch, size_t* scratch_bytes, fh_candidate* out,
                       int32_t cap, int32_t* counts, int32_t* n_out, hipStream_t s) {
  const int m = (int)rects.size();
  std::vector<SelMap> tab(m);
  long long rows = 0, squares = 0;
  for (int i = 0; i < m; ++i) {
    const Rect& q = rects[i];
    if (o.sq_k > q.n_rows || o.sq_x0 > std::min(q.c1 - q.c0, kMaxSelectSegments)) return FH_EINVAL;
    tab[i] = SelMap{q.map, q.n_rows, q.p->n_x0, q.c0, q.c1, (int32_t)rows, (int32_t)squares};
    rows += q.n_rows;
    squares += (long long)o.sq_k * o.sq_x0;
  }
  for (int i = 0; i < n_owners; ++i) counts[i] = 0;
  if (m == 0) {
    *n_out = 0;
    return FH_OK;
  }
  if (rows * o.sq_x0 >= (1LL << 31) || squares >= (1LL << 31)) return FH_ERANGE;
  const size_t tab_bytes = ((sizeof(SelMap) * (size_t)m + 255) / 256) * 256;
  const size_t row_words = (size_t)rows * o.sq_x0 * 3;
  const size_t sq_words = (size_t)squares * kSqWords;
  const size_t need = tab_bytes + 8 * (row_words + sq_words);
  if (need > *scratch_bytes) {
    if (*scratch) (void)hipFree(*scratch);
    *scratch = nullptr;
    *scratch_bytes = 0;
    void* v = nullptr;
    const fh_status st = device_alloc(&v, need);
    if (st != FH_OK) return st;
    *scratch = static_cast<unsigned long long*>(v);
    *scratch_bytes = need;
  }
  SelMap* d_tab = reinterpret_cast<SelMap*>(*scratch);
  unsigned long long* d_rows = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(*scratch) + tab_bytes);
  unsigned long long* d_sq = d_rows + row_words;
  if (hipMemcpyAsync(d_tab, tab.data(), sizeof(SelMap) * m, hipMemcpyHostToDevice, s) != hipSuccess)
    return FH_EDEVICE;
  const long long n_items = rows * o.sq_x0;
  hipLaunchKernelGGL(k_select_rows_batch, dim3((unsigned)((n_items + kBatchSelWaves - 1) / kBatchSelWaves)),
                     dim3(kBatchSelWaves * 64), 0, s, d_tab, m, n_items, o.sq_x0, d_rows);
  hipLaunchKernelGGL(k_select_squares_batch, dim3((unsigned)squares), dim3(kSelThreads), 0, s, d_tab, m, o.sq_k,
                     o.sq_x0, o.min_dk, d_rows, d_sq);
  if (hipGetLastError() != hipSuccess) return FH_EDEVICE;
  std::vector<unsigned long long> sq(sq_words);
  if (hipMemcpyAsync(sq.data(), d_sq, sq_words * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FH_EDEVICE;
  int32_t total = 0, written = 0;
  for (int i = 0; i < m; ++i) {
    const Rect& q = rects[i];
    fh_select_opts ro = o;
    ro.col_lo = q.c0;
    ro.col_hi = q.c1;
    int32_t n = 0;
    const int32_t room = cap - written;
    emit_squares(*q.p, ro, sq.data() + (size_t)tab[i].sq0 * kSqWords, 0, o.sq_k * o.sq_x0, out ? out + written : nullptr,
                 room, &n, q.n_rows, q.r0);
    counts[owner[i]] += n;
    written += std::min(n, room);
    total += n;
  }
  *n_out = total;
  return FH_OK;
}

}  // namespace

extern "C" fh_status fh_select_tiles(fh_plan_t h, const int32_t* map, const fh_select_opts* o, int32_t n_tiles,
                                     const int32_t* tiles, fh_candidate* out, int32_t cap, int32_t* counts,
                                     int32_t* n_out, void* stream) {
  if (!h || !map || !o || !n_out || n_tiles < 0 || (n_tiles > 0 && (!tiles || !counts)) || cap < 0 ||
      (cap > 0 && !out))
    return FH_EINVAL;
  Plan& p = reinterpret_cast<Plan&>(*h);
  fh_select_opts r = *o;
  r.col_hi = o->col_hi > 0 ? o->col_hi : p.n_x0;
  if (r.col_lo < 0 || r.col_hi > p.n_x0 || r.col_hi <= r.col_lo || r.sq_k < 1 || r.sq_x0 < 1) return FH_EINVAL;
  const int n_tiles_map = ((p.desc.n_k + kTile - 1) / kTile) * ((p.n_x0 + kTile - 1) / kTile);
  std::vector<Rect> rects;
  std::vector<int32_t> owner;
  for (int i = 0; i < n_tiles; ++i) {
    if (tiles[i] < 0 || tiles[i] >= n_tiles_map) return FH_EINVAL;
    Rect q;
    if (tile_rect(p, map, r, tiles[i], &q)) {
      rects.push_back(q);
      owner.push_back(i);
    }
  }
  // the plan's selection scratch, after a pending fused selection of the plan
  if (p.sel_pending && hipEventSynchronize(p.ev_sel) != hipSuccess) return FH_EDEVICE;
  size_t bytes = p.sel_words * 8;
  unsigned long long* scr = p.dSel;
  const fh_status st = select_rects(rects, owner, n_tiles, r, &scr, &bytes, out, cap, counts, n_out,
                                    (hipStream_t)stream);
  p.dSel = scr;
  p.sel_words = bytes / 8;
  return st;
}

extern "C" fh_status fh_batch_select_tiles(fh_batch_t b, const fh_select_opts* o, int32_t n_req, const int32_t* req,
                                           fh_candidate* out, int32_t cap, int32_t* counts, int32_t* n_out,
                                           void* stream) {
  if (!b || !o || !n_out || n_req < 0 || (n_req > 0 && (!req || !counts)) || cap < 0 || (cap > 0 && !out))
    return FH_EINVAL;
  if (o->sq_k < 1 || o->sq_x0 < 1) return FH_EINVAL;
  std::vector<Rect> rects;
  std::vector<int32_t> owner;
  for (int i = 0; i < n_req; ++i) {
    const int mi = req[2 * i], t = req[2 * i + 1];
    if (mi < 0 || mi >= b->m) return FH_EINVAL;
    const Plan& p = *b->plans[mi];
    fh_select_opts r = *o;
    r.col_hi = o->col_hi > 0 ? std::min(o->col_hi, p.n_x0) : p.n_x0;
    const int n_tiles_map = ((p.desc.n_k + kTile - 1) / kTile) * ((p.n_x0 + kTile - 1) / kTile);
    if (t < 0 || t >= n_tiles_map || r.col_lo < 0) return FH_EINVAL;
    Rect q;
    if (r.col_lo < r.col_hi && tile_rect(p, b->maps[mi], r, t, &q)) {
      rects.push_back(q);
      owner.push_back(i);
    }
  }
  return select_rects(rects, owner, n_req, *o, &b->d_sel, &b->sel_bytes, out, cap, counts, n_out,
                      (hipStream_t)stream);
}

extern "C" fh_status fh_batch_select(fh_batch_t b, const fh_select_opts* o, fh_candidate* out, int32_t cap,
                                     int32_t* counts, int32_t* n_out, void* stream) {
  if (!b || !o || !counts || !n_out || cap < 0 || (cap > 0 && !out)) return FH_EINVAL;
  const int m = b->m;
  std::vector<SelMap> tab(m);
  std::vector<fh_select_opts> res(m);
  long long rows = 0, squares = 0;
  for (int i = 0; i < m; ++i) {
    const Plan& p = *b->plans[i];
    const fh_status st = check_opts(p, o, &res[i]);
    if (st != FH_OK) return st;
    tab[i] = SelMap{b->maps[i], p.desc.n_k, p.n_x0, res[i].col_lo, res[i].col_hi, (int32_t)rows, (int32_t)squares};
    rows += p.desc.n_k;
    squares += (long long)o->sq_k * o->sq_x0;
  }
  if (rows * o->sq_x0 >= (1LL << 31) || squares >= (1LL << 31)) return FH_ERANGE;
  const size_t tab_bytes = ((sizeof(SelMap) * (size_t)m + 255) / 256) * 256;
  const size_t row_words = (size_t)rows * o->sq_x0 * 3;
  const size_t sq_words = (size_t)squares * kSqWords;
  const size_t need = tab_bytes + 8 * (row_words + sq_words);
  hipStream_t s = (hipStream_t)stream;
  if (need > b->sel_bytes) {  // the previous batched selection has completed (this call synchronises)
    if (b->d_sel) (void)hipFree(b->d_sel);
    b->d_sel = nullptr;
    b->sel_bytes = 0;
    void* v = nullptr;
    const fh_status st = device_alloc(&v, need);
    if (st != FH_OK) return st;
    b->d_sel = static_cast<unsigned long long*>(v);
    b->sel_bytes = need;
  }
  SelMap* d_tab = reinterpret_cast<SelMap*>(b->d_sel);
  unsigned long long* d_rows = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(b->d_sel) + tab_bytes);
  unsigned long long* d_sq = d_rows + row_words;
  if (hipMemcpyAsync(d_tab, tab.data(), sizeof(SelMap) * m, hipMemcpyHostToDevice, s) != hipSuccess)
    return FH_EDEVICE;
  const long long n_items = rows * o->sq_x0;
  hipLaunchKernelGGL(k_select_rows_batch, dim3((unsigned)((n_items + kBatchSelWaves - 1) / kBatchSelWaves)),
                     dim3(kBatchSelWaves * 64), 0, s, d_tab, m, n_items, o->sq_x0, d_rows);
  hipLaunchKernelGGL(k_select_squares_batch, dim3((unsigned)squares), dim3(kSelThreads), 0, s, d_tab, m, o->sq_k,
                     o->sq_x0, o->min_dk, d_rows, d_sq);
  if (hipGetLastError() != hipSuccess) return FH_EDEVICE;
  std::vector<unsigned long long> sq(sq_words);
  if (hipMemcpyAsync(sq.data(), d_sq, sq_words * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FH_EDEVICE;
  int32_t total = 0, written = 0;
  for (int i = 0; i < m; ++i) {
    int32_t n = 0;
    const int32_t room = cap - written;
    emit_candidates(*b->plans[i], res[i], sq.data() + (size_t)tab[i].sq0 * kSqWords, out ? out + written : nullptr,
                    room, &n);
    counts[i] = n;
    written += std::min(n, room);
    total += n;
  }
  *n_out = total;
  return FH_OK;
}
