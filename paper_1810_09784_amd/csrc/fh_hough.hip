// Generalized FrequencyHough kernels for gfx950 (Sec. IV of the paper: every
// peak (t_i, f) of the peakmap becomes, after x = f^(1-n), the line
// x0 = x - (n-1) k (t_i - t0) in the (x0, k) plane; the Hough map counts the
// lines through each cell).
//
// Work decomposition.  The map is cut into tiles of `rows` k-rows x `cols`
// x0-columns (optionally also into `tsplit` ranges of FFTs).  One work-group
// owns one tile: it keeps a differential copy of the tile in LDS (int32,
// one spare column per row), adds +1 at the first and -1 after the last
// column of every (peak, row) interval that meets the tile (LDS atomics),
// then prefix-sums every row with wavefront DPP scans and stores it with
// coalesced dword writes (or atomically adds it when time is split).
//
// Index arithmetic (identical on the host tables and here): for bin j, row r,
// FFT i:  u = fma(-C_r, T_i, A_j);  the interval is [floor(u_lo), floor(u_hi)]
// with u_lo from A_{j+1}, u_hi from A_j, clipped to the map / tile.
//
// Two ways to find the peaks of a tile:
//  - whole-FFT mode: every FFT that can reach the tile is read completely
//    (small maps: all peaks of an FFT usually land in the tile);
//  - windowed mode: per (row, FFT) the bins whose image can reach the tile's
//    columns are found from a column->bin table J and a per-FFT rank
//    structure (32-bin words: peaks below the word + bit mask), so wide maps
//    read only the peaks they need.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "fh_internal.h"

namespace fh {

// v_cvt_i32_f64: truncation toward zero; out-of-range inputs saturate to
// INT_MIN / INT_MAX (documented behaviour of the instruction; C's (int)
// conversion would be undefined there).
__device__ __forceinline__ int cvt_sat_i32(double x) {
  int r;
  asm("v_cvt_i32_f64_e32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

__device__ __forceinline__ bool is_negative(double x) {
  return (long long)__builtin_bit_cast(unsigned long long, x) < 0;
}

// Inclusive prefix sum over the 64 lanes of a wavefront (DPP row shifts and
// row broadcasts; all VALU, no LDS traffic).
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// One (peak, row) pair: the +1/-1 edges of its clipped interval in the tile.
// Drow points at the tile row; the slot at index (c1 - c0) absorbs right edges
// that fall outside the tile.
__device__ __forceinline__ void edge_update(int* Drow, double C, double T, double a_lo, double a_hi, int c0, int c1,
                                            bool valid) {
  const double u_lo = __builtin_fma(-C, T, a_lo);
  const double u_hi = __builtin_fma(-C, T, a_hi);
  // max(floor(u), c0) == max(trunc(u), c0) for c0 >= 0; floor(u_hi) < 0 iff u_hi < 0
  const int lo = max(cvt_sat_i32(u_lo), c0);
  const int hi = min(cvt_sat_i32(u_hi), c1 - 1);
  if (valid && !is_negative(u_hi) && lo <= hi) {
    atomicAdd(&Drow[lo - c0], 1);
    atomicAdd(&Drow[hi + 1 - c0], -1);
  }
}

// rank(i, j): number of peaks of FFT i with bin < j (0 <= j <= n_f).
__device__ __forceinline__ int peak_rank(const MapArgs& M, int i, int j) {
  const uint2 e = M.rank[(size_t)i * M.n_words + (j >> 5)];
  const unsigned below = (j & 31) ? ((1u << (j & 31)) - 1u) : 0u;
  return (int)e.x + __builtin_popcount(e.y & below);
}

// FFT range [ia, ib) whose shift s = C T_i can bring the band's image
// (A_{n_f} - s, A_0 - s] onto columns [c0, c1); one column of margin.
__device__ void fft_range(const MapArgs& M, double C, int c0, int c1, int i_lo, int i_hi, int* ia, int* ib) {
  const double hi_s = M.A[0] - (double)c0 + 1.0;
  const double lo_s = M.A[M.n_f] - (double)c1 - 1.0;
  if (C == 0.0) {
    const bool ok = lo_s <= 0.0 && 0.0 <= hi_s;
    *ia = i_lo;
    *ib = ok ? i_hi : i_lo;
    return;
  }
  const double tl = lo_s / C, th = hi_s / C;
  int a, b;
  if (M.t_uniform) {
    // T_i = (i + 0.5) tfft: widen by two FFTs, the exact clip decides
    const double fl = tl / M.tfft - 0.5, fh = th / M.tfft - 0.5;
    a = fl < (double)i_lo ? i_lo : (fl > (double)i_hi ? i_hi : (int)fl - 2);
    b = fh < (double)i_lo ? i_lo : (fh > (double)i_hi ? i_hi : (int)fh + 3);
    a = max(a, i_lo);
    b = min(max(b, a), i_hi);
  } else {
    int x = i_lo, y = i_hi;
    while (x < y) {
      int m = (x + y) >> 1;
      if (M.T[m] < tl) x = m + 1; else y = m;
    }
    a = x;
    y = i_hi;
    while (x < y) {
      int m = (x + y) >> 1;
      if (M.T[m] <= th) x = m + 1; else y = m;
    }
    b = x;
  }
  *ia = a;
  *ib = b;
}

template <int THREADS, bool ALDS>
__device__ void tile_body(const MapArgs& M, int tile, char* smem) {
  constexpr int NW = THREADS / kWave;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = uniform(tid >> 6);

  const int nxy = M.tiles_x * M.tiles_y;
  const int ts = tile / nxy;
  const int rem = tile - ts * nxy;
  const int rt = rem / M.tiles_x;
  const int ct = rem - rt * M.tiles_x;
  const int r0 = rt * M.rows;
  const int nrows = min(M.rows, M.n_k - r0);
  const int c0 = ct * M.cols;
  const int c1 = min(c0 + M.cols, M.n_x0);
  const int W = c1 - c0;
  const int i_lo = (int)((long long)M.n_fft * ts / M.tsplit);
  const int i_hi = (int)((long long)M.n_fft * (ts + 1) / M.tsplit);
  const int pitch = M.pitch;

  double* A_s = reinterpret_cast<double*>(smem);
  double* C_s = A_s + (ALDS ? (M.n_f + 1) : 0);
  int* ia_s = reinterpret_cast<int*>(C_s + M.rows);
  int* ib_s = ia_s + M.rows;
  int* wtot = ib_s + M.rows;           // per-wave partial sums (16 ints)
  int* span = wtot + 16;               // FFT union range (2 ints)
  int* D = span + 2 + ((4 - ((M.rows * 2 + 18) & 3)) & 3);
  const double* A = ALDS ? A_s : M.A;

  if (ALDS)
    for (int j = tid; j <= M.n_f; j += THREADS) A_s[j] = M.A[j];
  for (int x = tid; x < nrows * pitch; x += THREADS) D[x] = 0;
  if (tid < nrows) {
    const double C = M.C[r0 + tid];
    C_s[tid] = C;
    int a, b;
    fft_range(M, C, c0, c1, i_lo, i_hi, &a, &b);
    ia_s[tid] = a;
    ib_s[tid] = b;
  }
  __syncthreads();

  const bool count_bad = (rt == 0 && ct == 0);  // each (FFT, peak) counted by one tile

  if (M.mode == kModeWhole) {
    int i_start = i_hi, i_end = i_lo;
    for (int r = 0; r < nrows; ++r) {
      if (ia_s[r] < ib_s[r]) {
        i_start = min(i_start, ia_s[r]);
        i_end = max(i_end, ib_s[r]);
      }
    }
    if (count_bad) {
      i_start = i_lo;
      i_end = i_hi;
    }
    i_start = uniform(i_start);
    i_end = uniform(i_end);
    for (int i = i_start + wave; i < i_end; i += NW) {
      const bool act = lane < nrows && ia_s[lane] <= i && i < ib_s[lane];
      const unsigned long long amask = __ballot(act);
      if (!amask && !count_bad) continue;
      const int pa = uniform(min(max(M.row_ptr[i], 0), M.n_peaks));
      const int pb = uniform(min(max(M.row_ptr[i + 1], pa), M.n_peaks));
      const int m = pb - pa;
      if (m <= 0) continue;
      const double T = M.T[i];
      const int lsh = m >= 64 ? 6 : (m <= 1 ? 0 : 32 - __builtin_clz((unsigned)(m - 1)));  // ceil(log2 m)
      const int mp = 1 << lsh;
      const int q = lane >> lsh;      // row slot
      const int slot = lane & (mp - 1);
      const int ra = amask ? __builtin_ctzll(amask) : 0;
      const int rb = amask ? 64 - __builtin_clzll(amask) : 0;
      const int G = kWave >> lsh;
      for (int pc = pa; pc < pb; pc += kWave) {
        const int p = pc + slot;
        const bool pv = p < pb;
        const int j = M.bin[pv ? p : pa];  // in bounds: pa < pb <= n_peaks
        const bool jv = pv && (unsigned)j < (unsigned)M.n_f;
        if (count_bad && q == 0 && pv && !jv) atomicAdd(M.err, 1ull);
        const int jc = jv ? j : 0;
        const double a_hi = A[jc];
        const double a_lo = A[jc + 1];
        for (int rg = ra; rg < rb; rg += G) {
          const int rl = rg + q;
          const bool v = jv && rl < rb;
          const int rs = v ? rl : 0;
          edge_update(D + rs * pitch, C_s[rs], T, a_lo, a_hi, c0, c1, v);
        }
      }
    }
  } else {
    for (int rl = 0; rl < nrows; ++rl) {
      const int ia = ia_s[rl], ib = ib_s[rl];
      const double C = C_s[rl];
      int* Drow = D + rl * pitch;
      for (int i = ia + wave; i < ib; i += NW) {
        const double T = M.T[i];
        const double s = C * T;
        // a superset of the bins whose image can meet [c0, c1): A_j >= c0 + s and
        // A_{j+1} < c1 + s, each widened by one column against rounding
        const double y0 = (double)c0 + s - 1.0;
        const double y1 = (double)c1 + s + 1.0;
        int jb, ja;
        if (y0 < 0.0) jb = M.n_f - 1;
        else if (y0 >= (double)(M.n_J - 1)) jb = -1;
        else jb = min(M.J[(int)y0], M.n_f - 1);
        if (y1 <= 0.0) ja = 0;
        else if (y1 >= (double)(M.n_J - 1)) ja = M.J[M.n_J - 1];
        else ja = M.J[(int)__builtin_ceil(y1)];
        ja = max(ja, 0);
        if (jb < ja) continue;
        const int base = min(max(M.row_ptr[i], 0), M.n_peaks);
        const int end = min(max(M.row_ptr[i + 1], base), M.n_peaks);
        const int pa = uniform(min(base + peak_rank(M, i, ja), end));
        const int pb = uniform(min(base + peak_rank(M, i, jb + 1), end));
        for (int pc = pa; pc < pb; pc += kWave) {
          const int p = pc + lane;
          const bool pv = p < pb;
          const int j = M.bin[pv ? p : pa];  // in bounds: pa < pb <= n_peaks
          const bool jv = pv && (unsigned)j < (unsigned)M.n_f;
          const int jc = jv ? j : 0;
          const double a_hi = A[jc];
          const double a_lo = A[jc + 1];
          edge_update(Drow, C, T, a_lo, a_hi, c0, c1, jv);
        }
      }
    }
  }
  __syncthreads();

  // prefix sums along x0 and the store
  const bool accumulate = M.tsplit > 1;
  if (nrows >= NW) {
    for (int rl = wave; rl < nrows; rl += NW) {
      const int* Drow = D + rl * pitch;
      int32_t* out = M.map + (size_t)(r0 + rl) * M.n_x0 + c0;
      int carry = 0;
      for (int x0 = 0; x0 < W; x0 += kWave) {
        const int x = x0 + lane;
        const int v = x < W ? Drow[x] : 0;
        const int s = wave_incl_scan(v) + carry;
        if (x < W) {
          if (accumulate) {
            if (s) atomicAdd(&out[x], s);
          } else {
            out[x] = s;
          }
        }
        carry = __builtin_amdgcn_readlane(s, 63);
      }
    }
  } else {
    // few rows: all waves share each row, one segment per wave
    const int seg = ((W + NW - 1) / NW + kWave - 1) / kWave * kWave;
    for (int rl = 0; rl < nrows; ++rl) {
      const int* Drow = D + rl * pitch;
      const int xs = wave * seg, xe = min(W, xs + seg);
      int part = 0;
      for (int x0 = xs; x0 < xe; x0 += kWave) {
        const int x = x0 + lane;
        part += x < xe ? Drow[x] : 0;
      }
      part = wave_incl_scan(part);
      if (lane == 63) wtot[wave] = part;
      __syncthreads();
      int carry = 0;
      for (int w = 0; w < wave; ++w) carry += wtot[w];
      int32_t* out = M.map + (size_t)(r0 + rl) * M.n_x0 + c0;
      for (int x0 = xs; x0 < xe; x0 += kWave) {
        const int x = x0 + lane;
        const int v = x < xe ? Drow[x] : 0;
        const int s = wave_incl_scan(v) + carry;
        if (x < xe) {
          if (accumulate) {
            if (s) atomicAdd(&out[x], s);
          } else {
            out[x] = s;
          }
        }
        carry = __builtin_amdgcn_readlane(s, 63);
      }
      __syncthreads();
    }
  }
}

template <int THREADS, bool ALDS>
__global__ void __launch_bounds__(THREADS) k_hough(MapArgs M) {
  extern __shared__ __align__(16) char smem[];
  tile_body<THREADS, ALDS>(M, blockIdx.x, smem);
}

// Persistent batched kernel: work-groups claim (map, tile) entries of a queue
// (ordered longest first) until it is empty.
template <int THREADS>
__global__ void __launch_bounds__(THREADS) k_hough_batched(const MapArgs* __restrict__ maps,
                                                          const int2* __restrict__ queue, int n_queue, int* head) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(head, 1);
    __syncthreads();
    const int q = s_item;
    __syncthreads();
    if (q >= n_queue) break;
    const int2 e = queue[q];
    const MapArgs M = maps[e.x];
    tile_body<THREADS, true>(M, e.y, smem);
    __syncthreads();
  }
}

// Rank structure of the windowed mode and bad-peak counting: one thread per
// (FFT, 32-bin word).
__device__ void prepare_one(const MapArgs& M, long long t) {
  const int i = (int)(t / M.n_words);
  const int w = (int)(t - (long long)i * M.n_words);
  const int lo = min(max(M.row_ptr[i], 0), M.n_peaks);
  const int hi = min(max(M.row_ptr[i + 1], lo), M.n_peaks);
  const int key = w * 32;
  int a = lo, b = hi;
  while (a < b) {
    const int m = (a + b) >> 1;
    if (M.bin[m] < key) a = m + 1; else b = m;
  }
  unsigned mask = 0;
  unsigned long long bad = 0;
  int q = a;
  for (; q < hi; ++q) {
    const int j = M.bin[q];
    if (j >= key + 32) break;
    if (j < M.n_f) mask |= 1u << (j - key); else ++bad;
    if (q > lo && M.bin[q - 1] >= j) ++bad;
  }
  if (w == 0) bad += (unsigned long long)(a - lo);
  if (w == M.n_words - 1) bad += (unsigned long long)(hi - q);
  const_cast<uint2*>(M.rank)[(size_t)i * M.n_words + w] = make_uint2((unsigned)(a - lo), mask);
  if (bad) atomicAdd(M.err, bad);
}

__global__ void k_prepare(MapArgs M) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (long long)M.n_fft * M.n_words) prepare_one(M, t);
}

// All windowed maps of a batch, one after the other over the whole grid.
__global__ void k_prepare_batch(const MapArgs* __restrict__ maps, int m) {
  const long long st = (long long)gridDim.x * blockDim.x;
  for (int q = 0; q < m; ++q) {
    const MapArgs M = maps[q];
    if (M.mode != kModeWindowed) continue;
    const long long n = (long long)M.n_fft * M.n_words;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += st) prepare_one(M, t);
  }
}

// Error words of every map, and the maps of time-split plans, cleared.
__global__ void k_clear_batch(const MapArgs* __restrict__ maps, int m) {
  const long long st = (long long)gridDim.x * blockDim.x;
  for (int q = 0; q < m; ++q) {
    const MapArgs M = maps[q];
    if (blockIdx.x == 0 && threadIdx.x == 0) *M.err = 0;
    if (M.tsplit <= 1) continue;
    const long long n = (long long)M.n_k * M.n_x0;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += st) M.map[x] = 0;
  }
}

__global__ void k_clear(int32_t* map, long long n, unsigned long long* err) {
  const long long st = (long long)gridDim.x * blockDim.x;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += st) map[x] = 0;
  if (err && blockIdx.x == 0 && threadIdx.x == 0) *err = 0;
}

__global__ void k_zero_i32(int32_t* p, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) p[x] = 0;
}

static fh_status check_launch() { return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE; }

template <int THREADS, bool ALDS>
static fh_status launch_tiles(const MapArgs& a, int64_t tiles, hipStream_t s) {
  if (a.lds_bytes > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_hough<THREADS, ALDS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              a.lds_bytes);
  hipLaunchKernelGGL((k_hough<THREADS, ALDS>), dim3((unsigned)tiles), dim3(THREADS), a.lds_bytes, s, a);
  return check_launch();
}

fh_status launch_hough(const Plan& p, const fh_peaks& pk, int32_t* map, hipStream_t s) {
  MapArgs a = p.args(pk, map);
  const int64_t tiles = p.n_tiles();
  if (tiles <= 0 || tiles > 0x7fffffff) return FH_ERANGE;
  const long long cells = a.tsplit > 1 ? (long long)a.n_k * a.n_x0 : 0;
  const int cgrid = cells ? (int)std::min<long long>((cells + 255) / 256, 4096) : 1;
  hipLaunchKernelGGL(k_clear, dim3(cgrid), dim3(256), 0, s, map, cells, a.err);
  if (check_launch() != FH_OK) return FH_EDEVICE;
  if (a.mode == kModeWindowed) {
    const long long n = (long long)a.n_fft * a.n_words;
    hipLaunchKernelGGL(k_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    if (check_launch() != FH_OK) return FH_EDEVICE;
  }
  const int th = p.tile.threads;
  if (th == 512) return a.a_lds ? launch_tiles<512, true>(a, tiles, s) : launch_tiles<512, false>(a, tiles, s);
  return a.a_lds ? launch_tiles<256, true>(a, tiles, s) : launch_tiles<256, false>(a, tiles, s);
}

}  // namespace fh

// ------------------------------------------------------------- batching --

using namespace fh;

struct fh_batch_s {
  int32_t m = 0;
  std::vector<const Plan*> plans;
  std::vector<fh_peaks> peaks;
  std::vector<int32_t*> maps;
  std::vector<MapArgs> args;
  MapArgs* d_maps = nullptr;
  int2* d_queue = nullptr;
  int32_t* d_head = nullptr;
  int32_t n_queue = 0;
  int32_t grid = 0;
  int32_t lds = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void batch_free(fh_batch_s* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_maps) (void)hipFree(b->d_maps);
  if (b->d_queue) (void)hipFree(b->d_queue);
  if (b->d_head) (void)hipFree(b->d_head);
  delete b;
}

// Estimated cost of one tile: (FFT, row) pairs that can reach it times the
// mean peaks per FFT, plus the store.
static double tile_cost(const Plan& p, const MapArgs& a, int tile) {
  const int nxy = a.tiles_x * a.tiles_y;
  const int ts = tile / nxy, rem = tile % nxy, rt = rem / a.tiles_x, ct = rem % a.tiles_x;
  const int r0 = rt * a.rows, nrows = std::min(a.rows, a.n_k - r0);
  const int c0 = ct * a.cols, c1 = std::min(c0 + a.cols, a.n_x0);
  const long long i_lo = (long long)a.n_fft * ts / a.tsplit, i_hi = (long long)a.n_fft * (ts + 1) / a.tsplit;
  const double ppf = (double)a.n_peaks / std::max(1, a.n_fft);
  double pairs = 0;
  for (int r = 0; r < nrows; ++r) {
    const double C = p.C[r0 + r];
    const double hi_s = p.A[0] - c0 + 1.0;
    double nf;
    if (C == 0.0) nf = (double)(i_hi - i_lo);
    else {
      const double th = hi_s / C;
      double lo_t = p.T[i_lo], hi_t = p.T[i_hi - 1];
      double frac = (th - lo_t) / std::max(hi_t - lo_t, 1e-30);
      nf = (double)(i_hi - i_lo) * std::min(1.0, std::max(0.0, frac));
    }
    pairs += nf * ppf;
  }
  const double width_frac = a.mode == kModeWindowed ? std::min(1.0, (double)(c1 - c0) / a.n_x0 * 3.0) : 1.0;
  return pairs * width_frac + 0.25 * (double)nrows * (c1 - c0);
}

extern "C" fh_status fh_batch_create(int32_t m, const fh_plan_t* plans, const fh_peaks* peaks, int32_t* const* maps,
                                     fh_batch_t* out) {
  if (m < 1 || !plans || !peaks || !maps || !out) return FH_EINVAL;
  fh_batch_s* b = new (std::nothrow) fh_batch_s();
  if (!b) return FH_ENOMEM;
  b->m = m;
  int lds = 0;
  std::vector<std::pair<double, int2>> items;
  for (int i = 0; i < m; ++i) {
    if (!plans[i] || !maps[i] || !peaks[i].row_ptr || peaks[i].n_peaks < 0 || peaks[i].n_peaks >= (1LL << 31) ||
        (peaks[i].n_peaks > 0 && !peaks[i].bin)) {
      batch_free(b);
      return FH_EINVAL;
    }
    const Plan& p = reinterpret_cast<const fh_plan_s*>(plans[i])->p;
    MapArgs a = p.args(peaks[i], maps[i]);
    if (!a.a_lds) {  // the persistent kernel stages A in LDS
      batch_free(b);
      return FH_ERANGE;
    }
    // one work-group size for the whole batch: re-derive the LDS need at 256 threads
    b->plans.push_back(&p);
    b->peaks.push_back(peaks[i]);
    b->maps.push_back(maps[i]);
    b->args.push_back(a);
    lds = std::max(lds, a.lds_bytes);
    const int64_t nt = p.n_tiles();
    for (int64_t t = 0; t < nt; ++t) items.push_back({tile_cost(p, a, (int)t), make_int2(i, (int)t)});
  }
  if (items.size() >= (size_t)0x7fffffff) {
    batch_free(b);
    return FH_ERANGE;
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const std::pair<double, int2>& x, const std::pair<double, int2>& y) { return x.first > y.first; });
  std::vector<int2> q(items.size());
  for (size_t i = 0; i < items.size(); ++i) q[i] = items[i].second;
  b->n_queue = (int32_t)q.size();
  b->lds = lds;
  if (hipMalloc((void**)&b->d_maps, sizeof(MapArgs) * m) != hipSuccess ||
      hipMalloc((void**)&b->d_queue, sizeof(int2) * q.size()) != hipSuccess ||
      hipMalloc((void**)&b->d_head, sizeof(int32_t)) != hipSuccess) {
    batch_free(b);
    return FH_ENOMEM;
  }
  if (hipMemcpy(b->d_maps, b->args.data(), sizeof(MapArgs) * m, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_queue, q.data(), sizeof(int2) * q.size(), hipMemcpyHostToDevice) != hipSuccess) {
    batch_free(b);
    return FH_EDEVICE;
  }
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_hough_batched<256>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  int per_cu = 0, dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_hough_batched<256>, 256, lds) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  b->grid = std::min<int64_t>((int64_t)per_cu * std::max(cus, 1), b->n_queue);
  // capture: clear the queue head, per-map clears / rank builds, one persistent kernel
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    batch_free(b);
    return FH_EDEVICE;
  }
  bool ok = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, b->cap, b->d_head, 1);
    bool any_split = false, any_windowed = false;
    for (int i = 0; i < m; ++i) {
      any_split |= b->args[i].tsplit > 1;
      any_windowed |= b->args[i].mode == kModeWindowed;
    }
    hipLaunchKernelGGL(k_clear_batch, dim3(any_split ? 2048 : 1), dim3(256), 0, b->cap, b->d_maps, m);
    if (any_windowed) hipLaunchKernelGGL(k_prepare_batch, dim3(2048), dim3(256), 0, b->cap, b->d_maps, m);
    hipLaunchKernelGGL(k_hough_batched<256>, dim3(b->grid), dim3(256), lds, b->cap, b->d_maps, b->d_queue,
                       b->n_queue, b->d_head);
    ok = hipStreamEndCapture(b->cap, &b->graph) == hipSuccess;
  }
  if (ok) ok = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
  if (!ok) {
    batch_free(b);
    return FH_EDEVICE;
  }
  *out = reinterpret_cast<fh_batch_t>(b);
  return FH_OK;
}

extern "C" fh_status fh_batch_launch(fh_batch_t h, void* stream) {
  if (!h) return FH_EINVAL;
  fh_batch_s* b = reinterpret_cast<fh_batch_s*>(h);
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? FH_OK : FH_EDEVICE;
}

extern "C" fh_status fh_batch_launch_plain(fh_batch_t h, void* stream) {
  if (!h) return FH_EINVAL;
  fh_batch_s* b = reinterpret_cast<fh_batch_s*>(h);
  for (int i = 0; i < b->m; ++i) {
    fh_status st = launch_hough(*b->plans[i], b->peaks[i], b->maps[i], (hipStream_t)stream);
    if (st != FH_OK) return st;
  }
  return FH_OK;
}

extern "C" void fh_batch_destroy(fh_batch_t h) { batch_free(reinterpret_cast<fh_batch_s*>(h)); }

extern "C" fh_status fh_hough_batched(int32_t m, const fh_plan_t* plans, const fh_peaks* peaks, int32_t* const* maps,
                                      void* stream) {
  fh_batch_t b = nullptr;
  fh_status st = fh_batch_create(m, plans, peaks, maps, &b);
  if (st != FH_OK) return st;
  st = fh_batch_launch(b, stream);
  if (st == FH_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) st = FH_EDEVICE;
  fh_batch_destroy(b);
  return st;
}
