// Generalized FrequencyHough kernels for gfx950 (Sec. IV of the paper: every
// peak (t_i, f) of the peakmap becomes, after x = f^(1-n), the line
// x0 = x - (n-1) k (t_i - t0) in the (x0, k) plane; the Hough map counts the
// lines through each cell).
//
// Work decomposition.  The map is cut into tiles of `rows` k-rows x `cols`
// x0-columns; a tile whose estimated work is large is further split into
// FFT ranges (work units).  A work-group runs one unit at a time from a
// queue ordered longest first: it keeps a differential copy of the tile in LDS (int32,
// one spare column per row), adds +1 at the first and -1 after the last
// column of every (peak, row) interval that meets the tile (LDS atomics),
// then prefix-sums every row with wavefront DPP scans and stores it with
// coalesced dword writes (or atomically adds it when the tile is split).
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
#include <climits>
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
  return (int)(__builtin_bit_cast(unsigned long long, x) >> 32) < 0;
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

// x of lane `l` (wave-uniform) as a double.
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// v_med3_i32: the middle of three values, here x clamped to [a, b] (a <= b).
__device__ __forceinline__ int med3_i32(int x, int a, int b) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(a), "v"(b));
  return r;
}

// One (peak, row) pair: +1 at the first column of its clipped interval in the
// tile and -1 one past the last.  Drow + c is column c of the tile row (its
// slot at c1 absorbs right edges outside the tile).  The columns are
// floor(u_lo) .. floor(u_hi); trunc (the conversion) equals floor for u >= 0,
// and clamped to c0 >= 0 the two agree for u_lo too.  For u_hi only tiles at
// column 0 can tell them apart: there an interval with u_hi < 0 lies left of
// the map and is dropped (ZERO_COL).  An empty interval (or one moved off the
// tile) makes no LDS access at all: the atomics are masked off.
// The clamp bounds of edge_update in vector registers (v_med3_i32 reads at
// most one scalar operand): c0, c1, c0 - 1, c1 - 1.  Copied once per tile by
// an instruction the compiler cannot move into the pair loops.
struct EdgeBounds {
  int c0, c1, c0m, c1m;
  __device__ __forceinline__ EdgeBounds(int a, int b) {
    asm volatile("v_mov_b32 %0, %1" : "=v"(c0) : "s"(a));
    asm volatile("v_mov_b32 %0, %1" : "=v"(c1) : "s"(b));
    asm volatile("v_mov_b32 %0, %1" : "=v"(c0m) : "s"(a - 1));
    asm volatile("v_mov_b32 %0, %1" : "=v"(c1m) : "s"(b - 1));
  }
};

template <bool ZERO_COL>
__device__ __forceinline__ void edge_update(int* Drow, double C, double T, double a_lo, double a_hi,
                                            const EdgeBounds& e) {
  const double u_lo = __builtin_fma(-C, T, a_lo);
  const double u_hi = __builtin_fma(-C, T, a_hi);
  const int lo = med3_i32(cvt_sat_i32(u_lo), e.c0, e.c1);
  const int hi = med3_i32(cvt_sat_i32(u_hi), e.c0m, e.c1m);  // the -1 goes to hi + 1
  if (lo <= hi && (!ZERO_COL || u_hi >= 0.0)) {
    atomicAdd(Drow + lo, 1);
    atomicAdd(Drow + hi + 1, -1);
  }
}

// The same update without a branch: an empty interval sends its +1 and -1 to
// the lane's own discard word (where they cancel), so every lane makes its two
// LDS accesses (the windowed pair loop, where most slots hold a pair).
template <bool ZERO_COL>
__device__ __forceinline__ void edge_update_nb(int* Drow, int* discard, double C, double T, double a_lo, double a_hi,
                                               const EdgeBounds& e) {
  const double u_lo = __builtin_fma(-C, T, a_lo);
  const double u_hi = __builtin_fma(-C, T, a_hi);
  const int lo = med3_i32(cvt_sat_i32(u_lo), e.c0, e.c1);
  const int hi = med3_i32(cvt_sat_i32(u_hi), e.c0m, e.c1m);
  const bool ok = lo <= hi && (!ZERO_COL || u_hi >= 0.0);
  int* plo = ok ? Drow + lo : discard;
  int* phi = ok ? Drow + hi : discard - 1;  // the -1 lands one past phi
  atomicAdd(plo, 1);
  atomicAdd(phi + 1, -1);
}

// Global-memory views of the map's arrays (address space 1), so that loads
// and stores are global (not flat) instructions and never ordered against LDS.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
typedef int v4i __attribute__((ext_vector_type(4)));

struct GMap {
  gptr<const double> A, C, T;
  gptr<const int> J, row_ptr, bin;
  gptr<const unsigned long long> rank;  // (bit mask << 32) | peaks below the word
  gptr<int> map;
  __device__ explicit GMap(const MapArgs& M)
      : A((gptr<const double>)M.A), C((gptr<const double>)M.C), T((gptr<const double>)M.T),
        J((gptr<const int>)M.J), row_ptr((gptr<const int>)M.row_ptr), bin((gptr<const int>)M.bin),
        rank((gptr<const unsigned long long>)M.rank), map((gptr<int>)M.map) {}
};

// rank(i, j): number of peaks of FFT i with bin < j (0 <= j <= n_f).
// T_i: the table entry, or for mid-FFT times the same binary64 expression the
// plan evaluates, ((double)i + 0.5) * tfft, without the load.
__device__ __forceinline__ double fft_time(const MapArgs& M, const GMap& G, int i) {
  return M.t_uniform ? ((double)i + 0.5) * M.tfft : G.T[i];
}

__device__ __forceinline__ int peak_rank(const MapArgs& M, const GMap& G, int i, int j) {
  const unsigned long long e = G.rank[(size_t)(j >> 5) * M.n_fft + i];
  const unsigned below = (j & 31) ? ((1u << (j & 31)) - 1u) : 0u;
  return (int)(unsigned)e + __builtin_popcount((unsigned)(e >> 32) & below);
}

// FFT range [ia, ib) whose shift s = C T_i can bring the band's image
// (A_{n_f} - s, A_0 - s] onto columns [c0, c1); one column of margin.
__device__ void fft_range(const MapArgs& M, const GMap& G, double C, int c0, int c1, int i_lo, int i_hi, int* ia,
                          int* ib) {
  const double hi_s = G.A[0] - (double)c0 + 1.0;
  const double lo_s = G.A[M.n_f] - (double)c1 - 1.0;
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
      if (G.T[m] < tl) x = m + 1; else y = m;
    }
    a = x;
    y = i_hi;
    while (x < y) {
      int m = (x + y) >> 1;
      if (G.T[m] <= th) x = m + 1; else y = m;
    }
    b = x;
  }
  *ia = a;
  *ib = b;
}

// Maximum over the wavefront (DPP, VALU only).
__device__ __forceinline__ int wave_max(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x111, 0xf, 0xf, false));  // row_shr:1
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x112, 0xf, 0xf, false));  // row_shr:2
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x114, 0xf, 0xf, false));  // row_shr:4
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x118, 0xf, 0xf, false));  // row_shr:8
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x142, 0xa, 0xf, false));  // row_bcast:15
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wave LDS scratch of the whole-FFT mode: one block of up to 64 FFTs.
struct WaveScratch {
  double T[kWave];     // time of each FFT of the block
  int rb[kWave];       // rows that can reach the tile at that FFT
  int rp[kWave + 4];   // CSR offsets of the block (65 used)
  int mark[kWave];     // per 64-peak chunk: FFT (in the block) starting at each position, else -1
};
static_assert(sizeof(WaveScratch) == kWaveScratchBytes, "per-wave LDS scratch size is part of the LDS budget");

// Inclusive maximum over the lanes of a wavefront (DPP, as wave_incl_scan).
__device__ __forceinline__ int wave_incl_max(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x111, 0xf, 0xf, false));  // row_shr:1
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x112, 0xf, 0xf, false));  // row_shr:2
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x114, 0xf, 0xf, false));  // row_shr:4
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x118, 0xf, 0xf, false));  // row_shr:8
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x142, 0xa, 0xf, false));  // row_bcast:15
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return x;
}


// Fused candidate selection.  The epilogue produces each tile row's final
// counts in ascending column runs per wavefront; SelRun adds them into the
// selection's per-(row, column segment) partials: the exact sums of y and
// y^2 and the largest count, packed as (count ^ 0x80000000) << 32 | ~0u (the
// column of the best cells is found afterwards, only for the rows the square
// reduction picks).  Lanes keep partials of the wave's current segment; a
// segment's partials are reduced over the wave and added with 64-bit global
// atomics when the segment ends inside the run or the run ends (a segment
// cut by tile or run boundaries gets several additions).  Segment b covers
// columns lo + floor(b (hi - lo) / sq) .. lo + floor((b + 1) (hi - lo) / sq) - 1.
// A 64-bit value moved by one DPP pattern (0 where the pattern has no source).
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)x, CTRL, ROWS, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(x >> 32), CTRL, ROWS, 0xf, false);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long x, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// Sum and maximum over the wavefront (the scan pattern of wave_incl_scan; lane
// 63 ends with the total), broadcast to every lane.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
  x += dpp_u64<0x111, 0xf>(x);
  x += dpp_u64<0x112, 0xf>(x);
  x += dpp_u64<0x114, 0xf>(x);
  x += dpp_u64<0x118, 0xf>(x);
  x += dpp_u64<0x142, 0xa>(x);
  x += dpp_u64<0x143, 0xc>(x);
  return readlane_u64(x, 63);
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
  unsigned long long y;
  y = dpp_u64<0x111, 0xf>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x112, 0xf>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x114, 0xf>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x118, 0xf>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x142, 0xa>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x143, 0xc>(x);
  x = y > x ? y : x;
  return readlane_u64(x, 63);
}

struct SelRun {
  gptr<unsigned long long> out;  // this row's partials, [sq][3]
  int sq, lo, hi;                // segments, analysed columns [lo, hi)
  int b, s0, s1;                 // current segment and its columns [s0, s1); b < 0: none (wave-uniform)
  unsigned long long sy, sy2;    // this lane's partials of segment b
  int best;
  int lane;

  // counts are >= 0 (maps written by the tile kernel), so best = -1 means none yet
  __device__ SelRun(const MapArgs& M, int row, int lane_)
      : out((gptr<unsigned long long>)M.sel + (size_t)row * M.sel_sq * 3), sq(M.sel_sq), lo(M.sel_lo),
        hi(M.sel_hi), b(-1), s0(0), s1(0), sy(0), sy2(0), best(-1), lane(lane_) {}

  __device__ int edge(int q) const { return lo + (int)((long long)q * (hi - lo) / sq); }
  // the segment holding column g (lo <= g < hi): the largest q with edge(q) <= g
  __device__ int segment_of(int g) const { return (int)(((long long)(g - lo + 1) * sq - 1) / (hi - lo)); }

  // Sums over four counts (pair sums fit 32 bits since counts <= n_fft < 2^31).
  __device__ __forceinline__ void sums4(const v4i& v) {
    sy += (unsigned long long)(unsigned)(v.x + v.y) + (unsigned long long)(unsigned)(v.z + v.w);
    sy2 += (unsigned long long)(unsigned)v.x * (unsigned)v.x + (unsigned long long)(unsigned)v.y * (unsigned)v.y +
           (unsigned long long)(unsigned)v.z * (unsigned)v.z + (unsigned long long)(unsigned)v.w * (unsigned)v.w;
  }
  // The four columns of a chunk with counts v, all counting.
  __device__ __forceinline__ void add4_all(const v4i& v) {
    sums4(v);
    best = max(max(best, v.x), max(max(v.y, v.z), v.w));
  }
  // Only the chunk's columns (g .. g+3) inside [a, e) count: the others enter
  // as 0 in the sums and as -1 (below every count) in the maximum.
  __device__ __forceinline__ void add4(const v4i& v, int g, int a, int e) {
    const v4i w = v4i{(g >= a && g < e) ? v.x : -1, (g + 1 >= a && g + 1 < e) ? v.y : -1,
                      (g + 2 >= a && g + 2 < e) ? v.z : -1, (g + 3 >= a && g + 3 < e) ? v.w : -1};
    best = max(max(best, w.x), max(max(w.y, w.z), w.w));
    sums4(v4i{max(w.x, 0), max(w.y, 0), max(w.z, 0), max(w.w, 0)});
  }
  __device__ __forceinline__ void flush() {
    if (b < 0) return;
    const unsigned long long key =
        best >= 0 ? ((unsigned long long)((unsigned)best ^ 0x80000000u) << 32) | 0xffffffffull : 0ull;
    const unsigned long long s = wave_sum_u64(sy), s2 = wave_sum_u64(sy2);
    const unsigned long long kmax = wave_max_u64(key);
    if (lane == 0) {
      gptr<unsigned long long> o = out + 3 * b;
      __hip_atomic_fetch_add(o, (unsigned long long)s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(o + 1, (unsigned long long)s2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_max(o + 2, kmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    sy = 0;
    sy2 = 0;
    best = -1;
    b = -1;
  }
  // One step of the wave's run: its chunks cover columns [ga, gb) (wave-
  // uniform); this lane's chunk holds columns g .. g + 3 with counts v.
  __device__ __forceinline__ void step(const v4i& v, int g, int ga, int gb) {
    const int a = max(ga, lo), e = min(gb, hi);
    if (a >= e) return;
    if (b < 0 || a < s0 || a >= s1) {  // the step starts a segment
      flush();
      b = segment_of(a);
      s0 = edge(b);
      s1 = edge(b + 1);
    }
    if (e <= s1) {
      if (a == ga && e == gb && gb - ga == 4 * kWave) add4_all(v);  // a full step inside the segment
      else add4(v, g, a, e);
      if (e == s1) flush();
      return;
    }
    for (int x = a; x < e;) {  // segment boundaries inside the step
      if (b < 0 || x < s0 || x >= s1) {
        flush();
        b = segment_of(x);
        s0 = edge(b);
        s1 = edge(b + 1);
      }
      const int y = min(e, s1);
      add4(v, g, x, y);
      if (y == s1) flush();
      x = y;
    }
  }
};

// Epilogue helpers.  A tile row of the differential D is read in chunks of 4
// columns (16-byte LDS accesses); pitch is a multiple of 4 and covers the pad
// column W, so every chunk of a row lies inside it.

// Sum of chunks [k0, k1) of a D row over the wave's lanes (result per lane).
__device__ __forceinline__ int sum_chunks(const int* Drow, int k0, int k1, int lane) {
  int s = 0;
#pragma unroll 4
  for (int kb = k0; kb < k1; kb += kWave) {
    const int k = kb + lane;
    const v4i v = *reinterpret_cast<const v4i*>(Drow + 4 * min(k, k1 - 1));
    s += k < k1 ? (v.x + v.y) + (v.z + v.w) : 0;
  }
  return s;
}

// Inclusive prefix sums of chunks [k0, k1) of a D row on top of `carry`:
// columns below W go to `out`, and every chunk is left zero for the next
// unit.  Plain stores go out as 16-byte chunks when `vec`; atomic adds (split
// tiles) go through the row in LDS so that each instruction covers 64
// consecutive columns.  `sr` (plain stores only): the fused selection of the
// row, whose tile column 0 is map column gc0.  Returns the carry after the
// last chunk.
__device__ __forceinline__ int scan_chunks(int* Drow, int k0, int k1, int carry, int W, gptr<int> out, bool vec,
                                           bool atomic, int lane, SelRun* sr = nullptr, int gc0 = 0) {
  for (int kb = k0; kb < k1; kb += kWave) {
    const int k = kb + lane;
    const bool in = k < k1;
    v4i* slot = reinterpret_cast<v4i*>(Drow + 4 * min(k, k1 - 1));
    v4i v = *slot;
    if (!in) v = v4i{0, 0, 0, 0};
    v.y += v.x;
    v.z += v.y;
    v.w += v.z;
    const int incl = wave_incl_scan(v.w);
    v += carry + incl - v.w;
    if (in) {
      const int c = 4 * k;
      if (atomic) {
        *slot = v;  // the counts, for the column pass below
      } else {
        *slot = v4i{0, 0, 0, 0};
        if (vec && c + 3 < W) {
          *(gptr<v4i>)(out + c) = v;
        } else {
          if (c < W) out[c] = v.x;
          if (c + 1 < W) out[c + 1] = v.y;
          if (c + 2 < W) out[c + 2] = v.z;
          if (c + 3 < W) out[c + 3] = v.w;
        }
      }
    }
    if (sr) sr->step(v, gc0 + 4 * k, gc0 + 4 * kb, gc0 + min(4 * min(kb + kWave, k1), W));
    carry += __builtin_amdgcn_readlane(incl, 63);
  }
  if (sr) sr->flush();
  if (atomic) {  // this wave's own columns, in order (LDS is in order within a wave)
    for (int x = 4 * k0 + lane; x < 4 * k1; x += kWave) {
      const int y = Drow[x];
      Drow[x] = 0;
      if (x < W && y) __hip_atomic_fetch_add(out + x, y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  return carry;
}

constexpr int kWinQuads = 2;  // windowed mode: 16-byte bin groups per loop step (8 peaks)

// Shared state of one unit, set up by tile_body.
struct TileCtx {
  const double* A_s;      // A table in LDS (n_f + 2 entries) when ALDS
  const double* C_s;      // C of the tile's rows in LDS
  WaveScratch* wsc;       // per-wave scratch of the whole-FFT mode
  const int* ia_s;        // per tile row: FFT range [ia, ib) that can reach the tile
  const int* ib_s;
  int* flags;             // [0]: ib non-increasing over the rows, [1] [2]: union FFT range, [3]: blocks claimed
  int* discard;           // this lane's sink of empty intervals (windowed mode)
  int* D;                 // differential tile, rows x pitch
  int rt, ct, r0, nrows, c0, c1, pitch, i_lo, i_hi, lane, wave;
};

// All (peak, row) pairs of a unit into the differential tile.  ZERO_COL: the
// tile starts at column 0 (the only case that needs the sign test of u_hi).
// MODE: kModeWhole or kModeWindowed compiles only that path; 0 takes the
// map's mode at run time (batches of mixed maps).
template <int THREADS, bool ALDS, int MODE, bool ZERO_COL>
__device__ __forceinline__ void tile_pairs(const MapArgs& M, const GMap& G, const TileCtx& X) {
  constexpr int NW = THREADS / kWave;
  const double* A_s = X.A_s;
  const double* C_s = X.C_s;
  const int* ia_s = X.ia_s;
  const int* ib_s = X.ib_s;
  int* discard = X.discard;
  int* D = X.D;
  const int rt = X.rt, ct = X.ct, nrows = X.nrows, c0 = X.c0, c1 = X.c1, pitch = X.pitch;
  const int i_lo = X.i_lo, i_hi = X.i_hi, lane = X.lane, wave = X.wave;
  if (MODE == 0 ? M.mode == kModeWhole : MODE == kModeWhole) {
    // Waves take blocks of 64 FFTs; lanes take the blocks' peaks 64 at a time
    // (coalesced) and loop over the tile rows that can reach the tile.
    const bool count_bad = (rt == 0 && ct == 0);  // each peak counted by one tile
    const int mono = X.flags[0];
    const int i_start = uniform(count_bad ? i_lo : X.flags[1]);
    const int i_end = uniform(count_bad ? i_hi : max(X.flags[2], X.flags[1]));
    WaveScratch& S = X.wsc[wave];
    const EdgeBounds eb(c0, c1);
    // C of the tile's rows through the scalar cache (uniform row index)
    const __attribute__((address_space(4))) double* Cg = (const __attribute__((address_space(4))) double*)M.C + X.r0;
    int prev_last = INT_MIN;  // bin of the previous chunk's last peak (bad-peak count)
    // C of the tile's first eight rows, held for every chunk (most chunks reach no further)
    double c_first[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c_first[q] = Cg[q];
    // waves claim blocks of FFTs in order until the range is done, so that
    // no wave idles while another still has several blocks to go; a wave claims
    // its next block, and loads that block's CSR offsets, while it works on the
    // current one (lane l < nb: start of FFT f0 + l; lanes >= nb: the block's end)
    int* claim = X.flags + 3;
    int f0_next = 0, rp_next = 0, rpe_next = 0;
    // blocks of up to 64 FFTs, fewer when the unit's range is short, so that
    // every wave of the work-group gets about two blocks
    const int BS = uniform(max(8, min(kWave, (i_end - i_start + 2 * NW - 1) / (2 * NW))));
    auto claim_block = [&]() {
      int bi = 0;
      if (lane == 0) bi = atomicAdd(claim, 1);
      f0_next = i_start + BS * uniform(__builtin_amdgcn_readlane(bi, 0));
      if (f0_next < i_end) {
        const int nbn = min(BS, i_end - f0_next);
        rp_next = G.row_ptr[f0_next + min(lane, nbn)];
        rpe_next = G.row_ptr[f0_next + nbn];
      }
    };
    claim_block();
    for (;;) {
      const int f0 = f0_next;
      if (f0 >= i_end) break;
      const int nb = min(BS, i_end - f0);
      const int fi = f0 + min(lane, nb - 1);
      const int rp_l = min(max(rp_next, 0), M.n_peaks);
      const int rp_e = uniform(min(max(rpe_next, 0), M.n_peaks));
      const int Pa = uniform(rp_l);
      const int Pb = max(rp_e, Pa);
      // the first chunk's bins, loaded before the block's set-up
      int j_next = Pa < Pb ? G.bin[min(Pa + lane, Pb - 1)] : 0;
      claim_block();
      const double Tf = fft_time(M, G, fi);
      int rb = nrows;
      if (mono) {
        int u = 0, w = nrows;  // first r with ib_r <= fi
        while (u < w) {
          const int mid = (u + w) >> 1;
          if (ib_s[mid] > fi) u = mid + 1; else w = mid;
        }
        rb = u;
      }
      // FFT l starts a run of peaks when it has any (the next FFT's start is larger)
      int rp_n = __shfl_down(rp_l, 1);
      if (lane == kWave - 1) rp_n = rp_e;
      const bool starts = lane < nb && rp_n > rp_l;
      wave_sync_lds();
      S.rp[lane] = rp_l;
      if (lane == 0) S.rp[kWave] = rp_e;
      S.T[lane] = Tf;
      S.rb[lane] = lane < nb ? rb : 0;
      S.mark[lane] = -1;
      wave_sync_lds();
      int u_carry = 0;  // FFT of the previous chunk's last peak
      for (int pc = Pa; pc < Pb; pc += kWave) {
        const int p = pc + lane;
        const bool pv = p < Pb;
        const int pcl = pv ? p : Pa;
        const int j = j_next;
        if (pc + kWave < Pb) j_next = G.bin[min(pc + kWave + lane, Pb - 1)];  // one chunk ahead
        // FFT of each peak: every FFT marks the chunk position of its first peak,
        // and a running maximum over the lanes carries the marks forward
        const int sft = rp_l - pc;
        if (starts && sft >= 0 && sft < kWave) S.mark[sft] = lane;
        wave_sync_lds();
        const int mk = S.mark[lane];
        S.mark[lane] = -1;  // each lane clears the slot it read (in order within the wave)
        const int u = wave_incl_max(max(mk, u_carry));
        u_carry = __builtin_amdgcn_readlane(u, 63);
        const double T = S.T[u];
        const int rb_u = S.rb[u];
        const bool jv = pv && (unsigned)j < (unsigned)M.n_f;
        if (count_bad) {
          // a bad peak: bin outside [0, n_f) or not above the previous bin of its
          // FFT; counted once (this tile sees every peak once)
          int jm = __shfl_up(j, 1);
          if (lane == 0) jm = prev_last;
          prev_last = __shfl(j, kWave - 1);
          const bool first = pcl == S.rp[u];
          if (pv && (!jv || (!first && j <= jm))) atomicAdd(M.err, 1ull);
        }
        // invalid lanes and bad bins read the pad entry A[n_f + 1] = +huge: an
        // interval right of every tile, which writes nothing
        const int jc = jv ? j : M.n_f;
        const double a_hi = ALDS ? A_s[jc] : G.A[jc];
        const double a_lo = ALDS ? A_s[jc + 1] : G.A[jc + 1];
        // rows that can reach the tile: largest for the chunk's first FFT (lane
        // 0's) when the rows' FFT ranges nest, else the largest over the lanes
        const int rmax = mono ? uniform(rb_u) : wave_max(rb_u);
        // eight rows per step; past the first eight, their C read with one scalar
        // load (the table has kCPad entries of padding after the last row)
        int* Drow = D - c0;
        for (int r = 0; r < rmax; r += 8, Drow += 8 * pitch) {
          double c[8];
          if (r == 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = c_first[q];
          } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = Cg[r + q];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (r + q < rmax) edge_update<ZERO_COL>(Drow + q * pitch, c[q], T, a_lo, a_hi, eb);
        }
      }
    }
  } else {
    // Per row: each lane owns one FFT, finds the peaks whose image can reach
    // the tile's columns and walks them eight at a time.
    const EdgeBounds eb(c0, c1);
    for (int rl = 0; rl < nrows; ++rl) {
      const int ia = ia_s[rl], ib = ib_s[rl];
      const double C = C_s[rl];
      int* Drow = D + rl * pitch - c0;
      for (int qb = ia + wave * kWave; qb < ib; qb += NW * kWave) {
        const int i = qb + lane;
        const bool iv = i < ib;
        const int ic = iv ? i : ia;
        const double T = fft_time(M, G, ic);
        const double s = C * T;
        // a superset of the bins whose image can meet [c0, c1): A_j >= c0 + s and
        // A_{j+1} < c1 + s, each widened by one column against rounding
        const double y0 = (double)c0 + s - 1.0;
        const double y1 = (double)c1 + s + 1.0;
        int jb, ja;
        if (y0 < 0.0) jb = M.n_f - 1;
        else if (y0 >= (double)(M.n_J - 1)) jb = -1;
        else jb = min(G.J[(int)y0], M.n_f - 1);
        if (y1 <= 0.0) ja = 0;
        else if (y1 >= (double)(M.n_J - 1)) ja = G.J[M.n_J - 1];
        else ja = G.J[(int)__builtin_ceil(y1)];
        ja = max(ja, 0);
        const int base = min(max(G.row_ptr[ic], 0), M.n_peaks);
        const int end = min(max(G.row_ptr[ic + 1], base), M.n_peaks);
        int pa = 0, pe = 0;
        if (iv && jb >= ja) {
          pa = min(base + peak_rank(M, G, ic, ja), end);
          pe = max(min(base + peak_rank(M, G, ic, jb + 1), end), pa);
        }
        // 16-byte aligned groups of four bins, kWinQuads groups per step
        for (int g = pa & ~3; g < pe; g += 4 * kWinQuads) {
          int jj[4 * kWinQuads];
#pragma unroll
          for (int k = 0; k < kWinQuads; ++k) {
            const int q = g + 4 * k;
            if (q + 3 < M.n_peaks && q < pe) {
              const v4i v = *(gptr<const v4i>)(G.bin + q);
              jj[4 * k] = v.x;
              jj[4 * k + 1] = v.y;
              jj[4 * k + 2] = v.z;
              jj[4 * k + 3] = v.w;
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e) jj[4 * k + e] = G.bin[min(q + e, M.n_peaks - 1)];
            }
          }
#pragma unroll
          for (int h = 0; h < kWinQuads; ++h) {
            double alo[4], ahi[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {  // table reads of four peaks before their atomics
              const int q = g + 4 * h + e;
              // peaks outside the window and bad bins read the pad entry A[n_f + 1]
              // = +huge: an interval right of every tile, which writes nothing
              const int jc = (q >= pa && q < pe) ? (int)min((unsigned)jj[4 * h + e], (unsigned)M.n_f) : M.n_f;
              ahi[e] = ALDS ? A_s[jc] : G.A[jc];
              alo[e] = ALDS ? A_s[jc + 1] : G.A[jc + 1];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) edge_update_nb<ZERO_COL>(Drow, discard, C, T, alo[e], ahi[e], eb);
          }
        }
      }
    }
  }
}

// Fused selection of the split tiles.  Their counts are final only when
// every unit has added its part, so a pass after the tile kernel reads them
// back from the map: grid (split tiles, kSelSplitParts), each work-group
// takes a run of the tile's columns, cut into kSelSplitWaves pieces, and its
// waves take the (row, piece) pairs.
constexpr int kSelSplitParts = 4;
constexpr int kSelSplitWaves = 4;

constexpr int kSelSplitUnroll = 4;  // steps whose loads are in flight together

__device__ void sel_chunks(const MapArgs& M, const GMap& G, int r, int c0, int W, int k0, int k1, int lane) {
  SelRun sr(M, r, lane);
  const gptr<const int> row = (gptr<const int>)G.map + (size_t)r * M.n_x0 + c0;
  for (int kb = k0; kb < k1; kb += kSelSplitUnroll * kWave) {
    v4i v[kSelSplitUnroll];
#pragma unroll
    for (int u = 0; u < kSelSplitUnroll; ++u) {
      const int k = kb + u * kWave + lane;
      const int c = 4 * k;
      v[u] = v4i{0, 0, 0, 0};
      if (k < k1) {
        if (c < W) v[u].x = row[c];
        if (c + 1 < W) v[u].y = row[c + 1];
        if (c + 2 < W) v[u].z = row[c + 2];
        if (c + 3 < W) v[u].w = row[c + 3];
      }
    }
#pragma unroll
    for (int u = 0; u < kSelSplitUnroll; ++u) {
      const int ks = kb + u * kWave;
      if (ks < k1) sr.step(v[u], c0 + 4 * (ks + lane), c0 + 4 * ks, c0 + min(4 * min(ks + kWave, k1), W));
    }
  }
  sr.flush();
}

__global__ void __launch_bounds__(kSelSplitWaves * 64) k_select_split(MapArgs M, const int4* __restrict__ clears,
                                                                        int n_clears) {
  const GMap G(M);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  for (int c = blockIdx.x; c < n_clears; c += gridDim.x) {
    const int tile = clears[c].y;
    const int rt = tile / M.tiles_x, ct = tile - rt * M.tiles_x;
    const int r0 = rt * M.rows, nrows = min(M.rows, M.n_k - r0);
    const int c0 = ct * M.cols, W = min(M.cols, M.n_x0 - c0);
    const long long P4 = (W + 3) >> 2;
    const int pieces = (int)gridDim.y * kSelSplitWaves;
    for (int it = wave; it < nrows * kSelSplitWaves; it += kSelSplitWaves) {
      const int rl = it / kSelSplitWaves;
      const int q = (int)blockIdx.y * kSelSplitWaves + it % kSelSplitWaves;
      const int k0 = (int)(P4 * q / pieces), k1 = (int)(P4 * (q + 1) / pieces);
      sel_chunks(M, G, r0 + rl, c0, W, k0, k1, lane);
    }
  }
}

// One unit: tile `tile` of map M over FFTs [i_lo, i_hi); `atomic` when the
// tile is split over several units (the map region was cleared beforehand).
// `clean`: leading words of the differential tile at LDS offset `clean_at`
// known to be zero (each epilogue leaves the rows it used zero).
template <int THREADS, bool ALDS, int MODE, bool SEL>
__device__ void tile_body(const MapArgs& M, int tile, int i_lo, int i_hi, bool atomic, bool load_a, char* smem,
                          int& clean, int& clean_at) {
  constexpr int NW = THREADS / kWave;
  const GMap G(M);
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = uniform(tid >> 6);

  const int rt = tile / M.tiles_x;
  const int ct = tile - rt * M.tiles_x;
  const int r0 = rt * M.rows;
  const int nrows = min(M.rows, M.n_k - r0);
  const int c0 = ct * M.cols;
  const int c1 = min(c0 + M.cols, M.n_x0);
  const int W = c1 - c0;
  const int pitch = M.pitch;

  // LDS: [A (n_f+2) doubles][C rows doubles][wave scratch x NW][ia rows][ib rows][wtot 16][flags 4][discard 64]
  //      [D rows*pitch, 16-byte aligned]
  // (no wave scratch in the windowed-only instantiation: its pair loop has no use for it)
  constexpr int NWS = MODE == kModeWindowed ? 0 : NW;
  double* A_s = reinterpret_cast<double*>(smem);
  double* C_s = A_s + (ALDS ? (M.n_f + 2) : 0);
  WaveScratch* wsc = reinterpret_cast<WaveScratch*>(C_s + M.rows);
  int* ia_s = reinterpret_cast<int*>(wsc + NWS);
  int* ib_s = ia_s + M.rows;
  int* wtot = ib_s + M.rows;  // per-wave partial sums (16 ints)
  int* flags = wtot + 16;     // [0]: ib non-increasing over the rows, [1] [2]: union FFT range
  int* discard = flags + 4 + lane;  // per-lane sink of empty intervals (64 ints)
  const int d_at = ((int)(reinterpret_cast<char*>(flags + 4 + kWave) - smem) + 15) & ~15;
  int* D = reinterpret_cast<int*>(smem + d_at);

  if (ALDS && load_a)
    for (int j = tid; j <= M.n_f + 1; j += THREADS) A_s[j] = G.A[j];
  if (clean_at != d_at || clean < nrows * pitch)
    for (int x = tid; x < nrows * pitch; x += THREADS) D[x] = 0;
  if (wave == 0) {
    // the rows' FFT ranges (one lane per row, nrows <= 64), whether they nest
    // (ib non-increasing over the rows) and their union, by wave reductions
    int a = i_hi, b = i_lo, b_prev = INT_MAX;
    if (lane < nrows) {
      const double C = G.C[r0 + lane];
      C_s[lane] = C;
      fft_range(M, G, C, c0, c1, i_lo, i_hi, &a, &b);
      ia_s[lane] = a;
      ib_s[lane] = b;
    }
    b_prev = __shfl_up(b, 1);
    const bool breaks = lane > 0 && lane < nrows && b > b_prev;
    const bool some = a < b;
    const int lo = -wave_max(some ? -a : INT_MIN + 1);
    const int hi = wave_max(some ? b : INT_MIN);
    if (lane == 0) {
      flags[0] = __builtin_amdgcn_ballot_w64(breaks) == 0;
      flags[1] = lo > i_hi ? i_hi : lo;  // no row reaches the tile: an empty range
      flags[2] = hi < i_lo ? i_lo : hi;
      flags[3] = 0;  // blocks of FFTs claimed so far (whole-FFT mode)
    }
  }
  __syncthreads();

  const TileCtx X{A_s, C_s, wsc, ia_s, ib_s, flags, discard, D, rt, ct, r0, nrows, c0, c1, pitch, i_lo, i_hi, lane,
                  wave};
  if (c0 == 0) tile_pairs<THREADS, ALDS, MODE, true>(M, G, X);
  else tile_pairs<THREADS, ALDS, MODE, false>(M, G, X);
  __syncthreads();

  // prefix sums along x0 and the store; D is left zero
  const int P4 = pitch >> 2;
  if (nrows >= NW) {
    for (int rl = wave; rl < nrows; rl += NW) {
      gptr<int> out = G.map + (size_t)(r0 + rl) * M.n_x0 + c0;
      const bool vec = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
      if (SEL && !atomic) {
        SelRun sr(M, r0 + rl, lane);
        scan_chunks(D + rl * pitch, 0, P4, 0, W, out, vec, false, lane, &sr, c0);
      } else {
        scan_chunks(D + rl * pitch, 0, P4, 0, W, out, vec, atomic, lane);
      }
    }
  } else {
    // few rows: all waves share each row, one run of chunks per wave (with the
    // fused selection, runs of whole 64-chunk steps)
    const int segc = SEL ? (((P4 + NW - 1) / NW + kWave - 1) & ~(kWave - 1)) : (P4 + NW - 1) / NW;
    const int k0 = min(wave * segc, P4), k1 = min(k0 + segc, P4);
    for (int rl = 0; rl < nrows; ++rl) {
      int* Drow = D + rl * pitch;
      const int part = wave_incl_scan(sum_chunks(Drow, k0, k1, lane));
      if (lane == 63) wtot[wave] = part;
      __syncthreads();
      int carry = 0;
      for (int w = 0; w < wave; ++w) carry += wtot[w];
      gptr<int> out = G.map + (size_t)(r0 + rl) * M.n_x0 + c0;
      const bool vec = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
      if (SEL && !atomic) {
        SelRun sr(M, r0 + rl, lane);
        scan_chunks(Drow, k0, k1, carry, W, out, vec, false, lane, &sr, c0);
      } else {
        scan_chunks(Drow, k0, k1, carry, W, out, vec, atomic, lane);
      }
      __syncthreads();
    }
  }
  clean = nrows * pitch;
  clean_at = d_at;
}

// Persistent work-queue kernel: work-groups claim units (ordered longest
// first) through an atomic counter until the queue is empty.  maps == nullptr:
// every unit belongs to M0.
template <int THREADS, bool ALDS, int MODE, bool SEL = false>
__global__ void __launch_bounds__(THREADS) k_queue(MapArgs M0, const MapArgs* __restrict__ maps,
                                                  const Unit* __restrict__ units, int n_units, int* head) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_item;
  int loaded = -1;  // map whose A table is in LDS
  int clean = 0, clean_at = -1;  // zero part of the differential tile
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(head, 1);
    __syncthreads();
    const int q = s_item;
    __syncthreads();
    if (q >= n_units) break;
    const Unit u = units[q];
    const int mi = u.x & ~kUnitAtomic;
    if (maps) {
      const MapArgs M = maps[mi];
      tile_body<THREADS, ALDS, MODE, SEL>(M, u.y, u.z, u.w, (u.x & kUnitAtomic) != 0, mi != loaded, smem, clean,
                                          clean_at);
    } else {
      tile_body<THREADS, ALDS, MODE, SEL>(M0, u.y, u.z, u.w, (u.x & kUnitAtomic) != 0, mi != loaded, smem, clean,
                                     clean_at);
    }
    loaded = mi;
    __syncthreads();
  }
}

// Before a launch: queue head and error words to zero, split tiles cleared.
// Grid: (clears, kClearSplit); block y clears its share of the columns of
// every row of the tile.
constexpr int kClearSplit = 8;
__global__ void k_prologue(MapArgs M0, const MapArgs* __restrict__ maps, int n_maps, const int4* __restrict__ clears,
                           int n_clears, int* head) {
  if (blockIdx.x == 0 && blockIdx.y == 0) {
    if (threadIdx.x == 0) *head = 0;
    for (int m = threadIdx.x; m < n_maps; m += blockDim.x) *(maps ? maps[m].err : M0.err) = 0;
  }
  if (M0.sel) {  // fused selection of a single-map launch: its partials to zero
    const int nth = (int)(gridDim.x * gridDim.y * blockDim.x);
    const int t = (int)((blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x);
    const long long n_sel = (long long)M0.n_k * M0.sel_sq * 3;
    for (long long x = t; x < n_sel; x += nth) ((gptr<unsigned long long>)M0.sel)[x] = 0;
  }
  for (int c = blockIdx.x; c < n_clears; c += gridDim.x) {
    const int4 e = clears[c];
    const MapArgs& M = maps ? maps[e.x] : M0;
    const int rt = e.y / M.tiles_x, ct = e.y % M.tiles_x;
    const int r0 = rt * M.rows, nrows = min(M.rows, M.n_k - r0);
    const int c0 = ct * M.cols, W = min(M.cols, M.n_x0 - c0);
    const int per = (W + (int)gridDim.y - 1) / (int)gridDim.y;
    const int xa = (int)blockIdx.y * per, xb = min(W, xa + per);
    for (int r = 0; r < nrows; ++r) {
      gptr<int> row = (gptr<int>)M.map + (size_t)(r0 + r) * M.n_x0 + c0;
      for (int x = xa + (int)threadIdx.x; x < xb; x += blockDim.x) row[x] = 0;
    }
  }
}

// Rank structure of the windowed mode and bad-peak counting.  A work-group
// takes a group of F consecutive FFTs, one wavefront per FFT: the FFT's peaks
// (lanes, coalesced) add into per-word counts and OR their bits into per-word
// masks in the wave's LDS scratch; an exclusive scan of the counts gives the
// peaks below each word.  The group's entries collect in LDS and leave as
// runs of F consecutive FFTs: entry w of FFT i is stored at
// rank[w * n_fft + i] as (mask << 32 | peaks below), so that the tile
// kernel's lanes (consecutive FFTs) read it coalesced.  Maps with more words
// than the LDS holds take the per-(FFT, word) binary search instead.
// The work-group's LDS is sized to its map (at most 20 KB, 13 KB for 126
// words), so that it fits beside a windowed tile kernel's work-group on a CU
// and a rank build can run while another map's tiles are in flight.
constexpr int kPrepWaves = 4;
constexpr int kPrepMaxWords = 512;
constexpr int kPrepLdsTarget = 4096;  // LDS words a group aims for (16 KB)
constexpr int kPrepUnroll = 8;        // peaks per lane loaded ahead (512 per wavefront step)

// FFTs per group: the largest power of two <= 64 whose entries (row pitch
// F + 1 u64) fit in the target beside the waves' scratch; at least one.
__host__ __device__ __forceinline__ int prep_group(int n_words) {
  int F = 64;
  while (F > 1 && (F + 1) * n_words * 2 + kPrepWaves * 2 * n_words > kPrepLdsTarget) F >>= 1;
  return F;
}

// Dynamic LDS of a rank-build work-group for a map of n_words words.
static int prep_lds_bytes(int n_words) {
  if (n_words > kPrepMaxWords) return 0;  // the per-(FFT, word) search uses none
  return ((prep_group(n_words) + 1) * n_words * 2 + kPrepWaves * 2 * n_words) * 4;
}

// The first kPrepUnroll * 64 bins of peaks [lo, hi), one per lane and step.
__device__ __forceinline__ void prep_bins(const GMap& G, int lo, int hi, int lane, int* jv) {
#pragma unroll
  for (int u = 0; u < kPrepUnroll; ++u) {
    const int p = lo + u * kWave + lane;
    jv[u] = p < hi ? G.bin[p] : 0;
  }
}

// One FFT (peaks [lo, hi)) into the wave's LDS counts and masks, then its
// rank words into rbuf; j0 holds its first step of bins, loaded beforehand.
__device__ void prepare_fft_lds(const MapArgs& M, int lo, int hi, const int* j0, int lane, unsigned* cnt,
                                unsigned* msk, unsigned long long* rbuf, int pitch) {
  const GMap G(M);
  for (int w = lane; w < M.n_words; w += kWave) {
    cnt[w] = 0;
    msk[w] = 0;
  }
  wave_sync_lds();
  int bad = 0, neg = 0;
  int last = INT_MIN;  // bin of the previous peak of this FFT
  for (int p0 = lo; p0 < hi; p0 += kPrepUnroll * kWave) {
    int jv[kPrepUnroll];  // all loads of the step in flight before the first use
    if (p0 == lo) {
#pragma unroll
      for (int u = 0; u < kPrepUnroll; ++u) jv[u] = j0[u];
    } else {
      prep_bins(G, p0, hi, lane, jv);
    }
#pragma unroll
    for (int u = 0; u < kPrepUnroll; ++u) {
      if (p0 + u * kWave >= hi) break;
      const int p = p0 + u * kWave + lane;
      const bool v = p < hi;
      const int j = jv[u];
      int jm = __shfl_up(j, 1);
      if (lane == 0) jm = last;
      last = __shfl(j, kWave - 1);
      if (v) {
        const bool out = j < 0 || j >= M.n_f;
        bad += out || j <= jm;  // out of the band or not ascending: one bad peak
        if (out) {
          neg += j < 0;
        } else {
          atomicAdd(&cnt[j >> 5], 1u);
          atomicOr(&msk[j >> 5], 1u << (j & 31));
        }
      }
    }
  }
  wave_sync_lds();
  // negative bins sit before word 0: they shift every word's position
  neg = wave_incl_scan(neg);
  unsigned carry = (unsigned)__builtin_amdgcn_readlane(neg, 63);
  for (int w0 = 0; w0 < M.n_words; w0 += kWave) {
    const int w = w0 + lane;
    const unsigned c = w < M.n_words ? cnt[w] : 0u;
    const unsigned incl = (unsigned)wave_incl_scan((int)c) + carry;
    if (w < M.n_words) rbuf[(size_t)w * pitch] = ((unsigned long long)msk[w] << 32) | (incl - c);
    carry = (unsigned)__builtin_amdgcn_readlane((int)incl, 63);
  }
  bad = wave_incl_scan(bad);
  if (lane == 63 && bad) atomicAdd(M.err, (unsigned long long)bad);
  wave_sync_lds();
}

// Fallback for very wide bands: one thread per (FFT, word), binary search in
// the FFT's bins.
__device__ void prepare_word(const MapArgs& M, long long t) {
  const GMap G(M);
  const int i = (int)(t % M.n_fft);
  const int w = (int)(t / M.n_fft);
  const int lo = min(max(G.row_ptr[i], 0), M.n_peaks);
  const int hi = min(max(G.row_ptr[i + 1], lo), M.n_peaks);
  const int key = w * 32;
  int a = lo, b = hi;
  while (a < b) {
    const int m = (a + b) >> 1;
    if (G.bin[m] < key) a = m + 1; else b = m;
  }
  unsigned mask = 0;
  unsigned long long bad = 0;
  int q = a;
  for (; q < hi; ++q) {
    const int j = G.bin[q];
    if (j >= key + 32) break;
    if (j < M.n_f) mask |= 1u << (j & 31);
    bad += j >= M.n_f || (q > lo && G.bin[q - 1] >= j);  // out of the band or not ascending: one bad peak
  }
  if (w == 0) bad += (unsigned long long)(a - lo);
  if (w == M.n_words - 1) bad += (unsigned long long)(hi - q);
  ((gptr<unsigned long long>)M.rank)[(size_t)w * M.n_fft + i] = ((unsigned long long)mask << 32) | (unsigned)(a - lo);
  if (bad) atomicAdd(M.err, bad);
}

// Whole grid over one map.  Every branch and trip count around the barriers
// is uniform over the work-group.
__device__ void prepare_map(const MapArgs& M, unsigned* lds) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (M.n_words <= kPrepMaxWords) {
    const int F = prep_group(M.n_words);
    const int pitch = F + 1;
    unsigned* cnt = lds + wave * 2 * M.n_words;
    unsigned long long* rbuf = (unsigned long long*)(lds + kPrepWaves * 2 * M.n_words);
    gptr<unsigned long long> rank = (gptr<unsigned long long>)M.rank;
    const int n_groups = (M.n_fft + F - 1) / F;
    for (int g = blockIdx.x; g < n_groups; g += gridDim.x) {
      const int i0 = g * F;
      const int nf = min(F, M.n_fft - i0);
      // the wave's FFTs in pairs: both CSR ranges, then both first steps of
      // bins are in flight before the first FFT is processed
      const GMap G(M);
      for (int f = wave; f < nf; f += 2 * kPrepWaves) {
        const int fb = f + kPrepWaves;
        const bool two = fb < nf;  // uniform over the wavefront
        const int ia = uniform(i0 + f), ibb = uniform(i0 + (two ? fb : f));
        const int loA = min(max(G.row_ptr[ia], 0), M.n_peaks);
        const int hiA = min(max(G.row_ptr[ia + 1], loA), M.n_peaks);
        const int loB = min(max(G.row_ptr[ibb], 0), M.n_peaks);
        const int hiB = min(max(G.row_ptr[ibb + 1], loB), M.n_peaks);
        int jA[kPrepUnroll], jB[kPrepUnroll];
        prep_bins(G, loA, hiA, lane, jA);
        if (two) prep_bins(G, loB, hiB, lane, jB);
        prepare_fft_lds(M, loA, hiA, jA, lane, cnt, cnt + M.n_words, rbuf + f, pitch);
        if (two) prepare_fft_lds(M, loB, hiB, jB, lane, cnt, cnt + M.n_words, rbuf + fb, pitch);
      }
      __syncthreads();
      const int n = M.n_words * F;
      for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int w = e / F, f = e - w * F;
        if (f < nf) rank[(size_t)w * M.n_fft + i0 + f] = rbuf[w * pitch + f];
      }
      __syncthreads();
    }
  } else {
    const long long n = (long long)M.n_fft * M.n_words;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
      prepare_word(M, t);
  }
}

__global__ void __launch_bounds__(kPrepWaves * 64) k_prepare(MapArgs M) {
  extern __shared__ unsigned prep_lds[];
  prepare_map(M, prep_lds);
}

// All windowed maps of a batch, one after the other over the whole grid.
__global__ void __launch_bounds__(kPrepWaves * 64) k_prepare_batch(const MapArgs* __restrict__ maps, int m) {
  extern __shared__ unsigned prep_lds[];
  for (int q = 0; q < m; ++q) {
    const MapArgs M = maps[q];
    if (M.mode == kModeWindowed) prepare_map(M, prep_lds);
  }
}

static fh_status check_launch() { return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE; }

template <int THREADS, bool ALDS, int MODE, bool SEL = false>
static void set_lds_attr(int lds) {
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_queue<THREADS, ALDS, MODE, SEL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

template <int MODE>
static const void* queue_fn(int threads) {
  return threads == 1024 ? (const void*)k_queue<1024, true, MODE>
         : threads == 512 ? (const void*)k_queue<512, true, MODE> : (const void*)k_queue<256, true, MODE>;
}

int occupancy_grid(int threads, int lds_bytes, int n_units, int mode) {
  int per_cu = 0, dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  const void* fn = mode == kModeWhole ? queue_fn<kModeWhole>(threads)
                   : mode == kModeWindowed ? queue_fn<kModeWindowed>(threads) : queue_fn<0>(threads);
  if (lds_bytes > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds_bytes) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const long long g = (long long)per_cu * cus;
  return (int)std::min<long long>(g, std::max(n_units, 1));
}

template <int THREADS, bool ALDS, int MODE, bool SEL>
static fh_status launch_queue(const MapArgs& a, const Plan& p, hipStream_t s) {
  set_lds_attr<THREADS, ALDS, MODE, SEL>(a.lds_bytes);
  hipLaunchKernelGGL((k_queue<THREADS, ALDS, MODE, SEL>), dim3((unsigned)p.grid), dim3(THREADS), a.lds_bytes, s, a,
                     (const MapArgs*)nullptr, (const Unit*)p.dUnits, (int)p.units.size(), p.dHead);
  return check_launch();
}

// SEL: the tile kernel with the fused selection in its epilogue, a separate
// instantiation so that the plain kernel keeps its register budget.
template <int MODE, bool SEL>
static fh_status launch_queue_mode(const MapArgs& a, const Plan& p, hipStream_t s) {
  const int th = p.tile.threads;
  if (th == 1024)
    return a.a_lds ? launch_queue<1024, true, MODE, SEL>(a, p, s) : launch_queue<1024, false, MODE, SEL>(a, p, s);
  if (th == 512)
    return a.a_lds ? launch_queue<512, true, MODE, SEL>(a, p, s) : launch_queue<512, false, MODE, SEL>(a, p, s);
  return a.a_lds ? launch_queue<256, true, MODE, SEL>(a, p, s) : launch_queue<256, false, MODE, SEL>(a, p, s);
}

fh_status launch_hough(const Plan& p, const fh_peaks& pk, int32_t* map, hipStream_t s, const SelArgs* sel) {
  MapArgs a = p.args(pk, map);
  if (sel) {
    a.sel = sel->rows;
    a.sel_sq = sel->sq;
    a.sel_lo = sel->lo;
    a.sel_hi = sel->hi;
  }
  if (p.units.empty()) return FH_EINVAL;
  const int n_clears = (int)p.clears.size();
  hipLaunchKernelGGL(k_prologue, dim3((unsigned)std::max(1, std::min(n_clears, 1024)), kClearSplit), dim3(256), 0, s, a,
                     (const MapArgs*)nullptr, 1, (const int4*)p.dClears, n_clears, p.dHead);
  if (check_launch() != FH_OK) return FH_EDEVICE;
  if (a.mode == kModeWindowed) {
    hipLaunchKernelGGL(k_prepare, dim3(2048), dim3(kPrepWaves * 64), prep_lds_bytes(a.n_words), s, a);
    if (check_launch() != FH_OK) return FH_EDEVICE;
  }
  if (p.ev_start && hipEventRecord(p.ev_start, s) != hipSuccess) return FH_EDEVICE;
  fh_status st;
  if (sel)
    st = a.mode == kModeWhole ? launch_queue_mode<kModeWhole, true>(a, p, s)
                              : launch_queue_mode<kModeWindowed, true>(a, p, s);
  else
    st = a.mode == kModeWhole ? launch_queue_mode<kModeWhole, false>(a, p, s)
                              : launch_queue_mode<kModeWindowed, false>(a, p, s);
  if (st == FH_OK && p.ev_stop && hipEventRecord(p.ev_stop, s) != hipSuccess) return FH_EDEVICE;
  if (st == FH_OK && sel && n_clears > 0) {
    const dim3 grid((unsigned)std::min(n_clears, 4096), kSelSplitParts);
    hipLaunchKernelGGL(k_select_split, grid, dim3(kSelSplitWaves * 64), 0, s, a, (const int4*)p.dClears, n_clears);
    return check_launch();
  }
  return st;
}

}  // namespace fh

// ------------------------------------------------------------- batching --

using namespace fh;

constexpr int kBatchWholeThreads = 512;  // batches of whole-FFT maps whose plans differ in work-group size

static void batch_free(fh_batch_s* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_maps) (void)hipFree(b->d_maps);
  if (b->d_queue) (void)hipFree(b->d_queue);
  if (b->d_clears) (void)hipFree(b->d_clears);
  if (b->d_head) (void)hipFree(b->d_head);
  if (b->d_sel) (void)hipFree(b->d_sel);
  delete b;
}

extern "C" fh_status fh_batch_create(int32_t m, const fh_plan_t* plans, const fh_peaks* peaks, int32_t* const* maps,
                                     fh_batch_t* out) {
  if (m < 1 || m >= kUnitAtomic || !plans || !peaks || !maps || !out) return FH_EINVAL;
  fh_batch_s* b = new (std::nothrow) fh_batch_s();
  if (!b) return FH_ENOMEM;
  b->m = m;
  int lds = 0, prep_lds = 0;
  double total = 0;
  bool any_windowed = false;
  // all whole-FFT maps: a kernel compiled for that mode alone, with the
  // work-group size the plans agree on (else 512 threads); otherwise both modes
  // with 256 threads
  bool all_whole = true, same_threads = true;
  for (int i = 0; i < m; ++i) {
    if (!plans[i]) {
      batch_free(b);
      return FH_EINVAL;
    }
    const fh_tile_cfg& t = reinterpret_cast<const fh_plan_s*>(plans[i])->p.tile;
    all_whole &= t.mode == kModeWhole;
    same_threads &= t.threads == reinterpret_cast<const fh_plan_s*>(plans[0])->p.tile.threads;
  }
  const int common = reinterpret_cast<const fh_plan_s*>(plans[0])->p.tile.threads;
  b->threads = all_whole ? (same_threads ? common : kBatchWholeThreads) : 256;
  b->mode = all_whole ? (int)kModeWhole : 0;
  for (int i = 0; i < m; ++i) {
    if (!plans[i] || !maps[i] || check_peaks(&peaks[i]) != FH_OK) {
      batch_free(b);
      return FH_EINVAL;
    }
    const Plan& p = reinterpret_cast<const fh_plan_s*>(plans[i])->p;
    MapArgs a = p.args(peaks[i], maps[i]);
    // one work-group size for the whole batch, A staged in LDS
    a.lds_bytes = lds_bytes_for_shape(a.n_f, a.rows, a.cols, 1, b->threads, &a.pitch);
    a.a_lds = 1;
    if (a.lds_bytes > kLdsBudget) {
      batch_free(b);
      return FH_ERANGE;
    }
    any_windowed |= a.mode == kModeWindowed;
    if (a.mode == kModeWindowed) prep_lds = std::max(prep_lds, prep_lds_bytes(a.n_words));
    b->plans.push_back(&p);
    b->peaks.push_back(peaks[i]);
    b->maps.push_back(maps[i]);
    b->args.push_back(a);
    lds = std::max(lds, a.lds_bytes);
    total += p.total_cost;
  }
  // units of all maps sized against the whole batch, longest first
  const int resident = occupancy_grid(b->threads, lds, 1 << 30, b->mode);
  const double target = total / (4.0 * std::max(resident, 1));
  std::vector<Unit> units;
  std::vector<double> cost;
  std::vector<int4> clears;
  for (int i = 0; i < m; ++i) split_units(*b->plans[i], i, target, units, cost, clears);
  std::vector<size_t> order(units.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
  std::vector<Unit> q(order.size());
  for (size_t i = 0; i < order.size(); ++i) q[i] = units[order[i]];
  if (q.empty() || q.size() >= (size_t)0x7fffffff) {
    batch_free(b);
    return FH_ERANGE;
  }
  b->n_queue = (int32_t)q.size();
  b->n_clears = (int32_t)clears.size();
  b->lds = lds;
  b->grid = std::max(1, std::min(resident, b->n_queue));
  {
    void *vm = nullptr, *vq = nullptr, *vc = nullptr, *vh = nullptr;
    fh_status st = device_alloc(&vm, sizeof(MapArgs) * m);
    b->d_maps = static_cast<MapArgs*>(vm);
    if (st == FH_OK) st = device_alloc(&vq, sizeof(Unit) * q.size());
    b->d_queue = static_cast<Unit*>(vq);
    if (st == FH_OK) st = device_alloc(&vc, sizeof(int4) * std::max<size_t>(1, clears.size()));
    b->d_clears = static_cast<int4*>(vc);
    if (st == FH_OK) st = device_alloc(&vh, sizeof(int32_t));
    b->d_head = static_cast<int32_t*>(vh);
    if (st != FH_OK) {
      batch_free(b);
      return st;
    }
  }
  if (hipMemcpy(b->d_maps, b->args.data(), sizeof(MapArgs) * m, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_queue, q.data(), sizeof(Unit) * q.size(), hipMemcpyHostToDevice) != hipSuccess ||
      (!clears.empty() &&
       hipMemcpy(b->d_clears, clears.data(), sizeof(int4) * clears.size(), hipMemcpyHostToDevice) != hipSuccess)) {
    batch_free(b);
    return FH_EDEVICE;
  }
  if (b->mode == kModeWhole) {
    if (b->threads == 1024) set_lds_attr<1024, true, kModeWhole>(lds);
    else if (b->threads == 512) set_lds_attr<512, true, kModeWhole>(lds);
    else set_lds_attr<256, true, kModeWhole>(lds);
  } else {
    set_lds_attr<256, true, 0>(lds);
  }
  // capture: prologue (queue head, error words, split tiles cleared), rank
  // structures of windowed maps, one persistent kernel
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    batch_free(b);
    return FH_EDEVICE;
  }
  MapArgs none{};
  bool ok = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(k_prologue, dim3((unsigned)std::max(1, std::min(b->n_clears, 1024)), kClearSplit), dim3(256), 0,
                       b->cap,
                       none, (const MapArgs*)b->d_maps, m, (const int4*)b->d_clears, b->n_clears, b->d_head);
    if (any_windowed)
      hipLaunchKernelGGL(k_prepare_batch, dim3(2048), dim3(kPrepWaves * 64), prep_lds, b->cap, b->d_maps, m);
    if (b->mode == kModeWhole && b->threads == 1024)
      hipLaunchKernelGGL((k_queue<1024, true, kModeWhole>), dim3(b->grid), dim3(1024), lds, b->cap, none,
                         (const MapArgs*)b->d_maps, (const Unit*)b->d_queue, b->n_queue, b->d_head);
    else if (b->mode == kModeWhole && b->threads == 512)
      hipLaunchKernelGGL((k_queue<512, true, kModeWhole>), dim3(b->grid), dim3(512), lds, b->cap, none,
                         (const MapArgs*)b->d_maps, (const Unit*)b->d_queue, b->n_queue, b->d_head);
    else if (b->mode == kModeWhole)
      hipLaunchKernelGGL((k_queue<256, true, kModeWhole>), dim3(b->grid), dim3(256), lds, b->cap, none,
                         (const MapArgs*)b->d_maps, (const Unit*)b->d_queue, b->n_queue, b->d_head);
    else
      hipLaunchKernelGGL((k_queue<256, true, 0>), dim3(b->grid), dim3(256), lds, b->cap, none,
                         (const MapArgs*)b->d_maps, (const Unit*)b->d_queue, b->n_queue, b->d_head);
    ok = hipStreamEndCapture(b->cap, &b->graph) == hipSuccess;
  }
  if (ok) ok = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
  if (ok && fake_device_error("graph")) ok = false;  // test hook: as if instantiation had failed
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
