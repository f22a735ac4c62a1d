// Tile CNN on Hough maps: proposes the 64 x 64 tiles of a map worth the
// plain candidate selection's attention.  Not part of the paper's method: its
// closing section only plans machine learning for the search; here a small
// network is trained on maps the method itself produces from synthetic
// injections, and the plain selection still decides.
//
// Network: tile (1 channel, counts normalised per map row) -> 4 x [conv 3x3,
// stride 1, zero padding, bias, ReLU] with 1 -> 16 -> 32 -> 64 -> 64 channels
// -> global average pool -> linear 64 -> 1 -> logistic.  60289 parameters.
//
// Numerics: activations, weights and activation gradients are BF16 (round to
// nearest even); every product sum accumulates in FP32.  conv2..conv4 and
// their backward passes are implicit GEMMs on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16 / 16x16x16); conv1 (one input channel) and the
// head are plain FP32 VALU code.  Master weights and Adam state are FP32.
//
// Layouts: activations NHWC [B][64][64][C] bf16; conv weights [Cout][9*Cin]
// with k = (dy*3 + dx)*Cin + ci; flat parameter vector (FP32) in the order
// w1, b1, w2, b2, w3, b3, w4, b4, w5, b5.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "fh_internal.h"

namespace fh {
namespace cnn {

constexpr int HW = 64;           // tile side
constexpr int NPIX = HW * HW;
constexpr int C1 = 16, C2 = 32, C3 = 64, C4 = 64;
constexpr int NW1 = C1 * 9, NW2 = C2 * 9 * C1, NW3 = C3 * 9 * C2, NW4 = C4 * 9 * C3;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NW1, OFF_W2 = OFF_B1 + C1, OFF_B2 = OFF_W2 + NW2;
constexpr int OFF_W3 = OFF_B2 + C2, OFF_B3 = OFF_W3 + NW3, OFF_W4 = OFF_B3 + C3, OFF_B4 = OFF_W4 + NW4;
constexpr int OFF_W5 = OFF_B4 + C4, OFF_B5 = OFF_W5 + C4, NPARAM = OFF_B5 + 1;
static_assert(NPARAM == 60289, "parameter count of the tile network");

typedef unsigned short bf16_t;
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef short s8 __attribute__((ext_vector_type(8)));

__host__ __device__ inline bf16_t f2bf(float f) {
  unsigned u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)(u >> 16);  // inf / nan kept
  u += 0x7fffu + ((u >> 16) & 1u);                                  // round to nearest even
  return (bf16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(bf16_t h) {
  unsigned u = (unsigned)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

template <int KW>
struct Frag;
template <>
struct Frag<16> {
  typedef s4 T;
};
template <>
struct Frag<32> {
  typedef s8 T;
};

template <int KW>
__device__ __forceinline__ f4 mfma(typename Frag<KW>::T a, typename Frag<KW>::T b, f4 c) {
  if constexpr (KW == 32)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------ conv (GEMM) --
// Implicit-GEMM 3x3 convolution on the matrix cores.  One work-group = 32
// output rows of one tile, in groups of kConvWaves rows (a wavefront per row:
// 4 pixel tiles of 16 x all output-channel tiles of 16).  The whole weight
// matrix is staged in LDS once per work-group, and for each group the input
// rows y0-1 .. y0+kConvWaves (with the zero border), all with 16-byte loads.
//   FWD:  out = bf16(relu(bias + conv(in, w)))
//   BWD:  out = bf16(conv(in, w) * (mask > 0))   (in = dY, w = flipped w^T,
//         mask = the forward input of the layer: the ReLU derivative)
// EPI (forward only): 0 stores out; 1 stores out and the row sums of every
// output channel, rowsum[b][y][co] = sum over x of out (the global pool's
// partial sums, added in a fixed order); 2 writes the row sums alone (the
// last layer when nothing needs its activations).
constexpr int kConvWaves = 8;       // output rows per group
constexpr int kConvRowsPerWG = 32;  // output rows per work-group

// LDS bank spreading.  A fragment's 16 lanes read 16 consecutive pixels of
// the staged input (stride CIN bf16) or 16 consecutive weight rows (stride K
// bf16) at the same offset; with those strides a multiple of 128 bytes they
// would all hit the same banks.  So the 16-byte chunks of a pixel (of a
// weight row) are stored permuted: chunk q at slot q ^ sw, sw taken from the
// pixel (row) index such that the 8 lanes of each 128 bytes land on distinct
// bank groups.
//   pixels: VPP chunks per pixel (a power of two <= 8): sw = (P / (8 / VPP)) % VPP
//   weight rows: K / 8 = GW * odd chunks per row, GW the largest power of two
//   dividing it (<= 8): sw = (co / (8 / GW)) % GW
template <int VPP>
__device__ __forceinline__ int pix_swz(int P) {
  static_assert(VPP == 1 || VPP == 2 || VPP == 4 || VPP == 8, "chunks per pixel");
  return VPP == 1 ? 0 : (P / (8 / VPP)) & (VPP - 1);
}
template <int K>
constexpr int row_group() {
  return (K / 8) % 8 == 0 ? 8 : (K / 8) % 4 == 0 ? 4 : (K / 8) % 2 == 0 ? 2 : 1;
}
template <int K>
__device__ __forceinline__ int row_swz(int co) {
  constexpr int GW = row_group<K>();
  return GW == 1 ? 0 : (co / (8 / GW)) & (GW - 1);
}

// dY of the last convolution, made from its activations where it is read:
// the head spreads dL/dpool[c] / NPIX evenly over the pixels and the ReLU
// passes it where the activation is positive.  a: 8 activations of one pixel,
// g: the BF16 gradients of the same 8 channels (per tile).
__device__ __forceinline__ uint4 head_dy(uint4 a, uint4 g) {
  auto two = [](unsigned x, unsigned gw) {
    const unsigned lo = __uint_as_float(x << 16) > 0.f ? (gw & 0xffffu) : 0u;
    const unsigned hi = __uint_as_float(x & 0xffff0000u) > 0.f ? (gw & 0xffff0000u) : 0u;
    return lo | hi;
  };
  return uint4{two(a.x, g.x), two(a.y, g.y), two(a.z, g.z), two(a.w, g.w)};
}

// HDY (data gradient of the last convolution): `in` holds its activations and
// `hdy` the head's per-(tile, channel) gradient; dY is head_dy of the two.
template <int CIN, int COUT, bool BWD, int EPI = 0, bool HDY = false>
__global__ void __launch_bounds__(kConvWaves * 64) k_conv(const bf16_t* __restrict__ in, const bf16_t* __restrict__ w,
                                                          const float* __restrict__ bias,
                                                          const bf16_t* __restrict__ mask, bf16_t* __restrict__ out,
                                                          float* __restrict__ rowsum, const bf16_t* __restrict__ hdy) {
  static_assert(!BWD || EPI == 0, "row sums of the forward output only");
  static_assert(!HDY || BWD, "dY from the head only in a data gradient");
  static_assert(CIN % 8 == 0 && (COUT * 9 * CIN) % 8 == 0 && HW % kConvRowsPerWG == 0 &&
                    kConvRowsPerWG % kConvWaves == 0, "conv layout");
  constexpr int K = 9 * CIN;
  constexpr int KW = (K % 32 == 0) ? 32 : 16;
  constexpr int NCT = COUT / 16;
  constexpr int ROWS = kConvWaves + 2, COLS = HW + 2;
  constexpr int NT = kConvWaves * 64;
  constexpr int VPP = CIN / 8;  // 16-byte vectors per pixel
  constexpr int PARTS = HW / kConvRowsPerWG;
  extern __shared__ __align__(16) unsigned char smem[];
  bf16_t* xin = reinterpret_cast<bf16_t*>(smem);  // [ROWS][COLS][CIN]
  bf16_t* wl = xin + ROWS * COLS * CIN;           // [COUT][K]
  const int b = blockIdx.x / PARTS;
  const int yb = (blockIdx.x % PARTS) * kConvRowsPerWG;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    const uint4* src = reinterpret_cast<const uint4*>(w);
    uint4* dst = reinterpret_cast<uint4*>(wl);
    constexpr int RC = K / 8;  // chunks per weight row
    for (int e = tid; e < COUT * RC; e += NT) {
      const int co = e / RC, kq = e - co * RC;
      dst[co * RC + (kq ^ row_swz<K>(co))] = src[e];
    }
  }
  const bf16_t* inb = in + (size_t)b * NPIX * CIN;
  bf16_t* ob = out + (size_t)b * NPIX * COUT;
  const int g = lane >> 4, m = lane & 15;
  constexpr int EL = KW / 4;  // bf16 per lane per fragment
  // A group's input rows are loaded into registers while the previous group
  // computes and written to LDS after it (SPT 16-byte chunks per thread), so
  // staging overlaps the MFMA work.  (The K loop below is unrolled by two
  // only: fully unrolled, the 64 -> 32 data gradient needed more registers
  // than a lane has with these chunks in flight.)
  constexpr int NCHUNK = ROWS * COLS * VPP;
  constexpr int SPT = (NCHUNK + NT - 1) / NT;
  uint4 pre[SPT];
  // a thread's chunks all hold the same 8 channels (NT is a multiple of VPP)
  static_assert(NT % VPP == 0, "one channel group per thread");
  uint4 hg = uint4{0u, 0u, 0u, 0u};
  if constexpr (HDY) hg = reinterpret_cast<const uint4*>(hdy + (size_t)b * CIN)[tid % VPP];
  auto chunk = [&](int y0, int e) {
    const int v = e % VPP, P = e / VPP, col = P % COLS, row = P / COLS;
    const int y = y0 - 1 + row, x = col - 1;
    uint4 val = uint4{0u, 0u, 0u, 0u};
    if (e < NCHUNK && y >= 0 && y < HW && x >= 0 && x < HW)
      val = reinterpret_cast<const uint4*>(inb + ((size_t)y * HW + x) * CIN)[v];
    return val;
  };
  // HDY: dY is formed here, when the chunk goes to LDS, so that a prefetched
  // load is not waited for early (head_dy of a zero chunk is zero)
  auto put = [&](int e, uint4 val) {
    const int v = e % VPP, P = e / VPP;
    if constexpr (HDY) val = head_dy(val, hg);
    reinterpret_cast<uint4*>(xin)[P * VPP + (v ^ pix_swz<VPP>(P))] = val;
  };
#pragma unroll
  for (int q = 0; q < SPT; ++q) pre[q] = chunk(yb, tid + q * NT);
  for (int y0 = yb; y0 < yb + kConvRowsPerWG; y0 += kConvWaves) {
    __syncthreads();  // the previous group is done with xin
#pragma unroll
    for (int q = 0; q < SPT; ++q)
      if (tid + q * NT < NCHUNK) put(tid + q * NT, pre[q]);
    __syncthreads();
    if (y0 + kConvWaves < yb + kConvRowsPerWG) {
#pragma unroll
      for (int q = 0; q < SPT; ++q) pre[q] = chunk(y0 + kConvWaves, tid + q * NT);
    }
    f4 acc[4][NCT];
#pragma unroll
    for (int pt = 0; pt < 4; ++pt)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[pt][ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int kc = 0; kc < K; kc += KW) {
      const int k = kc + g * EL;  // EL consecutive k inside one 16-byte chunk
      const int tap = k / CIN, ci = k % CIN;
      const int dy = tap / 3, dx = tap % 3;
      const int kq = k >> 3, kh = k & 7, cq = ci >> 3;
      typename Frag<KW>::T bf[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const int co = ct * 16 + m;
        bf[ct] = *reinterpret_cast<const typename Frag<KW>::T*>(wl + (co * (K / 8) + (kq ^ row_swz<K>(co))) * 8 + kh);
      }
#pragma unroll
      for (int pt = 0; pt < 4; ++pt) {
        const int P = (wave + dy) * COLS + (pt * 16 + m + dx);
        const typename Frag<KW>::T af =
            *reinterpret_cast<const typename Frag<KW>::T*>(xin + (P * VPP + (cq ^ pix_swz<VPP>(P))) * 8 + kh);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[pt][ct] = mfma<KW>(af, bf[ct], acc[pt][ct]);
      }
    }
    const int y = y0 + wave;
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int co = ct * 16 + m;
      float rs = 0.f;  // this lane's 16 pixels of channel co (EPI > 0)
#pragma unroll
      for (int pt = 0; pt < 4; ++pt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int x = pt * 16 + g * 4 + i;
          const size_t o = ((size_t)y * HW + x) * COUT + co;
          float v = acc[pt][ct][i];
          if (BWD) {
            v = bf2f(mask[(size_t)b * NPIX * COUT + o]) > 0.f ? v : 0.f;
          } else {
            v = fmaxf(v + bias[co], 0.f);
          }
          const bf16_t h = f2bf(v);
          if constexpr (EPI != 2) ob[o] = h;
          if constexpr (EPI != 0) rs += bf2f(h);
        }
      if constexpr (EPI != 0) {
        // the four lanes of channel co (g = 0..3) add their parts: (g0 + g1) + (g2 + g3)
        rs += __shfl_xor(rs, 16);
        rs += __shfl_xor(rs, 32);
        if (g == 0) rowsum[((size_t)b * HW + y) * COUT + co] = rs;
      }
    }
  }
}

template <int CIN, int COUT>
constexpr int conv_lds() {
  return ((kConvWaves + 2) * (HW + 2) * CIN + COUT * 9 * CIN) * 2;
}

// Weight gradient of a 3x3 convolution on the matrix cores: dW[co][k] +=
// sum over pixels of dY[p][co] * in_col[p][k].  Grid (tile, dx): a
// work-group takes one tile and the three taps of one column offset dx.  Per
// output row it uses dY transposed ([co][x]) and the input rows y-1..y+1
// shifted by dx and transposed (four [ci][x] slots of a ring, zero outside
// the tile; two output rows, so two new input rows, per step), so that every
// fragment is one aligned LDS read; the partial sums are added into dW
// (and, for dx = 0, dbias) with atomics at the end.  Each wavefront owns a
// quarter of the work-group's K tiles for every output-channel tile, so each
// fragment it loads feeds several MFMAs.  The transposed rows are 128 bytes
// (64 pixels) long; their 16-byte chunks sit at slot chunk ^ tsw(row), so
// that 16 consecutive rows read at one chunk, and the staging stores of rows
// 8 apart, spread over the banks.
__device__ __forceinline__ int tsw(int r) { return (r ^ (r >> 3)) & 7; }
__device__ __forceinline__ int tidx(int r, int x) {  // element (r, x) of a transposed [rows][64] array
  return r * HW + (((x >> 3) ^ tsw(r)) << 3) + (x & 7);
}

template <int CIN, int COUT, bool HDY = false>
__global__ void __launch_bounds__(256) k_conv_wgrad(const bf16_t* __restrict__ in, const bf16_t* __restrict__ dy,
                                                    float* __restrict__ dw, float* __restrict__ db,
                                                    const bf16_t* __restrict__ hdy) {
  static_assert(CIN % 16 == 0 && COUT % 8 == 0 && HW == 64, "16-byte staging of 8 channels, 128-byte rows, K tiles within a tap");
  constexpr int K = 9 * CIN;      // columns of dW
  constexpr int KX = 3 * CIN;     // this work-group's columns: taps (0, dx), (1, dx), (2, dx)
  constexpr int MT = COUT / 16, NT = KX / 16;
  static_assert(KX % 16 == 0, "K tiles of 16");
  constexpr int NTW = (NT + 3) / 4;  // K tiles per wavefront
  extern __shared__ __align__(16) unsigned char smem[];
  bf16_t* dyT = reinterpret_cast<bf16_t*>(smem);  // [2][COUT][HW]
  bf16_t* xT = dyT + 2 * COUT * HW;                // [4 slots][CIN][HW]
  const int b = blockIdx.x, ddx = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, m = lane & 15;
  const bf16_t* inb = in + (size_t)b * NPIX * CIN;
  const bf16_t* dyb = dy + (size_t)b * NPIX * COUT;
  f4 acc[MT][NTW];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < NTW; ++j) acc[mt][j] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;  // dbias partial (dx = 0): threads 4 co .. 4 co + 3 hold channel co, 16 pixels each
  // Two output rows per step.  Input rows live in a ring of four slots (row yy
  // in slot (yy + 4) % 4), so each step stages two new input rows and two dY
  // rows, all loaded into registers while the previous step's MFMAs run.  A thread takes two adjacent
  // pixels (or columns) x, x+1 (x even) and 8 channels: two 16-byte loads, the
  // pair of every channel stored as one aligned 32-bit word.
  constexpr int ND = (HW / 2) * (COUT / 8), NX = (HW / 2) * (CIN / 8);
  constexpr int PD = (ND + 255) / 256, PX = (NX + 255) / 256;
  uint4 rd[2][PD][2], rx[2][PX][2];
  // HDY: `dy` holds the last convolution's activations and `hdy` the head's
  // per-(tile, channel) gradient; a thread's dY chunks all hold the channels
  // (tid % (COUT / 8)) * 8 .. + 8 (256 is a multiple of COUT / 8)
  static_assert(256 % (COUT / 8) == 0, "one channel group per thread");
  uint4 hg = uint4{0u, 0u, 0u, 0u};
  if constexpr (HDY) hg = reinterpret_cast<const uint4*>(hdy + (size_t)b * COUT)[tid % (COUT / 8)];
  auto load_dy = [&](int y, int h) {
#pragma unroll
    for (int p = 0; p < PD; ++p) {
      const int e = tid + 256 * p;
      rd[h][p][0] = rd[h][p][1] = uint4{0u, 0u, 0u, 0u};
      if (e < ND && y < HW) {
        const int x = (e / (COUT / 8)) * 2, c8 = (e % (COUT / 8)) * 8;
        rd[h][p][0] = *reinterpret_cast<const uint4*>(dyb + ((size_t)y * HW + x) * COUT + c8);
        rd[h][p][1] = *reinterpret_cast<const uint4*>(dyb + ((size_t)y * HW + x + 1) * COUT + c8);
      }
    }
  };
  auto store_dy = [&](int h) {
    bf16_t* dT = dyT + h * COUT * HW;
#pragma unroll
    for (int p = 0; p < PD; ++p) {
      const int e = tid + 256 * p;
      if (e < ND) {
        if constexpr (HDY) {  // dY formed at the store, not at the (early) load; zero stays zero
          rd[h][p][0] = head_dy(rd[h][p][0], hg);
          rd[h][p][1] = head_dy(rd[h][p][1], hg);
        }
        const int x = (e / (COUT / 8)) * 2, c8 = (e % (COUT / 8)) * 8;
        const unsigned a[4] = {rd[h][p][0].x, rd[h][p][0].y, rd[h][p][0].z, rd[h][p][0].w};
        const unsigned c[4] = {rd[h][p][1].x, rd[h][p][1].y, rd[h][p][1].z, rd[h][p][1].w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          *reinterpret_cast<unsigned*>(dT + tidx(c8 + 2 * i, x)) = (a[i] & 0xffffu) | (c[i] << 16);
          *reinterpret_cast<unsigned*>(dT + tidx(c8 + 2 * i + 1, x)) = (a[i] >> 16) | (c[i] & 0xffff0000u);
        }
      }
    }
  };
  // input row yy shifted by dx: column x holds X[yy][x + dx - 1] (zero outside the tile)
  auto load_x = [&](int yy, int h) {
#pragma unroll
    for (int p = 0; p < PX; ++p) {
      const int e = tid + 256 * p;
      const int c8 = (e % (CIN / 8)) * 8, x = (e / (CIN / 8)) * 2;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int xx = x + ddx - 1 + q;
        rx[h][p][q] = uint4{0u, 0u, 0u, 0u};
        if (e < NX && yy >= 0 && yy < HW && xx >= 0 && xx < HW)
          rx[h][p][q] = *reinterpret_cast<const uint4*>(inb + ((size_t)yy * HW + xx) * CIN + c8);
      }
    }
  };
  auto store_x = [&](int yy, int h) {
    const int slot = (yy + 4) % 4;
#pragma unroll
    for (int p = 0; p < PX; ++p) {
      const int e = tid + 256 * p;
      if (e < NX) {
        const int c8 = (e % (CIN / 8)) * 8, x = (e / (CIN / 8)) * 2;
        const int r0 = slot * CIN + c8;
        const unsigned lo4[4] = {rx[h][p][0].x, rx[h][p][0].y, rx[h][p][0].z, rx[h][p][0].w};
        const unsigned hi4[4] = {rx[h][p][1].x, rx[h][p][1].y, rx[h][p][1].z, rx[h][p][1].w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const unsigned lo = lo4[i], hi = hi4[i];  // pixels x + dx - 1 and x + dx
          *reinterpret_cast<unsigned*>(xT + tidx(r0 + 2 * i, x)) = (lo & 0xffffu) | (hi << 16);
          *reinterpret_cast<unsigned*>(xT + tidx(r0 + 2 * i + 1, x)) = (lo >> 16) | (hi & 0xffff0000u);
        }
      }
    }
  };
  load_x(-1, 0);
  store_x(-1, 0);
  load_x(0, 0);
  store_x(0, 0);
  load_dy(0, 0);
  load_dy(1, 1);
  load_x(1, 0);
  load_x(2, 1);
  for (int y = 0; y < HW; y += 2) {
    __syncthreads();  // the previous rows' MFMAs are done with dyT and with the slots reused now
    store_dy(0);
    store_dy(1);
    store_x(y + 1, 0);
    store_x(y + 2, 1);
    __syncthreads();
    if (y + 2 < HW) {
      load_dy(y + 2, 0);
      load_dy(y + 3, 1);
      load_x(y + 3, 0);
      load_x(y + 4, 1);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bf16_t* dT = dyT + h * COUT * HW;
      if (ddx == 0 && tid < 4 * COUT) {
        const int co = tid >> 2;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const uint4 v = *reinterpret_cast<const uint4*>(dT + tidx(co, (tid & 3) * 16 + hh * 8));
          const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int i = 0; i < 4; ++i) bsum += __uint_as_float(w[i] << 16) + __uint_as_float(w[i] & 0xffff0000u);
        }
      }
      const int yo = y + h;
      for (int pc = 0; pc < HW; pc += 32) {  // 32 pixels per MFMA step
        const int x = pc + g * 8;
        s8 a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[mt] = *reinterpret_cast<const s8*>(dT + tidx(mt * 16 + m, x));
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
          const int nt = wave * NTW + j;
          if (nt < NT) {
            const int kx = nt * 16, ddy = kx / CIN;  // a K tile never spans two taps (CIN % 16 == 0)
            const int row = ((yo + ddy - 1 + 4) % 4) * CIN + (kx - ddy * CIN) + m;
            const s8 bb = *reinterpret_cast<const s8*>(xT + tidx(row, x));
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][j] = mfma<32>(a[mt], bb, acc[mt][j]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NTW; ++j) {
    const int nt = wave * NTW + j;
    if (nt < NT) {
      const int kx = nt * 16 + m, ddy = kx / CIN, ci = kx % CIN;
      const int k = (ddy * 3 + ddx) * CIN + ci;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) atomicAdd(&dw[(mt * 16 + g * 4 + i) * K + k], acc[mt][j][i]);
    }
  }
  if (ddx == 0) {
    bsum += __shfl_xor(bsum, 1);
    bsum += __shfl_xor(bsum, 2);
    if (tid < 4 * COUT && (tid & 3) == 0) atomicAdd(&db[tid >> 2], bsum);
  }
}

// ---------------------------------------------------------- conv1 (VALU) --
// w1r: the conv1 weights already rounded to BF16 (as FP32), then the FP32
// biases (pack_param); every thread reads them at the same addresses, so
// they come through the scalar cache.
__global__ void __launch_bounds__(256) k_conv1_fwd(const bf16_t* __restrict__ in, const float* __restrict__ w1r,
                                                   bf16_t* __restrict__ out, int B) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // one pixel
  if (t >= (long long)B * NPIX) return;
  const int b = (int)(t / NPIX), p = (int)(t % NPIX), y = p / HW, x = p % HW;
  float v[9];
  for (int tap = 0; tap < 9; ++tap) {
    const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
    v[tap] = (yy >= 0 && yy < HW && xx >= 0 && xx < HW) ? bf2f(in[(size_t)b * NPIX + yy * HW + xx]) : 0.f;
  }
  static_assert(C1 % 8 == 0, "16-byte stores of 8 channels");
  unsigned pk[C1 / 2];  // the pixel's C1 channels, packed in pairs
#pragma unroll
  for (int co = 0; co < C1; ++co) {
    float s = 0.f;
    for (int tap = 0; tap < 9; ++tap) s += w1r[co * 9 + tap] * v[tap];
    const unsigned h = f2bf(fmaxf(s + w1r[NW1 + co], 0.f));
    pk[co / 2] = (co & 1) ? (pk[co / 2] | (h << 16)) : h;
  }
  uint4* o = reinterpret_cast<uint4*>(out + (size_t)t * C1);
#pragma unroll
  for (int q = 0; q < C1 / 8; ++q) o[q] = uint4{pk[4 * q], pk[4 * q + 1], pk[4 * q + 2], pk[4 * q + 3]};
}

// dW1[co][tap] = sum_p dY1[p][co] * in[p + tap]; kConv1WgradParts work-groups
// per tile, each over a run of its pixels (two: 160 accumulators and two
// pixels' loads per thread fit two wavefronts per SIMD, so two work-groups
// share a CU; one work-group per tile with four pixels in flight took 42
// against 33 us per 256 tiles, four parts 47 us).
constexpr int kConv1WgradParts = 2;
__global__ void __launch_bounds__(256) k_conv1_wgrad(const bf16_t* __restrict__ in, const bf16_t* __restrict__ dy,
                                                     float* __restrict__ dw, float* __restrict__ db) {
  constexpr int NA = C1 * 9 + C1, PU = 2;  // accumulators per thread; pixels whose loads are in flight together
  constexpr int NP = NPIX / kConv1WgradParts;  // pixels of one work-group
  static_assert(C1 == 16 && NP % (256 * PU) == 0, "reduction layout: 16 channels, whole pixel steps");
  static_assert(C1 % 8 == 0, "16-byte loads of 8 channels");
  __shared__ float part[256][C1 + 1];
  __shared__ float part2[16][C1 + 1];
  const int b = blockIdx.x / kConv1WgradParts, pb = (blockIdx.x % kConv1WgradParts) * NP, tid = threadIdx.x;
  float acc[NA];
  for (int e = 0; e < NA; ++e) acc[e] = 0.f;
  for (int p0 = pb + tid; p0 < pb + NP; p0 += 256 * PU) {
    float v[PU][9];
    uint4 dq[PU][C1 / 8];
#pragma unroll
    for (int u = 0; u < PU; ++u) {  // every load of PU pixels before the first use
      const int p = p0 + 256 * u, y = p / HW, x = p % HW;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        v[u][tap] = (yy >= 0 && yy < HW && xx >= 0 && xx < HW) ? bf2f(in[(size_t)b * NPIX + yy * HW + xx]) : 0.f;
      }
#pragma unroll
      for (int q = 0; q < C1 / 8; ++q) dq[u][q] = reinterpret_cast<const uint4*>(dy + ((size_t)b * NPIX + p) * C1)[q];
    }
#pragma unroll
    for (int u = 0; u < PU; ++u)
#pragma unroll
      for (int q = 0; q < C1 / 8; ++q) {
        const unsigned wd[4] = {dq[u][q].x, dq[u][q].y, dq[u][q].z, dq[u][q].w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int co = 8 * q + e;
          const float d = bf2f((bf16_t)(wd[e >> 1] >> (16 * (e & 1))));
#pragma unroll
          for (int tap = 0; tap < 9; ++tap) acc[co * 9 + tap] += d * v[u][tap];
          acc[C1 * 9 + co] += d;
        }
      }
  }
  // per group of 16 accumulators: 256 partials -> 16 (each thread adds 16 rows of
  // one channel) -> 1 (16 threads), then one atomic per accumulator
  for (int e = 0; e < NA; e += C1) {
    for (int q = 0; q < C1; ++q) part[tid][q] = acc[e + q];
    __syncthreads();
    {
      const int q = tid & 15, r0 = (tid >> 4) * 16;
      float s = 0.f;
      for (int r = 0; r < 16; ++r) s += part[r0 + r][q];
      part2[tid >> 4][q] = s;
    }
    __syncthreads();
    if (tid < C1) {
      float s = 0.f;
      for (int r = 0; r < 16; ++r) s += part2[r][tid];
      const int idx = e + tid;
      if (idx < C1 * 9) atomicAdd(&dw[idx], s); else atomicAdd(&db[idx - C1 * 9], s);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ head --
// The head from the last layer's row sums: feat[b][c] = (sum over rows y in
// order of rowsum[b][y][c]) / NPIX; logit = b5 + sum over c in order of
// feat[c] w5[c].  One 64-thread work-group per tile.
__global__ void __launch_bounds__(C4) k_head_pool(const float* __restrict__ rowsum, const float* __restrict__ w5,
                                                  const float* __restrict__ b5, float* __restrict__ feat,
                                                  float* __restrict__ logit) {
  __shared__ float red[C4];
  const int b = blockIdx.x, t = threadIdx.x;
  const float* rb = rowsum + (size_t)b * HW * C4 + t;
  float f = 0.f;
  for (int y = 0; y < HW; ++y) f += rb[(size_t)y * C4];
  f *= 1.0f / NPIX;
  feat[b * C4 + t] = f;
  red[t] = f * w5[t];
  __syncthreads();
  if (t == 0) {
    float z = b5[0];
    for (int e = 0; e < C4; ++e) z += red[e];
    logit[b] = z;
  }
}

// Binary cross-entropy of the batch (mean) and the head's gradients.  One
// 64-thread work-group per tile, a thread per channel: dW5, db5 and the loss
// by atomics, and the gradient that the pool hands to every pixel of channel
// c, w5[c] dz / NPIX, rounded to BF16 (`hdy`).  The last convolution's
// backward kernels read it with the activations and apply the ReLU there
// (head_dy), so the per-pixel dY is never written out.
static_assert(C4 == 64, "a thread per channel in one wavefront");
__global__ void __launch_bounds__(C4) k_head_bwd(const float* __restrict__ feat, const float* __restrict__ logit,
                                                 const float* __restrict__ label, const float* __restrict__ w5,
                                                 float* __restrict__ dw5, float* __restrict__ db5,
                                                 float* __restrict__ loss, bf16_t* __restrict__ hdy, int B) {
  const int b = blockIdx.x, c = threadIdx.x;
  const float z = logit[b], yv = label[b];
  const float pr = 1.f / (1.f + expf(-z));
  const float dz = (pr - yv) / (float)B;
  atomicAdd(&dw5[c], dz * feat[b * C4 + c]);
  if (c == 0) {
    atomicAdd(db5, dz);
    // log(1 + e^-|z|) form of -[y log p + (1 - y) log(1 - p)]
    const float l = fmaxf(z, 0.f) - z * yv + log1pf(expf(-fabsf(z)));
    atomicAdd(loss, l / (float)B);
  }
  hdy[b * C4 + c] = f2bf(dz * w5[c] * (1.0f / NPIX));
}

// The copies of the parameters that the kernels read, made from the FP32
// master values: conv1's weights rounded to BF16 (kept as FP32) followed by
// its FP32 biases (w1r), and for conv2..conv4 the BF16 weights w ([Cout][9 Cin])
// and their flipped transpose wt ([Cin][9 Cout], k' = ((2-dy)*3 + (2-dx))*Cout
// + co), which the data gradient uses.  One parameter (flat index e, value v)
// at a time, so that the optimiser's update writes them as it goes.
struct PackDst {
  float* w1r;
  bf16_t *w2, *w2t, *w3, *w3t, *w4, *w4t;
};

__device__ __forceinline__ void pack_conv(int e, int cin, int cout, float v, bf16_t* w, bf16_t* wt) {
  const int co = e / (9 * cin), k = e % (9 * cin), tap = k / cin, ci = k % cin;
  const bf16_t h = f2bf(v);
  w[e] = h;
  wt[(size_t)ci * 9 * cout + (8 - tap) * cout + co] = h;
}

__device__ __forceinline__ void pack_param(const PackDst& d, int e, float v) {
  static_assert(OFF_W1 == 0 && OFF_B1 == NW1, "conv1's biases follow its weights at the start");
  if (e < OFF_B1) d.w1r[e] = bf2f(f2bf(v));
  else if (e < OFF_W2) d.w1r[e] = v;
  else if (e >= OFF_W2 && e < OFF_W2 + NW2) pack_conv(e - OFF_W2, C1, C2, v, d.w2, d.w2t);
  else if (e >= OFF_W3 && e < OFF_W3 + NW3) pack_conv(e - OFF_W3, C2, C3, v, d.w3, d.w3t);
  else if (e >= OFF_W4 && e < OFF_W4 + NW4) pack_conv(e - OFF_W4, C3, C4, v, d.w4, d.w4t);
}

__global__ void k_pack(const float* __restrict__ p, PackDst d) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < NPARAM) pack_param(d, e, p[e]);
}

// ------------------------------------------------------------- optimiser --
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, int n, float lr, float b1, float b2, float eps, float c1, float c2,
                       PackDst d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  const float pi = p[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
  p[i] = pi;
  pack_param(d, i, pi);  // the kernels' copies of the updated parameter
}

// ---------------------------------------------------------- tile inputs --
// Per map row: mean and 1/std of the counts over the whole row (exact int64
// sums, FP64 statistics).
__global__ void __launch_bounds__(256) k_row_stats(const int32_t* __restrict__ map, int n_x0, float* __restrict__ mean,
                                                   float* __restrict__ istd) {
  __shared__ long long s1[256], s2[256];
  const int r = blockIdx.x;
  long long a = 0, q = 0;
  for (int c = threadIdx.x; c < n_x0; c += 256) {
    const long long v = map[(size_t)r * n_x0 + c];
    a += v;
    q += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = q;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mu = (double)s1[0] / n_x0;
    const double var = (double)s2[0] / n_x0 - mu * mu;
    mean[r] = (float)mu;
    istd[r] = var > 0 ? (float)(1.0 / sqrt(var)) : 0.f;
  }
}

// tiles[t][y][x] = bf16((map[r0+y][c0+x] - mean[r0+y]) * istd[r0+y]), zero outside the map
__global__ void __launch_bounds__(256) k_gather(const int32_t* __restrict__ map, int n_k, int n_x0,
                                                const float* __restrict__ mean, const float* __restrict__ istd,
                                                const int2* __restrict__ origin, bf16_t* __restrict__ tiles) {
  const int t = blockIdx.x;
  const int2 o = origin[t];
  for (int e = threadIdx.x; e < NPIX; e += 256) {
    const int y = e / HW, x = e % HW, r = o.x + y, c = o.y + x;
    float v = 0.f;
    if (r >= 0 && r < n_k && c >= 0 && c < n_x0) v = ((float)map[(size_t)r * n_x0 + c] - mean[r]) * istd[r];
    tiles[(size_t)t * NPIX + e] = f2bf(v);
  }
}

// Batched proposals: one map of the batch.  Its rows are global rows [row0,
// row0 + n_k) of the row statistics, its tiles global tiles [tile0, tile0 +
// ta * tb), tile l at origin ((l / tb) * HW, (l % tb) * HW).
struct PMap {
  const int32_t* map;
  int32_t n_k, n_x0, tb;
  int32_t row0, tile0;
};

template <typename F>
__device__ __forceinline__ int find_pmap(const PMap* maps, int m, int g, F first) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(maps[mid]) <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Row statistics of every map of the batch: one work-group per global row.
__global__ void __launch_bounds__(256) k_row_stats_batch(const PMap* __restrict__ maps, int m,
                                                         float* __restrict__ mean, float* __restrict__ istd) {
  const int g = blockIdx.x;
  const PMap M = maps[find_pmap(maps, m, g, [](const PMap& x) { return x.row0; })];
  const int r = g - M.row0;
  __shared__ long long s1[256], s2[256];
  long long a = 0, q = 0;
  for (int c = threadIdx.x; c < M.n_x0; c += 256) {
    const long long v = M.map[(size_t)r * M.n_x0 + c];
    a += v;
    q += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = q;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mu = (double)s1[0] / M.n_x0;
    const double var = (double)s2[0] / M.n_x0 - mu * mu;
    mean[g] = (float)mu;
    istd[g] = var > 0 ? (float)(1.0 / sqrt(var)) : 0.f;
  }
}

// Tiles t0 .. t0 + gridDim.x - 1 of the batch (global tile indices), as k_gather.
__global__ void __launch_bounds__(256) k_gather_batch(const PMap* __restrict__ maps, int m, int t0,
                                                      const float* __restrict__ mean, const float* __restrict__ istd,
                                                      bf16_t* __restrict__ tiles) {
  const int g = t0 + blockIdx.x;
  const PMap M = maps[find_pmap(maps, m, g, [](const PMap& x) { return x.tile0; })];
  const int l = g - M.tile0;
  const int r0 = (l / M.tb) * HW, c0 = (l % M.tb) * HW;
  for (int e = threadIdx.x; e < NPIX; e += 256) {
    const int y = e / HW, x = e % HW, r = r0 + y, c = c0 + x;
    float v = 0.f;
    if (r < M.n_k && c < M.n_x0)
      v = ((float)M.map[(size_t)r * M.n_x0 + c] - mean[M.row0 + r]) * istd[M.row0 + r];
    tiles[(size_t)blockIdx.x * NPIX + e] = f2bf(v);
  }
}

}  // namespace cnn
}  // namespace fh

// ===================================================================== ABI ==
using namespace fh::cnn;

struct fh_cnn_s {
  int max_batch = 0;
  float *params = nullptr, *grads = nullptr, *m1 = nullptr, *m2 = nullptr;
  float* w1r = nullptr;  // conv1 weights rounded to BF16, then its biases
  bf16_t *w2 = nullptr, *w3 = nullptr, *w4 = nullptr, *w2t = nullptr, *w3t = nullptr, *w4t = nullptr;
  bf16_t *x = nullptr, *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *a4 = nullptr;  // activations
  bf16_t *d1 = nullptr, *d2 = nullptr, *d3 = nullptr;  // activation gradients
  bf16_t* hdy = nullptr;  // [max_batch][C4]: the head's gradient per tile and channel
  float *feat = nullptr, *logit = nullptr, *loss = nullptr;
  float* rowsum = nullptr;  // [max_batch][64][64]: the last layer's row sums per channel
  float *row_mean = nullptr, *row_istd = nullptr;
  int row_cap = 0;
  int2* origins = nullptr;
  PMap* ptab = nullptr;  // batched proposals: the map table
  int ptab_cap = 0;
  int steps = 0;
  int last_batch = 0;
};

namespace {

template <typename T>
bool dalloc(T** p, size_t n) {
  void* v = nullptr;
  const bool ok = fh::device_alloc(&v, sizeof(T) * (n ? n : 1)) == FH_OK;
  *p = static_cast<T*>(v);
  return ok;
}

void cnn_free(fh_cnn_s* c) {
  if (!c) return;
  void* ptrs[] = {c->params, c->grads, c->m1,  c->m2,   c->w1r, c->w2,    c->w3,    c->w4, c->w2t, c->w3t, c->w4t, c->x,
                  c->a1,     c->a2,    c->a3,  c->a4,   c->d1,    c->d2,    c->d3, c->hdy, c->feat, c->logit,
                  c->loss,   c->row_mean, c->row_istd, c->origins, c->ptab, c->rowsum};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
}

template <int CIN, int COUT, bool BWD, int EPI = 0, bool HDY = false>
fh_status launch_conv(const bf16_t* in, const bf16_t* w, const float* bias, const bf16_t* mask, bf16_t* out, int B,
                      hipStream_t s, float* rowsum = nullptr, const bf16_t* hdy = nullptr) {
  constexpr int lds = conv_lds<CIN, COUT>();
  (void)hipFuncSetAttribute((const void*)k_conv<CIN, COUT, BWD, EPI, HDY>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds);
  static_assert(lds <= 160 * 1024, "conv LDS");
  hipLaunchKernelGGL((k_conv<CIN, COUT, BWD, EPI, HDY>), dim3(B * (HW / kConvRowsPerWG)), dim3(kConvWaves * 64), lds,
                     s, in, w, bias, mask, out, rowsum, hdy);
  return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE;
}

// LDS of one weight-gradient work-group: two transposed dY rows and four input-row slots.
template <int CIN, int COUT>
constexpr int wgrad_lds() {
  return (2 * COUT + 4 * CIN) * HW * 2;
}

template <int CIN, int COUT, bool HDY = false>
fh_status launch_wgrad(const bf16_t* in, const bf16_t* dy, float* dw, float* db, int B, hipStream_t s,
                       const bf16_t* hdy = nullptr) {
  constexpr int lds = wgrad_lds<CIN, COUT>();
  (void)hipFuncSetAttribute((const void*)k_conv_wgrad<CIN, COUT, HDY>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds);
  hipLaunchKernelGGL((k_conv_wgrad<CIN, COUT, HDY>), dim3(B, 3), dim3(256), lds, s, in, dy, dw, db, hdy);
  return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE;
}

PackDst pack_dst(const fh_cnn_s* c) { return PackDst{c->w1r, c->w2, c->w2t, c->w3, c->w3t, c->w4, c->w4t}; }

fh_status pack(fh_cnn_s* c, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3((NPARAM + 255) / 256), dim3(256), 0, s, c->params, pack_dst(c));
  return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE;
}

}  // namespace

extern "C" fh_status fh_cnn_create(int32_t max_batch, fh_cnn_t* out) {
  if (max_batch < 1 || max_batch > 65536 || !out) return FH_EINVAL;
  fh_cnn_s* c = new (std::nothrow) fh_cnn_s();
  if (!c) return FH_ENOMEM;
  c->max_batch = max_batch;
  const size_t P = (size_t)max_batch * NPIX;
  bool ok = dalloc(&c->params, NPARAM) && dalloc(&c->grads, NPARAM) && dalloc(&c->m1, NPARAM) &&
            dalloc(&c->m2, NPARAM) && dalloc(&c->w1r, NW1 + C1) && dalloc(&c->w2, NW2) && dalloc(&c->w3, NW3) && dalloc(&c->w4, NW4) &&
            dalloc(&c->w2t, NW2) && dalloc(&c->w3t, NW3) && dalloc(&c->w4t, NW4) && dalloc(&c->x, P) &&
            dalloc(&c->a1, P * C1) && dalloc(&c->a2, P * C2) && dalloc(&c->a3, P * C3) && dalloc(&c->a4, P * C4) &&
            dalloc(&c->d1, P * C1) && dalloc(&c->d2, P * C2) && dalloc(&c->d3, P * C3) &&
            dalloc(&c->hdy, (size_t)max_batch * C4) &&
            dalloc(&c->feat, (size_t)max_batch * C4) && dalloc(&c->logit, max_batch) && dalloc(&c->loss, 1) &&
            dalloc(&c->rowsum, (size_t)max_batch * HW * C4) &&
            dalloc(&c->origins, max_batch);
  if (!ok) {
    cnn_free(c);
    return FH_ENOMEM;
  }
  if (hipMemset(c->params, 0, NPARAM * 4) != hipSuccess || hipMemset(c->m1, 0, NPARAM * 4) != hipSuccess ||
      hipMemset(c->m2, 0, NPARAM * 4) != hipSuccess || hipMemset(c->grads, 0, NPARAM * 4) != hipSuccess ||
      pack(c, nullptr) != FH_OK || hipDeviceSynchronize() != hipSuccess) {
    cnn_free(c);
    return FH_EDEVICE;
  }
  *out = reinterpret_cast<fh_cnn_t>(c);
  return FH_OK;
}

extern "C" void fh_cnn_destroy(fh_cnn_t h) { cnn_free(reinterpret_cast<fh_cnn_s*>(h)); }

extern "C" int64_t fh_cnn_num_params(void) { return NPARAM; }

extern "C" fh_status fh_cnn_set_params(fh_cnn_t h, const float* host, int64_t n) {
  if (!h || !host || n != NPARAM) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  if (hipMemcpy(c->params, host, NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess) return FH_EDEVICE;
  if (hipMemset(c->m1, 0, NPARAM * 4) != hipSuccess || hipMemset(c->m2, 0, NPARAM * 4) != hipSuccess)
    return FH_EDEVICE;
  c->steps = 0;
  if (pack(c, nullptr) != FH_OK || hipDeviceSynchronize() != hipSuccess) return FH_EDEVICE;
  return FH_OK;
}

extern "C" fh_status fh_cnn_get_params(fh_cnn_t h, float* host, float* grads_host, int64_t n) {
  if (!h || n != NPARAM) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  if (hipDeviceSynchronize() != hipSuccess) return FH_EDEVICE;
  if (host && hipMemcpy(host, c->params, NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess) return FH_EDEVICE;
  if (grads_host && hipMemcpy(grads_host, c->grads, NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return FH_EDEVICE;
  return FH_OK;
}

extern "C" fh_status fh_cnn_set_grads(fh_cnn_t h, const float* grads_host, int64_t n) {
  if (!h || !grads_host || n != NPARAM) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  if (hipDeviceSynchronize() != hipSuccess) return FH_EDEVICE;
  return hipMemcpy(c->grads, grads_host, NPARAM * 4, hipMemcpyHostToDevice) == hipSuccess ? FH_OK : FH_EDEVICE;
}

extern "C" fh_status fh_cnn_get_state(fh_cnn_t h, float* m1_host, float* m2_host, int64_t n, int64_t* steps) {
  if (!h || n != NPARAM) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  if (hipDeviceSynchronize() != hipSuccess) return FH_EDEVICE;
  if (m1_host && hipMemcpy(m1_host, c->m1, NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess) return FH_EDEVICE;
  if (m2_host && hipMemcpy(m2_host, c->m2, NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess) return FH_EDEVICE;
  if (steps) *steps = c->steps;
  return FH_OK;
}

extern "C" fh_status fh_cnn_set_state(fh_cnn_t h, const float* m1_host, const float* m2_host, int64_t n,
                                      int64_t steps) {
  if (!h || !m1_host || !m2_host || n != NPARAM || steps < 0 || steps > INT32_MAX) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  if (hipDeviceSynchronize() != hipSuccess) return FH_EDEVICE;
  if (hipMemcpy(c->m1, m1_host, NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->m2, m2_host, NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess)
    return FH_EDEVICE;
  c->steps = (int)steps;
  return FH_OK;
}

extern "C" fh_status fh_cnn_activations(fh_cnn_t h, int32_t layer, uint16_t* out_host, int64_t n) {
  if (!h || !out_host || layer < 0 || layer > 4) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  if (c->last_batch < 1) return FH_EINVAL;
  const int ch[5] = {1, C1, C2, C3, C4};
  const bf16_t* src[5] = {c->x, c->a1, c->a2, c->a3, c->a4};
  const int64_t want = (int64_t)c->last_batch * NPIX * ch[layer];
  if (n != want) return FH_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return FH_EDEVICE;
  return hipMemcpy(out_host, src[layer], (size_t)want * 2, hipMemcpyDeviceToHost) == hipSuccess ? FH_OK : FH_EDEVICE;
}

extern "C" fh_status fh_cnn_forward(fh_cnn_t h, const uint16_t* tiles, int32_t B, float* logits, void* stream) {
  if (!h || !tiles || B < 1) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  if (B > c->max_batch) return FH_ERANGE;
  hipStream_t s = (hipStream_t)stream;
  if (tiles != c->x &&
      hipMemcpyAsync(c->x, tiles, (size_t)B * NPIX * 2, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return FH_EDEVICE;
  const long long npx = (long long)B * NPIX;
  hipLaunchKernelGGL(k_conv1_fwd, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, s, c->x, c->w1r, c->a1, B);
  fh_status st = launch_conv<C1, C2, false>(c->a1, c->w2, c->params + OFF_B2, nullptr, c->a2, B, s);
  if (st == FH_OK) st = launch_conv<C2, C3, false>(c->a2, c->w3, c->params + OFF_B3, nullptr, c->a3, B, s);
  if (st == FH_OK)
    st = launch_conv<C3, C4, false, 1>(c->a3, c->w4, c->params + OFF_B4, nullptr, c->a4, B, s, c->rowsum);
  if (st != FH_OK) return st;
  hipLaunchKernelGGL(k_head_pool, dim3(B), dim3(C4), 0, s, c->rowsum, c->params + OFF_W5, c->params + OFF_B5, c->feat,
                     c->logit);
  if (logits && hipMemcpyAsync(logits, c->logit, (size_t)B * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return FH_EDEVICE;
  c->last_batch = B;
  return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE;
}


namespace {
// The forward for proposals: the same layers and the same logits as
// fh_cnn_forward, but the last layer writes only its row sums (nothing will
// take a gradient), so its 512 KB of activations per tile are neither stored
// nor read back.  No backward may follow: the network's last batch is reset.
fh_status forward_scores(fh_cnn_s* c, int B, float* logits, hipStream_t s) {
  const long long npx = (long long)B * NPIX;
  hipLaunchKernelGGL(k_conv1_fwd, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, s, c->x, c->w1r, c->a1, B);
  fh_status st = launch_conv<C1, C2, false>(c->a1, c->w2, c->params + OFF_B2, nullptr, c->a2, B, s);
  if (st == FH_OK) st = launch_conv<C2, C3, false>(c->a2, c->w3, c->params + OFF_B3, nullptr, c->a3, B, s);
  if (st == FH_OK)
    st = launch_conv<C3, C4, false, 2>(c->a3, c->w4, c->params + OFF_B4, nullptr, nullptr, B, s, c->rowsum);
  if (st != FH_OK) return st;
  hipLaunchKernelGGL(k_head_pool, dim3(B), dim3(C4), 0, s, c->rowsum, c->params + OFF_W5, c->params + OFF_B5, c->feat,
                     logits);
  c->last_batch = 0;
  return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE;
}
}  // namespace

extern "C" fh_status fh_cnn_scores(fh_cnn_t h, const uint16_t* tiles, int32_t B, float* logits, void* stream) {
  if (!h || !tiles || !logits || B < 1) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  if (B > c->max_batch) return FH_ERANGE;
  hipStream_t s = (hipStream_t)stream;
  if (tiles != c->x &&
      hipMemcpyAsync(c->x, tiles, (size_t)B * NPIX * 2, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return FH_EDEVICE;
  return forward_scores(c, B, logits, s);
}

extern "C" fh_status fh_cnn_backward(fh_cnn_t h, const float* labels, int32_t B, float* loss, void* stream) {
  if (!h || !labels || B < 1) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  if (B != c->last_batch) return FH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemsetAsync(c->grads, 0, NPARAM * 4, s) != hipSuccess || hipMemsetAsync(c->loss, 0, 4, s) != hipSuccess)
    return FH_EDEVICE;
  hipLaunchKernelGGL(k_head_bwd, dim3(B), dim3(C4), 0, s, c->feat, c->logit, labels, c->params + OFF_W5,
                     c->grads + OFF_W5, c->grads + OFF_B5, c->loss, c->hdy, B);
  // the last convolution's dY: from its activations a4 and the head's gradient
  fh_status st = launch_wgrad<C3, C4, true>(c->a3, c->a4, c->grads + OFF_W4, c->grads + OFF_B4, B, s, c->hdy);
  if (st == FH_OK) st = launch_conv<C4, C3, true, 0, true>(c->a4, c->w4t, nullptr, c->a3, c->d3, B, s, nullptr, c->hdy);
  if (st == FH_OK) st = launch_wgrad<C2, C3>(c->a2, c->d3, c->grads + OFF_W3, c->grads + OFF_B3, B, s);
  if (st == FH_OK) st = launch_conv<C3, C2, true>(c->d3, c->w3t, nullptr, c->a2, c->d2, B, s);
  if (st == FH_OK) st = launch_wgrad<C1, C2>(c->a1, c->d2, c->grads + OFF_W2, c->grads + OFF_B2, B, s);
  if (st == FH_OK) st = launch_conv<C2, C1, true>(c->d2, c->w2t, nullptr, c->a1, c->d1, B, s);
  if (st != FH_OK) return st;
  hipLaunchKernelGGL(k_conv1_wgrad, dim3(B * kConv1WgradParts), dim3(256), 0, s, c->x, c->d1, c->grads + OFF_W1,
                     c->grads + OFF_B1);
  if (loss && hipMemcpyAsync(loss, c->loss, 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return FH_EDEVICE;
  return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE;
}

extern "C" fh_status fh_cnn_step(fh_cnn_t h, float lr, void* stream) {
  if (!h || !(lr >= 0.f)) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  hipStream_t s = (hipStream_t)stream;
  c->steps += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)c->steps), c2 = 1.f - std::pow(b2, (float)c->steps);
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, c->params, c->grads, c->m1, c->m2, NPARAM,
                     lr, b1, b2, 1e-8f, c1, c2, pack_dst(c));
  return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE;
}

extern "C" fh_status fh_tiles(const int32_t* map, int32_t n_k, int32_t n_x0, const int32_t* origins, int32_t n_tiles,
                              uint16_t* tiles, float* row_mean, float* row_istd, void* stream) {
  if (!map || !origins || !tiles || !row_mean || !row_istd || n_k < 1 || n_x0 < 1 || n_tiles < 0) return FH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_row_stats, dim3(n_k), dim3(256), 0, s, map, n_x0, row_mean, row_istd);
  if (n_tiles > 0)
    hipLaunchKernelGGL(k_gather, dim3(n_tiles), dim3(256), 0, s, map, n_k, n_x0, row_mean, row_istd,
                       reinterpret_cast<const int2*>(origins), tiles);
  return hipGetLastError() == hipSuccess ? FH_OK : FH_EDEVICE;
}

extern "C" fh_status fh_propose(fh_cnn_t h, fh_plan_t ph, const int32_t* map, float* scores, int32_t n_top,
                                int32_t* tile_ids, void* stream) {
  if (!h || !ph || !map || !scores || n_top < 0 || (n_top > 0 && !tile_ids)) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  const fh::Plan& p = reinterpret_cast<const fh::Plan&>(*ph);
  const int n_k = p.desc.n_k, n_x0 = p.n_x0;
  const int ta = (n_k + HW - 1) / HW, tb = (n_x0 + HW - 1) / HW;
  const int n_tiles = ta * tb;
  if (n_top > n_tiles) return FH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (c->row_cap < n_k) {
    if (c->row_mean) (void)hipFree(c->row_mean);
    if (c->row_istd) (void)hipFree(c->row_istd);
    c->row_mean = c->row_istd = nullptr;
    c->row_cap = 0;
    if (!dalloc(&c->row_mean, n_k) || !dalloc(&c->row_istd, n_k)) return FH_ENOMEM;
    c->row_cap = n_k;
  }
  std::vector<int2> org(n_tiles);
  for (int a = 0; a < ta; ++a)
    for (int b = 0; b < tb; ++b) org[(size_t)a * tb + b] = make_int2(a * HW, b * HW);
  hipLaunchKernelGGL(k_row_stats, dim3(n_k), dim3(256), 0, s, map, n_x0, c->row_mean, c->row_istd);
  for (int t0 = 0; t0 < n_tiles; t0 += c->max_batch) {
    const int B = std::min(c->max_batch, n_tiles - t0);
    if (hipMemcpyAsync(c->origins, org.data() + t0, sizeof(int2) * B, hipMemcpyHostToDevice, s) != hipSuccess)
      return FH_EDEVICE;
    hipLaunchKernelGGL(k_gather, dim3(B), dim3(256), 0, s, map, n_k, n_x0, c->row_mean, c->row_istd, c->origins,
                       c->x);
    // the network reads its input buffer in place
    fh_status st = forward_scores(c, B, scores + t0, s);
    if (st != FH_OK) return st;
    // the origins buffer is reused by the next batch: finish this one first
    if (hipStreamSynchronize(s) != hipSuccess) return FH_EDEVICE;
  }
  std::vector<float> sc(n_tiles);
  if (hipMemcpyAsync(sc.data(), scores, sizeof(float) * n_tiles, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FH_EDEVICE;
  std::vector<int32_t> idx(n_tiles);
  for (int i = 0; i < n_tiles; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return sc[x] > sc[y]; });
  for (int i = 0; i < n_top; ++i) tile_ids[i] = idx[i];
  return FH_OK;
}

extern "C" fh_status fh_batch_propose(fh_cnn_t h, fh_batch_t b, float* scores, const int32_t* n_top,
                                      int32_t* tile_ids, void* stream) {
  if (!h || !b || !scores || !n_top) return FH_EINVAL;
  fh_cnn_s* c = reinterpret_cast<fh_cnn_s*>(h);
  const int m = b->m;
  std::vector<PMap> tab(m);
  long long rows = 0, tiles = 0, picks = 0;
  for (int i = 0; i < m; ++i) {
    const fh::Plan& p = *b->plans[i];
    const int n_k = p.desc.n_k, n_x0 = p.n_x0;
    const int ta = (n_k + HW - 1) / HW, tb = (n_x0 + HW - 1) / HW;
    if (n_top[i] < 0 || n_top[i] > ta * tb) return FH_EINVAL;
    tab[i] = PMap{b->maps[i], n_k, n_x0, tb, (int32_t)rows, (int32_t)tiles};
    rows += n_k;
    tiles += (long long)ta * tb;
    picks += n_top[i];
  }
  if (rows >= (1LL << 31) || tiles >= (1LL << 31)) return FH_ERANGE;
  if (picks > 0 && !tile_ids) return FH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (c->row_cap < rows) {
    if (c->row_mean) (void)hipFree(c->row_mean);
    if (c->row_istd) (void)hipFree(c->row_istd);
    c->row_mean = c->row_istd = nullptr;
    c->row_cap = 0;
    if (!dalloc(&c->row_mean, (size_t)rows) || !dalloc(&c->row_istd, (size_t)rows)) return FH_ENOMEM;
    c->row_cap = (int)rows;
  }
  if (c->ptab_cap < m) {
    if (c->ptab) (void)hipFree(c->ptab);
    c->ptab = nullptr;
    c->ptab_cap = 0;
    if (!dalloc(&c->ptab, (size_t)m)) return FH_ENOMEM;
    c->ptab_cap = m;
  }
  if (hipMemcpyAsync(c->ptab, tab.data(), sizeof(PMap) * m, hipMemcpyHostToDevice, s) != hipSuccess)
    return FH_EDEVICE;
  hipLaunchKernelGGL(k_row_stats_batch, dim3((unsigned)rows), dim3(256), 0, s, c->ptab, m, c->row_mean, c->row_istd);
  // chunks of the network's batch; every step is ordered on `stream`
  for (long long t0 = 0; t0 < tiles; t0 += c->max_batch) {
    const int B = (int)std::min<long long>(c->max_batch, tiles - t0);
    hipLaunchKernelGGL(k_gather_batch, dim3(B), dim3(256), 0, s, c->ptab, m, (int)t0, c->row_mean, c->row_istd, c->x);
    const fh_status st = forward_scores(c, B, scores + t0, s);
    if (st != FH_OK) return st;
  }
  std::vector<float> sc((size_t)tiles);
  if (hipMemcpyAsync(sc.data(), scores, sizeof(float) * (size_t)tiles, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FH_EDEVICE;
  long long at = 0;
  std::vector<int32_t> idx;
  for (int i = 0; i < m; ++i) {
    const int n = (int)((i + 1 < m ? tab[i + 1].tile0 : tiles) - tab[i].tile0);
    const float* si = sc.data() + tab[i].tile0;
    idx.resize(n);
    for (int k = 0; k < n; ++k) idx[k] = k;
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return si[x] > si[y]; });
    for (int k = 0; k < n_top[i]; ++k) tile_ids[at + k] = idx[k];
    at += n_top[i];
  }
  return FH_OK;
}
