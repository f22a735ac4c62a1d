// Measured ceilings of the gfx950 units the library's kernels lean on, so
// that their rooflines can be read against what the chip delivers as well as
// against its data-sheet peaks:
//   - FP64 fma, and fma + v_cvt_i32_f64 pairs (the transform's index math);
//   - LDS 32-bit atomic adds without return: consecutive words, a random
//     scatter (the pattern of the tile kernel's edge updates) and a stride of
//     32 words (every lane on one bank);
//   - HBM: read-only streaming, a copy, and a store;
//   - dense BF16 matrix cores (v_mfma_f32_16x16x32_bf16, the CNN's instruction);
//   - VALU issue: independent 32-bit integer adds, one wave instruction each.
// Every loop has a fixed trip count and every index is masked into its
// buffer.  Prints one JSON object per line.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#define CK(x)                                                                  \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      std::printf("{\"error\":\"%s\",\"line\":%d}\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                                \
    }                                                                          \
  } while (0)

constexpr int kIters = 4096;
constexpr int kLdsWords = 16384;  // 64 KB of LDS per work-group

__global__ void __launch_bounds__(256) k_fma(double* out, double b, double c) {
  double a[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) a[q] = threadIdx.x + q;
  for (int i = 0; i < kIters; ++i)
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = __builtin_fma(a[q], b, c);
  double s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += a[q];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_fma_cvt(int* out, double b, double c) {
  double a[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) a[q] = threadIdx.x + q;
  int s = 0;
  for (int i = 0; i < kIters; ++i)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      a[q] = __builtin_fma(a[q], b, c);
      s ^= (int)a[q];
    }
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Eight independent chains of v_add_u32 per lane (written as instructions so
// that the count is exact): the VALU issue rate with every operand ready.
__global__ void __launch_bounds__(256) k_valu(unsigned* out, unsigned b) {
  unsigned a[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) a[q] = threadIdx.x + q;
  for (int i = 0; i < kIters; ++i)
#pragma unroll
    for (int q = 0; q < 8; ++q) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[q]) : "v"(b));
  unsigned s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s ^= a[q];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// MODE 0: lane t adds to word t + 64 i; 1: a random word per add (LCG per
// lane); 2: word 32 t + i, all 64 lanes on one bank.
template <int MODE>
__global__ void __launch_bounds__(256) k_lds_atomic(unsigned* out) {
  __shared__ unsigned buf[kLdsWords];
  for (int i = threadIdx.x; i < kLdsWords; i += blockDim.x) buf[i] = 0;
  __syncthreads();
  const unsigned t = threadIdx.x;
  unsigned h = t * 2654435761u + blockIdx.x;
  for (int i = 0; i < kIters; ++i) {
    unsigned idx;
    if (MODE == 0) {
      idx = (t + (unsigned)i * 64u) & (kLdsWords - 1);
    } else if (MODE == 1) {
      h = h * 1664525u + 1013904223u;
      idx = h >> 18;  // 14 bits
    } else {
      idx = (t * 32u + (unsigned)i) & (kLdsWords - 1);
    }
    atomicAdd(&buf[idx], 1u);
  }
  __syncthreads();
  unsigned s = 0;
  for (int i = threadIdx.x; i < kLdsWords; i += blockDim.x) s += buf[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Four 16-byte loads of each thread in flight per step.
__global__ void __launch_bounds__(256) k_read(const int4* __restrict__ a, size_t n, int* out) {
  const size_t st = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int acc = 0;
  for (; i + 3 * st < n; i += 4 * st) {
    const int4 v0 = a[i], v1 = a[i + st], v2 = a[i + 2 * st], v3 = a[i + 3 * st];
    acc ^= v0.x ^ v1.y ^ v2.z ^ v3.w;
  }
  for (; i < n; i += st) acc ^= a[i].x;
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ void __launch_bounds__(256) k_copy(const int4* __restrict__ a, int4* __restrict__ b, size_t n) {
  const size_t st = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * st < n; i += 4 * st) {
    const int4 v0 = a[i], v1 = a[i + st], v2 = a[i + 2 * st], v3 = a[i + 3 * st];
    b[i] = v0;
    b[i + st] = v1;
    b[i + 2 * st] = v2;
    b[i + 3 * st] = v3;
  }
  for (; i < n; i += st) b[i] = a[i];
}

__global__ void __launch_bounds__(256) k_store(int4* __restrict__ b, size_t n) {
  const size_t st = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int4 v = make_int4((int)i, 1, 2, 3);
  for (; i < n; i += st) b[i] = v;
}

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Eight independent accumulators per wavefront, operands in registers.
__global__ void __launch_bounds__(256) k_mfma(float* out, float seed) {
  bf8 a, b;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    a[q] = (__bf16)(seed + threadIdx.x + q);
    b[q] = (__bf16)(seed - q);
  }
  f4 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < kIters / 4; ++i)
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <typename F>
static float time_ms(F launch, int reps) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
  launch();
  (void)hipDeviceSynchronize();
  (void)hipEventRecord(e0);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

int main() {
  hipDeviceProp_t p;
  CK(hipGetDeviceProperties(&p, 0));
  std::printf("{\"gpu\":\"%s\",\"arch\":\"%s\",\"cus\":%d,\"clock_khz\":%d}\n", p.name, p.gcnArchName,
              p.multiProcessorCount, p.clockRate);
  const int blocks = p.multiProcessorCount * 16, threads = 256;
  const double lanes = (double)blocks * threads;
  void* out = nullptr;
  CK(hipMalloc(&out, (size_t)blocks * threads * 8));
  float ms = time_ms([&] { k_fma<<<blocks, threads>>>((double*)out, 1.0000001, 1e-9); }, 5);
  std::printf("{\"test\":\"fp64_fma\",\"ms\":%.4f,\"tflops\":%.2f}\n", ms, 2.0 * lanes * kIters * 8 / ms / 1e9);
  ms = time_ms([&] { k_fma_cvt<<<blocks, threads>>>((int*)out, 1.0000001, 1e-9); }, 5);
  std::printf("{\"test\":\"fp64_fma_plus_cvt_i32\",\"ms\":%.4f,\"g_pairs_per_s\":%.1f}\n", ms,
              lanes * kIters * 8 / ms / 1e6);
  CK(hipGetLastError());
  const int lb = p.multiProcessorCount * 8;  // two 256-thread groups of 64 KB per CU at a time
  const double llanes = (double)lb * threads;
  ms = time_ms([&] { k_lds_atomic<0><<<lb, threads>>>((unsigned*)out); }, 5);
  std::printf("{\"test\":\"lds_atomic_add_consecutive\",\"ms\":%.4f,\"g_lane_ops_per_s\":%.1f}\n", ms,
              llanes * kIters / ms / 1e6);
  ms = time_ms([&] { k_lds_atomic<1><<<lb, threads>>>((unsigned*)out); }, 5);
  std::printf("{\"test\":\"lds_atomic_add_random\",\"ms\":%.4f,\"g_lane_ops_per_s\":%.1f}\n", ms,
              llanes * kIters / ms / 1e6);
  ms = time_ms([&] { k_lds_atomic<2><<<lb, threads>>>((unsigned*)out); }, 5);
  std::printf("{\"test\":\"lds_atomic_add_one_bank\",\"ms\":%.4f,\"g_lane_ops_per_s\":%.1f}\n", ms,
              llanes * kIters / ms / 1e6);
  CK(hipGetLastError());
  const size_t nbytes = (size_t)1 << 30, n4 = nbytes / 16;
  void *a = nullptr, *b = nullptr;
  CK(hipMalloc(&a, nbytes));
  CK(hipMalloc(&b, nbytes));
  CK(hipMemset(a, 1, nbytes));
  CK(hipMemset(b, 0, nbytes));
  const int sb = p.multiProcessorCount * 32;
  CK(hipMemset(out, 0, (size_t)blocks * threads * 8));
  ms = time_ms([&] { k_read<<<sb, threads>>>((const int4*)a, n4, (int*)out); }, 10);
  std::printf("{\"test\":\"hbm_read_1GiB\",\"ms\":%.4f,\"gb_per_s\":%.1f}\n", ms, 1.0 * nbytes / ms / 1e6);
  ms = time_ms([&] { k_copy<<<sb, threads>>>((const int4*)a, (int4*)b, n4); }, 10);
  std::printf("{\"test\":\"hbm_copy_1GiB\",\"ms\":%.4f,\"gb_per_s\":%.1f}\n", ms, 2.0 * nbytes / ms / 1e6);
  ms = time_ms([&] { k_store<<<sb, threads>>>((int4*)b, n4); }, 10);
  std::printf("{\"test\":\"hbm_store_1GiB\",\"ms\":%.4f,\"gb_per_s\":%.1f}\n", ms, 1.0 * nbytes / ms / 1e6);
  CK(hipGetLastError());
  ms = time_ms([&] { k_mfma<<<blocks, threads>>>((float*)out, 0.5f); }, 5);
  const double waves = (double)blocks * threads / 64;
  std::printf("{\"test\":\"mfma_bf16_16x16x32\",\"ms\":%.4f,\"tflops\":%.1f}\n", ms,
              waves * (kIters / 4) * 8 * 16384.0 / ms / 1e9);
  ms = time_ms([&] { k_valu<<<blocks, threads>>>((unsigned*)out, 3u); }, 5);
  const double vi = waves * kIters * 8.0 / (ms * 1e-3);  // wave instructions per second
  std::printf("{\"test\":\"valu_issue_i32\",\"ms\":%.4f,\"g_wave_instr_per_s\":%.1f,\"per_cu_cycle_at_clock\":%.3f}\n",
              ms, vi / 1e9, vi / (p.multiProcessorCount * (p.clockRate * 1e3)));
  CK(hipDeviceSynchronize());
  CK(hipFree(a));
  CK(hipFree(b));
  CK(hipFree(out));
  return 0;
}
