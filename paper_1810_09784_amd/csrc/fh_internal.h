// Internal declarations of the generalized FrequencyHough library (product
// side only).  The plan holds the host-computed FP64 tables of the canonical
// index arithmetic and their device copies; the kernels read only these.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "fh.h"

namespace fh {

constexpr int kWave = 64;
constexpr int kMaxRowsPerTile = 64;     // rows of one tile (fits one wave's ballot)
constexpr int kLdsBudget = 160 * 1024;  // gfx950 LDS per work-group
constexpr int kMaxJTable = 1 << 24;     // largest column->bin table of the windowed mode

enum Mode : int32_t { kModeAuto = 0, kModeWhole = 1, kModeWindowed = 2 };

// Everything a tile of one map needs, by value (kernel argument or queue entry).
struct MapArgs {
  const double* A;         // [n_f + 1] column coordinate of each bin edge
  const double* C;         // [n_k] column shift per second of each row
  const double* T;         // [n_fft] time of each FFT
  const int32_t* J;        // [n_J] last bin edge j with A_j >= c (windowed mode)
  const uint2* rank;       // [n_fft][n_words] (#peaks below word, bit mask) (windowed mode)
  const int32_t* row_ptr;  // [n_fft + 1] peak CSR
  const int32_t* bin;      // [n_peaks]
  int32_t* map;            // [n_k][n_x0]
  unsigned long long* err; // bad-peak counter
  double tfft;             // FFT length (uniform times when t_uniform)
  int32_t t_uniform;       // T_i = (i + 0.5) * tfft
  int32_t n_peaks;
  int32_t n_f, n_x0, n_k, n_fft;
  int32_t n_words, n_J;
  int32_t rows, cols, mode;
  int32_t tiles_x, tiles_y, tsplit;
  int32_t pitch;           // LDS row pitch of the differential tile (ints)
  int32_t a_lds;           // A table staged in LDS
  int32_t lds_bytes;       // dynamic LDS of one tile
};

struct Plan {
  fh_map_desc desc{};       // scalars (array pointers cleared)
  int32_t n_f = 0, n_x0 = 0, n_J = 0, n_words = 0, t_uniform = 1;
  double x0_min = 0, dx0 = 0;
  fh_tile_cfg tile{};
  std::vector<double> A, C, T;
  std::vector<int32_t> J;
  // device
  double *dA = nullptr, *dC = nullptr, *dT = nullptr;
  int32_t* dJ = nullptr;
  uint2* dRank = nullptr;
  unsigned long long* dErr = nullptr;
  int device = 0;
  MapArgs args(const fh_peaks& pk, int32_t* map) const;
  int64_t n_tiles() const;
};

// implemented in fh_hough.hip
fh_status launch_hough(const Plan& p, const fh_peaks& pk, int32_t* map, hipStream_t s);
int lds_bytes_for(const Plan& p);
fh_status launch_batched(const MapArgs* d_maps, const int2* d_queue, int32_t n_queue, int32_t* d_head, int lds_max,
                         int32_t grid, hipStream_t s);
fh_status launch_prepare(const MapArgs& a, hipStream_t s);
fh_status launch_zero(unsigned long long* p, int n, hipStream_t s);
fh_status launch_zero_i32(int32_t* p, int n, hipStream_t s);

}  // namespace fh

struct fh_plan_s {
  fh::Plan p;
};
