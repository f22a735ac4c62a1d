// Internal declarations of the generalized FrequencyHough library (product
// side only).  The plan holds the host-computed FP64 tables of the canonical
// index arithmetic, their device copies, and the work units of the map.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "fh.h"

namespace fh {

constexpr int kWave = 64;
constexpr int kMaxRowsPerTile = 64;     // rows of one tile
constexpr int kLdsBudget = 160 * 1024;  // gfx950 LDS per work-group
constexpr int kMaxJTable = 1 << 24;     // largest column->bin table of the windowed mode
constexpr int kProfileSamples = 128;    // FFT samples of a tile's cost profile
constexpr int kUnitAtomic = 1 << 30;    // flag bit of a unit's map field: add into the map
constexpr int kMaxSelectSegments = 256; // squares along x0 in candidate selection
constexpr int kWaveScratchBytes = 1296; // per-wave LDS scratch of the whole-FFT pair loop
constexpr int kCPad = 8;                // zero entries after the last row of the device C table

enum Mode : int32_t { kModeAuto = 0, kModeWhole = 1, kModeWindowed = 2 };

// Everything a tile of one map needs, by value (kernel argument or table entry).
struct MapArgs {
  const double* A;         // [n_f + 2] column coordinate of each bin edge, then a pad +huge
  const double* C;         // [n_k + kCPad] column shift per second of each row, then zeros
  const double* T;         // [n_fft] time of each FFT
  const int32_t* J;        // [n_J] last bin edge j with A_j >= c (windowed mode)
  uint2* rank;             // [n_fft][n_words] (#peaks below word, bit mask) (windowed mode)
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
  int32_t tiles_x, tiles_y;
  int32_t pitch;           // LDS row pitch of the differential tile (ints)
  int32_t a_lds;           // A table staged in LDS
  int32_t lds_bytes;       // dynamic LDS of one tile
  // fused candidate selection (single-map launches; sel == nullptr: none)
  unsigned long long* sel; // [n_k][sel_sq][3] per row and column segment: Sy, Sy2, best-cell key
  int32_t sel_sq;          // column segments (squares along x0)
  int32_t sel_lo, sel_hi;  // analysed columns [sel_lo, sel_hi)
};

// Selection attached to a single-map launch: the row segment partials the
// tile kernel adds into (cleared by the launch).
struct SelArgs {
  unsigned long long* rows;
  int32_t sq, lo, hi;
};

// A unit of work: one tile over an FFT range.  x = map index | kUnitAtomic
// when the tile is split over several units (they add into a cleared map),
// y = tile index (row tile * tiles_x + column tile), [z, w) = FFT range.
using Unit = int4;

// Estimated cost of a tile as a function of its FFT range: cum[q] is the cost
// of FFTs [lo, lo + (hi - lo) * q / kProfileSamples).
struct TileProfile {
  int32_t lo = 0, hi = 0;
  float cum[kProfileSamples + 1];
};

struct Plan {
  fh_map_desc desc{};       // scalars (array pointers cleared)
  int32_t n_f = 0, n_x0 = 0, n_J = 0, n_words = 0, t_uniform = 1;
  double x0_min = 0, dx0 = 0;
  fh_tile_cfg tile{};
  std::vector<double> A, C, T, K;
  std::vector<int32_t> J;
  std::vector<TileProfile> prof;  // per tile
  double total_cost = 0;
  // work units of a single-map launch, and the tiles to clear before it
  std::vector<Unit> units;
  std::vector<double> unit_cost;
  std::vector<int4> clears;  // (map index, tile index, 0, 0)
  // device
  double *dA = nullptr, *dC = nullptr, *dT = nullptr;
  int32_t* dJ = nullptr;
  uint2* dRank = nullptr;
  unsigned long long* dErr = nullptr;
  Unit* dUnits = nullptr;
  int4* dClears = nullptr;
  int32_t* dHead = nullptr;
  unsigned long long* dSel = nullptr;  // fh_select scratch: row segment partials, then square results
  size_t sel_words = 0;               // its capacity in 64-bit words (grows on demand)
  unsigned long long* hSq = nullptr;  // pinned host copy of the square results of fh_hough_select
  size_t hsq_words = 0;
  hipEvent_t ev_sel = nullptr;        // recorded after that copy
  int32_t sel_pending = 0;            // results of an fh_hough_select not yet fetched
  fh_select_opts sel_opts{};          // its options (col_hi resolved)
  int32_t* dProj = nullptr;           // fh_project scratch: candidate flags, one drift table
  size_t proj_words = 0;
  int32_t grid = 0;  // persistent work-groups of a single-map launch
  int device = 0;
  int n_cu = 256;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;  // optional profiling hook
  MapArgs args(const fh_peaks& pk, int32_t* map) const;
  int64_t n_tiles() const;
};

// Dynamic LDS of one tile.  wave_scratch: room for the per-wave scratch that
// the whole-FFT pair loop uses (kernels compiled for windowed maps only have none).
int lds_bytes_for_shape(int n_f, int rows, int cols, int a_lds, int threads, int* pitch_out, int wave_scratch = 1);

// Split the plan's tiles into units of about `target` cost (at most
// tile.tsplit pieces per tile), append them (map index `mi`) to units/cost and
// the split tiles to clears.
void split_units(const Plan& p, int32_t mi, double target, std::vector<Unit>& units, std::vector<double>& cost,
                 std::vector<int4>& clears);

// Device allocation of the library (hipMalloc); FH_ENOMEM on out-of-memory,
// FH_EDEVICE on other failures.  Test hook: with the environment variable
// FH_FAKE_OOM set every such allocation fails with FH_ENOMEM.
fh_status device_alloc(void** p, size_t bytes);
// Test hook: true when the environment variable FH_FAKE_DEVICE_ERROR names
// `what` ("graph": graph instantiation of a batch fails).
bool fake_device_error(const char* what);
// Host checks of a peak list: row_ptr set, 0 <= n_peaks < 2^31, bin set when
// n_peaks > 0 and 16-byte aligned (the windowed tiles read it 16 bytes at a time).
fh_status check_peaks(const fh_peaks* pk);

// implemented in fh_hough.hip
fh_status launch_hough(const Plan& p, const fh_peaks& pk, int32_t* map, hipStream_t s,
                       const SelArgs* sel = nullptr);
int occupancy_grid(int threads, int lds_bytes, int n_units, int mode);

}  // namespace fh

struct fh_plan_s {
  fh::Plan p;
};

// A batch of maps launched as one persistent, graph-captured queue
// (fh_batch_*), and the scratch of its batched selection (fh_batch_select).
struct fh_batch_s {
  int32_t m = 0;
  std::vector<const fh::Plan*> plans;
  std::vector<fh_peaks> peaks;
  std::vector<int32_t*> maps;
  std::vector<fh::MapArgs> args;
  fh::MapArgs* d_maps = nullptr;
  fh::Unit* d_queue = nullptr;
  int4* d_clears = nullptr;
  int32_t* d_head = nullptr;
  int32_t n_queue = 0, n_clears = 0;
  int32_t grid = 0;
  int32_t lds = 0;
  int32_t threads = 256, mode = 0;  // persistent kernel: work-group size, compiled mode (0: per map)
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned long long* d_sel = nullptr;  // batched selection: map table, row partials, square results
  size_t sel_bytes = 0;
};
