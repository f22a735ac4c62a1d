/*
 * fh.h -- C ABI of the MI355X (gfx950) generalized FrequencyHough library.
 *
 * Method (Miller et al., "A method to search for long duration gravitational
 * wave transients from isolated neutron stars using the generalized
 * FrequencyHough"):
 *   Sec. II, Eqs. diff_powlaws/powlaws: the signal model fdot = -k f^n.
 *   Sec. IV, Eq. transform: x = f^(1-n) turns it into x = x0 + (n-1) k (t - t0),
 *     so each peakmap peak (t, f) is a line in the (x0, k) plane and the Hough
 *     map is the histogram of those lines.
 *   Sec. VI.B: the k grid (given here as an explicit ascending array).
 *   Sec. VI.C: the uniform x0 grid with step (n-1) df / f_max^n from f_max^(1-n).
 *   Sec. IV (candidate selection, Eq. for CR): squares, critical ratio.
 *
 * Conventions for every entry point:
 *   - Return FH_OK or a negative fh_status; arguments are validated before any
 *     work is enqueued, so an error return means nothing was written.
 *   - No exceptions, aborts or exits cross this boundary.
 *   - Device pointers are HIP device allocations on the current device,
 *     owned by the caller.  Host pointers are read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls that take a stream are asynchronous on it unless stated.
 *   - A plan owns scratch: its fh_hough calls (and the batches holding it) run
 *     one at a time, on one stream at a time; its fh_select calls likewise.
 *     The two kinds use separate scratch, so a selection of one map may run
 *     on another stream while the plan transforms the next map.
 *   - Different plans share nothing: their calls may run at the same time on
 *     different streams (no kernel of the library waits on another
 *     work-group, so overlapping launches always finish).  Two plans of one
 *     map description alternating over two streams let one call's rank build
 *     and selection overlap the other's tile kernel.
 *   - Fault injection for tests of callers' error paths, read at each use:
 *     with FH_FAKE_OOM set in the environment every device allocation of the
 *     library fails (FH_ENOMEM); FH_FAKE_DEVICE_ERROR=graph makes the graph
 *     instantiation of fh_batch_create fail (FH_EDEVICE).  Either way the call
 *     returns before anything is launched and frees what it had allocated.
 *
 * The peak bin b of FFT i stands for the frequency bin [f_min + b df,
 * f_min + (b+1) df), df = 1/tfft.  Its x-image is shifted, at row r and time
 * T_i, to x0-columns floor(u_lo) .. floor(u_hi), clipped to [0, n_x0), with
 *   u = fma(-C_r, T_i, A_b)   (binary64, one rounding)
 *   A_b = (pow(f_min + b*df, 1-n) - x0_min) * (1/dx0),  C_r = ((n-1)*k_r) * (1/dx0),
 *   T_i = t[i] if given, else (i + 0.5) * tfft  (FFT mid-time, t0 = start),
 * u_lo using the bin's upper edge b+1 and u_hi its lower edge b.  Every
 * operation is one IEEE binary64 operation rounded to nearest, no
 * contraction, on the host (tables) and on the device (u); counts are exact.
 */
#ifndef FH_H
#define FH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FH_OK = 0,
  FH_EINVAL = -1,   /* invalid argument (description, sizes, pointers) */
  FH_ENOMEM = -2,   /* device or host allocation failed */
  FH_EDEVICE = -3,  /* a HIP call failed (launch, copy, graph) */
  FH_ERANGE = -4    /* sizes exceed the library's limits (e.g. n_k*n_x0 >= 2^31) */
} fh_status;

typedef struct fh_plan_s* fh_plan_t;

/* One Hough map (Sec. IV/VI).  All arrays are HOST memory, read by fh_plan. */
typedef struct {
  double n;          /* braking index; finite, n > 1 (Sec. II) */
  double tfft;       /* FFT length in s; df = 1/tfft (Sec. VI.A) */
  double f_min;      /* band of the peakmap in Hz; 0 < f_min < f_max and */
  double f_max;      /*   (f_max - f_min)*tfft integral within 1e-9 */
  int32_t n_fft;     /* number of FFTs (time rows of the peakmap), >= 1 */
  const double* t;   /* [n_fft] t_i - t0 in s, ascending, finite; NULL = (i+0.5)*tfft */
  int32_t n_k;       /* rows of the map, >= 1 */
  const double* k;   /* [n_k] ascending, finite, k >= 0 (Sec. VI.B) */
  double x0_min;     /* x0 of column 0; used only if dx0 != 0 */
  double dx0;        /* column width; 0 = defaults x0_min = f_max^(1-n), */
                     /*   dx0 = ((n-1)/tfft) f_max^-n (Sec. VI.C); else > 0 */
  int32_t n_x0;      /* columns; 0 = ceil(f_max((f_max/f_min)^(n-1)-1)/((n-1)df) - 1e-9) */
} fh_map_desc;

/* Peakmap as a CSR by FFT, DEVICE memory: FFT i owns bin[row_ptr[i] ..
 * row_ptr[i+1]), frequency-bin indices strictly ascending within an FFT.
 * row_ptr has n_fft+1 entries, row_ptr[0] = 0, non-decreasing, row_ptr[n_fft]
 * = n_peaks (not checked on the host: it lives on the device).  Bins outside
 * [0, n_f) are skipped and counted in the plan's device error word; a
 * non-ascending FFT is counted there too and leaves that FFT's counts in the
 * windowed mode unspecified (never out-of-bounds memory access). */
typedef struct {
  const int32_t* row_ptr;
  const int32_t* bin;      /* 16-byte aligned (read 16 bytes at a time) */
  int64_t n_peaks;
} fh_peaks;

/* Host checks that every entry point taking peaks makes before it enqueues
 * anything: row_ptr not NULL, 0 <= n_peaks < 2^31, bin not NULL when
 * n_peaks > 0, and bin 16-byte aligned (torch and hipMalloc allocations are).
 * FH_OK or FH_EINVAL; touches no memory and no device. */
fh_status fh_peaks_validate(const fh_peaks* peaks);

/* Tile shape of the Hough kernel; zeros = automatic.  mode 1 = every tile
 * reads whole FFTs (small maps), mode 2 = tiles read only the peaks whose
 * image can reach their columns (wide maps). */
typedef struct {
  int32_t rows;     /* k rows per tile, 1..64 */
  int32_t cols;     /* x0 columns per tile */
  int32_t threads;  /* work-group size: 256 or 512 */
  int32_t mode;     /* 0 auto, 1 whole-FFT, 2 windowed */
  int32_t tsplit;   /* the FFTs are split into this many ranges, one tile each; */
                    /*   > 1: tiles add into the map with atomics after a clear */
} fh_tile_cfg;

typedef struct {
  int32_t n_f, n_x0, n_k, n_fft;
  double x0_min, dx0;
  fh_tile_cfg tile;      /* the resolved tile shape */
  int64_t n_tiles;
  int64_t workspace_bytes;
} fh_plan_info;

/* Validate a map description, compute the FP64 tables on the host and upload
 * them, choose the tile shape (cfg NULL or zeros = automatic) and allocate the
 * plan's device workspace on the current device.  Synchronous.
 * Errors: FH_EINVAL (bad description), FH_ERANGE (n_k*n_x0 >= 2^31 or
 * n_f > 2^24), FH_ENOMEM, FH_EDEVICE.  *out is set only on FH_OK. */
fh_status fh_plan(const fh_map_desc* desc, const fh_tile_cfg* cfg, fh_plan_t* out);
fh_status fh_plan_get_info(fh_plan_t plan, fh_plan_info* out);
/* Host copies of the plan's tables: A [n_f+1], C [n_k], T [n_fft]; any may be NULL. */
fh_status fh_plan_tables(fh_plan_t plan, double* A, double* C, double* T);
void fh_plan_destroy(fh_plan_t plan);

/* The generalized FrequencyHough of one peakmap (Sec. IV): writes every cell
 * of map (DEVICE int32 [n_k][n_x0], row-major, x0 ascending = frequency
 * descending), so the caller need not clear it.  Counts are exact.
 * Errors (nothing enqueued): FH_EINVAL for NULL pointers or peaks failing
 * fh_peaks_validate (sizes, a bin array that is not 16-byte aligned);
 * FH_EDEVICE if a launch fails. */
fh_status fh_hough(fh_plan_t plan, const fh_peaks* peaks, int32_t* map, void* stream);

/* Profiling hook: when start/stop (hipEvent_t, passed as void*) are set,
 * every later fh_hough of this plan records `start` on its stream right before
 * the Hough tile kernel and `stop` right after it, so the kernel alone can be
 * timed on the stream it runs on.  NULL, NULL clears the hook. */
fh_status fh_plan_set_events(fh_plan_t plan, void* start, void* stop);

/* Number of bad peaks seen by the last fh_hough / batch launch of this plan:
 * a peak is bad when its bin is outside [0, n_f) or not above the previous
 * bin of its FFT, and each bad peak counts once.  (Bands of more than 16384
 * bins find each FFT's words by bisection: there an FFT that is not ascending
 * apart from out-of-band bins at its two ends counts at least one.)
 * Synchronises `stream`. */
fh_status fh_device_errors(fh_plan_t plan, void* stream, uint64_t* out);

/* ---------------------------------------------------------- selection --
 * Candidate selection of Sec. IV: the analysed part of the map (all rows,
 * columns [col_lo, col_hi)) is divided into sq_k x sq_x0 "squares" (row
 * boundaries floor(a * n_k / sq_k), column boundaries col_lo + floor(b * W /
 * sq_x0), W = col_hi - col_lo).  In every square the cell with the highest
 * count is a candidate (ties: smallest row, then smallest column), and so is
 * the best cell at least min_dk rows away from it (same tie rule).  Each gets
 * the critical ratio CR = (y - mu) / sigma, mu and sigma being the mean and
 * population standard deviation of the square's counts, computed from exact
 * integer sums Sy, Sy2 over its N cells as
 *     mu = Sy / N,  var = Sy2 / N - mu * mu,  sigma = sqrt(var)
 * (binary64, this order, no contraction).  Squares with sigma = 0 give no
 * candidate.  Candidates with CR >= cr_thr are returned in square order
 * (best before second).  x0 and k are the cell centre x0_min + (col + 0.5) dx0
 * and k[row]; f0 = x0^(1/(1-n)) and fdot0 = -k f0^n invert the transform. */
typedef struct {
  int32_t sq_k, sq_x0;   /* squares along k and along x0, >= 1 */
  int32_t min_dk;        /* row distance of a second candidate (the paper: ~3); < 1 = none */
  int32_t col_lo, col_hi;/* analysed columns [col_lo, col_hi); col_hi <= 0 means n_x0 */
  double cr_thr;         /* keep candidates with CR >= cr_thr */
} fh_select_opts;

typedef struct {
  int32_t row, col;      /* cell: k row, x0 column */
  int32_t count;         /* Hough count y */
  int32_t square;        /* square index a * sq_x0 + b */
  int32_t second;        /* 0: best of its square, 1: the second candidate */
  int32_t pad;
  double cr, mu, sigma;  /* critical ratio and the square's statistics */
  double x0, k, f0, fdot0;
} fh_candidate;

/* Select candidates of a Hough map (DEVICE int32 [n_k][n_x0], counts >= 0, as
 * written by fh_hough with this plan).  Reads the map once on `stream` (per
 * row and column segment: exact sums and best cell), reduces the rows of each
 * square on the device, copies 48 bytes per square to the host and evaluates
 * mu, sigma and CR there; synchronises `stream`.  The plan's selection scratch
 * (8 (3 n_k sq_x0 + 6 sq_k sq_x0) bytes) is allocated on first use or growth.
 * Writes min(total, cap) candidates to `out` (HOST) and the total number with
 * CR >= cr_thr to *n_out.  Errors: FH_EINVAL (NULL pointers, sq_k outside
 * [1, n_k], sq_x0 outside [1, min(W, 256)], bad column range), FH_EDEVICE. */
fh_status fh_select(fh_plan_t plan, const int32_t* map, const fh_select_opts* opts, fh_candidate* out, int32_t cap,
                    int32_t* n_out, void* stream);

/* fh_select for callers that cannot allocate memory (code under HIP graph
 * capture, serving loops, hosts that forbid allocation at run time): the same
 * kernels, results and errors as fh_select, but its scratch is a fixed array
 * of 4 MiB (524288 64-bit words) in the library's device image, one copy per
 * GPU, held until the process ends, and the host finish works through a
 * buffer on the stack.  It calls no allocating routine.  Needs
 * 3 n_k sq_x0 + 6 sq_k sq_x0 <= 524288 words, else FH_ERANGE (nothing is
 * enqueued).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (several threads or streams) race, so serialise them.
 * Synchronises `stream`.  Does not touch the plan's own selection scratch. */
fh_status fh_select_noalloc(fh_plan_t plan, const int32_t* map, const fh_select_opts* opts, fh_candidate* out,
                            int32_t cap, int32_t* n_out, void* stream);

/* The transform and the selection in one pass (Sec. IV: the Hough map, then
 * its candidates): writes the same map as fh_hough and prepares the same
 * candidates as fh_select with `opts` would, without reading the map back.
 * The tile kernel adds each tile row's exact sums and largest count per
 * column segment as it stores the counts (tiles split over several units:
 * a short pass over their part of the map after the tile kernel); after the
 * square reduction, the first column holding the largest count is searched
 * in the two rows each square picks.  Asynchronous on
 * `stream`: the square results are copied to pinned host memory owned by the
 * plan and an event is recorded; fetch them with fh_select_results.  A new
 * fh_hough_select of the same plan first waits for a pending one and drops
 * its results if they were not fetched; an fh_select of the plan also waits
 * for it (those results stay available).  The plan's scratch is shared, so
 * one plan serves one such call at a time (use two plans of the same map
 * description to overlap steps).  Errors: those of fh_hough and fh_select,
 * FH_ENOMEM for the pinned buffer. */
fh_status fh_hough_select(fh_plan_t plan, const fh_peaks* peaks, int32_t* map, const fh_select_opts* opts,
                          void* stream);

/* Candidates of the last fh_hough_select of this plan, as fh_select returns
 * them (min(total, cap) records to `out` (HOST), the total to *n_out).  Waits
 * for that call's event (not for the whole stream).  FH_EINVAL when no
 * results are pending. */
fh_status fh_select_results(fh_plan_t plan, fh_candidate* out, int32_t cap, int32_t* n_out);

/* ---------------------------------------------------------- tile CNN --
 * A learned proposer of 64 x 64 map tiles (not in the paper, whose last
 * section only plans machine learning): tile (counts normalised by their map
 * row's mean and standard deviation) -> 4 x [3x3 conv, zero padding, bias,
 * ReLU] with 1 -> 16 -> 32 -> 64 -> 64 channels -> global average pool ->
 * linear 64 -> 1 -> logistic; 60289 FP32 parameters, flat order w1 [16][9],
 * b1, w2 [32][9*16], b2, w3 [64][9*32], b3, w4 [64][9*64], b4, w5 [64], b5,
 * conv weight index (co, k = (dy*3 + dx)*Cin + ci).  Activations, weights and
 * activation gradients are BF16 (round to nearest even), sums FP32 (matrix
 * cores for conv2..4).  Tiles are DEVICE BF16 [B][64][64] (row = k, col = x0).
 * A network object owns its parameters, Adam state and the activations of
 * up to max_batch tiles; it is used from one stream at a time. */
typedef struct fh_cnn_s* fh_cnn_t;

fh_status fh_cnn_create(int32_t max_batch, fh_cnn_t* out);          /* parameters zero */
void fh_cnn_destroy(fh_cnn_t net);
int64_t fh_cnn_num_params(void);                                    /* 60289 */
/* HOST float [n] in the flat order; resets the Adam state.  Synchronous. */
fh_status fh_cnn_set_params(fh_cnn_t net, const float* params, int64_t n);
/* HOST copies of the parameters and of the last backward's gradients (either may be NULL). */
fh_status fh_cnn_get_params(fh_cnn_t net, float* params, float* grads, int64_t n);
/* Replace the gradients that the next fh_cnn_step applies (HOST float [n] in
 * the flat order; n = 60289).  For callers that combine gradients outside the
 * library (several processes' gradients summed before one step) and for tests
 * of the optimiser alone.  Synchronous.  Errors: FH_EINVAL, FH_EDEVICE. */
fh_status fh_cnn_set_grads(fh_cnn_t net, const float* grads, int64_t n);
/* Adam's state, for a training checkpoint: HOST copies of the first and second
 * moments (float [n] in the flat order, n = 60289; either may be NULL) and the
 * number of steps taken (may be NULL).  Synchronous.  Errors: FH_EINVAL, FH_EDEVICE. */
fh_status fh_cnn_get_state(fh_cnn_t net, float* m1, float* m2, int64_t n, int64_t* steps);
/* Restore that state (after fh_cnn_set_params, which resets it): the next
 * fh_cnn_step continues as the network that saved it would have (bias
 * corrections of step `steps` + 1).  0 <= steps < 2^31.  Synchronous.
 * Errors: FH_EINVAL, FH_EDEVICE. */
fh_status fh_cnn_set_state(fh_cnn_t net, const float* m1, const float* m2, int64_t n, int64_t steps);
/* HOST copy of the BF16 activations of the last forward: layer 0 = the input
 * tiles [B][64][64], layer l = 1..4 = the ReLU output of conv l, NHWC
 * [B][64][64][C_l] with C = 16, 32, 64, 64 (B of that forward; n must equal
 * the element count).  Synchronous.  Errors: FH_EINVAL (no forward yet, layer
 * outside 0..4, wrong n), FH_EDEVICE. */
fh_status fh_cnn_activations(fh_cnn_t net, int32_t layer, uint16_t* out, int64_t n);
/* logits (DEVICE float [B], may be NULL) of B <= max_batch tiles; keeps the activations. */
fh_status fh_cnn_forward(fh_cnn_t net, const uint16_t* tiles, int32_t B, float* logits, void* stream);
/* Logits (DEVICE float [B]) of B <= max_batch tiles for proposals: the same
 * arithmetic as fh_cnn_forward, bit for bit, but the last layer keeps only its
 * per-row channel sums for the pool and its activations are not stored: a
 * backward or fh_cnn_activations may not follow (they return FH_EINVAL).  Errors: FH_EINVAL, FH_ERANGE (B), FH_EDEVICE. */
fh_status fh_cnn_scores(fh_cnn_t net, const uint16_t* tiles, int32_t B, float* logits, void* stream);
/* Mean binary cross-entropy of the last forward against labels (DEVICE float [B], 0/1)
 * and its gradients (replacing the previous ones); loss: DEVICE float, may be NULL. */
fh_status fh_cnn_backward(fh_cnn_t net, const float* labels, int32_t B, float* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr. */
fh_status fh_cnn_step(fh_cnn_t net, float lr, void* stream);
/* Normalised tiles of a DEVICE int32 map [n_k][n_x0]: per-row mean and 1/std
 * (DEVICE float [n_k] each, written) and tiles (DEVICE BF16 [n_tiles][64][64])
 * at origins (DEVICE int32 [n_tiles][2] = (row, col)); zero outside the map. */
fh_status fh_tiles(const int32_t* map, int32_t n_k, int32_t n_x0, const int32_t* origins, int32_t n_tiles,
                   uint16_t* tiles, float* row_mean, float* row_istd, void* stream);
/* Score every 64 x 64 tile of a Hough map of `plan` (tile (a, b) at row 64a,
 * column 64b; scores: DEVICE float [ceil(n_k/64) * ceil(n_x0/64)], the
 * logits, row-major over (a, b)) and return the n_top best tile indices
 * (HOST int32, best first) in tile_ids.  Uses the network's activations as
 * scratch; allocates a row-statistics buffer on first use or growth.
 * Synchronises `stream`. */
fh_status fh_propose(fh_cnn_t net, fh_plan_t plan, const int32_t* map, float* scores, int32_t n_top,
                     int32_t* tile_ids, void* stream);

/* Declared with the batches below: fh_batch_propose, fh_propose over every
 * map of a batch. */

/* ----------------------------------------------------------- batching --
 * Many maps of uneven size in one persistent launch: every tile of every map
 * goes into one work queue, longest (estimated) first, claimed by a grid of
 * resident work-groups through an atomic counter; the launch is captured in a
 * hipGraph once and replayed.  Each map i uses plans[i] (its grid and tile
 * shape), peaks[i] and maps[i]; several maps may share one peakmap. */
typedef struct fh_batch_s* fh_batch_t;

/* Build the work queue and the graph.  Host arrays of length m (>= 1) are read
 * during the call; the plans must outlive the batch; the peak and map device
 * buffers must stay valid while the batch is launched.  The persistent launch
 * uses one work-group size: that of the plans' tile shapes when they all have
 * the same one and read whole FFTs, else 512 threads (whole-FFT maps only) or
 * 256 (mixed).  Synchronous. */
fh_status fh_batch_create(int32_t m, const fh_plan_t* plans, const fh_peaks* peaks, int32_t* const* maps,
                          fh_batch_t* out);
/* Enqueue one replay of the batch on `stream`. */
fh_status fh_batch_launch(fh_batch_t batch, void* stream);
/* Same work without the graph or the queue: one fh_hough launch per map. */
fh_status fh_batch_launch_plain(fh_batch_t batch, void* stream);
void fh_batch_destroy(fh_batch_t batch);

/* Candidate selection (as fh_select, same options for every map; col_hi <= 0
 * means each map's own n_x0) on every map of the batch, as written by its
 * last launch: one row pass and one square reduction over all maps on
 * `stream`, one copy of the square results, the CR finish on the host;
 * synchronises `stream`.  Candidates go to `out` (HOST) map after map, at most
 * cap in all; counts[i] (HOST [m]) gets map i's number with CR >= cr_thr and
 * *n_out their sum.  The batch owns the scratch (grown on demand).  Errors:
 * FH_EINVAL (options invalid for some map), FH_ERANGE (more than 2^31 row
 * segments or squares), FH_ENOMEM, FH_EDEVICE. */
fh_status fh_batch_select(fh_batch_t batch, const fh_select_opts* opts, fh_candidate* out, int32_t cap,
                          int32_t* counts, int32_t* n_out, void* stream);

/* The selection re-checking given 64 x 64 tiles only (the tiles a proposer
 * such as fh_propose picked): tile t = a * ceil(n_x0/64) + b is the rectangle
 * rows 64a .. min(64a + 64, n_k) - 1, columns 64b .. min(64b + 64, n_x0) - 1
 * (fh_propose's numbering), intersected with the analysed columns
 * [col_lo, col_hi).  Each rectangle is selected on its own, as fh_select does a
 * whole map: sq_k x sq_x0 squares over the rectangle, their statistics (mu,
 * sigma, CR) from the rectangle's cells alone.  Candidates carry map rows and
 * columns; `square` numbers the squares within their tile.  Only the listed
 * tiles are read.  fh_select_tiles: n_tiles tile indices (HOST) of one map;
 * fh_batch_select_tiles: n_req (map index, tile index) pairs (HOST int32
 * [n_req][2]) over the maps of a batch (as written by its last launch).
 * Candidates go to `out` (HOST) request after request, at most cap in all;
 * counts[i] (HOST) gets request i's number with CR >= cr_thr (0 for a tile
 * outside the analysed columns) and *n_out their sum.  The scratch is the
 * plan's selection scratch, or the batch's; synchronises `stream`.  Errors:
 * FH_EINVAL (a tile index outside the map, sq_k above a rectangle's rows or
 * sq_x0 above its columns or 256), FH_ERANGE, FH_ENOMEM, FH_EDEVICE. */
fh_status fh_select_tiles(fh_plan_t plan, const int32_t* map, const fh_select_opts* opts, int32_t n_tiles,
                          const int32_t* tiles, fh_candidate* out, int32_t cap, int32_t* counts, int32_t* n_out,
                          void* stream);
fh_status fh_batch_select_tiles(fh_batch_t batch, const fh_select_opts* opts, int32_t n_req, const int32_t* req,
                                fh_candidate* out, int32_t cap, int32_t* counts, int32_t* n_out, void* stream);

/* fh_propose on every map of the batch (as written by its last launch) with
 * one network: row statistics of all maps in one launch, then the tiles of
 * all maps in the network's batches (tiles of several maps share a forward
 * pass; each tile's score does not depend on its batch-mates), one copy of the
 * scores.  scores: DEVICE float [sum of the maps' tile counts], map after
 * map, each map's tiles in fh_propose's order.  n_top: HOST [m], each within
 * [0, that map's tile count].  tile_ids: HOST, sum of n_top, map after map,
 * each map's best tiles first (ties: lower tile index first).  Synchronises
 * `stream`.  Errors: FH_EINVAL, FH_ERANGE (2^31 rows or tiles), FH_ENOMEM,
 * FH_EDEVICE. */
fh_status fh_batch_propose(fh_cnn_t net, fh_batch_t batch, float* scores, const int32_t* n_top, int32_t* tile_ids,
                           void* stream);

/* One-shot convenience: create, launch on `stream`, synchronise, destroy. */
fh_status fh_hough_batched(int32_t m, const fh_plan_t* plans, const fh_peaks* peaks, int32_t* const* maps,
                           void* stream);

/* ------------------------------------------------------- coincidences --
 * Sec. IV: candidates from two lists (two detectors, or two T_FFT portions of
 * Sec. VI.D) are in coincidence when their distance in bins
 *   d = sqrt(u*u + v*v),  u = (x0_b - x0_a') / dx,  v = (k_b - k_a) / dk
 * is at most max_d (the paper uses 3), with dx = (dx0_a + dx0_b) / 2 and
 * dk = (dk_a + dk_b) / 2 the mean bin sizes of the two candidates (dk is the
 * local step of a non-uniform k grid).  x0_a' = x0_a + (nm1 * k_a) * dt moves
 * a candidate of an earlier portion to the later portion's start along its
 * line x = x0 + (n-1) k t (Sec. IV, Eq. transform): nm1 = n - 1 and dt are
 * per segment; with dt = 0 (or NULL arrays) x0_a' = x0_a.  Every operation
 * is one binary64 operation in this order, no contraction.
 * Lists are grouped by segment (a map, or a braking index for portions):
 * a_off / b_off (DEVICE int32 [n_seg + 1], non-decreasing) delimit each
 * segment's points, and only points of the same segment are compared. */
typedef struct {
  double x0, k;     /* candidate cell */
  double dx0, dk;   /* bin sizes of its map at that cell */
} fh_point;

/* Pairs (DEVICE int32 [cap][2], indices into a and b) of all coincident
 * points, in no particular order, their distances (DEVICE double [cap], may
 * be NULL) and the total number of pairs (*count, DEVICE int32, set by the
 * call; pairs beyond cap are counted but not written).  a holds na points and
 * a_off[n_seg] = na, b holds nb points and b_off[n_seg] = nb (offsets outside
 * [0, na] / [0, nb] are clipped).  nm1, dt: DEVICE double [n_seg] or NULL.
 * Asynchronous on `stream`; allocates nothing.  Errors: FH_EINVAL (negative
 * sizes, NULL arrays that are needed, max_d not finite or < 0). */
fh_status fh_coincide(int32_t n_seg, int32_t na, const int32_t* a_off, const fh_point* a, int32_t nb,
                      const int32_t* b_off, const fh_point* b, const double* nm1, const double* dt, double max_d,
                      int32_t* pairs, double* dist, int32_t cap, int32_t* count, void* stream);

/* --------------------------------------------------------- follow-up --
 * The synthetic part of the follow-up of Sec. V: with a candidate's source
 * parameters (f0, k) every peak (i, j) of the peakmap is moved by the drift
 * of the power law of Eq. powlaws, j -> j - (b_i - b_0) with
 *   b_i = floor((f(T_i) - f_min) * tfft),  b_0 = floor((f0 - f_min) * tfft),
 *   f(T) = f0 / (1 + ((k * (n-1)) * pow(f0, n-1)) * T)^(1/(n-1))  (pow),
 * so that the source's peaks gather in bin b_0; the moved peaks are then
 * projected on the frequency axis and the count y in bin b_0 gets the
 * critical ratio CR = (y - mu) / sigma against the bins b_0 - w .. b_0 + w
 * outside b_0 - guard .. b_0 + guard (population statistics from exact sums,
 * binary64: mu = S/N, var = S2/N - mu^2, sigma = sqrt(var); sigma = 0 gives
 * CR = NaN).  Peaks with a bin outside [0, n_f) are skipped.  The plan gives
 * n, tfft, f_min and the times T_i.  Each FFT's window of bins is found by
 * binary search, so a non-ascending FFT leaves its contribution unspecified.
 * pow is the host C library's: the device evaluates the drift with its own
 * pow and, for a candidate where some (f(T_i) - f_min) * tfft lies within
 * rounding distance of an integer, the host evaluates that candidate's drift
 * table and the candidate is projected again (host_drift = 1). */
typedef struct {
  int32_t y;                 /* peaks in bin b_0 after the move */
  int32_t host_drift;        /* 1: this candidate's drift came from the host's table */
  double mu, sigma, cr;
} fh_projection;

/* n_cand candidates, f0 and k DEVICE double [n_cand]; hist DEVICE int32
 * [n_cand][2w+1] (bin b_0 + d at index w + d) written; out HOST [n_cand].
 * 1 <= w <= 4096, 0 <= guard < w.  The plan's projection scratch (4 (n_cand
 * + n_fft) bytes) is allocated on first use or growth.  Synchronises
 * `stream`.  Errors: FH_EINVAL, FH_ENOMEM, FH_EDEVICE. */
fh_status fh_project(fh_plan_t plan, const fh_peaks* peaks, int32_t n_cand, const double* f0, const double* k,
                     int32_t w, int32_t guard, int32_t* hist, fh_projection* out, void* stream);

const char* fh_status_str(fh_status s);
/* Library version string, and the gfx architecture it was built for. */
const char* fh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FH_H */
