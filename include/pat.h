/*
 * pat.h -- C ABI of the MI355X (gfx950) library for variational photoacoustic
 * tomography (PAT) reconstruction with preconditioned PDHGM.
 *
 * Method: Boink et al., "A Framework for Directional and Higher-Order
 * Reconstruction in Photoacoustic Tomography" (arXiv:1707.02245).
 *
 *   min_u 1/2 ||A u - f||^2 + R(u)                      (Sec. 2, eq. min_prob)
 *
 * with R = TV (eq. min_TV), TGV2 (eq. min_TGV), directional TV, the l1 norm
 * of dual-tree wavelet coefficients (eq. min_wav) or Tikhonov (LS-T, Sec. 2),
 * solved in saddle-point form (Sec. 3.1) by the first-order
 * primal-dual algorithm PDHGM (Algorithms 1 and 2) with diagonal or two-block
 * step sizes (Sec. 3.3.2) and the primal-dual gap as stopping rule (Sec. 3.3.3).
 *
 * Conventions shared by every entry point:
 *  - Data buffers are owned by the caller. Pointers named d_* are device
 *    pointers (HIP global memory on the current device), borrowed for the
 *    duration of the stream-ordered call; the library never frees them.
 *  - Handles (pat_geometry, pat_precond_h, pat_unet) are owned by the
 *    library and released only by their *_destroy function.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    Calls are asynchronous with respect to the host unless documented.
 *  - Images are row-major [ny][nx] with y increasing with the row index and
 *    pixel (ix, iy) centred at (x_min + (ix+1/2) h, y_min + (iy+1/2) h).
 *    Data are row-major [n_det][n_t] (bin b = d * n_t + k).
 *  - Element type is fixed per geometry: float (PAT_F32) or double (PAT_F64).
 *  - Return value < 0: error, outputs untouched, pat_last_error() explains.
 *    Return value > 0: warning, outputs valid. Handles may be used by one
 *    host thread at a time. No C++ exception crosses this boundary.
 */
#ifndef PAT_H
#define PAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PAT_OK = 0,
  PAT_NOT_CONVERGED = 1,      /* iteration cap reached before the gap target */
  PAT_ERR_INVALID_ARG = -1,   /* rejected before any device work */
  PAT_ERR_OOM = -2,           /* device allocation failed */
  PAT_ERR_DEVICE = -3,        /* HIP runtime error (message in pat_last_error) */
  PAT_ERR_NUMERIC = -4,       /* non-finite gap during iteration */
  PAT_ERR_UNSUPPORTED = -5    /* valid request this build does not implement */
} pat_status;

typedef enum { PAT_F32 = 0, PAT_F64 = 1 } pat_dtype;

typedef struct pat_geometry_s* pat_geometry;
typedef struct pat_precond_s* pat_precond_h;

/*
 * Acquisition geometry (Sec. 3.3.1 discretisation; Sec. 4.1 eq. K_def).
 *
 * Point detectors sit on a circle arc of radius det_radius about
 * (det_cx, det_cy): a closed circle (arc_span = 2 pi) places detector d at
 * angle arc_center + 2 pi d / n_det; a shorter arc spaces them evenly from
 * arc_center - arc_span/2 to arc_center + arc_span/2, both ends included.
 * If det_xy is non-NULL it gives explicit host positions [n_det][2] instead.
 *
 * Time sample k measures the mean of the image over the circle of radius
 * r_k = c (t0 + k dt) about the detector, sampled at M_k = max(1,
 * 4 ceil(2 pi r_k samples_per_pixel / (4 h))) points (the arc length in
 * samples rounded up to a multiple of four, so each circle's samples are
 * invariant under quarter turns) at angles 2 pi (m + 1/2) / M_k, each read by
 * bilinear interpolation with zero outside the grid:
 *
 *   A[(d,k), j] = (1/M_k) sum_m hat((X_dkm - x_j)/h) hat((Y_dkm - y_j)/h),
 *   hat(t) = max(0, 1 - |t|).
 *
 * Validation (PAT_ERR_INVALID_ARG): nx, ny >= 2; non-square pixels; n_det < 1;
 * n_t < 2; dt, c or samples_per_pixel <= 0; t0 < 0; any non-finite scalar;
 * nx, ny > 16384 or n_det * n_t > 2^28.
 */
typedef struct {
  int32_t nx, ny;
  double x_min, x_max, y_min, y_max;
  int32_t n_det;
  double det_cx, det_cy, det_radius, arc_center, arc_span;
  const double* det_xy;  /* optional host array [n_det][2]; NULL: use the arc */
  int32_t n_t;
  double t0, dt, c;
  double samples_per_pixel;
} pat_geometry_desc;

typedef struct {
  int32_t nx, ny, n_det, n_t;
  int64_t n_pix, n_bins;
  int64_t n_samples;      /* sum over bins of M_k (all arc samples) */
  int64_t n_window;       /* arc samples inside the clip windows (work per apply) */
  int32_t dtype;          /* pat_dtype */
  int32_t fwd_lanes_log2, adj_tile, adj_det_group; /* launch parameters */
  int32_t adj_mode;       /* 0 tile scatter, 1 stored CSR of A^T, 2 the CSR with
                           * LDS-staged input windows (in effect) */
  int64_t csr_nnz;        /* non-zeros of the stored A^T (-1: not built) */
  int32_t csr_tile_side;  /* pixel tile side of mode 2 (8 or 4; 0: none) */
  int32_t csr_win_max;    /* largest staged window of a tile, per quarter-turn
                           * slot (elements) */
  int32_t csr_rot;        /* 4: the stored A^T holds the rows of the first
                           * n_det/4 detectors only and the others follow by
                           * quarter turns; 1: all detectors stored */
  int32_t sym_rot;        /* 4: the geometry is quarter-turn symmetric (nx ==
                           * ny, n_det a multiple of 4, detector d + n_det/4 at
                           * the quarter turn of detector d about the grid
                           * centre, to 64 ulps); 1: not */
  int32_t csr_waves;      /* waves per workgroup of mode 2 (4, 8 or 16) */
  int32_t csr_lanes;      /* lanes per matrix row in mode 2 (16 or 64) */
  int32_t fwd_path;      /* forward: 0/1 gather (radius-/detector-major), 2 LDS tiles */
  int64_t fwd_pairs;      /* (bin, sample range) pairs of path 2 */
  int32_t fwd_sym;        /* 4: the forward runs in quarter-turn form (see
                           * pat_geometry_set_forward_symmetry); 1: not */
  int64_t fwd_entries;    /* non-zeros of the stored A of forward path 3
                           * (-1: not built, 0: not available) */
} pat_geometry_info;

/* Build the geometry tables on the device (FP64 host computation, rounded to
 * the element type) and the stored transpose A^T (CSR, rows = pixels, columns
 * sorted bins; Sec. 3.3.1 computes the matrix once). Synchronous with respect
 * to `stream` on return. Memory: about (6 + element size) bytes per non-zero,
 * roughly 3.7 non-zeros per (pixel, detector) pair, over a quarter of the
 * detectors on quarter-turn symmetric geometries. */
pat_status pat_geometry_create(const pat_geometry_desc* desc, pat_dtype dtype,
                               void* stream, pat_geometry* out);
pat_status pat_geometry_destroy(pat_geometry g);
pat_status pat_geometry_get_info(pat_geometry g, pat_geometry_info* out);
/* Launch parameters of the projector kernels (autotuner hook): forward lanes
 * per bin (log2: 4, 5 or 6 for 16, 32 or 64 lanes), adjoint tile edge (16, 32
 * or 64 pixels; FP64 uses 32 for 64) and detectors per adjoint workgroup
 * (1..n_det). Invalid values: PAT_ERR_INVALID_ARG. */
pat_status pat_geometry_set_launch(pat_geometry g, int32_t fwd_lanes_log2,
                                   int32_t adj_tile, int32_t adj_det_group);

/* How pat_adjoint and the solvers apply A^T: 0 = matrix-free tile scatter
 * (no stored matrix), 1 = stored CSR of A^T (built at geometry creation),
 * 2 = the same CSR read per 8x8 (or 4x4) pixel tile with the tile's input
 * windows staged in LDS and 16-bit window offsets (default; falls back to 1
 * when a tile's windows exceed 64 KB of LDS, reported by get_info). All give
 * the transpose of the same matrix (FP64 sample positions and the same weight
 * products); results agree to rounding order. Invalid mode:
 * PAT_ERR_INVALID_ARG. */
pat_status pat_geometry_set_adjoint(pat_geometry g, int32_t mode, void* stream);

/* How pat_forward and the solvers apply A (autotuner hook). 0 and 1: one
 * group of lanes per bin gathers its arc samples' 2x2 cells from the cached
 * image; a workgroup takes one radius for several detectors (0) or several
 * consecutive radii of one detector (1); both give the same result bit for
 * bit. 2: the image is cut into tiles of 64 x 64 cells staged in LDS; each
 * workgroup sums, for a chunk of the tile's (bin, sample range) pairs, the
 * samples whose cell lies in the tile, and a second pass adds each bin's
 * partial sums in a fixed order (same operator, different summation order).
 * 3 (quarter-turn symmetric geometries with the symmetric A^T storage): the
 * stored A of the first n_det/4 detectors, the stored quarter of A^T read the
 * other way (Sec. 3.3.1: the matrix computed once), grouped by 16 x 16 pixel
 * tiles; a workgroup stages its tile of the image turned by 0..3 quarter
 * turns in LDS and streams the tile's entries (one-byte pixel, weight) once
 * for the four quarters of the ring, and a second pass adds each bin's
 * per-tile partials in tile order. It is the exact transpose of the stored
 * A^T (same entries). About (1 + element size) bytes per stored non-zero.
 * Selecting path 2 or 3 builds its tables (synchronous on `stream`); path 3
 * on a geometry that does not allow it: PAT_ERR_UNSUPPORTED (also when a
 * tile touches more than 12288 bins); pat_geometry_set_symmetry(0) returns
 * the forward to path 0. Invalid path: PAT_ERR_INVALID_ARG. */
pat_status pat_geometry_set_forward_path(pat_geometry g, int32_t path, void* stream);

/* Workgroup shape of adjoint mode 2 (autotuner hook): waves per workgroup
 * (4, 8 or 16) and lanes per matrix row (16 or 64). Any valid pair gives the
 * same result up to summation order. Invalid values: PAT_ERR_INVALID_ARG. */
pat_status pat_geometry_set_tiled_launch(pat_geometry g, int32_t waves, int32_t row_lanes);

/* Whether the forward may use the quarter-turn symmetry (default 0;
 * pat_geometry_autotune turns it off; takes effect on symmetric geometries,
 * info.sym_rot == 4, with gather paths 0 and 1). The weights obey w(d + t n_det/4, k, R^t p) = w(d, k, p) for the quarter
 * turn R of the pixel grid, so the bins of detector d + t n_det/4 are those of
 * detector d on the image turned by t quarter turns: the gather then runs over
 * the first n_det/4 detectors and each arc sample's table entry, position and
 * cell serve four bins, read from the image and three turned copies (built by
 * a padding pass in stand-alone applies and by the primal step in the
 * solvers). Same operator; bins of the last three quarters agree with the
 * direct evaluation to rounding of the sample positions, and pat_adjoint with
 * the quarter-turn CSR is then its exact transpose. Solver instances take the
 * setting in effect when the solve starts. Invalid handle:
 * PAT_ERR_INVALID_ARG. */
pat_status pat_geometry_set_forward_symmetry(pat_geometry g, int32_t enable);

/* Whether the stored A^T may use the quarter-turn symmetry (default 1). On a
 * symmetric geometry (info.sym_rot == 4) the CSR then holds the rows of the
 * first n_det/4 detectors only, a quarter of the non-zeros, and modes 1 and 2
 * apply it to the four quarters of the data with the output turned by 0..3
 * quarter turns (w(d + n_det/4, k, R p) = w(d, k, p) for the quarter turn R
 * of the pixel grid). The result equals the full matrix's to rounding of the
 * sample positions. Rebuilds the CSR (synchronous on `stream`) when the choice
 * changes. Invalid handle: PAT_ERR_INVALID_ARG. */
pat_status pat_geometry_set_symmetry(pat_geometry g, int32_t enable, void* stream);

/* Autotuner of the projector launch parameters. Times, with HIP events over
 * `reps` stand-alone applies on `stream`, the forward with 16/32/64 lanes per
 * bin in either block order, by LDS tiles and (symmetric geometries) by the
 * stored A, and the adjoint as stored CSR or as tile scatter (tiles 16/32/64,
 * several detector-group sizes), and keeps the fastest of each; the
 * quarter-turn form of the gather is left off. If
 * cache_path is non-NULL the choice is read from / appended to that text
 * file, keyed by device architecture, geometry shape and element type, so a
 * later call with the same key times nothing. `out` may be NULL. */
typedef struct {
  int32_t fwd_lanes_log2, adj_mode, adj_tile, adj_det_group;
  double forward_ms, adjoint_ms;  /* measured (or cached) time per apply */
  int32_t from_cache;
} pat_autotune_result;
pat_status pat_geometry_autotune(pat_geometry g, const char* cache_path, int32_t reps,
                                 void* stream, pat_autotune_result* out);

/* f = A u (Sec. 4.1 eq. K_def, discretised as above).
 * d_u: device [ny][nx]; d_f: device [n_det][n_t]; element type of g. */
pat_status pat_forward(pat_geometry g, const void* d_u, void* d_f, void* stream);

/* u = A^T f, the exact matrix transpose of pat_forward (Sec. 3.3.1 uses the
 * transposed matrix, not a separately discretised adjoint). Deterministic.
 * d_f: device [n_det][n_t]; d_u: device [ny][nx]. */
pat_status pat_adjoint(pat_geometry g, const void* d_f, void* d_u, void* stream);

/* f = A u from a zero-bordered copy of the image, the form the solvers keep
 * (no padding pass). d_upad: device [ny + 2][nx + 2] with u at rows 1..ny,
 * columns 1..nx and zeros on the border (a non-zero border is read as image
 * and gives a different result); d_f: device [n_det][n_t]. */
pat_status pat_forward_padded(pat_geometry g, const void* d_upad, void* d_f, void* stream);

/* A^T f as the stored matrix computes it before any summation: in modes 1
 * and 2, info.csr_rot partial images (one per quarter turn) whose sum in
 * order 0, 1, ... is pat_adjoint's result; the solvers fold that sum into
 * their primal update. d_parts: device [csr_rot][ny][nx]. Mode 0 (matrix-free
 * scatter): PAT_ERR_UNSUPPORTED. */
pat_status pat_adjoint_partials(pat_geometry g, const void* d_f, void* d_parts, void* stream);

/* pat_adjoint for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result bit for bit, with the partial images that
 * pat_adjoint sums into d_u kept in a fixed 16 MiB device array of the
 * library (one per GPU, held until the process ends) instead of memory the
 * geometry allocates on first use. Nothing is allocated.
 * Needs csr_rot * N (stored A^T) or detector groups * N (matrix-free scatter)
 * elements of scratch, none when pat_adjoint writes d_u directly; more than
 * 16 MiB -> PAT_ERR_INVALID_ARG. The stored A^T must already exist in modes 1
 * and 2 (geometry creation or pat_geometry_set_adjoint builds it), else
 * PAT_ERR_INVALID_ARG. Calls on one GPU share its array: calls that overlap
 * in time on one GPU (different streams or host threads) race; calls ordered
 * on one stream do not. Arguments as pat_adjoint. */
pat_status pat_adjoint_noalloc(pat_geometry g, const void* d_f, void* d_u, void* stream);

/* Regulariser (Sec. 2.1, 2.2; Sec. 3.1 eqs. PD_TV, PD_TGV).
 *  TV      : lambda ||grad u||_{2,1}
 *  TGV     : lambda ||grad u - v||_{2,1} + tgv_alpha0 ||E v||_{F,1}
 *            (lambda = alpha, tgv_alpha0 = alpha beta in the paper's notation)
 *  DTV     : lambda ||D grad u||_{2,1}, D = I - (1 - dtv_eta) xi xi^T,
 *            xi = (-sin theta, cos theta), theta = d_dtv_theta [ny][nx]
 *            (device, element type of the geometry)
 *  TIKHONOV: lambda/2 ||u||^2 (LS-T, a test problem with a closed form)
 *  WAVELET : lambda ||W u||_1 (Sec. 2.2, eq. min_wav), W the dual-tree
 *            transform of pat_wavelet_forward with wav_levels levels; the
 *            dual variable holds one number per coefficient (4 N of them)
 * grad uses unit-spacing forward differences with a zero last difference;
 * E uses the backward differences -grad^T and counts the off-diagonal twice.
 * Validation: lambda < 0 or non-finite, tgv_alpha0 < 0, dtv_eta not in
 * (0, 1], DTV without d_dtv_theta, WAVELET with wav_levels outside 1..8 or
 * nx, ny not multiples of 2^wav_levels -> PAT_ERR_INVALID_ARG. */
typedef enum {
  PAT_REG_TV = 0, PAT_REG_TGV = 1, PAT_REG_DTV = 2, PAT_REG_TIKHONOV = 3, PAT_REG_WAVELET = 4
} pat_reg_kind;
typedef struct {
  int32_t kind;           /* pat_reg_kind */
  double lambda;
  double tgv_alpha0;
  double dtv_eta;
  const void* d_dtv_theta;
  int32_t wav_levels;     /* WAVELET: decomposition levels J (1..8) */
} pat_regulariser;

/* The dual-tree wavelet transform W of the wavelet model (Sec. 2.2, eq.
 * min_wav, which takes W from the dual-tree complex wavelet transform; the
 * paper does not print its filters, so this library fixes them):
 *  - 1-D filters: the orthonormal 4-tap Daubechies lowpass
 *    h = (1 + s, 3 + s, 3 - s, 1 - s) / (4 sqrt 2), s = sqrt 3, and its
 *    mirror highpass g[k] = (-1)^k h[3 - k]; periodic analysis
 *    y[i] = sum_k c[k] x[(2 i + k + shift) mod n].
 *  - Trees a and b: at level 1 tree b filters the signal advanced by one
 *    sample (shift 1), from level 2 on it uses the time-reversed filters of
 *    tree a (shift 0); tree a always uses h, g with shift 0.
 *  - 2-D: four separable trees (row tree, column tree) in {a, b}^2, each a
 *    J-level orthonormal transform recursing on its own lowpass band; per
 *    level and orientation (LH: lowpass along y, highpass along x; HL; HH)
 *    the four trees' bands combine into p = (aa - bb)/sqrt2,
 *    q = (aa + bb)/sqrt2, s = (ab + ba)/sqrt2, t = (ab - ba)/sqrt2; the four
 *    level-J lowpass bands stay per tree. All scaled by 1/2, so that
 *    W^T W = I and ||W|| = 1.
 *  - Coefficient order (4 N): for level j = 1..J, for orientation LH, HL,
 *    HH, for band p, q, s, t, the (ny/2^j) x (nx/2^j) band row-major; then
 *    the level-J lowpass bands of trees aa, ab, ba, bb.
 * pat_wavelet_forward: d_c = W d_u; pat_wavelet_adjoint: d_u = W^T d_c.
 * d_u: device [ny][nx], d_c: device [4 nx ny], element type `dtype`
 * (pat_dtype); arithmetic in the element type. d_work: device work buffer
 * for the lowpass bands between levels, at least pat_wavelet_work_elems
 * elements (nx ny + ceil(nx ny / 4)) of the element type, 16-byte aligned,
 * owned by the caller
 * (the call is then stream-ordered and allocates nothing); NULL: the call
 * allocates one and returns once `stream` has finished. Validation: levels
 * outside 1..8, nx or ny not a positive multiple of 2^levels, NULL d_u or
 * d_c, unknown dtype -> PAT_ERR_INVALID_ARG. */
int64_t pat_wavelet_work_elems(int32_t nx, int32_t ny);
pat_status pat_wavelet_forward(int32_t dtype, int32_t nx, int32_t ny, int32_t levels,
                               const void* d_u, void* d_c, void* d_work, void* stream);
pat_status pat_wavelet_adjoint(int32_t dtype, int32_t nx, int32_t ny, int32_t levels,
                               const void* d_c, void* d_u, void* d_work, void* stream);

/* Step sizes (Sec. 3.3.2).
 *  DIAG : sigma_i = 1 / sum_j |K_ij|, tau_j = 1 / sum_i |K_ij| over the
 *         stacked operator K = [A; B] (TGV: [A 0; grad -I; 0 E]); the rows of
 *         one pixel's dual vector share the smallest of their sigmas; rows
 *         with no entries get sigma = 1. WAVELET: the rows of W take
 *         sigma = 1 and tau_j = 1 / (sum_i |A_ij| + 1): with W^T W = I,
 *         ||W x|| = ||x|| takes the place of W's column sums in the bound
 *         ||Sigma^(1/2) K T^(1/2)|| <= 1.
 *  BLOCK: scalar sigma1 (data), sigma2 (regulariser) and tau with
 *         sigma_i tau L_i^2 = 0.99/4, tau = 1/(2 max(L1, L2)), L1 = ||A||,
 *         L2 = ||B|| (TGV: the block [grad -I; 0 E]); norms by 1000 power
 *         iterations times 1.05 (WAVELET: L2 = ||W||, the same way). */
typedef enum { PAT_PRECOND_DIAG = 0, PAT_PRECOND_BLOCK = 1 } pat_precond_kind;

/* Compute step sizes for (g, reg). The handle keeps device arrays and must
 * be used with the same geometry and regulariser. Synchronous on return. */
pat_status pat_precond(pat_geometry g, const pat_regulariser* reg, int32_t kind,
                       void* stream, pat_precond_h* out);
/* Export one step-size array to caller memory (device, element type of g):
 * which = 0 sigma_q [n_bins], 1 sigma_r [N] (WAVELET: [4 N]), 2 sigma_s [N] (TGV),
 * 3 tau_u [N], 4 tau_v [2][N] (TGV). Missing arrays: PAT_ERR_INVALID_ARG. */
pat_status pat_precond_get(pat_precond_h p, int32_t which, void* d_dst, void* stream);
pat_status pat_precond_destroy(pat_precond_h p);

/* Solver state for warm restarts and resume, in one device buffer of the
 * geometry's element type, concatenated in this order:
 *   u [N], ubar [N], q [n_bins], r [2][N] (TV, TGV, DTV) or [4 N] (WAVELET,
 *   in the coefficient order of pat_wavelet_forward),
 *   TGV only: v [2][N], vbar [2][N], s [3][N] (s_xx, s_xy, s_yy).
 * pat_state_elems gives the length in elements. */
pat_status pat_state_elems(pat_geometry g, int32_t reg_kind, int64_t* out);

typedef struct {
  int32_t max_iter;       /* iterations to run (cap); > 0 */
  double gap_tol;         /* stop when rel_gap <= gap_tol; <= 0: run max_iter */
  int32_t gap_every;      /* gap interval in iterations (>= 1) */
  int32_t graph_block;    /* iterations per captured HIP graph (>= 0; 0 = off),
                           * rounded up to a multiple of gap_every. The gap is
                           * evaluated, and stopping decided, once per block:
                           * every graph_block iterations (every gap_every with
                           * graphs off) and at max_iter. */
  double theta;           /* extrapolation, 1.0 */
  double gap_box;         /* C of the box-restricted gap; > 0 */
  const void* d_u0;       /* optional warm start [ny][nx]; NULL = zero */
  const void* d_y0;       /* optional dual start with d_u0 (TV, dTV): q [n_bins]
                           * then r [2][N]; NULL = zero */
  const void* d_state_in; /* optional full state to resume from; NULL = none */
  void* d_state_out;      /* optional: receives the final state */
  pat_precond_h precond;  /* NULL: DIAG computed for this call */
  /* Accelerated PDHGM (Sec. 3.3: the O(1/n^2) variant, Chambolle and Pock's
   * Algorithm 2) on the preconditioned steps: iteration n uses the dual steps
   * b_n Sigma and the primal steps a_n T and extrapolates with theta_n,
   *   a_0 = b_0 = 1, theta_n = 1/sqrt(1 + 2 accel_gamma a_n),
   *   a_{n+1} = theta_n a_n, b_{n+1} = b_n / theta_n,
   * until an update would take b above accel_step_max; from then on
   * theta = 1 and the steps stay fixed (plain PDHGM with steps a T, b Sigma,
   * so the solve converges to a saddle point of the same problem).
   * accel_gamma is the modulus of strong convexity of G in the metric of T
   * (Tikhonov: lambda times the smallest tau_u); for TV, TGV and dTV (G = 0)
   * a positive value is a step-ratio schedule, not a rate guarantee.
   * accel_gamma = 0: plain PDHGM with `theta` (accel_step_max unused).
   * accel_gamma > 0 needs theta = 1 and accel_step_max >= 1. The schedule
   * restarts from a = b = 1 on d_state_in. */
  double accel_gamma;
  double accel_step_max;
} pat_solve_opts;

typedef struct {
  int32_t iters, converged, fallback;
  double rel_gap, gap, primal, fstar, kty_l1, residual, seconds;
} pat_solve_info;

/* PDHGM (Algorithm 1 for TV/DTV/WAVELET/LS-T, Algorithm 2 for TGV) with theta
 * extrapolation, from zero, from d_u0, or from d_state_in. The gap of
 * Sec. 3.3.3 is taken with x restricted to the box ||x||_inf <= gap_box
 * (the printed gap is infinite when G = 0):
 *   gap = P(x) + 1/2||q||^2 + <q, f> + gap_box ||K^T y||_1, rel_gap = gap / P(x).
 * A warm start that is non-finite (u0, or y0 when given) or has
 * P(u0) > P(0) = 1/2||f||^2 is replaced by zero (info->fallback = 1); ubar
 * starts at u0.
 * d_f: device data [n_det][n_t]; d_u_out: device image [ny][nx].
 * Returns PAT_OK when rel_gap <= gap_tol (or max_iter ran with gap_tol <= 0),
 * PAT_NOT_CONVERGED at the cap, PAT_ERR_NUMERIC on a non-finite gap.
 * Synchronous on return (info is filled). */
pat_status pat_pdhg_solve(pat_geometry g, const void* d_f, const pat_regulariser* reg,
                          const pat_solve_opts* opts, void* d_u_out,
                          pat_solve_info* info, void* stream);

/* n independent reconstructions advanced together: every kernel launch covers
 * all active instances (one element type for the whole batch), instances
 * that share a geometry share each pass over its stored A^T (up to 8 per
 * pass), iterations run in captured HIP graphs of opts[0].graph_block
 * iterations (gap every opts[0].gap_every), and instances whose gap reaches
 * their gap_tol retire at block ends. Arrays have n entries; per instance the
 * arguments mean what they mean for pat_pdhg_solve. Returns PAT_OK if all
 * converged, PAT_NOT_CONVERGED if any hit its cap. Synchronous on return. */
pat_status pat_pdhg_solve_batched(int32_t n, const pat_geometry* g, const void* const* d_f,
                                  const pat_regulariser* reg, const pat_solve_opts* opts,
                                  void* const* d_u_out, pat_solve_info* info, void* stream);

/* Per-kernel timing of the solver's iteration (a benchmark and tuning hook):
 * sets up the n instances as pat_pdhg_solve_batched does (zero start; each
 * instance's own step sizes unless opts[i].precond is given), then times
 * each launch of an iteration with HIP events on `stream`, `reps` launches
 * after one untimed launch, and writes the average per launch in ms:
 *   ms[0] the forward launch (A ubar with the dual data step, Sec. 3.2 prox of
 *         F1*, and the regulariser's dual step in the same launch),
 *   ms[1] the regulariser's dual step alone (r, and s for TGV; WAVELET: the
 *         transform's dual step and W^T r, which run outside the forward),
 *   ms[2] A^T q into the partial images,
 *   ms[3] the primal step (u, v and the extrapolation).
 * Every launch covers all instances. The state the timed launches leave is
 * discarded. Arguments as pat_pdhg_solve_batched (d_u0, d_y0 and d_state_in
 * must be NULL); reps >= 1. Synchronous on return. */
pat_status pat_pdhg_kernel_times(int32_t n, const pat_geometry* g, const void* const* d_f,
                                 const pat_regulariser* reg, const pat_solve_opts* opts,
                                 int32_t reps, double* ms, void* stream);

/* ---- Learned warm start -------------------------------------------------
 * A U-Net (`levels` levels, base_ch channels at the top, doubling per level;
 * 3x3 convolutions with ReLU, 2x2 max pooling, 2x2 stride-2 transposed
 * convolutions, skip concatenation, 1x1 head with out_ch outputs) maps the
 * normalised backprojection x = (A^T f / A^T 1) / s, s = mean |A^T f / A^T 1|,
 * to the normalised TV reconstruction u / s (output 0) and, with out_ch = 3,
 * its dual variable r / lambda (outputs 1, 2). Weights are FP32 masters used
 * as bf16 in the matrix-core convolutions (FP32 accumulation); activations
 * and the gradients passed between layers are bf16. The network only changes
 * where PDHG starts (pat_solve_opts.d_u0, d_y0); the gap decides the result.
 * Inputs are device FP32 [n][h][w]; outputs and targets device FP32 channel
 * planes [n][out_ch][h][w]; h and w divisible by 2^(levels-1).
 * Parameters are one FP32 vector in the order: per level l = 0..levels-1 two
 * 3x3 convolutions (weights [Cout][3][3][Cin], bias [Cout]); per decoder level
 * l = levels-2..0 the transposed convolution ([2][2][Cin][Cout], [Cout]) and
 * two 3x3 convolutions; the head ([out_ch][C0], [out_ch]). */
typedef struct pat_unet_s* pat_unet;
typedef struct {
  int32_t epochs, batch;  /* passes over the data; images per Adam step */
  double lr;              /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
  uint64_t seed;          /* shuffling order */
} pat_train_opts;

/* He-normal weights from `seed`, zero biases; levels in [2, 6], base_ch a
 * multiple of 4 in [4, 256], out_ch in [1, 4]. */
pat_status pat_warmstart_create(int32_t levels, int32_t base_ch, int32_t out_ch, uint64_t seed,
                                pat_unet* out);
pat_status pat_warmstart_destroy(pat_unet n);
pat_status pat_warmstart_num_params(pat_unet n, int64_t* out);
/* Tile rule of the matrix-core convolution GEMMs, process-wide (a tuning and
 * test hook): 0 automatic (128x128 or 128x64 tiles only where the launch has
 * at least 1024 workgroups, else 64x64), 1 the largest tile the column count
 * allows, 2 128x64, 3 64x64; layers with at most 32 output columns always
 * take 128x32, and products of at most 32 rows (the weight gradients of
 * 32-channel layers) 32x64. The tiles differ only in how output elements are grouped into
 * workgroups; each element accumulates along k in the same chunks. Invalid
 * mode: PAT_ERR_INVALID_ARG. */
pat_status pat_warmstart_set_gemm_tiles(int32_t mode);
/* Copy the FP32 parameter vector to / from device memory (set resets Adam). */
pat_status pat_warmstart_get_params(pat_unet n, float* d_dst, void* stream);
pat_status pat_warmstart_set_params(pat_unet n, const float* d_src, void* stream);
/* y = net(x) for `batch` images: d_in [batch][h][w], d_out [batch][out_ch][h][w]. */
pat_status pat_warmstart_forward(pat_unet n, int32_t batch, int32_t h, int32_t w, const float* d_in,
                                 float* d_out, void* stream);
/* Mean squared error of net(x) against d_target (over all outputs) and its
 * gradient with respect to every parameter (device FP32 [num_params]);
 * *loss (host) if non-NULL. */
pat_status pat_warmstart_grad(pat_unet n, int32_t batch, int32_t h, int32_t w, const float* d_in,
                              const float* d_target, float* d_grad, double* loss, void* stream);
/* Adam on the mean squared error over `count` pairs, `epochs` shuffled passes
 * in batches of opts->batch (count / batch steps per epoch). *final_loss
 * (host): mean loss of the last epoch. PAT_ERR_NUMERIC if it is non-finite. */
pat_status pat_warmstart_train(pat_unet n, int32_t count, int32_t h, int32_t w, const float* d_inputs,
                               const float* d_targets, const pat_train_opts* opts, double* final_loss,
                               void* stream);
/* Checkpoint: parameters and Adam state, raw little-endian with a header
 * ("PATUNET2", levels, base_ch, out_ch, num_params, step as int64). */
pat_status pat_warmstart_save(pat_unet n, const char* path);
pat_status pat_warmstart_load(pat_unet n, const char* path);
/* Network input (and target) of one measurement: d_f data of g (element type
 * of g). Outputs FP32: d_x [ny][nx] the normalised backprojection and
 * d_scale[0] = s. With d_state (a solver state of g, layout of
 * pat_state_elems, e.g. pat_solve_opts.d_state_out of a TV solve) the target
 * planes d_t [t_channels][ny][nx]: u / s, and with t_channels = 3 also
 * r_x / lambda, r_y / lambda (reg: the TV regulariser of that solve). */
pat_status pat_warmstart_normalize(pat_geometry g, const pat_regulariser* reg, const void* d_f,
                                   const void* d_state, float* d_x, float* d_t, int32_t t_channels,
                                   float* d_scale, void* stream);
/* Starting point for pat_pdhg_solve from data d_f of g (element type of g):
 * d_u0 = s net(x)[0]. With d_y0 (out_ch = 3, reg TV) also the dual start
 * q0 = A u0 - f [n_bins] followed by r0 = lambda P(net(x)[1], net(x)[2])
 * [2][N], P the projection onto the unit disc per pixel. Synchronous. */
pat_status pat_warmstart_infer(pat_unet n, pat_geometry g, const pat_regulariser* reg, const void* d_f,
                               void* d_u0, void* d_y0, void* stream);

/* ---- Calibrated forward model and preprocessing (Sec. 4.1, 4.2) ----------
 * The measured pressure at detector x_d is the circular projection of the
 * image convolved in time with the calibration measurement of a point source
 * at x_p taken at retarded time (eq. FW_full). With the circular-mean
 * operator A of this library, (1/t) K u = 2 pi c A u, so
 *   p_d = s_d (A u)_d *_t pcal_d(. + tau_d),
 *   s_d = 2 pi c |x_d - x_p|,  tau_d = |x_d - x_p| / c,
 * where the sampled convolution is dt sum_j a_j b_{k-j}. Preprocessing
 * deconvolves with the regularised filter of eq. deconv and rescales
 * (eq. f_rewrite):
 *   f_d = F^-1{ F{p_d} conj(D_d) / (|D_d|^2 + eps) } / s_d,
 *   D_d = dt F{pcal_d} exp(i omega tau_d),
 * which gives A u back when the calibration spectrum has no zeros and eps is
 * small. Every transform is an L-point DFT, L the smallest power of two
 * >= 2 n_t (zero padding; at most 4096), so the retarded shift is a phase
 * ramp. Signals are device arrays [n_det][n_t] in the element type of the
 * geometry, sampled like the data; the transforms run in FP64. */
typedef struct pat_calib_s* pat_calib;
/* Spectra of the calibration d_pcal [n_det][n_t] (the pressure each detector
 * recorded from a point source at (xp, yp)) with regularisation eps > 0,
 * computed once on the device. A detector at the source, eps <= 0 or
 * non-finite values: PAT_ERR_INVALID_ARG; n_t > 2048: PAT_ERR_UNSUPPORTED.
 * The handle keeps g, which must outlive it. Synchronous. */
pat_status pat_calib_create(pat_geometry g, const void* d_pcal, double xp, double yp, double eps, void* stream,
                            pat_calib* out);
pat_status pat_calib_destroy(pat_calib c);
/* d_p = measured pressure of image d_u [ny][nx] (eq. FW_full). */
pat_status pat_pressure_forward(pat_calib c, const void* d_u, void* d_p, void* stream);
/* d_f = data for the reconstruction from measured pressure d_p (eqs. deconv,
 * f_rewrite). d_p and d_f may not overlap. */
pat_status pat_preprocess(pat_calib c, const void* d_p, void* d_f, void* stream);

/* Peak signal-to-noise ratio of an image against its ground truth (Sec. 5.4),
 * in the form the paper prints (maximum of the ground truth not squared)
 * and in the standard form:
 *   printed  = 10 log10(max(u_gt) / (||u - u_gt||^2 / n)),
 *   standard = 10 log10(max(u_gt)^2 / (||u - u_gt||^2 / n)).
 * d_u, d_gt: device arrays of n elements of `dtype`; FP64 reductions on the
 * GPU in a fixed order. Results to host doubles; +inf when u == u_gt.
 * n < 1, NULL pointers: PAT_ERR_INVALID_ARG; max(u_gt) <= 0 or non-finite
 * values: PAT_ERR_NUMERIC. Synchronous on return. */
pat_status pat_psnr(int32_t dtype, int64_t n, const void* d_u, const void* d_gt, double* psnr_printed,
                    double* psnr_standard, void* stream);

const char* pat_status_string(pat_status s);
/* Message of the last error on the calling thread ("" if none). */
const char* pat_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PAT_H */
