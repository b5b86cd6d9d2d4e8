// Host-side structures and launcher declarations of libpat.
#pragma once

#include "pat_common.hpp"

// The opaque handle of pat.h.
struct pat_geometry_s {
  pat_geometry_desc desc{};
  std::vector<double> det_xy;  // [n_det][2] world coordinates
  int dtype = PAT_F32;
  int nx = 0, ny = 0, n_det = 0, n_t = 0;
  double h = 0.0;
  std::vector<int> M, off;     // arc samples per radius and table offsets
  std::vector<double> radius;  // r_k
  int64_t n_samples_per_det = 0;
  int64_t n_window = 0;        // samples inside the clip windows, all bins
  pat::DevBuf d_det, d_rad, d_moff, d_cs, d_win;
  // launch parameters
  int lanes_log2 = 6, tile = 32, det_group = 16;
  int fwd_path = 0;  // forward path: 0/1 gather (see fwd_grid), 2 LDS tiles, 3 stored A
  // LDS-tiled forward (path 2): pairs {bin, m0, m1, partial slot} in tile
  // order, workgroup descriptors {cell x0, cell y0, first pair, end pair},
  // per-bin offsets of the partial sums (bin-major)
  pat::DevBuf fwd_pair, fwd_block, fwd_bin_off, scratch_fpart;
  int64_t fwd_n_pairs = -1;  // -1: not built
  int fwd_n_blocks = 0;
  // adjoint: 0 = tile scatter (matrix-free), 1 = stored CSR of A^T,
  // 2 = stored CSR with the input windows of pixel tiles staged in LDS
  int adj_mode = 2;
  pat::DevBuf csr_ptr, csr_col, csr_val;
  int64_t csr_nnz = -1;  // -1: not built
  // quarter-turn symmetry: sym_rot = 4 when detector d + n_det/4 sits at the
  // quarter turn of detector d about the centre of a square grid (1 if not);
  // csr_rot = 4 when the stored A^T holds the first n_det/4 detectors only
  int sym_rot = 1, csr_rot = 1;
  bool sym_enabled = true;
  // the forward in quarter-turn form on symmetric geometries (gather paths;
  // off by default, the autotuner times it)
  bool fwd_sym = false;
  bool fwd_qt() const { return fwd_sym && sym_rot == 4 && fwd_path < 2; }
  // pixel tiles of the stored A^T (side 0: windows too large for LDS);
  // csr_win_max is per quarter-turn slot
  int csr_side = 0, csr_tiles_x = 0, csr_tiles_y = 0, csr_win_max = 0;
  // waves per workgroup of the tiled kernel (4, 8 or 16) and lanes per row
  // (16 or 64)
  int csr_waves = 4, csr_lanes = 16;
  pat::DevBuf csr_lcol, csr_win;  // uint16 per non-zero; int4 per (tile, detector)
  // scratch of the stand-alone applies
  pat::DevBuf scratch_pad, scratch_part;
  // radii by decreasing samples in their clip windows (over all detectors)
  pat::DevBuf d_kord;
  // forward path 3: the stored A of the first n_det/4 detectors by pixel
  // tiles (GeomDev fm_*); fm_entries -1: not built, 0: not available
  pat::DevBuf fm_off, fm_w, fm_seg, fm_chunk, fm_binseg, fm_segidx;
  int64_t fm_entries = -1;
  int fm_nseg = 0, fm_nchunk = 0, fm_tiles_x = 0;
  void ensure_fmat(hipStream_t s);
  void drop_fmat();

  void build_host();
  void upload(hipStream_t stream);
  void set_launch(int lanes_log2, int tile, int det_group);
  void default_launch();
  pat::GeomDev dev() const;
  void ensure_csr(hipStream_t s);
  void ensure_fwd_tiles(hipStream_t s);
  int n_csr_tiles() const { return csr_tiles_x * csr_tiles_y; }
  int csr_det() const { return n_det / csr_rot; }  // detectors in the stored A^T
  void drop_csr();
  // the adjoint mode in effect (2 falls back to 1 without tiles)
  int effective_adj_mode() const { return adj_mode == 2 && csr_side == 0 ? 1 : adj_mode; }
  int64_t n_bins() const { return (int64_t)n_det * n_t; }
  int64_t n_pix() const { return (int64_t)nx * ny; }
  int n_groups() const { return (n_det + det_group - 1) / det_group; }
  int adj_blocks() const {
    return ((nx + tile - 1) / tile) * ((ny + tile - 1) / tile) * n_groups();
  }
};

// Step sizes of one (geometry, regulariser) pair.
struct pat_precond_s {
  pat_geometry g = nullptr;
  int reg_kind = 0;
  int kind = PAT_PRECOND_DIAG;
  double L1 = 0.0, L2 = 0.0;  // BLOCK mode norms
  // WAVELET: every coefficient's dual step is this one value (DIAG 1, BLOCK
  // sigma2); sigma_r holds it per coefficient for export only
  double sigma_w = 1.0;
  pat::DevBuf sigma_q, sigma_r, sigma_s, tau_u, tau_v;
};

namespace pat {

void validate_geometry_desc(const pat_geometry_desc* d);
void validate_regulariser(const pat_geometry_s* g, const pat_regulariser* r);

enum FwdMode { FWD_PLAIN = 0, FWD_DUAL = 1, FWD_GAP = 2, FWD_ROWSUM = 3 };

constexpr int kThreads = 256;

// Forward grid (the blocks whose epilogue writes bins and gap sums): paths 0
// and 1 gather with one block per group of 256/lanes bins, path 0 (radius-
// major) grouping detectors of one radius, path 1 (detector-major) radii of
// one detector; path 2 sums partials with one thread per bin.
inline int fwd_grid(int n_det, int n_t, int lanes_log2, int path) {
  const int bpb = kThreads >> lanes_log2;
  if (path == 2) return (int)(((int64_t)n_det * n_t + kThreads - 1) / kThreads);
  return path == 1 ? n_det * ((n_t + bpb - 1) / bpb) : ((n_det + bpb - 1) / bpb) * n_t;
}
// LDS-tiled forward: tile side in cells, pairs and threads per workgroup
constexpr int kFwdTile = 64;
constexpr int kFwdChunk = 256;
constexpr int kFwdTileThreads = 256;
inline int pix_blocks(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

// Batched launch tables: args arrays and instance block offsets on the device.
template <class T>
struct Launch {
  int n = 0;
  DevBuf fwd, fwd_gap, adj, inst, gapfin;  // FwdArgs x2 / AdjArgs / InstDev / GapFinishArgs
  DevBuf fwd_start, adj_start, pix_start;
  int fwd_total = 0, adj_total = 0, pix_total = 0;
  // instances whose adjoint is the stored CSR of A^T
  DevBuf csr, csr_start;
  int n_adj = 0, n_csr = 0, csr_total = 0, csr_max_rhs = 1;
  bool csr_tiled = false;  // LDS-staged kernel for every CSR group
  size_t csr_shm = 0;      // its dynamic LDS per workgroup
  int csr_waves = 4;       // its waves per workgroup
  int csr_lanes = 16;      // its lanes per row
  // LDS-tiled forward for every instance: gather blocks (per-instance
  // workgroup descriptors) before the per-bin sums
  bool fwd_tiled = false;
  DevBuf fwdt_start;
  int fwdt_total = 0;
  // instances grouped by geometry, up to four per group (gather forward):
  // each forward block serves a whole group. fwd_ni slots per group (the
  // largest group; unused slots have no image), group block offsets in
  // fwdg_start; fwd_ni == 1 when no two instances share a geometry
  DevBuf fwdg, fwdg_gap, fwdg_start;
  int fwd_ni = 1, fwd_ni_blocks = 0, fwd_ni_groups = 0;
  // instances whose forward is the stored A (path 3): their slot-form args
  // (dual / gap), workgroup offsets of the tile pass and of the per-bin pass
  DevBuf fm, fm_gap, fm_start, fmr_start;
  int fm_n = 0, fm_total = 0, fmr_total = 0;
  int lanes_log2 = 6;   // shared by every instance of one launch
  int max_tile = 32;    // shared by every instance of one launch
};

// ---- launchers (projector.hip)
template <class T>
void launch_pad(const T* u, T* upad, int nx, int ny, hipStream_t s);
template <class T>
void launch_forward(int mode, const FwdArgs<T>& a, int lanes_log2, hipStream_t s);
// quarter-turn forward: the padded image and its turned copies (slots), and
// the gather over a quarter of the detectors in slot form (PLAIN or DUAL)
template <class T>
void launch_rot_pad(const T* src, bool src_padded, T* dst, int n, int slots, hipStream_t s);
template <class T>
void launch_forward_qt(int mode, const FwdArgs<T>& a, int lanes_log2, hipStream_t s);
template <class T>
void launch_forward_batched(int mode, const Launch<T>& L, int lanes_log2, hipStream_t s);
// forward with the data term's dual step and the regulariser's dual step in
// one launch (two launches for the LDS-tiled forward)
template <class T>
void launch_forward_reg_batched(const Launch<T>& L, int lanes_log2, hipStream_t s);
template <class T>
void attach_fwd_part(pat_geometry_s* g, FwdArgs<T>& a);
template <class T>
void launch_adjoint(const AdjArgs<T>& a, hipStream_t s);
template <class T>
void launch_adjoint_batched(const Launch<T>& L, hipStream_t s);
template <class T>
void launch_reduce_groups(const T* part, T* out, int n_groups, int64_t n, hipStream_t s);

// Stand-alone applies (scratch owned by the geometry; adjoint by its mode).
template <class T>
void apply_forward(pat_geometry_s* g, const T* u, T* f, hipStream_t s);
template <class T>
void apply_adjoint(pat_geometry_s* g, const T* f, T* u, hipStream_t s);
// Bytes of partial images the stand-alone A^T sums into its output (0: it
// writes the output directly), and A^T with those partials in caller-given
// device memory (nothing allocated; the stored A^T must already exist in
// modes 1 and 2).
size_t adjoint_scratch_bytes(const pat_geometry_s* g);
template <class T>
void apply_adjoint_scratch(pat_geometry_s* g, const T* f, T* u, T* scratch, hipStream_t s);

// ---- stored A by pixel tiles, forward path 3 (fmat.hip)
constexpr int kFmSide = 16;             // tile side (a pixel in one byte)
constexpr int kFmChunkEntries = 4096;   // entries per workgroup (whole segments)
template <class T>
void build_fmat(pat_geometry_s* geo, hipStream_t s);
// workgroups of the per-bin pass over n_det (a quarter) x n_t bins
inline int fmat_reduce_blocks(int n_det, int n_t) { return (int)(((int64_t)n_det * n_t + 15) / 16); }
// A u of one instance in quarter-turn slot form (a.g.n_det the quarter,
// a.part 4 partials per segment, slot fields set); mode PLAIN
template <class T>
void launch_forward_fmat(int mode, const FwdArgs<T>& a, hipStream_t s);
// the path-3 instances of a batch (L.fm*), mode DUAL (with the regulariser's
// dual step of every instance in the same launch when fused) or GAP
template <class T>
void launch_fmat_batched(int mode, bool fused_reg, const Launch<T>& L, hipStream_t s);

// ---- stored A^T (csr.hip)
template <class T>
void build_csr_adjoint(pat_geometry_s* geo, hipStream_t s);
void build_csr_tiles(pat_geometry_s* geo, size_t esz, hipStream_t s);
// per pixel tile (side x side) and stored detector: {first radius, radii, 0, 0}
// of the tile's non-zeros in the stored A^T
void launch_csr_windows(const pat_geometry_s* geo, int side, int tiles_x, int64_t n_tiles, int4* win,
                        hipStream_t s);
template <class T>
void launch_csr_spmv(const CsrArgs<T>& a, hipStream_t s);
template <class T>
void launch_csr_spmv_batched(const CsrArgs<T>* arr, const int* starts, int n_inst, int total_blocks,
                             hipStream_t s, bool wide = false);
template <class T>
void launch_csr_spmm_batched(const CsrMultiArgs<T>* arr, const int* starts, int n_grp, int total_blocks,
                             hipStream_t s, bool wide, int max_rhs);
// LDS-staged variant: one block per pixel tile, the input windows of every
// right-hand side staged in dynamic LDS (shm bytes: max_rhs times the largest
// lds_stride of the groups, times sizeof(T); every slot up to max_rhs is
// read). A geometry gets tiles when one
// right-hand side fits kCsrLdsBytes; groups of several right-hand sides may use
// up to the workgroup LDS of the device (prepare_csr_tiled raises the kernels'
// limit beyond 64 KB, outside any graph capture).
constexpr int kCsrLdsBytes = 64 * 1024;
constexpr int64_t kCsrSlack = 256;  // zero entries after the values and window offsets
int device_lds_per_block();
template <class T>
void launch_csr_tiled(const CsrMultiArgs<T>& a, hipStream_t s, bool wide, int waves, int lanes);
template <class T>
void launch_csr_tiled_batched(const CsrMultiArgs<T>* arr, const int* starts, int n_grp, int total_blocks,
                              size_t shm, hipStream_t s, bool wide, int max_rhs, int waves, int lanes);
// Default workgroup shape of the tiled kernel for a dynamic LDS size and
// element size: 16 waves when the windows leave room for a single workgroup
// per CU (160 KB of LDS), 8 for 4-byte elements (their wide loads leave each
// wave fewer instructions to issue) or when at most two workgroups fit, else
// 4 (three or more workgroups per CU).
inline int csr_waves_for(size_t shm, size_t esz) {
  if (shm > 80 * 1024) return 16;
  return (esz == 4 || 3 * shm > 160 * 1024) ? 8 : 4;
}
// Default lanes per row for a mean row length (entries): 64 for long rows.
inline int csr_lanes_for(double mean_row) { return mean_row >= 512.0 ? 64 : 16; }
// Multi-RHS plain kernel for one group given on the host.
template <class T>
void launch_csr_spmm(const CsrMultiArgs<T>& a, hipStream_t s, bool wide);
template <class T>
void prepare_csr_tiled(int max_rhs, size_t shm);

// ---- dual-tree wavelet transform W (wavelet.hip)
constexpr int kWavMaxLevels = 8;
// The image W reads: img[y * pitch + x], y < ny, x < nx (nx, ny multiples of 2^levels).
template <class T>
struct WavInput {
  int nx, ny, levels;
  const T* img;
  int pitch;
};
// Where the coefficients go: coef (W u), the dual step on r, or the gap sum.
template <class T>
struct WavDual {
  T* coef;
  T* r;                // dual variable [4 N]
  T sigma;             // its step size (one value for all coefficients)
  const double* mult;  // step multipliers of the accelerated schedule, or null
  T lam;
  double* red;         // gap: wav_gap_blocks partial sums
};
// Work buffer of the lowpass bands between levels (elements of the arithmetic type).
int64_t wav_work_elems(int nx, int ny);
// Partial sums the gap pass writes (one per workgroup, levels in order).
int wav_gap_blocks(int nx, int ny, int levels);
void check_wavelet_shape(int nx, int ny, int levels);
// coef = W img
template <class T>
void launch_wav_forward(const WavInput<T>& in, T* coef, T* work, hipStream_t s);
// r <- clip(r + sigma mult[0] W img, -lam, lam)
template <class T>
void launch_wav_dual(const WavInput<T>& in, const WavDual<T>& d, T* work, hipStream_t s);
// red[b] = lam sum |W img| over the coefficients of workgroup b (FP64 arithmetic)
template <class T>
void launch_wav_gap(const WavInput<T>& in, T lam, double* red, double* work, hipStream_t s);
// out = W^T coef, arithmetic and output in A (T, or FP64 for the gap of FP32)
template <class T, class A>
void launch_wav_adjoint(int nx, int ny, int levels, const T* coef, A* out, A* work, hipStream_t s);

// ---- launchers (pdhg.hip)
template <class T>
void launch_reg_dual(const Launch<T>& L, hipStream_t s);
template <class T>
void launch_primal(const Launch<T>& L, bool check, hipStream_t s);
template <class T>
void launch_pattern(T* x, int64_t n, hipStream_t s);
template <class T>
void launch_gap_reg(const Launch<T>& L, hipStream_t s);
// Step multipliers of iteration t of a block for every instance:
// cur[i][0..2] = sched[i][t][0..2] (sched holds `block` iterations per instance).
void launch_accel_step(const double* sched, double* cur, int n_inst, int block, int t, hipStream_t s);
// Sum the partial sums of every instance: out[inst][slot] (double).
void launch_gap_finish(const GapFinishArgs* args, int n_inst, double* out, hipStream_t s);
template <class T>
void launch_precond_pix(int reg_kind, int nx, int ny, const T* colsum_a, const T* dmat,
                        T* sigma_r, T* sigma_s, T* tau_u, T* tau_v, hipStream_t s);
template <class T>
void launch_dmat(const T* theta, T eta, T* dmat, int64_t n, hipStream_t s);
template <class T>
void launch_fill(T* p, T v, int64_t n, hipStream_t s);
template <class T>
void launch_reg_apply(int reg_kind, int nx, int ny, const T* dmat, const T* xu, const T* xv,
                      T* z, hipStream_t s);
template <class T>
void launch_reg_apply_t(int reg_kind, int nx, int ny, const T* dmat, const T* z, T* yu, T* yv,
                        hipStream_t s);
template <class T>
void launch_dot(const T* a, const T* b, int64_t n, double* partial, int n_part, double* out,
                hipStream_t s);
template <class T>
void launch_scale_copy(T* y, const T* x, const double* denom, int64_t n, hipStream_t s);

}  // namespace pat
