// Solve driver of preconditioned PDHGM (arXiv:1707.02245, Algorithms 1 and 2)
// with the step-size rules of Sec. 3.3.2 and the gap stopping rule of
// Sec. 3.3.3, for one instance or many instances sharing every launch.
//
// One iteration is three launches over all active instances:
//   1. the forward of ubar with the dual data step fused (q update), and in
//      the same launch the regulariser's dual step (r, and s for TGV); with
//      the stored A by pixel tiles (forward path 3) its tile pass carries the
//      regulariser's step and a per-bin pass the dual data step
//   2. A^T q into one partial image per quarter turn (stored CSR) or per
//      detector group (matrix-free scatter)
//   3. primal step (sums the partials, u and v updates, extrapolation)
// The wavelet model adds one analysis launch per level with its dual step
// after 1 and one synthesis launch per level (W^T r) before 3.
// The last iteration of a block adds the gap: forward gather of u+ with the
// data and F* terms reduced, the regulariser value reduced, and an ordered
// final sum per instance. Blocks of iterations are captured once as a HIP
// graph and replayed; the only device-to-host traffic is the gap sums per
// block, and stopping is decided there.

#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <string>

#include "pat_internal.hpp"

namespace pat {

void validate_regulariser(const pat_geometry_s* g, const pat_regulariser* r) {
  PAT_CHECK_ARG(r != nullptr, "regulariser is NULL");
  PAT_CHECK_ARG(r->kind >= PAT_REG_TV && r->kind <= PAT_REG_WAVELET, "unknown regulariser kind");
  PAT_CHECK_ARG(std::isfinite(r->lambda) && r->lambda >= 0.0, "lambda must be finite and >= 0");
  if (r->kind == PAT_REG_TGV)
    PAT_CHECK_ARG(std::isfinite(r->tgv_alpha0) && r->tgv_alpha0 >= 0.0,
                  "tgv_alpha0 must be finite and >= 0");
  if (r->kind == PAT_REG_DTV) {
    PAT_CHECK_ARG(std::isfinite(r->dtv_eta) && r->dtv_eta > 0.0 && r->dtv_eta <= 1.0,
                  "dtv_eta must be in (0, 1]");
    PAT_CHECK_ARG(r->d_dtv_theta != nullptr, "DTV needs d_dtv_theta");
  }
  if (r->kind == PAT_REG_TIKHONOV) PAT_CHECK_ARG(r->lambda > 0.0, "Tikhonov lambda must be > 0");
  if (r->kind == PAT_REG_WAVELET) check_wavelet_shape(g->nx, g->ny, r->wav_levels);
}

static void validate_opts(const pat_solve_opts* o) {
  PAT_CHECK_ARG(o != nullptr, "opts is NULL");
  PAT_CHECK_ARG(o->max_iter > 0, "max_iter must be > 0");
  PAT_CHECK_ARG(std::isfinite(o->gap_tol), "gap_tol must be finite");
  PAT_CHECK_ARG(o->gap_every >= 1, "gap_every must be >= 1");
  PAT_CHECK_ARG(o->graph_block >= 0, "graph_block must be >= 0");
  PAT_CHECK_ARG(std::isfinite(o->theta) && o->theta >= 0.0 && o->theta <= 1.0,
                "theta must be in [0, 1]");
  PAT_CHECK_ARG(std::isfinite(o->gap_box) && o->gap_box > 0.0, "gap_box must be > 0");
  PAT_CHECK_ARG(std::isfinite(o->accel_gamma) && o->accel_gamma >= 0.0, "accel_gamma must be finite and >= 0");
  if (o->accel_gamma > 0.0) {
    PAT_CHECK_ARG(!std::isnan(o->accel_step_max) && o->accel_step_max >= 1.0,
                  "accel_step_max must be >= 1 with accel_gamma > 0");
    PAT_CHECK_ARG(o->theta == 1.0, "the accelerated schedule sets theta itself: pass theta = 1");
  }
}

// ------------------------------------------------------------------ step sizes

template <class T>
static void compute_dmat(pat_geometry g, const pat_regulariser* reg, DevBuf& dmat, hipStream_t s) {
  if (reg->kind != PAT_REG_DTV) return;
  dmat.ensure(sizeof(T) * 3 * g->n_pix());
  launch_dmat<T>(static_cast<const T*>(reg->d_dtv_theta), (T)reg->dtv_eta, ptr<T>(dmat), g->n_pix(), s);
}

template <class T>
static void precond_diag(pat_precond_s* pc, const pat_regulariser* reg, const T* dmat, hipStream_t s) {
  pat_geometry g = pc->g;
  const int64_t N = g->n_pix(), nb = g->n_bins();
  DevBuf ones(sizeof(T) * std::max<int64_t>(N, nb)), pad, colsum(sizeof(T) * N);
  launch_fill<T>(ptr<T>(ones), T(1), std::max<int64_t>(N, nb), s);
  // sigma_q = 1 / (A 1): A >= 0 so this is the absolute row sum
  pad.ensure(sizeof(T) * (size_t)(g->nx + 2) * (g->ny + 2));
  launch_pad<T>(ptr<T>(ones), ptr<T>(pad), g->nx, g->ny, s);
  FwdArgs<T> a{};
  a.g = g->dev();
  a.upad = ptr<T>(pad);
  a.out = ptr<T>(pc->sigma_q);
  attach_fwd_part<T>(g, a);
  launch_forward<T>(FWD_ROWSUM, a, g->lanes_log2, s);
  // column sums of A: A^T 1
  apply_adjoint<T>(g, ptr<T>(ones), ptr<T>(colsum), s);
  launch_precond_pix<T>(reg->kind, g->nx, g->ny, ptr<T>(colsum), dmat, ptr<T>(pc->sigma_r),
                        ptr<T>(pc->sigma_s), ptr<T>(pc->tau_u), ptr<T>(pc->tau_v), s);
  PAT_HIP(hipStreamSynchronize(s));
}

constexpr int kPowerIters = 1000;
constexpr double kPowerSafety = 1.05;

// ||M|| by power iteration on M^T M from x_j = 1 + (j mod 5)/4 (normalised).
template <class T, class Apply>
static double power_norm(int64_t n, hipStream_t s, Apply&& normal_op) {
  DevBuf x(sizeof(T) * n), y(sizeof(T) * n), part(sizeof(double) * 512), acc(sizeof(double));
  launch_pattern<T>(ptr<T>(x), n, s);
  launch_dot<T>(ptr<T>(x), ptr<T>(x), n, ptr<double>(part), 512, ptr<double>(acc), s);
  launch_scale_copy<T>(ptr<T>(x), ptr<T>(x), ptr<double>(acc), n, s);
  for (int it = 0; it < kPowerIters; ++it) {
    normal_op(ptr<T>(x), ptr<T>(y));
    launch_dot<T>(ptr<T>(y), ptr<T>(y), n, ptr<double>(part), 512, ptr<double>(acc), s);
    launch_scale_copy<T>(ptr<T>(x), ptr<T>(y), ptr<double>(acc), n, s);
  }
  double lam2 = 0.0;
  PAT_HIP(hipMemcpyAsync(&lam2, acc.p, sizeof(double), hipMemcpyDeviceToHost, s));
  PAT_HIP(hipStreamSynchronize(s));
  return std::sqrt(std::sqrt(lam2));  // ||M^T M x|| -> ||M||^2
}

template <class T>
static void precond_block(pat_precond_s* pc, const pat_regulariser* reg, const T* dmat, hipStream_t s) {
  pat_geometry g = pc->g;
  const int64_t N = g->n_pix(), nb = g->n_bins();
  DevBuf tmp_b(sizeof(T) * nb);
  const double L1 = kPowerSafety * power_norm<T>(N, s, [&](const T* x, T* y) {
    apply_forward<T>(g, x, ptr<T>(tmp_b), s);
    apply_adjoint<T>(g, ptr<T>(tmp_b), y, s);
  });
  double L2 = 0.0;
  if (reg->kind == PAT_REG_WAVELET) {
    DevBuf z(sizeof(T) * 4 * N), work(sizeof(T) * wav_work_elems(g->nx, g->ny));
    L2 = kPowerSafety * power_norm<T>(N, s, [&](const T* x, T* y) {
      WavInput<T> in{g->nx, g->ny, reg->wav_levels, x, g->nx};
      launch_wav_forward<T>(in, ptr<T>(z), ptr<T>(work), s);
      launch_wav_adjoint<T, T>(g->nx, g->ny, reg->wav_levels, ptr<T>(z), y, ptr<T>(work), s);
    });
  } else if (reg->kind != PAT_REG_TIKHONOV) {
    const bool tgv = reg->kind == PAT_REG_TGV;
    const int64_t nx_ = tgv ? 3 * N : N;
    DevBuf z(sizeof(T) * (tgv ? 5 : 2) * N);
    L2 = kPowerSafety * power_norm<T>(nx_, s, [&](const T* x, T* y) {
      launch_reg_apply<T>(reg->kind, g->nx, g->ny, dmat, x, tgv ? x + N : nullptr, ptr<T>(z), s);
      launch_reg_apply_t<T>(reg->kind, g->nx, g->ny, dmat, ptr<T>(z), y, tgv ? y + N : nullptr, s);
    });
  }
  pc->L1 = L1;
  pc->L2 = L2;
  const double tau = 1.0 / (2.0 * std::max(L1, L2));
  const double s1 = 0.99 / (4.0 * tau * L1 * L1);
  const double s2 = L2 > 0.0 ? 0.99 / (4.0 * tau * L2 * L2) : 1.0;
  if (reg->kind == PAT_REG_WAVELET) pc->sigma_w = s2;
  launch_fill<T>(ptr<T>(pc->sigma_q), (T)s1, nb, s);
  launch_fill<T>(ptr<T>(pc->tau_u), (T)tau, N, s);
  if (pc->sigma_r.p) launch_fill<T>(ptr<T>(pc->sigma_r), (T)s2, (int64_t)(pc->sigma_r.bytes / sizeof(T)), s);
  if (pc->sigma_s.p) launch_fill<T>(ptr<T>(pc->sigma_s), (T)s2, N, s);
  if (pc->tau_v.p) launch_fill<T>(ptr<T>(pc->tau_v), (T)tau, N, s);
  PAT_HIP(hipStreamSynchronize(s));
}

static pat_precond_s* make_precond(pat_geometry g, const pat_regulariser* reg, int kind, hipStream_t s) {
  std::unique_ptr<pat_precond_s> pc(new pat_precond_s());
  pc->g = g;
  pc->reg_kind = reg->kind;
  pc->kind = kind;
  const size_t es = dtype_size(g->dtype);
  const int64_t N = g->n_pix();
  pc->sigma_q.alloc(es * g->n_bins());
  pc->tau_u.alloc(es * N);
  // one step per pixel's dual vector; the wavelet's one per coefficient
  if (reg->kind != PAT_REG_TIKHONOV) pc->sigma_r.alloc(es * (reg->kind == PAT_REG_WAVELET ? 4 : 1) * N);
  if (reg->kind == PAT_REG_TGV) {
    pc->sigma_s.alloc(es * N);
    pc->tau_v.alloc(es * N);
  }
  DevBuf dmat;
  if (g->dtype == PAT_F64) {
    compute_dmat<double>(g, reg, dmat, s);
    if (kind == PAT_PRECOND_DIAG) precond_diag<double>(pc.get(), reg, ptr<double>(dmat), s);
    else precond_block<double>(pc.get(), reg, ptr<double>(dmat), s);
  } else {
    compute_dmat<float>(g, reg, dmat, s);
    if (kind == PAT_PRECOND_DIAG) precond_diag<float>(pc.get(), reg, ptr<float>(dmat), s);
    else precond_block<float>(pc.get(), reg, ptr<float>(dmat), s);
  }
  return pc.release();
}

// ------------------------------------------------------------------ solver state

int64_t state_elems(const pat_geometry_s* g, int kind) {
  const int64_t N = g->n_pix(), nb = g->n_bins();
  int64_t n = 2 * N + nb;
  if (kind == PAT_REG_WAVELET) n += 4 * N;
  else if (kind != PAT_REG_TIKHONOV) n += 2 * N;
  if (kind == PAT_REG_TGV) n += 7 * N;
  return n;
}

template <class T>
struct Inst {
  pat_geometry g = nullptr;
  pat_regulariser reg{};
  pat_solve_opts opts{};
  const T* f = nullptr;
  T* u_out = nullptr;
  pat_solve_info* info = nullptr;
  DevBuf u, ubar_pad, q, r, v, vbar, s, upad_gap, atq_part, atq64, red, dmat, fpart;
  // wavelet model: W^T r (and in FP64 for the gap of FP32), the transform's
  // work buffer (FP64-sized), and the gap pass's partial sums
  DevBuf wtr, wtr64, wwork;
  int n_reg = 0;
  pat_precond_s* pc = nullptr;
  std::unique_ptr<pat_precond_s> own_pc;
  int n_fwd = 0, n_pix = 0, n_adj = 0, n_csr = 0, red_stride = 0;
  bool csr = false;  // adjoint by the stored CSR of A^T
  // forward in quarter-turn form: ubar_pad and upad_gap hold four slots (the
  // image and its copies turned by 1..3 quarter turns)
  bool qt = false;
  // forward by the stored A of the first n_det/4 detectors (path 3): fpart
  // holds its four partials per segment
  bool fm = false;
  int iters = 0;
  bool active = true, converged = false;
  int fallback = 0;
  pat_status status = PAT_NOT_CONVERGED;
  double last[GAP_NSLOTS] = {0, 0, 0, 0, 0, 0};
  double rel_gap = INFINITY, gap = INFINITY, primal = 0, fstar = 0, kty = 0, residual = 0;
  // accelerated schedule (Chambolle-Pock Algorithm 2 on the preconditioned
  // steps): multipliers of the next iteration's dual (acc_b) and primal
  // (acc_a) steps; frozen once the dual steps would grow beyond accel_step_max
  bool accel = false, acc_frozen = false;
  double acc_a = 1.0, acc_b = 1.0;

  // the next iteration's {dual, primal, theta}; advances the schedule
  void next_mult(double* m) {
    double th = accel ? 1.0 : opts.theta;
    if (accel && !acc_frozen) {
      th = 1.0 / std::sqrt(1.0 + 2.0 * opts.accel_gamma * acc_a);
      if (acc_b / th > opts.accel_step_max) {
        acc_frozen = true;
        th = 1.0;
      }
    }
    m[0] = acc_b;
    m[1] = acc_a;
    m[2] = th;
    if (accel && !acc_frozen) {
      acc_a *= th;
      acc_b /= th;
    }
  }

  GeomDev gdev(int lanes_log2, int tile) const {
    GeomDev d = g->dev();
    d.lanes_log2 = lanes_log2;
    d.tile = tile;
    d.tiles_x = (g->nx + tile - 1) / tile;
    d.tiles_y = (g->ny + tile - 1) / tile;
    return d;
  }
};

template <class T>
class Solver {
 public:
  std::vector<std::unique_ptr<Inst<T>>> inst;
  std::vector<int> act;  // indices of active instances
  Launch<T> L;
  hipStream_t s = nullptr;
  int gap_every = 10, graph_block = 50;
  int lanes_log2 = 6, tile = 32;
  DevBuf results;        // [max_checks][n_active][GAP_NSLOTS]
  double* h_results = nullptr;
  int max_checks = 0;
  // accelerated schedule: multipliers of every instance for one block
  // [n_inst][block][3] (host pinned and device), the current iteration's
  // [n_inst][3] read by the kernels
  bool any_accel = false;
  bool accel_live = false;  // some instance's multipliers still change
  int sched_block = 1;
  DevBuf sched, cur;
  double* h_sched = nullptr;
  std::map<std::string, hipGraphExec_t> graphs;

  ~Solver() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (h_results) (void)hipHostFree(h_results);
    if (h_sched) (void)hipHostFree(h_sched);
  }

  void setup(hipStream_t stream) {
    s = stream;
    lanes_log2 = inst[0]->g->lanes_log2;
    tile = inst[0]->g->tile;
    if (sizeof(T) == 8 && tile == 64) tile = 32;
    for (auto& ip : inst) alloc_instance(*ip);
    act.clear();
    for (size_t i = 0; i < inst.size(); ++i) act.push_back((int)i);
    max_checks = 1;  // one gap evaluation per block
    results.alloc(sizeof(double) * max_checks * inst.size() * GAP_NSLOTS);
    PAT_HIP(hipHostMalloc((void**)&h_results, sizeof(double) * max_checks * inst.size() * GAP_NSLOTS,
                          hipHostMallocDefault));
    for (auto& ip : inst) {
      ip->accel = ip->opts.accel_gamma > 0.0;
      any_accel = any_accel || ip->accel;
    }
    accel_live = any_accel;
    if (any_accel) {
      sched_block = graph_block > 0 ? graph_block : gap_every;
      const size_t n = inst.size();
      sched.alloc(sizeof(double) * 3 * n * sched_block);
      cur.alloc(sizeof(double) * 3 * n);
      PAT_HIP(hipHostMalloc((void**)&h_sched, sizeof(double) * 3 * n * sched_block, hipHostMallocDefault));
      // plain multipliers until the first block's are uploaded
      for (size_t i = 0; i < n * sched_block; ++i) {
        h_sched[3 * i] = h_sched[3 * i + 1] = 1.0;
        h_sched[3 * i + 2] = inst[i / sched_block]->accel ? 1.0 : inst[i / sched_block]->opts.theta;
      }
      PAT_HIP(hipMemcpyAsync(cur.p, h_sched, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
      PAT_HIP(hipStreamSynchronize(s));
    }
  }

  // Multipliers of the next `steps` iterations of every active instance.
  // Once every active accelerated instance's schedule has frozen, its fixed
  // multipliers are written to the kernels' slot once and later blocks run
  // without the per-iteration selection launch.
  void upload_schedule(int steps) {
    if (!accel_live) return;
    bool all_frozen = true;
    for (int k : act) all_frozen = all_frozen && (!inst[k]->accel || inst[k]->acc_frozen);
    if (all_frozen) {
      for (int k : act) inst[k]->next_mult(h_sched + (size_t)k * 3);
      PAT_HIP(hipMemcpyAsync(cur.p, h_sched, cur.bytes, hipMemcpyHostToDevice, s));
      accel_live = false;
      return;
    }
    for (int k : act) {
      Inst<T>& I = *inst[k];
      for (int t = 0; t < steps; ++t) I.next_mult(h_sched + ((size_t)k * sched_block + t) * 3);
    }
    PAT_HIP(hipMemcpyAsync(sched.p, h_sched, sched.bytes, hipMemcpyHostToDevice, s));
  }

  void alloc_instance(Inst<T>& I) {
    pat_geometry g = I.g;
    const int64_t N = g->n_pix(), nb = g->n_bins();
    const size_t P = (size_t)(g->nx + 2) * (g->ny + 2);
    const int kind = I.reg.kind;
    I.qt = g->fwd_qt();
    const int slots = I.qt ? 4 : 1;
    I.u.alloc(sizeof(T) * N);
    I.ubar_pad.alloc(sizeof(T) * slots * P);
    I.upad_gap.alloc(sizeof(T) * slots * P);
    I.q.alloc(sizeof(T) * nb);
    if (kind == PAT_REG_WAVELET) {
      I.r.alloc(sizeof(T) * 4 * N);
      I.wtr.alloc(sizeof(T) * N);
      if (sizeof(T) == 4) I.wtr64.alloc(sizeof(double) * N);
      I.wwork.alloc(sizeof(double) * wav_work_elems(g->nx, g->ny));
    } else if (kind != PAT_REG_TIKHONOV) {
      I.r.alloc(sizeof(T) * 2 * N);
    }
    if (kind == PAT_REG_TGV) {
      I.v.alloc(sizeof(T) * 2 * N);
      I.vbar.alloc(sizeof(T) * 2 * N);
      I.s.alloc(sizeof(T) * 3 * N);
    }
    const GeomDev gd = I.gdev(lanes_log2, tile);
    I.csr = g->adj_mode != 0;
    if (I.csr) g->ensure_csr(s);
    // the stored A^T with quarter turns writes one partial image per turn
    I.atq_part.alloc(sizeof(T) * (I.csr ? g->csr_rot : gd.n_groups) * N);
    // FP64-accumulated A^T q for the gap: only FP32 needs a separate pass
    if (I.csr && sizeof(T) == 4) I.atq64.alloc(sizeof(double) * g->csr_rot * N);
    // gap partial sums: enough blocks for any forward path (build_launch
    // picks the path of the batch)
    I.n_fwd = std::max({fwd_grid(g->n_det, g->n_t, lanes_log2, 0), fwd_grid(g->n_det, g->n_t, lanes_log2, 1),
                        fwd_grid(g->n_det, g->n_t, lanes_log2, 2)});
    // quarter-turn form: four slots of partials over a quarter's blocks
    if (I.qt)
      I.n_fwd = std::max({I.n_fwd, 4 * fwd_grid(g->n_det / 4, g->n_t, lanes_log2, 0),
                          4 * fwd_grid(g->n_det / 4, g->n_t, lanes_log2, 1)});
    if (g->fwd_path == 2) I.fpart.alloc(sizeof(T) * (size_t)std::max<int64_t>(g->fwd_n_pairs, 1));
    I.fm = g->fwd_path == 3 && g->fm_entries > 0;
    if (I.fm) {
      I.fpart.alloc(sizeof(T) * 4 * (size_t)std::max(g->fm_nseg, 1));
      // the per-bin pass writes gap partials per turn and block
      I.n_fwd = std::max(I.n_fwd, 4 * fmat_reduce_blocks(g->n_det / 4, g->n_t));
    }
    I.n_pix = pix_blocks(N);
    I.n_adj = I.csr ? 0 : gd.tiles_x * gd.tiles_y * gd.n_groups;
    I.n_csr = I.csr ? (int)((N + 3) / 4) : 0;
    I.n_reg = kind == PAT_REG_WAVELET ? wav_gap_blocks(g->nx, g->ny, I.reg.wav_levels) : I.n_pix;
    I.red_stride = std::max({I.n_fwd, I.n_pix, I.n_reg});
    I.red.alloc(sizeof(double) * GAP_NSLOTS * I.red_stride);
    compute_dmat<T>(g, &I.reg, I.dmat, s);
    if (I.opts.precond) {
      PAT_CHECK_ARG(I.opts.precond->g == g && I.opts.precond->reg_kind == kind,
                    "precond handle was made for another geometry or regulariser");
      I.pc = I.opts.precond;
    } else {
      I.own_pc.reset(make_precond(g, &I.reg, PAT_PRECOND_DIAG, s));
      I.pc = I.own_pc.get();
    }
  }

  InstDev<T> inst_dev(const Inst<T>& I) const {
    InstDev<T> d{};
    const GeomDev gd = I.gdev(lanes_log2, tile);
    d.nx = I.g->nx;
    d.ny = I.g->ny;
    d.n_groups = I.csr ? I.g->csr_rot : gd.n_groups;
    d.n_bins = (int)I.g->n_bins();
    d.kind = I.reg.kind;
    d.lam = (T)I.reg.lambda;
    d.alpha0 = (T)I.reg.tgv_alpha0;
    d.theta_ex = (T)I.opts.theta;
    d.dmat = ptr<T>(I.dmat);
    d.u = ptr<T>(I.u);
    d.ubar_pad = ptr<T>(I.ubar_pad);
    d.r = ptr<T>(I.r);
    d.v = ptr<T>(I.v);
    d.vbar = ptr<T>(I.vbar);
    d.s = ptr<T>(I.s);
    d.sigma_r = ptr<T>(I.pc->sigma_r);
    d.sigma_s = ptr<T>(I.pc->sigma_s);
    d.tau_u = ptr<T>(I.pc->tau_u);
    d.tau_v = ptr<T>(I.pc->tau_v);
    d.atq_part = ptr<T>(I.atq_part);
    d.atq64 = ptr<double>(I.atq64);
    d.upad_gap = ptr<T>(I.upad_gap);
    d.red = ptr<double>(I.red);
    d.red_stride = I.red_stride;
    d.mult = I.accel ? ptr<double>(cur) + 3 * inst_index(I) : nullptr;
    d.rot_slots = I.qt ? 4 : 1;
    d.wtr = ptr<T>(I.wtr);
    d.wtr64 = ptr<double>(I.wtr64);
    return d;
  }

  int inst_index(const Inst<T>& I) const {
    for (size_t i = 0; i < inst.size(); ++i)
      if (inst[i].get() == &I) return (int)i;
    return 0;
  }

  // Upload the launch tables of the active instances.
  void build_launch() {
    const int n = (int)act.size();
    // the LDS-tiled forward when every instance's geometry uses it, else the
    // gather kernel (radius-major for those that chose tiles)
    bool fwd_tiled = n > 0;
    for (int k = 0; k < n; ++k) fwd_tiled = fwd_tiled && inst[act[k]]->g->fwd_path == 2 && inst[act[k]]->fpart.p;
    // instances in quarter-turn form (gather forward only) and instances
    // whose forward is the stored A (path 3, outside the gather launches)
    std::vector<bool> qt(n, false), fm(n, false);
    for (int k = 0; k < n; ++k) {
      qt[k] = !fwd_tiled && inst[act[k]]->qt;
      fm[k] = inst[act[k]]->fm;
    }
    std::vector<FwdArgs<T>> fmd, fmg;
    std::vector<int> fms(1, 0), fmrs(1, 0);
    std::vector<int> ts(n + 1, 0);
    std::vector<FwdArgs<T>> fd(n), fg(n);
    std::vector<AdjArgs<T>> ad;
    std::vector<CsrMultiArgs<T>> cd;
    std::vector<InstDev<T>> id(n);
    std::vector<GapFinishArgs> gf(n);
    std::vector<int> fs(n + 1), as(1, 0), cs(1, 0), ps(n + 1);
    std::vector<pat_geometry> csr_geo;  // geometry of each CSR group
    const int lds_max = device_lds_per_block();
    fs[0] = ps[0] = 0;
    for (int k = 0; k < n; ++k) {
      const Inst<T>& I = *inst[act[k]];
      const GeomDev gd = I.gdev(lanes_log2, tile);
      fd[k] = FwdArgs<T>{};
      fd[k].g = gd;
      fd[k].upad = ptr<T>(I.ubar_pad);
      fd[k].out = ptr<T>(I.q);
      fd[k].f = I.f;
      fd[k].sigma = ptr<T>(I.pc->sigma_q);
      fd[k].mult = I.accel ? ptr<double>(cur) + 3 * act[k] : nullptr;
      fg[k] = FwdArgs<T>{};
      fg[k].g = gd;
      fg[k].upad = ptr<T>(I.upad_gap);
      fg[k].f = I.f;
      fg[k].q = ptr<T>(I.q);
      fg[k].red = ptr<double>(I.red);
      fg[k].red_stride = I.red_stride;
      const int path = fwd_tiled ? 2 : (I.g->fwd_path >= 2 ? 0 : I.g->fwd_path);
      fd[k].g.fwd_path = fg[k].g.fwd_path = path;
      fd[k].part = fg[k].part = ptr<T>(I.fpart);
      int n_fwd = fwd_grid(I.g->n_det, I.g->n_t, lanes_log2, path);
      int n_fwd_parts = n_fwd;  // gap partials of the forward
      if (qt[k]) {
        // a quarter of the detectors; the group's four slots (below) read the
        // image turned by t quarter turns for the bins of detectors t n_det/4 ..
        const int q = I.g->n_det / 4;
        fd[k].g.n_det = fg[k].g.n_det = q;
        n_fwd = fwd_grid(q, I.g->n_t, lanes_log2, path);
        n_fwd_parts = 4 * n_fwd;
      } else if (fm[k]) {
        // no gather blocks: the stored A's two passes in slot form
        const int q = I.g->n_det / 4;
        const int nrb = fmat_reduce_blocks(q, I.g->n_t);
        FwdArgs<T> x = fd[k], y = fg[k];
        x.g = y.g = I.g->dev();
        x.g.n_det = y.g.n_det = q;
        x.slot_bins = y.slot_bins = (int64_t)q * I.g->n_t;
        y.slot_red = nrb;
        fmd.push_back(x);
        fmg.push_back(y);
        fms.push_back(fms.back() + I.g->fm_nchunk);
        fmrs.push_back(fmrs.back() + nrb);
        n_fwd = 0;
        n_fwd_parts = 4 * nrb;
      }
      ts[k + 1] = ts[k] + (fwd_tiled ? I.g->fwd_n_blocks : 0);
      if (I.csr) {
        // instances sharing a geometry share one pass over its stored A^T: up
        // to kMaxRhs slots (rot per instance), and for the tiled kernel as
        // many as their staged windows fit the workgroup LDS
        const int rot = I.g->csr_rot;
        int cap = kMaxRhs;
        if (I.g->effective_adj_mode() == 2) {
          // a kernel instance of R slots (1, 2, 4 or 8) stages R windows
          const int fit = lds_max / (int)(sizeof(T) * I.g->csr_win_max);
          cap = fit >= kMaxRhs ? kMaxRhs : (fit >= 4 ? 4 : (fit >= 2 ? 2 : 1));
        }
        CsrMultiArgs<T>* grp = nullptr;
        for (auto& c : cd)
          if (c.ptr == ptr<int64_t>(I.g->csr_ptr) && c.nrhs + rot <= cap) grp = &c;
        if (!grp) {
          cd.push_back(CsrMultiArgs<T>{});
          grp = &cd.back();
          pat_geometry g = I.g;
          grp->ptr = ptr<int64_t>(g->csr_ptr);
          grp->col = ptr<int>(g->csr_col);
          grp->val = ptr<T>(g->csr_val);
          grp->n_rows = g->n_pix();
          grp->nrhs = 0;
          if (g->effective_adj_mode() == 2) {
            grp->lcol = ptr<uint16_t>(g->csr_lcol);
            grp->win = ptr<int4>(g->csr_win);
            grp->side = g->csr_side;
            grp->tiles_x = g->csr_tiles_x;
            grp->lds_stride = g->csr_win_max;
          }
          grp->nx = g->nx;
          grp->ny = g->ny;
          grp->n_det = g->csr_det();
          grp->n_t = g->n_t;
          grp->rot = rot;
          csr_geo.push_back(g);
        }
        for (int r = 0; r < rot; ++r) {
          grp->x[grp->nrhs] = ptr<T>(I.q) + (int64_t)r * grp->n_det * grp->n_t;
          grp->y[grp->nrhs] = ptr<T>(I.atq_part) + (int64_t)r * I.g->n_pix();
          grp->y64[grp->nrhs] = I.atq64.p ? ptr<double>(I.atq64) + (int64_t)r * I.g->n_pix() : nullptr;
          ++grp->nrhs;
        }
      } else {
        AdjArgs<T> a{};
        a.g = gd;
        a.data = ptr<T>(I.q);
        a.part = ptr<T>(I.atq_part);
        ad.push_back(a);
        as.push_back(as.back() + I.n_adj);
      }
      id[k] = inst_dev(I);
      gf[k] = GapFinishArgs{ptr<double>(I.red), I.red_stride, n_fwd_parts, I.n_pix, I.n_reg};
      fs[k + 1] = fs[k] + n_fwd;
      ps[k + 1] = ps[k] + I.n_pix;
    }
    // CSR groups: the LDS-staged kernel when every group has tiles and the
    // windows of all its right-hand sides fit the LDS budget, else the plain one
    int max_rhs = 1, max_stride = 0;
    bool tiled = !cd.empty();
    for (size_t c = 0; c < cd.size(); ++c) {
      max_rhs = std::max(max_rhs, cd[c].nrhs);
      tiled = tiled && cd[c].lcol != nullptr;
      max_stride = std::max(max_stride, cd[c].lds_stride);
    }
    // the kernel instance for max_rhs reads every slot of every group
    const int r_inst = max_rhs <= 2 ? max_rhs : (max_rhs <= 4 ? 4 : kMaxRhs);
    const size_t shm = sizeof(T) * (size_t)max_stride * (size_t)r_inst;
    tiled = tiled && shm <= (size_t)lds_max;
    if (tiled) prepare_csr_tiled<T>(max_rhs, shm);
    // workgroup shape: the geometry's tuned choice for a single group, else by LDS
    int waves = csr_waves_for(shm, sizeof(T));
    double mean_row = 0.0;
    for (pat_geometry g : csr_geo) mean_row = std::max(mean_row, (double)g->csr_nnz / (double)g->n_pix());
    int lanes = csr_lanes_for(mean_row);
    if (tiled && cd.size() == 1 && cd[0].nrhs == csr_geo[0]->csr_rot) {
      waves = csr_geo[0]->csr_waves;
      lanes = csr_geo[0]->csr_lanes;
    }
    for (size_t c = 0; c < cd.size(); ++c) {
      const int blocks = tiled ? csr_geo[c]->n_csr_tiles() : (int)((cd[c].n_rows + 3) / 4);
      cs.push_back(cs.back() + blocks);
    }
    // forward groups (gather forward only): instances on one geometry, up to
    // four per group, share each forward block; an instance in quarter-turn
    // form is a group of its own whose four slots are its turned images
    std::vector<std::vector<int>> fgrp;
    if (!fwd_tiled) {
      for (int k = 0; k < n; ++k) {
        if (fm[k]) continue;
        std::vector<int>* into = nullptr;
        if (!qt[k])
          for (auto& gr : fgrp)
            if (!qt[gr[0]] && gr.size() < 4 && inst[act[gr[0]]]->g == inst[act[k]]->g) {
              into = &gr;
              break;
            }
        if (into) into->push_back(k);
        else fgrp.push_back({k});
      }
    }
    int ni = 1;
    for (const auto& gr : fgrp) ni = std::max(ni, qt[gr[0]] ? 4 : (int)gr.size());
    std::vector<FwdArgs<T>> gdual, ggap;
    std::vector<int> gs(1, 0);
    if (ni > 1) {
      for (const auto& gr : fgrp) {
        for (int i = 0; i < ni; ++i) {
          FwdArgs<T> x = fd[gr[0]], y = fg[gr[0]];
          if (qt[gr[0]]) {
            // slot i: the image turned by i quarter turns and the bins, data,
            // steps and gap partials of detectors i n_det/4 ..
            const Inst<T>& I = *inst[act[gr[0]]];
            const int64_t P = (int64_t)(I.g->nx + 2) * (I.g->ny + 2);
            const int64_t ob = (int64_t)i * x.g.n_det * x.g.n_t;
            x.upad += i * P;
            x.out += ob;
            x.f += ob;
            x.sigma += ob;
            y.upad += i * P;
            y.f += ob;
            y.q += ob;
            y.red += (int64_t)i * (fs[gr[0] + 1] - fs[gr[0]]);
          } else if (i < (int)gr.size()) {
            x = fd[gr[i]];
            y = fg[gr[i]];
          } else {
            x.upad = y.upad = nullptr;  // unused slot
          }
          gdual.push_back(x);
          ggap.push_back(y);
        }
        gs.push_back(gs.back() + (fs[gr[0] + 1] - fs[gr[0]]));
      }
    }
    auto up = [&](DevBuf& b, const void* src, size_t bytes) {
      b.ensure(bytes);
      PAT_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s));
    };
    if (ni > 1) {
      up(L.fwdg, gdual.data(), sizeof(FwdArgs<T>) * gdual.size());
      up(L.fwdg_gap, ggap.data(), sizeof(FwdArgs<T>) * ggap.size());
      up(L.fwdg_start, gs.data(), sizeof(int) * gs.size());
    }
    up(L.fwd, fd.data(), sizeof(FwdArgs<T>) * n);
    up(L.fwd_gap, fg.data(), sizeof(FwdArgs<T>) * n);
    if (!ad.empty()) up(L.adj, ad.data(), sizeof(AdjArgs<T>) * ad.size());
    if (!cd.empty()) up(L.csr, cd.data(), sizeof(CsrMultiArgs<T>) * cd.size());
    up(L.inst, id.data(), sizeof(InstDev<T>) * n);
    up(L.gapfin, gf.data(), sizeof(GapFinishArgs) * n);
    up(L.fwd_start, fs.data(), sizeof(int) * (n + 1));
    up(L.fwdt_start, ts.data(), sizeof(int) * (n + 1));
    up(L.adj_start, as.data(), sizeof(int) * as.size());
    up(L.csr_start, cs.data(), sizeof(int) * cs.size());
    up(L.pix_start, ps.data(), sizeof(int) * (n + 1));
    if (!fmd.empty()) {
      up(L.fm, fmd.data(), sizeof(FwdArgs<T>) * fmd.size());
      up(L.fm_gap, fmg.data(), sizeof(FwdArgs<T>) * fmg.size());
      up(L.fm_start, fms.data(), sizeof(int) * fms.size());
      up(L.fmr_start, fmrs.data(), sizeof(int) * fmrs.size());
    }
    PAT_HIP(hipStreamSynchronize(s));  // host vectors go out of scope
    L.fm_n = (int)fmd.size();
    L.fm_total = fms.back();
    L.fmr_total = fmrs.back();
    L.n = n;
    L.fwd_total = fs[n];
    L.fwd_tiled = fwd_tiled;
    L.fwd_ni = ni;
    L.fwd_ni_blocks = ni > 1 ? gs.back() : 0;
    L.fwd_ni_groups = ni > 1 ? (int)fgrp.size() : 0;
    L.fwdt_total = ts[n];
    L.adj_total = as.back();
    L.n_adj = (int)ad.size();
    L.n_csr = (int)cd.size();
    L.csr_max_rhs = max_rhs;
    L.csr_tiled = tiled;
    L.csr_shm = shm;
    L.csr_waves = waves;
    L.csr_lanes = lanes;
    L.csr_total = cs.back();
    L.pix_total = ps[n];
    L.lanes_log2 = lanes_log2;
    L.max_tile = tile;
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }

  // gap evaluation at the current (u, v, q, r, s) into results slot c
  void enqueue_gap(int c) {
    // the gap forward uses the second FwdArgs table (input u+, gap epilogue)
    std::swap(L.fwd, L.fwd_gap);
    std::swap(L.fwdg, L.fwdg_gap);
    std::swap(L.fm, L.fm_gap);
    launch_forward_batched<T>(FWD_GAP, L, lanes_log2, s);
    std::swap(L.fwd, L.fwd_gap);
    std::swap(L.fwdg, L.fwdg_gap);
    std::swap(L.fm, L.fm_gap);
    launch_gap_reg<T>(L, s);
    enqueue_wavelet_gap();
    launch_gap_finish(ptr<GapFinishArgs>(L.gapfin), L.n,
                      ptr<double>(results) + (size_t)c * L.n * GAP_NSLOTS, s);
  }

  void enqueue_iteration(int t, bool check, int c) {
    if (accel_live) launch_accel_step(ptr<double>(sched), ptr<double>(cur), (int)inst.size(), sched_block, t, s);
    launch_forward_reg_batched<T>(L, lanes_log2, s);
    enqueue_wavelet_dual();
    enqueue_wavelet_synthesis(check);
    enqueue_adjoint(check);
    launch_primal<T>(L, check, s);
    if (check) enqueue_gap(c);
  }

  // Wavelet model, one launch per level and instance. The transform reads the
  // interior of a padded state image.
  WavInput<T> wav_input(const Inst<T>& I, const DevBuf& upad) const {
    const int P = I.g->nx + 2;
    return WavInput<T>{I.g->nx, I.g->ny, I.reg.wav_levels, ptr<T>(upad) + P + 1, P};
  }

  // The dual step r <- clip(r + sigma W ubar, -lam, lam).
  void enqueue_wavelet_dual() {
    for (int k : act) {
      Inst<T>& I = *inst[k];
      if (I.reg.kind != PAT_REG_WAVELET) continue;
      WavDual<T> d{};
      d.r = ptr<T>(I.r);
      d.sigma = (T)I.pc->sigma_w;
      d.mult = I.accel ? ptr<double>(cur) + 3 * k : nullptr;
      d.lam = (T)I.reg.lambda;
      launch_wav_dual<T>(wav_input(I, I.ubar_pad), d, ptr<T>(I.wwork), s);
    }
  }

  // W^T r of the new r for the primal step (on check iterations of FP32 also
  // in FP64, for the gap's dual residual).
  void enqueue_wavelet_synthesis(bool check) {
    for (int k : act) {
      Inst<T>& I = *inst[k];
      if (I.reg.kind != PAT_REG_WAVELET) continue;
      launch_wav_adjoint<T, T>(I.g->nx, I.g->ny, I.reg.wav_levels, ptr<T>(I.r), ptr<T>(I.wtr), ptr<T>(I.wwork), s);
      if (check && I.wtr64.p)
        launch_wav_adjoint<T, double>(I.g->nx, I.g->ny, I.reg.wav_levels, ptr<T>(I.r), ptr<double>(I.wtr64),
                                      ptr<double>(I.wwork), s);
    }
  }

  // The gap's lam ||W u+||_1 into the regulariser partials.
  void enqueue_wavelet_gap() {
    for (int k : act) {
      Inst<T>& I = *inst[k];
      if (I.reg.kind != PAT_REG_WAVELET) continue;
      launch_wav_gap<T>(wav_input(I, I.upad_gap), (T)I.reg.lambda,
                        ptr<double>(I.red) + (size_t)GAP_REG * I.red_stride, ptr<double>(I.wwork), s);
    }
  }

  // A^T q of every active instance into its partial images
  void enqueue_adjoint(bool check) {
    if (L.n_adj > 0) launch_adjoint_batched<T>(L, s);
    if (L.n_csr > 0) {
      // check iterations: A^T q once more with FP64 accumulation for the gap
      // (FP32 only; the FP64 pass already accumulates in FP64)
      for (int wide = 0; wide <= (check && sizeof(T) == 4 ? 1 : 0); ++wide) {
        if (L.csr_tiled)
          launch_csr_tiled_batched<T>(ptr<CsrMultiArgs<T>>(L.csr), ptr<int>(L.csr_start), L.n_csr,
                                      L.csr_total, L.csr_shm, s, wide != 0, L.csr_max_rhs, L.csr_waves, L.csr_lanes);
        else
          launch_csr_spmm_batched<T>(ptr<CsrMultiArgs<T>>(L.csr), ptr<int>(L.csr_start), L.n_csr,
                                     L.csr_total, s, wide != 0, L.csr_max_rhs);
      }
    }
  }

  // Padded copy of an image into a state buffer (and its turned copies in
  // quarter-turn form).
  void pad_slots(const Inst<T>& I, const T* src, T* dst) {
    if (I.qt) launch_rot_pad<T>(src, false, dst, I.g->nx, 4, s);
    else launch_pad<T>(src, dst, I.g->nx, I.g->ny, s);
  }

  void init_state() {
    for (int k : act) {
      Inst<T>& I = *inst[k];
      pat_geometry g = I.g;
      const int64_t N = g->n_pix(), nb = g->n_bins();
      const size_t P = (size_t)(g->nx + 2) * (g->ny + 2);
      PAT_HIP(hipMemsetAsync(I.u.p, 0, sizeof(T) * N, s));
      PAT_HIP(hipMemsetAsync(I.ubar_pad.p, 0, I.ubar_pad.bytes, s));
      PAT_HIP(hipMemsetAsync(I.upad_gap.p, 0, I.upad_gap.bytes, s));
      PAT_HIP(hipMemsetAsync(I.q.p, 0, sizeof(T) * nb, s));
      if (I.r.p) PAT_HIP(hipMemsetAsync(I.r.p, 0, I.r.bytes, s));
      if (I.v.p) PAT_HIP(hipMemsetAsync(I.v.p, 0, I.v.bytes, s));
      if (I.vbar.p) PAT_HIP(hipMemsetAsync(I.vbar.p, 0, I.vbar.bytes, s));
      if (I.s.p) PAT_HIP(hipMemsetAsync(I.s.p, 0, I.s.bytes, s));
      if (I.opts.d_state_in) {
        const T* st = static_cast<const T*>(I.opts.d_state_in);
        PAT_HIP(hipMemcpyAsync(I.u.p, st, sizeof(T) * N, hipMemcpyDeviceToDevice, s));
        pad_slots(I, st + N, ptr<T>(I.ubar_pad));
        int64_t o = 2 * N;
        PAT_HIP(hipMemcpyAsync(I.q.p, st + o, sizeof(T) * nb, hipMemcpyDeviceToDevice, s));
        o += nb;
        if (I.r.p) {
          PAT_HIP(hipMemcpyAsync(I.r.p, st + o, I.r.bytes, hipMemcpyDeviceToDevice, s));
          o += (int64_t)(I.r.bytes / sizeof(T));
        }
        if (I.reg.kind == PAT_REG_TGV) {
          PAT_HIP(hipMemcpyAsync(I.v.p, st + o, sizeof(T) * 2 * N, hipMemcpyDeviceToDevice, s));
          PAT_HIP(hipMemcpyAsync(I.vbar.p, st + o + 2 * N, sizeof(T) * 2 * N, hipMemcpyDeviceToDevice, s));
          PAT_HIP(hipMemcpyAsync(I.s.p, st + o + 4 * N, sizeof(T) * 3 * N, hipMemcpyDeviceToDevice, s));
        }
      }
    }
    // warm starts: accept only a finite (u0[, y0]) with P(u0) <= P(0) = 1/2 ||f||^2
    bool any_u0 = false;
    for (int k : act) any_u0 |= (inst[k]->opts.d_u0 != nullptr && !inst[k]->opts.d_state_in);
    if (!any_u0) return;
    for (int k : act) {
      Inst<T>& I = *inst[k];
      if (!I.opts.d_u0 || I.opts.d_state_in) continue;
      PAT_HIP(hipMemcpyAsync(I.u.p, I.opts.d_u0, sizeof(T) * I.g->n_pix(), hipMemcpyDeviceToDevice, s));
      pad_slots(I, ptr<T>(I.u), ptr<T>(I.upad_gap));
    }
    enqueue_gap(0);
    read_results(1);
    DevBuf part(sizeof(double) * 512), acc(sizeof(double));
    for (size_t a = 0; a < act.size(); ++a) {
      Inst<T>& I = *inst[act[a]];
      if (!I.opts.d_u0 || I.opts.d_state_in) continue;
      const double* r = h_results + a * GAP_NSLOTS;
      const double P0 = r[GAP_DATA] + r[GAP_REG];
      const int64_t nb = I.g->n_bins(), N = I.g->n_pix();
      launch_dot<T>(I.f, I.f, nb, ptr<double>(part), 512, ptr<double>(acc), s);
      double ff = 0.0, yy = 0.0;
      PAT_HIP(hipMemcpyAsync(&ff, acc.p, sizeof(double), hipMemcpyDeviceToHost, s));
      PAT_HIP(hipStreamSynchronize(s));
      const T* y0 = static_cast<const T*>(I.opts.d_y0);
      if (y0) {
        // q0 [n_bins] then r0 [2][N]: a finite sum of squares means finite entries
        launch_dot<T>(y0, y0, nb + 2 * N, ptr<double>(part), 512, ptr<double>(acc), s);
        PAT_HIP(hipMemcpyAsync(&yy, acc.p, sizeof(double), hipMemcpyDeviceToHost, s));
        PAT_HIP(hipStreamSynchronize(s));
      }
      if (!std::isfinite(P0) || P0 > 0.5 * ff || !std::isfinite(yy)) {
        I.fallback = 1;
        PAT_HIP(hipMemsetAsync(I.u.p, 0, I.u.bytes, s));
      } else {
        pad_slots(I, ptr<T>(I.u), ptr<T>(I.ubar_pad));
        if (y0) {
          PAT_HIP(hipMemcpyAsync(I.q.p, y0, sizeof(T) * nb, hipMemcpyDeviceToDevice, s));
          PAT_HIP(hipMemcpyAsync(I.r.p, y0 + nb, sizeof(T) * 2 * N, hipMemcpyDeviceToDevice, s));
        }
      }
    }
    PAT_HIP(hipStreamSynchronize(s));
  }

  void read_results(int n_checks) {
    const size_t bytes = sizeof(double) * (size_t)n_checks * L.n * GAP_NSLOTS;
    PAT_HIP(hipMemcpyAsync(h_results, results.p, bytes, hipMemcpyDeviceToHost, s));
    PAT_HIP(hipStreamSynchronize(s));
  }

  // Evaluate check c for the active instance at position a.
  pat_status evaluate(int c, int a, int n_done) {
    Inst<T>& I = *inst[act[a]];
    const double* r = h_results + ((size_t)c * L.n + a) * GAP_NSLOTS;
    const double P = r[GAP_DATA] + r[GAP_REG];
    const double Fs = r[GAP_FSTAR];
    double gap;
    if (I.reg.kind == PAT_REG_TIKHONOV) gap = P + Fs + r[GAP_KTY] / (2.0 * I.reg.lambda);
    else gap = P + Fs + I.opts.gap_box * r[GAP_KTY];
    I.primal = P;
    I.fstar = Fs;
    I.kty = r[GAP_KTY];
    I.gap = gap;
    I.rel_gap = P > 0.0 ? gap / P : (gap == 0.0 ? 0.0 : INFINITY);
    I.residual = r[GAP_U2] > 0.0 ? std::sqrt(r[GAP_DU2] / r[GAP_U2]) : INFINITY;
    I.iters = n_done;
    if (!std::isfinite(gap)) {
      set_error("non-finite primal-dual gap at iteration %d", n_done);
      return PAT_ERR_NUMERIC;
    }
    return PAT_OK;
  }

  hipGraphExec_t graph_for(int steps, const std::vector<int>& checks) {
    std::string key = std::to_string(steps) + (accel_live ? "s" : "");
    for (int c : checks) key += "," + std::to_string(c);
    auto it = graphs.find(key);
    if (it != graphs.end()) return it->second;
    hipGraph_t graph;
    PAT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    try {
      run_direct(steps, checks);
    } catch (...) {
      hipGraph_t tmp;
      (void)hipStreamEndCapture(s, &tmp);
      if (tmp) (void)hipGraphDestroy(tmp);
      throw;
    }
    PAT_HIP(hipStreamEndCapture(s, &graph));
    hipGraphExec_t exec;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    PAT_HIP(e);
    graphs[key] = exec;
    return exec;
  }

  void run_direct(int steps, const std::vector<int>& checks) {
    size_t c = 0;
    for (int t = 0; t < steps; ++t) {
      const bool chk = c < checks.size() && checks[c] == t;
      enqueue_iteration(t, chk, (int)c);
      if (chk) ++c;
    }
  }

  // Run all instances to convergence or their caps.
  pat_status run(double* seconds) {
    int n_done = 0;
    hipEvent_t e0, e1;
    PAT_HIP(hipEventCreate(&e0));
    PAT_HIP(hipEventCreate(&e1));
    PAT_HIP(hipEventRecord(e0, s));
    pat_status worst = PAT_OK;
    int max_cap = 0;
    for (auto& ip : inst) max_cap = std::max(max_cap, ip->opts.max_iter);
    while (!act.empty()) {
      int cap = max_cap;
      for (int k : act) cap = std::min(cap, inst[k]->opts.max_iter);
      const int block = graph_block > 0 ? graph_block : gap_every;
      const int steps = std::min(block, cap - n_done);
      // the gap is evaluated once per block, at its last iteration (the
      // block ends at a multiple of gap_every or at the cap): a check inside
      // a block could not stop the solve there
      const std::vector<int> checks(1, steps - 1);
      upload_schedule(steps);
      if (graph_block > 0) {
        PAT_HIP(hipGraphLaunch(graph_for(steps, checks), s));
      } else {
        run_direct(steps, checks);
      }
      n_done += steps;
      read_results((int)checks.size());
      // decide on the last check of the block
      const int c = (int)checks.size() - 1;
      std::vector<int> keep;
      for (size_t a = 0; a < act.size(); ++a) {
        Inst<T>& I = *inst[act[a]];
        const pat_status st = evaluate(c, (int)a, n_done);
        if (st != PAT_OK) {
          I.status = st;
          I.active = false;
          worst = st;
          continue;
        }
        if (I.opts.gap_tol > 0.0 && I.rel_gap <= I.opts.gap_tol) {
          I.converged = true;
          I.status = PAT_OK;
          I.active = false;
        } else if (n_done >= I.opts.max_iter) {
          I.status = I.opts.gap_tol > 0.0 ? PAT_NOT_CONVERGED : PAT_OK;
          I.converged = false;
          I.active = false;
        } else {
          keep.push_back(act[a]);
        }
        if (!I.active) finish_instance(I);
      }
      if (keep.size() != act.size()) {
        act = keep;
        if (!act.empty()) build_launch();
      }
    }
    PAT_HIP(hipEventRecord(e1, s));
    PAT_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    PAT_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *seconds = ms * 1e-3;
    for (auto& ip : inst) {
      if (ip->status < 0) return ip->status;
      if (ip->status == PAT_NOT_CONVERGED) worst = worst == PAT_OK ? PAT_NOT_CONVERGED : worst;
    }
    return worst;
  }

  void finish_instance(Inst<T>& I) {
    pat_geometry g = I.g;
    const int64_t N = g->n_pix(), nb = g->n_bins();
    if (I.status >= 0) {
      PAT_HIP(hipMemcpyAsync(I.u_out, I.u.p, sizeof(T) * N, hipMemcpyDeviceToDevice, s));
      if (I.opts.d_state_out) {
        T* st = static_cast<T*>(I.opts.d_state_out);
        PAT_HIP(hipMemcpyAsync(st, I.u.p, sizeof(T) * N, hipMemcpyDeviceToDevice, s));
        const int P = g->nx + 2;
        PAT_HIP(hipMemcpy2DAsync(st + N, sizeof(T) * g->nx, ptr<T>(I.ubar_pad) + P + 1, sizeof(T) * P,
                                 sizeof(T) * g->nx, g->ny, hipMemcpyDeviceToDevice, s));
        int64_t o = 2 * N;
        PAT_HIP(hipMemcpyAsync(st + o, I.q.p, sizeof(T) * nb, hipMemcpyDeviceToDevice, s));
        o += nb;
        if (I.r.p) {
          PAT_HIP(hipMemcpyAsync(st + o, I.r.p, I.r.bytes, hipMemcpyDeviceToDevice, s));
          o += (int64_t)(I.r.bytes / sizeof(T));
        }
        if (I.reg.kind == PAT_REG_TGV) {
          PAT_HIP(hipMemcpyAsync(st + o, I.v.p, sizeof(T) * 2 * N, hipMemcpyDeviceToDevice, s));
          PAT_HIP(hipMemcpyAsync(st + o + 2 * N, I.vbar.p, sizeof(T) * 2 * N, hipMemcpyDeviceToDevice, s));
          PAT_HIP(hipMemcpyAsync(st + o + 4 * N, I.s.p, sizeof(T) * 3 * N, hipMemcpyDeviceToDevice, s));
        }
      }
    }
    if (I.info) {
      I.info->iters = I.iters;
      I.info->converged = I.converged ? 1 : 0;
      I.info->fallback = I.fallback;
      I.info->rel_gap = I.rel_gap;
      I.info->gap = I.gap;
      I.info->primal = I.primal;
      I.info->fstar = I.fstar;
      I.info->kty_l1 = I.kty;
      I.info->residual = I.residual;
    }
  }
};

// The library stream: a caller's NULL stream cannot be captured into a graph,
// so solves on NULL run on a blocking stream of the library (ordered with NULL).
static hipStream_t solve_stream(void* user, hipStream_t* owned) {
  *owned = nullptr;
  if (user) return static_cast<hipStream_t>(user);
  PAT_HIP(hipStreamCreate(owned));
  return *owned;
}

template <class T>
static pat_status solve_impl(int n, const pat_geometry* g, const void* const* d_f,
                             const pat_regulariser* reg, const pat_solve_opts* opts,
                             void* const* d_u_out, pat_solve_info* info, void* stream) {
  hipStream_t owned = nullptr;
  hipStream_t s = solve_stream(stream, &owned);
  struct StreamGuard {
    hipStream_t h;
    ~StreamGuard() {
      if (h) { (void)hipStreamSynchronize(h); (void)hipStreamDestroy(h); }
    }
  } guard{owned};
  Solver<T> S;
  S.gap_every = opts[0].gap_every;
  S.graph_block = opts[0].graph_block;
  if (S.graph_block > 0 && S.graph_block % S.gap_every != 0)
    S.graph_block = ((S.graph_block + S.gap_every - 1) / S.gap_every) * S.gap_every;
  for (int i = 0; i < n; ++i) {
    auto I = std::make_unique<Inst<T>>();
    I->g = g[i];
    I->reg = reg[i];
    I->opts = opts[i];
    I->f = static_cast<const T*>(d_f[i]);
    I->u_out = static_cast<T*>(d_u_out[i]);
    I->info = info ? &info[i] : nullptr;
    S.inst.push_back(std::move(I));
  }
  S.setup(s);
  S.build_launch();
  S.init_state();
  double secs = 0.0;
  const pat_status st = S.run(&secs);
  PAT_HIP(hipStreamSynchronize(s));
  if (info)
    for (int i = 0; i < n; ++i) info[i].seconds = secs;
  return st;
}

// Average duration (ms) of each launch of the solver's iteration, by HIP
// events over `reps` launches after one untimed launch, on instances set up
// as the batched solver sets them up (zero start).
template <class T>
static void kernel_times_impl(int n, const pat_geometry* g, const void* const* d_f, const pat_regulariser* reg,
                              const pat_solve_opts* opts, int reps, double* ms, void* stream) {
  hipStream_t owned = nullptr;
  hipStream_t s = solve_stream(stream, &owned);
  struct StreamGuard {
    hipStream_t h;
    ~StreamGuard() {
      if (h) { (void)hipStreamSynchronize(h); (void)hipStreamDestroy(h); }
    }
  } guard{owned};
  Solver<T> S;
  S.gap_every = opts[0].gap_every;
  S.graph_block = opts[0].graph_block;
  for (int i = 0; i < n; ++i) {
    auto I = std::make_unique<Inst<T>>();
    I->g = g[i];
    I->reg = reg[i];
    I->opts = opts[i];
    I->f = static_cast<const T*>(d_f[i]);
    S.inst.push_back(std::move(I));
  }
  S.setup(s);
  S.build_launch();
  S.init_state();
  hipEvent_t e0, e1;
  PAT_HIP(hipEventCreate(&e0));
  PAT_HIP(hipEventCreate(&e1));
  auto timeit = [&](auto&& fn) {
    fn();
    PAT_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) fn();
    PAT_HIP(hipEventRecord(e1, s));
    PAT_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    PAT_HIP(hipEventElapsedTime(&t, e0, e1));
    return (double)t / reps;
  };
  try {
    ms[0] = timeit([&] { launch_forward_reg_batched<T>(S.L, S.lanes_log2, s); });
    ms[1] = timeit([&] {
      launch_reg_dual<T>(S.L, s);
      S.enqueue_wavelet_dual();
      S.enqueue_wavelet_synthesis(false);
    });
    ms[2] = timeit([&] { S.enqueue_adjoint(false); });
    ms[3] = timeit([&] { launch_primal<T>(S.L, false, s); });
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

static void validate_instance(pat_geometry g, const void* f, const pat_regulariser* reg,
                              const pat_solve_opts* o, void* u) {
  PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
  PAT_CHECK_ARG(f != nullptr && u != nullptr, "NULL data or output buffer");
  validate_regulariser(g, reg);
  validate_opts(o);
  if (o->precond)
    PAT_CHECK_ARG(o->precond->g == g && o->precond->reg_kind == reg->kind,
                  "precond handle was made for another geometry or regulariser");
  if (o->d_y0) {
    PAT_CHECK_ARG(o->d_u0 != nullptr && o->d_state_in == nullptr, "d_y0 goes with d_u0 and no d_state_in");
    PAT_CHECK_ARG(reg->kind == PAT_REG_TV || reg->kind == PAT_REG_DTV, "d_y0 needs a TV or dTV regulariser");
  }
}

}  // namespace pat

using pat::guarded;

extern "C" pat_status pat_precond(pat_geometry g, const pat_regulariser* reg, int32_t kind,
                                  void* stream, pat_precond_h* out) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr && out != nullptr, "NULL argument");
    pat::validate_regulariser(g, reg);
    PAT_CHECK_ARG(kind == PAT_PRECOND_DIAG || kind == PAT_PRECOND_BLOCK, "unknown precond kind");
    hipStream_t owned = nullptr;
    hipStream_t s = pat::solve_stream(stream, &owned);
    pat_status st = PAT_OK;
    try {
      *out = pat::make_precond(g, reg, kind, s);
    } catch (...) {
      if (owned) (void)hipStreamDestroy(owned);
      throw;
    }
    if (owned) (void)hipStreamDestroy(owned);
    return st;
  });
}

extern "C" pat_status pat_precond_get(pat_precond_h p, int32_t which, void* d_dst, void* stream) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(p != nullptr && d_dst != nullptr, "NULL argument");
    const pat::DevBuf* b = nullptr;
    switch (which) {
      case 0: b = &p->sigma_q; break;
      case 1: b = &p->sigma_r; break;
      case 2: b = &p->sigma_s; break;
      case 3: b = &p->tau_u; break;
      case 4: b = &p->tau_v; break;
      default: break;
    }
    PAT_CHECK_ARG(b != nullptr && b->p != nullptr, "step-size array not present for this regulariser");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (which == 4) {
      // both components of v share one step size: export [2][N]
      PAT_HIP(hipMemcpyAsync(d_dst, b->p, b->bytes, hipMemcpyDeviceToDevice, s));
      PAT_HIP(hipMemcpyAsync(static_cast<char*>(d_dst) + b->bytes, b->p, b->bytes,
                             hipMemcpyDeviceToDevice, s));
    } else {
      PAT_HIP(hipMemcpyAsync(d_dst, b->p, b->bytes, hipMemcpyDeviceToDevice, s));
    }
    return PAT_OK;
  });
}

extern "C" pat_status pat_precond_destroy(pat_precond_h p) {
  return guarded([&]() -> pat_status {
    delete p;
    return PAT_OK;
  });
}

extern "C" pat_status pat_state_elems(pat_geometry g, int32_t reg_kind, int64_t* out) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr && out != nullptr, "NULL argument");
    PAT_CHECK_ARG(reg_kind >= PAT_REG_TV && reg_kind <= PAT_REG_WAVELET, "unknown regulariser kind");
    *out = pat::state_elems(g, reg_kind);
    return PAT_OK;
  });
}

extern "C" pat_status pat_pdhg_solve(pat_geometry g, const void* d_f, const pat_regulariser* reg,
                                     const pat_solve_opts* opts, void* d_u_out,
                                     pat_solve_info* info, void* stream) {
  return guarded([&]() -> pat_status {
    pat::validate_instance(g, d_f, reg, opts, d_u_out);
    if (g->dtype == PAT_F64)
      return pat::solve_impl<double>(1, &g, &d_f, reg, opts, &d_u_out, info, stream);
    return pat::solve_impl<float>(1, &g, &d_f, reg, opts, &d_u_out, info, stream);
  });
}

extern "C" pat_status pat_pdhg_solve_batched(int32_t n, const pat_geometry* g, const void* const* d_f,
                                             const pat_regulariser* reg, const pat_solve_opts* opts,
                                             void* const* d_u_out, pat_solve_info* info,
                                             void* stream) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(n >= 1, "n must be >= 1");
    PAT_CHECK_ARG(g && d_f && reg && opts && d_u_out, "NULL array");
    for (int i = 0; i < n; ++i) {
      pat::validate_instance(g[i], d_f[i], &reg[i], &opts[i], d_u_out[i]);
      PAT_CHECK_ARG(g[i]->dtype == g[0]->dtype, "batched solves need one element type");
    }
    if (g[0]->dtype == PAT_F64)
      return pat::solve_impl<double>(n, g, d_f, reg, opts, d_u_out, info, stream);
    return pat::solve_impl<float>(n, g, d_f, reg, opts, d_u_out, info, stream);
  });
}

extern "C" pat_status pat_pdhg_kernel_times(int32_t n, const pat_geometry* g, const void* const* d_f,
                                            const pat_regulariser* reg, const pat_solve_opts* opts,
                                            int32_t reps, double* ms, void* stream) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(n >= 1, "n must be >= 1");
    PAT_CHECK_ARG(reps >= 1, "reps must be >= 1");
    PAT_CHECK_ARG(g && d_f && reg && opts && ms, "NULL array");
    for (int i = 0; i < n; ++i) {
      PAT_CHECK_ARG(g[i] != nullptr && d_f[i] != nullptr, "NULL geometry or data");
      pat::validate_regulariser(g[i], &reg[i]);
      PAT_CHECK_ARG(opts[i].d_u0 == nullptr && opts[i].d_y0 == nullptr && opts[i].d_state_in == nullptr,
                    "kernel timing starts from zero (no warm start or state)");
      PAT_CHECK_ARG(opts[i].gap_every >= 1 && opts[i].graph_block >= 0, "bad gap_every or graph_block");
      if (opts[i].precond)
        PAT_CHECK_ARG(opts[i].precond->g == g[i] && opts[i].precond->reg_kind == reg[i].kind,
                      "precond handle was made for another geometry or regulariser");
      PAT_CHECK_ARG(g[i]->dtype == g[0]->dtype, "one element type for all instances");
    }
    if (g[0]->dtype == PAT_F64) pat::kernel_times_impl<double>(n, g, d_f, reg, opts, reps, ms, stream);
    else pat::kernel_times_impl<float>(n, g, d_f, reg, opts, reps, ms, stream);
    return PAT_OK;
  });
}
