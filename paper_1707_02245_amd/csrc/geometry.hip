// Geometry tables of the circular-mean operator (arXiv:1707.02245, Sec. 3.3.1
// discretisation of eq. K_def in Sec. 4.1) and the C-ABI entry points that
// create and describe them.
//
// Every arc sample is addressed by (detector d, radius k, sample m). Its
// position in continuous pixel-index units (pixel i has its centre at gx = i) is
//
//     gx = gdx_d + rho_k cos(phi_km),  gy = gdy_d + rho_k sin(phi_km),
//     phi_km = 2 pi (m + 1/2) / M_k,   rho_k = r_k / h,
//     M_k = max(1, 4 ceil(2 pi r_k s / (4 h)))   (a multiple of four, so each
//     circle's samples are invariant under quarter turns),
//
// evaluated in FP64 from FP64 tables by every kernel that touches samples, so
// the forward and the adjoint see bit-identical positions and weights.
// Per bin, the host computes up to four ranges of m whose samples can carry a
// non-zero weight (the arc clipped to the grid's support box), so the forward
// kernel skips the arc outside the image.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <thread>

#include "pat_internal.hpp"

namespace pat {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct Range {
  int a, b;  // [a, b)
};

// Sample ranges of one circle (centre (cx, cy), radius rho, M samples) whose
// samples may fall in the closed box [x0,x1]x[y0,y1] (grid index units).
// Conservative: one extra sample on each side of every angular interval.
int circle_box_ranges(double cx, double cy, double rho, int M, double x0, double x1,
                      double y0, double y1, Range out[4]) {
  const double eps = 1e-3;  // box growth, far above the FP64 position error
  x0 -= eps; y0 -= eps; x1 += eps; y1 += eps;
  auto inside = [&](double a) {
    const double x = cx + rho * std::cos(a), y = cy + rho * std::sin(a);
    return x >= x0 && x <= x1 && y >= y0 && y <= y1;
  };
  // distance bounds: skip circles that cannot meet the box
  const double dx = std::max({x0 - cx, 0.0, cx - x1});
  const double dy = std::max({y0 - cy, 0.0, cy - y1});
  const double dmin = std::hypot(dx, dy);
  double dmax = 0.0;
  for (double sx : {x0, x1})
    for (double sy : {y0, y1}) dmax = std::max(dmax, std::hypot(sx - cx, sy - cy));
  if (rho < dmin - eps || rho > dmax + eps) return 0;
  if (M == 1 || rho == 0.0) {
    if (inside(0.5 * kTwoPi)) { out[0] = {0, M}; return 1; }
    return 0;
  }
  // crossing angles with the four box lines
  double cand[10];
  int nc = 0;
  cand[nc++] = 0.0;
  for (double xv : {x0, x1}) {
    const double t = (xv - cx) / rho;
    if (t > -1.0 && t < 1.0) {
      const double a = std::acos(t);
      cand[nc++] = a;
      cand[nc++] = kTwoPi - a;
    }
  }
  for (double yh : {y0, y1}) {
    const double t = (yh - cy) / rho;
    if (t > -1.0 && t < 1.0) {
      double a = std::asin(t);
      if (a < 0) a += kTwoPi;
      cand[nc++] = a;
      double b = 0.5 * kTwoPi - std::asin(t);
      if (b < 0) b += kTwoPi;
      cand[nc++] = b;
    }
  }
  std::sort(cand, cand + nc);
  // sub-arcs between consecutive crossings are entirely inside or outside
  Range raw[12];
  int nr = 0;
  for (int i = 0; i < nc; ++i) {
    const double a = cand[i], b = (i + 1 < nc) ? cand[i + 1] : kTwoPi;
    if (b - a <= 0.0) continue;
    if (!inside(0.5 * (a + b))) continue;
    // samples with phi in [a, b]: m + 1/2 in [a M / 2pi, b M / 2pi]
    int lo = (int)std::floor(a * M / kTwoPi - 0.5) - 1;
    int hi = (int)std::ceil(b * M / kTwoPi - 0.5) + 1;  // inclusive
    if (hi - lo + 1 >= M) { out[0] = {0, M}; return 1; }
    // split at the wrap so every range lies in [0, M)
    if (lo < 0) {
      raw[nr++] = {lo + M, M};
      lo = 0;
    }
    if (hi >= M) {
      raw[nr++] = {0, hi - M + 1};
      hi = M - 1;
    }
    if (lo <= hi) raw[nr++] = {lo, hi + 1};
  }
  if (nr == 0) return 0;
  std::sort(raw, raw + nr, [](const Range& p, const Range& q) { return p.a < q.a; });
  // merge overlapping or touching ranges
  Range mg[12];
  int nm = 0;
  for (int i = 0; i < nr; ++i) {
    if (nm > 0 && raw[i].a <= mg[nm - 1].b) {
      mg[nm - 1].b = std::max(mg[nm - 1].b, raw[i].b);
    } else {
      mg[nm++] = raw[i];
    }
  }
  // at most four ranges: close the smallest gaps (still exact, more work)
  while (nm > 4) {
    int best = 0;
    for (int i = 1; i + 1 < nm; ++i)
      if (mg[i + 1].a - mg[i].b < mg[best + 1].a - mg[best].b) best = i;
    mg[best].b = mg[best + 1].b;
    for (int i = best + 1; i + 1 < nm; ++i) mg[i] = mg[i + 1];
    --nm;
  }
  for (int i = 0; i < nm; ++i) out[i] = mg[i];
  return nm;
}

static bool finite_all(std::initializer_list<double> xs) {
  for (double x : xs)
    if (!std::isfinite(x)) return false;
  return true;
}

void validate_geometry_desc(const pat_geometry_desc* d) {
  PAT_CHECK_ARG(d != nullptr, "desc is NULL");
  PAT_CHECK_ARG(d->nx >= 2 && d->ny >= 2, "nx and ny must be >= 2");
  PAT_CHECK_ARG(d->nx <= 16384 && d->ny <= 16384, "nx and ny must be <= 16384");
  PAT_CHECK_ARG(d->n_det >= 1, "n_det must be >= 1");
  PAT_CHECK_ARG(d->n_t >= 2, "n_t must be >= 2");
  PAT_CHECK_ARG((int64_t)d->n_det * d->n_t <= (int64_t(1) << 28), "n_det * n_t too large");
  PAT_CHECK_ARG(finite_all({d->x_min, d->x_max, d->y_min, d->y_max, d->det_cx, d->det_cy,
                            d->det_radius, d->arc_center, d->arc_span, d->t0, d->dt, d->c,
                            d->samples_per_pixel}),
                "non-finite scalar in geometry");
  PAT_CHECK_ARG(d->x_max > d->x_min && d->y_max > d->y_min, "empty image domain");
  const double hx = (d->x_max - d->x_min) / d->nx, hy = (d->y_max - d->y_min) / d->ny;
  PAT_CHECK_ARG(std::fabs(hx - hy) <= 1e-9 * std::max(hx, hy), "pixels must be square");
  PAT_CHECK_ARG(d->dt > 0.0 && d->c > 0.0 && d->samples_per_pixel > 0.0,
                "dt, c and samples_per_pixel must be > 0");
  PAT_CHECK_ARG(d->t0 >= 0.0, "t0 must be >= 0");
  if (d->det_xy) {
    for (int i = 0; i < 2 * d->n_det; ++i)
      PAT_CHECK_ARG(std::isfinite(d->det_xy[i]), "non-finite detector position");
  } else {
    PAT_CHECK_ARG(d->arc_span > 0.0 && d->arc_span <= kTwoPi + 1e-12,
                  "arc_span must be in (0, 2 pi]");
    PAT_CHECK_ARG(d->det_radius >= 0.0, "det_radius must be >= 0");
  }
  const double r_max = d->c * (d->t0 + d->dt * (d->n_t - 1));
  const double m_max = 4.0 * std::ceil(kTwoPi * r_max * d->samples_per_pixel / (4.0 * hx));
  PAT_CHECK_ARG(m_max < 4.0e6, "too many arc samples per circle");
}

}  // namespace pat

using pat::Range;

void pat_geometry_s::build_host() {
  const pat_geometry_desc& d = desc;
  using pat::kTwoPi;
  nx = d.nx; ny = d.ny; n_det = d.n_det; n_t = d.n_t;
  h = (d.x_max - d.x_min) / nx;
  det_xy.resize(2 * (size_t)n_det);
  if (d.det_xy) {
    std::memcpy(det_xy.data(), d.det_xy, sizeof(double) * 2 * n_det);
  } else {
    const bool closed = std::fabs(d.arc_span - kTwoPi) < 1e-12;
    for (int i = 0; i < n_det; ++i) {
      double a;
      if (closed) a = d.arc_center + kTwoPi * i / n_det;
      else if (n_det == 1) a = d.arc_center;
      else a = d.arc_center - 0.5 * d.arc_span + d.arc_span * i / (n_det - 1);
      det_xy[2 * i] = d.det_cx + d.det_radius * std::cos(a);
      det_xy[2 * i + 1] = d.det_cy + d.det_radius * std::sin(a);
    }
  }
  M.resize(n_t);
  off.resize(n_t);
  radius.resize(n_t);
  int64_t acc = 0;
  for (int k = 0; k < n_t; ++k) {
    const double r = d.c * (d.t0 + k * d.dt);
    radius[k] = r;
    const double m = 4.0 * std::ceil(kTwoPi * r * d.samples_per_pixel / (4.0 * h));
    M[k] = std::max(1, (int)m);
    off[k] = acc;
    acc += M[k];
  }
  n_samples_per_det = acc;
  PAT_CHECK_ARG(acc < (int64_t(1) << 31), "sample table too large");
  // Quarter-turn symmetry: in grid index units the quarter turn about the
  // centre c = (n-1)/2 of a square grid maps (gx, gy) to (n-1-gy, gx); the
  // ring is symmetric when detector d + n_det/4 sits there for every d (to 64
  // ulps of the coordinates). With every M_k a multiple of four (or the single
  // sample of r = 0, at the detector itself) the sample sets follow.
  sym_rot = 1;
  if (nx == ny && n_det % 4 == 0) {
    const int q = n_det / 4;
    bool ok = true;
    auto gx = [&](int i) { return (det_xy[2 * i] - d.x_min) / h - 0.5; };
    auto gy = [&](int i) { return (det_xy[2 * i + 1] - d.y_min) / h - 0.5; };
    for (int i = 0; i < n_det && ok; ++i) {
      const int j = (i + q) % n_det;
      const double ex = (double)(nx - 1) - gy(i), ey = gx(i);
      const double tol = 64.0 * 2.220446049250313e-16 *
                         std::max({1.0, std::fabs(ex), std::fabs(ey), std::fabs(gx(j)), std::fabs(gy(j))});
      ok = std::fabs(gx(j) - ex) <= tol && std::fabs(gy(j) - ey) <= tol;
    }
    for (int k = 0; k < n_t && ok; ++k) ok = (M[k] % 4 == 0) || radius[k] == 0.0;
    if (ok) sym_rot = 4;
  }
}

void pat_geometry_s::upload(hipStream_t stream) {
  using pat::kTwoPi;
  using pat::DevBuf;
  // detector positions and radii in grid index units
  std::vector<double2> h_det(n_det), h_rad(n_t), h_cs(n_samples_per_det);
  std::vector<int2> h_moff(n_t);
  for (int i = 0; i < n_det; ++i) {
    h_det[i].x = (det_xy[2 * i] - desc.x_min) / h - 0.5;
    h_det[i].y = (det_xy[2 * i + 1] - desc.y_min) / h - 0.5;
  }
  for (int k = 0; k < n_t; ++k) {
    h_rad[k].x = radius[k] / h;
    h_rad[k].y = 1.0 / M[k];
    h_moff[k] = make_int2(M[k], off[k]);
    for (int m = 0; m < M[k]; ++m) {
      const double phi = kTwoPi * (m + 0.5) / M[k];
      h_cs[off[k] + m] = make_double2(std::cos(phi), std::sin(phi));
    }
  }
  // clip windows: ranges of m whose samples can carry weight on the grid,
  // i.e. lie in the box [-1, nx] x [-1, ny] of index space
  const int64_t nb = (int64_t)n_det * n_t;
  std::vector<int4> h_win(2 * nb);
  std::vector<int64_t> work(n_t, 0);
  n_window = 0;
  for (int i = 0; i < n_det; ++i) {
    for (int k = 0; k < n_t; ++k) {
      Range rg[4];
      const int n = pat::circle_box_ranges(h_det[i].x, h_det[i].y, h_rad[k].x, M[k], -1.0,
                                      (double)nx, -1.0, (double)ny, rg);
      int v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int j = 0; j < n; ++j) {
        v[2 * j] = rg[j].a;
        v[2 * j + 1] = rg[j].b;
        n_window += rg[j].b - rg[j].a;
        work[k] += rg[j].b - rg[j].a;
      }
      const int64_t b = (int64_t)i * n_t + k;
      h_win[2 * b] = make_int4(v[0], v[1], v[2], v[3]);
      h_win[2 * b + 1] = make_int4(v[4], v[5], v[6], v[7]);
    }
  }
  d_det.alloc(sizeof(double2) * n_det);
  d_rad.alloc(sizeof(double2) * n_t);
  d_moff.alloc(sizeof(int2) * n_t);
  // the table is FP64 for every element type (positions are FP64)
  d_cs.alloc(sizeof(double2) * n_samples_per_det);
  d_win.alloc(sizeof(int4) * 2 * nb);
  // the radius-major gather takes its heaviest radii first, so that the
  // light ones fill the end of the launch
  std::vector<int> kord(n_t);
  std::iota(kord.begin(), kord.end(), 0);
  std::stable_sort(kord.begin(), kord.end(), [&](int a, int b) { return work[a] > work[b]; });
  d_kord.alloc(sizeof(int) * n_t);
  PAT_HIP(hipMemcpyAsync(d_kord.p, kord.data(), d_kord.bytes, hipMemcpyHostToDevice, stream));
  PAT_HIP(hipMemcpyAsync(d_det.p, h_det.data(), d_det.bytes, hipMemcpyHostToDevice, stream));
  PAT_HIP(hipMemcpyAsync(d_rad.p, h_rad.data(), d_rad.bytes, hipMemcpyHostToDevice, stream));
  PAT_HIP(hipMemcpyAsync(d_moff.p, h_moff.data(), d_moff.bytes, hipMemcpyHostToDevice, stream));
  PAT_HIP(hipMemcpyAsync(d_cs.p, h_cs.data(), d_cs.bytes, hipMemcpyHostToDevice, stream));
  PAT_HIP(hipMemcpyAsync(d_win.p, h_win.data(), d_win.bytes, hipMemcpyHostToDevice, stream));
  PAT_HIP(hipStreamSynchronize(stream));
}

// Pairs of the LDS-tiled forward. Cell (cx, cy) = (ix + 1, iy + 1) of a
// sample at grid position (gx, gy), ix = floor(gx), reads padded-image pixels
// cx..cx+1, cy..cy+1; cells in [0, nx] x [0, ny] can carry weight. Tile
// (tx, ty) holds cells [tx TS, tx TS + TS) x [ty TS, ty TS + TS), i.e. the
// samples with gx in [tx TS - 1, tx TS + TS - 1) (likewise y). For every bin
// and tile the conservative sample ranges of the circle inside that box
// (circle_box_ranges) become pairs; the kernel keeps the samples whose cell
// is in the tile, so every sample counts in exactly one tile.
void pat_geometry_s::ensure_fwd_tiles(hipStream_t stream) {
  if (fwd_n_pairs >= 0) return;
  const int TS = pat::kFwdTile;
  const int ntx = (nx + 1 + TS - 1) / TS, nty = (ny + 1 + TS - 1) / TS, ntiles = ntx * nty;
  std::vector<std::vector<int4>> per_tile(ntiles);
  auto work = [&](int t0, int t1) {
    for (int t = t0; t < t1; ++t) {
      const int tx = t % ntx, ty = t / ntx;
      const double x0 = tx * TS - 1.0, x1 = std::min(tx * TS + TS, nx + 1) - 1.0;
      const double y0 = ty * TS - 1.0, y1 = std::min(ty * TS + TS, ny + 1) - 1.0;
      std::vector<int4>& out = per_tile[t];
      for (int d = 0; d < n_det; ++d) {
        const double cx = (det_xy[2 * d] - desc.x_min) / h - 0.5;
        const double cy = (det_xy[2 * d + 1] - desc.y_min) / h - 0.5;
        for (int k = 0; k < n_t; ++k) {
          Range rg[4];
          const int n = pat::circle_box_ranges(cx, cy, radius[k] / h, M[k], x0, x1, y0, y1, rg);
          for (int j = 0; j < n; ++j) out.push_back(make_int4(d * n_t + k, rg[j].a, rg[j].b, 0));
        }
      }
    }
  };
  const int nthr = std::max(1, std::min(8, ntiles));
  std::vector<std::thread> th;
  for (int w = 0; w < nthr; ++w) th.emplace_back(work, (int)((int64_t)ntiles * w / nthr), (int)((int64_t)ntiles * (w + 1) / nthr));
  for (auto& x : th) x.join();
  // longest pairs first within a tile, so that the pairs a group of lanes
  // works on together have similar lengths (ties keep bin order)
  for (auto& v : per_tile)
    std::stable_sort(v.begin(), v.end(), [](const int4& p, const int4& q) { return p.z - p.y > q.z - q.y; });
  // partial slots bin-major (each bin's pairs in tile order), workgroups of
  // up to kFwdChunk pairs of one tile
  const int64_t nb = n_bins();
  std::vector<int> bin_off(nb + 1, 0);
  int64_t np = 0;
  for (const auto& v : per_tile) {
    np += (int64_t)v.size();
    for (const int4& p : v) ++bin_off[p.x + 1];
  }
  PAT_CHECK_ARG(np < (int64_t(1) << 31), "too many forward tile pairs");
  for (int64_t b = 0; b < nb; ++b) bin_off[b + 1] += bin_off[b];
  std::vector<int> fill(bin_off.begin(), bin_off.end() - 1);
  std::vector<int4> pairs;
  pairs.reserve(np);
  std::vector<int4> blocks;
  for (int t = 0; t < ntiles; ++t) {
    const int p0 = (int)pairs.size();
    for (int4 p : per_tile[t]) {
      p.w = fill[p.x]++;
      pairs.push_back(p);
    }
    const int p1 = (int)pairs.size();
    for (int c = p0; c < p1; c += pat::kFwdChunk)
      blocks.push_back(make_int4((t % ntx) * TS, (t / ntx) * TS, c, std::min(p1, c + pat::kFwdChunk)));
  }
  fwd_pair.alloc(sizeof(int4) * std::max<int64_t>(np, 1));
  fwd_block.alloc(sizeof(int4) * std::max<size_t>(blocks.size(), 1));
  fwd_bin_off.alloc(sizeof(int) * (nb + 1));
  if (np > 0)
    PAT_HIP(hipMemcpyAsync(fwd_pair.p, pairs.data(), sizeof(int4) * np, hipMemcpyHostToDevice, stream));
  if (!blocks.empty())
    PAT_HIP(hipMemcpyAsync(fwd_block.p, blocks.data(), sizeof(int4) * blocks.size(), hipMemcpyHostToDevice, stream));
  PAT_HIP(hipMemcpyAsync(fwd_bin_off.p, bin_off.data(), sizeof(int) * (nb + 1), hipMemcpyHostToDevice, stream));
  PAT_HIP(hipStreamSynchronize(stream));
  fwd_n_pairs = np;
  fwd_n_blocks = (int)blocks.size();
}

void pat_geometry_s::set_launch(int lanes_log2_, int tile_, int det_group_) {
  PAT_CHECK_ARG(lanes_log2_ >= 4 && lanes_log2_ <= 6, "forward lanes per bin must be 16, 32 or 64");
  PAT_CHECK_ARG(tile_ == 16 || tile_ == 32 || tile_ == 64, "adjoint tile must be 16, 32 or 64");
  PAT_CHECK_ARG(det_group_ >= 1 && det_group_ <= n_det, "adjoint detector group out of range");
  lanes_log2 = lanes_log2_;
  tile = tile_;
  det_group = det_group_;
}

void pat_geometry_s::default_launch() {
  // Scatter adjoint: enough workgroups to fill 256 CUs several times over.
  tile = 32;
  const int tiles = ((nx + tile - 1) / tile) * ((ny + tile - 1) / tile);
  int groups = std::max(1, (2048 + tiles - 1) / tiles);
  groups = std::min(groups, n_det);
  det_group = (n_det + groups - 1) / groups;
  // Forward: 16 lanes per bin keep each lane on several arc samples at the
  // workload sizes (about 200-450 in-window samples per bin); wider groups
  // only for very long arcs. The autotuner refines this per geometry.
  const double per_bin = n_bins() > 0 ? (double)n_window / (double)n_bins() : 0.0;
  lanes_log2 = per_bin > 2048.0 ? 6 : (per_bin > 1024.0 ? 5 : 4);
}

using pat::guarded;

extern "C" pat_status pat_geometry_create(const pat_geometry_desc* desc, pat_dtype dtype,
                                          void* stream, pat_geometry* out) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(out != nullptr, "out is NULL");
    PAT_CHECK_ARG(dtype == PAT_F32 || dtype == PAT_F64, "dtype must be PAT_F32 or PAT_F64");
    pat::validate_geometry_desc(desc);
    std::unique_ptr<pat_geometry_s> g(new pat_geometry_s());
    g->desc = *desc;
    g->desc.det_xy = nullptr;  // the host copy lives in det_xy
    if (desc->det_xy) {
      g->det_xy.assign(desc->det_xy, desc->det_xy + 2 * (size_t)desc->n_det);
      g->desc.det_xy = g->det_xy.data();
    }
    g->dtype = dtype;
    g->build_host();
    g->upload(static_cast<hipStream_t>(stream));
    g->default_launch();
    g->ensure_csr(static_cast<hipStream_t>(stream));
    *out = g.release();
    return PAT_OK;
  });
}

extern "C" pat_status pat_geometry_destroy(pat_geometry g) {
  return guarded([&]() -> pat_status {
    delete g;
    return PAT_OK;
  });
}

extern "C" pat_status pat_geometry_get_info(pat_geometry g, pat_geometry_info* out) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr && out != nullptr, "NULL argument");
    out->nx = g->nx;
    out->ny = g->ny;
    out->n_det = g->n_det;
    out->n_t = g->n_t;
    out->n_pix = (int64_t)g->nx * g->ny;
    out->n_bins = (int64_t)g->n_det * g->n_t;
    out->n_samples = g->n_samples_per_det * g->n_det;
    out->n_window = g->n_window;
    out->dtype = g->dtype;
    out->fwd_lanes_log2 = g->lanes_log2;
    out->adj_tile = g->tile;
    out->adj_det_group = g->det_group;
    out->adj_mode = g->adj_mode != 0 ? g->effective_adj_mode() : 0;
    out->csr_nnz = g->csr_nnz;
    out->csr_tile_side = g->csr_side;
    out->csr_win_max = g->csr_win_max;
    out->csr_rot = g->csr_nnz >= 0 ? g->csr_rot : 1;
    out->sym_rot = g->sym_rot;
    out->csr_waves = g->csr_waves;
    out->csr_lanes = g->csr_lanes;
    out->fwd_path = g->fwd_path;
    out->fwd_pairs = g->fwd_n_pairs;
    out->fwd_sym = g->fwd_qt() ? 4 : 1;
    out->fwd_entries = g->fm_entries;
    return PAT_OK;
  });
}

extern "C" pat_status pat_geometry_set_launch(pat_geometry g, int32_t lanes_log2, int32_t tile,
                                              int32_t det_group) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    g->set_launch(lanes_log2, tile, det_group);
    return PAT_OK;
  });
}

extern "C" pat_status pat_geometry_set_adjoint(pat_geometry g, int32_t mode, void* stream) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    PAT_CHECK_ARG(mode >= 0 && mode <= 2, "adjoint mode must be 0 (scatter), 1 (CSR) or 2 (tiled CSR)");
    if (mode != 0) g->ensure_csr(static_cast<hipStream_t>(stream));
    g->adj_mode = mode;
    return PAT_OK;
  });
}

extern "C" pat_status pat_geometry_set_forward_path(pat_geometry g, int32_t path, void* stream) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    PAT_CHECK_ARG(path >= 0 && path <= 3, "forward path must be 0, 1, 2 or 3");
    if (path == 2) g->ensure_fwd_tiles(static_cast<hipStream_t>(stream));
    if (path == 3) {
      if (g->sym_rot != 4 || !g->sym_enabled) {
        pat::set_error("forward path 3 needs a quarter-turn symmetric geometry with the symmetric A^T storage");
        return PAT_ERR_UNSUPPORTED;
      }
      g->ensure_fmat(static_cast<hipStream_t>(stream));
      if (g->fm_entries <= 0) {
        pat::set_error("forward path 3: a pixel tile touches more bins than its build supports");
        return PAT_ERR_UNSUPPORTED;
      }
    }
    g->fwd_path = path;
    return PAT_OK;
  });
}

extern "C" pat_status pat_geometry_set_tiled_launch(pat_geometry g, int32_t waves, int32_t row_lanes) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    PAT_CHECK_ARG(waves == 4 || waves == 8 || waves == 16, "waves per workgroup must be 4, 8 or 16");
    PAT_CHECK_ARG(row_lanes == 16 || row_lanes == 64, "lanes per row must be 16 or 64");
    g->csr_waves = waves;
    g->csr_lanes = row_lanes;
    return PAT_OK;
  });
}

extern "C" pat_status pat_geometry_set_forward_symmetry(pat_geometry g, int32_t enable) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    g->fwd_sym = enable != 0;
    return PAT_OK;
  });
}

extern "C" pat_status pat_geometry_set_symmetry(pat_geometry g, int32_t enable, void* stream) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    const bool want = enable != 0;
    if (want == g->sym_enabled) return PAT_OK;
    g->sym_enabled = want;
    const int rot = (want && g->sym_rot == 4) ? 4 : 1;
    if (g->csr_nnz >= 0 && rot != g->csr_rot) {
      hipStream_t s = static_cast<hipStream_t>(stream);
      PAT_HIP(hipStreamSynchronize(s));  // no apply may still read the old matrix
      g->drop_csr();
      g->ensure_csr(s);
    }
    // the stored A (path 3) is the quarter-turn storage read the other way
    if (g->fwd_path == 3 && g->csr_rot != 4) g->fwd_path = 0;
    return PAT_OK;
  });
}
