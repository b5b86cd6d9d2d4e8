// Launch-parameter autotuner of the projector kernels, with an on-disk cache.
//
// Candidates: forward lanes per bin (16, 32, 64), block order (radius- or
// detector-major), the LDS-tiled gather, the stored A by pixel tiles
// (symmetric geometries), and the adjoint path (stored
// CSR, plain or with LDS-staged input windows in workgroups of 4, 8 or 16 waves
// and 16 or 64 lanes per row,
// or the matrix-free tile scatter with 16/32/64-pixel tiles and a few
// detector-group sizes). Each candidate is timed with HIP events over `reps`
// stand-alone applies on the caller's stream; the fastest of each kind is
// kept. Results are cached per (device architecture, geometry shape, element
// type, quarter-turn use) in a plain text file: one line per key,
// "key lanes fwd_path fwd_sym adj_mode tile group waves row_lanes t_forward
// t_adjoint".

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>

#include "pat_internal.hpp"

namespace pat {

namespace {

std::string cache_key(const pat_geometry_s* g) {
  hipDeviceProp_t prop;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  char buf[512];
  const int rot = (g->sym_enabled && g->sym_rot == 4) ? 4 : 1;
  std::snprintf(buf, sizeof(buf), "v7|%s|nx=%d|ny=%d|ndet=%d|nt=%d|dt=%d|span=%.6f|r=%.6f|spp=%.4f|t=%.6g|rot=%d",
                arch.c_str(), g->nx, g->ny, g->n_det, g->n_t, g->dtype, g->desc.arc_span,
                g->desc.det_radius, g->desc.samples_per_pixel, g->desc.dt * g->desc.c / g->h, rot);
  return buf;
}

std::map<std::string, std::string> read_cache(const char* path) {
  std::map<std::string, std::string> m;
  if (!path) return m;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t sp = line.find(' ');
    if (sp == std::string::npos) continue;
    m[line.substr(0, sp)] = line.substr(sp + 1);
  }
  return m;
}

void write_cache(const char* path, const std::map<std::string, std::string>& m) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return;  // cache is optional: an unwritable path only skips saving
    for (const auto& kv : m) out << kv.first << ' ' << kv.second << '\n';
  }
  std::rename(tmp.c_str(), path);
}

template <class T>
double time_op(hipStream_t s, int reps, const std::function<void()>& op) {
  op();  // warm-up (first use may build tables)
  hipEvent_t e0, e1;
  PAT_HIP(hipEventCreate(&e0));
  PAT_HIP(hipEventCreate(&e1));
  PAT_HIP(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i) op();
  PAT_HIP(hipEventRecord(e1, s));
  PAT_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  PAT_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (double)ms / reps;
}

template <class T>
void tune(pat_geometry_s* g, int reps, hipStream_t s, pat_autotune_result* res) {
  const int64_t N = g->n_pix(), nb = g->n_bins();
  DevBuf u(sizeof(T) * N), f(sizeof(T) * nb), out_f(sizeof(T) * nb), out_u(sizeof(T) * N);
  launch_pattern<T>(ptr<T>(u), N, s);
  launch_pattern<T>(ptr<T>(f), nb, s);
  // forward: lanes per bin
  double best_f = 1e30;
  int best_l = g->lanes_log2, best_o = g->fwd_path;
  // the quarter-turn form of the gather is left off: timed alone it carries a
  // padding pass that the solver does not run, and in the solver its gain is
  // spent on the primal step's turned copies
  g->fwd_sym = false;
  g->ensure_fwd_tiles(s);
  // the stored A (path 3) where the geometry allows it
  if (g->sym_rot == 4 && g->sym_enabled) g->ensure_fmat(s);
  const int max_path = g->fm_entries > 0 ? 3 : 2;
  for (int o = 0; o <= max_path; ++o)
    for (int l = 4; l <= 6; ++l) {
      if (o >= 2 && l != 4) continue;  // the tiled and stored paths have one shape
      g->lanes_log2 = l;
      g->fwd_path = o;
      const double t = time_op<T>(s, reps, [&] { apply_forward<T>(g, ptr<T>(u), ptr<T>(out_f), s); });
      // a later candidate replaces the best only when clearly faster (3%), so
      // that shapes within run-to-run noise of each other keep the first
      // (the 16-lane radius-major gather), whose batched form shares work
      // between instances on one geometry; the stored A (path 3) only when 10%
      // faster: in the solver its per-bin pass carries the dual data step
      // (11 us at 256^2 in FP64 against 7 us alone) and batched instances on
      // one geometry do not share its stream
      const double margin = o == 3 ? 0.90 : 0.97;
      if (best_f > 1e29 || t < margin * best_f) {
        best_f = t;
        best_l = l;
        best_o = o;
      }
    }
  g->lanes_log2 = best_l;
  g->fwd_path = best_o;
  // adjoint: stored CSR (plain and LDS-staged) vs scatter variants
  double best_a = 1e30;
  int best_mode = 1, best_tile = g->tile, best_group = g->det_group;
  g->adj_mode = 1;
  g->ensure_csr(s);
  int best_wg = g->csr_waves, best_lanes = g->csr_lanes;
  best_a = time_op<T>(s, reps, [&] { apply_adjoint<T>(g, ptr<T>(f), ptr<T>(out_u), s); });
  if (g->csr_side > 0) {
    g->adj_mode = 2;
    for (int lanes : {16, 64})
      for (int wg : {4, 8, 16}) {
        g->csr_waves = wg;
        g->csr_lanes = lanes;
        const double t = time_op<T>(s, reps, [&] { apply_adjoint<T>(g, ptr<T>(f), ptr<T>(out_u), s); });
        if (t < best_a) { best_a = t; best_mode = 2; best_wg = wg; best_lanes = lanes; }
      }
  }
  const int tiles[3] = {16, 32, 64};
  for (int ti = 0; ti < 3; ++ti) {
    const int tile = tiles[ti];
    if (sizeof(T) == 8 && tile == 64) continue;
    const int n_tiles = ((g->nx + tile - 1) / tile) * ((g->ny + tile - 1) / tile);
    for (int target : {1024, 2048, 4096}) {
      int groups = std::min(g->n_det, std::max(1, (target + n_tiles - 1) / n_tiles));
      const int group = (g->n_det + groups - 1) / groups;
      g->adj_mode = 0;
      g->tile = tile;
      g->det_group = group;
      const double t = time_op<T>(s, reps, [&] { apply_adjoint<T>(g, ptr<T>(f), ptr<T>(out_u), s); });
      if (t < best_a) { best_a = t; best_mode = 0; best_tile = tile; best_group = group; }
    }
  }
  g->adj_mode = best_mode;
  g->csr_waves = best_wg;
  g->csr_lanes = best_lanes;
  if (best_mode == 0) {
    g->tile = best_tile;
    g->det_group = best_group;
  }
  res->forward_ms = best_f;
  res->adjoint_ms = best_a;
}

}  // namespace

}  // namespace pat

extern "C" pat_status pat_geometry_autotune(pat_geometry g, const char* cache_path, int32_t reps,
                                            void* stream, pat_autotune_result* out) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    PAT_CHECK_ARG(reps >= 1 && reps <= 10000, "reps must be in [1, 10000]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    pat_autotune_result res{};
    res.from_cache = 0;
    const std::string key = pat::cache_key(g);
    auto cache = pat::read_cache(cache_path);
    auto it = cache.find(key);
    bool applied = false;
    if (it != cache.end()) {
      std::istringstream in(it->second);
      int lanes = 0, mode = -1, tile = 0, group = 0, wg = -1, rl = -1, fo = -1, fsym = -1;
      double tf = 0, ta = 0;
      if (in >> lanes >> fo >> fsym >> mode >> tile >> group >> wg >> rl >> tf >> ta && lanes >= 4 && lanes <= 6 &&
          (fo >= 0 && fo <= 3) && (fsym == 0 || fsym == 1) &&
          (mode >= 0 && mode <= 2) && (tile == 16 || tile == 32 || tile == 64) && group >= 1 &&
          group <= g->n_det && (wg == 4 || wg == 8 || wg == 16) && (rl == 16 || rl == 64)) {
        g->lanes_log2 = lanes;
        if (fo == 2) g->ensure_fwd_tiles(s);
        if (fo == 3) {
          g->ensure_fmat(s);
          if (g->fm_entries <= 0) fo = 0;  // not buildable here: the gather
        }
        g->fwd_path = fo;
        g->fwd_sym = fsym != 0;
        g->tile = tile;
        g->det_group = group;
        if (mode != 0) g->ensure_csr(s);
        g->adj_mode = mode;
        g->csr_waves = wg;
        g->csr_lanes = rl;
        res.forward_ms = tf;
        res.adjoint_ms = ta;
        res.from_cache = 1;
        applied = true;
      }
    }
    if (!applied) {
      if (g->dtype == PAT_F64) pat::tune<double>(g, reps, s, &res);
      else pat::tune<float>(g, reps, s, &res);
      char buf[128];
      std::snprintf(buf, sizeof(buf), "%d %d %d %d %d %d %d %d %.6f %.6f", g->lanes_log2, g->fwd_path,
                    g->fwd_sym ? 1 : 0, g->adj_mode, g->tile, g->det_group, g->csr_waves, g->csr_lanes,
                    res.forward_ms, res.adjoint_ms);
      cache[key] = buf;
      pat::write_cache(cache_path, cache);
    }
    res.fwd_lanes_log2 = g->lanes_log2;
    res.adj_mode = g->adj_mode;
    res.adj_tile = g->tile;
    res.adj_det_group = g->det_group;
    if (out) *out = res;
    return PAT_OK;
  });
}
