// Circular-mean projector A and its exact transpose on gfx950
// (arXiv:1707.02245, Sec. 4.1 eq. K_def; Sec. 3.3.1: K applied as a matrix,
// its transpose as the adjoint).
//
// Forward (bin-major gather): a group of 16..64 lanes owns one bin (d, k) and
// walks the arc samples inside the bin's clip windows; each sample reads the
// 2x2 neighbourhood of a zero-bordered copy of the image (L1/L2 resident)
// and adds the bilinear weights times the values. The group sum times 1/M_k
// is the bin's value; epilogues fuse the dual data step of PDHGM, the gap
// terms or the row sums of the preconditioner.
//
// Adjoint (tile scatter): a workgroup owns a square pixel tile and a group of
// detectors; each wave walks, for its detectors, the radii whose circles meet
// the tile and the arc samples in the tile's angular window, and adds weight
// times data into a private LDS accumulator (tile plus one-pixel halo). The
// four waves' accumulators are summed in a fixed order and written as one
// partial image per detector group; partials are summed in a fixed order by
// the consumer. Positions and weights use the same FP64 formula as the
// forward, so the two are transposes of the same matrix, and the result is
// run-to-run deterministic (one wave per accumulator, no cross-wave atomics).

#include "pat_internal.hpp"
#include "reg_dual.hpp"
#include "fwd_epilogue.hpp"

namespace pat {

constexpr double kTwoPiD = 6.283185307179586476925286766559;

__device__ __forceinline__ int find_inst(const int* __restrict__ starts, int n, int blk) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (starts[mid] <= blk) lo = mid; else hi = mid;
  }
  return lo;
}

// Position of arc sample (d, k, m) in pixel-index units and its bilinear cell.
struct Sample {
  int ix, iy;
  double tx, ty;
};

__device__ __forceinline__ Sample arc_sample(const double2 p, const double rho, const double2 cs) {
  const double gx = fma(rho, cs.x, p.x);
  const double gy = fma(rho, cs.y, p.y);
  const double fx = floor(gx), fy = floor(gy);
  Sample s;
  s.ix = (int)fx;
  s.iy = (int)fy;
  s.tx = gx - fx;
  s.ty = gy - fy;
  return s;
}

// ------------------------------------------------------------------ padding

template <class T>
__global__ __launch_bounds__(256) void pad_kernel(const T* __restrict__ u, T* __restrict__ upad,
                                                  int nx, int ny) {
  const int P = nx + 2;
  const int64_t n = (int64_t)P * (ny + 2);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % P) - 1, y = (int)(i / P) - 1;
    upad[i] = (x >= 0 && x < nx && y >= 0 && y < ny) ? u[(int64_t)y * nx + x] : T(0);
  }
}

template <class T>
void launch_pad(const T* u, T* upad, int nx, int ny, hipStream_t s) {
  const int64_t n = (int64_t)(nx + 2) * (ny + 2);
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(pad_kernel<T>, dim3(blocks), dim3(256), 0, s, u, upad, nx, ny);
  PAT_HIP(hipGetLastError());
}

// Padded copies of an n x n image for the quarter-turn forward: slot t (at
// dst + t (n+2)^2) holds the padded image turned by t quarter turns, slot_t(x,
// y) = upad(R^t (x, y)) on the (n+2) x (n+2) padded grid (the border maps to
// the border). src is the image [n][n] or, with src_padded, its padded copy.
template <class T>
__global__ __launch_bounds__(256) void rot_pad_kernel(const T* __restrict__ src, int src_padded,
                                                      T* __restrict__ dst, int n, int slots) {
  const int P = n + 2;
  const int64_t np = (int64_t)P * P;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < np * slots;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(idx / np);
    const int64_t q = idx - t * np;
    int a, b;
    quarter_turn_xy((int)(q % P), (int)(q / P), P, t, a, b);
    T v;
    if (src_padded) {
      v = src[(int64_t)b * P + a];
    } else {
      const int i = a - 1, j = b - 1;
      v = (i >= 0 && i < n && j >= 0 && j < n) ? src[(int64_t)j * n + i] : T(0);
    }
    dst[idx] = v;
  }
}

template <class T>
void launch_rot_pad(const T* src, bool src_padded, T* dst, int n, int slots, hipStream_t s) {
  const int64_t total = (int64_t)(n + 2) * (n + 2) * slots;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(rot_pad_kernel<T>, dim3(blocks), dim3(256), 0, s, src, src_padded ? 1 : 0, dst, n, slots);
  PAT_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ forward

// With FUSED the launch also carries the regulariser's dual step, which reads
// the same extrapolated image as the forward's dual data step and writes
// disjoint state: blocks from n_fwd on run it (so filling the forward's last
// wave of blocks) and the blocks before them the forward. With NI > 1 arr
// holds groups of NI slots, each group's instances on one geometry (slots
// after the group's last instance have no image), and starts the groups'
// block offsets: each block serves a whole group, a sample's table entry,
// position and cell computed once and its 2x2 taps read from each
// instance's image. On a quarter-turn symmetric geometry the bins of detector
// d + t n_det/4 are those of detector d on the image turned by t quarter
// turns, so a group's slots can also be the four turned images of one
// instance over the first n_det/4 detectors (the solvers build such slot
// arrays); with QT (NI = 4) a0 alone describes the four slots (its slot
// fields), the form of the stand-alone forward.
template <class T, int MODE, int LANES, bool FUSED = false, int NI = 1, bool QT = false>
__global__ __launch_bounds__(256) void fwd_kernel(FwdArgs<T> a0, const FwdArgs<T>* __restrict__ arr,
                                                  const int* __restrict__ starts, int n_inst, int n_fwd,
                                                  const InstDev<T>* __restrict__ rarr,
                                                  const int* __restrict__ rstarts, int rn) {
  int blk = blockIdx.x;
  if constexpr (FUSED) {
    if (blk >= n_fwd) {
      reg_dual_block<T>(rarr, rstarts, rn, blk - n_fwd);
      return;
    }
  }
  FwdArgs<T> a;
  int cnt = 1;  // instances in this block's group
  if constexpr (QT) {
    static_assert(NI == 4, "quarter-turn slots come in fours");
    a = a0;
    cnt = NI;
  } else if constexpr (NI > 1) {
    const int gi = find_inst(starts, n_inst, blk);
    arr += (int64_t)NI * gi;
    blk -= starts[gi];
    a = arr[0];
#pragma unroll
    for (int i = 1; i < NI; ++i) cnt += arr[i].upad != nullptr;
  } else if (arr) {
    const int i = find_inst(starts, n_inst, blk);
    a = arr[i];
    blk -= starts[i];
  } else {
    a = a0;
  }
  const GeomDev& g = a.g;
  constexpr int BPB = 256 / LANES;
  const int sub = threadIdx.x / LANES, lane = threadIdx.x % LANES;
  // radius-major order: a block takes one radius for BPB detectors (the
  // radius' (cos, sin) table is shared); detector-major: BPB consecutive
  // radii of one detector, concentric arcs whose samples at similar angles
  // share cache lines
  int k, d;
  if (g.fwd_path == 1) {
    const int n_kg = (g.n_t + BPB - 1) / BPB;
    d = blk / n_kg;
    k = (blk - d * n_kg) * BPB + sub;
  } else {
    const int n_dg = (g.n_det + BPB - 1) / BPB;
    k = blk / n_dg;
    d = (blk - k * n_dg) * BPB + sub;
    if (g.kord) k = g.kord[k];
  }
  const bool valid = d < g.n_det && k < g.n_t;
  const int b = d * g.n_t + k;
  T acc[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) acc[i] = T(0);
  double inv_m = 0.0;
  if (valid) {
    const int4 w0 = g.win[2 * (int64_t)b], w1 = g.win[2 * (int64_t)b + 1];
    const double2 p = g.det[d];
    const double2 rr = g.rad[k];
    inv_m = rr.y;
    const int toff = g.moff[k].y;
    gptr<const char> ub[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i)
      ub[i] = as_global(reinterpret_cast<const char*>(QT ? a.upad + i * a.slot_img : (NI > 1 ? arr[i].upad : a.upad)));
    const int P = g.pitch;
    const unsigned rowb = (unsigned)P * (unsigned)sizeof(T);
    const int nx = g.nx, ny = g.ny;
    // Bilinear value of one arc sample from its 2x2 cell, as three linear
    // interpolations (the same function as the weight products). Branch free:
    // a sample whose cell is not inside the padded grid reads the cell at
    // offset P - 1 instead (last border column of row 0 and, wrapping, the
    // first border column of rows 1 and 2: all four taps are zero), so the
    // loads of both samples in flight issue together.
    auto tap = [&](const double2 cs, T* t) {
      const Sample s = arc_sample(p, rr.x, cs);
      const bool in = ((unsigned)(s.ix + 1) <= (unsigned)nx) & ((unsigned)(s.iy + 1) <= (unsigned)ny);
      const int o = in ? (int)__umul24((unsigned)(s.iy + 1), (unsigned)P) + (s.ix + 1) : P - 1;
      const T tx = (T)s.tx, ty = (T)s.ty;
      // 32-bit byte offsets from the uniform base (the padded image is far
      // below 4 GB): scalar-base loads without 64-bit address arithmetic
      const unsigned off = (unsigned)o * (unsigned)sizeof(T);
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        if (NI > 1 && !QT && i >= cnt) {
          t[i] = T(0);
          continue;
        }
        const gptr<const T> q0 = (gptr<const T>)(ub[i] + off), q1 = (gptr<const T>)(ub[i] + (off + rowb));
        const T q00 = q0[0], q10 = q0[1], q01 = q1[0], q11 = q1[1];
        const T lo = fma(tx, q10 - q00, q00);
        const T hi = fma(tx, q11 - q01, q01);
        t[i] = fma(ty, hi - lo, lo);
      }
    };
    const int rng[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m1 = rng[2 * r + 1];
      int m = rng[2 * r] + lane;
      // two samples per lane in flight
      for (; m + LANES < m1; m += 2 * LANES) {
        const double2 c0 = table_cs<T>(g, toff + m), c1 = table_cs<T>(g, toff + m + LANES);
        T t0[NI], t1[NI];
        tap(c0, t0);
        tap(c1, t1);
#pragma unroll
        for (int i = 0; i < NI; ++i) acc[i] += t0[i] + t1[i];
      }
      if (m < m1) {
        T t0[NI];
        tap(table_cs<T>(g, toff + m), t0);
#pragma unroll
        for (int i = 0; i < NI; ++i) acc[i] += t0[i];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NI; ++i) acc[i] = group_sum<LANES>(acc[i]);
  if constexpr (QT) {
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      FwdArgs<T> ai = a;
      const int64_t ob = i * a.slot_bins;
      if (ai.out) ai.out += ob;
      if (ai.f) ai.f += ob;
      if (ai.sigma) ai.sigma += ob;
      if (ai.q) ai.q += ob;
      if (ai.red) ai.red += i * a.slot_red;
      fwd_epilogue<T, MODE>(ai, blk, valid && lane == 0, b, acc[i] * (T)inv_m);
    }
  } else if constexpr (NI == 1) {
    fwd_epilogue<T, MODE>(a, blk, valid && lane == 0, b, acc[0] * (T)inv_m);
  } else {
#pragma unroll
    for (int i = 0; i < NI; ++i)
      if (i < cnt) fwd_epilogue<T, MODE>(arr[i], blk, valid && lane == 0, b, acc[i] * (T)inv_m);
  }
}

// LDS-tiled forward, gather pass: a workgroup stages tile cells [x0, x0 +
// TS] x [y0, y0 + TS] of the padded image in LDS and sums, 16 lanes per pair,
// the samples of its pairs whose cell lies in the tile; each pair's sum goes
// to its partial slot. A group of 16 lanes works on four pairs at once (their
// record, detector, radius and table loads issue together) so that the short
// per-pair chains of dependent loads overlap.
template <class T, int NT>
__global__ __launch_bounds__(NT) void fwd_tiled_kernel(FwdArgs<T> a0, const FwdArgs<T>* __restrict__ arr,
                                                       const int* __restrict__ starts, int n_inst) {
  constexpr int TS = kFwdTile, W = TS + 1, NG = NT / 16, J = 4;
  __shared__ T tile[W * W];
  int blk = blockIdx.x;
  const FwdArgs<T>* ap = &a0;
  if (arr) {
    const int i = find_inst(starts, n_inst, blk);
    ap = arr + i;
    blk -= starts[i];
  }
  const FwdArgs<T>& a = *ap;
  const GeomDev& g = a.g;
  const int4 bd = g.fblock[blk];
  const int x0 = bd.x, y0 = bd.y;
  const int P = g.pitch, PR = g.ny + 2;
  const gptr<const T> up = as_global(a.upad);
  for (int i = threadIdx.x; i < W * W; i += NT) {
    const int r = i / W, c = i - r * W;
    const int px = x0 + c, py = y0 + r;
    tile[i] = (px < P && py < PR) ? up[(int64_t)py * P + px] : T(0);
  }
  __syncthreads();
  const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15;
  const int4* __restrict__ pairs = g.fpair;
  for (int q0 = bd.z + grp; q0 < bd.w; q0 += J * NG) {
    int m0[J], len[J], slot[J], toff[J];
    double2 p[J];
    double rho[J];
    int bins[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int q = q0 + j * NG;
      int4 pr = make_int4(0, 0, 0, -1);
      if (q < bd.w) pr = pairs[q];
      bins[j] = pr.x;
      m0[j] = pr.y;
      len[j] = pr.z - pr.y;
      slot[j] = pr.w;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int d = bins[j] / g.n_t, k = bins[j] - d * g.n_t;
      p[j] = g.det[d];
      rho[j] = g.rad[k].x;
      toff[j] = g.moff[k].y + m0[j];
    }
    const int cnt = max(max(len[0], len[1]), max(len[2], len[3]));
    T acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = T(0);
    for (int s = gl; s < cnt; s += 16) {
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const bool live = s < len[j];
        const Sample sm = arc_sample(p[j], rho[j], table_cs<T>(g, live ? toff[j] + s : 0));
        const int cx = sm.ix + 1 - x0, cy = sm.iy + 1 - y0;
        const bool in = live & ((unsigned)cx < (unsigned)TS) & ((unsigned)cy < (unsigned)TS);
        const int o = in ? cy * W + cx : 0;
        const T tx = (T)sm.tx, ty = (T)sm.ty;
        const T q00 = tile[o], q10 = tile[o + 1], q01 = tile[o + W], q11 = tile[o + W + 1];
        const T lo = fma(tx, q10 - q00, q00);
        const T hi = fma(tx, q11 - q01, q01);
        acc[j] += in ? fma(ty, hi - lo, lo) : T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const T sum = row16_sum(acc[j]);
      if (gl == 0 && slot[j] >= 0) a.part[slot[j]] = sum;
    }
  }
}

// LDS-tiled forward, per-bin pass: the bin's partial sums in slot order,
// times 1/M_k, into the epilogue.
template <class T, int MODE>
__global__ __launch_bounds__(256) void fwd_reduce_kernel(FwdArgs<T> a0, const FwdArgs<T>* __restrict__ arr,
                                                         const int* __restrict__ starts, int n_inst) {
  int blk = blockIdx.x;
  const FwdArgs<T>* ap = &a0;
  if (arr) {
    const int i = find_inst(starts, n_inst, blk);
    ap = arr + i;
    blk -= starts[i];
  }
  const FwdArgs<T>& a = *ap;
  const GeomDev& g = a.g;
  const int64_t nb = (int64_t)g.n_det * g.n_t;
  const int64_t b = (int64_t)blk * 256 + threadIdx.x;
  const bool valid = b < nb;
  T val = T(0);
  if (valid) {
    T acc = T(0);
    const int s1 = g.fbin_off[b + 1];
    for (int s = g.fbin_off[b]; s < s1; ++s) acc += a.part[s];
    val = acc * (T)g.rad[b % g.n_t].y;
  }
  fwd_epilogue<T, MODE>(a, blk, valid, b, val);
}

template <class T, int MODE>
static void fwd_dispatch(int lanes_log2, int blocks, const FwdArgs<T>& a0, const FwdArgs<T>* arr,
                         const int* starts, int n, hipStream_t s) {
  switch (lanes_log2) {
    case 4: hipLaunchKernelGGL((fwd_kernel<T, MODE, 16>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n, blocks,
                         nullptr, nullptr, 0); break;
    case 5: hipLaunchKernelGGL((fwd_kernel<T, MODE, 32>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n, blocks,
                         nullptr, nullptr, 0); break;
    default: hipLaunchKernelGGL((fwd_kernel<T, MODE, 64>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n, blocks,
                         nullptr, nullptr, 0); break;
  }
}

template <class T>
static void fwd_mode_dispatch(int mode, int lanes_log2, int blocks, const FwdArgs<T>& a0,
                              const FwdArgs<T>* arr, const int* starts, int n, hipStream_t s) {
  if (blocks <= 0) return;
  switch (mode) {
    case FWD_PLAIN: fwd_dispatch<T, FWD_PLAIN>(lanes_log2, blocks, a0, arr, starts, n, s); break;
    case FWD_DUAL: fwd_dispatch<T, FWD_DUAL>(lanes_log2, blocks, a0, arr, starts, n, s); break;
    case FWD_GAP: fwd_dispatch<T, FWD_GAP>(lanes_log2, blocks, a0, arr, starts, n, s); break;
    default: fwd_dispatch<T, FWD_ROWSUM>(lanes_log2, blocks, a0, arr, starts, n, s); break;
  }
  PAT_HIP(hipGetLastError());
}

template <class T>
static void reduce_mode_dispatch(int mode, int blocks, const FwdArgs<T>& a0, const FwdArgs<T>* arr,
                                 const int* starts, int n, hipStream_t s) {
  if (blocks <= 0) return;
  switch (mode) {
    case FWD_PLAIN: hipLaunchKernelGGL((fwd_reduce_kernel<T, FWD_PLAIN>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n); break;
    case FWD_DUAL: hipLaunchKernelGGL((fwd_reduce_kernel<T, FWD_DUAL>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n); break;
    case FWD_GAP: hipLaunchKernelGGL((fwd_reduce_kernel<T, FWD_GAP>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n); break;
    default: hipLaunchKernelGGL((fwd_reduce_kernel<T, FWD_ROWSUM>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n); break;
  }
  PAT_HIP(hipGetLastError());
}

template <class T>
void launch_forward(int mode, const FwdArgs<T>& a, int lanes_log2, hipStream_t s) {
  const int blocks = fwd_grid(a.g.n_det, a.g.n_t, lanes_log2, a.g.fwd_path);
  if (a.g.fwd_path == 2) {
    PAT_CHECK_ARG(a.g.fpair != nullptr && a.part != nullptr, "tiled forward without its tables");
    if (a.g.n_fblocks > 0)
      hipLaunchKernelGGL((fwd_tiled_kernel<T, kFwdTileThreads>), dim3(a.g.n_fblocks), dim3(kFwdTileThreads), 0, s, a,
                         (const FwdArgs<T>*)nullptr, (const int*)nullptr, 1);
    PAT_HIP(hipGetLastError());
    reduce_mode_dispatch<T>(mode, blocks, a, nullptr, nullptr, 1, s);
    return;
  }
  fwd_mode_dispatch<T>(mode, lanes_log2, blocks, a, nullptr, nullptr, 1, s);
}

// Stand-alone forward in quarter-turn form: a.g holds a quarter of the
// detectors and the slot fields of a locate the turned images and the other
// quarters' bins (the solvers use the slot-array form of the NI = 4 gather).
template <class T>
void launch_forward_qt(int mode, const FwdArgs<T>& a, int lanes_log2, hipStream_t s) {
  PAT_CHECK_ARG(mode == FWD_PLAIN, "quarter-turn stand-alone forward: plain mode only");
  const int blocks = fwd_grid(a.g.n_det, a.g.n_t, lanes_log2, a.g.fwd_path);
  if (blocks <= 0) return;
  const FwdArgs<T>* none = nullptr;
  switch (lanes_log2) {
    case 4:
      hipLaunchKernelGGL((fwd_kernel<T, FWD_PLAIN, 16, false, 4, true>), dim3(blocks), dim3(256), 0, s, a, none,
                         nullptr, 1, blocks, nullptr, nullptr, 0);
      break;
    case 5:
      hipLaunchKernelGGL((fwd_kernel<T, FWD_PLAIN, 32, false, 4, true>), dim3(blocks), dim3(256), 0, s, a, none,
                         nullptr, 1, blocks, nullptr, nullptr, 0);
      break;
    default:
      hipLaunchKernelGGL((fwd_kernel<T, FWD_PLAIN, 64, false, 4, true>), dim3(blocks), dim3(256), 0, s, a, none,
                         nullptr, 1, blocks, nullptr, nullptr, 0);
      break;
  }
  PAT_HIP(hipGetLastError());
}

// Instances grouped by geometry: every block serves a group of up to NI; with
// FUSED the regulariser's dual step of all instances follows in extra blocks
template <class T, int MODE, bool FUSED, int NI>
static void fwd_ni_launch(int lanes_log2, const Launch<T>& L, const FwdArgs<T>* arr, hipStream_t s) {
  const int* gs = ptr<int>(L.fwdg_start);
  const int ng = L.fwd_ni_groups;
  const int n_fwd = L.fwd_ni_blocks;
  const dim3 grid((unsigned)(n_fwd + (FUSED ? L.pix_total : 0)));
  const InstDev<T>* ra = FUSED ? ptr<InstDev<T>>(L.inst) : nullptr;
  const int* rs = FUSED ? ptr<int>(L.pix_start) : nullptr;
  const int rn = FUSED ? L.n : 0;
  switch (lanes_log2) {
    case 4:
      hipLaunchKernelGGL((fwd_kernel<T, MODE, 16, FUSED, NI>), grid, dim3(256), 0, s, FwdArgs<T>{}, arr, gs, ng,
                         n_fwd, ra, rs, rn);
      break;
    case 5:
      hipLaunchKernelGGL((fwd_kernel<T, MODE, 32, FUSED, NI>), grid, dim3(256), 0, s, FwdArgs<T>{}, arr, gs, ng,
                         n_fwd, ra, rs, rn);
      break;
    default:
      hipLaunchKernelGGL((fwd_kernel<T, MODE, 64, FUSED, NI>), grid, dim3(256), 0, s, FwdArgs<T>{}, arr, gs, ng,
                         n_fwd, ra, rs, rn);
      break;
  }
  PAT_HIP(hipGetLastError());
}

template <class T, int MODE, bool FUSED>
static void fwd_ni_dispatch(int lanes_log2, const Launch<T>& L, hipStream_t s) {
  const FwdArgs<T>* arr = ptr<FwdArgs<T>>(L.fwdg);
  if (L.fwd_ni == 2) fwd_ni_launch<T, MODE, FUSED, 2>(lanes_log2, L, arr, s);
  else if (L.fwd_ni == 3) fwd_ni_launch<T, MODE, FUSED, 3>(lanes_log2, L, arr, s);
  else fwd_ni_launch<T, MODE, FUSED, 4>(lanes_log2, L, arr, s);
}

template <class T>
static void launch_gather_batched(int mode, const Launch<T>& L, int lanes_log2, hipStream_t s);

template <class T>
void launch_forward_reg_batched(const Launch<T>& L, int lanes_log2, hipStream_t s) {
  if (L.fm_n > 0) {
    // the gather instances without the regulariser, which runs in the stored
    // forward's tile pass
    launch_gather_batched<T>(FWD_DUAL, L, lanes_log2, s);
    launch_fmat_batched<T>(FWD_DUAL, true, L, s);
    return;
  }
  if (!L.fwd_tiled && L.fwd_ni > 1 && L.fwd_ni_blocks > 0 && L.pix_total > 0) {
    fwd_ni_dispatch<T, FWD_DUAL, true>(lanes_log2, L, s);
    return;
  }
  if (L.fwd_tiled || L.fwd_total <= 0 || L.pix_total <= 0) {
    launch_forward_batched<T>(FWD_DUAL, L, lanes_log2, s);
    launch_reg_dual<T>(L, s);
    return;
  }
  const dim3 grid((unsigned)(L.fwd_total + L.pix_total));
  const FwdArgs<T>* fa = ptr<FwdArgs<T>>(L.fwd);
  const InstDev<T>* ra = ptr<InstDev<T>>(L.inst);
  switch (lanes_log2) {
    case 4:
      hipLaunchKernelGGL((fwd_kernel<T, FWD_DUAL, 16, true>), grid, dim3(256), 0, s, FwdArgs<T>{}, fa,
                         ptr<int>(L.fwd_start), L.n, L.fwd_total, ra, ptr<int>(L.pix_start), L.n);
      break;
    case 5:
      hipLaunchKernelGGL((fwd_kernel<T, FWD_DUAL, 32, true>), grid, dim3(256), 0, s, FwdArgs<T>{}, fa,
                         ptr<int>(L.fwd_start), L.n, L.fwd_total, ra, ptr<int>(L.pix_start), L.n);
      break;
    default:
      hipLaunchKernelGGL((fwd_kernel<T, FWD_DUAL, 64, true>), grid, dim3(256), 0, s, FwdArgs<T>{}, fa,
                         ptr<int>(L.fwd_start), L.n, L.fwd_total, ra, ptr<int>(L.pix_start), L.n);
      break;
  }
  PAT_HIP(hipGetLastError());
}

template <class T>
void launch_forward_batched(int mode, const Launch<T>& L, int lanes_log2, hipStream_t s) {
  launch_gather_batched<T>(mode, L, lanes_log2, s);
  if (L.fm_n > 0) launch_fmat_batched<T>(mode, false, L, s);
}

template <class T>
static void launch_gather_batched(int mode, const Launch<T>& L, int lanes_log2, hipStream_t s) {
  if (!L.fwd_tiled && L.fwd_ni > 1 && L.fwd_ni_blocks > 0 && (mode == FWD_DUAL || mode == FWD_GAP)) {
    if (mode == FWD_DUAL) fwd_ni_dispatch<T, FWD_DUAL, false>(lanes_log2, L, s);
    else fwd_ni_dispatch<T, FWD_GAP, false>(lanes_log2, L, s);
    return;
  }
  FwdArgs<T> dummy{};
  if (L.fwd_tiled) {
    if (L.fwdt_total > 0)
      hipLaunchKernelGGL((fwd_tiled_kernel<T, kFwdTileThreads>), dim3(L.fwdt_total), dim3(kFwdTileThreads), 0, s, dummy,
                         ptr<FwdArgs<T>>(L.fwd), ptr<int>(L.fwdt_start), L.n);
    PAT_HIP(hipGetLastError());
    reduce_mode_dispatch<T>(mode, L.fwd_total, dummy, ptr<FwdArgs<T>>(L.fwd), ptr<int>(L.fwd_start), L.n, s);
    return;
  }
  fwd_mode_dispatch<T>(mode, lanes_log2, L.fwd_total, dummy, ptr<FwdArgs<T>>(L.fwd),
                       ptr<int>(L.fwd_start), L.n, s);
}

// ------------------------------------------------------------------ adjoint

template <class T, int TILE>
__global__ __launch_bounds__(256) void adj_kernel(AdjArgs<T> a0, const AdjArgs<T>* __restrict__ arr,
                                                  const int* __restrict__ starts, int n_inst) {
  constexpr int S = TILE + 2;  // tile plus a one-pixel halo on each side
  __shared__ T acc[4 * S * S];
  int blk = blockIdx.x;
  AdjArgs<T> a;
  if (arr) {
    const int i = find_inst(starts, n_inst, blk);
    a = arr[i];
    blk -= starts[i];
  } else {
    a = a0;
  }
  const GeomDev& g = a.g;
  const int n_tiles = g.tiles_x * g.tiles_y;
  const int grp = blk / n_tiles, t = blk - grp * n_tiles;
  const int I0 = (t % g.tiles_x) * TILE, J0 = (t / g.tiles_x) * TILE;
  for (int i = threadIdx.x; i < 4 * S * S; i += 256) acc[i] = T(0);
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  T* __restrict__ my = acc + wave * S * S;
  // samples whose cell (ix, iy) lies in [I0-1, I0+TILE-1] x [J0-1, J0+TILE-1]
  // touch the tile; their positions lie in this closed box
  const double bx0 = I0 - 1.0, bx1 = I0 + (double)TILE, by0 = J0 - 1.0, by1 = J0 + (double)TILE;
  const int d_begin = grp * g.det_group;
  const int d_end = min(g.n_det, d_begin + g.det_group);
  for (int d = d_begin + wave; d < d_end; d += 4) {
    const double2 p = g.det[d];
    const double ex = fmax(fmax(bx0 - p.x, 0.0), p.x - bx1);
    const double ey = fmax(fmax(by0 - p.y, 0.0), p.y - by1);
    const double rmin = sqrt(ex * ex + ey * ey);
    const double cx0 = bx0 - p.x, cx1 = bx1 - p.x, cy0 = by0 - p.y, cy1 = by1 - p.y;
    const double rmax = sqrt(fmax(cx0 * cx0, cx1 * cx1) + fmax(cy0 * cy0, cy1 * cy1));
    const int k0 = max(0, (int)floor(rmin * g.kscale - g.koff) - 1);
    const int k1 = min(g.n_t - 1, (int)ceil(rmax * g.kscale - g.koff) + 1);
    // angular window of the box seen from the detector; the whole circle when
    // the detector is within two pixels of the box
    const bool full = rmin < 2.0;
    double a_lo = 0.0, a_hi = 0.0;
    if (!full) {
      const double pc = atan2(0.5 * (cy0 + cy1), 0.5 * (cx0 + cx1));
      double dmin = 0.0, dmax = 0.0;
      const double cxs[2] = {cx0, cx1}, cys[2] = {cy0, cy1};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double dd = atan2(cys[c >> 1], cxs[c & 1]) - pc;
        dd -= kTwoPiD * rint(dd / kTwoPiD);
        dmin = fmin(dmin, dd);
        dmax = fmax(dmax, dd);
      }
      a_lo = pc + dmin - 1e-9;
      a_hi = pc + dmax + 1e-9;
    }
    for (int k = k0; k <= k1; ++k) {
      const T gk = a.data[(int64_t)d * g.n_t + k];
      if (gk == T(0)) continue;
      const int2 mo = g.moff[k];
      const double2 rr = g.rad[k];
      const int M = mo.x;
      int mlo = 0, cnt = M;
      if (!full) {
        mlo = (int)floor(a_lo * M / kTwoPiD - 0.5) - 1;
        const int mhi = (int)ceil(a_hi * M / kTwoPiD - 0.5) + 1;
        cnt = min(M, mhi - mlo + 1);
        mlo %= M;
        if (mlo < 0) mlo += M;
      }
      const T gw = gk * (T)rr.y;
      for (int j = lane; j < cnt; j += 64) {
        int m = mlo + j;
        if (m >= M) m -= M;
        const Sample s = arc_sample(p, rr.x, table_cs<T>(g, mo.y + m));
        const int lx = s.ix - (I0 - 1), ly = s.iy - (J0 - 1);
        if ((unsigned)lx <= (unsigned)TILE && (unsigned)ly <= (unsigned)TILE) {
          const T tx = (T)s.tx, ty = (T)s.ty;
          const T w00 = (T(1) - tx) * (T(1) - ty), w10 = tx * (T(1) - ty);
          const T w01 = (T(1) - tx) * ty, w11 = tx * ty;
          T* c = my + ly * S + lx;
          atomicAdd(c, gw * w00);
          atomicAdd(c + 1, gw * w10);
          atomicAdd(c + S, gw * w01);
          atomicAdd(c + S + 1, gw * w11);
        }
      }
    }
  }
  __syncthreads();
  const int64_t N = (int64_t)g.nx * g.ny;
  T* __restrict__ out = a.part + grp * N;
  for (int idx = threadIdx.x; idx < TILE * TILE; idx += 256) {
    const int i = idx % TILE, j = idx / TILE;
    const int X = I0 + i, Y = J0 + j;
    if (X < g.nx && Y < g.ny) {
      const int l = (j + 1) * S + (i + 1);
      out[(int64_t)Y * g.nx + X] = ((acc[l] + acc[S * S + l]) + acc[2 * S * S + l]) + acc[3 * S * S + l];
    }
  }
}

template <class T>
static void adj_dispatch(int tile, int blocks, const AdjArgs<T>& a0, const AdjArgs<T>* arr,
                         const int* starts, int n, hipStream_t s) {
  if (blocks <= 0) return;
  switch (tile) {
    case 16: hipLaunchKernelGGL((adj_kernel<T, 16>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n); break;
    case 64:
      if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL((adj_kernel<T, 64>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n);
        break;
      }
      [[fallthrough]];
    default: hipLaunchKernelGGL((adj_kernel<T, 32>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n); break;
  }
  PAT_HIP(hipGetLastError());
}

template <class T>
void launch_adjoint(const AdjArgs<T>& a, hipStream_t s) {
  const int blocks = a.g.tiles_x * a.g.tiles_y * a.g.n_groups;
  adj_dispatch<T>(a.g.tile, blocks, a, nullptr, nullptr, 1, s);
}

template <class T>
void launch_adjoint_batched(const Launch<T>& L, hipStream_t s) {
  AdjArgs<T> dummy{};
  adj_dispatch<T>(L.max_tile, L.adj_total, dummy, ptr<AdjArgs<T>>(L.adj),
                  ptr<int>(L.adj_start), L.n_adj, s);
}

template <class T>
__global__ __launch_bounds__(256) void reduce_groups_kernel(const T* __restrict__ part,
                                                            T* __restrict__ out, int n_groups,
                                                            int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    T s = T(0);
    for (int gi = 0; gi < n_groups; ++gi) s += part[gi * n + i];
    out[i] = s;
  }
}

template <class T>
void launch_reduce_groups(const T* part, T* out, int n_groups, int64_t n, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(reduce_groups_kernel<T>, dim3(blocks), dim3(256), 0, s, part, out, n_groups, n);
  PAT_HIP(hipGetLastError());
}

#define PAT_INST_PROJ(T)                                                                    \
  template void launch_pad<T>(const T*, T*, int, int, hipStream_t);                         \
  template void launch_rot_pad<T>(const T*, bool, T*, int, int, hipStream_t);               \
  template void launch_forward_qt<T>(int, const FwdArgs<T>&, int, hipStream_t);             \
  template void launch_forward<T>(int, const FwdArgs<T>&, int, hipStream_t);                \
  template void launch_forward_batched<T>(int, const Launch<T>&, int, hipStream_t);        \
  template void launch_forward_reg_batched<T>(const Launch<T>&, int, hipStream_t);          \
  template void launch_adjoint<T>(const AdjArgs<T>&, hipStream_t);                          \
  template void launch_adjoint_batched<T>(const Launch<T>&, hipStream_t);                   \
  template void launch_reduce_groups<T>(const T*, T*, int, int64_t, hipStream_t);
PAT_INST_PROJ(float)
PAT_INST_PROJ(double)

}  // namespace pat

// ------------------------------------------------------------------ geometry view + C ABI

pat::GeomDev pat_geometry_s::dev() const {
  pat::GeomDev g{};
  g.nx = nx;
  g.ny = ny;
  g.n_det = n_det;
  g.n_t = n_t;
  g.pitch = nx + 2;
  g.det = pat::ptr<double2>(d_det);
  g.rad = pat::ptr<double2>(d_rad);
  g.moff = pat::ptr<int2>(d_moff);
  g.cs = d_cs.p;
  g.win = pat::ptr<int4>(d_win);
  g.kord = pat::ptr<int>(d_kord);
  g.kscale = h / (desc.c * desc.dt);
  g.koff = desc.t0 / desc.dt;
  g.lanes_log2 = lanes_log2;
  g.fwd_path = fwd_path;
  g.fpair = fwd_n_pairs >= 0 ? pat::ptr<int4>(fwd_pair) : nullptr;
  g.fblock = fwd_n_pairs >= 0 ? pat::ptr<int4>(fwd_block) : nullptr;
  g.fbin_off = fwd_n_pairs >= 0 ? pat::ptr<int>(fwd_bin_off) : nullptr;
  g.n_fblocks = fwd_n_blocks;
  g.tile = (dtype == PAT_F64 && tile == 64) ? 32 : tile;
  g.tiles_x = (nx + g.tile - 1) / g.tile;
  g.tiles_y = (ny + g.tile - 1) / g.tile;
  g.det_group = det_group;
  g.n_groups = n_groups();
  const bool fm = fm_entries > 0;
  g.fm_off = fm ? pat::ptr<uint8_t>(fm_off) : nullptr;
  g.fm_w = fm ? fm_w.p : nullptr;
  g.fm_seg = fm ? pat::ptr<int4>(fm_seg) : nullptr;
  g.fm_chunk = fm ? pat::ptr<int4>(fm_chunk) : nullptr;
  g.fm_binseg = fm ? pat::ptr<int>(fm_binseg) : nullptr;
  g.fm_segidx = fm ? pat::ptr<int>(fm_segidx) : nullptr;
  g.fm_nseg = fm ? fm_nseg : 0;
  g.fm_tiles_x = fm_tiles_x;
  g.fm_nchunk = fm ? fm_nchunk : 0;
  return g;
}

void pat_geometry_s::ensure_fmat(hipStream_t s) {
  if (fm_entries >= 0) return;
  ensure_csr(s);
  if (dtype == PAT_F64) pat::build_fmat<double>(this, s);
  else pat::build_fmat<float>(this, s);
}

void pat_geometry_s::drop_fmat() {
  fm_off.release();
  fm_w.release();
  fm_seg.release();
  fm_chunk.release();
  fm_binseg.release();
  fm_segidx.release();
  fm_entries = -1;
  fm_nseg = fm_nchunk = fm_tiles_x = 0;
}

void pat_geometry_s::ensure_csr(hipStream_t s) {
  if (csr_nnz >= 0) return;
  if (dtype == PAT_F64) pat::build_csr_adjoint<double>(this, s);
  else pat::build_csr_adjoint<float>(this, s);
  const size_t esz = dtype == PAT_F64 ? 8 : 4;
  csr_waves = pat::csr_waves_for(csr_side ? esz * (size_t)csr_win_max * csr_rot : 0, esz);
  csr_lanes = pat::csr_lanes_for(n_pix() > 0 ? (double)csr_nnz / (double)n_pix() : 0.0);
}

void pat_geometry_s::drop_csr() {
  drop_fmat();  // built from the CSR
  csr_ptr.release();
  csr_col.release();
  csr_val.release();
  csr_lcol.release();
  csr_win.release();
  csr_nnz = -1;
  csr_rot = 1;
  csr_side = csr_tiles_x = csr_tiles_y = csr_win_max = 0;
}

namespace {

// Quarter-turn form of a stand-alone forward: the four turned padded copies
// of the input in the geometry's scratch, then the gather over the first
// quarter of the detectors.
template <class T>
void forward_qt_impl(pat_geometry g, const T* src, bool src_padded, T* f, hipStream_t s) {
  const int64_t P = (int64_t)(g->nx + 2) * (g->ny + 2);
  g->scratch_pad.ensure(sizeof(T) * (size_t)(4 * P));
  T* slots = pat::ptr<T>(g->scratch_pad);
  pat::launch_rot_pad<T>(src, src_padded, slots, g->nx, 4, s);
  pat::FwdArgs<T> a{};
  a.g = g->dev();
  a.g.n_det = g->n_det / 4;
  a.upad = slots;
  a.out = f;
  a.slot_img = P;
  a.slot_bins = (int64_t)a.g.n_det * g->n_t;
  pat::launch_forward_qt<T>(pat::FWD_PLAIN, a, g->lanes_log2, s);
}

// The stored A by pixel tiles (path 3) from a padded image: four partials per
// segment in the geometry's scratch, then the per-bin pass.
template <class T>
void forward_fmat_impl(pat_geometry g, const T* upad, T* f, hipStream_t s) {
  PAT_CHECK_ARG(g->fm_entries > 0, "forward path 3 without its stored matrix");
  g->scratch_fpart.ensure(sizeof(T) * 4 * (size_t)std::max(g->fm_nseg, 1));
  pat::FwdArgs<T> a{};
  a.g = g->dev();
  a.g.n_det = g->n_det / 4;
  a.upad = upad;
  a.out = f;
  a.part = pat::ptr<T>(g->scratch_fpart);
  a.slot_bins = (int64_t)a.g.n_det * g->n_t;
  pat::launch_forward_fmat<T>(pat::FWD_PLAIN, a, s);
}

template <class T>
void forward_impl(pat_geometry g, const void* d_u, void* d_f, hipStream_t s) {
  if (g->fwd_path == 3) {
    g->scratch_pad.ensure(sizeof(T) * (size_t)(g->nx + 2) * (g->ny + 2));
    T* upad = pat::ptr<T>(g->scratch_pad);
    pat::launch_pad<T>(static_cast<const T*>(d_u), upad, g->nx, g->ny, s);
    forward_fmat_impl<T>(g, upad, static_cast<T*>(d_f), s);
    return;
  }
  if (g->fwd_qt()) {
    forward_qt_impl<T>(g, static_cast<const T*>(d_u), false, static_cast<T*>(d_f), s);
    return;
  }
  g->scratch_pad.ensure(sizeof(T) * (size_t)(g->nx + 2) * (g->ny + 2));
  T* upad = pat::ptr<T>(g->scratch_pad);
  pat::launch_pad<T>(static_cast<const T*>(d_u), upad, g->nx, g->ny, s);
  pat::FwdArgs<T> a{};
  a.g = g->dev();
  a.upad = upad;
  a.out = static_cast<T*>(d_f);
  pat::attach_fwd_part<T>(g, a);
  pat::launch_forward<T>(pat::FWD_PLAIN, a, g->lanes_log2, s);
}

}  // namespace

namespace pat {
// Partial-sum scratch of the tiled forward (path 2) for stand-alone applies.
template <class T>
void attach_fwd_part(pat_geometry g, FwdArgs<T>& a) {
  if (g->fwd_path != 2) return;
  g->scratch_fpart.ensure(sizeof(T) * (size_t)std::max<int64_t>(g->fwd_n_pairs, 1));
  a.part = ptr<T>(g->scratch_fpart);
}
template void attach_fwd_part<float>(pat_geometry, FwdArgs<float>&);
template void attach_fwd_part<double>(pat_geometry, FwdArgs<double>&);
}  // namespace pat

namespace {

template <class T>
void forward_padded_impl(pat_geometry g, const void* d_upad, void* d_f, hipStream_t s) {
  if (g->fwd_path == 3) {
    forward_fmat_impl<T>(g, static_cast<const T*>(d_upad), static_cast<T*>(d_f), s);
    return;
  }
  if (g->fwd_qt()) {
    forward_qt_impl<T>(g, static_cast<const T*>(d_upad), true, static_cast<T*>(d_f), s);
    return;
  }
  pat::FwdArgs<T> a{};
  a.g = g->dev();
  a.upad = static_cast<const T*>(d_upad);
  a.out = static_cast<T*>(d_f);
  pat::attach_fwd_part<T>(g, a);
  pat::launch_forward<T>(pat::FWD_PLAIN, a, g->lanes_log2, s);
}

// parts: csr_rot partial images (or null: sum into d_u). scratch: device
// memory for the partial images that are summed into d_u (at least
// pat::adjoint_scratch_bytes(g) bytes), or null to use the geometry's own
// (allocated on first use); with a scratch given nothing is allocated and a
// missing stored A^T is an error instead of being built.
template <class T>
void adjoint_impl(pat_geometry g, const void* d_f, void* d_u, hipStream_t s, T* parts = nullptr,
                  T* scratch = nullptr) {
  if (g->adj_mode != 0) {
    if (scratch) PAT_CHECK_ARG(g->csr_nnz >= 0, "the stored A^T is not built (pat_geometry_set_adjoint builds it)");
    else g->ensure_csr(s);
  }
  const int mode = g->effective_adj_mode();
  if (mode != 0) {
    const int64_t N = g->n_pix();
    const int rot = g->csr_rot;
    pat::CsrMultiArgs<T> c{};
    c.ptr = pat::ptr<int64_t>(g->csr_ptr);
    c.col = pat::ptr<int>(g->csr_col);
    c.val = pat::ptr<T>(g->csr_val);
    c.n_rows = N;
    c.nx = g->nx;
    c.ny = g->ny;
    c.n_det = g->csr_det();
    c.n_t = g->n_t;
    c.rot = rot;
    c.nrhs = rot;
    // with quarter turns each slot writes a partial image, summed in order
    T* part = parts ? parts : static_cast<T*>(d_u);
    if (rot > 1 && !parts) {
      if (scratch) {
        part = scratch;
      } else {
        g->scratch_part.ensure(sizeof(T) * (size_t)rot * N);
        part = pat::ptr<T>(g->scratch_part);
      }
    }
    for (int r = 0; r < rot; ++r) {
      c.x[r] = static_cast<const T*>(d_f) + (int64_t)r * c.n_det * g->n_t;
      c.y[r] = part + (int64_t)r * N;
    }
    if (mode == 2) {
      c.lcol = pat::ptr<uint16_t>(g->csr_lcol);
      c.win = pat::ptr<int4>(g->csr_win);
      c.side = g->csr_side;
      c.tiles_x = g->csr_tiles_x;
      c.lds_stride = g->csr_win_max;
      pat::launch_csr_tiled<T>(c, s, false, g->csr_waves, g->csr_lanes);
    } else if (rot > 1) {
      pat::launch_csr_spmm<T>(c, s, false);
    } else {
      pat::CsrArgs<T> p{};
      p.ptr = c.ptr;
      p.col = c.col;
      p.val = c.val;
      p.x = c.x[0];
      p.y = c.y[0];
      p.n_rows = N;
      pat::launch_csr_spmv<T>(p, s);
    }
    if (rot > 1 && !parts) pat::launch_reduce_groups<T>(part, static_cast<T*>(d_u), rot, N, s);
    return;
  }
  PAT_CHECK_ARG(parts == nullptr, "partial images need a stored A^T (adjoint mode 1 or 2)");
  pat::AdjArgs<T> a{};
  a.g = g->dev();
  a.data = static_cast<const T*>(d_f);
  const int ng = a.g.n_groups;
  if (ng == 1) {
    a.part = static_cast<T*>(d_u);
    pat::launch_adjoint<T>(a, s);
    return;
  }
  if (scratch) {
    a.part = scratch;
  } else {
    g->scratch_part.ensure(sizeof(T) * (size_t)ng * g->n_pix());
    a.part = pat::ptr<T>(g->scratch_part);
  }
  pat::launch_adjoint<T>(a, s);
  pat::launch_reduce_groups<T>(a.part, static_cast<T*>(d_u), ng, g->n_pix(), s);
}

}  // namespace

namespace pat {
size_t adjoint_scratch_bytes(const pat_geometry_s* g) {
  const size_t es = dtype_size(g->dtype);
  if (g->adj_mode != 0 && g->effective_adj_mode() != 0)
    return g->csr_rot > 1 ? es * (size_t)g->csr_rot * (size_t)g->n_pix() : 0;
  const int ng = g->n_groups();
  return ng > 1 ? es * (size_t)ng * (size_t)g->n_pix() : 0;
}
template <class T>
void apply_adjoint_scratch(pat_geometry g, const T* f, T* u, T* scratch, hipStream_t s) {
  adjoint_impl<T>(g, f, u, s, nullptr, scratch);
}
template void apply_adjoint_scratch<float>(pat_geometry, const float*, float*, float*, hipStream_t);
template void apply_adjoint_scratch<double>(pat_geometry, const double*, double*, double*, hipStream_t);
template <class T>
void apply_forward(pat_geometry g, const T* u, T* f, hipStream_t s) { forward_impl<T>(g, u, f, s); }
template <class T>
void apply_adjoint(pat_geometry g, const T* f, T* u, hipStream_t s) { adjoint_impl<T>(g, f, u, s); }
template void apply_forward<float>(pat_geometry, const float*, float*, hipStream_t);
template void apply_forward<double>(pat_geometry, const double*, double*, hipStream_t);
template void apply_adjoint<float>(pat_geometry, const float*, float*, hipStream_t);
template void apply_adjoint<double>(pat_geometry, const double*, double*, hipStream_t);
}  // namespace pat

extern "C" pat_status pat_forward(pat_geometry g, const void* d_u, void* d_f, void* stream) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    PAT_CHECK_ARG(d_u != nullptr && d_f != nullptr, "NULL buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->dtype == PAT_F64) forward_impl<double>(g, d_u, d_f, s);
    else forward_impl<float>(g, d_u, d_f, s);
    return PAT_OK;
  });
}

extern "C" pat_status pat_forward_padded(pat_geometry g, const void* d_upad, void* d_f, void* stream) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    PAT_CHECK_ARG(d_upad != nullptr && d_f != nullptr, "NULL buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->dtype == PAT_F64) forward_padded_impl<double>(g, d_upad, d_f, s);
    else forward_padded_impl<float>(g, d_upad, d_f, s);
    return PAT_OK;
  });
}

extern "C" pat_status pat_adjoint_partials(pat_geometry g, const void* d_f, void* d_parts, void* stream) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    PAT_CHECK_ARG(d_parts != nullptr && d_f != nullptr, "NULL buffer");
    if (g->adj_mode == 0) {
      pat::set_error("partial images need a stored A^T (adjoint mode 1 or 2)");
      return PAT_ERR_UNSUPPORTED;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->dtype == PAT_F64) adjoint_impl<double>(g, d_f, nullptr, s, static_cast<double*>(d_parts));
    else adjoint_impl<float>(g, d_f, nullptr, s, static_cast<float*>(d_parts));
    return PAT_OK;
  });
}

extern "C" pat_status pat_adjoint(pat_geometry g, const void* d_f, void* d_u, void* stream) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr, "geometry is NULL");
    PAT_CHECK_ARG(d_u != nullptr && d_f != nullptr, "NULL buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->dtype == PAT_F64) adjoint_impl<double>(g, d_f, d_u, s);
    else adjoint_impl<float>(g, d_f, d_u, s);
    return PAT_OK;
  });
}
