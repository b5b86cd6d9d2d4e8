// The stored forward matrix by pixel tiles: forward path 3 on quarter-turn
// symmetric geometries (arXiv:1707.02245, Sec. 3.3.1: the discretised matrix
// is computed once and applied; Sec. 4.1 eq. K_def).
//
// Layout. The non-zeros of A for the first n_det/4 detectors, which are the
// stored quarter of A^T read the other way (the same values), grouped by
// 16 x 16 pixel tile, within a tile by bin (a segment), within a segment by
// pixel. An entry is its pixel within the tile (one byte) and its weight; a
// segment is padded with zero entries to a multiple of four, so that a lane
// reads four entries with two 16-byte (FP64) or one 16-byte (FP32) weight
// load and one 4-byte offset load. A segment's four partial sums (one per
// quarter turn) sit side by side in tile order; segidx[binseg[b] ..
// binseg[b+1]) lists bin b's segments in tile order.
//
// Apply, two passes. Tile pass: a workgroup stages its tile of the image
// turned by 0..3 quarter turns in LDS, a pixel's four turns side by side (the
// weights obey w(d + t n_det/4, k, R^t p) = w(d, k, p), so the bins of
// detector d + t n_det/4 are those of detector d on the image turned t
// times) and sums, 4 lanes per segment and 4 entries per lane and step,
// weight times pixel for the four turns into the segment's four partials.
// Bin pass: a thread per bin of the first quarter adds its partials in tile
// order, per turn, and hands each value to the forward's epilogue (data, the
// dual data step, gap terms). Both passes are deterministic; the result is
// the transpose of the stored A^T exactly (the same matrix entries), summed
// in pixel order.
//
// Build. From the stored quarter of A^T: per tile and detector the run of
// radii its rows touch (the tile's local bins); a count pass and a placement
// pass over the tile's rows in pixel order, one row at a time (a row's
// entries have distinct bins, so the per-bin counters need no atomics and the
// placement is the same on every build).

#include <algorithm>
#include <vector>

#include "pat_internal.hpp"
#include "reg_dual.hpp"
#include "fwd_epilogue.hpp"

namespace pat {

namespace {

constexpr int kFmLocalMax = 12288;  // local bins per tile (LDS counters, 48 KB)
constexpr int64_t kFmSlack = 64;    // zero entries past the end

__device__ __forceinline__ int find_blk(const int* __restrict__ starts, int n, int blk) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (starts[mid] <= blk) lo = mid; else hi = mid;
  }
  return lo;
}

// Count (place == false: counts of every local bin to cnt_out) or place the
// entries of one tile's rows (one workgroup per tile).
template <class T, bool PLACE>
__global__ __launch_bounds__(256) void fmat_tile_kernel(const int64_t* __restrict__ ptr, const int* __restrict__ col,
                                                        const T* __restrict__ val, const int4* __restrict__ win,
                                                        const int64_t* __restrict__ lbase, int nx, int ny,
                                                        int tiles_x, int nd, int n_t, int* __restrict__ cnt_out,
                                                        const int* __restrict__ seg_of,
                                                        const int4* __restrict__ seg, uint8_t* __restrict__ off_out,
                                                        T* __restrict__ w_out) {
  extern __shared__ int cnt[];
  const int t = blockIdx.x;
  const int n_local = (int)(lbase[t + 1] - lbase[t]);
  for (int i = threadIdx.x; i < n_local; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  const int x0 = (t % tiles_x) * kFmSide, y0 = (t / tiles_x) * kFmSide;
  for (int r = 0; r < kFmSide * kFmSide; ++r) {
    const int i = x0 + r % kFmSide, j = y0 + r / kFmSide;
    if (i < nx && j < ny) {
      const int64_t p = (int64_t)j * nx + i;
      for (int64_t e = ptr[p] + threadIdx.x; e < ptr[p + 1]; e += blockDim.x) {
        const int c = col[e];
        const int d = c / n_t, k = c - d * n_t;
        const int4 w = win[(int64_t)t * nd + d];
        const int lb = w.z + k - w.x;
        if (PLACE) {
          const int s = seg_of[lbase[t] + lb];
          const int q = seg[s].x + cnt[lb];
          off_out[q] = (uint8_t)r;
          w_out[q] = val[e];
        }
        cnt[lb] += 1;  // distinct bins within a row
      }
    }
    __syncthreads();
  }
  if (!PLACE)
    for (int i = threadIdx.x; i < n_local; i += blockDim.x) cnt_out[lbase[t] + i] = cnt[i];
}

// Tile pass (see the file comment); with FUSED the regulariser's dual step of
// every instance runs in the blocks from n_fwd on.
template <class T, bool FUSED>
__global__ __launch_bounds__(256) void fmat_kernel(FwdArgs<T> a0, const FwdArgs<T>* __restrict__ arr,
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
  if (arr) {
    const int i = find_blk(starts, n_inst, blk);
    a = arr[i];
    blk -= starts[i];
  } else {
    a = a0;
  }
  const GeomDev& g = a.g;
  constexpr int S2 = kFmSide * kFmSide;
  // pixel r's four turns at img[4 r .. 4 r + 3]: slot t holds the image
  // turned by t quarter turns, u_t(p) = u(R^t p)
  constexpr int kPix = 4;
  __shared__ __align__(16) T img[kPix * S2];
  const int4 ch = g.fm_chunk[blk];
  const int x0 = (ch.x % g.fm_tiles_x) * kFmSide, y0 = (ch.x / g.fm_tiles_x) * kFmSide;
  const int n = g.nx, P = g.pitch;
  const gptr<const T> up = as_global(a.upad);
  for (int e = threadIdx.x; e < 4 * S2; e += blockDim.x) {
    const int t = e / S2, r = e - t * S2;
    const int i = x0 + r % kFmSide, j = y0 + r / kFmSide;
    T v = T(0);
    if (i < n && j < n) {
      int x, y;
      quarter_turn_xy(i, j, n, t, x, y);
      v = up[(int64_t)(y + 1) * P + (x + 1)];
    }
    img[kPix * r + t] = v;
  }
  __syncthreads();
  const gptr<const uint32_t> off4 = as_global(reinterpret_cast<const uint32_t*>(g.fm_off));
  const gptr<const T> wt = as_global(static_cast<const T*>(g.fm_w));
  typedef T T2 __attribute__((ext_vector_type(2)));
  typedef T T4 __attribute__((ext_vector_type(4)));
  // The chunk's segments are contiguous: its entries, in groups of four (no
  // group straddles two segments), run from the first segment's first entry.
  // Thread t takes groups t, t + 256, ... (consecutive lanes on consecutive
  // groups, so a wave's loads are contiguous), all loaded before any is used,
  // and leaves each group's four turn sums in LDS; then a thread per segment
  // adds its groups' sums in order.
  __shared__ __align__(16) T4 gsum[kFmChunkEntries / 4];
  const int e0 = g.fm_seg[ch.y].x;
  const int4 last = g.fm_seg[ch.z - 1];
  const int ng = (last.x + last.y - e0) >> 2;  // at most kFmChunkEntries / 4
  constexpr int kPer = kFmChunkEntries / 4 / 256;
  uint32_t o4[kPer];
  T w[kPer][4];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int q = threadIdx.x + 256 * i;
    o4[i] = 0;
    w[i][0] = w[i][1] = w[i][2] = w[i][3] = T(0);
    if (q < ng) {
      const int e = e0 + 4 * q;
      o4[i] = __builtin_nontemporal_load(off4 + (e >> 2));
      if constexpr (sizeof(T) == 8) {
        const gptr<const T2> w2 = (gptr<const T2>)(wt + e);
        const T2 wa = __builtin_nontemporal_load(w2), wb = __builtin_nontemporal_load(w2 + 1);
        w[i][0] = wa.x;
        w[i][1] = wa.y;
        w[i][2] = wb.x;
        w[i][3] = wb.y;
      } else {
        const T4 wa = __builtin_nontemporal_load((gptr<const T4>)(wt + e));
        w[i][0] = wa.x;
        w[i][1] = wa.y;
        w[i][2] = wa.z;
        w[i][3] = wa.w;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int q = threadIdx.x + 256 * i;
    if (q < ng) {
      T acc0 = T(0), acc1 = T(0), acc2 = T(0), acc3 = T(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const T4 px = *reinterpret_cast<const T4*>(img + kPix * ((o4[i] >> (8 * k)) & 0xFF));
        acc0 = fma(w[i][k], px.x, acc0);
        acc1 = fma(w[i][k], px.y, acc1);
        acc2 = fma(w[i][k], px.z, acc2);
        acc3 = fma(w[i][k], px.w, acc3);
      }
      T4 v;
      v.x = acc0;
      v.y = acc1;
      v.z = acc2;
      v.w = acc3;
      gsum[q] = v;
    }
  }
  __syncthreads();
  // a segment's four partials side by side, segments in tile order: a
  // workgroup writes one contiguous run
  for (int s = ch.y + threadIdx.x; s < ch.z; s += 256) {
    const int4 sd = g.fm_seg[s];
    T4 acc = gsum[(sd.x - e0) >> 2];
    for (int q = ((sd.x - e0) >> 2) + 1, qe = (sd.x + sd.y - e0) >> 2; q < qe; ++q) acc += gsum[q];
    *reinterpret_cast<T4*>(a.part + 4 * (int64_t)s) = acc;
  }
}

// Bin pass (see the file comment): 16 lanes per bin of the first quarter,
// 16 bins per workgroup; a bin's segments (listed in tile order) are added
// across its lanes, each lane's in order, then over the lanes in a fixed
// tree.
template <class T, int MODE>
__global__ __launch_bounds__(256) void fmat_reduce_kernel(FwdArgs<T> a0, const FwdArgs<T>* __restrict__ arr,
                                                          const int* __restrict__ starts, int n_inst) {
  int blk = blockIdx.x;
  FwdArgs<T> a;
  if (arr) {
    const int i = find_blk(starts, n_inst, blk);
    a = arr[i];
    blk -= starts[i];
  } else {
    a = a0;
  }
  const GeomDev& g = a.g;
  const int64_t nb = (int64_t)g.n_det * g.n_t;
  const int gl = threadIdx.x & 15;
  const int64_t b = (int64_t)blk * 16 + (threadIdx.x >> 4);
  const bool valid = b < nb;
  // the dual data step's operands of the four turns, loaded before the
  // partials so that both round trips overlap (the same arithmetic as the
  // forward's epilogue)
  T dq[4], df[4], ds[4];
  if (MODE == FWD_DUAL && valid && gl == 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t bt = b + t * a.slot_bins;
      dq[t] = a.out[bt];
      df[t] = a.f[bt];
      ds[t] = a.sigma[bt];
    }
  }
  T v[4] = {T(0), T(0), T(0), T(0)};
  if (valid) {
    typedef T T4 __attribute__((ext_vector_type(4)));
    const int s0 = g.fm_binseg[b], s1 = g.fm_binseg[b + 1];
    for (int i = s0 + gl; i < s1; i += 16) {
      const T4 p = *reinterpret_cast<const T4*>(a.part + 4 * (int64_t)g.fm_segidx[i]);
      v[0] += p.x;
      v[1] += p.y;
      v[2] += p.z;
      v[3] += p.w;
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = row16_sum(v[t]);
  if (MODE == FWD_DUAL) {
    if (valid && gl == 0) {
      const T dm = a.mult ? (T)a.mult[0] : T(1);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        // q <- (q + sigma (A ubar - f)) / (1 + sigma), as fwd_epilogue
        const T sg = a.mult ? ds[t] * dm : ds[t];
        a.out[b + t * a.slot_bins] = (dq[t] + sg * (v[t] - df[t])) / (T(1) + sg);
      }
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    FwdArgs<T> at = a;
    const int64_t ob = t * a.slot_bins;
    if (at.out) at.out += ob;
    if (at.f) at.f += ob;
    if (at.sigma) at.sigma += ob;
    if (at.q) at.q += ob;
    if (at.red) at.red += t * a.slot_red;
    fwd_epilogue<T, MODE>(at, blk, valid && gl == 0, b, v[t]);
  }
}

}  // namespace

template <class T>
void build_fmat(pat_geometry_s* geo, hipStream_t s) {
  geo->drop_fmat();
  geo->fm_entries = 0;  // not available unless built below
  if (geo->sym_rot != 4 || geo->csr_rot != 4 || geo->csr_nnz <= 0 || geo->nx != geo->ny) return;
  const int nd = geo->csr_det(), n_t = geo->n_t, nx = geo->nx, ny = geo->ny;
  const int tx = (nx + kFmSide - 1) / kFmSide, ty = (ny + kFmSide - 1) / kFmSide;
  const int64_t nt = (int64_t)tx * ty;
  DevBuf win(sizeof(int4) * nt * nd);
  launch_csr_windows(geo, kFmSide, tx, nt, ptr<int4>(win), s);
  std::vector<int4> h(nt * nd);
  PAT_HIP(hipMemcpyAsync(h.data(), win.p, sizeof(int4) * h.size(), hipMemcpyDeviceToHost, s));
  PAT_HIP(hipStreamSynchronize(s));
  // local bins of a tile: its detectors' radius runs, one after another
  std::vector<int64_t> lbase(nt + 1, 0);
  int64_t local_max = 0;
  for (int64_t t = 0; t < nt; ++t) {
    int64_t o = 0;
    for (int d = 0; d < nd; ++d) {
      int4& w = h[t * nd + d];
      w.z = (int)o;
      o += w.y;
    }
    lbase[t + 1] = lbase[t] + o;
    local_max = std::max(local_max, o);
  }
  if (local_max > kFmLocalMax) return;  // too many bins per tile for the LDS counters
  const int64_t n_local = lbase[nt];
  DevBuf d_lbase(sizeof(int64_t) * (nt + 1)), cnt(sizeof(int) * std::max<int64_t>(n_local, 1));
  PAT_HIP(hipMemcpyAsync(win.p, h.data(), sizeof(int4) * h.size(), hipMemcpyHostToDevice, s));
  PAT_HIP(hipMemcpyAsync(d_lbase.p, lbase.data(), d_lbase.bytes, hipMemcpyHostToDevice, s));
  const size_t shm = sizeof(int) * (size_t)std::max<int64_t>(local_max, 1);
  const T* val = ptr<T>(geo->csr_val);
  hipLaunchKernelGGL((fmat_tile_kernel<T, false>), dim3((unsigned)nt), dim3(256), shm, s, ptr<int64_t>(geo->csr_ptr),
                     ptr<int>(geo->csr_col), val, ptr<int4>(win), ptr<int64_t>(d_lbase), nx, ny, tx, nd, n_t,
                     ptr<int>(cnt), (const int*)nullptr, (const int4*)nullptr, (uint8_t*)nullptr, (T*)nullptr);
  PAT_HIP(hipGetLastError());
  std::vector<int> h_cnt(n_local);
  if (n_local > 0)
    PAT_HIP(hipMemcpyAsync(h_cnt.data(), cnt.p, sizeof(int) * n_local, hipMemcpyDeviceToHost, s));
  PAT_HIP(hipStreamSynchronize(s));
  // segments in tile-major order, partials numbered bin-major (tile order
  // within a bin), workgroups of whole segments
  const int64_t nbq = (int64_t)nd * n_t;
  std::vector<int> seg_of(std::max<int64_t>(n_local, 1), -1), seg_bin;
  std::vector<int4> seg, chunk;
  std::vector<int> binseg(nbq + 1, 0);
  int64_t entries = 0, real = 0;
  for (int64_t t = 0; t < nt; ++t) {
    int64_t ch_entries = 0;
    for (int d = 0; d < nd; ++d) {
      const int4 w = h[t * nd + d];
      for (int kk = 0; kk < w.y; ++kk) {
        const int64_t li = lbase[t] + w.z + kk;
        const int c = h_cnt[li];
        if (c == 0) continue;
        if (chunk.empty() || chunk.back().x != (int)t || ch_entries + c + 3 > kFmChunkEntries) {
          if (!chunk.empty() && chunk.back().x == (int)t) chunk.back().z = (int)seg.size();
          chunk.push_back(make_int4((int)t, (int)seg.size(), (int)seg.size(), 0));
          ch_entries = 0;
        }
        const int c4 = (c + 3) & ~3;  // padded with zero entries
        ch_entries += c4;
        seg_of[li] = (int)seg.size();
        seg.push_back(make_int4((int)entries, c4, 0, 0));
        const int bin = d * n_t + w.x + kk;
        seg_bin.push_back(bin);
        binseg[bin + 1] += 1;
        entries += c4;
        real += c;
      }
    }
    if (!chunk.empty() && chunk.back().x == (int)t) chunk.back().z = (int)seg.size();
  }
  PAT_CHECK_ARG(real == geo->csr_nnz, "stored forward: entries do not match the stored A^T");
  PAT_CHECK_ARG(entries < (int64_t(1) << 31) - kFmSlack, "stored forward: too many entries");
  for (int64_t b = 0; b < nbq; ++b) binseg[b + 1] += binseg[b];
  // each bin's segments in tile order
  std::vector<int> segidx(std::max<size_t>(seg.size(), 1), 0);
  {
    std::vector<int> cur(binseg.begin(), binseg.end() - 1);
    for (size_t i = 0; i < seg.size(); ++i) segidx[cur[seg_bin[i]]++] = (int)i;
  }
  const int64_t nseg = (int64_t)seg.size();
  PAT_CHECK_ARG(nseg < (int64_t(1) << 31) / 4, "stored forward: too many segments");
  DevBuf d_seg_of(sizeof(int) * seg_of.size());
  geo->fm_seg.alloc(sizeof(int4) * std::max<int64_t>(nseg, 1));
  geo->fm_chunk.alloc(sizeof(int4) * std::max<size_t>(chunk.size(), 1));
  geo->fm_binseg.alloc(sizeof(int) * binseg.size());
  geo->fm_segidx.alloc(sizeof(int) * segidx.size());
  geo->fm_off.alloc(entries + kFmSlack);
  geo->fm_w.alloc(sizeof(T) * (entries + kFmSlack));
  PAT_HIP(hipMemsetAsync(geo->fm_off.p, 0, geo->fm_off.bytes, s));
  PAT_HIP(hipMemsetAsync(geo->fm_w.p, 0, geo->fm_w.bytes, s));
  PAT_HIP(hipMemcpyAsync(d_seg_of.p, seg_of.data(), d_seg_of.bytes, hipMemcpyHostToDevice, s));
  if (nseg > 0) PAT_HIP(hipMemcpyAsync(geo->fm_seg.p, seg.data(), sizeof(int4) * nseg, hipMemcpyHostToDevice, s));
  if (!chunk.empty())
    PAT_HIP(hipMemcpyAsync(geo->fm_chunk.p, chunk.data(), sizeof(int4) * chunk.size(), hipMemcpyHostToDevice, s));
  PAT_HIP(hipMemcpyAsync(geo->fm_binseg.p, binseg.data(), geo->fm_binseg.bytes, hipMemcpyHostToDevice, s));
  PAT_HIP(hipMemcpyAsync(geo->fm_segidx.p, segidx.data(), geo->fm_segidx.bytes, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL((fmat_tile_kernel<T, true>), dim3((unsigned)nt), dim3(256), shm, s, ptr<int64_t>(geo->csr_ptr),
                     ptr<int>(geo->csr_col), val, ptr<int4>(win), ptr<int64_t>(d_lbase), nx, ny, tx, nd, n_t,
                     (int*)nullptr, ptr<int>(d_seg_of), ptr<int4>(geo->fm_seg), ptr<uint8_t>(geo->fm_off),
                     ptr<T>(geo->fm_w));
  PAT_HIP(hipGetLastError());
  PAT_HIP(hipStreamSynchronize(s));  // host tables go out of scope
  geo->fm_entries = real;
  geo->fm_nseg = (int)nseg;
  geo->fm_nchunk = (int)chunk.size();
  geo->fm_tiles_x = tx;
}

template <class T>
void launch_forward_fmat(int mode, const FwdArgs<T>& a, hipStream_t s) {
  PAT_CHECK_ARG(mode == FWD_PLAIN, "stored forward stand-alone: plain mode only");
  if (a.g.fm_nchunk > 0)
    hipLaunchKernelGGL((fmat_kernel<T, false>), dim3((unsigned)a.g.fm_nchunk), dim3(256), 0, s, a,
                       (const FwdArgs<T>*)nullptr, (const int*)nullptr, 1, a.g.fm_nchunk,
                       (const InstDev<T>*)nullptr, (const int*)nullptr, 0);
  PAT_HIP(hipGetLastError());
  const int blocks = fmat_reduce_blocks(a.g.n_det, a.g.n_t);
  if (blocks > 0)
    hipLaunchKernelGGL((fmat_reduce_kernel<T, FWD_PLAIN>), dim3((unsigned)blocks), dim3(256), 0, s, a,
                       (const FwdArgs<T>*)nullptr, (const int*)nullptr, 1);
  PAT_HIP(hipGetLastError());
}

template <class T>
void launch_fmat_batched(int mode, bool fused_reg, const Launch<T>& L, hipStream_t s) {
  const FwdArgs<T> none{};
  const FwdArgs<T>* arr = ptr<FwdArgs<T>>(L.fm);  // the gap's table when the caller swapped it in
  const int extra = fused_reg ? L.pix_total : 0;
  if (L.fm_total + extra > 0) {
    if (fused_reg)
      hipLaunchKernelGGL((fmat_kernel<T, true>), dim3((unsigned)(L.fm_total + extra)), dim3(256), 0, s, none, arr,
                         ptr<int>(L.fm_start), L.fm_n, L.fm_total, ptr<InstDev<T>>(L.inst), ptr<int>(L.pix_start),
                         L.n);
    else
      hipLaunchKernelGGL((fmat_kernel<T, false>), dim3((unsigned)L.fm_total), dim3(256), 0, s, none, arr,
                         ptr<int>(L.fm_start), L.fm_n, L.fm_total, (const InstDev<T>*)nullptr, (const int*)nullptr,
                         0);
    PAT_HIP(hipGetLastError());
  }
  if (L.fmr_total <= 0) return;
  if (mode == FWD_DUAL)
    hipLaunchKernelGGL((fmat_reduce_kernel<T, FWD_DUAL>), dim3((unsigned)L.fmr_total), dim3(256), 0, s, none, arr,
                       ptr<int>(L.fmr_start), L.fm_n);
  else if (mode == FWD_GAP)
    hipLaunchKernelGGL((fmat_reduce_kernel<T, FWD_GAP>), dim3((unsigned)L.fmr_total), dim3(256), 0, s, none, arr,
                       ptr<int>(L.fmr_start), L.fm_n);
  else
    PAT_CHECK_ARG(false, "stored forward in a batch: dual or gap mode only");
  PAT_HIP(hipGetLastError());
}

template void build_fmat<float>(pat_geometry_s*, hipStream_t);
template void build_fmat<double>(pat_geometry_s*, hipStream_t);
template void launch_forward_fmat<float>(int, const FwdArgs<float>&, hipStream_t);
template void launch_forward_fmat<double>(int, const FwdArgs<double>&, hipStream_t);
template void launch_fmat_batched<float>(int, bool, const Launch<float>&, hipStream_t);
template void launch_fmat_batched<double>(int, bool, const Launch<double>&, hipStream_t);

}  // namespace pat
