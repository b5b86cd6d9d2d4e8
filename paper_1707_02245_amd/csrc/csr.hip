// The stored transpose of the circular-mean operator: A^T as a CSR matrix
// (rows = pixels, columns = bins, sorted), built once on the device and
// applied by a sparse matrix-vector product (arXiv:1707.02245, Sec. 3.3.1:
// compute the discretised matrix once and use its transpose as the adjoint).
//
// Build: one wave per pixel; lane d enumerates, for detector d, the radii
// whose circles pass within sqrt(2) pixels of the pixel centre and the arc
// samples in the pixel's angular window, computes each sample's position and
// bilinear weights with exactly the arithmetic of the forward kernel, keeps
// the weight that falls on this pixel and sums it per radius. Entries come
// out in bin order (detector-major, then radius), so the build is
// deterministic and needs no sort. A count pass and a fill pass share the
// enumeration; the row offsets are a host prefix sum.
//
// Apply: the rows of one pixel tile (8 x 8, or 4 x 4 when the windows would
// not fit) touch, per detector, a short run of consecutive radii (the circles
// through the tile). The tiled kernel stages these windows of the input in
// LDS once per tile and reads the non-zeros with 16-bit window offsets, so
// the input gathers hit LDS instead of the L2 and each non-zero streams 2
// index bytes instead of 4.
//
// Quarter turns: when detector d + n_det/4 sits at the quarter turn R of
// detector d about the centre of a square grid and every circle's sample set
// is invariant under quarter turns (M_k a multiple of four), the weights obey
// w(d + t n_det/4, k, R^t p) = w(d, k, p). The matrix then stores the rows of
// the first n_det/4 detectors only; one pass over it serves four slots, slot t
// reading the data of detectors t n_det/4 .. (t+1) n_det/4 - 1 and writing
// its partial image at the pixels turned by t quarter turns. The four partial
// images are summed by the consumer in a fixed order.

#include <numeric>
#include <type_traits>

#include "pat_internal.hpp"

namespace pat {

constexpr double kTwoPiC = 6.283185307179586476925286766559;

// Enumerate the non-zeros of row `pix` of A^T contributed by detector d.
// With out_col == nullptr only counts; otherwise writes (bin, value) pairs.
template <class T>
__device__ int enum_pixel_detector(const GeomDev& g, int i, int j, int d, int* out_col, T* out_val) {
  const double2 p = g.det[d];
  const double dx = (double)i - p.x, dy = (double)j - p.y;
  const double rho = sqrt(dx * dx + dy * dy);
  const int k0 = max(0, (int)floor((rho - 1.5) * g.kscale - g.koff) - 1);
  const int k1 = min(g.n_t - 1, (int)ceil((rho + 1.5) * g.kscale - g.koff) + 1);
  const bool full = rho < 2.0;
  double a_lo = 0.0, a_hi = 0.0;
  if (!full) {
    const double psi = atan2(dy, dx);
    const double del = asin(fmin(1.0, 1.5 / rho)) + 1e-9;
    a_lo = psi - del;
    a_hi = psi + del;
  }
  int n = 0;
  for (int k = k0; k <= k1; ++k) {
    const int2 mo = g.moff[k];
    const double2 rr = g.rad[k];
    const int M = mo.x;
    int mlo = 0, cnt = M;
    if (!full) {
      mlo = (int)floor(a_lo * M / kTwoPiC - 0.5) - 1;
      const int mhi = (int)ceil(a_hi * M / kTwoPiC - 0.5) + 1;
      cnt = min(M, mhi - mlo + 1);
      mlo %= M;
      if (mlo < 0) mlo += M;
    }
    T wsum = T(0);
    for (int t = 0; t < cnt; ++t) {
      int m = mlo + t;
      if (m >= M) m -= M;
      const double2 cs = table_cs<T>(g, mo.y + m);
      const double gx = fma(rr.x, cs.x, p.x);
      const double gy = fma(rr.x, cs.y, p.y);
      const double fx = floor(gx), fy = floor(gy);
      const int ix = (int)fx, iy = (int)fy;
      const int ox = i - ix, oy = j - iy;
      if ((unsigned)ox <= 1u && (unsigned)oy <= 1u) {
        const T tx = (T)(gx - fx), ty = (T)(gy - fy);
        const T wx = ox ? tx : (T(1) - tx);
        const T wy = oy ? ty : (T(1) - ty);
        wsum += wx * wy;
      }
    }
    if (wsum != T(0)) {
      if (out_col) {
        out_col[n] = d * g.n_t + k;
        out_val[n] = wsum * (T)rr.y;
      }
      ++n;
    }
  }
  return n;
}

__device__ __forceinline__ int wave_excl_scan(int v, int lane, int* total) {
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

template <class T>
__global__ __launch_bounds__(256) void csr_build_kernel(GeomDev g, int nd, int* __restrict__ row_cnt,
                                                        const int64_t* __restrict__ row_ptr,
                                                        int* __restrict__ col, T* __restrict__ val) {
  const int64_t N = (int64_t)g.nx * g.ny;
  const int64_t pix = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (pix >= N) return;  // whole wave
  const int i = (int)(pix % g.nx), j = (int)(pix / g.nx);
  int64_t pos = row_ptr ? row_ptr[pix] : 0;
  int total = 0;
  for (int d0 = 0; d0 < nd; d0 += 64) {
    const int d = d0 + lane;
    const int c = d < nd ? enum_pixel_detector<T>(g, i, j, d, nullptr, nullptr) : 0;
    int sum;
    const int excl = wave_excl_scan(c, lane, &sum);
    if (row_ptr && c > 0) enum_pixel_detector<T>(g, i, j, d, col + pos + excl, val + pos + excl);
    pos += sum;
    total += sum;
  }
  if (!row_ptr && lane == 0) row_cnt[pix] = total;
}

// Per tile and detector: the smallest and largest radius index of the
// non-zeros of the tile's rows (rows hold bins in increasing order, so each
// detector is one run found by binary search).
__global__ __launch_bounds__(256) void csr_window_kernel(const int64_t* __restrict__ ptr, const int* __restrict__ col,
                                                         int nx, int ny, int side, int tiles_x, int n_det, int n_t,
                                                         int4* __restrict__ win) {
  const int t = blockIdx.x;
  const int tx = t % tiles_x, ty = t / tiles_x;
  for (int d = threadIdx.x; d < n_det; d += blockDim.x) {
    const int c0 = d * n_t, c1 = c0 + n_t;
    int lo = n_t, hi = -1;
    for (int r = 0; r < side * side; ++r) {
      const int i = tx * side + r % side, j = ty * side + r / side;
      if (i >= nx || j >= ny) continue;
      const int64_t p = (int64_t)j * nx + i;
      int64_t a = ptr[p], b = ptr[p + 1];
      const int64_t end = b;
      while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (col[m] < c0) a = m + 1; else b = m;
      }
      for (int64_t e = a; e < end && col[e] < c1; ++e) {
        const int k = col[e] - c0;
        lo = min(lo, k);
        hi = max(hi, k);
      }
    }
    win[(int64_t)t * n_det + d] = hi < 0 ? make_int4(0, 0, 0, 0) : make_int4(lo, hi - lo + 1, 0, 0);
  }
}

// lcol[e] = off + k - k0 of the entry's tile and detector (one wave per row)
__global__ __launch_bounds__(256) void csr_lcol_kernel(const int64_t* __restrict__ ptr, const int* __restrict__ col,
                                                       const int4* __restrict__ win, int nx, int ny, int side,
                                                       int tiles_x, int n_det, int n_t,
                                                       uint16_t* __restrict__ lcol) {
  const int64_t N = (int64_t)nx * ny;
  const int64_t pix = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (pix >= N) return;
  const int i = (int)(pix % nx), j = (int)(pix / nx);
  const int64_t t = (int64_t)(j / side) * tiles_x + i / side;
  for (int64_t e = ptr[pix] + lane; e < ptr[pix + 1]; e += 64) {
    const int c = col[e];
    const int d = c / n_t, k = c - d * n_t;
    const int4 w = win[t * n_det + d];
    lcol[e] = (uint16_t)(w.z + k - w.x);
  }
}

void launch_csr_windows(const pat_geometry_s* geo, int side, int tiles_x, int64_t n_tiles, int4* win,
                        hipStream_t s) {
  hipLaunchKernelGGL(csr_window_kernel, dim3((unsigned)n_tiles), dim3(256), 0, s, ptr<int64_t>(geo->csr_ptr),
                     ptr<int>(geo->csr_col), geo->nx, geo->ny, side, tiles_x, geo->csr_det(), geo->n_t, win);
  PAT_HIP(hipGetLastError());
}

void build_csr_tiles(pat_geometry_s* geo, size_t esz, hipStream_t s) {
  geo->csr_side = 0;
  geo->csr_tiles_x = geo->csr_tiles_y = geo->csr_win_max = 0;
  const int64_t N = geo->n_pix();
  if (geo->csr_nnz <= 0) return;
  const int nd = geo->csr_det();
  for (int side : {8, 4}) {
    const int tx = (geo->nx + side - 1) / side, ty = (geo->ny + side - 1) / side;
    const int64_t nt = (int64_t)tx * ty;
    DevBuf win(sizeof(int4) * nt * nd);
    hipLaunchKernelGGL(csr_window_kernel, dim3((unsigned)nt), dim3(256), 0, s, ptr<int64_t>(geo->csr_ptr),
                       ptr<int>(geo->csr_col), geo->nx, geo->ny, side, tx, nd, geo->n_t, ptr<int4>(win));
    PAT_HIP(hipGetLastError());
    std::vector<int4> h(nt * nd);
    PAT_HIP(hipMemcpyAsync(h.data(), win.p, sizeof(int4) * h.size(), hipMemcpyDeviceToHost, s));
    PAT_HIP(hipStreamSynchronize(s));
    int64_t win_max = 0;
    for (int64_t t = 0; t < nt; ++t) {
      int64_t off = 0;
      for (int d = 0; d < nd; ++d) {
        int4& w = h[t * nd + d];
        w.z = (int)off;
        off += w.y;
      }
      win_max = std::max(win_max, off);
    }
    // the 16-bit offsets and one right-hand side (all its quarter-turn slots)
    // must fit the LDS budget
    if (win_max < 1 || win_max > 65535 || (int64_t)esz * win_max * geo->csr_rot > kCsrLdsBytes) continue;
    PAT_HIP(hipMemcpyAsync(win.p, h.data(), sizeof(int4) * h.size(), hipMemcpyHostToDevice, s));
    geo->csr_lcol.alloc(sizeof(uint16_t) * (geo->csr_nnz + kCsrSlack));
    PAT_HIP(hipMemsetAsync(ptr<uint16_t>(geo->csr_lcol) + geo->csr_nnz, 0, sizeof(uint16_t) * kCsrSlack, s));
    hipLaunchKernelGGL(csr_lcol_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s,
                       ptr<int64_t>(geo->csr_ptr), ptr<int>(geo->csr_col), ptr<int4>(win), geo->nx, geo->ny,
                       side, tx, nd, geo->n_t, ptr<uint16_t>(geo->csr_lcol));
    PAT_HIP(hipGetLastError());
    PAT_HIP(hipStreamSynchronize(s));
    geo->csr_win = std::move(win);
    geo->csr_side = side;
    geo->csr_tiles_x = tx;
    geo->csr_tiles_y = ty;
    geo->csr_win_max = (int)win_max;
    return;
  }
}

template <class T>
void build_csr_adjoint(pat_geometry_s* geo, hipStream_t s) {
  const GeomDev g = geo->dev();
  const int64_t N = geo->n_pix();
  geo->csr_rot = (geo->sym_enabled && geo->sym_rot == 4) ? 4 : 1;
  const int nd = geo->csr_det();
  DevBuf cnt(sizeof(int) * N);
  const int blocks = (int)((N + 3) / 4);
  hipLaunchKernelGGL(csr_build_kernel<T>, dim3(blocks), dim3(256), 0, s, g, nd, ptr<int>(cnt),
                     (const int64_t*)nullptr, (int*)nullptr, (T*)nullptr);
  PAT_HIP(hipGetLastError());
  std::vector<int> h_cnt(N);
  PAT_HIP(hipMemcpyAsync(h_cnt.data(), cnt.p, sizeof(int) * N, hipMemcpyDeviceToHost, s));
  PAT_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> h_ptr(N + 1);
  h_ptr[0] = 0;
  for (int64_t r = 0; r < N; ++r) h_ptr[r + 1] = h_ptr[r] + h_cnt[r];
  const int64_t nnz = h_ptr[N];
  PAT_CHECK_ARG(nnz <= (int64_t(1) << 31) - 512, "A^T has too many non-zeros for 32-bit indices");
  geo->csr_ptr.alloc(sizeof(int64_t) * (N + 1));
  geo->csr_col.alloc(sizeof(int) * std::max<int64_t>(nnz, 1));
  // kCsrSlack zero entries past the end: the tiled kernel's aligned loads may
  // read (and discard) up to 255 entries beyond a row
  geo->csr_val.alloc(sizeof(T) * (nnz + kCsrSlack));
  PAT_HIP(hipMemsetAsync(ptr<T>(geo->csr_val) + nnz, 0, sizeof(T) * kCsrSlack, s));
  PAT_HIP(hipMemcpyAsync(geo->csr_ptr.p, h_ptr.data(), sizeof(int64_t) * (N + 1),
                         hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(csr_build_kernel<T>, dim3(blocks), dim3(256), 0, s, g, nd, (int*)nullptr,
                     ptr<int64_t>(geo->csr_ptr), ptr<int>(geo->csr_col), ptr<T>(geo->csr_val));
  PAT_HIP(hipGetLastError());
  PAT_HIP(hipStreamSynchronize(s));
  geo->csr_nnz = nnz;
  build_csr_tiles(geo, sizeof(T), s);
}

// y[row] = sum_e val[e] x[col[e]]: one wave per row, lanes stride the row.
// The matrix streams through once per apply (non-temporal loads keep the
// vectors and the solver state resident in the caches). WIDE accumulates in
// FP64 into y64 (used for the gap's dual residual).
template <class T, bool WIDE>
__global__ __launch_bounds__(256) void csr_spmv_kernel(CsrArgs<T> a0, const CsrArgs<T>* __restrict__ arr,
                                                       const int* __restrict__ starts, int n_inst) {
  int blk = blockIdx.x;
  CsrArgs<T> a;
  if (arr) {
    int lo = 0, hi = n_inst;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (starts[mid] <= blk) lo = mid; else hi = mid;
    }
    a = arr[lo];
    blk -= starts[lo];
  } else {
    a = a0;
  }
  const int64_t row = (int64_t)blk * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= a.n_rows) return;  // whole wave
  const gptr<const int64_t> rowp = as_global(a.ptr);
  const int64_t e0 = rowp[row], e1 = rowp[row + 1];
  using Acc = typename std::conditional<WIDE, double, T>::type;
  Acc acc0 = Acc(0), acc1 = Acc(0), acc2 = Acc(0), acc3 = Acc(0);
  const gptr<const T> val = as_global(a.val);
  const gptr<const int> col = as_global(a.col);
  const gptr<const T> x = as_global(a.x);
  int64_t e = e0 + lane;
  // four independent entries per lane in flight: the column loads of all four
  // are issued before the dependent gathers of x
  for (; e + 192 < e1; e += 256) {
    const int c0 = __builtin_nontemporal_load(col + e);
    const int c1 = __builtin_nontemporal_load(col + e + 64);
    const int c2 = __builtin_nontemporal_load(col + e + 128);
    const int c3 = __builtin_nontemporal_load(col + e + 192);
    const T v0 = __builtin_nontemporal_load(val + e);
    const T v1 = __builtin_nontemporal_load(val + e + 64);
    const T v2 = __builtin_nontemporal_load(val + e + 128);
    const T v3 = __builtin_nontemporal_load(val + e + 192);
    acc0 += (Acc)v0 * (Acc)x[c0];
    acc1 += (Acc)v1 * (Acc)x[c1];
    acc2 += (Acc)v2 * (Acc)x[c2];
    acc3 += (Acc)v3 * (Acc)x[c3];
  }
  for (; e < e1; e += 64) {
    const int c = __builtin_nontemporal_load(col + e);
    acc0 += (Acc)__builtin_nontemporal_load(val + e) * (Acc)x[c];
  }
  Acc acc = (acc0 + acc1) + (acc2 + acc3);
  acc = group_sum<64>(acc);
  if (lane == 0) {
    if (WIDE) a.y64[row] = (double)acc;
    else a.y[row] = (T)acc;
  }
}

// Multi-RHS variant: one wave per row; every (column, value) pair loaded once
// serves all slots of the group (right-hand sides, or their quarter turns).
template <class T, bool WIDE, int R>
__global__ __launch_bounds__(256) void csr_spmm_kernel(CsrMultiArgs<T> a0, const CsrMultiArgs<T>* __restrict__ arr,
                                                       const int* __restrict__ starts, int n_grp) {
  int blk = blockIdx.x;
  const CsrMultiArgs<T>* ap = &a0;
  if (arr) {
    int lo = 0, hi = n_grp;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (starts[mid] <= blk) lo = mid; else hi = mid;
    }
    ap = arr + lo;
    blk -= starts[lo];
  }
  const CsrMultiArgs<T>& a = *ap;
  const int64_t row = (int64_t)blk * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= a.n_rows) return;  // whole wave
  const int nr = a.nrhs;
  using Acc = typename std::conditional<WIDE, double, T>::type;
  Acc acc[R];
  gptr<const T> xs[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    acc[r] = Acc(0);
    xs[r] = as_global(a.x[r]);
  }
  const gptr<const int64_t> rowp = as_global(a.ptr);
  const int64_t e0 = rowp[row], e1 = rowp[row + 1];
  const gptr<const T> val = as_global(a.val);
  const gptr<const int> col = as_global(a.col);
  int64_t e = e0 + lane;
  for (; e + 64 < e1; e += 128) {
    const int c0 = __builtin_nontemporal_load(col + e);
    const int c1 = __builtin_nontemporal_load(col + e + 64);
    const T v0 = __builtin_nontemporal_load(val + e);
    const T v1 = __builtin_nontemporal_load(val + e + 64);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < nr) acc[r] += (Acc)v0 * (Acc)xs[r][c0] + (Acc)v1 * (Acc)xs[r][c1];
  }
  if (e < e1) {
    const int c0 = __builtin_nontemporal_load(col + e);
    const T v0 = __builtin_nontemporal_load(val + e);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < nr) acc[r] += (Acc)v0 * (Acc)xs[r][c0];
  }
  const int rot = a.rot;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r < nr) {
      const Acc t = group_sum<64>(acc[r]);
      if (lane == 0) {
        const int64_t out = rot <= 1 ? row : quarter_turn((int)(row % a.nx), (int)(row / a.nx), a.nx, r % rot);
        if (WIDE) a.y64[r][out] = (double)t;
        else a.y[r][out] = (T)t;
      }
    }
  }
}

template <class T, bool WIDE>
static void spmm_dispatch(int max_rhs, const CsrMultiArgs<T>& a0, const CsrMultiArgs<T>* arr, const int* starts,
                          int n_grp, int blocks, hipStream_t s) {
  PAT_CHECK_ARG(max_rhs >= 1 && max_rhs <= kMaxRhs, "bad right-hand side count");
  if (max_rhs <= 1)
    hipLaunchKernelGGL((csr_spmm_kernel<T, WIDE, 1>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n_grp);
  else if (max_rhs <= 2)
    hipLaunchKernelGGL((csr_spmm_kernel<T, WIDE, 2>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n_grp);
  else if (max_rhs <= 4)
    hipLaunchKernelGGL((csr_spmm_kernel<T, WIDE, 4>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n_grp);
  else
    hipLaunchKernelGGL((csr_spmm_kernel<T, WIDE, kMaxRhs>), dim3(blocks), dim3(256), 0, s, a0, arr, starts, n_grp);
}

template <class T>
void launch_csr_spmm_batched(const CsrMultiArgs<T>* arr, const int* starts, int n_grp, int total_blocks,
                             hipStream_t s, bool wide, int max_rhs) {
  if (total_blocks <= 0) return;
  CsrMultiArgs<T> dummy{};
  if (wide) spmm_dispatch<T, true>(max_rhs, dummy, arr, starts, n_grp, total_blocks, s);
  else spmm_dispatch<T, false>(max_rhs, dummy, arr, starts, n_grp, total_blocks, s);
  PAT_HIP(hipGetLastError());
}

template <class T>
void launch_csr_spmm(const CsrMultiArgs<T>& a, hipStream_t s, bool wide) {
  const int blocks = (int)((a.n_rows + 3) / 4);
  if (blocks <= 0) return;
  if (wide) spmm_dispatch<T, true>(a.nrhs, a, nullptr, nullptr, 1, blocks, s);
  else spmm_dispatch<T, false>(a.nrhs, a, nullptr, nullptr, 1, blocks, s);
  PAT_HIP(hipGetLastError());
}

template void launch_csr_spmm<float>(const CsrMultiArgs<float>&, hipStream_t, bool);
template void launch_csr_spmm<double>(const CsrMultiArgs<double>&, hipStream_t, bool);

template void launch_csr_spmm_batched<float>(const CsrMultiArgs<float>*, const int*, int, int, hipStream_t, bool, int);
template void launch_csr_spmm_batched<double>(const CsrMultiArgs<double>*, const int*, int, int, hipStream_t, bool, int);

template <class T>
void launch_csr_spmv(const CsrArgs<T>& a, hipStream_t s) {
  const int blocks = (int)((a.n_rows + 3) / 4);
  if (blocks <= 0) return;
  hipLaunchKernelGGL((csr_spmv_kernel<T, false>), dim3(blocks), dim3(256), 0, s, a,
                     (const CsrArgs<T>*)nullptr, (const int*)nullptr, 1);
  PAT_HIP(hipGetLastError());
}

template <class T>
void launch_csr_spmv_batched(const CsrArgs<T>* arr, const int* starts, int n_inst, int total_blocks,
                             hipStream_t s, bool wide) {
  if (total_blocks <= 0) return;
  CsrArgs<T> dummy{};
  if (wide)
    hipLaunchKernelGGL((csr_spmv_kernel<T, true>), dim3(total_blocks), dim3(256), 0, s, dummy, arr,
                       starts, n_inst);
  else
    hipLaunchKernelGGL((csr_spmv_kernel<T, false>), dim3(total_blocks), dim3(256), 0, s, dummy, arr,
                       starts, n_inst);
  PAT_HIP(hipGetLastError());
}

// One block per pixel tile (NT / 64 waves): stage the tile's input windows of
// every slot in LDS, then LPR lanes per matrix row with the gathers served by
// LDS. Rows outside the image (ragged tiles) store nothing. The workgroup size
// (4, 8 or 16 waves) and LPR are launch choices (the autotuner's): large
// staged windows leave room for one workgroup per CU, where 16 waves keep
// enough loads in flight; the waves of a workgroup share one copy of the
// windows.
template <class T, bool WIDE, int R, int NT, int LPR>
__global__ __launch_bounds__(NT) void csr_tiled_kernel(CsrMultiArgs<T> a0, const CsrMultiArgs<T>* __restrict__ arr,
                                                       const int* __restrict__ starts, int n_grp) {
  constexpr int NW = NT / 64;
  constexpr int RPW = 64 / LPR;  // rows a wave works on at once
  extern __shared__ char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  int blk = blockIdx.x;
  const CsrMultiArgs<T>* ap = &a0;
  if (arr) {
    int lo = 0, hi = n_grp;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (starts[mid] <= blk) lo = mid; else hi = mid;
    }
    ap = arr + lo;
    blk -= starts[lo];
  }
  const CsrMultiArgs<T>& a = *ap;
  const int nr = a.nrhs;
  const int side = a.side;
  const int stride = a.lds_stride;
  const int tx = blk % a.tiles_x, ty = blk / a.tiles_x;
  const int n_det = a.n_det, n_t = a.n_t, nx = a.nx, ny = a.ny;
  const int4* __restrict__ win = a.win + (int64_t)blk * n_det;
  // staging: one thread per (slot, detector) window, four loads in flight
  const int n_pairs = (R == 1 ? 1 : nr) * n_det;
  for (int p = threadIdx.x; p < n_pairs; p += NT) {
    const int r = R == 1 ? 0 : p / n_det, d = R == 1 ? p : p - r * n_det;
    const int4 w = win[d];
    const gptr<const T> src = as_global(a.x[r]) + (int64_t)d * n_t + w.x;
    T* dst = lds + r * stride + w.z;
    int i = 0;
    for (; i + 4 <= w.y; i += 4) {
      const T v0 = src[i], v1 = src[i + 1], v2 = src[i + 2], v3 = src[i + 3];
      dst[i] = v0;
      dst[i + 1] = v1;
      dst[i + 2] = v2;
      dst[i + 3] = v3;
    }
    for (; i < w.y; ++i) dst[i] = src[i];
  }
  __syncthreads();
  // Rows: LPR lanes per row (16 or 64), so a wave works on RPW rows at once
  // (batch b of wave w holds rows rr0 + RPW b + 0..RPW-1); with 16 lanes a
  // row reduces over its lanes by DPP moves instead of LDS permutes. Short
  // rows (quarter-turn storage, about 240 entries) favour 16 lanes, long rows
  // 64. Entry indices fit 32 bits (the matrix is limited to 2^31 - 512
  // entries).
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int grp = lane / LPR, gl = lane % LPR;
  const int rows = side * side, per_wave = (rows + NW - 1) / NW;
  const int rr0 = wave * per_wave, rr1 = min(rows, rr0 + per_wave);
  const int n_batch = rr1 > rr0 ? (rr1 - rr0 + RPW - 1) / RPW : 0;
  using Acc = typename std::conditional<WIDE, double, T>::type;
  const gptr<const int64_t> rowp = as_global(a.ptr);
  const gptr<const uint16_t> lcol = as_global(a.lcol);
  const gptr<const T> val = as_global(a.val);
  // row of this lane's group in batch b: [e0, e1) (empty outside the tile's
  // rows or the image)
  auto row_range = [&](int b, int& e0, int& e1) {
    const int rr = rr0 + RPW * b + grp;
    e0 = e1 = 0;
    if (rr < rr1) {
      const int i = tx * side + rr % side, j = ty * side + rr / side;
      if (i < nx && j < ny) {
        const int64_t pix = (int64_t)j * nx + i;
        e0 = (int)rowp[pix];
        e1 = (int)rowp[pix + 1];
      }
    }
  };
  // Software pipeline: a group of G LPR-entry blocks per row (block-
  // aligned) is loaded one step ahead: the row's next group, the row's last
  // group again (marked stale, all lanes masked) once the row is done and
  // other rows of the batch go on, or the next batch's first group. Every
  // group starts at or before its row's end and spans G LPR <= 256 entries,
  // so its loads stay within the 256 entries of slack after the matrix.
  // Lanes outside [e0, e1) contribute a zero product.
  //
  // Entries per lane: runs of K consecutive entries, K = 16 bytes of values
  // (2 doubles or 4 floats): one 16-byte value load and one 4- or 8-byte
  // offset load per run, consecutive lanes on consecutive runs, so a wave's
  // value load covers 1 KB contiguous. Lane gl's entry u of a group is
  // base + K gl + K LPR (u / K) + u % K. With 8-byte values, 16-lane rows and
  // four slots a lane takes G = 8 entries per step (more bytes in flight per
  // wave at no loss of occupancy), else 4; a lane's entries and the order of
  // its additions are the same for both (an 8-entry step adds its products as
  // two 4-entry steps would), so G may follow the slot count. Group bases are
  // multiples of LPR and the arrays start 256-byte aligned, so every wide
  // load is aligned.
  constexpr int K = 16 / (int)sizeof(T);
  constexpr int G = (sizeof(T) == 8 && LPR == 16 && R == 4) ? 8 : 4;
  static_assert(G % K == 0 && (G == 4 || G == 8) && G * LPR <= kCsrSlack, "a group must stay within the slack");
  typedef T T2 __attribute__((ext_vector_type(2)));
  typedef T T4 __attribute__((ext_vector_type(4)));
  int c[G];  // 16-bit offsets held unpacked (packing would wait on the loads)
  T v[G];
  // Lanes whose run starts at or after their row's end (hi) load the row's
  // last run instead (or the group's first when the row has nothing there):
  // the values are masked out of the sums either way, and the loads stay
  // unconditional and in flight together but touch no cache line beyond
  // the row's own.
  auto load_group = [&](int base, int hi, int* cc, T* vv) {
    const int last = max(base, (hi - 1) & ~(K - 1));
#pragma unroll
    for (int q = 0; q < G / K; ++q) {
      const int e = min(base + K * gl + K * LPR * q, last);
      if constexpr (K == 2) {
        const uint32_t w = __builtin_nontemporal_load((gptr<const uint32_t>)(lcol + e));
        cc[2 * q] = (int)(w & 0xffffu);
        cc[2 * q + 1] = (int)(w >> 16);
        const T2 p = __builtin_nontemporal_load((gptr<const T2>)(val + e));
        vv[2 * q] = p.x;
        vv[2 * q + 1] = p.y;
      } else {
        const uint64_t w = __builtin_nontemporal_load((gptr<const uint64_t>)(lcol + e));
#pragma unroll
        for (int t = 0; t < 4; ++t) cc[4 * q + t] = (int)((w >> (16 * t)) & 0xffffu);
        const T4 p = __builtin_nontemporal_load((gptr<const T4>)(val + e));
        vv[4 * q] = p.x;
        vv[4 * q + 1] = p.y;
        vv[4 * q + 2] = p.z;
        vv[4 * q + 3] = p.w;
      }
    }
  };
  if (n_batch > 0) {
    int e0, e1;
    row_range(0, e0, e1);
    int base = e0 & ~(LPR - 1);
    load_group(base, e1, c, v);
    for (int b = 0; b < n_batch; ++b) {
      const bool has_next = b + 1 < n_batch;
      int ne0 = 0, ne1 = 0;
      if (has_next) row_range(b + 1, ne0, ne1);
      // a row without entries stores an exact zero: in a pixel tile that no
      // arc reaches nothing is staged, and its masked lanes would multiply 0
      // by whatever the LDS holds (possibly a NaN)
      const bool row_empty = e0 == e1;
      // one accumulator per slot; each 4 entries of a lane add their products
      // as a fixed tree, so a slot's summation order does not depend on how
      // many slots the launch carries (batched and single solves agree
      // bitwise)
      Acc acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = Acc(0);
      bool stale = false;
      while (true) {
        const int nb = base + G * LPR;
        const bool more = !stale && nb < e1;
        const bool any = __any(more);
        const int next = any ? (more ? nb : base) : (has_next ? (ne0 & ~(LPR - 1)) : base);
        // the row end of the next step's entries: this row's while it has
        // more, the next batch's row, or none (a stale placeholder)
        const int nhi = any ? (more ? e1 : 0) : (has_next ? ne1 : 0);
        int cn[G];
        T vn[G];
        load_group(next, nhi, cn, vn);
        // every slot is computed (slots past nrhs read stale LDS and are not
        // stored): no per-slot branches between the LDS reads
        Acc vm[G];
        int cu[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int e = base + K * gl + K * LPR * (u / K) + u % K;
          const bool ok = !stale && e >= e0 && e < e1;
          vm[u] = ok ? (Acc)v[u] : Acc(0);
          cu[u] = ok ? c[u] : 0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T* x = lds + r * stride;
          Acc p[G / 2];
#pragma unroll
          for (int h = 0; h < G / 2; ++h) p[h] = fma(vm[2 * h + 1], (Acc)x[cu[2 * h + 1]], vm[2 * h] * (Acc)x[cu[2 * h]]);
#pragma unroll
          for (int h = 0; h < G / 2; h += 2) acc[r] += p[h] + p[h + 1];
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
          c[u] = cn[u];
          v[u] = vn[u];
        }
        if (!any) break;
        stale = !more;
        base = next;
      }
      const int rr = rr0 + RPW * b + grp;
      const int i = tx * side + rr % side, j = ty * side + rr / side;
      const bool store = gl == 0 && rr < rr1 && i < nx && j < ny;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (R == 1 || r < nr) {
          const Acc tot = LPR == 16 ? row16_sum(acc[r]) : group_sum<64>(acc[r]);
          const Acc sum = row_empty ? Acc(0) : tot;
          if (store) {
            const int64_t out = (R == 1 || a.rot <= 1) ? (int64_t)j * nx + i : quarter_turn(i, j, nx, r % a.rot);
            if (WIDE) a.y64[r][out] = (double)sum;
            else a.y[r][out] = (T)sum;
          }
        }
      }
      e0 = ne0;
      e1 = ne1;
      base = ne0 & ~(LPR - 1);
    }
  }
}

template <class T, bool WIDE, int R, int NT>
static void tiled_launch_nt(size_t shm, const CsrMultiArgs<T>& a0, const CsrMultiArgs<T>* arr, const int* starts,
                            int n_grp, int blocks, hipStream_t s, int lanes) {
  if (lanes == 64)
    hipLaunchKernelGGL((csr_tiled_kernel<T, WIDE, R, NT, 64>), dim3(blocks), dim3(NT), shm, s, a0, arr, starts, n_grp);
  else
    hipLaunchKernelGGL((csr_tiled_kernel<T, WIDE, R, NT, 16>), dim3(blocks), dim3(NT), shm, s, a0, arr, starts, n_grp);
}

template <class T, bool WIDE, int R>
static void tiled_launch(size_t shm, const CsrMultiArgs<T>& a0, const CsrMultiArgs<T>* arr, const int* starts,
                         int n_grp, int blocks, hipStream_t s, int waves, int lanes) {
  if (waves == 16) tiled_launch_nt<T, WIDE, R, 1024>(shm, a0, arr, starts, n_grp, blocks, s, lanes);
  else if (waves == 8) tiled_launch_nt<T, WIDE, R, 512>(shm, a0, arr, starts, n_grp, blocks, s, lanes);
  else tiled_launch_nt<T, WIDE, R, 256>(shm, a0, arr, starts, n_grp, blocks, s, lanes);
}

template <class T, bool WIDE>
static void tiled_dispatch(int max_rhs, const CsrMultiArgs<T>& a0, const CsrMultiArgs<T>* arr, const int* starts,
                           int n_grp, int blocks, size_t shm, hipStream_t s, int waves, int lanes) {
  PAT_CHECK_ARG(waves == 4 || waves == 8 || waves == 16, "tiled workgroups carry 4, 8 or 16 waves");
  PAT_CHECK_ARG(lanes == 16 || lanes == 64, "tiled rows take 16 or 64 lanes");
  PAT_CHECK_ARG(max_rhs >= 1 && max_rhs <= kMaxRhs, "bad right-hand side count");
  PAT_CHECK_ARG(shm <= (size_t)device_lds_per_block(), "staged windows exceed the LDS of a workgroup");
  if (max_rhs <= 1) tiled_launch<T, WIDE, 1>(shm, a0, arr, starts, n_grp, blocks, s, waves, lanes);
  else if (max_rhs <= 2) tiled_launch<T, WIDE, 2>(shm, a0, arr, starts, n_grp, blocks, s, waves, lanes);
  else if (max_rhs <= 4) tiled_launch<T, WIDE, 4>(shm, a0, arr, starts, n_grp, blocks, s, waves, lanes);
  else tiled_launch<T, WIDE, kMaxRhs>(shm, a0, arr, starts, n_grp, blocks, s, waves, lanes);
  PAT_HIP(hipGetLastError());
}

int device_lds_per_block() {
  static thread_local int cached_dev = -1, cached = 0;
  int dev = 0;
  PAT_HIP(hipGetDevice(&dev));
  if (dev != cached_dev) {
    int v = 0;
    PAT_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    cached = v;
    cached_dev = dev;
  }
  return cached;
}

template <class T, bool WIDE, int R, int LPR>
static void raise_lds_l(size_t shm) {
  PAT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&csr_tiled_kernel<T, WIDE, R, 256, LPR>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  PAT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&csr_tiled_kernel<T, WIDE, R, 512, LPR>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  PAT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&csr_tiled_kernel<T, WIDE, R, 1024, LPR>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
}

template <class T, bool WIDE, int R>
static void raise_lds(size_t shm) {
  raise_lds_l<T, WIDE, R, 16>(shm);
  raise_lds_l<T, WIDE, R, 64>(shm);
}

template <class T>
void prepare_csr_tiled(int max_rhs, size_t shm) {
  if (shm <= 65536) return;
  PAT_CHECK_ARG(shm <= (size_t)device_lds_per_block(), "staged windows exceed the LDS of a workgroup");
  if (max_rhs <= 1) { raise_lds<T, false, 1>(shm); raise_lds<T, true, 1>(shm); }
  else if (max_rhs <= 2) { raise_lds<T, false, 2>(shm); raise_lds<T, true, 2>(shm); }
  else if (max_rhs <= 4) { raise_lds<T, false, 4>(shm); raise_lds<T, true, 4>(shm); }
  else { raise_lds<T, false, kMaxRhs>(shm); raise_lds<T, true, kMaxRhs>(shm); }
}

template <class T>
void launch_csr_tiled(const CsrMultiArgs<T>& a, hipStream_t s, bool wide, int waves, int lanes) {
  const int blocks = a.tiles_x * ((a.ny + a.side - 1) / a.side);
  if (blocks <= 0) return;
  // every slot of the kernel instance is staged (1, 2, 4 or kMaxRhs)
  const int r_inst = a.nrhs <= 2 ? a.nrhs : (a.nrhs <= 4 ? 4 : kMaxRhs);
  const size_t shm = sizeof(T) * (size_t)a.lds_stride * (size_t)r_inst;
  prepare_csr_tiled<T>(a.nrhs, shm);
  if (wide) tiled_dispatch<T, true>(a.nrhs, a, nullptr, nullptr, 1, blocks, shm, s, waves, lanes);
  else tiled_dispatch<T, false>(a.nrhs, a, nullptr, nullptr, 1, blocks, shm, s, waves, lanes);
}

template <class T>
void launch_csr_tiled_batched(const CsrMultiArgs<T>* arr, const int* starts, int n_grp, int total_blocks,
                              size_t shm, hipStream_t s, bool wide, int max_rhs, int waves, int lanes) {
  if (total_blocks <= 0) return;
  CsrMultiArgs<T> dummy{};
  if (wide) tiled_dispatch<T, true>(max_rhs, dummy, arr, starts, n_grp, total_blocks, shm, s, waves, lanes);
  else tiled_dispatch<T, false>(max_rhs, dummy, arr, starts, n_grp, total_blocks, shm, s, waves, lanes);
}

template void launch_csr_tiled<float>(const CsrMultiArgs<float>&, hipStream_t, bool, int, int);
template void launch_csr_tiled<double>(const CsrMultiArgs<double>&, hipStream_t, bool, int, int);
template void launch_csr_tiled_batched<float>(const CsrMultiArgs<float>*, const int*, int, int, size_t, hipStream_t,
                                              bool, int, int, int);
template void launch_csr_tiled_batched<double>(const CsrMultiArgs<double>*, const int*, int, int, size_t, hipStream_t,
                                               bool, int, int, int);
template void prepare_csr_tiled<float>(int, size_t);
template void prepare_csr_tiled<double>(int, size_t);

template void build_csr_adjoint<float>(pat_geometry_s*, hipStream_t);
template void build_csr_adjoint<double>(pat_geometry_s*, hipStream_t);
template void launch_csr_spmv<float>(const CsrArgs<float>&, hipStream_t);
template void launch_csr_spmv<double>(const CsrArgs<double>&, hipStream_t);
template void launch_csr_spmv_batched<float>(const CsrArgs<float>*, const int*, int, int, hipStream_t, bool);
template void launch_csr_spmv_batched<double>(const CsrArgs<double>*, const int*, int, int, hipStream_t, bool);

}  // namespace pat
