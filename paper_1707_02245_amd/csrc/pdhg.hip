// Pixel kernels of preconditioned PDHGM (arXiv:1707.02245, Algorithms 1 and 2;
// proximal maps of Sec. 3.2; step sizes of Sec. 3.3.2; gap of Sec. 3.3.3).
//
// Discretisation (Sec. 3.3.1, matrix versions of grad and E):
//   (dx+ w)_p = w_{p+x} - w_p if ix < nx-1 else 0          (same in y)
//   grad^T r   = -dx+^T rx - dy+^T ry
//   (dx- w)_p  = w_p [ix < nx-1] - w_{p-x} [ix >= 1]        (= -(dx+)^T w)
//   E v = [dx- vx, (dy- vx + dx- vy)/2, (dy- vx + dx- vy)/2, dy- vy]; the two
//   equal middle rows are stored once (s_xy) and counted twice in norms.
//   Directional TV: B = D grad with D = I - (1 - eta) xi xi^T per pixel.
//
// Each kernel handles one pixel per thread, reads its neighbours through the
// cache and writes only its own pixel, so no kernel races with itself. Work of
// many instances shares one launch (block ranges per instance).

#include "pat_internal.hpp"
#include "reg_dual.hpp"

namespace pat {

// ------------------------------------------------------------------ dual step of B

template <class T>
__global__ __launch_bounds__(256) void reg_dual_kernel(const InstDev<T>* __restrict__ arr,
                                                       const int* __restrict__ starts, int n_inst) {
  reg_dual_block<T>(arr, starts, n_inst, blockIdx.x);
}

template <class T>
void launch_reg_dual(const Launch<T>& L, hipStream_t s) {
  if (L.pix_total <= 0) return;
  hipLaunchKernelGGL(reg_dual_kernel<T>, dim3(L.pix_total), dim3(256), 0, s,
                     ptr<InstDev<T>>(L.inst), ptr<int>(L.pix_start), L.n);
  PAT_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ primal step

// (B^T r)_p for TV/TGV (B = grad) and DTV (B = D grad; D symmetric), in
// arithmetic type A (the element type, or FP64 for the gap's dual residual).
template <class T, class A = T>
__device__ __forceinline__ A bt_r(const InstDev<T>& a, int64_t p, int i, int j, int64_t N) {
  const int nx = a.nx, ny = a.ny;
  const bool ax = i < nx - 1, ay = j < ny - 1, bx = i >= 1, by = j >= 1;
  const T* __restrict__ rx = a.r;
  const T* __restrict__ ry = a.r + N;
  if (a.kind == PAT_REG_DTV) {
    const T* __restrict__ D = a.dmat;
    auto w1 = [&](int64_t q) { return (A)D[q] * (A)rx[q] + (A)D[N + q] * (A)ry[q]; };
    auto w2 = [&](int64_t q) { return (A)D[N + q] * (A)rx[q] + (A)D[2 * N + q] * (A)ry[q]; };
    A t = A(0);
    if (ax) t -= w1(p);
    if (bx) t += w1(p - 1);
    if (ay) t -= w2(p);
    if (by) t += w2(p - nx);
    return t;
  }
  A t = A(0);
  if (ax) t -= (A)rx[p];
  if (bx) t += (A)rx[p - 1];
  if (ay) t -= (A)ry[p];
  if (by) t += (A)ry[p - nx];
  return t;
}

template <class T, bool CHECK>
__global__ __launch_bounds__(256) void primal_kernel(const InstDev<T>* __restrict__ arr,
                                                     const int* __restrict__ starts, int n_inst) {
  int blk = blockIdx.x;
  const int ii = find_inst_p(starts, n_inst, blk);
  const InstDev<T> a = arr[ii];
  blk -= starts[ii];
  const int nx = a.nx, ny = a.ny;
  const int64_t N = (int64_t)nx * ny;
  const int64_t p = (int64_t)blk * 256 + threadIdx.x;
  double kty = 0.0, du2 = 0.0, u2 = 0.0;
  if (p < N) {
    const int i = (int)(p % nx), j = (int)(p / nx);
    T atq = T(0);
    for (int gi = 0; gi < a.n_groups; ++gi) atq += a.atq_part[gi * N + p];
    const T u_old = a.u[p];
    // the accelerated schedule scales every primal step of the iteration and
    // sets its extrapolation
    const T pm = a.mult ? (T)a.mult[1] : T(1);
    const T th = a.mult ? (T)a.mult[2] : a.theta_ex;
    const T tau = a.mult ? a.tau_u[p] * pm : a.tau_u[p];
    T un;
    // the gap's dual residual K^T y: FP64 A^T q when available
    double atq_d = (double)atq;
    if (CHECK && a.atq64) {
      atq_d = 0.0;
      for (int gi = 0; gi < a.n_groups; ++gi) atq_d += a.atq64[gi * N + p];
    }
    if (a.kind == PAT_REG_TIKHONOV) {
      // u <- prox_{tau G}(u - tau A^T q), G = lam/2 ||u||^2
      un = (u_old - tau * atq) / (T(1) + tau * a.lam);
      if (CHECK) kty = atq_d * atq_d;
    } else if (a.kind == PAT_REG_WAVELET) {
      // B^T r = W^T r, synthesised after the dual step of this iteration
      un = u_old - tau * (atq + a.wtr[p]);
      if (CHECK) kty = fabs(atq_d + (a.wtr64 ? a.wtr64[p] : (double)a.wtr[p]));
    } else {
      const T gdir = atq + bt_r(a, p, i, j, N);
      un = u_old - tau * gdir;
      if (CHECK) kty = fabs(atq_d + bt_r<T, double>(a, p, i, j, N));
    }
    a.u[p] = un;
    const T ubar = un + th * (un - u_old);
    const int P = nx + 2;
    a.ubar_pad[(int64_t)(j + 1) * P + (i + 1)] = ubar;
    if (CHECK) {
      du2 = (double)(un - u_old) * (double)(un - u_old);
      u2 = (double)u_old * (double)u_old;
      a.upad_gap[(int64_t)(j + 1) * P + (i + 1)] = un;
    }
    if (a.rot_slots == 4) {
      // the quarter-turn forward's copies: slot t holds the image turned by t
      // quarter turns, so this pixel's value lands where t turns bring it here
      const int64_t PP = (int64_t)P * (ny + 2);
#pragma unroll
      for (int t = 1; t < 4; ++t) {
        int x, y;
        quarter_turn_xy(i, j, nx, (4 - t) & 3, x, y);
        const int64_t o = t * PP + (int64_t)(y + 1) * P + (x + 1);
        a.ubar_pad[o] = ubar;
        if (CHECK) a.upad_gap[o] = un;
      }
    }
    if (a.kind == PAT_REG_TGV) {
      // v <- v - tau_v (E^T s - r); (E^T s)_x = -dx+ sxx - dy+ sxy, (E^T s)_y = -dx+ sxy - dy+ syy
      const bool ax = i < nx - 1, ay = j < ny - 1;
      const T* __restrict__ sxx = a.s;
      const T* __restrict__ sxy = a.s + N;
      const T* __restrict__ syy = a.s + 2 * N;
      const T c_xx = sxx[p], c_xy = sxy[p], c_yy = syy[p];
      const T dx_xx = ax ? sxx[p + 1] - c_xx : T(0);
      const T dy_xy = ay ? sxy[p + nx] - c_xy : T(0);
      const T dx_xy = ax ? sxy[p + 1] - c_xy : T(0);
      const T dy_yy = ay ? syy[p + nx] - c_yy : T(0);
      const T gvx = -dx_xx - dy_xy - a.r[p];
      const T gvy = -dx_xy - dy_yy - a.r[N + p];
      const T tv = a.mult ? a.tau_v[p] * pm : a.tau_v[p];
      const T vx = a.v[p], vy = a.v[N + p];
      const T vxn = vx - tv * gvx, vyn = vy - tv * gvy;
      a.v[p] = vxn;
      a.v[N + p] = vyn;
      a.vbar[p] = vxn + th * (vxn - vx);
      a.vbar[N + p] = vyn + th * (vyn - vy);
      if (CHECK) {
        const double ex = -((ax ? (double)sxx[p + 1] : (double)c_xx) - (double)c_xx) -
                          ((ay ? (double)sxy[p + nx] : (double)c_xy) - (double)c_xy) - (double)a.r[p];
        const double ey = -((ax ? (double)sxy[p + 1] : (double)c_xy) - (double)c_xy) -
                          ((ay ? (double)syy[p + nx] : (double)c_yy) - (double)c_yy) - (double)a.r[N + p];
        kty += fabs(ex) + fabs(ey);
      }
    }
  }
  if (CHECK) {
    __shared__ double lds[8];
    const double s0 = block_sum<256>(kty, lds);
    const double s1 = block_sum<256>(du2, lds);
    const double s2 = block_sum<256>(u2, lds);
    if (threadIdx.x == 0) {
      a.red[GAP_KTY * (int64_t)a.red_stride + blk] = s0;
      a.red[GAP_DU2 * (int64_t)a.red_stride + blk] = s1;
      a.red[GAP_U2 * (int64_t)a.red_stride + blk] = s2;
    }
  }
}

template <class T>
void launch_primal(const Launch<T>& L, bool check, hipStream_t s) {
  if (L.pix_total <= 0) return;
  if (check)
    hipLaunchKernelGGL((primal_kernel<T, true>), dim3(L.pix_total), dim3(256), 0, s,
                       ptr<InstDev<T>>(L.inst), ptr<int>(L.pix_start), L.n);
  else
    hipLaunchKernelGGL((primal_kernel<T, false>), dim3(L.pix_total), dim3(256), 0, s,
                       ptr<InstDev<T>>(L.inst), ptr<int>(L.pix_start), L.n);
  PAT_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ accelerated schedule

// cur[i] = sched[i][t] for every instance i (3 doubles each): the step
// multipliers of iteration t of the current block, read by the iteration's
// forward, regulariser and primal launches.
__global__ __launch_bounds__(256) void accel_step_kernel(const double* __restrict__ sched,
                                                         double* __restrict__ cur, int n_inst,
                                                         int block, int t) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= 3 * n_inst) return;
  const int i = e / 3, k = e % 3;
  cur[e] = sched[((int64_t)i * block + t) * 3 + k];
}

void launch_accel_step(const double* sched, double* cur, int n_inst, int block, int t, hipStream_t s) {
  const int blocks = (3 * n_inst + 255) / 256;
  hipLaunchKernelGGL(accel_step_kernel, dim3(blocks), dim3(256), 0, s, sched, cur, n_inst, block, t);
  PAT_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ gap: regulariser value

template <class T>
__global__ __launch_bounds__(256) void gap_reg_kernel(const InstDev<T>* __restrict__ arr,
                                                      const int* __restrict__ starts, int n_inst) {
  int blk = blockIdx.x;
  const int ii = find_inst_p(starts, n_inst, blk);
  const InstDev<T> a = arr[ii];
  // the wavelet value lam ||W u||_1 comes from the transform's own gap pass
  if (a.kind == PAT_REG_WAVELET) return;
  blk -= starts[ii];
  const int nx = a.nx, ny = a.ny;
  const int64_t N = (int64_t)nx * ny;
  const int64_t p = (int64_t)blk * 256 + threadIdx.x;
  double val = 0.0;
  if (p < N) {
    const int i = (int)(p % nx), j = (int)(p / nx);
    const bool ax = i < nx - 1, ay = j < ny - 1;
    const T* __restrict__ u = a.u;
    const double c = u[p];
    if (a.kind == PAT_REG_TIKHONOV) {
      val = 0.5 * (double)a.lam * c * c;
    } else {
      double gx = ax ? (double)u[p + 1] - c : 0.0;
      double gy = ay ? (double)u[p + nx] - c : 0.0;
      if (a.kind == PAT_REG_DTV) {
        const double d11 = a.dmat[p], d12 = a.dmat[N + p], d22 = a.dmat[2 * N + p];
        const double bx = d11 * gx + d12 * gy, by = d12 * gx + d22 * gy;
        gx = bx;
        gy = by;
      }
      if (a.kind == PAT_REG_TGV) {
        const T* __restrict__ vx = a.v;
        const T* __restrict__ vy = a.v + N;
        const double cx = vx[p], cy = vy[p];
        gx -= cx;
        gy -= cy;
        const bool bx = i >= 1, by = j >= 1;
        const double vx_l = bx ? (double)vx[p - 1] : 0.0, vy_l = bx ? (double)vy[p - 1] : 0.0;
        const double vx_d = by ? (double)vx[p - nx] : 0.0, vy_d = by ? (double)vy[p - nx] : 0.0;
        const double e1 = (ax ? cx : 0.0) - vx_l;
        const double e4 = (ay ? cy : 0.0) - vy_d;
        const double e2 = 0.5 * (((ay ? cx : 0.0) - vx_d) + ((ax ? cy : 0.0) - vy_l));
        val = (double)a.alpha0 * sqrt(e1 * e1 + 2.0 * e2 * e2 + e4 * e4);
      }
      val += (double)a.lam * sqrt(gx * gx + gy * gy);
    }
  }
  __shared__ double lds[8];
  const double s0 = block_sum<256>(val, lds);
  if (threadIdx.x == 0) a.red[GAP_REG * (int64_t)a.red_stride + blk] = s0;
}

template <class T>
void launch_gap_reg(const Launch<T>& L, hipStream_t s) {
  if (L.pix_total <= 0) return;
  hipLaunchKernelGGL(gap_reg_kernel<T>, dim3(L.pix_total), dim3(256), 0, s,
                     ptr<InstDev<T>>(L.inst), ptr<int>(L.pix_start), L.n);
  PAT_HIP(hipGetLastError());
}

// One workgroup per instance sums every slot in a fixed order.
__global__ __launch_bounds__(256) void gap_finish_kernel(const GapFinishArgs* __restrict__ args,
                                                         double* __restrict__ out_base) {
  const GapFinishArgs a = args[blockIdx.x];
  double* out = out_base + (int64_t)blockIdx.x * GAP_NSLOTS;
  __shared__ double lds[8];
  for (int slot = 0; slot < GAP_NSLOTS; ++slot) {
    const int cnt = (slot == GAP_DATA || slot == GAP_FSTAR) ? a.n_fwd : (slot == GAP_REG ? a.n_reg : a.n_pix);
    double v = 0.0;
    for (int b = threadIdx.x; b < cnt; b += 256) v += a.red[slot * (int64_t)a.stride + b];
    const double s = block_sum<256>(v, lds);
    if (threadIdx.x == 0) out[slot] = s;
  }
}

void launch_gap_finish(const GapFinishArgs* args, int n_inst, double* out, hipStream_t s) {
  if (n_inst <= 0) return;
  hipLaunchKernelGGL(gap_finish_kernel, dim3(n_inst), dim3(256), 0, s, args, out);
  PAT_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ preconditioner

// Closed-form absolute row and column sums of the regulariser part of the
// stacked operator K; colsum_a holds A^T 1 (A >= 0).
template <class T>
__global__ __launch_bounds__(256) void precond_pix_kernel(int kind, int nx, int ny,
                                                          const T* __restrict__ colsum_a,
                                                          const T* __restrict__ D,
                                                          T* __restrict__ sigma_r,
                                                          T* __restrict__ sigma_s,
                                                          T* __restrict__ tau_u,
                                                          T* __restrict__ tau_v) {
  const int64_t N = (int64_t)nx * ny;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int i = (int)(p % nx), j = (int)(p / nx);
  const double ax = i < nx - 1, ay = j < ny - 1, bx = i >= 1, by = j >= 1;
  const double ca = colsum_a[p];
  auto inv_or_one = [](double s) { return s > 0.0 ? 1.0 / s : 1.0; };
  if (kind == PAT_REG_TIKHONOV) {
    tau_u[p] = (T)inv_or_one(ca);
    return;
  }
  if (kind == PAT_REG_WAVELET) {
    // W^T W = I: ||W x|| = ||x|| stands in for W's column sums, so 1 is added
    // to A's, and W's rows take sigma = 1 (four coefficients per pixel)
    tau_u[p] = (T)(1.0 / (ca + 1.0));
#pragma unroll
    for (int k = 0; k < 4; ++k) sigma_r[k * N + p] = T(1);
    return;
  }
  if (kind == PAT_REG_TV) {
    // rows of grad: |-1| + |+1| where the difference exists
    sigma_r[p] = (T)fmin(inv_or_one(2.0 * ax), inv_or_one(2.0 * ay));
    tau_u[p] = (T)(1.0 / (ca + (ax + bx) + (ay + by)));
  } else if (kind == PAT_REG_DTV) {
    const double d11 = D[p], d12 = D[N + p], d22 = D[2 * N + p];
    const double row1 = fabs(d11 * ax + d12 * ay) + fabs(d11) * ax + fabs(d12) * ay;
    const double row2 = fabs(d12 * ax + d22 * ay) + fabs(d12) * ax + fabs(d22) * ay;
    sigma_r[p] = (T)fmin(inv_or_one(row1), inv_or_one(row2));
    double col = fabs(d11 * ax + d12 * ay) + fabs(d12 * ax + d22 * ay);
    if (bx) col += fabs((double)D[p - 1]) + fabs((double)D[N + p - 1]);
    if (by) col += fabs((double)D[N + p - nx]) + fabs((double)D[2 * N + p - nx]);
    tau_u[p] = (T)(1.0 / (ca + col));
  } else {  // TGV
    sigma_r[p] = (T)fmin(1.0 / (2.0 * ax + 1.0), 1.0 / (2.0 * ay + 1.0));
    // rows of E: dx- vx (ax + bx), the two middle rows (ax+bx+ay+by)/2, dy- vy (ay + by)
    const double ex = ax + bx, ey = ay + by;
    sigma_s[p] = (T)(1.0 / fmax(fmax(ex, ey), 0.5 * (ex + ey)));
    tau_u[p] = (T)(1.0 / (ca + ex + ey));
    // columns of v: -I (1), E: dx- column 2ax, two middle rows 2 * (1/2) * 2ay, ...
    tau_v[p] = (T)(1.0 / (1.0 + 2.0 * ax + 2.0 * ay));
  }
}

template <class T>
void launch_precond_pix(int reg_kind, int nx, int ny, const T* colsum_a, const T* dmat,
                        T* sigma_r, T* sigma_s, T* tau_u, T* tau_v, hipStream_t s) {
  const int64_t N = (int64_t)nx * ny;
  hipLaunchKernelGGL(precond_pix_kernel<T>, dim3(pix_blocks(N)), dim3(256), 0, s, reg_kind, nx, ny,
                     colsum_a, dmat, sigma_r, sigma_s, tau_u, tau_v);
  PAT_HIP(hipGetLastError());
}

// D = I - (1 - eta) xi xi^T, xi = (-sin theta, cos theta)
template <class T>
__global__ __launch_bounds__(256) void dmat_kernel(const T* __restrict__ theta, T eta,
                                                   T* __restrict__ D, int64_t N) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= N) return;
  double sn, cs;
  sincos((double)theta[p], &sn, &cs);
  const double xx = -sn, xy = cs, g = 1.0 - (double)eta;
  D[p] = (T)(1.0 - g * xx * xx);
  D[N + p] = (T)(-g * xx * xy);
  D[2 * N + p] = (T)(1.0 - g * xy * xy);
}

template <class T>
void launch_dmat(const T* theta, T eta, T* dmat, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(dmat_kernel<T>, dim3(pix_blocks(n)), dim3(256), 0, s, theta, eta, dmat, n);
  PAT_HIP(hipGetLastError());
}

template <class T>
__global__ __launch_bounds__(256) void fill_kernel(T* __restrict__ p, T v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <class T>
void launch_fill(T* p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_kernel<T>, dim3(blocks), dim3(256), 0, s, p, v, n);
  PAT_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ operator norms (BLOCK mode)

// z = B x: TV/DTV z = [2][N]; TGV z = [5][N] = (grad xu - xv, e1, e2, e4) of E xv.
template <class T>
__global__ __launch_bounds__(256) void reg_apply_kernel(int kind, int nx, int ny,
                                                        const T* __restrict__ D,
                                                        const T* __restrict__ xu,
                                                        const T* __restrict__ xv,
                                                        T* __restrict__ z) {
  const int64_t N = (int64_t)nx * ny;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int i = (int)(p % nx), j = (int)(p / nx);
  const bool ax = i < nx - 1, ay = j < ny - 1, bx = i >= 1, by = j >= 1;
  const T c = xu[p];
  T gx = ax ? xu[p + 1] - c : T(0), gy = ay ? xu[p + nx] - c : T(0);
  if (kind == PAT_REG_DTV) {
    const T d11 = D[p], d12 = D[N + p], d22 = D[2 * N + p];
    const T tx = d11 * gx + d12 * gy, ty = d12 * gx + d22 * gy;
    gx = tx;
    gy = ty;
  }
  if (kind == PAT_REG_TGV) {
    const T* vx = xv;
    const T* vy = xv + N;
    const T cx = vx[p], cy = vy[p];
    gx -= cx;
    gy -= cy;
    const T vx_l = bx ? vx[p - 1] : T(0), vy_l = bx ? vy[p - 1] : T(0);
    const T vx_d = by ? vx[p - nx] : T(0), vy_d = by ? vy[p - nx] : T(0);
    z[2 * N + p] = (ax ? cx : T(0)) - vx_l;
    z[3 * N + p] = T(0.5) * (((ay ? cx : T(0)) - vx_d) + ((ax ? cy : T(0)) - vy_l));
    z[4 * N + p] = (ay ? cy : T(0)) - vy_d;
  }
  z[p] = gx;
  z[N + p] = gy;
}

// y = B^T z with the four-row convention of E (middle row counted twice).
template <class T>
__global__ __launch_bounds__(256) void reg_apply_t_kernel(int kind, int nx, int ny,
                                                          const T* __restrict__ D,
                                                          const T* __restrict__ z,
                                                          T* __restrict__ yu, T* __restrict__ yv) {
  const int64_t N = (int64_t)nx * ny;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int i = (int)(p % nx), j = (int)(p / nx);
  const bool ax = i < nx - 1, ay = j < ny - 1, bx = i >= 1, by = j >= 1;
  const T* zx = z;
  const T* zy = z + N;
  T t = T(0);
  if (kind == PAT_REG_DTV) {
    auto w1 = [&](int64_t q) { return D[q] * zx[q] + D[N + q] * zy[q]; };
    auto w2 = [&](int64_t q) { return D[N + q] * zx[q] + D[2 * N + q] * zy[q]; };
    if (ax) t -= w1(p);
    if (bx) t += w1(p - 1);
    if (ay) t -= w2(p);
    if (by) t += w2(p - nx);
  } else {
    if (ax) t -= zx[p];
    if (bx) t += zx[p - 1];
    if (ay) t -= zy[p];
    if (by) t += zy[p - nx];
  }
  yu[p] = t;
  if (kind == PAT_REG_TGV) {
    const T* e1 = z + 2 * N;
    const T* e2 = z + 3 * N;
    const T* e4 = z + 4 * N;
    const T d_e1 = ax ? e1[p + 1] - e1[p] : T(0);
    const T dy_e2 = ay ? e2[p + nx] - e2[p] : T(0);
    const T dx_e2 = ax ? e2[p + 1] - e2[p] : T(0);
    const T d_e4 = ay ? e4[p + nx] - e4[p] : T(0);
    yv[p] = -d_e1 - dy_e2 - zx[p];
    yv[N + p] = -dx_e2 - d_e4 - zy[p];
  }
}

template <class T>
void launch_reg_apply(int reg_kind, int nx, int ny, const T* dmat, const T* xu, const T* xv,
                      T* z, hipStream_t s) {
  const int64_t N = (int64_t)nx * ny;
  hipLaunchKernelGGL(reg_apply_kernel<T>, dim3(pix_blocks(N)), dim3(256), 0, s, reg_kind, nx, ny,
                     dmat, xu, xv, z);
  PAT_HIP(hipGetLastError());
}

template <class T>
void launch_reg_apply_t(int reg_kind, int nx, int ny, const T* dmat, const T* z, T* yu, T* yv,
                        hipStream_t s) {
  const int64_t N = (int64_t)nx * ny;
  hipLaunchKernelGGL(reg_apply_t_kernel<T>, dim3(pix_blocks(N)), dim3(256), 0, s, reg_kind, nx,
                     ny, dmat, z, yu, yv);
  PAT_HIP(hipGetLastError());
}

// <a, b> in FP64: per-block partials then one ordered final block.
template <class T>
__global__ __launch_bounds__(256) void dot_partial_kernel(const T* __restrict__ a,
                                                          const T* __restrict__ b, int64_t n,
                                                          double* __restrict__ part) {
  double v = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v += (double)a[i] * (double)b[i];
  __shared__ double lds[8];
  const double s = block_sum<256>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sum_partial_kernel(const double* __restrict__ part, int n,
                                                          double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += part[i];
  __shared__ double lds[8];
  const double s = block_sum<256>(v, lds);
  if (threadIdx.x == 0) *out = s;
}

template <class T>
void launch_dot(const T* a, const T* b, int64_t n, double* partial, int n_part, double* out,
                hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel<T>, dim3(n_part), dim3(256), 0, s, a, b, n, partial);
  hipLaunchKernelGGL(sum_partial_kernel, dim3(1), dim3(256), 0, s, partial, n_part, out);
  PAT_HIP(hipGetLastError());
}

// y = x / sqrt(*denom) (power iteration normalisation; denom = ||x||^2)
template <class T>
__global__ __launch_bounds__(256) void scale_copy_kernel(T* __restrict__ y, const T* __restrict__ x,
                                                         const double* __restrict__ denom,
                                                         int64_t n) {
  const double d = *denom;
  const double f = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (T)((double)x[i] * f);
}

template <class T>
void launch_scale_copy(T* y, const T* x, const double* denom, int64_t n, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(scale_copy_kernel<T>, dim3(blocks), dim3(256), 0, s, y, x, denom, n);
  PAT_HIP(hipGetLastError());
}

// x_j = 1 + (j mod 5) / 4: deterministic start of the power iteration
template <class T>
__global__ __launch_bounds__(256) void pattern_kernel(T* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (T)(1.0 + (double)(i % 5) / 4.0);
}

template <class T>
void launch_pattern(T* x, int64_t n, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(pattern_kernel<T>, dim3(blocks), dim3(256), 0, s, x, n);
  PAT_HIP(hipGetLastError());
}

#define PAT_INST_PDHG(T)                                                                          \
  template void launch_reg_dual<T>(const Launch<T>&, hipStream_t);                                \
  template void launch_primal<T>(const Launch<T>&, bool, hipStream_t);                            \
  template void launch_gap_reg<T>(const Launch<T>&, hipStream_t);                                 \
  template void launch_precond_pix<T>(int, int, int, const T*, const T*, T*, T*, T*, T*,          \
                                      hipStream_t);                                               \
  template void launch_dmat<T>(const T*, T, T*, int64_t, hipStream_t);                            \
  template void launch_fill<T>(T*, T, int64_t, hipStream_t);                                      \
  template void launch_reg_apply<T>(int, int, int, const T*, const T*, const T*, T*, hipStream_t); \
  template void launch_reg_apply_t<T>(int, int, int, const T*, const T*, T*, T*, hipStream_t);     \
  template void launch_dot<T>(const T*, const T*, int64_t, double*, int, double*, hipStream_t);   \
  template void launch_scale_copy<T>(T*, const T*, const double*, int64_t, hipStream_t);        \
  template void launch_pattern<T>(T*, int64_t, hipStream_t);
PAT_INST_PDHG(float)
PAT_INST_PDHG(double)

}  // namespace pat
