// Dual step of the regulariser B (arXiv:1707.02245, Algorithms 1 and 2: the
// r and s updates with the projections that are the proximal maps of the
// conjugate norms, Sec. 3.2), one pixel per thread, as a device function so
// that the solver can also run it inside the forward's launch (it reads only
// ubar and vbar, which the forward's dual data step also reads, and writes
// only r and s). Discretisation of grad and E as in pdhg.hip.
#pragma once

#include "pat_internal.hpp"

namespace pat {

__device__ __forceinline__ int find_inst_p(const int* __restrict__ starts, int n, int blk) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (starts[mid] <= blk) lo = mid; else hi = mid;
  }
  return lo;
}

template <class T>
__device__ __forceinline__ void project2(T& a, T& b, T rad) {
  // prox of the conjugate of rad ||.||_2: projection on the ball of radius rad
  const T n = sqrt(a * a + b * b);
  if (n > rad) {
    const T s = rad / n;
    a *= s;
    b *= s;
  }
}

// Pixels [256 blk, 256 blk + 256) of the instances' concatenated block
// ranges (starts: first block of each instance, n_inst entries).
template <class T>
__device__ __forceinline__ void reg_dual_block(const InstDev<T>* __restrict__ arr, const int* __restrict__ starts,
                                               int n_inst, int blk) {
  const int ii = find_inst_p(starts, n_inst, blk);
  const InstDev<T> a = arr[ii];
  blk -= starts[ii];
  const int nx = a.nx, ny = a.ny;
  const int64_t N = (int64_t)nx * ny;
  const int64_t p = (int64_t)blk * 256 + threadIdx.x;
  if (p >= N || a.kind == PAT_REG_TIKHONOV || a.kind == PAT_REG_WAVELET) return;
  const int i = (int)(p % nx), j = (int)(p / nx);
  const int P = nx + 2;
  const T* __restrict__ ub = a.ubar_pad + (int64_t)(j + 1) * P + (i + 1);
  const bool ax = i < nx - 1, ay = j < ny - 1;
  const T c = ub[0];
  const T gx = ax ? ub[1] - c : T(0);
  const T gy = ay ? ub[P] - c : T(0);
  T rx = a.r[p], ry = a.r[N + p];
  // the accelerated schedule scales every dual step of the iteration
  const T dm = a.mult ? (T)a.mult[0] : T(1);
  const T sr = a.mult ? a.sigma_r[p] * dm : a.sigma_r[p];
  if (a.kind == PAT_REG_TV) {
    rx += sr * gx;
    ry += sr * gy;
    project2(rx, ry, a.lam);
  } else if (a.kind == PAT_REG_DTV) {
    const T d11 = a.dmat[p], d12 = a.dmat[N + p], d22 = a.dmat[2 * N + p];
    rx += sr * (d11 * gx + d12 * gy);
    ry += sr * (d12 * gx + d22 * gy);
    project2(rx, ry, a.lam);
  } else {  // TGV: r <- P_alpha1(r + sigma (grad ubar - vbar)), s <- P_alpha0(s + sigma E vbar)
    const T* __restrict__ vbx = a.vbar;
    const T* __restrict__ vby = a.vbar + N;
    const T vx = vbx[p], vy = vby[p];
    rx += sr * (gx - vx);
    ry += sr * (gy - vy);
    project2(rx, ry, a.lam);
    const bool bx = i >= 1, by = j >= 1;
    const T vx_l = bx ? vbx[p - 1] : T(0), vy_l = bx ? vby[p - 1] : T(0);
    const T vx_d = by ? vbx[p - nx] : T(0), vy_d = by ? vby[p - nx] : T(0);
    const T e1 = (ax ? vx : T(0)) - vx_l;
    const T e4 = (ay ? vy : T(0)) - vy_d;
    const T e2 = T(0.5) * (((ay ? vx : T(0)) - vx_d) + ((ax ? vy : T(0)) - vy_l));
    const T ss = a.mult ? a.sigma_s[p] * dm : a.sigma_s[p];
    T s1 = a.s[p] + ss * e1, s2 = a.s[N + p] + ss * e2, s4 = a.s[2 * N + p] + ss * e4;
    const T n = sqrt(s1 * s1 + T(2) * s2 * s2 + s4 * s4);
    if (n > a.alpha0) {
      const T f = a.alpha0 / n;
      s1 *= f;
      s2 *= f;
      s4 *= f;
    }
    a.s[p] = s1;
    a.s[N + p] = s2;
    a.s[2 * N + p] = s4;
  }
  a.r[p] = rx;
  a.r[N + p] = ry;
}

}  // namespace pat
