// Calibrated forward model of the measured pressure and the preprocessing
// that turns measured pressure into data for the reconstruction
// (arXiv:1707.02245, Sec. 4.1 eq. FW_full; Sec. 4.2 eqs. FW_conv, f_rewrite,
// conv_thm2, deconv).
//
// With the circular-mean operator A of this library, (1/t) K u = 2 pi c A u
// (K the circular integral over the circle of radius c t), so the model is
//   p_d = s_d (A u)_d *_t pcal_d(. + tau_d),  s_d = 2 pi c |x_d - x_p|,
//   tau_d = |x_d - x_p| / c  (the calibration trace at retarded time),
// with the sampled convolution dt sum_j a_j b_{k-j}, and the preprocessing is
//   f_d = F^-1{ F{p_d} conj(D_d) / (|D_d|^2 + eps) } / s_d,
//   D_d = dt F{pcal_d} exp(i omega tau_d).
// Every transform is an L-point DFT (L the smallest power of two >= 2 n_t,
// zero padding), so the retarded shift is a phase ramp (band-limited and
// exact for whole samples) and the convolutions are linear within the
// n_t-sample window.
//
// Kernels: one workgroup per detector row transforms the zero-padded row in
// LDS (radix-2, decimation in time, FP64 complex), applies the row's
// spectrum and transforms back. The per-row spectra are computed once per
// calibration by the same kernel.

#include <cmath>
#include <memory>
#include <vector>

#include "pat_internal.hpp"

struct pat_calib_s {
  pat_geometry g = nullptr;
  int L = 0, log2L = 0;
  double xp = 0.0, yp = 0.0, eps = 0.0;
  pat::DevBuf hfwd, hdec;   // [n_det][L] complex (double2): s_d D_d and conj(D_d) / (|D_d|^2 + eps) / s_d
  pat::DevBuf au;           // [n_det][n_t] scratch (element type of g): A u of the pressure forward
  pat::DevBuf st;           // [n_det] {s_d, tau_d}
};

namespace pat {
namespace {

constexpr int kFftThreads = 256;
constexpr int kMaxFftLog2 = 12;  // L <= 4096 (64 KB of FP64 complex in LDS)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place radix-2 transform of x[0..L) in LDS (input in bit-reversed
// order): sign -1 forward, +1 inverse (unscaled).
__device__ void fft_lds(double2* x, int L, int log2L, double sign) {
  for (int s = 1; s <= log2L; ++s) {
    const int m = 1 << s, half = m >> 1;
    for (int b = threadIdx.x; b < (L >> 1); b += kFftThreads) {
      const int grp = b >> (s - 1), j = b & (half - 1);
      const int k = grp * m + j;
      double sn, cs;
      sincospi(sign * 2.0 * (double)j / (double)m, &sn, &cs);
      const double2 t = cmul(make_double2(cs, sn), x[k + half]);
      const double2 u = x[k];
      x[k] = make_double2(u.x + t.x, u.y + t.y);
      x[k + half] = make_double2(u.x - t.x, u.y - t.y);
    }
    __syncthreads();
  }
}

// In-place radix-2 transform of x[0..L) in LDS by decimation in frequency:
// natural-order input, output in bit-reversed order; sign as fft_lds.
__device__ void fft_lds_dif(double2* x, int L, int log2L, double sign) {
  for (int s = log2L; s >= 1; --s) {
    const int m = 1 << s, half = m >> 1;
    for (int b = threadIdx.x; b < (L >> 1); b += kFftThreads) {
      const int grp = b >> (s - 1), j = b & (half - 1);
      const int k = grp * m + j;
      double sn, cs;
      sincospi(sign * 2.0 * (double)j / (double)m, &sn, &cs);
      const double2 u = x[k], v = x[k + half];
      x[k] = make_double2(u.x + v.x, u.y + v.y);
      x[k + half] = cmul(make_double2(u.x - v.x, u.y - v.y), make_double2(cs, sn));
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int bitrev(int i, int log2L) {
  return (int)(__brev((unsigned)i) >> (32 - log2L));
}

// Load row d (n_t samples, zero padded to L) into LDS in bit-reversed order.
template <class T>
__device__ void load_row(double2* x, const T* __restrict__ src, int n_t, int L, int log2L) {
  for (int i = threadIdx.x; i < L; i += kFftThreads) {
    const double v = i < n_t ? (double)src[i] : 0.0;
    x[bitrev(i, log2L)] = make_double2(v, 0.0);
  }
  __syncthreads();
}

// Spectra of the calibration at retarded time, per detector row:
// D = dt F{pcal} exp(i omega tau); hfwd = s D, hdec = conj(D) / (|D|^2 + eps) / s.
template <class T>
__global__ __launch_bounds__(kFftThreads) void calib_kernel(const T* __restrict__ pcal, int n_t, int L, int log2L,
                                                            const double2* __restrict__ st, double dt, double eps,
                                                            double2* __restrict__ hfwd, double2* __restrict__ hdec) {
  extern __shared__ double2 x[];
  const int d = blockIdx.x;
  load_row<T>(x, pcal + (int64_t)d * n_t, n_t, L, log2L);
  fft_lds(x, L, log2L, -1.0);
  const double s = st[d].x, tau = st[d].y;
  for (int j = threadIdx.x; j < L; j += kFftThreads) {
    // omega_j = 2 pi f_j, f_j = j / (L dt) below L/2, (j - L) / (L dt) from L/2 on
    const int jj = j < (L >> 1) ? j : j - L;
    double sn, cs;
    sincospi(2.0 * (double)jj * tau / ((double)L * dt), &sn, &cs);
    const double2 D = cmul(make_double2(dt * x[j].x, dt * x[j].y), make_double2(cs, sn));
    const double den = (D.x * D.x + D.y * D.y + eps) * s;
    hfwd[(int64_t)d * L + j] = make_double2(s * D.x, s * D.y);
    hdec[(int64_t)d * L + j] = make_double2(D.x / den, -D.y / den);
  }
}

// out_d = first n_t samples of F^-1{ F{in_d} h_d } (real part).
template <class T>
__global__ __launch_bounds__(kFftThreads) void filter_kernel(const T* __restrict__ in, T* __restrict__ out, int n_t,
                                                             int L, int log2L, const double2* __restrict__ h) {
  extern __shared__ double2 x[];
  const int d = blockIdx.x;
  load_row<T>(x, in + (int64_t)d * n_t, n_t, L, log2L);
  fft_lds(x, L, log2L, -1.0);
  // multiply by the row's spectrum in natural order, then the inverse by
  // decimation in frequency (natural in, bit-reversed out)
  for (int j = threadIdx.x; j < L; j += kFftThreads) x[j] = cmul(x[j], h[(int64_t)d * L + j]);
  __syncthreads();
  fft_lds_dif(x, L, log2L, 1.0);
  const double scale = 1.0 / (double)L;
  for (int i = threadIdx.x; i < n_t; i += kFftThreads)
    out[(int64_t)d * n_t + i] = (T)(x[bitrev(i, log2L)].x * scale);
}

template <class T>
void calib_build(pat_calib_s* c, const void* pcal, hipStream_t s) {
  pat_geometry g = c->g;
  const size_t shm = sizeof(double2) * (size_t)c->L;
  hipLaunchKernelGGL(calib_kernel<T>, dim3(g->n_det), dim3(kFftThreads), shm, s, static_cast<const T*>(pcal), g->n_t,
                     c->L, c->log2L, ptr<double2>(c->st), g->desc.dt, c->eps, ptr<double2>(c->hfwd),
                     ptr<double2>(c->hdec));
  PAT_HIP(hipGetLastError());
}

template <class T>
void filter_rows(const pat_calib_s* c, const void* in, void* out, const pat::DevBuf& h, hipStream_t s) {
  const size_t shm = sizeof(double2) * (size_t)c->L;
  hipLaunchKernelGGL(filter_kernel<T>, dim3(c->g->n_det), dim3(kFftThreads), shm, s, static_cast<const T*>(in),
                     static_cast<T*>(out), c->g->n_t, c->L, c->log2L, ptr<double2>(h));
  PAT_HIP(hipGetLastError());
}

}  // namespace
}  // namespace pat

extern "C" pat_status pat_calib_create(pat_geometry g, const void* d_pcal, double xp, double yp, double eps,
                                       void* stream, pat_calib* out) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr && d_pcal != nullptr && out != nullptr, "NULL argument");
    PAT_CHECK_ARG(std::isfinite(xp) && std::isfinite(yp), "source position must be finite");
    PAT_CHECK_ARG(std::isfinite(eps) && eps > 0.0, "eps must be finite and > 0");
    int log2L = 0;
    while ((1 << log2L) < 2 * g->n_t) ++log2L;
    if (log2L > pat::kMaxFftLog2) {
      pat::set_error("n_t = %d needs a %d-point transform; at most %d is supported", g->n_t, 1 << log2L,
                     1 << pat::kMaxFftLog2);
      return PAT_ERR_UNSUPPORTED;
    }
    for (int d = 0; d < g->n_det; ++d)
      PAT_CHECK_ARG(std::hypot(g->det_xy[2 * d] - xp, g->det_xy[2 * d + 1] - yp) > 0.0,
                    "a detector sits on the calibration source");
    std::unique_ptr<pat_calib_s> c(new pat_calib_s());
    c->g = g;
    c->log2L = log2L;
    c->L = 1 << log2L;
    c->xp = xp;
    c->yp = yp;
    c->eps = eps;
    c->hfwd.alloc(sizeof(double2) * (size_t)g->n_det * c->L);
    c->hdec.alloc(sizeof(double2) * (size_t)g->n_det * c->L);
    c->au.alloc(pat::dtype_size(g->dtype) * (size_t)g->n_bins());
    // per detector: s_d = 2 pi c |x_d - x_p| and the travel time tau_d = |x_d - x_p| / c
    std::vector<double> st(2 * (size_t)g->n_det);
    for (int d = 0; d < g->n_det; ++d) {
      const double dist = std::hypot(g->det_xy[2 * d] - xp, g->det_xy[2 * d + 1] - yp);
      st[2 * d] = 2.0 * M_PI * g->desc.c * dist;
      st[2 * d + 1] = dist / g->desc.c;
    }
    c->st.alloc(sizeof(double) * st.size());
    hipStream_t s = static_cast<hipStream_t>(stream);
    PAT_HIP(hipMemcpyAsync(c->st.p, st.data(), sizeof(double) * st.size(), hipMemcpyHostToDevice, s));
    if (g->dtype == PAT_F64) pat::calib_build<double>(c.get(), d_pcal, s);
    else pat::calib_build<float>(c.get(), d_pcal, s);
    PAT_HIP(hipStreamSynchronize(s));
    *out = c.release();
    return PAT_OK;
  });
}

extern "C" pat_status pat_calib_destroy(pat_calib c) {
  return pat::guarded([&]() -> pat_status {
    delete c;
    return PAT_OK;
  });
}

extern "C" pat_status pat_pressure_forward(pat_calib c, const void* d_u, void* d_p, void* stream) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(c != nullptr && d_u != nullptr && d_p != nullptr, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (c->g->dtype == PAT_F64) {
      pat::apply_forward<double>(c->g, static_cast<const double*>(d_u), pat::ptr<double>(c->au), s);
      pat::filter_rows<double>(c, c->au.p, d_p, c->hfwd, s);
    } else {
      pat::apply_forward<float>(c->g, static_cast<const float*>(d_u), pat::ptr<float>(c->au), s);
      pat::filter_rows<float>(c, c->au.p, d_p, c->hfwd, s);
    }
    return PAT_OK;
  });
}

extern "C" pat_status pat_preprocess(pat_calib c, const void* d_p, void* d_f, void* stream) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(c != nullptr && d_p != nullptr && d_f != nullptr, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (c->g->dtype == PAT_F64) pat::filter_rows<double>(c, d_p, d_f, c->hdec, s);
    else pat::filter_rows<float>(c, d_p, d_f, c->hdec, s);
    return PAT_OK;
  });
}
