// Image quality of a reconstruction against its ground truth (arXiv:1707.02245,
// Sec. 5.4): the peak signal-to-noise ratio, in the form the paper prints it
// (the maximum of the ground truth not squared) and in the standard form,
//   printed  = 10 log10(max(u_gt) / (||u - u_gt||^2 / N)),
//   standard = 10 log10(max(u_gt)^2 / (||u - u_gt||^2 / N)).
// Both reductions (sum of squared differences, maximum of the ground truth)
// run in FP64 on the GPU: per-block partials, then one block that combines
// them in a fixed order, so the result does not depend on scheduling.

#include "pat_internal.hpp"

namespace pat {
namespace {

constexpr int kPsnrBlocks = 512;

template <class T>
__global__ __launch_bounds__(256) void psnr_partial_kernel(const T* __restrict__ u, const T* __restrict__ gt,
                                                           int64_t n, double* __restrict__ part) {
  double sse = 0.0, mx = -INFINITY;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double g = (double)gt[i];
    const double d = (double)u[i] - g;
    sse = fma(d, d, sse);
    mx = fmax(mx, g);
  }
  __shared__ double lds[8];
  const double s = block_sum<256>(sse, lds);
  const double m = block_max<256>(mx, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    part[kPsnrBlocks + blockIdx.x] = m;
  }
}

// out = {printed, standard, sse, max}
__global__ __launch_bounds__(256) void psnr_finish_kernel(const double* __restrict__ part, int nb, int64_t n,
                                                          double* __restrict__ out) {
  double s = 0.0, m = -INFINITY;
  for (int b = threadIdx.x; b < nb; b += 256) {
    s += part[b];
    m = fmax(m, part[kPsnrBlocks + b]);
  }
  __shared__ double lds[8];
  const double sse = block_sum<256>(s, lds);
  const double mx = block_max<256>(m, lds);
  if (threadIdx.x == 0) {
    const double mse = sse / (double)n;
    out[0] = 10.0 * log10(mx / mse);
    out[1] = 10.0 * log10(mx * mx / mse);
    out[2] = sse;
    out[3] = mx;
  }
}

template <class T>
void psnr_impl(int64_t n, const void* u, const void* gt, double* host4, hipStream_t s) {
  DevBuf part(sizeof(double) * 2 * kPsnrBlocks), out(sizeof(double) * 4);
  const int nb = (int)std::min<int64_t>(kPsnrBlocks, (n + 255) / 256);
  hipLaunchKernelGGL(psnr_partial_kernel<T>, dim3(nb), dim3(256), 0, s, static_cast<const T*>(u),
                     static_cast<const T*>(gt), n, ptr<double>(part));
  hipLaunchKernelGGL(psnr_finish_kernel, dim3(1), dim3(256), 0, s, ptr<double>(part), nb, n, ptr<double>(out));
  PAT_HIP(hipGetLastError());
  PAT_HIP(hipMemcpyAsync(host4, out.p, sizeof(double) * 4, hipMemcpyDeviceToHost, s));
  PAT_HIP(hipStreamSynchronize(s));
}

}  // namespace
}  // namespace pat

extern "C" pat_status pat_psnr(int32_t dtype, int64_t n, const void* d_u, const void* d_gt,
                               double* psnr_printed, double* psnr_standard, void* stream) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(dtype == PAT_F32 || dtype == PAT_F64, "unknown dtype");
    PAT_CHECK_ARG(n >= 1, "n must be >= 1");
    PAT_CHECK_ARG(d_u != nullptr && d_gt != nullptr && psnr_printed != nullptr && psnr_standard != nullptr,
                  "NULL argument");
    double r[4];
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == PAT_F64) pat::psnr_impl<double>(n, d_u, d_gt, r, s);
    else pat::psnr_impl<float>(n, d_u, d_gt, r, s);
    if (!(r[3] > 0.0) || std::isnan(r[2])) {
      pat::set_error("PSNR needs a ground truth with a positive maximum and finite images (max %g, sse %g)",
                     r[3], r[2]);
      return PAT_ERR_NUMERIC;
    }
    *psnr_printed = r[0];
    *psnr_standard = r[1];
    return PAT_OK;
  });
}
