// Epilogue of the forward projections: where the value of one bin goes
// (shared by the gather, the LDS-tiled and the stored-matrix forwards).
#pragma once

#include "pat_internal.hpp"

namespace pat {

// The value val = (A x)_b of bin b, computed by this thread (writer), goes
// to its destination: the data (PLAIN), the dual data step of PDHGM (DUAL),
// the reciprocal row sum (ROWSUM) or the block's gap sums (GAP: every thread
// of the block takes part in the reduction).
template <class T, int MODE>
__device__ __forceinline__ void fwd_epilogue(const FwdArgs<T>& a, int blk, bool writer, int64_t b, T val) {
  if (MODE == FWD_GAP) {
    __shared__ double lds[8];
    double d_data = 0.0, d_fs = 0.0;
    if (writer) {
      const double res = (double)val - (double)a.f[b];
      const double qb = (double)a.q[b];
      d_data = 0.5 * res * res;
      d_fs = 0.5 * qb * qb + qb * (double)a.f[b];
    }
    const double s0 = block_sum<256>(d_data, lds);
    const double s1 = block_sum<256>(d_fs, lds);
    if (threadIdx.x == 0) {
      a.red[GAP_DATA * (int64_t)a.red_stride + blk] = s0;
      a.red[GAP_FSTAR * (int64_t)a.red_stride + blk] = s1;
    }
    return;
  }
  if (!writer) return;
  if (MODE == FWD_PLAIN) {
    a.out[b] = val;
  } else if (MODE == FWD_DUAL) {
    // q <- prox_{sigma F1*}(q + sigma A ubar) = (q + sigma (A ubar - f)) / (1 + sigma)
    const T sg = a.mult ? a.sigma[b] * (T)a.mult[0] : a.sigma[b];
    a.out[b] = (a.out[b] + sg * (val - a.f[b])) / (T(1) + sg);
  } else if (MODE == FWD_ROWSUM) {
    // A >= 0, so the absolute row sum is A 1; empty rows get sigma = 1
    a.out[b] = val > T(0) ? T(1) / val : T(1);
  }
}

}  // namespace pat
