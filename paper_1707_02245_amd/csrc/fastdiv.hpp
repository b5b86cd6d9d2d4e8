// Division of 32-bit unsigned integers by a divisor fixed at launch time, by a
// multiply-high and two shifts (Granlund and Montgomery, "Division by
// invariant integers using multiplication", PLDI 1994, Fig. 4.1):
//   l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
//   t = mulhi(m, n), n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0),
// exact for every n < 2^32 and 1 <= d < 2^31. Used where kernels split flat
// indices into image coordinates and channels with sizes known only at run
// time (an integer division by a run-time value costs tens of instructions).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pat {

struct FastDiv {
  uint32_t d = 1, m = 1;
  int s1 = 0, s2 = 0;
};

// d = 0 (a size that is never divided by) is taken as 1.
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d == 0 ? 1 : d;
  int l = 0;
  while ((1ull << l) < f.d) ++l;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - f.d)) / f.d + 1);
  f.s1 = l < 1 ? l : 1;
  f.s2 = l > 1 ? l - 1 : 0;
  return f;
}

__host__ __device__ __forceinline__ uint32_t fast_div(uint32_t n, const FastDiv& f) {
  const uint32_t t = (uint32_t)(((uint64_t)f.m * n) >> 32);
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

// n / d and n % d together
__host__ __device__ __forceinline__ void fast_divmod(uint32_t n, const FastDiv& f, uint32_t& q, uint32_t& r) {
  q = fast_div(n, f);
  r = n - q * f.d;
}

}  // namespace pat
