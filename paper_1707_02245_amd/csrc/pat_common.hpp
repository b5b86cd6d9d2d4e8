// Internal definitions shared by the translation units of libpat.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "pat.h"

namespace pat {

// ---------------------------------------------------------------- errors

struct Error {
  pat_status status;
};

void set_error(const char* fmt, ...);
void clear_error();

[[noreturn]] inline void fail(pat_status s, const char* msg) {
  set_error("%s", msg);
  throw Error{s};
}

#define PAT_CHECK_ARG(cond, msg)                                      \
  do {                                                                \
    if (!(cond)) {                                                    \
      ::pat::set_error("invalid argument: %s", msg);                  \
      throw ::pat::Error{PAT_ERR_INVALID_ARG};                        \
    }                                                                 \
  } while (0)

#define PAT_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::pat::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                      \
      throw ::pat::Error{e_ == hipErrorOutOfMemory ? PAT_ERR_OOM : PAT_ERR_DEVICE};    \
    }                                                                                  \
  } while (0)

// Run a body and translate exceptions into a status (nothing crosses the ABI).
template <class F>
pat_status guarded(F&& body) {
  try {
    clear_error();
    return body();
  } catch (const Error& e) {
    return e.status;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return PAT_ERR_OOM;
  } catch (...) {
    set_error("unexpected internal error");
    return PAT_ERR_DEVICE;
  }
}

// ---------------------------------------------------------------- device memory

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    PAT_HIP(hipMalloc(&p, n));
    bytes = n;
  }
  // grow-only reuse
  void ensure(size_t n) { if (n > bytes) alloc(n); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

template <class T> inline T* ptr(const DevBuf& b) { return static_cast<T*>(b.p); }

// Global-memory view of a device pointer read from an argument table: loads
// through generic pointers compile to flat loads, which also count against
// the LDS counter and so serialise with LDS reads.
template <class T> using gptr = __attribute__((address_space(1))) T*;
template <class T> __device__ __forceinline__ gptr<const T> as_global(const T* p) {
  return (gptr<const T>)p;
}

inline size_t dtype_size(int dt) { return dt == PAT_F64 ? sizeof(double) : sizeof(float); }

// ---------------------------------------------------------------- device helpers

template <class T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
template <class T> using vec2_t = typename Vec2<T>::type;

// Sum over the lanes of a group of W consecutive lanes (W a power of two <= 64).
template <int W, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

// Sum over each row of 16 lanes by DPP moves (rotate by 8 and 4 within the
// row, then swap lanes 2 and 1 apart within quads); every lane of the row
// ends with the row's sum, lane 0 of the row in a fixed order.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <class T>
__device__ __forceinline__ T row16_sum(T x) {
  x += dpp_move<0x128>(x);  // row_ror:8
  x += dpp_move<0x124>(x);  // row_ror:4
  x += dpp_move<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_move<0xB1>(x);   // quad_perm [1,0,3,2]
  return x;
}

// Sum over the four lanes of a quad (every lane gets it).
template <class T>
__device__ __forceinline__ T quad_sum(T x) {
  x += dpp_move<0x4E>(x);  // quad_perm [2,3,0,1]
  x += dpp_move<0xB1>(x);  // quad_perm [1,0,3,2]
  return x;
}

// Deterministic block reduction into one value per block (blockDim.x = NT).
template <int NT, class T>
__device__ __forceinline__ T block_sum(T v, T* lds) {
  v = group_sum<64>(v);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  T s = T(0);
  if (threadIdx.x == 0) {
    for (int w = 0; w < NT / 64; ++w) s += lds[w];
  }
  __syncthreads();
  return s;  // valid in thread 0
}

// Block maximum (valid in thread 0), same layout as block_sum.
template <int NT, class T>
__device__ __forceinline__ T block_max(T v, T* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  T m = lds[0];
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / 64; ++w) m = fmax(m, lds[w]);
  }
  __syncthreads();
  return m;  // valid in thread 0
}

// ---------------------------------------------------------------- per-instance descriptor

// Gap partial sums, one double per block and slot.
enum GapSlot {
  GAP_DATA = 0,     // 1/2 ||A u - f||^2
  GAP_REG = 1,      // regulariser value at (u, v)
  GAP_FSTAR = 2,    // 1/2 ||q||^2 + <q, f>
  GAP_KTY = 3,      // ||K^T y||_1 (LS-T: ||A^T q||^2)
  GAP_DU2 = 4,      // ||u+ - u||^2
  GAP_U2 = 5,       // ||u||^2 before the update
  GAP_NSLOTS = 6
};

// Geometry tables on the device plus launch parameters. Sample positions are
// evaluated in FP64 for every element type.
struct GeomDev {
  int nx, ny, n_det, n_t;
  int pitch;             // nx + 2 (padded image row length)
  const double2* det;    // [n_det] detector position in pixel-index units
  const double2* rad;    // [n_t] (r_k / h, 1 / M_k)
  const int2* moff;      // [n_t] (M_k, offset of radius k in the table)
  const void* cs;        // [sum M_k] (cos, sin) of 2 pi (m + 1/2) / M_k, FP64
  const int4* win;       // [n_bins][2]: four sample ranges [m0,m1) per bin
  const int* kord;       // [n_t] radii by decreasing window samples (the
                         // radius-major gather's block order; null: 0..n_t-1)
  double kscale, koff;   // radius index of a radius rho in pixel units: rho*kscale - koff
  int lanes_log2;        // forward: lanes per bin, log2 (4..6)
  int fwd_path;          // forward: 0/1 gather (radius-/detector-major), 2 LDS tiles
  const int4* fpair;     // path 2: pairs {bin, m0, m1, partial slot}
  const int4* fblock;    // path 2: workgroups {cell x0, cell y0, pair0, pair1}
  const int* fbin_off;   // path 2: [n_bins + 1] partial offsets per bin
  int n_fblocks;         // path 2: workgroups
  int tile;              // adjoint: tile edge in pixels
  int tiles_x, tiles_y;
  int det_group;         // adjoint: detectors per workgroup
  int n_groups;          // ceil(n_det / det_group)
  // path 3, the stored A of the first n_det/4 detectors by 16 x 16 pixel
  // tiles (quarter-turn symmetric geometries): entries grouped by tile, then
  // by bin (segments), then by pixel; partial sums numbered bin-major
  const uint8_t* fm_off;   // [entries] pixel of the entry within its tile
  const void* fm_w;        // [entries] weight, element type
  const int4* fm_seg;      // [segments, tile-major] {first entry, entries, 0, 0}
  const int4* fm_chunk;    // [workgroups] {tile, first segment, end segment, 0}
  const int* fm_binseg;    // [n_det/4 n_t + 1] each bin's range in fm_segidx
  const int* fm_segidx;    // [segments] each bin's segments, in tile order
  int fm_nseg, fm_tiles_x, fm_nchunk;
};

// (cos, sin) of an arc sample from the FP64 table (every element type: an FP32
// table would put errors of r_k / h times 6e-8 pixels into the positions).
template <class T>
__device__ __forceinline__ double2 table_cs(const GeomDev& g, int idx) {
  const gptr<const double> c = as_global(static_cast<const double*>(g.cs)) + 2 * (int64_t)idx;
  return make_double2(c[0], c[1]);
}

// Forward projection of one instance.
template <class T>
struct FwdArgs {
  GeomDev g;
  const T* upad;      // padded image [(ny+2)(nx+2)]
  T* out;             // PLAIN: A u; DUAL: q (in/out); ROWSUM: sigma_q
  const T* f;         // DUAL, GAP: data
  const T* sigma;     // DUAL: sigma_q
  const T* q;         // GAP: dual variable for F*
  double* red;        // GAP: partial sums [GAP_NSLOTS][red_stride]
  int red_stride;
  T* part;            // path 2: partial sums [pairs]
  const double* mult; // DUAL: step multipliers {dual, primal, theta} of this
                      // iteration (accelerated schedule; null: plain steps)
  // Quarter-turn slots (the gather's QT form): g.n_det is a quarter of the
  // detectors and slot t (0..3) reads the image turned by t quarter turns at
  // upad + t slot_img, writes the bins of detectors t n_det/4 .. at out + t
  // slot_bins (f, sigma and q likewise) and its gap partials at red + t slot_red.
  int64_t slot_img, slot_bins;
  int slot_red;
};

// Adjoint projection of one instance into per-detector-group partial images.
template <class T>
struct AdjArgs {
  GeomDev g;
  const T* data;      // [n_det][n_t]
  T* part;            // [n_groups][ny][nx]
};

// One PDHG instance as seen by the pixel kernels.
template <class T>
struct InstDev {
  int nx, ny, n_groups, n_bins;
  int kind;           // pat_reg_kind
  T lam, alpha0;
  T theta_ex;         // extrapolation parameter
  const T* dmat;      // [3][N] (D11, D12, D22) of the directional gradient (DTV)
  // state
  T* u;               // [N]
  T* ubar_pad;        // [(ny+2)(nx+2)], zero border
  T* r;               // [2][N] (WAVELET: [4 N], coefficient order)
  T* v;               // [2][N]  (TGV)
  T* vbar;            // [2][N]  (TGV)
  T* s;               // [3][N]  (TGV)
  // step sizes
  const T* sigma_r;   // [N]
  const T* sigma_s;   // [N]
  const T* tau_u;     // [N]
  const T* tau_v;     // [N] (both components share one value)
  const T* atq_part;  // [n_groups][N] partial A^T q per detector group
  const double* atq64;  // [n_groups][N] A^T q accumulated in FP64 (check iterations; may be null)
  T* upad_gap;        // [(ny+2)(nx+2)] padded u+ written on check iterations
  double* red;        // partial sums [GAP_NSLOTS][red_stride]
  int red_stride;
  const double* mult; // step multipliers {dual, primal, theta} of this
                      // iteration (accelerated schedule; null: plain steps)
  const T* wtr;       // WAVELET: W^T r [N] of this iteration
  const double* wtr64;  // WAVELET, FP32 check iterations: W^T r in FP64 (else null)
  int rot_slots;      // 4: ubar_pad and upad_gap hold, after the image, its
                      // copies turned by 1, 2 and 3 quarter turns (padded
                      // size apart) for the quarter-turn forward; else 1
};

// y = M x for a CSR matrix M (rows n_rows).
template <class T>
struct CsrArgs {
  const int64_t* ptr;
  const int* col;
  const T* val;
  const T* x;
  T* y;
  double* y64;        // wide variant: FP64 accumulation and output
  int64_t n_rows;
};

// Y_r = M X_r for up to kMaxRhs right-hand sides sharing one CSR matrix (the
// matrix streams once for all of them).
constexpr int kMaxRhs = 8;
template <class T>
struct CsrMultiArgs {
  const int64_t* ptr;
  const int* col;
  const T* val;
  int64_t n_rows;
  int nrhs;
  const T* x[kMaxRhs];
  T* y[kMaxRhs];
  double* y64[kMaxRhs];
  // LDS-staged variant: rows grouped in side x side pixel tiles; per tile and
  // detector the window {k0, len, off, 0} of the bins its rows touch, staged
  // at LDS offset off; lcol = off + k - k0 replaces col
  const uint16_t* lcol;
  const int4* win;
  int side, tiles_x, nx, ny, n_det, n_t;  // n_det: detectors of the stored matrix
  int lds_stride;  // staged elements per slot (the geometry's largest window)
  // quarter-turn slots: with rot = 4 the matrix holds the first n_det rows of
  // a ring of 4 n_det detectors and slot r writes y[r] at the pixel turned by
  // r % 4 quarter turns; x[r] is then the data of detectors from
  // (r % 4) n_det on. rot = 1: no turn.
  int rot;
};

// Pixel (i, j) of a square n x n grid turned by t quarter turns (counter-
// clockwise, about the grid centre): (i, j) -> (n-1-j, i), as coordinates
// (a, b) and as the linear index b n + a.
__device__ __forceinline__ void quarter_turn_xy(int i, int j, int n, int t, int& a, int& b) {
  a = i;
  b = j;
  if (t & 2) { a = n - 1 - i; b = n - 1 - j; }
  if (t & 1) { const int c = a; a = n - 1 - b; b = c; }
}

__device__ __forceinline__ int64_t quarter_turn(int i, int j, int n, int t) {
  int a, b;
  quarter_turn_xy(i, j, n, t, a, b);
  return (int64_t)b * n + a;
}

// Ordered final sum of one instance's gap partials.
struct GapFinishArgs {
  const double* red;
  int stride, n_fwd, n_pix;
  int n_reg;  // partials of the regulariser value (n_pix, or the wavelet gap's workgroups)
};

}  // namespace pat
