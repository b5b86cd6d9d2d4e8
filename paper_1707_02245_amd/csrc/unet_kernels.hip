// Kernels of the warm-start network: a generic implicit-GEMM on the bf16 matrix
// cores (FP32 accumulation) that can serve every convolution of the network in
// the forward pass and both backward passes; direct kernels on staged pixel
// tiles for the 3x3 convolutions whose shapes allow them (forward and data
// gradient, weight and bias gradients, the one-channel first layer); plus
// pooling, the 1x1 head, the loss, bias gradients, split-K reduction, Adam and
// weight re-layout.
//
// Tensors are NHWC. Every activation view carries a channel pitch and offset,
// so a transposed convolution writes the first half and an encoder
// convolution the second half of one concatenation buffer without copies.
//
// The GEMM computes C[m][n] = sum_k A(m,k) B(n,k). A and B are fetched
// element-wise through index maps (direct, 3x3 im2col with +/- tap offsets,
// 2x2 sub-pixel gathers, transposed views), staged through LDS in 32-wide k
// chunks and multiplied with the gfx950 instruction
// __builtin_amdgcn_mfma_f32_16x16x32_bf16: lane l supplies A[l%16][8(l/16)+j]
// and B[8(l/16)+j][l%16], j = 0..7 (one 16-byte LDS read per operand; any
// grouping of k that A and B share gives the same product), and receives
// D[4(l/16)+r][l%16], r = 0..3.

#include <climits>

#include "unet_internal.hpp"

namespace pat {
namespace nn {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}

// Pixel index -> (batch, row, column) of a view, and a 3x3 tap index -> offsets.
__device__ __forceinline__ void pix_split(int m, const FastDiv& dw, const FastDiv& dh, int& b, int& y, int& x) {
  uint32_t t, r;
  fast_divmod((uint32_t)m, dw, t, r);
  x = (int)r;
  uint32_t bb, yy;
  fast_divmod(t, dh, bb, yy);
  y = (int)yy;
  b = (int)bb;
}
__device__ __forceinline__ void chan_split(int k, const FastDiv& dc, int& tap, int& c) {
  uint32_t q, r;
  fast_divmod((uint32_t)k, dc, q, r);
  tap = (int)q;
  c = (int)r;
}

// ------------------------------------------------------------------ operand fetch

__device__ __forceinline__ uint16_t fetch_a(const GemmDesc& d, int m, int k) {
  if (m >= d.M || k >= d.K) return 0;
  const View& v = d.a;
  switch (d.a_mode) {
    case A_DIRECT:
      return v.p[(int64_t)m * v.pitch + v.off + k];
    case A_CONV: {
      int tap, c, b, y, x;
      chan_split(k, v.dC, tap, c);
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      pix_split(m, v.dW, v.dH, b, y, x);
      const int yy = y + d.a_sign * dy, xx = x + d.a_sign * dx;
      if (yy < 0 || yy >= v.H || xx < 0 || xx >= v.W) return 0;
      return v.p[((int64_t)(b * v.H + yy) * v.W + xx) * v.pitch + v.off + c];
    }
    case A_G22: {  // m: low-res pixel on (H/2, W/2); k = sub * C + c; source at full res
      int sub, c, b, y, x;
      chan_split(k, v.dC, sub, c);
      pix_split(m, v.dW2, v.dH2, b, y, x);
      const int yy = 2 * y + (sub >> 1), xx = 2 * x + (sub & 1);
      return v.p[((int64_t)(b * v.H + yy) * v.W + xx) * v.pitch + v.off + c];
    }
    case A_T:  // m = channel, k = pixel
      return v.p[(int64_t)k * v.pitch + v.off + m];
    case A_TG22: {  // m = sub * C + c, k = low-res pixel; source at full res
      int sub, c, b, y, x;
      chan_split(m, v.dC, sub, c);
      pix_split(k, v.dW2, v.dH2, b, y, x);
      const int yy = 2 * y + (sub >> 1), xx = 2 * x + (sub & 1);
      return v.p[((int64_t)(b * v.H + yy) * v.W + xx) * v.pitch + v.off + c];
    }
  }
  return 0;
}

__device__ __forceinline__ uint16_t fetch_b(const GemmDesc& d, int n, int k) {
  if (n >= d.N || k >= d.K) return 0;
  const View& v = d.b;
  switch (d.b_mode) {
    case B_W:
      return d.w[(int64_t)n * d.K + k];
    case B_IM2COL: {  // n = tap * C + c, k = pixel
      int tap, c, b, y, x;
      chan_split(n, v.dC, tap, c);
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      pix_split(k, v.dW, v.dH, b, y, x);
      const int yy = y + dy, xx = x + dx;
      if (yy < 0 || yy >= v.H || xx < 0 || xx >= v.W) return 0;
      return v.p[((int64_t)(b * v.H + yy) * v.W + xx) * v.pitch + v.off + c];
    }
    case B_T:  // n = channel, k = pixel
      return v.p[(int64_t)k * v.pitch + v.off + n];
  }
  return 0;
}

// Address of 8 consecutive operand elements (nullptr: all zero padding).
// Along k: A(m, k..k+7) or B(n, k..k+7); along m / n: A(m..m+7, k) or
// B(n..n+7, k). Only called when launch_gemm found the layout aligned.
__device__ __forceinline__ const uint16_t* addr8_a(const GemmDesc& d, int m, int k) {
  const View& v = d.a;
  switch (d.a_mode) {
    case A_DIRECT:
      return v.p + (int64_t)m * v.pitch + v.off + k;
    case A_CONV: {
      int tap, c, b, y, x;
      chan_split(k, v.dC, tap, c);
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      pix_split(m, v.dW, v.dH, b, y, x);
      const int yy = y + d.a_sign * dy, xx = x + d.a_sign * dx;
      if (yy < 0 || yy >= v.H || xx < 0 || xx >= v.W) return nullptr;
      return v.p + ((int64_t)(b * v.H + yy) * v.W + xx) * v.pitch + v.off + c;
    }
    case A_G22: {
      int sub, c, b, y, x;
      chan_split(k, v.dC, sub, c);
      pix_split(m, v.dW2, v.dH2, b, y, x);
      const int yy = 2 * y + (sub >> 1), xx = 2 * x + (sub & 1);
      return v.p + ((int64_t)(b * v.H + yy) * v.W + xx) * v.pitch + v.off + c;
    }
    case A_T:
      return v.p + (int64_t)k * v.pitch + v.off + m;
    case A_TG22: {
      int sub, c, b, y, x;
      chan_split(m, v.dC, sub, c);
      pix_split(k, v.dW2, v.dH2, b, y, x);
      const int yy = 2 * y + (sub >> 1), xx = 2 * x + (sub & 1);
      return v.p + ((int64_t)(b * v.H + yy) * v.W + xx) * v.pitch + v.off + c;
    }
  }
  return nullptr;
}

__device__ __forceinline__ const uint16_t* addr8_b(const GemmDesc& d, int n, int k) {
  const View& v = d.b;
  switch (d.b_mode) {
    case B_W:
      return d.w + (int64_t)n * d.K + k;
    case B_IM2COL: {
      int tap, c, b, y, x;
      chan_split(n, v.dC, tap, c);
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      pix_split(k, v.dW, v.dH, b, y, x);
      const int yy = y + dy, xx = x + dx;
      if (yy < 0 || yy >= v.H || xx < 0 || xx >= v.W) return nullptr;
      return v.p + ((int64_t)(b * v.H + yy) * v.W + xx) * v.pitch + v.off + c;
    }
    case B_T:
      return v.p + (int64_t)k * v.pitch + v.off + n;
  }
  return nullptr;
}

// Stage a ROWS x KC chunk of one operand into LDS (row-major, leading dim LD).
// VEC >= 0: the vector mode fixed at compile time (the other paths compiled
// out); -1: read from the descriptor.
template <bool IS_A, int ROWS, int KC, int LD, int VEC>
__device__ __forceinline__ void stage(const GemmDesc& d, uint16_t* S, int row0, int k0, int ke, int t) {
  const int vec = VEC >= 0 ? VEC : (IS_A ? d.a_vec : d.b_vec);
  const int nrows = IS_A ? d.M : d.N;
  if (vec == 1) {  // 8 consecutive k of one row: one 16-byte load, one 16-byte LDS store
    for (int e = t; e < ROWS * KC / 8; e += 256) {
      const int r = e / (KC / 8), kv = (e % (KC / 8)) * 8;
      const int row = row0 + r, k = k0 + kv;
      uint4 w = make_uint4(0, 0, 0, 0);
      if (row < nrows) {
        if (k + 8 <= ke) {
          const uint16_t* p = IS_A ? addr8_a(d, row, k) : addr8_b(d, row, k);
          if (p) w = *reinterpret_cast<const uint4*>(p);
        } else {
          uint16_t h[8];
#pragma unroll
          for (int i = 0; i < 8; ++i)
            h[i] = (k + i < ke) ? (IS_A ? fetch_a(d, row, k + i) : fetch_b(d, row, k + i)) : (uint16_t)0;
          w = make_uint4(h[0] | (uint32_t)h[1] << 16, h[2] | (uint32_t)h[3] << 16, h[4] | (uint32_t)h[5] << 16,
                         h[6] | (uint32_t)h[7] << 16);
        }
      }
      *reinterpret_cast<uint4*>(S + r * LD + kv) = w;
    }
  } else if (vec == 2) {
    // 8 consecutive rows at one k: one 16-byte load, 8 LDS stores; launch_gemm
    // takes this path only when the row count is a multiple of 8, so a group
    // of 8 rows is wholly inside or wholly outside
#pragma unroll 1
    for (int e = t; e < ROWS / 8 * KC; e += 256) {
      const int rv = (e / KC) * 8, kk = e % KC;
      const int row = row0 + rv, k = k0 + kk;
      uint4 w = make_uint4(0, 0, 0, 0);
      if (k < ke && row < nrows) {
        const uint16_t* p = IS_A ? addr8_a(d, row, k) : addr8_b(d, row, k);
        if (p) w = *reinterpret_cast<const uint4*>(p);
      }
      const uint32_t dw[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int i = 0; i < 8; ++i) S[(rv + i) * LD + kk] = (uint16_t)(dw[i >> 1] >> (16 * (i & 1)));
    }
  } else {
#pragma unroll 1
    for (int e = t; e < ROWS * KC; e += 256) {
      const int r = e / KC, kk = e % KC;
      S[r * LD + kk] = (k0 + kk < ke) ? (IS_A ? fetch_a(d, row0 + r, k0 + kk) : fetch_b(d, row0 + r, k0 + kk))
                                      : (uint16_t)0;
    }
  }
}

// One operand chunk (ROWS x KC) of a fixed vector mode held in registers
// between its global loads and its LDS stores, so that the loads of the next
// chunk are in flight while the current one is multiplied. VEC 1: 8
// consecutive k of one row per 16-byte vector; 2: 8 consecutive rows at one k
// (launch_gemm guarantees K, the split-K chunks and, for 2, the row count to
// be multiples of 8, so a vector is wholly inside or outside the operand).
template <bool IS_A, int ROWS, int KC, int LD, int VEC>
struct ChunkRegs {
  static constexpr int NV = VEC == 1 ? ROWS * KC / 8 : ROWS / 8 * KC;
  static constexpr int SLOTS = (NV + 255) / 256;
  uint4 r[SLOTS];

  __device__ __forceinline__ void load(const GemmDesc& d, int row0, int k0, int ke, int t) {
    const int nrows = IS_A ? d.M : d.N;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int e = t + 256 * s;
      r[s] = make_uint4(0, 0, 0, 0);
      if (e >= NV) continue;
      const int row = row0 + (VEC == 1 ? e / (KC / 8) : (e / KC) * 8);
      const int k = k0 + (VEC == 1 ? (e % (KC / 8)) * 8 : e % KC);
      if (row < nrows && k < ke) {
        const uint16_t* p = IS_A ? addr8_a(d, row, k) : addr8_b(d, row, k);
        if (p) r[s] = *reinterpret_cast<const uint4*>(p);
      }
    }
  }

  __device__ __forceinline__ void store(uint16_t* S, int t) const {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int e = t + 256 * s;
      if (e >= NV) continue;
      if (VEC == 1) {
        *reinterpret_cast<uint4*>(S + (e / (KC / 8)) * LD + (e % (KC / 8)) * 8) = r[s];
      } else {
        const int rv = (e / KC) * 8, kk = e % KC;
        const uint32_t dw[4] = {r[s].x, r[s].y, r[s].z, r[s].w};
#pragma unroll
        for (int i = 0; i < 8; ++i) S[(rv + i) * LD + kk] = (uint16_t)(dw[i >> 1] >> (16 * (i & 1)));
      }
    }
  }
};

// ------------------------------------------------------------------ direct 3x3 convolution

// The 3x3 convolutions (M = every pixel of the batch, N = output channels, a
// multiple of 32, K = 9 C) as a direct convolution: a workgroup of 8 waves
// takes a 16 x 16 pixel tile of one image (two rows per wave) and 32 of the
// output channels (blockIdx.y), stages the tile's input with its one-pixel
// halo (18 x 18 pixels, 32 channels at a time) and the weights of those
// channels for the nine taps in LDS once, and multiplies each tap's
// shifted view of the halo with the 16x16x32 MFMA, so a pixel's input is read
// from memory once per channel chunk instead of once per tap. Channels and
// weight rows are padded to 40 elements in LDS (an 80-byte stride puts the 16
// rows a fragment reads in distinct banks). a_sign = -1 (the data gradient)
// reads the taps mirrored, as the GEMM's index map does. Accumulation: per
// chunk of 32 channels, taps in order. (16 x 16 tiles took the training step
// 2.64 -> 2.51 ms against 8 x 16 tiles of 4 waves: the weights are staged for
// twice as many pixels.)
constexpr int kCvTH = 16, kCvTW = 16, kCvHH = kCvTH + 2, kCvHW = kCvTW + 2, kCvLD = 40, kCvThreads = 512;

__global__ __launch_bounds__(kCvThreads) void conv3_kernel(GemmDesc d) {
  __shared__ __align__(16) uint16_t halo[kCvHH * kCvHW * kCvLD];
  __shared__ __align__(16) uint16_t wts[9 * 32 * kCvLD];
  const View& v = d.a;
  const int H = v.H, W = v.W, C = v.C;
  const int tiles_x = W / kCvTW, tiles_y = H / kCvTH;
  int blk = blockIdx.x;
  const int tx = blk % tiles_x;
  blk /= tiles_x;
  const int ty = blk % tiles_y, b = blk / tiles_y;
  const int x0 = tx * kCvTW, y0 = ty * kCvTH;
  const int n0 = 32 * blockIdx.y;  // the workgroup's output channels n0 .. n0 + 31
  const int t = threadIdx.x, wave = t / 64, lane = t % 64;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int c0 = 0; c0 < C; c0 += 32) {
    // halo: 10 x 18 pixels x 32 channels as 16-byte vectors of 8 channels
    for (int e = t; e < kCvHH * kCvHW * 4; e += kCvThreads) {
      const int cv = e % 4, px = e / 4;
      const int hx = px % kCvHW, hy = px / kCvHW;
      const int yy = y0 + hy - 1, xx = x0 + hx - 1;
      uint4 w = make_uint4(0, 0, 0, 0);
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        w = *reinterpret_cast<const uint4*>(v.p + ((int64_t)(b * H + yy) * W + xx) * v.pitch + v.off + c0 + 8 * cv);
      *reinterpret_cast<uint4*>(halo + px * kCvLD + 8 * cv) = w;
    }
    // weights of the chunk: w[n0 + n][tap C + c0 + c] for 32 n, 9 taps, 32 c
    for (int e = t; e < 9 * 32 * 4; e += kCvThreads) {
      const int cv = e % 4, row = e / 4;  // row = tap * 32 + n
      const int tap = row / 32, n = row % 32;
      const uint4 w = *reinterpret_cast<const uint4*>(d.w + (int64_t)(n0 + n) * d.K + tap * C + c0 + 8 * cv);
      *reinterpret_cast<uint4*>(wts + row * kCvLD + 8 * cv) = w;
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = d.a_sign * (tap / 3 - 1), dx = d.a_sign * (tap % 3 - 1);
      v8bf a[2], bw[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int hy = wave * 2 + i + 1 + dy, hx = lane % 16 + 1 + dx;
        a[i] = *reinterpret_cast<const v8bf*>(halo + (hy * kCvHW + hx) * kCvLD + 8 * (lane / 16));
      }
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bw[j] = *reinterpret_cast<const v8bf*>(wts + (tap * 32 + j * 16 + lane % 16) * kCvLD + 8 * (lane / 16));
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bw[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue as the GEMM's E_ACT: fragment i covers tile row wave * 2 + i,
  // D[4(l/16)+r][l%16] -> pixel column 4(l/16)+r, output channel j * 16 + l % 16.
  // Bias, ReLU and bf16 per element into LDS (the halo's space: the last
  // chunk's barrier has passed), then each pixel's 32 channels leave as four
  // 16-byte stores, with the mask applied per element.
  uint16_t* ost = halo;  // [256 pixels][kCvLD]
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int nl = j * 16 + lane % 16;
    const float bn = d.bias ? d.bias[n0 + nl] : 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float val = acc[i][j][r];
        if (d.bias) val += bn;
        if (d.relu) val = fmaxf(val, 0.f);
        ost[((wave * 2 + i) * kCvTW + 4 * (lane / 16) + r) * kCvLD + nl] = f2bf(val);
      }
    }
  }
  __syncthreads();
  for (int e = t; e < kCvTH * kCvTW * 4; e += kCvThreads) {
    const int px = e / 4, cv = e % 4;
    const int64_t m = (int64_t)(b * H + y0 + px / kCvTW) * W + x0 + px % kCvTW;
    uint4 o = *reinterpret_cast<const uint4*>(ost + px * kCvLD + 8 * cv);
    if (d.mask.p) {
      const uint4 mk = *reinterpret_cast<const uint4*>(d.mask.p + m * d.mask.pitch + d.mask.off + n0 + 8 * cv);
      uint32_t ow[4] = {o.x, o.y, o.z, o.w};
      const uint32_t mw[4] = {mk.x, mk.y, mk.z, mk.w};
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (!(bf2f((uint16_t)(mw[k >> 1] >> (16 * (k & 1)))) > 0.f)) ow[k >> 1] &= ~(0xFFFFu << (16 * (k & 1)));
      o = make_uint4(ow[0], ow[1], ow[2], ow[3]);
    }
    *reinterpret_cast<uint4*>(d.out.p16 + m * d.out.pitch + d.out.off + n0 + 8 * cv) = o;
  }
}

// Whether conv3_kernel serves this product (else the generic GEMM).
static bool conv3_applies(const GemmDesc& d) {
  const View& v = d.a;
  auto vec_out = [](const View& o, const void* p) {
    return o.pitch % 8 == 0 && o.off % 8 == 0 && (reinterpret_cast<uintptr_t>(p) & 15) == 0;
  };
  return d.a_mode == A_CONV && d.b_mode == B_W && d.out_mode == E_ACT && d.a_vec == 1 && d.b_vec == 1 &&
         d.N % 32 == 0 && d.ksplit >= d.K && v.C % 32 == 0 && d.K == 9 * v.C && v.H % kCvTH == 0 &&
         v.W % kCvTW == 0 && v.H > 0 && v.W > 0 && d.M % (v.H * v.W) == 0 && vec_out(d.out, d.out.p16) &&
         (!d.mask.p || vec_out(d.mask, d.mask.p));
}

// A 3x3 convolution of a one-channel input (the network's first layer,
// K = 9): one thread per pixel reads its nine taps once and writes its N
// outputs (N a multiple of 8, at most 64) as 16-byte vectors, each output the
// FP32 sum of the nine products in tap order, then bias, ReLU, bf16 and the
// mask as the GEMM's E_ACT epilogue. The bf16 weights sit in LDS as floats
// (every thread reads the same weight: broadcast). a_sign = -1 mirrors the
// taps, as the GEMM's index map does.
constexpr int kCiMaxN = 64;

__global__ __launch_bounds__(256) void conv_in_kernel(GemmDesc d) {
  __shared__ float wl[kCiMaxN * 9];
  __shared__ float bl[kCiMaxN];
  for (int e = threadIdx.x; e < d.N * 9; e += blockDim.x) wl[e] = bf2f(d.w[e]);
  for (int e = threadIdx.x; e < d.N; e += blockDim.x) bl[e] = d.bias ? d.bias[e] : 0.f;
  __syncthreads();
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= d.M) return;
  const View& v = d.a;
  int b, y, x;
  pix_split(m, v.dW, v.dH, b, y, x);
  float xv[9];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int yy = y + d.a_sign * (tap / 3 - 1), xx = x + d.a_sign * (tap % 3 - 1);
    xv[tap] = (yy >= 0 && yy < v.H && xx >= 0 && xx < v.W)
                  ? bf2f(v.p[((int64_t)(b * v.H + yy) * v.W + xx) * v.pitch + v.off])
                  : 0.f;
  }
  for (int c0 = 0; c0 < d.N; c0 += 8) {
    uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int n = c0 + i;
      float acc = 0.f;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) acc = fmaf(xv[tap], wl[n * 9 + tap], acc);
      if (d.bias) acc += bl[n];
      if (d.relu) acc = fmaxf(acc, 0.f);
      uint16_t h = f2bf(acc);
      if (d.mask.p && !(bf2f(d.mask.p[(int64_t)m * d.mask.pitch + d.mask.off + n]) > 0.f)) h = 0;
      o[i >> 1] |= (uint32_t)h << (16 * (i & 1));
    }
    *reinterpret_cast<uint4*>(d.out.p16 + (int64_t)m * d.out.pitch + d.out.off + c0) =
        make_uint4(o[0], o[1], o[2], o[3]);
  }
}

static bool conv_in_applies(const GemmDesc& d) {
  const View& v = d.a;
  return d.a_mode == A_CONV && d.b_mode == B_W && d.out_mode == E_ACT && v.C == 1 && d.K == 9 &&
         d.ksplit >= d.K && d.N % 8 == 0 && d.N <= kCiMaxN && d.out.pitch % 8 == 0 && d.out.off % 8 == 0 &&
         (reinterpret_cast<uintptr_t>(d.out.p16) & 15) == 0 && v.H > 0 && v.W > 0 && d.M % (v.H * v.W) == 0;
}

// The weight gradient of a 3x3 convolution as a direct product over pixel
// tiles: dW[co][tap C + ci] = sum_p g[p][co] x[p + off(tap)][ci], off(tap) =
// (tap / 3 - 1, tap % 3 - 1), zero outside the image (the product the GEMM
// takes with B = im2col(x)). A workgroup of 4 waves takes 32 output channels
// (blockIdx.y), 32 input channels (blockIdx.z) and the 16 x 16-pixel tiles
// blockIdx.x, blockIdx.x + gridDim.x, ... For each tile it stages the
// gradient transposed, gT[co][pixel], and the input's 18 x 18 halo transposed
// in three copies shifted by 0, 1 and 2 columns, xs[dx][ci][row][col], so that
// every MFMA operand is one aligned 16-byte LDS read of 8 consecutive pixels
// (the halo is read from memory once instead of once per tap). k = pixels, 32
// per MFMA: tile rows 2s and 2s + 1, lane group q = l / 16 holding row
// 2s + q / 2, columns 8 (q % 2) .. + 7, in both operands. Wave w takes the k
// steps s = w and w + 4 of every tile for all 2 x 2 channel fragments and nine
// taps (two A and eighteen B reads per 36 products); the four waves' sums are
// added in wave order at the end and written to the split-K partials
// [blockIdx.x][co][tap C + ci]. Both stagings move blocks of
// 8 pixels x 8 channels (eight 16-byte loads, a transpose in registers, eight
// 16-byte LDS stores). The bias gradient's column
// sums sum_p g[p][co] come from the same staged gradient: the workgroups of
// the first input-channel chunk multiply it by a ones operand in one more
// accumulator per output-channel fragment and write bpart[blockIdx.x][co]. Rows are padded by 8 elements in LDS against bank
// conflicts.
// v[p] holds 8 bf16 channels of pixel p (p = 0..7); store channel c's 8
// pixels as one 16-byte row at dst + c * ld (16-byte aligned).
__device__ __forceinline__ void transpose8_store(const uint4 (&v)[8], uint16_t* dst, int ld) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t w0 = (&v[2 * k].x)[c >> 1], w1 = (&v[2 * k + 1].x)[c >> 1];
      o[k] = (c & 1) ? ((w0 >> 16) | (w1 & 0xFFFF0000u)) : ((w0 & 0xFFFFu) | (w1 << 16));
    }
    *reinterpret_cast<uint4*>(dst + c * ld) = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

constexpr int kWgT = 16, kWgGLD = kWgT * kWgT + 8, kWgXLD = (kWgT + 2) * kWgT + 8;
constexpr int kWgTargetBlocks = 512;

__global__ __launch_bounds__(256, 2) void wgrad3_kernel(View x, View g, float* __restrict__ part,
                                                     float* __restrict__ bpart, int cout, int cin, int n_tiles) {
  __shared__ __align__(16) uint16_t gT[32 * kWgGLD];
  __shared__ __align__(16) uint16_t xs[3 * 32 * kWgXLD];
  const int H = x.H, W = x.W;
  const int tiles_x = W / kWgT, tiles_y = H / kWgT;
  const int co0 = 32 * blockIdx.y, ci0 = 32 * blockIdx.z;
  const int t = threadIdx.x, wave = t / 64, lane = t % 64;
  const int q = lane / 16, r16 = lane % 16;
  const bool bias = blockIdx.z == 0;
  v8bf ones;
#pragma unroll
  for (int j = 0; j < 8; ++j) ones[j] = (__bf16)1.0f;
  // [output-channel fragment][input-channel fragment][tap], and the bias
  // column per output-channel fragment
  v4f acc[2][2][9], accb[2];
#pragma unroll
  for (int cf = 0; cf < 2; ++cf) {
    accb[cf] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nf = 0; nf < 2; ++nf)
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) acc[cf][nf][tap] = v4f{0.f, 0.f, 0.f, 0.f};
  }
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    int tt = tile;
    const int tx = tt % tiles_x;
    tt /= tiles_x;
    const int ty = tt % tiles_y, b = tt / tiles_y;
    const int x0 = tx * kWgT, y0 = ty * kWgT;
    // the gradient's 256 pixels x 32 channels by blocks of 8 pixels (a row
    // run) x 8 channels: eight 16-byte loads, a transpose in registers, eight
    // 16-byte LDS stores of 8 pixels of one channel
    if (t < 128) {
      const int pg = t % 32, cg = t / 32;
      const int row = pg / 2, col0 = 8 * (pg % 2);
      uint4 v[8];
#pragma unroll
      for (int p = 0; p < 8; ++p)
        v[p] = *reinterpret_cast<const uint4*>(g.p + ((int64_t)(b * H + y0 + row) * W + x0 + col0 + p) * g.pitch +
                                               g.off + co0 + 8 * cg);
      transpose8_store(v, gT + (8 * cg) * kWgGLD + row * kWgT + col0, kWgGLD);
    }
    // the input's halo: copy dx, row hy, columns 8 h .. 8 h + 7 hold the
    // pixels hx = dx + 8 h .. (image column x0 + hx - 1), zero outside
    for (int e = t; e < 3 * (kWgT + 2) * 2 * 4; e += 256) {
      const int cg = e % 4, h = (e / 4) % 2, hy = (e / 8) % (kWgT + 2), dx = e / (8 * (kWgT + 2));
      const int yy = y0 + hy - 1;
      uint4 v[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int xx = x0 + dx + 8 * h + p - 1;
        v[p] = make_uint4(0, 0, 0, 0);
        if (yy >= 0 && yy < H && xx >= 0 && xx < W)
          v[p] = *reinterpret_cast<const uint4*>(x.p + ((int64_t)(b * H + yy) * W + xx) * x.pitch + x.off + ci0 +
                                                 8 * cg);
      }
      transpose8_store(v, xs + (dx * 32 + 8 * cg) * kWgXLD + hy * kWgT + 8 * h, kWgXLD);
    }
    __syncthreads();
    // wave w: k steps w and w + 4 (tile rows 2 st, 2 st + 1), all four fragments
#pragma unroll
    for (int sw = 0; sw < kWgT / 8; ++sw) {
      const int st = wave + 4 * sw;
      const int row = 2 * st + (q >> 1), col = 8 * (q & 1);
      v8bf a[2];
#pragma unroll
      for (int cf = 0; cf < 2; ++cf)
        a[cf] = *reinterpret_cast<const v8bf*>(gT + (16 * cf + r16) * kWgGLD + row * kWgT + col);
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
#pragma unroll
        for (int nf = 0; nf < 2; ++nf) {
          const v8bf bx =
              *reinterpret_cast<const v8bf*>(xs + (dx * 32 + 16 * nf + r16) * kWgXLD + (row + dy) * kWgT + col);
#pragma unroll
          for (int cf = 0; cf < 2; ++cf)
            acc[cf][nf][tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cf], bx, acc[cf][nf][tap], 0, 0, 0);
        }
      }
      if (bias)
#pragma unroll
        for (int cf = 0; cf < 2; ++cf) accb[cf] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cf], ones, accb[cf], 0, 0, 0);
    }
    __syncthreads();
  }
  // the four waves' sums, added in wave order through LDS (the staging space:
  // the last tile's barrier has passed), one fragment pair (cf, nf) at a time;
  // D[4 q + r][r16]: output channel co0 + 16 cf + 4 q + r, input channel
  // ci0 + 16 nf + r16
  float* red = reinterpret_cast<float*>(xs);  // [wave][tap][r][lane]: 4 x 2304 floats
  const int64_t N = 9 * (int64_t)cin;
  float* out = part + (int64_t)blockIdx.x * cout * N;
#pragma unroll
  for (int pr = 0; pr < 4; ++pr) {
    const int cf = pr >> 1, nf = pr & 1;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[((wave * 9 + tap) * 4 + r) * 64 + lane] = acc[cf][nf][tap][r];
    __syncthreads();
    for (int e = t; e < 9 * 4 * 64; e += 256) {
      const float v = ((red[e] + red[2304 + e]) + red[2 * 2304 + e]) + red[3 * 2304 + e];
      const int tap = e / 256, r = (e / 64) % 4, l = e % 64;
      out[(int64_t)(co0 + 16 * cf + 4 * (l / 16) + r) * N + tap * cin + ci0 + 16 * nf + l % 16] = v;
    }
    __syncthreads();
  }
  if (bias) {
    // every column of the ones product holds the sum; column 0 is used
#pragma unroll
    for (int cf = 0; cf < 2; ++cf)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[((wave * 2 + cf) * 4 + r) * 64 + lane] = accb[cf][r];
    __syncthreads();
    if (t < 2 * 4 * 4) {
      const int cf = t / 16, r = (t / 4) % 4, qq = t % 4;
      const int e = (cf * 4 + r) * 64 + 16 * qq;
      const float v = ((red[e] + red[512 + e]) + red[2 * 512 + e]) + red[3 * 512 + e];
      bpart[(int64_t)blockIdx.x * cout + co0 + 16 * cf + 4 * qq + r] = v;
    }
  }
}

bool wgrad3_applies(const View& x, const View& g, int cin, int cout) {
  auto vec_ok = [](const View& v) {
    return v.pitch % 8 == 0 && v.off % 8 == 0 && (reinterpret_cast<uintptr_t>(v.p) & 15) == 0;
  };
  return cin % 32 == 0 && cout % 32 == 0 && x.C == cin && g.C == cout && x.H == g.H && x.W == g.W &&
         x.H > 0 && x.W > 0 && x.H % kWgT == 0 && x.W % kWgT == 0 && vec_ok(x) && vec_ok(g);
}

int wgrad3_splits(const View& x, int B, int cin, int cout) {
  const int n_tiles = B * (x.H / kWgT) * (x.W / kWgT);
  const int slices = (cout / 32) * (cin / 32);
  return std::max(1, std::min(n_tiles, kWgTargetBlocks / slices));
}

void launch_wgrad3(const View& x, const View& g, int B, int cin, int cout, int nsplit, float* part, float* bpart,
                   hipStream_t s) {
  const int n_tiles = B * (x.H / kWgT) * (x.W / kWgT);
  hipLaunchKernelGGL(wgrad3_kernel, dim3((unsigned)nsplit, (unsigned)(cout / 32), (unsigned)(cin / 32)),
                     dim3(256), 0, s, x, g, part, bpart, cout, cin, n_tiles);
  PAT_HIP(hipGetLastError());
}

// The weight and bias gradients of a 3x3 convolution of a one-channel input
// (the first layer): dW[co][tap] = sum_p g[p][co] x[p + off(tap)] and
// db[co] = sum_p g[p][co] in one MFMA per output-channel fragment and k step,
// the 16 columns of B being the nine taps' shifted views of the input, a
// ones column (the bias) and zeros. Per 16 x 16-pixel tile the gradient is
// staged transposed as in wgrad3_kernel and the input's one-channel halo in
// three column-shifted copies; wave w takes output channels 16 w .. + 15
// (cout / 16 waves). Partials: part[blockIdx.x][co][tap], bpart[blockIdx.x][co].
constexpr int kW1MaxC = 64;

__global__ __launch_bounds__(256) void wgrad1_kernel(View x, View g, float* __restrict__ part,
                                                     float* __restrict__ bpart, int cout, int n_tiles) {
  __shared__ __align__(16) uint16_t gT[kW1MaxC * kWgGLD];
  __shared__ __align__(16) uint16_t xs[3 * kWgXLD];
  const int H = x.H, W = x.W;
  const int tiles_x = W / kWgT, tiles_y = H / kWgT;
  const int t = threadIdx.x, nt = blockDim.x, cf = t / 64, lane = t % 64, q = lane / 16, r16 = lane % 16;
  const int gv = cout / 8;  // 16-byte vectors per gradient pixel
  v8bf ones, zeros;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    ones[j] = (__bf16)1.0f;
    zeros[j] = (__bf16)0.0f;
  }
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    int tt = tile;
    const int tx = tt % tiles_x;
    tt /= tiles_x;
    const int ty = tt % tiles_y, b = tt / tiles_y;
    const int x0 = tx * kWgT, y0 = ty * kWgT;
    for (int e = t; e < kWgT * kWgT * gv; e += nt) {
      const int px = e % (kWgT * kWgT), cv = e / (kWgT * kWgT);
      const int yy = y0 + px / kWgT, xx = x0 + px % kWgT;
      const uint4 v = *reinterpret_cast<const uint4*>(g.p + ((int64_t)(b * H + yy) * W + xx) * g.pitch + g.off + 8 * cv);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 8; ++i) gT[(8 * cv + i) * kWgGLD + px] = (uint16_t)(w[i >> 1] >> (16 * (i & 1)));
    }
    for (int px = t; px < (kWgT + 2) * (kWgT + 2); px += nt) {
      const int hy = px / (kWgT + 2), hx = px % (kWgT + 2);
      const int yy = y0 + hy - 1, xx = x0 + hx - 1;
      const uint16_t v = (yy >= 0 && yy < H && xx >= 0 && xx < W)
                             ? x.p[((int64_t)(b * H + yy) * W + xx) * x.pitch + x.off]
                             : (uint16_t)0;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int col = hx - dx;
        if (col >= 0 && col < kWgT) xs[dx * kWgXLD + hy * kWgT + col] = v;
      }
    }
    __syncthreads();
    for (int st = 0; st < kWgT / 2; ++st) {
      const int row = 2 * st + (q >> 1), col = 8 * (q & 1);
      const v8bf a = *reinterpret_cast<const v8bf*>(gT + (16 * cf + r16) * kWgGLD + row * kWgT + col);
      v8bf bx = zeros;
      if (r16 < 9)
        bx = *reinterpret_cast<const v8bf*>(xs + (r16 % 3) * kWgXLD + (row + r16 / 3) * kWgT + col);
      else if (r16 == 9)
        bx = ones;
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bx, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // D[4 q + r][r16]: output channel 16 cf + 4 q + r; column r16 a tap (< 9) or the bias (9)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int co = 16 * cf + 4 * q + r;
    if (r16 < 9) part[((int64_t)blockIdx.x * cout + co) * 9 + r16] = acc[r];
    else if (r16 == 9) bpart[(int64_t)blockIdx.x * cout + co] = acc[r];
  }
}

bool wgrad1_applies(const View& x, const View& g, int cin, int cout) {
  return cin == 1 && x.C == 1 && g.C == cout && cout % 16 == 0 && cout <= kW1MaxC && x.H == g.H &&
         x.W == g.W && x.H > 0 && x.W > 0 && x.H % kWgT == 0 && x.W % kWgT == 0 && g.pitch % 8 == 0 &&
         g.off % 8 == 0 && (reinterpret_cast<uintptr_t>(g.p) & 15) == 0;
}

int wgrad1_splits(const View& x, int B) {
  const int n_tiles = B * (x.H / kWgT) * (x.W / kWgT);
  return std::max(1, std::min(n_tiles, kWgTargetBlocks));
}

void launch_wgrad1(const View& x, const View& g, int B, int cout, int nsplit, float* part, float* bpart,
                   hipStream_t s) {
  const int n_tiles = B * (x.H / kWgT) * (x.W / kWgT);
  hipLaunchKernelGGL(wgrad1_kernel, dim3((unsigned)nsplit), dim3(64 * (cout / 16)), 0, s, x, g, part, bpart, cout,
                     n_tiles);
  PAT_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ the GEMM

// WM x WN waves, each computing FM x FN 16x16 fragments: a TM x TN tile with
// TM = 16 WM FM, TN = 16 WN FN. AV, BV: the operands' vector modes when fixed
// at compile time (-1: from the descriptor).
template <int WM, int WN, int FM, int FN, int AV, int BV>
__global__ __launch_bounds__(256) void gemm_kernel(GemmDesc d) {
  // 64-wide k chunks for the row-major operands of the weight gradients (long k,
  // split across workgroups), 32 elsewhere (fewer registers, more workgroups per CU)
  constexpr int TM = 16 * WM * FM, TN = 16 * WN * FN, KC = (AV == 2 && BV == 2) ? 64 : 32, LD = KC + 8;
  __shared__ __align__(16) uint16_t As[TM * LD];
  __shared__ __align__(16) uint16_t Bs[TN * LD];
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
  const int kb = blockIdx.z * d.ksplit;
  const int ke = min(d.K, kb + d.ksplit);
  const int t = threadIdx.x, wave = t / 64, lane = t % 64;
  const int wm = wave / WN, wn = wave % WN;
  v4f acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  // fixed vector modes: chunk n + 1 is loaded into registers while chunk n is
  // multiplied
  constexpr bool PIPE = AV > 0 && BV > 0;
  ChunkRegs<true, TM, KC, LD, PIPE ? AV : 1> ca;
  ChunkRegs<false, TN, KC, LD, PIPE ? BV : 1> cb;
  if (PIPE) {
    ca.load(d, m0, kb, ke, t);
    cb.load(d, n0, kb, ke, t);
  }
  for (int k0 = kb; k0 < ke; k0 += KC) {
    // stage A (TM x KC) and B (TN x KC); element (row, kk) -> row * LD + kk
    if (PIPE) {
      ca.store(As, t);
      cb.store(Bs, t);
    } else {
      stage<true, TM, KC, LD, AV>(d, As, m0, k0, ke, t);
      stage<false, TN, KC, LD, BV>(d, Bs, n0, k0, ke, t);
    }
    __syncthreads();
    if (PIPE && k0 + KC < ke) {
      ca.load(d, m0, k0 + KC, ke, t);
      cb.load(d, n0, k0 + KC, ke, t);
    }
#pragma unroll
    for (int ks = 0; ks < KC; ks += 32) {
      v8bf a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        a[i] = *reinterpret_cast<const v8bf*>(As + (wm * 16 * FM + i * 16 + lane % 16) * LD + ks + 8 * (lane / 16));
#pragma unroll
      for (int j = 0; j < FN; ++j)
        b[j] = *reinterpret_cast<const v8bf*>(Bs + (wn * 16 * FN + j * 16 + lane % 16) * LD + ks + 8 * (lane / 16));
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue
  if (d.out_mode == E_SHUF && d.out.C % 8 == 0 && d.out.pitch % 8 == 0 && d.out.off % 8 == 0 &&
      (reinterpret_cast<uintptr_t>(d.out.p16) & 15) == 0) {
    // m: low-res pixel (b, y, x), n = sub * C + c -> output pixel
    // (2y + sub / 2, 2x + sub % 2), channel c. The tile leaves through LDS (the
    // A staging space, free after the last chunk's barrier) in passes of 32
    // columns: bias and bf16 per element, then 16-byte stores of 8 columns
    // (8 consecutive channels of one output pixel, C being a multiple of 8)
    const View& o = d.out;
    constexpr int SLD = 40;
    static_assert(SLD <= LD, "a staged pass must fit the A staging space");
#pragma unroll
    for (int pass = 0; pass < TN / 32; ++pass) {
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int cl = wn * 16 * FN + j * 16;  // the fragment's first column in the tile
        if (cl / 32 != pass) continue;
        const int n = n0 + cl + lane % 16;
        float bc = 0.f;
        if (d.bias && n < d.N) {
          int sub, c;
          chan_split(n, o.dC, sub, c);
          bc = d.bias[c];
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float v = acc[i][j][r];
            if (d.bias) v += bc;
            As[(wm * 16 * FM + i * 16 + 4 * (lane / 16) + r) * SLD + cl % 32 + lane % 16] = f2bf(v);
          }
      }
      __syncthreads();
      for (int e = t; e < TM * 4; e += 256) {
        const int row = e / 4, cv = e % 4;
        const int m = m0 + row, n = n0 + 32 * pass + 8 * cv;
        if (m < d.M && n < d.N) {
          int b, y, x, sub, c;
          pix_split(m, o.dW2, o.dH2, b, y, x);
          chan_split(n, o.dC, sub, c);
          const int yy = 2 * y + (sub >> 1), xx = 2 * x + (sub & 1);
          *reinterpret_cast<uint4*>(o.p16 + ((int64_t)(b * o.H + yy) * o.W + xx) * o.pitch + o.off + c) =
              *reinterpret_cast<const uint4*>(As + row * SLD + 8 * cv);
        }
      }
      __syncthreads();
    }
    return;
  }
  if (d.out_mode == E_SHUF) {
    // the same element by element (channel counts that are not multiples
    // of 8): each row's pixel and each column's sub-pixel offset split once
    const View& o = d.out;
    int64_t base[FM][4];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 16 * FM + i * 16 + 4 * (lane / 16) + r;
        base[i][r] = -1;
        if (m < d.M) {
          int b, y, x;
          pix_split(m, o.dW2, o.dH2, b, y, x);
          base[i][r] = ((int64_t)(b * o.H + 2 * y) * o.W + 2 * x) * o.pitch + o.off;
        }
      }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn * 16 * FN + j * 16 + lane % 16;
      if (n >= d.N) continue;
      int sub, c;
      chan_split(n, o.dC, sub, c);
      const int64_t so = ((int64_t)(sub >> 1) * o.W + (sub & 1)) * o.pitch + c;
      const float bc = d.bias ? d.bias[c] : 0.f;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (base[i][r] < 0) continue;
          float v = acc[i][j][r];
          if (d.bias) v += bc;
          o.p16[base[i][r] + so] = f2bf(v);
        }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn * 16 * FN + j * 16 + lane % 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 16 * FM + i * 16 + 4 * (lane / 16) + r;
        if (m >= d.M || n >= d.N) continue;
        float v = acc[i][j][r];
        if (d.out_mode == E_SPLIT) {
          d.out_f32[((int64_t)blockIdx.z * d.M + m) * d.N + n] = v;
          continue;
        }
        if (d.out_mode == E_ACT) {
          if (d.bias) v += d.bias[n];
          if (d.relu) v = fmaxf(v, 0.f);
          uint16_t h = f2bf(v);
          if (d.mask.p && !(bf2f(d.mask.p[(int64_t)m * d.mask.pitch + d.mask.off + n]) > 0.f)) h = 0;
          d.out.p16[(int64_t)m * d.out.pitch + d.out.off + n] = h;
        }
      }
    }
  }
}

static bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// 8-element vectors stay inside one tensor row (a tap or sub-pixel block of
// C channels) and are 16-byte aligned when channel counts, pitches, offsets
// and base pointers are multiples of 8 elements and split-K chunks start on
// multiples of 8.
static void choose_vec(GemmDesc& d) {
  d.a_vec = d.b_vec = 0;
  if (d.ksplit % 8 != 0) return;
  const View& a = d.a;
  if (d.K % 8 != 0) return;
  const bool a_rows = a.p && al16(a.p) && a.pitch % 8 == 0 && a.off % 8 == 0;
  // along rows (mode 2): also whole groups of 8 rows
  switch (d.a_mode) {
    case A_DIRECT: if (a_rows) d.a_vec = 1; break;
    case A_CONV:
    case A_G22: if (a_rows && a.C % 8 == 0) d.a_vec = 1; break;
    case A_T: if (a_rows && d.M % 8 == 0) d.a_vec = 2; break;
    case A_TG22: if (a_rows && a.C % 8 == 0 && d.M % 8 == 0) d.a_vec = 2; break;
  }
  const View& b = d.b;
  const bool b_rows = b.p && al16(b.p) && b.pitch % 8 == 0 && b.off % 8 == 0;
  switch (d.b_mode) {
    case B_W: if (d.w && al16(d.w) && d.K % 8 == 0) d.b_vec = 1; break;
    case B_IM2COL: if (b_rows && b.C % 8 == 0 && d.N % 8 == 0) d.b_vec = 2; break;
    case B_T: if (b_rows && d.N % 8 == 0) d.b_vec = 2; break;
  }
}

// Tile rule of launch_gemm (process-wide): 0 automatic, 1 the largest tile
// the column count allows, 2 128x64, 3 64x64 (for N > 32 and M > 32; N <= 32
// always takes 128x32, M <= 32 32x64). Each output element accumulates along
// k in the same chunks.
static int g_gemm_tiles = 0;
void set_gemm_tiles(int mode) { g_gemm_tiles = mode; }

// Launch one tile shape with the operands' vector modes as template arguments
// where they are the common pairs (both along k, both along rows).
template <int WM, int WN, int FM, int FN>
static void launch_tile(const GemmDesc& d, dim3 grid, hipStream_t s) {
  if (d.a_vec == 1 && d.b_vec == 1)
    hipLaunchKernelGGL((gemm_kernel<WM, WN, FM, FN, 1, 1>), grid, dim3(256), 0, s, d);
  else if (d.a_vec == 2 && d.b_vec == 2)
    hipLaunchKernelGGL((gemm_kernel<WM, WN, FM, FN, 2, 2>), grid, dim3(256), 0, s, d);
  else
    hipLaunchKernelGGL((gemm_kernel<WM, WN, FM, FN, -1, -1>), grid, dim3(256), 0, s, d);
}

void launch_gemm(const GemmDesc& d_in, hipStream_t s) {
  GemmDesc d = d_in;
  d.a.prep_div();
  d.b.prep_div();
  d.out.prep_div();
  choose_vec(d);
  const int nsplit = (d.K + d.ksplit - 1) / d.ksplit;
  // the largest tile that still gives every CU a few workgroups
  const int64_t min_blocks = g_gemm_tiles == 1 ? 0 : (g_gemm_tiles >= 2 ? INT64_MAX : 1024);
  auto blocks = [&](int tm, int tn) { return (int64_t)((d.M + tm - 1) / tm) * ((d.N + tn - 1) / tn) * nsplit; };
  if (conv3_applies(d)) {
    const int64_t n_blk = (int64_t)(d.M / (d.a.H * d.a.W)) * (d.a.H / kCvTH) * (d.a.W / kCvTW);
    hipLaunchKernelGGL(conv3_kernel, dim3((unsigned)n_blk, (unsigned)(d.N / 32)), dim3(kCvThreads), 0, s, d);
  } else if (conv_in_applies(d)) {
    hipLaunchKernelGGL(conv_in_kernel, dim3((unsigned)((d.M + 255) / 256)), dim3(256), 0, s, d);
  } else if (d.N <= 32) {
    launch_tile<4, 1, 2, 2>(d, dim3((d.M + 127) / 128, (d.N + 31) / 32, nsplit), s);
  } else if (d.M <= 32) {
    // the weight gradients of 32-channel layers: 32 x 64 tiles
    launch_tile<2, 2, 1, 2>(d, dim3((d.M + 31) / 32, (d.N + 63) / 64, nsplit), s);
  } else if (d.N >= 128 && blocks(128, 128) >= min_blocks) {
    launch_tile<2, 2, 4, 4>(d, dim3((d.M + 127) / 128, (d.N + 127) / 128, nsplit), s);
  } else if (g_gemm_tiles == 2 || blocks(128, 64) >= min_blocks) {
    launch_tile<2, 2, 4, 2>(d, dim3((d.M + 127) / 128, (d.N + 63) / 64, nsplit), s);
  } else {
    launch_tile<2, 2, 2, 2>(d, dim3((d.M + 63) / 64, (d.N + 63) / 64, nsplit), s);
  }
  PAT_HIP(hipGetLastError());
}

// out[m][n] (with optional [ci][co] <- [(a,e,co)][ci] permutation) = sum_z part[z][m][n]
// A thread takes V consecutive elements (V = 4: 16-byte loads, when M N is a
// multiple of 4) and a workgroup 256 V / lanes of them; the lanes of an
// element group add the partials z = lane, lane + lanes, ... and then the
// lane sums in lane order. lanes (8 or 32) follows from the shape alone: more
// lanes when the partials are many and the elements too few to fill the
// device.
template <int V>
__device__ __forceinline__ void splitk_reduce_block(const float* __restrict__ part, int nsplit, int M, int N,
                                                    float* __restrict__ out, int permute_cout, int lanes,
                                                    int blk, float* lds) {
  const int els = 256 / lanes;
  const int64_t total = (int64_t)M * N;
  const int el = threadIdx.x % els, zl = threadIdx.x / els;
  const int64_t i = ((int64_t)blk * els + el) * V;
  float s[V];
#pragma unroll
  for (int j = 0; j < V; ++j) s[j] = 0.f;
  if (i < total) {
    for (int z = zl; z < nsplit; z += lanes) {
      if constexpr (V == 4) {
        const float4 v = *reinterpret_cast<const float4*>(part + (int64_t)z * total + i);
        s[0] += v.x;
        s[1] += v.y;
        s[2] += v.z;
        s[3] += v.w;
      } else {
        s[0] += part[(int64_t)z * total + i];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < V; ++j) lds[j * 256 + threadIdx.x] = s[j];
  __syncthreads();
  if (zl == 0 && i < total) {
#pragma unroll
    for (int j = 0; j < V; ++j) {
      float sj = s[j];
      for (int l = 1; l < lanes; ++l) sj += lds[j * 256 + l * els + el];
      const int64_t ij = i + j;
      if (permute_cout > 0) {
        // row m = sub * Cout + co, column n = ci -> [sub][ci][co]
        const int m = (int)(ij / N), n = (int)(ij % N);
        const int sub = m / permute_cout, co = m % permute_cout;
        out[((int64_t)sub * N + n) * permute_cout + co] = sj;
      } else {
        out[ij] = sj;
      }
    }
  }
}

static int splitk_lanes(int nsplit, int64_t groups) {
  int lanes = 8;
  if (4 * lanes <= nsplit && (groups * lanes + 255) / 256 < 1024) lanes *= 4;
  return lanes;
}

// out[c] = sum over the nblk rows of part[.][c] (ld floats per row), one
// workgroup per column
__device__ __forceinline__ void part_reduce_block(const float* __restrict__ part, int nblk, int ld,
                                                  float* __restrict__ out, int c) {
  float s = 0.f;
  for (int b = threadIdx.x; b < nblk; b += 256) s += part[(int64_t)b * ld + c];
  __shared__ float lds[8];
  s = block_sum<256>(s, lds);
  if (threadIdx.x == 0) out[c] = s;
}

// Every weight gradient's two reductions of a backward pass in one launch:
// entry k of the table owns workgroups [first_block, next entry's): the first
// nb_split sum its split-K partials, the next bC the bias column sums'
// per-workgroup partials (bnblk rows of bC). Each entry's partials have their
// own buffers, so the reductions wait only for the end of the backward pass.
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(WgReduceTable tb) {
  __shared__ float lds[256 * 4];
  int li = 0;
  for (int k = 1; k < tb.count; ++k)
    if ((int)blockIdx.x >= tb.e[k].first_block) li = k;
  const WgReduce r = tb.e[li];
  const int blk = (int)blockIdx.x - r.first_block;
  if (blk < r.nb_split) {
    if (r.vec)
      splitk_reduce_block<4>(r.part, r.nsplit, r.M, r.N, r.out, r.permute_cout, r.lanes, blk, lds);
    else
      splitk_reduce_block<1>(r.part, r.nsplit, r.M, r.N, r.out, r.permute_cout, r.lanes, blk, lds);
  } else {
    part_reduce_block(r.bpart, r.bnblk, r.bC, r.bout, blk - r.nb_split);
  }
}

void wgrad_reduce_add(WgReduceTable& tb, const float* part, int nsplit, int M, int N, float* out, int permute_cout,
                      const float* bpart, int bnblk, int bC, float* bout) {
  PAT_CHECK_ARG(tb.count < kMaxWgReduce, "too many weight gradients for one reduction launch");
  const int64_t total = (int64_t)M * N;
  WgReduce& r = tb.e[tb.count];
  r.part = part;
  r.out = out;
  r.bpart = bpart;
  r.bout = bout;
  r.nsplit = nsplit;
  r.M = M;
  r.N = N;
  r.permute_cout = permute_cout;
  r.bnblk = bnblk;
  r.bC = bC;
  r.vec = total % 4 == 0 && (reinterpret_cast<uintptr_t>(part) & 15) == 0;
  const int64_t groups = r.vec ? total / 4 : total;
  r.lanes = splitk_lanes(nsplit, groups);
  r.nb_split = (int)((groups + 256 / r.lanes - 1) / (256 / r.lanes));
  r.first_block = tb.count == 0 ? 0 : tb.e[tb.count - 1].first_block + tb.e[tb.count - 1].nb_split + tb.e[tb.count - 1].bC;
  ++tb.count;
}

void launch_wgrad_reduce(const WgReduceTable& tb, hipStream_t s) {
  if (tb.count == 0) return;
  const WgReduce& last = tb.e[tb.count - 1];
  const int blocks = last.first_block + last.nb_split + last.bC;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, tb);
  PAT_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ pooling

// y[b][i][j][c] = max of the 2x2 window; idx = first maximum (row-major window order)
__global__ __launch_bounds__(256) void maxpool_kernel(View in, View out, uint8_t* __restrict__ idx,
                                                      int B) {
  const int H2 = in.H / 2, W2 = in.W / 2, C = in.C;
  const int64_t total = (int64_t)B * H2 * W2 * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t p = e / C;
    const int x = (int)(p % W2), t = (int)(p / W2), y = t % H2, b = t / H2;
    float best = -INFINITY;
    int bi = 0;
    for (int q = 0; q < 4; ++q) {
      const int yy = 2 * y + (q >> 1), xx = 2 * x + (q & 1);
      const float v = bf2f(in.p[((int64_t)(b * in.H + yy) * in.W + xx) * in.pitch + in.off + c]);
      if (v > best) { best = v; bi = q; }
    }
    out.p16[p * out.pitch + out.off + c] = f2bf(best);
    idx[e] = (uint8_t)bi;
  }
}

// g_in = bf16(route(g_out) + g_skip) * (act > 0), over the full-resolution grid
__global__ __launch_bounds__(256) void maxpool_back_kernel(View gout, const uint8_t* __restrict__ idx,
                                                           View gskip, View act, View gin, int B) {
  const int H = gin.H, W = gin.W, C = gin.C, W2 = W / 2, H2 = H / 2;
  const int64_t total = (int64_t)B * H * W * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t p = e / C;
    const int x = (int)(p % W), t = (int)(p / W), y = t % H, b = t / H;
    const int64_t q = ((int64_t)(b * H2 + y / 2) * W2 + x / 2);
    const int pos = ((y & 1) << 1) | (x & 1);
    float v = (idx[q * C + c] == pos) ? bf2f(gout.p[q * gout.pitch + gout.off + c]) : 0.f;
    v += bf2f(gskip.p[p * gskip.pitch + gskip.off + c]);
    uint16_t h = f2bf(v);
    if (!(bf2f(act.p[p * act.pitch + act.off + c]) > 0.f)) h = 0;
    gin.p16[p * gin.pitch + gin.off + c] = h;
  }
}

// The same two operations on 8 channels per thread (16-byte loads and stores of
// the activations, 8-byte ones of the window indices), element by element the
// same arithmetic; taken when every view's channels, pitch and offset are
// multiples of 8 and the pointers 16-byte aligned. Index e runs over
// (pixel, channel group) pairs; the divisions by C / 8, the width and the
// height take their host-computed multiply-high constants.
__device__ __forceinline__ uint16_t half16(const uint32_t (&w)[4], int i) {
  return (uint16_t)(w[i >> 1] >> (16 * (i & 1)));
}

__global__ __launch_bounds__(256) void maxpool8_kernel(View in, View out, uint8_t* __restrict__ idx,
                                                       uint32_t total, FastDiv dG, FastDiv dW2, FastDiv dH2) {
  const int C = in.C;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    uint32_t p, cg, t, x, b, y;
    fast_divmod(e, dG, p, cg);
    fast_divmod(p, dW2, t, x);
    fast_divmod(t, dH2, b, y);
    const int c = 8 * (int)cg;
    uint32_t w[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t src = (int64_t)(b * in.H + 2 * y + (q >> 1)) * in.W + 2 * x + (q & 1);
      const uint4 v = *reinterpret_cast<const uint4*>(in.p + src * in.pitch + in.off + c);
      w[q][0] = v.x; w[q][1] = v.y; w[q][2] = v.z; w[q][3] = v.w;
    }
    uint32_t o[4] = {0u, 0u, 0u, 0u}, ix[2] = {0u, 0u};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float best = -INFINITY;
      int bi = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float v = bf2f(half16(w[q], i));
        if (v > best) { best = v; bi = q; }
      }
      o[i >> 1] |= (uint32_t)f2bf(best) << (16 * (i & 1));
      ix[i >> 2] |= (uint32_t)bi << (8 * (i & 3));
    }
    *reinterpret_cast<uint4*>(out.p16 + (int64_t)p * out.pitch + out.off + c) = make_uint4(o[0], o[1], o[2], o[3]);
    *reinterpret_cast<uint2*>(idx + (int64_t)p * C + c) = make_uint2(ix[0], ix[1]);
  }
}

__global__ __launch_bounds__(256) void maxpool_back8_kernel(View gout, const uint8_t* __restrict__ idx,
                                                            View gskip, View act, View gin, uint32_t total,
                                                            FastDiv dG, FastDiv dW, FastDiv dH) {
  const int C = gin.C, W2 = gin.W / 2, H2 = gin.H / 2;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    uint32_t p, cg, t, x, b, y;
    fast_divmod(e, dG, p, cg);
    fast_divmod(p, dW, t, x);
    fast_divmod(t, dH, b, y);
    const int c = 8 * (int)cg;
    const int64_t q = (int64_t)(b * H2 + y / 2) * W2 + x / 2;
    const uint32_t pos = ((y & 1) << 1) | (x & 1);
    const uint2 iv = *reinterpret_cast<const uint2*>(idx + q * C + c);
    const uint4 go = *reinterpret_cast<const uint4*>(gout.p + q * gout.pitch + gout.off + c);
    const uint4 gs = *reinterpret_cast<const uint4*>(gskip.p + (int64_t)p * gskip.pitch + gskip.off + c);
    const uint4 av = *reinterpret_cast<const uint4*>(act.p + (int64_t)p * act.pitch + act.off + c);
    const uint32_t wo[4] = {go.x, go.y, go.z, go.w}, ws[4] = {gs.x, gs.y, gs.z, gs.w},
                   wa[4] = {av.x, av.y, av.z, av.w}, wi[2] = {iv.x, iv.y};
    uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t sel = (wi[i >> 2] >> (8 * (i & 3))) & 0xffu;
      float v = (sel == pos) ? bf2f(half16(wo, i)) : 0.f;
      v += bf2f(half16(ws, i));
      uint16_t h = f2bf(v);
      if (!(bf2f(half16(wa, i)) > 0.f)) h = 0;
      o[i >> 1] |= (uint32_t)h << (16 * (i & 1));
    }
    *reinterpret_cast<uint4*>(gin.p16 + (int64_t)p * gin.pitch + gin.off + c) = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

static bool vec8_view(const View& v) {
  return v.C % 8 == 0 && v.pitch % 8 == 0 && v.off % 8 == 0 &&
         (reinterpret_cast<uintptr_t>(v.p) & 15) == 0;
}

void launch_maxpool(const View& in, const View& out, uint8_t* idx, int B, hipStream_t s) {
  const int64_t total = (int64_t)B * (in.H / 2) * (in.W / 2) * in.C;
  if (vec8_view(in) && vec8_view(out) && (reinterpret_cast<uintptr_t>(idx) & 7) == 0 && total / 8 < (1ll << 31)) {
    const int64_t groups = total / 8;
    const int blocks = (int)std::min<int64_t>((groups + 255) / 256, 16384);
    hipLaunchKernelGGL(maxpool8_kernel, dim3(blocks), dim3(256), 0, s, in, out, idx, (uint32_t)groups,
                       make_fastdiv((uint32_t)(in.C / 8)), make_fastdiv((uint32_t)(in.W / 2)),
                       make_fastdiv((uint32_t)(in.H / 2)));
  } else {
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(maxpool_kernel, dim3(blocks), dim3(256), 0, s, in, out, idx, B);
  }
  PAT_HIP(hipGetLastError());
}

void launch_maxpool_back(const View& gout, const uint8_t* idx, const View& gskip, const View& act,
                         const View& gin, int B, hipStream_t s) {
  const int64_t total = (int64_t)B * gin.H * gin.W * gin.C;
  if (vec8_view(gout) && vec8_view(gskip) && vec8_view(act) && vec8_view(gin) &&
      (reinterpret_cast<uintptr_t>(idx) & 7) == 0 && total / 8 < (1ll << 31)) {
    const int64_t groups = total / 8;
    const int blocks = (int)std::min<int64_t>((groups + 255) / 256, 16384);
    hipLaunchKernelGGL(maxpool_back8_kernel, dim3(blocks), dim3(256), 0, s, gout, idx, gskip, act, gin,
                       (uint32_t)groups, make_fastdiv((uint32_t)(gin.C / 8)), make_fastdiv((uint32_t)gin.W),
                       make_fastdiv((uint32_t)gin.H));
  } else {
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(maxpool_back_kernel, dim3(blocks), dim3(256), 0, s, gout, idx, gskip, act, gin, B);
  }
  PAT_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ head, loss, biases

// y[k] plane of pixel p = sum_c h[p][c] bf16(w[k][c]) + b[k]  (one thread per
// pixel). Outputs are channel planes: y[((p / hw) K + k) hw + p % hw].
__global__ __launch_bounds__(256) void head_kernel(View h, const float* __restrict__ w,
                                                   const float* __restrict__ b, float* __restrict__ y,
                                                   int64_t P, int K, int64_t hw, FastDiv dhw) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h.C % 8 == 0 && h.C <= 256 && h.pitch % 8 == 0 && h.off % 8 == 0 && K <= 4 &&
      (reinterpret_cast<uintptr_t>(h.p) & 15) == 0 && P < (int64_t)UINT32_MAX) {
    // the bf16-rounded weights in LDS; the pixel's channels in 16-byte loads;
    // each output adds over c in order
    __shared__ float wl[4 * 256];
    for (int e = threadIdx.x; e < K * h.C; e += blockDim.x) wl[e] = bf2f(f2bf(w[e]));
    __syncthreads();
    if (p >= P) return;
    uint32_t img, pix;
    fast_divmod((uint32_t)p, dhw, img, pix);
    const int64_t base = (int64_t)img * K * hw + pix;
    const uint16_t* row = h.p + p * h.pitch + h.off;
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < h.C; c0 += 8) {
      const uint4 v = *reinterpret_cast<const uint4*>(row + c0);
      const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const float x = bf2f((uint16_t)(dw[i >> 1] >> (16 * (i & 1))));
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < K) s[k] += x * wl[k * h.C + c0 + i];
      }
    }
    for (int k = 0; k < K; ++k) y[base + k * hw] = s[k] + b[k];
    return;
  }
  if (p >= P) return;
  const int64_t base = (p / hw) * K * hw + p % hw;
  const uint16_t* row = h.p + p * h.pitch + h.off;
  for (int k = 0; k < K; ++k) {
    float s = 0.f;
    for (int c = 0; c < h.C; ++c) s += bf2f(row[c]) * bf2f(f2bf(w[k * h.C + c]));
    y[base + k * hw] = s + b[k];
  }
}

void launch_head(const View& h, const float* w, const float* b, float* y, int64_t P, int K, int64_t hw,
                 hipStream_t s) {
  hipLaunchKernelGGL(head_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, h, w, b, y, P, K, hw,
                     make_fastdiv((uint32_t)hw));
  PAT_HIP(hipGetLastError());
}

// gy = 2 (y - t) / P; per-block partial sums of (y - t)^2 for the loss
__global__ __launch_bounds__(256) void mse_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                  float* __restrict__ gy, double* __restrict__ part,
                                                  int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double v = 0.0;
  if (p < P) {
    const float d = y[p] - t[p];
    gy[p] = 2.f * d / (float)P;
    v = (double)d * d;
  }
  __shared__ double lds[8];
  const double s = block_sum<256>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sum_part_kernel(const double* __restrict__ part, int n,
                                                       double scale, double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += part[i];
  __shared__ double lds[8];
  const double s = block_sum<256>(v, lds);
  if (threadIdx.x == 0) *out = s * scale;
}

void launch_mse(const float* y, const float* t, float* gy, double* part, double* loss, int64_t P,
                hipStream_t s) {
  const int blocks = (int)((P + 255) / 256);
  hipLaunchKernelGGL(mse_kernel, dim3(blocks), dim3(256), 0, s, y, t, gy, part, P);
  hipLaunchKernelGGL(sum_part_kernel, dim3(1), dim3(256), 0, s, part, blocks, 1.0 / (double)P, loss);
  PAT_HIP(hipGetLastError());
}

// head backward: gh[p][c] = bf16(sum_k gy[p][k] bf16(w[k][c])) * (h > 0), with
// gy in channel planes like y; per-block partial sums part[block][0, K C) for
// gw[k][c] = sum_p gy[p][k] h[p][c] and part[block][K C + k] for gb[k].
__global__ __launch_bounds__(256) void head_back_kernel(View h, const float* __restrict__ w,
                                                        const float* __restrict__ gy, View gh,
                                                        float* __restrict__ part, int64_t P, int K,
                                                        int64_t hw, int rows_per_block, FastDiv dhw) {
  const int C = h.C;
  const int64_t p0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t p1 = min(P, p0 + rows_per_block);
  if (C % 8 == 0 && C <= 256 && 256 % (C / 8) == 0 && K <= 4 && h.pitch % 8 == 0 && h.off % 8 == 0 &&
      gh.pitch % 8 == 0 && gh.off % 8 == 0 && (reinterpret_cast<uintptr_t>(h.p) & 15) == 0 &&
      (reinterpret_cast<uintptr_t>(gh.p16) & 15) == 0) {
    // thread t: channels 8 (t % (C/8)) .. + 7 of every (256 / (C/8))-th pixel
    // from the (t / (C/8))-th, by 16-byte loads and stores; lane sums added
    // in lane order
    const int groups = C / 8, lanes = 256 / groups, cg = threadIdx.x % groups, r = threadIdx.x / groups;
    float sw[4][8], sb[4] = {0.f, 0.f, 0.f, 0.f}, wq[4][8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        sw[k][i] = 0.f;
        wq[k][i] = k < K ? bf2f(f2bf(w[k * C + 8 * cg + i])) : 0.f;
      }
    }
    for (int64_t p = p0 + r; p < p1; p += lanes) {
      const uint4 hv4 = *reinterpret_cast<const uint4*>(h.p + p * h.pitch + h.off + 8 * cg);
      const uint32_t hw32[4] = {hv4.x, hv4.y, hv4.z, hv4.w};
      uint32_t img, pix;
      fast_divmod((uint32_t)p, dhw, img, pix);
      const int64_t g0 = (int64_t)img * K * hw + pix;
      float g[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        g[k] = k < K ? gy[g0 + k * hw] : 0.f;
        sb[k] += g[k];
      }
      uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const float hv = bf2f((uint16_t)(hw32[i >> 1] >> (16 * (i & 1))));
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (k < K) {
            sw[k][i] += g[k] * hv;
            acc += g[k] * wq[k][i];
          }
        }
        uint16_t v = f2bf(acc);
        if (!(hv > 0.f)) v = 0;
        o[i >> 1] |= (uint32_t)v << (16 * (i & 1));
      }
      *reinterpret_cast<uint4*>(gh.p16 + p * gh.pitch + gh.off + 8 * cg) = make_uint4(o[0], o[1], o[2], o[3]);
    }
    // one output k at a time through 8 KB of LDS
    __shared__ float l8[8][256];
    float* out = part + (int64_t)blockIdx.x * K * (C + 1);
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int i = 0; i < 8; ++i) l8[i][threadIdx.x] = sw[k][i];
      __syncthreads();
      if (threadIdx.x < C) {
        const int c = threadIdx.x, g8 = c / 8, i = c % 8;
        float s = l8[i][g8];
        for (int l = 1; l < lanes; ++l) s += l8[i][l * groups + g8];
        out[k * C + c] = s;
      }
      __syncthreads();
    }
    // the bias sums: the lanes of channel group 0 saw every pixel once
#pragma unroll
    for (int k = 0; k < 4; ++k) l8[k][threadIdx.x] = sb[k];
    __syncthreads();
    if (threadIdx.x < K) {
      const int k = threadIdx.x;
      float s = l8[k][0];
      for (int l = 1; l < lanes; ++l) s += l8[k][l * groups];
      out[K * C + k] = s;
    }
    return;
  } else if (C <= 256 && 256 % C == 0 && K <= 4) {
    // thread t: channel t % C over every (256 / C)-th pixel from the (t / C)-th;
    // lane sums added in lane order
    // with the data gradient of the same pixels and channel
    const int lanes = 256 / C, c = threadIdx.x % C, r = threadIdx.x / C;
    float sw[4] = {0.f, 0.f, 0.f, 0.f}, sb[4] = {0.f, 0.f, 0.f, 0.f}, wq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) wq[k] = k < K ? bf2f(f2bf(w[k * C + c])) : 0.f;
    for (int64_t p = p0 + r; p < p1; p += lanes) {
      const float hv = bf2f(h.p[p * h.pitch + h.off + c]);
      uint32_t img, pix;
      fast_divmod((uint32_t)p, dhw, img, pix);
      const int64_t g0 = (int64_t)img * K * hw + pix;
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < K) {
          const float g = gy[g0 + k * hw];
          sw[k] += g * hv;
          sb[k] += g;
          acc += g * wq[k];
        }
      }
      uint16_t v = f2bf(acc);
      if (!(hv > 0.f)) v = 0;
      gh.p16[p * gh.pitch + gh.off + c] = v;
    }
    __shared__ float lw[4][256];
    __shared__ float lb[4][256];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lw[k][threadIdx.x] = sw[k];
      lb[k][threadIdx.x] = sb[k];
    }
    __syncthreads();
    float* out = part + (int64_t)blockIdx.x * K * (C + 1);
    if (r == 0) {
      for (int k = 0; k < K; ++k) {
        float s = lw[k][c];
        for (int l = 1; l < lanes; ++l) s += lw[k][l * C + c];
        out[k * C + c] = s;
      }
    }
    // the bias sums: the lanes of channel 0 saw every pixel once
    if (threadIdx.x < K) {
      const int k = threadIdx.x;
      float s = lb[k][0];
      for (int l = 1; l < lanes; ++l) s += lb[k][l * C];
      out[K * C + k] = s;
    }
    return;
  } else {
    for (int e = threadIdx.x; e < K * (C + 1); e += blockDim.x) {
      const int k = e < K * C ? e / C : e - K * C;
      const int c = e < K * C ? e % C : -1;
      float s = 0.f;
      for (int64_t p = p0; p < p1; ++p) {
        const float g = gy[((p / hw) * K + k) * hw + p % hw];
        s += (c >= 0) ? g * bf2f(h.p[p * h.pitch + h.off + c]) : g;
      }
      part[(int64_t)blockIdx.x * K * (C + 1) + e] = s;
    }
  }
  for (int64_t e = p0 * C + threadIdx.x; e < p1 * C; e += blockDim.x) {
    const int64_t p = e / C;
    const int c = (int)(e % C);
    const int64_t g0 = (p / hw) * K * hw + p % hw;
    float acc = 0.f;
    for (int k = 0; k < K; ++k) acc += gy[g0 + k * hw] * bf2f(f2bf(w[k * C + c]));
    uint16_t v = f2bf(acc);
    if (!(bf2f(h.p[p * h.pitch + h.off + c]) > 0.f)) v = 0;
    gh.p16[p * gh.pitch + gh.off + c] = v;
  }
}

void launch_head_back(const View& h, const float* w, const float* gy, const View& gh, float* part,
                      int64_t P, int K, int64_t hw, int rows_per_block, hipStream_t s) {
  const int blocks = (int)((P + rows_per_block - 1) / rows_per_block);
  hipLaunchKernelGGL(head_back_kernel, dim3(blocks), dim3(256), 0, s, h, w, gy, gh, part, P, K, hw,
                     rows_per_block, make_fastdiv((uint32_t)hw));
  PAT_HIP(hipGetLastError());
}

// column sums of a bf16 NHWC gradient view: part[block][c] over a pixel range
// When C divides 256, thread t adds channel t % C over every (256 / C)-th
// pixel of the range from the (t / C)-th, and the 256 / C lane sums of a
// channel are added in lane order; else one thread per channel.
__global__ __launch_bounds__(256) void colsum_kernel(View g, float* __restrict__ part, int64_t P,
                                                     int rows_per_block) {
  const int64_t p0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t p1 = min(P, p0 + rows_per_block);
  const int C = g.C;
  if (C % 8 == 0 && C <= 256 && 256 % (C / 8) == 0 && g.pitch % 8 == 0 && g.off % 8 == 0 &&
      (reinterpret_cast<uintptr_t>(g.p) & 15) == 0) {
    // 16-byte loads: thread t adds channels 8 (t % (C/8)) .. + 7 over every
    // (256 / (C/8))-th pixel from the (t / (C/8))-th; lane sums in lane order
    const int groups = C / 8, lanes = 256 / groups, cg = threadIdx.x % groups, r = threadIdx.x / groups;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int64_t p = p0 + r; p < p1; p += lanes) {
      const uint4 v = *reinterpret_cast<const uint4*>(g.p + p * g.pitch + g.off + 8 * cg);
      const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 8; ++i) s[i] += bf2f((uint16_t)(dw[i >> 1] >> (16 * (i & 1))));
    }
    __shared__ float lds8[8][256];
#pragma unroll
    for (int i = 0; i < 8; ++i) lds8[i][threadIdx.x] = s[i];
    __syncthreads();
    if (threadIdx.x < C) {
      const int c = threadIdx.x, g8 = c / 8, i = c % 8;
      float acc = 0.f;
      for (int l = 0; l < lanes; ++l) acc += lds8[i][l * groups + g8];
      part[(int64_t)blockIdx.x * C + c] = acc;
    }
    return;
  }
  if (C <= 256 && 256 % C == 0) {
    const int lanes = 256 / C, c = threadIdx.x % C, r = threadIdx.x / C;
    float s = 0.f;
    for (int64_t p = p0 + r; p < p1; p += lanes) s += bf2f(g.p[p * g.pitch + g.off + c]);
    __shared__ float lds[256];
    lds[threadIdx.x] = s;
    __syncthreads();
    if (r == 0) {
      for (int l = 1; l < lanes; ++l) s += lds[l * C + c];
      part[(int64_t)blockIdx.x * C + c] = s;
    }
    return;
  }
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    float s = 0.f;
    for (int64_t p = p0; p < p1; ++p) s += bf2f(g.p[p * g.pitch + g.off + c]);
    part[(int64_t)blockIdx.x * C + c] = s;
  }
}

// the bias column sums' per-workgroup partials (rows_per_block pixels each);
// returns the number of partial rows
int launch_colsum_partials(const View& g, float* part, int64_t P, int rows_per_block, hipStream_t s) {
  const int nblk = (int)((P + rows_per_block - 1) / rows_per_block);
  hipLaunchKernelGGL(colsum_kernel, dim3(nblk), dim3(256), 0, s, g, part, P, rows_per_block);
  PAT_HIP(hipGetLastError());
  return nblk;
}

// ------------------------------------------------------------------ parameters

// Adam (Kingma & Ba) on the FP32 master copy; bc1 = 1 - beta1^t, bc2 = 1 - beta2^t
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                   float lr, float b1, float b2, float eps, float bc1,
                                                   float bc2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                 float eps, float bc1, float bc2, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
  PAT_HIP(hipGetLastError());
}

// bf16 weight layouts from the FP32 master:
//  conv3x3 [Cout][9][Cin]: forward B = same layout; dgrad B[ci][tap*Cout+co]
//  convT  [2][2][Cin][Cout]: forward B[(sub*Cout+co)][ci]; dgrad B[ci][sub*Cout+co]
// Every layer's bf16 weight copies in one launch: workgroup b serves the
// layer whose range of workgroups holds b, one weight per thread. A 3x3
// layer's weights [co][tap][ci] go to wf as they are and to wd as
// [ci][tap][co]; a transposed layer's [sub][ci][co] go to wf as
// [sub][co][ci] and to wd as [ci][sub][co].
__global__ __launch_bounds__(256) void prep_all_kernel(const float* __restrict__ params, uint16_t* __restrict__ wf,
                                                       uint16_t* __restrict__ wd, PrepTable t) {
  int li = 0;
  for (int k = 1; k < t.count; ++k)
    if ((int)blockIdx.x >= t.L[k].first_block) li = k;
  const PrepLayer L = t.L[li];
  const int64_t i = (int64_t)((int)blockIdx.x - L.first_block) * 256 + threadIdx.x;
  if (L.kind == 0) {
    if (i >= (int64_t)L.cout * 9 * L.cin) return;
    const int ci = (int)(i % L.cin);
    const int64_t r = i / L.cin;
    const int tap = (int)(r % 9), co = (int)(r / 9);
    const uint16_t h = f2bf(params[L.w + i]);
    wf[L.wf + i] = h;
    wd[L.wd + ((int64_t)ci * 9 + tap) * L.cout + co] = h;
  } else {
    if (i >= (int64_t)4 * L.cin * L.cout) return;
    const int co = (int)(i % L.cout);
    const int64_t r = i / L.cout;
    const int ci = (int)(r % L.cin), sub = (int)(r / L.cin);
    const uint16_t h = f2bf(params[L.w + i]);
    wf[L.wf + ((int64_t)sub * L.cout + co) * L.cin + ci] = h;
    wd[L.wd + (int64_t)ci * 4 * L.cout + sub * L.cout + co] = h;
  }
}

void launch_prep_all(const float* params, uint16_t* wf, uint16_t* wd, const PrepTable& t, int blocks,
                     hipStream_t s) {
  hipLaunchKernelGGL(prep_all_kernel, dim3((unsigned)blocks), dim3(256), 0, s, params, wf, wd, t);
  PAT_HIP(hipGetLastError());
}

// A training batch gathered by the epoch's order: batch image j is sample
// order[base + j], its input (img floats) to x and its target (timg floats)
// to t; workgroup row j serves image j, 4 floats per thread when VEC.
template <bool VEC>
__global__ __launch_bounds__(256) void batch_gather_kernel(const float* __restrict__ inputs,
                                                           const float* __restrict__ targets,
                                                           const int* __restrict__ order, int base, int64_t img,
                                                           int64_t timg, float* __restrict__ x,
                                                           float* __restrict__ t) {
  const int j = blockIdx.y;
  const int64_t src = order[base + j];
  const int64_t w = VEC ? 4 : 1, n_in = img / w, n = (img + timg) / w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const bool in = e < n_in;
    const float* from = in ? inputs + src * img + e * w : targets + src * timg + (e - n_in) * w;
    float* to = in ? x + j * img + e * w : t + j * timg + (e - n_in) * w;
    if (VEC) *reinterpret_cast<float4*>(to) = *reinterpret_cast<const float4*>(from);
    else *to = *from;
  }
}

void launch_batch_gather(const float* inputs, const float* targets, const int* order, int base, int B,
                         int64_t img, int64_t timg, float* x, float* t, hipStream_t s) {
  const bool vec = img % 4 == 0 && timg % 4 == 0 && (reinterpret_cast<uintptr_t>(inputs) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(targets) & 15) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(t) & 15) == 0;
  const int64_t n = (img + timg) / (vec ? 4 : 1);
  const dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 1024), (unsigned)B);
  if (vec)
    hipLaunchKernelGGL(batch_gather_kernel<true>, grid, dim3(256), 0, s, inputs, targets, order, base, img, timg, x, t);
  else
    hipLaunchKernelGGL(batch_gather_kernel<false>, grid, dim3(256), 0, s, inputs, targets, order, base, img, timg, x, t);
  PAT_HIP(hipGetLastError());
}

// f32 [P] -> bf16 NHWC view with one channel
__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ x, View out, int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < P) out.p16[p * out.pitch + out.off] = f2bf(x[p]);
}

void launch_to_bf16(const float* x, const View& out, int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, x, out, P);
  PAT_HIP(hipGetLastError());
}

}  // namespace nn
}  // namespace pat
