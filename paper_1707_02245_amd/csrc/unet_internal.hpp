// Internal definitions of the warm-start network kernels.
#pragma once

#include "fastdiv.hpp"
#include "pat_internal.hpp"

namespace pat {
namespace nn {

// NHWC bf16 view: element (pixel p, channel c) at p * pitch + off + c.
struct View {
  const uint16_t* p = nullptr;
  uint16_t* p16 = nullptr;
  int H = 0, W = 0, C = 0, pitch = 0, off = 0;
  // divisions by C, W, H, W/2 and H/2 in the kernels (set by prep_div)
  FastDiv dC, dW, dH, dW2, dH2;
  void prep_div() {
    dC = make_fastdiv((uint32_t)C);
    dW = make_fastdiv((uint32_t)W);
    dH = make_fastdiv((uint32_t)H);
    dW2 = make_fastdiv((uint32_t)(W / 2));
    dH2 = make_fastdiv((uint32_t)(H / 2));
  }
};

inline View view(uint16_t* base, int H, int W, int C, int pitch, int off) {
  View v;
  v.p = base;
  v.p16 = base;
  v.H = H;
  v.W = W;
  v.C = C;
  v.pitch = pitch;
  v.off = off;
  return v;
}

enum AMode { A_DIRECT = 0, A_CONV = 1, A_G22 = 2, A_T = 3, A_TG22 = 4 };
enum BMode { B_W = 0, B_IM2COL = 1, B_T = 2 };
enum EMode { E_ACT = 0, E_SHUF = 1, E_SPLIT = 2 };

struct GemmDesc {
  int M = 0, N = 0, K = 0, ksplit = 0;
  int a_mode = A_DIRECT, a_sign = 1;
  View a;
  int b_mode = B_W;
  View b;
  const uint16_t* w = nullptr;  // B_W: [N][K]
  int out_mode = E_ACT;
  View out;                     // E_ACT, E_SHUF
  float* out_f32 = nullptr;     // E_SPLIT: [nsplit][M][N]
  const float* bias = nullptr;
  int relu = 0;
  View mask;                    // E_ACT: zero where mask <= 0 (null p: no mask)
  // staging in 8-element (16-byte) vectors, set by launch_gemm when the
  // layout allows it: 0 element-wise, 1 along k, 2 along m (A) / n (B)
  int a_vec = 0, b_vec = 0;
};

void launch_gemm(const GemmDesc& d, hipStream_t s);
// weight gradient of a 3x3 convolution by pixel tiles (when wgrad3_applies):
// writes nsplit (wgrad3_splits) partials [split][cout][9 cin] to part and the
// bias column sums' partials [split][cout] to bpart
bool wgrad3_applies(const View& x, const View& g, int cin, int cout);
int wgrad3_splits(const View& x, int B, int cin, int cout);
void launch_wgrad3(const View& x, const View& g, int B, int cin, int cout, int nsplit, float* part, float* bpart,
                   hipStream_t s);
// the same for a one-channel input (partials [split][cout][9] and [split][cout])
bool wgrad1_applies(const View& x, const View& g, int cin, int cout);
int wgrad1_splits(const View& x, int B);
void launch_wgrad1(const View& x, const View& g, int B, int cout, int nsplit, float* part, float* bpart,
                   hipStream_t s);
void set_gemm_tiles(int mode);
// the reductions of a backward pass's weight gradients, gathered and then
// launched together (each entry: nsplit partials of M x N, the result in out,
// permuted [sub][ci][co] when permute_cout > 0; bnblk bias partial rows of bC)
struct WgReduce {
  const float* part;
  float* out;
  const float* bpart;
  float* bout;
  int nsplit, M, N, permute_cout, bnblk, bC, lanes, vec, nb_split, first_block;
};
constexpr int kMaxWgReduce = 32;
struct WgReduceTable {
  WgReduce e[kMaxWgReduce];
  int count;
};
void wgrad_reduce_add(WgReduceTable& tb, const float* part, int nsplit, int M, int N, float* out, int permute_cout,
                      const float* bpart, int bnblk, int bC, float* bout);
void launch_wgrad_reduce(const WgReduceTable& tb, hipStream_t s);
void launch_maxpool(const View& in, const View& out, uint8_t* idx, int B, hipStream_t s);
void launch_maxpool_back(const View& gout, const uint8_t* idx, const View& gskip, const View& act,
                         const View& gin, int B, hipStream_t s);
void launch_head(const View& h, const float* w, const float* b, float* y, int64_t P, int K, int64_t hw,
                 hipStream_t s);
void launch_mse(const float* y, const float* t, float* gy, double* part, double* loss, int64_t P,
                hipStream_t s);
void launch_head_back(const View& h, const float* w, const float* gy, const View& gh, float* part,
                      int64_t P, int K, int64_t hw, int rows_per_block, hipStream_t s);
int launch_colsum_partials(const View& g, float* part, int64_t P, int rows_per_block, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                 float eps, float bc1, float bc2, hipStream_t s);
// one layer of launch_prep_all: offsets in the FP32 parameters and in the two
// bf16 weight buffers, its kind (0 3x3, 1 transposed 2x2), channels, and its
// first workgroup in the launch
struct PrepLayer {
  int64_t w, wf, wd;
  int kind, cout, cin, first_block;
};
constexpr int kMaxPrepLayers = 32;
struct PrepTable {
  PrepLayer L[kMaxPrepLayers];
  int count;
};
void launch_prep_all(const float* params, uint16_t* wf, uint16_t* wd, const PrepTable& t, int blocks,
                     hipStream_t s);
void launch_to_bf16(const float* x, const View& out, int64_t P, hipStream_t s);
void launch_batch_gather(const float* inputs, const float* targets, const int* order, int base, int B,
                         int64_t img, int64_t timg, float* x, float* t, hipStream_t s);

}  // namespace nn
}  // namespace pat
