// Warm-start network driver: a 4-level U-Net whose forward and backward passes
// and Adam updates run in this library's kernels (bf16 matrix cores, FP32
// accumulation and FP32 master weights), trained on (normalised
// backprojection, PDHG solution) pairs; at inference it maps the normalised
// backprojection of new data to a starting point for PDHG. The solver's gap
// decides whether the start is kept (fallback to zero otherwise), so the
// fixed point of the reconstruction never depends on the network.
//
// Parameter order and layouts are those of the reference network: per level
// l = 0..3 the two encoder 3x3 convolutions ([Cout][3][3][Cin] + bias), then
// per decoder level l = 2..0 the 2x2 transposed convolution
// ([2][2][Cin][Cout] + bias) and two 3x3 convolutions, then the 1x1 head
// ([cout][C0] + bias). Outputs and targets are FP32 channel planes
// [batch][cout][h][w].

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <memory>
#include <random>

#include "unet_internal.hpp"

namespace pat {
namespace nn {

struct Layer {
  int kind;        // 0 conv3x3, 1 convT 2x2
  int cin, cout;
  int64_t w, b;    // offsets in the FP32 parameter vector
  int64_t wf, wd;  // offsets in the bf16 weight buffers
};

struct Act {
  int B = 0, H = 0, W = 0;
  // sized for the largest supported network (6 levels)
  DevBuf x0, y, gy, t, idx[5];
  DevBuf a[6], cat[5], s3, p[5], ua[5], ub[5];
  DevBuf g_ub[5], g_ua[5], g_cat[5], g_s3, g_a[6], g_p[5], g_s[5];
  DevBuf part, loss_part, loss;
  // per layer: its weight gradient's split partials and bias partials, kept
  // until the backward pass's one reduction launch (wred)
  DevBuf lws[kMaxWgReduce], lbp[kMaxWgReduce];
  WgReduceTable wred{};
};

}  // namespace nn
}  // namespace pat

struct pat_unet_s {
  int levels = 4, base = 32, cout = 1;
  std::vector<pat::nn::Layer> layers;  // in parameter order (head excluded)
  int64_t head_w = 0, head_b = 0, n_params = 0, n_wbf16 = 0;
  pat::DevBuf params, grads, adam_m, adam_v, wf, wd;
  int64_t step = 0;
  pat::nn::Act act;
  int ch(int l) const { return base << l; }
};

namespace pat {
namespace nn {

constexpr size_t kWorkspace = 64ull << 20;  // bound on one layer's split-K partials (bytes)

static void build_layers(pat_unet_s* n) {
  int64_t off = 0, woff = 0;
  auto add = [&](int kind, int cin, int cout) {
    Layer L{};
    L.kind = kind;
    L.cin = cin;
    L.cout = cout;
    const int64_t nw = kind == 0 ? (int64_t)cout * 9 * cin : (int64_t)4 * cin * cout;
    L.w = off;
    off += nw;
    L.b = off;
    off += cout;
    L.wf = woff;
    L.wd = woff;
    woff += nw;
    n->layers.push_back(L);
  };
  int c = 1;
  for (int l = 0; l < n->levels; ++l) {
    add(0, c, n->ch(l));
    add(0, n->ch(l), n->ch(l));
    c = n->ch(l);
  }
  for (int l = n->levels - 2; l >= 0; --l) {
    add(1, n->ch(l + 1), n->ch(l));
    add(0, 2 * n->ch(l), n->ch(l));
    add(0, n->ch(l), n->ch(l));
  }
  n->head_w = off;
  off += (int64_t)n->cout * n->ch(0);
  n->head_b = off;
  off += n->cout;
  n->n_params = off;
  n->n_wbf16 = woff;
}

// layer index helpers (parameter order)
static int enc(int l, int j) { return 2 * l + j; }                      // j = 0 (a), 1 (b)
static int dec(const pat_unet_s* n, int l, int j) {                     // j = 0 (t), 1 (a), 2 (b)
  return 2 * n->levels + 3 * (n->levels - 2 - l) + j;
}

static void prep_weights(pat_unet_s* n, hipStream_t s) {
  PAT_CHECK_ARG(n->layers.size() <= (size_t)kMaxPrepLayers, "too many layers for the weight table");
  PrepTable t{};
  int blocks = 0;
  for (const Layer& L : n->layers) {
    PrepLayer& e = t.L[t.count++];
    e.w = L.w;
    e.wf = L.wf;
    e.wd = L.wd;
    e.kind = L.kind;
    e.cout = L.cout;
    e.cin = L.cin;
    e.first_block = blocks;
    const int64_t elems = (int64_t)(L.kind == 0 ? 9 : 4) * L.cin * L.cout;
    blocks += (int)((elems + 255) / 256);
  }
  launch_prep_all(ptr<float>(n->params), ptr<uint16_t>(n->wf), ptr<uint16_t>(n->wd), t, blocks, s);
}

static void ensure_act(pat_unet_s* n, int B, int H, int W) {
  Act& a = n->act;
  if (a.B == B && a.H == H && a.W == W) return;
  PAT_CHECK_ARG(H % (1 << (n->levels - 1)) == 0 && W % (1 << (n->levels - 1)) == 0,
                "image size must be divisible by 2^(levels-1)");
  a = Act();
  a.B = B;
  a.H = H;
  a.W = W;
  auto px = [&](int l) { return (int64_t)B * (H >> l) * (W >> l); };
  const size_t h = sizeof(uint16_t);
  a.x0.alloc(h * px(0));
  a.y.alloc(sizeof(float) * px(0) * n->cout);
  a.gy.alloc(sizeof(float) * px(0) * n->cout);  // also stages the input batch
  a.t.alloc(sizeof(float) * px(0) * n->cout);
  for (int l = 0; l < n->levels; ++l) {
    a.a[l].alloc(h * px(l) * n->ch(l));
    a.g_a[l].alloc(h * px(l) * n->ch(l));
  }
  for (int l = 0; l < n->levels - 1; ++l) {
    a.cat[l].alloc(h * px(l) * 2 * n->ch(l));
    a.g_cat[l].alloc(h * px(l) * 2 * n->ch(l));
    a.p[l].alloc(h * px(l + 1) * n->ch(l));
    a.g_p[l].alloc(h * px(l + 1) * n->ch(l));
    a.idx[l].alloc(px(l + 1) * n->ch(l));
    a.ua[l].alloc(h * px(l) * n->ch(l));
    a.ub[l].alloc(h * px(l) * n->ch(l));
    a.g_ua[l].alloc(h * px(l) * n->ch(l));
    a.g_ub[l].alloc(h * px(l) * n->ch(l));
    a.g_s[l].alloc(h * px(l) * n->ch(l));
  }
  const int L3 = n->levels - 1;
  a.s3.alloc(h * px(L3) * n->ch(L3));
  a.g_s3.alloc(h * px(L3) * n->ch(L3));
  // per-block partial sums: bias gradients (256 pixels per block, up to 2 C
  // channels) and the head (256 pixels per block, cout (C0 + 1) sums)
  int64_t part = (px(0) + 255) / 256 * n->cout * (n->ch(0) + 1);
  for (int l = 0; l < n->levels; ++l) part = std::max<int64_t>(part, (px(l) + 255) / 256 * 2 * n->ch(l));
  a.part.alloc(sizeof(float) * part);
  a.loss_part.alloc(sizeof(double) * ((px(0) * n->cout + 255) / 256 + 1));
  a.loss.alloc(sizeof(double));
}

// ---------------------------------------------------------------- layer ops

static void conv_fwd(pat_unet_s* n, const Layer& L, const View& in, const View& out, bool relu,
                     hipStream_t s) {
  GemmDesc d;
  d.M = n->act.B * in.H * in.W;
  d.N = L.cout;
  d.K = 9 * L.cin;
  d.ksplit = d.K;
  d.a_mode = A_CONV;
  d.a_sign = 1;
  d.a = in;
  d.b_mode = B_W;
  d.w = ptr<uint16_t>(n->wf) + L.wf;
  d.out_mode = E_ACT;
  d.out = out;
  d.bias = ptr<float>(n->params) + L.b;
  d.relu = relu ? 1 : 0;
  launch_gemm(d, s);
}

static void convt_fwd(pat_unet_s* n, const Layer& L, const View& in, const View& out, hipStream_t s) {
  GemmDesc d;
  d.M = n->act.B * in.H * in.W;
  d.N = 4 * L.cout;
  d.K = L.cin;
  d.ksplit = d.K;
  d.a_mode = A_DIRECT;
  d.a = in;
  d.b_mode = B_W;
  d.w = ptr<uint16_t>(n->wf) + L.wf;
  d.out_mode = E_SHUF;
  d.out = out;
  d.bias = ptr<float>(n->params) + L.b;
  launch_gemm(d, s);
}

// split so that tiles x splits fill the device and the partials fit the workspace
static int choose_ksplit(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int64_t nsplit = std::max<int64_t>(1, 1024 / std::max<int64_t>(tiles, 1));
  nsplit = std::min<int64_t>(nsplit, (K + 31) / 32);
  while (nsplit > 1 && nsplit * M * N * (int64_t)sizeof(float) > (int64_t)kWorkspace) --nsplit;
  int64_t ks = (K + nsplit - 1) / nsplit;
  ks = (ks + 31) / 32 * 32;
  return (int)ks;
}

// weight gradient of a 3x3 convolution: dW[co][tap*Cin+ci] = sum_p g[p][co] X[p+tap][ci]
// (by pixel tiles where the shapes allow, else the implicit GEMM split over k);
// the partials go to the layer's own buffers and their reduction joins the
// backward pass's table
static void conv_wgrad(pat_unet_s* n, const Layer& L, const View& x, const View& g, hipStream_t s) {
  Act& a = n->act;
  const int li = (int)(&L - n->layers.data());
  const int64_t P = (int64_t)a.B * x.H * x.W;
  const size_t f = sizeof(float);
  int nsplit, bnblk;
  if (wgrad3_applies(x, g, L.cin, L.cout)) {
    // the bias partials come from the same launch, one row per split
    nsplit = wgrad3_splits(x, a.B, L.cin, L.cout);
    a.lws[li].ensure(f * nsplit * L.cout * 9 * L.cin);
    a.lbp[li].ensure(f * nsplit * L.cout);
    launch_wgrad3(x, g, a.B, L.cin, L.cout, nsplit, ptr<float>(a.lws[li]), ptr<float>(a.lbp[li]), s);
    bnblk = nsplit;
  } else if (wgrad1_applies(x, g, L.cin, L.cout)) {
    nsplit = wgrad1_splits(x, a.B);
    a.lws[li].ensure(f * nsplit * L.cout * 9);
    a.lbp[li].ensure(f * nsplit * L.cout);
    launch_wgrad1(x, g, a.B, L.cout, nsplit, ptr<float>(a.lws[li]), ptr<float>(a.lbp[li]), s);
    bnblk = nsplit;
  } else {
    bnblk = (int)((P + 255) / 256);
    a.lbp[li].ensure(f * bnblk * g.C);
    launch_colsum_partials(g, ptr<float>(a.lbp[li]), P, 256, s);
    GemmDesc d;
    d.M = L.cout;
    d.N = 9 * L.cin;
    d.K = (int)P;
    d.ksplit = choose_ksplit(d.M, d.N, d.K);
    nsplit = (d.K + d.ksplit - 1) / d.ksplit;
    a.lws[li].ensure(f * nsplit * d.M * d.N);
    d.a_mode = A_T;
    d.a = g;
    d.b_mode = B_IM2COL;
    d.b = x;
    d.out_mode = E_SPLIT;
    d.out_f32 = ptr<float>(a.lws[li]);
    launch_gemm(d, s);
  }
  wgrad_reduce_add(a.wred, ptr<float>(a.lws[li]), nsplit, L.cout, 9 * L.cin, ptr<float>(n->grads) + L.w, 0,
                   ptr<float>(a.lbp[li]), bnblk, g.C, ptr<float>(n->grads) + L.b);
}

// input gradient of a 3x3 convolution (flipped taps), rounded to bf16 and masked
static void conv_dgrad(pat_unet_s* n, const Layer& L, const View& g, const View& out, const View& mask,
                       hipStream_t s) {
  GemmDesc d;
  d.M = n->act.B * g.H * g.W;
  d.N = L.cin;
  d.K = 9 * L.cout;
  d.ksplit = d.K;
  d.a_mode = A_CONV;
  d.a_sign = -1;
  d.a = g;
  d.b_mode = B_W;
  d.w = ptr<uint16_t>(n->wd) + L.wd;
  d.out_mode = E_ACT;
  d.out = out;
  d.mask = mask;
  launch_gemm(d, s);
}

// transposed convolution: x is the low-resolution input, g the full-resolution
// output gradient
static void convt_wgrad(pat_unet_s* n, const Layer& L, const View& x, const View& g, hipStream_t s) {
  Act& a = n->act;
  const int li = (int)(&L - n->layers.data());
  const size_t f = sizeof(float);
  GemmDesc d;
  d.M = 4 * L.cout;
  d.N = L.cin;
  d.K = a.B * x.H * x.W;
  d.ksplit = choose_ksplit(d.M, d.N, d.K);
  const int nsplit = (d.K + d.ksplit - 1) / d.ksplit;
  a.lws[li].ensure(f * nsplit * d.M * d.N);
  d.a_mode = A_TG22;
  d.a = g;
  d.b_mode = B_T;
  d.b = x;
  d.out_mode = E_SPLIT;
  d.out_f32 = ptr<float>(a.lws[li]);
  const int64_t P = (int64_t)a.B * g.H * g.W;
  const int bnblk = (int)((P + 255) / 256);
  a.lbp[li].ensure(f * bnblk * g.C);
  launch_colsum_partials(g, ptr<float>(a.lbp[li]), P, 256, s);
  launch_gemm(d, s);
  wgrad_reduce_add(a.wred, d.out_f32, nsplit, d.M, d.N, ptr<float>(n->grads) + L.w, L.cout, ptr<float>(a.lbp[li]),
                   bnblk, g.C, ptr<float>(n->grads) + L.b);
}

static void convt_dgrad(pat_unet_s* n, const Layer& L, const View& g, const View& out, const View& mask,
                        hipStream_t s) {
  GemmDesc d;
  d.M = n->act.B * (g.H / 2) * (g.W / 2);
  d.N = L.cin;
  d.K = 4 * L.cout;
  d.ksplit = d.K;
  d.a_mode = A_G22;
  d.a = g;
  d.b_mode = B_W;
  d.w = ptr<uint16_t>(n->wd) + L.wd;
  d.out_mode = E_ACT;
  d.out = out;
  d.mask = mask;
  launch_gemm(d, s);
}

// ---------------------------------------------------------------- network passes

struct Views {
  View x0, a[6], s[5], cat[5], t[5], p[5], s3, ua[5], ub[5];
};

static Views views(pat_unet_s* n) {
  Act& a = n->act;
  Views v;
  auto Hl = [&](int l) { return a.H >> l; };
  auto Wl = [&](int l) { return a.W >> l; };
  v.x0 = view(ptr<uint16_t>(a.x0), a.H, a.W, 1, 1, 0);
  for (int l = 0; l < n->levels; ++l) v.a[l] = view(ptr<uint16_t>(a.a[l]), Hl(l), Wl(l), n->ch(l), n->ch(l), 0);
  for (int l = 0; l < n->levels - 1; ++l) {
    const int C = n->ch(l);
    v.cat[l] = view(ptr<uint16_t>(a.cat[l]), Hl(l), Wl(l), 2 * C, 2 * C, 0);
    v.t[l] = view(ptr<uint16_t>(a.cat[l]), Hl(l), Wl(l), C, 2 * C, 0);
    v.s[l] = view(ptr<uint16_t>(a.cat[l]), Hl(l), Wl(l), C, 2 * C, C);
    v.p[l] = view(ptr<uint16_t>(a.p[l]), Hl(l + 1), Wl(l + 1), C, C, 0);
    v.ua[l] = view(ptr<uint16_t>(a.ua[l]), Hl(l), Wl(l), C, C, 0);
    v.ub[l] = view(ptr<uint16_t>(a.ub[l]), Hl(l), Wl(l), C, C, 0);
  }
  const int L3 = n->levels - 1;
  v.s3 = view(ptr<uint16_t>(a.s3), Hl(L3), Wl(L3), n->ch(L3), n->ch(L3), 0);
  return v;
}

static void forward(pat_unet_s* n, const float* x, hipStream_t s) {
  Act& a = n->act;
  const Views v = views(n);
  const int64_t P0 = (int64_t)a.B * a.H * a.W;
  launch_to_bf16(x, v.x0, P0, s);
  View in = v.x0;
  for (int l = 0; l < n->levels; ++l) {
    conv_fwd(n, n->layers[enc(l, 0)], in, v.a[l], true, s);
    const View sk = l < n->levels - 1 ? v.s[l] : v.s3;
    conv_fwd(n, n->layers[enc(l, 1)], v.a[l], sk, true, s);
    if (l < n->levels - 1) {
      launch_maxpool(sk, v.p[l], ptr<uint8_t>(a.idx[l]), a.B, s);
      in = v.p[l];
    }
  }
  View h = v.s3;
  for (int l = n->levels - 2; l >= 0; --l) {
    convt_fwd(n, n->layers[dec(n, l, 0)], h, v.t[l], s);
    conv_fwd(n, n->layers[dec(n, l, 1)], v.cat[l], v.ua[l], true, s);
    conv_fwd(n, n->layers[dec(n, l, 2)], v.ua[l], v.ub[l], true, s);
    h = v.ub[l];
  }
  launch_head(h, ptr<float>(n->params) + n->head_w, ptr<float>(n->params) + n->head_b, ptr<float>(a.y),
              P0, n->cout, (int64_t)a.H * a.W, s);
}

static void backward(pat_unet_s* n, hipStream_t s) {
  Act& a = n->act;
  const Views v = views(n);
  a.wred.count = 0;
  const int64_t P0 = (int64_t)a.B * a.H * a.W;
  auto gview = [&](DevBuf& b, int l, int C, int pitch, int off) {
    return view(ptr<uint16_t>(b), a.H >> l, a.W >> l, C, pitch, off);
  };
  View none;
  // head: gh = bf16(sum_k gy_k w_k) * (ub0 > 0)
  const int C0 = n->ch(0);
  View g = gview(a.g_ub[0], 0, C0, C0, 0);
  const int rows = 256;
  const int nblk = (int)((P0 + rows - 1) / rows);
  launch_head_back(v.ub[0], ptr<float>(n->params) + n->head_w, ptr<float>(a.gy), g, ptr<float>(a.part), P0,
                   n->cout, (int64_t)a.H * a.W, rows, s);
  // part rows are [cout][C0] weight sums then cout bias sums: the head's
  // parameter layout, so one column reduction (an entry without split
  // partials in the backward pass's reduction launch) fills both
  const int hk = n->cout * (C0 + 1);
  wgrad_reduce_add(a.wred, nullptr, 0, 0, 0, nullptr, 0, ptr<float>(a.part), nblk, hk,
                   ptr<float>(n->grads) + n->head_w);
  // decoder, level 0 up to levels-2
  for (int l = 0; l < n->levels - 1; ++l) {
    const int C = n->ch(l);
    const Layer& Lb = n->layers[dec(n, l, 2)];
    const Layer& La = n->layers[dec(n, l, 1)];
    const Layer& Lt = n->layers[dec(n, l, 0)];
    // g is the masked gradient of ub[l]
    conv_wgrad(n, Lb, v.ua[l], g, s);
    const View gua = gview(a.g_ua[l], l, C, C, 0);
    conv_dgrad(n, Lb, g, gua, v.ua[l], s);
    conv_wgrad(n, La, v.cat[l], gua, s);
    const View gcat = gview(a.g_cat[l], l, 2 * C, 2 * C, 0);
    conv_dgrad(n, La, gua, gcat, none, s);
    // transposed convolution: gradient of its output is the first half of gcat
    const View gt = gview(a.g_cat[l], l, C, 2 * C, 0);
    const View xin = (l + 1 < n->levels - 1) ? v.ub[l + 1] : v.s3;
    convt_wgrad(n, Lt, xin, gt, s);
    const int Cn = n->ch(l + 1);
    View gnext;
    if (l + 1 < n->levels - 1) gnext = gview(a.g_ub[l + 1], l + 1, Cn, Cn, 0);
    else gnext = gview(a.g_s3, l + 1, Cn, Cn, 0);
    convt_dgrad(n, Lt, gt, gnext, xin, s);
    g = gnext;
  }
  // encoder, bottom level up
  for (int l = n->levels - 1; l >= 0; --l) {
    const int C = n->ch(l);
    const Layer& Lb = n->layers[enc(l, 1)];
    const Layer& La = n->layers[enc(l, 0)];
    if (l < n->levels - 1) {
      // g_s = bf16(route(g_p) + g_skip) * (s > 0)
      const View gp = view(ptr<uint16_t>(a.g_p[l]), a.H >> (l + 1), a.W >> (l + 1), C, C, 0);
      const View gskip = gview(a.g_cat[l], l, C, 2 * C, C);
      const View gs = gview(a.g_s[l], l, C, C, 0);
      launch_maxpool_back(gp, ptr<uint8_t>(a.idx[l]), gskip, v.s[l], gs, a.B, s);
      g = gs;
    }
    conv_wgrad(n, Lb, v.a[l], g, s);
    const View ga = gview(a.g_a[l], l, C, C, 0);
    conv_dgrad(n, Lb, g, ga, v.a[l], s);
    const View xin = l > 0 ? v.p[l - 1] : v.x0;
    conv_wgrad(n, La, xin, ga, s);
    if (l > 0) {
      const View gp = view(ptr<uint16_t>(a.g_p[l - 1]), a.H >> l, a.W >> l, n->ch(l - 1), n->ch(l - 1), 0);
      conv_dgrad(n, La, ga, gp, none, s);
      g = gp;
    }
  }
  launch_wgrad_reduce(a.wred, s);
}

static void init_params(pat_unet_s* n, uint64_t seed, hipStream_t s) {
  std::vector<float> h(n->n_params, 0.f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (const Layer& L : n->layers) {
    const int64_t nw = L.kind == 0 ? (int64_t)L.cout * 9 * L.cin : (int64_t)4 * L.cin * L.cout;
    const double fan_in = L.kind == 0 ? 9.0 * L.cin : (double)L.cin;
    const double sd = std::sqrt(2.0 / fan_in);
    for (int64_t i = 0; i < nw; ++i) h[L.w + i] = (float)(sd * nd(rng));
  }
  const double sd = std::sqrt(2.0 / n->ch(0));
  for (int64_t c = 0; c < (int64_t)n->cout * n->ch(0); ++c) h[n->head_w + c] = (float)(sd * nd(rng));
  PAT_HIP(hipMemcpyAsync(n->params.p, h.data(), sizeof(float) * n->n_params, hipMemcpyHostToDevice, s));
  PAT_HIP(hipMemsetAsync(n->adam_m.p, 0, n->adam_m.bytes, s));
  PAT_HIP(hipMemsetAsync(n->adam_v.p, 0, n->adam_v.bytes, s));
  PAT_HIP(hipStreamSynchronize(s));
}

static double train_step(pat_unet_s* n, const float* x, const float* t, double lr, hipStream_t s,
                         bool update) {
  Act& a = n->act;
  const int64_t P0 = (int64_t)a.B * a.H * a.W;
  forward(n, x, s);
  launch_mse(ptr<float>(a.y), t, ptr<float>(a.gy), ptr<double>(a.loss_part), ptr<double>(a.loss),
             P0 * n->cout, s);
  backward(n, s);
  if (update) {
    ++n->step;
    const double b1 = 0.9, b2 = 0.999;
    launch_adam(ptr<float>(n->params), ptr<float>(n->grads), ptr<float>(n->adam_m), ptr<float>(n->adam_v),
                n->n_params, (float)lr, (float)b1, (float)b2, 1e-8f, (float)(1.0 - std::pow(b1, (double)n->step)),
                (float)(1.0 - std::pow(b2, (double)n->step)), s);
    prep_weights(n, s);
  }
  return 0.0;
}

}  // namespace nn

// ---------------------------------------------------------------- warm-start pre/post-processing

template <class T>
__global__ __launch_bounds__(256) void bp_ratio_kernel(const T* __restrict__ atf, const T* __restrict__ at1,
                                                       float* __restrict__ bp, double* __restrict__ part,
                                                       int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double d = (double)at1[i];
    const double r = d > 0.0 ? (double)atf[i] / d : 0.0;
    bp[i] = (float)r;
    v = fabs(r);
  }
  __shared__ double lds[8];
  const double s = block_sum<256>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// scale = max(mean |bp|, 1e-12); x = bp / scale; target planes (if u):
// t[0] = u / scale, and with tc = 3 also t[1], t[2] = r_x / lambda, r_y / lambda
template <class T>
__global__ __launch_bounds__(256) void normalise_kernel(const double* __restrict__ part, int nblk, int64_t n,
                                                        float* __restrict__ x, const T* __restrict__ u,
                                                        const T* __restrict__ r, double inv_lam,
                                                        float* __restrict__ t, int tc,
                                                        float* __restrict__ scale_out) {
  __shared__ double sc;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b];
    sc = fmax(s / (double)n, 1e-12);
    if (blockIdx.x == 0 && scale_out) *scale_out = (float)sc;
  }
  __syncthreads();
  const double inv = 1.0 / sc;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] = (float)(x[i] * inv);
    if (u && t) {
      t[i] = (float)((double)u[i] * inv);
      if (tc == 3) {
        t[n + i] = (float)((double)r[i] * inv_lam);
        t[2 * n + i] = (float)((double)r[n + i] * inv_lam);
      }
    }
  }
}

// u0 = scale y[0]; with r0: r0 = lambda P(y[1], y[2]), P the projection onto
// the unit disc (the dual ball of TV scaled to 1)
template <class T>
__global__ __launch_bounds__(256) void rescale_kernel(const float* __restrict__ y, const float* __restrict__ scale,
                                                      T* __restrict__ u, T* __restrict__ r, double lam, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  u[i] = (T)((double)y[i] * (double)*scale);
  if (r) {
    const double a = y[n + i], b = y[2 * n + i];
    const double m = fmax(1.0, sqrt(a * a + b * b));
    r[i] = (T)(lam * a / m);
    r[n + i] = (T)(lam * b / m);
  }
}

// q0 = A u0 - f (already holding A u0)
template <class T>
__global__ __launch_bounds__(256) void residual_kernel(T* __restrict__ q, const T* __restrict__ f, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) q[i] = q[i] - f[i];
}

template <class T>
static void normalise_impl(pat_geometry g, const pat_regulariser* reg, const void* d_f, const void* d_state,
                           float* d_x, float* d_t, int tc, float* d_scale, hipStream_t s) {
  const int64_t N = g->n_pix(), nb = g->n_bins();
  DevBuf atf(sizeof(T) * N), at1(sizeof(T) * N), ones(sizeof(T) * nb);
  apply_adjoint<T>(g, static_cast<const T*>(d_f), ptr<T>(atf), s);
  launch_fill<T>(ptr<T>(ones), T(1), nb, s);
  apply_adjoint<T>(g, ptr<T>(ones), ptr<T>(at1), s);
  const int nblk = (int)((N + 255) / 256);
  DevBuf part(sizeof(double) * nblk);
  hipLaunchKernelGGL(bp_ratio_kernel<T>, dim3(nblk), dim3(256), 0, s, ptr<T>(atf), ptr<T>(at1), d_x,
                     ptr<double>(part), N);
  const T* u = static_cast<const T*>(d_state);
  const T* r = u ? u + 2 * N + nb : nullptr;  // state layout: u, ubar, q, r
  const double inv_lam = (u && tc == 3) ? 1.0 / reg->lambda : 0.0;  // reg checked by the caller then
  hipLaunchKernelGGL(normalise_kernel<T>, dim3(std::min(nblk, 1024)), dim3(256), 0, s, ptr<double>(part), nblk,
                     N, d_x, u, r, inv_lam, d_t, tc, d_scale);
  PAT_HIP(hipGetLastError());
  PAT_HIP(hipStreamSynchronize(s));  // temporaries go out of scope
}

}  // namespace pat

using pat::guarded;
using pat::nn::Act;

static void check_net(pat_unet n) { PAT_CHECK_ARG(n != nullptr, "network is NULL"); }

extern "C" pat_status pat_warmstart_create(int32_t levels, int32_t base_ch, int32_t out_ch, uint64_t seed,
                                           pat_unet* out) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(out != nullptr, "out is NULL");
    PAT_CHECK_ARG(levels >= 2 && levels <= 6, "levels must be in [2, 6]");
    PAT_CHECK_ARG(base_ch >= 4 && base_ch <= 256 && base_ch % 4 == 0, "base_ch must be a multiple of 4 in [4, 256]");
    PAT_CHECK_ARG(out_ch >= 1 && out_ch <= 4, "out_ch must be in [1, 4]");
    std::unique_ptr<pat_unet_s> n(new pat_unet_s());
    n->levels = levels;
    n->base = base_ch;
    n->cout = out_ch;
    pat::nn::build_layers(n.get());
    n->params.alloc(sizeof(float) * n->n_params);
    n->grads.alloc(sizeof(float) * n->n_params);
    n->adam_m.alloc(sizeof(float) * n->n_params);
    n->adam_v.alloc(sizeof(float) * n->n_params);
    n->wf.alloc(sizeof(uint16_t) * n->n_wbf16);
    n->wd.alloc(sizeof(uint16_t) * n->n_wbf16);
    hipStream_t s = nullptr;
    pat::nn::init_params(n.get(), seed, s);
    pat::nn::prep_weights(n.get(), s);
    PAT_HIP(hipStreamSynchronize(s));
    *out = n.release();
    return PAT_OK;
  });
}

extern "C" pat_status pat_warmstart_destroy(pat_unet n) {
  return guarded([&]() -> pat_status {
    delete n;
    return PAT_OK;
  });
}

extern "C" pat_status pat_warmstart_set_gemm_tiles(int32_t mode) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(mode >= 0 && mode <= 3, "gemm tile mode must be 0..3");
    pat::nn::set_gemm_tiles(mode);
    return PAT_OK;
  });
}

extern "C" pat_status pat_warmstart_num_params(pat_unet n, int64_t* out) {
  return guarded([&]() -> pat_status {
    check_net(n);
    PAT_CHECK_ARG(out != nullptr, "out is NULL");
    *out = n->n_params;
    return PAT_OK;
  });
}

extern "C" pat_status pat_warmstart_get_params(pat_unet n, float* d_dst, void* stream) {
  return guarded([&]() -> pat_status {
    check_net(n);
    PAT_CHECK_ARG(d_dst != nullptr, "NULL buffer");
    PAT_HIP(hipMemcpyAsync(d_dst, n->params.p, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)));
    return PAT_OK;
  });
}

extern "C" pat_status pat_warmstart_set_params(pat_unet n, const float* d_src, void* stream) {
  return guarded([&]() -> pat_status {
    check_net(n);
    PAT_CHECK_ARG(d_src != nullptr, "NULL buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    PAT_HIP(hipMemcpyAsync(n->params.p, d_src, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, s));
    PAT_HIP(hipMemsetAsync(n->adam_m.p, 0, n->adam_m.bytes, s));
    PAT_HIP(hipMemsetAsync(n->adam_v.p, 0, n->adam_v.bytes, s));
    n->step = 0;
    pat::nn::prep_weights(n, s);
    return PAT_OK;
  });
}

extern "C" pat_status pat_warmstart_forward(pat_unet n, int32_t batch, int32_t h, int32_t w, const float* d_in,
                                            float* d_out, void* stream) {
  return guarded([&]() -> pat_status {
    check_net(n);
    PAT_CHECK_ARG(batch >= 1 && h >= 1 && w >= 1 && d_in && d_out, "invalid forward arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    pat::nn::ensure_act(n, batch, h, w);
    pat::nn::forward(n, d_in, s);
    PAT_HIP(hipMemcpyAsync(d_out, n->act.y.p, sizeof(float) * (size_t)batch * n->cout * h * w,
                           hipMemcpyDeviceToDevice, s));
    return PAT_OK;
  });
}

extern "C" pat_status pat_warmstart_grad(pat_unet n, int32_t batch, int32_t h, int32_t w, const float* d_in,
                                         const float* d_target, float* d_grad, double* loss, void* stream) {
  return guarded([&]() -> pat_status {
    check_net(n);
    PAT_CHECK_ARG(batch >= 1 && h >= 1 && w >= 1 && d_in && d_target && d_grad, "invalid grad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    pat::nn::ensure_act(n, batch, h, w);
    pat::nn::train_step(n, d_in, d_target, 0.0, s, false);
    PAT_HIP(hipMemcpyAsync(d_grad, n->grads.p, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, s));
    if (loss) {
      PAT_HIP(hipMemcpyAsync(loss, n->act.loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
      PAT_HIP(hipStreamSynchronize(s));
    }
    return PAT_OK;
  });
}

extern "C" pat_status pat_warmstart_train(pat_unet n, int32_t count, int32_t h, int32_t w, const float* d_inputs,
                                          const float* d_targets, const pat_train_opts* opts, double* final_loss,
                                          void* stream) {
  return guarded([&]() -> pat_status {
    check_net(n);
    PAT_CHECK_ARG(opts != nullptr && d_inputs && d_targets, "NULL argument");
    PAT_CHECK_ARG(count >= 1 && opts->batch >= 1 && opts->batch <= count && opts->epochs >= 1,
                  "invalid training sizes");
    PAT_CHECK_ARG(std::isfinite(opts->lr) && opts->lr > 0.0, "lr must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int B = opts->batch;
    pat::nn::ensure_act(n, B, h, w);
    const int64_t img = (int64_t)h * w, timg = img * n->cout;
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::mt19937_64 rng(opts->seed);
    const int per_epoch = count / B;
    std::vector<double> losses;
    pat::DevBuf loss_hist(sizeof(double) * (size_t)per_epoch);
    pat::DevBuf order_d(sizeof(int) * (size_t)count);
    double last = 0.0;
    for (int ep = 0; ep < opts->epochs; ++ep) {
      std::shuffle(order.begin(), order.end(), rng);
      // the epoch's order on the device (the copy has read the host vector when
      // it returns; the vector is reshuffled only after the epoch's synchronisation)
      PAT_HIP(hipMemcpyAsync(order_d.p, order.data(), sizeof(int) * (size_t)count, hipMemcpyHostToDevice, s));
      for (int bi = 0; bi < per_epoch; ++bi) {
        // the input batch is staged in gy (overwritten by the loss gradient after the forward)
        pat::nn::launch_batch_gather(d_inputs, d_targets, pat::ptr<int>(order_d), bi * B, B, img, timg,
                                     pat::ptr<float>(n->act.gy), pat::ptr<float>(n->act.t), s);
        pat::nn::forward(n, pat::ptr<float>(n->act.gy), s);
        pat::nn::launch_mse(pat::ptr<float>(n->act.y), pat::ptr<float>(n->act.t), pat::ptr<float>(n->act.gy),
                            pat::ptr<double>(n->act.loss_part), pat::ptr<double>(loss_hist) + bi,
                            (int64_t)B * timg, s);
        pat::nn::backward(n, s);
        ++n->step;
        const double b1 = 0.9, b2 = 0.999;
        pat::nn::launch_adam(pat::ptr<float>(n->params), pat::ptr<float>(n->grads), pat::ptr<float>(n->adam_m),
                             pat::ptr<float>(n->adam_v), n->n_params, (float)opts->lr, (float)b1, (float)b2, 1e-8f,
                             (float)(1.0 - std::pow(b1, (double)n->step)),
                             (float)(1.0 - std::pow(b2, (double)n->step)), s);
        pat::nn::prep_weights(n, s);
      }
      std::vector<double> h_l(per_epoch);
      PAT_HIP(hipMemcpyAsync(h_l.data(), loss_hist.p, sizeof(double) * per_epoch, hipMemcpyDeviceToHost, s));
      PAT_HIP(hipStreamSynchronize(s));
      double sum = 0.0;
      for (double v : h_l) sum += v;
      last = sum / per_epoch;
      if (!std::isfinite(last)) {
        pat::set_error("training loss became non-finite in epoch %d", ep);
        return PAT_ERR_NUMERIC;
      }
    }
    if (final_loss) *final_loss = last;
    return PAT_OK;
  });
}

extern "C" pat_status pat_warmstart_save(pat_unet n, const char* path) {
  return guarded([&]() -> pat_status {
    check_net(n);
    PAT_CHECK_ARG(path != nullptr, "path is NULL");
    std::vector<float> p(n->n_params), m(n->n_params), v(n->n_params);
    PAT_HIP(hipMemcpy(p.data(), n->params.p, sizeof(float) * n->n_params, hipMemcpyDeviceToHost));
    PAT_HIP(hipMemcpy(m.data(), n->adam_m.p, sizeof(float) * n->n_params, hipMemcpyDeviceToHost));
    PAT_HIP(hipMemcpy(v.data(), n->adam_v.p, sizeof(float) * n->n_params, hipMemcpyDeviceToHost));
    std::ofstream out(path, std::ios::binary | std::ios::trunc);
    PAT_CHECK_ARG((bool)out, "cannot open checkpoint for writing");
    const char magic[8] = {'P', 'A', 'T', 'U', 'N', 'E', 'T', '2'};
    const int64_t hdr[5] = {n->levels, n->base, n->cout, n->n_params, n->step};
    out.write(magic, 8);
    out.write(reinterpret_cast<const char*>(hdr), sizeof(hdr));
    out.write(reinterpret_cast<const char*>(p.data()), sizeof(float) * n->n_params);
    out.write(reinterpret_cast<const char*>(m.data()), sizeof(float) * n->n_params);
    out.write(reinterpret_cast<const char*>(v.data()), sizeof(float) * n->n_params);
    PAT_CHECK_ARG((bool)out, "checkpoint write failed");
    return PAT_OK;
  });
}

extern "C" pat_status pat_warmstart_load(pat_unet n, const char* path) {
  return guarded([&]() -> pat_status {
    check_net(n);
    PAT_CHECK_ARG(path != nullptr, "path is NULL");
    std::ifstream in(path, std::ios::binary);
    PAT_CHECK_ARG((bool)in, "cannot open checkpoint");
    char magic[8];
    int64_t hdr[5];
    in.read(magic, 8);
    in.read(reinterpret_cast<char*>(hdr), sizeof(hdr));
    PAT_CHECK_ARG((bool)in && std::string(magic, 8) == "PATUNET2", "not a network checkpoint");
    PAT_CHECK_ARG(hdr[0] == n->levels && hdr[1] == n->base && hdr[2] == n->cout && hdr[3] == n->n_params,
                  "checkpoint was written for another network shape");
    std::vector<float> p(n->n_params), m(n->n_params), v(n->n_params);
    in.read(reinterpret_cast<char*>(p.data()), sizeof(float) * n->n_params);
    in.read(reinterpret_cast<char*>(m.data()), sizeof(float) * n->n_params);
    in.read(reinterpret_cast<char*>(v.data()), sizeof(float) * n->n_params);
    PAT_CHECK_ARG((bool)in, "truncated checkpoint");
    PAT_HIP(hipMemcpy(n->params.p, p.data(), sizeof(float) * n->n_params, hipMemcpyHostToDevice));
    PAT_HIP(hipMemcpy(n->adam_m.p, m.data(), sizeof(float) * n->n_params, hipMemcpyHostToDevice));
    PAT_HIP(hipMemcpy(n->adam_v.p, v.data(), sizeof(float) * n->n_params, hipMemcpyHostToDevice));
    n->step = hdr[4];
    pat::nn::prep_weights(n, nullptr);
    PAT_HIP(hipDeviceSynchronize());
    return PAT_OK;
  });
}

static void check_dual_reg(const pat_regulariser* reg) {
  PAT_CHECK_ARG(reg != nullptr, "a dual start needs the regulariser");
  PAT_CHECK_ARG(reg->kind == PAT_REG_TV, "dual starts are defined for TV only");
  PAT_CHECK_ARG(std::isfinite(reg->lambda) && reg->lambda > 0.0, "lambda must be > 0");
}

extern "C" pat_status pat_warmstart_normalize(pat_geometry g, const pat_regulariser* reg, const void* d_f,
                                              const void* d_state, float* d_x, float* d_t, int32_t t_channels,
                                              float* d_scale, void* stream) {
  return guarded([&]() -> pat_status {
    PAT_CHECK_ARG(g != nullptr && d_f != nullptr && d_x != nullptr && d_scale != nullptr, "NULL argument");
    PAT_CHECK_ARG((d_state == nullptr) == (d_t == nullptr), "d_state and d_t go together");
    PAT_CHECK_ARG(t_channels == 1 || t_channels == 3, "t_channels must be 1 or 3");
    if (d_state && t_channels == 3) check_dual_reg(reg);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->dtype == PAT_F64) pat::normalise_impl<double>(g, reg, d_f, d_state, d_x, d_t, t_channels, d_scale, s);
    else pat::normalise_impl<float>(g, reg, d_f, d_state, d_x, d_t, t_channels, d_scale, s);
    return PAT_OK;
  });
}

template <class T>
static void infer_impl(pat_unet n, pat_geometry g, const pat_regulariser* reg, const void* d_f, void* d_u0,
                       void* d_y0, hipStream_t s) {
  const int64_t N = g->n_pix(), nb = g->n_bins();
  pat::DevBuf x(sizeof(float) * N), sc(sizeof(float));
  pat::normalise_impl<T>(g, reg, d_f, nullptr, pat::ptr<float>(x), nullptr, 1, pat::ptr<float>(sc), s);
  pat::nn::ensure_act(n, 1, g->ny, g->nx);
  pat::nn::forward(n, pat::ptr<float>(x), s);
  T* u0 = static_cast<T*>(d_u0);
  T* q0 = static_cast<T*>(d_y0);
  T* r0 = q0 ? q0 + nb : nullptr;
  const unsigned blocks = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(pat::rescale_kernel<T>, dim3(blocks), dim3(256), 0, s, pat::ptr<float>(n->act.y),
                     pat::ptr<float>(sc), u0, r0, r0 ? reg->lambda : 0.0, N);
  PAT_HIP(hipGetLastError());
  if (q0) {
    pat::apply_forward<T>(g, u0, q0, s);
    hipLaunchKernelGGL(pat::residual_kernel<T>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, q0,
                       static_cast<const T*>(d_f), nb);
    PAT_HIP(hipGetLastError());
  }
  PAT_HIP(hipStreamSynchronize(s));
}

extern "C" pat_status pat_warmstart_infer(pat_unet n, pat_geometry g, const pat_regulariser* reg, const void* d_f,
                                          void* d_u0, void* d_y0, void* stream) {
  return guarded([&]() -> pat_status {
    check_net(n);
    PAT_CHECK_ARG(g != nullptr && d_f != nullptr && d_u0 != nullptr, "NULL argument");
    if (d_y0) {
      check_dual_reg(reg);
      PAT_CHECK_ARG(n->cout == 3, "a dual start needs a network with 3 outputs");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->dtype == PAT_F64) infer_impl<double>(n, g, reg, d_f, d_u0, d_y0, s);
    else infer_impl<float>(n, g, reg, d_f, d_u0, d_y0, s);
    return PAT_OK;
  });
}
