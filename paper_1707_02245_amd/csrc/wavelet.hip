// Dual-tree wavelet transform W of the wavelet model (arXiv:1707.02245,
// Sec. 2.2 eq. min_wav: lam ||W u||_1 with W from the dual-tree complex
// wavelet transform, ||W|| = 1 and W^T as its inverse) and the solver's
// wavelet steps (Algorithm 1 with grad -> W and div -> W^T).
//
// Filters (the paper does not print them): the orthonormal 4-tap Daubechies
// pair h = (1 + s, 3 + s, 3 - s, 1 - s) / (4 sqrt 2), s = sqrt 3, and
// g[k] = (-1)^k h[3 - k]; periodic analysis y[i] = sum_k c[k] x[(2i + k +
// shift) mod n]. Tree a: (h, g), shift 0. Tree b: at level 1 (h, g) on the
// signal advanced by one sample, from level 2 on the time-reversed pair with
// shift 0. The 2-D transform runs the four trees (row tree, column tree) in
// {a, b}^2, each recursing on its own lowpass band; per level the detail
// bands of the trees combine into the oriented bands p, q, s, t (sums and
// differences over sqrt 2), and everything carries a factor 1/2 so that
// W^T W = I. Coefficient order: level-major, then orientation (LH, HL, HH),
// then band (p, q, s, t), row-major inside a band; the level-J lowpass bands
// of trees aa, ab, ba, bb at the end.
//
// One launch per level. Analysis: one thread per coefficient position of the
// level reads the 4 x 4 input taps of each tree (cached loads; the level-1
// input is the image shared by all trees), forms the 16 tree subbands and
// writes the 12 oriented detail coefficients and the 4 lowpass values (the
// next level's input, or the last level's lowpass coefficients). The
// coefficients go out as W u (stand-alone), into the dual step
// r <- clip(r + sigma c, -lam, lam) (the prox of the conjugate of
// lam ||.||_1, Sec. 3.2), or into lam sum |c| (the gap's regulariser value).
// Synthesis (W^T): one thread per coefficient position of the level reads the
// 16 values of the positions whose taps reach its 2 x 2 block of input
// samples (4 positions, 9 at level 1 where tree b is shifted), undoes the
// band combination and writes the block for every tree (the image, summed
// over the trees, at level 1).

#include "pat_internal.hpp"

namespace pat {

namespace {

// Filters of one level: [tree a, tree b] lowpass, highpass and shift.
struct WavFilters {
  double lo[2][4], hi[2][4];
  int shift[2];
  double kc;  // 1 / (2 sqrt 2): the band combination's 1/sqrt 2 times the frame's 1/2
};

WavFilters wav_filters(int level) {
  const double s3 = std::sqrt(3.0), d = 4.0 * std::sqrt(2.0);
  const double h[4] = {(1.0 + s3) / d, (3.0 + s3) / d, (3.0 - s3) / d, (1.0 - s3) / d};
  WavFilters f{};
  for (int t = 0; t < 2; ++t) {
    const bool rev = t == 1 && level >= 2;
    double c[4];
    for (int k = 0; k < 4; ++k) c[k] = rev ? h[3 - k] : h[k];
    for (int k = 0; k < 4; ++k) {
      f.lo[t][k] = c[k];
      f.hi[t][k] = (k % 2 ? -1.0 : 1.0) * c[3 - k];
    }
    f.shift[t] = (t == 1 && level == 1) ? 1 : 0;
  }
  f.kc = 0.5 / std::sqrt(2.0);
  return f;
}

enum { WAV_PLAIN = 0, WAV_DUAL = 1, WAV_GAP = 2 };

// Workgroups go to the 8 XCDs in turn (block b to XCD b mod 8). Numbering the
// position ranges so that each XCD takes one contiguous run keeps the rows a
// position row shares with its neighbours (the filters' overlapping taps) in
// that XCD's L2. Measured at 4096^2 it helps the levels from 2 on (synthesis
// 91 -> 76 and 25 -> 21 us); the level-1 analysis, which reads the image, was
// no faster with it and keeps launch order.
__device__ __forceinline__ int64_t xcd_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  return nb % 8 == 0 ? (int64_t)(b % 8) * (nb / 8) + b / 8 : (int64_t)b;
}

// One analysis level. Input grid cy x cx (the image at level 1, else the
// previous level's four lowpass bands); output grid (cy/2) x (cx/2).
template <class T, class A>
struct WavAnaArgs {
  int cx, cy;
  const T* img;        // level 1: img[y * pitch + x]
  int pitch;
  const A* ll_in;      // levels >= 2: [4][cy][cx]
  A* ll_out;           // not the last level: [4][cy/2][cx/2]
  int64_t band_off;    // first detail band of the level in the coefficient vector
  int64_t ll_off;      // last level: the lowpass bands; else -1
  T* coef;             // PLAIN: W u
  T* r;                // DUAL: the dual variable (coefficient order)
  T sigma;             // DUAL: its step size
  const double* mult;  // DUAL: {dual, primal, theta} multipliers or null
  T lam;               // DUAL: clip bound; GAP: weight
  double* red;         // GAP: one partial sum per workgroup
  WavFilters f;
};

template <class T, class A, int MODE, bool FIRST>
__global__ __launch_bounds__(256) void wav_analysis_kernel(WavAnaArgs<T, A> a) {
  const int hx = a.cx >> 1, hy = a.cy >> 1;
  const int64_t S = (int64_t)hx * hy;
  const int64_t e = (FIRST ? (int64_t)blockIdx.x : xcd_block()) * 256 + threadIdx.x;
  double gap = 0.0;
  if (e < S) {
    const int ix = (int)(e % hx), iy = (int)(e / hx);
    A sub[4][4];  // [tree aa, ab, ba, bb][LL, LH, HL, HH]
    // level 1: the 5 x 5 patch at (2 iy, 2 ix) serves every tree (shifts 0, 1)
    A patch[FIRST ? 5 : 1][FIRST ? 5 : 1];
    if (FIRST) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const int y = (2 * iy + k) % a.cy;
#pragma unroll
        for (int m = 0; m < 5; ++m) patch[k][m] = (A)a.img[(int64_t)y * a.pitch + (2 * ix + m) % a.cx];
      }
    }
    // from level 2 on every shift is 0 and the four taps of a row are two
    // aligned pairs unless they wrap around the right edge
    const bool pairs = !FIRST && 2 * ix + 3 < a.cx;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ty = t >> 1, tx = t & 1;
      const int sy = FIRST ? ty : 0, sx = FIRST ? tx : 0;
      A rl[4], rh[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        A x[4];
        if (FIRST) {
#pragma unroll
          for (int m = 0; m < 4; ++m) x[m] = patch[k + sy][m + sx];
        } else {
          const A* in = a.ll_in + (int64_t)t * a.cx * a.cy + (int64_t)((2 * iy + k) % a.cy) * a.cx;
          if (pairs) {
            using A2 = typename Vec2<A>::type;
            const A2 p0 = *reinterpret_cast<const A2*>(in + 2 * ix);
            const A2 p1 = *reinterpret_cast<const A2*>(in + 2 * ix + 2);
            x[0] = p0.x;
            x[1] = p0.y;
            x[2] = p1.x;
            x[3] = p1.y;
          } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) x[m] = in[(2 * ix + m) % a.cx];
          }
        }
        A l = A(0), h = A(0);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          l += (A)a.f.lo[tx][m] * x[m];
          h += (A)a.f.hi[tx][m] * x[m];
        }
        rl[k] = l;
        rh[k] = h;
      }
      A ll = A(0), lh = A(0), hl = A(0), hh = A(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ll += (A)a.f.lo[ty][k] * rl[k];
        lh += (A)a.f.lo[ty][k] * rh[k];
        hl += (A)a.f.hi[ty][k] * rl[k];
        hh += (A)a.f.hi[ty][k] * rh[k];
      }
      sub[t][0] = ll;
      sub[t][1] = lh;
      sub[t][2] = hl;
      sub[t][3] = hh;
    }
    // the coefficients of this position: oriented bands p = (aa - bb),
    // q = (aa + bb), s = (ab + ba), t = (ab - ba), each over sqrt 2, times the
    // frame factor 1/2; on the last level the four lowpass bands times 1/2
    const bool last = a.ll_off >= 0;
    const A kc = (A)a.f.kc;
    A val[16];
    int64_t idx[16];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      const A aa = sub[0][o + 1], ab = sub[1][o + 1], ba = sub[2][o + 1], bb = sub[3][o + 1];
      const int64_t base = a.band_off + (int64_t)(4 * o) * S + e;
      val[4 * o] = kc * (aa - bb);
      val[4 * o + 1] = kc * (aa + bb);
      val[4 * o + 2] = kc * (ab + ba);
      val[4 * o + 3] = kc * (ab - ba);
#pragma unroll
      for (int b = 0; b < 4; ++b) idx[4 * o + b] = base + b * S;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      val[12 + t] = A(0.5) * sub[t][0];
      idx[12 + t] = a.ll_off + t * S + e;
      if (!last) a.ll_out[t * S + e] = sub[t][0];
    }
    const int n_out = last ? 16 : 12;
    if (MODE == WAV_PLAIN) {
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < n_out) a.coef[idx[k]] = (T)val[k];
    } else if (MODE == WAV_DUAL) {
      // every load of r before the first store, so that the loads overlap
      const T sr = a.mult ? a.sigma * (T)a.mult[0] : a.sigma;
      T rv[16];
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < n_out) rv[k] = a.r[idx[k]];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (k < n_out) {
          const T rr = rv[k] + sr * (T)val[k];
          a.r[idx[k]] = rr > a.lam ? a.lam : (rr < -a.lam ? -a.lam : rr);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < n_out) gap += fabs((double)val[k]);
    }
  }
  if (MODE == WAV_GAP) {
    __shared__ double lds[8];
    const double s = block_sum<256>(gap * (double)a.lam, lds);
    if (threadIdx.x == 0) a.red[blockIdx.x] = s;
  }
}

// One synthesis level: the level's subbands (grid (cy/2) x (cx/2)) back to
// its input grid cy x cx.
template <class T, class A>
struct WavSynArgs {
  int cx, cy;
  const T* coef;       // the coefficient vector
  int64_t band_off;    // first detail band of the level
  int64_t ll_off;      // last level: the lowpass bands; else -1
  const A* ll_in;      // not the last level: [4][cy/2][cx/2] (from the level above)
  A* ll_out;           // levels >= 2: [4][cy][cx]
  A* out;              // level 1: the image [cy][cx], summed over the trees
  WavFilters f;
};

// One thread per position (X, Y) of the level writes the 2 x 2 block of
// samples (2Y + dy, 2X + dx) of its input grid. Tap k of the analysis at
// position i reaches sample 2 i + k + shift, so sample 2Y + dy takes tap
// k = 2 a + dy - shift from position Y - a (mod cy/2), for a = 0, 1 (and 2
// when the shift is 1, at level 1), each valid k once: the positions of
// offsets a, b in {0, 1, 2} hold every term. Their 16 values (12 oriented
// detail bands, 4 lowpass) are turned back into the trees' subbands (the
// transposed band combination). This kernel serves the levels from 2 on
// (no shifts: offsets 0 and 1), reading each position's values once per
// thread; level 1, and levels of many positions, take the tiled kernel below.
template <class T, class A>
__global__ __launch_bounds__(256) void wav_synthesis_kernel(WavSynArgs<T, A> a) {
  const int hx = a.cx >> 1, hy = a.cy >> 1;
  const int64_t S = (int64_t)hx * hy;
  const int64_t e = xcd_block() * 256 + threadIdx.x;
  if (e >= S) return;
  const int X = (int)(e % hx), Y = (int)(e / hx);
  const A kc = (A)a.f.kc;
  constexpr int NA = 2;
  A acc[4][2][2];  // [tree][dy][dx]
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) acc[t][dy][dx] = A(0);
#pragma unroll
  for (int ay = 0; ay < NA; ++ay) {
    const int iy = (Y - ay + hy) % hy;
#pragma unroll
    for (int ax = 0; ax < NA; ++ax) {
      const int ix = (X - ax + hx) % hx;
      const int64_t pos = (int64_t)iy * hx + ix;
      A sub[4][4];  // [tree][LL, LH, HL, HH]
#pragma unroll
      for (int t = 0; t < 4; ++t)
        sub[t][0] = a.ll_off >= 0 ? A(0.5) * (A)a.coef[a.ll_off + t * S + pos] : a.ll_in[t * S + pos];
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        const T* c = a.coef + a.band_off + (int64_t)(4 * o) * S + pos;
        const A p = (A)c[0], q = (A)c[S], s = (A)c[2 * S], u = (A)c[3 * S];
        sub[0][o + 1] = kc * (p + q);  // aa
        sub[1][o + 1] = kc * (s + u);  // ab
        sub[2][o + 1] = kc * (s - u);  // ba
        sub[3][o + 1] = kc * (q - p);  // bb
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int ty = t >> 1, tx = t & 1;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
          const int ky = 2 * ay + dy;
          const A ly = (A)a.f.lo[ty][ky], gy = (A)a.f.hi[ty][ky];
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const int kx = 2 * ax + dx;
            const A lx = (A)a.f.lo[tx][kx], gx = (A)a.f.hi[tx][kx];
            acc[t][dy][dx] += ly * (lx * sub[t][0] + gx * sub[t][1]) + gy * (lx * sub[t][2] + gx * sub[t][3]);
          }
        }
      }
    }
  }
  const int64_t n = (int64_t)a.cx * a.cy;
#pragma unroll
  for (int dy = 0; dy < 2; ++dy) {
    const int64_t row = (int64_t)(2 * Y + dy) * a.cx + 2 * X;
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
#pragma unroll
      for (int t = 0; t < 4; ++t) a.ll_out[t * n + row + dx] = acc[t][dy][dx];
    }
  }
}

// The same by tiles of 16 x 16 positions: the positions a tile's threads
// reach (the tile and the NA - 1 position rows and columns before it,
// periodic; NA = 3 at level 1, else 2) are turned into the trees' subbands
// once and kept in LDS, band-major (conflict-free 8-byte reads), so that every
// coefficient is read from memory (1 + (NA - 1) / 16)^2 times instead of once
// per neighbour that uses it (NA^2 times); each thread then sums its
// neighbourhood in the same order and with the same values as the
// per-position kernel. Level 1 (FIRST: the tree shifts) writes the image
// summed over the trees, the other levels each tree's lowpass band. Used at
// level 1 and wherever a level has many tiles (at 4096^2 the levels 2 and 3
// went 78 -> 67 and 22 -> 20 us); a level of a few tiles is latency-bound and
// keeps one thread per position (at 256^2 the tiles' extra barrier and LDS
// round trip cost 4.9 -> 6.8 us at level 2).
constexpr int kWsT = 16, kWsTiledMin = 256;

template <class T, class A, bool FIRST>
__global__ __launch_bounds__(256) void wav_synthesis_tiled_kernel(WavSynArgs<T, A> a) {
  constexpr int NA = FIRST ? 3 : 2, HALO = NA - 1, TH = kWsT + HALO, TP = TH * TH;
  __shared__ A sl[16][TP];  // [tree * 4 + band][position in the haloed tile]
  const int hx = a.cx >> 1, hy = a.cy >> 1;
  const int64_t S = (int64_t)hx * hy;
  const int tiles_x = (hx + kWsT - 1) / kWsT;
  const int64_t tile = xcd_block();
  const int X0 = (int)(tile % tiles_x) * kWsT, Y0 = (int)(tile / tiles_x) * kWsT;
  const A kc = (A)a.f.kc;
  for (int q = threadIdx.x; q < TP; q += 256) {
    const int ly = q / TH, lx = q - ly * TH;
    const int iy = ((Y0 - HALO + ly) % hy + hy) % hy, ix = ((X0 - HALO + lx) % hx + hx) % hx;
    const int64_t pos = (int64_t)iy * hx + ix;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      sl[4 * t][q] = a.ll_off >= 0 ? A(0.5) * (A)a.coef[a.ll_off + t * S + pos] : a.ll_in[t * S + pos];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      const T* c = a.coef + a.band_off + (int64_t)(4 * o) * S + pos;
      const A p = (A)c[0], r = (A)c[S], s = (A)c[2 * S], u = (A)c[3 * S];
      sl[o + 1][q] = kc * (p + r);       // aa
      sl[4 + o + 1][q] = kc * (s + u);   // ab
      sl[8 + o + 1][q] = kc * (s - u);   // ba
      sl[12 + o + 1][q] = kc * (r - p);  // bb
    }
  }
  __syncthreads();
  const int tx = threadIdx.x % kWsT, ty = threadIdx.x / kWsT;
  const int X = X0 + tx, Y = Y0 + ty;
  if (X >= hx || Y >= hy) return;
  A acc[4][2][2];  // [tree][dy][dx]
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) acc[t][dy][dx] = A(0);
#pragma unroll
  for (int ay = 0; ay < NA; ++ay) {
#pragma unroll
    for (int ax = 0; ax < NA; ++ax) {
      const int q = (ty + HALO - ay) * TH + (tx + HALO - ax);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int fy = t >> 1, fx = t & 1;
        const int sy = FIRST ? fy : 0, sx = FIRST ? fx : 0;
        const A s0 = sl[4 * t][q], s1 = sl[4 * t + 1][q], s2 = sl[4 * t + 2][q], s3 = sl[4 * t + 3][q];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
          const int ky = 2 * ay + dy - sy;
          if (ky < 0 || ky > 3) continue;
          const A ly = (A)a.f.lo[fy][ky], gy = (A)a.f.hi[fy][ky];
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const int kx = 2 * ax + dx - sx;
            if (kx < 0 || kx > 3) continue;
            const A lx = (A)a.f.lo[fx][kx], gx = (A)a.f.hi[fx][kx];
            acc[t][dy][dx] += ly * (lx * s0 + gx * s1) + gy * (lx * s2 + gx * s3);
          }
        }
      }
    }
  }
  const int64_t n = (int64_t)a.cx * a.cy;
#pragma unroll
  for (int dy = 0; dy < 2; ++dy) {
    const int64_t row = (int64_t)(2 * Y + dy) * a.cx + 2 * X;
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      if (FIRST) {
        a.out[row + dx] = (acc[0][dy][dx] + acc[1][dy][dx]) + (acc[2][dy][dx] + acc[3][dy][dx]);
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) a.ll_out[t * n + row + dx] = acc[t][dy][dx];
      }
    }
  }
}

inline int64_t band_size(int nx, int ny, int j) { return (int64_t)(nx >> j) * (ny >> j); }

// Start of level j's detail bands (j = levels + 1: the lowpass bands).
inline int64_t level_offset(int nx, int ny, int j) {
  int64_t o = 0;
  for (int l = 1; l < j; ++l) o += 12 * band_size(nx, ny, l);
  return o;
}

// Lowpass bands of level l in the work buffer: odd levels at 0, even at N.
template <class A>
inline A* ll_region(A* work, int nx, int ny, int l) {
  return (l & 1) ? work : work + (int64_t)nx * ny;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int64_t wav_work_elems(int nx, int ny) { return (int64_t)nx * ny + ((int64_t)nx * ny + 3) / 4; }

int wav_gap_blocks(int nx, int ny, int levels) {
  int b = 0;
  for (int j = 1; j <= levels; ++j) b += (int)blocks_for(band_size(nx, ny, j));
  return b;
}

template <class T, class A>
static void analysis(int mode, const WavInput<T>& in, const WavDual<T>& d, A* work, hipStream_t s) {
  const int nx = in.nx, ny = in.ny, J = in.levels;
  double* red = d.red;
  for (int j = 1; j <= J; ++j) {
    WavAnaArgs<T, A> a{};
    a.cx = nx >> (j - 1);
    a.cy = ny >> (j - 1);
    a.img = in.img;
    a.pitch = in.pitch;
    a.ll_in = j >= 2 ? ll_region(work, nx, ny, j - 1) : nullptr;
    a.ll_out = j < J ? ll_region(work, nx, ny, j) : nullptr;
    a.band_off = level_offset(nx, ny, j);
    a.ll_off = j == J ? level_offset(nx, ny, J + 1) : -1;
    a.coef = d.coef;
    a.r = d.r;
    a.sigma = d.sigma;
    a.mult = d.mult;
    a.lam = d.lam;
    a.red = red;
    a.f = wav_filters(j);
    const unsigned grid = blocks_for(band_size(nx, ny, j));
#define PAT_WAV_ANA(M, F) \
  hipLaunchKernelGGL((wav_analysis_kernel<T, A, M, F>), dim3(grid), dim3(256), 0, s, a)
    if (mode == WAV_PLAIN) { if (j == 1) PAT_WAV_ANA(WAV_PLAIN, true); else PAT_WAV_ANA(WAV_PLAIN, false); }
    else if (mode == WAV_DUAL) { if (j == 1) PAT_WAV_ANA(WAV_DUAL, true); else PAT_WAV_ANA(WAV_DUAL, false); }
    else { if (j == 1) PAT_WAV_ANA(WAV_GAP, true); else PAT_WAV_ANA(WAV_GAP, false); }
#undef PAT_WAV_ANA
    PAT_HIP(hipGetLastError());
    if (red) red += grid;
  }
}

template <class T, class A>
static void synthesis(int nx, int ny, int J, const T* coef, A* out, A* work, hipStream_t s) {
  for (int j = J; j >= 1; --j) {
    WavSynArgs<T, A> a{};
    a.cx = nx >> (j - 1);
    a.cy = ny >> (j - 1);
    a.coef = coef;
    a.band_off = level_offset(nx, ny, j);
    a.ll_off = j == J ? level_offset(nx, ny, J + 1) : -1;
    a.ll_in = j < J ? ll_region(work, nx, ny, j) : nullptr;
    a.ll_out = j >= 2 ? ll_region(work, nx, ny, j - 1) : nullptr;
    a.out = j == 1 ? out : nullptr;
    a.f = wav_filters(j);
    const unsigned grid = blocks_for(band_size(nx, ny, j));
    const int hx = a.cx >> 1, hy = a.cy >> 1;
    const unsigned tiles = (unsigned)(((hx + kWsT - 1) / kWsT) * ((hy + kWsT - 1) / kWsT));
    if (j == 1)
      hipLaunchKernelGGL((wav_synthesis_tiled_kernel<T, A, true>), dim3(tiles), dim3(256), 0, s, a);
    else if (tiles >= (unsigned)kWsTiledMin)
      hipLaunchKernelGGL((wav_synthesis_tiled_kernel<T, A, false>), dim3(tiles), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((wav_synthesis_kernel<T, A>), dim3(grid), dim3(256), 0, s, a);
    PAT_HIP(hipGetLastError());
  }
}

template <class T>
void launch_wav_forward(const WavInput<T>& in, T* coef, T* work, hipStream_t s) {
  WavDual<T> d{};
  d.coef = coef;
  analysis<T, T>(WAV_PLAIN, in, d, work, s);
}

template <class T>
void launch_wav_dual(const WavInput<T>& in, const WavDual<T>& d, T* work, hipStream_t s) {
  analysis<T, T>(WAV_DUAL, in, d, work, s);
}

template <class T>
void launch_wav_gap(const WavInput<T>& in, T lam, double* red, double* work, hipStream_t s) {
  WavDual<T> d{};
  d.lam = lam;
  d.red = red;
  analysis<T, double>(WAV_GAP, in, d, work, s);
}

template <class T, class A>
void launch_wav_adjoint(int nx, int ny, int levels, const T* coef, A* out, A* work, hipStream_t s) {
  synthesis<T, A>(nx, ny, levels, coef, out, work, s);
}

#define PAT_INST_WAV(T)                                                                          \
  template void launch_wav_forward<T>(const WavInput<T>&, T*, T*, hipStream_t);                 \
  template void launch_wav_dual<T>(const WavInput<T>&, const WavDual<T>&, T*, hipStream_t);     \
  template void launch_wav_gap<T>(const WavInput<T>&, T, double*, double*, hipStream_t);        \
  template void launch_wav_adjoint<T, T>(int, int, int, const T*, T*, T*, hipStream_t);
PAT_INST_WAV(float)
PAT_INST_WAV(double)
template void launch_wav_adjoint<float, double>(int, int, int, const float*, double*, double*, hipStream_t);

void check_wavelet_shape(int nx, int ny, int levels) {
  PAT_CHECK_ARG(levels >= 1 && levels <= kWavMaxLevels, "wavelet levels must be in 1..8");
  PAT_CHECK_ARG(nx > 0 && ny > 0 && nx % (1 << levels) == 0 && ny % (1 << levels) == 0,
                "the image sides must be positive multiples of 2^levels");
}

}  // namespace pat

// ------------------------------------------------------------------ C ABI

template <class T>
static void wavelet_apply(bool adjoint, int nx, int ny, int levels, const void* in, void* out, void* d_work,
                          hipStream_t s) {
  pat::DevBuf own;
  T* work = static_cast<T*>(d_work);
  if (!work) {
    own.alloc(sizeof(T) * (size_t)pat::wav_work_elems(nx, ny));
    work = pat::ptr<T>(own);
  }
  if (adjoint) {
    pat::launch_wav_adjoint<T, T>(nx, ny, levels, static_cast<const T*>(in), static_cast<T*>(out), work, s);
  } else {
    const pat::WavInput<T> w{nx, ny, levels, static_cast<const T*>(in), nx};
    pat::launch_wav_forward<T>(w, static_cast<T*>(out), work, s);
  }
  // a work buffer of the call's own is freed on return
  if (own.p) PAT_HIP(hipStreamSynchronize(s));
}

static pat_status wavelet_entry(bool adjoint, int32_t dtype, int32_t nx, int32_t ny, int32_t levels,
                                const void* in, void* out, void* d_work, void* stream) {
  return pat::guarded([&]() -> pat_status {
    PAT_CHECK_ARG(dtype == PAT_F32 || dtype == PAT_F64, "unknown dtype");
    PAT_CHECK_ARG(in != nullptr && out != nullptr, "NULL argument");
    PAT_CHECK_ARG((reinterpret_cast<uintptr_t>(d_work) & 15) == 0, "d_work must be 16-byte aligned");
    pat::check_wavelet_shape(nx, ny, levels);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == PAT_F64) wavelet_apply<double>(adjoint, nx, ny, levels, in, out, d_work, s);
    else wavelet_apply<float>(adjoint, nx, ny, levels, in, out, d_work, s);
    return PAT_OK;
  });
}

extern "C" int64_t pat_wavelet_work_elems(int32_t nx, int32_t ny) {
  return nx > 0 && ny > 0 ? pat::wav_work_elems(nx, ny) : 0;
}

extern "C" pat_status pat_wavelet_forward(int32_t dtype, int32_t nx, int32_t ny, int32_t levels,
                                          const void* d_u, void* d_c, void* d_work, void* stream) {
  return wavelet_entry(false, dtype, nx, ny, levels, d_u, d_c, d_work, stream);
}

extern "C" pat_status pat_wavelet_adjoint(int32_t dtype, int32_t nx, int32_t ny, int32_t levels,
                                          const void* d_c, void* d_u, void* d_work, void* stream) {
  return wavelet_entry(true, dtype, nx, ny, levels, d_c, d_u, d_work, stream);
}
