// Kernels of the warm-start network (include/clb_nn.h): implicit-GEMM 3x3
// convolutions on the gfx950 matrix cores (bf16 MFMA, FP32 accumulation),
// their weight gradients, and the elementwise layers, loss and optimizer.
//
// Matrix-core operand layout (v_mfma_f32_16x16x32_bf16, one wave of 64 lanes):
//   A (16 x 32):  lane l holds row l % 16, columns 8 (l / 16) .. + 7;
//   B (32 x 16):  lane l holds column l % 16, rows 8 (l / 16) .. + 7;
//   D (16 x 16):  lane l holds column l % 16, rows 4 (l / 16) .. + 3.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "clb.h"
#include "clb_nn.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kPixTile = 64;  // pixels per workgroup of the convolution (4 waves x 16)
constexpr int kCoTile = 64;   // output channels per workgroup (4 MFMA column tiles)

__device__ __forceinline__ f4 mfma16(const bf16x8 &a, const bf16x8 &b, const f4 &c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Forward 3x3 convolution as a GEMM: rows = pixels (b, i, j), columns =
// output channels, reduction index k = t * cin + c (tap-major, channels
// contiguous).  The reduction runs in steps of 32 (one 16x16x32 MFMA per
// 16-channel column tile); cin is a multiple of 16, so a lane's 8
// consecutive k lie in one tap and are 16 contiguous bytes of the input and
// of the weight row.  The input is read through a ConvSrc: its first ca
// channels come from tensor a (at half resolution, nearest-neighbour
// upsampled, when up != 0), the other cb from tensor b, so the upsampled and
// the concatenated tensors of a decoder level are never formed.  The output
// may be split by channels (ConvDst) into two tensors, as the input gradient
// of such a convolution feeds its two sources.  A workgroup (4 waves)
// computes up to 64 output channels for
//   - KSPLIT = false: 64 PT pixels, wave w the pixel tiles 16 (w + 4 p),
//     p < PT.  The weight slice of each step (64 channels x 32 k) is loaded
//     once per workgroup into LDS (double-buffered) and read by all four
//     waves for all PT tiles;
//   - KSPLIT = true (few pixels, deep layers): 16 pixels, wave w the steps
//     w, w + 4, ...; the four partial sums are added in wave order through
//     LDS, which gives four times as many workgroups and a quarter of the
//     sequential steps per wave.
// Both load the next step's operands before the current step's MFMAs.
constexpr int kWRow = 32 + 8;  // LDS row of the weight slice in bf16 (padded)

struct ConvSrc {
  const bf16 *a;  // first ca channels: (B, H >> up, W >> up, ca)
  const bf16 *b;  // then cb channels: (B, H, W, cb); null when cb = 0
  int ca, cb, up;
};

struct ConvDst {
  void *y0;  // output channels [0, split): (B, H, W, split)
  void *y1;  // output channels [split, cout): (B, H, W, cout - split); null when split = cout
  int split;
  // Gradient through a leaky ReLU (bf16 output, one part): the rounded
  // value v is stored as v (act_y > 0) or act_slope v, act_y being the
  // activation's output in the output's layout; null for none.
  const bf16 *act_y = nullptr;
  float act_slope = 0.0f;
};

struct ConvPixel {
  int n, py, px;
  bool ok;
};

__device__ __forceinline__ ConvPixel conv_pixel(int m, int M, int H, int W) {
  ConvPixel p{0, 0, 0, m < M};
  if (p.ok) {
    p.n = m / (H * W);
    const int r = m - p.n * H * W;
    p.py = r / W;
    p.px = r - p.py * W;
  }
  return p;
}

// 8 consecutive input channels c .. c + 7 of pixel (n, yy, xx) of the
// virtual input (zero outside the image).
__device__ __forceinline__ bf16x8 src_load(const ConvSrc &x, int n, int yy, int xx, int c,
                                           int H, int W) {
  bf16x8 v = {};
  if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
    if (c < x.ca) {
      const int ha = H >> x.up, wa = W >> x.up;
      v = *reinterpret_cast<const bf16x8 *>(
          x.a + ((size_t)(n * ha + (yy >> x.up)) * wa + (xx >> x.up)) * x.ca + c);
    } else {
      v = *reinterpret_cast<const bf16x8 *>(x.b + ((size_t)(n * H + yy) * W + xx) * x.cb +
                                            (c - x.ca));
    }
  }
  return v;
}

// 8 consecutive k of one pixel (zero outside the image or beyond K).
__device__ __forceinline__ bf16x8 conv_a(const ConvSrc &x, const ConvPixel &p, int k, int K,
                                         int H, int W, int cin) {
  bf16x8 a = {};
  if (k < K && p.ok) {
    const int tap = k / cin, c = k - tap * cin;
    a = src_load(x, p.n, p.py + tap / 3 - 1, p.px + tap % 3 - 1, c, H, W);
  }
  return a;
}

// Bias, activation and store of one wave's 16 pixels x nt (<= NT) column tiles.
template <int NT>
__device__ __forceinline__ void conv_store(const f4 *acc, int nt, int m0, int M, int co0,
                                           int lane, const float *__restrict__ bias, int cout,
                                           int act, float slope, const ConvDst &dst,
                                           int y_fp32) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t >= nt) continue;
    const int co = co0 + 16 * t + (lane & 15);
    const float bb = bias ? bias[co] : 0.0f;
    // a column tile of 16 channels lies in one part (split is a multiple of 16)
    const bool hi = co >= dst.split;
    void *y = hi ? dst.y1 : dst.y0;
    const int ld = hi ? cout - dst.split : dst.split, cc = hi ? co - dst.split : co;
    for (int e = 0; e < 4; ++e) {
      const int mm = m0 + 4 * (lane >> 4) + e;
      if (mm >= M) continue;
      float v = acc[t][e] + bb;
      if (act) v = v > 0.0f ? v : v * slope;
      if (y_fp32) {
        static_cast<float *>(y)[(size_t)mm * ld + cc] = v;
      } else if (dst.act_y) {
        const float r = (float)(bf16)v;
        static_cast<bf16 *>(y)[(size_t)mm * ld + cc] =
            (bf16)((float)dst.act_y[(size_t)mm * ld + cc] > 0.0f ? r : dst.act_slope * r);
      } else {
        static_cast<bf16 *>(y)[(size_t)mm * ld + cc] = (bf16)v;
      }
    }
  }
}

template <bool KSPLIT, int PT, int NT>
__global__ void __launch_bounds__(256) conv3x3_kernel(
    ConvSrc x, int B, int H, int W, const bf16 *__restrict__ wt, const float *__restrict__ bias,
    int cout, int act, float slope, ConvDst dst, int y_fp32) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cin = x.ca + x.cb;
  const int M = B * H * W, K = 9 * cin, nsteps = (K + 31) / 32;
  const int co0 = blockIdx.y * kCoTile;
  const int nt = min(NT, (cout - co0) >> 4);  // column tiles of this workgroup (<= NT)
  const int row = lane & 15, kq = 8 * (lane >> 4);
  const bf16x8 zero = {};
  if constexpr (!KSPLIT) {
    __shared__ __attribute__((aligned(16))) bf16 sw[2][kCoTile * kWRow];
    f4 acc[PT][4];
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[p][t] = f4{0.f, 0.f, 0.f, 0.f};
    const int mb = blockIdx.x * kPixTile * PT;
    ConvPixel px[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) px[p] = conv_pixel(mb + 16 * (wave + 4 * p) + row, M, H, W);
    // weight loading role: channel wo of the slice, k offset 8 wk
    const int wo = threadIdx.x >> 2, wk = 8 * (threadIdx.x & 3);
    const bool wok = co0 + wo < cout;
    const bf16 *wrow = wt + (size_t)(co0 + wo) * K;
    bf16x8 a[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) a[p] = conv_a(x, px[p], kq, K, H, W, cin);
    bf16x8 wv = (wok && wk < K) ? *reinterpret_cast<const bf16x8 *>(wrow + wk) : zero;
    *reinterpret_cast<bf16x8 *>(&sw[0][wo * kWRow + wk]) = wv;
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
      const int cur = s & 1;
      const int kn = 32 * (s + 1);
      bf16x8 an[PT];
#pragma unroll
      for (int p = 0; p < PT; ++p) an[p] = zero;
      if (s + 1 < nsteps) {
#pragma unroll
        for (int p = 0; p < PT; ++p) an[p] = conv_a(x, px[p], kn + kq, K, H, W, cin);
        wv = (wok && kn + wk < K) ? *reinterpret_cast<const bf16x8 *>(wrow + kn + wk) : zero;
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t < nt) {
          const bf16x8 b =
              *reinterpret_cast<const bf16x8 *>(&sw[cur][(16 * t + row) * kWRow + kq]);
#pragma unroll
          for (int p = 0; p < PT; ++p) acc[p][t] = mfma16(a[p], b, acc[p][t]);
        }
      }
      if (s + 1 < nsteps) *reinterpret_cast<bf16x8 *>(&sw[cur ^ 1][wo * kWRow + wk]) = wv;
      __syncthreads();
#pragma unroll
      for (int p = 0; p < PT; ++p) a[p] = an[p];
    }
#pragma unroll
    for (int p = 0; p < PT; ++p)
      conv_store<NT>(acc[p], nt, mb + 16 * (wave + 4 * p), M, co0, lane, bias, cout, act, slope,
                     dst, y_fp32);
  } else {
    __shared__ f4 red[3][4][64];
    f4 acc[4];
    for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    const int m0 = blockIdx.x * 16;
    const ConvPixel px = conv_pixel(m0 + row, M, H, W);
    const bf16 *wrow = wt + (size_t)(co0 + row) * K;  // column tile t adds 16 t rows
    auto load_b = [&](int k, int t) {
      return k < K ? *reinterpret_cast<const bf16x8 *>(wrow + (size_t)16 * t * K + k) : zero;
    };
    int s = wave;
    bf16x8 a = zero, b[4] = {zero, zero, zero, zero};
    if (s < nsteps) {
      a = conv_a(x, px, 32 * s + kq, K, H, W, cin);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nt) b[t] = load_b(32 * s + kq, t);
    }
    for (; s < nsteps; s += 4) {
      bf16x8 an = zero, bn[4] = {zero, zero, zero, zero};
      if (s + 4 < nsteps) {
        an = conv_a(x, px, 32 * (s + 4) + kq, K, H, W, cin);
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t < nt) bn[t] = load_b(32 * (s + 4) + kq, t);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nt) acc[t] = mfma16(a, b[t], acc[t]);
      a = an;
#pragma unroll
      for (int t = 0; t < 4; ++t) b[t] = bn[t];
    }
    if (wave > 0)
#pragma unroll
      for (int t = 0; t < 4; ++t) red[wave - 1][t][lane] = acc[t];
    __syncthreads();
    if (wave == 0) {
      for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] += red[w][t][lane];
      conv_store<4>(acc, nt, m0, M, co0, lane, bias, cout, act, slope, dst, y_fp32);
    }
  }
}

// Forward 3x3 convolution for layers with few pixels and long reductions
// (deep levels): a workgroup of 16 waves computes 64 pixels x 64 output
// channels.  The waves form 4 groups; group g takes the reduction steps
// g, g + 4, ... (32 k each), wave q of a group the pixel tile 16 q, all four
// column tiles.  Each group stages its step's weight slice (64 channels x 32
// k) in its own double-buffered LDS slice, read by its four waves; the A
// operand is gathered as in conv3x3_kernel.  The groups' sums are added in
// group order through LDS before the epilogue.
constexpr int kGroups = 4;

__global__ void __launch_bounds__(1024) conv3x3_kgroups_kernel(
    ConvSrc x, int B, int H, int W, const bf16 *__restrict__ wt, const float *__restrict__ bias,
    int cout, int act, float slope, ConvDst dst, int y_fp32) {
  // weight slices: [group][buffer][64 x kWRow]; reused for the reduction
  __shared__ __attribute__((aligned(16))) char lds_raw[(kGroups - 1) * 4 * 4 * 64 * 16];
  static_assert(sizeof(lds_raw) >= kGroups * 2 * kCoTile * kWRow * sizeof(bf16), "LDS");
  bf16 *sw_all = reinterpret_cast<bf16 *>(lds_raw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = wave >> 2, q = wave & 3, gt = tid & 255;  // group, wave in group, thread in group
  const int cin = x.ca + x.cb;
  const int M = B * H * W, K = 9 * cin, nsteps = (K + 31) / 32;
  const int rounds = (nsteps + kGroups - 1) / kGroups;
  const int co0 = blockIdx.y * kCoTile;
  const int nt = min(4, (cout - co0) >> 4);
  const int row = lane & 15, kq = 8 * (lane >> 4);
  const bf16x8 zero = {};
  bf16 *sw = sw_all + g * 2 * kCoTile * kWRow;
  const int m0 = blockIdx.x * 64 + 16 * q;
  const ConvPixel px = conv_pixel(m0 + row, M, H, W);
  // weight loading role within the group: channel wo of the slice, k offset 8 wk
  const int wo = gt >> 2, wk = 8 * (gt & 3);
  const bool wok = co0 + wo < cout;
  const bf16 *wrow = wt + (size_t)(co0 + wo) * K;
  f4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
  // step of round r for this group: s = kGroups r + g (none beyond nsteps)
  auto step_k = [&](int r) { return 32 * (kGroups * r + g); };
  int k = step_k(0);
  bf16x8 a = conv_a(x, px, k + kq, K, H, W, cin);
  bf16x8 wv = (wok && k + wk < K) ? *reinterpret_cast<const bf16x8 *>(wrow + k + wk) : zero;
  *reinterpret_cast<bf16x8 *>(&sw[wo * kWRow + wk]) = wv;
  __syncthreads();
  for (int r = 0; r < rounds; ++r) {
    const int cur = r & 1;
    const int kn = step_k(r + 1);
    bf16x8 an = zero;
    if (r + 1 < rounds) {
      an = conv_a(x, px, kn + kq, K, H, W, cin);
      wv = (wok && kn + wk < K) ? *reinterpret_cast<const bf16x8 *>(wrow + kn + wk) : zero;
    }
    if (k < K) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < nt) {
          const bf16x8 b = *reinterpret_cast<const bf16x8 *>(
              &sw[cur * kCoTile * kWRow + (16 * t + row) * kWRow + kq]);
          acc[t] = mfma16(a, b, acc[t]);
        }
      }
    }
    if (r + 1 < rounds)
      *reinterpret_cast<bf16x8 *>(&sw[(cur ^ 1) * kCoTile * kWRow + wo * kWRow + wk]) = wv;
    __syncthreads();
    a = an;
    k = kn;
  }
  // groups 1..3 hand their sums to group 0, which adds them in group order
  f4 *red = reinterpret_cast<f4 *>(lds_raw);  // [group - 1][wave in group][tile][64]
  if (g > 0)
#pragma unroll
    for (int t = 0; t < 4; ++t) red[(((g - 1) * 4 + q) * 4 + t) * 64 + lane] = acc[t];
  __syncthreads();
  if (g == 0) {
    for (int h = 0; h < kGroups - 1; ++h)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] += red[((h * 4 + q) * 4 + t) * 64 + lane];
    conv_store<4>(acc, nt, m0, M, co0, lane, bias, cout, act, slope, dst, y_fp32);
  }
}

// Forward 3x3 convolution over bands of image rows, for inputs small enough
// to stage in LDS: a workgroup computes the R W = 64 PT pixels of R rows of
// one image for 16 NT output channels.  It copies the input rows band - 1 ..
// band + R with a zero column on each side ((R + 2) x (W + 2) pixels x cin
// channels, through the ConvSrc, so the upsampled and concatenated decoder
// inputs work as in conv3x3_kernel) and the 16 NT weight rows into LDS once;
// every tap then reads its shifted pixels from LDS (channels contiguous: a
// lane's 8 k are 16 aligned bytes).  The GEMM is that of conv3x3_kernel
// (rows = pixels, columns = output channels, k = tap x channel in steps of
// 32); wave w takes the pixel tiles 16 (w + 4 p), p < PT.
template <int PT, int NT, bool WLDS>
__global__ void __launch_bounds__(256) conv3x3_rows_kernel(
    ConvSrc x, int B, int H, int W, const bf16 *__restrict__ wt, const float *__restrict__ bias,
    int cout, int act, float slope, ConvDst dst, int y_fp32, int R, int PS) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cin = x.ca + x.cb, K = 9 * cin, KP = K + 8, nsteps = (K + 31) / 32;
  const int WP = W + 2;
  // [R + 2][W + 2] pixels of PS >= cin elements (a multiple of 8)
  bf16 *sin = reinterpret_cast<bf16 *>(lds_raw);
  bf16 *sw = sin + (size_t)(R + 2) * WP * PS;      // [16 NT][K + 8]
  const int bands_img = H / R;
  const int n = blockIdx.x / bands_img, y0 = (blockIdx.x - n * bands_img) * R;
  const int co0 = blockIdx.y * kCoTile;
  const int nt = min(NT, (cout - co0) >> 4);
  const int row = lane & 15, kq = 8 * (lane >> 4);
  // input rows y0 - 1 .. y0 + R, columns -1 .. W (zero outside the image)
  const int cg = cin / 8, nvec = (R + 2) * WP * cg;
  for (int v = threadIdx.x; v < nvec; v += 256) {
    const int c8 = v % cg, pix = v / cg;
    const int r = pix / WP, cc = pix - r * WP;
    const bf16x8 val = src_load(x, n, y0 - 1 + r, cc - 1, 8 * c8, H, W);
    *reinterpret_cast<bf16x8 *>(sin + (size_t)pix * PS + 8 * c8) = val;
  }
  // the weight rows of this workgroup's output channels (WLDS; else they are
  // read from global memory, which leaves LDS to the input band)
  if constexpr (WLDS) {
    const int kv = K / 8;
    for (int v = threadIdx.x; v < 16 * NT * kv; v += 256) {
      const int o = v / kv, k8 = v - o * kv;
      bf16x8 val = {};
      if (o < 16 * nt)
        val = *reinterpret_cast<const bf16x8 *>(wt + (size_t)(co0 + o) * K + 8 * k8);
      *reinterpret_cast<bf16x8 *>(sw + o * KP + 8 * k8) = val;
    }
  }
  __syncthreads();
  f4 acc[PT][NT];
#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[p][t] = f4{0.f, 0.f, 0.f, 0.f};
  int base[PT];  // LDS pixel index of each tile's pixel at tap (0, 0), i.e. (y - 1, x - 1)
#pragma unroll
  for (int p = 0; p < PT; ++p) {
    const int m = 16 * (wave + 4 * p) + row;
    const int r = m / W, c = m - r * W;
    base[p] = r * WP + c;
  }
  const bf16x8 zero = {};
  for (int s = 0; s < nsteps; ++s) {
    const int k = 32 * s + kq;
    const bool kok = k < K;
    const int tap = kok ? k / cin : 0, c = k - tap * cin;
    const int toff = (tap / 3) * WP + tap % 3;
    bf16x8 a[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p)
      a[p] = kok ? *reinterpret_cast<const bf16x8 *>(sin + (size_t)(base[p] + toff) * PS + c)
                 : zero;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t < nt) {
        bf16x8 b = zero;
        if (kok)
          b = WLDS ? *reinterpret_cast<const bf16x8 *>(sw + (16 * t + row) * KP + k)
                   : *reinterpret_cast<const bf16x8 *>(wt + (size_t)(co0 + 16 * t + row) * K + k);
#pragma unroll
        for (int p = 0; p < PT; ++p) acc[p][t] = mfma16(a[p], b, acc[p][t]);
      }
    }
  }
  const int mb = ((n * H) + y0) * W;
#pragma unroll
  for (int p = 0; p < PT; ++p)
    conv_store<NT>(acc[p], nt, mb + 16 * (wave + 4 * p), B * H * W, co0, lane, bias, cout, act,
                   slope, dst, y_fp32);
}

// Weight gradient as a GEMM: rows = output channels o, columns = k = t*cin + c,
// reduction over the pixels of one chunk.  A workgroup (4 waves) computes a
// (16 OB) x 64 tile of (o, k), OB = 1, 2 or 4 output blocks of 16 channels;
// the 4 waves form OB output blocks x 4/OB pixel groups, so that small
// layers (16 or 32 channels) keep every wave busy.  Per step of 128/OB pixels
// the workgroup loads dy[pixels, 16 OB o] and the tap-shifted x[pixels, 64 k]
// with 16-byte vector loads (8 channels per load; cin and cout are multiples
// of 16, so 8 consecutive k lie in one tap) and stores both transposed in LDS,
// pixels contiguous, the layout the MFMA reduction reads; wave (ob, pg) runs
// its output block against the four 16-column tiles over its 32 pixels.  The
// pixel groups' sums are added through LDS in group order.  Partial sums per
// chunk go to `part` (and, for the first k tile, the bias partial sums to
// `partb`).
constexpr int kWgK = 64;  // k columns per workgroup

template <int OB>
__global__ void __launch_bounds__(256) wgrad_kernel(const bf16 *__restrict__ dy, ConvSrc x,
                                                     int B, int H, int W, int cout, int chunk,
                                                     float *__restrict__ part,
                                                     float *__restrict__ partb) {
  const int cin = x.ca + x.cb;
  constexpr int PG = 4 / OB;         // pixel groups
  constexpr int PX = 32 * PG;        // pixels per step
  constexpr int ROW = PX + 8;        // LDS row length in bf16 (padding: fewer bank conflicts)
  __shared__ __attribute__((aligned(16))) bf16 sA[16 * OB * ROW];  // dy^T: [o][pixel]
  __shared__ __attribute__((aligned(16))) bf16 sB[kWgK * ROW];     // x^T:  [k][pixel]
  __shared__ f4 red[PG > 1 ? PG - 1 : 1][OB][4][64];
  __shared__ float redb[PG > 1 ? PG - 1 : 1][OB][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ob = wave % OB, pg = wave / OB;
  const int HW = H * W, M = B * HW, K = 9 * cin;
  const int o0 = blockIdx.x * 16 * OB, k0 = blockIdx.y * kWgK;
  const int p0 = blockIdx.z * chunk, p1 = min(M, p0 + chunk);
  // loading roles: dy pixel ap with channels 8 ag..; x pixels tid/8 + 32 j with k 8 kg..
  const int ap = tid / (2 * OB), ag = tid % (2 * OB), kg = tid & 7;
  const int lo = o0 + 8 * ag, lk = k0 + 8 * kg;
  const bool o_ok = lo < cout, k_ok = lk < K;
  int lc = 0, oy = 0, ox = 0;
  if (k_ok) {
    const int tap = lk / cin;
    lc = lk - tap * cin;
    oy = tap / 3 - 1;
    ox = tap % 3 - 1;
  }
  // MFMA role: A row (output channel) and 8 pixels of the reduction
  const int row = lane & 15, q = 32 * pg + 8 * (lane >> 4);
  const bool bias = partb && blockIdx.y == 0;
  f4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.0f;
  const bf16x8 zero = {};
  for (int p = p0; p < p1; p += PX) {
    bf16x8 va = zero, vb[PG];
    const int ma = p + ap;
    if (ma < p1 && o_ok) va = *reinterpret_cast<const bf16x8 *>(dy + (size_t)ma * cout + lo);
#pragma unroll
    for (int j = 0; j < PG; ++j) {
      vb[j] = zero;
      const int mm = p + (tid >> 3) + 32 * j;
      if (mm < p1 && k_ok) {
        const int n = mm / HW, r = mm - n * HW;
        const int py = r / W;
        vb[j] = src_load(x, n, py + oy, r - py * W + ox, lc, H, W);
      }
    }
    __syncthreads();  // the previous step's LDS reads are done
#pragma unroll
    for (int e = 0; e < 8; ++e) sA[(8 * ag + e) * ROW + ap] = va[e];
#pragma unroll
    for (int j = 0; j < PG; ++j)
#pragma unroll
      for (int e = 0; e < 8; ++e) sB[(8 * kg + e) * ROW + (tid >> 3) + 32 * j] = vb[j][e];
    __syncthreads();
    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(sA + (16 * ob + row) * ROW + q);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf16x8 b = *reinterpret_cast<const bf16x8 *>(sB + (16 * t + row) * ROW + q);
      acc[t] = mfma16(a, b, acc[t]);
    }
    if (bias)
#pragma unroll
      for (int e = 0; e < 8; ++e) bsum += (float)a[e];
  }
  if constexpr (PG > 1) {  // add the pixel groups' sums in group order
    if (pg > 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) red[pg - 1][ob][t][lane] = acc[t];
      redb[pg - 1][ob][lane] = bsum;
    }
    __syncthreads();
    if (pg == 0)
      for (int g = 0; g < PG - 1; ++g) {
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] += red[g][ob][t][lane];
        bsum += redb[g][ob][lane];
      }
  }
  if (pg != 0) return;
  // D: lane holds column k0 + 16 t + row, output channels o0 + 16 ob + 4 (lane / 16) + e
  const size_t base = (size_t)blockIdx.z * cout * K;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int kk = k0 + 16 * t + row;
    if (kk >= K) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int o = o0 + 16 * ob + 4 * (lane >> 4) + e;
      if (o < cout) part[base + (size_t)o * K + kk] = acc[t][e];
    }
  }
  if (bias) {
    bsum += __shfl_xor(bsum, 16, 64);
    bsum += __shfl_xor(bsum, 32, 64);
    const int o = o0 + 16 * ob + row;
    if (lane < 16 && o < cout) partb[(size_t)blockIdx.z * cout + o] = bsum;
  }
}

// Weight gradient over bands of image rows (W a multiple of 8, at most 512):
// a workgroup owns 16 OB output channels x 16 CB input channels for all nine
// taps and runs over bands of R rows of one image (P = R W <= 512 pixels, R
// as large as 64 KB of LDS allows).  Per band it loads dy[band, o tile] and the input rows
// band - 1 .. band + R of its channel tile; each thread takes blocks of 8
// pixels x 8 channels (eight 16-byte loads), transposes them in registers
// (v_perm) and stores 8 pixel-contiguous 16-byte rows to LDS.  Every tap then
// reads the same LDS rows: the row shift of a tap is a row offset, the column
// shift comes from two aligned 16-byte reads joined by v_alignbyte.  The four
// waves take every fourth 32-pixel reduction step of the band and add their
// sums in wave order at the end.  Partial sums per chunk of bands go to
// `part` (bias partial sums, for the first channel tile, to `partb`), laid
// out as for wgrad_kernel.
constexpr int kRowPix = 512;             // pixels per band at most
constexpr int kDyPitch = kRowPix + 8;    // LDS row of dy^T in bf16
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

// Row r of an 8 x 8 block in registers (8 pixels x 8 channels, pixel-major)
// into 8 channel rows of 8 pixels: channel 2k takes the low halves of dword
// k of the pixels, channel 2k + 1 the high halves.
__device__ __forceinline__ void transpose8(const u4 in[8], u4 out[8]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      out[2 * k][j] = __builtin_amdgcn_perm(in[2 * j + 1][k], in[2 * j][k], 0x05040100u);
      out[2 * k + 1][j] = __builtin_amdgcn_perm(in[2 * j + 1][k], in[2 * j][k], 0x07060302u);
    }
}

// The 8 bf16 that start 2 bytes before (sh = -1) or after (sh = +1) the
// aligned block b of a row whose neighbours are a (before) and c (after).
__device__ __forceinline__ u4 shift_left1(const u4 &a, const u4 &b) {  // a[7], b[0..6]
  return u4{__builtin_amdgcn_alignbyte(b[0], a[3], 2), __builtin_amdgcn_alignbyte(b[1], b[0], 2),
            __builtin_amdgcn_alignbyte(b[2], b[1], 2), __builtin_amdgcn_alignbyte(b[3], b[2], 2)};
}
__device__ __forceinline__ u4 shift_right1(const u4 &b, const u4 &c) {  // b[1..7], c[0]
  return u4{__builtin_amdgcn_alignbyte(b[1], b[0], 2), __builtin_amdgcn_alignbyte(b[2], b[1], 2),
            __builtin_amdgcn_alignbyte(b[3], b[2], 2), __builtin_amdgcn_alignbyte(c[0], b[3], 2)};
}

__device__ __forceinline__ bf16x8 as_bf16x8(const u4 &v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

template <int OB, int CB>
__global__ void __launch_bounds__(256) wgrad_rows_kernel(const bf16 *__restrict__ dy, ConvSrc x,
                                                          int B, int H, int W, int cout, int R,
                                                          int bands_per_chunk,
                                                          float *__restrict__ part,
                                                          float *__restrict__ partb) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  constexpr int NO = 16 * OB, NC = 16 * CB;
  const int cin = x.ca + x.cb, K = 9 * cin;
  const int XP = W + 16;                 // LDS input row: 8 zeros, W pixels, 8 zeros
  const int P = R * W, ksteps = P / 32;  // pixels and 32-pixel steps of a band
  bf16 *sdy = reinterpret_cast<bf16 *>(lds_raw);            // [NO][kDyPitch]
  bf16 *sx = sdy + NO * kDyPitch;                          // [NC][R + 2][XP]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int o0 = blockIdx.x * NO, c0 = blockIdx.y * NC;
  const int bands_img = H / R, nbands = B * bands_img;
  const int b0 = blockIdx.z * bands_per_chunk, b1 = min(nbands, b0 + bands_per_chunk);
  const bool bias = partb && blockIdx.y == 0;
  // the zero columns left and right of every input row
  for (int i = tid; i < NC * (R + 2); i += 256) {
    *reinterpret_cast<u4 *>(sx + i * XP) = u4{0, 0, 0, 0};
    *reinterpret_cast<u4 *>(sx + i * XP + W + 8) = u4{0, 0, 0, 0};
  }
  f4 acc[OB][9][CB];
#pragma unroll
  for (int ob = 0; ob < OB; ++ob)
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[ob][t][cb] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum[OB];
#pragma unroll
  for (int ob = 0; ob < OB; ++ob) bsum[ob] = 0.0f;
  const int row = lane & 15, g8 = 8 * (lane >> 4);
  const int dy_units = (P / 8) * (NO / 8), x_units = (R + 2) * (W / 8) * (NC / 8);
  for (int band = b0; band < b1; ++band) {
    const int n = band / bands_img, y0 = (band - n * bands_img) * R;
    const size_t m0 = ((size_t)n * H + y0) * W;
    __syncthreads();  // the previous band's LDS reads are done
    for (int u = tid; u < dy_units + x_units; u += 256) {
      u4 in[8], tr[8];
      if (u < dy_units) {  // 8 pixels x 8 output channels of dy
        const int pb = u / (NO / 8), cg = u - pb * (NO / 8);
        const bf16 *src = dy + (m0 + 8 * pb) * cout + o0 + 8 * cg;
#pragma unroll
        for (int i = 0; i < 8; ++i) in[i] = *reinterpret_cast<const u4 *>(src + (size_t)i * cout);
        transpose8(in, tr);
#pragma unroll
        for (int c = 0; c < 8; ++c)
          *reinterpret_cast<u4 *>(sdy + (8 * cg + c) * kDyPitch + 8 * pb) = tr[c];
      } else {  // 8 pixels x 8 input channels of input row y0 - 1 + r
        const int v = u - dy_units;
        const int cg = v % (NC / 8), rest = v / (NC / 8);
        const int xb = rest % (W / 8), r = rest / (W / 8);
        const int yy = y0 - 1 + r;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const bf16x8 t = src_load(x, n, yy, 8 * xb + i, c0 + 8 * cg, H, W);
          __builtin_memcpy(&in[i], &t, 16);
        }
        transpose8(in, tr);
#pragma unroll
        for (int c = 0; c < 8; ++c)
          *reinterpret_cast<u4 *>(sx + ((8 * cg + c) * (R + 2) + r) * XP + 8 + 8 * xb) = tr[c];
      }
    }
    __syncthreads();
    for (int ks = wave; ks < ksteps; ks += 4) {
      const int p = 32 * ks + g8;  // this lane's 8 pixels: row pr, columns px .. px + 7
      const int pr = p / W, px = p - pr * W;
      bf16x8 a[OB];
#pragma unroll
      for (int ob = 0; ob < OB; ++ob) {
        a[ob] = *reinterpret_cast<const bf16x8 *>(sdy + (16 * ob + row) * kDyPitch + p);
        if (bias)
#pragma unroll
          for (int e = 0; e < 8; ++e) bsum[ob] += (float)a[ob][e];
      }
#pragma unroll
      for (int ty = 0; ty < 3; ++ty)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const bf16 *xr = sx + ((16 * cb + row) * (R + 2) + pr + ty) * XP + px;
          const u4 lo = *reinterpret_cast<const u4 *>(xr);       // columns px - 8 .. px - 1
          const u4 mid = *reinterpret_cast<const u4 *>(xr + 8);  // px .. px + 7
          const u4 hi = *reinterpret_cast<const u4 *>(xr + 16);  // px + 8 .. px + 15
          const bf16x8 bl = as_bf16x8(shift_left1(lo, mid)), bm = as_bf16x8(mid),
                       bh = as_bf16x8(shift_right1(mid, hi));
#pragma unroll
          for (int ob = 0; ob < OB; ++ob) {
            acc[ob][3 * ty][cb] = mfma16(a[ob], bl, acc[ob][3 * ty][cb]);
            acc[ob][3 * ty + 1][cb] = mfma16(a[ob], bm, acc[ob][3 * ty + 1][cb]);
            acc[ob][3 * ty + 2][cb] = mfma16(a[ob], bh, acc[ob][3 * ty + 2][cb]);
          }
        }
    }
  }
  // add the four waves' sums in wave order through LDS, one tile at a time
  f4 *red = reinterpret_cast<f4 *>(lds_raw);  // [3][64]
  float *redb = reinterpret_cast<float *>(red + 3 * 64);  // [3][OB][64]
  __syncthreads();
  if (wave > 0)
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) redb[((wave - 1) * OB + ob) * 64 + lane] = bsum[ob];
#pragma unroll
  for (int ob = 0; ob < OB; ++ob)
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        if (wave > 0) red[(wave - 1) * 64 + lane] = acc[ob][t][cb];
        __syncthreads();
        if (wave == 0) acc[ob][t][cb] = ((acc[ob][t][cb] + red[lane]) + red[64 + lane]) +
                                        red[128 + lane];
        __syncthreads();
      }
  if (wave != 0) return;
  // D: lane holds input channel c0 + 16 cb + row, output channels
  // o0 + 16 ob + 4 (lane / 16) + e
  const size_t base = (size_t)blockIdx.z * cout * K;
#pragma unroll
  for (int ob = 0; ob < OB; ++ob)
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int o = o0 + 16 * ob + 4 * (lane >> 4) + e;
          part[base + (size_t)o * K + t * cin + c0 + 16 * cb + row] = acc[ob][t][cb][e];
        }
  if (bias)
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      float b = ((bsum[ob] + redb[ob * 64 + lane]) + redb[(OB + ob) * 64 + lane]) +
                redb[(2 * OB + ob) * 64 + lane];
      b += __shfl_xor(b, 16, 64);
      b += __shfl_xor(b, 32, 64);
      if (lane < 16) partb[(size_t)blockIdx.z * cout + o0 + 16 * ob + lane] = b;
    }
}

// Sum over the nsplit chunks of one partial-sum array in a fixed order.
// Up to kThreadSplits chunks, each thread adds the chunks of one output in
// increasing order (256 outputs per workgroup).  Beyond that, the 256
// threads of a workgroup cover 64 consecutive outputs x 4 waves; wave w adds
// the chunks w, w + 4, w + 8, ... in increasing order (64 consecutive outputs
// per load: coalesced), and the four wave sums of an output are added in wave
// order.  out(i, v) receives output i's sum.
constexpr int kThreadSplits = 32;

__host__ __device__ inline int sum_outputs_per_block(int nsplit) {
  return nsplit <= kThreadSplits ? 256 : 64;
}

template <typename Src, typename Out>
__device__ __forceinline__ void sum_chunks(int nsplit, int b, size_t count, const Src &src,
                                           const Out &out) {
  __shared__ float lds[4][64];
  if (nsplit <= kThreadSplits) {
    const size_t i = (size_t)b * 256 + threadIdx.x;
    if (i >= count) return;
    float s = 0.0f;
    for (int z = 0; z < nsplit; ++z) s += src(i, z);
    out(i, s);
    return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const size_t i = (size_t)b * 64 + lane;
  float s = 0.0f;
  if (i < count) {
#pragma unroll 8
    for (int z = w; z < nsplit; z += 4) s += src(i, z);
  }
  lds[w][lane] = s;
  __syncthreads();
  if (w == 0 && i < count) out(i, ((lds[0][lane] + lds[1][lane]) + lds[2][lane]) + lds[3][lane]);
}

// Sums of `nsplit` partial arrays, for two arrays at once: outputs i < n add
// part[z n + i] into out[i], outputs n <= i < n + nb add partb[z nb + i - n]
// into outb[i - n].
__global__ void __launch_bounds__(256) sum_parts_kernel(const float *__restrict__ part,
                                                        int nsplit, size_t n,
                                                        float *__restrict__ out,
                                                        const float *__restrict__ partb,
                                                        size_t nb, float *__restrict__ outb) {
  sum_chunks(
      nsplit, blockIdx.x, n + nb,
      [&](size_t i, int z) { return i < n ? part[(size_t)z * n + i] : partb[(size_t)z * nb + i - n]; },
      [&](size_t i, float v) {
        if (i < n)
          out[i] = v;
        else
          outb[i - n] = v;
      });
}

__global__ void __launch_bounds__(256) weights_kernel(const float *__restrict__ w32, int cout,
                                                      int cin, bf16 *__restrict__ wf,
                                                      bf16 *__restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cout * 9 * cin) return;
  const int o = i / (9 * cin), r = i - o * 9 * cin, t = r / cin, c = r - t * cin;
  const bf16 v = (bf16)w32[i];
  wf[i] = v;
  wb[((size_t)c * 9 + (8 - t)) * cout + o] = v;
}

// The layer table of weights_layers_kernel: the workgroups of layer l are
// [block0[l], block0[l + 1]).
struct WeightLayers {
  int n;
  int cout[CLB_NN_MAX_LAYERS], cin[CLB_NN_MAX_LAYERS];
  long long offset[CLB_NN_MAX_LAYERS];
  int block0[CLB_NN_MAX_LAYERS + 1];
};

__global__ void __launch_bounds__(256) weights_layers_kernel(const float *__restrict__ w32,
                                                             WeightLayers L,
                                                             bf16 *__restrict__ wf,
                                                             bf16 *__restrict__ wb) {
  int l = 0;
  while (l + 1 < L.n && (int)blockIdx.x >= L.block0[l + 1]) ++l;
  const int cout = L.cout[l], cin = L.cin[l];
  const int i = (blockIdx.x - L.block0[l]) * blockDim.x + threadIdx.x;
  if (i >= cout * 9 * cin) return;
  const int o = i / (9 * cin), r = i - o * 9 * cin, t = r / cin, c = r - t * cin;
  const size_t base = (size_t)L.offset[l];
  const bf16 v = (bf16)w32[base + i];
  wf[base + i] = v;
  wb[base + ((size_t)c * 9 + (8 - t)) * cout + o] = v;
}

__global__ void __launch_bounds__(256) pool2_kernel(const bf16 *__restrict__ x, int B, int H,
                                                    int W, int C, bf16 *__restrict__ y) {
  const size_t n = (size_t)B * (H / 2) * (W / 2) * C;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = i % C;
  size_t r = i / C;
  const int j = r % (W / 2);
  r /= (W / 2);
  const int ii = r % (H / 2);
  const int b = r / (H / 2);
  const size_t s = (((size_t)b * H + 2 * ii) * W + 2 * j) * C + c;
  const float v = (float)x[s] + (float)x[s + C] + (float)x[s + (size_t)W * C] +
                  (float)x[s + (size_t)W * C + C];
  y[i] = (bf16)(0.25f * v);
}

__global__ void __launch_bounds__(256) pool2_grad_kernel(const bf16 *__restrict__ dy, int B,
                                                         int H, int W, int C,
                                                         bf16 *__restrict__ dx) {
  const size_t n = (size_t)B * H * W * C;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = i % C;
  size_t r = i / C;
  const int j = r % W;
  r /= W;
  const int ii = r % H;
  const int b = r / H;
  dx[i] = (bf16)(0.25f * (float)dy[(((size_t)b * (H / 2) + ii / 2) * (W / 2) + j / 2) * C + c]);
}

__global__ void __launch_bounds__(256) up2_kernel(const bf16 *__restrict__ x, int B, int H, int W,
                                                  int C, bf16 *__restrict__ y) {
  const size_t n = (size_t)B * 2 * H * 2 * W * C;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = i % C;
  size_t r = i / C;
  const int j = r % (2 * W);
  r /= (2 * W);
  const int ii = r % (2 * H);
  const int b = r / (2 * H);
  y[i] = x[(((size_t)b * H + ii / 2) * W + j / 2) * C + c];
}

__global__ void __launch_bounds__(256) up2_grad_kernel(const bf16 *__restrict__ dy, int B, int H,
                                                       int W, int C, bf16 *__restrict__ dx) {
  const size_t n = (size_t)B * H * W * C;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = i % C;
  size_t r = i / C;
  const int j = r % W;
  r /= W;
  const int ii = r % H;
  const int b = r / H;
  const size_t s = (((size_t)b * 2 * H + 2 * ii) * 2 * W + 2 * j) * C + c;
  const size_t row = (size_t)2 * W * C;
  const float v = (float)dy[s] + (float)dy[s + C] + (float)dy[s + row] + (float)dy[s + row + C];
  dx[i] = (bf16)v;
}

__global__ void __launch_bounds__(256) concat_kernel(const bf16 *__restrict__ a, int ca,
                                                     const bf16 *__restrict__ b, int cb,
                                                     size_t npix, bf16 *__restrict__ y) {
  const int C = ca + cb;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix * C) return;
  const size_t p = i / C;
  const int c = i - p * C;
  y[i] = c < ca ? a[p * ca + c] : b[p * cb + (c - ca)];
}

__global__ void __launch_bounds__(256) split_kernel(const bf16 *__restrict__ y, int ca, int cb,
                                                    size_t npix, bf16 *__restrict__ a,
                                                    bf16 *__restrict__ b) {
  const int C = ca + cb;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix * C) return;
  const size_t p = i / C;
  const int c = i - p * C;
  if (c < ca)
    a[p * ca + c] = y[i];
  else
    b[p * cb + (c - ca)] = y[i];
}

// The same layers on groups of 8 channels (16 bytes per load and store) for
// channel counts that are multiples of 8: grid.y runs over the image rows of
// the output (batch x height), grid.x over (column, channel group), so each
// thread needs one 32-bit division.
__global__ void __launch_bounds__(256) pool2_v8_kernel(const bf16x8 *__restrict__ x, int H, int W,
                                                       int C8, bf16x8 *__restrict__ y) {
  const int Wo = W / 2, Ho = H / 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Wo * C8) return;
  const int j = i / C8, c = i - j * C8;
  const int row = blockIdx.y, b = row / Ho, ii = row - b * Ho;  // output row
  const size_t s = ((size_t)(b * H + 2 * ii) * W + 2 * j) * C8 + c;
  const size_t dn = (size_t)W * C8;
  const bf16x8 v0 = x[s], v1 = x[s + C8], v2 = x[s + dn], v3 = x[s + dn + C8];
  bf16x8 o;
#pragma unroll
  for (int e = 0; e < 8; ++e)
    o[e] = (bf16)(0.25f * ((float)v0[e] + (float)v1[e] + (float)v2[e] + (float)v3[e]));
  y[(size_t)row * Wo * C8 + i] = o;
}

// The pooling and upsampling gradients below optionally finish the gradient
// through a leaky ReLU whose output y has the result's layout (y null: none):
// s = result (+ add, the tensor's other gradient contribution, rounded to
// bfloat16 as clb_nn_act_grad adds), then s (y > 0) or slope s.
__device__ __forceinline__ bf16x8 act_finish(bf16x8 o, const bf16x8 *add, const bf16x8 *y,
                                             size_t i, float slope) {
  if (!y) return o;
  const bf16x8 yy = y[i];
  bf16x8 a = {};
  if (add) a = add[i];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float s = (float)o[e];
    if (add) s = (float)(bf16)((float)a[e] + s);
    o[e] = (bf16)((float)yy[e] > 0.0f ? s : slope * s);
  }
  return o;
}

__global__ void __launch_bounds__(256) pool2_grad_v8_kernel(const bf16x8 *__restrict__ dy, int H,
                                                            int W, int C8,
                                                            bf16x8 *__restrict__ dx,
                                                            const bf16x8 *__restrict__ add,
                                                            const bf16x8 *__restrict__ y,
                                                            float slope) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * C8) return;
  const int j = i / C8, c = i - j * C8;
  const int row = blockIdx.y, b = row / H, ii = row - b * H;  // row of dx
  const bf16x8 v = dy[((size_t)(b * (H / 2) + ii / 2) * (W / 2) + j / 2) * C8 + c];
  bf16x8 o;
#pragma unroll
  for (int e = 0; e < 8; ++e) o[e] = (bf16)(0.25f * (float)v[e]);
  const size_t k = (size_t)row * W * C8 + i;
  dx[k] = act_finish(o, add, y, k, slope);
}

__global__ void __launch_bounds__(256) up2_grad_v8_kernel(const bf16x8 *__restrict__ dy, int H,
                                                          int W, int C8, bf16x8 *__restrict__ dx,
                                                          const bf16x8 *__restrict__ y,
                                                          float slope) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * C8) return;
  const int j = i / C8, c = i - j * C8;
  const int row = blockIdx.y, b = row / H, ii = row - b * H;  // row of dx (H x W)
  const size_t s = ((size_t)(b * 2 * H + 2 * ii) * 2 * W + 2 * j) * C8 + c;
  const size_t dn = (size_t)2 * W * C8;
  const bf16x8 v0 = dy[s], v1 = dy[s + C8], v2 = dy[s + dn], v3 = dy[s + dn + C8];
  bf16x8 o;
#pragma unroll
  for (int e = 0; e < 8; ++e) o[e] = (bf16)((float)v0[e] + (float)v1[e] + (float)v2[e] + (float)v3[e]);
  const size_t k = (size_t)row * W * C8 + i;
  dx[k] = act_finish(o, nullptr, y, k, slope);
}

__global__ void __launch_bounds__(256) act_grad_v8_kernel(const bf16x8 *__restrict__ g0,
                                                          const bf16x8 *__restrict__ g1,
                                                          const bf16x8 *__restrict__ out,
                                                          size_t n8, float slope,
                                                          bf16x8 *__restrict__ dz) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n8) return;
  const bf16x8 a = g0[i], o = out[i];
  bf16x8 b = {};
  if (g1) b = g1[i];
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float s = (float)a[e];
    if (g1) s = (float)(bf16)(s + (float)b[e]);
    r[e] = (bf16)((float)o[e] > 0.0f ? s : slope * s);
  }
  dz[i] = r;
}

__global__ void __launch_bounds__(256) act_grad_kernel(const bf16 *__restrict__ g0,
                                                       const bf16 *__restrict__ g1,
                                                       const bf16 *__restrict__ out, size_t n,
                                                       float slope, bf16 *__restrict__ dz) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = (float)g0[i];
  if (g1) s = (float)(bf16)(s + (float)g1[i]);
  dz[i] = (bf16)((float)out[i] > 0.0f ? s : slope * s);
}

constexpr int kMseBlocks = 1024;

__global__ void __launch_bounds__(256) mse_kernel(const float *__restrict__ out, int ldo,
                                                  const float *__restrict__ tgt, int nch,
                                                  size_t npix, bf16 *__restrict__ dout,
                                                  double *__restrict__ part) {
  __shared__ double lds[4];
  const double scale = 2.0 / ((double)npix * nch);
  double s = 0.0;
  // 8 consecutive channels of one pixel per thread and iteration (ldo is a
  // multiple of 8 here): two 16-byte loads of out, one 16-byte store
  const int groups = ldo / 8;
  const size_t units = npix * groups;
  for (size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x; u < units;
       u += (size_t)gridDim.x * blockDim.x) {
    const size_t p = u / groups;
    const int c0 = 8 * (int)(u - p * groups);
    const f4 o0 = *reinterpret_cast<const f4 *>(out + p * ldo + c0);
    const f4 o1 = *reinterpret_cast<const f4 *>(out + p * ldo + c0 + 4);
    bf16x8 g;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = c0 + e;
      float v = 0.0f;
      if (c < nch) {
        const float d = (e < 4 ? o0[e] : o1[e - 4]) - tgt[p * nch + c];
        s += (double)d * d;
        v = (float)(scale * d);
      }
      g[e] = (bf16)v;
    }
    *reinterpret_cast<bf16x8 *>(dout + p * ldo + c0) = g;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

__global__ void __launch_bounds__(256) mse_finalize_kernel(const double *__restrict__ part,
                                                           int nparts, double count,
                                                           double *__restrict__ loss) {
  __shared__ double lds[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *loss = (lds[0] + lds[1] + lds[2] + lds[3]) / count;
}

__global__ void __launch_bounds__(256) adamw_kernel(float *__restrict__ p,
                                                    const float *__restrict__ g,
                                                    float *__restrict__ m, float *__restrict__ v,
                                                    size_t n, float lr, float b1, float b2,
                                                    float eps, float wd, float c1, float c2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  p[i] = p[i] - lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
}

// AdamW (adamw_kernel) followed, for the elements that are convolution
// weights of the layer table L (offsets ascending), by the two bfloat16
// copies of weights_layers_kernel.
__global__ void __launch_bounds__(256) adamw_layers_kernel(
    float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
    float *__restrict__ v, size_t n, float lr, float b1, float b2, float eps, float wd, float c1,
    float c2, WeightLayers L, bf16 *__restrict__ wf, bf16 *__restrict__ wb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  const float pi = p[i] - lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
  p[i] = pi;
  // the last layer that starts at or before i
  int lo = 0, hi = L.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((size_t)L.offset[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  const size_t base = (size_t)L.offset[lo];
  if (i < base) return;
  const int cout = L.cout[lo], cin = L.cin[lo];
  const size_t j = i - base;
  if (j >= (size_t)cout * 9 * cin) return;  // a bias or a gap
  const int o = (int)(j / (9 * cin)), r = (int)(j - (size_t)o * 9 * cin), t = r / cin,
            c = r - t * cin;
  const bf16 b = (bf16)pi;
  wf[i] = b;
  wb[base + ((size_t)c * 9 + (8 - t)) * cout + o] = b;
}

__global__ void __launch_bounds__(256) features_kernel(const float *__restrict__ eps_all,
                                                       const float *__restrict__ groups,
                                                       int ngroups, const int32_t *__restrict__ idx,
                                                       int B, int H, int W, bf16 *__restrict__ x) {
  const size_t n = (size_t)B * H * W * 16;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = i & 15;
  size_t r = i >> 4;
  const int j = r % W;
  r /= W;
  const int ii = r % H;
  const int b = r / H;
  const int s = idx[b];
  float v = 0.0f;
  if (c == 0)
    v = (eps_all[((size_t)s * H + ii) * W + j] - 0.625f) * 5.0f;
  else if (c <= ngroups)
    v = groups[(size_t)s * ngroups + (c - 1)];
  else if (c == ngroups + 1)
    v = W > 1 ? 2.0f * j / (W - 1) - 1.0f : 0.0f;
  else if (c == ngroups + 2)
    v = H > 1 ? 2.0f * ii / (H - 1) - 1.0f : 0.0f;
  x[i] = (bf16)v;
}

__global__ void __launch_bounds__(256) gather_kernel(const float *__restrict__ src, int nch,
                                                     const int32_t *__restrict__ idx, int B,
                                                     size_t npix, float *__restrict__ out) {
  const size_t per = npix * nch;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)B * per) return;
  const size_t b = i / per, r = i - b * per;
  out[i] = src[(size_t)idx[b] * per + r];
}

// ------------------------------------------------------------------ host side

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

clb_status launched() {
  return hipGetLastError() == hipSuccess ? CLB_OK : CLB_ERR_HIP;
}

unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

// Output blocks of 16 channels per weight-gradient workgroup.
int wgrad_ob(int cout) { return cout % 64 == 0 ? 4 : (cout % 32 == 0 ? 2 : 1); }

// Workgroup tiles of the weight gradient ((16 OB) output channels x 64 k).
int64_t wgrad_tiles(int cin, int cout) {
  return (int64_t)(cout / (16 * wgrad_ob(cout))) * ((9LL * cin + kWgK - 1) / kWgK);
}

// Split of the pixel reduction of the weight gradient: enough chunks for
// about 2048 workgroups, each chunk a multiple of 128 pixels (a whole number
// of steps for every OB) and >= 512.
void wgrad_plan(int64_t M, int64_t tiles, int *nsplit, int *chunk) {
  int64_t ns = std::max<int64_t>(1, (2048 + tiles - 1) / tiles);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, M / 512));
  int64_t ch = (M + ns - 1) / ns;
  ch = (ch + 127) / 128 * 128;
  *chunk = (int)ch;
  *nsplit = (int)((M + ch - 1) / ch);
}

bool dims_ok(int32_t b, int32_t h, int32_t w) {
  return b > 0 && h > 0 && w > 0 && (int64_t)b * h * w < (1LL << 31);
}

}  // namespace

namespace {

// Launch of the forward kernel: pixel tiles (64 PT pixels per workgroup, the
// largest PT in {4, 2, 1} that still gives about 1024 workgroups), or the
// split reduction below that.
// LDS bytes of conv3x3_rows_kernel for bands of r rows, or 0 if it exceeds
// 64 KiB.
size_t conv_rows_lds(int r, int w, int cin, int ps, int nt, bool wlds) {
  const size_t b = sizeof(bf16) * ((size_t)(r + 2) * (w + 2) * ps +
                                   (wlds ? (size_t)16 * nt * (9 * cin + 8) : 0));
  return b <= 65536 ? b : 0;
}

void conv_launch(const ConvSrc &x, int32_t batch, int32_t h, int32_t w, const bf16 *wb,
                 const float *bias, int32_t cout, int32_t act, float slope, const ConvDst &dst,
                 int32_t y_fp32, hipStream_t s) {
  const int64_t M = (int64_t)batch * h * w;
  const unsigned cot = (unsigned)((cout + kCoTile - 1) / kCoTile);
  auto blocks = [&](int pix) { return (unsigned)((M + pix - 1) / pix); };
  // column tiles per workgroup: 16 channels (NT = 1), 32 (2) or up to 64 (4)
  const int nt = cout >= 64 ? 4 : (cout > 16 ? (cout > 32 ? 4 : 2) : 1);
  const int cin = x.ca + x.cb;
  // Bands of rows staged in LDS: 64 PT pixels per workgroup (PT = 4, 2, 1),
  // whole rows, bands tiling the image height, at least 256 workgroups.
  for (int pt = 4; pt >= 1; pt /= 2) {
    const int pix = 64 * pt;
    if (pix % w || h % (pix / w)) continue;
    const int r = pix / w;
    const int ps = cin;  // pixel stride in LDS (padding it measured no faster)
    // band and weights within 64 KB of LDS; for 16 output channels the
    // weights are read from global memory instead where the two exceed 48 KB
    // (three workgroups then fit a CU instead of two; with more output
    // channels that measured slower)
    const size_t with_w = conv_rows_lds(r, w, cin, ps, nt, true);
    const int64_t wgs = (int64_t)batch * (h / r) * cot;
    if (!with_w || wgs < 256) continue;
    const bool wlds = nt > 1 || with_w <= 49152;
    const size_t lds = conv_rows_lds(r, w, cin, ps, nt, wlds);
    const dim3 grid((unsigned)(batch * (h / r)), cot);
    auto go = [&](auto pt_tag, auto nt_tag) {
      constexpr int PT = decltype(pt_tag)::value, NT = decltype(nt_tag)::value;
      if (wlds)
        hipLaunchKernelGGL((conv3x3_rows_kernel<PT, NT, true>), grid, dim3(256), lds, s, x, batch,
                           h, w, wb, bias, cout, act, slope, dst, y_fp32, r, ps);
      else
        hipLaunchKernelGGL((conv3x3_rows_kernel<PT, NT, false>), grid, dim3(256), lds, s, x,
                           batch, h, w, wb, bias, cout, act, slope, dst, y_fp32, r, ps);
    };
    auto pick = [&](auto pt_tag) {
      if (nt == 1)
        go(pt_tag, std::integral_constant<int, 1>{});
      else if (nt == 2)
        go(pt_tag, std::integral_constant<int, 2>{});
      else
        go(pt_tag, std::integral_constant<int, 4>{});
    };
    if (pt == 4)
      pick(std::integral_constant<int, 4>{});
    else if (pt == 2)
      pick(std::integral_constant<int, 2>{});
    else
      pick(std::integral_constant<int, 1>{});
    return;
  }
  auto go = [&](auto pt_tag, auto nt_tag) {
    constexpr int PT = decltype(pt_tag)::value, NT = decltype(nt_tag)::value;
    hipLaunchKernelGGL((conv3x3_kernel<false, PT, NT>), dim3(blocks(PT * kPixTile), cot),
                       dim3(256), 0, s, x, batch, h, w, wb, bias, cout, act, slope, dst, y_fp32);
  };
  auto pick_nt = [&](auto pt_tag) {
    if (nt == 1)
      go(pt_tag, std::integral_constant<int, 1>{});
    else if (nt == 2)
      go(pt_tag, std::integral_constant<int, 2>{});
    else
      go(pt_tag, std::integral_constant<int, 4>{});
  };
  if ((int64_t)blocks(4 * kPixTile) * cot >= 1024)
    pick_nt(std::integral_constant<int, 4>{});
  else if ((int64_t)blocks(2 * kPixTile) * cot >= 1024)
    pick_nt(std::integral_constant<int, 2>{});
  else if ((int64_t)blocks(kPixTile) * cot >= 1024)
    pick_nt(std::integral_constant<int, 1>{});
  else
    hipLaunchKernelGGL(conv3x3_kgroups_kernel, dim3(blocks(64), cot), dim3(1024), 0, s, x, batch,
                       h, w, wb, bias, cout, act, slope, dst, y_fp32);
}

bool cat_ok(const void *a, int32_t ca, int32_t up, const void *b, int32_t cb, int32_t h,
            int32_t w) {
  return a && b && ca > 0 && ca % 16 == 0 && cb > 0 && cb % 16 == 0 && (up == 0 || up == 1) &&
         (!up || (h % 2 == 0 && w % 2 == 0)) && aligned16(a) && aligned16(b);
}

// LDS bytes of wgrad_rows_kernel<OB, CB> for bands of r rows of width w.
size_t wgrad_rows_lds(int ob, int cb, int r, int w) {
  return sizeof(bf16) * ((size_t)16 * ob * kDyPitch + (size_t)16 * cb * (r + 2) * (w + 16));
}

// Rows per band of the row-band weight gradient, or 0 where it does not
// apply: the width must be a multiple of 8 and at most kRowPix, the bands
// (as tall as kRowPix pixels and 64 KB of LDS allow) must tile the image
// height, and a band must hold whole 32-pixel steps.
int wgrad_rows(int32_t h, int32_t w, int ob, int cb) {
  if (w % 8 || w > kRowPix) return 0;
  // 512-pixel bands for wide images (fewer halo rows), 256 below (more bands)
  int r = std::min<int>(h, (w >= 128 ? kRowPix : kRowPix / 2) / w);
  while (r > 1 && wgrad_rows_lds(ob, cb, r, w) > 65536) r /= 2;
  return (wgrad_rows_lds(ob, cb, r, w) <= 65536 && h % r == 0 && (r * w) % 32 == 0) ? r : 0;
}

// Output x input channel blocks (of 16) of a row-band weight-gradient workgroup.
void wgrad_rows_blocks(int cin, int cout, int *ob, int *cb) {
  *ob = cout % 32 == 0 ? 2 : 1;
  *cb = (*ob == 1 && cin % 32 == 0) ? 2 : 1;
}

template <int OB, int CB>
void wgrad_rows_launch(const bf16 *dyb, const ConvSrc &x, int32_t batch, int32_t h, int32_t w,
                       int32_t cout, int r, int bpc, int nsplit, float *part, float *partb,
                       hipStream_t s) {
  const int cin = x.ca + x.cb;
  const size_t lds = wgrad_rows_lds(OB, CB, r, w);
  const dim3 grid((unsigned)(cout / (16 * OB)), (unsigned)(cin / (16 * CB)), (unsigned)nsplit);
  hipLaunchKernelGGL((wgrad_rows_kernel<OB, CB>), grid, dim3(256), lds, s, dyb, x, batch, h, w,
                     cout, r, bpc, part, partb);
}

// Launch of the weight-gradient partial sums: nsplit chunks of cout x 9 cin
// weight sums at part, then (dbias requested) nsplit chunks of cout bias sums
// right after them.  Returns nsplit, at most the chunk count that
// clb_nn_wgrad_workspace_bytes provides for.
int wgrad_parts_launch(const bf16 *dyb, const ConvSrc &x, int32_t batch, int32_t h, int32_t w,
                       int32_t cout, bool with_bias, float *part, hipStream_t s) {
  const int cin = x.ca + x.cb;
  int nsplit, chunk;
  const int64_t K = 9LL * cin, M = (int64_t)batch * h * w;
  wgrad_plan(M, wgrad_tiles(cin, cout), &nsplit, &chunk);
  int rob, rcb;
  wgrad_rows_blocks(cin, cout, &rob, &rcb);
  const int r = wgrad_rows(h, w, rob, rcb);
  int bpc = 0;
  if (r) {  // bands of rows: chunks of whole bands, about 768 workgroups (the
            // workgroup tiles are larger than wgrad_kernel's, so fewer chunks,
            // and fewer partial sums to add, fill the GPU)
    const int nbands = batch * (h / r);
    const int tiles = (cout / (16 * rob)) * (cin / (16 * rcb));
    const int cap = std::min(std::min(nbands, nsplit), std::max(1, (768 + tiles - 1) / tiles));
    bpc = (nbands + cap - 1) / cap;
    nsplit = (nbands + bpc - 1) / bpc;
  }
  float *partb = with_bias ? part + (size_t)nsplit * cout * K : nullptr;
  if (r) {
    if (rob == 2)
      wgrad_rows_launch<2, 1>(dyb, x, batch, h, w, cout, r, bpc, nsplit, part, partb, s);
    else if (rcb == 2)
      wgrad_rows_launch<1, 2>(dyb, x, batch, h, w, cout, r, bpc, nsplit, part, partb, s);
    else
      wgrad_rows_launch<1, 1>(dyb, x, batch, h, w, cout, r, bpc, nsplit, part, partb, s);
    return nsplit;
  }
  const int ob = wgrad_ob(cout);
  const dim3 grid((unsigned)(cout / (16 * ob)), (unsigned)((K + kWgK - 1) / kWgK), nsplit);
  if (ob == 4)
    hipLaunchKernelGGL(wgrad_kernel<4>, grid, dim3(256), 0, s, dyb, x, batch, h, w, cout, chunk,
                       part, partb);
  else if (ob == 2)
    hipLaunchKernelGGL(wgrad_kernel<2>, grid, dim3(256), 0, s, dyb, x, batch, h, w, cout, chunk,
                       part, partb);
  else
    hipLaunchKernelGGL(wgrad_kernel<1>, grid, dim3(256), 0, s, dyb, x, batch, h, w, cout, chunk,
                       part, partb);
  return nsplit;
}

void wgrad_launch(const bf16 *dyb, const ConvSrc &x, int32_t batch, int32_t h, int32_t w,
                  int32_t cout, float *dweight, float *dbias, void *workspace, hipStream_t s) {
  float *part = static_cast<float *>(workspace);
  const int nsplit = wgrad_parts_launch(dyb, x, batch, h, w, cout, dbias != nullptr, part, s);
  const size_t n = (size_t)cout * 9 * (x.ca + x.cb), nb = dbias ? (size_t)cout : 0;
  const size_t per = sum_outputs_per_block(nsplit);
  hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((n + nb + per - 1) / per)), dim3(256), 0,
                     s, part, nsplit, n, dweight, part + (size_t)nsplit * n, nb, dbias);
}

// The layer table of sum_parts_layers_kernel: layer l adds nsplit[l] chunks
// of n[l] weight and nb[l] bias partial sums at part[l] into w[l] and b[l];
// its workgroups are [block0[l], block0[l + 1]).
struct PartLayers {
  int n_layers;
  const float *part[CLB_NN_MAX_LAYERS];
  float *w[CLB_NN_MAX_LAYERS];
  float *b[CLB_NN_MAX_LAYERS];
  int nsplit[CLB_NN_MAX_LAYERS], n[CLB_NN_MAX_LAYERS], nb[CLB_NN_MAX_LAYERS];
  int block0[CLB_NN_MAX_LAYERS + 1];
};

// sum_parts_kernel for many layers in one launch (same order of additions).
__global__ void __launch_bounds__(256) sum_parts_layers_kernel(PartLayers L) {
  int l = 0;
  while (l + 1 < L.n_layers && (int)blockIdx.x >= L.block0[l + 1]) ++l;
  const size_t n = L.n[l], nb = L.nb[l];
  const float *part = L.part[l], *partb = L.part[l] + (size_t)L.nsplit[l] * n;
  float *w = L.w[l], *b = L.b[l];
  sum_chunks(
      L.nsplit[l], blockIdx.x - L.block0[l], n + nb,
      [&](size_t i, int z) { return i < n ? part[(size_t)z * n + i] : partb[(size_t)z * nb + i - n]; },
      [&](size_t i, float v) {
        if (i < n)
          w[i] = v;
        else
          b[i - n] = v;
      });
}

}  // namespace

extern "C" clb_status clb_nn_conv3x3(const clb_bf16 *x, int32_t batch, int32_t h, int32_t w,
                                     int32_t cin, const clb_bf16 *weight, const float *bias,
                                     int32_t cout, int32_t act, float slope, void *y,
                                     int32_t y_fp32, void *stream) {
  if (!x || !weight || !y || !dims_ok(batch, h, w) || cin <= 0 || cin % 16 || cout <= 0 ||
      cout % 16 || (act != 0 && act != 1) || !aligned16(x) || !aligned16(weight))
    return CLB_ERR_ARG;
  const ConvSrc src{reinterpret_cast<const bf16 *>(x), nullptr, cin, 0, 0};
  const ConvDst dst{y, nullptr, cout};
  conv_launch(src, batch, h, w, reinterpret_cast<const bf16 *>(weight), bias, cout, act, slope,
              dst, y_fp32, static_cast<hipStream_t>(stream));
  return launched();
}

extern "C" clb_status clb_nn_conv3x3_cat(const clb_bf16 *a, int32_t ca, int32_t up_a,
                                         const clb_bf16 *b, int32_t cb, int32_t batch, int32_t h,
                                         int32_t w, const clb_bf16 *weight, const float *bias,
                                         int32_t cout, int32_t act, float slope, void *y,
                                         int32_t y_fp32, void *stream) {
  if (!cat_ok(a, ca, up_a, b, cb, h, w) || !weight || !y || !dims_ok(batch, h, w) || cout <= 0 ||
      cout % 16 || (act != 0 && act != 1) || !aligned16(weight))
    return CLB_ERR_ARG;
  const ConvSrc src{reinterpret_cast<const bf16 *>(a), reinterpret_cast<const bf16 *>(b), ca, cb,
                    up_a};
  const ConvDst dst{y, nullptr, cout};
  conv_launch(src, batch, h, w, reinterpret_cast<const bf16 *>(weight), bias, cout, act, slope,
              dst, y_fp32, static_cast<hipStream_t>(stream));
  return launched();
}

extern "C" clb_status clb_nn_conv3x3_split(const clb_bf16 *x, int32_t batch, int32_t h,
                                           int32_t w, int32_t cin, const clb_bf16 *weight,
                                           int32_t cout, int32_t split, clb_bf16 *y0,
                                           clb_bf16 *y1, void *stream) {
  if (!x || !weight || !y0 || !y1 || !dims_ok(batch, h, w) || cin <= 0 || cin % 16 ||
      cout <= 0 || cout % 16 || split <= 0 || split >= cout || split % 16 || !aligned16(x) ||
      !aligned16(weight))
    return CLB_ERR_ARG;
  const ConvSrc src{reinterpret_cast<const bf16 *>(x), nullptr, cin, 0, 0};
  const ConvDst dst{y0, y1, split};
  conv_launch(src, batch, h, w, reinterpret_cast<const bf16 *>(weight), nullptr, cout, 0, 0.0f,
              dst, 0, static_cast<hipStream_t>(stream));
  return launched();
}

extern "C" clb_status clb_nn_conv3x3_act_grad(const clb_bf16 *dy, int32_t batch, int32_t h,
                                              int32_t w, int32_t cin, const clb_bf16 *weight,
                                              int32_t cout, const clb_bf16 *y, float slope,
                                              clb_bf16 *dz, void *stream) {
  if (!dy || !weight || !y || !dz || !dims_ok(batch, h, w) || cin <= 0 || cin % 16 ||
      cout <= 0 || cout % 16 || !aligned16(dy) || !aligned16(weight))
    return CLB_ERR_ARG;
  const ConvSrc src{reinterpret_cast<const bf16 *>(dy), nullptr, cin, 0, 0};
  ConvDst dst{dz, nullptr, cout};
  dst.act_y = reinterpret_cast<const bf16 *>(y);
  dst.act_slope = slope;
  conv_launch(src, batch, h, w, reinterpret_cast<const bf16 *>(weight), nullptr, cout, 0, 0.0f,
              dst, 0, static_cast<hipStream_t>(stream));
  return launched();
}

extern "C" clb_status clb_nn_wgrad_workspace_bytes(int32_t batch, int32_t h, int32_t w,
                                                   int32_t cin, int32_t cout, size_t *bytes) {
  if (!bytes || !dims_ok(batch, h, w) || cin <= 0 || cin % 16 || cout <= 0 || cout % 16)
    return CLB_ERR_ARG;
  int nsplit, chunk;
  const int64_t K = 9LL * cin;
  wgrad_plan((int64_t)batch * h * w, wgrad_tiles(cin, cout), &nsplit, &chunk);
  *bytes = sizeof(float) * (size_t)nsplit * (cout * K + cout);
  return CLB_OK;
}

extern "C" clb_status clb_nn_conv3x3_wgrad(const clb_bf16 *dy, const clb_bf16 *x, int32_t batch,
                                           int32_t h, int32_t w, int32_t cin, int32_t cout,
                                           float *dweight, float *dbias, void *workspace,
                                           size_t bytes, void *stream) {
  size_t need = 0;
  if (clb_nn_wgrad_workspace_bytes(batch, h, w, cin, cout, &need) != CLB_OK || !dy || !x ||
      !dweight || !workspace || bytes < need || !aligned16(dy) || !aligned16(x))
    return CLB_ERR_ARG;
  const ConvSrc src{reinterpret_cast<const bf16 *>(x), nullptr, cin, 0, 0};
  wgrad_launch(reinterpret_cast<const bf16 *>(dy), src, batch, h, w, cout, dweight, dbias,
               workspace, static_cast<hipStream_t>(stream));
  return launched();
}

extern "C" clb_status clb_nn_conv3x3_wgrad_cat(const clb_bf16 *dy, const clb_bf16 *a, int32_t ca,
                                               int32_t up_a, const clb_bf16 *b, int32_t cb,
                                               int32_t batch, int32_t h, int32_t w, int32_t cout,
                                               float *dweight, float *dbias, void *workspace,
                                               size_t bytes, void *stream) {
  size_t need = 0;
  if (!cat_ok(a, ca, up_a, b, cb, h, w) ||
      clb_nn_wgrad_workspace_bytes(batch, h, w, ca + cb, cout, &need) != CLB_OK || !dy ||
      !dweight || !workspace || bytes < need || !aligned16(dy))
    return CLB_ERR_ARG;
  const ConvSrc src{reinterpret_cast<const bf16 *>(a), reinterpret_cast<const bf16 *>(b), ca, cb,
                    up_a};
  wgrad_launch(reinterpret_cast<const bf16 *>(dy), src, batch, h, w, cout, dweight, dbias,
               workspace, static_cast<hipStream_t>(stream));
  return launched();
}

extern "C" clb_status clb_nn_conv3x3_wgrad_parts(const clb_bf16 *dy, const clb_bf16 *x,
                                                 int32_t batch, int32_t h, int32_t w, int32_t cin,
                                                 int32_t cout, int32_t with_bias, void *workspace,
                                                 size_t bytes, int32_t *nsplit, void *stream) {
  size_t need = 0;
  if (clb_nn_wgrad_workspace_bytes(batch, h, w, cin, cout, &need) != CLB_OK || !dy || !x ||
      !workspace || !nsplit || bytes < need || !aligned16(dy) || !aligned16(x) ||
      !aligned16(workspace))
    return CLB_ERR_ARG;
  const ConvSrc src{reinterpret_cast<const bf16 *>(x), nullptr, cin, 0, 0};
  *nsplit = wgrad_parts_launch(reinterpret_cast<const bf16 *>(dy), src, batch, h, w, cout,
                               with_bias != 0, static_cast<float *>(workspace),
                               static_cast<hipStream_t>(stream));
  return launched();
}

extern "C" clb_status clb_nn_conv3x3_wgrad_cat_parts(const clb_bf16 *dy, const clb_bf16 *a,
                                                     int32_t ca, int32_t up_a, const clb_bf16 *b,
                                                     int32_t cb, int32_t batch, int32_t h,
                                                     int32_t w, int32_t cout, int32_t with_bias,
                                                     void *workspace, size_t bytes,
                                                     int32_t *nsplit, void *stream) {
  size_t need = 0;
  if (!cat_ok(a, ca, up_a, b, cb, h, w) ||
      clb_nn_wgrad_workspace_bytes(batch, h, w, ca + cb, cout, &need) != CLB_OK || !dy ||
      !workspace || !nsplit || bytes < need || !aligned16(dy) || !aligned16(workspace))
    return CLB_ERR_ARG;
  const ConvSrc src{reinterpret_cast<const bf16 *>(a), reinterpret_cast<const bf16 *>(b), ca, cb,
                    up_a};
  *nsplit = wgrad_parts_launch(reinterpret_cast<const bf16 *>(dy), src, batch, h, w, cout,
                               with_bias != 0, static_cast<float *>(workspace),
                               static_cast<hipStream_t>(stream));
  return launched();
}

extern "C" clb_status clb_nn_wgrad_reduce_layers(int32_t nlayers, void *const *parts,
                                                 const int32_t *nsplit, const int32_t *cout,
                                                 const int32_t *cin, float *const *dweight,
                                                 float *const *dbias, void *stream) {
  if (nlayers < 1 || nlayers > CLB_NN_MAX_LAYERS || !parts || !nsplit || !cout || !cin ||
      !dweight || !dbias)
    return CLB_ERR_ARG;
  PartLayers L{};
  L.n_layers = nlayers;
  int64_t blocks = 0;
  for (int l = 0; l < nlayers; ++l) {
    const int64_t n = (int64_t)cout[l] * 9 * cin[l];
    if (!parts[l] || !dweight[l] || nsplit[l] < 1 || cout[l] <= 0 || cin[l] <= 0 ||
        n + cout[l] >= (1LL << 31))
      return CLB_ERR_ARG;
    L.part[l] = static_cast<const float *>(parts[l]);
    L.w[l] = dweight[l];
    L.b[l] = dbias[l];
    L.nsplit[l] = nsplit[l];
    L.n[l] = (int)n;
    L.nb[l] = dbias[l] ? cout[l] : 0;
    L.block0[l] = (int)blocks;
    const int per = sum_outputs_per_block(nsplit[l]);
    blocks += (n + L.nb[l] + per - 1) / per;
    if (blocks >= (1LL << 31)) return CLB_ERR_ARG;
  }
  L.block0[nlayers] = (int)blocks;
  hipLaunchKernelGGL(sum_parts_layers_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), L);
  return launched();
}

// ----------------------------------------------- weight gradient, no allocation

// Scratch of clb_nn_conv3x3_wgrad_static: the per-chunk partial sums that
// clb_nn_conv3x3_wgrad keeps in its caller's workspace.  Each GPU the library
// runs on holds one copy (32 MiB) until the process ends.  Host code never
// passes this name to a kernel: its device address is looked up per device.
constexpr size_t kWgradScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) float scratch[kWgradScratchBytes / sizeof(float)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
clb_status scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CLB_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CLB_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CLB_OK;
}
}  // namespace

extern "C" size_t clb_nn_wgrad_static_max_bytes(void) { return kWgradScratchBytes; }

extern "C" clb_status clb_nn_conv3x3_wgrad_static(const clb_bf16 *dy, const clb_bf16 *x,
                                                  int32_t batch, int32_t h, int32_t w,
                                                  int32_t cin, int32_t cout, float *dweight,
                                                  float *dbias, void *stream) {
  size_t need = 0;
  if (clb_nn_wgrad_workspace_bytes(batch, h, w, cin, cout, &need) != CLB_OK || !dy || !x ||
      !dweight || !aligned16(dy) || !aligned16(x))
    return CLB_ERR_ARG;
  if (need > kWgradScratchBytes) return CLB_ERR_WORKSPACE;
  void *ws = nullptr;
  const clb_status st = scratch_address(&ws);
  if (st != CLB_OK) return st;
  // the same kernels as clb_nn_conv3x3_wgrad; every partial sum they read is
  // written first by the same call, so nothing needs clearing
  return clb_nn_conv3x3_wgrad(dy, x, batch, h, w, cin, cout, dweight, dbias, ws, need, stream);
}

extern "C" clb_status clb_nn_weights_bf16(const float *w32, int32_t cout, int32_t cin,
                                          clb_bf16 *w_fwd, clb_bf16 *w_bwd, void *stream) {
  if (!w32 || !w_fwd || !w_bwd || cout <= 0 || cin <= 0) return CLB_ERR_ARG;
  const size_t n = (size_t)cout * 9 * cin;
  hipLaunchKernelGGL(weights_kernel, dim3(blocks_for(n)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), w32, cout, cin,
                     reinterpret_cast<bf16 *>(w_fwd), reinterpret_cast<bf16 *>(w_bwd));
  return launched();
}

extern "C" clb_status clb_nn_weights_bf16_layers(const float *w32, int32_t nlayers,
                                                 const int32_t *cout, const int32_t *cin,
                                                 const int64_t *offset, clb_bf16 *w_fwd,
                                                 clb_bf16 *w_bwd, void *stream) {
  if (!w32 || !w_fwd || !w_bwd || !cout || !cin || !offset || nlayers < 1 ||
      nlayers > CLB_NN_MAX_LAYERS)
    return CLB_ERR_ARG;
  WeightLayers L{};
  L.n = nlayers;
  int64_t blocks = 0;
  for (int l = 0; l < nlayers; ++l) {
    if (cout[l] <= 0 || cin[l] <= 0 || offset[l] < 0 ||
        (int64_t)cout[l] * 9 * cin[l] >= (1LL << 31))
      return CLB_ERR_ARG;
    L.cout[l] = cout[l];
    L.cin[l] = cin[l];
    L.offset[l] = offset[l];
    L.block0[l] = (int)blocks;
    blocks += ((int64_t)cout[l] * 9 * cin[l] + 255) / 256;
    if (blocks >= (1LL << 31)) return CLB_ERR_ARG;
  }
  L.block0[nlayers] = (int)blocks;
  hipLaunchKernelGGL(weights_layers_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), w32, L, reinterpret_cast<bf16 *>(w_fwd),
                     reinterpret_cast<bf16 *>(w_bwd));
  return launched();
}

extern "C" clb_status clb_nn_pool2(const clb_bf16 *x, int32_t batch, int32_t h, int32_t w,
                                   int32_t c, clb_bf16 *y, void *stream) {
  if (!x || !y || !dims_ok(batch, h, w) || h % 2 || w % 2 || c <= 0) return CLB_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c % 8 == 0 && aligned16(x) && aligned16(y) && (int64_t)(w / 2) * (c / 8) < (1 << 30) &&
      (int64_t)batch * (h / 2) < 65536) {
    const int C8 = c / 8;
    hipLaunchKernelGGL(pool2_v8_kernel, dim3(blocks_for((size_t)(w / 2) * C8), batch * (h / 2)),
                       dim3(256), 0, s, reinterpret_cast<const bf16x8 *>(x), h, w, C8,
                       reinterpret_cast<bf16x8 *>(y));
    return launched();
  }
  const size_t n = (size_t)batch * (h / 2) * (w / 2) * c;
  hipLaunchKernelGGL(pool2_kernel, dim3(blocks_for(n)), dim3(256), 0, s,
                     reinterpret_cast<const bf16 *>(x), batch, h, w, c, reinterpret_cast<bf16 *>(y));
  return launched();
}

extern "C" clb_status clb_nn_pool2_grad(const clb_bf16 *dy, int32_t batch, int32_t h, int32_t w,
                                        int32_t c, clb_bf16 *dx, void *stream) {
  if (!dy || !dx || !dims_ok(batch, h, w) || h % 2 || w % 2 || c <= 0) return CLB_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c % 8 == 0 && aligned16(dy) && aligned16(dx) && (int64_t)w * (c / 8) < (1 << 30) &&
      (int64_t)batch * h < 65536) {
    const int C8 = c / 8;
    hipLaunchKernelGGL(pool2_grad_v8_kernel, dim3(blocks_for((size_t)w * C8), batch * h),
                       dim3(256), 0, s, reinterpret_cast<const bf16x8 *>(dy), h, w, C8,
                       reinterpret_cast<bf16x8 *>(dx), nullptr, nullptr, 0.0f);
    return launched();
  }
  const size_t n = (size_t)batch * h * w * c;
  hipLaunchKernelGGL(pool2_grad_kernel, dim3(blocks_for(n)), dim3(256), 0, s,
                     reinterpret_cast<const bf16 *>(dy), batch, h, w, c,
                     reinterpret_cast<bf16 *>(dx));
  return launched();
}

extern "C" clb_status clb_nn_up2(const clb_bf16 *x, int32_t batch, int32_t h, int32_t w,
                                 int32_t c, clb_bf16 *y, void *stream) {
  if (!x || !y || !dims_ok(batch, 2 * h, 2 * w) || c <= 0) return CLB_ERR_ARG;
  const size_t n = (size_t)batch * 4 * h * w * c;
  hipLaunchKernelGGL(up2_kernel, dim3(blocks_for(n)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), reinterpret_cast<const bf16 *>(x), batch,
                     h, w, c, reinterpret_cast<bf16 *>(y));
  return launched();
}

extern "C" clb_status clb_nn_pool2_grad_act(const clb_bf16 *dy, int32_t batch, int32_t h,
                                            int32_t w, int32_t c, const clb_bf16 *add,
                                            const clb_bf16 *y, float slope, clb_bf16 *dz,
                                            void *stream) {
  if (!dy || !y || !dz || !dims_ok(batch, h, w) || h % 2 || w % 2 || c <= 0 || c % 8 ||
      !aligned16(dy) || !aligned16(y) || !aligned16(dz) || (add && !aligned16(add)) ||
      (int64_t)w * (c / 8) >= (1 << 30) || (int64_t)batch * h >= 65536)
    return CLB_ERR_ARG;
  const int C8 = c / 8;
  hipLaunchKernelGGL(pool2_grad_v8_kernel, dim3(blocks_for((size_t)w * C8), batch * h),
                     dim3(256), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const bf16x8 *>(dy), h, w, C8, reinterpret_cast<bf16x8 *>(dz),
                     reinterpret_cast<const bf16x8 *>(add), reinterpret_cast<const bf16x8 *>(y),
                     slope);
  return launched();
}

extern "C" clb_status clb_nn_up2_grad_act(const clb_bf16 *dy, int32_t batch, int32_t h, int32_t w,
                                          int32_t c, const clb_bf16 *y, float slope, clb_bf16 *dz,
                                          void *stream) {
  if (!dy || !y || !dz || !dims_ok(batch, 2 * h, 2 * w) || c <= 0 || c % 8 || !aligned16(dy) ||
      !aligned16(y) || !aligned16(dz) || (int64_t)w * (c / 8) >= (1 << 30) ||
      (int64_t)batch * h >= 65536)
    return CLB_ERR_ARG;
  const int C8 = c / 8;
  hipLaunchKernelGGL(up2_grad_v8_kernel, dim3(blocks_for((size_t)w * C8), batch * h), dim3(256),
                     0, static_cast<hipStream_t>(stream), reinterpret_cast<const bf16x8 *>(dy), h,
                     w, C8, reinterpret_cast<bf16x8 *>(dz), reinterpret_cast<const bf16x8 *>(y),
                     slope);
  return launched();
}

extern "C" clb_status clb_nn_up2_grad(const clb_bf16 *dy, int32_t batch, int32_t h, int32_t w,
                                      int32_t c, clb_bf16 *dx, void *stream) {
  if (!dy || !dx || !dims_ok(batch, 2 * h, 2 * w) || c <= 0) return CLB_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c % 8 == 0 && aligned16(dy) && aligned16(dx) && (int64_t)w * (c / 8) < (1 << 30) &&
      (int64_t)batch * h < 65536) {
    const int C8 = c / 8;
    hipLaunchKernelGGL(up2_grad_v8_kernel, dim3(blocks_for((size_t)w * C8), batch * h), dim3(256),
                       0, s, reinterpret_cast<const bf16x8 *>(dy), h, w, C8,
                       reinterpret_cast<bf16x8 *>(dx), nullptr, 0.0f);
    return launched();
  }
  const size_t n = (size_t)batch * h * w * c;
  hipLaunchKernelGGL(up2_grad_kernel, dim3(blocks_for(n)), dim3(256), 0, s,
                     reinterpret_cast<const bf16 *>(dy), batch, h, w, c,
                     reinterpret_cast<bf16 *>(dx));
  return launched();
}

extern "C" clb_status clb_nn_concat(const clb_bf16 *a, int32_t ca, const clb_bf16 *b, int32_t cb,
                                    int64_t npix, clb_bf16 *y, void *stream) {
  if (!a || !b || !y || ca <= 0 || cb <= 0 || npix <= 0) return CLB_ERR_ARG;
  const size_t n = (size_t)npix * (ca + cb);
  hipLaunchKernelGGL(concat_kernel, dim3(blocks_for(n)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), reinterpret_cast<const bf16 *>(a), ca,
                     reinterpret_cast<const bf16 *>(b), cb, (size_t)npix,
                     reinterpret_cast<bf16 *>(y));
  return launched();
}

extern "C" clb_status clb_nn_split(const clb_bf16 *y, int32_t ca, int32_t cb, int64_t npix,
                                   clb_bf16 *a, clb_bf16 *b, void *stream) {
  if (!a || !b || !y || ca <= 0 || cb <= 0 || npix <= 0) return CLB_ERR_ARG;
  const size_t n = (size_t)npix * (ca + cb);
  hipLaunchKernelGGL(split_kernel, dim3(blocks_for(n)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), reinterpret_cast<const bf16 *>(y), ca, cb,
                     (size_t)npix, reinterpret_cast<bf16 *>(a), reinterpret_cast<bf16 *>(b));
  return launched();
}

extern "C" clb_status clb_nn_act_grad(const clb_bf16 *g0, const clb_bf16 *g1,
                                      const clb_bf16 *out, int64_t n, float slope, clb_bf16 *dz,
                                      void *stream) {
  if (!g0 || !out || !dz || n <= 0) return CLB_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n % 8 == 0 && aligned16(g0) && (!g1 || aligned16(g1)) && aligned16(out) && aligned16(dz)) {
    hipLaunchKernelGGL(act_grad_v8_kernel, dim3(blocks_for((size_t)n / 8)), dim3(256), 0, s,
                       reinterpret_cast<const bf16x8 *>(g0), reinterpret_cast<const bf16x8 *>(g1),
                       reinterpret_cast<const bf16x8 *>(out), (size_t)n / 8, slope,
                       reinterpret_cast<bf16x8 *>(dz));
    return launched();
  }
  hipLaunchKernelGGL(act_grad_kernel, dim3(blocks_for((size_t)n)), dim3(256), 0, s,
                     reinterpret_cast<const bf16 *>(g0), reinterpret_cast<const bf16 *>(g1),
                     reinterpret_cast<const bf16 *>(out), (size_t)n, slope,
                     reinterpret_cast<bf16 *>(dz));
  return launched();
}

extern "C" clb_status clb_nn_mse_workspace_bytes(int64_t npix, size_t *bytes) {
  if (!bytes || npix <= 0) return CLB_ERR_ARG;
  *bytes = sizeof(double) * kMseBlocks;
  return CLB_OK;
}

extern "C" clb_status clb_nn_mse(const float *out, int32_t ldo, const float *target, int32_t nch,
                                 int64_t npix, clb_bf16 *dout, double *d_loss, void *workspace,
                                 size_t bytes, void *stream) {
  if (!out || !target || !dout || !d_loss || !workspace || nch <= 0 || ldo < nch || npix <= 0 ||
      bytes < sizeof(double) * kMseBlocks)
    return CLB_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ldo % 8 || !aligned16(out) || !aligned16(dout)) return CLB_ERR_ARG;
  const unsigned nb = (unsigned)std::min<size_t>(kMseBlocks, blocks_for((size_t)npix * (ldo / 8)));
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, s, out, ldo, target, nch, (size_t)npix,
                     reinterpret_cast<bf16 *>(dout), static_cast<double *>(workspace));
  hipLaunchKernelGGL(mse_finalize_kernel, dim3(1), dim3(256), 0, s,
                     static_cast<const double *>(workspace), (int)nb, (double)npix * nch, d_loss);
  return launched();
}

extern "C" clb_status clb_nn_adamw(float *p, const float *g, float *m, float *v, int64_t n,
                                   float lr, float b1, float b2, float eps, float wd, int32_t t,
                                   void *stream) {
  if (!p || !g || !m || !v || n <= 0 || t < 1) return CLB_ERR_ARG;
  const float c1 = (float)(1.0 - std::pow((double)b1, t));
  const float c2 = (float)(1.0 - std::pow((double)b2, t));
  hipLaunchKernelGGL(adamw_kernel, dim3(blocks_for((size_t)n)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), p, g, m, v, (size_t)n, lr, b1, b2, eps, wd,
                     c1, c2);
  return launched();
}

extern "C" clb_status clb_nn_adamw_layers(float *p, const float *g, float *m, float *v,
                                          int64_t n, float lr, float b1, float b2, float eps,
                                          float wd, int32_t t, int32_t nlayers,
                                          const int32_t *cout, const int32_t *cin,
                                          const int64_t *offset, clb_bf16 *w_fwd,
                                          clb_bf16 *w_bwd, void *stream) {
  if (!p || !g || !m || !v || n <= 0 || t < 1 || !w_fwd || !w_bwd || !cout || !cin || !offset ||
      nlayers < 1 || nlayers > CLB_NN_MAX_LAYERS)
    return CLB_ERR_ARG;
  WeightLayers L{};
  L.n = nlayers;
  for (int l = 0; l < nlayers; ++l) {
    if (cout[l] <= 0 || cin[l] <= 0 || offset[l] < 0 || (l && offset[l] <= offset[l - 1]) ||
        offset[l] + (int64_t)cout[l] * 9 * cin[l] > n)
      return CLB_ERR_ARG;
    L.cout[l] = cout[l];
    L.cin[l] = cin[l];
    L.offset[l] = offset[l];
  }
  const float c1 = (float)(1.0 - std::pow((double)b1, t));
  const float c2 = (float)(1.0 - std::pow((double)b2, t));
  hipLaunchKernelGGL(adamw_layers_kernel, dim3(blocks_for((size_t)n)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), p, g, m, v, (size_t)n, lr, b1, b2, eps, wd,
                     c1, c2, L, reinterpret_cast<bf16 *>(w_fwd), reinterpret_cast<bf16 *>(w_bwd));
  return launched();
}

extern "C" clb_status clb_nn_features(const float *eps_all, const float *groups_all,
                                      int32_t ngroups, const int32_t *idx, int32_t batch,
                                      int32_t h, int32_t w, clb_bf16 *x, void *stream) {
  if (!eps_all || !idx || !x || ngroups < 0 || ngroups > 13 || (ngroups && !groups_all) ||
      !dims_ok(batch, h, w))
    return CLB_ERR_ARG;
  const size_t n = (size_t)batch * h * w * 16;
  hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), eps_all, groups_all, ngroups, idx, batch,
                     h, w, reinterpret_cast<bf16 *>(x));
  return launched();
}

extern "C" clb_status clb_nn_gather(const float *fields_all, int32_t nch, const int32_t *idx,
                                    int32_t batch, int64_t npix, float *out, void *stream) {
  if (!fields_all || !idx || !out || nch <= 0 || batch <= 0 || npix <= 0) return CLB_ERR_ARG;
  const size_t n = (size_t)batch * npix * nch;
  hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(n)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), fields_all, nch, idx, batch, (size_t)npix,
                     out);
  return launched();
}
