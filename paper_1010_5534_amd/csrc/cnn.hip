// Depth-proposal network on gfx950: 3x3 convolutions as implicit GEMMs on
// the bf16 matrix cores (v_mfma_f32_16x16x32_bf16, float32 accumulation),
// its backward pass, the weighted cross-entropy and Adam.
//
// Tensors are NHWC: pixel p = (map * h + y) * w + x, channels contiguous.
// Activations and back-propagated gradients are bf16 (round to nearest
// even), logits float32.  A convolution
//   y[p, o] = bias[o] + sum_{ky, kx, c} x[p shifted by (ky-1, kx-1), c] W[o, ky, kx, c]
// is the product D = A B with A = W as a [rows][K] matrix (K = 9 taps x
// stored input channels, padded to 32) and B[k][p] = the shifted input; a
// block stages a 16 x 16 pixel tile of the input with its halo in LDS and
// its waves compute 16-pixel column blocks for every output row, holding all
// of A in registers, each lane reading its pixel's 8 consecutive channels
// of one tap with a single 16-byte LDS load.  The input
// gradient is the same product with the flipped, transposed weights; the
// weight gradient stages 8 x 8 pixel tiles of both operands transposed in
// LDS (the input once per tile, with its halo) and reduces over pixels into
// per-block partials that one more kernel sums in a fixed order.
#include <algorithm>
#include <cmath>

#include "cnn.h"

namespace air {
namespace cnn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;
constexpr uint16_t BF16_ONE = 0x3f80;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);                     // nearest, ties to even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ bool bf_pos(uint16_t h) { return !(h & 0x8000u) && (h & 0x7fffu); }

__device__ __forceinline__ f32x4 mfma(const u16x8& a, const u16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// stored channels of each layer's input and output, and the rows of its
// forward matrix
constexpr int CS_IN[LAYERS] = {XC, HID, HID, HID};
constexpr int CS_OUT[LAYERS] = {HID, HID, HID, ZC};
constexpr int ROWS[LAYERS] = {HID, HID, HID, 16};

struct Prep {
  const float* theta;
  uint16_t* wf[LAYERS];
  uint16_t* wt[LAYERS];
  int woff[LAYERS];
};

// bf16 operand matrices from the float32 parameters
__global__ __launch_bounds__(256) void k_prep(Prep P) {
  const int l = blockIdx.y;
  const int cin = CIN[l], cout = COUT[l], csi = CS_IN[l], cso = CS_OUT[l];
  const float* w = P.theta + P.woff[l];
  // forward: wf[r][k], k = tap * csi + c
  const int kpf = KPAD(csi), nf = ROWS[l] * kpf;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += gridDim.x * blockDim.x) {
    const int r = e / kpf, k = e % kpf, tap = k / csi, c = k % csi;
    float val = 0.0f;
    if (r < cout && k < 9 * csi && c < cin) val = w[(r * 9 + tap) * cin + c];
    P.wf[l][e] = f2bf(val);
  }
  if (l == 0) return;
  // input gradient: wt[c][k], k = tap' * cso + o, tap' = (2 - ky) * 3 + (2 - kx)
  const int kpt = KPAD(cso), nt = HID * kpt;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nt; e += gridDim.x * blockDim.x) {
    const int c = e / kpt, k = e % kpt, tp = k / cso, o = k % cso;
    float val = 0.0f;
    if (k < 9 * cso && o < cout && c < cin) {
      const int ky = 2 - tp / 3, kx = 2 - tp % 3;
      val = w[(o * 9 + ky * 3 + kx) * cin + c];
    }
    P.wt[l][e] = f2bf(val);
  }
}

struct Norm {
  float mean[FEAT], inv_std[FEAT];
};

// standardised bf16 input maps, channels 4..7 zero
__global__ __launch_bounds__(256) void k_input(const float* feat, int64_t P, Norm nm, uint16_t* x) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    u16x8 o = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < FEAT; ++c) o[c] = f2bf((feat[p * FEAT + c] - nm.mean[c]) * nm.inv_std[c]);
    *reinterpret_cast<u16x8*>(x + p * XC) = o;
  }
}

enum { MODE_HIDDEN = 0, MODE_LOGITS = 1, MODE_MASK = 2 };

// D[rows][pixels] = A[rows][K] B[K][pixels]; CS = stored input channels,
// CSO = stored output channels, NBIAS = real output channels (bias length).
// A block takes 16 x 16 output pixels of one map at a time: the input tile
// with its one-pixel halo (18 x 18 pixels) is staged in LDS once, so an
// input pixel leaves L2 about 1.27 times instead of once per tap, and the
// B operands are 16-byte LDS reads; each wave computes four of the tile's
// rows as 16-pixel column blocks with all of A in registers (loaded once per
// block through LDS).  Tiles are taken in a grid-stride loop, the next
// tile's input loaded while the current one is multiplied.
constexpr int CT = 16;         // output tile edge
constexpr int CTH = CT + 2;    // with the halo
constexpr int CONV_MAX_BLOCKS = 1024;
// bf16 per staged pixel: 32 channels padded to 40 spread a column block's
// 16-byte reads over the LDS banks
template <int CS>
constexpr int conv_px_stride() {
  return CS == 32 ? 40 : CS;
}

template <int CS, int RW, int CSO, int MODE>
__global__ __launch_bounds__(256) void k_conv(const uint16_t* __restrict__ wmat, const float* __restrict__ bias,
                                              int nbias, const uint16_t* __restrict__ x,
                                              const uint16_t* __restrict__ act, int n, int h, int w,
                                              void* __restrict__ out) {
  constexpr int K = 9 * CS, KP = (K + 31) / 32 * 32, KS = KP / 32, MB = RW / 16, PS = conv_px_stride<CS>();
  constexpr int OCT = CS / 8, ROWS_PER_WAVE = CT / 4;
  static_assert(CS % 8 == 0 && RW % 16 == 0, "operand shapes");
  __shared__ __attribute__((aligned(16))) uint16_t xt[CTH * CTH * PS];
  __shared__ __attribute__((aligned(16))) uint16_t at[RW * KP];
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE, g = lane >> 4, c16 = lane & 15;
  for (int e = threadIdx.x; e < RW * KP / 8; e += blockDim.x)
    *reinterpret_cast<u16x8*>(at + 8 * e) = *reinterpret_cast<const u16x8*>(wmat + 8 * e);
  __syncthreads();
  u16x8 a[MB][KS];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      a[mb][ks] = *reinterpret_cast<const u16x8*>(at + (mb * 16 + c16) * KP + ks * 32 + 8 * g);
  const int tx = (w + CT - 1) / CT, ty = (h + CT - 1) / CT, tiles = n * tx * ty;  // n h w < 2^25
  // the halo tile's 16-byte pieces, held in registers between their load
  // and their LDS store so that the next tile's loads fly during this
  // tile's products
  constexpr int HL = (CTH * CTH * OCT + 255) / 256;
  u16x8 hv[HL];
  auto load_halo = [&](int t) {
    const int b = t / (tx * ty), r = t - b * (tx * ty), y0 = (r / tx) * CT, x0 = (r % tx) * CT;
#pragma unroll
    for (int q = 0; q < HL; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int o = e % OCT, px = e / OCT, yy = y0 - 1 + px / CTH, xx = x0 - 1 + px % CTH;
      hv[q] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (e < CTH * CTH * OCT && (unsigned)yy < (unsigned)h && (unsigned)xx < (unsigned)w)
        hv[q] = *reinterpret_cast<const u16x8*>(x + ((b * h + yy) * w + xx) * CS + 8 * o);
    }
  };
  if (blockIdx.x < tiles) load_halo(blockIdx.x);
  for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int b = t / (tx * ty), r = t - b * (tx * ty), y0 = (r / tx) * CT, x0 = (r % tx) * CT;
    __syncthreads();  // the previous tile's reads of xt are done
#pragma unroll
    for (int q = 0; q < HL; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < CTH * CTH * OCT) *reinterpret_cast<u16x8*>(xt + (e / OCT) * PS + 8 * (e % OCT)) = hv[q];
    }
    __syncthreads();
    if (t + (int)gridDim.x < tiles) load_halo(t + gridDim.x);
#pragma unroll 1
    for (int rr = 0; rr < ROWS_PER_WAVE; ++rr) {
      const int row = wv * ROWS_PER_WAVE + rr, y = y0 + row, xq = x0 + c16;
      f32x4 acc[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k0 = ks * 32 + 8 * g;
        const int tap = k0 / CS, c0 = k0 % CS, dy = tap / 3, dx = tap % 3;
        u16x8 bv = {0, 0, 0, 0, 0, 0, 0, 0};
        if (k0 < K) bv = *reinterpret_cast<const u16x8*>(xt + ((row + dy) * CTH + c16 + dx) * PS + c0);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = mfma(a[mb][ks], bv, acc[mb]);
      }
      if (y >= h || xq >= w) continue;
      const int64_t p = ((int64_t)b * h + y) * w + xq;
      // lane holds rows mb*16 + 4g + i of pixel p
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int r0 = mb * 16 + 4 * g;
        if (r0 >= CSO) continue;
        if constexpr (MODE == MODE_LOGITS) {
          float4 o;
          o.x = acc[mb][0] + (r0 + 0 < nbias ? bias[r0 + 0] : 0.0f);
          o.y = acc[mb][1] + (r0 + 1 < nbias ? bias[r0 + 1] : 0.0f);
          o.z = acc[mb][2] + (r0 + 2 < nbias ? bias[r0 + 2] : 0.0f);
          o.w = acc[mb][3] + (r0 + 3 < nbias ? bias[r0 + 3] : 0.0f);
          *reinterpret_cast<float4*>(static_cast<float*>(out) + p * CSO + r0) = o;
        } else {
          u16x4 o;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float v = acc[mb][i];
            if constexpr (MODE == MODE_HIDDEN) {
              v = fmaxf(v + (r0 + i < nbias ? bias[r0 + i] : 0.0f), 0.0f);
            } else {
              v = bf_pos(act[p * CSO + r0 + i]) ? v : 0.0f;
            }
            o[i] = f2bf(v);
          }
          *reinterpret_cast<u16x4*>(static_cast<uint16_t*>(out) + p * CSO + r0) = o;
        }
      }
    }
  }
}

// weight gradient: G[o][n] = sum_p dy[p, o] X[p, n], n = tap * CS + c, plus
// the bias column n = 9 CS of ones.  CS = stored input channels, DC = stored
// dy channels, RW = padded rows.  The reduction runs over pixels, taken in
// 8 x 8 tiles of one map (64 pixels, two MFMA k-steps; pixel k of a tile is
// row k / 8, column k % 8).  dy of the tile is transposed into LDS; the
// input's 10 x 10 halo is transposed into LDS three times, shifted by the
// tap's column offset, so the B operand of tap (ky, kx) for a lane's 8
// pixels (one tile row) is one aligned 16-byte LDS read of copy kx at halo
// row row + ky.  A thread transposes an 8 x 8 block (8 pixels x 8
// channels) in registers and stores it as 8 rows of 16 bytes, so an input
// pixel is loaded at most three times (once per column offset) instead of
// nine, and no LDS store is narrower than 16 bytes.  The next tile's loads are issued
// before the current tile's products; each wave owns every fourth 16-column
// block of G with all row blocks.
constexpr int WG_BLOCKS = 512;
constexpr int WG_MAX_FLOATS = HID * ((9 * HID + 1 + 15) / 16 * 16);
constexpr int WG_T = 8;               // tile edge
constexpr int WG_H = WG_T + 2;        // halo edge
constexpr int WG_LD = WG_T * WG_T + 8;  // dy row stride in bf16 (144 bytes: conflict-free 16-byte reads)
constexpr int WG_HR = WG_H + 1;       // halo rows per channel, padded (176 bytes between channels)

template <int CS, int DC, int RW>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t* __restrict__ dy, const uint16_t* __restrict__ x,
                                               int n, int h, int w, float* __restrict__ partial) {
  constexpr int N = 9 * CS + 1, NBK = (N + 15) / 16, NP = NBK * 16, MB = RW / 16, NBPW = (NBK + 3) / 4;
  constexpr int DO = DC / 8, XO = CS / 8;
  // task e: one tile row of dy (8 pixels x 8 channels, e < DT), or one halo
  // row's 8 pixels starting at column kx (one copy) x 8 channels of the
  // input; its 8 x 8 block is transposed in registers and stored as 8 rows
  // of 16 bytes.  Neighbouring tasks take neighbouring rows, whose 16-byte
  // pieces sit 16 bytes apart in LDS (a channel octet's rows lie a multiple
  // of 128 bytes apart, so octet-major order would put a store's lanes on
  // the same banks)
  constexpr int DT = WG_T * DO, TT = DT + WG_H * XO * 3;
  static_assert(TT <= 256, "one task per thread");
  static_assert(DC % 8 == 0 && CS % 8 == 0 && DC <= RW && RW % 16 == 0, "operand shapes");
  __shared__ __attribute__((aligned(16))) uint16_t dT[RW * WG_LD];                // [o][pixel]
  __shared__ __attribute__((aligned(16))) uint16_t hT[3 * CS * WG_HR * WG_T];     // [kx][c][halo row][column]
  const int tid = threadIdx.x, wv = tid / WAVE, lane = tid & (WAVE - 1), g = lane >> 4, c16 = lane & 15;
  const int tx_n = (w + WG_T - 1) / WG_T, ty_n = (h + WG_T - 1) / WG_T, tiles = n * tx_n * ty_n;  // P < 2^25

  // dy rows no tile writes stay zero
  for (int e = tid; e < (RW - DC) * WG_LD; e += 256) dT[DC * WG_LD + e] = 0;
  u16x8 v[WG_T];
  auto load = [&](int t) {
    const int b = t / (tx_n * ty_n), r = t - b * (tx_n * ty_n), y0 = (r / tx_n) * WG_T, x0 = (r % tx_n) * WG_T;
    int yy, xs, stride, oct;
    const uint16_t* base;
    if (tid < DT) {
      oct = tid / WG_T;
      yy = y0 + tid % WG_T;
      xs = x0;
      base = dy;
      stride = DC;
    } else {
      const int f = tid - DT, rest = f / WG_H, kx = rest % 3;
      oct = rest / 3;
      yy = y0 - 1 + f % WG_H;
      xs = x0 - 1 + kx;
      base = x;
      stride = CS;
    }
    const bool row_ok = tid < TT && (unsigned)yy < (unsigned)h;
#pragma unroll
    for (int j = 0; j < WG_T; ++j) {
      v[j] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (row_ok && (unsigned)(xs + j) < (unsigned)w)
        v[j] = *reinterpret_cast<const u16x8*>(base + ((b * h + yy) * w + xs + j) * stride + 8 * oct);
    }
  };
  auto store = [&]() {
    if (tid >= TT) return;
    uint16_t* dst;
    int row_stride;
    if (tid < DT) {
      dst = dT + (8 * (tid / WG_T)) * WG_LD + (tid % WG_T) * WG_T;
      row_stride = WG_LD;
    } else {
      const int f = tid - DT, rest = f / WG_H, kx = rest % 3;
      dst = hT + ((kx * CS + 8 * (rest / 3)) * WG_HR + f % WG_H) * WG_T;
      row_stride = WG_HR * WG_T;
    }
    // transpose: row i (channel) holds the 8 pixels' channel i
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      uint4 q;
      q.x = (uint32_t)v[0][i] | ((uint32_t)v[1][i] << 16);
      q.y = (uint32_t)v[2][i] | ((uint32_t)v[3][i] << 16);
      q.z = (uint32_t)v[4][i] | ((uint32_t)v[5][i] << 16);
      q.w = (uint32_t)v[6][i] | ((uint32_t)v[7][i] << 16);
      *reinterpret_cast<uint4*>(dst + i * row_stride) = q;
    }
  };

  f32x4 acc[NBPW][MB];
#pragma unroll
  for (int t = 0; t < NBPW; ++t)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[t][mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  int t = blockIdx.x;  // the launch has at most `tiles` blocks
  load(t);
  for (; t < tiles; t += gridDim.x) {
    __syncthreads();  // the previous tile's products have read dT and hT
    store();
    __syncthreads();
    if (t + (int)gridDim.x < tiles) load(t + gridDim.x);
    u16x8 a[MB][2];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
        a[mb][kk] = *reinterpret_cast<const u16x8*>(&dT[(mb * 16 + c16) * WG_LD + kk * 32 + 8 * g]);
#pragma unroll
    for (int q = 0; q < NBPW; ++q) {
      const int nb = wv + 4 * q;
      if (nb >= NBK) break;  // uniform per wave
      const int col = nb * 16 + c16, tap = col / CS, c = col % CS, ky = tap / 3, kx = tap % 3;
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        u16x8 bv = {0, 0, 0, 0, 0, 0, 0, 0};
        if (col < 9 * CS)
          bv = *reinterpret_cast<const u16x8*>(&hT[((kx * CS + c) * WG_HR + 4 * kk + g + ky) * WG_T]);
        else if (col == 9 * CS)
          bv = u16x8{BF16_ONE, BF16_ONE, BF16_ONE, BF16_ONE, BF16_ONE, BF16_ONE, BF16_ONE, BF16_ONE};
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[q][mb] = mfma(a[mb][kk], bv, acc[q][mb]);
      }
    }
  }
  float* out = partial + (int64_t)blockIdx.x * RW * NP;
#pragma unroll
  for (int q = 0; q < NBPW; ++q) {
    const int nb = wv + 4 * q;
    if (nb >= NBK) break;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) out[(mb * 16 + 4 * g + i) * NP + nb * 16 + c16] = acc[q][mb][i];
  }
}

// sum the per-block partials into the flat gradient: 64 entries per block,
// each wave adds a contiguous quarter of the partial blocks in order and the
// quarters are added in wave order (a fixed order: the result is
// deterministic)
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ partial, int nblocks, int rw, int np,
                                                      int cs, int cin, int cout, float* gw, float* gb) {
  __shared__ float sh[4][WAVE];
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const int total = rw * np, e = blockIdx.x * WAVE + lane;
  float s = 0.0f;
  if (e < total) {
    const int per = (nblocks + 3) / 4, b0 = min(nblocks, wv * per), b1 = min(nblocks, b0 + per);
    int b = b0;
    for (; b + 8 <= b1; b += 8) {
      float t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = partial[(int64_t)(b + u) * total + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += t[u];
    }
    for (; b < b1; ++b) s += partial[(int64_t)b * total + e];
  }
  sh[wv][lane] = s;
  __syncthreads();
  if (wv != 0 || e >= total) return;
  s = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
  const int o = e / np, col = e % np;
  if (o >= cout || col > 9 * cs) return;
  if (col == 9 * cs)
    gb[o] = s;
  else if (col % cs < cin)
    gw[(o * 9 + col / cs) * cin + col % cs] = s;
}

struct ClassW {
  float w[CLASSES];
};
constexpr int LOSS_BLOCKS = 256;

__device__ __forceinline__ int label_at(const int32_t* labels, int64_t p) {
  return min(max((int)labels[p], 0), CLASSES - 1);
}

__device__ __forceinline__ double block_sum_f64(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// per block: sum of class weights and of weighted negative log-likelihoods
__global__ __launch_bounds__(256) void k_loss_partial(const float* z, const int32_t* labels, int64_t P, ClassW cw,
                                                      double* partial) {
  __shared__ double sh[256];
  double sw = 0.0, sl = 0.0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    const float* zp = z + p * ZC;
    const int t = label_at(labels, p);
    float m = zp[0];
    for (int c = 1; c < CLASSES; ++c) m = fmaxf(m, zp[c]);
    double se = 0.0;
    for (int c = 0; c < CLASSES; ++c) se += exp((double)zp[c] - (double)m);
    const double wt = cw.w[t];
    sw += wt;
    sl += wt * ((double)m + log(se) - (double)zp[t]);
  }
  sw = block_sum_f64(sw, sh);
  sl = block_sum_f64(sl, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sw;
    partial[2 * blockIdx.x + 1] = sl;
  }
}

__global__ __launch_bounds__(256) void k_loss_final(const double* partial, int nblocks, double* out) {
  __shared__ double sh[256];
  double sw = 0.0, sl = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) {
    sw += partial[2 * b];
    sl += partial[2 * b + 1];
  }
  sw = block_sum_f64(sw, sh);
  sl = block_sum_f64(sl, sh);
  if (threadIdx.x == 0) {
    out[0] = sw;
    out[1] = sw > 0.0 ? sl / sw : 0.0;
  }
}

// dz = (softmax(z) - onehot) w_t / sum w, bf16, channels 6 and 7 zero
__global__ __launch_bounds__(256) void k_dz(const float* z, const int32_t* labels, int64_t P, ClassW cw,
                                            const double* out, uint16_t* dz) {
  const double sw = out[0];
  const float inv = sw > 0.0 ? (float)(1.0 / sw) : 0.0f;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    const float* zp = z + p * ZC;
    const int t = label_at(labels, p);
    float m = zp[0];
    for (int c = 1; c < CLASSES; ++c) m = fmaxf(m, zp[c]);
    float e[CLASSES], se = 0.0f;
    for (int c = 0; c < CLASSES; ++c) {
      e[c] = expf(zp[c] - m);
      se += e[c];
    }
    const float scale = cw.w[t] * inv;
    u16x8 o = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < CLASSES; ++c) o[c] = f2bf((e[c] / se - (c == t ? 1.0f : 0.0f)) * scale);
    *reinterpret_cast<u16x8*>(dz + p * ZC) = o;
  }
}

__global__ __launch_bounds__(256) void k_adam(float* theta, float* m, float* v, const float* g, int P, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < P; k += gridDim.x * blockDim.x) {
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    theta[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
  }
}

int conv_blocks(int n, int h, int w) {
  const int64_t tiles = (int64_t)n * ((h + CT - 1) / CT) * ((w + CT - 1) / CT);
  return (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), CONV_MAX_BLOCKS);
}

// ---------------------------------------------------------------- inference
// All four layers for one IT x IT output tile of one map: the input rows of
// an (IT+8)^2 region (4-pixel halo) and each hidden layer's (IT+6)^2,
// (IT+4)^2, (IT+2)^2 region stay in LDS as bf16 NHWC; positions outside the
// image are zero, as the layer-by-layer kernels' zero padding.  Every output
// pixel sees the same MFMA sequence (same operands, same K order) as in
// k_conv, so the logits are bit-identical to the layer-by-layer path and do
// not depend on IT.  The last layer's logits go through LDS to the depth
// choice, one thread per pixel.  IT = 16 for large maps; 8 when the 16x16
// tiles would not give every compute unit a block (the four layers of a
// tile run one after another, so small tiles shorten the launch); 4 when
// even the 8x8 tiles would fill under a quarter of the compute units (one
// 32x32 map), though their halos are recomputed about 9 times.
template <int IT, int CS, int RW>
__device__ __forceinline__ void fused_layer(const uint16_t* __restrict__ wmat, const float* __restrict__ bias,
                                            int nbias, const uint16_t* in, int rin, uint16_t* out, float* zout,
                                            int y0, int x0, int h, int w) {
  constexpr int K = 9 * CS, KP = (K + 31) / 32 * 32, KS = KP / 32, MB = RW / 16;
  const int lane = threadIdx.x & (WAVE - 1), g = lane >> 4, c16 = lane & 15, wv = threadIdx.x / WAVE;
  const int rout = rin - 2, npx = rout * rout;
  u16x8 a[MB][KS];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      a[mb][ks] = *reinterpret_cast<const u16x8*>(wmat + (mb * 16 + c16) * KP + ks * 32 + 8 * g);
  for (int t = wv; t * 16 < npx; t += 4) {
    const int p = t * 16 + c16;
    const bool ok = p < npx;
    const int py = ok ? p / rout : 0, px = ok ? p % rout : 0;
    f32x4 acc[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k0 = ks * 32 + 8 * g;
      u16x8 bv = {0, 0, 0, 0, 0, 0, 0, 0};
      if (ok && k0 < K) {
        const int tap = k0 / CS, c0 = k0 % CS;
        bv = *reinterpret_cast<const u16x8*>(in + ((py + tap / 3) * rin + (px + tap % 3)) * CS + c0);
      }
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[mb] = mfma(a[mb][ks], bv, acc[mb]);
    }
    if (!ok) continue;
    // global position of this output pixel: region origin is tile origin
    // minus the remaining halo
    const int halo = (rout - IT) / 2;
    const int gy = y0 - halo + py, gx = x0 - halo + px;
    const bool inside = gy >= 0 && gy < h && gx >= 0 && gx < w;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int r0 = mb * 16 + 4 * g;
      if (zout) {  // logits (last layer): channels 0..7 of the 16 rows
        if (r0 < 8)
#pragma unroll
          for (int i = 0; i < 4; ++i) zout[p * 8 + r0 + i] = acc[mb][i] + (r0 + i < nbias ? bias[r0 + i] : 0.0f);
      } else {
        u16x4 o;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          o[i] = inside ? f2bf(fmaxf(acc[mb][i] + (r0 + i < nbias ? bias[r0 + i] : 0.0f), 0.0f)) : (uint16_t)0;
        *reinterpret_cast<u16x4*>(out + p * HID + r0) = o;
      }
    }
  }
}

template <int IT>
__global__ __launch_bounds__(256) void k_infer(Prep W, const float* theta, const uint16_t* x, int h, int w, int dmax,
                                               float c_ray, float c_sweep, uint8_t* depth,
                                               unsigned long long* spec_off, unsigned long long* spec_total) {
  constexpr int R0 = IT + 8, R1 = IT + 6, R2 = IT + 4, R3 = IT + 2;
  constexpr int NA = R0 * R0 * XC > R2 * R2 * HID ? R0 * R0 * XC : R2 * R2 * HID;
  __shared__ __attribute__((aligned(16))) uint16_t bufA[NA];             // input rows, then layer-1 output
  __shared__ __attribute__((aligned(16))) uint16_t bufB[R1 * R1 * HID];  // layer-0 output, then layer-2 output
  __shared__ float z[IT * IT * 8];
  const int tiles_x = (w + IT - 1) / IT, tiles_y = (h + IT - 1) / IT;
  const int map = blockIdx.x / (tiles_x * tiles_y), tix = blockIdx.x % (tiles_x * tiles_y);
  const int y0 = (tix / tiles_x) * IT, x0 = (tix % tiles_x) * IT;
  const uint16_t* xm = x + (int64_t)map * h * w * XC;
  // input rows of the region (zero outside the image)
  for (int e = threadIdx.x; e < R0 * R0; e += 256) {
    const int gy = y0 - 4 + e / R0, gx = x0 - 4 + e % R0;
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    if (gy >= 0 && gy < h && gx >= 0 && gx < w) v = *reinterpret_cast<const u16x8*>(xm + ((int64_t)gy * w + gx) * XC);
    *reinterpret_cast<u16x8*>(bufA + e * XC) = v;
  }
  __syncthreads();
  const Offsets o = offsets();
  fused_layer<IT, XC, HID>(W.wf[0], theta + o.b[0], HID, bufA, R0, bufB, nullptr, y0, x0, h, w);
  __syncthreads();
  fused_layer<IT, HID, HID>(W.wf[1], theta + o.b[1], HID, bufB, R1, bufA, nullptr, y0, x0, h, w);
  __syncthreads();
  fused_layer<IT, HID, HID>(W.wf[2], theta + o.b[2], HID, bufA, R2, bufB, nullptr, y0, x0, h, w);
  __syncthreads();
  fused_layer<IT, HID, 16>(W.wf[3], theta + o.b[3], CLASSES, bufB, R3, nullptr, z, y0, x0, h, w);
  __syncthreads();
  // depth choice, then each pixel's speculative rays get a range of the
  // work list: a block prefix sum and one atomic reservation per block
  __shared__ unsigned long long wsum[256 / WAVE], base;
  const int py = threadIdx.x / IT, px = threadIdx.x % IT, gy = y0 + py, gx = x0 + px;
  const bool in = threadIdx.x < IT * IT && gy < h && gx < w;
  const int64_t e = (int64_t)map * h * w + (int64_t)gy * w + gx;
  unsigned long long n = 0;
  if (in) {
    const int d = depth_choice(z + threadIdx.x * 8, dmax, c_ray, c_sweep);
    depth[e] = (uint8_t)d;
    n = subtree_rays(d);
  }
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  unsigned long long pre = n;  // inclusive prefix over the wave
  for (int o = 1; o < WAVE; o <<= 1) {
    const unsigned long long y = __shfl_up(pre, o);
    if (lane >= o) pre += y;
  }
  if (lane == WAVE - 1) wsum[wv] = pre;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < 256 / WAVE; ++q) t += wsum[q];
    base = t ? atomicAdd(spec_total, t) : 0ull;
  }
  __syncthreads();
  unsigned long long before = base + pre - n;
  for (int q = 0; q < wv; ++q) before += wsum[q];
  if (in) spec_off[e] = before;
}

}  // namespace

hipError_t prep_weights(const Net& net, hipStream_t s) {
  Prep P;
  P.theta = net.theta;
  const Offsets o = offsets();
  for (int l = 0; l < LAYERS; ++l) {
    P.wf[l] = net.wf[l];
    P.wt[l] = net.wt[l];
    P.woff[l] = o.w[l];
  }
  hipLaunchKernelGGL(k_prep, dim3(16, LAYERS), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t input_maps(const float* feat, int64_t P, const float* mean, const float* stdv, uint16_t* x,
                      hipStream_t s) {
  Norm nm;
  for (int c = 0; c < FEAT; ++c) {
    nm.mean[c] = mean[c];
    nm.inv_std[c] = 1.0f / stdv[c];
  }
  const int blocks = (int)std::min<int64_t>((P + 255) / 256 + 1, 4096);
  hipLaunchKernelGGL(k_input, dim3(blocks), dim3(256), 0, s, feat, P, nm, x);
  return hipGetLastError();
}

hipError_t conv_forward(int l, const Net& net, const uint16_t* x, int n, int h, int w, void* y, hipStream_t s) {
  const Offsets o = offsets();
  const float* bias = net.theta + o.b[l];
  const int blocks = conv_blocks(n, h, w);
  switch (l) {
    case 0:
      hipLaunchKernelGGL((k_conv<XC, HID, HID, MODE_HIDDEN>), dim3(blocks), dim3(256), 0, s, net.wf[0], bias, HID, x,
                         nullptr, n, h, w, y);
      break;
    case 1:
    case 2:
      hipLaunchKernelGGL((k_conv<HID, HID, HID, MODE_HIDDEN>), dim3(blocks), dim3(256), 0, s, net.wf[l], bias, HID,
                         x, nullptr, n, h, w, y);
      break;
    default:
      hipLaunchKernelGGL((k_conv<HID, 16, ZC, MODE_LOGITS>), dim3(blocks), dim3(256), 0, s, net.wf[3], bias, CLASSES,
                         x, nullptr, n, h, w, y);
  }
  return hipGetLastError();
}

hipError_t conv_input_grad(int l, const Net& net, const uint16_t* dy, const uint16_t* act, int n, int h, int w,
                           uint16_t* dx, hipStream_t s) {
  const int blocks = conv_blocks(n, h, w);
  if (l == 3)
    hipLaunchKernelGGL((k_conv<ZC, HID, HID, MODE_MASK>), dim3(blocks), dim3(256), 0, s, net.wt[3], nullptr, 0, dy,
                       act, n, h, w, dx);
  else
    hipLaunchKernelGGL((k_conv<HID, HID, HID, MODE_MASK>), dim3(blocks), dim3(256), 0, s, net.wt[l], nullptr, 0, dy,
                       act, n, h, w, dx);
  return hipGetLastError();
}

size_t wgrad_partial_floats() { return (size_t)WG_BLOCKS * WG_MAX_FLOATS; }

hipError_t conv_weight_grad(int l, const Net& net, const uint16_t* dy, const uint16_t* x, int n, int h, int w,
                            float* partial, hipStream_t s) {
  const int64_t P = (int64_t)n * h * w;
  if (P < 1 || P >= ((int64_t)1 << 25)) return hipErrorInvalidValue;  // the kernel indexes pixels in 32 bits
  const int64_t tiles = (int64_t)n * ((h + WG_T - 1) / WG_T) * ((w + WG_T - 1) / WG_T);
  const int blocks = (int)std::min<int64_t>(tiles, WG_BLOCKS);
  const Offsets o = offsets();
  int cs, rw;
  if (l == 0) {
    hipLaunchKernelGGL((k_wgrad<XC, HID, HID>), dim3(blocks), dim3(256), 0, s, dy, x, n, h, w, partial);
    cs = XC;
    rw = HID;
  } else if (l < 3) {
    hipLaunchKernelGGL((k_wgrad<HID, HID, HID>), dim3(blocks), dim3(256), 0, s, dy, x, n, h, w, partial);
    cs = HID;
    rw = HID;
  } else {
    hipLaunchKernelGGL((k_wgrad<HID, ZC, 16>), dim3(blocks), dim3(256), 0, s, dy, x, n, h, w, partial);
    cs = HID;
    rw = 16;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int np = (9 * cs + 1 + 15) / 16 * 16;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((rw * np + WAVE - 1) / WAVE), dim3(256), 0, s, partial, blocks, rw, np, cs,
                     CIN[l], COUT[l],
                     net.grad + o.w[l], net.grad + o.b[l]);
  return hipGetLastError();
}

size_t loss_partial_doubles() { return 2 * LOSS_BLOCKS; }

hipError_t loss_and_dz(const float* z, const int32_t* labels, int64_t P, const float* class_w, double* partial,
                       double* out, uint16_t* dz, hipStream_t s) {
  ClassW cw;
  for (int c = 0; c < CLASSES; ++c) cw.w[c] = class_w[c];
  hipLaunchKernelGGL(k_loss_partial, dim3(LOSS_BLOCKS), dim3(256), 0, s, z, labels, P, cw, partial);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, partial, LOSS_BLOCKS, out);
  const int blocks = (int)std::min<int64_t>((P + 255) / 256 + 1, 4096);
  hipLaunchKernelGGL(k_dz, dim3(blocks), dim3(256), 0, s, z, labels, P, cw, out, dz);
  return hipGetLastError();
}

hipError_t infer_depth(const Net& net, const uint16_t* x, int n, int h, int w, int dmax, float c_ray, float c_sweep,
                       uint8_t* depth, unsigned long long* spec_off, unsigned long long* spec_total, hipStream_t s) {
  Prep P;
  P.theta = net.theta;
  for (int l = 0; l < LAYERS; ++l) {
    P.wf[l] = net.wf[l];
    P.wt[l] = net.wt[l];
    P.woff[l] = 0;
  }
  const int tiles16 = ((w + 15) / 16) * ((h + 15) / 16) * n;
  if (tiles16 >= 256) {
    hipLaunchKernelGGL(k_infer<16>, dim3(tiles16), dim3(256), 0, s, P, net.theta, x, h, w, dmax, c_ray, c_sweep, depth,
                       spec_off, spec_total);
  } else if (((w + 7) / 8) * ((h + 7) / 8) * n >= 64) {
    const int tiles8 = ((w + 7) / 8) * ((h + 7) / 8) * n;
    hipLaunchKernelGGL(k_infer<8>, dim3(tiles8), dim3(256), 0, s, P, net.theta, x, h, w, dmax, c_ray, c_sweep, depth,
                       spec_off, spec_total);
  } else {
    const int tiles4 = ((w + 3) / 4) * ((h + 3) / 4) * n;
    hipLaunchKernelGGL(k_infer<4>, dim3(tiles4), dim3(256), 0, s, P, net.theta, x, h, w, dmax, c_ray, c_sweep, depth,
                       spec_off, spec_total);
  }
  return hipGetLastError();
}

hipError_t adam(Net& net, int P, float lr, float beta1, float beta2, float eps, hipStream_t s) {
  net.step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)net.step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)net.step)));
  hipLaunchKernelGGL(k_adam, dim3((P + 255) / 256), dim3(256), 0, s, net.theta, net.m, net.v, net.grad, P, lr, beta1,
                     beta2, eps, c1, c2);
  net.dirty = true;
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace air
