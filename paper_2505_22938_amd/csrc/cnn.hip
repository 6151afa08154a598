// Bracket-proposal CNN kernels (not in the paper): 3x3 convolutions on a
// grid of 8x8-pixel cells, bfloat16 operands on MFMA with float32
// accumulation, their backward passes, the pinball loss and an Adam step.
//
// Layouts
//   activations  bf16 [H][W][32]        (cell-major, 32 channels, 64 B/cell)
//   weights      bf16 [cout][9][32]     (tap = 3 * (dy + 1) + (dx + 1))
//   bias         f32  [cout]
//   cout is 32 for hidden layers and 16 for the output layer (channels 0, 1
//   = lo, hi; 2..15 zero weights).
//
// A convolution is an implicit GEMM: rows = 16 consecutive cells of one
// grid row, columns = 16 output channels, and the reduction runs over
// (tap, input channel) in 9 chunks of 32, one v_mfma_f32_16x16x32_bf16 per
// chunk per column block.  Operand fragments (one wave, lane l, g = l / 16):
//   A: row l % 16, reduction index 8g .. 8g + 7   (8 bf16, one 16-byte load)
//   B: column l % 16, reduction index 8g .. 8g + 7
//   D: column l % 16, rows 4g .. 4g + 3           (4 f32)
// mf_mfma_probe checks this layout against a host matrix product.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "mf_internal.h"

namespace mf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kC = 32;       // channels of every activation tensor
constexpr int kTaps = 9;
constexpr int kCell = 8;     // pixels per cell side

__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                              // nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ bf16x8 zero8() {
  return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
}

// ------------------------------------------------------------------ probe

__global__ void mfma_probe_kernel(const uint16_t* A, const uint16_t* B, float* D) {
  // A: 16 x 32 row-major, B: 32 x 16 row-major, D: 16 x 16 row-major
  const int l = threadIdx.x, g = l >> 4, r = l & 15;
  uint16_t a[8], b[8];
  for (int j = 0; j < 8; ++j) {
    a[j] = A[r * 32 + 8 * g + j];
    b[j] = B[(8 * g + j) * 16 + r];
  }
  const bf16x8 av = __builtin_bit_cast(bf16x8, *reinterpret_cast<uint4*>(a));
  const bf16x8 bv = __builtin_bit_cast(bf16x8, *reinterpret_cast<uint4*>(b));
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  for (int i = 0; i < 4; ++i) D[(4 * g + i) * 16 + r] = acc[i];
}

// ------------------------------------------------------------------ forward

enum { EPI_RELU_BF16 = 0, EPI_F32 = 1, EPI_MASK_BF16 = 2 };

// One wave: 16 cells (x0 .. x0+15 of row y) x all COUT channels.
// EPI_RELU_BF16: y = bf16(relu(acc + b));  EPI_F32: y = acc + b (f32);
// EPI_MASK_BF16: y = bf16(acc * [mask > 0]) with mask a bf16 activation.
template <int COUT, int EPI>
__global__ __launch_bounds__(256) void conv3x3_kernel(const uint16_t* __restrict__ x, int H, int W,
                                                      const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias,
                                                      const uint16_t* __restrict__ mask,
                                                      void* __restrict__ y) {
  const int lane = threadIdx.x & 63, wave = (blockIdx.x * 4) + (threadIdx.x >> 6);
  const int segs = (W + 15) / 16;
  if (wave >= segs * H) return;
  const int yy = wave / segs, x0 = (wave - yy * segs) * 16;
  const int g = lane >> 4, r = lane & 15;
  constexpr int NB = COUT / 16;
  floatx4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < kTaps; ++t) {
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    const int sy = yy + dy, sx = x0 + r + dx;
    bf16x8 av = zero8();
    if (sy >= 0 && sy < H && sx >= 0 && sx < W) av = load8(x + ((long long)sy * W + sx) * kC + 8 * g);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = nb * 16 + r;
      const bf16x8 bv = load8(w + ((long long)co * kTaps + t) * kC + 8 * g);
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int co = nb * 16 + r;
    const float bco = bias ? bias[co] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int xx = x0 + 4 * g + i;
      if (xx >= W) continue;
      const long long cell = (long long)yy * W + xx;
      float v = acc[nb][i] + bco;
      if (EPI == EPI_F32) {
        static_cast<float*>(y)[cell * COUT + co] = v;
      } else {
        if (EPI == EPI_RELU_BF16) v = v > 0.f ? v : 0.f;
        if (EPI == EPI_MASK_BF16) v = bf16_bits_to_f32(mask[cell * kC + co]) > 0.f ? v : 0.f;
        static_cast<uint16_t*>(y)[cell * kC + co] = f32_to_bf16_bits(v);
      }
    }
  }
}

// Backward-data weights: wf[ci][t][co] = w[co][8 - t][ci] (zero for co >= cout).
__global__ void flip_weights_kernel(const uint16_t* __restrict__ w, int cout,
                                    uint16_t* __restrict__ wf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kC * kTaps * kC) return;
  const int ci = i / (kTaps * kC), t = (i / kC) % kTaps, co = i % kC;
  wf[i] = co < cout ? w[((long long)co * kTaps + (kTaps - 1 - t)) * kC + ci] : (uint16_t)0;
}

// ------------------------------------------------------------------ backward weights

// Partial weight and bias gradients over a chunk of cells.  Block = 4
// waves; grid = one block per kChunkCells cells in row-major order.  The
// block stages, per 32-cell row segment, dY (32 cells x 32 ch) and the
// three input rows around it (34 cells x 32 ch each) in LDS, then
// accumulates dW[co][t*32+ci] += sum_cells dY[cell][co] * X[cell+off(t)][ci]
// with MFMA (rows = co, columns = (t, ci), reduction = cells).
constexpr int kSeg = 32;
template <int COUT>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(const uint16_t* __restrict__ x,
                                                         const uint16_t* __restrict__ dy, int H,
                                                         int W, int segs_per_block,
                                                         float* __restrict__ part_w,
                                                         float* __restrict__ part_b) {
  __shared__ uint16_t s_dy[kSeg * kC];
  __shared__ uint16_t s_x[3][(kSeg + 2) * kC];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  constexpr int MB = COUT / 16, NBT = kTaps * kC / 16;   // 18 column blocks
  constexpr int NBW = (NBT + 3) / 4;                      // per wave
  floatx4 acc[MB][NBW];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int j = 0; j < NBW; ++j) acc[mb][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;   // thread t < COUT accumulates db[t]
  const int segs_row = (W + kSeg - 1) / kSeg;
  const int total_segs = segs_row * H;
  for (int s = 0; s < segs_per_block; ++s) {
    const int seg = blockIdx.x * segs_per_block + s;
    if (seg >= total_segs) break;
    const int yy = seg / segs_row, x0 = (seg - yy * segs_row) * kSeg;
    __syncthreads();
    for (int i = threadIdx.x; i < kSeg * kC; i += 256) {
      const int c = i / kC, ch = i % kC, xx = x0 + c;
      s_dy[i] = (xx < W && ch < COUT) ? dy[((long long)yy * W + xx) * kC + ch] : (uint16_t)0;
    }
    for (int i = threadIdx.x; i < 3 * (kSeg + 2) * kC; i += 256) {
      const int row = i / ((kSeg + 2) * kC), rem = i % ((kSeg + 2) * kC);
      const int c = rem / kC, ch = rem % kC;
      const int sy = yy + row - 1, sx = x0 + c - 1;
      s_x[row][rem] = (sy >= 0 && sy < H && sx >= 0 && sx < W) ? x[((long long)sy * W + sx) * kC + ch]
                                                               : (uint16_t)0;
    }
    __syncthreads();
    if (threadIdx.x < COUT)
      for (int c = 0; c < kSeg; ++c) bsum += bf16_bits_to_f32(s_dy[c * kC + threadIdx.x]);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      uint16_t a[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] = s_dy[(8 * g + j) * kC + mb * 16 + r];
      const bf16x8 av = __builtin_bit_cast(bf16x8, *reinterpret_cast<uint4*>(a));
#pragma unroll
      for (int j = 0; j < NBW; ++j) {
        const int nb = wv + 4 * j;
        if (nb >= NBT) continue;
        const int n = nb * 16 + r, t = n / kC, ci = n % kC;
        const int dyy = t / 3, dxx = t % 3;   // row in s_x, column shift
        uint16_t b[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) b[q] = s_x[dyy][(8 * g + q + dxx) * kC + ci];
        const bf16x8 bv = __builtin_bit_cast(bf16x8, *reinterpret_cast<uint4*>(b));
        acc[mb][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[mb][j], 0, 0, 0);
      }
    }
  }
  float* pw = part_w + (long long)blockIdx.x * COUT * kTaps * kC;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int j = 0; j < NBW; ++j) {
      const int nb = wv + 4 * j;
      if (nb >= NBT) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) pw[(mb * 16 + 4 * g + i) * (kTaps * kC) + nb * 16 + r] = acc[mb][j][i];
    }
  if (threadIdx.x < COUT) part_b[(long long)blockIdx.x * COUT + threadIdx.x] = bsum;
}

// Sum the per-block partials (deterministic order).
__global__ void reduce_partials_kernel(const float* __restrict__ part, int nblocks, int n,
                                       float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int b = 0; b < nblocks; ++b) s += part[(long long)b * n + i];
  out[i] = s;
}

// ------------------------------------------------------------------ loss, features, Adam

// Pinball loss of out[cell][0] (lo) and out[cell][1] (hi) against targets
// tgt[cell][2]; writes dOut (gradient of the SUM over cells) as a 32-channel
// bf16 tensor and per-block loss partial sums.
__global__ void pinball_kernel(const float* __restrict__ out, int out_ch,
                               const float* __restrict__ tgt, int ncell, float tau_lo,
                               float tau_hi, uint16_t* __restrict__ dout,
                               float* __restrict__ part_loss) {
  __shared__ float s[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < ncell) {
    const float u0 = tgt[2 * i] - out[(long long)i * out_ch];
    const float u1 = tgt[2 * i + 1] - out[(long long)i * out_ch + 1];
    const float w0 = tau_lo - (u0 < 0.f ? 1.f : 0.f), w1 = tau_hi - (u1 < 0.f ? 1.f : 0.f);
    l = u0 * w0 + u1 * w1;
    uint16_t* d = dout + (long long)i * kC;
    d[0] = f32_to_bf16_bits(-w0);
    d[1] = f32_to_bf16_bits(-w1);
    for (int c = 2; c < kC; ++c) d[c] = 0;
  }
  s[threadIdx.x] = l;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part_loss[blockIdx.x] = s[0];
}

// Network input per cell: channel 0 = mean of the cell's pixels / maxval,
// channel 1 = radius / 64, channels 2..31 = 0.
template <typename T>
__global__ void features_kernel(const T* __restrict__ img, long long stride, int w, int h,
                                float inv_max, float rplane, uint16_t* __restrict__ feat) {
  const int hc = (h + kCell - 1) / kCell, wc = (w + kCell - 1) / kCell;
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= hc * wc) return;
  const int cy = cell / wc, cx = cell - cy * wc;
  float s = 0.f;
  int n = 0;
  for (int y = cy * kCell; y < min(h, cy * kCell + kCell); ++y)
    for (int x = cx * kCell; x < min(w, cx * kCell + kCell); ++x) {
      s += (float)img[(long long)y * stride + x];
      ++n;
    }
  uint16_t* f = feat + (long long)cell * kC;
  f[0] = f32_to_bf16_bits(s / (float)n * inv_max);
  f[1] = f32_to_bf16_bits(rplane);
  for (int c = 2; c < kC; ++c) f[c] = 0;
}

// ------------------------------------------------------------------ fused inference

// The whole network in one launch (inference only: no activation is kept).
// A workgroup computes a 16x16-cell block of the output.  Each 3x3 layer
// needs one more cell of input on every side, so the block's features are
// taken over 24x24 cells and the three hidden layers over 22x22, 20x20 and
// 18x18 cells, all in LDS (two buffers used in turn).  Cells outside the
// cell grid hold zero at every layer, which is the layer-by-layer kernels'
// zero padding, so the result equals theirs bit for bit: the MFMA sequence
// per output cell (tap order, reduction chunks), the bias add, ReLU and bf16
// rounding are the same, and the cell sums of the features are exact in
// float32 (at most 64 values below 2^16), whatever their order.
// A layer's row of output cells is covered by 16-cell MFMA row blocks at
// x = 0 and x = width - 16; where the two overlap, both write the same
// values.  All four layers' weights are staged in LDS once, tap-major
// ([tap][cout][32], so the 16 lanes of an MFMA operand read 1 KB of
// consecutive bytes), while the block's pixels are being read.
constexpr int kNetOB = 16;          // output cells per block side
constexpr int kNetIn = kNetOB + 8;  // feature cells per block side
constexpr int kNetThreads = 1024;
constexpr int kNetW = kTaps * 32 * kC;            // bf16 weights of a 32-channel layer
constexpr int kNetWAll = 3 * kNetW + kTaps * 16 * kC;

struct NetWeights {
  const uint16_t* w[4];   // bf16 [cout][9][32]
  const float* b[4];      // f32 [cout]
};

template <int WIN, int NB, bool LAST>
__device__ __forceinline__ void net_layer(const uint16_t* __restrict__ in,
                                          uint16_t* __restrict__ ob, float* __restrict__ gout,
                                          const uint16_t* __restrict__ ws,
                                          const float* __restrict__ bias, int oy0, int ox0, int H,
                                          int W) {
  constexpr int WOUT = WIN - 2, NXB = WOUT > 16 ? 2 : 1, NW = kNetThreads / 64;
  constexpr int COUT = 16 * NB;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  float bco[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) bco[nb] = bias[nb * 16 + r];
  for (int task = wv; task < WOUT * NXB; task += NW) {
    const int yo = task / NXB, xb = (task % NXB) ? WOUT - 16 : 0;
    floatx4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      const int dy = t / 3, dx = t % 3;   // input cell = output cell + (dy - 1, dx - 1) + 1
      const bf16x8 av = load8(in + ((yo + dy) * WIN + xb + r + dx) * kC + 8 * g);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bf16x8 bv = load8(ws + (t * COUT + nb * 16 + r) * kC + 8 * g);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nb], 0, 0, 0);
      }
    }
    const int gy = oy0 + yo;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = nb * 16 + r;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int xo = xb + 4 * g + i, gx = ox0 + xo;
        const float v = acc[nb][i] + bco[nb];
        const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
        if (LAST) {
          if (inside) gout[((long long)gy * W + gx) * 16 + co] = v;
        } else {
          ob[(yo * WOUT + xo) * kC + co] = inside ? f32_to_bf16_bits(v > 0.f ? v : 0.f) : (uint16_t)0;
        }
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kNetThreads) void net_forward_kernel(const T* __restrict__ img,
                                                                  long long stride, int w, int h,
                                                                  float inv_max, float rplane,
                                                                  NetWeights nw,
                                                                  float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint16_t wsm[kNetWAll];
  __shared__ __attribute__((aligned(16))) uint16_t buf_a[kNetIn * kNetIn * kC];
  __shared__ __attribute__((aligned(16))) uint16_t buf_b[(kNetIn - 2) * (kNetIn - 2) * kC];
  const int H = (h + kCell - 1) / kCell, W = (w + kCell - 1) / kCell;
  const int cx0 = blockIdx.x * kNetOB, cy0 = blockIdx.y * kNetOB;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // weights, 16 bytes per load: source [cout][tap][32] -> LDS [tap][cout][32]
  for (int i = t; i < kNetWAll / 8; i += kNetThreads) {
    const int e = i * 8;
    const int l = e < 3 * kNetW ? e / kNetW : 3;
    const int cout = l == 3 ? 16 : 32, le = e - l * kNetW;
    const int co = le / (kTaps * kC), tap = (le / kC) % kTaps, c = le % kC;
    *reinterpret_cast<uint4*>(wsm + l * kNetW + (tap * cout + co) * kC + c) =
        *reinterpret_cast<const uint4*>(nw.w[l] + le);
  }
  // features over the 24x24 cells around the block: a wave takes rows of
  // cells, its lanes adjacent pixels of each pixel row (3 x 64 = 192 pixels)
  constexpr int NW = kNetThreads / 64;
  for (int cr = wv; cr < kNetIn; cr += NW) {
    const int gcy = cy0 - 4 + cr;
    float s[3] = {0.f, 0.f, 0.f};
    if (gcy >= 0 && gcy < H) {
#pragma unroll
      for (int py = 0; py < kCell; ++py) {
        const int y = gcy * kCell + py;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const int x = (cx0 - 4) * kCell + lane + 64 * j;
          if (y < h && x >= 0 && x < w) s[j] += (float)img[(long long)y * stride + x];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      s[j] += __shfl_xor(s[j], 1, 64);
      s[j] += __shfl_xor(s[j], 2, 64);
      s[j] += __shfl_xor(s[j], 4, 64);
    }
    const int k = lane & 7;   // this lane writes channels 4k .. 4k+3
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int cc = (lane >> 3) + 8 * j, gcx = cx0 - 4 + cc;
      uint2 v = make_uint2(0u, 0u);
      if (k == 0 && gcy >= 0 && gcy < H && gcx >= 0 && gcx < W) {
        const int n = min(kCell, w - gcx * kCell) * min(kCell, h - gcy * kCell);
        v.x = (uint32_t)f32_to_bf16_bits(s[j] / (float)n * inv_max) |
              ((uint32_t)f32_to_bf16_bits(rplane) << 16);
      }
      *reinterpret_cast<uint2*>(buf_a + (cr * kNetIn + cc) * kC + 4 * k) = v;
    }
  }
  __syncthreads();
  net_layer<kNetIn, 2, false>(buf_a, buf_b, nullptr, wsm, nw.b[0], cy0 - 3, cx0 - 3, H, W);
  __syncthreads();
  net_layer<kNetIn - 2, 2, false>(buf_b, buf_a, nullptr, wsm + kNetW, nw.b[1], cy0 - 2, cx0 - 2,
                                  H, W);
  __syncthreads();
  net_layer<kNetIn - 4, 2, false>(buf_a, buf_b, nullptr, wsm + 2 * kNetW, nw.b[2], cy0 - 1,
                                  cx0 - 1, H, W);
  __syncthreads();
  net_layer<kNetIn - 6, 1, true>(buf_b, nullptr, out, wsm + 3 * kNetW, nw.b[3], cy0, cx0, H, W);
}

// Training targets per cell: min and max of the exact median image / maxval.
template <typename T>
__global__ void targets_kernel(const T* __restrict__ med, long long stride, int w, int h,
                               float inv_max, float* __restrict__ tgt) {
  const int hc = (h + kCell - 1) / kCell, wc = (w + kCell - 1) / kCell;
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= hc * wc) return;
  const int cy = cell / wc, cx = cell - cy * wc;
  float lo = 3.4e38f, hi = -3.4e38f;
  for (int y = cy * kCell; y < min(h, cy * kCell + kCell); ++y)
    for (int x = cx * kCell; x < min(w, cx * kCell + kCell); ++x) {
      const float v = (float)med[(long long)y * stride + x];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
  tgt[2 * cell] = lo * inv_max;
  tgt[2 * cell + 1] = hi * inv_max;
}

// Adam on float32 master parameters; refreshes the bf16 copy.  Parameter
// i of a weight tensor is also weight element i (same layout).
__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ grad, int n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2, uint16_t* __restrict__ p_bf16) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * g, vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  p[i] = pi;
  if (p_bf16) p_bf16[i] = f32_to_bf16_bits(pi);
}

}  // namespace mf

// ------------------------------------------------------------------ C ABI

namespace {
int launch_ok() { return hipGetLastError() == hipSuccess ? MF_OK : MF_ERR_HIP; }
}  // namespace

extern "C" {

int mf_mfma_probe(const void* a, const void* b, float* d, hipStream_t stream) {
  if (!a || !b || !d) return MF_ERR_INVALID_ARG;
  hipLaunchKernelGGL(mf::mfma_probe_kernel, dim3(1), dim3(64), 0, stream,
                     static_cast<const uint16_t*>(a), static_cast<const uint16_t*>(b), d);
  return launch_ok();
}

int mf_cnn_conv_forward(const void* x, int H, int W, const void* w, const float* bias, int cout,
                        int mode, const void* mask, void* y, hipStream_t stream) {
  if (!x || !w || !y || H <= 0 || W <= 0 || (cout != 32 && cout != 16)) return MF_ERR_INVALID_ARG;
  if (mode < 0 || mode > 2 || (mode == 2 && (!mask || cout != 32)) || (mode == 0 && cout != 32))
    return MF_ERR_INVALID_ARG;
  const long long waves = (long long)((W + 15) / 16) * H;
  const dim3 grid((unsigned)((waves + 3) / 4));
  const auto* xs = static_cast<const uint16_t*>(x);
  const auto* ws = static_cast<const uint16_t*>(w);
  const auto* ms = static_cast<const uint16_t*>(mask);
  if (cout == 16)
    hipLaunchKernelGGL((mf::conv3x3_kernel<16, mf::EPI_F32>), grid, dim3(256), 0, stream, xs, H, W,
                       ws, bias, ms, y);
  else if (mode == 0)
    hipLaunchKernelGGL((mf::conv3x3_kernel<32, mf::EPI_RELU_BF16>), grid, dim3(256), 0, stream, xs,
                       H, W, ws, bias, ms, y);
  else if (mode == 1)
    hipLaunchKernelGGL((mf::conv3x3_kernel<32, mf::EPI_F32>), grid, dim3(256), 0, stream, xs, H, W,
                       ws, bias, ms, y);
  else
    hipLaunchKernelGGL((mf::conv3x3_kernel<32, mf::EPI_MASK_BF16>), grid, dim3(256), 0, stream, xs,
                       H, W, ws, bias, ms, y);
  return launch_ok();
}

int mf_cnn_flip_weights(const void* w, int cout, void* wf, hipStream_t stream) {
  if (!w || !wf || (cout != 32 && cout != 16)) return MF_ERR_INVALID_ARG;
  hipLaunchKernelGGL(mf::flip_weights_kernel, dim3((32 * 9 * 32 + 255) / 256), dim3(256), 0,
                     stream, static_cast<const uint16_t*>(w), cout, static_cast<uint16_t*>(wf));
  return launch_ok();
}

// Workspace floats needed by mf_cnn_conv_wgrad for an H x W grid.
long long mf_cnn_wgrad_workspace(int H, int W, int cout, int segs_per_block) {
  if (H <= 0 || W <= 0 || segs_per_block <= 0) return -1;
  const long long segs = (long long)((W + 31) / 32) * H;
  const long long blocks = (segs + segs_per_block - 1) / segs_per_block;
  return blocks * (long long)cout * (9 * 32 + 1);
}

int mf_cnn_conv_wgrad(const void* x, const void* dy, int H, int W, int cout, int segs_per_block,
                      float* workspace, float* dw, float* db, hipStream_t stream) {
  if (!x || !dy || !workspace || !dw || !db || H <= 0 || W <= 0 || segs_per_block <= 0 ||
      (cout != 32 && cout != 16))
    return MF_ERR_INVALID_ARG;
  const long long segs = (long long)((W + 31) / 32) * H;
  const int blocks = (int)((segs + segs_per_block - 1) / segs_per_block);
  float* pw = workspace;
  float* pb = workspace + (long long)blocks * cout * 9 * 32;
  const auto* xs = static_cast<const uint16_t*>(x);
  const auto* ds = static_cast<const uint16_t*>(dy);
  if (cout == 32)
    hipLaunchKernelGGL(mf::conv_wgrad_kernel<32>, dim3(blocks), dim3(256), 0, stream, xs, ds, H,
                       W, segs_per_block, pw, pb);
  else
    hipLaunchKernelGGL(mf::conv_wgrad_kernel<16>, dim3(blocks), dim3(256), 0, stream, xs, ds, H,
                       W, segs_per_block, pw, pb);
  int rc = launch_ok();
  if (rc) return rc;
  const int nw = cout * 9 * 32;
  hipLaunchKernelGGL(mf::reduce_partials_kernel, dim3((nw + 255) / 256), dim3(256), 0, stream, pw,
                     blocks, nw, dw);
  hipLaunchKernelGGL(mf::reduce_partials_kernel, dim3(1), dim3(256), 0, stream, pb, blocks, cout,
                     db);
  return launch_ok();
}

int mf_cnn_pinball(const float* out, int out_ch, const float* tgt, int ncell, float tau_lo,
                   float tau_hi, void* dout, float* part_loss, hipStream_t stream) {
  if (!out || !tgt || !dout || !part_loss || ncell <= 0 || out_ch < 2) return MF_ERR_INVALID_ARG;
  hipLaunchKernelGGL(mf::pinball_kernel, dim3((ncell + 255) / 256), dim3(256), 0, stream, out,
                     out_ch, tgt, ncell, tau_lo, tau_hi, static_cast<uint16_t*>(dout), part_loss);
  return launch_ok();
}

int mf_cnn_features(const void* img, int w, int h, size_t stride_bytes, int dtype, int radius,
                    void* feat, hipStream_t stream) {
  if (!img || !feat || w <= 0 || h <= 0 || (dtype != MF_U8 && dtype != MF_U16))
    return MF_ERR_INVALID_ARG;
  const int ncell = ((w + 7) / 8) * ((h + 7) / 8);
  const float rp = radius / 64.0f;
  if (dtype == MF_U8)
    hipLaunchKernelGGL(mf::features_kernel<uint8_t>, dim3((ncell + 255) / 256), dim3(256), 0,
                       stream, static_cast<const uint8_t*>(img), (long long)stride_bytes, w, h,
                       1.0f / 255.0f, rp, static_cast<uint16_t*>(feat));
  else
    hipLaunchKernelGGL(mf::features_kernel<uint16_t>, dim3((ncell + 255) / 256), dim3(256), 0,
                       stream, static_cast<const uint16_t*>(img), (long long)(stride_bytes / 2), w,
                       h, 1.0f / 65535.0f, rp, static_cast<uint16_t*>(feat));
  return launch_ok();
}

int mf_cnn_net_forward(const void* img, int w, int h, size_t stride_bytes, int dtype, int radius,
                       const void* const* w_bf16, const float* const* bias, float* out,
                       hipStream_t stream) {
  if (!img || !out || !w_bf16 || !bias || w <= 0 || h <= 0 || radius < 0 ||
      (dtype != MF_U8 && dtype != MF_U16))
    return MF_ERR_INVALID_ARG;
  const size_t es = dtype == MF_U8 ? 1 : 2;
  if (stride_bytes < (size_t)w * es || stride_bytes % es) return MF_ERR_INVALID_ARG;
  mf::NetWeights nw;
  for (int l = 0; l < 4; ++l) {
    if (!w_bf16[l] || !bias[l] || (reinterpret_cast<uintptr_t>(w_bf16[l]) & 15u))
      return MF_ERR_INVALID_ARG;
    nw.w[l] = static_cast<const uint16_t*>(w_bf16[l]);
    nw.b[l] = bias[l];
  }
  const int H = (h + 7) / 8, W = (w + 7) / 8;
  const dim3 grid((unsigned)((W + mf::kNetOB - 1) / mf::kNetOB),
                  (unsigned)((H + mf::kNetOB - 1) / mf::kNetOB));
  const float rp = radius / 64.0f;
  if (dtype == MF_U8)
    hipLaunchKernelGGL(mf::net_forward_kernel<uint8_t>, grid, dim3(mf::kNetThreads), 0, stream,
                       static_cast<const uint8_t*>(img), (long long)stride_bytes, w, h,
                       1.0f / 255.0f, rp, nw, out);
  else
    hipLaunchKernelGGL(mf::net_forward_kernel<uint16_t>, grid, dim3(mf::kNetThreads), 0, stream,
                       static_cast<const uint16_t*>(img), (long long)(stride_bytes / 2), w, h,
                       1.0f / 65535.0f, rp, nw, out);
  return launch_ok();
}

int mf_cnn_targets(const void* med, int w, int h, size_t stride_bytes, int dtype, float* tgt,
                   hipStream_t stream) {
  if (!med || !tgt || w <= 0 || h <= 0 || (dtype != MF_U8 && dtype != MF_U16))
    return MF_ERR_INVALID_ARG;
  const int ncell = ((w + 7) / 8) * ((h + 7) / 8);
  if (dtype == MF_U8)
    hipLaunchKernelGGL(mf::targets_kernel<uint8_t>, dim3((ncell + 255) / 256), dim3(256), 0,
                       stream, static_cast<const uint8_t*>(med), (long long)stride_bytes, w, h,
                       1.0f / 255.0f, tgt);
  else
    hipLaunchKernelGGL(mf::targets_kernel<uint16_t>, dim3((ncell + 255) / 256), dim3(256), 0,
                       stream, static_cast<const uint16_t*>(med), (long long)(stride_bytes / 2), w,
                       h, 1.0f / 65535.0f, tgt);
  return launch_ok();
}

int mf_cnn_adam(float* p, float* m, float* v, const float* grad, int n, float lr, float b1,
                float b2, float eps, int step, void* p_bf16, hipStream_t stream) {
  if (!p || !m || !v || !grad || n <= 0 || step < 1) return MF_ERR_INVALID_ARG;
  // bias corrections 1 - beta^t in double: in float32, 1 - powf(0.999f, 2)
  // keeps only a few correct bits (the power is within one ulp of 1)
  const float bc1 = (float)(1.0 - std::pow((double)b1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)b2, (double)step));
  hipLaunchKernelGGL(mf::adam_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, m, v, grad,
                     n, lr, b1, b2, eps, bc1, bc2, static_cast<uint16_t*>(p_bf16));
  return launch_ok();
}

}  // extern "C"
