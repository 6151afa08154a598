// Learned bracket proposal (not in the paper) around the exact engine.
//
// A four-layer 3x3 CNN on 8x8-pixel cells (input: cell mean and the radius
// plane) predicts per cell a bracket [lo, hi] for the medians of the cell's
// pixels.  A tile's bracket is the union over the cells it covers, widened
// by a calibrated margin.  The bracketed tile kernel ranks only the box
// pixels inside the bracket (exact counts, see tile_body's BR mode); a tile
// where some median falls outside is flagged and recomputed by the plain
// engine, so the output is always exact.  Training runs the network's own
// forward, backward and Adam kernels (cnn.hip) on targets made from exact
// median images.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "../../include/mf_cnn.h"
#include "mf_internal.h"
#include "tile_engine.h"

namespace mf {

// Parameter layout (floats): W1 b1 W2 b2 W3 b3 W4 b4; weights are
// [cout][9][32], W4 has 16 output rows (0 = lo, 1 = hi, rest zero).
constexpr int kW = 32 * 9 * 32, kW4 = 16 * 9 * 32;
constexpr int kOffW[4] = {0, kW + 32, 2 * (kW + 32), 3 * (kW + 32)};
constexpr int kOffB[4] = {kW, 2 * kW + 32, 3 * kW + 64, 3 * (kW + 32) + kW4};
constexpr int kParams = 3 * (kW + 32) + kW4 + 16;

__device__ __forceinline__ void count_fallback(const ImageDesc& a, int tile,
                                               unsigned long long* fail_px) {
  const int tx0 = (tile % a.tiles_x) * a.tw, ty0 = (tile / a.tiles_x) * a.th;
  const long long n = (long long)min(a.tw, a.w - tx0) * min(a.th, a.h - ty0);
  atomicAdd(fail_px, (unsigned long long)n);
}

// Bracketed tiles: one workgroup per tile; writes the tile's fail flag
// (median outside the bracket, or more in-bracket pixels than fit).
template <int KT, int SHAPE, int IMAX>
__global__ __launch_bounds__(kThreads) void mf_bracket_tile_kernel(ImageDesc a, int* tile_fail) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const bool bad = tile_body<KT, SHAPE, IMAX, false, true>(a, tile, smem, nullptr);
  if (threadIdx.x == 0) tile_fail[tile] = bad ? 1 : 0;
}

// The bracketed tile holding fallback tile `tile`: fallback tiles have the
// bracketed tiles' width and 1/ratio of their height.
__device__ __forceinline__ int parent_tile(const ImageDesc& f, int tile, int ratio) {
  const int tx = tile % f.tiles_x, ty = tile / f.tiles_x;
  return (ty / ratio) * f.tiles_x + tx;
}

// Plain pass over the flagged tiles, LDS variant: one workgroup per tile.
template <int KT, int SHAPE, int IMAX>
__global__ __launch_bounds__(kThreads) void mf_fallback_kernel(ImageDesc f, const int* tile_fail,
                                                               unsigned long long* fail_px,
                                                               int ratio) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile_fail[parent_tile(f, tile, ratio)] == 0) return;   // uniform per workgroup
  tile_body<KT, SHAPE, IMAX, false, false>(f, tile, smem, nullptr);
  if (threadIdx.x == 0) count_fallback(f, tile, fail_px);
}

// Plain pass over the flagged tiles, global-scratch variant: a persistent
// grid, one scratch slot per workgroup.
template <int KT, int SHAPE>
__global__ __launch_bounds__(kThreads) void mf_fallback_gs_kernel(ImageDesc f,
                                                                  const int* tile_fail,
                                                                  unsigned long long* fail_px,
                                                                  int ratio) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  unsigned char* slot = f.scratch + (long long)blockIdx.x * f.slot_bytes;
  const int ntiles = f.tiles_x * f.tiles_y;
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const int tile = xcd_tile(v, ntiles);
    if (tile_fail[parent_tile(f, tile, ratio)] == 0) continue;   // uniform per workgroup
    tile_body<KT, SHAPE, 1, true>(f, tile, smem, slot);
    if (threadIdx.x == 0) count_fallback(f, tile, fail_px);
    __syncthreads();
  }
}

// Per-pixel exact fallback: one workgroup (four waves) per listed pixel
// (index y * w + x) selects the rank-k value of its window straight from
// the image by radix selection on the value bits: a 256-bin histogram of
// the top byte finds the byte holding rank k, then (16-bit) a histogram of
// the low byte among the values with that top byte.  The four waves take
// the window's rows in turn, eight rows (up to 256 taps each) of loads in
// flight per wave, and keep the values in LDS for the second histogram
// when the window fits the staging buffer (the launch's dynamic LDS of
// stage_cap taps, which the host sizes to the window when it has at most
// kSelStage taps, else empty: the window is then read again).  Sized to the
// window, the buffer leaves room for more workgroups per CU under small
// windows.  Adds the list length to fail_px.
constexpr int kSelStage = 16384, kSelMaxRows = 512;
template <int KT>
__global__ __launch_bounds__(256) void mf_pixel_select_kernel(ImageDesc f,
                                                              const unsigned int* miss,
                                                              const unsigned int* miss_count,
                                                              unsigned long long* fail_px,
                                                              int stage_cap) {
  constexpr int kRows = 8;
  __shared__ uint32_t hist[256];
  extern __shared__ __attribute__((aligned(16))) uint16_t stage[];   // stage_cap entries
  __shared__ int rowbase[kSelMaxRows + 1];   // staged position of each row's first tap
  __shared__ int sel[2];                     // bin holding rank k, count below the bin
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int n = (int)*miss_count;
  if (blockIdx.x == 0 && t == 0 && n > 0) atomicAdd(fail_px, (unsigned long long)n);
  if ((int)blockIdx.x >= n) return;   // uniform per workgroup
  const int nrows = f.nrows;          // <= kSelMaxRows (host-checked)
  // rowbase = exclusive prefix sum of the row widths (wave 0, 64 rows per step)
  __shared__ int widest;
  if (wid == 0) {
    int carry = 0, wmax = 0;
    for (int r0 = 0; r0 <= nrows; r0 += 64) {
      const int r = r0 + lane;
      const int wdt = r < nrows ? f.spans[r].y - f.spans[r].x + 1 : 0;
      const int incl = (int)wave_inclusive_scan((uint32_t)wdt, lane);
      if (r <= nrows) rowbase[r] = carry + incl - wdt;
      carry += __shfl(incl, 63, 64);
      wmax = max(wmax, wdt);
    }
    for (int d = 32; d >= 1; d >>= 1) wmax = max(wmax, __shfl_xor(wmax, d, 64));
    if (lane == 0) widest = wmax;
  }
  __syncthreads();
  const int N = rowbase[nrows];
  const int nq = min(4, (widest + 63) >> 6);   // 64-tap slices of the widest row (<= 255)
  const bool staged = N <= stage_cap;
  constexpr int kPasses = KT == KEY_U8 ? 1 : 2;
  for (int i = (int)blockIdx.x; i < n; i += (int)gridDim.x) {
    const uint32_t idx = miss[i];
    const int y = (int)(idx / (uint32_t)f.w), x = (int)(idx - (uint32_t)y * (uint32_t)f.w);
    int target = f.rank;
    uint32_t prefix = 0;
    for (int pass = 0; pass < kPasses; ++pass) {
      const int sh = (kPasses - 1 - pass) * 8;
      hist[t] = 0;
      __syncthreads();
      if (pass == 1 && staged) {
        for (int j = t; j < N; j += 256) {
          const uint32_t v = stage[j];
          if ((v >> 8) == prefix) atomicAdd(&hist[v & 255u], 1u);
        }
      } else {
        // this wave's rows: wid, wid + 4, ...; kRows of them per batch, each
        // row read in nq slices of 64 taps, all loads of a batch in flight
        for (int b0 = wid; b0 < nrows; b0 += 4 * kRows) {
          uint32_t v[kRows][4];
          bool ok[kRows][4];
#pragma unroll
          for (int j = 0; j < kRows; ++j) {
            const int rr = b0 + 4 * j, r = min(rr, nrows - 1);
            const short2 sp = f.spans[r];
            const long long rowoff =
                (long long)remap(y + f.dy_min + r, f.h, f.boundary) * f.stride;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int dx = sp.x + lane + 64 * q;
              ok[j][q] = q < nq && rr < nrows && dx <= sp.y;
              v[j][q] = 0;
              if (q < nq) {   // uniform
                const int gx = remap(x + min(dx, (int)sp.y), f.w, f.boundary);
                v[j][q] = KT == KEY_U8
                              ? (uint32_t)static_cast<const uint8_t*>(f.img)[rowoff + gx]
                              : (uint32_t)static_cast<const uint16_t*>(f.img)[rowoff + gx];
              }
            }
          }
#pragma unroll
          for (int j = 0; j < kRows; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (ok[j][q]) {
                const int pos = rowbase[b0 + 4 * j] + lane + 64 * q;
                if (pass == 0 && staged) stage[pos] = (uint16_t)v[j][q];
                if (pass == 0 || (v[j][q] >> 8) == prefix)
                  atomicAdd(&hist[(v[j][q] >> sh) & 255u], 1u);
              }
        }
      }
      __syncthreads();
      if (wid == 0) {
        uint32_t h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) h[j] = hist[lane * 4 + j];
        const uint32_t sum = h[0] + h[1] + h[2] + h[3];
        uint32_t cum = wave_inclusive_scan(sum, lane) - sum;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // exactly one bin holds rank `target` (a non-empty one)
          if (cum <= (uint32_t)target && (uint32_t)target < cum + h[j]) {
            sel[0] = lane * 4 + j;
            sel[1] = (int)cum;
          }
          cum += h[j];
        }
      }
      __syncthreads();
      target -= sel[1];
      prefix = pass == 0 ? (uint32_t)sel[0] : ((prefix << 8) | (uint32_t)sel[0]);
      __syncthreads();   // sel and hist are rewritten by the next pass or pixel
    }
    if (t == 0) {
      const long long o = (long long)y * f.stride + x;
      if (KT == KEY_U8) static_cast<uint8_t*>(f.out)[o] = (uint8_t)prefix;
      else static_cast<uint16_t*>(f.out)[o] = (uint16_t)prefix;
    }
  }
}

// One wave per tile: tile bracket = union of the predicted brackets of the
// cells the tile covers, widened by `margin` (normalised units), rounded
// outward to keys and clamped to [0, maxval].  Block 0 also clears the
// fallback pixel count and the miss list.
__global__ __launch_bounds__(256) void bracket_kernel(const float* __restrict__ out, int hc,
                                                      int wc, int tw, int th, int tiles_x,
                                                      int ntiles, float maxval, float margin,
                                                      uint2* __restrict__ br,
                                                      unsigned long long* fail_px,
                                                      unsigned int* miss_count) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *fail_px = 0;
    *miss_count = 0;
  }
  const int tile = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), lane = threadIdx.x & 63;
  if (tile >= ntiles) return;   // uniform per wave
  const int tx0 = (tile % tiles_x) * tw, ty0 = (tile / tiles_x) * th;
  int c0 = tx0 / 8, c1 = min(wc, (tx0 + tw + 7) / 8);
  int r0 = ty0 / 8, r1 = min(hc, (ty0 + th + 7) / 8);
  // cells within kEdge of the image border see the convolutions' zero
  // padding and predict poorly; a tile with other cells ignores them (a
  // border pixel whose median then escapes is recomputed exactly)
  constexpr int kEdge = 4;
  const int ic0 = max(c0, kEdge), ic1 = min(c1, wc - kEdge);
  const int ir0 = max(r0, kEdge), ir1 = min(r1, hc - kEdge);
  if (ic0 < ic1 && ir0 < ir1) {
    c0 = ic0;
    c1 = ic1;
    r0 = ir0;
    r1 = ir1;
  }
  const int ncx = c1 - c0, ncell = ncx * (r1 - r0);
  float lo = 3.4e38f, hi = -3.4e38f;
  for (int i = lane; i < ncell; i += 64) {
    const int r = r0 + i / ncx, c = c0 + i % ncx;
    const float2 v = *reinterpret_cast<const float2*>(out + ((long long)r * wc + c) * 16);
    lo = fminf(lo, fminf(v.x, v.y));
    hi = fmaxf(hi, fmaxf(v.x, v.y));
  }
  for (int d = 32; d >= 1; d >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, d, 64));
    hi = fmaxf(hi, __shfl_xor(hi, d, 64));
  }
  if (lane == 0) {
    float L = floorf((lo - margin) * maxval), H = ceilf((hi + margin) * maxval);
    L = fminf(fmaxf(L, 0.f), maxval);
    H = fminf(fmaxf(H, 0.f), maxval);
    // empty, NaN, or wider than 0.3 of the value range: no bracket (lo > hi),
    // the tile goes straight to the plain pass
    if (!(L <= H) || H - L > 0.3f * maxval) br[tile] = make_uint2(1u, 0u);
    else br[tile] = make_uint2((unsigned)L, (unsigned)H);
  }
}

// Caller-supplied brackets: clear the fallback count and the miss list.
__global__ void clear_count_kernel(unsigned long long* fail_px, unsigned int* miss_count) {
  *fail_px = 0;
  *miss_count = 0;
}

}  // namespace mf

struct mf_learned {
  int dev = 0;
  float* p = nullptr;        // master parameters
  float* m = nullptr;
  float* v = nullptr;
  float* g = nullptr;
  uint16_t* wbf = nullptr;   // bf16 copy, same element offsets as p
  float margin = 0.0f;
  int step = 0;
  // cell workspace
  long long cells_cap = 0;
  int grid_w = 0, grid_h = 0;
  uint16_t* act[4] = {nullptr, nullptr, nullptr, nullptr};
  float* out = nullptr;
  float* tgt = nullptr;
  uint16_t* dout = nullptr;
  uint16_t* dbuf[2] = {nullptr, nullptr};
  uint16_t* wflip = nullptr;
  float* wsp = nullptr;
  long long wsp_floats = 0;
  float* loss_part = nullptr;
  // inference output (f32 [cells][16]) of the one-launch forward pass
  float* iout = nullptr;
  long long iout_cap = 0;
  // tile workspace
  long long tiles_cap = 0;
  uint2* brackets = nullptr;
  int* tile_fail = nullptr;
  // per-pixel misses: list of y * w + x, capacity miss_cap, count on device
  unsigned int* miss = nullptr;
  unsigned int* miss_count = nullptr;
  long long miss_cap = 0;
  unsigned long long* fail_px = nullptr;
};

namespace {

constexpr int kSegsPerBlock = 8;

void free_cells(mf_learned* n) {
  for (auto& a : n->act) (void)hipFree(a), a = nullptr;
  (void)hipFree(n->out);
  (void)hipFree(n->tgt);
  (void)hipFree(n->dout);
  (void)hipFree(n->dbuf[0]);
  (void)hipFree(n->dbuf[1]);
  (void)hipFree(n->wsp);
  (void)hipFree(n->loss_part);
  n->out = n->tgt = n->wsp = n->loss_part = nullptr;
  n->dout = n->dbuf[0] = n->dbuf[1] = nullptr;
  n->cells_cap = 0;
}

// Make sure the cell workspace fits an H x W cell grid.
int ensure_cells(mf_learned* n, int H, int W) {
  const long long cells = (long long)H * W;
  const long long wsf = std::max(mf_cnn_wgrad_workspace(H, W, 32, kSegsPerBlock),
                                 mf_cnn_wgrad_workspace(H, W, 16, kSegsPerBlock));
  if (cells <= n->cells_cap && wsf <= n->wsp_floats) {
    n->grid_w = W;
    n->grid_h = H;
    return MF_OK;
  }
  if (hipDeviceSynchronize() != hipSuccess) return MF_ERR_HIP;
  free_cells(n);
  bool ok = true;
  for (auto& a : n->act) ok = ok && hipMalloc(&a, cells * 32 * 2) == hipSuccess;
  ok = ok && hipMalloc(&n->out, cells * 16 * 4) == hipSuccess;
  ok = ok && hipMalloc(&n->tgt, cells * 2 * 4) == hipSuccess;
  ok = ok && hipMalloc(&n->dout, cells * 32 * 2) == hipSuccess;
  ok = ok && hipMalloc(&n->dbuf[0], cells * 32 * 2) == hipSuccess;
  ok = ok && hipMalloc(&n->dbuf[1], cells * 32 * 2) == hipSuccess;
  ok = ok && hipMalloc(&n->wsp, wsf * 4) == hipSuccess;
  ok = ok && hipMalloc(&n->loss_part, ((cells + 255) / 256) * 4) == hipSuccess;
  if (!ok) {
    free_cells(n);
    return MF_ERR_NOMEM;
  }
  n->cells_cap = cells;
  n->wsp_floats = wsf;
  n->grid_w = W;
  n->grid_h = H;
  return MF_OK;
}

int ensure_tiles(mf_learned* n, long long tiles) {
  if (tiles <= n->tiles_cap) return MF_OK;
  if (hipDeviceSynchronize() != hipSuccess) return MF_ERR_HIP;
  (void)hipFree(n->brackets);
  (void)hipFree(n->tile_fail);
  n->brackets = nullptr;
  n->tile_fail = nullptr;
  n->tiles_cap = 0;
  if (hipMalloc(&n->brackets, tiles * sizeof(uint2)) != hipSuccess ||
      hipMalloc(&n->tile_fail, tiles * sizeof(int)) != hipSuccess)
    return MF_ERR_NOMEM;
  n->tiles_cap = tiles;
  return MF_OK;
}

int ensure_miss(mf_learned* n, long long px) {
  if (px <= n->miss_cap) return MF_OK;
  if (hipDeviceSynchronize() != hipSuccess) return MF_ERR_HIP;
  (void)hipFree(n->miss);
  n->miss = nullptr;
  n->miss_cap = 0;
  if (hipMalloc(&n->miss, px * sizeof(unsigned int)) != hipSuccess) return MF_ERR_NOMEM;
  n->miss_cap = px;
  return MF_OK;
}

int footprint_radius(const mf_footprint* fp) {
  return std::max(std::max(-fp->dx_min, fp->dx_max), std::max(-fp->dy_min, fp->dy_max));
}

// Inference output buffer for an H x W cell grid.
int ensure_iout(mf_learned* n, long long cells) {
  if (cells <= n->iout_cap) return MF_OK;
  if (hipDeviceSynchronize() != hipSuccess) return MF_ERR_HIP;
  (void)hipFree(n->iout);
  n->iout = nullptr;
  n->iout_cap = 0;
  if (hipMalloc(&n->iout, cells * 16 * 4) != hipSuccess) return MF_ERR_NOMEM;
  n->iout_cap = cells;
  return MF_OK;
}

// Inference: the whole network in one launch; results in n->iout.
int net_infer(mf_learned* n, const void* img, int w, int h, size_t stride, int dtype, int radius,
              hipStream_t s) {
  const long long cells = (long long)((w + 7) / 8) * ((h + 7) / 8);
  int rc = ensure_iout(n, cells);
  if (rc) return rc;
  const void* wl[4];
  const float* bl[4];
  for (int l = 0; l < 4; ++l) {
    wl[l] = n->wbf + mf::kOffW[l];
    bl[l] = n->p + mf::kOffB[l];
  }
  return mf_cnn_net_forward(img, w, h, stride, dtype, radius, wl, bl, n->iout, s);
}

// Training forward pass over the cells of an image (every activation
// kept for the backward pass); results in n->out.
int net_forward(mf_learned* n, const void* img, int w, int h, size_t stride, int dtype,
                int radius, hipStream_t s) {
  const int H = (h + 7) / 8, W = (w + 7) / 8;
  int rc = ensure_cells(n, H, W);
  if (rc) return rc;
  if ((rc = mf_cnn_features(img, w, h, stride, dtype, radius, n->act[0], s))) return rc;
  for (int l = 0; l < 3; ++l)
    if ((rc = mf_cnn_conv_forward(n->act[l], H, W, n->wbf + mf::kOffW[l], n->p + mf::kOffB[l], 32,
                                  0, nullptr, n->act[l + 1], s)))
      return rc;
  return mf_cnn_conv_forward(n->act[3], H, W, n->wbf + mf::kOffW[3], n->p + mf::kOffB[3], 16, 1,
                             nullptr, n->out, s);
}

using BrKernel = void (*)(mf::ImageDesc, int*);
using FbKernel = void (*)(mf::ImageDesc, const int*, unsigned long long*, int);

template <int KT, int SHAPE>
void pick(const mf::ImageDesc& br, const mf::ImageDesc& fb, BrKernel* b, FbKernel* f) {
  switch (br.imax) {
    case 9: *b = mf::mf_bracket_tile_kernel<KT, SHAPE, 9>; break;
    case 17: *b = mf::mf_bracket_tile_kernel<KT, SHAPE, 17>; break;
    case 25: *b = mf::mf_bracket_tile_kernel<KT, SHAPE, 25>; break;
    default: *b = mf::mf_bracket_tile_kernel<KT, SHAPE, 0>; break;
  }
  if (fb.gs) {
    *f = mf::mf_fallback_gs_kernel<KT, SHAPE>;
    return;
  }
  switch (fb.imax) {
    case 9: *f = mf::mf_fallback_kernel<KT, SHAPE, 9>; break;
    case 17: *f = mf::mf_fallback_kernel<KT, SHAPE, 17>; break;
    case 25: *f = mf::mf_fallback_kernel<KT, SHAPE, 25>; break;
    default: *f = mf::mf_fallback_kernel<KT, SHAPE, 33>; break;
  }
}

// Tile plans of the learned path: the bracketed layout `br` on the tallest
// tile shape that fits LDS, and the plain layout `fb` of the pass over the
// tiles that fail.  The plain pass takes the plain filter's own plan for the
// image when its tiles split the bracketed tiles evenly (same width, a
// height dividing theirs: `ratio` fallback tiles per bracketed tile), so a
// pass over many failed tiles is as well balanced as the plain filter;
// otherwise the bracketed tiles' shape (LDS if it fits, else global
// scratch).  Measured on 2048x2048 uint16 (i.i.d. and natural-like, radius
// 16 and 32): bracketed tiles of the plain filter's shorter shape were
// slower than the tall ones (radius 32, i.i.d.: 417 against 383 us), and
// they fail on more pixels.
struct LearnedPlan {
  mf::ImageDesc br, fb;
  mf::DeviceInfo di;
  int dev;
  int ratio;
};

int learned_plan(int dtype, const mf_footprint* fp, int w, int h, LearnedPlan* lp) {
  if (hipGetDevice(&lp->dev) != hipSuccess) return MF_ERR_HIP;
  int rc = mf::device_info(lp->dev, &lp->di);
  if (rc) return rc;
  lp->ratio = 1;
  mf::ImageDesc own{};
  const bool have_own =
      w > 0 && h > 0 &&
      mf::choose_plan(dtype, fp, lp->di.lds_max, 33, &own, w, h, lp->di.cus) == MF_OK;
  mf::ImageDesc base{};
  if ((rc = mf::choose_plan_tall(dtype, fp, lp->di.lds_max, 33, &base))) return rc;
  if ((rc = mf::make_plan_br(dtype, fp, lp->di.lds_max, base.tw, base.th, &lp->br)))
    return rc;
  if (have_own && own.tw == base.tw && own.th <= base.th && base.th % own.th == 0) {
    lp->fb = own;
    lp->ratio = base.th / own.th;
    return MF_OK;
  }
  if (mf::make_plan(dtype, fp, lp->di.lds_max, base.tw, base.th, &lp->fb) != MF_OK ||
      lp->fb.imax > 33)
    if ((rc = mf::make_plan_gs(dtype, fp, lp->di.lds_max, base.tw, base.th, &lp->fb)))
      return rc;
  return MF_OK;
}

// Bracketed filter with per-tile brackets in `br` (the fallback count
// already cleared on `s`), then the plain pass over the flagged tiles.
int bracketed_filter(mf_learned* n, const uint2* br, const void* img, int w, int h,
                     size_t stride, int dtype, const mf_footprint* fp, int boundary, void* out,
                     unsigned long long* fallback_px, hipStream_t s, const LearnedPlan& lp) {
  if (lp.fb.nrows > mf::kSelMaxRows) return MF_ERR_UNSUPPORTED;   // (boxes are <= 256 tall)
  const void* table = nullptr;
  int rc = mf::footprint_device_table(fp, lp.dev, &table, s);
  if (rc) return rc;
  mf::ImageDesc a = lp.br, f = lp.fb;
  const int rank = (fp->taps - 1) / 2;
  mf::bind_image(&a, img, w, h, stride, dtype, fp, boundary, rank, table);
  mf::bind_image(&f, img, w, h, stride, dtype, fp, boundary, rank, table);
  a.out = f.out = out;
  a.brackets = br;
  a.miss = n->miss;
  a.miss_count = n->miss_count;
  a.counters = f.counters = mf::work_counters_ptr();
  const long long ntiles = (long long)a.tiles_x * a.tiles_y;
  BrKernel bk = nullptr;
  FbKernel fk = nullptr;
  if (dtype == MF_U8) {
    if (a.shape == mf::SHAPE_DISC) pick<mf::KEY_U8, mf::SHAPE_DISC>(a, f, &bk, &fk);
    else pick<mf::KEY_U8, mf::SHAPE_SPANS>(a, f, &bk, &fk);
  } else {
    if (a.shape == mf::SHAPE_DISC) pick<mf::KEY_U16, mf::SHAPE_DISC>(a, f, &bk, &fk);
    else pick<mf::KEY_U16, mf::SHAPE_SPANS>(a, f, &bk, &fk);
  }
  const long long fntiles = (long long)f.tiles_x * f.tiles_y;
  long long fgrid = fntiles;
  if (f.gs) {
    const int occ = std::max(1, std::min(2, lp.di.lds_max / std::max(1, f.lds_bytes)));
    fgrid = std::min<long long>(fntiles, (long long)lp.di.cus * occ);
    void* scr = nullptr;
    if ((rc = mf::get_scratch(lp.dev, s, (size_t)fgrid * (size_t)f.slot_bytes, &scr))) return rc;
    f.scratch = static_cast<unsigned char*>(scr);
  }
  (void)hipFuncSetAttribute((const void*)bk, hipFuncAttributeMaxDynamicSharedMemorySize,
                            a.lds_bytes);
  (void)hipFuncSetAttribute((const void*)fk, hipFuncAttributeMaxDynamicSharedMemorySize,
                            f.lds_bytes);
  hipLaunchKernelGGL(bk, dim3((unsigned)ntiles), dim3(mf::kThreads), a.lds_bytes, s, a,
                     n->tile_fail);
  hipLaunchKernelGGL(fk, dim3((unsigned)fgrid), dim3(mf::kThreads), f.lds_bytes, s, f,
                     (const int*)n->tile_fail, n->fail_px, lp.ratio);
  const long long pgrid = std::max(1, lp.di.cus) * 8LL;   // 8 pixels at a time per CU
  // staging buffer: the window's taps (the kernel stages windows of at most
  // kSelStage taps)
  const int stage_cap = fp->taps <= mf::kSelStage ? fp->taps : 0;
  const size_t stage_bytes = (size_t)stage_cap * 2;
  if (dtype == MF_U8)
    hipLaunchKernelGGL(mf::mf_pixel_select_kernel<mf::KEY_U8>, dim3((unsigned)pgrid), dim3(256),
                       stage_bytes, s, f, (const unsigned int*)n->miss,
                       (const unsigned int*)n->miss_count, n->fail_px, stage_cap);
  else
    hipLaunchKernelGGL(mf::mf_pixel_select_kernel<mf::KEY_U16>, dim3((unsigned)pgrid), dim3(256),
                       stage_bytes, s, f, (const unsigned int*)n->miss,
                       (const unsigned int*)n->miss_count, n->fail_px, stage_cap);
  if (hipGetLastError() != hipSuccess) return MF_ERR_HIP;
  if (fallback_px) {
    if (hipMemcpyAsync(fallback_px, n->fail_px, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return MF_ERR_HIP;
  }
  return MF_OK;
}

}  // namespace

extern "C" {

int mf_learned_param_count(void) { return mf::kParams; }

void mf_learned_destroy(mf_learned* n) {
  if (!n) return;
  (void)hipDeviceSynchronize();
  free_cells(n);
  (void)hipFree(n->p);
  (void)hipFree(n->m);
  (void)hipFree(n->v);
  (void)hipFree(n->g);
  (void)hipFree(n->wbf);
  (void)hipFree(n->wflip);
  (void)hipFree(n->brackets);
  (void)hipFree(n->tile_fail);
  (void)hipFree(n->fail_px);
  (void)hipFree(n->miss_count);
  (void)hipFree(n->miss);
  (void)hipFree(n->iout);
  delete n;
}

int mf_learned_set_params(mf_learned* n, const float* host) {
  if (!n || !host) return MF_ERR_INVALID_ARG;
  std::vector<uint16_t> bf(mf::kParams);
  for (int i = 0; i < mf::kParams; ++i) {
    uint32_t u;
    std::memcpy(&u, &host[i], 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    bf[i] = (uint16_t)(u >> 16);
  }
  if (hipMemcpy(n->p, host, mf::kParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(n->wbf, bf.data(), mf::kParams * 2, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(n->m, 0, mf::kParams * 4) != hipSuccess ||
      hipMemset(n->v, 0, mf::kParams * 4) != hipSuccess ||
      hipMemset(n->g, 0, mf::kParams * 4) != hipSuccess)
    return MF_ERR_HIP;
  n->step = 0;
  return MF_OK;
}

int mf_learned_get_params(const mf_learned* n, float* host) {
  if (!n || !host) return MF_ERR_INVALID_ARG;
  return hipMemcpy(host, n->p, mf::kParams * 4, hipMemcpyDeviceToHost) == hipSuccess ? MF_OK
                                                                                      : MF_ERR_HIP;
}

int mf_learned_get_grads(const mf_learned* n, float* host) {
  if (!n || !host) return MF_ERR_INVALID_ARG;
  return hipMemcpy(host, n->g, mf::kParams * 4, hipMemcpyDeviceToHost) == hipSuccess ? MF_OK
                                                                                      : MF_ERR_HIP;
}

int mf_learned_create(unsigned long long seed, mf_learned** out) {
  if (!out) return MF_ERR_INVALID_ARG;
  *out = nullptr;
  auto* n = new (std::nothrow) mf_learned;
  if (!n) return MF_ERR_NOMEM;
  if (hipGetDevice(&n->dev) != hipSuccess) {
    delete n;
    return MF_ERR_HIP;
  }
  if (hipMalloc(&n->p, mf::kParams * 4) != hipSuccess ||
      hipMalloc(&n->m, mf::kParams * 4) != hipSuccess ||
      hipMalloc(&n->v, mf::kParams * 4) != hipSuccess ||
      hipMalloc(&n->g, mf::kParams * 4) != hipSuccess ||
      hipMalloc(&n->wbf, mf::kParams * 2) != hipSuccess ||
      hipMalloc(&n->wflip, 32 * 9 * 32 * 2) != hipSuccess ||
      hipMalloc(&n->fail_px, sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&n->miss_count, sizeof(unsigned int)) != hipSuccess) {
    mf_learned_destroy(n);
    return MF_ERR_NOMEM;
  }
  // He-normal weights over the real fan-in (layer 1 sees 2 input channels),
  // zero biases except the output layer, which starts at the full range
  // (lo = 0, hi = 1) so an untrained net brackets everything.
  std::mt19937_64 rng(seed);
  std::vector<float> h(mf::kParams, 0.0f);
  for (int l = 0; l < 4; ++l) {
    const int cout = l == 3 ? 2 : 32, cin = l == 0 ? 2 : 32;
    std::normal_distribution<float> nd(0.0f, std::sqrt(2.0f / (9.0f * cin)) * (l == 3 ? 0.1f : 1.0f));
    for (int co = 0; co < cout; ++co)
      for (int t = 0; t < 9; ++t)
        for (int ci = 0; ci < cin; ++ci) h[mf::kOffW[l] + (co * 9 + t) * 32 + ci] = nd(rng);
  }
  h[mf::kOffB[3]] = 0.0f;
  h[mf::kOffB[3] + 1] = 1.0f;
  const int rc = mf_learned_set_params(n, h.data());
  if (rc) {
    mf_learned_destroy(n);
    return rc;
  }
  *out = n;
  return MF_OK;
}

int mf_learned_set_margin(mf_learned* n, float margin) {
  if (!n || !(margin >= 0.0f)) return MF_ERR_INVALID_ARG;
  n->margin = margin;
  return MF_OK;
}

int mf_learned_forward(mf_learned* n, const void* img, int w, int h, size_t stride_bytes,
                       int dtype, int radius, float* out_cells, hipStream_t s) {
  if (!n || !img || !out_cells || w <= 0 || h <= 0 || radius < 0 ||
      (dtype != MF_U8 && dtype != MF_U16))
    return MF_ERR_INVALID_ARG;
  int rc = net_infer(n, img, w, h, stride_bytes, dtype, radius, s);
  if (rc) return rc;
  const long long cells = (long long)((w + 7) / 8) * ((h + 7) / 8);
  return hipMemcpyAsync(out_cells, n->iout, cells * 16 * 4, hipMemcpyDeviceToDevice, s) ==
                 hipSuccess
             ? MF_OK
             : MF_ERR_HIP;
}

int mf_learned_train_step(mf_learned* n, const void* img, const void* median, int w, int h,
                          size_t stride_bytes, int dtype, int radius, float lr, float* loss,
                          hipStream_t s) {
  if (!n || !img || !median || w <= 0 || h <= 0 || !(lr > 0) ||
      (dtype != MF_U8 && dtype != MF_U16))
    return MF_ERR_INVALID_ARG;
  int rc = net_forward(n, img, w, h, stride_bytes, dtype, radius, s);
  if (rc) return rc;
  const int H = n->grid_h, W = n->grid_w;
  const int cells = H * W;
  if ((rc = mf_cnn_targets(median, w, h, stride_bytes, dtype, n->tgt, s))) return rc;
  if ((rc = mf_cnn_pinball(n->out, 16, n->tgt, cells, 0.02f, 0.98f, n->dout, n->loss_part, s)))
    return rc;
  // backward through the four layers
  const uint16_t* dcur = n->dout;
  for (int l = 3; l >= 0; --l) {
    const int cout = l == 3 ? 16 : 32;
    if ((rc = mf_cnn_conv_wgrad(n->act[l], dcur, H, W, cout, kSegsPerBlock, n->wsp,
                                n->g + mf::kOffW[l], n->g + mf::kOffB[l], s)))
      return rc;
    if (l == 0) break;
    uint16_t* dnext = n->dbuf[l & 1];
    if ((rc = mf_cnn_flip_weights(n->wbf + mf::kOffW[l], cout, n->wflip, s)) ||
        (rc = mf_cnn_conv_forward(dcur, H, W, n->wflip, nullptr, 32, 2, n->act[l], dnext, s)))
      return rc;
    dcur = dnext;
  }
  // zero the gradients of the unused output rows and input channels
  (void)hipMemsetAsync(n->g + mf::kOffW[3] + 2 * 9 * 32, 0, (16 - 2) * 9 * 32 * 4, s);
  (void)hipMemsetAsync(n->g + mf::kOffB[3] + 2, 0, 14 * 4, s);
  n->step += 1;
  if ((rc = mf_cnn_adam(n->p, n->m, n->v, n->g, mf::kParams, lr, 0.9f, 0.999f, 1e-8f, n->step,
                        n->wbf, s)))
    return rc;
  if (loss) {
    std::vector<float> part((cells + 255) / 256);
    if (hipMemcpyAsync(part.data(), n->loss_part, part.size() * 4, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return MF_ERR_HIP;
    double sum = 0;
    for (float f : part) sum += f;
    *loss = (float)(sum / cells);
  }
  return MF_OK;
}

int median_filter_bracketed(const void* img, int w, int h, size_t stride_bytes, int dtype,
                            const mf_footprint* fp, int boundary, const unsigned int* tile_brackets,
                            mf_learned* net, void* out, unsigned long long* fallback_px,
                            hipStream_t stream) {
  int rc = mf::validate_image(img, w, h, stride_bytes, dtype, fp, boundary, out);
  if (rc) return rc;
  if (!net || !tile_brackets || (dtype != MF_U8 && dtype != MF_U16)) return MF_ERR_INVALID_ARG;
  if (w == 0 || h == 0) {
    if (fallback_px) *fallback_px = 0;
    return MF_OK;
  }
  LearnedPlan lp;
  if ((rc = learned_plan(dtype, fp, w, h, &lp))) return rc;
  const long long ntiles =
      (long long)((w + lp.br.tw - 1) / lp.br.tw) * ((h + lp.br.th - 1) / lp.br.th);
  if (ntiles > 0x7fffffffLL) return MF_ERR_UNSUPPORTED;
  if ((long long)w * h > 0xffffffffLL) return MF_ERR_UNSUPPORTED;
  if ((rc = ensure_tiles(net, ntiles)) || (rc = ensure_miss(net, (long long)w * h))) return rc;
  hipLaunchKernelGGL(mf::clear_count_kernel, dim3(1), dim3(1), 0, stream, net->fail_px,
                     net->miss_count);
  if (hipGetLastError() != hipSuccess) return MF_ERR_HIP;
  return bracketed_filter(net, reinterpret_cast<const uint2*>(tile_brackets), img, w, h,
                          stride_bytes, dtype, fp, boundary, out, fallback_px, stream, lp);
}

int median_filter_learned(const void* img, int w, int h, size_t stride_bytes, int dtype,
                          const mf_footprint* fp, int boundary, mf_learned* net, void* out,
                          unsigned long long* fallback_px, hipStream_t stream) {
  int rc = mf::validate_image(img, w, h, stride_bytes, dtype, fp, boundary, out);
  if (rc) return rc;
  if (!net || (dtype != MF_U8 && dtype != MF_U16)) return MF_ERR_INVALID_ARG;
  if (w == 0 || h == 0) {
    if (fallback_px) *fallback_px = 0;
    return MF_OK;
  }
  LearnedPlan lp;
  if ((rc = learned_plan(dtype, fp, w, h, &lp))) return rc;
  const int tiles_x = (w + lp.br.tw - 1) / lp.br.tw, tiles_y = (h + lp.br.th - 1) / lp.br.th;
  const long long ntiles = (long long)tiles_x * tiles_y;
  if (ntiles > 0x7fffffffLL / 64 || (long long)w * h > 0xffffffffLL) return MF_ERR_UNSUPPORTED;
  if ((rc = ensure_tiles(net, ntiles)) || (rc = ensure_miss(net, (long long)w * h))) return rc;
  if ((rc = net_infer(net, img, w, h, stride_bytes, dtype, footprint_radius(fp), stream)))
    return rc;
  const float maxval = dtype == MF_U8 ? 255.0f : 65535.0f;
  hipLaunchKernelGGL(mf::bracket_kernel, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, stream,
                     net->iout, (h + 7) / 8, (w + 7) / 8, lp.br.tw, lp.br.th, tiles_x, (int)ntiles,
                     maxval, net->margin, net->brackets, net->fail_px, net->miss_count);
  if (hipGetLastError() != hipSuccess) return MF_ERR_HIP;
  return bracketed_filter(net, net->brackets, img, w, h, stride_bytes, dtype, fp, boundary, out,
                          fallback_px, stream, lp);
}

int mf_learned_tile_grid(int w, int h, int dtype, const mf_footprint* fp, int* tiles_x,
                         int* tiles_y, int* bracket_capacity, int* tile_w, int* tile_h) {
  if (!fp || w <= 0 || h <= 0 || (dtype != MF_U8 && dtype != MF_U16)) return MF_ERR_INVALID_ARG;
  LearnedPlan lp;
  const int rc = learned_plan(dtype, fp, w, h, &lp);
  if (rc) return rc;
  if (tiles_x) *tiles_x = (w + lp.br.tw - 1) / lp.br.tw;
  if (tiles_y) *tiles_y = (h + lp.br.th - 1) / lp.br.th;
  if (bracket_capacity) *bracket_capacity = lp.br.br_cap;
  if (tile_w) *tile_w = lp.br.tw;
  if (tile_h) *tile_h = lp.br.th;
  return MF_OK;
}

}  // extern "C"
