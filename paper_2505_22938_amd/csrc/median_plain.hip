// Plain median filter: one workgroup per output tile.
//
// Per tile (paper, "Method Summary" and "GPU"):
//   1. load the input box = output tile grown by the window extent, with the
//      boundary rule applied, into registers;
//   2. ordinal transform: sort {key, location} in LDS, giving the reverse
//      map C (sorted keys) and the omnigram (sorted locations);
//   3. pivot/count sliding over bands of output rows with omnigram scans
//      (tile_engine.h);
//   4. write C[m] for the ordinal m found.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>

#include "mf_internal.h"
#include "tile_engine.h"

namespace mf {

template <int KT, int SHAPE, int IMAX>
__global__ __launch_bounds__(kThreads) void mf_plain_kernel(ImageDesc a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  tile_body<KT, SHAPE, IMAX>(a, blockIdx.x, smem);
}

// ---------------------------------------------------------------- host side

namespace {

constexpr int kItemChoices[] = {9, 17, 25, 33};

struct DeviceInfo {
  int lds_max = 0;
};

int device_info(int dev, DeviceInfo* out) {
  static std::mutex mu;
  static DeviceInfo cache[64];
  static bool have[64] = {};
  if (dev < 0 || dev >= 64) return MF_ERR_HIP;
  std::lock_guard<std::mutex> lock(mu);
  if (!have[dev]) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MF_ERR_HIP;
    cache[dev].lds_max = (int)prop.sharedMemPerBlock;
    have[dev] = true;
  }
  *out = cache[dev];
  return MF_OK;
}

std::mutex g_override_mu;
int g_tile_w = 0, g_tile_h = 0;

int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace

// Fill the geometry and LDS layout of `d` for an output tile of tw x th.
int make_plan(int dtype, const mf_footprint* fp, int lds_max, int tw, int th, ImageDesc* d,
              int* imax) {
  if (tw < 1 || tw > 64 || 64 % tw) return MF_ERR_UNSUPPORTED;
  const int segs = 64 / tw;
  if (th % (kWaves * segs)) return MF_ERR_UNSUPPORTED;
  const int R = th / (kWaves * segs);
  if (R < 1) return MF_ERR_UNSUPPORTED;
  const int ext_x = fp->dx_max - fp->dx_min, ext_y = fp->dy_max - fp->dy_min;
  const int bw = tw + ext_x, bh = th + ext_y;
  if (bw > 255 || bh > 256) return MF_ERR_UNSUPPORTED;   // (255, 255) must lie outside the box
  const int T = bw * bh;
  const int need_items = ((T + kThreads - 1) / kThreads) | 1;
  int im = 0;
  for (int c : kItemChoices)
    if (need_items <= c) {
      im = c;
      break;
    }
  if (!im) return MF_ERR_UNSUPPORTED;
  // ordinal-image row pitch (16-bit elements): pitch/2 odd, so consecutive
  // rows start in different LDS banks
  int pitch = round_up(bw, 2);
  if ((pitch / 2) % 2 == 0) pitch += 2;
  const int nrows = (int)fp->row_lo.size(), ncols = (int)fp->col_lo.size();
  // region A: sort exchange (4T); afterwards the omnigram (2T) and the
  // reverse map (2T) for 8/16-bit keys, or keys (4T) + locations (2T) for
  // float keys.  Region B: digit counts during the sort, then the ordinal
  // image and the per-wave seed histograms.
  // omega and C each hold T entries plus 16 padding entries, 16-byte aligned
  const int TP = round_up(T, 8) + 16;
  const int kb = dtype == MF_F32 ? 4 * round_up(T, 4) : 4 * TP;
  const int pb = dtype == MF_F32 ? 2 * TP : 0;
  const int ib = round_up(2 * pitch * bh, 16);
  const int hb = kWaves * 128 * 4;
  const int B = std::max(kCounterBytes, ib + hb);
  const int nr4 = round_up(nrows, 4);
  const int tab = 64 + 4 * nr4 + 8 * nr4 + 16 * ncols;
  d->tw = tw;
  d->th = th;
  d->bw = bw;
  d->bh = bh;
  d->T = T;
  d->pitch = pitch;
  d->segs = segs;
  d->band_rows = R;
  int hs = 0;
  while (((T - 1) >> hs) >= 256) ++hs;
  d->hist_shift = hs;
  d->off_p = kb;
  d->off_C = 2 * TP;
  d->off_B = kb + pb;
  d->off_hist = d->off_B + ib;
  d->off_tab = d->off_B + B;
  d->lds_bytes = d->off_tab + tab;
  d->dx_min = fp->dx_min;
  d->dy_min = fp->dy_min;
  d->nrows = nrows;
  d->ncols = ncols;
  d->limit = (int)fp->limit;
  *imax = im;
  if (d->lds_bytes > lds_max) return MF_ERR_UNSUPPORTED;
  return MF_OK;
}

// Automatic tile shape: the widest band layout that fits, preferring taller
// bands (fewer seed rows per output pixel) up to 8 rows.
int choose_plan(int dtype, const mf_footprint* fp, int lds_max, ImageDesc* d, int* imax) {
  {
    std::lock_guard<std::mutex> lock(g_override_mu);
    if (g_tile_w > 0) return make_plan(dtype, fp, lds_max, g_tile_w, g_tile_h, d, imax);
  }
  static const int tws[] = {64, 32, 16, 8};
  for (int tw : tws) {
    const int segs = 64 / tw;
    for (int R = 8; R >= 1; R /= 2)
      if (make_plan(dtype, fp, lds_max, tw, kWaves * segs * R, d, imax) == MF_OK) return MF_OK;
  }
  return MF_ERR_UNSUPPORTED;
}

namespace {

using KernelFn = void (*)(ImageDesc);

template <int KT, int SHAPE>
KernelFn pick_imax(int imax) {
  switch (imax) {
    case 9: return mf_plain_kernel<KT, SHAPE, 9>;
    case 17: return mf_plain_kernel<KT, SHAPE, 17>;
    case 25: return mf_plain_kernel<KT, SHAPE, 25>;
    default: return mf_plain_kernel<KT, SHAPE, 33>;
  }
}

KernelFn pick_kernel(int dtype, int shape, int imax) {
  if (dtype == MF_U8) return shape == SHAPE_DISC ? pick_imax<KEY_U8, SHAPE_DISC>(imax)
                                                 : pick_imax<KEY_U8, SHAPE_SPANS>(imax);
  if (dtype == MF_U16) return shape == SHAPE_DISC ? pick_imax<KEY_U16, SHAPE_DISC>(imax)
                                                  : pick_imax<KEY_U16, SHAPE_SPANS>(imax);
  return shape == SHAPE_DISC ? pick_imax<KEY_F32, SHAPE_DISC>(imax)
                             : pick_imax<KEY_F32, SHAPE_SPANS>(imax);
}

unsigned long long* g_counters = nullptr;  // device work counters, enabled on request

}  // namespace

int validate_image(const void* img, int w, int h, size_t stride_bytes, int dtype,
                   const mf_footprint* fp, int boundary, const void* out) {
  if (dtype != MF_U8 && dtype != MF_U16 && dtype != MF_F32) return MF_ERR_INVALID_ARG;
  if (boundary != MF_CLAMP && boundary != MF_MIRROR) return MF_ERR_INVALID_ARG;
  if (!fp || w < 0 || h < 0) return MF_ERR_INVALID_ARG;
  if (w == 0 || h == 0) return MF_OK;
  if (!img || !out) return MF_ERR_INVALID_ARG;
  const size_t es = (size_t)elem_size(dtype);
  if (stride_bytes < (size_t)w * es || stride_bytes % es) return MF_ERR_INVALID_ARG;
  const size_t span = stride_bytes * (size_t)(h - 1) + (size_t)w * es;
  const uintptr_t a0 = (uintptr_t)img, b0 = (uintptr_t)out;
  if (a0 < b0 + span && b0 < a0 + span) return MF_ERR_ALIAS;
  return MF_OK;
}

int launch_plain(const void* img, int w, int h, size_t stride_bytes, int dtype,
                 const mf_footprint* fp, int boundary, int rank, void* out, hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MF_ERR_HIP;
  DeviceInfo di;
  int rc = device_info(dev, &di);
  if (rc) return rc;
  const void* table = nullptr;
  rc = footprint_device_table(fp, dev, &table);
  if (rc) return rc;
  ImageDesc a{};
  int imax = 0;
  rc = choose_plan(dtype, fp, di.lds_max, &a, &imax);
  if (rc) return rc;
  a.img = img;
  a.out = out;
  a.stride = (long long)(stride_bytes / (size_t)elem_size(dtype));
  a.w = w;
  a.h = h;
  a.boundary = boundary;
  a.tiles_x = (w + a.tw - 1) / a.tw;
  a.tiles_y = (h + a.th - 1) / a.th;
  a.rank = rank;
  a.spans = static_cast<const short2*>(table);
  a.counters = g_counters;
  const int shape = fp->kind == 0 ? SHAPE_DISC : SHAPE_SPANS;
  KernelFn k = pick_kernel(dtype, shape, imax);
  (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                            a.lds_bytes);
  const long long ntiles = (long long)a.tiles_x * a.tiles_y;
  if (ntiles > 0x7fffffffLL) return MF_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(kThreads), a.lds_bytes, stream, a);
  if (hipGetLastError() != hipSuccess) return MF_ERR_HIP;
  return MF_OK;
}

int query_plan(int dtype, const mf_footprint* fp, ImageDesc* d, int* imax) {
  int dev = 0;
  DeviceInfo di;
  if (hipGetDevice(&dev) != hipSuccess || device_info(dev, &di) != MF_OK) di.lds_max = 160 * 1024;
  return choose_plan(dtype, fp, di.lds_max, d, imax);
}

int set_counters(int enable) {
  if (enable && !g_counters) {
    if (hipMalloc(&g_counters, CNT_SLOTS * sizeof(unsigned long long)) != hipSuccess) {
      g_counters = nullptr;
      return MF_ERR_NOMEM;
    }
  }
  if (g_counters && hipMemset(g_counters, 0, CNT_SLOTS * sizeof(unsigned long long)) != hipSuccess)
    return MF_ERR_HIP;
  if (!enable && g_counters) {
    (void)hipFree(g_counters);
    g_counters = nullptr;
  }
  return MF_OK;
}

int read_counters(unsigned long long* host) {
  if (!g_counters) return MF_ERR_INVALID_ARG;
  if (hipMemcpy(host, g_counters, CNT_SLOTS * sizeof(unsigned long long),
                hipMemcpyDeviceToHost) != hipSuccess)
    return MF_ERR_HIP;
  return MF_OK;
}

}  // namespace mf

extern "C" {

const char* mf_status_string(int s) {
  switch (s) {
    case MF_OK: return "MF_OK";
    case MF_ERR_INVALID_ARG: return "MF_ERR_INVALID_ARG";
    case MF_ERR_ALIAS: return "MF_ERR_ALIAS";
    case MF_ERR_UNSUPPORTED: return "MF_ERR_UNSUPPORTED";
    case MF_ERR_NOMEM: return "MF_ERR_NOMEM";
    case MF_ERR_HIP: return "MF_ERR_HIP";
    default: return "MF_ERR_UNKNOWN";
  }
}

int median_filter_rank(const void* img, int w, int h, size_t stride_bytes, int dtype,
                       const mf_footprint* fp, int boundary, int rank, void* out,
                       hipStream_t stream) {
  int rc = mf::validate_image(img, w, h, stride_bytes, dtype, fp, boundary, out);
  if (rc != MF_OK) return rc;
  if (rank < 0 || rank >= fp->taps) return MF_ERR_INVALID_ARG;
  if (w == 0 || h == 0) return MF_OK;
  return mf::launch_plain(img, w, h, stride_bytes, dtype, fp, boundary, rank, out, stream);
}

int median_filter(const void* img, int w, int h, size_t stride_bytes, int dtype,
                  const mf_footprint* fp, int boundary, void* out, hipStream_t stream) {
  if (!fp) return MF_ERR_INVALID_ARG;
  return median_filter_rank(img, w, h, stride_bytes, dtype, fp, boundary, (fp->taps - 1) / 2,
                            out, stream);
}

int mf_set_tile_override(int tile_w, int tile_h) {
  if (tile_w < 0 || tile_h < 0 || (tile_w == 0) != (tile_h == 0)) return MF_ERR_INVALID_ARG;
  if (tile_w && (tile_w > 64 || 64 % tile_w || tile_w < 8 || tile_h > 256 ||
                 tile_h % (16 * (64 / tile_w))))
    return MF_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(mf::g_override_mu);
  mf::g_tile_w = tile_w;
  mf::g_tile_h = tile_h;
  return MF_OK;
}

int mf_query_plan(int w, int h, int dtype, const mf_footprint* fp, int* tile_w, int* tile_h,
                  int* box_w, int* box_h, int* lds) {
  (void)w;
  (void)h;
  if (!fp || (dtype != MF_U8 && dtype != MF_U16 && dtype != MF_F32)) return MF_ERR_INVALID_ARG;
  mf::ImageDesc d{};
  int imax = 0;
  const int rc = mf::query_plan(dtype, fp, &d, &imax);
  if (rc) return rc;
  if (tile_w) *tile_w = d.tw;
  if (tile_h) *tile_h = d.th;
  if (box_w) *box_w = d.bw;
  if (box_h) *box_h = d.bh;
  if (lds) *lds = d.lds_bytes;
  return MF_OK;
}

int mf_work_counters(int enable, unsigned long long* out8) {
  if (enable < 0) return out8 ? mf::read_counters(out8) : MF_ERR_INVALID_ARG;
  return mf::set_counters(enable);
}

}  // extern "C"
