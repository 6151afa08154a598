// Plain median filter: one workgroup per output tile.
//
// Per tile (paper, "Method Summary" and "GPU"):
//   1. load the input box = output tile grown by the window extent, with the
//      boundary rule applied, into registers;
//   2. ordinal transform: sort {key, location} in LDS, giving the reverse
//      map C (sorted keys) and the omnigram (sorted locations);
//   3. solve each output pixel's rank by scanning the omnigram in blocks of
//      64 ordinals: one wave tests 64 omnigram entries against the window
//      (Eq. 3 or a span lookup), ballots them into a 64-bit mask and counts
//      it with popcount (paper, "Implementation": the 64-element bitmask and
//      popcount refinement);
//   4. write C[m] for the ordinal m found.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>

#include "mf_internal.h"
#include "tile_common.h"

namespace mf {

struct PlainArgs {
  const void* img;
  void* out;
  long long stride;  // elements
  int w, h, boundary;
  int tw, th, tiles_x;
  int bw, bh, T, items;
  int dx_min, dy_min, nrows;
  int rank;
  int limit;                 // disc: dx^2 + dy^2 <= limit
  const short2* spans;       // row spans, index dy - dy_min
};

template <int SHAPE>
__device__ __forceinline__ bool member(int ox, int oy, int nrows, int dy_min, int limit,
                                       const short2* sp) {
  if (SHAPE == SHAPE_DISC) return ox * ox + oy * oy <= limit;
  const int r = oy - dy_min;
  if ((unsigned)r >= (unsigned)nrows) return false;
  const short2 s = sp[r];
  return ox >= s.x && ox <= s.y;
}

template <int KT, int SHAPE, int IMAX>
__global__ __launch_bounds__(kThreads) void mf_plain_scan_kernel(PlainArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int T = a.T;
  uint32_t* kbuf = reinterpret_cast<uint32_t*>(smem);                         // 4T
  uint16_t* pbuf = reinterpret_cast<uint16_t*>(smem + 4 * ((T + 3) & ~3));  // 2T (f32)
  unsigned char* after = smem + 4 * ((T + 3) & ~3) + (KT == KEY_F32 ? 2 * ((T + 7) & ~7) : 0);
  uint16_t* cnt = reinterpret_cast<uint16_t*>(after);                        // kCounterBytes
  uint32_t* wsum = reinterpret_cast<uint32_t*>(after + kCounterBytes);       // kWaves
  short2* sp = reinterpret_cast<short2*>(after + kCounterBytes + 4 * kWaves);

  const int t = threadIdx.x;
  const int tile = blockIdx.x;
  const int tx0 = (tile % a.tiles_x) * a.tw, ty0 = (tile / a.tiles_x) * a.th;
  const int gx0 = tx0 + a.dx_min, gy0 = ty0 + a.dy_min;

  if (SHAPE == SHAPE_SPANS)
    for (int i = t; i < a.nrows; i += kThreads) sp[i] = a.spans[i];

  // 1. load the box, striped: element e = i*kThreads + t, row-major in the box
  uint32_t key[IMAX];
  uint16_t pos[IMAX];
  {
    int lx = t % a.bw, ly = t / a.bw;
    const int sx = kThreads % a.bw, sy = kThreads / a.bw;
#pragma unroll
    for (int i = 0; i < IMAX; ++i) {
      const int e = i * kThreads + t;
      uint32_t k = 0, q = 0;
      if (e < T) {
        const int gx = remap(gx0 + lx, a.w, a.boundary);
        const int gy = remap(gy0 + ly, a.h, a.boundary);
        const long long off = (long long)gy * a.stride + gx;
        const uint32_t p = (uint32_t)((ly << 8) | lx);
        if (KT == KEY_U8) k = ((uint32_t)static_cast<const uint8_t*>(a.img)[off] << 16) | p;
        if (KT == KEY_U16) k = ((uint32_t)static_cast<const uint16_t*>(a.img)[off] << 16) | p;
        if (KT == KEY_F32) {
          k = f32_to_key(static_cast<const uint32_t*>(a.img)[off]);
          q = p;
        }
      }
      key[i] = k;
      pos[i] = (uint16_t)q;
      lx += sx;
      ly += sy;
      if (lx >= a.bw) {
        lx -= a.bw;
        ly += 1;
      }
    }
  }

  // 2. ordinal transform
  if (KT == KEY_U8)
    block_radix_sort<IMAX, false>(key, pos, T, 16, 2, kbuf, pbuf, cnt, wsum);
  else if (KT == KEY_U16)
    block_radix_sort<IMAX, false>(key, pos, T, 16, 4, kbuf, pbuf, cnt, wsum);
  else
    block_radix_sort<IMAX, true>(key, pos, T, 0, 8, kbuf, pbuf, cnt, wsum);

  // 3. rank selection by omnigram scan, one output pixel per wave at a time
  const int lane = t & 63, wid = t >> 6;
  const int nblk = (T + 63) >> 6;
  const int npix = a.tw * a.th;
  for (int p = wid; p < npix; p += kWaves) {
    const int ox = p % a.tw, oy = p / a.tw;
    const int gx = tx0 + ox, gy = ty0 + oy;
    if (gx >= a.w || gy >= a.h) continue;
    const int cx = ox - a.dx_min, cy = oy - a.dy_min;
    int need = a.rank;
    for (int b = 0; b < nblk; ++b) {
      const int v = (b << 6) + lane;
      bool in = false;
      if (v < T) {
        const uint32_t loc = KT == KEY_F32 ? (uint32_t)pbuf[v] : (kbuf[v] & 0xffffu);
        in = member<SHAPE>((int)(loc & 255u) - cx, (int)(loc >> 8) - cy, a.nrows, a.dy_min,
                           a.limit, sp);
      }
      const uint64_t mask = __ballot(in);
      const int pc = __popcll(mask);
      if (need < pc) {
        const int below = __popcll(mask & ((1ull << lane) - 1ull));
        const uint64_t hit = __ballot(in && below == need);
        const int m = (b << 6) + (__ffsll((unsigned long long)hit) - 1);
        if (lane == 0) {
          const long long o = (long long)gy * a.stride + gx;
          if (KT == KEY_U8) static_cast<uint8_t*>(a.out)[o] = (uint8_t)(kbuf[m] >> 16);
          if (KT == KEY_U16) static_cast<uint16_t*>(a.out)[o] = (uint16_t)(kbuf[m] >> 16);
          if (KT == KEY_F32) static_cast<uint32_t*>(a.out)[o] = key_to_f32(kbuf[m]);
        }
        break;
      }
      need -= pc;
    }
  }
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

struct Plan {
  int tw, th, bw, bh, T, items, imax, lds;
};

int lds_bytes(int T, int dtype, int nrows) {
  const int a = 4 * ((T + 3) & ~3) + (dtype == MF_F32 ? 2 * ((T + 7) & ~7) : 0);
  return a + kCounterBytes + 4 * kWaves + 4 * nrows;
}

int plan_for(int dtype, const mf_footprint* fp, int lds_max, int tw, int th, Plan* p) {
  const int ext_x = fp->dx_max - fp->dx_min, ext_y = fp->dy_max - fp->dy_min;
  p->tw = tw;
  p->th = th;
  p->bw = tw + ext_x;
  p->bh = th + ext_y;
  if (p->bw > 256 || p->bh > 256) return MF_ERR_UNSUPPORTED;
  p->T = p->bw * p->bh;
  int items = (p->T + kThreads - 1) / kThreads;
  items |= 1;
  p->items = items;
  p->imax = 0;
  for (int c : kItemChoices)
    if (items <= c) {
      p->imax = c;
      break;
    }
  if (!p->imax) return MF_ERR_UNSUPPORTED;
  p->lds = lds_bytes(p->T, dtype, (int)fp->row_lo.size());
  if (p->lds > lds_max) return MF_ERR_UNSUPPORTED;
  return MF_OK;
}

int choose_plan(int w, int h, int dtype, const mf_footprint* fp, int lds_max, Plan* p) {
  {
    std::lock_guard<std::mutex> lock(g_override_mu);
    if (g_tile_w > 0) return plan_for(dtype, fp, lds_max, g_tile_w, g_tile_h, p);
  }
  (void)w;
  (void)h;
  static const int sizes[] = {64, 56, 48, 40, 32, 24, 16, 8};
  for (int s : sizes)
    if (plan_for(dtype, fp, lds_max, s, s, p) == MF_OK) return MF_OK;
  return MF_ERR_UNSUPPORTED;
}

using KernelFn = void (*)(PlainArgs);

template <int KT, int SHAPE>
KernelFn pick_imax(int imax) {
  switch (imax) {
    case 9: return mf_plain_scan_kernel<KT, SHAPE, 9>;
    case 17: return mf_plain_scan_kernel<KT, SHAPE, 17>;
    case 25: return mf_plain_scan_kernel<KT, SHAPE, 25>;
    default: return mf_plain_scan_kernel<KT, SHAPE, 33>;
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
  Plan p;
  rc = choose_plan(w, h, dtype, fp, di.lds_max, &p);
  if (rc) return rc;

  PlainArgs a;
  a.img = img;
  a.out = out;
  a.stride = (long long)(stride_bytes / (size_t)elem_size(dtype));
  a.w = w;
  a.h = h;
  a.boundary = boundary;
  a.tw = p.tw;
  a.th = p.th;
  a.tiles_x = (w + p.tw - 1) / p.tw;
  const int tiles_y = (h + p.th - 1) / p.th;
  a.bw = p.bw;
  a.bh = p.bh;
  a.T = p.T;
  a.items = p.items;
  a.dx_min = fp->dx_min;
  a.dy_min = fp->dy_min;
  a.nrows = (int)fp->row_lo.size();
  a.rank = rank;
  a.limit = (int)fp->limit;
  a.spans = static_cast<const short2*>(table);
  const int shape = fp->kind == 0 ? SHAPE_DISC : SHAPE_SPANS;
  KernelFn k = pick_kernel(dtype, shape, p.imax);
  (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, p.lds);
  const long long ntiles = (long long)a.tiles_x * tiles_y;
  if (ntiles > 0x7fffffffLL) return MF_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(kThreads), p.lds, stream, a);
  if (hipGetLastError() != hipSuccess) return MF_ERR_HIP;
  return MF_OK;
}

int query_plan(int w, int h, int dtype, const mf_footprint* fp, Plan* p) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  DeviceInfo di;
  if (dev < 0 || device_info(dev, &di) != MF_OK) di.lds_max = 160 * 1024;
  return choose_plan(w, h, dtype, fp, di.lds_max, p);
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
  if (tile_w && (tile_w % 8 || tile_h % 8 || tile_w > 64 || tile_h > 256))
    return MF_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(mf::g_override_mu);
  mf::g_tile_w = tile_w;
  mf::g_tile_h = tile_h;
  return MF_OK;
}

int mf_query_plan(int w, int h, int dtype, const mf_footprint* fp, int* tile_w, int* tile_h,
                  int* box_w, int* box_h, int* lds) {
  if (!fp || (dtype != MF_U8 && dtype != MF_U16 && dtype != MF_F32)) return MF_ERR_INVALID_ARG;
  mf::Plan p;
  const int rc = mf::query_plan(w, h, dtype, fp, &p);
  if (rc) return rc;
  if (tile_w) *tile_w = p.tw;
  if (tile_h) *tile_h = p.th;
  if (box_w) *box_w = p.bw;
  if (box_h) *box_h = p.bh;
  if (lds) *lds = p.lds;
  return MF_OK;
}

}  // extern "C"
