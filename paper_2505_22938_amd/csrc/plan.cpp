// Host-side planning: tile geometry, LDS and scratch layout, the tuned-shape
// table and its JSON cache, the per-(device, stream) scratch cache.
//
// A plan fixes the output tile (tw x th), the input box (tile grown by the
// window extent, paper "Method Summary" step 1: input tiles padded by the
// filter radius), the band layout of the 16 waves and where each per-tile
// structure lives.  Input boxes are limited to 255 x 256 pixels so a box
// location fits the omnigram's 8+8-bit encoding (paper, "Implementation":
// input tiles up to 256x256, 16-bit omnigram entries) and (255, 255) lies
// outside every box (the omnigram's padding location).

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mf_internal.h"

namespace mf {

namespace {

constexpr int kItemChoices[] = {9, 17, 25, 33};

int round_up(int x, int m) { return (x + m - 1) / m * m; }

std::mutex g_override_mu;
int g_tile_w = 0, g_tile_h = 0;

// Band layout shared by both variants; fills geometry fields.
int band_geometry(const mf_footprint* fp, int tw, int th, ImageDesc* d) {
  if (tw < 1 || tw > 64 || th < 1) return MF_ERR_UNSUPPORTED;
  const int segs = 64 / tw;                                // bands per wave
  const int R = (th + kWaves * segs - 1) / (kWaves * segs);   // rows per band
  const int bw = tw + fp->dx_max - fp->dx_min, bh = th + fp->dy_max - fp->dy_min;
  if (bw > 255 || bh > 256) return MF_ERR_UNSUPPORTED;
  const int T = bw * bh;
  if (T > 65535) return MF_ERR_UNSUPPORTED;
  // ordinal-image row pitch (16-bit elements): pitch/2 odd, so consecutive
  // rows start in different LDS banks
  int pitch = round_up(bw, 2);
  if ((pitch / 2) % 2 == 0) pitch += 2;
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
  d->dx_min = fp->dx_min;
  d->dy_min = fp->dy_min;
  d->nrows = (int)fp->row_lo.size();
  d->ncols = (int)fp->col_lo.size();
  d->limit = (int)fp->limit;
  d->shape = fp->kind == 0 ? SHAPE_DISC : SHAPE_SPANS;
  return MF_OK;
}

int table_bytes(const ImageDesc* d) {
  const int nr4 = round_up(d->nrows, 4);
  return 128 + 4 * nr4 + 8 * nr4 + 16 * d->ncols;   // scan words, spans, offsets
}

}  // namespace

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
    cache[dev].cus = prop.multiProcessorCount;
    have[dev] = true;
  }
  *out = cache[dev];
  return MF_OK;
}

int make_plan(int dtype, const mf_footprint* fp, int lds_max, int tw, int th, ImageDesc* d) {
  int rc = band_geometry(fp, tw, th, d);
  if (rc) return rc;
  const int T = d->T;
  const int need_items = ((T + kThreads - 1) / kThreads) | 1;
  int im = 0;
  for (int c : kItemChoices)
    if (need_items <= c) {
      im = c;
      break;
    }
  if (!im) return MF_ERR_UNSUPPORTED;
  // Region A: the sort exchange (u32 words; float keys: u32 keys, then a
  // 16-bit payload array).  After the sort it holds the omnigram (T + 16
  // padding entries, 16-bit) and the ordinal image, which takes the part of
  // the exchange buffer the omnigram leaves free.  The reverse map is not
  // kept: an output reads its value back from the image at the omnigram's
  // location.  Region B: digit counts during the sort, then the per-wave
  // seed histograms.
  const int TP = round_up(T, 8) + 16;
  const int ib = round_up(2 * d->pitch * d->bh, 16);
  const int hb = kHistBytes;
  int A;
  if (dtype == MF_F32) {
    const int kb = std::max(4 * (round_up(T, 4) + 4), ib);   // keys, then the ordinal image
    d->off_p = kb;                                          // payload = omnigram
    d->off_I = 0;
    A = kb + 2 * TP;
  } else {
    d->off_p = 0;
    d->off_I = 2 * TP;                                      // after the omnigram
    A = std::max(4 * TP, 2 * TP + ib);
  }
  d->off_C = 0;
  d->off_B = A;
  d->off_hist = A;
  d->off_tab = A + std::max(kCounterBytes, hb);
  d->lds_bytes = d->off_tab + table_bytes(d);
  d->kt = dtype;
  d->gs = 0;
  d->imax = im;
  d->slot_bytes = 0;
  d->off_x1 = d->off_lr = d->ipt = 0;
  if (d->lds_bytes > lds_max) return MF_ERR_UNSUPPORTED;
  return MF_OK;
}

int make_plan_br(int dtype, const mf_footprint* fp, int lds_max, int tw, int th, ImageDesc* d) {
  if (dtype != MF_U8 && dtype != MF_U16) return MF_ERR_UNSUPPORTED;
  int rc = band_geometry(fp, tw, th, d);
  if (rc) return rc;
  const int T = d->T;
  const int ib = round_up(2 * d->pitch * d->bh, 16);
  const int hb = kHistBytes;
  const int B = std::max(kCounterBytes, ib + hb);
  const int tb = table_bytes(d);
  // region A: TPc 32-bit words (candidate exchange), afterwards omega and C
  // (16-bit, ordinals 0..Tc plus 16 padding entries each)
  const int avail = lds_max - B - tb;
  if (avail <= 0) return MF_ERR_UNSUPPORTED;
  int cap = (avail / 4) - 32;
  cap = std::min(cap, std::min(T, 17 * kThreads));
  if (cap < kThreads) return MF_ERR_UNSUPPORTED;
  // Region A capped at a quarter of the box: a bracket holding more of the
  // box saves less than three quarters of the sort, and its tile goes to the
  // plain pass right after the load instead of ranking most of its box
  // twice (on smooth images most tiles are such); a tight bracket holds far
  // fewer pixels (about a tenth of the box on i.i.d. input).
  cap = std::min(cap, std::max(kThreads, T / 4));
  const int TPc = round_up(cap + 1, 8) + 16;
  d->off_p = 0;
  d->off_C = 2 * TPc;
  d->off_B = 4 * TPc;
  d->off_I = d->off_B;
  d->off_hist = d->off_B + ib;
  d->off_tab = d->off_B + B;
  d->lds_bytes = d->off_tab + tb;
  d->kt = dtype;
  d->gs = 0;
  // register-held box load for boxes of up to 25 pixels per thread, else
  // the box streams through LDS (imax 0)
  const int need_items = ((T + kThreads - 1) / kThreads) | 1;
  d->imax = need_items <= 9 ? 9 : need_items <= 17 ? 17 : need_items <= 25 ? 25 : 0;
  d->slot_bytes = 0;
  d->off_x1 = d->off_lr = d->ipt = 0;
  d->br_cap = cap;
  if (d->lds_bytes > lds_max) return MF_ERR_UNSUPPORTED;
  return MF_OK;
}

int make_plan_gs(int dtype, const mf_footprint* fp, int lds_max, int tw, int th, ImageDesc* d) {
  int rc = band_geometry(fp, tw, th, d);
  if (rc) return rc;
  const int T = d->T;
  const int TP = round_up(T, 8) + 16;
  const int ib = round_up(2 * d->pitch * d->bh, 16);
  const int hb = kHistBytes;
  const int B0 = std::max(kCounterBytes, ib + hb);
  // slot: 8/16-bit keys: the omnigram (TP u16 entries), written by the
  // counting pass.  Float keys: x0 and x1, TP 32-bit words each, for the
  // stable passes over the high key bits; the last pass writes the omnigram
  // over x0.  The output is read back from the image (no reverse map).
  // Region B also holds the sort's packed 16-bit key counters (2^16 of
  // them for 16-bit and float keys, 2^8 for 8-bit keys).
  const int B = std::max(B0, dtype == MF_U8 ? 512 : 131072);
  d->off_p = 0;
  d->off_C = 0;
  d->off_x1 = 4 * TP;
  d->off_lr = 0;
  d->slot_bytes = round_up(dtype == MF_F32 ? 8 * TP : 2 * TP, 256);
  d->ipt = (T + kThreads - 1) / kThreads;
  d->off_B = 0;
  d->off_I = 0;
  d->off_hist = ib;
  d->off_tab = B;
  d->lds_bytes = B + table_bytes(d);
  d->kt = dtype;
  d->gs = 1;
  d->imax = 0;
  if (d->lds_bytes > lds_max) return MF_ERR_UNSUPPORTED;
  return MF_OK;
}

void get_override(int* tw, int* th) {
  std::lock_guard<std::mutex> lock(g_override_mu);
  *tw = g_tile_w;
  *th = g_tile_h;
}

static int plan_shape(int dtype, const mf_footprint* fp, int lds_max, int imax_cap, int tw,
                      int th, ImageDesc* d) {
  if (make_plan(dtype, fp, lds_max, tw, th, d) == MF_OK && d->imax <= imax_cap) return MF_OK;
  return make_plan_gs(dtype, fp, lds_max, tw, th, d);
}

// Global-scratch plans (large windows): the tile shape with the least box
// amplification T / (tw * th) among shapes that keep at least 3/4 of the
// lanes and half of the waves busy in the band phase.  Widths need not
// divide 64 (a wave then owns one band and some lanes sit out).
int best_gs_plan(int dtype, const mf_footprint* fp, int lds_max, ImageDesc* d) {
  static const int tws[] = {64, 56, 54, 48, 32, 16, 8};
  static const int ths[] = {128, 112, 96, 80, 64, 56, 54, 48, 32, 16, 8};
  double best = 1e300;
  ImageDesc pick{};
  bool found = false;
  for (int w : tws) {
    const int segs = 64 / w;
    if (w * segs < 48) continue;
    for (int h : ths) {
      ImageDesc c{};
      if (make_plan_gs(dtype, fp, lds_max, w, h, &c) != MF_OK) continue;
      const int bands = (h + c.band_rows - 1) / c.band_rows;
      if (bands * 2 < kWaves * segs && h > kWaves) continue;
      const double amp = (double)c.T / ((double)w * h);
      if (amp < best) {
        best = amp;
        pick = c;
        found = true;
      }
    }
  }
  if (!found) return MF_ERR_UNSUPPORTED;
  *d = pick;
  return MF_OK;
}

// Tallest output tile for the default choice, by the window's extent e (its
// largest offset from the centre).  Small windows hold few members among
// the box's ordinals, so the omnigram walks between neighbouring outputs
// get longer as the box grows; measured on 2048^2 and 4096^2 images of
// every key type (smooth and i.i.d. content), the best heights are about
// 16 (e <= 1), 32 (e <= 3), 48 (e <= 5), 64 (e <= 16) and the tallest that
// fits beyond.
static int default_th_cap(const mf_footprint* fp) {
  const int e = std::max(std::max(fp->dx_max, -fp->dx_min), std::max(fp->dy_max, -fp->dy_min));
  if (e <= 1) return 16;
  if (e <= 3) return 32;
  if (e <= 5) return 48;
  if (e <= 16) return 64;
  return 128;
}

// The first LDS shape that fits (widest, then tallest first, heights up to
// th_cap), unless a global-scratch shape re-reads enough fewer box pixels
// per output pixel (small LDS tiles under large windows).  Measured
// crossover, as the ratio of the LDS plan's amplification to the
// global-scratch plan's: about 1.25 for 8/16-bit keys (4096^2 uint16 disc:
// radius 48, ratio 1.14, 1.91 ms in LDS against 2.06; radius 52, 1.27,
// 2.22 against 2.19; radius 56, 1.47, 2.56 against 2.33; radius 60, 3.15
// against 2.42) and about 1.7 for float keys, whose global-scratch sort
// has two more passes (3840x2160 float32 disc: radius 40, ratio 1.5, 1.07
// against 1.29 ms; radius 44, 1.68, 1.38 against 1.40).  fill_tiles > 0:
// a kept 64-wide LDS shape steps down in height (not below 64) while the
// image would have fewer tiles than that (fewer tiles per CU than needed
// to balance tiles of uneven cost).
static int default_plan(int dtype, const mf_footprint* fp, int lds_max, int imax_cap, int th_cap,
                        int w, int h, long long fill_tiles, ImageDesc* d) {
  ImageDesc gs{};
  const bool have_gs = best_gs_plan(dtype, fp, lds_max, &gs) == MF_OK;
  // a 64-wide global-scratch plan steps down in height (not below 64) while
  // the image would give fewer tiles than CUs (fill_tiles / 4): on 1024^2
  // uint16 natural-like, radius 56/64, 64x64 tiles take 0.22/0.28 ms against
  // 0.47/0.51 ms for the 128 tiles of 64x128; at 2048^2 (512 tiles of
  // 64x128) shorter tiles lose on i.i.d. input (radius 64: 0.76 ms for 64x64
  // against 0.59)
  if (have_gs && fill_tiles > 0 && gs.tw == 64) {
    auto tiles = [&](const ImageDesc& c) {
      return (long long)((w + c.tw - 1) / c.tw) * ((h + c.th - 1) / c.th);
    };
    for (int t2 = gs.th - 16; t2 >= 64 && tiles(gs) * 4 < fill_tiles; t2 -= 16) {
      ImageDesc c{};
      if (make_plan_gs(dtype, fp, lds_max, 64, t2, &c) == MF_OK) gs = c;
    }
  }
  auto finish = [&](ImageDesc* c) {
    const double amp = (double)c->T / ((double)c->tw * c->th);
    const double amp_gs = have_gs ? (double)gs.T / ((double)gs.tw * gs.th) : 1e300;
    if (amp > (dtype == MF_F32 ? 1.7 : 1.25) * amp_gs) *c = gs;
    return MF_OK;
  };
  // 64 wide, heights in steps of 16 (the tallest that fits is weighed
  // against the global-scratch plan before any step down)
  for (int th = th_cap; th >= 16; th -= 16) {
    if (make_plan(dtype, fp, lds_max, 64, th, d) != MF_OK || d->imax > imax_cap) continue;
    finish(d);
    if (d->gs) return MF_OK;
    if (fill_tiles > 0) {
      for (int t2 = th - 16; t2 >= 64; t2 -= 16) {
        const long long tiles = (long long)((w + 63) / 64) * ((h + d->th - 1) / d->th);
        if (tiles * 20 >= fill_tiles * 19) break;   // within 5 % of the target
        ImageDesc c{};
        if (make_plan(dtype, fp, lds_max, 64, t2, &c) == MF_OK && c.imax <= imax_cap) *d = c;
      }
    }
    return MF_OK;
  }
  // narrower tiles for windows whose 64-wide boxes do not fit
  static const int tws[] = {32, 16, 8};
  for (int tw : tws) {
    const int segs = 64 / tw;
    for (int R = 8; R >= 1; R /= 2)
      if (make_plan(dtype, fp, lds_max, tw, kWaves * segs * R, d) == MF_OK && d->imax <= imax_cap)
        return finish(d);
  }
  if (!have_gs) return MF_ERR_UNSUPPORTED;
  *d = gs;
  return MF_OK;
}

int choose_plan(int dtype, const mf_footprint* fp, int lds_max, int imax_cap, ImageDesc* d,
                int w, int h, int cus) {
  int tw = 0, th = 0;
  get_override(&tw, &th);
  if (tw > 0) return plan_shape(dtype, fp, lds_max, imax_cap, tw, th, d);
  if (tuned_shape(dtype, fp, &tw, &th) &&
      plan_shape(dtype, fp, lds_max, imax_cap, tw, th, d) == MF_OK)
    return MF_OK;
  const long long fill = w > 0 && h > 0 && cus > 0 ? 4LL * cus : 0;
  return default_plan(dtype, fp, lds_max, imax_cap, default_th_cap(fp), w, h, fill, d);
}

int choose_plan_tall(int dtype, const mf_footprint* fp, int lds_max, int imax_cap,
                     ImageDesc* d) {
  int tw = 0, th = 0;
  get_override(&tw, &th);
  if (tw > 0) return plan_shape(dtype, fp, lds_max, imax_cap, tw, th, d);
  return default_plan(dtype, fp, lds_max, imax_cap, 128, 0, 0, 0, d);
}

std::vector<ImageDesc> candidate_plans(int dtype, const mf_footprint* fp, int lds_max,
                                       int imax_cap) {
  std::vector<ImageDesc> out;
  static const int tws[] = {64, 32, 16, 8};
  auto add = [&](int w, int th) {
    ImageDesc d{};
    if (make_plan(dtype, fp, lds_max, w, th, &d) == MF_OK && d.imax <= imax_cap)
      out.push_back(d);
    else if (make_plan_gs(dtype, fp, lds_max, w, th, &d) == MF_OK)
      out.push_back(d);
  };
  for (int w : tws) {
    const int segs = 64 / w;
    for (int R = 1; R <= 16; R *= 2) add(w, kWaves * segs * R);
  }
  add(64, 48);
  add(64, 96);
  ImageDesc g{};
  if (best_gs_plan(dtype, fp, lds_max, &g) == MF_OK) {
    bool seen = false;
    for (const ImageDesc& c : out) seen = seen || (c.tw == g.tw && c.th == g.th && c.gs);
    if (!seen) out.push_back(g);
  }
  return out;
}

void bind_image(ImageDesc* d, const void* img, int w, int h, size_t stride_bytes, int dtype,
                const mf_footprint* fp, int boundary, int rank, const void* spans) {
  (void)fp;
  d->img = img;
  d->w = w;
  d->h = h;
  d->stride = (long long)(stride_bytes / (size_t)elem_size(dtype));
  d->boundary = boundary;
  d->tiles_x = (w + d->tw - 1) / d->tw;
  d->tiles_y = (h + d->th - 1) / d->th;
  d->rank = rank;
  d->spans = static_cast<const short2*>(spans);
  d->counters = nullptr;
  d->scratch = nullptr;
  d->brackets = nullptr;
  d->miss = nullptr;
  d->miss_count = nullptr;
}

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

// ------------------------------------------------------------------ scratch

namespace {
struct ScratchEntry {
  int dev;
  hipStream_t stream;
  void* ptr;
  size_t bytes;
  bool captured;   // a graph captured on the stream may still use ptr
};
std::mutex g_scratch_mu;
std::vector<ScratchEntry> g_scratch;
std::vector<std::pair<int, void*>> g_retired;   // outgrown but possibly captured
}  // namespace

// Cached per (device, stream).  A stream under graph capture never
// allocates: a buffer that is already large enough is used (and kept alive
// until mf_release_scratch, since the graph refers to it), anything else
// returns MF_ERR_UNSUPPORTED.  Outside capture a buffer that is too small is
// replaced; if a captured graph may refer to the old one it is retired, not
// freed.
int get_scratch(int dev, hipStream_t stream, size_t bytes, void** out) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap) != hipSuccess) return MF_ERR_HIP;
  const bool capturing = cap != hipStreamCaptureStatusNone;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  for (auto& e : g_scratch) {
    if (e.dev == dev && e.stream == stream) {
      if (e.bytes < bytes) {
        if (capturing) return MF_ERR_UNSUPPORTED;
        if (hipStreamSynchronize(stream) != hipSuccess) return MF_ERR_HIP;
        if (e.captured) g_retired.push_back({dev, e.ptr});
        else (void)hipFree(e.ptr);
        e.ptr = nullptr;
        e.bytes = 0;
        e.captured = false;
        if (hipMalloc(&e.ptr, kClaimBytes + bytes) != hipSuccess) return MF_ERR_NOMEM;
        if (hipMemsetAsync(e.ptr, 0, kClaimBytes, stream) != hipSuccess) return MF_ERR_HIP;
        e.bytes = bytes;
      }
      e.captured = e.captured || capturing;
      *out = static_cast<unsigned char*>(e.ptr) + kClaimBytes;
      return MF_OK;
    }
  }
  if (capturing) return MF_ERR_UNSUPPORTED;
  void* p = nullptr;
  if (hipMalloc(&p, kClaimBytes + bytes) != hipSuccess) return MF_ERR_NOMEM;
  if (hipMemsetAsync(p, 0, kClaimBytes, stream) != hipSuccess) {
    (void)hipFree(p);
    return MF_ERR_HIP;
  }
  g_scratch.push_back({dev, stream, p, bytes, false});
  *out = static_cast<unsigned char*>(p) + kClaimBytes;
  return MF_OK;
}

int release_scratch() {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return MF_ERR_HIP;
  if (hipDeviceSynchronize() != hipSuccess) return MF_ERR_HIP;
  int rc = MF_OK;
  auto drop = [&](int dev, void* ptr) {
    if (hipSetDevice(dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        hipFree(ptr) != hipSuccess)
      rc = MF_ERR_HIP;
  };
  for (auto& e : g_scratch) drop(e.dev, e.ptr);
  for (auto& r : g_retired) drop(r.first, r.second);
  g_scratch.clear();
  g_retired.clear();
  (void)hipSetDevice(cur);
  return rc;
}

// ------------------------------------------------------------------ tuning table

namespace {
struct Tuned {
  int tw, th;
  double ms;
};
std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tune;
}  // namespace

// Key: dtype, footprint kind, squared limit (discs), extents, taps and a
// hash of the spans, so different shapes never share an entry.
std::string tune_key(int dtype, const mf_footprint* fp) {
  unsigned long long h = 1469598103934665603ull;
  for (size_t i = 0; i < fp->row_lo.size(); ++i) {
    h = (h ^ (unsigned long long)(fp->row_lo[i] + 1024)) * 1099511628211ull;
    h = (h ^ (unsigned long long)(fp->row_hi[i] + 1024)) * 1099511628211ull;
  }
  char buf[192];
  std::snprintf(buf, sizeof buf, "%s/%s/L%lld/x%d:%d/y%d:%d/n%d/h%016llx",
                dtype == MF_U8 ? "u8" : dtype == MF_U16 ? "u16" : "f32",
                fp->kind == 0 ? "disc" : "spans", fp->kind == 0 ? fp->limit : -1LL, fp->dx_min,
                fp->dx_max, fp->dy_min, fp->dy_max, fp->taps, h);
  return buf;
}

bool tuned_shape(int dtype, const mf_footprint* fp, int* tw, int* th) {
  const std::string k = tune_key(dtype, fp);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(k);
  if (it == g_tune.end()) return false;
  *tw = it->second.tw;
  *th = it->second.th;
  return true;
}

void record_tuned_shape(int dtype, const mf_footprint* fp, int tw, int th, double ms) {
  const std::string k = tune_key(dtype, fp);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[k] = {tw, th, ms};
}

void erase_tuned_shape(int dtype, const mf_footprint* fp) {
  const std::string k = tune_key(dtype, fp);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.erase(k);
}

// Cache format: a JSON array with one object per line,
//   {"key": "<tune_key>", "tile_w": 64, "tile_h": 128, "ms": 2.16}
int tune_cache_load(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return MF_ERR_INVALID_ARG;
  char line[512];
  int n = 0;
  while (std::fgets(line, sizeof line, f)) {
    char key[256];
    int tw = 0, th = 0;
    double ms = 0;
    const char* p = std::strstr(line, "\"key\"");
    if (!p) continue;
    if (std::sscanf(p, "\"key\": \"%255[^\"]\", \"tile_w\": %d, \"tile_h\": %d, \"ms\": %lf", key,
                    &tw, &th, &ms) >= 3) {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      g_tune[key] = {tw, th, ms};
      ++n;
    }
  }
  std::fclose(f);
  return n >= 0 ? MF_OK : MF_ERR_INVALID_ARG;
}

int tune_cache_save(const char* path) {
  FILE* f = std::fopen(path, "w");
  if (!f) return MF_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  std::fprintf(f, "[\n");
  size_t i = 0;
  for (const auto& kv : g_tune) {
    std::fprintf(f, "  {\"key\": \"%s\", \"tile_w\": %d, \"tile_h\": %d, \"ms\": %.4f}%s\n",
                 kv.first.c_str(), kv.second.tw, kv.second.th, kv.second.ms,
                 ++i < g_tune.size() ? "," : "");
  }
  std::fprintf(f, "]\n");
  std::fclose(f);
  return MF_OK;
}

}  // namespace mf

extern "C" int mf_release_scratch(void) { return mf::release_scratch(); }

extern "C" int mf_set_tile_override(int tile_w, int tile_h) {
  if (tile_w < 0 || tile_h < 0 || (tile_w == 0) != (tile_h == 0)) return MF_ERR_INVALID_ARG;
  if (tile_w && (tile_w > 64 || tile_h > 256)) return MF_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(mf::g_override_mu);
  mf::g_tile_w = tile_w;
  mf::g_tile_h = tile_h;
  return MF_OK;
}
