// General rank outputs: several rank planes from one ordinal transform per
// tile, each at a constant rank or at a rank given per pixel.
//
// The paper's filter is a general percentile filter (Conclusion); its
// discussion of multi-parameter filtering notes that one ordinal transform
// can serve several percentiles (e.g. the 25th, 50th and 75th), and its
// varying-percentile figure lets the percentile change across the image.
// Here the tile body sorts the box once and then runs its bands once per
// requested plane (tile_engine.h, GEN); a pixel's rank only changes the
// target of the omnigram scans, so sliding and counting are unchanged.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "mf_internal.h"
#include "tile_engine.h"

namespace mf {

template <int KT, int SHAPE, int IMAX>
__global__ __launch_bounds__(kThreads) void mf_general_kernel(ImageDesc a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  tile_body<KT, SHAPE, IMAX, false, false, true>(a, xcd_tile(blockIdx.x, gridDim.x), smem,
                                                 nullptr);
}

template <int KT, int SHAPE>
__global__ __launch_bounds__(kThreads) void mf_general_gs_kernel(ImageDesc a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int claimed;
  unsigned char* slot = a.scratch + (long long)blockIdx.x * a.slot_bytes;
  const int ntiles = a.tiles_x * a.tiles_y;
  int run = 0;
  for (int tile; (tile = claim_tile(a.claim, ntiles, run, &claimed)) >= 0;) {
    tile_body<KT, SHAPE, 1, true, false, true>(a, tile, smem, slot);
    __syncthreads();
  }
  claim_done(a.claim);
}

namespace {

template <int KT, int SHAPE>
PlainKernelFn pick_general_variant(const ImageDesc& d) {
  if (d.gs) return mf_general_gs_kernel<KT, SHAPE>;
  switch (d.imax) {
    case 9: return mf_general_kernel<KT, SHAPE, 9>;
    case 17: return mf_general_kernel<KT, SHAPE, 17>;
    case 25: return mf_general_kernel<KT, SHAPE, 25>;
    default: return mf_general_kernel<KT, SHAPE, 33>;
  }
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

}  // namespace

namespace {
std::atomic<int> g_fuse_all{0};
}  // namespace

bool window_fusion_all() { return g_fuse_all.load() != 0; }
void set_window_fusion_all(int all) { g_fuse_all.store(all ? 1 : 0); }

// One pass of median_filter_windows over the windows outs[idx[0..n)]
// (arguments already validated): the plan of the smallest offset rectangle
// holding all of them, each plane with its own window tables.
int launch_window_pass(const void* img, int w, int h, size_t stride_bytes, int dtype,
                       int boundary, const mf_window_output* outs, const int* idx, int n,
                       int dev, const DeviceInfo& di, hipStream_t stream) {
  // the box: row and column spans of the hull are per-row / per-column
  // extremes (only the planner reads them; the tiles use each window's own
  // tables)
  mf_footprint hull;
  hull.kind = 0;
  hull.dx_min = hull.dy_min = 1 << 30;
  hull.dx_max = hull.dy_max = -(1 << 30);
  for (int i = 0; i < n; ++i) {
    const mf_footprint* fp = outs[idx[i]].footprint;
    if (fp->kind != 0) hull.kind = 1;
    hull.limit = std::max(hull.limit, fp->limit);
    hull.dx_min = std::min(hull.dx_min, fp->dx_min);
    hull.dx_max = std::max(hull.dx_max, fp->dx_max);
    hull.dy_min = std::min(hull.dy_min, fp->dy_min);
    hull.dy_max = std::max(hull.dy_max, fp->dy_max);
    hull.taps = std::max(hull.taps, fp->taps);
  }
  if (hull.kind != 0) hull.limit = 0;
  const int hr = hull.dy_max - hull.dy_min + 1, hc = hull.dx_max - hull.dx_min + 1;
  hull.row_lo.assign(hr, 0);
  hull.row_hi.assign(hr, 0);
  hull.col_lo.assign(hc, 0);
  hull.col_hi.assign(hc, 0);
  for (int i = 0; i < n; ++i) {
    const mf_footprint* fp = outs[idx[i]].footprint;
    for (size_t k = 0; k < fp->row_lo.size(); ++k) {
      const int r = fp->dy_min + (int)k - hull.dy_min;
      hull.row_lo[r] = std::min(hull.row_lo[r], fp->row_lo[k]);
      hull.row_hi[r] = std::max(hull.row_hi[r], fp->row_hi[k]);
    }
    for (size_t k = 0; k < fp->col_lo.size(); ++k) {
      const int c = fp->dx_min + (int)k - hull.dx_min;
      hull.col_lo[c] = std::min(hull.col_lo[c], fp->col_lo[k]);
      hull.col_hi[c] = std::max(hull.col_hi[c], fp->col_hi[k]);
    }
  }
  if (n == 1) {   // one window: the single-window entry points
    const mf_window_output& o = outs[idx[0]];
    if (o.rank_map)
      return median_filter_rank_map(img, w, h, stride_bytes, dtype, o.footprint, boundary,
                                    o.rank_map, o.rank_map_stride_bytes, o.out, stream);
    return median_filter_rank(img, w, h, stride_bytes, dtype, o.footprint, boundary,
                              o.rank < 0 ? (o.footprint->taps - 1) / 2 : o.rank, o.out, stream);
  }
  int rc;
  ImageDesc a{};
  if ((rc = choose_plan(dtype, &hull, di.lds_max, 33, &a, w, h, di.cus))) {
    if (rc != MF_ERR_UNSUPPORTED) return rc;
    // windows that each fit but whose rectangle does not (off-centre
    // shapes on opposite sides): one pass per window
    for (int i = 0; i < n; ++i)
      if ((rc = launch_window_pass(img, w, h, stride_bytes, dtype, boundary, outs, idx + i, 1,
                                   dev, di, stream)))
        return rc;
    return MF_OK;
  }
  const void* table0 = nullptr;
  if ((rc = footprint_device_table(outs[idx[0]].footprint, dev, &table0, stream))) return rc;
  bind_image(&a, img, w, h, stride_bytes, dtype, &hull, boundary, 0, table0);
  a.out = outs[idx[0]].out;
  a.nq = n;
  a.multi_fp = 1;
  for (int q = 0; q < n; ++q) {
    const mf_window_output& o = outs[idx[q]];
    const mf_footprint* fp = o.footprint;
    const void* table = nullptr;
    if ((rc = footprint_device_table(fp, dev, &table, stream))) return rc;
    PlaneFp& pf = a.pfp[q];
    pf.spans = static_cast<const short2*>(table);
    pf.dx_min = fp->dx_min;
    pf.dy_min = fp->dy_min;
    pf.nrows = (int)fp->row_lo.size();
    pf.ncols = (int)fp->col_lo.size();
    pf.limit = (int)fp->limit;
    pf.rank_hi = fp->taps - 1;
    if (pf.nrows > a.nrows || pf.ncols > a.ncols) return MF_ERR_UNSUPPORTED;   // not reached
    a.outs[q] = o.out;
    a.rmaps[q] = o.rank_map;
    a.rmap_strides[q] = (long long)(o.rank_map_stride_bytes / 4);
    a.ranks[q] = o.rank_map || o.rank < 0 ? (fp->taps - 1) / 2 : o.rank;
  }
  a.rank = a.ranks[0];
  a.rank_hi = a.pfp[0].rank_hi;
  return launch_with_plan(a, dev, di, stream);
}

PlainKernelFn pick_general_kernel(const ImageDesc& d) {
  if (d.kt == MF_U8) return d.shape == SHAPE_DISC ? pick_general_variant<KEY_U8, SHAPE_DISC>(d)
                                                  : pick_general_variant<KEY_U8, SHAPE_SPANS>(d);
  if (d.kt == MF_U16) return d.shape == SHAPE_DISC
                                 ? pick_general_variant<KEY_U16, SHAPE_DISC>(d)
                                 : pick_general_variant<KEY_U16, SHAPE_SPANS>(d);
  return d.shape == SHAPE_DISC ? pick_general_variant<KEY_F32, SHAPE_DISC>(d)
                               : pick_general_variant<KEY_F32, SHAPE_SPANS>(d);
}

}  // namespace mf

extern "C" {

int median_filter_ranks(const void* img, int w, int h, size_t stride_bytes, int dtype,
                        const mf_footprint* fp, int boundary, const mf_rank_output* outs,
                        int nouts, hipStream_t stream) {
  using namespace mf;
  if (!outs || nouts < 1 || nouts > MF_MAX_RANK_OUTPUTS) return MF_ERR_INVALID_ARG;
  for (int q = 0; q < nouts; ++q) {
    const int rc = validate_image(img, w, h, stride_bytes, dtype, fp, boundary, outs[q].out);
    if (rc != MF_OK) return rc;
  }
  if (w == 0 || h == 0) return MF_OK;
  const size_t span =
      stride_bytes * (size_t)(h - 1) + (size_t)w * (size_t)elem_size(dtype);
  for (int q = 0; q < nouts; ++q) {
    const mf_rank_output& o = outs[q];
    if (o.rank_map) {
      if (o.rank_map_stride_bytes < (size_t)w * 4 || o.rank_map_stride_bytes % 4)
        return MF_ERR_INVALID_ARG;
      const size_t mspan = o.rank_map_stride_bytes * (size_t)(h - 1) + (size_t)w * 4;
      for (int j = 0; j < nouts; ++j)
        if (overlaps(o.rank_map, mspan, outs[j].out, span)) return MF_ERR_ALIAS;
    } else if (o.rank < 0 || o.rank >= fp->taps) {
      return MF_ERR_INVALID_ARG;
    }
    for (int j = 0; j < q; ++j)
      if (overlaps(o.out, span, outs[j].out, span)) return MF_ERR_ALIAS;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MF_ERR_HIP;
  DeviceInfo di;
  int rc = device_info(dev, &di);
  if (rc) return rc;
  const void* table = nullptr;
  if ((rc = footprint_device_table(fp, dev, &table, stream))) return rc;
  ImageDesc a{};
  if ((rc = choose_plan(dtype, fp, di.lds_max, 33, &a, w, h, di.cus))) return rc;
  bind_image(&a, img, w, h, stride_bytes, dtype, fp, boundary, (fp->taps - 1) / 2, table);
  a.out = outs[0].out;
  a.nq = nouts;
  a.rank_hi = fp->taps - 1;
  for (int q = 0; q < nouts; ++q) {
    a.outs[q] = outs[q].out;
    a.rmaps[q] = outs[q].rank_map;
    a.rmap_strides[q] = (long long)(outs[q].rank_map_stride_bytes / 4);
    a.ranks[q] = outs[q].rank_map ? (fp->taps - 1) / 2 : outs[q].rank;
  }
  return launch_with_plan(a, dev, di, stream);
}

int median_filter_windows(const void* img, int w, int h, size_t stride_bytes, int dtype,
                          int boundary, const mf_window_output* outs, int nouts,
                          hipStream_t stream) {
  using namespace mf;
  if (!outs || nouts < 1 || nouts > MF_MAX_RANK_OUTPUTS) return MF_ERR_INVALID_ARG;
  for (int q = 0; q < nouts; ++q) {
    const int rc =
        validate_image(img, w, h, stride_bytes, dtype, outs[q].footprint, boundary, outs[q].out);
    if (rc != MF_OK) return rc;
  }
  if (w == 0 || h == 0) return MF_OK;
  const size_t span =
      stride_bytes * (size_t)(h - 1) + (size_t)w * (size_t)elem_size(dtype);
  for (int q = 0; q < nouts; ++q) {
    const mf_window_output& o = outs[q];
    if (o.rank_map) {
      if (o.rank_map_stride_bytes < (size_t)w * 4 || o.rank_map_stride_bytes % 4)
        return MF_ERR_INVALID_ARG;
      const size_t mspan = o.rank_map_stride_bytes * (size_t)(h - 1) + (size_t)w * 4;
      for (int j = 0; j < nouts; ++j)
        if (overlaps(o.rank_map, mspan, outs[j].out, span)) return MF_ERR_ALIAS;
    } else if (o.rank >= o.footprint->taps) {
      return MF_ERR_INVALID_ARG;
    }
    for (int j = 0; j < q; ++j)
      if (overlaps(o.out, span, outs[j].out, span)) return MF_ERR_ALIAS;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MF_ERR_HIP;
  DeviceInfo di;
  int rc = device_info(dev, &di);
  if (rc) return rc;
  // Passes: windows in decreasing order of their own plan's box (T_q
  // pixels for tiles of P_q pixels); a window joins the current pass, whose
  // first (largest) window has the box T_0, while
  //   (T_q / P_q) * N_q >= kFuse * (T_0 - T_q),
  // else it starts a pass of its own.  Left: the sort work the shared
  // ordinal transform saves per output pixel (the window's box
  // amplification); right: the extra ordinals a walk crosses per window
  // member in the larger box, times the member density N_q / T that the
  // walks see -- a small window in a large box crosses the extra box pixels
  // as non-members at every step.  kFuse separates the measured cases at
  // 4096^2 uint16 (one pass faster than separate calls: radii 24+32, 32+48,
  // 28+32+40, 24+32+40; slower: 8+16, 8+32, 16+64, 8+16+32) and keeps the
  // float32 disc 48 + ellipse 60x20 + hexagon R=40 set in one pass (1.19x
  // at 3840x2160).
  constexpr double kFuse = 0.25;
  int order[MF_MAX_RANK_OUTPUTS];
  long long boxT[MF_MAX_RANK_OUTPUTS];
  double gain[MF_MAX_RANK_OUTPUTS];
  for (int q = 0; q < nouts; ++q) {
    ImageDesc p{};
    if ((rc = choose_plan(dtype, outs[q].footprint, di.lds_max, 33, &p, w, h, di.cus))) return rc;
    boxT[q] = p.T;
    gain[q] = (double)p.T / ((double)p.tw * p.th) * (double)outs[q].footprint->taps;
    order[q] = q;
  }
  std::stable_sort(order, order + nouts, [&](int x, int y) { return boxT[x] > boxT[y]; });
  const bool fuse_all = window_fusion_all();
  for (int g0 = 0; g0 < nouts;) {
    const long long t0 = boxT[order[g0]];
    int g1 = g0 + 1;
    while (g1 < nouts &&
           (fuse_all || gain[order[g1]] >= kFuse * (double)(t0 - boxT[order[g1]])))
      ++g1;
    if ((rc = launch_window_pass(img, w, h, stride_bytes, dtype, boundary, outs, order + g0,
                                 g1 - g0, dev, di, stream)))
      return rc;
    g0 = g1;
  }
  return MF_OK;
}

int mf_set_window_fusion(int all) {
  mf::set_window_fusion_all(all);
  return MF_OK;
}

int median_filter_rank_map(const void* img, int w, int h, size_t stride_bytes, int dtype,
                           const mf_footprint* fp, int boundary, const int* rank_map,
                           size_t rank_map_stride_bytes, void* out, hipStream_t stream) {
  if (!rank_map && w > 0 && h > 0) return MF_ERR_INVALID_ARG;
  mf_rank_output o{out, 0, rank_map, rank_map_stride_bytes};
  return median_filter_ranks(img, w, h, stride_bytes, dtype, fp, boundary, &o, 1, stream);
}

}  // extern "C"
