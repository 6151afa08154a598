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
  unsigned char* slot = a.scratch + (long long)blockIdx.x * a.slot_bytes;
  const int ntiles = a.tiles_x * a.tiles_y;
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    tile_body<KT, SHAPE, 1, true, false, true>(a, xcd_tile(v, ntiles), smem, slot);
    __syncthreads();
  }
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
  if ((rc = footprint_device_table(fp, dev, &table))) return rc;
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

int median_filter_rank_map(const void* img, int w, int h, size_t stride_bytes, int dtype,
                           const mf_footprint* fp, int boundary, const int* rank_map,
                           size_t rank_map_stride_bytes, void* out, hipStream_t stream) {
  if (!rank_map && w > 0 && h > 0) return MF_ERR_INVALID_ARG;
  mf_rank_output o{out, 0, rank_map, rank_map_stride_bytes};
  return median_filter_ranks(img, w, h, stride_bytes, dtype, fp, boundary, &o, 1, stream);
}

}  // extern "C"
