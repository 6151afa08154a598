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
#include <vector>

#include "mf_internal.h"
#include "tile_engine.h"

namespace mf {

template <int KT, int SHAPE, int IMAX>
__global__ __launch_bounds__(kThreads) void mf_plain_kernel(ImageDesc a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  tile_body<KT, SHAPE, IMAX, false>(a, xcd_tile(blockIdx.x, gridDim.x), smem, nullptr);
}

// Large boxes: a persistent grid, one global scratch slot per workgroup,
// tiles claimed at run time.
template <int KT, int SHAPE>
__global__ __launch_bounds__(kThreads) void mf_plain_gs_kernel(ImageDesc a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int claimed;
  unsigned char* slot = a.scratch + (long long)blockIdx.x * a.slot_bytes;
  const int ntiles = a.tiles_x * a.tiles_y;
  int run = 0;
  for (int tile; (tile = claim_tile(a.claim, ntiles, run, &claimed)) >= 0;) {
    tile_body<KT, SHAPE, 1, true>(a, tile, smem, slot);
    __syncthreads();
  }
  claim_done(a.claim);
}

// Chained tiles: workgroup (x, c) walks tiles c * S .. c * S + S - 1 of
// tile column x top to bottom, each tile after the first re-ranking the
// box part it shares with the one above and starting its first band from
// the forwarded last-row solutions (tile_body, CHAIN).
template <int KT, int SHAPE, int IMAX>
__global__ __launch_bounds__(kThreads) void mf_chain_kernel(ImageDesc a, int S) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tx = (int)blockIdx.x % a.tiles_x;
  const int ty0 = ((int)blockIdx.x / a.tiles_x) * S;
  const int ty1 = min(ty0 + S, a.tiles_y);
  for (int ty = ty0; ty < ty1; ++ty) {
    tile_body<KT, SHAPE, IMAX, false, false, false, true>(a, ty * a.tiles_x + tx, smem, nullptr,
                                                         ty > ty0 ? 1 : 0);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- host side

namespace {

using KernelFn = PlainKernelFn;

template <int KT, int SHAPE>
KernelFn pick_imax(int imax) {
  switch (imax) {
    case 9: return mf_plain_kernel<KT, SHAPE, 9>;
    case 17: return mf_plain_kernel<KT, SHAPE, 17>;
    case 25: return mf_plain_kernel<KT, SHAPE, 25>;
    default: return mf_plain_kernel<KT, SHAPE, 33>;
  }
}

template <int KT, int SHAPE>
KernelFn pick_variant(const ImageDesc& d) {
  return d.gs ? mf_plain_gs_kernel<KT, SHAPE> : pick_imax<KT, SHAPE>(d.imax);
}

KernelFn pick_kernel(const ImageDesc& d) {
  if (d.kt == MF_U8) return d.shape == SHAPE_DISC ? pick_variant<KEY_U8, SHAPE_DISC>(d)
                                                  : pick_variant<KEY_U8, SHAPE_SPANS>(d);
  if (d.kt == MF_U16) return d.shape == SHAPE_DISC ? pick_variant<KEY_U16, SHAPE_DISC>(d)
                                                   : pick_variant<KEY_U16, SHAPE_SPANS>(d);
  return d.shape == SHAPE_DISC ? pick_variant<KEY_F32, SHAPE_DISC>(d)
                               : pick_variant<KEY_F32, SHAPE_SPANS>(d);
}

using ChainFn = void (*)(ImageDesc, int);

template <int KT, int SHAPE>
ChainFn pick_chain_imax(int imax) {
  switch (imax) {
    case 9: return mf_chain_kernel<KT, SHAPE, 9>;
    case 17: return mf_chain_kernel<KT, SHAPE, 17>;
    case 25: return mf_chain_kernel<KT, SHAPE, 25>;
    default: return mf_chain_kernel<KT, SHAPE, 33>;
  }
}

ChainFn pick_chain(const ImageDesc& d) {
  if (d.kt == MF_U8) return d.shape == SHAPE_DISC ? pick_chain_imax<KEY_U8, SHAPE_DISC>(d.imax)
                                                  : pick_chain_imax<KEY_U8, SHAPE_SPANS>(d.imax);
  if (d.kt == MF_U16) return d.shape == SHAPE_DISC ? pick_chain_imax<KEY_U16, SHAPE_DISC>(d.imax)
                                                   : pick_chain_imax<KEY_U16, SHAPE_SPANS>(d.imax);
  return d.shape == SHAPE_DISC ? pick_chain_imax<KEY_F32, SHAPE_DISC>(d.imax)
                               : pick_chain_imax<KEY_F32, SHAPE_SPANS>(d.imax);
}

unsigned long long* g_counters = nullptr;  // device work counters, enabled on request

}  // namespace

unsigned long long* work_counters_ptr() { return g_counters; }

// Launch one plain filter with a complete plan `a` (geometry + image bound);
// a.nq > 0 selects the general-rank kernels.
int launch_with_plan(ImageDesc a, int dev, const DeviceInfo& di, hipStream_t stream,
                     unsigned char* ext_scratch, size_t ext_bytes) {
  a.counters = g_counters;
  KernelFn k = a.nq > 0 ? pick_general_kernel(a) : pick_kernel(a);
  (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                            a.lds_bytes);
  const long long ntiles = (long long)a.tiles_x * a.tiles_y;
  if (ntiles > 0x7fffffffLL) return MF_ERR_UNSUPPORTED;
  long long grid = ntiles;
  if (a.gs) {
    const int occ = std::max(1, std::min(2, di.lds_max / std::max(1, a.lds_bytes)));
    grid = std::min<long long>(ntiles, (long long)di.cus * occ);
    if (ext_scratch) {
      // claim words first (zero-initialised, left zero by every launch)
      if (ext_bytes < (size_t)kClaimBytes) return MF_ERR_SCRATCH_LIMIT;
      const long long fit = (long long)((ext_bytes - kClaimBytes) / (size_t)a.slot_bytes);
      if (fit < 1) return MF_ERR_SCRATCH_LIMIT;
      grid = std::min(grid, fit);
      a.scratch = ext_scratch + kClaimBytes;
    } else {
      void* scr = nullptr;
      const int rc = get_scratch(dev, stream, (size_t)grid * (size_t)a.slot_bytes, &scr);
      if (rc) return rc;
      a.scratch = static_cast<unsigned char*>(scr);
    }
    a.claim = reinterpret_cast<unsigned int*>(a.scratch - kClaimBytes);
  }
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kThreads), a.lds_bytes, stream, a);
  if (hipGetLastError() != hipSuccess) return MF_ERR_HIP;
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
  rc = footprint_device_table(fp, dev, &table, stream);
  if (rc) return rc;
  ImageDesc a{};
  rc = choose_plan(dtype, fp, di.lds_max, 33, &a, w, h, di.cus);
  if (rc) return rc;
  bind_image(&a, img, w, h, stride_bytes, dtype, fp, boundary, rank, table);
  a.out = out;
  return launch_with_plan(a, dev, di, stream);
}

// Chained tiles (median_filter_chained): the plan of the footprint with an
// empty row on top, LDS variants only, 128 bytes more LDS for the forwarded
// locations.
int launch_chained(const void* img, int w, int h, size_t stride_bytes, int dtype,
                   const mf_footprint* fp, int boundary, int chain, void* out,
                   hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MF_ERR_HIP;
  DeviceInfo di;
  int rc = device_info(dev, &di);
  if (rc) return rc;
  const mf_footprint* fx = footprint_with_top_row(fp);
  const void* table = nullptr;
  if ((rc = footprint_device_table(fx, dev, &table, stream))) return rc;
  ImageDesc a{};
  if ((rc = choose_plan(dtype, fx, di.lds_max - 128, 33, &a, w, h, di.cus))) return rc;
  if (a.gs) return MF_ERR_UNSUPPORTED;   // chained tiles re-rank in LDS
  a.off_fwd = a.lds_bytes;
  a.lds_bytes += 128;
  bind_image(&a, img, w, h, stride_bytes, dtype, fx, boundary, (fp->taps - 1) / 2, table);
  a.out = out;
  a.counters = g_counters;
  ChainFn k = pick_chain(a);
  (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                            a.lds_bytes);
  const long long chains = (long long)a.tiles_x * ((a.tiles_y + chain - 1) / chain);
  if (chains > 0x7fffffffLL) return MF_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k, dim3((unsigned)chains), dim3(kThreads), a.lds_bytes, stream, a, chain);
  if (hipGetLastError() != hipSuccess) return MF_ERR_HIP;
  return MF_OK;
}

int query_plan(int w, int h, int dtype, const mf_footprint* fp, ImageDesc* d) {
  int dev = 0;
  DeviceInfo di;
  if (hipGetDevice(&dev) != hipSuccess || device_info(dev, &di) != MF_OK) {
    di.lds_max = 160 * 1024;
    di.cus = 256;
  }
  return choose_plan(dtype, fp, di.lds_max, 33, d, w, h, di.cus);
}

int set_counters(int enable) {
  if (enable && !g_counters) {
    if (hipMalloc(&g_counters, CNT_SLOTS * sizeof(unsigned long long)) != hipSuccess) {
      g_counters = nullptr;
      return MF_ERR_NOMEM;
    }
  }
  if (g_counters &&
      hipMemset(g_counters, 0, CNT_SLOTS * sizeof(unsigned long long)) != hipSuccess)
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
    case MF_ERR_SCRATCH_LIMIT: return "MF_ERR_SCRATCH_LIMIT";
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

int median_filter_chained(const void* img, int w, int h, size_t stride_bytes, int dtype,
                          const mf_footprint* fp, int boundary, int chain, void* out,
                          hipStream_t stream) {
  int rc = mf::validate_image(img, w, h, stride_bytes, dtype, fp, boundary, out);
  if (rc != MF_OK) return rc;
  if (chain < 1) return MF_ERR_INVALID_ARG;
  if (w == 0 || h == 0) return MF_OK;
  return mf::launch_chained(img, w, h, stride_bytes, dtype, fp, boundary, chain, out, stream);
}

int mf_query_plan(int w, int h, int dtype, const mf_footprint* fp, int* tile_w, int* tile_h,
                  int* box_w, int* box_h, int* lds) {
  if (!fp || w < 0 || h < 0 || (dtype != MF_U8 && dtype != MF_U16 && dtype != MF_F32))
    return MF_ERR_INVALID_ARG;
  mf::ImageDesc d{};
  const int rc = mf::query_plan(w, h, dtype, fp, &d);
  if (rc) return rc;
  if (tile_w) *tile_w = d.tw;
  if (tile_h) *tile_h = d.th;
  if (box_w) *box_w = d.bw;
  if (box_h) *box_h = d.bh;
  if (lds) *lds = d.lds_bytes;
  return MF_OK;
}

int mf_work_counters(int enable, unsigned long long* out10) {
  if (enable < 0) return out10 ? mf::read_counters(out10) : MF_ERR_INVALID_ARG;
  return mf::set_counters(enable);
}

int mf_autotune(const void* img, int w, int h, size_t stride_bytes, int dtype,
                const mf_footprint* fp, int boundary, void* out, hipStream_t stream, int reps,
                int* best_tw, int* best_th, float* best_ms) {
  int rc = mf::validate_image(img, w, h, stride_bytes, dtype, fp, boundary, out);
  if (rc != MF_OK) return rc;
  if (w == 0 || h == 0 || reps < 1) return MF_ERR_INVALID_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MF_ERR_HIP;
  mf::DeviceInfo di;
  if ((rc = mf::device_info(dev, &di))) return rc;
  const void* table = nullptr;
  if ((rc = mf::footprint_device_table(fp, dev, &table, stream))) return rc;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MF_ERR_HIP;
  float best = 1e30f;
  int btw = 0, bth = 0;
  for (mf::ImageDesc d : mf::candidate_plans(dtype, fp, di.lds_max, 33)) {
    mf::bind_image(&d, img, w, h, stride_bytes, dtype, fp, boundary, (fp->taps - 1) / 2, table);
    d.out = out;
    if (mf::launch_with_plan(d, dev, di, stream) != MF_OK) continue;   // warm-up
    (void)hipEventRecord(e0, stream);
    bool ok = true;
    for (int i = 0; i < reps && ok; ++i) ok = mf::launch_with_plan(d, dev, di, stream) == MF_OK;
    (void)hipEventRecord(e1, stream);
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = MF_ERR_HIP;
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)reps;
    if (ok && ms < best) {
      best = ms;
      btw = d.tw;
      bth = d.th;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (!btw) return MF_ERR_UNSUPPORTED;
  mf::record_tuned_shape(dtype, fp, btw, bth, best);
  if (best_tw) *best_tw = btw;
  if (best_th) *best_th = bth;
  if (best_ms) *best_ms = best;
  return MF_OK;
}

int mf_tune_cache_load(const char* path) {
  return path ? mf::tune_cache_load(path) : MF_ERR_INVALID_ARG;
}

int mf_tune_cache_save(const char* path) {
  return path ? mf::tune_cache_save(path) : MF_ERR_INVALID_ARG;
}

}  // extern "C"
