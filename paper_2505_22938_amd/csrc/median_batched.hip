// Batched filtering: many images (any sizes, dtypes, footprints) in one
// persistent launch, optionally captured in a hipGraph.  Not in the paper;
// the per-tile work is the same engine as the plain filter.
//
// mf_plan_create builds, per image, the plain filter's plan (tuned shape if
// one is recorded), a device descriptor table, and one queue of all tiles of
// all images, ordered longest-estimated-first.  The kernel runs one
// workgroup per resident slot (CUs x occupancy); each workgroup pops tiles
// from the queue with an atomic counter and runs them.  The last workgroup
// to find the queue empty resets the counters, so a launch needs no memset
// and can be replayed from a graph.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mf_internal.h"
#include "tile_engine.h"

namespace mf {

constexpr int kBatchItems = 25;   // register capacity of LDS plans in a batch

template <int KT, int SHAPE>
__device__ __forceinline__ void run_tile(const ImageDesc& d, int tile, unsigned char* smem,
                                         unsigned char* slot) {
  if (d.gs) tile_body<KT, SHAPE, 1, true>(d, tile, smem, slot);
  else tile_body<KT, SHAPE, kBatchItems, false>(d, tile, smem, nullptr);
}

__global__ __launch_bounds__(kThreads) void mf_batched_kernel(const ImageDesc* __restrict__ descs,
                                                              const int2* __restrict__ queue,
                                                              int ntotal, int* counters,
                                                              unsigned char* scratch,
                                                              long long slot_bytes) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int s_item;
  unsigned char* slot = scratch ? scratch + (long long)blockIdx.x * slot_bytes : nullptr;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&counters[0], 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= ntotal) break;
    const int2 q = queue[item];
    const int img = __builtin_amdgcn_readfirstlane(q.x);
    const int tile = __builtin_amdgcn_readfirstlane(q.y);
    const ImageDesc d = descs[img];
    switch (d.kt * 2 + d.shape) {
      case KEY_U8 * 2 + SHAPE_DISC: run_tile<KEY_U8, SHAPE_DISC>(d, tile, smem, slot); break;
      case KEY_U8 * 2 + SHAPE_SPANS: run_tile<KEY_U8, SHAPE_SPANS>(d, tile, smem, slot); break;
      case KEY_U16 * 2 + SHAPE_DISC: run_tile<KEY_U16, SHAPE_DISC>(d, tile, smem, slot); break;
      case KEY_U16 * 2 + SHAPE_SPANS: run_tile<KEY_U16, SHAPE_SPANS>(d, tile, smem, slot); break;
      case KEY_F32 * 2 + SHAPE_DISC: run_tile<KEY_F32, SHAPE_DISC>(d, tile, smem, slot); break;
      default: run_tile<KEY_F32, SHAPE_SPANS>(d, tile, smem, slot); break;
    }
    __syncthreads();
  }
  // the last workgroup out resets the queue for the next launch
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&counters[1], 1) == (int)gridDim.x - 1) {
      atomicExch(&counters[0], 0);
      atomicExch(&counters[1], 0);
    }
  }
}

namespace {

// Relative tile cost for longest-first ordering: sort work over the box plus
// slide and scan work over the tile's pixels.
double tile_cost(const ImageDesc& d) {
  const int passes = d.kt == MF_U8 ? 2 : d.kt == MF_U16 ? 4 : 8;
  return (double)d.T * passes * 4.0 + (double)d.tw * d.th * (2.0 * d.ncols + 160.0) +
         (d.gs ? (double)d.T * passes * 8.0 : 0.0);
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

}  // namespace

}  // namespace mf

struct mf_plan {
  int dev = 0;
  int n = 0;
  int ntotal = 0;
  int grid = 0;
  int lds_bytes = 0;
  long long slot_bytes = 0;
  mf::ImageDesc* d_descs = nullptr;
  int2* d_queue = nullptr;
  int* d_counters = nullptr;
  unsigned char* d_scratch = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

void mf_plan_destroy(mf_plan* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->dev);
  (void)hipDeviceSynchronize();
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  (void)hipFree(p->d_descs);
  (void)hipFree(p->d_queue);
  (void)hipFree(p->d_counters);
  (void)hipFree(p->d_scratch);
  (void)hipSetDevice(cur);
  delete p;
}

int mf_plan_create(const mf_image_desc* descs, int n, const char* tune_cache_path,
                   mf_plan** out) {
  using namespace mf;
  if (!out || n < 0 || (n > 0 && !descs)) return MF_ERR_INVALID_ARG;
  *out = nullptr;
  if (tune_cache_path && *tune_cache_path) (void)tune_cache_load(tune_cache_path);
  // argument checks, including aliasing between any output and any buffer
  std::vector<size_t> span(n);
  for (int i = 0; i < n; ++i) {
    const mf_image_desc& e = descs[i];
    int rc = validate_image(e.img, e.w, e.h, e.stride_bytes, e.dtype, e.fp, e.boundary, e.out);
    if (rc) return rc;
    span[i] = e.w && e.h ? e.stride_bytes * (size_t)(e.h - 1) + (size_t)e.w * elem_size(e.dtype)
                         : 0;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (!span[i] || !span[j]) continue;
      if (overlaps(descs[i].out, span[i], descs[j].img, span[j])) return MF_ERR_ALIAS;
      if (i < j && overlaps(descs[i].out, span[i], descs[j].out, span[j])) return MF_ERR_ALIAS;
    }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MF_ERR_HIP;
  DeviceInfo di;
  int rc = device_info(dev, &di);
  if (rc) return rc;

  auto* p = new (std::nothrow) mf_plan;
  if (!p) return MF_ERR_NOMEM;
  p->dev = dev;
  p->n = n;
  std::vector<ImageDesc> hd(n);
  std::vector<std::pair<double, int2>> items;
  for (int i = 0; i < n; ++i) {
    const mf_image_desc& e = descs[i];
    if (!e.w || !e.h) {
      hd[i] = ImageDesc{};
      continue;
    }
    const void* table = nullptr;
    if ((rc = footprint_device_table(e.fp, dev, &table)) ||
        (rc = choose_plan(e.dtype, e.fp, di.lds_max - 256, kBatchItems, &hd[i]))) {
      mf_plan_destroy(p);
      return rc;
    }
    bind_image(&hd[i], e.img, e.w, e.h, e.stride_bytes, e.dtype, e.fp, e.boundary,
               (e.fp->taps - 1) / 2, table);
    hd[i].out = e.out;
    p->lds_bytes = std::max(p->lds_bytes, hd[i].lds_bytes);
    if (hd[i].gs) p->slot_bytes = std::max(p->slot_bytes, hd[i].slot_bytes);
    const double c = tile_cost(hd[i]);
    const int nt = hd[i].tiles_x * hd[i].tiles_y;
    for (int t = 0; t < nt; ++t) items.push_back({c, make_int2(i, t)});
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const auto& a, const auto& b) { return a.first > b.first; });
  p->ntotal = (int)items.size();
  const int occ = std::max(1, std::min(2, di.lds_max / std::max(1, p->lds_bytes)));
  p->grid = std::max(1, std::min(p->ntotal, di.cus * occ));
  std::vector<int2> q(items.size());
  for (size_t i = 0; i < items.size(); ++i) q[i] = items[i].second;
  if (hipMalloc(&p->d_descs, sizeof(ImageDesc) * std::max(1, n)) != hipSuccess ||
      hipMalloc(&p->d_queue, sizeof(int2) * std::max<size_t>(1, q.size())) != hipSuccess ||
      hipMalloc(&p->d_counters, 2 * sizeof(int)) != hipSuccess ||
      (p->slot_bytes &&
       hipMalloc(&p->d_scratch, (size_t)p->grid * (size_t)p->slot_bytes) != hipSuccess)) {
    mf_plan_destroy(p);
    return MF_ERR_NOMEM;
  }
  if ((n && hipMemcpy(p->d_descs, hd.data(), sizeof(ImageDesc) * n, hipMemcpyHostToDevice) !=
                hipSuccess) ||
      (!q.empty() &&
       hipMemcpy(p->d_queue, q.data(), sizeof(int2) * q.size(), hipMemcpyHostToDevice) !=
           hipSuccess) ||
      hipMemset(p->d_counters, 0, 2 * sizeof(int)) != hipSuccess) {
    mf_plan_destroy(p);
    return MF_ERR_HIP;
  }
  (void)hipFuncSetAttribute((const void*)mf_batched_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, p->lds_bytes);
  *out = p;
  return MF_OK;
}

int mf_plan_launch(mf_plan* p, hipStream_t stream) {
  if (!p) return MF_ERR_INVALID_ARG;
  if (p->ntotal == 0) return MF_OK;
  hipLaunchKernelGGL(mf::mf_batched_kernel, dim3(p->grid), dim3(mf::kThreads), p->lds_bytes,
                     stream, p->d_descs, p->d_queue, p->ntotal, p->d_counters, p->d_scratch,
                     p->slot_bytes);
  return hipGetLastError() == hipSuccess ? MF_OK : MF_ERR_HIP;
}

int mf_plan_capture(mf_plan* p, hipStream_t stream) {
  if (!p || !stream) return MF_ERR_INVALID_ARG;
  if (p->exec) {
    (void)hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
  }
  if (p->graph) {
    (void)hipGraphDestroy(p->graph);
    p->graph = nullptr;
  }
  if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return MF_ERR_HIP;
  const int rc = mf_plan_launch(p, stream);
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(stream, &g) != hipSuccess || rc != MF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc != MF_OK ? rc : MF_ERR_HIP;
  }
  p->graph = g;
  if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    p->exec = nullptr;
    return MF_ERR_HIP;
  }
  return MF_OK;
}

int mf_plan_replay(mf_plan* p, hipStream_t stream) {
  if (!p || !p->exec) return MF_ERR_INVALID_ARG;
  return hipGraphLaunch(p->exec, stream) == hipSuccess ? MF_OK : MF_ERR_HIP;
}

int mf_plan_info(const mf_plan* p, int* tiles, int* grid, int* lds_bytes,
                 long long* scratch_bytes) {
  if (!p) return MF_ERR_INVALID_ARG;
  if (tiles) *tiles = p->ntotal;
  if (grid) *grid = p->grid;
  if (lds_bytes) *lds_bytes = p->lds_bytes;
  if (scratch_bytes) *scratch_bytes = (long long)p->grid * p->slot_bytes;
  return MF_OK;
}

int median_filter_batched(const mf_image_desc* descs, int n, hipStream_t stream) {
  mf_plan* p = nullptr;
  int rc = mf_plan_create(descs, n, nullptr, &p);
  if (rc) return rc;
  rc = mf_plan_launch(p, stream);
  if (rc == MF_OK && hipStreamSynchronize(stream) != hipSuccess) rc = MF_ERR_HIP;
  mf_plan_destroy(p);
  return rc;
}

}  // extern "C"
