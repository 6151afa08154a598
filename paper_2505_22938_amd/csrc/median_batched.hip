// Batched filtering: many images (any sizes, dtypes, footprints) in a few
// launches, optionally captured in a hipGraph.  Not in the paper; the
// per-tile work is the same engine as the plain filter.
//
// mf_plan_create builds, per image, the plain filter's plan (tuned shape if
// one is recorded) and a device descriptor table, then splits all tiles of
// all images into groups that share a kernel instance (key type, footprint
// form, register capacity or global scratch), so that each instance keeps
// the register allocation of the plain kernel for that variant.  A group is
// a slice of one tile queue, ordered longest-estimated-first, run by one
// launch: one workgroup per tile in queue order for LDS tiles, a persistent
// grid popping tiles with an atomic counter for global-scratch tiles.  The
// groups are spread over up to four streams (the caller's and three the plan
// owns, forked from and joined back into the caller's with events), longest
// total first, so that one group's tail overlaps the next group's start.
// Persistent launches reset their own counters when done, so launches need
// no memset and can be replayed from a graph.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "mf_internal.h"
#include "tile_engine.h"

namespace mf {

constexpr int kMaxItems = 33;  // register capacity allowed to batch plans (as plain)
constexpr int kLanes = 4;      // streams a launch spreads its groups over

// Descriptors are read through the constant address space, so the tile body
// loads each field with a scalar load where it is used, as it does a kernel
// argument, instead of holding a copy in registers.
using ConstDesc = const __attribute__((address_space(4))) ImageDesc;

// Register-capacity (LDS) groups: one workgroup per tile of the slice, in
// queue order, so the longest tiles are dispatched first.
template <int KT, int SHAPE, int IMAX>
__global__ __launch_bounds__(kThreads) void mf_batched_kernel(ConstDesc* descs,
                                                              const int2* __restrict__ queue,
                                                              int begin, int end, int* counters,
                                                              unsigned char* scratch,
                                                              long long slot_bytes) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int2 q = queue[begin + blockIdx.x];
  const int img = __builtin_amdgcn_readfirstlane(q.x);
  const int tile = __builtin_amdgcn_readfirstlane(q.y);
  tile_body<KT, SHAPE, IMAX, false>(descs[img], tile, smem, nullptr);
}

// Global-scratch groups: a persistent grid, one scratch slot per workgroup;
// workgroups pop tiles with an atomic counter.  The last workgroup to find
// the slice empty resets its counters for the next launch.
template <int KT, int SHAPE>
__global__ __launch_bounds__(kThreads) void mf_batched_gs_kernel(ConstDesc* descs,
                                                                 const int2* __restrict__ queue,
                                                                 int begin, int end,
                                                                 int* counters,
                                                                 unsigned char* scratch,
                                                                 long long slot_bytes) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  int* s_item = reinterpret_cast<int*>(smem);  // free between tiles
  unsigned char* slot = scratch + (long long)blockIdx.x * slot_bytes;
  for (;;) {
    if (threadIdx.x == 0) *s_item = begin + atomicAdd(&counters[0], 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(*s_item);
    __syncthreads();
    if (item >= end) break;
    const int2 q = queue[item];
    const int img = __builtin_amdgcn_readfirstlane(q.x);
    const int tile = __builtin_amdgcn_readfirstlane(q.y);
    tile_body<KT, SHAPE, 1, true>(descs[img], tile, smem, slot);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&counters[1], 1) == (int)gridDim.x - 1) {
      atomicExch(&counters[0], 0);
      atomicExch(&counters[1], 0);
    }
  }
}

namespace {

using BatchFn = void (*)(ConstDesc*, const int2*, int, int, int*, unsigned char*,
                         long long);

// Kernel variant of a planned image: 0..3 = register capacity 9/17/25/33,
// 4 = global scratch.
int variant_of(const ImageDesc& d) {
  if (d.gs) return 4;
  return d.imax <= 9 ? 0 : d.imax <= 17 ? 1 : d.imax <= 25 ? 2 : 3;
}

template <int KT, int SHAPE>
BatchFn pick_batched_variant(int v) {
  switch (v) {
    case 0: return mf_batched_kernel<KT, SHAPE, 9>;
    case 1: return mf_batched_kernel<KT, SHAPE, 17>;
    case 2: return mf_batched_kernel<KT, SHAPE, 25>;
    case 3: return mf_batched_kernel<KT, SHAPE, 33>;
    default: return mf_batched_gs_kernel<KT, SHAPE>;
  }
}

BatchFn pick_batched(int kt, int shape, int v) {
  if (kt == MF_U8) return shape == SHAPE_DISC ? pick_batched_variant<KEY_U8, SHAPE_DISC>(v)
                                              : pick_batched_variant<KEY_U8, SHAPE_SPANS>(v);
  if (kt == MF_U16) return shape == SHAPE_DISC ? pick_batched_variant<KEY_U16, SHAPE_DISC>(v)
                                               : pick_batched_variant<KEY_U16, SHAPE_SPANS>(v);
  return shape == SHAPE_DISC ? pick_batched_variant<KEY_F32, SHAPE_DISC>(v)
                             : pick_batched_variant<KEY_F32, SHAPE_SPANS>(v);
}

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

// One persistent launch of a batch plan: a slice of the queue run by one
// kernel instance.
struct BatchGroup {
  BatchFn fn = nullptr;
  int begin = 0, end = 0;   // queue slice
  int grid = 0;
  int lds_bytes = 0;
  long long slot_bytes = 0;
  long long scratch_off = 0;
  int lane = 0;             // 0 = caller's stream, 1.. = the plan's streams
  double cost = 0;
};

}  // namespace mf

struct mf_plan {
  int dev = 0;
  int n = 0;
  int ntotal = 0;
  int nlanes = 1;
  std::vector<mf::BatchGroup> groups;
  mf::ImageDesc* d_descs = nullptr;
  int2* d_queue = nullptr;
  int* d_counters = nullptr;
  unsigned char* d_scratch = nullptr;
  long long scratch_bytes = 0;
  hipStream_t side[mf::kLanes - 1] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[mf::kLanes - 1] = {};
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
  for (int i = 0; i < mf::kLanes - 1; ++i) {
    if (p->join[i]) (void)hipEventDestroy(p->join[i]);
    if (p->side[i]) (void)hipStreamDestroy(p->side[i]);
  }
  if (p->fork) (void)hipEventDestroy(p->fork);
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
  // (group key, -cost, image, tile): sorted, each group's tiles are one
  // contiguous slice, longest first
  struct Item {
    int key;
    double cost;
    int2 it;
  };
  std::vector<Item> items;
  for (int i = 0; i < n; ++i) {
    const mf_image_desc& e = descs[i];
    if (!e.w || !e.h) {
      hd[i] = ImageDesc{};
      continue;
    }
    const void* table = nullptr;
    if ((rc = footprint_device_table(e.fp, dev, &table, nullptr)) ||
        (rc = choose_plan(e.dtype, e.fp, di.lds_max, kMaxItems, &hd[i]))) {
      mf_plan_destroy(p);
      return rc;
    }
    bind_image(&hd[i], e.img, e.w, e.h, e.stride_bytes, e.dtype, e.fp, e.boundary,
               (e.fp->taps - 1) / 2, table);
    hd[i].out = e.out;
    const int key = (hd[i].kt * 2 + hd[i].shape) * 5 + variant_of(hd[i]);
    const double c = tile_cost(hd[i]);
    const int nt = hd[i].tiles_x * hd[i].tiles_y;
    for (int t = 0; t < nt; ++t) items.push_back({key, c, make_int2(i, t)});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
    return a.key != b.key ? a.key < b.key : a.cost > b.cost;
  });
  p->ntotal = (int)items.size();
  std::vector<int2> q(items.size());
  for (size_t i = 0; i < items.size(); ++i) q[i] = items[i].it;
  // one group per key, sized like the plain filter's launch of that variant
  for (size_t i = 0; i < items.size();) {
    size_t j = i;
    BatchGroup g;
    const ImageDesc& d0 = hd[items[i].it.x];
    g.fn = pick_batched(d0.kt, d0.shape, variant_of(d0));
    for (; j < items.size() && items[j].key == items[i].key; ++j) {
      const ImageDesc& d = hd[items[j].it.x];
      g.lds_bytes = std::max(g.lds_bytes, d.lds_bytes);
      if (d.gs) g.slot_bytes = std::max(g.slot_bytes, d.slot_bytes);
      g.cost += items[j].cost;
    }
    g.begin = (int)i;
    g.end = (int)j;
    const int occ = std::max(1, std::min(2, di.lds_max / std::max(1, g.lds_bytes)));
    g.grid = g.slot_bytes ? std::max(1, std::min(g.end - g.begin, di.cus * occ))
                          : g.end - g.begin;
    g.scratch_off = p->scratch_bytes;
    p->scratch_bytes += (long long)g.grid * g.slot_bytes;
    p->groups.push_back(g);
    i = j;
  }
  // longest group first, each onto the least loaded stream
  std::stable_sort(p->groups.begin(), p->groups.end(),
                   [](const BatchGroup& a, const BatchGroup& b) { return a.cost > b.cost; });
  p->nlanes = std::max(1, std::min<int>(kLanes, (int)p->groups.size()));
  {
    double load[kLanes] = {};
    for (BatchGroup& g : p->groups) {
      int best = 0;
      for (int l = 1; l < p->nlanes; ++l)
        if (load[l] < load[best]) best = l;
      g.lane = best;
      load[best] += g.cost;
    }
  }
  const size_t ng = std::max<size_t>(1, p->groups.size());
  if (hipMalloc(&p->d_descs, sizeof(ImageDesc) * std::max(1, n)) != hipSuccess ||
      hipMalloc(&p->d_queue, sizeof(int2) * std::max<size_t>(1, q.size())) != hipSuccess ||
      hipMalloc(&p->d_counters, 2 * sizeof(int) * ng) != hipSuccess ||
      (p->scratch_bytes && hipMalloc(&p->d_scratch, (size_t)p->scratch_bytes) != hipSuccess)) {
    mf_plan_destroy(p);
    return MF_ERR_NOMEM;
  }
  if ((n && hipMemcpy(p->d_descs, hd.data(), sizeof(ImageDesc) * n, hipMemcpyHostToDevice) !=
                hipSuccess) ||
      (!q.empty() &&
       hipMemcpy(p->d_queue, q.data(), sizeof(int2) * q.size(), hipMemcpyHostToDevice) !=
           hipSuccess) ||
      hipMemset(p->d_counters, 0, 2 * sizeof(int) * ng) != hipSuccess) {
    mf_plan_destroy(p);
    return MF_ERR_HIP;
  }
  if (p->nlanes > 1) {
    if (hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess) {
      p->fork = nullptr;
      mf_plan_destroy(p);
      return MF_ERR_HIP;
    }
    for (int l = 0; l < p->nlanes - 1; ++l)
      if (hipStreamCreateWithFlags(&p->side[l], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&p->join[l], hipEventDisableTiming) != hipSuccess) {
        mf_plan_destroy(p);
        return MF_ERR_HIP;
      }
  }
  for (const BatchGroup& g : p->groups)
    (void)hipFuncSetAttribute((const void*)g.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              g.lds_bytes);
  *out = p;
  return MF_OK;
}

int mf_plan_launch(mf_plan* p, hipStream_t stream) {
  if (!p) return MF_ERR_INVALID_ARG;
  if (p->ntotal == 0) return MF_OK;
  const bool fork = p->nlanes > 1;
  if (fork) {
    if (hipEventRecord(p->fork, stream) != hipSuccess) return MF_ERR_HIP;
    for (int l = 0; l < p->nlanes - 1; ++l)
      if (hipStreamWaitEvent(p->side[l], p->fork, 0) != hipSuccess) return MF_ERR_HIP;
  }
  int rc = MF_OK;
  for (size_t i = 0; i < p->groups.size(); ++i) {
    const mf::BatchGroup& g = p->groups[i];
    hipStream_t s = g.lane ? p->side[g.lane - 1] : stream;
    hipLaunchKernelGGL(g.fn, dim3(g.grid), dim3(mf::kThreads), g.lds_bytes, s,
                       (mf::ConstDesc*)p->d_descs, p->d_queue, g.begin, g.end, p->d_counters + 2 * i,
                       g.slot_bytes ? p->d_scratch + g.scratch_off : nullptr, g.slot_bytes);
    if (hipGetLastError() != hipSuccess) rc = MF_ERR_HIP;
  }
  if (fork)  // join every forked stream back, also after a failed launch
    for (int l = 0; l < p->nlanes - 1; ++l)
      if (hipEventRecord(p->join[l], p->side[l]) != hipSuccess ||
          hipStreamWaitEvent(stream, p->join[l], 0) != hipSuccess)
        rc = MF_ERR_HIP;
  return rc;
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
  int wg = 0, lds = 0;
  for (const mf::BatchGroup& g : p->groups) {
    wg += g.grid;
    lds = std::max(lds, g.lds_bytes);
  }
  if (tiles) *tiles = p->ntotal;
  if (grid) *grid = wg;
  if (lds_bytes) *lds_bytes = lds;
  if (scratch_bytes) *scratch_bytes = p->scratch_bytes;
  return MF_OK;
}

int mf_plan_groups(const mf_plan* p, int* groups, int* streams) {
  if (!p) return MF_ERR_INVALID_ARG;
  if (groups) *groups = (int)p->groups.size();
  if (streams) *streams = p->groups.empty() ? 0 : p->nlanes;
  return MF_OK;
}

int mf_plan_autotune(const mf_image_desc* descs, int n, hipStream_t stream, int reps,
                     float* before_ms, float* after_ms, int* dropped) {
  using namespace mf;
  if (n < 0 || (n > 0 && !descs) || reps < 1) return MF_ERR_INVALID_ARG;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return MF_ERR_HIP;
  }
  // batch time (ms per launch) under the tuned table as it stands
  auto time_batch = [&](float* ms) -> int {
    mf_plan* p = nullptr;
    int rc = mf_plan_create(descs, n, nullptr, &p);
    if (rc) return rc;
    rc = mf_plan_launch(p, stream);
    if (!rc && hipEventRecord(e0, stream) != hipSuccess) rc = MF_ERR_HIP;
    for (int i = 0; i < reps && !rc; ++i) rc = mf_plan_launch(p, stream);
    if (!rc && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
      rc = MF_ERR_HIP;
    float t = 0;
    if (!rc) (void)hipEventElapsedTime(&t, e0, e1);
    mf_plan_destroy(p);
    *ms = t / (float)reps;
    return rc;
  };
  // distinct (dtype, footprint) pairs with their share of the batch's work
  struct Grp {
    int dtype;
    const mf_footprint* fp;
    double cost;
  };
  std::vector<Grp> grps;
  for (int i = 0; i < n; ++i) {
    const mf_image_desc& e = descs[i];
    if (!e.fp || !e.w || !e.h) continue;
    const double c = (double)e.w * e.h * (2.0 * (e.fp->dx_max - e.fp->dx_min + 1) + 160.0);
    const std::string k = tune_key(e.dtype, e.fp);
    bool found = false;
    for (Grp& g : grps)
      if (g.dtype == e.dtype && tune_key(g.dtype, g.fp) == k) {
        g.cost += c;
        found = true;
        break;
      }
    if (!found) grps.push_back({e.dtype, e.fp, c});
  }
  std::stable_sort(grps.begin(), grps.end(), [](const Grp& a, const Grp& b) { return a.cost > b.cost; });
  float best = 0;
  int rc = time_batch(&best);
  const float first = best;
  int ndrop = 0;
  for (const Grp& g : grps) {
    if (rc) break;
    int tw = 0, th = 0;
    if (!tuned_shape(g.dtype, g.fp, &tw, &th)) continue;
    erase_tuned_shape(g.dtype, g.fp);
    float t = 0;
    if ((rc = time_batch(&t))) break;
    if (t < best) {
      best = t;
      ++ndrop;
    } else {
      record_tuned_shape(g.dtype, g.fp, tw, th, 0.0);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (before_ms) *before_ms = first;
  if (after_ms) *after_ms = best;
  if (dropped) *dropped = ndrop;
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
