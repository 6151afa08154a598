// Allocation-free variant of the plain median filter.
//
// The plain filter keeps two pieces of device memory besides the caller's
// planes: the footprint's span table (uploaded once per footprint and device)
// and, for windows whose box does not fit LDS, per-workgroup sort slots of
// the persistent global-scratch grid.  Here both come from one fixed
// file-scope device array, so a call allocates nothing.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol): the array's device address is looked up once per device
// with hipGetSymbolAddress and that pointer is used everywhere.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "mf_internal.h"

namespace mf {
namespace {

constexpr size_t kSpanRegion = 64 * 1024;   // span table at offset 0
constexpr size_t kScratchBytes = MF_NOALLOC_SCRATCH_BYTES;
constexpr size_t kSlotRegion = kScratchBytes - kSpanRegion;
static_assert(kScratchBytes > kSpanRegion, "scratch smaller than its span-table region");

// Span table as a kernel argument: boxes are at most 256 rows by 255
// columns, so a plan never has more than 511 row plus column spans.
constexpr int kMaxSpans = 512;
struct SpanArg {
  int n;
  short2 e[kMaxSpans];
};
static_assert(sizeof(SpanArg) <= 4096 - 8, "span table too large for a kernel argument");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Write the span table into the array's first region (one workgroup).
__global__ __launch_bounds__(256) void mf_noalloc_store_spans(SpanArg a, short2* dst) {
  for (int i = threadIdx.x; i < a.n; i += blockDim.x) dst[i] = a.e[i];
}

namespace {

// Device address of `scratch` on device `dev` (current), looked up once.
int scratch_ptr(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return MF_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MF_ERR_HIP;
    g_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_ptr[dev];
  return MF_OK;
}

}  // namespace
}  // namespace mf

extern "C" int median_filter_noalloc(const void* img, int w, int h, size_t stride_bytes,
                                     int dtype, const mf_footprint* fp, int boundary, void* out,
                                     hipStream_t stream) {
  using namespace mf;
  int rc = validate_image(img, w, h, stride_bytes, dtype, fp, boundary, out);
  if (rc != MF_OK) return rc;
  if (w == 0 || h == 0) return MF_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MF_ERR_HIP;
  DeviceInfo di;
  if ((rc = device_info(dev, &di))) return rc;
  unsigned char* base = nullptr;
  if ((rc = scratch_ptr(dev, &base))) return rc;

  ImageDesc a{};
  if ((rc = choose_plan(dtype, fp, di.lds_max, 33, &a, w, h, di.cus))) return rc;
  const size_t nspan = footprint_span_table_len(fp) / 2;
  if (nspan > (size_t)kMaxSpans || nspan * sizeof(short2) > kSpanRegion)
    return MF_ERR_SCRATCH_LIMIT;
  SpanArg sa;
  sa.n = (int)nspan;
  footprint_span_table(fp, reinterpret_cast<int16_t*>(sa.e));
  short2* table = reinterpret_cast<short2*>(base);
  hipLaunchKernelGGL(mf_noalloc_store_spans, dim3(1), dim3(256), 0, stream, sa, table);
  if (hipGetLastError() != hipSuccess) return MF_ERR_HIP;

  bind_image(&a, img, w, h, stride_bytes, dtype, fp, boundary, (fp->taps - 1) / 2, table);
  a.out = out;
  return launch_with_plan(a, dev, di, stream, base + kSpanRegion, kSlotRegion);
}
