// Internal declarations shared by the library's host sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/median_filter.h"

struct mf_footprint {
  // kind: 0 = disc given by an integer squared limit; 1 = general convex
  // shape given only by its spans.  Both carry the spans.
  int kind = 1;
  long long limit = 0;
  int dx_min = 0, dx_max = 0, dy_min = 0, dy_max = 0;
  int taps = 0;
  std::vector<int> row_lo, row_hi;  // index dy - dy_min: dx range of that row
  std::vector<int> col_lo, col_hi;  // index dx - dx_min: dy range of that column

  // Per-device copies of the span tables (int16 pairs: rows then columns).
  struct DevCopy {
    int device;
    void* ptr;
  };
  mutable std::mutex mu;
  mutable std::vector<DevCopy> dev;
};

namespace mf {

constexpr int kThreads = 1024;            // threads per tile workgroup
constexpr int kWaves = kThreads / 64;     // wave64
constexpr int kDigits = 16;               // 4-bit radix digits
constexpr int kCounterBytes = kDigits * kThreads * 2;
constexpr int kHistWords = 256;           // seed histogram bins per wave (32-bit)
constexpr int kHistBytes = kWaves * kHistWords * 4;

enum { KEY_U8 = 0, KEY_U16 = 1, KEY_F32 = 2 };
enum { SHAPE_DISC = 0, SHAPE_SPANS = 1 };

// Everything one tile needs to know about its image and plan.  Passed by
// value to the plain kernels and stored in the batched descriptor table.
constexpr int kMaxRankOutputs = MF_MAX_RANK_OUTPUTS;   // planes of one general-rank call

// Window of one output plane when the planes of a general-rank call use
// different footprints (all inside the plan's box): its device span table
// (rows then columns, as ImageDesc::spans), geometry, disc limit and the
// largest valid rank (taps - 1).
struct PlaneFp {
  const short2* spans;
  int dx_min, dy_min, nrows, ncols, limit, rank_hi;
};

struct ImageDesc {
  const void* img;
  void* out;
  long long stride;  // elements (image and output)
  int w, h, boundary;
  int tw, th, tiles_x, tiles_y;
  int bw, bh, T, pitch;
  int dx_min, dy_min, nrows, ncols;
  int rank, limit;
  int segs, band_rows, hist_shift;
  const short2* spans;  // nrows row spans (index dy - dy_min) then ncols column spans
  // LDS layout, bytes (off_I: the ordinal image)
  int off_p, off_C, off_B, off_I, off_hist, off_tab, lds_bytes;
  unsigned long long* counters;  // optional work counters (null: off)
  // global-scratch variant: per-workgroup slot of slot_bytes at scratch;
  // claim: the persistent grid's tile-claim words (zero between launches)
  unsigned char* scratch;
  long long slot_bytes;
  unsigned int* claim;
  int off_x1, off_lr, ipt;
  // kernel selection: key type, shape, 1 = global-scratch variant, and the
  // register capacity (elements per thread) of the LDS variant
  int kt, shape, gs, imax;
  // bracketed tiles (learned path): per-tile [lo, hi] keys, the number of
  // in-bracket pixels region A can hold, and the list (y * w + x) and count
  // of output pixels whose median fell outside their tile's bracket
  const uint2* brackets;
  int br_cap;
  unsigned int* miss;
  unsigned int* miss_count;
  // general ranks (kernels instantiated for them only): nq output planes
  // from one ordinal transform per tile; plane q is written to outs[q] at
  // rank ranks[q], or at the per-pixel rank rmaps[q][y * rmap_strides[q] +
  // x] (int32, clamped to [0, rank_hi]) where rmaps[q] is set.  nq = 0: the
  // single plane `out` at `rank`.
  int nq, rank_hi;
  void* outs[kMaxRankOutputs];
  const int* rmaps[kMaxRankOutputs];
  long long rmap_strides[kMaxRankOutputs];  // elements
  int ranks[kMaxRankOutputs];
  // multi_fp = 1: plane q uses the window pfp[q] instead of the plan's
  // (whose box, tables and kernel shape cover all of them)
  int multi_fp;
  PlaneFp pfp[kMaxRankOutputs];
  // chained tiles: LDS offset of the forwarded last-row locations (64 u16)
  int off_fwd;
};

struct DeviceInfo {
  int lds_max = 0;
  int cus = 0;
};
int device_info(int dev, DeviceInfo* out);

// Tile plans.  make_plan: everything in LDS; make_plan_gs: sort, omnigram and
// reverse map in a global scratch slot.  choose_plan picks the tuned shape
// for this (dtype, footprint) if one is recorded, else the widest layout
// that fits, LDS first; imax_cap bounds the register capacity of LDS plans.
int make_plan(int dtype, const mf_footprint* fp, int lds_max, int tw, int th, ImageDesc* d);
int make_plan_gs(int dtype, const mf_footprint* fp, int lds_max, int tw, int th, ImageDesc* d);
// w, h, cus (image size and compute units, 0 = unknown) let the default
// choice keep enough tiles per CU.  choose_plan_tall: the override or the
// tallest default shape, ignoring the tuned table (bracketed tiles).
int choose_plan(int dtype, const mf_footprint* fp, int lds_max, int imax_cap, ImageDesc* d,
                int w = 0, int h = 0, int cus = 0);
int choose_plan_tall(int dtype, const mf_footprint* fp, int lds_max, int imax_cap,
                     ImageDesc* d);
// Bracketed-tile plan (8/16-bit keys) for a given shape: region A holds only
// the in-bracket pixels (up to br_cap of them), region B the ordinal image
// of the whole box.  MF_ERR_UNSUPPORTED if fewer than 1024 fit.
int make_plan_br(int dtype, const mf_footprint* fp, int lds_max, int tw, int th, ImageDesc* d);
// Enumerate every valid plan (for the autotuner).
std::vector<ImageDesc> candidate_plans(int dtype, const mf_footprint* fp, int lds_max,
                                       int imax_cap);
// Fill the per-image fields of a plan.
void bind_image(ImageDesc* d, const void* img, int w, int h, size_t stride_bytes, int dtype,
                const mf_footprint* fp, int boundary, int rank, const void* spans);

int validate_image(const void* img, int w, int h, size_t stride_bytes, int dtype,
                   const mf_footprint* fp, int boundary, const void* out);

// Global scratch cached per (device, stream); never allocates while the
// stream is capturing (MF_ERR_UNSUPPORTED instead).  release_scratch frees
// every cached buffer (mf_release_scratch).  *out points to `bytes` of slot
// space; the kClaimBytes before it hold the tile-claim words (nine used),
// zeroed when the buffer is allocated and left zero by every launch that
// uses them.
constexpr int kClaimBytes = 256;
int get_scratch(int dev, hipStream_t stream, size_t bytes, void** out);
int release_scratch();

// Tuned tile shapes, keyed by dtype and footprint.
std::string tune_key(int dtype, const mf_footprint* fp);
bool tuned_shape(int dtype, const mf_footprint* fp, int* tw, int* th);
void record_tuned_shape(int dtype, const mf_footprint* fp, int tw, int th, double ms);
void erase_tuned_shape(int dtype, const mf_footprint* fp);
int tune_cache_load(const char* path);
int tune_cache_save(const char* path);

// Device work counters of the plain engine (null when counting is off).
unsigned long long* work_counters_ptr();

// Plain-filter launch with a complete plan (median_plain.hip); a.nq > 0
// runs the general-rank kernels (median_general.hip).
// ext_scratch (non-null): a global-scratch plan takes its slots from this
// buffer of ext_bytes bytes instead of the cached per-stream scratch, its
// persistent grid shrunk to the slots that fit (MF_ERR_SCRATCH_LIMIT if not
// even one does); nothing is allocated.
using PlainKernelFn = void (*)(ImageDesc);
int launch_with_plan(ImageDesc a, int dev, const DeviceInfo& di, hipStream_t stream,
                     unsigned char* ext_scratch = nullptr, size_t ext_bytes = 0);
PlainKernelFn pick_general_kernel(const ImageDesc& d);
// median_filter_windows: one pass for all windows (set by
// mf_set_window_fusion) instead of grouping them by box size.
bool window_fusion_all();
void set_window_fusion_all(int all);
int launch_window_pass(const void* img, int w, int h, size_t stride_bytes, int dtype,
                       int boundary, const mf_window_output* outs, const int* idx, int n,
                       int dev, const DeviceInfo& di, hipStream_t stream);

// Tile-shape override (measurement): 0 = off.
void get_override(int* tw, int* th);

// Upload (once per device) and return the device span table of `fp`:
// [row (lo,hi) pairs as int16][column (lo,hi) pairs as int16].
// MF_ERR_UNSUPPORTED if the table is not there yet and `stream` is capturing.
int footprint_device_table(const mf_footprint* fp, int device, const void** table,
                           hipStream_t stream);
// The same footprint with one empty row added above its first row (cached,
// owned by the library): a box planned for it has one extra row on top, the
// row whose windows chained tiles forward.
const mf_footprint* footprint_with_top_row(const mf_footprint* fp);
// The same table on the host: 2 * (rows + columns) int16 values written to
// `dst` (which holds at least that many); returns the count.
size_t footprint_span_table(const mf_footprint* fp, int16_t* dst);
size_t footprint_span_table_len(const mf_footprint* fp);

inline int elem_size(int dtype) { return dtype == MF_U8 ? 1 : dtype == MF_U16 ? 2 : 4; }

}  // namespace mf
