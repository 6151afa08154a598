// Brute-force CPU oracle for exact rank-order (median) filtering.
//
// TEST INFRASTRUCTURE ONLY.  This file is the independent checker for the
// GPU library; only the test-suite, the smoke check and the CPU-baseline leg
// of the benchmark may load it.  It shares no code, header or table with the
// GPU path.
//
// What it computes (paper, "Core concepts: Histograms, Pivots, and Counts"):
// the median of a window is the value at the midpoint rank of the window's
// sorted values -- for a 7x7 window the 25th of 49, i.e. zero-based rank
// k = (N-1)/2.  The paper's method reaches exactly this result (rank-order
// filtering is invariant under the ordinal transform, "The Ordinal Transform
// and Compound Histogram"), so the oracle is that definition written out:
//
//   out(x,y) = element of rank k (ascending, zero-based) of the multiset
//              { v(bx(x+dx), by(y+dy)) : (dx,dy) in F }
//
// with the window's N values gathered one by one and the rank-k element taken
// by std::nth_element (a library selection primitive).  No tiling, no reuse
// between pixels, no sharing of sorts.
//
// Readings where the paper is silent:
//  * Image boundary: clamp (replicate edge) or mirror (reflect-101: -1 -> 1,
//    w -> w-2, folded repeatedly with period 2(w-1); w == 1 degenerates to 0).
//  * Float order: IEEE 754 totalOrder (-0 < +0; -NaN below -inf, +NaN above
//    +inf).  The output is the input bit pattern of the selected element.
//  * The rank is a parameter; the median is k = (N-1)/2 (lower median when N
//    is even).  A rank may also be given per output pixel (a rank map; the
//    paper's Conclusion and its varying-percentile figure let the percentile
//    vary across the image); a map entry outside [0, N) selects the nearest
//    end (0 or N-1), i.e. the window minimum or maximum.
//
// Build: g++ -O3 -fopenmp -shared -fPIC (no -march=native: the library may
// run on a different host CPU from the one that built it).

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

enum { DT_U8 = 0, DT_U16 = 1, DT_F32 = 2 };
enum { BD_CLAMP = 0, BD_MIRROR = 1 };

// Boundary rule, written from its definition.
inline int remap(int x, int n, int boundary) {
  if (x >= 0 && x < n) return x;
  if (boundary == BD_CLAMP) return x < 0 ? 0 : n - 1;
  if (n == 1) return 0;
  const long long period = 2LL * (n - 1);
  long long m = ((long long)x % period + period) % period;
  if (m >= n) m = period - m;
  return (int)m;
}

// IEEE 754 totalOrder on binary32 bit patterns, from the definition:
// a value with the sign bit set precedes one without; among non-negative
// encodings a larger magnitude field is larger; among negative encodings a
// larger magnitude field is smaller.
inline bool total_order_less(uint32_t a, uint32_t b) {
  const bool na = (a >> 31) != 0, nb = (b >> 31) != 0;
  if (na != nb) return na;               // negative < non-negative
  const uint32_t ma = a & 0x7fffffffu, mb = b & 0x7fffffffu;
  if (!na) return ma < mb;               // both non-negative
  return ma > mb;                        // both negative
}

struct Args {
  const unsigned char* img;
  int w, h;
  long long stride;     // elements
  int dtype;
  const int* dx;
  const int* dy;
  int n;
  int rank;
  int boundary;
};

// Rank-k element of the window centred at (x, y); returns the bits.
template <typename T>
inline uint32_t window_rank(const Args& a, int x, int y, int k, std::vector<T>& buf) {
  const T* base = reinterpret_cast<const T*>(a.img);
  for (int i = 0; i < a.n; ++i) {
    const int sx = remap(x + a.dx[i], a.w, a.boundary);
    const int sy = remap(y + a.dy[i], a.h, a.boundary);
    buf[i] = base[(long long)sy * a.stride + sx];
  }
  if constexpr (sizeof(T) == 4) {
    std::nth_element(buf.begin(), buf.begin() + k, buf.end(), total_order_less);
  } else {
    std::nth_element(buf.begin(), buf.begin() + k, buf.end());
  }
  return (uint32_t)buf[k];
}

// Rank map entry -> rank in [0, n).
inline int clamp_rank(long long r, int n) { return r < 0 ? 0 : r >= n ? n - 1 : (int)r; }

// Whole plane; the rank of pixel (x, y) is rank_map[y * rmap_stride + x]
// (clamped) when rank_map is given, else a.rank.
template <typename T>
void filter_all(const Args& a, const int* rank_map, long long rmap_stride, T* out,
                long long out_stride, int nthreads) {
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<T> buf(a.n);
#pragma omp for schedule(dynamic, 1)
    for (int y = 0; y < a.h; ++y)
      for (int x = 0; x < a.w; ++x) {
        const int k = rank_map ? clamp_rank(rank_map[(long long)y * rmap_stride + x], a.n)
                               : a.rank;
        out[(long long)y * out_stride + x] = (T)window_rank<T>(a, x, y, k, buf);
      }
  }
}

// Listed pixels; ks[i] (clamped) is pixel i's rank when ks is given.
template <typename T>
void filter_points(const Args& a, const int* xs, const int* ys, const int* ks, int npts,
                   T* vals, int nthreads) {
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<T> buf(a.n);
#pragma omp for schedule(dynamic, 64)
    for (int i = 0; i < npts; ++i)
      vals[i] = (T)window_rank<T>(a, xs[i], ys[i], ks ? clamp_rank(ks[i], a.n) : a.rank, buf);
  }
}

int check(const Args& a) {
  if (!a.img || a.w <= 0 || a.h <= 0 || a.n <= 0 || !a.dx || !a.dy) return -1;
  if (a.rank < 0 || a.rank >= a.n || a.stride < a.w) return -1;
  if (a.dtype < 0 || a.dtype > 2 || (a.boundary != BD_CLAMP && a.boundary != BD_MIRROR)) return -1;
  return 0;
}

}  // namespace

extern "C" {

// Filter a whole plane.  Strides are in elements.  Returns 0 or -1 (bad args).
int oracle_filter(const void* img, int w, int h, long long stride, int dtype,
                  const int* dx, const int* dy, int n, int rank, int boundary,
                  void* out, long long out_stride, int nthreads) {
  Args a{(const unsigned char*)img, w, h, stride, dtype, dx, dy, n, rank, boundary};
  if (check(a) || !out || out_stride < w) return -1;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  if (dtype == DT_U8) filter_all<uint8_t>(a, nullptr, 0, (uint8_t*)out, out_stride, nthreads);
  else if (dtype == DT_U16)
    filter_all<uint16_t>(a, nullptr, 0, (uint16_t*)out, out_stride, nthreads);
  else filter_all<uint32_t>(a, nullptr, 0, (uint32_t*)out, out_stride, nthreads);
  return 0;
}

// Filter a whole plane with a rank per pixel: rank_map (int32, row stride
// rmap_stride elements); entries outside [0, n) are clamped to it.
int oracle_filter_rank_map(const void* img, int w, int h, long long stride, int dtype,
                           const int* dx, const int* dy, int n, const int* rank_map,
                           long long rmap_stride, int boundary, void* out,
                           long long out_stride, int nthreads) {
  Args a{(const unsigned char*)img, w, h, stride, dtype, dx, dy, n, 0, boundary};
  if (check(a) || !out || out_stride < w || !rank_map || rmap_stride < w) return -1;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  if (dtype == DT_U8)
    filter_all<uint8_t>(a, rank_map, rmap_stride, (uint8_t*)out, out_stride, nthreads);
  else if (dtype == DT_U16)
    filter_all<uint16_t>(a, rank_map, rmap_stride, (uint16_t*)out, out_stride, nthreads);
  else filter_all<uint32_t>(a, rank_map, rmap_stride, (uint32_t*)out, out_stride, nthreads);
  return 0;
}

// Filter only the listed pixels (xs[i], ys[i]); vals[i] receives the result.
int oracle_filter_points(const void* img, int w, int h, long long stride, int dtype,
                         const int* dx, const int* dy, int n, int rank, int boundary,
                         const int* xs, const int* ys, int npts, void* vals, int nthreads) {
  Args a{(const unsigned char*)img, w, h, stride, dtype, dx, dy, n, rank, boundary};
  if (check(a) || npts < 0 || (npts > 0 && (!xs || !ys || !vals))) return -1;
  for (int i = 0; i < npts; ++i)
    if (xs[i] < 0 || xs[i] >= w || ys[i] < 0 || ys[i] >= h) return -1;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  if (dtype == DT_U8) filter_points<uint8_t>(a, xs, ys, nullptr, npts, (uint8_t*)vals, nthreads);
  else if (dtype == DT_U16)
    filter_points<uint16_t>(a, xs, ys, nullptr, npts, (uint16_t*)vals, nthreads);
  else filter_points<uint32_t>(a, xs, ys, nullptr, npts, (uint32_t*)vals, nthreads);
  return 0;
}

// As oracle_filter_points with a rank per listed pixel (ks[i], clamped to
// [0, n)).
int oracle_filter_points_ranks(const void* img, int w, int h, long long stride, int dtype,
                               const int* dx, const int* dy, int n, const int* ks,
                               int boundary, const int* xs, const int* ys, int npts,
                               void* vals, int nthreads) {
  Args a{(const unsigned char*)img, w, h, stride, dtype, dx, dy, n, 0, boundary};
  if (check(a) || npts < 0 || (npts > 0 && (!xs || !ys || !vals || !ks))) return -1;
  for (int i = 0; i < npts; ++i)
    if (xs[i] < 0 || xs[i] >= w || ys[i] < 0 || ys[i] >= h) return -1;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  if (dtype == DT_U8) filter_points<uint8_t>(a, xs, ys, ks, npts, (uint8_t*)vals, nthreads);
  else if (dtype == DT_U16)
    filter_points<uint16_t>(a, xs, ys, ks, npts, (uint16_t*)vals, nthreads);
  else filter_points<uint32_t>(a, xs, ys, ks, npts, (uint32_t*)vals, nthreads);
  return 0;
}

// Boundary index map, exposed so tests can pin it against numpy padding.
int oracle_remap(int x, int n, int boundary) { return remap(x, n, boundary); }

// totalOrder comparison, exposed for the float-order pins.
int oracle_total_order_less(uint32_t a, uint32_t b) { return total_order_less(a, b) ? 1 : 0; }

// Ordinal transform of a list of values (paper, "The Ordinal Transform and
// Compound Histogram"; Eq. 4 and Eq. 5): a stable sort of {value, index}.
// C[v] = value of ordinal v (reverse map), omega[v] = index holding ordinal v,
// ordinal[i] = ordinal of element i.  Duplicates get consecutive ordinals in
// index order.
int oracle_ordinal_transform(const void* vals, int n, int dtype, void* C, int* omega,
                             int* ordinal) {
  if (n < 0 || (n > 0 && (!vals || !C || !omega || !ordinal)) || dtype < 0 || dtype > 2) return -1;
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  auto value_bits = [&](int i) -> uint32_t {
    if (dtype == DT_U8) return ((const uint8_t*)vals)[i];
    if (dtype == DT_U16) return ((const uint16_t*)vals)[i];
    return ((const uint32_t*)vals)[i];
  };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    const uint32_t va = value_bits(a), vb = value_bits(b);
    return dtype == DT_F32 ? total_order_less(va, vb) : va < vb;
  });
  for (int v = 0; v < n; ++v) {
    const int i = idx[v];
    omega[v] = i;
    ordinal[i] = v;
    if (dtype == DT_U8) ((uint8_t*)C)[v] = (uint8_t)value_bits(i);
    else if (dtype == DT_U16) ((uint16_t*)C)[v] = (uint16_t)value_bits(i);
    else ((uint32_t*)C)[v] = value_bits(i);
  }
  return 0;
}

}  // extern "C"
