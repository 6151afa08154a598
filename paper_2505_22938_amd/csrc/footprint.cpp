// Footprint construction: shapes -> integer row/column spans.
//
// The paper tests window membership analytically (Eq. 3 for a disc) and
// notes that other convex shapes follow by changing that test ("Arbitrary
// Convex Kernel Shapes").  Here each shape is rasterised once on the host
// into per-row dx spans and per-column dy spans; the sliding steps walk the
// spans (one entering and one leaving pixel per column or row) and the
// omnigram test is a span lookup, so no geometry runs on the GPU.

#include <cmath>
#include <cstring>
#include <new>

#include <hip/hip_runtime.h>

#include "mf_internal.h"

namespace {

constexpr int kMaxExtent = 255;  // |dx|, |dy| limit: box coordinates are 8-bit

long long isqrt_ll(long long v) {
  long long r = (long long)std::sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// Build spans from a membership predicate over the square [-R, R]^2.
template <typename Pred>
int from_predicate(int R, Pred member, mf_footprint* fp) {
  int y0 = 1 << 30, y1 = -(1 << 30);
  std::vector<int> lo(2 * R + 1, 1), hi(2 * R + 1, 0);
  for (int dy = -R; dy <= R; ++dy) {
    int first = 1 << 30, last = -(1 << 30), count = 0;
    for (int dx = -R; dx <= R; ++dx) {
      if (member(dx, dy)) {
        if (first == (1 << 30)) first = dx;
        last = dx;
        ++count;
      }
    }
    if (count == 0) continue;
    if (count != last - first + 1) return MF_ERR_UNSUPPORTED;  // row not convex
    lo[dy + R] = first;
    hi[dy + R] = last;
    if (dy < y0) y0 = dy;
    if (dy > y1) y1 = dy;
  }
  if (y0 > y1) return MF_ERR_INVALID_ARG;  // empty window
  fp->dy_min = y0;
  fp->dy_max = y1;
  fp->row_lo.assign(lo.begin() + (y0 + R), lo.begin() + (y1 + R) + 1);
  fp->row_hi.assign(hi.begin() + (y0 + R), hi.begin() + (y1 + R) + 1);
  return MF_OK;
}

// Derive column spans, extents and tap count from the row spans; check
// that the rows are contiguous and every column is a single run.
int finish(mf_footprint* fp) {
  const int nr = (int)fp->row_lo.size();
  int x0 = 1 << 30, x1 = -(1 << 30);
  long long taps = 0;
  for (int i = 0; i < nr; ++i) {
    if (fp->row_lo[i] > fp->row_hi[i]) return MF_ERR_UNSUPPORTED;  // gap between rows
    x0 = std::min(x0, fp->row_lo[i]);
    x1 = std::max(x1, fp->row_hi[i]);
    taps += fp->row_hi[i] - fp->row_lo[i] + 1;
  }
  if (x0 < -kMaxExtent || x1 > kMaxExtent || fp->dy_min < -kMaxExtent ||
      fp->dy_max > kMaxExtent)
    return MF_ERR_UNSUPPORTED;
  fp->dx_min = x0;
  fp->dx_max = x1;
  fp->taps = (int)taps;
  const int nc = x1 - x0 + 1;
  fp->col_lo.assign(nc, 0);
  fp->col_hi.assign(nc, 0);
  for (int dx = x0; dx <= x1; ++dx) {
    int first = 1 << 30, last = -(1 << 30), count = 0;
    for (int i = 0; i < nr; ++i) {
      if (fp->row_lo[i] <= dx && dx <= fp->row_hi[i]) {
        const int dy = fp->dy_min + i;
        if (first == (1 << 30)) first = dy;
        last = dy;
        ++count;
      }
    }
    if (count == 0 || count != last - first + 1) return MF_ERR_UNSUPPORTED;
    fp->col_lo[dx - x0] = first;
    fp->col_hi[dx - x0] = last;
  }
  return MF_OK;
}

int emit(mf_footprint* fp, int rc, mf_footprint** out) {
  if (rc == MF_OK) rc = finish(fp);
  if (rc != MF_OK) {
    delete fp;
    return rc;
  }
  *out = fp;
  return MF_OK;
}

}  // namespace

extern "C" {

int mf_footprint_disc_limit(long long limit, mf_footprint** out) {
  if (!out || limit < 0) return MF_ERR_INVALID_ARG;
  if (limit > (long long)kMaxExtent * kMaxExtent) return MF_ERR_UNSUPPORTED;
  auto* fp = new (std::nothrow) mf_footprint;
  if (!fp) return MF_ERR_NOMEM;
  fp->kind = 0;
  fp->limit = limit;
  // Row dy holds |dx| <= floor(sqrt(limit - dy^2)).
  const int R = (int)isqrt_ll(limit);
  fp->dy_min = -R;
  fp->dy_max = R;
  for (int dy = -R; dy <= R; ++dy) {
    const int half = (int)isqrt_ll(limit - (long long)dy * dy);
    fp->row_lo.push_back(-half);
    fp->row_hi.push_back(half);
  }
  return emit(fp, MF_OK, out);
}

int mf_footprint_disc(int r, mf_footprint** out) {
  if (r < 0) return MF_ERR_INVALID_ARG;
  if (r > kMaxExtent) return MF_ERR_UNSUPPORTED;
  return mf_footprint_disc_limit((long long)r * r, out);
}

int mf_footprint_ellipse(double a, double b, double theta_deg, mf_footprint** out) {
  if (!out || !(a > 0) || !(b > 0) || !std::isfinite(theta_deg)) return MF_ERR_INVALID_ARG;
  if (std::max(a, b) > kMaxExtent) return MF_ERR_UNSUPPORTED;
  auto* fp = new (std::nothrow) mf_footprint;
  if (!fp) return MF_ERR_NOMEM;
  const double t = theta_deg * M_PI / 180.0, c = std::cos(t), s = std::sin(t);
  const int R = (int)std::ceil(std::max(a, b)) + 1;
  const int rc = from_predicate(R, [&](int dx, int dy) {
    const double u = dx * c + dy * s, v = -dx * s + dy * c;
    return (u / a) * (u / a) + (v / b) * (v / b) <= 1.0 + 1e-9;
  }, fp);
  return emit(fp, rc, out);
}

int mf_footprint_polygon(const double* xy, int n, mf_footprint** out) {
  if (!out || !xy || n < 3) return MF_ERR_INVALID_ARG;
  double area2 = 0, scale = 0;
  for (int i = 0; i < n; ++i) {
    const double x0 = xy[2 * i], y0 = xy[2 * i + 1];
    const double x1 = xy[2 * ((i + 1) % n)], y1 = xy[2 * ((i + 1) % n) + 1];
    if (!std::isfinite(x0) || !std::isfinite(y0)) return MF_ERR_INVALID_ARG;
    area2 += x0 * y1 - x1 * y0;
    scale = std::max(scale, std::hypot(x0, y0));
  }
  if (area2 == 0) return MF_ERR_INVALID_ARG;
  if (scale > kMaxExtent) return MF_ERR_UNSUPPORTED;
  const double orient = area2 > 0 ? 1.0 : -1.0;
  // Convexity: every turn between consecutive edges goes the way of the
  // winding (or straight on), and the turns add up to one full turn (a
  // self-intersecting star turns the same way at every vertex but winds
  // more than once).  The edge half-planes would otherwise describe a
  // different set than the polygon.
  {
    double turn = 0;
    for (int i = 0; i < n; ++i) {
      const int j = (i + 1) % n, k = (i + 2) % n;
      const double ax = xy[2 * j] - xy[2 * i], ay = xy[2 * j + 1] - xy[2 * i + 1];
      const double bx = xy[2 * k] - xy[2 * j], by = xy[2 * k + 1] - xy[2 * j + 1];
      const double cr = ax * by - ay * bx, dt = ax * bx + ay * by;
      const double mag = std::hypot(ax, ay) * std::hypot(bx, by);
      if (orient * cr < -1e-12 * mag) return MF_ERR_INVALID_ARG;
      turn += std::atan2(orient * cr, dt);
    }
    if (std::fabs(turn - 2 * M_PI) > 1e-6) return MF_ERR_INVALID_ARG;
  }
  const double tol = 1e-9 * std::max(scale, 1.0);
  // Inward edge normals, normalised, so the test is a signed distance.
  std::vector<double> nx(n), ny(n), off(n);
  for (int i = 0; i < n; ++i) {
    const double x0 = xy[2 * i], y0 = xy[2 * i + 1];
    const double x1 = xy[2 * ((i + 1) % n)], y1 = xy[2 * ((i + 1) % n) + 1];
    const double len = std::hypot(x1 - x0, y1 - y0);
    if (len == 0) return MF_ERR_INVALID_ARG;
    nx[i] = -orient * (y1 - y0) / len;
    ny[i] = orient * (x1 - x0) / len;
    off[i] = nx[i] * x0 + ny[i] * y0;
  }
  auto* fp = new (std::nothrow) mf_footprint;
  if (!fp) return MF_ERR_NOMEM;
  const int R = (int)std::ceil(scale) + 1;
  const int rc = from_predicate(R, [&](int dx, int dy) {
    for (int i = 0; i < n; ++i)
      if (nx[i] * dx + ny[i] * dy - off[i] < -tol) return false;
    return true;
  }, fp);
  return emit(fp, rc, out);
}

int mf_footprint_regular_polygon(int n_sides, double circumradius, double rot_deg,
                                 mf_footprint** out) {
  if (n_sides < 3 || !(circumradius > 0) || !std::isfinite(rot_deg)) return MF_ERR_INVALID_ARG;
  std::vector<double> xy(2 * n_sides);
  for (int k = 0; k < n_sides; ++k) {
    const double t = (rot_deg + 360.0 * k / n_sides) * M_PI / 180.0;
    xy[2 * k] = circumradius * std::cos(t);
    xy[2 * k + 1] = circumradius * std::sin(t);
  }
  return mf_footprint_polygon(xy.data(), n_sides, out);
}

int mf_footprint_info(const mf_footprint* fp, int* taps, int* rank, int* dx_min, int* dx_max,
                      int* dy_min, int* dy_max) {
  if (!fp) return MF_ERR_INVALID_ARG;
  if (taps) *taps = fp->taps;
  if (rank) *rank = (fp->taps - 1) / 2;
  if (dx_min) *dx_min = fp->dx_min;
  if (dx_max) *dx_max = fp->dx_max;
  if (dy_min) *dy_min = fp->dy_min;
  if (dy_max) *dy_max = fp->dy_max;
  return MF_OK;
}

int mf_footprint_row_spans(const mf_footprint* fp, int* x_lo, int* x_hi) {
  if (!fp || !x_lo || !x_hi) return MF_ERR_INVALID_ARG;
  std::memcpy(x_lo, fp->row_lo.data(), fp->row_lo.size() * sizeof(int));
  std::memcpy(x_hi, fp->row_hi.data(), fp->row_hi.size() * sizeof(int));
  return MF_OK;
}

void mf_footprint_destroy(mf_footprint* fp) {
  if (!fp) return;
  for (auto& d : fp->dev) {
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess) {
      (void)hipSetDevice(d.device);
      (void)hipFree(d.ptr);
      (void)hipSetDevice(cur);
    }
  }
  delete fp;
}

}  // extern "C"

namespace mf {

size_t footprint_span_table_len(const mf_footprint* fp) {
  return 2 * (fp->row_lo.size() + fp->col_lo.size());
}

size_t footprint_span_table(const mf_footprint* fp, int16_t* dst) {
  const size_t nr = fp->row_lo.size(), nc = fp->col_lo.size();
  for (size_t i = 0; i < nr; ++i) {
    dst[2 * i] = (int16_t)fp->row_lo[i];
    dst[2 * i + 1] = (int16_t)fp->row_hi[i];
  }
  for (size_t i = 0; i < nc; ++i) {
    dst[2 * (nr + i)] = (int16_t)fp->col_lo[i];
    dst[2 * (nr + i) + 1] = (int16_t)fp->col_hi[i];
  }
  return 2 * (nr + nc);
}

const mf_footprint* footprint_with_top_row(const mf_footprint* fp) {
  static std::mutex mu;
  static std::vector<std::pair<std::string, mf_footprint*>> cache;
  const std::string k = tune_key(MF_U16, fp);
  std::lock_guard<std::mutex> lock(mu);
  for (auto& e : cache)
    if (e.first == k) return e.second;
  auto* x = new mf_footprint;
  x->kind = fp->kind;
  x->limit = fp->limit;
  x->dx_min = fp->dx_min;
  x->dx_max = fp->dx_max;
  x->dy_min = fp->dy_min - 1;
  x->dy_max = fp->dy_max;
  x->taps = fp->taps;
  x->row_lo.push_back(1);   // an empty span: no pixel of this row is in the window
  x->row_hi.push_back(0);
  x->row_lo.insert(x->row_lo.end(), fp->row_lo.begin(), fp->row_lo.end());
  x->row_hi.insert(x->row_hi.end(), fp->row_hi.begin(), fp->row_hi.end());
  x->col_lo = fp->col_lo;
  x->col_hi = fp->col_hi;
  cache.emplace_back(k, x);
  return x;
}

int footprint_device_table(const mf_footprint* fp, int device, const void** table,
                           hipStream_t stream) {
  std::lock_guard<std::mutex> lock(fp->mu);
  for (auto& d : fp->dev)
    if (d.device == device) {
      *table = d.ptr;
      return MF_OK;
    }
  // the upload allocates and copies synchronously: not while the caller's
  // stream is being captured into a graph
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap) != hipSuccess) return MF_ERR_HIP;
  if (cap != hipStreamCaptureStatusNone) return MF_ERR_UNSUPPORTED;
  std::vector<int16_t> host(footprint_span_table_len(fp));
  footprint_span_table(fp, host.data());
  void* p = nullptr;
  if (hipMalloc(&p, host.size() * sizeof(int16_t)) != hipSuccess) return MF_ERR_NOMEM;
  if (hipMemcpy(p, host.data(), host.size() * sizeof(int16_t), hipMemcpyHostToDevice) !=
      hipSuccess) {
    (void)hipFree(p);
    return MF_ERR_HIP;
  }
  fp->dev.push_back({device, p});
  *table = p;
  return MF_OK;
}

}  // namespace mf
