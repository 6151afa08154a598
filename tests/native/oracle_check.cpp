// Host check of the brute-force oracle (built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py): every entry
// point on small planes of every dtype, ragged sizes, padded strides, both
// boundaries, windows larger than the image, rank maps with entries outside
// [0, N), and the ordinal transform; plus two properties that need no
// second implementation (radius 0 is the identity, a constant plane is a
// fixed point).  Memory errors and undefined behaviour abort the run.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

extern "C" {
int oracle_filter(const void* img, int w, int h, long long stride, int dtype, const int* dx,
                  const int* dy, int n, int rank, int boundary, void* out, long long out_stride,
                  int nthreads);
int oracle_filter_rank_map(const void* img, int w, int h, long long stride, int dtype,
                           const int* dx, const int* dy, int n, const int* rank_map,
                           long long rmap_stride, int boundary, void* out, long long out_stride,
                           int nthreads);
int oracle_filter_points(const void* img, int w, int h, long long stride, int dtype,
                         const int* dx, const int* dy, int n, int rank, int boundary,
                         const int* xs, const int* ys, int npts, void* vals, int nthreads);
int oracle_filter_points_ranks(const void* img, int w, int h, long long stride, int dtype,
                               const int* dx, const int* dy, int n, const int* ks, int boundary,
                               const int* xs, const int* ys, int npts, void* vals,
                               int nthreads);
int oracle_ordinal_transform(const void* vals, int n, int dtype, void* C, int* omega,
                             int* ordinal);
}

namespace {

int failures = 0;

void expect(bool ok, const char* what, int w, int h, int dt, int r) {
  if (!ok) {
    if (failures < 20) std::fprintf(stderr, "FAIL %s (w %d h %d dtype %d r %d)\n", what, w, h, dt, r);
    ++failures;
  }
}

void disc(int r, std::vector<int>& dx, std::vector<int>& dy) {
  dx.clear();
  dy.clear();
  for (int y = -r; y <= r; ++y)
    for (int x = -r; x <= r; ++x)
      if (x * x + y * y <= r * r) {
        dx.push_back(x);
        dy.push_back(y);
      }
}

}  // namespace

int main() {
  std::mt19937 rng(7);
  const int es[3] = {1, 2, 4};
  const int sizes[][2] = {{1, 1}, {1, 9}, {9, 1}, {5, 7}, {17, 3}, {33, 21}};
  std::vector<int> dx, dy;
  for (int dt = 0; dt < 3; ++dt)
    for (const auto& s : sizes)
      for (int r : {0, 1, 3, 12}) {
        const int w = s[0], h = s[1];
        const long long stride = w + 3;   // padded rows
        std::vector<unsigned char> img(stride * h * es[dt]);
        for (auto& b : img) b = (unsigned char)rng();
        std::vector<unsigned char> out(stride * h * es[dt], 0xAB), out2(out);
        disc(r, dx, dy);
        const int n = (int)dx.size();
        for (int bd = 0; bd < 2; ++bd) {
          expect(oracle_filter(img.data(), w, h, stride, dt, dx.data(), dy.data(), n, (n - 1) / 2,
                               bd, out.data(), stride, 2) == 0,
                 "filter", w, h, dt, r);
          if (r == 0)
            for (int y = 0; y < h; ++y)
              expect(std::memcmp(&out[y * stride * es[dt]], &img[y * stride * es[dt]],
                                 (size_t)w * es[dt]) == 0,
                     "radius 0 identity", w, h, dt, r);
          std::vector<int> rmap(stride * h);
          for (auto& v : rmap) v = (int)(rng() % (unsigned)(n + 6)) - 3;
          expect(oracle_filter_rank_map(img.data(), w, h, stride, dt, dx.data(), dy.data(), n,
                                        rmap.data(), stride, bd, out2.data(), stride, 3) == 0,
                 "rank map", w, h, dt, r);
          std::vector<int> xs, ys, ks;
          for (int i = 0; i < 25; ++i) {
            xs.push_back((int)(rng() % (unsigned)w));
            ys.push_back((int)(rng() % (unsigned)h));
            ks.push_back((int)(rng() % (unsigned)(n + 4)) - 2);
          }
          std::vector<unsigned char> pv(25 * es[dt]);
          expect(oracle_filter_points(img.data(), w, h, stride, dt, dx.data(), dy.data(), n,
                                      (n - 1) / 2, bd, xs.data(), ys.data(), 25, pv.data(), 1) == 0,
                 "points", w, h, dt, r);
          for (int i = 0; i < 25; ++i)
            expect(std::memcmp(&pv[i * es[dt]], &out[((long long)ys[i] * stride + xs[i]) * es[dt]],
                               es[dt]) == 0,
                   "points agree with the plane", w, h, dt, r);
          expect(oracle_filter_points_ranks(img.data(), w, h, stride, dt, dx.data(), dy.data(), n,
                                            ks.data(), bd, xs.data(), ys.data(), 25, pv.data(),
                                            2) == 0,
                 "points with ranks", w, h, dt, r);
        }
        // constant plane: a fixed point
        std::vector<unsigned char> cst(img.size());
        for (size_t i = 0; i < cst.size(); i += es[dt]) std::memcpy(&cst[i], &img[0], es[dt]);
        expect(oracle_filter(cst.data(), w, h, stride, dt, dx.data(), dy.data(), n, (n - 1) / 2, 1,
                             out.data(), stride, 2) == 0,
               "constant", w, h, dt, r);
        for (int y = 0; y < h; ++y)
          expect(std::memcmp(&out[y * stride * es[dt]], &cst[y * stride * es[dt]],
                             (size_t)w * es[dt]) == 0,
                 "constant fixed point", w, h, dt, r);
      }
  for (int dt = 0; dt < 3; ++dt)
    for (int n : {0, 1, 2, 13, 300}) {
      std::vector<unsigned char> v(n * es[dt] + 1), C(n * es[dt] + 1);
      for (auto& b : v) b = (unsigned char)(rng() % 4);   // many ties
      std::vector<int> om(n + 1), ord(n + 1);
      expect(oracle_ordinal_transform(v.data(), n, dt, C.data(), om.data(), ord.data()) == 0,
             "ordinal transform", n, 1, dt, 0);
      for (int i = 0; i < n; ++i) expect(om[ord[i]] == i, "omega inverts the ordinals", n, 1, dt, 0);
    }
  // argument errors are reported, not undefined
  expect(oracle_filter(nullptr, 4, 4, 4, 0, dx.data(), dy.data(), 1, 0, 0, nullptr, 4, 1) == -1,
         "null image rejected", 4, 4, 0, 0);
  std::printf("oracle_check: %d failures\n", failures);
  return failures ? 1 : 0;
}
