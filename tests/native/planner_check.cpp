// Host check of the tile planner (built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py).
//
// For every dtype, every disc radius 0..123 and a set of other windows, it
// walks the candidate plans, the default and tallest choices, the
// global-scratch plans and the bracketed plans, and checks that each LDS
// region (sort exchange, digit counters, omnigram, ordinal image, seed
// histograms, footprint tables) and each global-scratch region lies inside
// its buffer and overlaps no region that is live in the same phase of the
// tile (sort, or bands).  A layout overlap would otherwise show only as a
// rare mismatch on the GPU.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "mf_internal.h"

namespace {

int failures = 0;
long long checked = 0;

struct Reg {
  const char* name;
  long long lo, hi;   // [lo, hi)
};

int ru(int x, int m) { return (x + m - 1) / m * m; }

void fail(const std::string& what, const mf::ImageDesc& d, int dtype) {
  if (failures < 20)
    std::fprintf(stderr, "FAIL dtype %d tile %dx%d box %dx%d T %d gs %d br_cap %d: %s\n", dtype,
                 d.tw, d.th, d.bw, d.bh, d.T, d.gs, d.br_cap, what.c_str());
  ++failures;
}

void disjoint(const std::vector<Reg>& rs, long long limit, const mf::ImageDesc& d, int dtype,
              const char* phase) {
  for (size_t i = 0; i < rs.size(); ++i) {
    if (rs[i].lo < 0 || rs[i].hi > limit || rs[i].lo > rs[i].hi)
      fail(std::string(phase) + ": " + rs[i].name + " outside its buffer", d, dtype);
    for (size_t j = i + 1; j < rs.size(); ++j)
      if (rs[i].lo < rs[j].hi && rs[j].lo < rs[i].hi && rs[i].lo < rs[i].hi &&
          rs[j].lo < rs[j].hi)
        fail(std::string(phase) + ": " + rs[i].name + " overlaps " + rs[j].name, d, dtype);
  }
}

void check_plan(const mf::ImageDesc& d, int dtype, int lds_max, bool br) {
  ++checked;
  const int T = d.T;
  const int TP = ru(T, 8) + 16;
  const int ib = ru(2 * d.pitch * d.bh, 16);
  const int hb = mf::kHistBytes;
  const int nr4 = ru(d.nrows, 4);
  const int tab = 128 + 12 * nr4 + 16 * d.ncols;
  const long long L = d.lds_bytes;
  if (L > lds_max) fail("lds_bytes above the device limit", d, dtype);
  if (d.off_tab + tab != L) fail("tables do not end at lds_bytes", d, dtype);
  if (d.pitch < d.bw || (d.pitch / 2) % 2 != 1) fail("ordinal-image pitch", d, dtype);
  if (d.bw > 255 || d.bh > 256 || T > 65535 || T != d.bw * d.bh) fail("box limits", d, dtype);
  if (d.tw < 1 || d.tw > 64 || d.segs != 64 / d.tw ||
      d.band_rows * mf::kWaves * d.segs < d.th)
    fail("band layout does not cover the tile", d, dtype);
  if (((T - 1) >> d.hist_shift) > 255) fail("seed histogram bins", d, dtype);
  const Reg tables{"tables", d.off_tab, L};
  const Reg counters{"digit counters", d.off_B, (long long)d.off_B + mf::kCounterBytes};
  const Reg hist{"seed histograms", d.off_hist, (long long)d.off_hist + hb};
  if (br) {
    const int cap = d.br_cap;
    const int TPc = ru(cap + 1, 8) + 16;
    if (cap < mf::kThreads || cap > T) fail("bracket capacity", d, dtype);
    const Reg kbuf{"candidate exchange", 0, 4LL * cap};
    const Reg om{"omnigram", 0, 2LL * TPc};
    const Reg crev{"reverse map", d.off_C, (long long)d.off_C + 2LL * TPc};
    const Reg vals{"streamed box values", d.off_I, (long long)d.off_I + 2LL * T};
    const Reg I{"ordinal image", d.off_I, (long long)d.off_I + ib};
    disjoint({kbuf, vals, tables}, L, d, dtype, "load");
    disjoint({kbuf, counters, tables}, L, d, dtype, "sort");
    disjoint({om, crev, I, hist, tables}, L, d, dtype, "bands");
    if (d.imax != 0 && (long long)d.imax * mf::kThreads < T) fail("register load capacity", d, dtype);
    return;
  }
  if (d.gs) {
    const long long S = d.slot_bytes;
    // LDS during the sort: packed 16-bit key counters (2^16 for 16-bit and
    // float keys, 2^8 for 8-bit keys), and the digit counters of the float
    // keys' stable passes, in region B
    const long long pc = dtype == MF_U8 ? 512 : 131072;
    const Reg pcnt{"packed key counters", d.off_B, (long long)d.off_B + pc};
    disjoint({pcnt, tables}, L, d, dtype, "sort");
    const Reg dcnt{"stable-pass digit counters", d.off_B, (long long)d.off_B + 4LL * 16 * 257};
    disjoint({dcnt, tables}, L, d, dtype, "sort");
    if (dtype == MF_F32) {
      const Reg x0{"scratch x0", 0, 4LL * TP};
      const Reg x1{"scratch x1", d.off_x1, (long long)d.off_x1 + 4LL * TP};
      disjoint({x0, x1}, S, d, dtype, "scratch sort");
      // the last stable pass reads x1 and writes the omnigram in x0
      const Reg om{"scratch omnigram", d.off_p, (long long)d.off_p + 2LL * TP};
      disjoint({om, x1}, S, d, dtype, "scratch bands");
      if (om.lo < x0.lo || om.hi > x0.hi) fail("omnigram outside x0", d, dtype);
    } else {
      // the counting pass writes the omnigram directly
      const Reg om{"scratch omnigram", 0, 2LL * TP};
      disjoint({om}, S, d, dtype, "scratch sort and bands");
    }
    const Reg I{"ordinal image", d.off_I, (long long)d.off_I + ib};
    disjoint({I, hist, tables}, L, d, dtype, "bands");
    if (d.ipt * mf::kThreads < T) fail("elements per thread", d, dtype);
    return;
  }
  if ((long long)d.imax * mf::kThreads < T || (d.imax & 1) == 0) fail("register capacity", d, dtype);
  if (dtype == MF_F32) {
    const Reg keys{"sort keys", 0, 4LL * T};
    const Reg pay{"sort payload / omnigram", d.off_p, (long long)d.off_p + 2LL * TP};
    const Reg I{"ordinal image", d.off_I, (long long)d.off_I + ib};
    disjoint({keys, pay, counters, tables}, L, d, dtype, "sort");
    disjoint({pay, I, hist, tables}, L, d, dtype, "bands");
  } else {
    const Reg ex{"sort exchange", 0, 4LL * T};
    const Reg om{"omnigram", 0, 2LL * TP};
    const Reg I{"ordinal image", d.off_I, (long long)d.off_I + ib};
    disjoint({ex, counters, tables}, L, d, dtype, "sort");
    disjoint({om, I, hist, tables}, L, d, dtype, "bands");
  }
}

void walk(const mf_footprint* fp, int lds_max) {
  for (int dtype : {MF_U8, MF_U16, MF_F32}) {
    for (const mf::ImageDesc& d : mf::candidate_plans(dtype, fp, lds_max, 33))
      check_plan(d, dtype, lds_max, false);
    mf::ImageDesc d{};
    const int sizes[][2] = {{0, 0}, {4096, 4096}, {257, 131}, {2048, 2048}, {1, 1}, {3840, 2160}};
    for (const auto& s : sizes)
      if (mf::choose_plan(dtype, fp, lds_max, 33, &d, s[0], s[1], 256) == MF_OK)
        check_plan(d, dtype, lds_max, false);
    if (mf::choose_plan_tall(dtype, fp, lds_max, 33, &d) == MF_OK) check_plan(d, dtype, lds_max, false);
    for (int tw : {64, 56, 48, 32, 16, 8})
      for (int th = 8; th <= 256; th += 8) {
        if (mf::make_plan_gs(dtype, fp, lds_max, tw, th, &d) == MF_OK)
          check_plan(d, dtype, lds_max, false);
        if (mf::make_plan(dtype, fp, lds_max, tw, th, &d) == MF_OK)
          check_plan(d, dtype, lds_max, false);
        if (dtype != MF_F32 && mf::make_plan_br(dtype, fp, lds_max, tw, th, &d) == MF_OK)
          check_plan(d, dtype, lds_max, true);
      }
  }
}

}  // namespace

int main() {
  const int lds_max = 160 * 1024;
  std::vector<mf_footprint*> fps;
  for (int r = 0; r <= 123; ++r) {
    mf_footprint* fp = nullptr;
    if (mf_footprint_disc(r, &fp) != MF_OK) return 2;
    fps.push_back(fp);
  }
  for (long long r : {2LL, 7LL, 48LL, 96LL}) {
    mf_footprint* fp = nullptr;
    if (mf_footprint_disc_limit(r * (r + 1), &fp) != MF_OK) return 2;
    fps.push_back(fp);
  }
  {
    mf_footprint* fp = nullptr;
    if (mf_footprint_ellipse(60, 20, 30, &fp) != MF_OK) return 2;
    fps.push_back(fp);
    if (mf_footprint_regular_polygon(6, 40, 0, &fp) != MF_OK) return 2;
    fps.push_back(fp);
    const double tri[] = {0, -30, 40, 20, -10, 25};
    if (mf_footprint_polygon(tri, 3, &fp) != MF_OK) return 2;
    fps.push_back(fp);
  }
  for (mf_footprint* fp : fps) walk(fp, lds_max);
  for (mf_footprint* fp : fps) mf_footprint_destroy(fp);
  std::printf("planner_check: %lld plans checked, %d failures\n", checked, failures);
  return failures ? 1 : 0;
}
