// The per-tile median engine (paper, "Method Summary" steps 1-5 and 7, and
// "GPU"), written as device functions so the plain kernel (one workgroup
// per tile) and the persistent batched kernel (tiles popped from a queue)
// share it.
//
// Tile pipeline, one workgroup of kThreads threads:
//   load    box = output tile grown by the window extent, boundary-remapped
//   sort    LSD radix sort of {key, location} -> W[v] (key and location of
//           ordinal v): the reverse map C and the omnigram (Eq. 4)
//   I       ordinal image, I(loc(v)) = v, 16-bit, row pitch chosen so rows
//           start in different LDS banks
//   bands   the tile is cut into bands of `band_rows` rows and each wave
//           owns `segs` bands side by side (a band is tw <= 64 columns, one
//           lane per column).  Per band:
//             seed  the first window of the band's first row is solved
//                   with a coarse histogram of its ordinals, refined by an
//                   omnigram scan (paper: seeds solved from low-precision
//                   histograms, then refined);
//             row   the rest of that row is solved by sliding the window
//                   right one pixel at a time, the wave testing one footprint
//                   row per lane for entering and leaving pixels (ballot +
//                   popcount) against the pivot, then scanning;
//             sweep every lane then slides its window down the band: count
//                   += #entering < pivot - #leaving < pivot over the window's
//                   columns (adjacent lanes read adjacent pixels), then each
//                   lane's window is refined by a wave-cooperative scan.
//   The pivot is the previous window's median ordinal m, whose count in the
//   previous window is exactly the rank k, so no separate count is stored
//   (the paper notes any pivot with a known count works).
//   out     C[m] for every output pixel inside the image.
#pragma once

#include "tile_common.h"

namespace mf {

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
  // LDS layout, bytes
  int off_p, off_B, off_hist, off_tab, lds_bytes;
  unsigned long long* counters;  // optional work counters (null: off)
};

// Work counters (accumulated only when ImageDesc::counters is set).
constexpr int kLaneBudget = 64;  // 4-ordinal groups a lane tests before the wave helps

enum {
  CNT_BLOCKS = 0,      // wave-cooperative omnigram blocks scanned (64 ordinals each)
  CNT_SEEDS = 1,       // seed windows solved from a histogram
  CNT_CYC_SORT = 2,    // shader clocks per wave: load + sort + ordinal image
  CNT_CYC_ROW = 3,     // shader clocks per wave: seeds + first rows of bands
  CNT_CYC_SWEEP = 4,   // shader clocks per wave: vertical sweeps
  CNT_WAVES = 5,       // waves that reported clocks
  CNT_GROUPS = 6,      // lane-parallel 4-ordinal groups tested (summed over lanes)
  CNT_SLOTS = 8
};

// Set lane L of a per-lane value to a wave-uniform value.
__device__ __forceinline__ int set_lane(int v, int L, int old) {
  return (int)(threadIdx.x & 63) == L ? v : old;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

template <int KT>
__device__ __forceinline__ uint32_t omega_at(const uint32_t* kbuf, const uint16_t* pbuf, int v) {
  return KT == KEY_F32 ? (uint32_t)pbuf[v] : (kbuf[v] & 0xffffu);
}

typedef short s2v __attribute__((ext_vector_type(2)));

// Window membership of an omnigram entry (paper, Eq. 2/3).  `w` holds the
// entry's box location in its low 16 bits (x: bits 0-7, y: bits 8-15);
// `cxy` is the window centre packed as x | y << 16.  The offset is formed
// with one byte permute and one packed 16-bit subtract; a disc then needs one
// 16-bit dot product, other shapes one span lookup by row.
template <int SHAPE>
__device__ __forceinline__ bool member_packed(uint32_t w, uint32_t cxy, int limit, int dy_min,
                                              int nrows, const short2* rsp) {
  const uint32_t pk = __builtin_amdgcn_perm(0u, w, 0x0c010c00u);
  const s2v d = __builtin_bit_cast(s2v, pk) - __builtin_bit_cast(s2v, cxy);
  if (SHAPE == SHAPE_DISC) return __builtin_amdgcn_sdot2(d, d, 0, false) <= limit;
  const int r = (int)d.y - dy_min;
  if ((unsigned)r >= (unsigned)nrows) return false;
  const short2 s = rsp[r];
  return (int)d.x >= (int)s.x && (int)d.x <= (int)s.y;
}

template <int SHAPE>
__device__ __forceinline__ bool in_window(uint32_t loc, int cx, int cy, int limit, int dy_min,
                                          int nrows, const short2* rsp) {
  return member_packed<SHAPE>(loc, (uint32_t)cx | ((uint32_t)cy << 16), limit, dy_min, nrows,
                              rsp);
}

// Load the four omnigram entries of aligned group q (q % 4 == 0).
template <int KT>
__device__ __forceinline__ void load_group(const uint32_t* kbuf, const uint16_t* pbuf, int q,
                                           uint32_t (&e)[4]) {
  if (KT == KEY_F32) {
    const uint2 g = *reinterpret_cast<const uint2*>(pbuf + q);
    e[0] = g.x;
    e[1] = g.x >> 16;
    e[2] = g.y;
    e[3] = g.y >> 16;
  } else {
    const uint4 g = *reinterpret_cast<const uint4*>(kbuf + q);
    e[0] = g.x;
    e[1] = g.y;
    e[2] = g.z;
    e[3] = g.w;
  }
}

// Rank selection for one window (wave-uniform arguments): given a pivot
// ordinal p and the number c of window members with ordinal < p, return the
// member ordinal m with exactly k members below it.  The omnigram is tested
// 64 ordinals per step, one per lane (Eq. 2/3), and the block's members
// counted with one ballot and popcount (paper, "Implementation").
template <int KT, int SHAPE>
__device__ __forceinline__ int scan_select(int p, int c, int k, int cx, int cy,
                                           const ImageDesc& a, const uint32_t* kbuf,
                                           const uint16_t* pbuf, const short2* rsp,
                                           int& blocks) {
  const int lane = threadIdx.x & 63;
  const int T = a.T;
  const int cap = (T >> 6) + 2;
  if (c <= k) {
    int need = k - c;
    int b = p;
    for (int it = 0; it < cap; ++it, b += 64) {
      const int v = b + lane;
      bool in = false;
      if (v < T) in = in_window<SHAPE>(omega_at<KT>(kbuf, pbuf, v), cx, cy, a.limit, a.dy_min,
                                       a.nrows, rsp);
      const uint64_t mask = __ballot(in);
      const int pc = __popcll(mask);
      ++blocks;
      if (need < pc) {
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        const uint64_t hit = __ballot(in && below == need);
        return b + (__ffsll((unsigned long long)hit) - 1);
      }
      need -= pc;
    }
  } else {
    int need = c - k;
    int b = p;
    for (int it = 0; it < cap; ++it, b -= 64) {
      const int v = b - 64 + lane;
      bool in = false;
      if (v >= 0 && v < T)
        in = in_window<SHAPE>(omega_at<KT>(kbuf, pbuf, v), cx, cy, a.limit, a.dy_min, a.nrows,
                              rsp);
      const uint64_t mask = __ballot(in);
      const int pc = __popcll(mask);
      ++blocks;
      if (need <= pc) {
        const int idx = pc - need;
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        const uint64_t hit = __ballot(in && below == idx);
        return b - 64 + (__ffsll((unsigned long long)hit) - 1);
      }
      need -= pc;
    }
  }
  return -1;  // unreachable for a consistent omnigram
}

// Lane-parallel rank selection: every lane refines its own window.  Same
// contract as scan_select, per lane: pivot p with c window members below it.
// The lane walks the omnigram from p upwards (c <= k) or downwards, four
// ordinals per LDS read (one aligned 16-byte group of W, or 8 bytes of the
// location array for float keys), counting members until the one of rank k
// is reached.  Used where windows move little between steps (vertical
// slides), so each lane walks a short distance.
template <int KT, int SHAPE>
__device__ __forceinline__ int lane_select(int& p, int& c, int k, uint32_t cxy, int budget,
                                           const ImageDesc& a, const uint32_t* kbuf,
                                           const uint16_t* pbuf, const short2* rsp, int& groups) {
  const bool up = c <= k;
  int need = up ? k - c : c - 1 - k;
  const int lo = up ? p : 0;
  const unsigned span = (unsigned)(up ? a.T - p : p);
  int q = up ? (p & ~3) : ((p - 1) & ~3);
  int below = c;                 // members below the scanned frontier
  int m = -1;
  int it = 0;
  while (q >= 0 && q < a.T && it < budget) {
    ++it;
    uint32_t e[4];
    load_group<KT>(kbuf, pbuf, q, e);
    uint32_t bits = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool ok = (unsigned)(q + j - lo) < span &&
                      member_packed<SHAPE>(e[j], cxy, a.limit, a.dy_min, a.nrows, rsp);
      bits |= (uint32_t)ok << j;
    }
    const int cnt = __builtin_popcount(bits);
    if (need < cnt) {
      int n = need, jsel = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int jj = up ? t : 3 - t;
        if ((bits >> jj) & 1u) {
          if (n == 0) jsel = jj;
          --n;
        }
      }
      m = q + jsel;
      break;
    }
    need -= cnt;
    if (up) {
      below += cnt;
      q += 4;
    } else {
      below -= cnt;
      q -= 4;
    }
  }
  groups += it;
  if (m < 0) {
    // frontier for a wave-cooperative finish: ordinals scanned so far lie
    // in [p, q) (up) or [q + 4, p) (down)
    p = up ? q : q + 4;
    if (p < 0) p = 0;
    if (p > a.T) p = a.T;
    c = below;
  }
  return m;
}

// Seed solve for the window centred at box (cx, cy): histogram of its
// ordinals >> hist_shift, pick the bin holding rank k, refine by scanning.
template <int KT, int SHAPE>
__device__ __forceinline__ int seed_solve(int cx, int cy, const ImageDesc& a,
                                          const uint32_t* kbuf, const uint16_t* pbuf,
                                          const uint16_t* I, uint32_t* hist, const short2* rsp,
                                          int& blocks) {
  const int lane = threadIdx.x & 63;
  const int k = a.rank;
#pragma unroll
  for (int j = 0; j < 4; ++j) hist[lane * 4 + j] = 0;
  wave_lds_sync();
  for (int i = lane; i < a.nrows; i += 64) {
    const short2 s = rsp[i];
    const int row = (cy + a.dy_min + i) * a.pitch + cx;
    for (int x = s.x; x <= s.y; ++x) atomicAdd(&hist[I[row + x] >> a.hist_shift], 1u);
  }
  wave_lds_sync();
  uint32_t h[4], sum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    h[j] = hist[lane * 4 + j];
    sum += h[j];
  }
  uint32_t cum = wave_inclusive_scan(sum, lane) - sum;
  int bin = -1;
  uint32_t base = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (bin < 0 && cum <= (uint32_t)k && (uint32_t)k < cum + h[j]) {
      bin = lane * 4 + j;
      base = cum;
    }
    cum += h[j];
  }
  const uint64_t who = __ballot(bin >= 0);
  const int src = __ffsll((unsigned long long)who) - 1;
  const int sbin = __builtin_amdgcn_readlane(bin, src);
  const int sbase = __builtin_amdgcn_readlane((int)base, src);
  return scan_select<KT, SHAPE>(sbin << a.hist_shift, sbase, k, cx, cy, a, kbuf, pbuf, rsp,
                                blocks);
}

// Count change when the window centred at box (cx, cy) moves right by one
// pixel, against pivot p: one footprint row per lane (rows beyond 64 in
// further passes); hrow[i] = (entering offset, leaving offset) of row i.
__device__ __forceinline__ int hstep_delta(int cx, int cy, int p, const ImageDesc& a,
                                           const uint16_t* I, const int2* hrow) {
  const int lane = threadIdx.x & 63;
  const int base = cy * a.pitch + cx;
  int delta = 0;
  for (int i0 = 0; i0 < a.nrows; i0 += 64) {
    const int i = i0 + lane;
    bool e = false, l = false;
    if (i < a.nrows) {
      const int2 o = hrow[i];
      e = I[base + o.x] < p;
      l = I[base + o.y] < p;
    }
    delta += __popcll(__ballot(e)) - __popcll(__ballot(l));
  }
  return delta;
}

template <int KT>
__device__ __forceinline__ void store_out(const ImageDesc& a, int gx, int gy, const uint32_t* kbuf,
                                          int m) {
  const long long o = (long long)gy * a.stride + gx;
  if (KT == KEY_U8) static_cast<uint8_t*>(a.out)[o] = (uint8_t)(kbuf[m] >> 16);
  if (KT == KEY_U16) static_cast<uint16_t*>(a.out)[o] = (uint16_t)(kbuf[m] >> 16);
  if (KT == KEY_F32) static_cast<uint32_t*>(a.out)[o] = key_to_f32(kbuf[m]);
}

// One output tile.  All threads of the workgroup must call it.
template <int KT, int SHAPE, int IMAX>
__device__ __forceinline__ void tile_body(const ImageDesc& a, int tile, unsigned char* smem) {
  const int T = a.T;
  uint32_t* kbuf = reinterpret_cast<uint32_t*>(smem);
  uint16_t* pbuf = reinterpret_cast<uint16_t*>(smem + a.off_p);
  uint16_t* cnt = reinterpret_cast<uint16_t*>(smem + a.off_B);
  uint16_t* I = reinterpret_cast<uint16_t*>(smem + a.off_B);
  uint32_t* hist_all = reinterpret_cast<uint32_t*>(smem + a.off_hist);
  uint32_t* wsum = reinterpret_cast<uint32_t*>(smem + a.off_tab);
  const int nr4 = (a.nrows + 3) & ~3;
  short2* rsp = reinterpret_cast<short2*>(smem + a.off_tab + 64);
  int2* hrow = reinterpret_cast<int2*>(smem + a.off_tab + 64 + 4 * nr4);
  int4* vtab = reinterpret_cast<int4*>(smem + a.off_tab + 64 + 12 * nr4);

  const int t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;
  const int tx0 = (tile % a.tiles_x) * a.tw, ty0 = (tile / a.tiles_x) * a.th;
  const long long clk0 = a.counters ? (long long)clock64() : 0;
  const int gx0 = tx0 + a.dx_min, gy0 = ty0 + a.dy_min;

  // footprint tables: row spans, per-row horizontal offsets, per-column
  // vertical offsets (down: entering, leaving; up: entering, leaving)
  for (int i = t; i < a.nrows; i += kThreads) {
    const short2 s = a.spans[i];
    rsp[i] = s;
    const int dy = a.dy_min + i;
    hrow[i] = make_int2(dy * a.pitch + s.y + 1, dy * a.pitch + s.x);
  }
  for (int j = t; j < a.ncols; j += kThreads) {
    const short2 s = a.spans[a.nrows + j];
    const int dx = a.dx_min + j;
    vtab[j] = make_int4((s.y + 1) * a.pitch + dx, s.x * a.pitch + dx,
                        (s.x - 1) * a.pitch + dx, s.y * a.pitch + dx);
  }

  // 1. load the box (striped order)
  uint32_t key[IMAX];
  uint16_t pos[IMAX];
  {
    int lx = t % a.bw, ly = t / a.bw;
    const int sx = kThreads % a.bw, sy = kThreads / a.bw;
#pragma unroll
    for (int i = 0; i < IMAX; ++i) {
      const int e = i * kThreads + t;
      uint32_t kk = 0, q = 0;
      if (e < T) {
        const int gx = remap(gx0 + lx, a.w, a.boundary);
        const int gy = remap(gy0 + ly, a.h, a.boundary);
        const long long off = (long long)gy * a.stride + gx;
        const uint32_t p = (uint32_t)((ly << 8) | lx);
        if (KT == KEY_U8) kk = ((uint32_t)static_cast<const uint8_t*>(a.img)[off] << 16) | p;
        if (KT == KEY_U16) kk = ((uint32_t)static_cast<const uint16_t*>(a.img)[off] << 16) | p;
        if (KT == KEY_F32) {
          kk = f32_to_key(static_cast<const uint32_t*>(a.img)[off]);
          q = p;
        }
      }
      key[i] = kk;
      pos[i] = (uint16_t)q;
      lx += sx;
      ly += sy;
      if (lx >= a.bw) {
        lx -= a.bw;
        ly += 1;
      }
    }
  }

  // 2. ordinal transform
  if (KT == KEY_U8)
    block_radix_sort<IMAX, false>(key, pos, T, 16, 2, kbuf, pbuf, cnt, wsum);
  else if (KT == KEY_U16)
    block_radix_sort<IMAX, false>(key, pos, T, 16, 4, kbuf, pbuf, cnt, wsum);
  else
    block_radix_sort<IMAX, true>(key, pos, T, 0, 8, kbuf, pbuf, cnt, wsum);

  // 3. ordinal image (overwrites the sort's count table)
  for (int v = t; v < T; v += kThreads) {
    const uint32_t loc = omega_at<KT>(kbuf, pbuf, v);
    I[(int)(loc >> 8) * a.pitch + (int)(loc & 255u)] = (uint16_t)v;
  }
  __syncthreads();
  const long long clk1 = a.counters ? (long long)clock64() : 0;

  // 4. bands
  const int k = a.rank;
  uint32_t* hist = hist_all + wid * 256;
  int blocks = 0, seeds = 0, seed_taps = 0, groups = 0;
  const int tw = a.tw, segs = a.segs, R = a.band_rows;
  const int seg = lane / tw, col = lane - seg * tw;
  const int band = wid * segs + seg;
  const int row0 = band * R;                 // first output row of this lane's band
  const int cxl = col - a.dx_min;            // lane's window centre, box coords
  int m = 0;

  // 4a. seed + first row of each band, one segment at a time
  for (int s = 0; s < segs; ++s) {
    const int cy = (wid * segs + s) * R - a.dy_min;
    int ms = seed_solve<KT, SHAPE>(0 - a.dx_min, cy, a, kbuf, pbuf, I, hist, rsp, blocks);
    ++seeds;
    m = set_lane(ms, s * tw, m);
    for (int c = 1; c < tw; ++c) {
      const int cxp = c - 1 - a.dx_min;
      const int cnt_new = k + hstep_delta(cxp, cy, ms, a, I, hrow);
      ms = scan_select<KT, SHAPE>(ms, cnt_new, k, cxp + 1, cy, a, kbuf, pbuf, rsp, blocks);
      m = set_lane(ms, s * tw + c, m);
    }
  }
  if (a.counters) seed_taps = seeds;  // taps per seed added on the host
  const long long clk2 = a.counters ? (long long)clock64() : 0;
  {
    const int gx = tx0 + col, gy = ty0 + row0;
    if (lane < segs * tw && gx < a.w && gy < a.h) store_out<KT>(a, gx, gy, kbuf, m);
  }

  // 4b. vertical sweep down each band
  const int lane_active = lane < segs * tw;
  for (int r = 1; r < R; ++r) {
    const int cy_prev = row0 + r - 1 - a.dy_min;
    const int lbase = cy_prev * a.pitch + cxl;
    int delta = 0;
    if (lane_active) {
      for (int j = 0; j < a.ncols; ++j) {
        const int4 o = vtab[j];
        delta += (int)(I[lbase + o.x] < m) - (int)(I[lbase + o.y] < m);
      }
    }
    int pl = m, cl = k + delta;
    int mnew = m;
    const uint32_t cxy = (uint32_t)cxl | ((uint32_t)(row0 + r - a.dy_min) << 16);
    if (lane_active)
      mnew = lane_select<KT, SHAPE>(pl, cl, k, cxy, kLaneBudget, a, kbuf, pbuf, rsp, groups);
    uint64_t left = __ballot(lane_active && mnew < 0);
    while (left) {
      const int L = __ffsll((unsigned long long)left) - 1;
      left &= left - 1;
      const int cxyL = __builtin_amdgcn_readlane((int)cxy, L);
      const int mL = scan_select<KT, SHAPE>(__builtin_amdgcn_readlane(pl, L),
                                            __builtin_amdgcn_readlane(cl, L), k, cxyL & 0xffff,
                                            cxyL >> 16, a, kbuf, pbuf, rsp, blocks);
      mnew = set_lane(mL, L, mnew);
    }
    m = mnew;
    const int gx = tx0 + col, gy = ty0 + row0 + r;
    if (lane_active && gx < a.w && gy < a.h) store_out<KT>(a, gx, gy, kbuf, m);
  }

  if (a.counters && lane == 0) {
    const long long clk3 = (long long)clock64();
    atomicAdd(&a.counters[CNT_BLOCKS], (unsigned long long)blocks);
    atomicAdd(&a.counters[CNT_SEEDS], (unsigned long long)seed_taps);
    atomicAdd(&a.counters[CNT_CYC_SORT], (unsigned long long)(clk1 - clk0));
    atomicAdd(&a.counters[CNT_CYC_ROW], (unsigned long long)(clk2 - clk1));
    atomicAdd(&a.counters[CNT_CYC_SWEEP], (unsigned long long)(clk3 - clk2));
    atomicAdd(&a.counters[CNT_WAVES], 1ull);
  }
  if (a.counters) {
    // lane-parallel groups differ per lane: sum over the wave
    unsigned long long gsum = (unsigned long long)groups;
    for (int d = 32; d >= 1; d >>= 1) gsum += __shfl_xor(gsum, d, 64);
    if (lane == 0) atomicAdd(&a.counters[CNT_GROUPS], gsum);
  }
}

}  // namespace mf
