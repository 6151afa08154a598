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

enum { CNT_BLOCKS = 0, CNT_SEEDS = 1, CNT_PIXELS = 2, CNT_SEED_TAPS = 3 };

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

template <int SHAPE>
__device__ __forceinline__ bool in_window(uint32_t loc, int cx, int cy, int limit, int dy_min,
                                          int nrows, const short2* rsp) {
  const int ox = (int)(loc & 255u) - cx, oy = (int)(loc >> 8) - cy;
  if (SHAPE == SHAPE_DISC) return ox * ox + oy * oy <= limit;
  const int r = oy - dy_min;
  if ((unsigned)r >= (unsigned)nrows) return false;
  const short2 s = rsp[r];
  return ox >= s.x && ox <= s.y;
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

  // 4. bands
  const int k = a.rank;
  uint32_t* hist = hist_all + wid * 256;
  int blocks = 0, seeds = 0, seed_taps = 0;
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
    const int cnew = k + delta;
    int mnew = m;
    for (int L = 0; L < segs * tw; ++L) {
      const int pL = __builtin_amdgcn_readlane(m, L);
      const int cL = __builtin_amdgcn_readlane(cnew, L);
      const int sL = L / tw;
      const int cxL = (L - sL * tw) - a.dx_min;
      const int cyL = (wid * segs + sL) * R + r - a.dy_min;
      const int mL = scan_select<KT, SHAPE>(pL, cL, k, cxL, cyL, a, kbuf, pbuf, rsp, blocks);
      mnew = set_lane(mL, L, mnew);
    }
    m = mnew;
    const int gx = tx0 + col, gy = ty0 + row0 + r;
    if (lane_active && gx < a.w && gy < a.h) store_out<KT>(a, gx, gy, kbuf, m);
  }

  if (a.counters && lane == 0) {
    atomicAdd(&a.counters[CNT_BLOCKS], (unsigned long long)blocks);
    atomicAdd(&a.counters[CNT_SEEDS], (unsigned long long)seed_taps);
  }
}

}  // namespace mf
