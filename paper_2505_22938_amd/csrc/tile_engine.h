// The per-tile median engine (paper, "Method Summary" steps 1-5 and 7, and
// "GPU"), written as device functions so the plain kernel (one workgroup
// per tile) and the persistent batched kernel (tiles popped from a queue)
// share it.
//
// Tile pipeline, one workgroup of kThreads threads:
//   load    box = output tile grown by the window extent, boundary-remapped
//   sort    radix sort of {key, location} -> the omnigram W[v] (location of
//           ordinal v; Eq. 4): one counting pass over the low key bits by
//           LDS atomics (order among equal digits free, since ties may take
//           their ordinals in any order), then stable 4-bit LSD passes
//   I       ordinal image, I(loc(v)) = v, 16-bit, row pitch chosen so rows
//           start in different LDS banks
//   bands   the tile is cut into bands of `band_rows` rows (the last one
//           may be shorter) and each wave owns `segs` = 64 / tw bands side
//           by side (a band is tw <= 64 columns, one lane per column; lanes
//           past segs * tw and bands past the tile sit out).  Per band:
//             seeds the band's first row is cut into chunks of 16 columns;
//                   the first chunk's window is solved with a coarse
//                   histogram of its ordinals refined by an omnigram scan
//                   (paper: seeds solved from low-precision histograms, then
//                   refined), each later chunk's by moving the previous
//                   chunk's window 16 columns right;
//             row   the four 16-lane rows of the wave take one chunk each
//                   and slide their windows right one pixel at a time in
//                   lockstep (paper: short horizontal slides from many
//                   seeds), counting entering and leaving pixels against
//                   the pivot across the row's lanes and refining by a
//                   row-wide omnigram scan;
//             sweep every lane then slides its window down the band: count
//                   += #entering < pivot - #leaving < pivot over the window's
//                   columns (adjacent lanes read adjacent pixels), then each
//                   lane walks the omnigram for its window's new median;
//                   lanes with long walks are finished four at a time by
//                   16-lane rows.
//   The pivot is the previous window's median ordinal m, whose count in the
//   previous window is exactly the rank k, so no separate count is stored
//   (the paper notes any pivot with a known count works).
//   out     C[m] for every output pixel inside the image.
#pragma once

#include <type_traits>

#include "tile_common.h"

namespace mf {


// Work counters (accumulated only when ImageDesc::counters is set).
constexpr int kLaneBudget = 32;  // 8-ordinal groups a lane tests before the wave helps

enum {
  CNT_BLOCKS = 0,      // wave-cooperative omnigram blocks scanned (64 ordinals each)
  CNT_SEEDS = 1,       // seed windows solved from a histogram
  CNT_CYC_SORT = 2,    // shader clocks per wave: load + sort + ordinal image
  CNT_CYC_ROW = 3,     // shader clocks per wave: seeds + first rows of bands
  CNT_CYC_SWEEP = 4,   // shader clocks per wave: vertical sweeps
  CNT_WAVES = 5,       // waves that reported clocks
  CNT_GROUPS = 6,      // lane-parallel 8-ordinal groups tested (summed over lanes)
  CNT_SORTED = 7,      // box pixels ranked by the ordinal transform (summed over tiles)
  CNT_CYC_SEED = 8,    // shader clocks per wave spent in seed solves (part of CNT_CYC_ROW)
  CNT_CYC_LOAD = 9,    // shader clocks per wave from tile start to box loaded (part of CNT_CYC_SORT)
  CNT_SLOTS = 10
};

// Set lane L of a per-lane value to a wave-uniform value.
__device__ __forceinline__ int set_lane(int v, int L, int old) {
  return (int)(threadIdx.x & 63) == L ? v : old;
}

// 64-lane mask of a per-lane condition (straight from the compare, no
// detour through an integer predicate).
__device__ __forceinline__ uint64_t wave_ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}


typedef short s2v __attribute__((ext_vector_type(2)));

// d.x * d.x + d.y * d.y + c as one VOP3P dot product (the addend from a
// scalar register, no accumulator copy).
__device__ __forceinline__ int dot2_sq_add(s2v d, int c) {
  int r;
  asm("v_dot2_i32_i16 %0, %1, %1, %2" : "=v"(r) : "v"(d), "s"(c));
  return r;
}

// Footprint geometry seen by the scans, walks and seed solves: the disc's
// squared-radius limit, the first row offset and the row count (row spans
// are in the LDS table rsp, index dy - dy_min).  One per output plane when
// planes use different windows.
struct Fp {
  int limit, dy_min, nrows;
};

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
  // dx^2 + dy^2 - (limit + 1) < 0: the threshold rides in the dot product's addend
  if (SHAPE == SHAPE_DISC) return dot2_sq_add(d, -limit - 1) < 0;
  const int r = (int)d.y - dy_min;
  if ((unsigned)r >= (unsigned)nrows) return false;
  const short2 s = rsp[r];
  return (int)d.x >= (int)s.x && (int)d.x <= (int)s.y;
}


// Membership of the eight omnigram entries in g (two per word), bit j for
// entry j.  Disc: per entry one byte permute, one packed subtract and one
// dot product whose sign bit is shifted into the mask (v_alignbit).
template <int SHAPE>
__device__ __forceinline__ uint32_t group_mask(const uint4& g, uint32_t cxy, const Fp& f,
                                               const short2* rsp) {
  const uint32_t wv[4] = {g.x, g.y, g.z, g.w};
  if constexpr (SHAPE == SHAPE_DISC) {
    const s2v c = __builtin_bit_cast(s2v, cxy);
    const int negl = -f.limit - 1;
    // all eight dot products first, then the sign bits shifted in (keeps
    // each product's consumer away from it)
    int r[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t pk = __builtin_amdgcn_perm(0u, wv[j >> 1], (j & 1) ? 0x0c030c02u : 0x0c010c00u);
      const s2v d = __builtin_bit_cast(s2v, pk) - c;
      r[j] = dot2_sq_add(d, negl);
    }
    uint32_t acc = 0;
#pragma unroll
    for (int j = 7; j >= 0; --j) acc = __builtin_amdgcn_alignbit(acc, (uint32_t)r[j], 31u);
    return acc;
  } else {
    uint32_t bits = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t e = (j & 1) ? (wv[j >> 1] >> 16) : wv[j >> 1];
      bits |= (uint32_t)member_packed<SHAPE>(e, cxy, f.limit, f.dy_min, f.nrows, rsp) << j;
    }
    return bits;
  }
}

// A 16-bit LDS load the compiler keeps where it is written (a volatile
// access in the LDS address space), so a prefetch is not sunk into the path
// that consumes it.  Only for arrays in LDS (OM_LDS: not the global-scratch
// omnigram of large boxes).
__device__ __forceinline__ uint32_t lds_load_early(const uint16_t* base, int i) {
  using lds_u16 = const volatile __attribute__((address_space(3))) uint16_t;
  return *((lds_u16*)base + i);
}

// Rank selection for one window (wave-uniform arguments): given a pivot
// ordinal p and the number c of window members with ordinal < p, return the
// member ordinal m with exactly k members below it.  The omnigram is tested
// 64 ordinals per step, one per lane (Eq. 2/3), and the block's members
// counted with one ballot and popcount (paper, "Implementation").  The next
// block is loaded while the current one is tested.  pre_up / pre_dn are
// this lane's entries of the first block above p ([p, p+64)) and below p
// ([p-64, p)), loaded by the caller (only the one for the taken direction
// is used).
// T bounds the valid ordinals ([0, T) here; entries beyond are padding).
// Returns -1 if no member of rank k exists among the valid ordinals (only
// possible when some pixels are outside the omnigram, see BR below); c_end
// then receives the number of members below the end reached (below T going
// up, below ordinal 0 going down).
template <int SHAPE, bool OM_LDS = true, typename D>
__device__ __forceinline__ int scan_core(int p, int c, int k, uint32_t cxy, int T,
                                         const D& a, const Fp& f, const uint16_t* om,
                                         const short2* rsp, int& blocks, uint32_t pre_up,
                                         uint32_t pre_dn, int& c_end) {
  const int lane = threadIdx.x & 63;
  const int cap = (T >> 6) + 2;
  if (c <= k) {
    int need = k - c;
    int b = p;
    uint32_t cur = pre_up;
    for (int it = 0; it < cap && b < T; ++it, b += 64) {
      // next block's entry, loaded before this block is tested (volatile:
      // the load stays here instead of sinking into the continue path)
      const int ni = min(max(b + 64 + lane, 0), T - 1);
      const uint32_t nxt = OM_LDS ? lds_load_early(om, ni) : (uint32_t)om[ni];
      // both tests evaluated (no branch; cur is always a loaded entry) and
      // combined as lane masks
      const uint64_t mask =
          wave_ballot(b + lane < T) &
          wave_ballot(member_packed<SHAPE>(cur, cxy, f.limit, f.dy_min, f.nrows, rsp));
      const int pc = __popcll(mask);
      ++blocks;
      if (need < pc) {
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        const uint64_t hit = mask & wave_ballot(below == need);
        return b + (__ffsll((unsigned long long)hit) - 1);
      }
      need -= pc;
      cur = nxt;
    }
    c_end = k - need;   // members below T
  } else {
    int need = c - k;
    int b = p;
    uint32_t cur = pre_dn;
    for (int it = 0; it < cap && b > 0; ++it, b -= 64) {
      const int ni = max(b - 128 + lane, 0);
      const uint32_t nxt = OM_LDS ? lds_load_early(om, ni) : (uint32_t)om[ni];
      const int v = b - 64 + lane;
      const uint64_t mask =
          wave_ballot((v >= 0) & (v < T)) &
          wave_ballot(member_packed<SHAPE>(cur, cxy, f.limit, f.dy_min, f.nrows, rsp));
      const int pc = __popcll(mask);
      ++blocks;
      if (need <= pc) {
        const int idx = pc - need;
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        const uint64_t hit = mask & wave_ballot(below == idx);
        return b - 64 + (__ffsll((unsigned long long)hit) - 1);
      }
      need -= pc;
      cur = nxt;
    }
    c_end = k + need;   // members below ordinal 0
  }
  return -1;
}

template <int KT, int SHAPE, bool OM_LDS = true, typename D>
__device__ __forceinline__ int scan_select(int p, int c, int k, int cx, int cy, int T,
                                           const D& a, const Fp& f, const uint16_t* om,
                                           const short2* rsp, int& blocks, int& c_end) {
  const int lane = threadIdx.x & 63;
  const uint32_t cxy = (uint32_t)cx | ((uint32_t)cy << 16);
  const bool up = c <= k;
  const uint32_t pre = up ? om[min(max(p + lane, 0), T - 1)] : om[max(p - 64 + lane, 0)];
  return scan_core<SHAPE, OM_LDS>(p, c, k, cxy, T, a, f, om, rsp, blocks, pre, pre, c_end);
}

// Lane-parallel rank selection: every lane refines its own window.  Same
// contract as scan_select, per lane: pivot p with c window members below it.
// The lane walks the omnigram from p upwards (c <= k) or downwards, eight
// ordinals per 16-byte LDS read, counting members until the one of rank k is
// reached.  Used where windows move little between steps (vertical slides),
// so each lane walks a short distance.  The omnigram is padded past T with
// entries located outside the box, so only the first group needs a range
// test.  After `budget` groups an unfinished lane returns -1 with (p, c) set
// to its frontier, for a wave-cooperative finish.
template <int SHAPE>
__device__ __forceinline__ int lane_select(int& p, int& c, int k, uint32_t cxy, int budget, int T,
                                           const Fp& f, const uint16_t* om,
                                           const short2* rsp, int& groups) {
  const bool up = c <= k;
  int need = up ? k - c : c - 1 - k;
  int q = up ? (p & ~7) : ((p - 1) & ~7);
  const int need0 = need;   // members passed = need0 - need
  int m = -1, it = 0;
  uint32_t bits = 0;
  // first (partial) group: only ordinals in [p, T) (up) or [0, p) (down);
  // p > 0 whenever the walk goes down, so q >= 0
  {
    const uint4 g = *reinterpret_cast<const uint4*>(om + max(q, 0));
    uint32_t range;
    if (up) {
      const int hi = T - q;   // entries j < hi are below T
      range = (0xffu << (p - q)) & (hi >= 8 ? 0xffu : ((1u << max(hi, 0)) - 1u));
    } else {
      range = (1u << (p - q)) - 1u;
    }
    bits = group_mask<SHAPE>(g, cxy, f, rsp) & range;
    const int cnt = __builtin_popcount(bits);
    ++it;
    if (need < cnt) {
      m = q;   // selection below
    } else {
      need -= cnt;
      q += up ? 8 : -8;
    }
  }
  // full groups: count members only
  while (m < 0 && (up ? q < T : q >= 0) && it < budget) {
    const uint4 g = *reinterpret_cast<const uint4*>(om + q);
    bits = group_mask<SHAPE>(g, cxy, f, rsp);
    const int cnt = __builtin_popcount(bits);
    ++it;
    if (need < cnt) {
      m = q;
      break;
    }
    need -= cnt;
    q += up ? 8 : -8;
  }
  if (m >= 0) {
    // the need-th member of the group from the bottom going up, from the
    // top going down (= member cnt - 1 - need from the bottom): the n-th set
    // bit of the 8-bit mask by halving (nibble, pair, bit)
    uint32_t x = bits;
    int n = up ? need : __builtin_popcount(bits) - 1 - need;
    int jsel = 0;
    int cn = __builtin_popcount(x & 15u);
    if (n >= cn) { n -= cn; jsel += 4; x >>= 4; }
    cn = __builtin_popcount(x & 3u);
    if (n >= cn) { n -= cn; jsel += 2; x >>= 2; }
    if (n >= (int)(x & 1u)) jsel += 1;
    m = q + jsel;
  }
  groups += it;
  if (m < 0) {
    p = up ? q : q + 8;
    if (p < 0) p = 0;
    if (p > T) p = T;
    c += up ? need0 - need : need - need0;   // members below the frontier
  }
  return m;
}

// Seed solve for the window centred at box (cx, cy): histogram of its
// ordinals >> hshift, pick the bin holding rank k (wave-uniform), refine by
// scanning.
// BR (bracketed tiles): ordinal 0 stands for every pixel below the bracket
// and 0xffff for every pixel above it.  If the median is below (above) the
// bracket, returns -1 with esc_p = 1 (T) and esc_c = the exact number of
// window members below that ordinal, so sliding can go on from there.
template <int KT, int SHAPE, bool BR, bool OM_LDS = true, typename D>
__device__ __forceinline__ int seed_solve(int cx, int cy, int T, int hshift, int k, const D& a,
                                          const Fp& f, const uint16_t* om, const uint16_t* I, uint32_t* hist,
                                          const short2* rsp, int& blocks, int& esc_p,
                                          int& esc_c) {
  const int lane = threadIdx.x & 63;
  int zeros = 0;
  // 256 bins of 32-bit counts (a bin's word address is the ordinal shifted,
  // no packing arithmetic per update).  Bracketed tiles: pixels below the
  // bracket (ordinal 0) are counted in a register and pixels above it
  // (0xffff) skipped, so the histogram holds only in-bracket ordinals and no
  // bin is hammered by atomics.
  reinterpret_cast<uint4*>(hist)[lane] = make_uint4(0u, 0u, 0u, 0u);
  wave_lds_sync();
  // one footprint row per lane; eight ordinals read before their eight
  // histogram updates, so the reads overlap instead of each waiting behind
  // the previous update
  constexpr int kBatch = 8;
  for (int i = lane; i < f.nrows; i += 64) {
    const short2 s = rsp[i];
    const int row = (cy + f.dy_min + i) * a.pitch + cx;
    for (int x0 = s.x; x0 <= s.y; x0 += kBatch) {
      uint32_t iv[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) iv[j] = I[row + min(x0 + j, (int)s.y)];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        if (x0 + j > s.y) break;
        if (BR) {
          zeros += iv[j] == 0;
          if (iv[j] == 0 || iv[j] == 0xffffu) continue;
        }
        atomicAdd(&hist[iv[j] >> hshift], 1u);
      }
    }
  }
  if (BR)
    for (int d = 32; d >= 1; d >>= 1) zeros += __shfl_xor(zeros, d, 64);
  wave_lds_sync();
  const int target = k - zeros;   // rank among the histogram's entries
  if (BR && target < 0) {          // median below the bracket
    esc_p = 1;
    esc_c = zeros;
    return -1;
  }
  const uint4 hw = reinterpret_cast<const uint4*>(hist)[lane];
  uint32_t h[4] = {hw.x, hw.y, hw.z, hw.w};
  const uint32_t sum = h[0] + h[1] + h[2] + h[3];
  uint32_t cum = wave_inclusive_scan(sum, lane) - sum;
  int bin = -1;
  uint32_t base = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (bin < 0 && cum <= (uint32_t)target && (uint32_t)target < cum + h[j]) {
      bin = lane * 4 + j;
      base = cum;
    }
    cum += h[j];
  }
  const uint64_t who = wave_ballot(bin >= 0);
  if (BR && who == 0) {             // median above the bracket
    esc_p = T;
    esc_c = zeros + __builtin_amdgcn_readlane((int)cum, 63);
    return -1;
  }
  const int src = __ffsll((unsigned long long)who) - 1;
  const int sbin = __builtin_amdgcn_readlane(bin, src);
  const int sbase = __builtin_amdgcn_readlane((int)base, src) + zeros;
  int p = sbin << hshift;
  if (BR && p == 0) p = 1;          // ordinal 1; entries below it are the zeros
  int c_end = 0;
  return scan_select<KT, SHAPE, OM_LDS>(p, sbase, k, cx, cy, T, a, f, om, rsp, blocks, c_end);
}

// 16-lane rows of a wave (DPP rows).  Call with every lane of the wave
// active; lanes that should not contribute pass 0.
// Sum over the lane's row, in every lane of the row.
__device__ __forceinline__ int row_sum16(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x128, 0xf, 0xf, false);   // row_ror:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x124, 0xf, 0xf, false);   // row_ror:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x122, 0xf, 0xf, false);   // row_ror:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x121, 0xf, 0xf, false);   // row_ror:1
  return x;
}
// Largest value over the lane's row, in every lane of the row.
__device__ __forceinline__ int row_max16(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x128, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x124, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x122, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x121, 0xf, 0xf, false));
  return x;
}
// Inclusive prefix sum along the lane's row (row_shr with zero fill).
__device__ __forceinline__ int row_incl_scan16(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);    // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);    // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);    // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);    // row_shr:8
  return x;
}

// Index (0..7) of the n-th set bit (from bit 0) of an 8-bit mask that has
// more than n set bits: halving by nibble, pair and bit.
__device__ __forceinline__ int nth_bit8(uint32_t x, int n) {
  int jsel = 0;
  int cn = __builtin_popcount(x & 15u);
  if (n >= cn) { n -= cn; jsel += 4; x >>= 4; }
  cn = __builtin_popcount(x & 3u);
  if (n >= cn) { n -= cn; jsel += 2; x >>= 2; }
  if (n >= (int)(x & 1u)) jsel += 1;
  return jsel;
}

// Rank selection for one window per 16-lane row, the row's lanes
// cooperating (row-uniform arguments; `act` false: the row has no window).
// Same contract as scan_select: pivot p with c window members below it;
// returns the member ordinal with exactly k members below it.  Each step of
// the loop tests 128 ordinals of the omnigram, eight per lane (one 16-byte
// read), upwards from p (c <= k) or downwards from p - 1, and a prefix sum
// of the lanes' member counts along the row locates the one holding rank k
// (paper, Eq. 2/3 and the block-wise refinement of "Implementation", with a
// block of 128).  Ordinals at or past T (going up) or below 0 (going down)
// are never members: -1 is returned with c_end = the number of members
// below T (up) or below ordinal 0 (down), as scan_core does.
template <int SHAPE>
__device__ __forceinline__ int row_select(bool act, int p, int c, int k, uint32_t cxy, int T,
                                          const Fp& f, const uint16_t* om, const short2* rsp,
                                          int& groups, int& c_end) {
  const int j = threadIdx.x & 15;
  const bool up = c <= k;
  int need = up ? k - c : c - 1 - k;   // members to pass before the one sought
  int q = up ? (p & ~7) : ((p - 1) & ~7);
  bool done = !act;
  int res = -1;
  const int cap = (T >> 7) + 2;
  for (int it = 0; it < cap; ++it) {
    if (wave_ballot(!done) == 0) break;
    const int qj = up ? q + 8 * j : q - 8 * j;
    const bool valid = !done && (up ? qj < T : qj >= 0);
    uint32_t bits = 0;
    if (valid) {
      const uint4 g = *reinterpret_cast<const uint4*>(om + qj);
      bits = group_mask<SHAPE>(g, cxy, f, rsp);
      if (it == 0 && j == 0) bits &= up ? (0xffu << (p - q)) : ((1u << (p - q)) - 1u);
      ++groups;
    }
    const int pc = __builtin_popcount(bits);
    const int incl = row_incl_scan16(pc);
    const int tot = __shfl(incl, (int)(threadIdx.x | 15u), 64);
    const int before = incl - pc;
    int cand = -1;
    if (valid && before <= need && need < incl) {
      const int n = need - before;
      cand = up ? qj + nth_bit8(bits, n) : qj + nth_bit8(bits, pc - 1 - n);
    }
    // (the row's candidate reaches its lanes only on an iteration where some
    // row finds its member)
    if (wave_ballot(!done && need < tot) != 0) cand = row_max16(cand);
    if (!done) {
      if (need < tot) {
        res = cand;
        done = true;
      } else {
        need -= tot;
        q += up ? 128 : -128;
        if (up ? q >= T : q < 0) {
          done = true;
          c_end = up ? k - need : k + 1 + need;
        }
      }
    }
  }
  return res;
}

// Rank selection for one window by the whole wave (wave-uniform
// arguments), 512 ordinals per step, eight per lane; otherwise as
// row_select.  Used where the member sought may lie far from the pivot.
template <int SHAPE>
__device__ __forceinline__ int wave_select(int p, int c, int k, uint32_t cxy, int T, const Fp& f,
                                           const uint16_t* om, const short2* rsp, int& groups,
                                           int& c_end) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const bool up = c <= k;
  int need = up ? k - c : c - 1 - k;
  int q = up ? (p & ~7) : ((p - 1) & ~7);
  const int cap = (T >> 9) + 2;
  for (int it = 0; it < cap; ++it) {
    const int ql = up ? q + 8 * lane : q - 8 * lane;
    const bool valid = up ? ql < T : ql >= 0;
    uint32_t bits = 0;
    if (valid) {
      const uint4 gv = *reinterpret_cast<const uint4*>(om + ql);
      bits = group_mask<SHAPE>(gv, cxy, f, rsp);
      if (it == 0 && lane == 0) bits &= up ? (0xffu << (p - q)) : ((1u << (p - q)) - 1u);
      ++groups;
    }
    const int pc = __builtin_popcount(bits);
    int incl = row_incl_scan16(pc);
    const int t0 = __builtin_amdgcn_readlane(incl, 15), t1 = __builtin_amdgcn_readlane(incl, 31);
    const int t2 = __builtin_amdgcn_readlane(incl, 47), t3 = __builtin_amdgcn_readlane(incl, 63);
    incl += (g >= 1 ? t0 : 0) + (g >= 2 ? t1 : 0) + (g >= 3 ? t2 : 0);
    const int tot = t0 + t1 + t2 + t3;
    if (need < tot) {
      const int before = incl - pc;
      const bool hit = valid && before <= need && need < incl;
      const uint64_t hm = wave_ballot(hit);
      int cand = 0;
      if (hit) {
        const int n = need - before;
        cand = up ? ql + nth_bit8(bits, n) : ql + nth_bit8(bits, pc - 1 - n);
      }
      return __builtin_amdgcn_readlane(cand, __ffsll((unsigned long long)hm) - 1);
    }
    need -= tot;
    q += up ? 512 : -512;
    if (up ? q >= T : q < 0) {
      c_end = up ? k - need : k + 1 + need;
      return -1;
    }
  }
  return -1;
}

// Sum over the whole wave, in every lane (all lanes active).
__device__ __forceinline__ int wave_sum(int x) {
  x = row_sum16(x);
  return __builtin_amdgcn_readlane(x, 0) + __builtin_amdgcn_readlane(x, 16) +
         __builtin_amdgcn_readlane(x, 32) + __builtin_amdgcn_readlane(x, 48);
}

// Reverse map (paper, "Method Summary" step 7): the output is C[m], the
// value of ordinal m.  GATHER (tiles sorted in LDS): no copy of C is kept;
// the value is read back from the image at the omnigram's box location of
// m through the boundary map, which yields exactly the bits the sort saw.
// Otherwise C is read from crev (16-bit keys) or kbuf (float keys); for
// bracketed tiles the stored key is relative to the bracket's low end lo.
template <int KT, bool GATHER, typename D>
__device__ __forceinline__ void store_out(const D& a, void* out, int gx, int gy,
                                          const uint32_t* kbuf, const uint16_t* crev,
                                          const uint16_t* om, int m, uint32_t lo, int gx0,
                                          int gy0) {
  const long long o = (long long)gy * a.stride + gx;
  if constexpr (GATHER) {
    const uint32_t loc = om[m];
    const int sx = remap(gx0 + (int)(loc & 255u), a.w, a.boundary);
    const int sy = remap(gy0 + (int)(loc >> 8), a.h, a.boundary);
    const long long src = (long long)sy * a.stride + sx;
    if (KT == KEY_U8) static_cast<uint8_t*>(out)[o] = static_cast<const uint8_t*>(a.img)[src];
    if (KT == KEY_U16) static_cast<uint16_t*>(out)[o] = static_cast<const uint16_t*>(a.img)[src];
    if (KT == KEY_F32) static_cast<uint32_t*>(out)[o] = static_cast<const uint32_t*>(a.img)[src];
  } else {
    if (KT == KEY_U8) static_cast<uint8_t*>(out)[o] = (uint8_t)(crev[m] + lo);
    if (KT == KEY_U16) static_cast<uint16_t*>(out)[o] = (uint16_t)(crev[m] + lo);
    if (KT == KEY_F32) static_cast<uint32_t*>(out)[o] = key_to_f32(kbuf[m] + lo);
  }
}

// Rank of output pixel (gx, gy) in plane q of the general form: the plane's
// rank map entry clamped to [0, N) where the plane has a map and the pixel
// is inside the image, else the plane's constant rank k0.  N is the plane's
// window size (its own window under multi_fp).
template <bool GEN, typename D>
__device__ __forceinline__ int rank_at(const D& a, int q, int k0, int gx, int gy, bool inside) {
  if (!GEN) return k0;
  const int* rm = a.rmaps[q];
  if (!rm || !inside) return k0;
  const int v = rm[(long long)gy * a.rmap_strides[q] + gx];
  return min(max(v, 0), a.multi_fp ? a.pfp[q].rank_hi : a.rank_hi);
}

// Bracketed tiles: append the flagged output pixels of the wave (index
// y * w + x) to the miss list.  Call with the whole wave.
template <typename D>
__device__ __forceinline__ void push_misses(const D& a, bool missed, int gx, int gy) {
  const uint64_t mb = wave_ballot(missed);
  if (mb == 0) return;
  const int lane = threadIdx.x & 63;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(a.miss_count, (uint32_t)__popcll(mb));
  base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
  if (missed)
    a.miss[base + (uint32_t)__popcll(mb & ((1ull << lane) - 1ull))] = (uint32_t)gy * (uint32_t)a.w +
                                                                       (uint32_t)gx;
}

// Bracketed tiles: sort the Ts candidate words held in kbuf (element e =
// kbuf[e]) with ITEMS elements per thread; ordinals are written to
// omega/crev from index 0 (callers pass the arrays shifted by one).
template <int ITEMS>
__device__ __forceinline__ void br_sort(uint32_t* kbuf, int Ts, int passes, uint16_t* omega,
                                        uint16_t* crev, uint16_t* cnt, uint32_t* wsum) {
  const int t = threadIdx.x;
  uint32_t key[ITEMS];
  uint16_t pos[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int e = i * kThreads + t;
    key[i] = e < Ts ? kbuf[e] : 0u;
    pos[i] = 0;
  }
  block_radix_sort<ITEMS, false>(key, pos, Ts, 16, passes, kbuf, nullptr, omega, crev, nullptr,
                                 cnt, wsum);
}

// Branch-free binary search over n sorted values at arr[0 .. n) (LDS):
// the number of entries whose value (VAL of the entry) is below v (LE:
// at or below v).
template <bool LE, typename F>
__device__ __forceinline__ int count_below(int n, uint32_t v, F val) {
  int lo = 0;
  while (n > 0) {
    const int h = n >> 1;
    const uint32_t x = val(lo + h);
    const bool go = LE ? x <= v : x < v;
    lo = go ? lo + h + 1 : lo;
    n = go ? n - h - 1 : h;
  }
  return lo;
}

// Chained tiles (paper, "Limitations and Future Work": reuse of the
// ordinal transform where adjacent input tiles overlap).  The tile below a
// finished tile in the same column keeps the part of its box the two boxes
// share, already ranked, and ranks only its new rows:
//   1. kept entries: the previous omnigram's entries whose box row is at
//      or below th, in their order, moved up by th rows, values read back
//      from the image;
//   2. the new rows (box rows bh - th .. bh - 1) are loaded and sorted;
//   3. the two sorted lists are merged by rank: a kept entry's ordinal is
//      its index plus the number of new values below it, a new entry's its
//      index plus the number of kept values at or below it.  Among equal
//      values kept entries come first, so the kept pixels keep their
//      relative order, which keeps forwarded solutions exact.
// Lists: new entries at 0 .. nn - 1 and kept ones at nn .. T - 1 of kbuf
// (words key << 16 | location; float keys: keys in kbuf, locations in
// pbuf).  Output: the omnigram om.
template <int KT, int IMAX, typename D>
__device__ __forceinline__ void chain_rerank(const D& a, int gx0, int gy0, uint32_t* kbuf,
                                             uint16_t* pbuf, uint16_t* om, uint16_t* cnt,
                                             uint32_t* wsum) {
  constexpr bool PL = KT == KEY_F32;
  const int t = threadIdx.x;
  const int T = a.T, th = a.th, bw = a.bw;
  const int nn = th * bw;
  auto pixel = [&](int x, int y) -> uint32_t {
    const int gx = remap(gx0 + x, a.w, a.boundary), gy = remap(gy0 + y, a.h, a.boundary);
    const long long off = (long long)gy * a.stride + gx;
    if (KT == KEY_U8) return static_cast<const uint8_t*>(a.img)[off];
    if (KT == KEY_U16) return static_cast<const uint16_t*>(a.img)[off];
    return f32_to_key(static_cast<const uint32_t*>(a.img)[off]);
  };
  // 1. kept entries, in the previous omnigram's order
  {
    uint32_t loc[IMAX];
    uint32_t nk = 0;
#pragma unroll
    for (int i = 0; i < IMAX; ++i) {
      const int o = t * IMAX + i;
      const uint32_t l = o < T ? (uint32_t)om[o] : 0u;
      const bool keep = o < T && (int)(l >> 8) >= th;
      nk += keep;
      loc[i] = keep ? (l | 0x10000u) : 0u;
    }
    // (the scan's barriers also separate the reads above from the writes)
    uint32_t pos = (uint32_t)nn + block_exclusive_scan(nk, wsum);
#pragma unroll
    for (int i = 0; i < IMAX; ++i) {
      if (loc[i] & 0x10000u) {
        const int x = (int)(loc[i] & 255u), y = (int)((loc[i] >> 8) & 255u) - th;
        const uint32_t nl = (uint32_t)((y << 8) | x);
        const uint32_t v = pixel(x, y);
        if (PL) {
          kbuf[pos] = v;
          pbuf[pos] = (uint16_t)nl;
        } else {
          kbuf[pos] = (v << 16) | nl;
        }
        ++pos;
      }
    }
  }
  // 2. the new rows, loaded in row order and sorted (words to kbuf[0, nn))
  {
    uint32_t key[IMAX];
    uint16_t pos[IMAX];
    const int r0 = a.bh - th;
    int lx = t % bw, ly = t / bw;
    const int sx = kThreads % bw, sy = kThreads / bw;
#pragma unroll
    for (int i = 0; i < IMAX; ++i) {
      const int e = i * kThreads + t;
      const uint32_t p = (uint32_t)(((r0 + ly) << 8) | lx);
      const uint32_t v = e < nn ? pixel(lx, r0 + ly) : 0u;
      key[i] = e < nn ? (PL ? v : ((v << 16) | p)) : 0u;
      pos[i] = (uint16_t)p;
      lx += sx;
      ly += sy;
      if (lx >= bw) {
        lx -= bw;
        ly += 1;
      }
    }
    __syncthreads();   // kept entries written
    uint32_t* bcnt = reinterpret_cast<uint32_t*>(cnt);
    if constexpr (KT == KEY_U8) {
      bucket_pass<IMAX, false, false>(key, pos, nn, 16, 8, kbuf, pbuf, om, bcnt, wsum);
    } else {
      const int sh = PL ? 0 : 16;
      bucket_pass<IMAX, PL, false>(key, pos, nn, sh, 12, kbuf, pbuf, om, bcnt, wsum);
#pragma unroll
      for (int i = 0; i < IMAX; ++i) {
        const int e = t * IMAX + i;
        key[i] = e < nn ? kbuf[e] : 0u;
        if (PL) pos[i] = e < nn ? pbuf[e] : (uint16_t)0;
      }
      if constexpr (PL)
        block_radix_sort<IMAX, true, true, true>(key, pos, nn, 12, 5, kbuf, pbuf, pbuf, nullptr,
                                                 kbuf, cnt, wsum);
      else
        block_radix_sort<IMAX, false, false, true, true>(key, pos, nn, 28, 1, kbuf, pbuf, om,
                                                         nullptr, nullptr, cnt, wsum);
    }
  }
  // 3. merge by rank
  {
    const int nk = T - nn;
    auto val = [&](int e) -> uint32_t { return PL ? kbuf[e] : kbuf[e] >> 16; };
    uint32_t res[IMAX];
#pragma unroll
    for (int i = 0; i < IMAX; ++i) {
      const int e = t * IMAX + i;
      res[i] = 0;
      if (e < T) {
        const uint32_t v = val(e);
        const uint32_t l = PL ? (uint32_t)pbuf[e] : (kbuf[e] & 0xffffu);
        const int r = e < nn ? e + count_below<true>(nk, v, [&](int j) { return val(nn + j); })
                             : (e - nn) + count_below<false>(nn, v, [&](int j) { return val(j); });
        res[i] = ((uint32_t)r << 16) | l;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IMAX; ++i)
      if (t * IMAX + i < T) om[res[i] >> 16] = (uint16_t)(res[i] & 0xffffu);
    __syncthreads();
  }
}

// One output tile.  All threads of the workgroup must call it.
// GS = false: the sort, the omnigram and the reverse map live in LDS.
// GS = true: they live in the workgroup's global scratch slot `gslot`
// (boxes too large for LDS); the ordinal image, histograms and footprint
// tables stay in LDS.
// BR = true (LDS variant only): the tile has a value bracket [lo, hi]
// (a.brackets[tile], keys).  Only box pixels inside it are sorted; they take
// ordinals 1..Tc, pixels below take ordinal 0 and pixels above 0xffff in the
// ordinal image, so every count stays exact.  A window whose median lies
// outside the bracket has no member of rank k among ordinals 1..Tc: its
// output pixel is appended to a.miss (to be recomputed by the per-pixel
// pass) and the sweep goes on.  Returns true, with nothing written, if the
// tile has more in-bracket pixels than region A holds (the caller then runs
// the plain body on it); always false without BR.
//
// GEN (general ranks): the bands run once per output plane q < a.nq, each
// writing a.outs[q] at a.ranks[q] or at the per-pixel ranks of a.rmaps[q],
// all from the one ordinal transform of the tile (the paper's
// multi-parameter and varying-percentile filtering).
//
// CHAIN (chained tiles, LDS variant, median only): `chain` = 1 for a tile
// whose upper neighbour in the column was just processed by this
// workgroup: its box is re-ranked from the neighbour's (chain_rerank) and
// its first band starts from the forwarded last-row solutions of the
// neighbour (paper, "Method Summary" step 6: the median pixel's offset from
// its window centre carries over, so its ordinal in the new tile is the
// pivot, with exactly rank-k members below it).  The plan's footprint has
// one empty row added on top, so the box holds the window of the row above
// the tile.  Each tile leaves the box locations of its last row's medians
// in the LDS array at a.off_fwd.
template <int KT, int SHAPE, int IMAX, bool GS, bool BR = false, bool GEN = false,
          bool CHAIN = false, typename D>
__device__ __forceinline__ bool tile_body(const D& a, int tile, unsigned char* smem,
                                          unsigned char* gslot, int chain = 0) {
  static_assert(!(CHAIN && (GS || BR || GEN)), "chained tiles: LDS median tiles only");
  const bool fw = CHAIN && chain != 0;   // forwarded solutions and a kept box part
  uint16_t* fwd = CHAIN ? reinterpret_cast<uint16_t*>(smem + a.off_fwd) : nullptr;
  static_assert(!(GS && BR), "bracketed tiles use the LDS variant");
  static_assert(!(GEN && BR), "bracketed tiles compute the median only");
  const int T = a.T;
  unsigned char* abase = GS ? gslot : smem;   // region holding the sorted arrays
  uint32_t* kbuf = reinterpret_cast<uint32_t*>(abase);                // sort exchange / f32 C
  uint16_t* pbuf = reinterpret_cast<uint16_t*>(abase + a.off_p);      // f32 locations
  uint16_t* om = KT == KEY_F32 ? pbuf : reinterpret_cast<uint16_t*>(abase);   // omnigram
  uint16_t* crev = reinterpret_cast<uint16_t*>(abase + a.off_C);      // u8/u16 reverse map
  uint16_t* cnt = reinterpret_cast<uint16_t*>(smem + a.off_B);
  uint16_t* I = reinterpret_cast<uint16_t*>(smem + a.off_I);
  constexpr bool GATHER = !BR;   // no reverse map kept (store_out)
  uint32_t* hist_all = reinterpret_cast<uint32_t*>(smem + a.off_hist);
  uint32_t* wsum = reinterpret_cast<uint32_t*>(smem + a.off_tab);
  const int nr4 = (a.nrows + 3) & ~3;
  short2* rsp = reinterpret_cast<short2*>(smem + a.off_tab + 128);   // after wsum (32 words)
  int2* hrow = reinterpret_cast<int2*>(smem + a.off_tab + 128 + 4 * nr4);
  int4* vtab = reinterpret_cast<int4*>(smem + a.off_tab + 128 + 12 * nr4);

  const int t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;
  const int tx0 = (tile % a.tiles_x) * a.tw, ty0 = (tile / a.tiles_x) * a.th;
  const long long clk0 = a.counters ? (long long)clock64() : 0;
  long long clk_load = clk0;
  const int gx0 = tx0 + a.dx_min, gy0 = ty0 + a.dy_min;
  uint32_t blo = 0, bhi = 0xffffffffu;   // bracket (keys)
  if (BR) {
    const uint2 b = a.brackets[tile];
    blo = b.x;
    bhi = b.y;
  }
  int Tv = T;        // ordinals [0, Tv) are valid omnigram entries
  int mlo = 0;       // smallest ordinal a member may have

  // footprint tables: row spans, per-row horizontal offsets, per-column
  // vertical offsets (down: entering, leaving; up: entering, leaving), all
  // relative to the window centre.  Planes with windows of their own
  // (multi_fp) rebuild them per plane inside the box of the plan, whose
  // offsets (a.dx_min, a.dy_min) still place the centres.
  auto build_tables = [&](const short2* spans, int nrows, int ncols, int dx_min, int dy_min) {
    for (int i = t; i < nrows; i += kThreads) {
      const short2 s = spans[i];
      rsp[i] = s;
      const int dy = dy_min + i;
      hrow[i] = make_int2(dy * a.pitch + s.y + 1, dy * a.pitch + s.x);
    }
    for (int j = t; j < ncols; j += kThreads) {
      const short2 s = spans[nrows + j];
      const int dx = dx_min + j;
      vtab[j] = make_int4((s.y + 1) * a.pitch + dx, s.x * a.pitch + dx,
                          (s.x - 1) * a.pitch + dx, s.y * a.pitch + dx);
    }
  };
  const bool mfp = GEN && a.multi_fp;
  Fp f{a.limit, a.dy_min, a.nrows};
  int fcols = a.ncols;
  if (mfp) {
    const auto& p0 = a.pfp[0];
    f = Fp{p0.limit, p0.dy_min, p0.nrows};
    fcols = p0.ncols;
    build_tables(p0.spans, p0.nrows, p0.ncols, p0.dx_min, p0.dy_min);
  } else {
    build_tables(a.spans, a.nrows, a.ncols, a.dx_min, a.dy_min);
  }

  // Box pixels that no window of the tile reaches (the corners of the
  // rounded rectangle the windows sweep; disc windows: farther than the
  // radius from every window centre of the tile) take the largest key, so
  // they rank above every pixel a window holds and the omnigram walks
  // between medians do not cross them (no window counts them, so the
  // results are unchanged).  Not for chained tiles, whose ranked box is
  // carried into the next tile, where these rows hold window pixels, nor
  // for passes with a window per plane.
  constexpr uint32_t kTopKey = KT == KEY_U8 ? 0xffu : KT == KEY_U16 ? 0xffffu : 0xffffffffu;
  const bool cut = SHAPE == SHAPE_DISC && !CHAIN && !BR && !(GEN && a.multi_fp);
  const int ccx0 = -a.dx_min, ccx1 = -a.dx_min + a.tw - 1;   // window centres, box coordinates
  const int ccy0 = -a.dy_min, ccy1 = -a.dy_min + a.th - 1;
  auto corner_cut = [&](int lx, int ly) -> bool {
    if (!cut) return false;
    const int ox = max(0, max(ccx0 - lx, lx - ccx1)), oy = max(0, max(ccy0 - ly, ly - ccy1));
    return ox * ox + oy * oy > a.limit;
  };
  uint64_t below_bits = 0, above_bits = 0;   // BR: classes of this thread's chunks
  if constexpr (BR) {
    static_assert(KT != KEY_F32, "bracketed tiles take 8/16-bit keys");
    if (blo > bhi) return true;   // no bracket: the plain pass takes the tile
    // 1. stream the box in chunks of kThreads pixels (pixel e = chunk *
    // kThreads + t).  Pixels inside the bracket are appended to the exchange
    // buffer, keyed relative to the bracket's low end; the class of the
    // others (below / above) is kept as bit `chunk` of two masks.
    uint32_t* ncand = wsum + 24;
    if (t == 0) *ncand = 0;
    __syncthreads();
    const int cap = a.br_cap;
    const int nch = (T + kThreads - 1) / kThreads;   // <= 64
    const uint64_t lt = (1ull << lane) - 1ull;
    const int sx = kThreads % a.bw, sy = kThreads / a.bw;
    if constexpr (IMAX > 0) {
      // boxes of at most IMAX * kThreads pixels: every pixel's value in a
      // register (loads all in flight), one LDS atomic per wave
      uint32_t kv[IMAX];
      int lx = t % a.bw, ly = t / a.bw;
      const int sx = kThreads % a.bw, sy = kThreads / a.bw;
#pragma unroll
      for (int i = 0; i < IMAX; ++i) {
        const int gx = remap(gx0 + lx, a.w, a.boundary);
        const int gy = remap(gy0 + ly, a.h, a.boundary);
        const long long off = (long long)gy * a.stride + gx;
        kv[i] = KT == KEY_U8 ? (uint32_t)static_cast<const uint8_t*>(a.img)[off]
                             : (uint32_t)static_cast<const uint16_t*>(a.img)[off];
        lx += sx;
        ly += sy;
        if (lx >= a.bw) {
          lx -= a.bw;
          ly += 1;
        }
      }
      uint32_t total = 0;
#pragma unroll
      for (int i = 0; i < IMAX; ++i) {
        const bool valid = i * kThreads + t < T;
        const bool below = valid && kv[i] < blo, above = valid && kv[i] > bhi;
        below_bits |= (uint64_t)below << i;
        above_bits |= (uint64_t)above << i;
        total += (uint32_t)__popcll(__ballot(valid && !below && !above));
      }
      uint32_t base = 0;
      if (lane == 0 && total != 0) base = atomicAdd(ncand, total);
      base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
      lx = t % a.bw;
      ly = t / a.bw;
#pragma unroll
      for (int i = 0; i < IMAX; ++i) {
        const bool cand = i * kThreads + t < T && !((below_bits >> i) & 1ull) &&
                          !((above_bits >> i) & 1ull);
        const uint64_t bal = __ballot(cand);
        const uint32_t o = base + (uint32_t)__popcll(bal & lt);
        if (cand && o < (uint32_t)cap)
          kbuf[o] = ((kv[i] - blo) << 16) | (uint32_t)((ly << 8) | lx);
        base += (uint32_t)__popcll(bal);
        lx += sx;
        ly += sy;
        if (lx >= a.bw) {
          lx -= a.bw;
          ly += 1;
        }
      }
    } else {
    // 1a. box values into region B (free until the sort; it later holds the
      // ordinal image): independent coalesced loads, many in flight
      uint16_t* vals = I;
      {
        int lx = t % a.bw, ly = t / a.bw;
  #pragma unroll 8
        for (int c = 0; c < nch; ++c) {
          const int e = c * kThreads + t;
          const int gx = remap(gx0 + lx, a.w, a.boundary);
          const int gy = remap(gy0 + ly, a.h, a.boundary);
          const long long off = (long long)gy * a.stride + gx;
          const uint16_t v = KT == KEY_U8 ? (uint16_t)static_cast<const uint8_t*>(a.img)[off]
                                          : static_cast<const uint16_t*>(a.img)[off];
          if (e < T) vals[e] = v;
          lx += sx;
          ly += sy;
          if (lx >= a.bw) {
            lx -= a.bw;
            ly += 1;
          }
        }
      }
      __syncthreads();
      // 1b. classify from LDS; append in-bracket pixels to the exchange buffer
      {
        int lx = t % a.bw, ly = t / a.bw;
        constexpr int kBatch = 8;   // chunks per LDS atomic
        for (int c0 = 0; c0 < nch; c0 += kBatch) {
          uint32_t kv[kBatch], loc[kBatch];
          uint64_t bal[kBatch];
          uint32_t total = 0;
  #pragma unroll
          for (int j = 0; j < kBatch; ++j) {
            const int e = (c0 + j) * kThreads + t;
            const bool valid = c0 + j < nch && e < T;
            kv[j] = valid ? (uint32_t)vals[e] : 0u;
            loc[j] = (uint32_t)((ly << 8) | lx);
            const bool below = valid && kv[j] < blo, above = valid && kv[j] > bhi;
            if (c0 + j < 64) {
              below_bits |= (uint64_t)below << (c0 + j);
              above_bits |= (uint64_t)above << (c0 + j);
            }
            bal[j] = __ballot(valid && !below && !above);
            total += (uint32_t)__popcll(bal[j]);
            lx += sx;
            ly += sy;
            if (lx >= a.bw) {
              lx -= a.bw;
              ly += 1;
            }
          }
          uint32_t base = 0;
          if (lane == 0 && total != 0) base = atomicAdd(ncand, total);
          base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
  #pragma unroll
          for (int j = 0; j < kBatch; ++j) {
            const uint32_t o = base + (uint32_t)__popcll(bal[j] & lt);
            if (((bal[j] >> lane) & 1ull) && o < (uint32_t)cap)
              kbuf[o] = ((kv[j] - blo) << 16) | loc[j];
            base += (uint32_t)__popcll(bal[j]);
          }
        }
      }
    }
    __syncthreads();
    clk_load = a.counters ? (long long)clock64() : 0;
    const int Ts = (int)*ncand;
    if (Ts > cap) return true;   // more in-bracket pixels than region A holds
    // 2. ordinal transform of the candidates, ordinals 1..Ts; passes cover
    // the bracket's span
    const uint32_t span = bhi - blo;
    int passes = 1;
    while (passes < 4 && (span >> (4 * passes)) != 0) ++passes;
    if (Ts <= 3 * kThreads) br_sort<3>(kbuf, Ts, passes, om + 1, crev + 1, cnt, wsum);
    else if (Ts <= 9 * kThreads) br_sort<9>(kbuf, Ts, passes, om + 1, crev + 1, cnt, wsum);
    else if (Ts <= 13 * kThreads) br_sort<13>(kbuf, Ts, passes, om + 1, crev + 1, cnt, wsum);
    else br_sort<17>(kbuf, Ts, passes, om + 1, crev + 1, cnt, wsum);
    Tv = Ts + 1;
    mlo = 1;
  } else if constexpr (!GS) {
   if (fw) {
    chain_rerank<KT, IMAX>(a, gx0, gy0, kbuf, pbuf, om, cnt, wsum);
    clk_load = a.counters ? (long long)clock64() : 0;
   } else {
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
        {
          // unconditional load (remap keeps coordinates inside the image);
          // elements numbered >= T are ignored by the sort
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
          if (corner_cut(lx, ly)) kk = KT == KEY_F32 ? kTopKey : ((kTopKey << 16) | p);
        }
        key[i] = e < T ? kk : 0u;
        pos[i] = (uint16_t)q;
        lx += sx;
        ly += sy;
        if (lx >= a.bw) {
          lx -= a.bw;
          ly += 1;
        }
      }
    }
    clk_load = a.counters ? (long long)clock64() : 0;
    // 2. ordinal transform: one bucket pass over the low 8 (8-bit keys) or
    // 12 key bits, then stable 4-bit passes over the rest (one for 16-bit
    // keys, five for float keys)
    uint32_t* bcnt = reinterpret_cast<uint32_t*>(cnt);
    if constexpr (KT == KEY_U8) {
      bucket_pass<IMAX, false, true>(key, pos, T, 16, 8, kbuf, pbuf, om, bcnt, wsum);
    } else {
      constexpr bool PL = KT == KEY_F32;
      const int sh = PL ? 0 : 16;
      bucket_pass<IMAX, PL, false>(key, pos, T, sh, 12, kbuf, pbuf, om, bcnt, wsum);
#pragma unroll
      for (int i = 0; i < IMAX; ++i) {
        const int e = t * IMAX + i;
        key[i] = e < T ? kbuf[e] : 0u;
        if (PL) pos[i] = e < T ? pbuf[e] : (uint16_t)0;
      }
      block_radix_sort<IMAX, PL, false, true>(key, pos, T, sh + 12, PL ? 5 : 1, kbuf, pbuf, om,
                                              nullptr, nullptr, cnt, wsum);
    }
   }
  } else {
    // One counting pass over the low 16 bits of the key (8-bit keys: all
    // 8): box pixels are counted per key value straight from the image by
    // LDS atomics on packed 16-bit counters, the counters are scanned, and
    // each pixel is read again and claims the next slot of its key value.
    // Ties take their slots in any order, which the ordinal transform
    // allows, so 8/16-bit keys are fully sorted: each slot receives just
    // the pixel's location, the omnigram entry (the output is read back
    // from the image, so no reverse map is kept).  Float keys go to x0 as
    // (high 16 key bits << 16 | location) words for two stable 8-bit
    // passes over the high bits.
    uint32_t* x0 = reinterpret_cast<uint32_t*>(gslot);
    uint32_t* x1 = reinterpret_cast<uint32_t*>(gslot + a.off_x1);
    uint32_t* pcnt = reinterpret_cast<uint32_t*>(cnt);
    constexpr int KB = KT == KEY_U8 ? 8 : 16;
    constexpr int NW = 1 << (KB - 1);   // counter words, two counters each
    // Both passes read the box kGB elements per thread at a time (element
    // e = e0 + j * kThreads + t, coordinates stepped as in the LDS load), the
    // loads of a batch in flight together, then apply the batch's atomics.
    constexpr int kGB = 8;
    const int sx = kThreads % a.bw, sy = kThreads / a.bw;
    auto load_batch = [&](int e0, int& lx, int& ly, uint32_t (&kk)[kGB], uint32_t (&ll)[kGB]) {
#pragma unroll
      for (int j = 0; j < kGB; ++j) {
        // unconditional (remap keeps coordinates inside the image); elements
        // numbered >= T are not used
        const int gx = remap(gx0 + lx, a.w, a.boundary);
        const int gy = remap(gy0 + ly, a.h, a.boundary);
        const long long off = (long long)gy * a.stride + gx;
        ll[j] = (uint32_t)((ly << 8) | lx);
        if (KT == KEY_U8) kk[j] = static_cast<const uint8_t*>(a.img)[off];
        if (KT == KEY_U16) kk[j] = static_cast<const uint16_t*>(a.img)[off];
        if (KT == KEY_F32) kk[j] = f32_to_key(static_cast<const uint32_t*>(a.img)[off]);
        if (corner_cut(lx, ly)) kk[j] = kTopKey;
        lx += sx;
        ly += sy;
        if (lx >= a.bw) {
          lx -= a.bw;
          ly += 1;
        }
      }
      (void)e0;
    };
    for (int b = t; b < NW; b += kThreads) pcnt[b] = 0;
    __syncthreads();
    {
      int lx = t % a.bw, ly = t / a.bw;
      for (int e0 = 0; e0 < T; e0 += kGB * kThreads) {
        uint32_t kk[kGB], ll[kGB];
        load_batch(e0, lx, ly, kk, ll);
#pragma unroll
        for (int j = 0; j < kGB; ++j)
          if (e0 + j * kThreads + t < T) {
            const uint32_t d = kk[j] & ((1u << KB) - 1u);
            atomicAdd(&pcnt[d >> 1], 1u << ((d & 1u) << 4));
          }
      }
    }
    __syncthreads();
    packed_exclusive_scan(pcnt, NW, wsum);
    __syncthreads();
    {
      int lx = t % a.bw, ly = t / a.bw;
      for (int e0 = 0; e0 < T; e0 += kGB * kThreads) {
        uint32_t kk[kGB], ll[kGB], slot[kGB];
        load_batch(e0, lx, ly, kk, ll);
#pragma unroll
        for (int j = 0; j < kGB; ++j)
          if (e0 + j * kThreads + t < T) {
            const uint32_t d = kk[j] & ((1u << KB) - 1u);
            const uint32_t sh = (d & 1u) << 4;
            slot[j] = (atomicAdd(&pcnt[d >> 1], 1u << sh) >> sh) & 0xffffu;
          }
#pragma unroll
        for (int j = 0; j < kGB; ++j)
          if (e0 + j * kThreads + t < T) {
            if (KT == KEY_F32) x0[slot[j]] = (kk[j] & 0xffff0000u) | ll[j];
            else om[slot[j]] = (uint16_t)ll[j];
          }
      }
    }
    __syncthreads();
    if (KT == KEY_F32) global_radix_sort(x0, x1, T, 16, 2, om, pcnt, wsum);
  }
  if (a.counters && t == 0) atomicAdd(&a.counters[CNT_SORTED], (unsigned long long)(Tv - mlo));
  // omnigram padding: locations outside the box (box width < 256)
  if (t < 16) om[Tv + t] = 0xffff;
  if (BR && t == 16) om[0] = 0xffff;
  // 3. ordinal image (overwrites the sort's count table); a global-scratch
  // omnigram is read kGI entries per thread at a time, loads in flight
  // together
  if constexpr (GS) {
    constexpr int kGI = 8;
    for (int v0 = mlo; v0 < Tv; v0 += kGI * kThreads) {
      uint32_t loc[kGI];
#pragma unroll
      for (int j = 0; j < kGI; ++j) {
        const int v = v0 + j * kThreads + t;
        loc[j] = v < Tv ? (uint32_t)om[v] : 0u;
      }
#pragma unroll
      for (int j = 0; j < kGI; ++j) {
        const int v = v0 + j * kThreads + t;
        if (v < Tv) I[(int)(loc[j] >> 8) * a.pitch + (int)(loc[j] & 255u)] = (uint16_t)v;
      }
    }
  } else {
    for (int v = mlo + t; v < Tv; v += kThreads) {
      const uint32_t loc = (uint32_t)om[v];
      I[(int)(loc >> 8) * a.pitch + (int)(loc & 255u)] = (uint16_t)v;
    }
  }
  if (BR) {
    // pixels outside the bracket: bit c of the masks is box pixel
    // c * kThreads + t (coordinates stepped per chunk, as in the load)
    const uint64_t rest = below_bits | above_bits;
    const int nch = (T + kThreads - 1) / kThreads;
    int lx = t % a.bw, ly = t / a.bw;
    const int sx = kThreads % a.bw, sy = kThreads / a.bw;
    for (int c = 0; c < nch; ++c) {
      if ((rest >> c) & 1ull)
        I[ly * a.pitch + lx] = ((below_bits >> c) & 1ull) ? (uint16_t)0 : (uint16_t)0xffff;
      lx += sx;
      ly += sy;
      if (lx >= a.bw) {
        lx -= a.bw;
        ly += 1;
      }
    }
  }
  __syncthreads();
  const long long clk1 = a.counters ? (long long)clock64() : 0;

  // 4. bands
  // seed histogram bins: ordinals >> hshift (bracketed tiles: sized to the
  // in-bracket ordinals)
  int hshift = a.hist_shift;
  if (BR) {
    hshift = 0;
    while (((Tv - 1) >> hshift) > 255) ++hshift;
  }
  uint32_t* hist = hist_all + wid * kHistWords;
  int blocks = 0, seeds = 0, seed_taps = 0, groups = 0;
  long long seed_clk = 0, row_clk = 0, sweep_clk = 0;
  const int tw = a.tw, segs = a.segs, R = a.band_rows;
  const int seg = lane / tw, col = lane - seg * tw;
  const int band = wid * segs + seg;
  const int row0 = band * R;                 // first output row of this lane's band
  const int cxl = col - a.dx_min;            // lane's window centre, box coords
  const int cols_in = min(tw, a.w - tx0);
  const int nq = GEN ? a.nq : 1;
  for (int q = 0; q < nq; ++q) {
  if (mfp && q > 0) {
    // this plane's window: every wave is done with the previous tables
    const auto& pq = a.pfp[q];
    __syncthreads();
    f = Fp{pq.limit, pq.dy_min, pq.nrows};
    fcols = pq.ncols;
    build_tables(pq.spans, pq.nrows, pq.ncols, pq.dx_min, pq.dy_min);
    __syncthreads();
  }
  void* const outq = GEN ? a.outs[q] : a.out;
  const int k0 = GEN ? a.ranks[q] : a.rank;
  const long long clkq = GEN && a.counters ? (long long)clock64() : clk1;
  // Lane state after each row: its window's selected ordinal m, and a pivot
  // vp with the exact number vc of window members below it (vp = m, vc = the
  // pixel's rank normally).  BR: a window whose median is outside the
  // bracket is a miss (recomputed per pixel afterwards); its pivot is then
  // the bracket end it left by (ordinal 1 or Tv) with the exact count there,
  // so sliding goes on and the median is picked up again once it re-enters
  // the bracket.
  int m = 0, vp = 0, vc = k0, miss = 0;

  // 4a. first rows of the wave's bands (paper, "GPU": seeds solved from
  // histograms, then short horizontal slides from each seed).  The columns
  // of each band's first row are cut into chunks of at most 16, each
  // starting from its own seed window; the four 16-lane rows of the wave
  // take one chunk each and slide their windows right in lockstep: lane j
  // of a row counts the entering and leaving pixels of footprint rows j,
  // j + 16, ... against the row's pivot, a row-wide sum gives the count,
  // and row_select refines it.  Windows outside the image are not
  // computed: chunks of bands below the tile or the image are skipped and
  // a chunk ends at the last column inside the image.  Results reach the
  // sweep's lanes (lane = seg * tw + col) by a lane shuffle per round.
  {
    const int g = lane >> 4, j = lane & 15;
    const int nchb = (cols_in + 15) >> 4;       // chunks per band row
    const int nch = segs * nchb;
    int lp = 0, lc = 0;   // pivot and count of the last seed solved
    for (int r0 = 0; r0 < nch; r0 += 4) {
      // this row's chunk: band s, first column c0, len columns
      const int ch = r0 + g;
      const int sb = ch / nchb, c0 = (ch - sb * nchb) << 4;
      const int brow = (wid * segs + sb) * R;
      const bool ok = ch < nch && brow < a.th && ty0 + brow < a.h && !(fw && wid == 0 && sb == 0);
      const int len = ok ? min(16, cols_in - c0) : 0;
      const int cy = brow - a.dy_min;
      // ranks of the chunk's pixels, lane j holding column c0 + j
      const int krow = rank_at<GEN>(a, q, k0, tx0 + c0 + j, ty0 + brow, ok && j < len);
      int hp = 0, hc = 0;                       // the row's pivot and count
      int m_l = 0, vp_l = 0, vc_l = k0, miss_l = 0;   // results, lane j = column c0 + j
      // seeds, one wave-wide solve per chunk of the round: a band's first
      // chunk from a histogram, each later chunk by moving the previous
      // chunk's seed window 16 columns right (entering and leaving pixels
      // of every footprint row counted against its pivot, then a wave-wide
      // omnigram scan)
      for (int gg = 0; gg < 4; ++gg) {
        const int chg = r0 + gg;
        if (chg >= nch) break;
        const int sg = chg / nchb, c0g = (chg - sg * nchb) << 4;
        const int browg = (wid * segs + sg) * R;
        if (browg >= a.th || ty0 + browg >= a.h || (fw && wid == 0 && sg == 0)) continue;
        const int kseed = GEN ? __builtin_amdgcn_readlane(krow, 16 * gg) : k0;
        const int cyg = browg - a.dy_min;
        const long long cs0 = a.counters ? (long long)clock64() : 0;
        int ms, sp, sc;
        if (c0g == 0) {
          int ep = 0, ec = 0;
          ms = seed_solve<KT, SHAPE, BR, !GS>(0 - a.dx_min, cyg, Tv, hshift, kseed, a, f, om, I,
                                              hist, rsp, blocks, ep, ec);
          ++seeds;
          sp = (BR && ms < 0) ? ep : ms;
          sc = (BR && ms < 0) ? ec : kseed;
        } else {
          const int cx0 = c0g - 16 - a.dx_min;   // previous seed's centre
          const int jb = cyg * a.pitch + cx0;
          int d = 0;
          for (int e = lane; e < (f.nrows << 4); e += 64) {
            const int2 o = hrow[e >> 4];
            const int tt = e & 15;
            d += (int)(I[jb + o.x + tt] < (uint32_t)lp) - (int)(I[jb + o.y + tt] < (uint32_t)lp);
          }
          const int cnt = lc + wave_sum(d);
          int c_end = 0;
          ms = wave_select<SHAPE>(lp, cnt, kseed, (uint32_t)(cx0 + 16) | ((uint32_t)cyg << 16),
                                  Tv, f, om, rsp, groups, c_end);
          sp = (!BR || ms >= 0) ? ms : (cnt <= kseed ? Tv : 1);
          sc = (!BR || ms >= 0) ? kseed : c_end;
        }
        lp = sp;
        lc = sc;
        if (a.counters) seed_clk += (long long)clock64() - cs0;
        if (g == gg) {
          hp = sp;
          hc = sc;
        }
        if (lane == 16 * gg) {
          m_l = ms;
          vp_l = sp;
          vc_l = sc;
          miss_l = ms < 0;
        }
      }
      // horizontal slides, all rows in lockstep; the lane's first five
      // footprint rows' offsets stay in registers

      const int steps = __builtin_amdgcn_readfirstlane(
          max(max(__shfl(len, 0, 64), __shfl(len, 16, 64)),
              max(__shfl(len, 32, 64), __shfl(len, 48, 64))));
      for (int t = 1; t < steps; ++t) {
        const bool act = t < len;
        const int kc = GEN ? __shfl(krow, (int)((threadIdx.x & ~15u) | (unsigned)t), 64) : k0;
        const int cxp = c0 + t - 1 - a.dx_min;   // previous centre, box x
        const int base = cy * a.pitch + cxp;
        int d = 0;
        if (act) {
          // rows beyond the footprint read the centre twice and cancel
          for (int i = j; i < f.nrows; i += 16) {
            const int2 o = hrow[i];
            d += (int)(I[base + o.x] < (uint32_t)hp) - (int)(I[base + o.y] < (uint32_t)hp);
          }
        }
        const int cnt = hc + row_sum16(d);
        int c_end = 0;
        const int ms = row_select<SHAPE>(act, hp, cnt, kc,
                                         (uint32_t)(cxp + 1) | ((uint32_t)cy << 16), Tv, f, om,
                                         rsp, groups, c_end);
        if (act) {
          if (!BR || ms >= 0) {
            hp = ms;
            hc = kc;
          } else {
            hp = cnt <= kc ? Tv : 1;
            hc = c_end;
          }
          if (j == t) {
            m_l = ms;
            vp_l = hp;
            vc_l = hc;
            miss_l = ms < 0;
          }
        }
      }
      // hand this round's columns to the sweep lanes
      const int chu = seg * nchb + (col >> 4);
      const bool mine = lane < segs * tw && col < cols_in && chu >= r0 && chu < r0 + 4;
      const int src = mine ? (((chu - r0) << 4) | (col & 15)) : 0;
      const int mv = __shfl(m_l, src, 64), pv = __shfl(vp_l, src, 64);
      const int cv = __shfl(vc_l, src, 64), xv = __shfl(miss_l, src, 64);
      if (mine) {
        m = mv;
        vp = pv;
        vc = cv;
        miss = xv;
      }
    }
  }
  if (a.counters) seed_taps = seeds;  // taps per seed added on the host
  const long long clk2 = a.counters ? (long long)clock64() : 0;
  // forwarded first row of the tile's first band: the pivot is the new
  // ordinal of the pixel that was the median of the window one row up
  const bool fw_lanes = fw && wid == 0 && seg == 0 && lane < tw && col < cols_in;
  if (fw_lanes) {
    const uint32_t l = fwd[col];
    vp = I[((int)(l >> 8) - a.th) * a.pitch + (int)(l & 255u)];
    vc = k0;
  }
  {
    const int gx = tx0 + col, gy = ty0 + row0;
    const bool own = lane < segs * tw && col < cols_in && row0 < a.th && gy < a.h &&
                     !(fw && wid == 0 && seg == 0);
    if (own && !miss) store_out<KT, GATHER>(a, outq, gx, gy, kbuf, crev, om, m, blo, gx0, gy0);
    if (BR) push_misses(a, own && miss, gx, gy);
    if (CHAIN && own && row0 == a.th - 1) fwd[col] = om[m];
  }

  // 4b. vertical sweep down each band (lanes whose column or row is
  // outside the image sit out)
  const bool in_cols = lane < segs * tw && col < cols_in;
  const int rows_lim = min(a.h - ty0, a.th);   // tile rows inside the image
  const int rows_in = rows_lim - row0;          // rows of this lane's band inside both
  const int r_end = min(R, __builtin_amdgcn_readfirstlane(max(0, rows_lim - wid * segs * R)));
  // (the forwarded band starts one row higher, at the row above the tile)
  const int r_begin = fw && wid == 0 ? 0 : 1;
  for (int r = r_begin; r < r_end; ++r) {
    const bool lane_active = in_cols && r < rows_in && (r > 0 || fw_lanes);
    const int gx = tx0 + col, gy = ty0 + row0 + r;
    const int kl = rank_at<GEN>(a, q, k0, gx, gy, lane_active);
    const int cy_prev = row0 + r - 1 - a.dy_min;
    const int lbase = cy_prev * a.pitch + cxl;
    int delta = 0;
    if (lane_active) {
#pragma unroll 4
      for (int j = 0; j < fcols; ++j) {
        const int4 o = vtab[j];
        delta += (int)(I[lbase + o.x] < vp) - (int)(I[lbase + o.y] < vp);
      }
    }
    int pl = vp, cl = vc + delta;
    int mnew = m, esc = 0;
    const uint32_t cxy = (uint32_t)cxl | ((uint32_t)(row0 + r - a.dy_min) << 16);
    if (lane_active) {
      mnew = lane_select<SHAPE>(pl, cl, kl, cxy, kLaneBudget, Tv, f, om, rsp, groups);
      if (BR && mnew < 0 && (pl <= 0 || pl >= Tv)) {
        // walked off an end of the bracket: a miss
        esc = 1;
        if (pl <= 0) pl = 1;
      }
    }
    // lanes still walking: four at a time, each finished by one 16-lane row
    // of the wave (row_select, 128 ordinals per step)
    uint64_t left = wave_ballot(lane_active && mnew < 0 && !esc);
    while (left) {
      int Ls[4];
#pragma unroll
      for (int gi = 0; gi < 4; ++gi) {
        Ls[gi] = left ? __ffsll((unsigned long long)left) - 1 : -1;
        left &= left - 1;
      }
      const int rg = lane >> 4;
      const int Lg = rg == 0 ? Ls[0] : rg == 1 ? Ls[1] : rg == 2 ? Ls[2] : Ls[3];
      const int Lsrc = max(Lg, 0);
      const int plg = __shfl(pl, Lsrc, 64), clg = __shfl(cl, Lsrc, 64);
      const int kg = GEN ? __shfl(kl, Lsrc, 64) : k0;
      const uint32_t cxyg = (uint32_t)__shfl((int)cxy, Lsrc, 64);
      int c_end = 0;
      const int mr = row_select<SHAPE>(Lg >= 0, plg, clg, kg, cxyg, Tv, f, om, rsp, groups, c_end);
      int slot = -1;
#pragma unroll
      for (int gi = 0; gi < 4; ++gi) slot = lane == Ls[gi] ? gi : slot;
      const int src = slot >= 0 ? slot << 4 : 0;
      const int mb = __shfl(mr, src, 64), ceb = __shfl(c_end, src, 64);
      if (slot >= 0) {
        mnew = mb;
        if (BR && mb < 0) {
          pl = cl <= kl ? Tv : 1;
          cl = ceb;
          esc = 1;
        }
      }
    }
    if (lane_active) {
      if (!BR || !esc) {
        m = mnew;
        vp = mnew;
        vc = kl;
      } else {
        vp = pl;
        vc = cl;
      }
    }
    if (lane_active && !esc)
      store_out<KT, GATHER>(a, outq, gx, gy, kbuf, crev, om, m, blo, gx0, gy0);
    if (BR) push_misses(a, lane_active && esc, gx, gy);
    if (CHAIN && lane_active && row0 + r == a.th - 1) fwd[col] = om[m];
  }
  if (a.counters) {
    const long long clk3 = (long long)clock64();
    row_clk += clk2 - clkq;
    sweep_clk += clk3 - clk2;
  }
  }  // planes
  if (a.counters && lane == 0) {
    atomicAdd(&a.counters[CNT_BLOCKS], (unsigned long long)blocks);
    atomicAdd(&a.counters[CNT_SEEDS], (unsigned long long)seed_taps);
    atomicAdd(&a.counters[CNT_CYC_SORT], (unsigned long long)(clk1 - clk0));
    atomicAdd(&a.counters[CNT_CYC_ROW], (unsigned long long)row_clk);
    atomicAdd(&a.counters[CNT_CYC_SWEEP], (unsigned long long)sweep_clk);
    atomicAdd(&a.counters[CNT_WAVES], 1ull);
    atomicAdd(&a.counters[CNT_CYC_SEED], (unsigned long long)seed_clk);
    atomicAdd(&a.counters[CNT_CYC_LOAD], (unsigned long long)(clk_load - clk0));
  }
  if (a.counters) {
    // lane-parallel groups differ per lane: sum over the wave
    // (one atomic per lane: a cross-lane reduction here would keep lane
    // indices live through the whole tile, and they spill)
    if (groups) atomicAdd(&a.counters[CNT_GROUPS], (unsigned long long)groups);
  }
  return false;
}

}  // namespace mf
