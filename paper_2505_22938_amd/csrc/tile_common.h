// Device-side building blocks shared by the plain, batched and learned
// kernels: boundary remap, key transform, tile load and the per-tile LDS
// radix sort that produces the reverse map C and the omnigram.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_internal.h"

namespace mf {

// Workgroups are dealt to the 8 XCDs round-robin by id.  Give XCD x a
// contiguous run of tiles instead, so neighbouring tiles, which read the same
// halo rows and columns, are processed under one L2.  Bijective on [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, j = b / kXcd, q = n / kXcd, rem = n % kXcd;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + j;
}

// Persistent grids claim their tiles at run time, so a workgroup whose
// tiles were cheap goes on to take more.  The tiles are cut into kXcd
// contiguous runs as xcd_tile cuts them; workgroup b takes tiles from run
// b % kXcd (the XCD it runs on) until that run is used up, then from the
// following runs.  claim[x] counts the claims made on run x (claims past
// its end included) and claim[kXcd] the workgroups done; the last
// workgroup to finish clears them, so every launch starts from zeros.
// `run` starts at 0 and is the workgroup's position in its order of runs;
// `sh` is one LDS word.  Returns the next tile, or -1 when every run is
// used up.  Contains barriers: call from all threads.
__device__ __forceinline__ int claim_tile(unsigned int* claim, int ntiles, int& run, int* sh) {
  constexpr int kXcd = 8;
  const int q = ntiles / kXcd, rem = ntiles % kXcd;
  while (run < kXcd) {
    const int x = ((int)blockIdx.x + run) % kXcd;
    if (threadIdx.x == 0) *sh = (int)atomicAdd(&claim[x], 1u);
    __syncthreads();
    const int j = *sh;
    __syncthreads();
    if (j < q + (x < rem ? 1 : 0)) return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + j;
    ++run;
  }
  return -1;
}
__device__ __forceinline__ void claim_done(unsigned int* claim) {
  constexpr int kXcd = 8;
  if (threadIdx.x == 0 && atomicAdd(&claim[kXcd], 1u) == gridDim.x - 1) {
#pragma unroll
    for (int i = 0; i <= kXcd; ++i) atomicExch(&claim[i], 0u);
  }
}

// Boundary rule: clamp repeats the edge pixel; mirror reflects about it
// without repeating it and folds with period 2(n-1).
__device__ __forceinline__ int remap(int x, int n, int boundary) {
  if ((unsigned)x < (unsigned)n) return x;
  if (boundary == 0) return x < 0 ? 0 : n - 1;
  if (n == 1) return 0;
  const int period = 2 * (n - 1);
  int m = x % period;
  if (m < 0) m += period;
  return m >= n ? period - m : m;
}

// float32 bits -> unsigned key whose unsigned order is IEEE totalOrder
// (paper, "Implementation": XOR exponent and mantissa by the sign bit and
// flip the sign bit).  key_to_f32 inverts it.
__device__ __forceinline__ uint32_t f32_to_key(uint32_t b) {
  return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}
__device__ __forceinline__ uint32_t key_to_f32(uint32_t k) {
  return k ^ (((k >> 31) - 1u) | 0x80000000u);
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan over the whole workgroup of one value per thread.
// `wsum` is kWaves words of LDS.  Contains barriers: call from all threads.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t incl = wave_inclusive_scan(v, lane);
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  uint32_t pre = 0;
  for (int j = 0; j < wid; ++j) pre += wsum[j];
  __syncthreads();
  return pre + incl - v;
}

// Per-tile key-value sort (paper, "Implementation", Eq. 4: the ordinal
// transform is a key-value sort of {value, location}).  LSD radix sort with
// 4-bit digits.  Each thread keeps `items` elements in registers; the
// per-thread digit counts give a stable rank (thread-blocked order), a flat
// scan over the digit-major count table gives each (digit, thread) its
// output offset, and the elements are scattered into LDS.  Between passes
// each thread reloads a contiguous run of `items` elements (items is odd,
// so the strided reload hits distinct LDS banks).
//
// Elements: `key[i]` holds the sort key in bits [shift0, shift0 + 4*passes);
// for float keys `pos[i]` is a 16-bit payload sorted alongside.  On entry
// element i of thread t is element number i*kThreads + t (any order is fine
// for the first pass), or t*ITEMS + i with BLOCKED0 (the first pass then
// keeps that order among equal digits); elements numbered >= T are absent.  ITEMS is odd and
// ITEMS * kThreads >= T.
//
// Output: with PAYLOAD (float keys) the last pass writes the sorted keys to
// kout[dst] and the payload to omega[dst].  Without PAYLOAD the element is
// one word key << 16 | loc; the last pass splits it into loc -> omega[dst]
// and key -> crev[dst].  KEEP_C = false writes only omega (the caller reads
// values back from the image through the omnigram's locations).  WORDS_OUT
// (without PAYLOAD): the last pass writes the whole words to kbuf as the
// earlier passes do.  kbuf/pbuf are the exchange buffers of earlier
// passes; the output arrays may alias them (the last pass reads only
// registers).
template <int ITEMS, bool PAYLOAD, bool KEEP_C = true, bool BLOCKED0 = false,
          bool WORDS_OUT = false>
__device__ __forceinline__ void block_radix_sort(uint32_t (&key)[ITEMS], uint16_t (&pos)[ITEMS],
                                                 int T, int shift0, int passes,
                                                 uint32_t* kbuf, uint16_t* pbuf,
                                                 uint16_t* omega, uint16_t* crev, uint32_t* kout,
                                                 uint16_t* cnt, uint32_t* wsum) {
  const int t = threadIdx.x;
  for (int pass = 0; pass < passes; ++pass) {
    const int sh = shift0 + 4 * pass;
    // 1. thread-local digit counts and local ranks
    uint64_t c_lo = 0, c_hi = 0;
    uint32_t lr[(ITEMS + 3) / 4];
#pragma unroll
    for (int j = 0; j < (ITEMS + 3) / 4; ++j) lr[j] = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int e = pass == 0 && !BLOCKED0 ? i * kThreads + t : t * ITEMS + i;
      if (e < T) {
        const uint32_t d = (key[i] >> sh) & 15u;
        const uint32_t s8 = (d & 7u) << 3;
        const uint64_t sel = d < 8 ? c_lo : c_hi;
        lr[i >> 2] |= ((uint32_t)(sel >> s8) & 0xffu) << ((i & 3) * 8);
        const uint64_t inc = 1ull << s8;
        if (d < 8) c_lo += inc; else c_hi += inc;
      }
    }
    // 2. counts to the digit-major table
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      cnt[d * kThreads + t] = (uint16_t)((c_lo >> (8 * d)) & 0xff);
      cnt[(d + 8) * kThreads + t] = (uint16_t)((c_hi >> (8 * d)) & 0xff);
    }
    __syncthreads();
    // 3. flat exclusive scan: thread t owns table entries [16t, 16t+16)
    {
      uint4* row = reinterpret_cast<uint4*>(cnt + 16 * t);
      uint4 a = row[0], b = row[1];
      uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
      uint32_t run = 0, ex[16];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t lo = w[j] & 0xffffu, hi = w[j] >> 16;
        ex[2 * j] = run;
        run += lo;
        ex[2 * j + 1] = run;
        run += hi;
      }
      const uint32_t base = block_exclusive_scan(run, wsum);
#pragma unroll
      for (int j = 0; j < 8; ++j) w[j] = ((ex[2 * j] + base) & 0xffffu) | ((ex[2 * j + 1] + base) << 16);
      row[0] = make_uint4(w[0], w[1], w[2], w[3]);
      row[1] = make_uint4(w[4], w[5], w[6], w[7]);
    }
    __syncthreads();
    // 4. scatter
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int e = pass == 0 && !BLOCKED0 ? i * kThreads + t : t * ITEMS + i;
      if (e < T) {
        const uint32_t d = (key[i] >> sh) & 15u;
        const uint32_t dst = (uint32_t)cnt[d * kThreads + t] + ((lr[i >> 2] >> ((i & 3) * 8)) & 0xffu);
        if (PAYLOAD) {
          if (pass + 1 < passes) {
            kbuf[dst] = key[i];
            pbuf[dst] = pos[i];
          } else {
            if (KEEP_C) kout[dst] = key[i];
            omega[dst] = pos[i];
          }
        } else if (pass + 1 < passes || WORDS_OUT) {
          kbuf[dst] = key[i];
        } else {
          omega[dst] = (uint16_t)key[i];
          if (KEEP_C) crev[dst] = (uint16_t)(key[i] >> 16);
        }
      }
    }
    __syncthreads();
    // 5. reload a contiguous run for the next pass
    if (pass + 1 < passes) {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int e = t * ITEMS + i;
        uint32_t k = 0;
        uint16_t q = 0;
        if (e < T) {
          k = kbuf[e];
          if (PAYLOAD) q = pbuf[e];
        }
        key[i] = k;
        if (PAYLOAD) pos[i] = q;
      }
    }
  }
}

// Counting pass on the low `bits` key bits (at bit `sh`) that does not keep
// the order of equal digits: bucket sizes by LDS atomics, an exclusive scan
// over the buckets, then each element claims the next slot of its bucket by
// a returning atomic on the bucket's running offset.  Ties between equal
// keys may be broken in any order (they get consecutive ordinals whose
// reverse-map value is the same), so this may serve as the least
// significant pass of the LSD sort; the stable passes of block_radix_sort
// (BLOCKED0) then order the higher bits.  Elements: as block_radix_sort's
// first pass (striped).  FINAL (8-bit keys, whose low 8 bits are the whole
// key): the location (low 16 bits of the word) goes straight to omega[slot];
// otherwise the word goes to kbuf[slot] (and the payload to pbuf[slot]).
// cnt holds 1 << bits words (bits <= 12); wsum as block_exclusive_scan.
template <int ITEMS, bool PAYLOAD, bool FINAL>
__device__ __forceinline__ void bucket_pass(const uint32_t (&key)[ITEMS],
                                            const uint16_t (&pos)[ITEMS], int T, int sh,
                                            int bits, uint32_t* kbuf, uint16_t* pbuf,
                                            uint16_t* omega, uint32_t* cnt, uint32_t* wsum) {
  const int t = threadIdx.x;
  const uint32_t mask = (1u << bits) - 1u;
  const int nb = 1 << bits;
  for (int b = t; b < nb; b += kThreads) cnt[b] = 0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i)
    if (i * kThreads + t < T) atomicAdd(&cnt[(key[i] >> sh) & mask], 1u);
  __syncthreads();
  // exclusive scan: thread t owns buckets [4t, 4t + 4)
  {
    uint32_t c[4] = {0, 0, 0, 0};
    const bool own = 4 * t < nb;
    if (own) {
      const uint4 v = reinterpret_cast<const uint4*>(cnt)[t];
      c[0] = v.x;
      c[1] = v.y;
      c[2] = v.z;
      c[3] = v.w;
    }
    const uint32_t sum = c[0] + c[1] + c[2] + c[3];
    const uint32_t base = block_exclusive_scan(sum, wsum);
    if (own)
      reinterpret_cast<uint4*>(cnt)[t] =
          make_uint4(base, base + c[0], base + c[0] + c[1], base + c[0] + c[1] + c[2]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (i * kThreads + t < T) {
      const uint32_t dst = atomicAdd(&cnt[(key[i] >> sh) & mask], 1u);
      if (FINAL) {
        omega[dst] = (uint16_t)key[i];
      } else {
        kbuf[dst] = key[i];
        if (PAYLOAD) pbuf[dst] = pos[i];
      }
    }
  }
  __syncthreads();
}

// Stable LSD radix sort of T elements in global memory, for boxes whose
// sort exchange does not fit in LDS.  Elements are 32-bit words (key bits
// << 16 | location); the passes sort bits [shift0, shift0 + 8*passes), 8 at
// a time.  Pass p reads xa (p even) or xb (p odd) and writes the other; the
// last pass writes neither but only each word's location, to omega[], which
// may alias the buffer that pass does not read.
//
// Wave v owns the contiguous elements [v*S, (v+1)*S) and walks them 64 at a
// time in order (coalesced loads).  A pass counts digits per (digit, wave),
// scans the counters digit-major, then walks again: an element's slot is its
// (digit, wave) counter plus its rank among the lanes of its step holding
// the same digit (eight ballots), and the highest such lane advances the
// counter, so equal digits keep their order.  Counters: cw[wave * 257 +
// digit] (the odd row pitch spreads a wave's digits and a scan thread's
// waves over the banks), 16 * 257 LDS words.
__device__ __forceinline__ uint64_t digit_peers8(uint32_t d, bool valid) {
  uint64_t p = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t m = __ballot((d >> b) & 1u);
    p &= ((d >> b) & 1u) ? m : ~m;
  }
  return p;
}

__device__ __forceinline__ void global_radix_sort(uint32_t* xa, uint32_t* xb, int T, int shift0,
                                                  int passes, uint16_t* omega, uint32_t* cw,
                                                  uint32_t* wsum) {
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  constexpr int kPitch = 257;
  const int S = (((T + kWaves - 1) / kWaves) + 63) & ~63;
  const int e0 = wid * S, e1 = min(e0 + S, T);
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t* mine = cw + wid * kPitch;
  for (int pass = 0; pass < passes; ++pass) {
    const uint32_t* src = (pass & 1) ? xb : xa;
    uint32_t* dst = (pass & 1) ? xa : xb;
    const int sh = shift0 + 8 * pass;
    const bool last = pass + 1 == passes;
    for (int i = t; i < kWaves * kPitch; i += kThreads) cw[i] = 0;
    __syncthreads();
    for (int e = e0 + lane; e < e1; e += 64) atomicAdd(&mine[(src[e] >> sh) & 255u], 1u);
    __syncthreads();
    {
      // thread t scans entries 4t .. 4t + 3 of the digit-major order
      // (digit t / 4, waves 4 (t % 4) .. 4 (t % 4) + 3)
      const int d = t >> 2, w0 = (t & 3) * 4;
      uint32_t c[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) c[j] = cw[(w0 + j) * kPitch + d];
      uint32_t b = block_exclusive_scan(c[0] + c[1] + c[2] + c[3], wsum);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cw[(w0 + j) * kPitch + d] = b;
        b += c[j];
      }
    }
    __syncthreads();
    for (int c0 = e0; c0 < e1; c0 += 64) {
      const int e = c0 + lane;
      const bool valid = e < e1;
      const uint32_t v = valid ? src[e] : 0u;
      const uint32_t d = (v >> sh) & 255u;
      const uint64_t peers = digit_peers8(d, valid);
      const uint32_t base = valid ? mine[d] : 0u;
      if (valid) {
        const uint32_t o = base + (uint32_t)__popcll(peers & lt);
        if (!last) dst[o] = v;
        else omega[o] = (uint16_t)v;
        if ((peers & ~lt) == (1ull << lane)) mine[d] = base + (uint32_t)__popcll(peers);
      }
    }
    __syncthreads();
  }
}

// Exclusive scan, in place, over the 2 * nw 16-bit counters packed two per
// word in w (counter 2i in the low half of word i); the totals stay below
// 65536.  Wave v owns the contiguous run of words [v * per, (v + 1) * per)
// and walks it 64 words at a time, lane l on word l of each step, so every
// LDS access of a step falls in its own bank (a run per thread would put
// all lanes of a wave on two banks).  Contains barriers.
__device__ __forceinline__ void packed_exclusive_scan(uint32_t* w, int nw, uint32_t* wsum) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int per = (nw + kWaves - 1) / kWaves;
  const int w0 = wid * per, w1 = min(w0 + per, nw);
  uint32_t sum = 0;
  for (int i = w0 + lane; i < w1; i += 64) {
    const uint32_t v = w[i];
    sum += (v & 0xffffu) + (v >> 16);
  }
  // the runs before this wave's: the exclusive prefix of one value per wave
  const uint32_t tot = __shfl(wave_inclusive_scan(sum, lane), 63, 64);
  uint32_t run = block_exclusive_scan(lane == 63 ? tot : 0u, wsum);
  for (int i0 = w0; i0 < w1; i0 += 64) {
    const int i = i0 + lane;
    const uint32_t v = i < w1 ? w[i] : 0u;
    const uint32_t lo = v & 0xffffu, s = lo + (v >> 16);
    const uint32_t incl = wave_inclusive_scan(s, lane);
    const uint32_t b = run + incl - s;
    if (i < w1) w[i] = b | ((b + lo) << 16);
    run += __shfl(incl, 63, 64);
  }
}

}  // namespace mf
