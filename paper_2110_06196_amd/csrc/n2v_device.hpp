// Device-side building blocks shared by the walk and prep kernels (gfx950,
// wave64).  Everything here is exact integer arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace n2v {

constexpr uint32_t kC16 = 65536u;  // alpha = 1 (common neighbour) in Q16

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xor bijection with the key advanced by the Weyl constants between
// rounds.  Key = (seed lo, seed hi), counter = (step, wid lo, wid hi, 0); the
// 64-bit draw is word0 | word1 << 32.
__device__ __forceinline__ void philox_words(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t out[4]) {
  uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    uint32_t lo0 = m0 * x0, hi0 = __umulhi(m0, x0);
    uint32_t lo1 = m1 * x2, hi1 = __umulhi(m1, x2);
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

__device__ __forceinline__ uint64_t philox_draw(uint64_t seed, uint32_t step, uint64_t wid) {
  uint32_t x0 = step, x1 = (uint32_t)wid, x2 = (uint32_t)(wid >> 32), x3 = 0u;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    uint32_t lo0 = m0 * x0, hi0 = __umulhi(m0, x0);
    uint32_t lo1 = m1 * x2, hi1 = __umulhi(m1, x2);
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return (uint64_t)x0 | ((uint64_t)x1 << 32);
}

// floor(r * total / 2^64): uniform in [0, total) (step 3 of the sampler).
__device__ __forceinline__ uint64_t scale_draw(uint64_t r, uint64_t total) {
  return __umul64hi(r, total);
}

// ---------------------------------------------------------------------------
// Whole-wavefront collectives on DPP (data-parallel primitives) and readlane,
// which stay in the vector ALU instead of the LDS permute pipe.  All 64 lanes
// must be active.
// ---------------------------------------------------------------------------
// Inclusive 64-lane scan of 32-bit values: row_shr 1, 2, 4, 8 scan each row of
// 16 lanes; row_bcast 15 and 31 then carry row totals into the later rows.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Exact 64-bit scan: three limbs of at most 22 bits, so every 64-lane partial
// sum of a limb fits in 32 bits; recombined modulo 2^64.
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x) {
  const uint32_t a = wave_incl_scan_u32((uint32_t)(x & 0x3FFFFFull));
  const uint32_t b = wave_incl_scan_u32((uint32_t)((x >> 22) & 0x3FFFFFull));
  const uint32_t c = wave_incl_scan_u32((uint32_t)(x >> 44));
  return (uint64_t)a + ((uint64_t)b << 22) + ((uint64_t)c << 44);
}

__device__ __forceinline__ uint64_t wave_read_u64(uint64_t x, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// ---------------------------------------------------------------------------
// Sub-wave groups of G lanes (G divides 64).  Control flow is uniform inside
// a group, so the cross-lane reads below only touch active lanes.  A group of
// 64 is the whole wavefront and uses the DPP / readlane forms.
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ uint64_t grp_sum(uint64_t x) {
  if constexpr (G == 64) {
    return wave_read_u64(wave_incl_scan_u64(x), 63);
  } else {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, G);
    return x;
  }
}

template <int G>
__device__ __forceinline__ uint64_t grp_incl_scan(uint64_t x, int gl) {
  if constexpr (G == 64) {
    (void)gl;
    return wave_incl_scan_u64(x);
  } else {
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      uint64_t y = __shfl_up(x, (unsigned)o, G);
      if (gl >= o) x += y;
    }
    return x;
  }
}

// src is the same for every lane of the group.
template <int G>
__device__ __forceinline__ uint64_t grp_bcast(uint64_t x, int src) {
  if constexpr (G == 64) return wave_read_u64(x, src);
  else return __shfl(x, src, G);
}

template <int G>
__device__ __forceinline__ int32_t grp_bcast_i32(int32_t x, int src) {
  if constexpr (G == 64) return __builtin_amdgcn_readlane(x, src);
  else return __shfl(x, src, G);
}

// Mask of the lanes of this group (bit i = group lane i) whose pred is true.
template <int G>
__device__ __forceinline__ uint64_t grp_ballot(bool pred, int gbase) {
  uint64_t m = __ballot(pred);
  if (G == 64) return m;
  return (m >> gbase) & ((1ull << G) - 1ull);
}

// Walk position e = e0 + d of a [rows][L] array split into (row, column),
// given e0 = row0 * L + i0.
__device__ __forceinline__ void split_pos(uint64_t row0, uint32_t i0, uint64_t d, uint32_t L, uint64_t* row,
                                          uint32_t* i) {
  const uint64_t s = (uint64_t)i0 + d;
  if (s < L) {
    *row = row0;
    *i = (uint32_t)s;
  } else {
    const uint64_t k = s / L;
    *row = row0 + k;
    *i = (uint32_t)(s - k * L);
  }
}

// First index j in [0, d) with R[j] > T (R non-decreasing); d if none.
template <typename RT>
__device__ __forceinline__ uint32_t upper_bound_gt(const RT* R, uint32_t d, uint64_t T) {
  uint32_t lo = 0, hi = d;
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    if ((uint64_t)R[mid] > T) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// First j in [0, d) with f(j) > T, for f non-decreasing with f(d - 1) = S > T
// (a row prefix, or one scaled and shifted at a single position), found with
// fewer dependent loads when f grows roughly linearly, as row prefixes of
// weights do: up to three rounds probe a window of 33 entries around the point
// where the line through the bracket's end values crosses T (both ends of the
// window in flight together), then a bisection finishes inside the bracket.
// Invariant: the answer lies in [lo, hi], f(lo - 1) <= T (flo; 0 before the
// row), f(hi) > T (fhi).
template <typename F>
__device__ __forceinline__ uint32_t first_above_interp(uint32_t d, uint64_t T, uint64_t S, F f) {
  uint32_t lo = 0, hi = d - 1;
  uint64_t flo = 0, fhi = S;
  for (int round = 0; round < 3 && hi - lo > 32; ++round) {
    const double frac = (double)(T - flo) / (double)(fhi - flo);
    uint32_t g = lo + (uint32_t)(frac * (double)(hi - lo));
    if (g > hi - 1) g = hi - 1;
    const uint32_t a = g > lo + 16 ? g - 16 : lo;
    const uint32_t b = g + 16 < hi - 1 ? g + 16 : hi - 1;
    const uint64_t fa = f(a), fb = f(b);
    if (fa > T) {
      hi = a;
      fhi = fa;
    } else if (fb > T) {
      lo = a + 1;
      flo = fa;
      hi = b;
      fhi = fb;
    } else {
      lo = b + 1;
      flo = fb;
    }
  }
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (f(mid) > T) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

template <typename RT>
__device__ __forceinline__ uint32_t upper_bound_interp(const RT* R, uint32_t d, uint64_t T, uint64_t S) {
  return first_above_interp(d, T, S, [&](uint32_t j) -> uint64_t { return (uint64_t)R[j]; });
}

// First index j in [0, d) with D[j] >= x; d if none.
__device__ __forceinline__ uint32_t lower_bound_i32(const int32_t* D, uint32_t d, int32_t x) {
  uint32_t lo = 0, hi = d;
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    if (D[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Floor search in a strictly increasing array: the largest index b in
// [base, base + len) with A[b] <= x, given vb = A[base] <= x (or base = 0 and
// vb = A[0] > x, when the answer stays base with a value other than x), and
// that value.  A membership test compares the value, so the found entry is
// never read a second time.  Needs len >= 1.
__device__ __forceinline__ uint32_t floor_search(const int32_t* A, uint32_t base, uint32_t len, int32_t vb,
                                                 int32_t x, int32_t& val) {
  while (len > 1) {
    const uint32_t half = len >> 1;
    const int32_t v = A[base + half];
    if (v <= x) {
      base += half;
      vb = v;
    }
    len -= half;
  }
  val = vb;
  return base;
}

}  // namespace n2v
