// Order-independent, correctly rounded summation of doubles with integer
// atomics.  A term v is converted exactly to a fixed-point integer
// v * 2^EX_SCALE split into EX_WORDS signed 32-bit chunks; chunk sums are
// accumulated in int64 words (any order, any grouping, no overflow below
// 2^31 terms per word) and the final value is the exact sum rounded once to
// the nearest double (ties to even).  Terms must satisfy |v| < 2^40; terms
// below 2^-68 in magnitude are rounded to the fixed-point grid first.
#pragma once
#include <stdint.h>

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#endif

#define EX_INLINE inline __attribute__((always_inline))

namespace fslbm {

constexpr int EX_WORDS = 5;
constexpr int EX_SCALE = 120;  // grid 2^-120

struct ExTerm {
  long long w[EX_WORDS];
};

// Chunks of v * 2^EX_SCALE: chunk c holds bits [32c, 32c + 32).
__host__ __device__ EX_INLINE ExTerm ex_split(double v) {
  ExTerm t;
#pragma unroll
  for (int c = 0; c < EX_WORDS; ++c) t.w[c] = 0;
  if (v == 0.0 || v != v) return t;
  union {
    double d;
    uint64_t u;
  } b;
  b.d = v;
  const bool neg = (b.u >> 63) != 0;
  const int ebits = (int)((b.u >> 52) & 0x7ff);
  uint64_t m = b.u & ((1ull << 52) - 1);
  int e;  // v = m * 2^e
  if (ebits == 0) {
    e = -1074;
  } else {
    m |= 1ull << 52;
    e = ebits - 1075;
  }
  int s = e + EX_SCALE;  // fixed value = m * 2^s
  if (s < 0) {
    // below the grid: round to nearest at 2^-EX_SCALE
    if (-s > 60) return t;
    const uint64_t half = 1ull << (-s - 1);
    m = (m + half) >> (-s);
    s = 0;
  }
  const uint64_t MASK = 0xffffffffull;
#pragma unroll
  for (int c = 0; c < EX_WORDS; ++c) {
    const int lo = 32 * c - s;  // lowest bit of m in this chunk
    uint64_t chunk;
    if (lo >= 64) chunk = 0;
    else if (lo >= 0) chunk = (m >> lo) & MASK;
    else if (lo > -32) chunk = (m & (MASK >> (-lo))) << (-lo);
    else chunk = 0;
    t.w[c] = neg ? -(long long)chunk : (long long)chunk;
  }
  return t;
}

// Exact value of sum_c w[c] 2^(32c - EX_SCALE), rounded to nearest even.
__host__ __device__ EX_INLINE double ex_value(const long long *win) {
  long long w[EX_WORDS];
#pragma unroll
  for (int c = 0; c < EX_WORDS; ++c) w[c] = win[c];
  // carry-normalise: w[0..3] in [0, 2^32), w[4] signed
#pragma unroll
  for (int c = 0; c < EX_WORDS - 1; ++c) {
    const long long carry = w[c] >> 32;  // floor division by 2^32
    w[c] = w[c] & 0xffffffffll;       // the non-negative remainder
    w[c + 1] += carry;
  }
  const bool neg = w[EX_WORDS - 1] < 0;
  // magnitude in three 64-bit limbs (bits 0..191)
  uint64_t L[3] = {0, 0, 0};
  {
    // value = w4 * 2^128 + (w3 w2 w1 w0 in 32-bit digits)
    uint64_t lo = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    uint64_t mid = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
    uint64_t hi = (uint64_t)w[4];  // two's complement if negative
    if (neg) {
      // negate the 192-bit two's-complement number (hi:mid:lo)
      lo = ~lo;
      mid = ~mid;
      hi = ~hi;
      lo += 1;
      if (lo == 0) {
        mid += 1;
        if (mid == 0) hi += 1;
      }
    }
    L[0] = lo;
    L[1] = mid;
    L[2] = hi;
  }
  // highest set bit
  int top;
  if (L[2]) top = 128 + 63 - __builtin_clzll(L[2]);
  else if (L[1]) top = 64 + 63 - __builtin_clzll(L[1]);
  else if (L[0]) top = 63 - __builtin_clzll(L[0]);
  else return 0.0;
  uint64_t mant, rbit = 0;
  bool sticky = false;
  const int sh = top - 52;  // bits below the 53 significant ones
  if (sh <= 0) {
    mant = L[0] << (-sh);  // the value fits in 53 bits (top < 64)
  } else {
    // mant = bits [sh, sh + 53); round bit sh - 1; sticky = bits below
    const int q = sh >> 6, r = sh & 63;
    const uint64_t a = q == 0 ? L[0] : (q == 1 ? L[1] : L[2]);
    const uint64_t b = q == 0 ? L[1] : (q == 1 ? L[2] : 0ull);
    mant = (r == 0 ? a : ((a >> r) | (b << (64 - r)))) & ((1ull << 53) - 1);
    const int rb = sh - 1;
    const int rq = rb >> 6, rr = rb & 63;
    const uint64_t rl = rq == 0 ? L[0] : (rq == 1 ? L[1] : L[2]);
    rbit = (rl >> rr) & 1ull;
    // sticky: any bit below rb
    const uint64_t below = rr == 0 ? 0ull : (rl & ((1ull << rr) - 1ull));
    bool lower = false;
    if (rq >= 1 && L[0]) lower = true;
    if (rq >= 2 && L[1]) lower = true;
    sticky = below != 0 || lower;
  }
  if (rbit && (sticky || (mant & 1ull))) {
    mant += 1;
    if (mant == (1ull << 53)) {
      mant >>= 1;
      top += 1;
    }
  }
  // value = mant * 2^(top - 52 - EX_SCALE)
  double r = (double)mant;
  int ex = top - 52 - EX_SCALE;
  while (ex > 0) {
    const int k = ex > 60 ? 60 : ex;
    r *= (double)(1ull << k);
    ex -= k;
  }
  while (ex < 0) {
    const int k = -ex > 60 ? 60 : -ex;
    r /= (double)(1ull << k);
    ex += k;
  }
  return neg ? -r : r;
}

}  // namespace fslbm
