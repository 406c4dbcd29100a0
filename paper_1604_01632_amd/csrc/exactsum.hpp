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

namespace fslbm {

constexpr int EX_WORDS = 5;
constexpr int EX_SCALE = 120;  // grid 2^-120

struct ExTerm {
  long long w[EX_WORDS];
};

// Chunks of v * 2^EX_SCALE: chunk c holds bits [32c, 32c + 32).
__host__ __device__ inline ExTerm ex_split(double v) {
  ExTerm t;
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
__host__ __device__ inline double ex_value(const long long *win) {
  long long w[EX_WORDS];
  for (int c = 0; c < EX_WORDS; ++c) w[c] = win[c];
  // carry-normalise: w[0..3] in [0, 2^32), w[4] signed
  for (int c = 0; c < EX_WORDS - 1; ++c) {
    const long long carry = w[c] >> 32;  // floor division by 2^32
    w[c] = w[c] & 0xffffffffll;       // the non-negative remainder
    w[c + 1] += carry;
  }
  const bool neg = w[EX_WORDS - 1] < 0;
  // magnitude in three 64-bit limbs (bits 0..191)
  uint64_t L[3];
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
  int top = -1;
  for (int k = 2; k >= 0 && top < 0; --k)
    if (L[k]) top = 64 * k + 63 - __builtin_clzll(L[k]);
  if (top < 0) return 0.0;
  auto bit = [&](int j) -> uint64_t { return j < 0 ? 0ull : (L[j >> 6] >> (j & 63)) & 1ull; };
  // 53 significant bits [top-52, top], round bit top-53, sticky below
  uint64_t mant = 0;
  for (int j = top; j >= top - 52; --j) mant = (mant << 1) | bit(j);
  const uint64_t rbit = bit(top - 53);
  bool sticky = false;
  for (int j = top - 54; j >= 0 && !sticky; --j)
    if (bit(j)) sticky = true;
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
  // scale by a power of two without rounding (|ex| is small)
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
