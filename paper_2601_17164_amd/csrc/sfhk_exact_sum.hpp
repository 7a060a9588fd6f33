// sfhk_exact_sum.hpp -- an order-independent, exact sum of binary64 values: the per-step
// accumulator of the dipole F(t_n) = sum_j f_j(t_n) (Eq. 2) and of the dipole velocity.
//
// Every finite binary64 value is an integer multiple of 2^-1074 below 2^1024, so it is a signed
// integer of at most 2098 bits in units of 2^-1074. The accumulator holds that integer as
// kExactBins signed 64-bit words, word b weighing 2^(32 b - 1074). A value's 53-bit significand
// lands in at most three consecutive words as 32-bit slices; adding the slices with 64-bit integer
// additions (atomic on the device) is exact and associative, so the total does not depend on the
// order in which values arrive, on how the work was split into tiles, launches or batches, or on
// which wave added what. Each word takes slices below 2^32 in magnitude, so up to 2^30 additions
// per word keep it below 2^62 (the propagation adds at most one value per tile and step). One
// more word collects non-finite values as flags (NaN, +inf, -inf). The final conversion propagates the carries and rounds the exact total once, to nearest
// with ties to even: the result is the correctly rounded sum of the values added.
//
// Plain C++ (no HIP types) so that the host test suite compiles it with a host compiler and checks
// it against exact rational arithmetic; SFHK_HD marks the functions for both sides.
#pragma once
#include <stdint.h>
#include <string.h>

#ifndef SFHK_HD
#if defined(__HIPCC__)
#define SFHK_HD __host__ __device__
#else
#define SFHK_HD
#endif
#endif

namespace sfhk_exact {

constexpr int kExactBins = 66;               // 66 x 32 = 2112 bits >= 2098
constexpr int kExactFlag = kExactBins;       // word of non-finite flags
constexpr int kExactWords = kExactBins + 2;  // + flags + padding: 544 bytes per accumulator
constexpr uint64_t kFlagNaN = 1, kFlagPosInf = 2, kFlagNegInf = 4;

// The slices of one value: word index of the lowest slice, the three signed slices (|s| < 2^32),
// or a flag for a non-finite value. A zero has no slices (n = 0).
struct Slices {
  int bin;
  int n;  // slices to add (0, 2 or 3)
  int64_t s[3];
  uint64_t flag;
};

SFHK_HD inline Slices slices_of(double v) {
  Slices r;
  r.bin = 0;
  r.n = 0;
  r.s[0] = r.s[1] = r.s[2] = 0;
  r.flag = 0;
  uint64_t u;
  memcpy(&u, &v, sizeof u);
  const bool neg = (u >> 63) != 0;
  const int e = (int)((u >> 52) & 0x7FF);
  uint64_t m = u & ((1ull << 52) - 1);
  if (e == 0x7FF) {
    r.flag = m ? kFlagNaN : (neg ? kFlagNegInf : kFlagPosInf);
    return r;
  }
  if (e == 0 && m == 0) return r;  // +-0
  int p;  // bit position of the significand's lowest bit, in units of 2^-1074
  if (e == 0) {
    p = 0;  // subnormal: m 2^-1074
  } else {
    m |= 1ull << 52;
    p = e - 1;  // m 2^(e - 1075) = m 2^-1074 2^(e - 1)
  }
  r.bin = p >> 5;
  const int sh = p & 31;
  // m << sh spans at most 53 + 31 = 84 bits: a low 64-bit part and a high part below 2^20
  const uint64_t lo = m << sh;
  const uint64_t hi = sh ? (m >> (64 - sh)) : 0;
  int64_t s0 = (int64_t)(lo & 0xFFFFFFFFull), s1 = (int64_t)(lo >> 32), s2 = (int64_t)hi;
  if (neg) {
    s0 = -s0;
    s1 = -s1;
    s2 = -s2;
  }
  r.s[0] = s0;
  r.s[1] = s1;
  r.s[2] = s2;
  r.n = hi ? 3 : 2;
  return r;
}

// Adds a value to an accumulator on the host (the device adds the same slices atomically).
inline void add_host(int64_t* acc, double v) {
  const Slices sl = slices_of(v);
  if (sl.flag) {
    acc[kExactFlag] |= (int64_t)sl.flag;
    return;
  }
  for (int i = 0; i < sl.n; ++i) acc[sl.bin + i] += sl.s[i];
}

// The accumulated exact total, rounded once to the nearest binary64 (ties to even); +-inf when it
// exceeds the binary64 range; NaN, or the infinity, when non-finite values were added.
SFHK_HD inline double round_total(const int64_t* acc) {
  const uint64_t fl = (uint64_t)acc[kExactFlag];
  const double kInf = __builtin_huge_val();
  if ((fl & kFlagNaN) || ((fl & kFlagPosInf) && (fl & kFlagNegInf))) return __builtin_nan("");
  if (fl & kFlagPosInf) return kInf;
  if (fl & kFlagNegInf) return -kInf;
  // carries: digits d_b in [0, 2^32) and a signed top carry
  uint32_t d[kExactBins];
  int64_t carry = 0;
  for (int b = 0; b < kExactBins; ++b) {
    const int64_t t = acc[b] + carry;  // |acc| < 2^62, |carry| < 2^31: no overflow
    d[b] = (uint32_t)((uint64_t)t & 0xFFFFFFFFull);
    carry = t >> 32;  // arithmetic shift: floor division by 2^32
  }
  bool neg = false;
  if (carry < 0) {  // negative total: two's complement of the digit string
    neg = true;
    uint64_t c = 1;
    for (int b = 0; b < kExactBins; ++b) {
      const uint64_t t = (uint64_t)(uint32_t)~d[b] + c;
      d[b] = (uint32_t)t;
      c = t >> 32;
    }
    carry = -carry - 1 + (int64_t)c;  // magnitude beyond the digits (0 unless out of range)
  }
  if (carry != 0) return neg ? -kInf : kInf;
  int top = kExactBins - 1;
  while (top >= 0 && d[top] == 0) --top;
  if (top < 0) return 0.0;
  // most significant bit position P (units of 2^-1074)
  const int lz = __builtin_clz(d[top]);
  const int P = 32 * top + 31 - lz;
  if (P < 53) {  // below 2^-1021: exact as a subnormal or small normal (multiple of 2^-1074)
    uint64_t v = d[0] | (top >= 1 ? ((uint64_t)d[1] << 32) : 0);
    double r = (double)v;  // v < 2^53: exact
    r = r * 0x1p-1074;     // exact: the result is a multiple of 2^-1074 below 2^-1021
    return neg ? -r : r;
  }
  // the 64 bits from P down (bit 63 of w is bit P), and a sticky bit for everything lower: the
  // 96-bit window of the top three digits, shifted left by the top digit's leading zeros
  const uint64_t d2 = d[top], d1 = top >= 1 ? d[top - 1] : 0, d0 = top >= 2 ? d[top - 2] : 0;
  const uint64_t hi = (d2 << 32) | d1;
  const uint64_t w = lz ? ((hi << lz) | (d0 >> (32 - lz))) : hi;
  bool sticky = lz ? (d0 & ((1ull << (32 - lz)) - 1)) != 0 : d0 != 0;
  for (int b = top - 3; b >= 0 && !sticky; --b) sticky = d[b] != 0;
  // keep 53 bits: w >> 11, with the 11 lower bits and the sticky bit deciding the rounding
  uint64_t mant = w >> 11;
  const uint64_t rest = w & 0x7FFull;
  const uint64_t half = 0x400ull;
  if (rest > half || (rest == half && (sticky || (mant & 1)))) ++mant;
  int expo = P - 52;  // value = mant 2^(expo - 1074)
  if (mant == (1ull << 53)) {
    mant >>= 1;
    ++expo;
  }
  if (expo - 1074 + 52 > 1023) return neg ? -kInf : kInf;
  // mant 2^(expo - 1074) with mant < 2^53 and expo >= 1: build the binary64 directly
  const uint64_t bexp = (uint64_t)(expo + 52 - 1074 + 1023);
  const uint64_t bits = ((uint64_t)neg << 63) | (bexp << 52) | (mant & ((1ull << 52) - 1));
  double r;
  memcpy(&r, &bits, sizeof r);
  return r;
}

}  // namespace sfhk_exact
