// Division of 32-bit indices by a divisor fixed at launch time, as a multiply
// and a shift (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, the round-up method): with s = ceil(log2 d) and
// m = floor(2^32 (2^s - d) / d) + 1,
//
//   floor(n / d) = (floor(m n / 2^32) + n) >> s      for 0 <= n < 2^31,
//
// where the sum stays below 2^32 because floor(m n / 2^32) < n.  Index
// arithmetic on the device uses this in place of the integer division
// sequence, which costs tens of instructions per quotient.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define JGB_HD __host__ __device__
#else
#define JGB_HD
#endif

namespace jgb {

struct FastDiv {
  uint32_t d = 1, m = 1, s = 0;

  FastDiv() = default;
  // d >= 1, d < 2^31
  explicit FastDiv(uint32_t d_) : d(d_), m(1), s(0) {
    while ((1u << s) < d) ++s;
    m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << s) - d)) / d + 1);
  }
  // n < 2^31
  JGB_HD uint32_t div(uint32_t n) const {
    const uint32_t hi = (uint32_t)(((uint64_t)m * n) >> 32);
    return (hi + n) >> s;
  }
  JGB_HD uint32_t mod(uint32_t n) const { return n - div(n) * d; }
};

}  // namespace jgb
