// Natural logarithm of x in [2^-53, 1] for the FP64 flight time -ln(1 - u)/nu'
// (eq. random_time), table-driven after P. T. P. Tang, "Table-driven implementation of the
// logarithm function in IEEE floating-point arithmetic", ACM TOMS 16 (1990):
//   x = 2^e m with m in [1, 2), and c = 1 + i/64 from the top six fraction bits of m;
//   with r = m RN(1/c) - 1 (one FMA, 0 <= r <= 2^-6),
//   ln x = e ln2 - ln RN(1/c) + log1p(r)   (exact in real arithmetic),
// the table holding RN(1/c) and -ln RN(1/c) as a sum of two doubles (hi + lo) for the 64
// values of i.  The lo part matters where e ln2 and -ln RN(1/c) nearly cancel (x just below
// 1 - 2^-7): their sum is then exact, and the table's own rounding would otherwise show.
// log1p(r) is its Taylor series to r^9 (truncation below 2^-57 relative).  Inputs within
// 2^-7 of 1 take r = x - 1 (exact) with e = 0 and no table term, so short flights keep full
// relative accuracy.  The table is built on the host in extended precision; the evaluation
// uses only IEEE-exact operations (FMA, frexp, products by powers of two), so host and
// device compute the same bits.
#pragma once

#include <cmath>
#include <cstdint>
#include <cstring>

namespace swarm_impl {

constexpr int kUnitLogEntries = 64;          // table entries
constexpr int kUnitLogStride = 4;            // doubles per entry: RN(1/c), hi, lo, 0

// Table: entry i holds RN(1/c_i) and -ln RN(1/c_i) = hi + lo, c_i = 1 + i/64 (hi rounded to
// double, lo the rounded remainder, from the extended-precision logarithm).
inline void unit_log_table(double* tab) {
  for (int i = 0; i < kUnitLogEntries; ++i) {
    const double c = 1.0 + static_cast<double>(i) / 64.0;
    const double inv = 1.0 / c;
    const long double l = -logl(static_cast<long double>(inv));
    const double hi = static_cast<double>(l);
    tab[kUnitLogStride * i] = inv;
    tab[kUnitLogStride * i + 1] = hi;
    tab[kUnitLogStride * i + 2] = static_cast<double>(l - static_cast<long double>(hi));
    tab[kUnitLogStride * i + 3] = 0.0;
  }
}

__host__ __device__ inline double unit_log(double x, const double* __restrict__ tab) {
  int e;
  const double mant = frexp(x, &e);          // x = mant 2^e, mant in [0.5, 1)
  // Within 2^-7 of 1, take m = x with exponent 0 and entry 0 (RN(1/c) = 1, no log term):
  // then r = x - 1 exactly.  Elsewhere m = 2 mant in [1, 2) with exponent e - 1.
  const bool near1 = x > 0x1.fcp-1;
  const double m = near1 ? x : 2.0 * mant;
  uint64_t bits;
  memcpy(&bits, &m, sizeof(bits));
  const int i = near1 ? 0 : static_cast<int>((bits >> 46) & 63u);   // top six fraction bits
  const double ed = near1 ? 0.0 : static_cast<double>(e - 1);
  const double* t = tab + kUnitLogStride * i;
  const double r = fma(m, t[0], -1.0);
  double p = 1.0 / 9.0;
  p = fma(p, r, -1.0 / 8.0);
  p = fma(p, r, 1.0 / 7.0);
  p = fma(p, r, -1.0 / 6.0);
  p = fma(p, r, 1.0 / 5.0);
  p = fma(p, r, -1.0 / 4.0);
  p = fma(p, r, 1.0 / 3.0);
  p = fma(p, r, -0.5);
  const double lp = fma(r * r, p, r);                     // log1p(r)
  const double ln2_hi = 0x1.62e42fefa3800p-1;             // 42 significant bits: ed ln2_hi exact
  const double ln2_lo = 0x1.ef35793c76730p-45;
  const double hi = fma(ed, ln2_hi, t[1]);                // exact where the two terms cancel
  const double lo = fma(ed, ln2_lo, t[2] + lp);
  return hi + lo;
}

}  // namespace swarm_impl
