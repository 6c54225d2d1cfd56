/*
 * opcount.cpp -- the oracle's op-counting build.  TEST INFRASTRUCTURE ONLY,
 * like the oracle itself: only the tests, the smoke check and the CPU leg of
 * the benchmark may load it, and the GPU library shares nothing with it.
 *
 * It compiles the oracle's own source (tk_oracle.c) as C++ with every double
 * replaced by or_counted, a scalar that holds one double and counts each
 * arithmetic operation it takes part in.  The values it computes are the
 * oracle's, bit for bit (the same IEEE operations in the same order); what it
 * adds is a count of the floating-point work of each routine, so that the
 * algorithmic flops per pair of every kernel are counted rather than
 * estimated (section "Hotspots" ranks the routines by time; the counts say
 * how much arithmetic each pair of each routine is).
 *
 * Counting rules: +, -, * and / count one flop each (negation none); fma
 * counts two; sqrt, exp, erfc, pow, cos and sin count one call each of their
 * own kind (their flops depend on the library, so they are reported apart);
 * rint, floor and fabs are counted as "other".  Comparisons and conversions
 * are not counted.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <type_traits>

namespace {
struct OpCounts {
  long long add, mul, div, fma, sqrt, exp, erfc, trig, pow, other;
};
OpCounts g_ops;
}  // namespace

struct or_counted {
  double v;
  or_counted() = default;
  constexpr or_counted(double x) : v(x) {}
  template <class I, class = typename std::enable_if<std::is_integral<I>::value>::type>
  constexpr or_counted(I x) : v((double)x) {}
  template <class I, class = typename std::enable_if<std::is_integral<I>::value>::type>
  explicit operator I() const { return (I)v; }
  or_counted operator-() const { return or_counted(-v); }
  or_counted& operator+=(or_counted o) { ++g_ops.add; v += o.v; return *this; }
  or_counted& operator-=(or_counted o) { ++g_ops.add; v -= o.v; return *this; }
  or_counted& operator*=(or_counted o) { ++g_ops.mul; v *= o.v; return *this; }
  or_counted& operator/=(or_counted o) { ++g_ops.div; v /= o.v; return *this; }
};
static_assert(sizeof(or_counted) == sizeof(double), "arrays of it are arrays of doubles");
static_assert(std::is_trivially_copyable<or_counted>::value, "memcpy-able like a double");

static inline or_counted operator+(or_counted a, or_counted b) { ++g_ops.add; return a.v + b.v; }
static inline or_counted operator-(or_counted a, or_counted b) { ++g_ops.add; return a.v - b.v; }
static inline or_counted operator*(or_counted a, or_counted b) { ++g_ops.mul; return a.v * b.v; }
static inline or_counted operator/(or_counted a, or_counted b) { ++g_ops.div; return a.v / b.v; }
static inline bool operator<(or_counted a, or_counted b) { return a.v < b.v; }
static inline bool operator>(or_counted a, or_counted b) { return a.v > b.v; }
static inline bool operator<=(or_counted a, or_counted b) { return a.v <= b.v; }
static inline bool operator>=(or_counted a, or_counted b) { return a.v >= b.v; }
static inline bool operator==(or_counted a, or_counted b) { return a.v == b.v; }
static inline bool operator!=(or_counted a, or_counted b) { return a.v != b.v; }
static inline bool operator!(or_counted a) { return !a.v; }

static inline or_counted fma(or_counted a, or_counted b, or_counted c) {
  ++g_ops.fma;
  return std::fma(a.v, b.v, c.v);
}
static inline or_counted sqrt(or_counted a) { ++g_ops.sqrt; return std::sqrt(a.v); }
static inline or_counted exp(or_counted a) { ++g_ops.exp; return std::exp(a.v); }
static inline or_counted erfc(or_counted a) { ++g_ops.erfc; return std::erfc(a.v); }
static inline or_counted cos(or_counted a) { ++g_ops.trig; return std::cos(a.v); }
static inline or_counted sin(or_counted a) { ++g_ops.trig; return std::sin(a.v); }
static inline or_counted pow(or_counted a, or_counted b) { ++g_ops.pow; return std::pow(a.v, b.v); }
static inline or_counted rint(or_counted a) { ++g_ops.other; return std::rint(a.v); }
static inline or_counted floor(or_counted a) { ++g_ops.other; return std::floor(a.v); }
static inline or_counted fabs(or_counted a) { ++g_ops.other; return std::fabs(a.v); }
static inline bool isfinite(or_counted a) { return std::isfinite(a.v); }

extern "C" {
// every double of the oracle below is the counting scalar
#define double or_counted
#include "tk_oracle.c"
#undef double

void or_ops_reset(void) { memset(&g_ops, 0, sizeof g_ops); }
/* out[10]: add/sub, mul, div, fma, sqrt, exp, erfc, cos+sin, pow, other (rint, floor, fabs) */
void or_ops_read(long long* out) {
  const long long v[10] = {g_ops.add, g_ops.mul, g_ops.div,  g_ops.fma, g_ops.sqrt,
                           g_ops.exp, g_ops.erfc, g_ops.trig, g_ops.pow, g_ops.other};
  memcpy(out, v, sizeof v);
}
}
