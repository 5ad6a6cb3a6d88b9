// opcount.cpp -- counts the floating-point operations the FP64 oracle
// performs (test infrastructure).  A copy of orc.c whose `double` is renamed
// `orc_real` (made by pyorc.build_opcount) is compiled here as C++ with
// orc_real a value type that tallies every +, -, *, /, sqrt and exp; the
// counts per flux evaluation and per cell-update give the algorithmic flop
// figures used for the arithmetic roofline.  Built without OpenMP so the
// tallies are exact.
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>

namespace opc {
struct Tally {
  long long add = 0, mul = 0, div = 0, sqrt = 0, exp = 0;
};
static Tally t;
struct D {
  double v;
  D() : v(0) {}
  D(double x) : v(x) {}
  D& operator+=(D o) { ++t.add; v += o.v; return *this; }
  D& operator-=(D o) { ++t.add; v -= o.v; return *this; }
  D& operator*=(D o) { ++t.mul; v *= o.v; return *this; }
  D& operator/=(D o) { ++t.div; v /= o.v; return *this; }
};
inline D operator+(D a, D b) { ++t.add; return D(a.v + b.v); }
inline D operator-(D a, D b) { ++t.add; return D(a.v - b.v); }
inline D operator-(D a) { return D(-a.v); }
inline D operator*(D a, D b) { ++t.mul; return D(a.v * b.v); }
inline D operator/(D a, D b) { ++t.div; return D(a.v / b.v); }
inline bool operator<(D a, D b) { return a.v < b.v; }
inline bool operator>(D a, D b) { return a.v > b.v; }
inline bool operator<=(D a, D b) { return a.v <= b.v; }
inline bool operator>=(D a, D b) { return a.v >= b.v; }
inline bool operator==(D a, D b) { return a.v == b.v; }
inline bool operator!=(D a, D b) { return a.v != b.v; }
inline D sqrt(D a) { ++t.sqrt; return D(std::sqrt(a.v)); }
inline D exp(D a) { ++t.exp; return D(std::exp(a.v)); }
inline D fabs(D a) { return D(std::fabs(a.v)); }
inline bool isfinite(D a) { return std::isfinite(a.v); }
}  // namespace opc

#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

using opc::exp;
using opc::fabs;
using opc::isfinite;
using opc::sqrt;
typedef opc::D orc_real;
#include ORC_REAL_SOURCE

extern "C" {
// Operation tallies since the last reset: add (incl. subtract), mul, div,
// sqrt, exp.
void opc_reset(void) { opc::t = opc::Tally(); }
void opc_get(long long out[5]) {
  out[0] = opc::t.add;
  out[1] = opc::t.mul;
  out[2] = opc::t.div;
  out[3] = opc::t.sqrt;
  out[4] = opc::t.exp;
}
}
