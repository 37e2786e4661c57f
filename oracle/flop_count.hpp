// Operation-counting scalar for the oracle -- TEST INFRASTRUCTURE ONLY.
// Instantiating the oracle with this type counts every floating-point add,
// subtract, multiply, divide and square root applied to state-dependent
// values (sign changes, absolute values and comparisons are free).  Work done
// on metric values alone (plain doubles in the oracle) is not counted.
#pragma once

#include <cmath>

namespace orc {

struct Counted {
  double v;
  static long long& n() { static long long c = 0; return c; }
  Counted() : v(0.0) {}
  Counted(double x) : v(x) {}
};

inline Counted operator+(Counted a, Counted b) { ++Counted::n(); return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { ++Counted::n(); return Counted(a.v - b.v); }
inline Counted operator*(Counted a, Counted b) { ++Counted::n(); return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { ++Counted::n(); return Counted(a.v / b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }
inline bool operator<=(Counted a, Counted b) { return a.v <= b.v; }
inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
inline Counted sqrt(Counted a) { ++Counted::n(); return Counted(std::sqrt(a.v)); }
inline Counted fabs(Counted a) { return Counted(std::fabs(a.v)); }

}  // namespace orc
