// tgks_opcount.hpp -- host-only scalar type that counts floating-point
// operations, used to evaluate the device math templates of tgks_device.hpp
// on the host and report the algorithmic operation count of the kernels:
// +, -, *, / and each of sqrt, exp, expm1, erfc count one operation (a fused
// multiply-add counts two); negation, comparisons and fabs count none.
#pragma once
#include <cmath>

namespace tgks_opcount {

struct Tally {
  long long add = 0, mul = 0, div = 0, sqrt = 0, exp = 0, expm1 = 0, erfc = 0;
  long long total() const { return add + mul + div + sqrt + exp + expm1 + erfc; }
};

inline Tally& tally() {
  static thread_local Tally t;
  return t;
}

struct F {
  double v;
  F() : v(0.0) {}
  F(double x) : v(x) {}
};

inline F operator+(F a, F b) { ++tally().add; return F(a.v + b.v); }
inline F operator-(F a, F b) { ++tally().add; return F(a.v - b.v); }
inline F operator*(F a, F b) { ++tally().mul; return F(a.v * b.v); }
inline F operator/(F a, F b) { ++tally().div; return F(a.v / b.v); }
inline F operator-(F a) { return F(-a.v); }
inline F& operator+=(F& a, F b) { return a = a + b; }
inline F& operator-=(F& a, F b) { return a = a - b; }
inline F& operator*=(F& a, F b) { return a = a * b; }
inline bool operator<(F a, F b) { return a.v < b.v; }
inline bool operator>(F a, F b) { return a.v > b.v; }
inline bool operator<=(F a, F b) { return a.v <= b.v; }
inline bool operator>=(F a, F b) { return a.v >= b.v; }
inline bool operator==(F a, F b) { return a.v == b.v; }
inline bool operator!=(F a, F b) { return a.v != b.v; }
inline F sqrt(F a) { ++tally().sqrt; return F(std::sqrt(a.v)); }
inline F exp(F a) { ++tally().exp; return F(std::exp(a.v)); }
inline F expm1(F a) { ++tally().expm1; return F(std::expm1(a.v)); }
inline F erfc(F a) { ++tally().erfc; return F(std::erfc(a.v)); }
inline F fabs(F a) { return F(std::fabs(a.v)); }

}  // namespace tgks_opcount
