// tgks_opcount.hpp -- host-only scalar type that counts the floating-point
// operations of the device math templates of tgks_device.hpp, evaluated on
// the host, to report the algorithmic operation count of the kernels.
//
// The count is the size of the computation's dataflow graph: every value
// carries an identity; an operation on operands already combined the same
// way (commutative operands in either order) returns the earlier result and
// is not counted again, as common-subexpression elimination does.  Constants
// with equal values share one identity.  +, -, *, / and each of sqrt, rsqrt,
// exp, expm1, erfc count one operation; negation, comparisons and fabs count
// none.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>

namespace tgks_opcount {

struct Tally {
  long long add = 0, mul = 0, div = 0, sqrt = 0, exp = 0, expm1 = 0, erfc = 0;
  long long total() const { return add + mul + div + sqrt + exp + expm1 + erfc; }
};

struct Graph {
  Tally t;
  long long next = 1;
  std::map<uint64_t, long long> consts;                          // value bits -> id
  std::map<std::tuple<int, long long, long long>, long long> ops;  // (op, a, b) -> id
  void reset() {
    t = Tally();
    next = 1;
    consts.clear();
    ops.clear();
  }
};

inline Graph& graph() {
  static thread_local Graph g;
  return g;
}
inline Tally& tally() { return graph().t; }

struct F {
  double v;
  long long id;
  F() : v(0.0), id(constant_id(0.0)) {}
  F(double x) : v(x), id(constant_id(x)) {}
  F(double x, long long i) : v(x), id(i) {}
  static long long constant_id(double x) {
    uint64_t b;
    std::memcpy(&b, &x, sizeof b);
    auto& g = graph();
    auto it = g.consts.find(b);
    if (it != g.consts.end()) return it->second;
    const long long id = g.next++;
    g.consts[b] = id;
    return id;
  }
  // a fresh input value (distinct from every other value)
  static F input(double x) { return F(x, graph().next++); }
};

enum Op { ADD, SUB, MUL, DIV, SQRT, RSQRT, EXP, EXPM1, ERFC, NEG };

inline F apply(Op op, F a, F b, double v, long long* counter) {
  long long x = a.id, y = b.id;
  if ((op == ADD || op == MUL) && x > y) std::swap(x, y);
  auto& g = graph();
  const auto key = std::make_tuple((int)op, x, y);
  auto it = g.ops.find(key);
  if (it != g.ops.end()) return F(v, it->second);
  const long long id = g.next++;
  g.ops[key] = id;
  if (counter) ++*counter;
  return F(v, id);
}

inline F operator+(F a, F b) { return apply(ADD, a, b, a.v + b.v, &tally().add); }
inline F operator-(F a, F b) { return apply(SUB, a, b, a.v - b.v, &tally().add); }
inline F operator*(F a, F b) { return apply(MUL, a, b, a.v * b.v, &tally().mul); }
inline F operator/(F a, F b) { return apply(DIV, a, b, a.v / b.v, &tally().div); }
inline F operator-(F a) { return apply(NEG, a, a, -a.v, nullptr); }
inline F& operator+=(F& a, F b) { return a = a + b; }
inline F& operator-=(F& a, F b) { return a = a - b; }
inline F& operator*=(F& a, F b) { return a = a * b; }
inline bool operator<(F a, F b) { return a.v < b.v; }
inline bool operator>(F a, F b) { return a.v > b.v; }
inline bool operator<=(F a, F b) { return a.v <= b.v; }
inline bool operator>=(F a, F b) { return a.v >= b.v; }
inline bool operator==(F a, F b) { return a.v == b.v; }
inline bool operator!=(F a, F b) { return a.v != b.v; }
inline F sqrt(F a) { return apply(SQRT, a, a, std::sqrt(a.v), &tally().sqrt); }
inline F exp(F a) { return apply(EXP, a, a, std::exp(a.v), &tally().exp); }
inline F expm1(F a) { return apply(EXPM1, a, a, std::expm1(a.v), &tally().expm1); }
inline F erfc(F a) { return apply(ERFC, a, a, std::erfc(a.v), &tally().erfc); }
inline F rsqrt(F a) { return apply(RSQRT, a, a, 1.0 / std::sqrt(a.v), &tally().sqrt); }
inline F fabs(F a) { return a.v < 0 ? -a : a; }

}  // namespace tgks_opcount
