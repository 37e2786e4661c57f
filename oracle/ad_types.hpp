// Automatic-differentiation scalars for the oracle -- TEST INFRASTRUCTURE ONLY.
//
// Dual: forward mode, value + one tangent (Jacobian-vector products).
// Var:  reverse mode on a global tape (vector-Jacobian products): every
//       operation appends a node with up to two parents and the local
//       partial derivatives; backward() sweeps the tape once in reverse.
// Non-smooth points follow fixed conventions: |x| has derivative sign(x)
// with sign(0) = 0; comparisons (branches, maxima) are taken on values, so
// a maximum propagates to the first maximal argument.
#pragma once

#include <cmath>
#include <vector>

namespace orc {

// ---------------------------------------------------------------- forward
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
inline Dual fabs(Dual a) { return Dual(std::fabs(a.v), a.v > 0 ? a.d : (a.v < 0 ? -a.d : 0.0)); }

// ---------------------------------------------------------------- reverse
struct TapeNode { int p0, p1; double d0, d1; };

struct Tape {
  std::vector<TapeNode> nodes;
  std::vector<double> adj;
  int push(int p0, double d0, int p1, double d1) {
    nodes.push_back({p0, p1, d0, d1});
    return (int)nodes.size() - 1;
  }
  void clear() { nodes.clear(); adj.clear(); }
  // seed adjoints are set in adj by the caller; propagate to the leaves
  void backward() {
    for (int i = (int)nodes.size() - 1; i >= 0; --i) {
      const TapeNode& n = nodes[i];
      const double a = adj[i];
      if (a == 0.0) continue;
      if (n.p0 >= 0) adj[n.p0] += a * n.d0;
      if (n.p1 >= 0) adj[n.p1] += a * n.d1;
    }
  }
  static Tape& get() { static Tape t; return t; }
};

struct Var {
  double v;
  int id;  // -1: constant
  Var() : v(0.0), id(-1) {}
  Var(double x) : v(x), id(-1) {}
  Var(double x, int i) : v(x), id(i) {}
  static Var leaf(double x) { return Var(x, Tape::get().push(-1, 0.0, -1, 0.0)); }
};

inline Var mk(double v, int p0, double d0, int p1, double d1) {
  if (p0 < 0 && p1 < 0) return Var(v);
  return Var(v, Tape::get().push(p0, d0, p1, d1));
}
inline Var operator+(Var a, Var b) { return mk(a.v + b.v, a.id, 1.0, b.id, 1.0); }
inline Var operator-(Var a, Var b) { return mk(a.v - b.v, a.id, 1.0, b.id, -1.0); }
inline Var operator*(Var a, Var b) { return mk(a.v * b.v, a.id, b.v, b.id, a.v); }
inline Var operator/(Var a, Var b) {
  const double q = a.v / b.v;
  return mk(q, a.id, 1.0 / b.v, b.id, -q / b.v);
}
inline Var operator-(Var a) { return mk(-a.v, a.id, -1.0, -1, 0.0); }
inline bool operator<=(Var a, Var b) { return a.v <= b.v; }
inline bool operator>(Var a, Var b) { return a.v > b.v; }
inline Var sqrt(Var a) {
  const double s = std::sqrt(a.v);
  return mk(s, a.id, 0.5 / s, -1, 0.0);
}
inline Var fabs(Var a) {
  const double g = a.v > 0 ? 1.0 : (a.v < 0 ? -1.0 : 0.0);
  return mk(std::fabs(a.v), a.id, g, -1, 0.0);
}

}  // namespace orc
