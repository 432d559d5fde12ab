// Scalar types the oracle is instantiated with.
//
// TEST INFRASTRUCTURE ONLY. The oracle is the slow, obviously correct FP64
// statement of the method that the tests, the smoke check and the CPU-baseline
// leg of the benchmark compare against. Nothing in the product path includes,
// links or calls it.
//
//   double    — the reference result.
//   Dual<N>   — forward-mode dual numbers: value plus N directional
//               derivatives, giving exact Jacobian-vector products of the
//               very same code (used to assemble the oracle's adjoint).
//   Counted   — a double that counts its floating-point operations
//               (add/sub/mul/div/sqrt/atan2/asin each count one), used to
//               measure the algorithmic work per environment step.
//   Traced    — a double that records every operation on a state- or
//               action-dependent value (a linear trace of the computation),
//               used to count the operations of one reverse (adjoint) sweep
//               through the step.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

namespace orc {

// ---------------------------------------------------------------- double
inline double val(double x) { return x; }
inline double osqrt(double x) { return std::sqrt(x); }
inline double oatan2(double y, double x) { return std::atan2(y, x); }
inline double oasin(double x) { return std::asin(x); }
inline double ocos(double x) { return std::cos(x); }
inline double osin(double x) { return std::sin(x); }

// ---------------------------------------------------------------- Dual<N>
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0) { for (int i = 0; i < N; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0; }  // NOLINT
};
template <int N> inline double val(const Dual<N>& a) { return a.v; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r;
}
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> inline Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> inline Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { a = a - b; return a; }
// Elementary functions: value and the chain rule with the textbook derivative.
template <int N> inline Dual<N> chain(double fv, double dfdx, const Dual<N>& x) {
  Dual<N> r; r.v = fv; for (int i = 0; i < N; ++i) r.d[i] = dfdx * x.d[i]; return r;
}
template <int N> inline Dual<N> osqrt(const Dual<N>& x) {
  double s = std::sqrt(x.v); return chain(s, 0.5 / s, x);
}
template <int N> inline Dual<N> oasin(const Dual<N>& x) {
  // d/dx asin x = 1/sqrt(1-x^2); at |x| = 1 the clamp upstream fixes the
  // convention that the derivative there is zero.
  double den = 1.0 - x.v * x.v;
  return chain(std::asin(x.v), den > 0 ? 1.0 / std::sqrt(den) : 0.0, x);
}
template <int N> inline Dual<N> ocos(const Dual<N>& x) { return chain(std::cos(x.v), -std::sin(x.v), x); }
template <int N> inline Dual<N> osin(const Dual<N>& x) { return chain(std::sin(x.v), std::cos(x.v), x); }
template <int N> inline Dual<N> oatan2(const Dual<N>& y, const Dual<N>& x) {
  // d atan2(y,x) = (x dy - y dx) / (x^2 + y^2)
  Dual<N> r; r.v = std::atan2(y.v, x.v);
  double den = x.v * x.v + y.v * y.v;
  for (int i = 0; i < N; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) / den;
  return r;
}

// ---------------------------------------------------------------- Counted
extern thread_local int64_t g_flops;
struct Counted {
  double v;
  Counted() : v(0) {}
  Counted(double x) : v(x) {}  // NOLINT
};
inline double val(const Counted& a) { return a.v; }
inline Counted operator+(Counted a, Counted b) { ++g_flops; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { ++g_flops; return Counted(a.v - b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }  // sign flip: free
inline Counted operator*(Counted a, Counted b) { ++g_flops; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { ++g_flops; return Counted(a.v / b.v); }
inline Counted& operator+=(Counted& a, Counted b) { a = a + b; return a; }
inline Counted& operator-=(Counted& a, Counted b) { a = a - b; return a; }
inline Counted osqrt(Counted x) { ++g_flops; return Counted(std::sqrt(x.v)); }
inline Counted oasin(Counted x) { ++g_flops; return Counted(std::asin(x.v)); }
inline Counted ocos(Counted x) { ++g_flops; return Counted(std::cos(x.v)); }
inline Counted osin(Counted x) { ++g_flops; return Counted(std::sin(x.v)); }
inline Counted oatan2(Counted y, Counted x) { ++g_flops; return Counted(std::atan2(y.v, x.v)); }

// ---------------------------------------------------------------- Traced
// Each value computed from the inputs is a node of a thread-local trace:
// (kind, up to two operand nodes; -1 marks a constant operand). Values built
// from constants only are constants and are not recorded. Comparisons and
// branches read the value and record nothing (a selected value passes
// through), so the trace holds exactly the arithmetic the outputs depend on
// along the branches taken.
enum TraceOp : int8_t { T_LEAF, T_ADD, T_SUB, T_NEG, T_MUL, T_DIV, T_SQRT, T_ASIN, T_SIN, T_COS, T_ATAN2 };
struct TraceNode {
  int8_t op;
  int32_t a, b;
};
extern thread_local std::vector<TraceNode>* g_trace;
struct Traced {
  double v;
  int32_t id;
  Traced() : v(0), id(-1) {}
  Traced(double x) : v(x), id(-1) {}  // NOLINT
};
inline Traced trace_leaf(double x) {
  Traced r(x);
  r.id = (int32_t)g_trace->size();
  g_trace->push_back(TraceNode{T_LEAF, -1, -1});
  return r;
}
inline Traced trace_op(double v, TraceOp op, int32_t a, int32_t b) {
  Traced r(v);
  if (a >= 0 || b >= 0) {
    r.id = (int32_t)g_trace->size();
    g_trace->push_back(TraceNode{op, a, b});
  }
  return r;
}
inline double val(const Traced& a) { return a.v; }
inline Traced operator+(Traced a, Traced b) { return trace_op(a.v + b.v, T_ADD, a.id, b.id); }
inline Traced operator-(Traced a, Traced b) { return trace_op(a.v - b.v, T_SUB, a.id, b.id); }
inline Traced operator-(Traced a) { return trace_op(-a.v, T_NEG, a.id, -1); }
inline Traced operator*(Traced a, Traced b) { return trace_op(a.v * b.v, T_MUL, a.id, b.id); }
inline Traced operator/(Traced a, Traced b) { return trace_op(a.v / b.v, T_DIV, a.id, b.id); }
inline Traced& operator+=(Traced& a, Traced b) { a = a + b; return a; }
inline Traced& operator-=(Traced& a, Traced b) { a = a - b; return a; }
inline Traced osqrt(Traced x) { return trace_op(std::sqrt(x.v), T_SQRT, x.id, -1); }
inline Traced oasin(Traced x) { return trace_op(std::asin(x.v), T_ASIN, x.id, -1); }
inline Traced ocos(Traced x) { return trace_op(std::cos(x.v), T_COS, x.id, -1); }
inline Traced osin(Traced x) { return trace_op(std::sin(x.v), T_SIN, x.id, -1); }
inline Traced oatan2(Traced y, Traced x) { return trace_op(std::atan2(y.v, x.v), T_ATAN2, y.id, x.id); }

}  // namespace orc
