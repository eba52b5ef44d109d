// ms_ad.hpp -- TEST INFRASTRUCTURE ONLY: scalar types for the CPU oracle.
//
//   adouble : reverse-mode tape (one thread-local tape per worker thread)
//   dual    : forward-mode tangent
//   cdouble : double that counts floating-point operations
//
// The oracle's step is written once as a template over the scalar; these
// types turn the same arithmetic into its exact VJP, JVP and operation count.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

inline double val(double x) { return x; }

// ------------------------------------------------------------------ adouble
struct Tape {
  struct Node { int32_t a, b; double da, db; };
  std::vector<Node> nodes;
  std::vector<double> adj;
  void clear() { nodes.clear(); }
  int32_t leaf() { nodes.push_back({-1, -1, 0.0, 0.0}); return (int32_t)nodes.size() - 1; }
  int32_t push(int32_t a, double da, int32_t b, double db) {
    nodes.push_back(Node{a, b, da, db});
    return (int32_t)nodes.size() - 1;
  }
  // Propagate adjoints from the seeds already written into adj.
  void reverse() {
    for (int64_t i = (int64_t)nodes.size() - 1; i >= 0; --i) {
      const Node& n = nodes[(size_t)i];
      double g = adj[(size_t)i];
      if (g == 0.0) continue;
      if (n.a >= 0) adj[(size_t)n.a] += g * n.da;
      if (n.b >= 0) adj[(size_t)n.b] += g * n.db;
    }
  }
};
extern thread_local Tape* g_tape;

struct adouble {
  double v;
  int32_t i;  // tape index, -1 for a constant
  adouble() : v(0.0), i(-1) {}
  adouble(double x) : v(x), i(-1) {}
  adouble(double x, int32_t idx) : v(x), i(idx) {}
  static adouble var(double x) { return adouble(x, g_tape->leaf()); }
  adouble& operator+=(const adouble& o);
  adouble& operator-=(const adouble& o);
  adouble& operator*=(const adouble& o);
  adouble& operator/=(const adouble& o);
};
inline double val(const adouble& x) { return x.v; }
inline adouble mk1(double v, const adouble& a, double da) {
  if (a.i < 0) return adouble(v);
  return adouble(v, g_tape->push(a.i, da, -1, 0.0));
}
inline adouble mk2(double v, const adouble& a, double da, const adouble& b, double db) {
  if (a.i < 0 && b.i < 0) return adouble(v);
  if (a.i < 0) return adouble(v, g_tape->push(b.i, db, -1, 0.0));
  if (b.i < 0) return adouble(v, g_tape->push(a.i, da, -1, 0.0));
  return adouble(v, g_tape->push(a.i, da, b.i, db));
}
inline adouble operator+(const adouble& a, const adouble& b) { return mk2(a.v + b.v, a, 1.0, b, 1.0); }
inline adouble operator-(const adouble& a, const adouble& b) { return mk2(a.v - b.v, a, 1.0, b, -1.0); }
inline adouble operator*(const adouble& a, const adouble& b) { return mk2(a.v * b.v, a, b.v, b, a.v); }
inline adouble operator/(const adouble& a, const adouble& b) {
  double r = a.v / b.v;
  return mk2(r, a, 1.0 / b.v, b, -r / b.v);
}
inline adouble operator-(const adouble& a) { return mk1(-a.v, a, -1.0); }
inline adouble operator+(const adouble& a, double b) { return mk1(a.v + b, a, 1.0); }
inline adouble operator+(double a, const adouble& b) { return mk1(a + b.v, b, 1.0); }
inline adouble operator-(const adouble& a, double b) { return mk1(a.v - b, a, 1.0); }
inline adouble operator-(double a, const adouble& b) { return mk1(a - b.v, b, -1.0); }
inline adouble operator*(const adouble& a, double b) { return mk1(a.v * b, a, b); }
inline adouble operator*(double a, const adouble& b) { return mk1(a * b.v, b, a); }
inline adouble operator/(const adouble& a, double b) { return mk1(a.v / b, a, 1.0 / b); }
inline adouble operator/(double a, const adouble& b) {
  double r = a / b.v;
  return mk1(r, b, -r / b.v);
}
inline adouble& adouble::operator+=(const adouble& o) { *this = *this + o; return *this; }
inline adouble& adouble::operator-=(const adouble& o) { *this = *this - o; return *this; }
inline adouble& adouble::operator*=(const adouble& o) { *this = *this * o; return *this; }
inline adouble& adouble::operator/=(const adouble& o) { *this = *this / o; return *this; }
inline adouble Sqrt(const adouble& a) {
  double r = std::sqrt(a.v);
  return mk1(r, a, r > 0.0 ? 0.5 / r : 0.0);
}
inline adouble Sin(const adouble& a) { return mk1(std::sin(a.v), a, std::cos(a.v)); }
inline adouble Cos(const adouble& a) { return mk1(std::cos(a.v), a, -std::sin(a.v)); }

// --------------------------------------------------------------------- dual
struct dual {
  double v, d;
  dual() : v(0.0), d(0.0) {}
  dual(double x) : v(x), d(0.0) {}
  dual(double x, double dx) : v(x), d(dx) {}
  dual& operator+=(const dual& o) { v += o.v; d += o.d; return *this; }
  dual& operator-=(const dual& o) { v -= o.v; d -= o.d; return *this; }
  dual& operator*=(const dual& o) { d = d * o.v + v * o.d; v *= o.v; return *this; }
  dual& operator/=(const dual& o) { double r = v / o.v; d = (d - r * o.d) / o.v; v = r; return *this; }
};
inline double val(const dual& x) { return x.v; }
inline dual operator+(dual a, const dual& b) { return a += b; }
inline dual operator-(dual a, const dual& b) { return a -= b; }
inline dual operator*(dual a, const dual& b) { return a *= b; }
inline dual operator/(dual a, const dual& b) { return a /= b; }
inline dual operator-(const dual& a) { return dual(-a.v, -a.d); }
inline dual operator+(const dual& a, double b) { return dual(a.v + b, a.d); }
inline dual operator+(double a, const dual& b) { return dual(a + b.v, b.d); }
inline dual operator-(const dual& a, double b) { return dual(a.v - b, a.d); }
inline dual operator-(double a, const dual& b) { return dual(a - b.v, -b.d); }
inline dual operator*(const dual& a, double b) { return dual(a.v * b, a.d * b); }
inline dual operator*(double a, const dual& b) { return dual(a * b.v, a * b.d); }
inline dual operator/(const dual& a, double b) { return dual(a.v / b, a.d / b); }
inline dual operator/(double a, const dual& b) { double r = a / b.v; return dual(r, -r * b.d / b.v); }
inline dual Sqrt(const dual& a) { double r = std::sqrt(a.v); return dual(r, r > 0.0 ? 0.5 * a.d / r : 0.0); }
inline dual Sin(const dual& a) { return dual(std::sin(a.v), std::cos(a.v) * a.d); }
inline dual Cos(const dual& a) { return dual(std::cos(a.v), -std::sin(a.v) * a.d); }

// ------------------------------------------------------------------ cdouble
extern thread_local uint64_t g_flops;
struct cdouble {
  double v;
  cdouble() : v(0.0) {}
  cdouble(double x) : v(x) {}
  cdouble& operator+=(const cdouble& o) { ++g_flops; v += o.v; return *this; }
  cdouble& operator-=(const cdouble& o) { ++g_flops; v -= o.v; return *this; }
  cdouble& operator*=(const cdouble& o) { ++g_flops; v *= o.v; return *this; }
  cdouble& operator/=(const cdouble& o) { ++g_flops; v /= o.v; return *this; }
};
inline double val(const cdouble& x) { return x.v; }
inline cdouble operator+(cdouble a, const cdouble& b) { return a += b; }
inline cdouble operator-(cdouble a, const cdouble& b) { return a -= b; }
inline cdouble operator*(cdouble a, const cdouble& b) { return a *= b; }
inline cdouble operator/(cdouble a, const cdouble& b) { return a /= b; }
inline cdouble operator-(const cdouble& a) { return cdouble(-a.v); }
inline cdouble operator+(const cdouble& a, double b) { ++g_flops; return cdouble(a.v + b); }
inline cdouble operator+(double a, const cdouble& b) { ++g_flops; return cdouble(a + b.v); }
inline cdouble operator-(const cdouble& a, double b) { ++g_flops; return cdouble(a.v - b); }
inline cdouble operator-(double a, const cdouble& b) { ++g_flops; return cdouble(a - b.v); }
inline cdouble operator*(const cdouble& a, double b) { ++g_flops; return cdouble(a.v * b); }
inline cdouble operator*(double a, const cdouble& b) { ++g_flops; return cdouble(a * b.v); }
inline cdouble operator/(const cdouble& a, double b) { ++g_flops; return cdouble(a.v / b); }
inline cdouble operator/(double a, const cdouble& b) { ++g_flops; return cdouble(a / b.v); }
inline cdouble Sqrt(const cdouble& a) { ++g_flops; return cdouble(std::sqrt(a.v)); }
inline cdouble Sin(const cdouble& a) { ++g_flops; return cdouble(std::sin(a.v)); }
inline cdouble Cos(const cdouble& a) { ++g_flops; return cdouble(std::cos(a.v)); }

// --------------------------------------------------------------------- f32s
// IEEE binary32 evaluation: every operation rounds to float, and a double
// operand (a parameter such as h, or a literal) is rounded to float first, so
// no intermediate is carried in double.  Used for the FP32 error floor.
struct f32s {
  float v;
  f32s() : v(0.0f) {}
  f32s(double x) : v((float)x) {}
  f32s& operator+=(const f32s& o) { v = v + o.v; return *this; }
  f32s& operator-=(const f32s& o) { v = v - o.v; return *this; }
  f32s& operator*=(const f32s& o) { v = v * o.v; return *this; }
  f32s& operator/=(const f32s& o) { v = v / o.v; return *this; }
};
inline double val(const f32s& x) { return x.v; }
inline f32s operator+(f32s a, const f32s& b) { return a += b; }
inline f32s operator-(f32s a, const f32s& b) { return a -= b; }
inline f32s operator*(f32s a, const f32s& b) { return a *= b; }
inline f32s operator/(f32s a, const f32s& b) { return a /= b; }
inline f32s operator-(const f32s& a) { f32s r; r.v = -a.v; return r; }
inline f32s operator+(const f32s& a, double b) { return a + f32s(b); }
inline f32s operator+(double a, const f32s& b) { return f32s(a) + b; }
inline f32s operator-(const f32s& a, double b) { return a - f32s(b); }
inline f32s operator-(double a, const f32s& b) { return f32s(a) - b; }
inline f32s operator*(const f32s& a, double b) { return a * f32s(b); }
inline f32s operator*(double a, const f32s& b) { return f32s(a) * b; }
inline f32s operator/(const f32s& a, double b) { return a / f32s(b); }
inline f32s operator/(double a, const f32s& b) { return f32s(a) / b; }
inline f32s Sqrt(const f32s& a) { f32s r; r.v = std::sqrt(a.v); return r; }
inline f32s Sin(const f32s& a) { f32s r; r.v = std::sin(a.v); return r; }
inline f32s Cos(const f32s& a) { f32s r; r.v = std::cos(a.v); return r; }

inline double Sqrt(double a) { return std::sqrt(a); }
inline double val(float x) { return x; }
inline float Sqrt(float a) { return std::sqrt(a); }
inline float Sin(float a) { return std::sin(a); }
inline float Cos(float a) { return std::cos(a); }
inline double Sin(double a) { return std::sin(a); }
inline double Cos(double a) { return std::cos(a); }
