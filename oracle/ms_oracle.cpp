// ms_oracle.cpp -- TEST INFRASTRUCTURE ONLY (see ms_oracle.hpp).
//
// FP64 CPU oracle of the batched rigid-body control step.  Plain loops, no
// blocking, fusion or reordering beyond what each definition states.  The
// whole step is a template over the scalar type so that the same arithmetic
// gives the forward result (double), the exact reverse-mode VJP (adouble),
// a forward-mode JVP (dual) and an operation count (cdouble).
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared (no fast-math).
#include "ms_oracle.hpp"
#include "ms_ad.hpp"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <type_traits>
#include <vector>

thread_local Tape* g_tape = nullptr;
thread_local uint64_t g_flops = 0;

namespace {

constexpr int ND = 16;
constexpr int SMX = 128;

// ------------------------------------------------------------ small algebra
template <class T> using V3 = std::array<T, 3>;
template <class T> using M3 = std::array<T, 9>;   // row-major
template <class T> using V6 = std::array<T, 6>;   // [angular; linear]
template <class T> using M6 = std::array<T, 36>;  // row-major

template <class T> V3<T> cv3(const double* p) { return {T(p[0]), T(p[1]), T(p[2])}; }
template <class T> V3<T> zero3() { return {T(0.0), T(0.0), T(0.0)}; }
template <class T> V3<T> add(const V3<T>& a, const V3<T>& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
template <class T> V3<T> sub(const V3<T>& a, const V3<T>& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
template <class T, class S> V3<T> scl(const V3<T>& a, const S& s) { return {a[0] * s, a[1] * s, a[2] * s}; }
template <class T> T dot(const V3<T>& a, const V3<T>& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <class T> V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
template <class T> M3<T> ident3() {
  M3<T> r;
  for (int i = 0; i < 9; ++i) r[i] = T(i % 4 == 0 ? 1.0 : 0.0);
  return r;
}
template <class T> M3<T> cm3(const double* p) {
  M3<T> r;
  for (int i = 0; i < 9; ++i) r[i] = T(p[i]);
  return r;
}
template <class T> V3<T> mv(const M3<T>& R, const V3<T>& v) {
  return {R[0] * v[0] + R[1] * v[1] + R[2] * v[2], R[3] * v[0] + R[4] * v[1] + R[5] * v[2],
          R[6] * v[0] + R[7] * v[1] + R[8] * v[2]};
}
template <class T> V3<T> mtv(const M3<T>& R, const V3<T>& v) {  // R^T v
  return {R[0] * v[0] + R[3] * v[1] + R[6] * v[2], R[1] * v[0] + R[4] * v[1] + R[7] * v[2],
          R[2] * v[0] + R[5] * v[1] + R[8] * v[2]};
}
template <class T> M3<T> mm(const M3<T>& A, const M3<T>& B) {
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i * 3 + j] = A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
  return C;
}
template <class T> M3<T> mmt(const M3<T>& A, const M3<T>& B) {  // A B^T
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] = A[i * 3] * B[j * 3] + A[i * 3 + 1] * B[j * 3 + 1] + A[i * 3 + 2] * B[j * 3 + 2];
  return C;
}

// rotation by angle th about unit axis k (Rodrigues): I + sin K + (1 - cos) K^2
template <class T> M3<T> rot_axis(const double* k, const T& th) {
  T s = Sin(th), c = Cos(th);
  T oc = 1.0 - c;
  double x = k[0], y = k[1], z = k[2];
  M3<T> R;
  R[0] = 1.0 + oc * (-(y * y + z * z));
  R[1] = -s * z + oc * (x * y);
  R[2] = s * y + oc * (x * z);
  R[3] = s * z + oc * (x * y);
  R[4] = 1.0 + oc * (-(x * x + z * z));
  R[5] = -s * x + oc * (y * z);
  R[6] = -s * y + oc * (x * z);
  R[7] = s * x + oc * (y * z);
  R[8] = 1.0 + oc * (-(x * x + y * y));
  return R;
}

template <class T> M3<T> quat_R(const std::array<T, 4>& q) {
  const T &w = q[0], &x = q[1], &y = q[2], &z = q[3];
  M3<T> R;
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
  return R;
}

void quat_R_d(const double* q, double* R) {
  std::array<double, 4> a{q[0], q[1], q[2], q[3]};
  M3<double> r = quat_R<double>(a);
  for (int i = 0; i < 9; ++i) R[i] = r[i];
}

// spatial algebra in world coordinates (Featherstone 2008, ch. 2)
template <class T> V6<T> zero6() {
  V6<T> r;
  for (auto& x : r) x = T(0.0);
  return r;
}
template <class T> V6<T> add6(const V6<T>& a, const V6<T>& b) {
  V6<T> r;
  for (int i = 0; i < 6; ++i) r[i] = a[i] + b[i];
  return r;
}
template <class T, class S> V6<T> scl6(const V6<T>& a, const S& s) {
  V6<T> r;
  for (int i = 0; i < 6; ++i) r[i] = a[i] * s;
  return r;
}
template <class T> T dot6(const V6<T>& a, const V6<T>& b) {
  T r = a[0] * b[0];
  for (int i = 1; i < 6; ++i) r = r + a[i] * b[i];
  return r;
}
template <class T> V6<T> mul6(const M6<T>& I, const V6<T>& v) {
  V6<T> r;
  for (int i = 0; i < 6; ++i) {
    T a = I[i * 6] * v[0];
    for (int j = 1; j < 6; ++j) a = a + I[i * 6 + j] * v[j];
    r[i] = a;
  }
  return r;
}
// motion cross product v x m
template <class T> V6<T> crm(const V6<T>& v, const V6<T>& m) {
  V3<T> w{v[0], v[1], v[2]}, vo{v[3], v[4], v[5]}, mw{m[0], m[1], m[2]}, mvv{m[3], m[4], m[5]};
  V3<T> a = cross(w, mw), b = add(cross(w, mvv), cross(vo, mw));
  return {a[0], a[1], a[2], b[0], b[1], b[2]};
}
// force cross product v x* f
template <class T> V6<T> crf(const V6<T>& v, const V6<T>& f) {
  V3<T> w{v[0], v[1], v[2]}, vo{v[3], v[4], v[5]}, n{f[0], f[1], f[2]}, fl{f[3], f[4], f[5]};
  V3<T> a = add(cross(w, n), cross(vo, fl)), b = cross(w, fl);
  return {a[0], a[1], a[2], b[0], b[1], b[2]};
}
// spatial inertia about the world origin of a body of mass m, COM c and
// rotational inertia Ic (about the COM, world axes)
template <class T> M6<T> spatial_inertia(double m, const V3<T>& c, const M3<T>& Ic) {
  M6<T> I;
  T cc = dot(c, c);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T v = Ic[i * 3 + j] - m * (c[i] * c[j]);
      if (i == j) v = v + m * cc;
      I[i * 6 + j] = v;
    }
  // m [c]x (top right) and its transpose (bottom left)
  T cx[9] = {T(0.0), -c[2], c[1], c[2], T(0.0), -c[0], -c[1], c[0], T(0.0)};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      I[i * 6 + 3 + j] = m * cx[i * 3 + j];
      I[(3 + i) * 6 + j] = m * cx[j * 3 + i];
      I[(3 + i) * 6 + 3 + j] = T(i == j ? m : 0.0);
    }
  return I;
}

// ------------------------------------------------------------- model data
struct ArtModel {
  int nb = 0;
  int parent[ND], jtype[ND], veldof[ND];
  double axis[ND][3], xtR[ND][9], xtp[ND][3], mass[ND], com[ND][3], Ic[ND][9], kp[ND], kd[ND];
  double armature[ND], damping[ND];
  int act_kind[ND];
  double act_scale[ND];
};

void load_robot(const or_scene* sc, int m, ArtModel& a) {
  a.nb = sc->model_nb[m];
  for (int i = 0; i < ND; ++i) {
    int k = m * ND + i;
    a.parent[i] = sc->model_parent[k];
    a.jtype[i] = sc->model_jtype[k];
    a.veldof[i] = sc->model_veldof[k];
    double qr[4];
    for (int t = 0; t < 4; ++t) qr[t] = sc->model_xt_rot[k * 4 + t];
    quat_R_d(qr, a.xtR[i]);
    for (int t = 0; t < 3; ++t) {
      a.axis[i][t] = sc->model_axis[k * 3 + t];
      a.xtp[i][t] = sc->model_xt_pos[k * 3 + t];
      a.com[i][t] = sc->model_com[k * 3 + t];
    }
    a.mass[i] = sc->model_mass[k];
    const float* in = sc->model_inertia + k * 6;  // xx yy zz xy xz yz
    double I[9] = {in[0], in[3], in[4], in[3], in[1], in[5], in[4], in[5], in[2]};
    for (int t = 0; t < 9; ++t) a.Ic[i][t] = I[t];
    a.kp[i] = sc->model_kp[k];
    a.kd[i] = sc->model_kd[k];
    a.armature[i] = sc->model_armature[k];
    a.damping[i] = sc->model_damping[k];
    a.act_kind[i] = sc->model_act_kind ? sc->model_act_kind[k] : 0;
    a.act_scale[i] = sc->model_act_scale ? sc->model_act_scale[k] : 0.0;
  }
}

void load_aux(const or_scene* sc, int x, ArtModel& a, double box[6], double lim[2]) {
  a.nb = 1;
  a.parent[0] = -1;
  a.jtype[0] = sc->aux_type[x];
  a.veldof[0] = 0;
  double qr[4];
  for (int t = 0; t < 4; ++t) qr[t] = sc->aux_rot[x * 4 + t];
  quat_R_d(qr, a.xtR[0]);
  for (int t = 0; t < 3; ++t) {
    a.axis[0][t] = sc->aux_axis[x * 3 + t];
    a.xtp[0][t] = sc->aux_pos[x * 3 + t];
    a.com[0][t] = sc->aux_box[x * 6 + t];
  }
  a.mass[0] = sc->aux_mass[x];
  for (int t = 0; t < 9; ++t) a.Ic[0][t] = 0.0;
  a.Ic[0][0] = sc->aux_inertia[x * 3 + 0];
  a.Ic[0][4] = sc->aux_inertia[x * 3 + 1];
  a.Ic[0][8] = sc->aux_inertia[x * 3 + 2];
  a.kp[0] = 0.0;
  a.kd[0] = 0.0;
  a.armature[0] = 0.0;
  a.damping[0] = 0.0;
  a.act_kind[0] = 0;
  a.act_scale[0] = 0.0;
  for (int t = 0; t < 6; ++t) box[t] = sc->aux_box[x * 6 + t];
  lim[0] = sc->aux_limit[x * 2 + 0];
  lim[1] = sc->aux_limit[x * 2 + 1];
}

// --------------------------------------------------------------- kinematics
template <class T> struct Kin {
  M3<T> R[ND];   // body rotation (world from body)
  V3<T> p[ND];   // body origin
  V3<T> a[ND];   // joint axis (world)
  V3<T> o[ND];   // joint origin (world)
  V6<T> s[ND];   // motion subspace (world)
  M6<T> I[ND];   // spatial inertia (world origin)
};

// Forward kinematics: X_i = X_parent * X_T(i) * X_J(q_i), in topological order.
template <class T> void fk(const ArtModel& m, const T* q, Kin<T>& k, bool inertia) {
  for (int i = 0; i < m.nb; ++i) {
    int par = m.parent[i];
    M3<T> Rj;
    V3<T> o;
    if (par < 0) {
      Rj = cm3<T>(m.xtR[i]);
      o = cv3<T>(m.xtp[i]);
    } else {
      Rj = mm(k.R[par], cm3<T>(m.xtR[i]));
      o = add(k.p[par], mv(k.R[par], cv3<T>(m.xtp[i])));
    }
    V3<T> a = mv(Rj, cv3<T>(m.axis[i]));
    k.a[i] = a;
    k.o[i] = o;
    if (m.jtype[i] == 0) {
      k.R[i] = mm(Rj, rot_axis<T>(m.axis[i], q[i]));
      k.p[i] = o;
      V3<T> oa = cross(o, a);
      k.s[i] = {a[0], a[1], a[2], oa[0], oa[1], oa[2]};
    } else {
      k.R[i] = Rj;
      k.p[i] = add(o, scl(a, q[i]));
      k.s[i] = {T(0.0), T(0.0), T(0.0), a[0], a[1], a[2]};
    }
    if (inertia) {
      V3<T> c = add(mv(k.R[i], cv3<T>(m.com[i])), k.p[i]);
      M3<T> Icw = mmt(mm(k.R[i], cm3<T>(m.Ic[i])), k.R[i]);
      k.I[i] = spatial_inertia<T>(m.mass[i], c, Icw);
    }
  }
}

// Composite-rigid-body algorithm: M_ij = s_i . (I^c_i s_j) for j an ancestor of i.
template <class T> void crba(const ArtModel& m, const Kin<T>& k, T* M) {
  M6<T> Ic[ND];
  for (int i = 0; i < m.nb; ++i) Ic[i] = k.I[i];
  for (int i = m.nb - 1; i >= 0; --i) {
    int par = m.parent[i];
    if (par >= 0)
      for (int t = 0; t < 36; ++t) Ic[par][t] = Ic[par][t] + Ic[i][t];
  }
  for (int i = 0; i < ND * ND; ++i) M[i] = T(0.0);
  for (int i = 0; i < m.nb; ++i) {
    V6<T> F = mul6(Ic[i], k.s[i]);
    M[i * ND + i] = dot6(k.s[i], F);
    for (int j = m.parent[i]; j >= 0; j = m.parent[j]) {
      T v = dot6(k.s[j], F);
      M[i * ND + j] = v;
      M[j * ND + i] = v;
    }
  }
}

// Recursive Newton-Euler inverse dynamics in world coordinates, gravity as a
// fictitious base acceleration -g.  qdd may be null (zero).
template <class T> void rnea(const ArtModel& m, const Kin<T>& k, const T* qd, const T* qdd, const double* g,
                             T* tau) {
  V6<T> v[ND], a[ND], f[ND];
  V6<T> a0 = {T(0.0), T(0.0), T(0.0), T(-g[0]), T(-g[1]), T(-g[2])};
  for (int i = 0; i < m.nb; ++i) {
    int par = m.parent[i];
    V6<T> vJ = scl6(k.s[i], qd[i]);
    v[i] = par < 0 ? vJ : add6(v[par], vJ);
    V6<T> ai = add6(par < 0 ? a0 : a[par], crm(v[i], vJ));
    if (qdd) ai = add6(ai, scl6(k.s[i], qdd[i]));
    a[i] = ai;
    f[i] = add6(mul6(k.I[i], a[i]), crf(v[i], mul6(k.I[i], v[i])));
  }
  for (int i = m.nb - 1; i >= 0; --i) {
    tau[i] = dot6(k.s[i], f[i]);
    int par = m.parent[i];
    if (par >= 0) f[par] = add6(f[par], f[i]);
  }
}

// In-place Cholesky factorisation A = L L^T (row-major, stride ND), lower part.
template <class T> bool cholesky(T* A, int n) {
  for (int j = 0; j < n; ++j) {
    T d = A[j * ND + j];
    for (int k = 0; k < j; ++k) d = d - A[j * ND + k] * A[j * ND + k];
    if (!(val(d) > 0.0)) return false;
    T l = Sqrt(d);
    A[j * ND + j] = l;
    for (int i = j + 1; i < n; ++i) {
      T s = A[i * ND + j];
      for (int k = 0; k < j; ++k) s = s - A[i * ND + k] * A[j * ND + k];
      A[i * ND + j] = s / l;
    }
  }
  return true;
}
template <class T> void chol_solve(const T* L, int n, T* b) {
  for (int i = 0; i < n; ++i) {
    T s = b[i];
    for (int k = 0; k < i; ++k) s = s - L[i * ND + k] * b[k];
    b[i] = s / L[i * ND + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    T s = b[i];
    for (int k = i + 1; k < n; ++k) s = s - L[k * ND + i] * b[k];
    b[i] = s / L[i * ND + i];
  }
}

// --------------------------------------------------------------- geometry
// Signed distance of a sphere (c, r) to a plane n.x = d; normal n; point c - r n.
template <class U> U g_plane(const V3<U>& c, double r, const double* pl, V3<U>& n, V3<U>& p) {
  n = {U(pl[0]), U(pl[1]), U(pl[2])};
  U phi = dot(n, c) - pl[3] - r;
  p = sub(c, scl(n, U(r)));
  return phi;
}
// Sphere vs box (centre bc, world-from-box rotation R, half extents e).
template <class U> U g_box(const V3<U>& c, double r, const V3<U>& bc, const M3<U>& R, const double* e, V3<U>& n,
                           V3<U>& p) {
  V3<U> y = mtv(R, sub(c, bc));
  bool outside = false;
  for (int i = 0; i < 3; ++i)
    if (std::fabs(val(y[i])) > e[i]) outside = true;
  U phi;
  V3<U> nl;
  if (outside) {
    V3<U> k;
    for (int i = 0; i < 3; ++i) {
      double yi = val(y[i]);
      k[i] = yi > e[i] ? U(e[i]) : (yi < -e[i] ? U(-e[i]) : y[i]);
    }
    V3<U> d = sub(y, k);
    U dist = Sqrt(dot(d, d));
    phi = dist - r;
    nl = scl(d, 1.0 / dist);
    if (!(val(dist) > 0.0)) nl = {U(0.0), U(0.0), U(1.0)};
  } else {
    int best = 0;
    double bestv = e[0] - std::fabs(val(y[0]));
    for (int i = 1; i < 3; ++i) {
      double v = e[i] - std::fabs(val(y[i]));
      if (v < bestv) { bestv = v; best = i; }
    }
    bool pos = val(y[best]) >= 0.0;
    U depth = pos ? U(e[best]) - y[best] : U(e[best]) + y[best];
    phi = -depth - r;
    nl = zero3<U>();
    nl[best] = U(pos ? 1.0 : -1.0);
  }
  n = mv(R, nl);
  p = sub(c, scl(n, U(r)));
  return phi;
}
template <class U> U g_sphere(const V3<U>& ca, double ra, const V3<U>& cb, double rb, V3<U>& n, V3<U>& p) {
  V3<U> d = sub(ca, cb);
  U dist = Sqrt(dot(d, d));
  U phi = dist - ra - rb;
  if (val(dist) < 1e-12)
    n = {U(0.0), U(0.0), U(1.0)};
  else
    n = scl(d, 1.0 / dist);
  p = sub(ca, scl(n, U(ra)));
  return phi;
}

// Orthonormal basis completing n (Duff et al. 2017, "Building an Orthonormal
// Basis, Revisited", JCGT 6(1)).
template <class U> void onb(const V3<U>& n, V3<U>& t1, V3<U>& t2) {
  double sg = std::copysign(1.0, val(n[2]));
  U a = -1.0 / (sg + n[2]);
  U b = n[0] * n[1] * a;
  t1 = {1.0 + sg * n[0] * n[0] * a, sg * b, -sg * n[0]};
  t2 = {b, sg + n[1] * n[1] * a, -n[1]};
}

uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ------------------------------------------------------------------ scenes
struct FreeC {
  int type;
  double half[3];
  double mass, Ib[3];
};
struct Sphere {
  int body, flags;
  double c[3], r;
};
struct SceneC {
  const ArtModel* robot;
  int robot_model;
  std::vector<Sphere> sph;
  std::vector<FreeC> fr;
  std::vector<std::array<double, 6>> boxes;
  std::vector<std::array<double, 4>> planes;
  std::vector<ArtModel> aux;
  std::vector<std::array<double, 6>> aux_box;
  std::vector<std::array<double, 2>> aux_lim;
  double hold[ND];
  int f0;  // global index of the scene's first free body
  int a0;  // global index of the scene's first door / drawer joint
  int nf_all;  // free bodies in the batch (rows of the gripper output before the joints)
};

void load_scene(const or_scene* sc, const std::vector<ArtModel>& robots, int s, SceneC& c) {
  int m = sc->scene_model[s];
  c.robot_model = m;
  c.robot = &robots[m];
  c.sph.clear();
  for (int k = 0; k < sc->model_nsph[m]; ++k) {
    Sphere sp;
    sp.body = sc->model_sph_body[m * SMX + k];
    sp.flags = sc->model_sph_flags[m * SMX + k];
    for (int t = 0; t < 3; ++t) sp.c[t] = sc->model_sph[(m * SMX + k) * 4 + t];
    sp.r = sc->model_sph[(m * SMX + k) * 4 + 3];
    c.sph.push_back(sp);
  }
  c.fr.clear();
  for (int f = sc->free_off[s]; f < sc->free_off[s + 1]; ++f) {
    FreeC fc;
    fc.type = sc->free_type[f];
    for (int t = 0; t < 3; ++t) {
      fc.half[t] = sc->free_size[f * 3 + t];
      fc.Ib[t] = sc->free_inertia[f * 3 + t];
    }
    fc.mass = sc->free_mass[f];
    c.fr.push_back(fc);
  }
  c.boxes.clear();
  for (int b = sc->static_off[s]; b < sc->static_off[s + 1]; ++b) {
    std::array<double, 6> x;
    for (int t = 0; t < 6; ++t) x[t] = sc->static_box[b * 6 + t];
    c.boxes.push_back(x);
  }
  c.planes.clear();
  for (int p = sc->plane_off[s]; p < sc->plane_off[s + 1]; ++p) {
    std::array<double, 4> x;
    for (int t = 0; t < 4; ++t) x[t] = sc->plane[p * 4 + t];
    c.planes.push_back(x);
  }
  int na = sc->aux_off[s + 1] - sc->aux_off[s];
  c.aux.resize(na);
  c.aux_box.resize(na);
  c.aux_lim.resize(na);
  for (int x = 0; x < na; ++x) load_aux(sc, sc->aux_off[s] + x, c.aux[x], c.aux_box[x].data(), c.aux_lim[x].data());
  for (int j = 0; j < ND; ++j) c.hold[j] = sc->scene_hold[s * ND + j];
  c.f0 = sc->free_off[s];
  c.a0 = sc->aux_off[s];
  c.nf_all = sc->free_off[sc->n_scenes];
}

template <class T> struct FreeS {
  V3<T> x;
  std::array<T, 4> Q;
  V3<T> v, w;
};
template <class T> struct StateS {
  T q[ND], qd[ND];
  std::vector<FreeS<T>> fr;
  std::vector<T> aq, aqd;
};

// a side of a contact: kind 0 static, 1 articulation (art 0 robot, 1+x aux), 2 free body
struct Side {
  int kind, art, body;
};
template <class T> struct Contact {
  Side A, B;
  T phi;
  V3<T> n, p;
  uint64_t key;
  bool robot_owner;
};
// per-direction row data of one side
template <class T> struct RowSide {
  T J[ND], w[ND];       // articulation: signed Jacobian row and M~^-1 J^T
  V3<T> lin, ang;       // free: signed linear / angular Jacobian
  V3<T> ilin, iang;     // free: M^-1 J^T
};
template <class T> struct Rows {
  V3<T> d[3];
  RowSide<T> side[2][3];
  T W[3];
  T bias;
  bool ok[3];
};

template <class T> struct Work {
  Kin<T> rk;
  std::vector<Kin<T>> ak;
  T L[ND * ND];                    // Cholesky factor of the robot's M~
  std::vector<std::array<T, 1>> aM;  // aux M~ (1x1)
  std::vector<M3<T>> fR, fIinv;
  std::vector<V3<T>> sphw;
};

template <class T> int art_ndof(const SceneC& c, int art) { return art == 0 ? c.robot->nb : 1; }

// Point-velocity Jacobian row d . dp/dq for a point p attached to `body`.
template <class T> void art_row(const ArtModel& m, const Kin<T>& k, int body, const V3<T>& p, const V3<T>& d,
                                double sgn, T* J) {
  for (int j = 0; j < ND; ++j) J[j] = T(0.0);
  for (int j = body; j >= 0; j = m.parent[j]) {
    T v = m.jtype[j] == 0 ? dot(d, cross(k.a[j], sub(p, k.o[j]))) : dot(d, k.a[j]);
    J[j] = v * sgn;
  }
}

template <class P> struct TestScalarT { using type = double; };

// Operation count of one emit decision (the signed distance alone), charged
// to the counting scalar in place of the decision's own evaluation, which
// also forms n and p and, for an axis-aligned box, multiplies by an identity
// rotation:  plane n.c - d - r: 7;  axis-aligned box c - m, clamp, |c - y| - r
// (inside: e - |c|): 13;  oriented box R^T (c - x) then as an axis-aligned
// box: 28;  sphere |c_A - c_B| - r_A - r_B: 11.
enum { COST_PLANE = 7, COST_AABB = 13, COST_OBB = 28, COST_SPHERE = 11 };
template <class T> void count_decision(int n) {
  if constexpr (std::is_same<T, cdouble>::value) g_flops += (uint64_t)n;
}

// One substep of one scene (see the header for the sequence of steps).
template <class T> void substep(const SceneC& c, const or_params& pr, StateS<T>& st, const T* u, int isub,
                                uint32_t& status, or_debug* dbg, int s, int n_sub) {
  using P = typename TestScalarT<T>::type;
  const ArtModel& rm = *c.robot;
  const int nb = rm.nb;
  const double h = pr.h;
  const int NF = (int)c.fr.size(), NA = (int)c.aux.size();
  Work<T> wk;

  // 1. drive -------------------------------------------------------------
  T tau[ND], arm[ND];
  for (int j = 0; j < ND; ++j) { tau[j] = T(0.0); arm[j] = T(0.0); }
  for (int j = 0; j < nb; ++j) {
    // implicit viscous damping: -damping * qd(t+h) moves h*damping to the left-hand side
    const double dmp = rm.damping[j];
    if (pr.control_mode == 0) {
      tau[j] = u[j] - dmp * st.qd[j];
      arm[j] = T(rm.armature[j] + h * dmp);
    } else {
      double kp = rm.kp[j], kd = rm.kd[j];
      T qt, vt, ff = T(0.0);
      if (pr.control_mode == 1) {
        qt = rm.veldof[j] ? T(0.0) : u[j];
        vt = rm.veldof[j] ? u[j] : T(0.0);
      } else {
        qt = T(rm.veldof[j] ? 0.0 : c.hold[j]);
        vt = T(rm.veldof[j] ? c.hold[j] : 0.0);
        ff = u[j];
      }
      if (rm.veldof[j]) kp = 0.0;
      // implicit PD: tau_PD evaluated at t+h with q(t+h) = q + h qd(t+h)
      tau[j] = ff + kp * (qt - st.q[j] - h * st.qd[j]) + kd * (vt - st.qd[j]) - dmp * st.qd[j];
      arm[j] = T(rm.armature[j] + h * (kd + dmp) + h * h * kp);
    }
  }

  // 2. kinematics -------------------------------------------------------
  fk(rm, st.q, wk.rk, true);
  wk.sphw.resize(c.sph.size());
  for (size_t k = 0; k < c.sph.size(); ++k) {
    const Sphere& sp = c.sph[k];
    wk.sphw[k] = add(mv(wk.rk.R[sp.body], cv3<T>(sp.c)), wk.rk.p[sp.body]);
  }
  wk.ak.resize(NA);
  for (int x = 0; x < NA; ++x) {
    T qx[1] = {st.aq[x]};
    fk(c.aux[x], qx, wk.ak[x], true);
  }
  wk.fR.resize(NF);
  wk.fIinv.resize(NF);
  for (int f = 0; f < NF; ++f) {
    wk.fR[f] = quat_R(st.fr[f].Q);
    M3<T> Dinv = cm3<T>(std::array<double, 9>{1.0 / c.fr[f].Ib[0], 0, 0, 0, 1.0 / c.fr[f].Ib[1], 0, 0, 0,
                                               1.0 / c.fr[f].Ib[2]}.data());
    wk.fIinv[f] = mmt(mm(wk.fR[f], Dinv), wk.fR[f]);
  }

  // 3. contacts (canonical order: owner class, owner index, target class, target index)
  std::vector<Contact<T>> con;
  bool overflow = false, robot_overflow = false;
  int n_robot = 0;
  const double margin = pr.margin;
  // caps: a robot-owned contact beyond robot_contact_cap is dropped first;
  // then any contact beyond contact_cap (both keep the canonical-order prefix)
  auto emit = [&](const Contact<T>& ct) {
    if (ct.robot_owner && n_robot >= pr.robot_contact_cap) {
      robot_overflow = true;
      return;
    }
    if ((int)con.size() < pr.contact_cap) {
      con.push_back(ct);
      if (ct.robot_owner) ++n_robot;
    } else {
      overflow = true;
    }
  };
  auto aux_obb = [&](int x, V3<T>& bc, M3<T>& R) {
    const Kin<T>& k = wk.ak[x];
    R = k.R[0];
    bc = add(mv(k.R[0], cv3<T>(c.aux_box[x].data())), k.p[0]);
  };
  auto val3 = [](const V3<T>& a) { return V3<P>{P(val(a[0])), P(val(a[1])), P(val(a[2]))}; };
  auto valM = [](const M3<T>& a) {
    M3<P> r;
    for (int i = 0; i < 9; ++i) r[i] = P(val(a[i]));
    return r;
  };
  // test one owner point against every allowed target
  auto owner_targets = [&](const V3<T>& cw, double r, Side A, uint64_t okey, bool skip_floor, int self_free,
                           bool is_vertex, bool is_sphere_owner, bool robot_owner) {
    V3<P> cp = val3(cw);
    V3<P> nP, pP;
    for (int pl = 0; pl < (int)c.planes.size(); ++pl) {
      if (pl == 0 && skip_floor) continue;
      count_decision<T>(COST_PLANE);
      P phi = g_plane<P>(cp, r, c.planes[pl].data(), nP, pP);
      if (val(phi) < margin) {
        Contact<T> ct;
        ct.A = A; ct.B = {0, -1, -1};
        ct.phi = g_plane<T>(cw, r, c.planes[pl].data(), ct.n, ct.p);
        ct.key = (okey << 32) | (uint64_t)((0u << 24) | (uint32_t)pl);
        ct.robot_owner = robot_owner;
        emit(ct);
      }
    }
    static const M3<double> I3 = ident3<double>();
    for (int b = 0; b < (int)c.boxes.size(); ++b) {
      const auto& bx = c.boxes[b];
      V3<P> bc{P(bx[0]), P(bx[1]), P(bx[2])};
      M3<P> RI;
      for (int i = 0; i < 9; ++i) RI[i] = P(I3[i]);
      count_decision<T>(COST_AABB);
      P phi = g_box<P>(cp, r, bc, RI, &bx[3], nP, pP);
      if (val(phi) < margin) {
        Contact<T> ct;
        ct.A = A; ct.B = {0, -1, -1};
        M3<T> RT = ident3<T>();
        ct.phi = g_box<T>(cw, r, cv3<T>(bx.data()), RT, &bx[3], ct.n, ct.p);
        ct.key = (okey << 32) | (uint64_t)((1u << 24) | (uint32_t)b);
        ct.robot_owner = robot_owner;
        emit(ct);
      }
    }
    for (int x = 0; x < NA; ++x) {
      V3<T> bc; M3<T> R;
      aux_obb(x, bc, R);
      count_decision<T>(COST_OBB);
      P phi = g_box<P>(cp, r, val3(bc), valM(R), &c.aux_box[x][3], nP, pP);
      if (val(phi) < margin) {
        Contact<T> ct;
        ct.A = A; ct.B = {1, 1 + x, 0};
        ct.phi = g_box<T>(cw, r, bc, R, &c.aux_box[x][3], ct.n, ct.p);
        ct.key = (okey << 32) | (uint64_t)((2u << 24) | (uint32_t)x);
        ct.robot_owner = robot_owner;
        emit(ct);
      }
    }
    for (int g = 0; g < NF; ++g) {
      if (g == self_free) continue;
      const FreeC& fg = c.fr[g];
      P phi;
      if (fg.type == 0) {
        count_decision<T>(COST_OBB);
        phi = g_box<P>(cp, r, val3(st.fr[g].x), valM(wk.fR[g]), fg.half, nP, pP);
      } else {
        if (is_vertex) continue;                      // box vertices do not test free spheres
        if (is_sphere_owner && g <= self_free) continue;  // sphere pairs counted once
        count_decision<T>(COST_SPHERE);
        phi = g_sphere<P>(cp, r, val3(st.fr[g].x), fg.half[0], nP, pP);
      }
      if (val(phi) < margin) {
        Contact<T> ct;
        ct.A = A; ct.B = {2, -1, g};
        if (fg.type == 0)
          ct.phi = g_box<T>(cw, r, st.fr[g].x, wk.fR[g], fg.half, ct.n, ct.p);
        else
          ct.phi = g_sphere<T>(cw, r, st.fr[g].x, fg.half[0], ct.n, ct.p);
        ct.key = (okey << 32) | (uint64_t)((3u << 24) | (uint32_t)g);
        ct.robot_owner = robot_owner;
        emit(ct);
      }
    }
  };
  for (size_t k = 0; k < c.sph.size(); ++k) {
    const Sphere& sp = c.sph[k];
    owner_targets(wk.sphw[k], sp.r, Side{1, 0, sp.body}, (uint64_t)k, (sp.flags & 1) != 0, -1, false, false, true);
  }
  for (int f = 0; f < NF; ++f) {
    const FreeC& fc = c.fr[f];
    uint64_t ok = (1ull << 24) | ((uint64_t)f << 3);
    if (fc.type == 0) {
      for (int v = 0; v < 8; ++v) {
        V3<double> loc{(v & 1) ? fc.half[0] : -fc.half[0], (v & 2) ? fc.half[1] : -fc.half[1],
                       (v & 4) ? fc.half[2] : -fc.half[2]};
        V3<T> cw = add(st.fr[f].x, mv(wk.fR[f], cv3<T>(loc.data())));
        owner_targets(cw, 0.0, Side{2, -1, f}, ok | (uint64_t)v, false, f, true, false, false);
      }
    } else {
      owner_targets(st.fr[f].x, fc.half[0], Side{2, -1, f}, ok, false, f, false, true, false);
    }
  }
  if (overflow) status |= 2u;
  if (robot_overflow) status |= 8u;

  // 4. unconstrained velocities ------------------------------------------
  T vR[ND];
  {
    T M[ND * ND], C[ND];
    crba(rm, wk.rk, M);
    rnea(rm, wk.rk, st.qd, (const T*)nullptr, pr.gravity, C);
    for (int j = 0; j < nb; ++j) M[j * ND + j] = M[j * ND + j] + arm[j];
    for (int i = 0; i < ND * ND; ++i) wk.L[i] = M[i];
    if (!cholesky(wk.L, nb)) status |= 4u;
    T rhs[ND];
    for (int j = 0; j < nb; ++j) rhs[j] = tau[j] - C[j];
    chol_solve(wk.L, nb, rhs);
    for (int j = 0; j < ND; ++j) vR[j] = j < nb ? st.qd[j] + h * rhs[j] : st.qd[j];
  }
  std::vector<T> vA(NA);
  wk.aM.resize(NA);
  for (int x = 0; x < NA; ++x) {
    T M[ND * ND], C[ND];
    T qdx[1] = {st.aqd[x]};
    crba(c.aux[x], wk.ak[x], M);
    rnea(c.aux[x], wk.ak[x], qdx, (const T*)nullptr, pr.gravity, C);
    wk.aM[x][0] = M[0];
    vA[x] = st.aqd[x] + h * ((T(0.0) - C[0]) / M[0]);
  }
  std::vector<V3<T>> vF(NF), wF(NF);
  for (int f = 0; f < NF; ++f) {
    const FreeS<T>& fs = st.fr[f];
    vF[f] = add(fs.v, scl(cv3<T>(pr.gravity), T(h)));
    M3<T> D = cm3<T>(std::array<double, 9>{c.fr[f].Ib[0], 0, 0, 0, c.fr[f].Ib[1], 0, 0, 0, c.fr[f].Ib[2]}.data());
    M3<T> Iw = mmt(mm(wk.fR[f], D), wk.fR[f]);
    V3<T> gyro = cross(fs.w, mv(Iw, fs.w));
    wF[f] = sub(fs.w, scl(mv(wk.fIinv[f], gyro), T(h)));
  }

  // 5. rows ----------------------------------------------------------------
  const int NC = (int)con.size();
  std::vector<Rows<T>> rows(NC);
  auto art_solve = [&](int art, T* b) {
    if (art == 0) chol_solve(wk.L, nb, b);
    else b[0] = b[0] / wk.aM[art - 1][0];
  };
  for (int ci = 0; ci < NC; ++ci) {
    const Contact<T>& ct = con[ci];
    Rows<T>& rw = rows[ci];
    rw.d[0] = ct.n;
    onb(ct.n, rw.d[1], rw.d[2]);
    for (int di = 0; di < 3; ++di) {
      T W = T(0.0);
      for (int sd = 0; sd < 2; ++sd) {
        const Side& S = sd == 0 ? ct.A : ct.B;
        double sgn = sd == 0 ? 1.0 : -1.0;
        RowSide<T>& r = rw.side[sd][di];
        if (S.kind == 1) {
          const ArtModel& am = S.art == 0 ? rm : c.aux[S.art - 1];
          const Kin<T>& kk = S.art == 0 ? wk.rk : wk.ak[S.art - 1];
          art_row(am, kk, S.body, ct.p, rw.d[di], sgn, r.J);
          for (int j = 0; j < ND; ++j) r.w[j] = r.J[j];
          art_solve(S.art, r.w);
          int n = S.art == 0 ? nb : 1;
          for (int j = 0; j < n; ++j) W = W + r.J[j] * r.w[j];
        } else if (S.kind == 2) {
          V3<T> rr = sub(ct.p, st.fr[S.body].x);
          r.lin = scl(rw.d[di], T(sgn));
          r.ang = scl(cross(rr, rw.d[di]), T(sgn));
          r.ilin = scl(r.lin, T(1.0 / c.fr[S.body].mass));
          r.iang = mv(wk.fIinv[S.body], r.ang);
          W = W + dot(r.lin, r.ilin) + dot(r.ang, r.iang);
        }
      }
      rw.W[di] = W;
      rw.ok[di] = val(W) >= 1e-12;
      if (!rw.ok[di]) status |= 4u;
    }
    rw.bias = val(ct.phi) >= 0.0 ? ct.phi / h : pr.baumgarte * ct.phi / h;
  }
  // joint-limit rows of the auxiliary articulations (first in the order)
  struct Lim { int x; double sgn; T bias; T W; };  // W = J M~^-1 J^T = 1 / M~
  std::vector<Lim> lims;
  for (int x = 0; x < NA; ++x) {
    double lo = c.aux_lim[x][0], hi = c.aux_lim[x][1];
    if (lo > hi) continue;
    T glo = st.aq[x] - lo, ghi = hi - st.aq[x];
    T Wx = 1.0 / wk.aM[x][0];
    if (val(glo) < margin) lims.push_back({x, 1.0, val(glo) >= 0.0 ? glo / h : pr.baumgarte * glo / h, Wx});
    if (val(ghi) < margin) lims.push_back({x, -1.0, val(ghi) >= 0.0 ? ghi / h : pr.baumgarte * ghi / h, Wx});
  }

  // 6. projected Gauss-Seidel ------------------------------------------
  auto rowvel = [&](int ci, int di) {
    const Contact<T>& ct = con[ci];
    T r = T(0.0);
    for (int sd = 0; sd < 2; ++sd) {
      const Side& S = sd == 0 ? ct.A : ct.B;
      const RowSide<T>& rs = rows[ci].side[sd][di];
      if (S.kind == 1) {
        if (S.art == 0) {
          for (int j = 0; j < nb; ++j) r = r + rs.J[j] * vR[j];
        } else {
          r = r + rs.J[0] * vA[S.art - 1];
        }
      } else if (S.kind == 2) {
        r = r + dot(rs.lin, vF[S.body]) + dot(rs.ang, wF[S.body]);
      }
    }
    return r;
  };
  auto apply = [&](int ci, int di, const T& dl) {
    const Contact<T>& ct = con[ci];
    for (int sd = 0; sd < 2; ++sd) {
      const Side& S = sd == 0 ? ct.A : ct.B;
      const RowSide<T>& rs = rows[ci].side[sd][di];
      if (S.kind == 1) {
        if (S.art == 0) {
          for (int j = 0; j < nb; ++j) vR[j] = vR[j] + rs.w[j] * dl;
        } else {
          vA[S.art - 1] = vA[S.art - 1] + rs.w[0] * dl;
        }
      } else if (S.kind == 2) {
        vF[S.body] = add(vF[S.body], scl(rs.ilin, dl));
        wF[S.body] = add(wF[S.body], scl(rs.iang, dl));
      }
    }
  };
  std::vector<std::array<T, 3>> lam(NC, {T(0.0), T(0.0), T(0.0)});
  std::vector<T> llam(lims.size(), T(0.0));
  uint64_t act = 0x12345ull;
  // diagnostics: pre-projection values of the last substep's row updates
  auto tape_y = [&](int it, int row, int slot, const T& y) {
    if (!dbg || !dbg->dump_y || isub != n_sub - 1 || row >= dbg->dump_cap) return;
    dbg->dump_y[(((size_t)s * pr.pgs_iters + it) * dbg->dump_cap + row) * 3 + slot] = val(y);
  };
  const int NLm = (int)lims.size();
  for (int it = 0; it < pr.pgs_iters; ++it) {
    for (size_t li = 0; li < lims.size(); ++li) {
      Lim& L = lims[li];
      T r = L.sgn * vA[L.x] + L.bias;
      T y = llam[li] - r / L.W;
      tape_y(it, (int)li, 0, y);
      bool on = val(y) > 0.0;
      T nl = on ? y : T(0.0);
      T dl = nl - llam[li];
      vA[L.x] = vA[L.x] + (L.sgn * L.W) * dl;
      llam[li] = nl;
      act = mix64(act ^ (on ? 3u : 5u));
    }
    for (int ci = 0; ci < NC; ++ci) {
      Rows<T>& rw = rows[ci];
      if (rw.ok[0]) {
        T r = rowvel(ci, 0) + rw.bias;
        T y = lam[ci][0] - r / rw.W[0];
        tape_y(it, NLm + ci, 0, y);
        bool on = val(y) > 0.0;
        T nl = on ? y : T(0.0);
        T dl = nl - lam[ci][0];
        apply(ci, 0, dl);
        lam[ci][0] = nl;
        act = mix64(act ^ (on ? 7u : 11u));
      }
      if (rw.ok[1] && rw.ok[2]) {
        T r1 = rowvel(ci, 1), r2 = rowvel(ci, 2);
        T y1 = lam[ci][1] - r1 / rw.W[1];
        T y2 = lam[ci][2] - r2 / rw.W[2];
        tape_y(it, NLm + ci, 1, y1);
        tape_y(it, NLm + ci, 2, y2);
        T lim = pr.mu * lam[ci][0];
        T nn = y1 * y1 + y2 * y2;
        bool proj = val(nn) > val(lim) * val(lim);
        if (proj) {
          if (val(lim) > 0.0) {
            T sc = lim / Sqrt(nn);
            y1 = y1 * sc;
            y2 = y2 * sc;
          } else {
            y1 = T(0.0);
            y2 = T(0.0);
          }
        }
        T d1 = y1 - lam[ci][1], d2 = y2 - lam[ci][2];
        apply(ci, 1, d1);
        apply(ci, 2, d2);
        lam[ci][1] = y1;
        lam[ci][2] = y2;
        act = mix64(act ^ (proj ? 13u : 17u));
      }
    }
  }

  // 7. integrate -------------------------------------------------------------
  for (int j = 0; j < ND; ++j) {
    st.qd[j] = vR[j];
    if (j < nb) st.q[j] = st.q[j] + h * st.qd[j];
  }
  for (int x = 0; x < NA; ++x) {
    st.aqd[x] = vA[x];
    st.aq[x] = st.aq[x] + h * st.aqd[x];
  }
  for (int f = 0; f < NF; ++f) {
    FreeS<T>& fs = st.fr[f];
    fs.v = vF[f];
    fs.w = wF[f];
    fs.x = add(fs.x, scl(fs.v, T(h)));
    V3<T> th = scl(fs.w, T(h));
    T n2 = dot(th, th);
    T cw, sk;  // cos(|th|/2) and sin(|th|/2)/|th|
    if (val(n2) < 1e-12) {
      cw = 1.0 - n2 / 8.0;
      sk = 0.5 - n2 / 48.0;
    } else {
      T nn = Sqrt(n2);
      cw = Cos(nn / 2.0);
      sk = Sin(nn / 2.0) / nn;
    }
    std::array<T, 4> e{cw, th[0] * sk, th[1] * sk, th[2] * sk};
    const std::array<T, 4>& Q = fs.Q;
    std::array<T, 4> r;
    r[0] = e[0] * Q[0] - (e[1] * Q[1] + e[2] * Q[2] + e[3] * Q[3]);
    r[1] = e[0] * Q[1] + Q[0] * e[1] + (e[2] * Q[3] - e[3] * Q[2]);
    r[2] = e[0] * Q[2] + Q[0] * e[2] + (e[3] * Q[1] - e[1] * Q[3]);
    r[3] = e[0] * Q[3] + Q[0] * e[3] + (e[1] * Q[2] - e[2] * Q[1]);
    T nq = Sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    for (int t = 0; t < 4; ++t) fs.Q[t] = r[t] / nq;
  }

  // diagnostics
  if (dbg) {
    if (dbg->n_contacts) dbg->n_contacts[(size_t)s * n_sub + isub] = NC;
    if (dbg->key_hash) {
      uint64_t hsum = 0;
      for (auto& ct : con) hsum += mix64(ct.key);
      dbg->key_hash[(size_t)s * n_sub + isub] = hsum;
    }
    if (dbg->act_hash) dbg->act_hash[(size_t)s * n_sub + isub] = act;
    if (dbg->robot_force) {
      double fsum = 0.0;
      for (int ci = 0; ci < NC; ++ci)
        if (con[ci].robot_owner) fsum += std::fabs(val(lam[ci][0])) / h;
      dbg->robot_force[s] += fsum;
    }
    if (dbg->robot_body_force) {
      // the impulse on the owner A is sum_d d lambda_d; the target B receives its negative
      for (int ci = 0; ci < NC; ++ci) {
        const Contact<T>& ct = con[ci];
        if (!ct.robot_owner || ct.B.kind != 2) continue;
        double* F = dbg->robot_body_force + (size_t)(c.f0 + ct.B.body) * 3;
        for (int t = 0; t < 3; ++t) {
          double P = 0.0;
          for (int d = 0; d < 3; ++d) P += val(rows[ci].d[d][t]) * val(lam[ci][d]);
          F[t] -= P / h;
        }
      }
    }
    if (dbg->grip) {
      // gripper contacts per free body / door-drawer joint: the normal force
      // of the end effector's bodies (summed over the substeps) and, in the
      // last substep, the smaller of the two fingers' normal forces
      const int nobj = (int)c.fr.size() + (int)c.aux.size();
      for (int o = 0; o < nobj; ++o) {
        const bool isf = o < (int)c.fr.size();
        double fe = 0.0, fl = 0.0, fr = 0.0;
        for (int ci = 0; ci < NC; ++ci) {
          const Contact<T>& ct = con[ci];
          if (!ct.robot_owner) continue;
          const bool hit = isf ? (ct.B.kind == 2 && ct.B.body == o)
                               : (ct.B.kind == 1 && ct.B.art == 1 + (o - (int)c.fr.size()));
          if (!hit) continue;
          const double fn = val(lam[ci][0]) / h;
          const int body = ct.A.body;
          if ((dbg->grip_ee >> body) & 1u) fe += fn;
          if (body == dbg->grip_finger_l) fl += fn;
          if (body == dbg->grip_finger_r) fr += fn;
        }
        double* g = dbg->grip + 2 * (isf ? (size_t)(c.f0 + o) : (size_t)c.nf_all + c.a0 + (o - (int)c.fr.size()));
        g[0] += fe;
        if (isub == n_sub - 1) g[1] = std::min(fl, fr);
      }
    }
    if (isub == n_sub - 1 && dbg->dump_cap > 0) {
      for (int ci = 0; ci < dbg->dump_cap; ++ci) {
        size_t o = (size_t)s * dbg->dump_cap + ci;
        bool has = ci < NC;
        if (dbg->dump_keys) dbg->dump_keys[o] = has ? con[ci].key : ~0ull;
        if (dbg->dump_phi) dbg->dump_phi[o] = has ? val(con[ci].phi) : 0.0;
        if (dbg->dump_lambda)
          for (int t = 0; t < 3; ++t) dbg->dump_lambda[o * 3 + t] = has ? val(lam[ci][t]) : 0.0;
      }
    }
  }
}

// Normalized actions in [-1, 1] to PD targets, once per control step from the
// state at its start (the action space of Sec. 4.1: joint delta position for
// arm, torso and head, base linear and angular velocity, gripper opening).
template <class T> T clip_unit(const T& a) { return val(a) > 1.0 ? T(1.0) : (val(a) < -1.0 ? T(-1.0) : a); }
template <class T> void actions_to_targets(const ArtModel& m, const T* q, const T* a, T* tgt) {
  int jx = -1, jyaw = -1;
  for (int j = 0; j < m.nb; ++j) {
    if (m.act_kind[j] == 1) jx = j;
    if (m.act_kind[j] == 3) jyaw = j;
  }
  for (int j = 0; j < ND; ++j) tgt[j] = T(0.0);
  for (int j = 0; j < m.nb; ++j) {
    const double sc = m.act_scale[j];
    const T aj = clip_unit(a[j]);
    switch (m.act_kind[j]) {
      case 0: tgt[j] = q[j] + aj * sc; break;
      case 1: tgt[j] = jyaw >= 0 ? aj * sc * Cos(q[jyaw]) : aj * sc; break;
      case 2: {
        const T ax = jx >= 0 ? clip_unit(a[jx]) : T(0.0);
        tgt[j] = jyaw >= 0 ? ax * sc * Sin(q[jyaw]) : T(0.0);
        break;
      }
      case 3: tgt[j] = aj * sc; break;
      default: tgt[j] = (aj + 1.0) * 0.5 * sc; break;
    }
  }
}
// One control step of one scene: n_sub substeps under zero-order hold.
template <class T> void control_step(const SceneC& c, const or_params& pr, StateS<T>& st, const T* us,
                                     uint32_t& status, or_debug* dbg, int s) {
  const T* uu = us;
  T tgt[ND];
  or_params p = pr;
  if (pr.control_mode == 3) {
    actions_to_targets(*c.robot, st.q, us, tgt);
    uu = tgt;
    p.control_mode = 1;
  }
  for (int k = 0; k < pr.n_sub; ++k) substep<T>(c, p, st, uu, k, status, dbg, s, pr.n_sub);
}

// --------------------------------------------------------- state packing
struct Layout {
  int S, NF, NA;
  size_t q(int s) const { return (size_t)s * ND; }
  size_t qd(int s) const { return (size_t)S * ND + (size_t)s * ND; }
  size_t fr(int f) const { return (size_t)S * 2 * ND + (size_t)f * 16; }
  size_t ax(int x) const { return (size_t)S * 2 * ND + (size_t)NF * 16 + (size_t)x * 4; }
};

Layout layout_of(const or_scene* sc) {
  return Layout{sc->n_scenes, sc->free_off[sc->n_scenes], sc->aux_off[sc->n_scenes]};
}

// Gather scene s's state, with `mk` turning each double into a T.
template <class T, class F> void gather(const or_scene* sc, const Layout& L, int s, const double* x, StateS<T>& st,
                                        F mk) {
  for (int j = 0; j < ND; ++j) {
    st.q[j] = mk(L.q(s) + j, x[L.q(s) + j]);
    st.qd[j] = mk(L.qd(s) + j, x[L.qd(s) + j]);
  }
  int f0 = sc->free_off[s], nf = sc->free_off[s + 1] - f0;
  st.fr.resize(nf);
  for (int f = 0; f < nf; ++f) {
    size_t o = L.fr(f0 + f);
    for (int t = 0; t < 3; ++t) {
      st.fr[f].x[t] = mk(o + t, x[o + t]);
      st.fr[f].v[t] = mk(o + 8 + t, x[o + 8 + t]);
      st.fr[f].w[t] = mk(o + 12 + t, x[o + 12 + t]);
    }
    for (int t = 0; t < 4; ++t) st.fr[f].Q[t] = mk(o + 4 + t, x[o + 4 + t]);
  }
  int a0 = sc->aux_off[s], na = sc->aux_off[s + 1] - a0;
  st.aq.resize(na);
  st.aqd.resize(na);
  for (int a = 0; a < na; ++a) {
    size_t o = L.ax(a0 + a);
    st.aq[a] = mk(o, x[o]);
    st.aqd[a] = mk(o + 1, x[o + 1]);
  }
}

// Visit every state slot of scene s with (flat index, T value).
template <class T, class F> void scatter(const or_scene* sc, const Layout& L, int s, const StateS<T>& st, F put) {
  for (int j = 0; j < ND; ++j) {
    put(L.q(s) + j, st.q[j]);
    put(L.qd(s) + j, st.qd[j]);
  }
  int f0 = sc->free_off[s], nf = sc->free_off[s + 1] - f0;
  for (int f = 0; f < nf; ++f) {
    size_t o = L.fr(f0 + f);
    for (int t = 0; t < 3; ++t) {
      put(o + t, st.fr[f].x[t]);
      put(o + 8 + t, st.fr[f].v[t]);
      put(o + 12 + t, st.fr[f].w[t]);
    }
    for (int t = 0; t < 4; ++t) put(o + 4 + t, st.fr[f].Q[t]);
    put(o + 3, T(0.0));
    put(o + 11, T(0.0));
    put(o + 15, T(0.0));
  }
  int a0 = sc->aux_off[s], na = sc->aux_off[s + 1] - a0;
  for (int a = 0; a < na; ++a) {
    size_t o = L.ax(a0 + a);
    put(o, st.aq[a]);
    put(o + 1, st.aqd[a]);
    put(o + 2, T(0.0));
    put(o + 3, T(0.0));
  }
}

template <class F> void parallel_scenes(int S, int threads, F fn) {
  if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
  threads = std::min(threads, std::max(S, 1));
  std::atomic<int> next{0};
  auto worker = [&]() {
    for (;;) {
      int s = next.fetch_add(1);
      if (s >= S) break;
      fn(s);
    }
  };
  if (threads == 1) {
    worker();
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
}

std::vector<ArtModel> load_models(const or_scene* sc) {
  std::vector<ArtModel> r(sc->n_models);
  for (int m = 0; m < sc->n_models; ++m) load_robot(sc, m, r[m]);
  return r;
}

bool finite_state(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

}  // namespace

// =========================================================================
extern "C" {

int or_step(const or_scene* sc, const or_params* pr, const double* x_in, const double* u, double* x_out,
            int threads, or_debug* dbg) {
  if (!sc || !pr || !x_in || !u || !x_out) return -1;
  std::vector<ArtModel> robots = load_models(sc);
  Layout L = layout_of(sc);
  const int S = sc->n_scenes;
  if (dbg && dbg->robot_force)
    for (int s = 0; s < S; ++s) dbg->robot_force[s] = 0.0;
  if (dbg && dbg->robot_body_force)
    for (size_t i = 0; i < (size_t)L.NF * 3; ++i) dbg->robot_body_force[i] = 0.0;
  if (dbg && dbg->grip)
    for (size_t i = 0; i < 2 * ((size_t)L.NF + L.NA); ++i) dbg->grip[i] = 0.0;
  std::vector<double> xin(x_in, x_in + (size_t)S * 2 * ND + (size_t)L.NF * 16 + (size_t)L.NA * 4);
  parallel_scenes(S, threads, [&](int s) {
    SceneC c;
    load_scene(sc, robots, s, c);
    StateS<double> st;
    gather(sc, L, s, xin.data(), st, [](size_t, double v) { return v; });
    uint32_t status = 0;
    const double* us = u + (size_t)s * ND;
    control_step<double>(c, *pr, st, us, status, dbg, s);
    std::vector<double> vals;
    scatter(sc, L, s, st, [&](size_t i, double v) { x_out[i] = v; vals.push_back(v); });
    if (!finite_state(vals)) status |= 1u;
    if (dbg && dbg->status) dbg->status[s] = status;
  });
  return 0;
}

// The same step evaluated in IEEE single precision (every operation rounds to
// float, parameters and literals included; contact decisions as in or_step):
// an estimate of the error floor of any FP32 evaluation of the step.
int or_step_f32(const or_scene* sc, const or_params* pr, const double* x_in, const double* u, double* x_out,
                int threads, or_debug* dbg) {
  if (!sc || !pr || !x_in || !u || !x_out) return -1;
  std::vector<ArtModel> robots = load_models(sc);
  Layout L = layout_of(sc);
  const int S = sc->n_scenes;
  std::vector<double> xin(x_in, x_in + (size_t)S * 2 * ND + (size_t)L.NF * 16 + (size_t)L.NA * 4);
  parallel_scenes(S, threads, [&](int s) {
    SceneC c;
    load_scene(sc, robots, s, c);
    StateS<f32s> st;
    gather(sc, L, s, xin.data(), st, [](size_t, double v) { return f32s(v); });
    f32s us[ND];
    for (int j = 0; j < ND; ++j) us[j] = f32s(u[(size_t)s * ND + j]);
    uint32_t status = 0;
    control_step<f32s>(c, *pr, st, us, status, dbg, s);
    scatter(sc, L, s, st, [&](size_t i, const f32s& v) { x_out[i] = val(v); });
  });
  return 0;
}

int or_vjp(const or_scene* sc, const or_params* pr, const double* x_in, const double* u, const double* gx_out,
           double* gx_in, double* gu, int threads) {
  if (!sc || !pr || !x_in || !u || !gx_out || !gx_in || !gu) return -1;
  std::vector<ArtModel> robots = load_models(sc);
  Layout L = layout_of(sc);
  const int S = sc->n_scenes;
  parallel_scenes(S, threads, [&](int s) {
    Tape tape;
    g_tape = &tape;
    SceneC c;
    load_scene(sc, robots, s, c);
    StateS<adouble> st;
    std::vector<std::pair<size_t, int32_t>> in_idx;
    gather(sc, L, s, x_in, st, [&](size_t i, double v) {
      adouble a = adouble::var(v);
      in_idx.push_back({i, a.i});
      return a;
    });
    adouble us[ND];
    int32_t u_idx[ND];
    for (int j = 0; j < ND; ++j) {
      us[j] = adouble::var(u[(size_t)s * ND + j]);
      u_idx[j] = us[j].i;
    }
    uint32_t status = 0;
    control_step<adouble>(c, *pr, st, us, status, nullptr, s);
    tape.adj.assign(tape.nodes.size(), 0.0);
    scatter(sc, L, s, st, [&](size_t i, const adouble& v) {
      if (v.i >= 0) tape.adj[(size_t)v.i] += gx_out[i];
    });
    tape.reverse();
    for (auto& p : in_idx) gx_in[p.first] = tape.adj[(size_t)p.second];
    for (int j = 0; j < ND; ++j) gu[(size_t)s * ND + j] = tape.adj[(size_t)u_idx[j]];
    g_tape = nullptr;
  });
  return 0;
}

int or_jvp(const or_scene* sc, const or_params* pr, const double* x_in, const double* u, const double* dx_in,
           const double* du, double* dx_out, int threads) {
  if (!sc || !pr || !x_in || !u || !dx_in || !du || !dx_out) return -1;
  std::vector<ArtModel> robots = load_models(sc);
  Layout L = layout_of(sc);
  const int S = sc->n_scenes;
  parallel_scenes(S, threads, [&](int s) {
    SceneC c;
    load_scene(sc, robots, s, c);
    StateS<dual> st;
    gather(sc, L, s, x_in, st, [&](size_t i, double v) { return dual(v, dx_in[i]); });
    dual us[ND];
    for (int j = 0; j < ND; ++j) us[j] = dual(u[(size_t)s * ND + j], du[(size_t)s * ND + j]);
    uint32_t status = 0;
    control_step<dual>(c, *pr, st, us, status, nullptr, s);
    scatter(sc, L, s, st, [&](size_t i, const dual& v) { dx_out[i] = v.d; });
  });
  return 0;
}

int or_flops(const or_scene* sc, const or_params* pr, const double* x_in, const double* u, double* flops) {
  std::vector<ArtModel> robots = load_models(sc);
  Layout L = layout_of(sc);
  const int S = sc->n_scenes;
  parallel_scenes(S, 0, [&](int s) {
    g_flops = 0;
    SceneC c;
    load_scene(sc, robots, s, c);
    StateS<cdouble> st;
    gather(sc, L, s, x_in, st, [](size_t, double v) { return cdouble(v); });
    cdouble us[ND];
    for (int j = 0; j < ND; ++j) us[j] = cdouble(u[(size_t)s * ND + j]);
    uint32_t status = 0;
    control_step<cdouble>(c, *pr, st, us, status, nullptr, s);
    flops[s] = (double)g_flops;
  });
  return 0;
}

int or_spawn_check(const or_scene* sc, const double* x, int32_t* collide, double* min_phi, int threads) {
  if (!sc || !x || !collide) return -1;
  std::vector<ArtModel> robots = load_models(sc);
  Layout L = layout_of(sc);
  parallel_scenes(sc->n_scenes, threads, [&](int s) {
    SceneC c;
    load_scene(sc, robots, s, c);
    StateS<double> st;
    gather(sc, L, s, x, st, [](size_t, double v) { return v; });
    Kin<double> rk;
    fk(*c.robot, st.q, rk, false);
    const int NA = (int)c.aux.size(), NF = (int)c.fr.size();
    std::vector<Kin<double>> ak(NA);
    for (int a = 0; a < NA; ++a) {
      double qa[1] = {st.aq[a]};
      fk(c.aux[a], qa, ak[a], false);
    }
    double mphi = 1e300;
    V3<double> n, p;
    auto see = [&](double phi) { mphi = std::min(mphi, phi); };
    for (const Sphere& sp : c.sph) {
      V3<double> cw = add(mv(rk.R[sp.body], cv3<double>(sp.c)), rk.p[sp.body]);
      for (int pl = 0; pl < (int)c.planes.size(); ++pl) {
        if (pl == 0 && (sp.flags & 1)) continue;
        see(g_plane<double>(cw, sp.r, c.planes[pl].data(), n, p));
      }
      for (const auto& bx : c.boxes)
        see(g_box<double>(cw, sp.r, cv3<double>(bx.data()), ident3<double>(), &bx[3], n, p));
      for (int a = 0; a < NA; ++a) {
        V3<double> bc = add(mv(ak[a].R[0], cv3<double>(c.aux_box[a].data())), ak[a].p[0]);
        see(g_box<double>(cw, sp.r, bc, ak[a].R[0], &c.aux_box[a][3], n, p));
      }
      for (int f = 0; f < NF; ++f) {
        const FreeC& fc = c.fr[f];
        if (fc.type == 0)
          see(g_box<double>(cw, sp.r, st.fr[f].x, quat_R(st.fr[f].Q), fc.half, n, p));
        else
          see(g_sphere<double>(cw, sp.r, st.fr[f].x, fc.half[0], n, p));
      }
    }
    collide[s] = mphi < 0.0 ? 1 : 0;
    if (min_phi) min_phi[s] = mphi;
  });
  return 0;
}

int or_fk(const or_scene* sc, int model, const double* q, double* sph_out, double* origin_out, double* rot_out) {
  ArtModel m;
  load_robot(sc, model, m);
  Kin<double> k;
  fk(m, q, k, false);
  int ns = sc->model_nsph[model];
  for (int i = 0; sph_out && i < ns; ++i) {
    int b = sc->model_sph_body[model * SMX + i];
    V3<double> lc{sc->model_sph[(model * SMX + i) * 4 + 0], sc->model_sph[(model * SMX + i) * 4 + 1],
                  sc->model_sph[(model * SMX + i) * 4 + 2]};
    V3<double> w = add(mv(k.R[b], lc), k.p[b]);
    for (int t = 0; t < 3; ++t) sph_out[i * 3 + t] = w[t];
  }
  for (int i = 0; i < m.nb; ++i) {
    for (int t = 0; origin_out && t < 3; ++t) origin_out[i * 3 + t] = k.p[i][t];
    for (int t = 0; rot_out && t < 9; ++t) rot_out[i * 9 + t] = k.R[i][t];
  }
  return m.nb;
}

int or_dynamics(const or_scene* sc, int model, const double* q, const double* qd, const double* g, double* M_out,
                double* C_out) {
  ArtModel m;
  load_robot(sc, model, m);
  Kin<double> k;
  fk(m, q, k, true);
  if (M_out) crba(m, k, M_out);
  if (C_out) {
    double C[ND] = {0};
    rnea(m, k, qd, (const double*)nullptr, g, C);
    for (int i = 0; i < ND; ++i) C_out[i] = i < m.nb ? C[i] : 0.0;
  }
  return m.nb;
}

// Articulated-body algorithm (Featherstone 2008, Table 7.1) written in world
// coordinates, where every transform between bodies is the identity.
int or_aba(const or_scene* sc, int model, const double* q, const double* qd, const double* tau, const double* arm,
           const double* g, double* qdd_out) {
  ArtModel m;
  load_robot(sc, model, m);
  Kin<double> k;
  fk(m, q, k, true);
  const int nb = m.nb;
  V6<double> v[ND], c[ND], pA[ND], U[ND], a[ND];
  M6<double> IA[ND];
  double D[ND], uu[ND];
  for (int i = 0; i < nb; ++i) {
    int par = m.parent[i];
    V6<double> vJ = scl6(k.s[i], qd[i]);
    v[i] = par < 0 ? vJ : add6(v[par], vJ);
    c[i] = crm(v[i], vJ);
    IA[i] = k.I[i];
    pA[i] = crf(v[i], mul6(k.I[i], v[i]));
  }
  for (int i = nb - 1; i >= 0; --i) {
    U[i] = mul6(IA[i], k.s[i]);
    D[i] = dot6(k.s[i], U[i]) + (arm ? arm[i] : 0.0);
    uu[i] = tau[i] - dot6(k.s[i], pA[i]);
    int par = m.parent[i];
    if (par >= 0) {
      M6<double> Ia;
      for (int r = 0; r < 6; ++r)
        for (int cc = 0; cc < 6; ++cc) Ia[r * 6 + cc] = IA[i][r * 6 + cc] - U[i][r] * U[i][cc] / D[i];
      V6<double> pa = add6(add6(pA[i], mul6(Ia, c[i])), scl6(U[i], uu[i] / D[i]));
      for (int t = 0; t < 36; ++t) IA[par][t] += Ia[t];
      pA[par] = add6(pA[par], pa);
    }
  }
  V6<double> a0 = {0, 0, 0, -g[0], -g[1], -g[2]};
  for (int i = 0; i < nb; ++i) {
    int par = m.parent[i];
    V6<double> ap = add6(par < 0 ? a0 : a[par], c[i]);
    double qdd = (uu[i] - dot6(U[i], ap)) / D[i];
    qdd_out[i] = qdd;
    a[i] = add6(ap, scl6(k.s[i], qdd));
  }
  for (int i = nb; i < ND; ++i) qdd_out[i] = 0.0;
  return nb;
}

double or_kinetic_energy(const or_scene* sc, int model, const double* q, const double* qd) {
  ArtModel m;
  load_robot(sc, model, m);
  Kin<double> k;
  fk(m, q, k, false);
  // link twist from joint rates; velocity of the COM and angular velocity
  double E = 0.0;
  V3<double> w[ND], vo[ND];  // angular velocity, velocity of body origin
  for (int i = 0; i < m.nb; ++i) {
    int par = m.parent[i];
    V3<double> wp = par < 0 ? zero3<double>() : w[par];
    V3<double> vp = par < 0 ? zero3<double>() : vo[par];
    V3<double> pp = par < 0 ? zero3<double>() : k.p[par];
    // velocity of the new origin as a point of the parent, plus the joint's own motion
    V3<double> vpt = add(vp, cross(wp, sub(k.p[i], pp)));
    if (m.jtype[i] == 0) {
      w[i] = add(wp, scl(k.a[i], qd[i]));
      vo[i] = vpt;
    } else {
      w[i] = wp;
      vo[i] = add(vpt, scl(k.a[i], qd[i]));
    }
    V3<double> rc = mv(k.R[i], cv3<double>(m.com[i]));
    V3<double> vc = add(vo[i], cross(w[i], rc));
    M3<double> Icw = mmt(mm(k.R[i], cm3<double>(m.Ic[i])), k.R[i]);
    E += 0.5 * m.mass[i] * dot(vc, vc) + 0.5 * dot(w[i], mv(Icw, w[i]));
  }
  return E;
}

int or_pair(int kind, const double* c, double r, const double* prim, double* out7) {
  V3<double> cc{c[0], c[1], c[2]}, n, p;
  double phi;
  if (kind == 0) {
    phi = g_plane<double>(cc, r, prim, n, p);
  } else if (kind == 1) {
    double R[9];
    quat_R_d(prim + 6, R);
    phi = g_box<double>(cc, r, V3<double>{prim[0], prim[1], prim[2]}, cm3<double>(R), prim + 3, n, p);
  } else {
    phi = g_sphere<double>(cc, r, V3<double>{prim[0], prim[1], prim[2]}, prim[3], n, p);
  }
  out7[0] = phi;
  for (int t = 0; t < 3; ++t) {
    out7[1 + t] = n[t];
    out7[4 + t] = p[t];
  }
  return 0;
}

void or_onb(const double* n, double* t1, double* t2) {
  V3<double> a, b;
  onb<double>(V3<double>{n[0], n[1], n[2]}, a, b);
  for (int t = 0; t < 3; ++t) {
    t1[t] = a[t];
    t2[t] = b[t];
  }
}

void or_quat_update(const double* Q, const double* w, double h, double* out) {
  // same arithmetic as the integrator's free-body orientation update
  V3<double> th{w[0] * h, w[1] * h, w[2] * h};
  double n2 = dot(th, th), cw, sk;
  if (n2 < 1e-12) {
    cw = 1.0 - n2 / 8.0;
    sk = 0.5 - n2 / 48.0;
  } else {
    double nn = std::sqrt(n2);
    cw = std::cos(nn / 2.0);
    sk = std::sin(nn / 2.0) / nn;
  }
  double e[4] = {cw, th[0] * sk, th[1] * sk, th[2] * sk};
  double r[4];
  r[0] = e[0] * Q[0] - (e[1] * Q[1] + e[2] * Q[2] + e[3] * Q[3]);
  r[1] = e[0] * Q[1] + Q[0] * e[1] + (e[2] * Q[3] - e[3] * Q[2]);
  r[2] = e[0] * Q[2] + Q[0] * e[2] + (e[3] * Q[1] - e[1] * Q[3]);
  r[3] = e[0] * Q[3] + Q[0] * e[3] + (e[1] * Q[2] - e[2] * Q[1]);
  double nq = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
  for (int t = 0; t < 4; ++t) out[t] = r[t] / nq;
}

}  // extern "C"
