// ms_kernels.hip -- fused control-step kernel of the batched rigid-body step (gfx950).
//
// One 64-lane wavefront (one workgroup) advances one scene through all
// substeps of a control step with the scene resident in LDS.  Per substep:
//   drive -> forward kinematics (pointer jumping over the tree, lane per body)
//   -> contact generation (lanes over (owner sphere, target) pairs in the
//      canonical order, compacted with ballots so the list stays ordered)
//   -> articulated-body algorithm in world coordinates (outward pass lane per
//      body, inward pass serial, outward pass and the 16 columns of the
//      inverse mass matrix as parallel triangular solves, one lane each)
//   -> contact rows (lane per contact; robot rows lane per DoF and direction)
//   -> level schedule of the canonical row order (lane per dynamic node)
//   -> projected Gauss-Seidel: levels in order, the level's robot row with a
//      16-lane shuffle reduction, the level's other rows one lane each
//   -> semi-implicit Euler.
// The mathematics follows the textbook definitions cited in the C header; no
// code is shared with the CPU oracle.
#include "ms_internal.h"

namespace msk {

// ------------------------------------------------------------ small helpers
struct f3 {
  float x, y, z;
};
__device__ __forceinline__ f3 mk3(float a, float b, float c) { return {a, b, c}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// row-major 3x3
__device__ __forceinline__ f3 mv(const float* R, f3 v) {
  return {R[0] * v.x + R[1] * v.y + R[2] * v.z, R[3] * v.x + R[4] * v.y + R[5] * v.z,
          R[6] * v.x + R[7] * v.y + R[8] * v.z};
}
__device__ __forceinline__ f3 mtv(const float* R, f3 v) {
  return {R[0] * v.x + R[3] * v.y + R[6] * v.z, R[1] * v.x + R[4] * v.y + R[7] * v.z,
          R[2] * v.x + R[5] * v.y + R[8] * v.z};
}
// symmetric 3x3 stored as xx yy zz xy xz yz
__device__ __forceinline__ f3 smv(const float* S, f3 v) {
  return {S[0] * v.x + S[3] * v.y + S[4] * v.z, S[3] * v.x + S[1] * v.y + S[5] * v.z,
          S[4] * v.x + S[5] * v.y + S[2] * v.z};
}
__device__ __forceinline__ void mm(const float* A, const float* B, float* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[i * 3 + j] = A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
}
__device__ __forceinline__ void quat_to_R(float w, float x, float y, float z, float* R) {
  R[0] = 1.f - 2.f * (y * y + z * z);
  R[1] = 2.f * (x * y - w * z);
  R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z);
  R[4] = 1.f - 2.f * (x * x + z * z);
  R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y);
  R[7] = 2.f * (y * z + w * x);
  R[8] = 1.f - 2.f * (x * x + y * y);
}
// rotation by angle th about unit axis k: I + sin K + (1 - cos) K^2
__device__ __forceinline__ void rot_axis(f3 k, float th, float* R) {
  float s, c;
  sincosf(th, &s, &c);
  float oc = 1.f - c;
  R[0] = 1.f - oc * (k.y * k.y + k.z * k.z);
  R[1] = -s * k.z + oc * k.x * k.y;
  R[2] = s * k.y + oc * k.x * k.z;
  R[3] = s * k.z + oc * k.x * k.y;
  R[4] = 1.f - oc * (k.x * k.x + k.z * k.z);
  R[5] = -s * k.x + oc * k.y * k.z;
  R[6] = -s * k.y + oc * k.x * k.z;
  R[7] = s * k.x + oc * k.y * k.z;
  R[8] = 1.f - oc * (k.x * k.x + k.y * k.y);
}
// Duff et al. 2017 orthonormal basis completing unit n
__device__ __forceinline__ void onb(f3 n, f3& t1, f3& t2) {
  float sg = copysignf(1.f, n.z);
  float a = -1.f / (sg + n.z);
  float b = n.x * n.y * a;
  t1 = {1.f + sg * n.x * n.x * a, sg * b, -sg * n.x};
  t2 = {b, sg + n.y * n.y * a, -n.y};
}
// the same basis from a precomputed a = -1 / (sign(n.z) + n.z) (bit for bit)
__device__ __forceinline__ void onb_a(f3 n, float a, f3& t1, f3& t2) {
  float sg = copysignf(1.f, n.z);
  float b = n.x * n.y * a;
  t1 = {1.f + sg * n.x * n.x * a, sg * b, -sg * n.x};
  t2 = {b, sg + n.y * n.y * a, -n.y};
}
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ int lane_id() { return threadIdx.x; }
// the lane index, opaque to the optimizer: address arithmetic on it stays
// where it is used instead of being hoisted out of the scene loop into
// registers that live (or spill) across the whole step
__device__ __forceinline__ int lane_fresh() {
  int l = lane_id();
  asm volatile("" : "+v"(l));
  return l;
}
__device__ __forceinline__ int prefix_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}
__device__ __forceinline__ float bcast(float v, int src) { return __shfl(v, src, WAVE); }
__device__ __forceinline__ int bcasti(int v, int src) { return __shfl(v, src, WAVE); }
// value of the lane N places along within its row of 16 lanes (DPP row
// rotation: a VALU operand modifier, no LDS crossbar)
template <int N>
__device__ __forceinline__ float row_ror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + N, 0xf, 0xf, false));
}
// sum over aligned groups of 16 lanes (result in every lane of the group)
__device__ __forceinline__ float sum16(float v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  return v;
}
// lane src's value in every lane (src uniform)
__device__ __forceinline__ float lane_val(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ void wave_sync() { __syncthreads(); }
// Ordering of LDS accesses between the lanes of the one wavefront of a
// workgroup: the LDS executes a wavefront's instructions in issue order, so a
// read issued after a write sees it; only the compiler must not move memory
// accesses across (no wait for outstanding accesses, unlike the barrier).
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

// spatial 6-vectors [angular; linear] in world coordinates
struct s6 {
  float v[6];
};
__device__ __forceinline__ void crm(const float* v, const float* m, float* out) {  // v x m
  f3 w = mk3(v[0], v[1], v[2]), vo = mk3(v[3], v[4], v[5]), mw = mk3(m[0], m[1], m[2]), ml = mk3(m[3], m[4], m[5]);
  f3 a = cross(w, mw), b = cross(w, ml) + cross(vo, mw);
  out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = b.x; out[4] = b.y; out[5] = b.z;
}
__device__ __forceinline__ void crf(const float* v, const float* f, float* out) {  // v x* f
  f3 w = mk3(v[0], v[1], v[2]), vo = mk3(v[3], v[4], v[5]), n = mk3(f[0], f[1], f[2]), fl = mk3(f[3], f[4], f[5]);
  f3 a = cross(w, n) + cross(vo, fl), b = cross(w, fl);
  out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = b.x; out[4] = b.y; out[5] = b.z;
}

// ------------------------------------------------------------ LDS views
struct Robot {
  float *q, *qd, *tau, *arm, *u;        // [16] each
  float *R, *p, *s;                     // [16][9], [16][3], [16][6]
  float *Minv;                          // [16][16]
  // dynamics scratch, valid only inside the dynamics phase (it shares the
  // LDS of the contact list and the robot contact rows, built afterwards):
  // per body COM, mass and world inertia about the COM [16][BI_FLOATS],
  // velocity-product accelerations and body forces [16][6] each, M~ [16][16],
  // tau - C [16], the per-body sums of the pair-lane reductions
  // [16][DSUM_FLOATS]
  float *bI, *cc, *fo, *Mt, *rhs, *dsum;
};
__device__ __forceinline__ Robot robot_view(float* base, float* dyn) {
  Robot r;
  float* o = base;
  r.q = o; o += ND;
  r.qd = o; o += ND;
  r.tau = o; o += ND;
  r.arm = o; o += ND;
  r.u = o; o += ND;
  r.R = o; o += ND * 9;
  r.p = o; o += ND * 3;
  r.s = o; o += ND * 6;
  r.Minv = o; o += ND * ND;
  o = dyn;
  r.bI = o; o += ND * BI_FLOATS;
  r.cc = o; o += ND * 6;
  r.fo = o; o += ND * 6;
  r.Mt = o; o += ND * ND;
  r.rhs = o; o += ND;
  r.dsum = o; o += ND * DSUM_FLOATS;
  return r;
}
// free-body fields (structure of arrays, stride fmax)
enum FF {
  F_X = 0, F_Q = 3, F_V = 7, F_W = 10, F_R = 13, F_II = 22, F_IM = 28, F_TYPE = 29, F_H = 30, F_IB = 33, F_N = 36
};
// force-output accumulators per free body (own region, force mode only)
enum FRF { R_FRC = 0, R_EE = 3, R_FMIN = 4 };
// aux fields (stride AMAX)
enum AF {
  A_Q = 0, A_QD = 1, A_V = 2, A_R = 3, A_P = 12, A_AX = 15, A_BC = 18, A_IM = 21, A_BH = 22, A_LO = 25, A_HI = 26,
  A_TYPE = 27, A_LIM = 28, A_M = 29, A_EE = 30, A_FMIN = 31, A_N = 32
};
// contact fields (structure of arrays, stride ccap)
// C_KEY: owner sphere index or box vertex (bits 0..7), target class (8..9),
// target index (10..31)
// From the rows phase on, the gap and key slots (dead by then: the gap is in
// the bias, the key in the record) hold the tangent basis factor C_ONB (see
// onb_a) and the normal-tangent couplings C_WTN = (t1, t2) . K n of the
// contact's two sides (K: inverse inertia at the contact point).
enum CF { C_INFO = 0, C_N = 1, C_P = 4, C_IW = 7, C_BIAS = 10, C_LAM = 11, C_PHI = 14, C_KEY = 16, C_ONB = 14, C_WTN = 15 };

// side kinds packed in a contact's info word: A in bits 0..15, B in 16..31,
// each (kind << 8) | index
enum { K_STATIC = 0, K_ROBOT = 1, K_FREE = 2, K_AUX = 3, K_LIMIT = 4 };
__device__ __forceinline__ int side_kind(int s) { return (s >> 8) & 0xff; }
__device__ __forceinline__ int side_idx(int s) { return s & 0xff; }
__device__ __forceinline__ int node_of(int s) {
  int k = side_kind(s);
  if (k == K_ROBOT) return 0;
  if (k == K_AUX || k == K_LIMIT) return 1 + side_idx(s);
  if (k == K_FREE) return 1 + AMAX + side_idx(s);
  return 63;  // static: a lane whose level never changes
}

// Box test: sphere (c, r) against an oriented box (centre bc, world-from-box
// R (null = axis aligned), half extents e).  Returns phi and the normal n
// pointing from the box to the sphere.
__device__ __forceinline__ float box_test(f3 c, float r, f3 bc, const float* R, f3 e, f3& n) {
  f3 d = c - bc;
  f3 y = R ? mtv(R, d) : d;
  bool out = fabsf(y.x) > e.x || fabsf(y.y) > e.y || fabsf(y.z) > e.z;
  float phi;
  f3 nl;
  if (out) {
    f3 k = mk3(fminf(fmaxf(y.x, -e.x), e.x), fminf(fmaxf(y.y, -e.y), e.y), fminf(fmaxf(y.z, -e.z), e.z));
    f3 dd = y - k;
    float dist = sqrtf(dot(dd, dd));
    phi = dist - r;
    float inv = dist > 0.f ? 1.f / dist : 0.f;
    nl = dd * inv;
    if (!(dist > 0.f)) nl = mk3(0.f, 0.f, 1.f);
  } else {
    float gx = e.x - fabsf(y.x), gy = e.y - fabsf(y.y), gz = e.z - fabsf(y.z);
    int best = 0;
    float bv = gx;
    if (gy < bv) { bv = gy; best = 1; }
    if (gz < bv) { bv = gz; best = 2; }
    float yc = best == 0 ? y.x : (best == 1 ? y.y : y.z);
    float sg = yc >= 0.f ? 1.f : -1.f;
    phi = -bv - r;
    nl = mk3(best == 0 ? sg : 0.f, best == 1 ? sg : 0.f, best == 2 ? sg : 0.f);
  }
  n = R ? mv(R, nl) : nl;
  return phi;
}

// ============================================================ the kernel
struct Scene {
  const DModel* M;
  const float* hold;  // [16] hold targets (global)
  int s, nb, nsph, nf, ns, np, na, nfo, f0, s0, p0, a0;
  float gx0, gy0, gix, giy;  // furniture grid: origin and inverse cell sizes (xy)
};

__device__ __forceinline__ void load_scene(const KArgs& a, const Scene& S, float* L, const Robot& rb) {
  const int lane = lane_id();
  const LdsLayout& Y = a.L;
  if (lane < ND) {
    const int ln = lane_fresh();
    rb.q[lane] = a.x_in[(size_t)S.s * ND + ln];
    rb.qd[lane] = a.x_in[(size_t)a.S * ND + (size_t)S.s * ND + ln];
    rb.u[lane] = a.u[(size_t)S.s * ND + ln];
  }
  float* F = L + Y.fr;
  const int fm = Y.fmax;
  for (int f = lane; f < S.nf; f += WAVE) {
    const float* xs = a.x_in + (size_t)a.S * 2 * ND + (size_t)(S.f0 + f) * 16;
    float4 x0 = *reinterpret_cast<const float4*>(xs);
    float4 x1 = *reinterpret_cast<const float4*>(xs + 4);
    float4 x2 = *reinterpret_cast<const float4*>(xs + 8);
    float4 x3 = *reinterpret_cast<const float4*>(xs + 12);
    F[(f) * FSTR + F_X + 0] = x0.x; F[(f) * FSTR + F_X + 1] = x0.y; F[(f) * FSTR + F_X + 2] = x0.z;
    F[(f) * FSTR + F_Q + 0] = x1.x; F[(f) * FSTR + F_Q + 1] = x1.y; F[(f) * FSTR + F_Q + 2] = x1.z;
    F[(f) * FSTR + F_Q + 3] = x1.w;
    F[(f) * FSTR + F_V + 0] = x2.x; F[(f) * FSTR + F_V + 1] = x2.y; F[(f) * FSTR + F_V + 2] = x2.z;
    F[(f) * FSTR + F_W + 0] = x3.x; F[(f) * FSTR + F_W + 1] = x3.y; F[(f) * FSTR + F_W + 2] = x3.z;
    DFree d = a.free[S.f0 + f];
    F[(f) * FSTR + F_IM] = 1.f / d.mass;
    F[(f) * FSTR + F_TYPE] = (float)d.type;
    F[(f) * FSTR + F_H + 0] = d.half[0]; F[(f) * FSTR + F_H + 1] = d.half[1]; F[(f) * FSTR + F_H + 2] = d.half[2];
    F[(f) * FSTR + F_IB + 0] = d.Ib[0]; F[(f) * FSTR + F_IB + 1] = d.Ib[1]; F[(f) * FSTR + F_IB + 2] = d.Ib[2];
  }
  // the zero record past the free bodies: the static side of a contact row
  // in the sweeps (no mass, no velocity)
  if (lane < FREE_FLOATS) F[fm * FSTR + lane] = 0.f;
  float* A = L + Y.aux;
  if (lane < S.na) {
    const float* xs = a.x_in + (size_t)a.S * 2 * ND + (size_t)a.NF * 16 + (size_t)(S.a0 + lane) * 4;
    DAux d = a.aux[S.a0 + lane];
    A[A_Q * AMAX + lane] = xs[0];
    A[A_QD * AMAX + lane] = xs[1];
    for (int t = 0; t < 3; ++t) {
      A[(A_P + t) * AMAX + lane] = d.p0[t];
      A[(A_BH + t) * AMAX + lane] = d.bh[t];
    }
    f3 ax = mv(d.R0, mk3(d.axis[0], d.axis[1], d.axis[2]));
    A[(A_AX + 0) * AMAX + lane] = ax.x; A[(A_AX + 1) * AMAX + lane] = ax.y; A[(A_AX + 2) * AMAX + lane] = ax.z;
    A[A_LO * AMAX + lane] = d.lo;
    A[A_HI * AMAX + lane] = d.hi;
    A[A_TYPE * AMAX + lane] = (float)d.type;
    A[A_LIM * AMAX + lane] = (float)d.has_limit;
  }
  if (Y.smax > 0) {
    float* St = L + Y.stat;
    const float* src = a.statics + (size_t)S.s0 * 6;
    for (int i = lane_fresh(); i < S.ns * 6; i += WAVE) St[i] = src[i];
  }
  float* Pl = L + Y.plane;
  if (lane < S.np) {
    float4 pl = a.planes[S.p0 + lane];
    Pl[lane * 4 + 0] = pl.x; Pl[lane * 4 + 1] = pl.y; Pl[lane * 4 + 2] = pl.z; Pl[lane * 4 + 3] = pl.w;
  }
  // owner table of free bodies: boxes own 8 vertices, spheres 1
  uint16_t* own = reinterpret_cast<uint16_t*>(L + Y.own);
  if (lane == 0) {
    int o = 0;
    for (int f = 0; f < S.nf; ++f) {
      int cnt = a.free[S.f0 + f].type == 0 ? 8 : 1;
      for (int k = 0; k < cnt; ++k) own[o++] = (uint16_t)((f << 3) | k);
    }
  }
  wave_sync();
}

__device__ __forceinline__ void store_scene(const KArgs& a, const Scene& S, float* L, const Robot& rb, uint32_t& status) {
  const int lane = lane_id();
  const LdsLayout& Y = a.L;
  bool bad = false;
  if (!a.x_out) return;  // record mode: the state goes to the record only
  if (lane < ND) {
    float q = rb.q[lane], qd = rb.qd[lane];
    bad |= !isfinite(q) || !isfinite(qd);
    const int ln = lane_fresh();
    a.x_out[(size_t)S.s * ND + ln] = q;
    a.x_out[(size_t)a.S * ND + (size_t)S.s * ND + ln] = qd;
  }
  const float* F = L + Y.fr;
  const int fm = Y.fmax;
  for (int f = lane; f < S.nf; f += WAVE) {
    float* xs = a.x_out + (size_t)a.S * 2 * ND + (size_t)(S.f0 + f) * 16;
    float4 x0 = make_float4(F[(f) * FSTR + F_X + 0], F[(f) * FSTR + F_X + 1], F[(f) * FSTR + F_X + 2], 0.f);
    float4 x1 = make_float4(F[(f) * FSTR + F_Q + 0], F[(f) * FSTR + F_Q + 1], F[(f) * FSTR + F_Q + 2],
                            F[(f) * FSTR + F_Q + 3]);
    float4 x2 = make_float4(F[(f) * FSTR + F_V + 0], F[(f) * FSTR + F_V + 1], F[(f) * FSTR + F_V + 2], 0.f);
    float4 x3 = make_float4(F[(f) * FSTR + F_W + 0], F[(f) * FSTR + F_W + 1], F[(f) * FSTR + F_W + 2], 0.f);
    bad |= !isfinite(x0.x + x0.y + x0.z + x1.x + x1.y + x1.z + x1.w + x2.x + x2.y + x2.z + x3.x + x3.y + x3.z);
    *reinterpret_cast<float4*>(xs) = x0;
    *reinterpret_cast<float4*>(xs + 4) = x1;
    *reinterpret_cast<float4*>(xs + 8) = x2;
    *reinterpret_cast<float4*>(xs + 12) = x3;
  }
  const float* A = L + Y.aux;
  if (lane < S.na) {
    float* xs = a.x_out + (size_t)a.S * 2 * ND + (size_t)a.NF * 16 + (size_t)(S.a0 + lane) * 4;
    float q = A[A_Q * AMAX + lane], qd = A[A_QD * AMAX + lane];
    bad |= !isfinite(q) || !isfinite(qd);
    *reinterpret_cast<float4*>(xs) = make_float4(q, qd, 0.f, 0.f);
  }
  if (__ballot(bad)) status |= 1u;
}

// ---------------------------------------------------------------- record for the adjoint
// state at a substep boundary (q, qd, free bodies, door/drawer joints)
__device__ __forceinline__ void rec_state(const KArgs& a, const Scene& S, const float* L, const Robot& rb, float* R) {
  const int lane = lane_id();
  const LdsLayout& Y = a.L;
  if (lane < ND) {
    R[lane] = rb.q[lane];
    R[ND + lane] = rb.qd[lane];
  }
  const float* F = L + Y.fr;
  const int fm = Y.fmax;
  for (int f = lane; f < S.nf; f += WAVE) {
    float* x = R + 32 + 16 * f;
    x[0] = F[(f) * FSTR + F_X + 0]; x[1] = F[(f) * FSTR + F_X + 1]; x[2] = F[(f) * FSTR + F_X + 2]; x[3] = 0.f;
    x[4] = F[(f) * FSTR + F_Q + 0]; x[5] = F[(f) * FSTR + F_Q + 1]; x[6] = F[(f) * FSTR + F_Q + 2];
    x[7] = F[(f) * FSTR + F_Q + 3];
    x[8] = F[(f) * FSTR + F_V + 0]; x[9] = F[(f) * FSTR + F_V + 1]; x[10] = F[(f) * FSTR + F_V + 2]; x[11] = 0.f;
    x[12] = F[(f) * FSTR + F_W + 0]; x[13] = F[(f) * FSTR + F_W + 1]; x[14] = F[(f) * FSTR + F_W + 2]; x[15] = 0.f;
  }
  const float* A = L + Y.aux;
  if (lane < AMAX) {
    float* x = R + 32 + 16 * fm + 4 * lane;
    bool on = lane < S.na;
    x[0] = on ? A[A_Q * AMAX + lane] : 0.f;
    x[1] = on ? A[A_QD * AMAX + lane] : 0.f;
    x[2] = 0.f;
    x[3] = 0.f;
  }
}
// the substep's contact list as emitted (before the rows overwrite it)
__device__ __forceinline__ void rec_contacts(const KArgs& a, const float* L, int NC, int NL, int NR, float* R) {
  const int lane = lane_id();
  if (lane == 0) {
    R[0] = __int_as_float(NC);
    R[1] = __int_as_float(NL);
    R[2] = __int_as_float(NR);
    R[3] = 0.f;
  }
  // the fields the contact phase wrote (side codes, normal, point, gap,
  // key; limit rows: side code and gap); the rest, which later phases fill
  // in LDS, as zeros so that the record holds no stale values
  const float* C = L + a.L.con;
  for (int i = lane; i < NC * CSTR; i += WAVE) {
    const int f = i % CSTR;
    const bool contact = i / CSTR >= NL;
    const bool keep = f == C_INFO || f == C_PHI || (contact && (f < C_IW || f == C_KEY));
    R[4 + i] = keep ? C[i] : 0.f;
  }
}

// ---------------------------------------------------------------- phases
__device__ __forceinline__ void phase_drive(const KArgs& a, const Scene& S, const Robot& rb) {
  const int j = lane_id();
  if (j < S.nb) {
    const DModel* M = S.M;
    float q = rb.q[j], qd = rb.qd[j], u = rb.u[j], dmp = M->damp[j];
    float tau, arm;
    if (a.mode == 0) {
      tau = u - dmp * qd;
      arm = M->arm[j] + a.h * dmp;
    } else {
      int vd = M->veldof[j];
      float kp = vd ? 0.f : M->kp[j], kd = M->kd[j];
      float qt, vt, ff = 0.f;
      if (a.mode == 1) {
        qt = vd ? 0.f : u;
        vt = vd ? u : 0.f;
      } else {
        qt = vd ? 0.f : S.hold[j];
        vt = vd ? S.hold[j] : 0.f;
        ff = u;
      }
      tau = ff + kp * (qt - q - a.h * qd) + kd * (vt - qd) - dmp * qd;
      arm = M->arm[j] + a.h * (kd + dmp) + a.h * a.h * kp;
    }
    rb.tau[j] = tau;
    rb.arm[j] = arm;
  }
}

// world frames by pointer jumping over the tree; spheres; free and aux frames
__device__ __forceinline__ void phase_kinematics(const KArgs& a, const Scene& S, float* L, const Robot& rb) {
  const int lane = lane_id();
  const DModel* M = S.M;
  const int nb = S.nb;
  float Rw[9], pw[3];
  int anc = -1;
  if (lane < nb) {
    f3 ax = mk3(M->axis[lane][0], M->axis[lane][1], M->axis[lane][2]);
    const float* RT = M->xtR[lane];
    float q = rb.q[lane];
    if (M->jtype[lane] == 0) {
      float RJ[9];
      rot_axis(ax, q, RJ);
      mm(RT, RJ, Rw);
      pw[0] = M->xtp[lane][0]; pw[1] = M->xtp[lane][1]; pw[2] = M->xtp[lane][2];
    } else {
      for (int t = 0; t < 9; ++t) Rw[t] = RT[t];
      f3 d = mv(RT, ax) * q;
      pw[0] = M->xtp[lane][0] + d.x; pw[1] = M->xtp[lane][1] + d.y; pw[2] = M->xtp[lane][2] + d.z;
    }
    anc = M->parent[lane];
  } else {
    for (int t = 0; t < 9; ++t) Rw[t] = t % 4 == 0 ? 1.f : 0.f;
    pw[0] = pw[1] = pw[2] = 0.f;
  }
  // W_i <- W_parent o W_i in depth order (round d composes the bodies of
  // depth d onto their finished parents).  A body's origin is then computed
  // as R_parent xtp + p_parent, the very operations that place a point of the
  // parent at the same local position: coincident spheres on adjacent links
  // (a capsule's end sphere and the next capsule's first) land on the same
  // world point bit for bit and give one consistent duplicated contact, not
  // two that differ by rounding and make Gauss-Seidel trade impulse between
  // them sweep after sweep.  (Composing by pointer jumping takes fewer
  // rounds but associates the products differently.)
  const int depth = lane < nb ? __popc(M->anc[lane]) - 1 : -1;
  for (int d = 1; d < ND; ++d) {
    if (!__ballot(depth >= d)) break;
    const int src = (depth == d && anc >= 0) ? anc : lane;
    float Ra[9], pa[3];
    for (int t = 0; t < 9; ++t) Ra[t] = bcast(Rw[t], src);
    for (int t = 0; t < 3; ++t) pa[t] = bcast(pw[t], src);
    if (depth == d && anc >= 0) {
      float Rn[9];
      mm(Ra, Rw, Rn);
      f3 pn = mv(Ra, mk3(pw[0], pw[1], pw[2]));
      for (int t = 0; t < 9; ++t) Rw[t] = Rn[t];
      pw[0] = pn.x + pa[0]; pw[1] = pn.y + pa[1]; pw[2] = pn.z + pa[2];
    }
  }
  if (lane < nb) {
    for (int t = 0; t < 9; ++t) rb.R[lane * 9 + t] = Rw[t];
    for (int t = 0; t < 3; ++t) rb.p[lane * 3 + t] = pw[t];
    f3 ax = mv(Rw, mk3(M->axis[lane][0], M->axis[lane][1], M->axis[lane][2]));
    float* s = rb.s + lane * 6;
    // motion subspace referred to the body's own origin (on the joint axis)
    if (M->jtype[lane] == 0) {
      s[0] = ax.x; s[1] = ax.y; s[2] = ax.z; s[3] = 0.f; s[4] = 0.f; s[5] = 0.f;
    } else {
      s[0] = 0.f; s[1] = 0.f; s[2] = 0.f; s[3] = ax.x; s[4] = ax.y; s[5] = ax.z;
    }
  }
  wave_sync();
  // sphere centres
  float* SW = L + a.L.sph;
  for (int k = lane; k < S.nsph; k += WAVE) {
    int b = M->sph_body[k];
    float4 sp = M->sph[k];
    f3 c = mv(rb.R + b * 9, mk3(sp.x, sp.y, sp.z)) + mk3(rb.p[b * 3], rb.p[b * 3 + 1], rb.p[b * 3 + 2]);
    SW[k * 4 + 0] = c.x; SW[k * 4 + 1] = c.y; SW[k * 4 + 2] = c.z; SW[k * 4 + 3] = sp.w;
  }
  // free bodies: rotation and world inverse inertia
  float* F = L + a.L.fr;
  const int fm = a.L.fmax;
  for (int f = lane; f < S.nf; f += WAVE) {
    float R[9];
    quat_to_R(F[(f) * FSTR + F_Q + 0], F[(f) * FSTR + F_Q + 1], F[(f) * FSTR + F_Q + 2], F[(f) * FSTR + F_Q + 3], R);
    float ib[3] = {1.f / F[(f) * FSTR + F_IB + 0], 1.f / F[(f) * FSTR + F_IB + 1], 1.f / F[(f) * FSTR + F_IB + 2]};
    for (int t = 0; t < 9; ++t) F[(f) * FSTR + F_R + t] = R[t];
    // world inverse inertia R diag(1/Ib) R^T, symmetric: xx yy zz xy xz yz
    const int ii_r[6] = {0, 1, 2, 0, 0, 1}, ii_c[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      int i = ii_r[e], j = ii_c[e];
      F[(f) * FSTR + F_II + e] = R[i * 3] * ib[0] * R[j * 3] + R[i * 3 + 1] * ib[1] * R[j * 3 + 1] +
                                 R[i * 3 + 2] * ib[2] * R[j * 3 + 2];
    }
  }
  // aux joints: moving frame and world box centre
  float* A = L + a.L.aux;
  if (lane < S.na) {
    DAux d = a.aux[S.a0 + lane];
    float q = A[A_Q * AMAX + lane];
    float R[9];
    f3 p = mk3(d.p0[0], d.p0[1], d.p0[2]);
    if (d.type == 0) {
      float RJ[9];
      rot_axis(mk3(d.axis[0], d.axis[1], d.axis[2]), q, RJ);
      mm(d.R0, RJ, R);
    } else {
      for (int t = 0; t < 9; ++t) R[t] = d.R0[t];
      p = p + mv(d.R0, mk3(d.axis[0], d.axis[1], d.axis[2])) * q;
    }
    f3 bc = mv(R, mk3(d.bc[0], d.bc[1], d.bc[2])) + p;
    for (int t = 0; t < 9; ++t) A[(A_R + t) * AMAX + lane] = R[t];
    A[(A_BC + 0) * AMAX + lane] = bc.x; A[(A_BC + 1) * AMAX + lane] = bc.y; A[(A_BC + 2) * AMAX + lane] = bc.z;
    // generalized inertia about the joint axis: s^T I s (world frame)
    f3 ax = mk3(A[(A_AX + 0) * AMAX + lane], A[(A_AX + 1) * AMAX + lane], A[(A_AX + 2) * AMAX + lane]);
    float Mq;
    if (d.type == 0) {
      // I_c about the axis through the COM plus m * (distance of the COM from the axis)^2
      f3 rc = bc - mk3(d.p0[0], d.p0[1], d.p0[2]);
      f3 lx = mtv(R, ax);  // axis in box coordinates
      float Ia = d.Ib[0] * lx.x * lx.x + d.Ib[1] * lx.y * lx.y + d.Ib[2] * lx.z * lx.z;
      f3 perp = rc - ax * dot(rc, ax);
      Mq = Ia + d.mass * dot(perp, perp);
    } else {
      Mq = d.mass;
    }
    A[A_M * AMAX + lane] = Mq;
    A[A_IM * AMAX + lane] = 1.f / Mq;
  }
  wave_sync();
}

// ---------------------------------------------------------------- contacts
__device__ __forceinline__ f3 body_p(const Robot& rb, int i) {
  return mk3(rb.p[i * 3], rb.p[i * 3 + 1], rb.p[i * 3 + 2]);
}
// Canonical order: owners (robot spheres by index, then free-body vertices /
// spheres by body and vertex), targets (planes, furniture boxes, door /
// drawer boxes, free bodies by index).  Both drivers below evaluate pairs
// with the same function and emit hits through the same ballot compaction in
// pair order, so the contact list is the canonical prefix of the hits.

struct ConCtx {
  const DModel* M;
  float* C;
  int cc;
  const float* SW;
  const float* F;
  int fm;
  const float* A;
  const float* Pl;
  const uint16_t* own;
  const float* St;
  int nsph, np, ns, na, nf, NT;
  float margin;
  bool hash;  // keep the contact-set hash (diagnostics only)
};

struct PairOut {
  float phi;
  f3 n, c;
  float r;
  int aside, bside, osub;
  uint32_t okey, tkey;
};

// owner o: robot sphere (o < nsph) or free-body owner o - nsph
__device__ __forceinline__ void owner_geom(const ConCtx& X, int o, f3& c, float& r, int& okind, int& oidx, int& of,
                                           int& ovk, int& oflags) {
  of = -1;
  ovk = 0;
  oflags = 0;
  if (o < X.nsph) {
    c = mk3(X.SW[o * 4], X.SW[o * 4 + 1], X.SW[o * 4 + 2]);
    r = X.SW[o * 4 + 3];
    oflags = X.M->sph_flags[o];
    oidx = X.M->sph_body[o];
    okind = 0;
  } else {
    int ow = X.own[o - X.nsph];
    of = ow >> 3;
    ovk = ow & 7;
    const float* F = X.F;
    const int fm = X.fm;
    f3 x = mk3(F[(of) * FSTR + F_X + 0], F[(of) * FSTR + F_X + 1], F[(of) * FSTR + F_X + 2]);
    oidx = of;
    if (F[(of) * FSTR + F_TYPE] == 0.f) {
      f3 hl = mk3((ovk & 1) ? F[(of) * FSTR + F_H + 0] : -F[(of) * FSTR + F_H + 0],
                  (ovk & 2) ? F[(of) * FSTR + F_H + 1] : -F[(of) * FSTR + F_H + 1],
                  (ovk & 4) ? F[(of) * FSTR + F_H + 2] : -F[(of) * FSTR + F_H + 2]);
      float Rf[9];
      for (int k = 0; k < 9; ++k) Rf[k] = F[(of) * FSTR + F_R + k];
      c = x + mv(Rf, hl);
      r = 0.f;
      okind = 1;
    } else {
      c = x;
      r = F[(of) * FSTR + F_H + 0];
      okind = 2;
    }
  }
}

// exact pair test of owner o against target t; false when the pair is not allowed
__device__ __forceinline__ bool eval_pair(const ConCtx& X, int o, int t, PairOut& out, bool& isrob) {
  f3 c;
  float r;
  int okind, oidx, of, ovk, oflags;
  owner_geom(X, o, c, r, okind, oidx, of, ovk, oflags);
  isrob = okind == 0;
  float phi = 1e30f;
  f3 nrm = mk3(0.f, 0.f, 1.f);
  int tkey = 0, bside = 0;
  bool allowed = true;
  const float* F = X.F;
  const int fm = X.fm;
  const float* A = X.A;
  if (t < X.np) {
    allowed = !(t == 0 && okind == 0 && (oflags & 1));
    if (allowed) {
      f3 pn = mk3(X.Pl[t * 4], X.Pl[t * 4 + 1], X.Pl[t * 4 + 2]);
      phi = dot(pn, c) - X.Pl[t * 4 + 3] - r;
      nrm = pn;
    }
    tkey = t;
    bside = K_STATIC << 8;
  } else {
    // box targets (furniture, door / drawer boxes, free boxes) share one box
    // test, so that a chunk of pairs with mixed targets runs it once; a
    // furniture box is axis-aligned (the identity rotation is exact)
    float Rb[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
    f3 bc, he;
    bool sphere = false;
    if (t < X.np + X.ns) {
      const int bi = t - X.np;
      const float* bx = X.St + bi * 6;
      bc = mk3(bx[0], bx[1], bx[2]);
      he = mk3(bx[3], bx[4], bx[5]);
      tkey = (1 << 24) | bi;
      bside = K_STATIC << 8;
    } else if (t < X.np + X.ns + X.na) {
      const int x = t - X.np - X.ns;
      for (int k = 0; k < 9; ++k) Rb[k] = A[(A_R + k) * AMAX + x];
      bc = mk3(A[(A_BC + 0) * AMAX + x], A[(A_BC + 1) * AMAX + x], A[(A_BC + 2) * AMAX + x]);
      he = mk3(A[(A_BH + 0) * AMAX + x], A[(A_BH + 1) * AMAX + x], A[(A_BH + 2) * AMAX + x]);
      tkey = (2 << 24) | x;
      bside = (K_AUX << 8) | x;
    } else {
      const int g = t - X.np - X.ns - X.na;
      const bool gbox = F[(g) * FSTR + F_TYPE] == 0.f;
      allowed = g != of;
      if (!gbox && okind == 1) allowed = false;           // box vertices skip free spheres
      if (!gbox && okind == 2 && g <= of) allowed = false;  // sphere pairs once
      bc = mk3(F[(g) * FSTR + F_X + 0], F[(g) * FSTR + F_X + 1], F[(g) * FSTR + F_X + 2]);
      he = mk3(F[(g) * FSTR + F_H + 0], F[(g) * FSTR + F_H + 1], F[(g) * FSTR + F_H + 2]);
      if (gbox)
        for (int k = 0; k < 9; ++k) Rb[k] = F[(g) * FSTR + F_R + k];
      sphere = !gbox;
      tkey = (3 << 24) | g;
      bside = (K_FREE << 8) | g;
    }
    if (allowed) {
      if (sphere) {
        f3 d = c - bc;
        float dist = sqrtf(dot(d, d));
        phi = dist - r - he.x;
        nrm = dist < 1e-12f ? mk3(0.f, 0.f, 1.f) : d * (1.f / dist);
      } else {
        phi = box_test(c, r, bc, Rb, he, nrm);
      }
    }
  }
  out.phi = phi;
  out.n = nrm;
  out.c = c;
  out.r = r;
  out.aside = okind == 0 ? ((K_ROBOT << 8) | oidx) : ((K_FREE << 8) | of);
  out.bside = bside;
  out.okey = okind == 0 ? (uint32_t)o : ((1u << 24) | ((uint32_t)of << 3) | (uint32_t)ovk);
  out.osub = okind == 0 ? o : ovk;
  out.tkey = (uint32_t)tkey;
  return allowed && phi < X.margin;
}

struct EmitState {
  int n, nr;
  bool over, rover;
  uint64_t ks;
};

// wave-collective: append this lane's hit at its canonical position
__device__ __forceinline__ void emit(const ConCtx& X, int rcap, bool hit, bool isrob, const PairOut& po,
                                     EmitState& E) {
  uint64_t mr = __ballot(hit && isrob);
  int rpos = E.nr + prefix_below(mr);
  bool keep = hit && (!isrob || rpos < rcap);
  if (hit && isrob && rpos >= rcap) E.rover = true;
  uint64_t mk = __ballot(keep);
  int pos = E.n + prefix_below(mk);
  if (keep && pos >= X.cc) {
    keep = false;
    E.over = true;
  }
  if (keep) {
    float* C = X.C;
    const int cc = X.cc;
    C[(pos) * CSTR + C_INFO] = __int_as_float(po.aside | (po.bside << 16));
    f3 p = po.c - po.n * po.r;
    C[(pos) * CSTR + C_N + 0] = po.n.x; C[(pos) * CSTR + C_N + 1] = po.n.y; C[(pos) * CSTR + C_N + 2] = po.n.z;
    C[(pos) * CSTR + C_P + 0] = p.x; C[(pos) * CSTR + C_P + 1] = p.y; C[(pos) * CSTR + C_P + 2] = p.z;
    C[(pos) * CSTR + C_PHI] = po.phi;
    C[(pos) * CSTR + C_KEY] = __int_as_float(po.osub | (int)((po.tkey >> 24) << 8) | (int)((po.tkey & 0xffffffu) << 10));
    if (X.hash) E.ks += mix64(((uint64_t)po.okey << 32) | po.tkey);
  }
  uint64_t mkept = __ballot(keep);
  E.n = min(E.n + __popcll(mkept), X.cc);
  E.nr += __popcll(__ballot(keep && isrob));
}

// q = i / n, r = i - q n for small non-negative i and n > 0
__device__ __forceinline__ void divmod(int i, int n, float inv, int& q, int& r) {
  q = (int)(((float)i + 0.5f) * inv);
  r = i - q * n;
  if (r < 0) { --q; r += n; }
  if (r >= n) { ++q; r -= n; }
}

// wave-collective ordered compaction: out[] = item(i) for the i in [0, N)
// with pred(item(i)), in increasing i
template <class I, class P>
__device__ __forceinline__ int compact(int N, uint16_t* out, I item, P pred) {
  int cnt = 0;
  for (int base = 0; base < N; base += WAVE) {
    int i = base + lane_id();
    int v = i < N ? item(i) : 0;
    bool m = i < N && pred(v);
    uint64_t mk = __ballot(m);
    if (m) out[cnt + prefix_below(mk)] = (uint16_t)v;
    cnt += __popcll(mk);
  }
  return cnt;
}

__device__ __forceinline__ float dist_point_box(f3 y, f3 e) {
  f3 d = mk3(fmaxf(fabsf(y.x) - e.x, 0.f), fmaxf(fabsf(y.y) - e.y, 0.f), fmaxf(fabsf(y.z) - e.z, 0.f));
  return sqrtf(dot(d, d));
}

// conservative test of a bounding sphere (c, R) against target t
__device__ __forceinline__ bool sphere_near_target(const ConCtx& X, f3 c, float R, int t, float slack) {
  const float* F = X.F;
  const int fm = X.fm;
  const float* A = X.A;
  if (t < X.np) {
    f3 pn = mk3(X.Pl[t * 4], X.Pl[t * 4 + 1], X.Pl[t * 4 + 2]);
    return dot(pn, c) - X.Pl[t * 4 + 3] - R < slack;
  }
  if (t < X.np + X.ns) {
    const float* bx = X.St + (t - X.np) * 6;
    return dist_point_box(c - mk3(bx[0], bx[1], bx[2]), mk3(bx[3], bx[4], bx[5])) - R < slack;
  }
  if (t < X.np + X.ns + X.na) {
    int x = t - X.np - X.ns;
    float Rx[9];
    for (int k = 0; k < 9; ++k) Rx[k] = A[(A_R + k) * AMAX + x];
    f3 y = mtv(Rx, c - mk3(A[(A_BC + 0) * AMAX + x], A[(A_BC + 1) * AMAX + x], A[(A_BC + 2) * AMAX + x]));
    return dist_point_box(y, mk3(A[(A_BH + 0) * AMAX + x], A[(A_BH + 1) * AMAX + x], A[(A_BH + 2) * AMAX + x])) - R <
           slack;
  }
  int g = t - X.np - X.ns - X.na;
  f3 xg = mk3(F[(g) * FSTR + F_X + 0], F[(g) * FSTR + F_X + 1], F[(g) * FSTR + F_X + 2]);
  if (F[(g) * FSTR + F_TYPE] == 0.f) {
    float Rg[9];
    for (int k = 0; k < 9; ++k) Rg[k] = F[(g) * FSTR + F_R + k];
    return dist_point_box(mtv(Rg, c - xg), mk3(F[(g) * FSTR + F_H + 0], F[(g) * FSTR + F_H + 1], F[(g) * FSTR + F_H + 2])) -
               R < slack;
  }
  f3 d = c - xg;
  return sqrtf(dot(d, d)) - R - F[(g) * FSTR + F_H + 0] < slack;
}

// conservative test of an axis-aligned box (centre bc, half extents he) against target t
__device__ __forceinline__ bool box_near_target(const ConCtx& X, f3 bc, f3 he, int t, float slack) {
  const float* F = X.F;
  const int fm = X.fm;
  const float* A = X.A;
  if (t < X.np) {
    f3 pn = mk3(X.Pl[t * 4], X.Pl[t * 4 + 1], X.Pl[t * 4 + 2]);
    float supp = fabsf(pn.x) * he.x + fabsf(pn.y) * he.y + fabsf(pn.z) * he.z;
    return dot(pn, bc) - supp - X.Pl[t * 4 + 3] < slack;
  }
  if (t < X.np + X.ns) {
    const float* bx = X.St + (t - X.np) * 6;
    return fabsf(bc.x - bx[0]) < he.x + bx[3] + slack && fabsf(bc.y - bx[1]) < he.y + bx[4] + slack &&
           fabsf(bc.z - bx[2]) < he.z + bx[5] + slack;
  }
  f3 c;
  float rad;
  if (t < X.np + X.ns + X.na) {
    int x = t - X.np - X.ns;
    c = mk3(A[(A_BC + 0) * AMAX + x], A[(A_BC + 1) * AMAX + x], A[(A_BC + 2) * AMAX + x]);
    f3 h = mk3(A[(A_BH + 0) * AMAX + x], A[(A_BH + 1) * AMAX + x], A[(A_BH + 2) * AMAX + x]);
    rad = sqrtf(dot(h, h));
  } else {
    int g = t - X.np - X.ns - X.na;
    c = mk3(F[(g) * FSTR + F_X + 0], F[(g) * FSTR + F_X + 1], F[(g) * FSTR + F_X + 2]);
    f3 h = mk3(F[(g) * FSTR + F_H + 0], F[(g) * FSTR + F_H + 1], F[(g) * FSTR + F_H + 2]);
    rad = F[(g) * FSTR + F_TYPE] == 0.f ? sqrtf(dot(h, h)) : h.x;
  }
  return dist_point_box(c - bc, he) - rad < slack;
}

// Bound of one culling target, held by a lane: a plane (n in ctr, offset pd)
// or an axis-aligned box (centre ctr, half extents half) grown by rt: planes
// exactly, furniture boxes as their boxes, door / drawer boxes and free
// bodies as bounding spheres.  g: the free body a target is (-1: none).
struct TBound {
  bool valid, isplane;
  f3 ctr, half;
  float rt, pd;
  int g, gbox;
};
__device__ __forceinline__ void target_bound(const ConCtx& X, int t, TBound& B) {
  B.valid = t >= 0 && t < X.NT;
  B.isplane = false;
  B.ctr = mk3(0.f, 0.f, 0.f);
  B.half = mk3(0.f, 0.f, 0.f);
  B.rt = 0.f;
  B.pd = 0.f;
  B.g = -1;
  B.gbox = 0;
  if (!B.valid) return;
  const float* F = X.F;
  const float* A = X.A;
  const int gbase = X.np + X.ns + X.na;
  if (t < X.np) {
    B.isplane = true;
    B.ctr = mk3(X.Pl[t * 4], X.Pl[t * 4 + 1], X.Pl[t * 4 + 2]);
    B.pd = X.Pl[t * 4 + 3];
  } else if (t < X.np + X.ns) {
    const float* bx = X.St + (t - X.np) * 6;
    B.ctr = mk3(bx[0], bx[1], bx[2]);
    B.half = mk3(bx[3], bx[4], bx[5]);
  } else if (t < gbase) {
    const int x = t - X.np - X.ns;
    B.ctr = mk3(A[(A_BC + 0) * AMAX + x], A[(A_BC + 1) * AMAX + x], A[(A_BC + 2) * AMAX + x]);
    f3 h = mk3(A[(A_BH + 0) * AMAX + x], A[(A_BH + 1) * AMAX + x], A[(A_BH + 2) * AMAX + x]);
    B.rt = sqrtf(dot(h, h));
  } else {
    const int g = t - gbase;
    B.g = g;
    B.ctr = mk3(F[(g) * FSTR + F_X + 0], F[(g) * FSTR + F_X + 1], F[(g) * FSTR + F_X + 2]);
    f3 h = mk3(F[(g) * FSTR + F_H + 0], F[(g) * FSTR + F_H + 1], F[(g) * FSTR + F_H + 2]);
    B.gbox = F[(g) * FSTR + F_TYPE] == 0.f ? 1 : 0;
    B.rt = B.gbox ? sqrtf(dot(h, h)) : h.x;
  }
}
// conservative: may sphere (c, R) come within `slack` of the bound?  Sphere-
// to-box distances are compared squared (slack covers the rounding).
__device__ __forceinline__ bool bound_near(const TBound& B, f3 c, float R, float slack) {
  if (B.isplane) return dot(B.ctr, c) - B.pd - R < slack;
  const f3 q = mk3(fmaxf(fabsf(c.x - B.ctr.x) - B.half.x, 0.f), fmaxf(fabsf(c.y - B.ctr.y) - B.half.y, 0.f),
                   fmaxf(fabsf(c.z - B.ctr.z) - B.half.z, 0.f));
  const float lim = R + B.rt + slack;
  return dot(q, q) < lim * lim;
}

// position of the k-th (from 0) set bit of m (k < popcount(m))
__device__ __forceinline__ int select_bit(uint64_t m, int k) {
  int pos = 0;
  uint32_t x = (uint32_t)m;
  int c = __popc(x);
  if (k >= c) {
    k -= c;
    pos = 32;
    x = (uint32_t)(m >> 32);
  }
  c = __popc(x & 0xffffu);
  if (k >= c) { k -= c; pos += 16; x >>= 16; }
  c = __popc(x & 0xffu);
  if (k >= c) { k -= c; pos += 8; x >>= 8; }
  c = __popc(x & 0xfu);
  if (k >= c) { k -= c; pos += 4; x >>= 4; }
  c = __popc(x & 0x3u);
  if (k >= c) { k -= c; pos += 2; x >>= 2; }
  if (k >= (int)(x & 1u)) pos += 1;
  return pos;
}

// Exact tests of bodies' owners against their culled candidates (body b:
// mem(b) owners from owner index obase(b); candidates: the set bits of its
// masks, bit j of chunk ch standing for target tgt(ch, j)), packed into full
// chunks: consecutive bodies are grouped while the group's pairs fit one
// chunk; a body with more than a chunk of pairs runs alone over several.
// Pairs are enumerated (body, owner, candidate) in increasing order, so the
// contacts come out in canonical order.  A lane finds its body by comparing
// its pair index with the members' first pairs, and its candidate as the
// set bit of that rank in the body's masks.
template <class Mem, class Obase, class Tgt>
__device__ __forceinline__ void exact_grouped(const ConCtx& X, int rcap, int nbod, const uint32_t* msk, int nch,
                                              Mem mem, Obase obase, Tgt tgt, EmitState& E) {
  const int lane = lane_id();
  auto mask_of = [&](int b, int ch) -> uint64_t {
    return (uint64_t)msk[(b * nch + ch) * 2] | ((uint64_t)msk[(b * nch + ch) * 2 + 1] << 32);
  };
  // lane b: body b's candidate count
  int bcnt = 0;
  if (lane < nbod)
    for (int ch = 0; ch < nch; ++ch) bcnt += __popcll(mask_of(lane, ch));
  int b = 0;
  while (b < nbod) {
    // lane gi: group member gi's first pair, candidates, owner base, body
    int ng = 0, pairs = 0;
    int gP = 0, gC = 1, gO = 0, gB = 0;
    while (b < nbod) {
      const int cnt = __builtin_amdgcn_readlane(bcnt, b);
      const int m = mem(b);
      if (cnt == 0 || m == 0) {
        ++b;
        continue;
      }
      if (ng > 0 && pairs + m * cnt > WAVE) break;
      if (lane == ng) {
        gP = pairs;
        gC = cnt;
        gO = obase(b);
        gB = b;
      }
      pairs += m * cnt;
      ++ng;
      ++b;
      if (pairs > WAVE) break;
    }
    if (ng == 0) break;
    for (int base = 0; base < pairs; base += WAVE) {
      const int idx = base + lane;
      int gi = 0;
      for (int j = 1; j < ng; ++j) gi += idx >= __builtin_amdgcn_readlane(gP, j) ? 1 : 0;
      const int P = __shfl(gP, gi, WAVE), Cn = __shfl(gC, gi, WAVE), O = __shfl(gO, gi, WAVE),
                Bb = __shfl(gB, gi, WAVE);
      PairOut po;
      bool isrob = false, hit = false;
      if (idx < pairs) {
        int k, ci;
        divmod(idx - P, Cn, 1.f / (float)Cn, k, ci);
        int ch = 0;
        uint64_t m = mask_of(Bb, 0);
        int c = __popcll(m);
        while (ci >= c) {
          ci -= c;
          ++ch;
          m = mask_of(Bb, ch);
          c = __popcll(m);
        }
        hit = eval_pair(X, O + k, tgt(ch, select_bit(m, ci)), po, isrob);
      }
      emit(X, rcap, hit, isrob, po, E);
    }
  }
}

__device__ __forceinline__ void phase_contacts(const KArgs& a, const Scene& S, float* L, const Robot& rb, int& NC, int& NR, int& NL,
                               uint32_t& status, uint64_t& keysum) {
  const int lane = lane_id();
  const LdsLayout& Y = a.L;
  ConCtx X;
  X.M = S.M;
  X.C = L + Y.con;
  X.cc = Y.ccap;
  X.SW = L + Y.sph;
  X.F = L + Y.fr;
  X.fm = Y.fmax;
  X.A = L + Y.aux;
  X.Pl = L + Y.plane;
  X.own = reinterpret_cast<const uint16_t*>(L + Y.own);
  X.St = Y.smax > 0 ? (L + Y.stat) : (a.statics + (size_t)S.s0 * 6);
  X.nsph = S.nsph; X.np = S.np; X.ns = S.ns; X.na = S.na; X.nf = S.nf;
  X.NT = S.np + S.ns + S.na + S.nf;
  X.margin = a.margin;
  X.hash = a.debug != nullptr;
  float* C = X.C;
  const int cc = X.cc;
  const float* Ax = X.A;

  int n = 0;
  // joint-limit rows of door / drawer joints come first in the canonical order
  if (lane == 0) {
    for (int x = 0; x < S.na; ++x) {
      if (Ax[A_LIM * AMAX + x] == 0.f) continue;
      float q = Ax[A_Q * AMAX + x];
      float gaps[2] = {q - Ax[A_LO * AMAX + x], Ax[A_HI * AMAX + x] - q};
      for (int e = 0; e < 2; ++e) {
        if (gaps[e] < a.margin && n < cc) {
          C[(n) * CSTR + C_INFO] = __int_as_float((K_LIMIT << 8 | x) | ((e == 0 ? 0 : 1) << 16));
          C[(n) * CSTR + C_PHI] = gaps[e];
          ++n;
        }
      }
    }
  }
  n = bcasti(n, 0);
  NL = n;
  EmitState E{n, 0, false, false, 0ull};
  const int NT = X.NT;
  if (!a.cull) {
    // brute force over every (owner, target) pair
    const int NO = S.nsph + S.nfo;
    const int total = NO * NT;
    const float invNT = NT > 0 ? 1.f / (float)NT : 0.f;
    for (int base = 0; base < total; base += WAVE) {
      int pair = base + lane;
      PairOut po;
      bool isrob = false, hit = false;
      if (pair < total) {
        int o, t;
        divmod(pair, NT, invNT, o, t);
        hit = eval_pair(X, o, t, po, isrob);
      }
      emit(X, a.rcap, hit, isrob, po, E);
    }
  } else {
    // bounding volumes first; the exact test runs on the surviving pairs only.
    // The slack covers single-precision rounding of the bounding tests.
    const float slack = a.margin + 1e-3f;
    uint16_t* listA = reinterpret_cast<uint16_t*>(L + Y.cand);
    uint16_t* listB = listA + Y.ntmax;
    const DModel* M = S.M;
    if (S.nsph > 0) {
      // axis-aligned box around the robot's body bounding spheres
      f3 lo = mk3(1e30f, 1e30f, 1e30f), hi = mk3(-1e30f, -1e30f, -1e30f);
      if (lane < S.nb && M->sph_count[lane] > 0) {
        float4 bs = M->bsph[lane];
        f3 c = mv(rb.R + lane * 9, mk3(bs.x, bs.y, bs.z)) + body_p(rb, lane);
        lo = mk3(c.x - bs.w, c.y - bs.w, c.z - bs.w);
        hi = mk3(c.x + bs.w, c.y + bs.w, c.z + bs.w);
      }
      for (int off = 32; off > 0; off >>= 1) {
        lo.x = fminf(lo.x, __shfl_xor(lo.x, off, WAVE)); lo.y = fminf(lo.y, __shfl_xor(lo.y, off, WAVE));
        lo.z = fminf(lo.z, __shfl_xor(lo.z, off, WAVE)); hi.x = fmaxf(hi.x, __shfl_xor(hi.x, off, WAVE));
        hi.y = fmaxf(hi.y, __shfl_xor(hi.y, off, WAVE)); hi.z = fmaxf(hi.z, __shfl_xor(hi.z, off, WAVE));
      }
      f3 bc = (lo + hi) * 0.5f, he = (hi - lo) * 0.5f;
      // the robot's candidate targets in increasing order; the furniture
      // boxes of four chunks are loaded together
      int nra = 0;
      for (int base = 0; base < NT; base += 4 * WAVE) {
        float bx[4][6];
        if (S.ns > 0) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int si = max(0, min(S.ns - 1, base + u * WAVE + lane - S.np));
#pragma unroll
            for (int e = 0; e < 6; ++e) bx[u][e] = X.St[si * 6 + e];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = base + u * WAVE + lane;
          bool m = false;
          if (t < NT) {
            if (t >= S.np && t < S.np + S.ns)
              m = fabsf(bc.x - bx[u][0]) < he.x + bx[u][3] + slack && fabsf(bc.y - bx[u][1]) < he.y + bx[u][4] + slack &&
                  fabsf(bc.z - bx[u][2]) < he.z + bx[u][5] + slack;
            else
              m = box_near_target(X, bc, he, t, slack);
          }
          const uint64_t mk = __ballot(m);
          if (m) listA[nra + prefix_below(mk)] = (uint16_t)t;
          nra += __popcll(mk);
        }
      }
      // the robot bodies' bounding spheres against the robot's candidates,
      // transposed as for the free bodies below: lanes over a chunk of the
      // candidates, a loop over the bodies, one ballot per (body, chunk)
      uint32_t* msk = reinterpret_cast<uint32_t*>(L + Y.cmask);
      const int ncA = (nra + WAVE - 1) / WAVE;
      // the bodies' bounding spheres (centre, radius; a body without spheres
      // radius -1) where every lane reads them with one broadcast load
      float4* rbd = reinterpret_cast<float4*>(L + Y.cmask + lds_align4((Y.fmax > ND ? Y.fmax : ND) * Y.nch * 2));
      if (lane < S.nb) {
        float4 bs = M->bsph[lane];
        const f3 c = mv(rb.R + lane * 9, mk3(bs.x, bs.y, bs.z)) + body_p(rb, lane);
        rbd[lane] = make_float4(c.x, c.y, c.z, M->sph_count[lane] > 0 ? bs.w : -1.f);
      }
      lds_order();
      for (int ch = 0; ch < ncA; ++ch) {
        const int i = ch * WAVE + lane;
        TBound B;
        target_bound(X, i < nra ? (int)listA[i] : -1, B);
#pragma unroll 4
        for (int b = 0; b < S.nb; ++b) {
          const float4 bd = rbd[b];
          const bool m = bd.w >= 0.f && B.valid && bound_near(B, mk3(bd.x, bd.y, bd.z), bd.w, slack);
          const uint64_t mk = __ballot(m);
          if (lane == 0) {
            msk[(b * ncA + ch) * 2] = (uint32_t)mk;
            msk[(b * ncA + ch) * 2 + 1] = (uint32_t)(mk >> 32);
          }
        }
      }
      wave_sync();
      exact_grouped(
          X, a.rcap, S.nb, msk, ncA, [&](int b) { return M->sph_count[b]; }, [&](int b) { return M->sph_first[b]; },
          [&](int ch, int j) { return (int)listA[ch * WAVE + j]; }, E);
    }
    // free bodies.  Bounding-sphere culling in two parts.  Furniture: each
    // body's lane looks up the cells of the scene's furniture grid its sphere
    // overlaps and tests only the boxes registered there.  Planes, door /
    // drawer boxes and free bodies, transposed: the lanes hold a chunk of
    // those targets' bounds, the loop runs over the bodies (their spheres by
    // broadcast loads from LDS), one ballot per body and chunk.  Both set the
    // bodies' bits in the mask table with LDS atomics; then the exact tests,
    // grouped.  The grid only skips boxes the bounding test would reject, so
    // the candidates are those of a test against every target.
    {
      const float* F = X.F;
      const int fm = X.fm;
      uint32_t* msk = reinterpret_cast<uint32_t*>(L + Y.cmask);
      unsigned long long* msk64 = reinterpret_cast<unsigned long long*>(msk);
      const int nch = (NT + WAVE - 1) / WAVE;
      // lane f: body f's bounding sphere, kind and first owner index
      f3 fc = mk3(0.f, 0.f, 0.f);
      float fR = 0.f;
      int fb = 0, fmem = 0;
      if (lane < S.nf) {
        fc = mk3(F[(lane) * FSTR + F_X + 0], F[(lane) * FSTR + F_X + 1], F[(lane) * FSTR + F_X + 2]);
        f3 h = mk3(F[(lane) * FSTR + F_H + 0], F[(lane) * FSTR + F_H + 1], F[(lane) * FSTR + F_H + 2]);
        fb = F[(lane) * FSTR + F_TYPE] == 0.f ? 1 : 0;
        fR = fb ? sqrtf(dot(h, h)) : h.x;
        fmem = fb ? 8 : 1;
      }
      int fob = fmem;  // inclusive scan of the owners per body
      for (int off = 1; off < WAVE; off <<= 1) {
        const int v = __shfl_up(fob, off, WAVE);
        if (lane >= off) fob += v;
      }
      fob += S.nsph - fmem;
      // the bodies' spheres (centre, radius; the radius negative for a free
      // sphere) where every lane reads them with one broadcast load
      float4* fbd = reinterpret_cast<float4*>(L + Y.cmask + lds_align4((Y.fmax > ND ? Y.fmax : ND) * Y.nch * 2));
      if (lane < S.nf) fbd[lane] = make_float4(fc.x, fc.y, fc.z, fb ? fR : -fR);
      for (int e = lane; e < S.nf * nch; e += WAVE) msk64[e] = 0ull;
      lds_order();
      // furniture, by the grid (lane per body): the words of every cell the
      // sphere overlaps are loaded together, then the candidates' boxes four
      // at a time
      if (lane < S.nf && S.ns > 0) {
        const int nw = a.sg_nw, nws = (S.ns + WAVE - 1) / WAVE;
        const unsigned long long* cells =
            reinterpret_cast<const unsigned long long*>(a.sgrid + (size_t)sgrid_floats(nw) * S.s + 4);
        const float reach = fR + slack + 2e-3f;
        const int x0 = max(0, min(SGRID - 1, (int)floorf((fc.x - reach - S.gx0) * S.gix)));
        const int x1 = max(0, min(SGRID - 1, (int)floorf((fc.x + reach - S.gx0) * S.gix)));
        const int y0 = max(0, min(SGRID - 1, (int)floorf((fc.y - reach - S.gy0) * S.giy)));
        const int y1 = max(0, min(SGRID - 1, (int)floorf((fc.y + reach - S.gy0) * S.giy)));
        const int ncell = (x1 - x0 + 1) * (y1 - y0 + 1);
        for (int wg = 0; wg < nws; wg += 4) {
          unsigned long long cw[4] = {0ull, 0ull, 0ull, 0ull};
          int cx = x0, cy = y0;
          for (int k0 = 0; k0 < ncell; k0 += 4) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
              const bool kv = k0 + kk < ncell;
              const unsigned long long* c = cells + (min(cy, y1) * SGRID + cx) * nw;
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const unsigned long long v = c[min(wg + u, nw - 1)];
                cw[u] |= (kv && wg + u < nws) ? v : 0ull;
              }
              if (++cx > x1) {
                cx = x0;
                ++cy;
              }
            }
          }
          // the candidates in increasing order, taken from the words in turn
          unsigned long long cur = cw[0], n1 = cw[1], n2 = cw[2], n3 = cw[3];
          int wb = wg * 64;
          auto refill = [&]() {
            while (cur == 0ull && (n1 | n2 | n3) != 0ull) {
              cur = n1;
              n1 = n2;
              n2 = n3;
              n3 = 0ull;
              wb += 64;
            }
          };
          refill();
          while (cur) {
            int bi[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              refill();
              bi[u] = cur ? wb + __ffsll((long long)cur) - 1 : -1;
              cur &= cur - 1ull;
            }
            float bx[4][6];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const float* src = X.St + (bi[u] >= 0 ? bi[u] : bi[0]) * 6;
#pragma unroll
              for (int e = 0; e < 6; ++e) bx[u][e] = src[e];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              TBound B;
              B.valid = true;
              B.isplane = false;
              B.ctr = mk3(bx[u][0], bx[u][1], bx[u][2]);
              B.half = mk3(bx[u][3], bx[u][4], bx[u][5]);
              B.rt = 0.f;
              B.pd = 0.f;
              B.g = -1;
              B.gbox = 0;
              if (bi[u] >= 0 && bound_near(B, fc, fR, slack)) {
                const int t = S.np + bi[u];
                atomicOr(msk64 + lane * nch + (t >> 6), 1ull << (t & 63));
              }
            }
            refill();
          }
        }
      }
      // planes, door / drawer boxes and free bodies (transposed).  With at
      // most 32 such targets both halves of the wave hold them, and each
      // ballot serves two bodies (the lower half's and the upper half's).
      const int NO = S.np + S.na + S.nf;
      if (NO <= WAVE / 2) {
        const int hh = lane >> 5, l = lane & 31;
        const int t = l < S.np ? l : S.ns + l;  // the target index of other-target l
        TBound B;
        target_bound(X, l < NO ? t : -1, B);
        uint64_t mym = 0;  // lane f: body f's bits over the other targets
#pragma unroll 2
        for (int f0 = 0; f0 < S.nf; f0 += 2) {
          const int f = f0 + hh;
          const float4 bd = fbd[f < S.nf ? f : S.nf - 1];
          const bool fbox = bd.w >= 0.f;
          bool m = f < S.nf && B.valid && bound_near(B, mk3(bd.x, bd.y, bd.z), fabsf(bd.w), slack);
          if (B.g >= 0 && (B.g == f || (!B.gbox && (fbox || B.g <= f)))) m = false;
          const uint64_t mk = __ballot(m);
          mym = lane == f0 ? (mk & 0xffffffffull) : (lane == f0 + 1 ? (mk >> 32) : mym);
        }
        if (lane < S.nf)
          while (mym) {
            const int bit = __ffsll((long long)mym) - 1;
            mym &= mym - 1ull;
            const int tt = bit < S.np ? bit : S.ns + bit;
            atomicOr(msk64 + lane * nch + (tt >> 6), 1ull << (tt & 63));
          }
      }
      for (int base = 0; NO > WAVE / 2 && base < NO; base += WAVE) {
        const int l = base + lane;
        const int t = l < S.np ? l : S.ns + l;  // the target index of other-target l
        TBound B;
        target_bound(X, l < NO ? t : -1, B);
        uint64_t mym = 0;  // lane f: body f's bits over this chunk of other targets
#pragma unroll 2
        for (int f = 0; f < S.nf; ++f) {
          const float4 bd = fbd[f];
          const bool fbox = bd.w >= 0.f;
          bool m = B.valid && bound_near(B, mk3(bd.x, bd.y, bd.z), fabsf(bd.w), slack);
          // pair rules of free-body targets: not itself; box vertices skip
          // free spheres; sphere pairs once
          if (B.g >= 0 && (B.g == f || (!B.gbox && (fbox || B.g <= f)))) m = false;
          const uint64_t mk = __ballot(m);
          mym = lane == f ? mk : mym;
        }
        if (lane < S.nf)
          while (mym) {
            const int bit = __ffsll((long long)mym) - 1;
            mym &= mym - 1ull;
            const int lo = base + bit;
            const int tt = lo < S.np ? lo : S.ns + lo;
            atomicOr(msk64 + lane * nch + (tt >> 6), 1ull << (tt & 63));
          }
      }
      wave_sync();
      exact_grouped(
          X, a.rcap, S.nf, msk, nch, [&](int f) { return __builtin_amdgcn_readlane(fmem, f); },
          [&](int f) { return __builtin_amdgcn_readlane(fob, f); }, [&](int ch, int j) { return ch * WAVE + j; }, E);
    }
  }
  uint64_t ks = E.ks;
  for (int off = 32; off > 0; off >>= 1) ks += __shfl_xor(ks, off, WAVE);
  keysum = ks;
  if (__ballot(E.over)) status |= 2u;
  if (__ballot(E.rover)) status |= 8u;
  NC = E.n;
  NR = E.nr;
  wave_sync();
}

// Joint-space dynamics of the robot: M~ = M + diag(arm) by the composite-
// rigid-body algorithm and the bias forces C(q, qd) by recursive Newton-Euler
// (Featherstone 2008, Sec. 6.2 and 5.3), then M~^-1 by Gauss-Jordan
// elimination and qdd = M~^-1 (tau - C).  Axes are world-aligned and each
// body's quantities are referred to its own origin p_i (on the joint axis):
// sums over a subtree take every member's inertia, force or motion straight
// to p_i with lever arms of link length, which keeps FP32 free of the
// cancellation that origin-referred inertias of distant links suffer, and no
// tree recursion runs serially over the bodies.

// motion vector m given at point P, expressed at point Q (d = Q - P)
__device__ __forceinline__ void shift_motion(const float* m, f3 d, float* out) {
  f3 w = mk3(m[0], m[1], m[2]);
  f3 v = mk3(m[3], m[4], m[5]) + cross(w, d);
  out[0] = m[0]; out[1] = m[1]; out[2] = m[2]; out[3] = v.x; out[4] = v.y; out[5] = v.z;
}
// force vector f given at point P, expressed at point Q (e = P - Q)
__device__ __forceinline__ void shift_force(const float* f, f3 e, float* out) {
  f3 n = mk3(f[0], f[1], f[2]) + cross(e, mk3(f[3], f[4], f[5]));
  out[0] = n.x; out[1] = n.y; out[2] = n.z; out[3] = f[3]; out[4] = f[4]; out[5] = f[5];
}
// motion subspace of joint k expressed at point q
__device__ __forceinline__ void s_at(const Robot& rb, const DModel* M, int k, f3 q, float* out) {
  const float* s = rb.s + k * 6;
  if (M->jtype[k] == 0) {
    f3 a = mk3(s[0], s[1], s[2]);
    f3 v = cross(a, q - body_p(rb, k));
    out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = v.x; out[4] = v.y; out[5] = v.z;
  } else {
    for (int t = 0; t < 6; ++t) out[t] = s[t];
  }
}
// A rigid (or composite) inertia about a point P: mass m, first moment
// h = m (c - P) and rotational inertia J about P (symmetric: xx yy zz xy xz
// yz).  As a spatial matrix [[J, h x], [(h x)^T, m 1]] applied to the motion
// (w, v): n = J w + h x v, f = m v - h x w.
struct RI {
  float m, h[3], J[6];
};
__device__ __forceinline__ void ri_apply(const RI& I, const float* mv6, float* out) {
  const f3 w = mk3(mv6[0], mv6[1], mv6[2]), v = mk3(mv6[3], mv6[4], mv6[5]), h = mk3(I.h[0], I.h[1], I.h[2]);
  const f3 hv = cross(h, v), hw = cross(h, w);
  out[0] = I.J[0] * w.x + I.J[3] * w.y + I.J[4] * w.z + hv.x;
  out[1] = I.J[3] * w.x + I.J[1] * w.y + I.J[5] * w.z + hv.y;
  out[2] = I.J[4] * w.x + I.J[5] * w.y + I.J[2] * w.z + hv.z;
  out[3] = I.m * v.x - hw.x;
  out[4] = I.m * v.y - hw.y;
  out[5] = I.m * v.z - hw.z;
}
// add a body (mass m, COM offset d from P, rotational inertia Jc about its
// COM) to an inertia about P (parallel axis: J += Jc + m (|d|^2 1 - d d^T))
__device__ __forceinline__ void ri_add(RI& I, float m, f3 d, const float* Jc) {
  const float dd = dot(d, d);
  I.m += m;
  I.h[0] += m * d.x; I.h[1] += m * d.y; I.h[2] += m * d.z;
  I.J[0] += Jc[0] + m * (dd - d.x * d.x);
  I.J[1] += Jc[1] + m * (dd - d.y * d.y);
  I.J[2] += Jc[2] + m * (dd - d.z * d.z);
  I.J[3] += Jc[3] - m * d.x * d.y;
  I.J[4] += Jc[4] - m * d.x * d.z;
  I.J[5] += Jc[5] - m * d.y * d.z;
}

__device__ __forceinline__ void phase_dynamics(const KArgs& a, const Scene& S, float* L, const Robot& rb, float& vR) {
  const int lane = lane_id();
  const DModel* M = S.M;
  const int nb = S.nb;
  // M~ starts as zero, with identity rows and columns past the robot's DoFs
  for (int e = lane; e < ND * ND; e += WAVE) {
    const int r = e / ND, c = e % ND;
    rb.Mt[e] = (r >= nb || c >= nb) && r == c ? 1.f : 0.f;
  }
  // The sums over a body's ancestors or descendants run over pair lanes: in
  // each of four rounds, row q (lanes 16 q .. 16 q + 15) serves body
  // i = 4 r + q and lane k of the row the other body k; the row's 16 terms
  // are added by a 16-lane reduction, and lane 0 of the row leaves the sum in
  // LDS for body i's own lane.  (One lane per body looping over the other
  // bodies made each sum a chain of 16 dependent LDS rounds.)
  const int lf = lane_fresh(), q = lf >> 4, kq = lf & 15;
  // pass 1 (lane per body): COM and world inertia about the COM (kept for the
  // subtree sums); (pair lanes) twist v_i = sum over k in anc-or-self(i) of
  // s_k qd_k at p_i; (lane per body) the velocity-product acceleration
  // c_i = v_i x (s_i qd_i) and force p_i = v_i x* (I_i v_i)
  RI Ib{0.f, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}};
  float vp[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  f3 pi = mk3(0.f, 0.f, 0.f);
  if (lane < nb) {
    const int i = lane_fresh();
    pi = body_p(rb, i);
    const float* R = rb.R + i * 9;
    const f3 d = mv(R, mk3(M->com[i][0], M->com[i][1], M->com[i][2]));
    const float* ic = M->Ic[i];
    const float Bb[9] = {ic[0], ic[3], ic[4], ic[3], ic[1], ic[5], ic[4], ic[5], ic[2]};
    float RB[9];
    mm(R, Bb, RB);
    float Jc[6];
    const int rr[6] = {0, 1, 2, 0, 0, 1}, cc6[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const int r = rr[t], qq = cc6[t];
      Jc[t] = RB[r * 3] * R[qq * 3] + RB[r * 3 + 1] * R[qq * 3 + 1] + RB[r * 3 + 2] * R[qq * 3 + 2];
    }
    const float m = M->mass[i];
    ri_add(Ib, m, d, Jc);
    float* bI = rb.bI + i * BI_FLOATS;
    bI[0] = pi.x + d.x; bI[1] = pi.y + d.y; bI[2] = pi.z + d.z;
    bI[3] = m;
    for (int t = 0; t < 6; ++t) bI[4 + t] = Jc[t];
  }
  for (int r0 = 0; r0 < nb; r0 += 4) {
    const int i = r0 + q;
    float t6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < nb && kq < nb && ((M->anc[i] >> kq) & 1)) {
      float sk[6];
      s_at(rb, M, kq, body_p(rb, i), sk);
      const float qd = rb.qd[kq];
      for (int t = 0; t < 6; ++t) t6[t] = sk[t] * qd;
    }
    for (int t = 0; t < 6; ++t) t6[t] = sum16(t6[t]);
    if (kq == 0 && i < nb)
      for (int t = 0; t < 6; ++t) rb.fo[i * 6 + t] = t6[t];  // v_i (fo is free until pass 2 ends)
  }
  lds_order();
  if (lane < nb) {
    const int i = lane;
    float v[6], vJ[6], Iv[6];
    for (int t = 0; t < 6; ++t) v[t] = rb.fo[i * 6 + t];
    const float qd = rb.qd[i];
    for (int t = 0; t < 6; ++t) vJ[t] = rb.s[i * 6 + t] * qd;
    crm(v, vJ, rb.cc + i * 6);
    ri_apply(Ib, v, Iv);
    crf(v, Iv, vp);
  }
  wave_sync();
  // pass 2 (pair lanes): bias acceleration (qdd = 0, gravity as the base's
  // acceleration -g) a_i = -g + sum over anc-or-self of c_k, taken to p_i;
  // the subtree's composite inertia about p_i; then (lane per body) the body
  // force f_i = I_i a_i + p_i
  for (int r0 = 0; r0 < nb; r0 += 4) {
    const int i = r0 + q;
    float ta[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    RI tc{0.f, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}};
    if (i < nb && kq < nb) {
      const f3 p_i = body_p(rb, i);
      if ((M->anc[i] >> kq) & 1) shift_motion(rb.cc + kq * 6, p_i - body_p(rb, kq), ta);
      if ((M->anc[kq] >> i) & 1) {
        const float* bk = rb.bI + kq * BI_FLOATS;
        ri_add(tc, bk[3], mk3(bk[0], bk[1], bk[2]) - p_i, bk + 4);
      }
    }
    for (int t = 0; t < 6; ++t) ta[t] = sum16(ta[t]);
    tc.m = sum16(tc.m);
    for (int t = 0; t < 3; ++t) tc.h[t] = sum16(tc.h[t]);
    for (int t = 0; t < 6; ++t) tc.J[t] = sum16(tc.J[t]);
    if (kq == 0 && i < nb) {
      float* o = rb.dsum + i * DSUM_FLOATS;
      for (int t = 0; t < 6; ++t) o[t] = ta[t];
      o[6] = tc.m;
      for (int t = 0; t < 3; ++t) o[7 + t] = tc.h[t];
      for (int t = 0; t < 6; ++t) o[10 + t] = tc.J[t];
    }
  }
  lds_order();
  RI Ic{0.f, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}};
  if (lane < nb) {
    const int i = lane;
    const float* o = rb.dsum + i * DSUM_FLOATS;
    float acc6[6] = {o[0], o[1], o[2], o[3] - a.g[0], o[4] - a.g[1], o[5] - a.g[2]};
    Ic.m = o[6];
    for (int t = 0; t < 3; ++t) Ic.h[t] = o[7 + t];
    for (int t = 0; t < 6; ++t) Ic.J[t] = o[10 + t];
    float fi[6];
    ri_apply(Ib, acc6, fi);
    for (int t = 0; t < 6; ++t) rb.fo[i * 6 + t] = fi[t] + vp[t];
  }
  wave_sync();
  // pass 3: (pair lanes) the subtree's body forces at p_i; (lane per body)
  // C_i = s_i . that sum, the right-hand side tau - C, G_i = I^c_i s_i and
  // M_ii; (pair lanes) M_ij = s_j . G_i for j a strict ancestor of i, all at
  // p_i, plus the armature on the diagonal
  for (int r0 = 0; r0 < nb; r0 += 4) {
    const int i = r0 + q;
    float tf[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < nb && kq < nb && ((M->anc[kq] >> i) & 1))
      shift_force(rb.fo + kq * 6, body_p(rb, kq) - body_p(rb, i), tf);
    for (int t = 0; t < 6; ++t) tf[t] = sum16(tf[t]);
    if (kq == 0 && i < nb)
      for (int t = 0; t < 6; ++t) rb.dsum[i * DSUM_FLOATS + t] = tf[t];
  }
  lds_order();
  if (lane < nb) {
    const int i = lane;
    const float* si = rb.s + i * 6;
    float C = 0.f, G[6];
    for (int t = 0; t < 6; ++t) C += si[t] * rb.dsum[i * DSUM_FLOATS + t];
    rb.rhs[i] = rb.tau[i] - C;
    ri_apply(Ic, si, G);
    float Mii = 0.f;
    for (int t = 0; t < 6; ++t) Mii += si[t] * G[t];
    rb.Mt[i * ND + i] = Mii + rb.arm[i];
    for (int t = 0; t < 6; ++t) rb.dsum[i * DSUM_FLOATS + 6 + t] = G[t];
  }
  lds_order();
  for (int r0 = 0; r0 < nb; r0 += 4) {
    const int i = r0 + q, j = kq;
    if (i < nb && j < i && ((M->anc[i] >> j) & 1)) {
      float sj[6];
      s_at(rb, M, j, body_p(rb, i), sj);
      const float* G = rb.dsum + i * DSUM_FLOATS + 6;
      float v = 0.f;
      for (int t = 0; t < 6; ++t) v += sj[t] * G[t];
      rb.Mt[i * ND + j] = v;
      rb.Mt[j * ND + i] = v;
    }
  }
  wave_sync();
  // M~^-1 by Gauss-Jordan elimination without pivoting (M~ is symmetric
  // positive definite) in registers: lane r < 16 holds row r, the pivot row
  // is read from its lane with readlane (the loops are unrolled, so every
  // register index is a constant); the identity past the robot's DoFs stays
  if (lane < ND) {
    float e[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) e[k] = rb.Mt[lane * ND + k];
#pragma unroll
    for (int p = 0; p < ND; ++p) {
      float prow[ND];
#pragma unroll
      for (int k = 0; k < ND; ++k) prow[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(e[k]), p));
      const float inv = 1.f / prow[p];
      const float f = e[p];
      const bool own = lane == p;
#pragma unroll
      for (int k = 0; k < ND; ++k) {
        if (k == p) e[k] = own ? inv : -f * inv;
        else e[k] = own ? prow[k] * inv : e[k] - f * (prow[k] * inv);
      }
    }
#pragma unroll
    for (int k = 0; k < ND; ++k) rb.Minv[lane * ND + k] = lane < nb && k < nb ? e[k] : 0.f;
  }
  wave_sync();
  // M~^-1 is symmetric, but the elimination rounds its two triangles
  // differently.  The rows read it row-wise for W = J M~^-1 J^T and the sweeps
  // column-wise for w = M~^-1 J^T; with the two triangles averaged both see
  // the same numbers in the same order, so a robot row's update applies
  // exactly the W its impulse was computed with (otherwise the mismatch
  // accumulates sweep after sweep on redundant contact sets, e.g. more robot
  // contacts than DoFs).
  for (int e = lane; e < ND * ND; e += WAVE) {
    const int i = e / ND, k = e % ND;
    if (i < k) {
      const float m = 0.5f * (rb.Minv[e] + rb.Minv[k * ND + i]);
      rb.Minv[e] = m;
      rb.Minv[k * ND + i] = m;
    }
  }
  wave_sync();
  // unconstrained robot velocity qd + h M~^-1 (tau - C): joint j in lane j
  // of each 16-lane row (the four copies are equal)
  {
    const int j = lane & 15;
    float qdd = 0.f;
    if (j < nb)
      for (int k = 0; k < nb; ++k) qdd += rb.Minv[j * ND + k] * rb.rhs[k];
    vR = rb.qd[j] + a.h * qdd;
  }
  // free bodies: v* = v + h g ; w* = w - h Iw^-1 (w x Iw w)
  float* F = L + a.L.fr;
  const int fm = a.L.fmax;
  for (int f = lane; f < S.nf; f += WAVE) {
    float R[9];
    for (int t = 0; t < 9; ++t) R[t] = F[(f) * FSTR + F_R + t];
    f3 w = mk3(F[(f) * FSTR + F_W + 0], F[(f) * FSTR + F_W + 1], F[(f) * FSTR + F_W + 2]);
    f3 wl = mtv(R, w);
    f3 Iwl = mk3(F[(f) * FSTR + F_IB + 0] * wl.x, F[(f) * FSTR + F_IB + 1] * wl.y, F[(f) * FSTR + F_IB + 2] * wl.z);
    f3 Iw = mv(R, Iwl);
    f3 gy = cross(w, Iw);
    float Ii[6];
    for (int t = 0; t < 6; ++t) Ii[t] = F[(f) * FSTR + F_II + t];
    f3 dw = smv(Ii, gy);
    F[(f) * FSTR + F_W + 0] = w.x - a.h * dw.x;
    F[(f) * FSTR + F_W + 1] = w.y - a.h * dw.y;
    F[(f) * FSTR + F_W + 2] = w.z - a.h * dw.z;
    for (int t = 0; t < 3; ++t) F[(f) * FSTR + F_V + t] += a.h * a.g[t];
  }
  // aux joints: passive single-DoF bodies; the gravity torque about the axis
  float* Ax = L + a.L.aux;
  if (lane < S.na) {
    DAux d = a.aux[S.a0 + lane];
    f3 ax = mk3(Ax[(A_AX + 0) * AMAX + lane], Ax[(A_AX + 1) * AMAX + lane], Ax[(A_AX + 2) * AMAX + lane]);
    f3 bc = mk3(Ax[(A_BC + 0) * AMAX + lane], Ax[(A_BC + 1) * AMAX + lane], Ax[(A_BC + 2) * AMAX + lane]);
    f3 gvec = mk3(a.g[0], a.g[1], a.g[2]);
    float gen;  // generalized gravity force
    if (d.type == 0) gen = dot(ax, cross(bc - mk3(d.p0[0], d.p0[1], d.p0[2]), gvec * d.mass));
    else gen = d.mass * dot(ax, gvec);
    float qd = Ax[A_QD * AMAX + lane];
    Ax[A_V * AMAX + lane] = qd + a.h * gen * Ax[A_IM * AMAX + lane];
  }
  wave_sync();
}

// Point-Jacobian column of aux joint x at world point p
__device__ __forceinline__ f3 aux_col(const float* A, int x, f3 p) {
  f3 ax = mk3(A[(A_AX + 0) * AMAX + x], A[(A_AX + 1) * AMAX + x], A[(A_AX + 2) * AMAX + x]);
  if (A[A_TYPE * AMAX + x] == 0.f) {
    f3 o = mk3(A[(A_P + 0) * AMAX + x], A[(A_P + 1) * AMAX + x], A[(A_P + 2) * AMAX + x]);
    return cross(ax, p - o);
  }
  return ax;
}

// Entry j of the robot's Jacobian row for direction d at the point p of a
// contact on body `body`: d . (a_j x (p - o_j)) for a revolute joint, d . a_j
// for a prismatic one, 0 when joint j does not move the body
__device__ __forceinline__ float robot_J(const DModel* M, const Robot& rb, int nb, int body, int j, f3 d, f3 p) {
  float J = 0.f;
  if (j < nb && ((M->anc[body] >> j) & 1)) {
    const float* s = rb.s + j * 6;
    if (M->jtype[j] == 0) J = dot(d, cross(mk3(s[0], s[1], s[2]), p - mk3(rb.p[j * 3], rb.p[j * 3 + 1], rb.p[j * 3 + 2])));
    else J = dot(d, mk3(s[3], s[4], s[5]));
  }
  return J;
}

__device__ __forceinline__ void phase_rows(const KArgs& a, const Scene& S, float* L, const Robot& rb, int NC, int NR, int NL,
                           uint32_t& status) {
  const int lane = lane_id();
  const LdsLayout& Y = a.L;
  float* C = L + Y.con;
  const int cc = Y.ccap;
  const float* F = L + Y.fr;
  const int fm = Y.fmax;
  const float* A = L + Y.aux;
  const DModel* M = S.M;
  // lane per contact: tangents, free / aux effective-mass parts, bias
  for (int ci = lane; ci < NC; ci += WAVE) {
    int info = __float_as_int(C[(ci) * CSTR + C_INFO]);
    int sA = info & 0xffff, sB = (info >> 16) & 0xffff;
    float phi = C[(ci) * CSTR + C_PHI];
    float bias = phi >= 0.f ? phi / a.h : a.beta * phi / a.h;
    if (side_kind(sA) == K_LIMIT) {
      int x = side_idx(sA);
      C[(ci) * CSTR + C_IW + 0] = A[A_IM * AMAX + x];  // W = 1 / M~ for J = +-1
      C[(ci) * CSTR + C_BIAS] = bias;
      for (int t = 0; t < 3; ++t) C[(ci) * CSTR + C_LAM + t] = 0.f;
      continue;
    }
    f3 n = mk3(C[(ci) * CSTR + C_N + 0], C[(ci) * CSTR + C_N + 1], C[(ci) * CSTR + C_N + 2]);
    f3 p = mk3(C[(ci) * CSTR + C_P + 0], C[(ci) * CSTR + C_P + 1], C[(ci) * CSTR + C_P + 2]);
    const float ta = -1.f / (copysignf(1.f, n.z) + n.z);
    f3 t1, t2;
    onb_a(n, ta, t1, t2);
    float W0 = 0.f, W1 = 0.f, W2 = 0.f, W1n = 0.f, W2n = 0.f;
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      int sv = sd == 0 ? sA : sB;
      int k = side_kind(sv), idx = side_idx(sv);
      if (k == K_FREE) {
        f3 r = p - mk3(F[(idx) * FSTR + F_X + 0], F[(idx) * FSTR + F_X + 1], F[(idx) * FSTR + F_X + 2]);
        float Ii[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) Ii[t] = F[(idx) * FSTR + F_II + t];
        float im = F[(idx) * FSTR + F_IM];
        f3 r0 = cross(r, n), r1 = cross(r, t1), r2 = cross(r, t2);
        const f3 k0 = smv(Ii, r0);
        W0 += im + dot(r0, k0);
        W1 += im + dot(r1, smv(Ii, r1));
        W2 += im + dot(r2, smv(Ii, r2));
        W1n += dot(r1, k0);
        W2n += dot(r2, k0);
      } else if (k == K_AUX) {
        f3 col = aux_col(A, idx, p);
        float im = A[A_IM * AMAX + idx];
        float J0 = dot(n, col), J1 = dot(t1, col), J2 = dot(t2, col);
        W0 += J0 * J0 * im;
        W1 += J1 * J1 * im;
        W2 += J2 * J2 * im;
        W1n += J1 * J0 * im;
        W2n += J2 * J0 * im;
      }
    }
    C[(ci) * CSTR + C_IW + 0] = W0;
    C[(ci) * CSTR + C_IW + 1] = W1;
    C[(ci) * CSTR + C_IW + 2] = W2;
    C[(ci) * CSTR + C_BIAS] = bias;
    C[(ci) * CSTR + C_ONB] = ta;
    C[(ci) * CSTR + C_WTN + 0] = W1n;
    C[(ci) * CSTR + C_WTN + 1] = W2n;
    for (int t = 0; t < 3; ++t) C[(ci) * CSTR + C_LAM + t] = 0.f;
  }
  wave_sync();
  // robot rows: lane (d, j) builds J[d][j] = d . (dp/dq_j) and W = J M~^-1 J^T
  float* Rw = L + Y.rows;
  const int d = lane >> 4, j = lane & 15;
  for (int rr = 0; rr < NR; ++rr) {
    const int ci = NL + rr;
    float* row = Rw + rr * ROW_FLOATS;
    int info = __float_as_int(C[(ci) * CSTR + C_INFO]);
    int body = side_idx(info & 0xffff);
    if (d < 3) {
      f3 n = mk3(C[(ci) * CSTR + C_N + 0], C[(ci) * CSTR + C_N + 1], C[(ci) * CSTR + C_N + 2]);
      f3 p = mk3(C[(ci) * CSTR + C_P + 0], C[(ci) * CSTR + C_P + 1], C[(ci) * CSTR + C_P + 2]);
      f3 t1, t2;
      onb_a(n, C[(ci) * CSTR + C_ONB], t1, t2);
      f3 dir = d == 0 ? n : (d == 1 ? t1 : t2);
      row[d * ND + j] = robot_J(M, rb, S.nb, body, j, dir, p);
    }
    wave_sync();
    float w = 0.f;
    if (d < 3) {
#pragma unroll
      for (int k = 0; k < ND; ++k) w += rb.Minv[j * ND + k] * row[d * ND + k];
    }
    const float wn = __shfl(w, j, WAVE);  // M~^-1 J_n^T
    if (d < 3) {
      // W_dd, and the couplings J_d M~^-1 J_n^T of the tangents (added to
      // the other side's part of C_WTN)
      const float Wr = sum16(row[d * ND + j] * w);
      const float Wc = sum16(row[d * ND + j] * wn);
      if (j == 0) {
        C[(ci) * CSTR + C_IW + d] += Wr;
        if (d > 0) C[(ci) * CSTR + C_WTN + d - 1] += Wc;
      }
    }
    wave_sync();
  }
  // inverse effective masses; rows below 1e-12 are skipped (inverse 0)
  bool degen = false;
  for (int ci = lane; ci < NC; ci += WAVE) {
    for (int dd = 0; dd < 3; ++dd) {
      float W = C[(ci) * CSTR + C_IW + dd];
      int info = __float_as_int(C[(ci) * CSTR + C_INFO]);
      bool lim = side_kind(info & 0xffff) == K_LIMIT;
      if (lim && dd > 0) continue;
      if (W >= 1e-12f) C[(ci) * CSTR + C_IW + dd] = 1.f / W;
      else {
        C[(ci) * CSTR + C_IW + dd] = 0.f;
        degen = true;
      }
    }
  }
  if (__ballot(degen)) status |= 4u;
  wave_sync();
}

// Level schedule.  Rows are first merged into groups: a run of consecutive
// rows (in canonical order) between one free body and static targets is one
// group, run by one lane in order with the body's state in registers; every
// other row is a group of its own.  level(g) = 1 + max level of earlier
// groups sharing a node, so that executing the levels in order performs the
// sequential row updates exactly.  Then an order list of the groups grouped
// by level; each level's robot row is kept apart.
// The nodes are the robot (0), the door / drawer joints (1 + x) and the free
// bodies (1 + AMAX + f); static targets are no node.  For every node a bit
// mask of the groups touching it (LDS atomics, one bit per group) gives each
// group the previous group on each of its nodes, and the levels are the
// longest-path depths of that DAG, relaxed over the lanes until no level
// changes (as many rounds as the deepest chain).
__device__ __forceinline__ void row_nodes(int inf, int& na, int& nbn) {
  na = node_of(inf & 0xffff);
  nbn = side_kind(inf & 0xffff) == K_LIMIT ? 63 : node_of((inf >> 16) & 0xffff);
}
// a row between a free body and a static target (may join its predecessor's group)
__device__ __forceinline__ bool row_single(int inf) {
  return side_kind(inf & 0xffff) == K_FREE && side_kind((inf >> 16) & 0xffff) == K_STATIC;
}
__device__ __forceinline__ int phase_levels(const KArgs& a, float* L, int NC, int NR, int NL) {
  const int lane = lane_id();
  const LdsLayout& Y = a.L;
  const float* C = L + Y.con;
  const int cc = Y.ccap;
  // per level the offset of its groups in `order` and its robot row (0xffff:
  // none); the groups of each level (first row | rows << 16); each group's
  // level and first row.  While the levels are found, loff and rob hold each
  // group's previous group on its first and second node (0xffff: none).
  uint16_t* loff = reinterpret_cast<uint16_t*>(L + Y.lvl);     // [cc + 2]
  uint16_t* rob = loff + cc + 2;                               // [cc + 2]
  uint32_t* order = reinterpret_cast<uint32_t*>(rob + cc + 2);  // [cc]
  uint16_t* lvl = reinterpret_cast<uint16_t*>(order + cc);     // [cc]
  uint16_t* gfirst = lvl + cc;                                 // [cc + 1]
  // group starts and first rows
  int NG = 0;
  for (int base = 0; base < NC; base += WAVE) {
    const int r = base + lane;
    bool st = false;
    if (r < NC) {
      const int inf = __float_as_int(C[r * CSTR + C_INFO]);
      st = true;
      if (r > 0 && row_single(inf)) {
        const int pinf = __float_as_int(C[(r - 1) * CSTR + C_INFO]);
        st = !(row_single(pinf) && (pinf & 0xffff) == (inf & 0xffff));
      }
    }
    const uint64_t mk = __ballot(st);
    if (st) gfirst[NG + prefix_below(mk)] = (uint16_t)r;
    NG += __popcll(mk);
  }
  if (lane == 0) gfirst[NG] = (uint16_t)NC;
  const int nch = (NG + WAVE - 1) / WAVE;
  const int nnode = 1 + AMAX + Y.fmax;
  unsigned long long* nm = reinterpret_cast<unsigned long long*>(L + Y.cand);  // [nnode][nch]
  for (int e = lane; e < nnode * nch; e += WAVE) nm[e] = 0ull;
  lds_order();
  for (int ch = 0; ch < nch; ++ch) {
    const int g = ch * WAVE + lane;
    if (g < NG) {
      int na, nbn;
      row_nodes(__float_as_int(C[gfirst[g] * CSTR + C_INFO]), na, nbn);
      const unsigned long long bit = 1ull << lane;
      atomicOr(nm + na * nch + ch, bit);
      if (nbn != 63) atomicOr(nm + nbn * nch + ch, bit);
    }
  }
  lds_order();
  // the previous group touching node n before group g (-1: none)
  auto prev = [&](int n, int g) {
    int w = g >> 6;
    unsigned long long m = nm[n * nch + w] & ((1ull << (g & 63)) - 1ull);
    while (m == 0ull && w > 0) {
      --w;
      m = nm[n * nch + w];
    }
    return m ? w * WAVE + 63 - __clzll((long long)m) : -1;
  };
  for (int ch = 0; ch < nch; ++ch) {
    const int g = ch * WAVE + lane;
    if (g < NG) {
      int na, nbn;
      row_nodes(__float_as_int(C[gfirst[g] * CSTR + C_INFO]), na, nbn);
      const int pa = prev(na, g), pb = nbn == 63 ? -1 : prev(nbn, g);
      loff[g] = (uint16_t)(pa < 0 ? 0xffff : pa);
      rob[g] = (uint16_t)(pb < 0 ? 0xffff : pb);
      lvl[g] = 1;
    }
  }
  lds_order();
  // relax: level(g) = 1 + max(level(prev on node A), level(prev on node B))
  for (;;) {
    bool changed = false;
    for (int ch = 0; ch < nch; ++ch) {
      const int g = ch * WAVE + lane;
      if (g < NG) {
        const int pa = loff[g], pb = rob[g];
        const int la = pa == 0xffff ? 0 : lvl[pa], lb = pb == 0xffff ? 0 : lvl[pb];
        const int nl = 1 + max(la, lb);
        if (nl != lvl[g]) {
          lvl[g] = (uint16_t)nl;
          changed = true;
        }
      }
    }
    if (!__ballot(changed)) break;
    lds_order();
  }
  int maxl = 0;
  for (int g = lane; g < NG; g += WAVE) maxl = max(maxl, (int)lvl[g]);
  for (int off = 32; off > 0; off >>= 1) maxl = max(maxl, __shfl_xor(maxl, off, WAVE));
  lds_order();
  for (int e = lane; e <= maxl + 1; e += WAVE) rob[e] = 0xffff;
  lds_order();
  // robot rows are groups of their own: rob[level] = the row
  for (int g = lane; g < NG; g += WAVE) {
    const int r = gfirst[g];
    if (r >= NL && r < NL + NR) rob[lvl[g]] = (uint16_t)r;
  }
  int pos = 0;
  for (int lv = 1; lv <= maxl; ++lv) {
    if (lane == 0) loff[lv - 1] = (uint16_t)pos;
    for (int base = 0; base < NG; base += WAVE) {
      const int g = base + lane;
      bool m = false;
      int r = 0;
      if (g < NG) {
        r = gfirst[g];
        m = !(r >= NL && r < NL + NR) && lvl[g] == lv;
      }
      uint64_t mk = __ballot(m);
      if (m) order[pos + prefix_below(mk)] = (uint32_t)r | ((uint32_t)(gfirst[g + 1] - r) << 16);
      pos += __popcll(mk);
    }
  }
  if (lane == 0) loff[maxl] = (uint16_t)pos;
  wave_sync();
  return maxl;
}

// One dynamic side of a contact held in registers during a row update:
// free body (x, v, w, 1/m, world inverse inertia) or door / drawer joint
// (point-Jacobian column at the contact point, joint velocity, 1/M~).
struct SideReg {
  int kind, idx;
  f3 x, v, w, col;
  float im, qv;
  // symmetric world inverse inertia (xx yy zz xy xz yz), named scalars so
  // that the whole side stays in registers
  float i0, i1, i2, i3, i4, i5;
};
__device__ __forceinline__ void side_load(const float* F, const float* A, int sv, f3 p, SideReg& S) {
  S.kind = side_kind(sv);
  S.idx = side_idx(sv);
  S.x = S.v = S.w = S.col = mk3(0.f, 0.f, 0.f);
  S.im = S.qv = 0.f;
  S.i0 = S.i1 = S.i2 = S.i3 = S.i4 = S.i5 = 0.f;
  if (S.kind == K_FREE) {
    const float* f = F + S.idx * FSTR;
    S.x = mk3(f[F_X], f[F_X + 1], f[F_X + 2]);
    S.v = mk3(f[F_V], f[F_V + 1], f[F_V + 2]);
    S.w = mk3(f[F_W], f[F_W + 1], f[F_W + 2]);
    S.im = f[F_IM];
    S.i0 = f[F_II + 0];
    S.i1 = f[F_II + 1];
    S.i2 = f[F_II + 2];
    S.i3 = f[F_II + 3];
    S.i4 = f[F_II + 4];
    S.i5 = f[F_II + 5];
  } else if (S.kind == K_AUX) {
    S.col = aux_col(A, S.idx, p);
    S.qv = A[A_V * AMAX + S.idx];
    S.im = A[A_IM * AMAX + S.idx];
  }
}
// velocity of the contact point p of a side
__device__ __forceinline__ f3 side_vel(const SideReg& S, f3 p) {
  if (S.kind == K_FREE) return S.v + cross(S.w, p - S.x);
  if (S.kind == K_AUX) return S.col * S.qv;
  return mk3(0.f, 0.f, 0.f);
}
// apply the impulse P at p
__device__ __forceinline__ void side_impulse(SideReg& S, f3 p, f3 P) {
  if (S.kind == K_FREE) {
    const f3 q = cross(p - S.x, P);
    S.v = S.v + P * S.im;
    S.w = S.w + mk3(S.i0 * q.x + S.i3 * q.y + S.i4 * q.z, S.i3 * q.x + S.i1 * q.y + S.i5 * q.z,
                    S.i4 * q.x + S.i5 * q.y + S.i2 * q.z);
  } else if (S.kind == K_AUX) {
    S.qv += dot(S.col, P) * S.im;
  }
}
__device__ __forceinline__ void side_store(float* F, float* A, const SideReg& S) {
  if (S.kind == K_FREE) {
    float* f = F + S.idx * FSTR;
    f[F_V] = S.v.x; f[F_V + 1] = S.v.y; f[F_V + 2] = S.v.z;
    f[F_W] = S.w.x; f[F_W + 1] = S.w.y; f[F_W + 2] = S.w.z;
  } else if (S.kind == K_AUX) {
    A[A_V * AMAX + S.idx] = S.qv;
  }
}
// friction pair: Jacobi step on both tangent rows from the same velocity,
// then projection onto the disk of radius mu * lambda_n
__device__ __forceinline__ void friction_disk(float l1, float l2, float r1, float r2, float iw1, float iw2, float lim,
                                              float& y1, float& y2) {
  y1 = l1 - r1 * iw1;
  y2 = l2 - r2 * iw2;
  const float nn = y1 * y1 + y2 * y2;
  // outside the disk: scaled onto it (onto 0 for a radius of 0); selects,
  // not branches, so the lanes of a level do not split
  const float sc = nn > lim * lim ? (lim > 0.f ? lim * rsqrtf(nn) : 0.f) : 1.f;
  y1 *= sc;
  y2 *= sc;
}

__device__ __forceinline__ void phase_pgs(const KArgs& a, const Scene& S, float* L, int NC, int NL, int maxl,
                                          float& vR, float* tape) {
  const int lane = lane_id();
  const LdsLayout& Y = a.L;
  float* C = L + Y.con;
  const int cc = Y.ccap;
  float* F = L + Y.fr;
  float* A = L + Y.aux;
  const float* Rw = L + Y.rows;
  const uint16_t* loff = reinterpret_cast<const uint16_t*>(L + Y.lvl);
  const uint16_t* rob = loff + cc + 2;
  const uint32_t* order = reinterpret_cast<const uint32_t*>(rob + cc + 2);
  const float mu = a.mu;
  const int j = lane & 15;
  // w = M~^-1 J^T of the first robot rows, kept over the sweeps: in the
  // robot's sphere centres and the culling lists (both dead until the next
  // substep's kinematics and contacts)
  float* wcA = L + Y.sph;
  float* wcB = L + Y.cand;
  const int wc1 = (Y.fr - Y.sph) / ROW_FLOATS, wc2 = (Y.frc - Y.cand) / ROW_FLOATS;
  const float* Minv = robot_view(L + Y.robot, L + Y.dyn).Minv;
  // the zero record's velocities (kept zero by every update that uses it)
  if (lane < 6) F[Y.fmax * FSTR + F_V + lane] = 0.f;
  wave_sync();
#pragma unroll 1
  for (int it = 0; it < a.K; ++it) {
    int o1 = 0;  // a level's rows start where the previous level's end
#pragma unroll 1
    for (int lv = 1; lv <= maxl; ++lv) {
      const int rc = rob[lv] == 0xffff ? -1 : (int)rob[lv];
      const int o0 = o1;
      o1 = loff[lv];
      if (rc >= 0) {
        // the level's robot row: lane j of each 16-lane row holds joint
        // velocity j; row d < 3 of the wave forms J_d . v in one reduction
        const float* row = Rw + (rc - NL) * ROW_FLOATS;
        const float* c = C + rc * CSTR;
        int info = __float_as_int(c[C_INFO]);
        f3 n = mk3(c[C_N], c[C_N + 1], c[C_N + 2]);
        f3 p = mk3(c[C_P], c[C_P + 1], c[C_P + 2]);
        float iw0 = c[C_IW], iw1 = c[C_IW + 1], iw2 = c[C_IW + 2];
        float bias = c[C_BIAS];
        float l0 = c[C_LAM], l1 = c[C_LAM + 1], l2 = c[C_LAM + 2];
        const float wtn1 = c[C_WTN], wtn2 = c[C_WTN + 1];
        const int dr = lane >> 4;
        const float Jd = row[(dr < 3 ? dr : 2) * ND + j];
        // lane j's entries of w = M~^-1 J^T: formed in the first sweep (M~^-1
        // is symmetric, so lane j reads its column: consecutive across the
        // lanes, no bank conflicts) and kept for the later ones where LDS
        // that is dead during the sweeps has room
        float wn = 0.f, w1 = 0.f, w2 = 0.f;
        const int rr = rc - NL;
        float* wc = rr < wc1 ? wcA + rr * ROW_FLOATS : (rr < wc1 + wc2 ? wcB + (rr - wc1) * ROW_FLOATS : nullptr);
        if (it == 0 || wc == nullptr) {
#pragma unroll 8
          for (int k = 0; k < ND; ++k) {
            const float m = Minv[k * ND + j];
            wn += m * row[k];
            w1 += m * row[ND + k];
            w2 += m * row[2 * ND + k];
          }
          if (wc != nullptr && dr < 3) wc[lane] = dr == 0 ? wn : (dr == 1 ? w1 : w2);
        } else {
          wn = wc[j];
          w1 = wc[ND + j];
          w2 = wc[2 * ND + j];
        }
        f3 t1, t2;
        onb_a(n, c[C_ONB], t1, t2);
        SideReg B;
        side_load(F, A, (info >> 16) & 0xffff, p, B);
        const float dsum = sum16(dr < 3 ? Jd * vR : 0.f);
        const float dn = lane_val(dsum, 0), d1 = lane_val(dsum, ND), d2 = lane_val(dsum, 2 * ND);
        const f3 uB = side_vel(B, p);
        float r = dn - dot(n, uB) + bias;
        float nl = l0;
        if (iw0 > 0.f) nl = fmaxf(0.f, l0 - r * iw0);
        if (tape && lane == 0) tape[it * a.RL.tsw + rc * 3] = l0 - r * iw0;
        const float dl = nl - l0;
        float dl1 = 0.f, dl2 = 0.f;
        if (iw1 > 0.f && iw2 > 0.f) {
          // the friction pair sees the velocity after the normal update:
          // t . u + dl (t . K n), the couplings of both sides from the rows
          // phase; the impulses are then applied together
          const float u1 = d1 - dot(t1, uB) + dl * wtn1, u2 = d2 - dot(t2, uB) + dl * wtn2;
          float y1, y2;
          friction_disk(l1, l2, u1, u2, iw1, iw2, mu * nl, y1, y2);
          if (tape && lane == 0) {
            tape[it * a.RL.tsw + rc * 3 + 1] = l1 - u1 * iw1;
            tape[it * a.RL.tsw + rc * 3 + 2] = l2 - u2 * iw2;
          }
          dl1 = y1 - l1;
          dl2 = y2 - l2;
          l1 = y1;
          l2 = y2;
        }
        vR += wn * dl + w1 * dl1 + w2 * dl2;
        side_impulse(B, p, (n * dl + t1 * dl1 + t2 * dl2) * (-1.f));
        if (lane == 0) {
          side_store(F, A, B);
          float* cw = C + rc * CSTR;
          cw[C_LAM] = nl;
          cw[C_LAM + 1] = l1;
          cw[C_LAM + 2] = l2;
        }
        // the per-lane rows below touch other nodes; the fence also keeps the
        // robot row's registers from living into them
        lds_order();
      }
      // the level's other rows, one lane each (they share no node)
#pragma unroll 1
      for (int e = o0 + lane; e < o1; e += WAVE) {
        const uint32_t ge = order[e];
        const int gn = ge >> 16;
        if (gn > 1) {
          // a group: consecutive rows between one free body and static
          // targets, in order, with the body's velocities in registers
          const int c0 = ge & 0xffff;
          float* fa = F + side_idx(__float_as_int(C[c0 * CSTR + C_INFO]) & 0xffff) * FSTR;
          const f3 xa = mk3(fa[F_X], fa[F_X + 1], fa[F_X + 2]);
          f3 va = mk3(fa[F_V], fa[F_V + 1], fa[F_V + 2]), wa = mk3(fa[F_W], fa[F_W + 1], fa[F_W + 2]);
          const float ima = fa[F_IM];
          const float i0 = fa[F_II], i1 = fa[F_II + 1], i2 = fa[F_II + 2], i3 = fa[F_II + 3], i4 = fa[F_II + 4],
                      i5 = fa[F_II + 5];
#pragma unroll 1
          for (int ci = c0; ci < c0 + gn; ++ci) {
            float* c = C + ci * CSTR;
            const f3 n = mk3(c[C_N], c[C_N + 1], c[C_N + 2]);
            const f3 p = mk3(c[C_P], c[C_P + 1], c[C_P + 2]);
            const float iw0 = c[C_IW], iw1 = c[C_IW + 1], iw2 = c[C_IW + 2], bias = c[C_BIAS];
            const float l0 = c[C_LAM];
            float l1 = c[C_LAM + 1], l2 = c[C_LAM + 2];
            const f3 ra = p - xa;
            const f3 u = va + cross(wa, ra);
            const float r = dot(n, u) + bias;
            float nl = l0;
            if (iw0 > 0.f) nl = fmaxf(0.f, l0 - r * iw0);
            if (tape) tape[it * a.RL.tsw + ci * 3] = l0 - r * iw0;
            const float dl = nl - l0;
            f3 P = n * dl;
            if (iw1 > 0.f && iw2 > 0.f) {
              f3 t1, t2;
              onb_a(n, c[C_ONB], t1, t2);
              const float u1 = dot(t1, u) + dl * c[C_WTN], u2 = dot(t2, u) + dl * c[C_WTN + 1];
              float y1, y2;
              friction_disk(l1, l2, u1, u2, iw1, iw2, mu * nl, y1, y2);
              if (tape) {
                tape[it * a.RL.tsw + ci * 3 + 1] = l1 - u1 * iw1;
                tape[it * a.RL.tsw + ci * 3 + 2] = l2 - u2 * iw2;
              }
              P = P + t1 * (y1 - l1) + t2 * (y2 - l2);
              l1 = y1;
              l2 = y2;
            }
            const f3 q = cross(ra, P);
            va = va + P * ima;
            wa = wa + mk3(i0 * q.x + i3 * q.y + i4 * q.z, i3 * q.x + i1 * q.y + i5 * q.z, i4 * q.x + i5 * q.y + i2 * q.z);
            c[C_LAM] = nl;
            c[C_LAM + 1] = l1;
            c[C_LAM + 2] = l2;
          }
          fa[F_V] = va.x; fa[F_V + 1] = va.y; fa[F_V + 2] = va.z;
          fa[F_W] = wa.x; fa[F_W + 1] = wa.y; fa[F_W + 2] = wa.z;
          continue;
        }
        const int ci = ge & 0xffff;
        float* c = C + ci * CSTR;
        const int info = __float_as_int(c[C_INFO]);
        const int sA = info & 0xffff, sB = (info >> 16) & 0xffff;
        float bias = c[C_BIAS];
        float l0 = c[C_LAM];
        if (side_kind(sA) == K_LIMIT) {
          int x = side_idx(sA);
          float sg = ((info >> 16) & 1) ? -1.f : 1.f;
          float iwl = c[C_IW];  // = 1 / W
          float r = sg * A[A_V * AMAX + x] + bias;
          float nl = fmaxf(0.f, l0 - r * iwl);
          if (tape) tape[it * a.RL.tsw + ci * 3] = l0 - r * iwl;
          A[A_V * AMAX + x] += sg * A[A_IM * AMAX + x] * (nl - l0);
          c[C_LAM] = nl;
          continue;
        }
        // side A is a free body (the owner); side B a free body, a door /
        // drawer or static.  A static B reads and writes the zero record past
        // the scene's free bodies (no mass, no velocity), so both sides run
        // the same loads and arithmetic without branches; a door / drawer
        // adds its joint's part in a branch of its own.
        const f3 n = mk3(c[C_N], c[C_N + 1], c[C_N + 2]);
        const f3 p = mk3(c[C_P], c[C_P + 1], c[C_P + 2]);
        const float iw0 = c[C_IW], iw1 = c[C_IW + 1], iw2 = c[C_IW + 2];
        float l1 = c[C_LAM + 1], l2 = c[C_LAM + 2];
        const int kB = side_kind(sB), xi = side_idx(sB);
        float* fa = F + side_idx(sA) * FSTR;
        float* fb = F + (kB == K_FREE ? xi : Y.fmax) * FSTR;
        const f3 xa = mk3(fa[F_X], fa[F_X + 1], fa[F_X + 2]), xb = mk3(fb[F_X], fb[F_X + 1], fb[F_X + 2]);
        f3 va = mk3(fa[F_V], fa[F_V + 1], fa[F_V + 2]), wa = mk3(fa[F_W], fa[F_W + 1], fa[F_W + 2]);
        f3 vb = mk3(fb[F_V], fb[F_V + 1], fb[F_V + 2]), wb = mk3(fb[F_W], fb[F_W + 1], fb[F_W + 2]);
        const f3 ra = p - xa, rb = p - xb;
        f3 u = (va + cross(wa, ra)) - (vb + cross(wb, rb));
        f3 col = mk3(0.f, 0.f, 0.f);
        float qv = 0.f, imx = 0.f;
        if (kB == K_AUX) {
          col = aux_col(A, xi, p);
          qv = A[A_V * AMAX + xi];
          imx = A[A_IM * AMAX + xi];
          u = u - col * qv;
        }
        float r = dot(n, u) + bias;
        float nl = l0;
        if (iw0 > 0.f) nl = fmaxf(0.f, l0 - r * iw0);
        if (tape) tape[it * a.RL.tsw + ci * 3] = l0 - r * iw0;
        float dl = nl - l0;
        f3 P = n * dl;
        if (iw1 > 0.f && iw2 > 0.f) {
          // the friction pair sees the velocity after the normal update: its
          // tangential parts are t . u + dl (t . K n), with the couplings
          // t . K n of the two sides' inverse inertias from the rows phase;
          // the normal and friction impulses are then applied together
          f3 t1, t2;
          onb_a(n, c[C_ONB], t1, t2);
          const float u1 = dot(t1, u) + dl * c[C_WTN], u2 = dot(t2, u) + dl * c[C_WTN + 1];
          float y1, y2;
          friction_disk(l1, l2, u1, u2, iw1, iw2, mu * nl, y1, y2);
          if (tape) {
            tape[it * a.RL.tsw + ci * 3 + 1] = l1 - u1 * iw1;
            tape[it * a.RL.tsw + ci * 3 + 2] = l2 - u2 * iw2;
          }
          P = P + t1 * (y1 - l1) + t2 * (y2 - l2);
          l1 = y1;
          l2 = y2;
        }
        {
          const float ima = fa[F_IM], imb = fb[F_IM];
          const f3 qa = cross(ra, P), qb = cross(rb, P);
          const float* ia = fa + F_II;
          const float* ib = fb + F_II;
          va = va + P * ima;
          wa = wa + mk3(ia[0] * qa.x + ia[3] * qa.y + ia[4] * qa.z, ia[3] * qa.x + ia[1] * qa.y + ia[5] * qa.z,
                        ia[4] * qa.x + ia[5] * qa.y + ia[2] * qa.z);
          vb = vb - P * imb;
          wb = wb - mk3(ib[0] * qb.x + ib[3] * qb.y + ib[4] * qb.z, ib[3] * qb.x + ib[1] * qb.y + ib[5] * qb.z,
                        ib[4] * qb.x + ib[5] * qb.y + ib[2] * qb.z);
          fa[F_V] = va.x; fa[F_V + 1] = va.y; fa[F_V + 2] = va.z;
          fa[F_W] = wa.x; fa[F_W + 1] = wa.y; fa[F_W + 2] = wa.z;
          fb[F_V] = vb.x; fb[F_V + 1] = vb.y; fb[F_V + 2] = vb.z;
          fb[F_W] = wb.x; fb[F_W + 1] = wb.y; fb[F_W + 2] = wb.z;
          if (kB == K_AUX) A[A_V * AMAX + xi] = qv - dot(col, P) * imx;
        }
        c[C_LAM] = nl;
        c[C_LAM + 1] = l1;
        c[C_LAM + 2] = l2;
      }
      lds_order();
    }
  }
}

__device__ __forceinline__ void phase_integrate(const KArgs& a, const Scene& S, float* L, const Robot& rb, float vR) {
  const int lane = lane_id();
  if (lane < ND) {
    rb.qd[lane] = vR;
    if (lane < S.nb) rb.q[lane] += a.h * vR;
  }
  float* F = L + a.L.fr;
  const int fm = a.L.fmax;
  for (int f = lane; f < S.nf; f += WAVE) {
    f3 v = mk3(F[(f) * FSTR + F_V + 0], F[(f) * FSTR + F_V + 1], F[(f) * FSTR + F_V + 2]);
    f3 w = mk3(F[(f) * FSTR + F_W + 0], F[(f) * FSTR + F_W + 1], F[(f) * FSTR + F_W + 2]);
    F[(f) * FSTR + F_X + 0] += a.h * v.x;
    F[(f) * FSTR + F_X + 1] += a.h * v.y;
    F[(f) * FSTR + F_X + 2] += a.h * v.z;
    f3 th = w * a.h;
    float n2 = dot(th, th);
    float cw, sk;
    if (n2 < 1e-12f) {
      cw = 1.f - n2 * 0.125f;
      sk = 0.5f - n2 * (1.f / 48.f);
    } else {
      float nn = sqrtf(n2);
      cw = cosf(0.5f * nn);
      sk = sinf(0.5f * nn) / nn;
    }
    float e0 = cw, e1 = th.x * sk, e2 = th.y * sk, e3 = th.z * sk;
    float q0 = F[(f) * FSTR + F_Q + 0], q1 = F[(f) * FSTR + F_Q + 1], q2 = F[(f) * FSTR + F_Q + 2],
          q3 = F[(f) * FSTR + F_Q + 3];
    float r0 = e0 * q0 - (e1 * q1 + e2 * q2 + e3 * q3);
    float r1 = e0 * q1 + q0 * e1 + (e2 * q3 - e3 * q2);
    float r2 = e0 * q2 + q0 * e2 + (e3 * q1 - e1 * q3);
    float r3 = e0 * q3 + q0 * e3 + (e1 * q2 - e2 * q1);
    float inv = 1.f / sqrtf(r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3);
    F[(f) * FSTR + F_Q + 0] = r0 * inv;
    F[(f) * FSTR + F_Q + 1] = r1 * inv;
    F[(f) * FSTR + F_Q + 2] = r2 * inv;
    F[(f) * FSTR + F_Q + 3] = r3 * inv;
  }
  float* A = L + a.L.aux;
  if (lane < S.na) {
    float v = A[A_V * AMAX + lane];
    A[A_QD * AMAX + lane] = v;
    A[A_Q * AMAX + lane] += a.h * v;
  }
  wave_sync();
}

// Contact-force outputs of a substep: the sum of the robot's normal impulses
// / h (all lanes hold it), and per free body the force the robot's contacts
// exert on it (the negative of the impulse on the robot side, / h),
// accumulated in the body's record.
__device__ __forceinline__ void phase_forces(const KArgs& a, const Scene& S, float* L, int NL, int NR, float& frc,
                                             bool last) {
  const int lane = lane_id();
  const float* C = L + a.L.con;
  float* FR = L + a.L.frc;
  if (a.grip) {
    // gripper contacts, one lane per free body / door-drawer joint: the
    // normal force of the end effector's bodies on it (accumulated), and in
    // the last substep the smaller of the two fingers' normal forces on it
    float* A = L + a.L.aux;
    for (int o = lane; o < S.nf + S.na; o += WAVE) {
      const bool isf = o < S.nf;
      const int want = isf ? ((K_FREE << 8) | o) : ((K_AUX << 8) | (o - S.nf));
      float fe = 0.f, fl = 0.f, fr = 0.f;
      for (int ci = NL; ci < NL + NR; ++ci) {
        const float* c = C + ci * CSTR;
        const int info = __float_as_int(c[C_INFO]);
        if (((info >> 16) & 0xffff) != want) continue;
        const int body = side_idx(info & 0xffff);  // a robot side carries its body
        const float fn = c[C_LAM] / a.h;
        if ((a.grip_ee >> body) & 1u) fe += fn;
        if (body == a.grip_fl) fl += fn;
        if (body == a.grip_fr) fr += fn;
      }
      if (isf) {
        FR[o * FRC_FLOATS + R_EE] += fe;
        if (last) FR[o * FRC_FLOATS + R_FMIN] = fminf(fl, fr);
      } else {
        A[A_EE * AMAX + o - S.nf] += fe;
        if (last) A[A_FMIN * AMAX + o - S.nf] = fminf(fl, fr);
      }
    }
  }
  if (!a.frc_robot) {
    wave_sync();
    return;
  }
  float part = 0.f;
  for (int ci = NL + lane; ci < NL + NR; ci += WAVE) part += C[ci * CSTR + C_LAM];
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, WAVE);
  frc += part / a.h;
  if (lane == 0) {
    for (int ci = NL; ci < NL + NR; ++ci) {
      const float* c = C + ci * CSTR;
      int bside = (__float_as_int(c[C_INFO]) >> 16) & 0xffff;
      if (side_kind(bside) != K_FREE) continue;
      int g = side_idx(bside);
      f3 n = mk3(c[C_N], c[C_N + 1], c[C_N + 2]), t1, t2;
      onb(n, t1, t2);
      f3 P = n * c[C_LAM] + t1 * c[C_LAM + 1] + t2 * c[C_LAM + 2];
      FR[(g) * FRC_FLOATS + R_FRC + 0] -= P.x / a.h;
      FR[(g) * FRC_FLOATS + R_FRC + 1] -= P.y / a.h;
      FR[(g) * FRC_FLOATS + R_FRC + 2] -= P.z / a.h;
    }
  }
  wave_sync();
}

// MODE 0: the plain step; 1: also the record of the control step for the
// adjoint; 2: also the contact-force outputs.  Separate instantiations, so
// the plain step keeps its register allocation.
template <int MODE>
__device__ __forceinline__ void run_scene(const KArgs& a, int s, float* L) {
  constexpr bool REC = MODE == 1;
  const int lane = lane_id();
  Scene S;
  const DScene ds = a.scenes[s];
  S.s = s;
  S.M = a.models + ds.model;
  S.nb = S.M->nb;
  S.nsph = S.M->nsph;
  S.nf = ds.nf; S.ns = ds.ns; S.np = ds.np; S.na = ds.na; S.nfo = ds.nown;
  S.f0 = ds.f0; S.s0 = ds.s0; S.p0 = ds.p0; S.a0 = ds.a0;
  S.hold = a.scenes[s].hold;
  {
    const float* g = a.sgrid + (size_t)sgrid_floats(a.sg_nw) * s;
    S.gx0 = g[0];
    S.gy0 = g[1];
    S.gix = g[2];
    S.giy = g[3];
  }
  Robot rb = robot_view(L + a.L.robot, L + a.L.dyn);
  const unsigned long long t_scene = a.cost ? clock64() : 0ull;
  const bool prof = a.phase_cycles != nullptr;
  unsigned long long cyc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long tc = prof ? clock64() : 0;
#define MS_PHASE(k)                          \
  if (prof) {                                \
    unsigned long long t2 = clock64();       \
    cyc[k] += t2 - tc;                       \
    tc = t2;                                 \
  }
  load_scene(a, S, L, rb);
  MS_PHASE(7)
  uint32_t status = 0;
  float frc = 0.f;
  if (MODE == 2) {
    // the force sums of the control step: a launch that resumes the step
    // (a.sub0 > 0) continues the sums so far, so that they add up in the
    // order of one launch over the whole step
    float* FR = L + a.L.frc;
    float* A = L + a.L.aux;
    const bool resume = a.sub0 > 0;
    for (int f = lane; f < S.nf; f += WAVE) {
      for (int t = 0; t < FRC_FLOATS; ++t) FR[(f) * FRC_FLOATS + t] = 0.f;
      if (resume && a.frc_body)
        for (int t = 0; t < 3; ++t) FR[(f) * FRC_FLOATS + R_FRC + t] = a.frc_body[(size_t)(S.f0 + f) * 4 + t];
      if (resume && a.grip) FR[(f) * FRC_FLOATS + R_EE] = a.grip[2 * (size_t)(S.f0 + f)];
    }
    if (lane < S.na) {
      A[A_EE * AMAX + lane] = resume && a.grip ? a.grip[2 * ((size_t)a.NF + S.a0 + lane)] : 0.f;
      A[A_FMIN * AMAX + lane] = 0.f;
    }
    if (resume && a.frc_robot) frc = a.frc_robot[s];
    wave_sync();
  }
  float* rec = REC ? a.rec + (size_t)s * a.RL.total : nullptr;
  // the largest contact lists of the step, for the next step's routing
  int max_nc = 0, max_nr = 0;
  for (int k = 0; k < a.n_sub; ++k) {
    int NC, NR, NL;
    uint64_t keysum = 0;
    float vR;
    const int ks = a.sub0 + k;
    if (rec) rec_state(a, S, L, rb, rec + ks * a.RL.ss);
    phase_drive(a, S, rb);
    phase_kinematics(a, S, L, rb);
    MS_PHASE(0)
    // unconstrained dynamics first: it needs only the frames, and its
    // articulated-body scratch is dead before the contact list is written
    // into the same LDS
    phase_dynamics(a, S, L, rb, vR);
    MS_PHASE(2)
    phase_contacts(a, S, L, rb, NC, NR, NL, status, keysum);
    // a launch in a smaller layout gives up a scene at its first overflowing
    // contact list; everything written so far the retry writes again alike
    if (a.fit_mode == 1 && (status & 10u)) break;
    if (rec) rec_contacts(a, L, NC, NL, NR, rec + a.RL.con + ks * a.RL.cstride);
    max_nc = max(max_nc, NC - NL);
    max_nr = max(max_nr, NR);
    MS_PHASE(1)
    phase_rows(a, S, L, rb, NC, NR, NL, status);
    MS_PHASE(3)
    int maxl = phase_levels(a, L, NC, NR, NL);
    MS_PHASE(4)
    phase_pgs(a, S, L, NC, NL, maxl, vR, rec ? rec + a.RL.tape + (size_t)ks * a.K * a.RL.tsw : nullptr);
    if (MODE == 2) phase_forces(a, S, L, NL, NR, frc, ks == a.n_sub_total - 1);
    MS_PHASE(5)
    phase_integrate(a, S, L, rb, vR);
    MS_PHASE(6)
    if (rec && ks == a.n_sub_total - 1) rec_state(a, S, L, rb, rec + (ks + 1) * a.RL.ss);
    if (a.debug && lane == 0) {
      uint32_t* d = a.debug + ((size_t)s * a.n_sub_total + a.sub0 + k) * 4;
      d[0] = (uint32_t)(NC - NL);
      d[1] = (uint32_t)NR;
      d[2] = (uint32_t)keysum;
      d[3] = (uint32_t)(keysum >> 32);
    }
  }
  // a launch in a smaller layout stores nothing of a scene whose lists
  // overflowed it: the retry launch steps it again in the full layout, from
  // the unchanged input state
  if (a.fit_mode == 1 && (status & 10u)) {
    if (lane == 0) a.retry[1 + atomicAdd(a.retry, 1)] = s;
    return;
  }
  store_scene(a, S, L, rb, status);
  if (MODE == 2 && a.grip) {
    const float* FR = L + a.L.frc;
    const float* A = L + a.L.aux;
    const bool last = a.sub0 + a.n_sub == a.n_sub_total;
    for (int o = lane; o < S.nf + S.na; o += WAVE) {
      const bool isf = o < S.nf;
      float* dst = a.grip + 2 * (isf ? (size_t)(S.f0 + o) : (size_t)a.NF + S.a0 + (o - S.nf));
      const float fe = isf ? FR[o * FRC_FLOATS + R_EE] : A[A_EE * AMAX + o - S.nf];
      dst[0] = fe;
      if (last) dst[1] = isf ? FR[o * FRC_FLOATS + R_FMIN] : A[A_FMIN * AMAX + o - S.nf];
    }
  }
  if (MODE == 2 && a.frc_robot) {
    const float* FR = L + a.L.frc;
    if (lane == 0) a.frc_robot[s] = frc;
    for (int f = lane; f < S.nf; f += WAVE) {
      float* dst = a.frc_body + (size_t)(S.f0 + f) * 4;
      for (int t = 0; t < 3; ++t) {
        float v = FR[(f) * FRC_FLOATS + R_FRC + t];
        dst[t] = v;
      }
      dst[3] = 0.f;
    }
  }
  MS_PHASE(7)
#undef MS_PHASE
  if (lane == 0) {
    if (a.sub0 == 0) a.status[s] = status;
    else a.status[s] |= status;
    if (a.cost) {
      // the scene's time in this launch (shader clock / 16) orders the next
      // step: a scene's time changes little from one step to the next
      const long long dt = (long long)((clock64() - t_scene) >> 4);
      const long long v = a.sub0 == 0 ? dt : (long long)a.cost[s] + dt;
      a.cost[s] = (int)(v < 0x7fffffffLL ? v : 0x7fffffffLL);
    }
    if (a.maxc) {
      const int m = a.sub0 == 0 ? 0 : a.maxc[s];
      a.maxc[s] = max(m & 0xffff, max_nc) | (max(m >> 16, max_nr) << 16);
    }
    if (prof) {
      for (int k = 0; k < 8; ++k) {
        if (a.sub0 == 0) a.phase_cycles[(size_t)s * 8 + k] = cyc[k];
        else a.phase_cycles[(size_t)s * 8 + k] += cyc[k];
      }
    }
  }
}

template <int MODE>
__device__ __forceinline__ void step_body(const KArgs& a, float* lds) {
  // one call site: the persistent form pulls positions from its work
  // counter, the plain form takes its block index once
  const int qi = a.fit_mode == 2 ? 1 : (a.fit_mode == 3 ? 2 : 0);
  const int base = a.fit_mode == 1 ? *a.n_over : 0;
  const int end = a.fit_mode == 2 ? *a.n_over : (a.fit_mode == 3 ? a.retry[0] : a.S);
  int pos = a.persistent ? 0 : base + (int)blockIdx.x;
  for (;;) {
    if (a.persistent) {
      int got = 0;
      if (threadIdx.x == 0) got = atomicAdd(a.queue + qi, 1);
      pos = base + __shfl(got, 0, WAVE);
    }
    if (pos >= end) break;
    run_scene<MODE>(a, a.fit_mode == 3 ? a.retry[1 + pos] : a.order[pos], lds);
    if (!a.persistent) break;
    __syncthreads();
  }
}

__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_step(KArgs a) {
  extern __shared__ float lds[];
  step_body<0>(a, lds);
}
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_step_rec(KArgs a) {
  extern __shared__ float lds[];
  step_body<1>(a, lds);
}
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_step_frc(KArgs a) {
  extern __shared__ float lds[];
  step_body<2>(a, lds);
}

__global__ void k_reset_queue(int* q) {
  if (threadIdx.x == 0) q[0] = 0;
}

// Spawn check of a reset: collide[s] = 1 where a robot sphere penetrates
// (phi < 0) another body; every (robot sphere, target) pair is tested with
// the contact phase's pair function and a zero margin.
__global__ __launch_bounds__(WAVE) void k_spawn_check(KArgs a, uint8_t* collide) {
  extern __shared__ float lds[];
  const int s = blockIdx.x;
  if (s >= a.S) return;
  const int lane = lane_id();
  Scene S;
  const DScene ds = a.scenes[s];
  S.s = s;
  S.M = a.models + ds.model;
  S.nb = S.M->nb;
  S.nsph = S.M->nsph;
  S.nf = ds.nf; S.ns = ds.ns; S.np = ds.np; S.na = ds.na; S.nfo = ds.nown;
  S.f0 = ds.f0; S.s0 = ds.s0; S.p0 = ds.p0; S.a0 = ds.a0;
  S.hold = a.scenes[s].hold;
  float* L = lds;
  Robot rb = robot_view(L + a.L.robot, L + a.L.dyn);
  load_scene(a, S, L, rb);
  phase_kinematics(a, S, L, rb);
  const LdsLayout& Y = a.L;
  ConCtx X;
  X.M = S.M;
  X.C = L + Y.con;
  X.cc = Y.ccap;
  X.SW = L + Y.sph;
  X.F = L + Y.fr;
  X.fm = Y.fmax;
  X.A = L + Y.aux;
  X.Pl = L + Y.plane;
  X.own = reinterpret_cast<const uint16_t*>(L + Y.own);
  X.St = Y.smax > 0 ? (L + Y.stat) : (a.statics + (size_t)S.s0 * 6);
  X.nsph = S.nsph; X.np = S.np; X.ns = S.ns; X.na = S.na; X.nf = S.nf;
  X.NT = S.np + S.ns + S.na + S.nf;
  X.margin = 0.f;
  X.hash = false;
  const int NT = X.NT, total = S.nsph * NT;
  const float invNT = NT > 0 ? 1.f / (float)NT : 0.f;
  bool hit = false;
  for (int base = 0; base < total; base += WAVE) {
    int pair = base + lane;
    if (pair < total) {
      int o, t;
      divmod(pair, NT, invNT, o, t);
      PairOut po;
      bool isrob;
      hit |= eval_pair(X, o, t, po, isrob);
    }
  }
  uint64_t any = __ballot(hit);
  if (lane == 0) collide[s] = any ? 1 : 0;
}

// Robot resets of the masked scenes: q = base + clip(noise, -c_j, c_j), qd = 0.
struct Clip16 {
  float c[ND];
};
__global__ void k_reset_robots(float* x, const uint8_t* mask, const float* base, const float* noise, Clip16 clip,
                               int S) {
  const int s = blockIdx.x * 4 + (threadIdx.x >> 4), j = threadIdx.x & 15;
  if (s >= S || (mask && !mask[s])) return;
  const size_t i = (size_t)s * ND + j;
  x[i] = base[i] + fminf(fmaxf(noise[i], -clip.c[j]), clip.c[j]);
  x[(size_t)S * ND + i] = 0.f;
}

// Normalized actions (clipped to [-1, 1]) to PD targets from the state at the
// control step's start: joint delta position, base linear velocity along the
// heading (world x and y shares), base angular velocity, gripper opening.
// One thread per (scene, DoF).
__device__ __forceinline__ float clip_unit(float a) { return fminf(fmaxf(a, -1.f), 1.f); }
__global__ void k_actions(const DModel* models, const DScene* scenes, const float* x, const float* a, float* tgt,
                          int S) {
  const int s = blockIdx.x * 4 + (threadIdx.x >> 4), j = threadIdx.x & 15;
  if (s >= S) return;
  const DModel& M = models[scenes[s].model];
  const float* q = x + (size_t)s * ND;
  const float* as = a + (size_t)s * ND;
  float t = 0.f;
  if (j < M.nb) {
    const float sc = M.act_scale[j], aj = clip_unit(as[j]);
    const float yaw = M.act_yaw >= 0 ? q[M.act_yaw] : 0.f;
    switch (M.act_kind[j]) {
      case 0: t = q[j] + aj * sc; break;
      case 1: t = M.act_yaw >= 0 ? aj * sc * cosf(yaw) : aj * sc; break;
      case 2: t = (M.act_x >= 0 && M.act_yaw >= 0) ? clip_unit(as[M.act_x]) * sc * sinf(yaw) : 0.f; break;
      case 3: t = aj * sc; break;
      default: t = (aj + 1.f) * 0.5f * sc; break;
    }
  }
  tgt[(size_t)s * ND + j] = t;
}
// Reverse of k_actions: given the adjoint of the targets, writes the adjoint of
// the actions and adds the targets' dependence on the start state into the
// state adjoint's joint positions.  One thread per scene.
__global__ void k_actions_bwd(const DModel* models, const DScene* scenes, const float* x, const float* a,
                              const float* gtgt, float* ga, float* gx, int S) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const DModel& M = models[scenes[s].model];
  const float* q = x + (size_t)s * ND;
  const float* as = a + (size_t)s * ND;
  const float* gt = gtgt + (size_t)s * ND;
  float gav[ND], gq[ND];
  for (int j = 0; j < ND; ++j) gav[j] = gq[j] = 0.f;
  const float yaw = M.act_yaw >= 0 ? q[M.act_yaw] : 0.f;
  const float cy = cosf(yaw), sy = sinf(yaw);
  for (int j = 0; j < M.nb; ++j) {
    const float sc = M.act_scale[j], g = gt[j];
    const bool in = as[j] >= -1.f && as[j] <= 1.f;  // the clip's slope (1 on the boundary)
    switch (M.act_kind[j]) {
      case 0:
        gq[j] += g;
        if (in) gav[j] += g * sc;
        break;
      case 1:
        if (M.act_yaw >= 0) {
          if (in) gav[j] += g * sc * cy;
          gq[M.act_yaw] -= g * clip_unit(as[j]) * sc * sy;
        } else if (in) {
          gav[j] += g * sc;
        }
        break;
      case 2:
        if (M.act_x >= 0 && M.act_yaw >= 0) {
          const float ax = as[M.act_x];
          if (ax >= -1.f && ax <= 1.f) gav[M.act_x] += g * sc * sy;
          gq[M.act_yaw] += g * clip_unit(ax) * sc * cy;
        }
        break;
      case 3:
        if (in) gav[j] += g * sc;
        break;
      default:
        if (in) gav[j] += g * 0.5f * sc;
        break;
    }
  }
  for (int j = 0; j < ND; ++j) {
    ga[(size_t)s * ND + j] = gav[j];
    gx[(size_t)s * ND + j] += gq[j];
  }
}

// dst[scene] = src[scene] where mask[scene] != 0; grid over scenes
__global__ void k_masked_copy(float* dst, const float* src, const uint8_t* mask, int S, int NF, int NA,
                              const int* free_off, const int* aux_off) {
  int s = blockIdx.x;
  if (s >= S || (mask && !mask[s])) return;
  int t = threadIdx.x;
  if (t < ND) {
    dst[(size_t)s * ND + t] = src[(size_t)s * ND + t];
    dst[(size_t)S * ND + (size_t)s * ND + t] = src[(size_t)S * ND + (size_t)s * ND + t];
  }
  size_t fb = (size_t)S * 2 * ND;
  for (int i = free_off[s] * 16 + t; i < free_off[s + 1] * 16; i += blockDim.x) dst[fb + i] = src[fb + i];
  size_t ab = fb + (size_t)NF * 16;
  for (int i = aux_off[s] * 4 + t; i < aux_off[s + 1] * 4; i += blockDim.x) dst[ab + i] = src[ab + i];
}

void launch_step(const KArgs& a, int grid, size_t lds_bytes, hipStream_t st) {
  if (a.rec) hipLaunchKernelGGL(k_step_rec, dim3(grid), dim3(WAVE), lds_bytes, st, a);
  else if (a.frc_robot || a.grip) hipLaunchKernelGGL(k_step_frc, dim3(grid), dim3(WAVE), lds_bytes, st, a);
  else hipLaunchKernelGGL(k_step, dim3(grid), dim3(WAVE), lds_bytes, st, a);
}
void launch_reset_queue(int* q, hipStream_t st) { hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, st, q); }

// counting sort of the scenes by (group, decreasing cost key): one
// workgroup of 1024 lanes, a histogram over 2 x 4096 slots in LDS, its
// exclusive prefix sum (eight entries per lane, then across the lanes), then
// a scatter
constexpr int NKEY = 4096;
__global__ __launch_bounds__(1024) void k_cost_order(const int* cost, const int* maxc, int S, int fit_c, int fit_r,
                                                     int* order, int* n_over, int* q, int* retry) {
  __shared__ int cnt[2 * NKEY];
  __shared__ int wsum[16];
  const int t = threadIdx.x;
  if (t < 3 && q) q[t] = 0;
  if (t == 0 && retry) retry[0] = 0;
  for (int i = t; i < 2 * NKEY; i += 1024) cnt[i] = 0;
  __syncthreads();
  // the key of a scene time v > 0: its base-2 logarithm in steps of 1/128
  auto slot_of = [&](int s) {
    const int v = cost[s];
    int k = 0;
    if (v > 0) {
      const int m = 31 - __clz(v);
      const uint32_t f = m >= 7 ? ((uint32_t)v >> (m - 7)) & 127u : ((uint32_t)v << (7 - m)) & 127u;
      k = min(NKEY - 1, m * 128 + (int)f);
    }
    int g = 1;
    if (fit_c > 0 && maxc) {
      const int m = maxc[s];
      if ((m & 0xffff) + 8 > fit_c || (m >> 16) + 2 > fit_r) g = 0;
    }
    return g * NKEY + (NKEY - 1 - k);
  };
  for (int s = t; s < S; s += 1024) atomicAdd(&cnt[slot_of(s)], 1);
  __syncthreads();
  int loc[8], sum = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    loc[i] = cnt[8 * t + i];
    sum += loc[i];
  }
  int inc = sum;
  const int lane = t & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(inc, o, 64);
    if (lane >= o) inc += v;
  }
  if (lane == 63) wsum[t >> 6] = inc;
  __syncthreads();
  int base = inc - sum;
  for (int w = 0; w < (t >> 6); ++w) base += wsum[w];
  // lane NKEY / 8 owns the first entry of group 1
  if (t == NKEY / 8 && n_over) *n_over = base;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    cnt[8 * t + i] = base;
    base += loc[i];
  }
  __syncthreads();
  for (int s = t; s < S; s += 1024) order[atomicAdd(&cnt[slot_of(s)], 1)] = s;
}

void launch_cost_order(const int* cost, const int* maxc, int S, int fit_c, int fit_r, int* order, int* n_over, int* q,
                       int* retry, hipStream_t st) {
  hipLaunchKernelGGL(k_cost_order, dim3(1), dim3(1024), 0, st, cost, maxc, S, fit_c, fit_r, order, n_over, q, retry);
}
void launch_actions(const DModel* models, const DScene* scenes, const float* x, const float* a, float* tgt, int S,
                    hipStream_t st) {
  if (S <= 0) return;
  hipLaunchKernelGGL(k_actions, dim3((S + 3) / 4), dim3(64), 0, st, models, scenes, x, a, tgt, S);
}
void launch_actions_bwd(const DModel* models, const DScene* scenes, const float* x, const float* a,
                        const float* gtgt, float* ga, float* gx, int S, hipStream_t st) {
  if (S <= 0) return;
  hipLaunchKernelGGL(k_actions_bwd, dim3((S + 63) / 64), dim3(64), 0, st, models, scenes, x, a, gtgt, ga, gx, S);
}
void launch_masked_copy(float* dst, const float* src, const uint8_t* mask, int S, int NF, int NA,
                        const int* free_off, const int* aux_off, hipStream_t st) {
  if (S <= 0) return;
  hipLaunchKernelGGL(k_masked_copy, dim3(S), dim3(64), 0, st, dst, src, mask, S, NF, NA, free_off, aux_off);
}
const void* step_kernel_ptr() { return reinterpret_cast<const void*>(&k_step); }
const void* step_rec_kernel_ptr() { return reinterpret_cast<const void*>(&k_step_rec); }
const void* step_frc_kernel_ptr() { return reinterpret_cast<const void*>(&k_step_frc); }
const void* spawn_check_kernel_ptr() { return reinterpret_cast<const void*>(&k_spawn_check); }
void launch_spawn_check(const KArgs& a, uint8_t* collide, size_t lds_bytes, hipStream_t st) {
  hipLaunchKernelGGL(k_spawn_check, dim3(a.S), dim3(WAVE), lds_bytes, st, a, collide);
}
void launch_reset_robots(float* x, const uint8_t* mask, const float* base, const float* noise, const float* clip,
                         int S, hipStream_t st) {
  if (S <= 0) return;
  Clip16 c;
  for (int j = 0; j < ND; ++j) c.c[j] = clip[j];
  hipLaunchKernelGGL(k_reset_robots, dim3((S + 3) / 4), dim3(64), 0, st, x, mask, base, noise, c, S);
}

}  // namespace msk
