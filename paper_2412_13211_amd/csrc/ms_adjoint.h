// ms_adjoint.h -- adjoint engine of one control step (reverse mode): the
// per-scene state, workspace layout and primitive reverses shared by the two
// adjoint kernels of ms_backward.hip.
//
// The vector-Jacobian product behind ms_step_backward walks the substeps of
// a control step backwards:
//   integrate^T -> Gauss-Seidel^T (velocities reconstructed from the recorded
//   pre-projection values) -> rows^T -> bias^T -> dynamics^T -> contacts^T ->
//   kinematics^T -> drive^T.
// Convention at the kinks: max(0, y) has slope 0 at y = 0, a friction disk
// projection exactly on the boundary counts as inside, contacts appear and
// disappear only between evaluations (the contact set is held fixed).
//
// Two users:
//   - the product path, k_step_bwd_wave (ms_backward.hip): one 64-lane
//     wavefront per scene with its workspace (ws_layout(..., wave = true)) in
//     LDS.  It reads the record the forward kernel wrote (substep states,
//     contact lists, Gauss-Seidel tape) and recomputes kinematics, dynamics,
//     M~^-1 and the rows across the lanes; the per-scene engine Eng below
//     supplies the record access, the row bookkeeping and the single-lane
//     pieces (limit rows, free-body and door / drawer sides);
//   - the reference schedule k_step_bwd (MS_SCHED_BWD_REFERENCE): one thread
//     per scene runs the whole engine alone, recomputing the step itself
//     (contacts, CRBA + Cholesky, sequential Gauss-Seidel in the canonical
//     order the level schedule reproduces), with derivatives of the mass
//     matrix and bias force by forward-mode tangents of CRBA / RNEA, in a
//     per-scene workspace in global memory.  It is the independent
//     cross-check of the wavefront kernel.
//
// The code is plain C++ (host and device) so that the engine also runs on
// the CPU.
#pragma once
#include "ms_internal.h"

#ifndef MSA_HD
#define MSA_HD __host__ __device__
#endif

namespace msa {
using namespace msk;

// ------------------------------------------------------------ 3-vectors
struct V {
  float x, y, z;
};
MSA_HD inline V mkv(float a, float b, float c) { return V{a, b, c}; }
MSA_HD inline V ld3(const float* p) { return V{p[0], p[1], p[2]}; }
MSA_HD inline void st3(float* p, V v) { p[0] = v.x; p[1] = v.y; p[2] = v.z; }
MSA_HD inline void add3(float* p, V v) { p[0] += v.x; p[1] += v.y; p[2] += v.z; }
MSA_HD inline V operator+(V a, V b) { return V{a.x + b.x, a.y + b.y, a.z + b.z}; }
MSA_HD inline V operator-(V a, V b) { return V{a.x - b.x, a.y - b.y, a.z - b.z}; }
MSA_HD inline V operator-(V a) { return V{-a.x, -a.y, -a.z}; }
MSA_HD inline V operator*(V a, float s) { return V{a.x * s, a.y * s, a.z * s}; }
MSA_HD inline float dot(V a, V b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
MSA_HD inline V cross(V a, V b) { return V{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
MSA_HD inline float norm(V a) { return sqrtf(dot(a, a)); }
MSA_HD inline V rmv(const float* R, V v) {
  return V{R[0] * v.x + R[1] * v.y + R[2] * v.z, R[3] * v.x + R[4] * v.y + R[5] * v.z,
           R[6] * v.x + R[7] * v.y + R[8] * v.z};
}
MSA_HD inline V rtmv(const float* R, V v) {
  return V{R[0] * v.x + R[3] * v.y + R[6] * v.z, R[1] * v.x + R[4] * v.y + R[7] * v.z,
           R[2] * v.x + R[5] * v.y + R[8] * v.z};
}
// symmetric 3x3 stored xx yy zz xy xz yz
MSA_HD inline V smv(const float* S, V v) {
  return V{S[0] * v.x + S[3] * v.y + S[4] * v.z, S[3] * v.x + S[1] * v.y + S[5] * v.z,
           S[4] * v.x + S[5] * v.y + S[2] * v.z};
}
// S_bar += sym part of a b^T, stored as the adjoint of the 6 free entries
MSA_HD inline void sym_outer_add(float* Sb, V a, V b, float s) {
  Sb[0] += s * a.x * b.x;
  Sb[1] += s * a.y * b.y;
  Sb[2] += s * a.z * b.z;
  Sb[3] += s * (a.x * b.y + a.y * b.x);
  Sb[4] += s * (a.x * b.z + a.z * b.x);
  Sb[5] += s * (a.y * b.z + a.z * b.y);
}
MSA_HD inline void mm3(const float* A, const float* B, float* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i * 3 + j] = A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
}
MSA_HD inline void quatR(const float* q, float* R) {
  float w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}
// adjoint of quatR: Rb (9) -> qb (4), accumulated
MSA_HD inline void quatR_bar(const float* q, const float* Rb, float* qb) {
  float w = q[0], x = q[1], y = q[2], z = q[3];
  qb[0] += 2.f * (-z * Rb[1] + y * Rb[2] + z * Rb[3] - x * Rb[5] - y * Rb[6] + x * Rb[7]);
  qb[1] += 2.f * (y * Rb[1] + z * Rb[2] + y * Rb[3] - 2.f * x * Rb[4] - w * Rb[5] + z * Rb[6] + w * Rb[7] -
                  2.f * x * Rb[8]);
  qb[2] += 2.f * (-2.f * y * Rb[0] + x * Rb[1] + w * Rb[2] + x * Rb[3] + z * Rb[5] - w * Rb[6] + z * Rb[7] -
                  2.f * y * Rb[8]);
  qb[3] += 2.f * (-2.f * z * Rb[0] - w * Rb[1] + x * Rb[2] + w * Rb[3] - 2.f * z * Rb[4] + y * Rb[5] + x * Rb[6] +
                  y * Rb[7]);
}
MSA_HD inline void rot_axis(V k, float th, float* R) {
  float s = sinf(th), c = cosf(th);
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
MSA_HD inline void onb(V n, V& t1, V& t2) {
  float sg = copysignf(1.f, n.z);
  float a = -1.f / (sg + n.z);
  float b = n.x * n.y * a;
  t1 = V{1.f + sg * n.x * n.x * a, sg * b, -sg * n.x};
  t2 = V{b, sg + n.y * n.y * a, -n.y};
}
// adjoint of onb: (t1b, t2b) -> nb, accumulated
MSA_HD inline void onb_bar(V n, V t1b, V t2b, float* nb) {
  float sg = copysignf(1.f, n.z);
  float a = -1.f / (sg + n.z);
  float a2 = a * a;
  nb[0] += sg * 2.f * n.x * a * t1b.x + sg * n.y * a * t1b.y - sg * t1b.z + n.y * a * t2b.x;
  nb[1] += sg * n.x * a * t1b.y + n.x * a * t2b.x + 2.f * n.y * a * t2b.y - t2b.z;
  nb[2] += sg * n.x * n.x * a2 * t1b.x + sg * n.x * n.y * a2 * t1b.y + n.x * n.y * a2 * t2b.x + n.y * n.y * a2 * t2b.y;
}


// ------------------------------------------------------------ workspace
// A scene's workspace is one float array.  On the GPU the arrays of all
// scenes are interleaved (element e of slot s at base[e * stride + s]) so
// that the lanes of a wavefront touch consecutive addresses.
struct Buf {
  float* p;
  long st;
  MSA_HD float& operator[](long e) const { return p[e * st]; }
};
MSA_HD inline V bl3(const Buf& b, long e) { return V{b[e], b[e + 1], b[e + 2]}; }
MSA_HD inline void bs3(const Buf& b, long e, V v) { b[e] = v.x; b[e + 1] = v.y; b[e + 2] = v.z; }
MSA_HD inline void ba3(const Buf& b, long e, V v) { b[e] += v.x; b[e + 1] += v.y; b[e + 2] += v.z; }

struct SceneRef {
  const DModel* M;
  const DFree* F;     // this scene's free bodies
  const float* St;    // this scene's static boxes (6 floats each)
  const float4* Pl;   // this scene's planes
  const DAux* A;      // this scene's door / drawer joints
  const float* hold;  // hold targets [16]
  int nf, ns, np, na;
};
struct Prm {
  float h, mu, beta, margin, g[3];
  int K, mode, ccap, rcap, nsub;
};

// per-scene state record: q[16] qd[16] | free[fmax][16] | aux[AMAX][4]
MSA_HD inline int state_rec_floats(int fmax) { return 32 + 16 * fmax + 4 * AMAX; }

// contact record: packed side codes, owner radius, phi, normal, contact
// point, tangents, W per direction, bias (the owner's centre is p + r n)
enum { C_ID = 0, C_R = 1, C_PHI = 2, C_N = 3, C_P = 6, C_T1 = 9, C_T2 = 12, C_W = 15, C_BIAS = 18, CR = 19 };
// side codes of a contact packed into the bits of one float: owner kind
// (bits 0-1), owner vertex (2-4), target kind (5-6), owner index (7-14),
// target index (15-30)
struct Ids {
  int ok, oi, ov, tk, ti;
};
MSA_HD inline float pack_ids(int ok, int oi, int ov, int tk, int ti) {
  return __builtin_bit_cast(float, ok | (ov << 2) | (tk << 5) | (oi << 7) | (ti << 15));
}
MSA_HD inline Ids unpack_ids(float f) {
  const int v = __builtin_bit_cast(int, f);
  return Ids{v & 3, (v >> 7) & 255, (v >> 2) & 7, (v >> 5) & 3, (v >> 15) & 0xffff};
}
// contact adjoint record: direction adjoints (n, t1, t2), contact point, W, bias
enum { B_D = 0, B_P = 9, B_W = 12, B_BIAS = 15, CB = 16 };
// free-body adjoint record
enum { F_XB = 0, F_RB = 3, F_IIB = 12, F_IWB = 21, FB = 30 };
// door / drawer adjoint record
enum { X_RB = 0, X_BCB = 9, X_QB = 12, XB = 16 };

// level schedule arrays (ints): level of row (then of group), groups by
// level, level offsets, robot row of each level, first row of each group,
// last level of each dynamic node, counters
MSA_HD inline int lv_rows(int ccap) { return 2 * AMAX + ccap; }
MSA_HD inline int lv_ints(int ccap) { return 5 * lv_rows(ccap) + 5 + 64 + 8; }

struct WS {
  int wave;  // the wavefront kernel's LDS layout
  int fmax, ntmax, ccap, rcap, K, nsub, ss;
  int st, gA, gB, ub, tape;
  int kR, kp, ka, ko, kc, kIcw, ks, kI, kIc, sph, tl;
  int fR, fIw, fIi, fim;  // fim: inverse masses of the free bodies
  int xR, xbc, xa, xo, xM, xC, xty;  // xty: door / drawer joint kinds (0 revolute, 1 prismatic)
  int tau, arm, L, z, rv, ra, rfl, rff;
  int vR, vA, vF, lam, llam, con, lim, rJ, rw;
  int vRb, vAb, vFb, lamb, llamb, limb, conb, rJb, rwb, fb, xb;
  int Mb, sb, Ib, Icb, fbar, abar, vbar, bacc;
  int lv;    // level schedule (wavefront kernel only)
  int tring;  // two sweeps of the tape staged from the record (wavefront kernel only)
  int trs;    // floats per staged sweep
  int Minv;  // explicit M~^-1 (wavefront kernel only)
  int lz;    // bias torques, then M~^-1 h vRbar (wavefront kernel only)
  int tF, tFb, tA, tV, tV2;  // per-body scratch of the wavefront dynamics^T
  int total;
};

// wave = true: the layout of the wavefront kernel's LDS block (one state
// record, the tape and candidate lists elsewhere, plus the level schedule)
MSA_HD inline WS ws_layout(int fmax, int ntmax, int ccap, int rcap, int K, int nsub, bool wave = false) {
  WS w;
  w.wave = wave ? 1 : 0;
  w.fmax = fmax < 1 ? 1 : fmax;
  w.ntmax = ntmax < 1 ? 1 : ntmax;
  w.ccap = ccap;
  w.rcap = rcap < 1 ? 1 : rcap;
  w.K = K;
  w.nsub = nsub;
  w.ss = state_rec_floats(w.fmax);
  const int fm = w.fmax;
  int o = 0;
  auto take = [&](int n) { int r = o; o += n; return r; };
  w.st = take((wave ? 1 : nsub + 1) * w.ss);
  w.gA = take(w.ss);
  w.gB = take(w.ss);
  w.ub = take(ND);
  w.tape = take(wave ? 0 : K * 3 * (2 * AMAX + ccap));
  w.kR = take(ND * 9); w.kp = take(ND * 3); w.ka = take(ND * 3); w.ko = take(ND * 3); w.kc = take(ND * 3);
  w.kIcw = take(ND * 6); w.ks = take(ND * 6); w.kI = take(ND * 36); w.kIc = take(ND * 36);
  w.sph = take(wave ? 0 : SPH * 3);  // sphere centres: only the lane kernel's contact search reads them
  w.tl = take(wave ? 0 : (ND + 1) * (w.ntmax + 1));
  w.fR = take(fm * 9); w.fIw = take(fm * 9); w.fIi = take(fm * 9); w.fim = take(fm);
  w.xR = take(AMAX * 9); w.xbc = take(AMAX * 3); w.xa = take(AMAX * 3); w.xo = take(AMAX * 3);
  w.xM = take(AMAX); w.xC = take(AMAX); w.xty = take(AMAX);
  w.tau = take(ND); w.arm = take(ND); w.L = take(ND * ND); w.z = take(ND);
  w.rv = take(ND * 6); w.ra = take(ND * 6); w.rfl = take(ND * 6); w.rff = take(ND * 6);
  w.vR = take(ND); w.vA = take(AMAX); w.vF = take(fm * 6);
  // impulses: working storage of the lane kernel's forward sweeps (the
  // reverse sweeps read them from the tape)
  w.lam = take(wave ? 0 : 3 * ccap); w.llam = take(wave ? 0 : 2 * AMAX);
  w.con = take(ccap * CR);
  w.lim = take(2 * AMAX * 4);
  w.rJ = take(w.rcap * 3 * ND); w.rw = take(w.rcap * 3 * ND);
  w.vRb = take(ND); w.vAb = take(AMAX); w.vFb = take(fm * 6);
  w.lamb = take(3 * ccap); w.llamb = take(2 * AMAX); w.limb = take(2 * AMAX);
  w.conb = take(ccap * CB);
  // the robot rows' adjoints (and in the wavefront kernel the staged tape)
  // are dead once rows^T is done; the dynamics^T scratch (written before it
  // is read) shares their space.  The wavefront kernel forms Ibar in place
  // of Icbar.
  w.trs = 3 * (2 * AMAX + ccap);
  const int rows_b = 2 * w.rcap * 3 * ND;
  const int live_b = rows_b + (wave ? 2 * w.trs : 0);
  const int dyn_b = ND * 6 + (wave ? 1 : 2) * ND * 36 + 8 * ND * 6;
  const int kb = take(live_b > dyn_b ? live_b : dyn_b);
  w.rJb = kb; w.rwb = kb + w.rcap * 3 * ND;
  w.tring = wave ? kb + rows_b : 0;
  w.sb = kb; w.Ib = w.sb + ND * 6; w.Icb = wave ? w.Ib : w.Ib + ND * 36;
  w.fbar = w.Icb + ND * 36; w.abar = w.fbar + ND * 6; w.vbar = w.abar + ND * 6;
  w.tF = w.vbar + ND * 6; w.tFb = w.tF + ND * 6; w.tA = w.tFb + ND * 6; w.tV = w.tA + ND * 6;
  w.tV2 = w.tV + ND * 6;
  w.fb = take(fm * FB); w.xb = take(AMAX * XB);
  w.Mb = take(ND * ND);
  w.bacc = take(ND * 9);
  w.lv = take(wave ? lv_ints(ccap) : 0);
  w.Minv = take(wave ? ND * ND : 0);
  w.lz = take(wave ? ND : 0);
  w.total = o;
  return w;
}

// ------------------------------------------------------------ small kernels of the step
// signed distance of sphere (c, r) to a box (centre bc, world-from-box R or
// identity when R is null, half extents e); normal from the box to the sphere
MSA_HD inline float box_phi(V c, float r, V bc, const float* R, V e, V& n) {
  V d = c - bc;
  V y = R ? rtmv(R, d) : d;
  bool out = fabsf(y.x) > e.x || fabsf(y.y) > e.y || fabsf(y.z) > e.z;
  float phi;
  V nl;
  if (out) {
    V k{fminf(fmaxf(y.x, -e.x), e.x), fminf(fmaxf(y.y, -e.y), e.y), fminf(fmaxf(y.z, -e.z), e.z)};
    V dd = y - k;
    float dist = sqrtf(dot(dd, dd));
    phi = dist - r;
    nl = dist > 0.f ? dd * (1.f / dist) : V{0.f, 0.f, 1.f};
  } else {
    float gx = e.x - fabsf(y.x), gy = e.y - fabsf(y.y), gz = e.z - fabsf(y.z);
    int best = 0;
    float bv = gx;
    if (gy < bv) { bv = gy; best = 1; }
    if (gz < bv) { bv = gz; best = 2; }
    float yc = best == 0 ? y.x : (best == 1 ? y.y : y.z);
    float sg = yc >= 0.f ? 1.f : -1.f;
    phi = -bv - r;
    nl = V{best == 0 ? sg : 0.f, best == 1 ? sg : 0.f, best == 2 ? sg : 0.f};
  }
  n = R ? rmv(R, nl) : nl;
  return phi;
}
// reverse of box_phi: (phib, nb) -> cb, bcb (+=), Rb (+= when R non-null)
MSA_HD inline void box_phi_bar(V c, V bc, const float* R, V e, float phib, V nb, V& cb, V& bcb, float* Rb) {
  V d = c - bc;
  V y = R ? rtmv(R, d) : d;
  bool out = fabsf(y.x) > e.x || fabsf(y.y) > e.y || fabsf(y.z) > e.z;
  V nl;
  V yb{0.f, 0.f, 0.f};
  if (out) {
    V k{fminf(fmaxf(y.x, -e.x), e.x), fminf(fmaxf(y.y, -e.y), e.y), fminf(fmaxf(y.z, -e.z), e.z)};
    V dd = y - k;
    float dist = sqrtf(dot(dd, dd));
    if (dist > 0.f) {
      nl = dd * (1.f / dist);
      V nlb = R ? rtmv(R, nb) : nb;
      V ddb = nl * phib + (nlb - nl * dot(nl, nlb)) * (1.f / dist);
      yb.x = fabsf(y.x) > e.x ? ddb.x : 0.f;
      yb.y = fabsf(y.y) > e.y ? ddb.y : 0.f;
      yb.z = fabsf(y.z) > e.z ? ddb.z : 0.f;
    } else {
      nl = V{0.f, 0.f, 1.f};
    }
  } else {
    float gx = e.x - fabsf(y.x), gy = e.y - fabsf(y.y), gz = e.z - fabsf(y.z);
    int best = 0;
    float bv = gx;
    if (gy < bv) { bv = gy; best = 1; }
    if (gz < bv) { bv = gz; best = 2; }
    float yc = best == 0 ? y.x : (best == 1 ? y.y : y.z);
    float sg = yc >= 0.f ? 1.f : -1.f;
    nl = V{best == 0 ? sg : 0.f, best == 1 ? sg : 0.f, best == 2 ? sg : 0.f};
    // phi = |y_best| - e_best - r
    if (best == 0) yb.x = sg * phib;
    else if (best == 1) yb.y = sg * phib;
    else yb.z = sg * phib;
  }
  V db;
  if (R) {
    // n = R nl
    Rb[0] += nb.x * nl.x; Rb[1] += nb.x * nl.y; Rb[2] += nb.x * nl.z;
    Rb[3] += nb.y * nl.x; Rb[4] += nb.y * nl.y; Rb[5] += nb.y * nl.z;
    Rb[6] += nb.z * nl.x; Rb[7] += nb.z * nl.y; Rb[8] += nb.z * nl.z;
    // y = R^T d
    db = rmv(R, yb);
    Rb[0] += d.x * yb.x; Rb[1] += d.x * yb.y; Rb[2] += d.x * yb.z;
    Rb[3] += d.y * yb.x; Rb[4] += d.y * yb.y; Rb[5] += d.y * yb.z;
    Rb[6] += d.z * yb.x; Rb[7] += d.z * yb.y; Rb[8] += d.z * yb.z;
  } else {
    db = yb;
  }
  cb = cb + db;
  bcb = bcb - db;
}
MSA_HD inline float dist_point_box(V y, V e) {
  V d{fmaxf(fabsf(y.x) - e.x, 0.f), fmaxf(fabsf(y.y) - e.y, 0.f), fmaxf(fabsf(y.z) - e.z, 0.f)};
  return sqrtf(dot(d, d));
}
// friction-disk projection of (y1, y2) onto radius lim; returns whether it projected
MSA_HD inline bool disk_proj(float y1, float y2, float lim, float& o1, float& o2) {
  float nn = y1 * y1 + y2 * y2;
  bool proj = nn > lim * lim;
  o1 = y1;
  o2 = y2;
  if (proj) {
    if (lim > 0.f) {
      float sc = lim / sqrtf(nn);
      o1 = y1 * sc;
      o2 = y2 * sc;
    } else {
      o1 = 0.f;
      o2 = 0.f;
    }
  }
  return proj;
}

// ------------------------------------------------------------ the engine
// Side codes of a contact: owner kind (0 robot sphere, 1 free-box vertex,
// 2 free sphere); target kind (0 plane, 1 static box, 2 door/drawer box,
// 3 free body).
struct Eng {
  SceneRef sc;
  Prm pr;
  WS w;
  Buf b;
  int nb, nsph, nc, nrob, nlim;
  uint32_t status;
  // pre-projection values of the row updates: sweep it, row r (limit rows
  // first, then contacts), slot d (normal, tangent 1, tangent 2)
  Buf tb;
  int tsw;    // floats per sweep
  int tmask;  // sweep index mask: all bits (the whole tape), or 1 (a two-sweep ring)
  MSA_HD float& tape_at(int it, int r, int d) const { return tb[(long)(it & tmask) * tsw + 3 * r + d]; }

  MSA_HD float& at(long e) const { return b[e]; }
  MSA_HD Ids ids(long e) const { return unpack_ids(b[e + C_ID]); }
  MSA_HD V v3(long e) const { return bl3(b, e); }
  MSA_HD void s3(long e, V v) const { bs3(b, e, v); }
  MSA_HD void a3(long e, V v) const { ba3(b, e, v); }
  MSA_HD void ld9(long e, float* R) const {
    for (int t = 0; t < 9; ++t) R[t] = b[e + t];
  }
  MSA_HD void zero(long e, int n) const {
    for (int t = 0; t < n; ++t) b[e + t] = 0.f;
  }
  MSA_HD long srec(int r) const { return (long)w.st + (long)r * w.ss; }
  MSA_HD int fro(int f) const { return 32 + 16 * f; }            // free body f in a state record
  MSA_HD int axo(int x) const { return 32 + 16 * w.fmax + 4 * x; }  // aux joint x in a state record

  // ---------------------------------------------------------------- drive
  MSA_HD void drive(long s, const float* u) {
    for (int j = 0; j < ND; ++j) drive_one(s, u, j);
  }
  MSA_HD void drive_one(long s, const float* u, int j) {
    const DModel& M = *sc.M;
    const float h = pr.h;
    {
      float tau = 0.f, arm = 0.f;
      if (j < nb) {
        float q = at(s + j), qd = at(s + ND + j), dmp = M.damp[j];
        if (pr.mode == 0) {
          tau = u[j] - dmp * qd;
          arm = M.arm[j] + h * dmp;
        } else {
          float kp = M.kp[j], kd = M.kd[j], qt, vt, ff = 0.f;
          bool vel = M.veldof[j] != 0;
          if (pr.mode == 1) {
            qt = vel ? 0.f : u[j];
            vt = vel ? u[j] : 0.f;
          } else {
            qt = vel ? 0.f : sc.hold[j];
            vt = vel ? sc.hold[j] : 0.f;
            ff = u[j];
          }
          if (vel) kp = 0.f;
          tau = ff + kp * (qt - q - h * qd) + kd * (vt - qd) - dmp * qd;
          arm = M.arm[j] + h * (kd + dmp) + h * h * kp;
        }
      }
      at(w.tau + j) = tau;
      at(w.arm + j) = arm;
    }
  }

  // ---------------------------------------------------------------- kinematics
  MSA_HD void kinematics(long s) {
    for (int i = 0; i < nb; ++i) {
      kin_pose(s, i);
      kin_body(i);
    }
    kin_spheres();
  }
  // world pose of body i (its parent's pose known): R, p, joint axis a and origin o
  MSA_HD void kin_pose(long s, int i) {
    const DModel& M = *sc.M;
    {
      int par = M.parent[i];
      float Rj[9], R[9];
      V o;
      if (par < 0) {
        for (int t = 0; t < 9; ++t) Rj[t] = M.xtR[i][t];
        o = ld3(M.xtp[i]);
      } else {
        float Rp[9];
        ld9(w.kR + par * 9, Rp);
        mm3(Rp, M.xtR[i], Rj);
        o = v3(w.kp + par * 3) + rmv(Rp, ld3(M.xtp[i]));
      }
      V ax = ld3(M.axis[i]);
      V a = rmv(Rj, ax);
      V p;
      if (M.jtype[i] == 0) {
        float Rr[9];
        rot_axis(ax, at(s + i), Rr);
        mm3(Rj, Rr, R);
        p = o;
      } else {
        for (int t = 0; t < 9; ++t) R[t] = Rj[t];
        p = o + a * at(s + i);
      }
      for (int t = 0; t < 9; ++t) at(w.kR + i * 9 + t) = R[t];
      s3(w.kp + i * 3, p);
      s3(w.ka + i * 3, a);
      s3(w.ko + i * 3, o);
    }
  }
  // per-body quantities from the pose: motion subspace, COM, inertias
  MSA_HD void kin_body(int i) {
    const DModel& M = *sc.M;
    {
      float R[9];
      ld9(w.kR + i * 9, R);
      const V a = v3(w.ka + i * 3), o = v3(w.ko + i * 3), p = v3(w.kp + i * 3);
      V top = M.jtype[i] == 0 ? a : V{0.f, 0.f, 0.f};
      V bot = M.jtype[i] == 0 ? cross(o, a) : a;
      s3(w.ks + i * 6, top);
      s3(w.ks + i * 6 + 3, bot);
      V c = rmv(R, ld3(M.com[i])) + p;
      s3(w.kc + i * 3, c);
      // Icw = R Ic R^T
      const float* I = M.Ic[i];
      float Ib[9] = {I[0], I[3], I[4], I[3], I[1], I[5], I[4], I[5], I[2]};
      float T[9], W[9];
      mm3(R, Ib, T);
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) W[r * 3 + q] = T[r * 3] * R[q * 3] + T[r * 3 + 1] * R[q * 3 + 1] + T[r * 3 + 2] * R[q * 3 + 2];
      float Sw[6] = {W[0], W[4], W[8], W[1], W[2], W[5]};
      for (int t = 0; t < 6; ++t) at(w.kIcw + i * 6 + t) = Sw[t];
      spatial_inertia(M.mass[i], c, W, w.kI + i * 36);
    }
  }
  MSA_HD void kin_spheres() {
    const DModel& M = *sc.M;
    for (int k = 0; k < nsph && !w.wave; ++k) {
      int bi = M.sph_body[k];
      float R[9];
      ld9(w.kR + bi * 9, R);
      float4 sp = M.sph[k];
      s3(w.sph + k * 3, rmv(R, V{sp.x, sp.y, sp.z}) + v3(w.kp + bi * 3));
    }
  }
  // 6x6 spatial inertia about the world origin (angular rows first)
  MSA_HD void spatial_inertia(float m, V c, const float* Ic, long dst) {
    float cc = dot(c, c);
    float cv[3] = {c.x, c.y, c.z};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        float v = Ic[i * 3 + j] - m * (cv[i] * cv[j]);
        if (i == j) v += m * cc;
        at(dst + i * 6 + j) = v;
      }
    float cx[9] = {0.f, -c.z, c.y, c.z, 0.f, -c.x, -c.y, c.x, 0.f};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        at(dst + i * 6 + 3 + j) = m * cx[i * 3 + j];
        at(dst + (3 + i) * 6 + j) = m * cx[j * 3 + i];
        at(dst + (3 + i) * 6 + 3 + j) = i == j ? m : 0.f;
      }
  }

  MSA_HD void aux_frames(long s) {
    for (int x = 0; x < sc.na; ++x) aux_frame(s, x);
  }
  MSA_HD void aux_frame(long s, int x) {
    {
      const DAux& A = sc.A[x];
      float q = at(s + axo(x));
      V ax = ld3(A.axis);
      V a = rmv(A.R0, ax);
      V o = ld3(A.p0);
      float R[9];
      V p = o;
      if (A.type == 0) {
        float Rr[9];
        rot_axis(ax, q, Rr);
        mm3(A.R0, Rr, R);
      } else {
        for (int t = 0; t < 9; ++t) R[t] = A.R0[t];
        p = o + a * q;
      }
      V bc = rmv(R, ld3(A.bc)) + p;
      for (int t = 0; t < 9; ++t) at(w.xR + x * 9 + t) = R[t];
      s3(w.xbc + x * 3, bc);
      s3(w.xa + x * 3, a);
      s3(w.xo + x * 3, o);
      V g{pr.g[0], pr.g[1], pr.g[2]};
      float Mx, Cx;
      if (A.type == 0) {
        V Ra = rtmv(R, a);
        float Iaa = A.Ib[0] * Ra.x * Ra.x + A.Ib[1] * Ra.y * Ra.y + A.Ib[2] * Ra.z * Ra.z;
        V ac = cross(a, bc - o);
        Mx = Iaa + A.mass * dot(ac, ac);
        Cx = -A.mass * dot(g, ac);
      } else {
        Mx = A.mass;
        Cx = -A.mass * dot(g, a);
      }
      at(w.xM + x) = Mx;
      at(w.xC + x) = Cx;
      at(w.xty + x) = (float)A.type;
    }
  }

  MSA_HD void free_frames(long s) {
    for (int f = 0; f < sc.nf; ++f) free_frame(s, f);
  }
  MSA_HD void free_frame(long s, int f) {
    {
      float Q[4] = {at(s + fro(f) + 4), at(s + fro(f) + 5), at(s + fro(f) + 6), at(s + fro(f) + 7)};
      float R[9];
      quatR(Q, R);
      const DFree& F = sc.F[f];
      float Iw[9], Ii[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          Iw[r * 3 + c] = R[r * 3] * F.Ib[0] * R[c * 3] + R[r * 3 + 1] * F.Ib[1] * R[c * 3 + 1] +
                          R[r * 3 + 2] * F.Ib[2] * R[c * 3 + 2];
          Ii[r * 3 + c] = R[r * 3] * (1.f / F.Ib[0]) * R[c * 3] + R[r * 3 + 1] * (1.f / F.Ib[1]) * R[c * 3 + 1] +
                          R[r * 3 + 2] * (1.f / F.Ib[2]) * R[c * 3 + 2];
        }
      at(w.fim + f) = 1.f / F.mass;
      for (int t = 0; t < 9; ++t) {
        at(w.fR + f * 9 + t) = R[t];
        at(w.fIw + f * 9 + t) = Iw[t];
        at(w.fIi + f * 9 + t) = Ii[t];
      }
    }
  }

  // ---------------------------------------------------------------- contacts
  MSA_HD int n_targets() const { return sc.np + sc.ns + sc.na + sc.nf; }
  // conservative test of a bounding sphere (c, R) against target t
  MSA_HD bool near_target(long s, V c, float Rad, int t, float slack) const {
    if (t < sc.np) {
      float4 pl = sc.Pl[t];
      return pl.x * c.x + pl.y * c.y + pl.z * c.z - pl.w - Rad < slack;
    }
    t -= sc.np;
    if (t < sc.ns) {
      const float* bx = sc.St + t * 6;
      return dist_point_box(c - V{bx[0], bx[1], bx[2]}, V{bx[3], bx[4], bx[5]}) - Rad < slack;
    }
    t -= sc.ns;
    if (t < sc.na) {
      float R[9];
      ld9(w.xR + t * 9, R);
      V y = rtmv(R, c - v3(w.xbc + t * 3));
      return dist_point_box(y, ld3(sc.A[t].bh)) - Rad < slack;
    }
    t -= sc.na;
    V xg = v3(s + fro(t));
    const DFree& G = sc.F[t];
    if (G.type == 0) {
      float R[9];
      ld9(w.fR + t * 9, R);
      return dist_point_box(rtmv(R, c - xg), ld3(G.half)) - Rad < slack;
    }
    V d = c - xg;
    return sqrtf(dot(d, d)) - Rad - G.half[0] < slack;
  }
  // exact pair test; returns whether the pair is allowed (phi, n valid then)
  MSA_HD bool pair(long s, V c, float r, int okind, int of, int oflags, int t, float& phi, V& n) const {
    if (t < sc.np) {
      if (t == 0 && okind == 0 && (oflags & 1)) return false;
      float4 pl = sc.Pl[t];
      n = V{pl.x, pl.y, pl.z};
      phi = dot(n, c) - pl.w - r;
      return true;
    }
    t -= sc.np;
    if (t < sc.ns) {
      const float* bx = sc.St + t * 6;
      phi = box_phi(c, r, V{bx[0], bx[1], bx[2]}, nullptr, V{bx[3], bx[4], bx[5]}, n);
      return true;
    }
    t -= sc.ns;
    if (t < sc.na) {
      float R[9];
      ld9(w.xR + t * 9, R);
      phi = box_phi(c, r, v3(w.xbc + t * 3), R, ld3(sc.A[t].bh), n);
      return true;
    }
    t -= sc.na;
    const DFree& G = sc.F[t];
    if (t == of) return false;
    if (G.type != 0 && okind == 1) return false;
    if (G.type != 0 && okind == 2 && t <= of) return false;
    V xg = v3(s + fro(t));
    if (G.type == 0) {
      float R[9];
      ld9(w.fR + t * 9, R);
      phi = box_phi(c, r, xg, R, ld3(G.half), n);
    } else {
      V d = c - xg;
      float dist = sqrtf(dot(d, d));
      phi = dist - r - G.half[0];
      n = dist < 1e-12f ? V{0.f, 0.f, 1.f} : d * (1.f / dist);
    }
    return true;
  }
  MSA_HD void emit(int okind, int oidx, int overt, int t, float r, V c, float phi, V n) {
    bool rob = okind == 0;
    if (rob && nrob >= pr.rcap) {
      status |= MS_ROBOT_OVERFLOW_BIT;
      return;
    }
    if (nc >= pr.ccap) {
      status |= MS_OVERFLOW_BIT;
      return;
    }
    long e = w.con + (long)nc * CR;
    int tk, ti;
    target_code(t, tk, ti);
    at(e + C_ID) = pack_ids(okind, oidx, overt, tk, ti);
    at(e + C_R) = r;
    at(e + C_PHI) = phi;
    s3(e + C_N, n);
    s3(e + C_P, c - n * r);
    ++nc;
    if (rob) ++nrob;
  }
  MSA_HD void target_code(int t, int& tk, int& ti) const {
    if (t < sc.np) { tk = 0; ti = t; return; }
    t -= sc.np;
    if (t < sc.ns) { tk = 1; ti = t; return; }
    t -= sc.ns;
    if (t < sc.na) { tk = 2; ti = t; return; }
    tk = 3;
    ti = t - sc.na;
  }
  static constexpr uint32_t MS_OVERFLOW_BIT = 2u, MS_DEGENERATE_BIT = 4u, MS_ROBOT_OVERFLOW_BIT = 8u;

  MSA_HD void contacts(long s) {
    const DModel& M = *sc.M;
    nc = 0;
    nrob = 0;
    const int NT = n_targets();
    const float slack = pr.margin + 1e-3f;
    // per-body candidate targets (bounding-sphere cull; the exact test decides)
    for (int bi = 0; bi < nb; ++bi) {
      int cnt = 0;
      if (M.sph_count[bi] > 0) {
        float R[9];
        ld9(w.kR + bi * 9, R);
        float4 bs = M.bsph[bi];
        V cb = rmv(R, V{bs.x, bs.y, bs.z}) + v3(w.kp + bi * 3);
        for (int t = 0; t < NT; ++t)
          if (near_target(s, cb, bs.w, t, slack)) at(w.tl + bi * (w.ntmax + 1) + 1 + cnt++) = (float)t;
      }
      at(w.tl + bi * (w.ntmax + 1)) = (float)cnt;
    }
    for (int k = 0; k < nsph; ++k) {
      int bi = M.sph_body[k];
      V c = v3(w.sph + k * 3);
      float r = M.sph[k].w;
      int fl = M.sph_flags[k];
      long lb = w.tl + bi * (w.ntmax + 1);
      int cnt = (int)at(lb);
      for (int q = 0; q < cnt; ++q) {
        int t = (int)at(lb + 1 + q);
        float phi;
        V n;
        if (pair(s, c, r, 0, -1, fl, t, phi, n) && phi < pr.margin) emit(0, k, 0, t, r, c, phi, n);
      }
    }
    for (int f = 0; f < sc.nf; ++f) {
      const DFree& F = sc.F[f];
      V x = v3(s + fro(f));
      // candidate targets of the body's bounding sphere (list reuses body slot 0's space)
      float brad = F.type == 0 ? sqrtf(F.half[0] * F.half[0] + F.half[1] * F.half[1] + F.half[2] * F.half[2])
                               : F.half[0];
      long lb = w.tl + (long)ND * (w.ntmax + 1);
      int cnt = 0;
      for (int t = 0; t < NT; ++t)
        if (near_target(s, x, brad, t, slack)) at(lb + cnt++) = (float)t;
      if (F.type == 0) {
        float R[9];
        ld9(w.fR + f * 9, R);
        for (int vtx = 0; vtx < 8; ++vtx) {
          V loc{(vtx & 1) ? F.half[0] : -F.half[0], (vtx & 2) ? F.half[1] : -F.half[1],
                (vtx & 4) ? F.half[2] : -F.half[2]};
          V c = x + rmv(R, loc);
          for (int q = 0; q < cnt; ++q) {
            int t = (int)at(lb + q);
            float phi;
            V n;
            if (pair(s, c, 0.f, 1, f, 0, t, phi, n) && phi < pr.margin) emit(1, f, vtx, t, 0.f, c, phi, n);
          }
        }
      } else {
        for (int q = 0; q < cnt; ++q) {
          int t = (int)at(lb + q);
          float phi;
          V n;
          if (pair(s, x, F.half[0], 2, f, 0, t, phi, n) && phi < pr.margin) emit(2, f, 0, t, F.half[0], x, phi, n);
        }
      }
    }
  }

  // ---------------------------------------------------------------- dynamics
  MSA_HD void chol_solve(float* x) const {
    for (int i = 0; i < nb; ++i) {
      float s = x[i];
      for (int k = 0; k < i; ++k) s -= at(w.L + i * ND + k) * x[k];
      x[i] = s / at(w.L + i * ND + i);
    }
    for (int i = nb - 1; i >= 0; --i) {
      float s = x[i];
      for (int k = i + 1; k < nb; ++k) s -= at(w.L + k * ND + i) * x[k];
      x[i] = s / at(w.L + i * ND + i);
    }
  }
  MSA_HD void mul6(long I, const float* v, float* r) const {
    for (int i = 0; i < 6; ++i) {
      float a = 0.f;
      for (int j = 0; j < 6; ++j) a += at(I + i * 6 + j) * v[j];
      r[i] = a;
    }
  }
  MSA_HD void mul6t(long I, const float* v, float* r) const {
    for (int i = 0; i < 6; ++i) {
      float a = 0.f;
      for (int j = 0; j < 6; ++j) a += at(I + j * 6 + i) * v[j];
      r[i] = a;
    }
  }
  MSA_HD void ld6(long e, float* v) const {
    for (int t = 0; t < 6; ++t) v[t] = at(e + t);
  }
  MSA_HD void st6(long e, const float* v) const {
    for (int t = 0; t < 6; ++t) at(e + t) = v[t];
  }
  MSA_HD void ad6(long e, const float* v) const {
    for (int t = 0; t < 6; ++t) at(e + t) += v[t];
  }
  static MSA_HD void crm6(const float* v, const float* m, float* r) {
    V w{v[0], v[1], v[2]}, vo{v[3], v[4], v[5]}, mw{m[0], m[1], m[2]}, mv{m[3], m[4], m[5]};
    V a = cross(w, mw), c = cross(w, mv) + cross(vo, mw);
    r[0] = a.x; r[1] = a.y; r[2] = a.z; r[3] = c.x; r[4] = c.y; r[5] = c.z;
  }
  static MSA_HD void crf6(const float* v, const float* f, float* r) {
    V w{v[0], v[1], v[2]}, vo{v[3], v[4], v[5]}, n{f[0], f[1], f[2]}, fl{f[3], f[4], f[5]};
    V a = cross(w, n) + cross(vo, fl), c = cross(w, fl);
    r[0] = a.x; r[1] = a.y; r[2] = a.z; r[3] = c.x; r[4] = c.y; r[5] = c.z;
  }

  MSA_HD void dynamics(long s, bool set_vel = true) {
    const DModel& M = *sc.M;
    const float h = pr.h;
    // composite inertias and the joint-space mass matrix (CRBA)
    for (int i = 0; i < nb * 36; ++i) at(w.kIc + i) = at(w.kI + i);
    for (int i = nb - 1; i >= 0; --i) {
      int par = M.parent[i];
      if (par >= 0)
        for (int t = 0; t < 36; ++t) at(w.kIc + par * 36 + t) += at(w.kIc + i * 36 + t);
    }
    for (int i = 0; i < ND * ND; ++i) at(w.L + i) = 0.f;
    for (int i = 0; i < nb; ++i) {
      float si[6], F[6];
      ld6(w.ks + i * 6, si);
      mul6(w.kIc + i * 36, si, F);
      for (int j = i; j >= 0; j = M.parent[j]) {
        float sj[6];
        ld6(w.ks + j * 6, sj);
        float v = 0.f;
        for (int t = 0; t < 6; ++t) v += sj[t] * F[t];
        at(w.L + i * ND + j) = v;
        at(w.L + j * ND + i) = v;
      }
    }
    // bias forces (RNEA with qdd = 0, gravity as a base acceleration -g)
    float C[ND];
    for (int i = 0; i < nb; ++i) {
      int par = M.parent[i];
      float si[6], vJ[6], v[6], a[6], t6[6], hv[6], fl[6];
      ld6(w.ks + i * 6, si);
      float qd = at(s + ND + i);
      for (int t = 0; t < 6; ++t) vJ[t] = si[t] * qd;
      if (par < 0) {
        for (int t = 0; t < 6; ++t) v[t] = vJ[t];
        a[0] = a[1] = a[2] = 0.f;
        a[3] = -pr.g[0]; a[4] = -pr.g[1]; a[5] = -pr.g[2];
      } else {
        ld6(w.rv + par * 6, v);
        for (int t = 0; t < 6; ++t) v[t] += vJ[t];
        ld6(w.ra + par * 6, a);
      }
      crm6(v, vJ, t6);
      for (int t = 0; t < 6; ++t) a[t] += t6[t];
      st6(w.rv + i * 6, v);
      st6(w.ra + i * 6, a);
      mul6(w.kI + i * 36, a, fl);
      mul6(w.kI + i * 36, v, hv);
      crf6(v, hv, t6);
      for (int t = 0; t < 6; ++t) fl[t] += t6[t];
      st6(w.rfl + i * 6, fl);
      st6(w.rff + i * 6, fl);
    }
    for (int i = nb - 1; i >= 0; --i) {
      float f[6], si[6];
      ld6(w.rff + i * 6, f);
      ld6(w.ks + i * 6, si);
      float tq = 0.f;
      for (int t = 0; t < 6; ++t) tq += si[t] * f[t];
      C[i] = tq;
      int par = M.parent[i];
      if (par >= 0) ad6(w.rff + par * 6, f);
    }
    // M~ = M + diag(arm), Cholesky in place (lower triangle)
    for (int j = 0; j < nb; ++j) at(w.L + j * ND + j) += at(w.arm + j);
    for (int j = 0; j < nb; ++j) {
      float d = at(w.L + j * ND + j);
      for (int k = 0; k < j; ++k) d -= at(w.L + j * ND + k) * at(w.L + j * ND + k);
      if (!(d > 0.f)) {
        status |= MS_DEGENERATE_BIT;
        d = 1e-30f;
      }
      float l = sqrtf(d);
      at(w.L + j * ND + j) = l;
      for (int i = j + 1; i < nb; ++i) {
        float sm = at(w.L + i * ND + j);
        for (int k = 0; k < j; ++k) sm -= at(w.L + i * ND + k) * at(w.L + j * ND + k);
        at(w.L + i * ND + j) = sm / l;
      }
    }
    float z[ND];
    for (int j = 0; j < nb; ++j) z[j] = at(w.tau + j) - C[j];
    chol_solve(z);
    for (int j = 0; j < ND; ++j) at(w.z + j) = j < nb ? z[j] : 0.f;
    if (!set_vel) return;
    for (int j = 0; j < ND; ++j) {
      float qd = at(s + ND + j);
      at(w.vR + j) = j < nb ? qd + h * z[j] : qd;
    }
    for (int x = 0; x < sc.na; ++x) at(w.vA + x) = at(s + axo(x) + 1) + h * ((0.f - at(w.xC + x)) / at(w.xM + x));
    for (int f = 0; f < sc.nf; ++f) {
      V v = v3(s + fro(f) + 8), om = v3(s + fro(f) + 12);
      V vF = v + V{pr.g[0], pr.g[1], pr.g[2]} * h;
      float Iw[9], Ii[9];
      ld9(w.fIw + f * 9, Iw);
      ld9(w.fIi + f * 9, Ii);
      V gy = cross(om, rmv(Iw, om));
      V wF = om - rmv(Ii, gy) * h;
      s3(w.vF + f * 6, vF);
      s3(w.vF + f * 6 + 3, wF);
    }
  }

  // ---------------------------------------------------------------- rows
  // contact direction di of contact ci: row data of the sides
  MSA_HD V dir(long e, int di) const { return v3(e + (di == 0 ? C_N : (di == 1 ? C_T1 : C_T2))); }
  // robot row J (into rJ) for contact ci (a robot contact), direction d
  MSA_HD void robot_row(int ci, int di, V d, V p, int body, float* J) const {
    const DModel& M = *sc.M;
    for (int j = 0; j < ND; ++j) J[j] = 0.f;
    int anc = M.anc[body];
    for (int j = 0; j < nb; ++j) {
      if (!((anc >> j) & 1)) continue;
      V a = v3(w.ka + j * 3);
      J[j] = M.jtype[j] == 0 ? dot(d, cross(a, p - v3(w.ko + j * 3))) : dot(d, a);
    }
  }
  MSA_HD float aux_J(int x, V d, V p, float sgn) const {
    V a = v3(w.xa + x * 3);
    return sgn * (at(w.xty + x) == 0.f ? dot(d, cross(a, p - v3(w.xo + x * 3))) : dot(d, a));
  }
  MSA_HD void rows() {
    const DModel& M = *sc.M;
    const float h = pr.h;
    for (int ci = 0; ci < nc; ++ci) {
      long e = w.con + (long)ci * CR;
      V n = v3(e + C_N), t1, t2;
      onb(n, t1, t2);
      s3(e + C_T1, t1);
      s3(e + C_T2, t2);
      V p = v3(e + C_P);
      const Ids id = ids(e);
      const int ok = id.ok, oi = id.oi, tk = id.tk, ti = id.ti;
      for (int di = 0; di < 3; ++di) {
        V d = di == 0 ? n : (di == 1 ? t1 : t2);
        float W = 0.f;
        if (ok == 0) {
          float J[ND], wv[ND];
          robot_row(ci, di, d, p, M.sph_body[oi], J);
          for (int j = 0; j < ND; ++j) wv[j] = J[j];
          chol_solve(wv);
          for (int j = 0; j < nb; ++j) W += J[j] * wv[j];
          long r = w.rJ + ((long)ci * 3 + di) * ND;
          long rr = w.rw + ((long)ci * 3 + di) * ND;
          for (int j = 0; j < ND; ++j) {
            at(r + j) = J[j];
            at(rr + j) = wv[j];
          }
        } else {
          W += free_W(oi, d, p, 1.f);
        }
        if (tk == 2) {
          float J = aux_J(ti, d, p, -1.f);
          W += J * (J / at(w.xM + ti));
        } else if (tk == 3) {
          W += free_W(ti, d, p, -1.f);
        }
        at(e + C_W + di) = W;
        if (!(W >= 1e-12f)) status |= MS_DEGENERATE_BIT;
      }
      float phi = at(e + C_PHI);
      at(e + C_BIAS) = phi >= 0.f ? phi / h : pr.beta * phi / h;
    }
    build_lims();
  }
  // joint-limit rows of the door / drawer joints (first in the canonical order)
  MSA_HD void build_lims() {
    nlim = 0;
    for (int x = 0; x < sc.na; ++x) {
      const DAux& A = sc.A[x];
      if (!A.has_limit) continue;
      float q = at(cur_s + axo(x));
      float glo = q - A.lo, ghi = A.hi - q;
      float Wx = 1.f / at(w.xM + x);
      if (glo < pr.margin) add_lim(x, 1.f, glo, Wx);
      if (ghi < pr.margin) add_lim(x, -1.f, ghi, Wx);
    }
  }
  long cur_s;  // state record of the substep being evaluated
  MSA_HD void add_lim(int x, float sgn, float gap, float Wx) {
    long e = w.lim + nlim * 4;
    at(e) = (float)x;
    at(e + 1) = sgn;
    at(e + 2) = gap >= 0.f ? gap / pr.h : pr.beta * gap / pr.h;
    at(e + 3) = Wx;
    ++nlim;
  }
  // free-body side: lin = sgn d, ang = sgn (p - x) x d; returns lin.M^-1 lin + ang.I^-1 ang
  MSA_HD void free_side(int f, V d, V p, float sgn, V& lin, V& ang) const {
    V rr = p - v3(cur_s + fro(f));
    lin = d * sgn;
    ang = cross(rr, d) * sgn;
  }
  MSA_HD float free_W(int f, V d, V p, float sgn) const {
    V lin, ang;
    free_side(f, d, p, sgn, lin, ang);
    float Ii[9];
    ld9(w.fIi + f * 9, Ii);
    V ilin = lin * at(w.fim + f);
    V iang = rmv(Ii, ang);
    return dot(lin, ilin) + dot(ang, iang);
  }

  // ---------------------------------------------------------------- Gauss-Seidel
  // side masks of a contact's row primitives: A = owner, B = target
  static constexpr int SA = 1, SB = 2, SAB = 3;
  MSA_HD float rowvel(int ci, int di, int sides = SAB) const {
    long e = w.con + (long)ci * CR;
    const Ids id = ids(e);
    const int ok = id.ok, oi = id.oi, tk = id.tk, ti = id.ti;
    V d = dir(e, di), p = v3(e + C_P);
    float r = 0.f;
    if (sides & SA) {
      if (ok == 0) {
        long rj = w.rJ + ((long)ci * 3 + di) * ND;
        for (int j = 0; j < nb; ++j) r += at(rj + j) * at(w.vR + j);
      } else {
        V lin, ang;
        free_side(oi, d, p, 1.f, lin, ang);
        r += dot(lin, v3(w.vF + oi * 6)) + dot(ang, v3(w.vF + oi * 6 + 3));
      }
    }
    if (sides & SB) {
      if (tk == 2) {
        r += aux_J(ti, d, p, -1.f) * at(w.vA + ti);
      } else if (tk == 3) {
        V lin, ang;
        free_side(ti, d, p, -1.f, lin, ang);
        r += dot(lin, v3(w.vF + ti * 6)) + dot(ang, v3(w.vF + ti * 6 + 3));
      }
    }
    return r;
  }
  MSA_HD void free_apply(int f, V lin, V ang, float dl) const {
    float Ii[9];
    ld9(w.fIi + f * 9, Ii);
    a3(w.vF + f * 6, lin * at(w.fim + f) * dl);
    a3(w.vF + f * 6 + 3, rmv(Ii, ang) * dl);
  }
  MSA_HD void apply(int ci, int di, float dl, int sides = SAB) const {
    long e = w.con + (long)ci * CR;
    const Ids id = ids(e);
    const int ok = id.ok, oi = id.oi, tk = id.tk, ti = id.ti;
    V d = dir(e, di), p = v3(e + C_P);
    if (sides & SA) {
      if (ok == 0) {
        long rw = w.rw + ((long)ci * 3 + di) * ND;
        for (int j = 0; j < nb; ++j) at(w.vR + j) += at(rw + j) * dl;
      } else {
        V lin, ang;
        free_side(oi, d, p, 1.f, lin, ang);
        free_apply(oi, lin, ang, dl);
      }
    }
    if (sides & SB) {
      if (tk == 2) {
        float J = aux_J(ti, d, p, -1.f);
        at(w.vA + ti) += (J / at(w.xM + ti)) * dl;
      } else if (tk == 3) {
        V lin, ang;
        free_side(ti, d, p, -1.f, lin, ang);
        free_apply(ti, lin, ang, dl);
      }
    }
  }
  MSA_HD bool row_ok(int ci, int di) const { return at(w.con + (long)ci * CR + C_W + di) >= 1e-12f; }

  // one limit row update (sweep it); records its pre-projection value
  MSA_HD void limit_update(int it, int li, bool tape) const {
    long e = w.lim + li * 4;
    int x = (int)at(e);
    float sgn = at(e + 1), bias = at(e + 2), W = at(e + 3);
    float r = sgn * at(w.vA + x) + bias;
    float y = at(w.llam + li) - r / W;
    if (tape) tape_at(it, li, 0) = y;
    float nl = y > 0.f ? y : 0.f;
    float dl = nl - at(w.llam + li);
    at(w.vA + x) += (sgn * W) * dl;
    at(w.llam + li) = nl;
  }
  // one contact's normal then friction-pair update (sweep it)
  MSA_HD void contact_update(int it, int ci, bool tape) const {
    long e = w.con + (long)ci * CR;
    long lm = w.lam + ci * 3;
    const int row = nlim + ci;
    if (row_ok(ci, 0)) {
      float r = rowvel(ci, 0) + at(e + C_BIAS);
      float y = at(lm) - r / at(e + C_W);
      if (tape) tape_at(it, row, 0) = y;
      float nl = y > 0.f ? y : 0.f;
      apply(ci, 0, nl - at(lm));
      at(lm) = nl;
    }
    if (row_ok(ci, 1) && row_ok(ci, 2)) {
      float r1 = rowvel(ci, 1), r2 = rowvel(ci, 2);
      float y1 = at(lm + 1) - r1 / at(e + C_W + 1);
      float y2 = at(lm + 2) - r2 / at(e + C_W + 2);
      if (tape) {
        tape_at(it, row, 1) = y1;
        tape_at(it, row, 2) = y2;
      }
      float o1, o2;
      disk_proj(y1, y2, pr.mu * at(lm), o1, o2);
      float d1 = o1 - at(lm + 1), d2 = o2 - at(lm + 2);
      apply(ci, 1, d1);
      apply(ci, 2, d2);
      at(lm + 1) = o1;
      at(lm + 2) = o2;
    }
  }
  MSA_HD void pgs(bool tape) {
    for (int i = 0; i < 3 * nc; ++i) at(w.lam + i) = 0.f;
    for (int i = 0; i < nlim; ++i) at(w.llam + i) = 0.f;
    for (int it = 0; it < pr.K; ++it) {
      for (int li = 0; li < nlim; ++li) limit_update(it, li, tape);
      for (int ci = 0; ci < nc; ++ci) contact_update(it, ci, tape);
    }
  }

  // ---------------------------------------------------------------- integrate
  MSA_HD static void quat_step(const float* Q, V om, float h, float* out, float* e, float* r, float& nq) {
    V th = om * h;
    float n2 = dot(th, th);
    float cw, sk;
    if (n2 < 1e-12f) {
      cw = 1.f - n2 / 8.f;
      sk = 0.5f - n2 / 48.f;
    } else {
      float nn = sqrtf(n2);
      cw = cosf(nn / 2.f);
      sk = sinf(nn / 2.f) / nn;
    }
    e[0] = cw; e[1] = th.x * sk; e[2] = th.y * sk; e[3] = th.z * sk;
    r[0] = e[0] * Q[0] - (e[1] * Q[1] + e[2] * Q[2] + e[3] * Q[3]);
    r[1] = e[0] * Q[1] + Q[0] * e[1] + (e[2] * Q[3] - e[3] * Q[2]);
    r[2] = e[0] * Q[2] + Q[0] * e[2] + (e[3] * Q[1] - e[1] * Q[3]);
    r[3] = e[0] * Q[3] + Q[0] * e[3] + (e[1] * Q[2] - e[2] * Q[1]);
    nq = sqrtf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    for (int t = 0; t < 4; ++t) out[t] = r[t] / nq;
  }
  MSA_HD void integrate(long s, long so) {
    const float h = pr.h;
    for (int j = 0; j < ND; ++j) {
      float v = at(w.vR + j);
      at(so + ND + j) = v;
      at(so + j) = j < nb ? at(s + j) + h * v : at(s + j);
    }
    for (int x = 0; x < AMAX; ++x) {
      if (x < sc.na) {
        float v = at(w.vA + x);
        at(so + axo(x) + 1) = v;
        at(so + axo(x)) = at(s + axo(x)) + h * v;
      } else {
        at(so + axo(x)) = at(s + axo(x));
        at(so + axo(x) + 1) = at(s + axo(x) + 1);
      }
      at(so + axo(x) + 2) = at(s + axo(x) + 2);
      at(so + axo(x) + 3) = at(s + axo(x) + 3);
    }
    for (int f = 0; f < sc.nf; ++f) {
      long fi = s + fro(f), fo = so + fro(f);
      V v = v3(w.vF + f * 6), om = v3(w.vF + f * 6 + 3);
      s3(fo, v3(fi) + v * h);
      at(fo + 3) = at(fi + 3);
      s3(fo + 8, v);
      at(fo + 11) = at(fi + 11);
      s3(fo + 12, om);
      at(fo + 15) = at(fi + 15);
      float Q[4] = {at(fi + 4), at(fi + 5), at(fi + 6), at(fi + 7)}, Qo[4], e[4], r[4], nq;
      quat_step(Q, om, h, Qo, e, r, nq);
      for (int t = 0; t < 4; ++t) at(fo + 4 + t) = Qo[t];
    }
  }

  // one substep from state record si to state record si + 1
  MSA_HD void forward_substep(int si, const float* u, bool tape) {
    long s = srec(si);
    cur_s = s;
    drive(s, u);
    kinematics(s);
    aux_frames(s);
    free_frames(s);
    contacts(s);
    dynamics(s);
    rows();
    pgs(tape);
    integrate(s, srec(si + 1));
  }

  // ================================================================ reverse
  // adjoints of the articulated quantities are gathered per body as
  // (sum of point adjoints F, sum of x cross xbar Mo, sum of direction
  // moments Md); joint k then receives a_k . (Mo - o_k x F + Md) over its
  // subtree (revolute) or a_k . F (prismatic).
  MSA_HD void acc_point(int bi, V x, V xb) const {
    a3(w.bacc + bi * 9, xb);
    a3(w.bacc + bi * 9 + 3, cross(x, xb));
  }
  MSA_HD void acc_dir(int bi, V d, V db) const { a3(w.bacc + bi * 9 + 6, cross(d, db)); }

  MSA_HD void integrate_bar(long s) {
    for (int j = 0; j < ND; ++j) integrate_bar_dof(j);
    for (int x = 0; x < AMAX; ++x) integrate_bar_aux(x);
    for (int f = 0; f < sc.nf; ++f) integrate_bar_free(s, f);
  }
  MSA_HD void integrate_bar_dof(int j) const {
    const float h = pr.h;
    long gA = w.gA, gB = w.gB;
    {
      float qb = at(gA + j), qdb = at(gA + ND + j);
      at(gB + j) += qb;
      at(w.vRb + j) = qdb + (j < nb ? h * qb : 0.f);
    }
  }
  MSA_HD void integrate_bar_aux(int x) const {
    const float h = pr.h;
    long gA = w.gA, gB = w.gB;
    {
      if (x < sc.na) {
        float qb = at(gA + axo(x)), qdb = at(gA + axo(x) + 1);
        at(gB + axo(x)) += qb;
        at(w.vAb + x) = qdb + h * qb;
      } else {
        at(gB + axo(x)) += at(gA + axo(x));
        at(gB + axo(x) + 1) += at(gA + axo(x) + 1);
      }
    }
  }
  MSA_HD void integrate_bar_free(long s, int f) const {
    const float h = pr.h;
    long gA = w.gA, gB = w.gB;
    {
      long go = gA + fro(f), gi = gB + fro(f);
      V xb = v3(go);
      a3(gi, xb);
      s3(w.vFb + f * 6, v3(go + 8) + xb * h);
      // Q+ = normalize(exp(h w+) (x) Q)
      long fi = s + fro(f);
      float Q[4] = {at(fi + 4), at(fi + 5), at(fi + 6), at(fi + 7)}, Qo[4], e[4], r[4], nq;
      V om = v3(w.vF + f * 6 + 3);
      quat_step(Q, om, h, Qo, e, r, nq);
      float Qob[4] = {at(go + 4), at(go + 5), at(go + 6), at(go + 7)};
      float pq = Qo[0] * Qob[0] + Qo[1] * Qob[1] + Qo[2] * Qob[2] + Qo[3] * Qob[3];
      float rb[4];
      for (int t = 0; t < 4; ++t) rb[t] = (Qob[t] - Qo[t] * pq) / nq;
      at(gi + 4) += e[0] * rb[0] + e[1] * rb[1] + e[2] * rb[2] + e[3] * rb[3];
      at(gi + 5) += -e[1] * rb[0] + e[0] * rb[1] + e[3] * rb[2] - e[2] * rb[3];
      at(gi + 6) += -e[2] * rb[0] - e[3] * rb[1] + e[0] * rb[2] + e[1] * rb[3];
      at(gi + 7) += -e[3] * rb[0] + e[2] * rb[1] - e[1] * rb[2] + e[0] * rb[3];
      float eb0 = Q[0] * rb[0] + Q[1] * rb[1] + Q[2] * rb[2] + Q[3] * rb[3];
      V eb{-Q[1] * rb[0] + Q[0] * rb[1] - Q[3] * rb[2] + Q[2] * rb[3],
           -Q[2] * rb[0] + Q[3] * rb[1] + Q[0] * rb[2] - Q[1] * rb[3],
           -Q[3] * rb[0] - Q[2] * rb[1] + Q[1] * rb[2] + Q[0] * rb[3]};
      V th = om * h;
      float n2 = dot(th, th);
      float sk, n2b;
      if (n2 < 1e-12f) {
        sk = 0.5f - n2 / 48.f;
        float skb = dot(th, eb);
        n2b = -eb0 / 8.f - skb / 48.f;
      } else {
        float nn = sqrtf(n2);
        float sn = sinf(nn / 2.f), cs = cosf(nn / 2.f);
        sk = sn / nn;
        float skb = dot(th, eb);
        float nnb = -0.5f * sn * eb0 + skb * (cs / (2.f * nn) - sn / (nn * nn));
        n2b = nnb / (2.f * nn);
      }
      V thb = eb * sk + th * (2.f * n2b);
      s3(w.vFb + f * 6 + 3, v3(go + 12) + thb * h);
    }
  }

  // --------------------------------------------------------------- Gauss-Seidel^T
  // adjoint of a free side's row vectors lin = sgn d, ang = sgn (p - x) x d,
  // folded at once into the direction, contact-point and body-position adjoints
  MSA_HD void free_row_bar(int ci, int di, int f, float sgn, V linb, V angb) const {
    long e = w.con + (long)ci * CR, cb = w.conb + (long)ci * CB;
    V d = dir(e, di), p = v3(e + C_P);
    V rr = p - v3(cur_s + fro(f));
    a3(cb + B_D + di * 3, linb * sgn + cross(angb, rr) * sgn);
    V rrb = cross(d, angb) * sgn;
    a3(cb + B_P, rrb);
    a3(w.fb + f * FB + F_XB, -rrb);
  }
  // a door / drawer target's Jacobian entry J = -(d . (a x (p - o))) (revolute)
  // or -(d . a) (prismatic): its adjoint Jb goes at once to the direction and
  // contact-point adjoints (the joint axis and origin do not move)
  MSA_HD void aux_J_bar(long e, long cb, int di, int ti, float Jb) const {
    V d = dir(e, di), a = v3(w.xa + ti * 3);
    if (at(w.xty + ti) == 0.f) {
      V ev = v3(e + C_P) - v3(w.xo + ti * 3);
      a3(cb + B_D + di * 3, -(cross(a, ev) * Jb));
      a3(cb + B_P, -(cross(d, a) * Jb));
    } else {
      a3(cb + B_D + di * 3, -(a * Jb));
    }
  }
  // adjoint of r = J . v (v = the velocities before the update): Jbar += rb v, vbar += rb J
  MSA_HD void rowvel_bar(int ci, int di, float rb, int sides = SAB) const {
    long e = w.con + (long)ci * CR;
    const Ids id = ids(e);
    const int ok = id.ok, oi = id.oi, tk = id.tk, ti = id.ti;
    V d = dir(e, di), p = v3(e + C_P);
    if (sides & SA) {
      if (ok == 0) {
        long rj = w.rJ + ((long)ci * 3 + di) * ND, rjb = w.rJb + ((long)ci * 3 + di) * ND;
        for (int j = 0; j < nb; ++j) {
          at(rjb + j) += rb * at(w.vR + j);
          at(w.vRb + j) += rb * at(rj + j);
        }
      } else {
        V lin, ang;
        free_side(oi, d, p, 1.f, lin, ang);
        free_row_bar(ci, di, oi, 1.f, v3(w.vF + oi * 6) * rb, v3(w.vF + oi * 6 + 3) * rb);
        a3(w.vFb + oi * 6, lin * rb);
        a3(w.vFb + oi * 6 + 3, ang * rb);
      }
    }
    if (sides & SB) {
      if (tk == 2) {
        float J = aux_J(ti, d, p, -1.f);
        aux_J_bar(e, w.conb + (long)ci * CB, di, ti, rb * at(w.vA + ti));
        at(w.vAb + ti) += rb * J;
      } else if (tk == 3) {
        V lin, ang;
        free_side(ti, d, p, -1.f, lin, ang);
        free_row_bar(ci, di, ti, -1.f, v3(w.vF + ti * 6) * rb, v3(w.vF + ti * 6 + 3) * rb);
        a3(w.vFb + ti * 6, lin * rb);
        a3(w.vFb + ti * 6 + 3, ang * rb);
      }
    }
  }
  // adjoint of a free side's v += (lin / m) dl, w += (I^-1 ang) dl; returns its part of dlbar
  MSA_HD float free_apply_bar(int ci, int di, int f, float sgn, float dl) const {
    long e = w.con + (long)ci * CR;
    V d = dir(e, di), p = v3(e + C_P);
    V lin, ang;
    free_side(f, d, p, sgn, lin, ang);
    float Ii[9];
    ld9(w.fIi + f * 9, Ii);
    float im = at(w.fim + f);
    V vb = v3(w.vFb + f * 6), wb = v3(w.vFb + f * 6 + 3);
    float dlb = dot(lin * im, vb) + dot(rmv(Ii, ang), wb);
    V iab = wb * dl;
    long ib = w.fb + f * FB + F_IIB;
    float iv[3] = {iab.x, iab.y, iab.z};
    for (int r = 0; r < 3; ++r) {
      at(ib + r * 3 + 0) += iv[r] * ang.x;
      at(ib + r * 3 + 1) += iv[r] * ang.y;
      at(ib + r * 3 + 2) += iv[r] * ang.z;
    }
    free_row_bar(ci, di, f, sgn, vb * (im * dl), rtmv(Ii, iab));
    return dlb;
  }
  // adjoint of v += w dl: returns dlbar = w . vbar and accumulates wbar += vbar dl
  MSA_HD float apply_bar(int ci, int di, float dl, int sides = SAB) const {
    long e = w.con + (long)ci * CR;
    const Ids id = ids(e);
    const int ok = id.ok, oi = id.oi, tk = id.tk, ti = id.ti;
    V d = dir(e, di), p = v3(e + C_P);
    float dlb = 0.f;
    if (sides & SA) {
      if (ok == 0) {
        long rw = w.rw + ((long)ci * 3 + di) * ND, rwb = w.rwb + ((long)ci * 3 + di) * ND;
        for (int j = 0; j < nb; ++j) {
          dlb += at(rw + j) * at(w.vRb + j);
          at(rwb + j) += at(w.vRb + j) * dl;
        }
      } else {
        dlb += free_apply_bar(ci, di, oi, 1.f, dl);
      }
    }
    if (sides & SB) {
      if (tk == 2) {
        float J = aux_J(ti, d, p, -1.f);
        float Mx = at(w.xM + ti);
        dlb += (J / Mx) * at(w.vAb + ti);
        aux_J_bar(e, w.conb + (long)ci * CB, di, ti, at(w.vAb + ti) * dl / Mx);
      } else if (tk == 3) {
        dlb += free_apply_bar(ci, di, ti, -1.f, dl);
      }
    }
    return dlb;
  }
  MSA_HD float prev_normal(int it, int ci) const {
    if (it == 0 || !row_ok(ci, 0)) return 0.f;
    float y = tape_at(it - 1, nlim + ci, 0);
    return y > 0.f ? y : 0.f;
  }
  MSA_HD void prev_fric(int it, int ci, float& o1, float& o2) const {
    o1 = o2 = 0.f;
    if (it == 0) return;
    disk_proj(tape_at(it - 1, nlim + ci, 1), tape_at(it - 1, nlim + ci, 2), pr.mu * prev_normal(it, ci), o1, o2);
  }
  // reverse of limit_update (sweep it): the velocities are set back to
  // their values before the update, the adjoints carried through it
  MSA_HD void limit_bar(int it, int li) const {
    long e = w.lim + li * 4;
    int x = (int)at(e);
    float sgn = at(e + 1), W = at(e + 3);
    float y = tape_at(it, li, 0);
    float nl = y > 0.f ? y : 0.f;
    float pl = 0.f;
    if (it > 0) {
      float yp = tape_at(it - 1, li, 0);
      pl = yp > 0.f ? yp : 0.f;
    }
    float dl = nl - pl;
    at(w.vA + x) -= (sgn * W) * dl;
    float dlb = sgn * W * at(w.vAb + x);
    float nlb = at(w.llamb + li) + dlb;
    float lold = -dlb;
    float yb = y > 0.f ? nlb : 0.f;
    lold += yb;
    float rb = -yb / W;
    at(w.vAb + x) += rb * sgn;
    at(w.limb + li) += rb;
    at(w.llamb + li) = lold;
  }
  // contact ci's normal impulse after sweep it's normal update (the
  // friction disk radius is mu times it)
  MSA_HD float normal_after(int it, int ci) const {
    if (!row_ok(ci, 0)) return 0.f;
    float y = tape_at(it, nlim + ci, 0);
    return y > 0.f ? y : 0.f;
  }
  // ---- register form of a contact's reverse update (free-body owner;
  // plane, furniture or free-body target): the sides' velocities, adjoints
  // and inverse inertias are read once, updated in registers and written
  // back once.  The arithmetic is that of apply / apply_bar / rowvel /
  // rowvel_bar / free_row_bar for these side kinds.
  struct FSide {
    int f;
    float sgn, im;
    V x, v, w, vb, wb, xb;
    float Ii[9], IIb[9];
  };
  MSA_HD void fs_load(FSide& S, int f, float sgn) const {
    S.f = f;
    S.sgn = sgn;
    S.im = at(w.fim + f);
    S.x = v3(cur_s + fro(f));
    ld9(w.fIi + f * 9, S.Ii);
    S.v = v3(w.vF + f * 6);
    S.w = v3(w.vF + f * 6 + 3);
    S.vb = v3(w.vFb + f * 6);
    S.wb = v3(w.vFb + f * 6 + 3);
    S.xb = V{0.f, 0.f, 0.f};
    for (int t = 0; t < 9; ++t) S.IIb[t] = 0.f;
  }
  MSA_HD void fs_store(const FSide& S) const {
    s3(w.vF + S.f * 6, S.v);
    s3(w.vF + S.f * 6 + 3, S.w);
    s3(w.vFb + S.f * 6, S.vb);
    s3(w.vFb + S.f * 6 + 3, S.wb);
    long fb = w.fb + S.f * FB;
    a3(fb + F_XB, S.xb);
    for (int t = 0; t < 9; ++t) at(fb + F_IIB + t) += S.IIb[t];
  }
  struct RowAcc {
    V p, d[3], db[3], pb;
  };
  // (lin, ang) of side S for direction d: lin = sgn d, ang = sgn (p - x) x d
  MSA_HD static void fs_row(const FSide& S, const RowAcc& A, int di, V& lin, V& ang) {
    lin = A.d[di] * S.sgn;
    ang = cross(A.p - S.x, A.d[di]) * S.sgn;
  }
  MSA_HD static void fs_row_bar(FSide& S, RowAcc& A, int di, V linb, V angb) {
    V rr = A.p - S.x;
    A.db[di] = A.db[di] + linb * S.sgn + cross(angb, rr) * S.sgn;
    V rrb = cross(A.d[di], angb) * S.sgn;
    A.pb = A.pb + rrb;
    S.xb = S.xb - rrb;
  }
  MSA_HD static void fs_apply(FSide& S, const RowAcc& A, int di, float dl) {
    V lin, ang;
    fs_row(S, A, di, lin, ang);
    S.v = S.v + lin * S.im * dl;
    S.w = S.w + rmv(S.Ii, ang) * dl;
  }
  MSA_HD static float fs_rowvel(const FSide& S, const RowAcc& A, int di) {
    V lin, ang;
    fs_row(S, A, di, lin, ang);
    return dot(lin, S.v) + dot(ang, S.w);
  }
  MSA_HD static float fs_apply_bar(FSide& S, RowAcc& A, int di, float dl) {
    V lin, ang;
    fs_row(S, A, di, lin, ang);
    float dlb = dot(lin * S.im, S.vb) + dot(rmv(S.Ii, ang), S.wb);
    V iab = S.wb * dl;
    float iv[3] = {iab.x, iab.y, iab.z}, av[3] = {ang.x, ang.y, ang.z};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) S.IIb[r * 3 + c] += iv[r] * av[c];
    fs_row_bar(S, A, di, S.vb * (S.im * dl), rtmv(S.Ii, iab));
    return dlb;
  }
  MSA_HD static void fs_rowvel_bar(FSide& S, RowAcc& A, int di, float rb) {
    V lin, ang;
    fs_row(S, A, di, lin, ang);
    fs_row_bar(S, A, di, S.v * rb, S.w * rb);
    S.vb = S.vb + lin * rb;
    S.wb = S.wb + ang * rb;
  }
  // a door / drawer target in registers: J = -(d . (a x (p - o))) (revolute)
  // or -(d . a) (prismatic), v += (J / M) dl; the arithmetic of the aux
  // branches of apply / apply_bar / rowvel / rowvel_bar / aux_J_bar, with the
  // direction and point adjoints accumulated in the RowAcc
  struct XSide {
    int x, type;
    V a, o;
    float M, v, vb;
  };
  MSA_HD void xs_load(XSide& X, int x) const {
    X.x = x;
    X.type = (int)at(w.xty + x);
    X.a = v3(w.xa + x * 3);
    X.o = v3(w.xo + x * 3);
    X.M = at(w.xM + x);
    X.v = at(w.vA + x);
    X.vb = at(w.vAb + x);
  }
  MSA_HD void xs_store(const XSide& X) const {
    at(w.vA + X.x) = X.v;
    at(w.vAb + X.x) = X.vb;
  }
  MSA_HD static float xs_J(const XSide& X, const RowAcc& A, int di) {
    return X.type == 0 ? -dot(A.d[di], cross(X.a, A.p - X.o)) : -dot(A.d[di], X.a);
  }
  MSA_HD static void xs_J_bar(const XSide& X, RowAcc& A, int di, float Jb) {
    if (X.type == 0) {
      A.db[di] = A.db[di] - cross(X.a, A.p - X.o) * Jb;
      A.pb = A.pb - cross(A.d[di], X.a) * Jb;
    } else {
      A.db[di] = A.db[di] - X.a * Jb;
    }
  }
  MSA_HD static void xs_apply(XSide& X, const RowAcc& A, int di, float dl) { X.v += (xs_J(X, A, di) / X.M) * dl; }
  MSA_HD static float xs_apply_bar(XSide& X, RowAcc& A, int di, float dl) {
    const float J = xs_J(X, A, di);
    xs_J_bar(X, A, di, X.vb * dl / X.M);
    return (J / X.M) * X.vb;
  }
  MSA_HD static float xs_rowvel(const XSide& X, const RowAcc& A, int di) { return xs_J(X, A, di) * X.v; }
  MSA_HD static void xs_rowvel_bar(XSide& X, RowAcc& A, int di, float rb) {
    const float J = xs_J(X, A, di);
    xs_J_bar(X, A, di, rb * X.v);
    X.vb += rb * J;
  }
  MSA_HD void contact_bar_reg(int it, int ci, int oi, int tk, int ti) const {
    const bool two = tk == 3;
    FSide A, B;
    fs_load(A, oi, 1.f);
    if (two) fs_load(B, ti, -1.f);
    contact_bar_core(it, ci, A, B, two);
    fs_store(A);
    if (two) fs_store(B);
  }
  // reverse of a run of rows ci0 .. ci0 + n - 1 between one free body and
  // static targets, last row first, with the body's side in registers
  MSA_HD void contact_group_bar(int it, int ci0, int n) const {
    FSide A, B;
    fs_load(A, ids(w.con + (long)ci0 * CR).oi, 1.f);
    for (int ci = ci0 + n - 1; ci >= ci0; --ci) contact_bar_core(it, ci, A, B, false);
    fs_store(A);
  }
  // the register form's arithmetic between the sides' load and store
  MSA_HD void contact_bar_core(int it, int ci, FSide& A, FSide& B, bool two) const {
    const long e = w.con + (long)ci * CR, cb = w.conb + (long)ci * CB, lb = w.lamb + ci * 3;
    const int row = nlim + ci;
    RowAcc R;
    R.p = v3(e + C_P);
    R.d[0] = v3(e + C_N);
    R.d[1] = v3(e + C_T1);
    R.d[2] = v3(e + C_T2);
    for (int k = 0; k < 3; ++k) R.db[k] = V{0.f, 0.f, 0.f};
    R.pb = V{0.f, 0.f, 0.f};
    const float W0 = at(e + C_W), W1 = at(e + C_W + 1), W2 = at(e + C_W + 2);
    float lb0 = at(lb), lb1 = at(lb + 1), lb2 = at(lb + 2);
    float Wb0 = 0.f, Wb1 = 0.f, Wb2 = 0.f, biasb = 0.f;
    if (W1 >= 1e-12f && W2 >= 1e-12f) {
      float y1 = tape_at(it, row, 1), y2 = tape_at(it, row, 2);
      float lim = pr.mu * normal_after(it, ci);
      float o1, o2, p1, p2;
      bool proj = disk_proj(y1, y2, lim, o1, o2);
      prev_fric(it, ci, p1, p2);
      float d1 = o1 - p1, d2 = o2 - p2;
      fs_apply(A, R, 2, -d2);
      if (two) fs_apply(B, R, 2, -d2);
      fs_apply(A, R, 1, -d1);
      if (two) fs_apply(B, R, 1, -d1);
      float d1b = fs_apply_bar(A, R, 1, d1);
      if (two) d1b += fs_apply_bar(B, R, 1, d1);
      float d2b = fs_apply_bar(A, R, 2, d2);
      if (two) d2b += fs_apply_bar(B, R, 2, d2);
      float yb1, yb2, limb;
      fric_bar(y1, y2, lim, proj, lb1 + d1b, lb2 + d2b, yb1, yb2, limb);
      lb0 += pr.mu * limb;
      float l1 = -d1b + yb1, l2 = -d2b + yb2;
      float r1 = fs_rowvel(A, R, 1) + (two ? fs_rowvel(B, R, 1) : 0.f);
      float r2 = fs_rowvel(A, R, 2) + (two ? fs_rowvel(B, R, 2) : 0.f);
      float rb1 = -yb1 / W1, rb2 = -yb2 / W2;
      Wb1 += yb1 * r1 / (W1 * W1);
      Wb2 += yb2 * r2 / (W2 * W2);
      fs_rowvel_bar(A, R, 1, rb1);
      if (two) fs_rowvel_bar(B, R, 1, rb1);
      fs_rowvel_bar(A, R, 2, rb2);
      if (two) fs_rowvel_bar(B, R, 2, rb2);
      lb1 = l1;
      lb2 = l2;
    }
    if (W0 >= 1e-12f) {
      float y = tape_at(it, row, 0);
      float nl = y > 0.f ? y : 0.f;
      float pl = prev_normal(it, ci);
      float dl = nl - pl;
      fs_apply(A, R, 0, -dl);
      if (two) fs_apply(B, R, 0, -dl);
      float dlb = fs_apply_bar(A, R, 0, dl);
      if (two) dlb += fs_apply_bar(B, R, 0, dl);
      float lold, yb;
      normal_bar(y, lb0 + dlb, dlb, lold, yb);
      float r = fs_rowvel(A, R, 0) + (two ? fs_rowvel(B, R, 0) : 0.f) + at(e + C_BIAS);
      float rb = -yb / W0;
      Wb0 += yb * r / (W0 * W0);
      biasb += rb;
      fs_rowvel_bar(A, R, 0, rb);
      if (two) fs_rowvel_bar(B, R, 0, rb);
      lb0 = lold;
    }
    at(lb) = lb0;
    at(lb + 1) = lb1;
    at(lb + 2) = lb2;
    for (int k = 0; k < 3; ++k) a3(cb + B_D + k * 3, R.db[k]);
    a3(cb + B_P, R.pb);
    at(cb + B_W) += Wb0;
    at(cb + B_W + 1) += Wb1;
    at(cb + B_W + 2) += Wb2;
    at(cb + B_BIAS) += biasb;
  }

  // reverse of contact_update (sweep it): friction pair, then normal
  MSA_HD void contact_bar(int it, int ci) const {
    {
      const Ids id = ids(w.con + (long)ci * CR);
      if (id.ok != 0 && id.tk != 2) {
        contact_bar_reg(it, ci, id.oi, id.tk, id.ti);
        return;
      }
    }
    long e = w.con + (long)ci * CR, cb = w.conb + (long)ci * CB;
    long lb = w.lamb + ci * 3;
    const int row = nlim + ci;
    if (row_ok(ci, 1) && row_ok(ci, 2)) {
      float y1 = tape_at(it, row, 1), y2 = tape_at(it, row, 2);
      float lim = pr.mu * normal_after(it, ci);
      float o1, o2, p1, p2;
      bool proj = disk_proj(y1, y2, lim, o1, o2);
      prev_fric(it, ci, p1, p2);
      float d1 = o1 - p1, d2 = o2 - p2;
      apply(ci, 2, -d2);
      apply(ci, 1, -d1);
      float d1b = apply_bar(ci, 1, d1), d2b = apply_bar(ci, 2, d2);
      float yb1, yb2, limb;
      fric_bar(y1, y2, lim, proj, at(lb + 1) + d1b, at(lb + 2) + d2b, yb1, yb2, limb);
      at(lb) += pr.mu * limb;
      float l1 = -d1b + yb1, l2 = -d2b + yb2;
      float W1 = at(e + C_W + 1), W2 = at(e + C_W + 2);
      float r1 = rowvel(ci, 1), r2 = rowvel(ci, 2);
      float rb1 = -yb1 / W1, rb2 = -yb2 / W2;
      at(cb + B_W + 1) += yb1 * r1 / (W1 * W1);
      at(cb + B_W + 2) += yb2 * r2 / (W2 * W2);
      rowvel_bar(ci, 1, rb1);
      rowvel_bar(ci, 2, rb2);
      at(lb + 1) = l1;
      at(lb + 2) = l2;
    }
    if (row_ok(ci, 0)) {
      float y = tape_at(it, row, 0);
      float nl = y > 0.f ? y : 0.f;
      float pl = prev_normal(it, ci);
      float dl = nl - pl;
      apply(ci, 0, -dl);
      float dlb = apply_bar(ci, 0, dl);
      float lold, yb;
      normal_bar(y, at(lb) + dlb, dlb, lold, yb);
      float W = at(e + C_W);
      float r = rowvel(ci, 0) + at(e + C_BIAS);
      float rb = -yb / W;
      at(cb + B_W) += yb * r / (W * W);
      at(cb + B_BIAS) += rb;
      rowvel_bar(ci, 0, rb);
      at(lb) = lold;
    }
  }
  // scalar parts of the reverse updates, shared with the wavefront kernel.
  // normal: nl = max(0, y), dl = nl - lold; given nlbar (incl. dlbar) and
  // dlbar, returns the adjoint of lold and ybar
  static MSA_HD void normal_bar(float y, float nlb, float dlb, float& lold, float& yb) {
    yb = y > 0.f ? nlb : 0.f;
    lold = -dlb + yb;
  }
  // friction pair: from the adjoints of the projected values (incl. dlbar)
  // to the adjoints of the unprojected values and of the disk radius
  static MSA_HD void fric_bar(float y1, float y2, float lim, bool proj, float yb1p, float yb2p, float& yb1,
                              float& yb2, float& limb) {
    yb1 = yb1p;
    yb2 = yb2p;
    limb = 0.f;
    if (proj) {
      if (lim > 0.f) {
        float nn = sqrtf(y1 * y1 + y2 * y2);
        float u1 = y1 / nn, u2 = y2 / nn;
        float g = u1 * yb1 + u2 * yb2;
        limb = g;
        float sc2 = lim / nn;
        yb1 = sc2 * (yb1 - u1 * g);
        yb2 = sc2 * (yb2 - u2 * g);
      } else {
        yb1 = 0.f;
        yb2 = 0.f;
      }
    }
  }
  MSA_HD void pgs_bar() {
    for (int i = 0; i < 3 * nc; ++i) at(w.lamb + i) = 0.f;
    for (int i = 0; i < nlim; ++i) at(w.llamb + i) = 0.f;
    for (int it = pr.K - 1; it >= 0; --it) {
      for (int ci = nc - 1; ci >= 0; --ci) contact_bar(it, ci);
      for (int li = nlim - 1; li >= 0; --li) limit_bar(it, li);
    }
  }

  // --------------------------------------------------------------- rows^T
  // adjoint of a free side's share of W, lin . lin / m + ang . I^-1 ang,
  // with lin = sgn d, ang = sgn (p - x) x d
  MSA_HD void free_side_bar(int f, V d, V p, float sgn, float Wb, V& db, V& pb) const {
    V lin, ang;
    free_side(f, d, p, sgn, lin, ang);
    float Ii[9];
    ld9(w.fIi + f * 9, Ii);
    float im = at(w.fim + f);
    V linb = lin * (2.f * Wb * im);
    V angb = (rmv(Ii, ang) + rtmv(Ii, ang)) * Wb;
    long ib = w.fb + f * FB + F_IIB;
    float av[3] = {ang.x, ang.y, ang.z};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) at(ib + r * 3 + c) += Wb * av[r] * av[c];
    V rr = p - v3(cur_s + fro(f));
    db = db + linb * sgn + cross(angb, rr) * sgn;
    V rrb = cross(d, angb) * sgn;
    pb = pb + rrb;
    a3(w.fb + f * FB + F_XB, -rrb);
  }
  // robot_side = false: the robot owners' rows are reversed elsewhere (the
  // wavefront kernel spreads them over lanes); M~bar must be zeroed before
  MSA_HD void rows_bar(bool robot_side = true) {
    for (int ci = 0; ci < nc; ++ci) rows_bar_one(ci, robot_side);
    for (int li = 0; li < nlim; ++li) rows_bar_limit(li);
  }
  // rows^T of contact ci (touches the contact's own adjoint record and its
  // sides' accumulators)
  MSA_HD void rows_bar_one(int ci, bool robot_side) const {
    const DModel& M = *sc.M;
    {
      long e = w.con + (long)ci * CR, cb = w.conb + (long)ci * CB;
      const Ids id = ids(e);
      const int ok = id.ok, oi = id.oi, tk = id.tk, ti = id.ti;
      V p = v3(e + C_P);
      V pb{0.f, 0.f, 0.f};
      for (int di = 0; di < 3; ++di) {
        V d = dir(e, di);
        V db{0.f, 0.f, 0.f};
        float Wb = at(cb + B_W + di);
        if (ok == 0 && !robot_side) {
          // nothing: this side is handled by the caller
        } else if (ok == 0) {
          long rj = w.rJ + ((long)ci * 3 + di) * ND, rwv = w.rw + ((long)ci * 3 + di) * ND;
          long rjb = w.rJb + ((long)ci * 3 + di) * ND, rwb = w.rwb + ((long)ci * 3 + di) * ND;
          float Jb[ND], al[ND];
          for (int j = 0; j < ND; ++j) {
            Jb[j] = at(rjb + j) + Wb * at(rwv + j);
            al[j] = at(rwb + j) + Wb * at(rj + j);
          }
          // w = M~^-1 J: Jbar += M~^-1 wbar, M~bar -= (M~^-1 wbar) w^T
          chol_solve(al);
          for (int r = 0; r < nb; ++r) {
            Jb[r] += al[r];
            for (int c = 0; c < nb; ++c) at(w.Mb + r * ND + c) -= al[r] * at(rwv + c);
          }
          int body = M.sph_body[oi];
          int anc = M.anc[body];
          for (int j = 0; j < nb; ++j) {
            if (!((anc >> j) & 1) || Jb[j] == 0.f) continue;
            V a = v3(w.ka + j * 3);
            if (M.jtype[j] == 0) {
              V o = v3(w.ko + j * 3);
              V ev = p - o;
              db = db + cross(a, ev) * Jb[j];
              acc_dir(j, a, cross(ev, d) * Jb[j]);
              V eb = cross(d, a) * Jb[j];
              pb = pb + eb;
              acc_point(j, o, -eb);
            } else {
              db = db + a * Jb[j];
              acc_dir(j, a, d * Jb[j]);
            }
          }
        } else {
          free_side_bar(oi, d, p, 1.f, Wb, db, pb);
        }
        if (tk == 2) {
          float J = aux_J(ti, d, p, -1.f);
          float Jb = Wb * 2.f * J / at(w.xM + ti);
          V a = v3(w.xa + ti * 3);
          if (sc.A[ti].type == 0) {
            V ev = p - v3(w.xo + ti * 3);
            db = db - cross(a, ev) * Jb;
            pb = pb - cross(d, a) * Jb;
          } else {
            db = db - a * Jb;
          }
        } else if (tk == 3) {
          free_side_bar(ti, d, p, -1.f, Wb, db, pb);
        }
        a3(cb + B_D + di * 3, db);
      }
      a3(cb + B_P, pb);
    }
  }
  // rows^T of joint-limit row li: its bias depends on the joint position
  MSA_HD void rows_bar_limit(int li) const {
    const float h = pr.h;
    {
      long e = w.lim + li * 4;
      int x = (int)at(e);
      float sgn = at(e + 1);
      const DAux& A = sc.A[x];
      float q = at(cur_s + axo(x));
      float gap = sgn > 0.f ? q - A.lo : A.hi - q;
      float k = gap >= 0.f ? 1.f / h : pr.beta / h;
      at(w.xb + x * XB + X_QB) += at(w.limb + li) * k * sgn;
    }
  }

  // --------------------------------------------------------------- dynamics^T
  // drive^T of DoF j, tb = the adjoint of its torque
  MSA_HD void drive_bar_one(int j, float tb) const {
    const DModel& M = *sc.M;
    const float h = pr.h;
    const long gB = w.gB;
    float dmp = M.damp[j];
    if (pr.mode == 0) {
      at(w.ub + j) += tb;
      at(gB + ND + j) -= dmp * tb;
    } else {
      bool vel = M.veldof[j] != 0;
      float kp = vel ? 0.f : M.kp[j], kd = M.kd[j];
      if (pr.mode == 1) at(w.ub + j) += (vel ? kd : kp) * tb;
      else at(w.ub + j) += tb;
      at(gB + j) -= kp * tb;
      at(gB + ND + j) -= (h * kp + kd + dmp) * tb;
    }
  }
  MSA_HD void dynamics_bar(long s, const float* u) {
    const DModel& M = *sc.M;
    const float h = pr.h;
    long gB = w.gB;
    // vR = qd + h z, z = M~^-1 (tau - C)
    float lz[ND];
    for (int j = 0; j < ND; ++j) {
      at(gB + ND + j) += at(w.vRb + j);
      lz[j] = j < nb ? h * at(w.vRb + j) : 0.f;
    }
    chol_solve(lz);
    for (int r = 0; r < nb; ++r)
      for (int c = 0; c < nb; ++c) at(w.Mb + r * ND + c) -= lz[r] * at(w.z + c);
    // drive^T (tau bar = lz)
    for (int j = 0; j < nb; ++j) drive_bar_one(j, lz[j]);
    // CRBA^T: M_ij = s_j . (Ic_i s_i), j an ancestor of i (or i)
    for (int i = 0; i < nb * 36; ++i) at(w.Ib + i) = 0.f;
    for (int i = 0; i < nb * 6; ++i) at(w.sb + i) = 0.f;
    for (int i = 0; i < nb; ++i) {
      float si[6], F[6], Fb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      ld6(w.ks + i * 6, si);
      mul6(w.kIc + i * 36, si, F);
      for (int j = i; j >= 0; j = M.parent[j]) {
        float c = j == i ? at(w.Mb + i * ND + i) : at(w.Mb + i * ND + j) + at(w.Mb + j * ND + i);
        float sj[6];
        ld6(w.ks + j * 6, sj);
        for (int t = 0; t < 6; ++t) {
          at(w.sb + j * 6 + t) += c * F[t];
          Fb[t] += c * sj[t];
        }
      }
      // F = Ic_i s_i
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) at(w.Icb + i * 36 + r * 6 + c) = Fb[r] * si[c];
      float t6[6];
      mul6t(w.kIc + i * 36, Fb, t6);
      ad6(w.sb + i * 6, t6);
    }
    // Ic_i = sum over the subtree of i of I_b
    for (int bi = 0; bi < nb; ++bi) {
      int par = M.parent[bi];
      for (int t = 0; t < 36; ++t)
        at(w.Ib + bi * 36 + t) = at(w.Icb + bi * 36 + t) + (par >= 0 ? at(w.Ib + par * 36 + t) : 0.f);
    }
    // RNEA^T with Cbar = -lz
    for (int i = 0; i < nb; ++i) {
      int par = M.parent[i];
      float si[6], fb[6], ff[6];
      ld6(w.ks + i * 6, si);
      ld6(w.rff + i * 6, ff);
      float Cb = -lz[i];
      for (int t = 0; t < 6; ++t) fb[t] = si[t] * Cb + (par >= 0 ? at(w.fbar + par * 6 + t) : 0.f);
      st6(w.fbar + i * 6, fb);
      for (int t = 0; t < 6; ++t) at(w.sb + i * 6 + t) += Cb * ff[t];
    }
    for (int i = 0; i < nb * 6; ++i) {
      at(w.abar + i) = 0.f;
      at(w.vbar + i) = 0.f;
    }
    for (int i = nb - 1; i >= 0; --i) {
      int par = M.parent[i];
      long I = w.kI + i * 36;
      float v[6], a[6], fb[6], t6[6], hv[6], ab[6], vb[6];
      ld6(w.rv + i * 6, v);
      ld6(w.ra + i * 6, a);
      ld6(w.fbar + i * 6, fb);
      // f = I a + v x* (I v)
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) at(w.Ib + i * 36 + r * 6 + c) += fb[r] * a[c];
      mul6t(I, fb, t6);
      ad6(w.abar + i * 6, t6);
      mul6(I, v, hv);
      V om{v[0], v[1], v[2]}, nu{v[3], v[4], v[5]}, hn{hv[0], hv[1], hv[2]}, hf{hv[3], hv[4], hv[5]};
      V fn{fb[0], fb[1], fb[2]}, ff{fb[3], fb[4], fb[5]};
      V omb = cross(hn, fn) + cross(hf, ff), nub = cross(hf, fn);
      V hnb = cross(fn, om), hfb = cross(fn, nu) + cross(ff, om);
      float hb[6] = {hnb.x, hnb.y, hnb.z, hfb.x, hfb.y, hfb.z};
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) at(w.Ib + i * 36 + r * 6 + c) += hb[r] * v[c];
      mul6t(I, hb, t6);
      float ovb[6] = {omb.x + t6[0], omb.y + t6[1], omb.z + t6[2], nub.x + t6[3], nub.y + t6[4], nub.z + t6[5]};
      ad6(w.vbar + i * 6, ovb);
      // a_i = a_par + v_i x (s_i qd_i)
      float si[6];
      ld6(w.ks + i * 6, si);
      float qd = at(s + ND + i);
      V vJw{si[0] * qd, si[1] * qd, si[2] * qd}, vJv{si[3] * qd, si[4] * qd, si[5] * qd};
      ld6(w.abar + i * 6, ab);
      V aw{ab[0], ab[1], ab[2]}, av{ab[3], ab[4], ab[5]};
      V omb2 = cross(vJw, aw) + cross(vJv, av), nub2 = cross(vJw, av);
      float ovb2[6] = {omb2.x, omb2.y, omb2.z, nub2.x, nub2.y, nub2.z};
      ad6(w.vbar + i * 6, ovb2);
      V vJwb = cross(aw, om) + cross(av, nu), vJvb = cross(av, om);
      if (par >= 0) ad6(w.abar + par * 6, ab);
      ld6(w.vbar + i * 6, vb);
      if (par >= 0) ad6(w.vbar + par * 6, vb);
      float vJb[6] = {vJwb.x + vb[0], vJwb.y + vb[1], vJwb.z + vb[2], vJvb.x + vb[3], vJvb.y + vb[4], vJvb.z + vb[5]};
      float qdb = 0.f;
      for (int t = 0; t < 6; ++t) {
        at(w.sb + i * 6 + t) += qd * vJb[t];
        qdb += si[t] * vJb[t];
      }
      at(gB + ND + i) += qdb;
    }
    for (int i = 0; i < nb; ++i) body_bar_one(i);
    for (int x = 0; x < sc.na; ++x) aux_dyn_bar_one(x);
    for (int f = 0; f < sc.nf; ++f) free_dyn_bar_one(s, f);
  }
  // I_i (spatial, about the origin) -> COM point and rotational inertia;
  // s_i -> axis and joint origin
  MSA_HD void body_bar_one(int i) const {
    const DModel& M = *sc.M;
    {
      long Ib = w.Ib + i * 36;
      float m = M.mass[i];
      V c = v3(w.kc + i * 3);
      float cv[3] = {c.x, c.y, c.z};
      float TL[9];
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) TL[r * 3 + q] = at(Ib + r * 6 + q);
      float tr = TL[0] + TL[4] + TL[8];
      float cb3[3];
      for (int k = 0; k < 3; ++k) {
        float sm = 0.f;
        for (int j = 0; j < 3; ++j) sm += (TL[k * 3 + j] + TL[j * 3 + k]) * cv[j];
        cb3[k] = m * (2.f * cv[k] * tr - sm);
      }
      // top right m [c]x, bottom left m [c]x^T
      float X[9];
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) X[r * 3 + q] = at(Ib + r * 6 + 3 + q) + at(Ib + (3 + q) * 6 + r);
      cb3[0] += m * (X[7] - X[5]);
      cb3[1] += m * (X[2] - X[6]);
      cb3[2] += m * (X[3] - X[1]);
      acc_point(i, c, V{cb3[0], cb3[1], cb3[2]});
      // rotational inertia R Ic R^T turns with the body
      float S6[6];
      for (int t = 0; t < 6; ++t) S6[t] = at(w.kIcw + i * 6 + t);
      float Iw[9] = {S6[0], S6[3], S6[4], S6[3], S6[1], S6[5], S6[4], S6[5], S6[2]};
      float B[9];
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
          float sm = 0.f;
          for (int k = 0; k < 3; ++k) sm += Iw[r * 3 + k] * TL[q * 3 + k] - TL[k * 3 + r] * Iw[k * 3 + q];
          B[r * 3 + q] = sm;
        }
      a3(w.bacc + i * 9 + 6, V{B[5] - B[7], B[6] - B[2], B[1] - B[3]});
      V a = v3(w.ka + i * 3);
      float sbv[6];
      ld6(w.sb + i * 6, sbv);
      V st{sbv[0], sbv[1], sbv[2]}, sbo{sbv[3], sbv[4], sbv[5]};
      if (M.jtype[i] == 0) {
        V o = v3(w.ko + i * 3);
        acc_dir(i, a, st + cross(sbo, o));
        acc_point(i, o, cross(a, sbo));
      } else {
        acc_dir(i, a, sbo);
      }
    }
  }
  // door / drawer joint x: vA = qd + h (-C / M)
  MSA_HD void aux_dyn_bar_one(int x) const {
    const float h = pr.h;
    const long gB = w.gB;
    V g{pr.g[0], pr.g[1], pr.g[2]};
    {
      float vb = at(w.vAb + x);
      at(gB + axo(x) + 1) += vb;
      if (sc.A[x].type == 0) {
        float Cb = -h * vb / at(w.xM + x);
        V a = v3(w.xa + x * 3);
        V dc = cross(a, cross(a, v3(w.xbc + x * 3) - v3(w.xo + x * 3)));
        at(w.xb + x * XB + X_QB) += Cb * (-sc.A[x].mass * dot(g, dc));
      }
    }
  }
  // free body f: v* = v + h g ; w* = w - h I^-1 (w x I w)
  MSA_HD void free_dyn_bar_one(long s, int f) const {
    const float h = pr.h;
    const long gB = w.gB;
    {
      long gi = gB + fro(f);
      a3(gi + 8, v3(w.vFb + f * 6));
      V wFb = v3(w.vFb + f * 6 + 3);
      V om = v3(s + fro(f) + 12);
      float Iw[9], Ii[9];
      ld9(w.fIw + f * 9, Iw);
      ld9(w.fIi + f * 9, Ii);
      V uu = rmv(Iw, om);
      V cc = cross(om, uu);
      V gyb = wFb * (-h);
      long ib = w.fb + f * FB;
      float gv[3] = {gyb.x, gyb.y, gyb.z}, cv[3] = {cc.x, cc.y, cc.z};
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) at(ib + F_IIB + r * 3 + q) += gv[r] * cv[q];
      V ccb = rtmv(Ii, gyb);
      V omb = wFb + cross(uu, ccb);
      V ub = cross(ccb, om);
      float uv[3] = {ub.x, ub.y, ub.z}, ov[3] = {om.x, om.y, om.z};
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) at(ib + F_IWB + r * 3 + q) += uv[r] * ov[q];
      omb = omb + rtmv(Iw, ub);
      a3(gi + 12, omb);
    }
  }

  // --------------------------------------------------------------- contacts^T
  MSA_HD void contacts_bar() {
    for (int ci = 0; ci < nc; ++ci) contact_geom_bar(ci);
  }
  // contacts^T of contact ci: from its point / direction / bias adjoints to
  // the geometry of its sides
  MSA_HD void contact_geom_bar(int ci) const {
    const DModel& M = *sc.M;
    const float h = pr.h;
    {
      long e = w.con + (long)ci * CR, cb = w.conb + (long)ci * CB;
      const Ids id = ids(e);
      const int ok = id.ok, oi = id.oi, ov = id.ov, tk = id.tk, ti = id.ti;
      float r = at(e + C_R), phi = at(e + C_PHI);
      V n = v3(e + C_N);
      V c = v3(e + C_P) + n * r;
      float phib = at(cb + B_BIAS) * (phi >= 0.f ? 1.f / h : pr.beta / h);
      float nbv[3] = {0.f, 0.f, 0.f};
      onb_bar(n, v3(cb + B_D + 3), v3(cb + B_D + 6), nbv);
      V nb3 = v3(cb + B_D) + V{nbv[0], nbv[1], nbv[2]};
      V pb = v3(cb + B_P);
      // p = c - r n
      V cbar = pb;
      nb3 = nb3 - pb * r;
      if (tk == 0) {
        float4 pl = sc.Pl[ti];
        cbar = cbar + V{pl.x, pl.y, pl.z} * phib;
      } else if (tk == 1) {
        const float* bx = sc.St + ti * 6;
        V bcb{0.f, 0.f, 0.f};
        box_phi_bar(c, V{bx[0], bx[1], bx[2]}, nullptr, V{bx[3], bx[4], bx[5]}, phib, nb3, cbar, bcb, nullptr);
      } else if (tk == 2) {
        float R[9], Rb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        ld9(w.xR + ti * 9, R);
        V bcb{0.f, 0.f, 0.f};
        box_phi_bar(c, v3(w.xbc + ti * 3), R, ld3(sc.A[ti].bh), phib, nb3, cbar, bcb, Rb);
        long xb = w.xb + ti * XB;
        for (int t = 0; t < 9; ++t) at(xb + X_RB + t) += Rb[t];
        a3(xb + X_BCB, bcb);
      } else {
        const DFree& G = sc.F[ti];
        V xg = v3(cur_s + fro(ti));
        long gb = w.fb + ti * FB;
        if (G.type == 0) {
          float R[9], Rb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
          ld9(w.fR + ti * 9, R);
          V xgb{0.f, 0.f, 0.f};
          box_phi_bar(c, xg, R, ld3(G.half), phib, nb3, cbar, xgb, Rb);
          for (int t = 0; t < 9; ++t) at(gb + F_RB + t) += Rb[t];
          a3(gb + F_XB, xgb);
        } else {
          V d = c - xg;
          float dist = sqrtf(dot(d, d));
          V db = d * 0.f;
          if (!(dist < 1e-12f)) {
            V nn = d * (1.f / dist);
            db = nn * phib + (nb3 - nn * dot(nn, nb3)) * (1.f / dist);
          }
          cbar = cbar + db;
          a3(gb + F_XB, -db);
        }
      }
      // owner point
      if (ok == 0) {
        acc_point(M.sph_body[oi], c, cbar);
      } else {
        long fb = w.fb + oi * FB;
        a3(fb + F_XB, cbar);
        if (ok == 1) {
          const DFree& F = sc.F[oi];
          V loc{(ov & 1) ? F.half[0] : -F.half[0], (ov & 2) ? F.half[1] : -F.half[1], (ov & 4) ? F.half[2] : -F.half[2]};
          float cv[3] = {cbar.x, cbar.y, cbar.z}, lv[3] = {loc.x, loc.y, loc.z};
          for (int rr = 0; rr < 3; ++rr)
            for (int q = 0; q < 3; ++q) at(fb + F_RB + rr * 3 + q) += cv[rr] * lv[q];
        }
      }
    }
  }

  // --------------------------------------------------------------- frames^T
  MSA_HD void frames_bar(long s) {
    for (int f = 0; f < sc.nf; ++f) free_frame_bar(s, f);
    for (int x = 0; x < sc.na; ++x) aux_frame_bar(x);
  }
  MSA_HD void free_frame_bar(long s, int f) const {
    const long gB = w.gB;
    {
      long fb = w.fb + f * FB;
      const DFree& F = sc.F[f];
      float R[9], Rb[9];
      ld9(w.fR + f * 9, R);
      for (int t = 0; t < 9; ++t) Rb[t] = at(fb + F_RB + t);
      // Iw = R D R^T, Ii = R D^-1 R^T: Rbar += (Xbar + Xbar^T) R D
      float D[3] = {F.Ib[0], F.Ib[1], F.Ib[2]};
      for (int pass = 0; pass < 2; ++pass) {
        long xo = fb + (pass == 0 ? F_IWB : F_IIB);
        float Xs[9];
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) Xs[r * 3 + q] = at(xo + r * 3 + q) + at(xo + q * 3 + r);
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) {
            float dq = pass == 0 ? D[q] : 1.f / D[q];
            Rb[r * 3 + q] += (Xs[r * 3 + 0] * R[0 * 3 + q] + Xs[r * 3 + 1] * R[1 * 3 + q] + Xs[r * 3 + 2] * R[2 * 3 + q]) * dq;
          }
      }
      float Q[4] = {at(s + fro(f) + 4), at(s + fro(f) + 5), at(s + fro(f) + 6), at(s + fro(f) + 7)};
      float Qb[4] = {0.f, 0.f, 0.f, 0.f};
      quatR_bar(Q, Rb, Qb);
      for (int t = 0; t < 4; ++t) at(gB + fro(f) + 4 + t) += Qb[t];
      a3(gB + fro(f), v3(fb + F_XB));
    }
  }
  MSA_HD void aux_frame_bar(int x) const {
    const long gB = w.gB;
    {
      long xb = w.xb + x * XB;
      float qb = at(xb + X_QB);
      V a = v3(w.xa + x * 3);
      V bcb = v3(xb + X_BCB);
      if (sc.A[x].type == 0) {
        float R[9];
        ld9(w.xR + x * 9, R);
        V m = cross(v3(w.xbc + x * 3) - v3(w.xo + x * 3), bcb);
        for (int col = 0; col < 3; ++col)
          m = m + cross(V{R[col], R[3 + col], R[6 + col]}, V{at(xb + X_RB + col), at(xb + X_RB + 3 + col), at(xb + X_RB + 6 + col)});
        qb += dot(a, m);
      } else {
        qb += dot(a, bcb);
      }
      at(gB + axo(x)) += qb;
    }
  }

  // --------------------------------------------------------------- kinematics^T
  MSA_HD void kin_bar() {
    const DModel& M = *sc.M;
    long gB = w.gB;
    for (int i = nb - 1; i >= 0; --i) {
      long ac = w.bacc + i * 9;
      V F = v3(ac), Mo = v3(ac + 3), Md = v3(ac + 6);
      V a = v3(w.ka + i * 3);
      float qb = M.jtype[i] == 0 ? dot(a, Mo + Md - cross(v3(w.ko + i * 3), F)) : dot(a, F);
      at(gB + i) += qb;
      int par = M.parent[i];
      if (par >= 0) {
        a3(w.bacc + par * 9, F);
        a3(w.bacc + par * 9 + 3, Mo);
        a3(w.bacc + par * 9 + 6, Md);
      }
    }
  }

  MSA_HD void reverse_substep(int si, const float* u) {
    long s = srec(si);
    cur_s = s;
    zero(w.gB, w.ss);
    zero(w.vRb, ND);
    zero(w.vAb, AMAX);
    zero(w.vFb, w.fmax * 6);
    zero(w.limb, 2 * AMAX);
    zero(w.conb, nc * CB);
    zero(w.rJb, nrob * 3 * ND);
    zero(w.rwb, nrob * 3 * ND);
    zero(w.fb, w.fmax * FB);
    zero(w.xb, AMAX * XB);
    zero(w.bacc, ND * 9);
    zero(w.Mb, ND * ND);
    integrate_bar(s);
    pgs_bar();
    rows_bar();
    dynamics_bar(s, u);
    contacts_bar();
    frames_bar(s);
    kin_bar();
    for (int t = 0; t < w.ss; ++t) at(w.gA + t) = at(w.gB + t);
  }

  // ---------------------------------------------------------------- driver
  // q, qd: the scene's rows of the robot state; fr: its first free body's
  // 16 floats; ax: its first door/drawer's 4 floats.  g* are the same views
  // of the output adjoint (in) and input adjoint (out); gu the control adjoint.
  MSA_HD void run(const float* q, const float* qd, const float* fr, const float* ax, const float* u, const float* gq,
                  const float* gqd, const float* gfr, const float* gax, float* oq, float* oqd, float* ofr, float* oax,
                  float* ou) {
    const DModel& M = *sc.M;
    nb = M.nb;
    nsph = M.nsph;
    status = 0;
    nc = nrob = nlim = 0;
    tb = Buf{b.p + (long)w.tape * b.st, b.st};
    tsw = 3 * (2 * AMAX + w.ccap);
    tmask = -1;
    long s0 = srec(0);
    zero(s0, w.ss);
    for (int j = 0; j < ND; ++j) {
      at(s0 + j) = q[j];
      at(s0 + ND + j) = qd[j];
    }
    for (int f = 0; f < sc.nf; ++f)
      for (int t = 0; t < 16; ++t) at(s0 + fro(f) + t) = fr[f * 16 + t];
    for (int x = 0; x < sc.na; ++x)
      for (int t = 0; t < 4; ++t) at(s0 + axo(x) + t) = ax[x * 4 + t];
    for (int si = 0; si < pr.nsub; ++si) forward_substep(si, u, false);
    zero(w.gA, w.ss);
    for (int j = 0; j < ND; ++j) {
      at(w.gA + j) = gq[j];
      at(w.gA + ND + j) = gqd[j];
    }
    for (int f = 0; f < sc.nf; ++f)
      for (int t = 0; t < 16; ++t) at(w.gA + fro(f) + t) = gfr[f * 16 + t];
    for (int x = 0; x < sc.na; ++x)
      for (int t = 0; t < 4; ++t) at(w.gA + axo(x) + t) = gax[x * 4 + t];
    zero(w.ub, ND);
    for (int si = pr.nsub - 1; si >= 0; --si) {
      forward_substep(si, u, true);
      reverse_substep(si, u);
    }
    for (int j = 0; j < ND; ++j) {
      oq[j] = at(w.gA + j);
      oqd[j] = at(w.gA + ND + j);
      ou[j] = at(w.ub + j);
    }
    for (int f = 0; f < sc.nf; ++f)
      for (int t = 0; t < 16; ++t) ofr[f * 16 + t] = at(w.gA + fro(f) + t);
    for (int x = 0; x < sc.na; ++x)
      for (int t = 0; t < 4; ++t) oax[x * 4 + t] = at(w.gA + axo(x) + t);
  }
};

}  // namespace msa
