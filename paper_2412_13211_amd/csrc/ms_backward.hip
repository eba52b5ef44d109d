// ms_backward.hip -- the adjoint of one control step on gfx950.
#include "ms_backward.h"

namespace msk {

// ============================================================ lane per scene
// (scenes taken in the cost-sorted order so that a wavefront holds scenes of
// similar size; workspace interleaved across the lanes)
__global__ __launch_bounds__(64) void k_step_bwd(BwdArgs a) {
  const int slot = blockIdx.x * 64 + threadIdx.x;
  if (slot >= a.S) return;
  const int s = a.order[slot];
  const DScene& D = a.scenes[s];
  msa::Eng E;
  E.sc = msa::SceneRef{a.models + D.model, a.free + D.f0, a.statics + 6 * (size_t)D.s0, a.planes + D.p0,
                       a.aux + D.a0, D.hold, D.nf, D.ns, D.np, D.na};
  E.pr = a.pr;
  E.w = a.w;
  E.b = msa::Buf{a.ws + slot, (long)a.stride};
  const size_t S = (size_t)a.S;
  const size_t q = 16 * (size_t)s, qd = 16 * S + 16 * (size_t)s;
  const size_t fo = 32 * S + 16 * (size_t)D.f0, ao = 32 * S + 16 * (size_t)a.NF + 4 * (size_t)D.a0;
  E.run(a.x + q, a.x + qd, a.x + fo, a.x + ao, a.u + 16 * (size_t)s, a.gxo + q, a.gxo + qd, a.gxo + fo, a.gxo + ao,
        a.gxi + q, a.gxi + qd, a.gxi + fo, a.gxi + ao, a.gu + 16 * (size_t)s);
  if (E.status) a.status[s] |= E.status;
}

void launch_step_bwd(const BwdArgs& a, hipStream_t st) {
  const int grid = (a.S + 63) / 64;
  hipLaunchKernelGGL(k_step_bwd, dim3(grid), dim3(64), 0, st, a);
}

// ============================================================ wavefront per scene
namespace {

__device__ __forceinline__ int lane_id() { return threadIdx.x; }
__device__ __forceinline__ void wsync() { __syncthreads(); }
// Ordering of LDS accesses between the lanes of the workgroup's one
// wavefront: the LDS executes a wavefront's instructions in issue order, so a
// read issued after a write sees it; only the compiler must not move memory
// accesses across (no wait for outstanding accesses, unlike the barrier).
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }
__device__ __forceinline__ float bcast0(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0)); }
// value of the lane N places along within its row of 16 lanes (DPP row
// rotation: a VALU operand modifier, no LDS crossbar)
template <int N>
__device__ __forceinline__ float row_ror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + N, 0xf, 0xf, false));
}
// sum within each 16-lane group, returned in every lane of the group
__device__ __forceinline__ float sum16(float v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  return v;
}
// sum over lanes 0..15 (other lanes pass 0), returned in every lane
__device__ __forceinline__ float sum16_b(float v) { return bcast0(sum16(v)); }
// the sum of 16-lane row q (q = 0..3), read by every lane
__device__ __forceinline__ float row_sum(float s16, int q) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s16), 16 * q));
}

// level-schedule views inside the LDS block
struct Lv {
  int *lvl, *order, *loff, *rob, *gfirst, *last, *cnt;
};
__device__ __forceinline__ Lv lv_view(float* L, const msa::WS& w) {
  Lv v;
  int* p = reinterpret_cast<int*>(L + w.lv);
  const int R = msa::lv_rows(w.ccap);
  v.lvl = p; p += R;
  v.order = p; p += R;
  v.loff = p; p += R + 2;
  v.rob = p; p += R + 2;
  v.gfirst = p; p += R + 1;
  v.last = p; p += 64;
  v.cnt = p;  // [0] nc, [1] nrob, [2] nlim, [3] maxl, [4] status
  return v;
}

// dynamic node of a row (robot 0, door/drawer 1 + x, free body 1 + AMAX + f; -1 none)
__device__ __forceinline__ void row_nodes(const msa::Eng& E, int r, int& na, int& nbn) {
  if (r < E.nlim) {
    na = 1 + (int)E.at(E.w.lim + r * 4);
    nbn = -1;
    return;
  }
  long e = E.w.con + (long)(r - E.nlim) * msa::CR;
  const msa::Ids id = E.ids(e);
  const int ok = id.ok, oi = id.oi, tk = id.tk, ti = id.ti;
  na = ok == 0 ? 0 : 1 + AMAX + oi;
  nbn = tk == 2 ? 1 + ti : (tk == 3 ? 1 + AMAX + ti : -1);
}

// Reverse of a robot contact's row updates in sweep it.  Lane j of each
// 16-lane row carries the robot's joint j in registers (the four copies
// equal); the target side (a free body or a door / drawer joint, none for
// furniture and planes) is carried in registers by every lane alike, so the
// sums over the joints are the only exchanges, and each 16-lane row forms
// one of them: the friction part's four sums come from one reduction, the
// normal part's two from another.  Lanes 0..15 write the joints back, lane 0
// the target side and the contact's adjoints.
__device__ void robot_contact_bar(msa::Eng& E, int it, int ci, float* L) {
  using namespace msa;
  const int lane = lane_id(), j = lane & 15, q = lane >> 4;
  const bool jv = j < E.nb;           // this lane holds joint j
  const bool own = lane < 16 && jv;   // and writes it back
  const WS& w = E.w;
  const long e = w.con + (long)ci * CR, cb = w.conb + (long)ci * CB, lb = w.lamb + ci * 3;
  const long rr = (long)ci * 3 * ND + j;
  const int row = E.nlim + ci;
  const float mu = E.pr.mu;
  const Ids id = E.ids(e);
  const bool tf = id.tk == 3, tx = id.tk == 2;
  // robot side: joint j's velocity, its adjoint, the three rows' J and
  // M~^-1 J entries and their adjoints
  float vr = 0.f, vrb = 0.f, J[3] = {0.f, 0.f, 0.f}, Wr[3] = {0.f, 0.f, 0.f};
  float Jb[3] = {0.f, 0.f, 0.f}, Wrb[3] = {0.f, 0.f, 0.f};
  if (jv) {
    vr = L[w.vR + j];
    vrb = L[w.vRb + j];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      J[k] = L[w.rJ + rr + k * ND];
      Wr[k] = L[w.rw + rr + k * ND];
    }
  }
  Eng::FSide B;
  Eng::XSide X;
  if (tf) E.fs_load(B, id.ti, -1.f);
  if (tx) E.xs_load(X, id.ti);
  Eng::RowAcc R;
  R.p = E.v3(e + C_P);
  R.d[0] = E.v3(e + C_N);
  R.d[1] = E.v3(e + C_T1);
  R.d[2] = E.v3(e + C_T2);
  for (int k = 0; k < 3; ++k) R.db[k] = V{0.f, 0.f, 0.f};
  R.pb = V{0.f, 0.f, 0.f};
  auto t_apply = [&](int di, float dl) {
    if (tf) Eng::fs_apply(B, R, di, dl);
    else if (tx) Eng::xs_apply(X, R, di, dl);
  };
  auto t_apply_bar = [&](int di, float dl) -> float {
    if (tf) return Eng::fs_apply_bar(B, R, di, dl);
    if (tx) return Eng::xs_apply_bar(X, R, di, dl);
    return 0.f;
  };
  auto t_rowvel = [&](int di) -> float {
    if (tf) return Eng::fs_rowvel(B, R, di);
    if (tx) return Eng::xs_rowvel(X, R, di);
    return 0.f;
  };
  auto t_rowvel_bar = [&](int di, float rb) {
    if (tf) Eng::fs_rowvel_bar(B, R, di, rb);
    else if (tx) Eng::xs_rowvel_bar(X, R, di, rb);
  };
  const float W0 = L[e + C_W], W1 = L[e + C_W + 1], W2 = L[e + C_W + 2];
  float lb0 = L[lb], lb1 = L[lb + 1], lb2 = L[lb + 2];
  float Wb0 = 0.f, Wb1 = 0.f, Wb2 = 0.f, biasb = 0.f;
  if (W1 >= 1e-12f && W2 >= 1e-12f) {
    const float y1 = E.tape_at(it, row, 1), y2 = E.tape_at(it, row, 2);
    const float lim = mu * E.normal_after(it, ci);
    float o1, o2, p1, p2;
    const bool proj = disk_proj(y1, y2, lim, o1, o2);
    E.prev_fric(it, ci, p1, p2);
    const float d1 = o1 - p1, d2 = o2 - p2;
    vr += Wr[2] * (-d2);
    vr += Wr[1] * (-d1);
    t_apply(2, -d2);
    t_apply(1, -d1);
    // rows 0..3: w_1 . vbar, w_2 . vbar, J_1 . v, J_2 . v
    const float part = !jv ? 0.f : (q == 0 ? Wr[1] * vrb : (q == 1 ? Wr[2] * vrb : (q == 2 ? J[1] * vr : J[2] * vr)));
    const float s4 = sum16(part);
    Wrb[1] += vrb * d1;
    Wrb[2] += vrb * d2;
    const float b1 = t_apply_bar(1, d1);
    const float b2 = t_apply_bar(2, d2);
    const float d1b = row_sum(s4, 0) + b1, d2b = row_sum(s4, 1) + b2;
    float yb1, yb2, limb;
    Eng::fric_bar(y1, y2, lim, proj, lb1 + d1b, lb2 + d2b, yb1, yb2, limb);
    const float l1 = -d1b + yb1, l2 = -d2b + yb2;
    const float r1 = row_sum(s4, 2) + t_rowvel(1);
    const float r2 = row_sum(s4, 3) + t_rowvel(2);
    const float rb1 = -yb1 / W1, rb2 = -yb2 / W2;
    lb0 += mu * limb;
    Wb1 += yb1 * r1 / (W1 * W1);
    Wb2 += yb2 * r2 / (W2 * W2);
    t_rowvel_bar(1, rb1);
    t_rowvel_bar(2, rb2);
    lb1 = l1;
    lb2 = l2;
    Jb[1] += rb1 * vr;
    Jb[2] += rb2 * vr;
    vrb += rb1 * J[1];
    vrb += rb2 * J[2];
  }
  if (W0 >= 1e-12f) {
    const float y = E.tape_at(it, row, 0);
    const float nl = y > 0.f ? y : 0.f;
    const float dl = nl - E.prev_normal(it, ci);
    vr += Wr[0] * (-dl);
    t_apply(0, -dl);
    // rows 0..1: w_n . vbar, J_n . v
    const float s2 = sum16(!jv ? 0.f : (q == 0 ? Wr[0] * vrb : J[0] * vr));
    Wrb[0] += vrb * dl;
    const float dlb = row_sum(s2, 0) + t_apply_bar(0, dl);
    float lold, yb;
    Eng::normal_bar(y, lb0 + dlb, dlb, lold, yb);
    const float r = row_sum(s2, 1) + t_rowvel(0) + L[e + C_BIAS];
    const float rb = -yb / W0;
    Wb0 += yb * r / (W0 * W0);
    biasb += rb;
    t_rowvel_bar(0, rb);
    Jb[0] += rb * vr;
    vrb += rb * J[0];
    lb0 = lold;
  }
  if (own) {
    L[w.vR + j] = vr;
    L[w.vRb + j] = vrb;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      L[w.rJb + rr + k * ND] += Jb[k];
      L[w.rwb + rr + k * ND] += Wrb[k];
    }
  }
  if (lane == 0) {
    L[lb] = lb0;
    L[lb + 1] = lb1;
    L[lb + 2] = lb2;
    for (int k = 0; k < 3; ++k) E.a3(cb + B_D + k * 3, R.db[k]);
    E.a3(cb + B_P, R.pb);
    L[cb + B_W] += Wb0;
    L[cb + B_W + 1] += Wb1;
    L[cb + B_W + 2] += Wb2;
    L[cb + B_BIAS] += biasb;
    if (tf) E.fs_store(B);
    if (tx) E.xs_store(X);
  }
}

__device__ __forceinline__ void zero_lds(float* L, long off, int n) {
  for (int i = lane_id(); i < n; i += 64) L[off + i] = 0.f;
}

// contact rows (the same quantities as the engine's rows(), limit rows
// excepted): one lane per contact for the tangents, bias and the free-body
// and door/drawer shares of W; then one lane per robot row (contact,
// direction) for J, w = M~^-1 J^T and the robot share of W
__device__ __forceinline__ void rows_wave(msa::Eng& E, float* L) {
  using namespace msa;
  const int lane = lane_id();
  const WS& w = E.w;
  const DModel& M = *E.sc.M;
  const float h = E.pr.h;
  for (int ci = lane; ci < E.nc; ci += 64) {
    const long e = w.con + (long)ci * CR;
    V n = E.v3(e + C_N), t1, t2;
    onb(n, t1, t2);
    E.s3(e + C_T1, t1);
    E.s3(e + C_T2, t2);
    const V p = E.v3(e + C_P);
    const Ids id = unpack_ids(L[e + C_ID]);
    const int ok = id.ok, oi = id.oi, tk = id.tk, ti = id.ti;
    for (int di = 0; di < 3; ++di) {
      const V d = di == 0 ? n : (di == 1 ? t1 : t2);
      float W = ok == 0 ? 0.f : E.free_W(oi, d, p, 1.f);
      if (tk == 2) {
        float J = E.aux_J(ti, d, p, -1.f);
        W += J * (J / L[w.xM + ti]);
      } else if (tk == 3) {
        W += E.free_W(ti, d, p, -1.f);
      }
      L[e + C_W + di] = W;
    }
    const float phi = L[e + C_PHI];
    L[e + C_BIAS] = phi >= 0.f ? phi / h : E.pr.beta * phi / h;
  }
  wsync();
  // robot rows, four at a time: lane j of a 16-lane group owns joint j
  const int g = lane >> 4, j = lane & 15, nr = 3 * E.nrob;
  for (int r0 = 0; r0 < nr; r0 += 4) {
    const int r = r0 + g;
    const bool act = r < nr;
    const int ci = r / 3, di = r - 3 * (r / 3);
    const long e = w.con + (long)ci * CR;
    float Jj = 0.f;
    if (act) {
      const int anc = M.anc[M.sph_body[unpack_ids(L[e + C_ID]).oi]];
      if (j < E.nb && ((anc >> j) & 1)) {
        const V a = E.v3(w.ka + j * 3), d = E.dir(e, di);
        Jj = M.jtype[j] == 0 ? dot(d, cross(a, E.v3(e + C_P) - E.v3(w.ko + j * 3))) : dot(d, a);
      }
      L[w.rJ + (long)r * ND + j] = Jj;
    }
    wsync();
    // w_j = sum_k (M~^-1)_jk J_k; Minv row k holds M~^-1 e_k
    float s = 0.f;
    if (act)
      for (int k = 0; k < ND; ++k) s += L[w.Minv + k * ND + j] * L[w.rJ + (long)r * ND + k];
    const float W = sum16(Jj * s);
    if (act) {
      L[w.rw + (long)r * ND + j] = s;
      if (j == 0) L[e + C_W + di] += W;
    }
  }
  wsync();
  bool bad = false;
  for (int ci = lane; ci < E.nc; ci += 64)
    for (int di = 0; di < 3; ++di) bad |= !(L[w.con + (long)ci * CR + C_W + di] >= 1e-12f);
  if (__ballot(bad)) E.status |= Eng::MS_DEGENERATE_BIT;
}

// adjoint of the robot rows (the robot owners' share; the engine's
// rows_bar(false) does the rest).  With w = M~^-1 J^T and W += J . w:
// Jbar += Wbar w + M~^-1 (wbar + Wbar J), M~bar -= M~^-1 (wbar + Wbar J) w^T;
// Jbar then reaches the directions, the contact point and the joint axes
__device__ __forceinline__ void robot_rows_bar_wave(msa::Eng& E, float* L) {
  using namespace msa;
  const int lane = lane_id();
  const WS& w = E.w;
  const DModel& M = *E.sc.M;
  const int nb = E.nb, nr = 3 * E.nrob;
  // robot rows four at a time (lane j of a 16-lane group owns entry j):
  // Jbar into rJb, alpha = M~^-1 (wbar + Wbar J) into rwb
  const int g = lane >> 4, jj = lane & 15;
  for (int r0 = 0; r0 < nr; r0 += 4) {
    const int r = r0 + g;
    const bool act = r < nr;
    const int ci = r / 3, di = r - 3 * (r / 3);
    const long rb = (long)r * ND + jj;
    float Wb = 0.f;
    if (act) {
      Wb = L[w.conb + (long)ci * CB + B_W + di];
      L[w.rwb + rb] += Wb * L[w.rJ + rb];
    }
    wsync();
    float s = 0.f;
    if (act)
      for (int k = 0; k < ND; ++k) s += L[w.Minv + k * ND + jj] * L[w.rwb + (long)r * ND + k];
    wsync();
    if (act) {
      L[w.rJb + rb] += Wb * L[w.rw + rb] + s;
      L[w.rwb + rb] = s;
    }
  }
  wsync();
  // M~bar: lane owns entries lane, lane + 64, ...
  for (int idx = lane; idx < ND * ND; idx += 64) {
    const int rr = idx / ND, cc = idx - ND * (idx / ND);
    float s = 0.f;
    for (int q = 0; q < nr; ++q) s += L[w.rwb + (long)q * ND + rr] * L[w.rw + (long)q * ND + cc];
    L[w.Mb + idx] -= s;
  }
  // lane per robot contact: direction and contact-point adjoints
  for (int ci = lane; ci < E.nrob; ci += 64) {
    const long e = w.con + (long)ci * CR, cb = w.conb + (long)ci * CB;
    const V p = E.v3(e + C_P);
    const int anc = M.anc[M.sph_body[unpack_ids(L[e + C_ID]).oi]];
    V pb{0.f, 0.f, 0.f};
    for (int di = 0; di < 3; ++di) {
      const V d = E.dir(e, di);
      const long rjb = w.rJb + ((long)ci * 3 + di) * ND;
      V db{0.f, 0.f, 0.f};
      for (int j = 0; j < nb; ++j) {
        const float Jb = L[rjb + j];
        if (!((anc >> j) & 1) || Jb == 0.f) continue;
        const V a = E.v3(w.ka + j * 3);
        if (M.jtype[j] == 0) {
          db = db + cross(a, p - E.v3(w.ko + j * 3)) * Jb;
          pb = pb + cross(d, a) * Jb;
        } else {
          db = db + a * Jb;
        }
      }
      E.a3(cb + B_D + di * 3, db);
    }
    E.a3(cb + B_P, pb);
  }
  // lane per joint: the joint's own body accumulators
  for (int j = lane; j < nb; j += 64) {
    const V a = E.v3(w.ka + j * 3), o = E.v3(w.ko + j * 3);
    const bool rev = M.jtype[j] == 0;
    for (int r = 0; r < nr; ++r) {
      const int ci = r / 3, di = r - 3 * ci;
      const long e = w.con + (long)ci * CR;
      const float Jb = L[w.rJb + (long)r * ND + j];
      if (!((M.anc[M.sph_body[unpack_ids(L[e + C_ID]).oi]] >> j) & 1) || Jb == 0.f) continue;
      const V d = E.dir(e, di);
      if (rev) {
        const V ev = E.v3(e + C_P) - o;
        E.acc_dir(j, a, cross(ev, d) * Jb);
        E.acc_point(j, o, -(cross(d, a) * Jb));
      } else {
        E.acc_dir(j, a, d * Jb);
      }
    }
  }
  wsync();
}

// Recompute of a substep's articulated quantities over the lanes: drive
// (lane per DoF), door/drawer and free-body frames (lane per joint / body),
// body poses by pointer jumping (lane per body, four doubling rounds),
// per-body quantities (lane per body); CRBA and RNEA with the tree
// recursions run down or up the tree by one lane per matrix or vector
// component, the per-body terms one lane per body; M~^-1 by Gauss-Jordan
// elimination over the lanes.  The bias torques are left in w.lz.
__device__ __forceinline__ void recompute_wave(msa::Eng& E, float* L, const float* u) {
  using namespace msa;
  const int lane = lane_id();
  const WS& w = E.w;
  const DModel& M = *E.sc.M;
  const int nb = E.nb;
  const long s = w.st;
  if (lane < ND) E.drive_one(s, u, lane);
  if (lane >= ND && lane < ND + E.sc.na) E.aux_frame(s, lane - ND);
  for (int f = lane; f < E.sc.nf; f += 64) E.free_frame(s, f);
  // body poses: each body's joint transform relative to its parent, then
  // X_i <- X_a X_i with a the current ancestor, a <- a's ancestor, until the
  // root (the ancestor index lives in w.z, free until z is solved)
  int anc = -1;
  if (lane < nb) {
    const int i = lane;
    const V ax = ld3(M.axis[i]);
    float R[9];
    V p = ld3(M.xtp[i]);
    if (M.jtype[i] == 0) {
      float Rr[9];
      rot_axis(ax, L[s + i], Rr);
      mm3(M.xtR[i], Rr, R);
    } else {
      for (int t = 0; t < 9; ++t) R[t] = M.xtR[i][t];
      p = p + rmv(M.xtR[i], ax) * L[s + i];
    }
    for (int t = 0; t < 9; ++t) L[w.kR + i * 9 + t] = R[t];
    E.s3(w.kp + i * 3, p);
    anc = M.parent[i];
    L[w.z + i] = __int_as_float(anc);
  }
  wsync();
  for (int round = 0; round < 4; ++round) {
    float Ra[9], R[9], Rn[9];
    V pa{0.f, 0.f, 0.f}, p{0.f, 0.f, 0.f};
    int anc2 = -1;
    const bool act = lane < nb && anc >= 0;
    if (act) {
      for (int t = 0; t < 9; ++t) {
        Ra[t] = L[w.kR + anc * 9 + t];
        R[t] = L[w.kR + lane * 9 + t];
      }
      pa = E.v3(w.kp + anc * 3);
      p = E.v3(w.kp + lane * 3);
      anc2 = __float_as_int(L[w.z + anc]);
    }
    wsync();
    if (act) {
      mm3(Ra, R, Rn);
      for (int t = 0; t < 9; ++t) L[w.kR + lane * 9 + t] = Rn[t];
      E.s3(w.kp + lane * 3, pa + rmv(Ra, p));
      anc = anc2;
      L[w.z + lane] = __int_as_float(anc);
    }
    wsync();
  }
  // joint axis and origin from the parent's world pose
  if (lane < nb) {
    const int i = lane, par = M.parent[i];
    float Rj[9];
    V o;
    if (par < 0) {
      for (int t = 0; t < 9; ++t) Rj[t] = M.xtR[i][t];
      o = ld3(M.xtp[i]);
    } else {
      float Rp[9];
      E.ld9(w.kR + par * 9, Rp);
      mm3(Rp, M.xtR[i], Rj);
      o = E.v3(w.kp + par * 3) + rmv(Rp, ld3(M.xtp[i]));
    }
    E.s3(w.ka + i * 3, rmv(Rj, ld3(M.axis[i])));
    E.s3(w.ko + i * 3, o);
  }
  wsync();
  if (lane < nb) E.kin_body(lane);
  wsync();
  // composite inertias (one lane per entry, up the tree) and velocities
  // v_i = v_par + s_i qd_i (one lane per component, down the tree)
  for (int idx = lane; idx < nb * 36; idx += 64) L[w.kIc + idx] = L[w.kI + idx];
  // M~: zero, identity past the robot's DoFs
  for (int e = lane; e < ND * ND; e += 64) {
    const int r = e >> 4, c = e & 15;
    L[w.L + e] = (r >= nb || c >= nb) && r == c ? 1.f : 0.f;
  }
  wsync();
  if (lane < 36) {
    for (int i = nb - 1; i > 0; --i) {
      const int par = M.parent[i];
      if (par >= 0) L[w.kIc + par * 36 + lane] += L[w.kIc + i * 36 + lane];
    }
  } else if (lane < 42) {
    const int t = lane - 36;
    for (int i = 0; i < nb; ++i) {
      const int par = M.parent[i];
      L[w.rv + i * 6 + t] = (par >= 0 ? L[w.rv + par * 6 + t] : 0.f) + L[w.ks + i * 6 + t] * L[s + ND + i];
    }
  }
  wsync();
  // mass matrix row / column i: M_ij = s_j . (Ic_i s_i), j an ancestor of i;
  // the terms v_i x (s_i qd_i) (into ra, summed down the tree below)
  if (lane < nb) {
    const int i = lane;
    float si[6], F[6];
    E.ld6(w.ks + i * 6, si);
    E.mul6(w.kIc + i * 36, si, F);
    for (int j = i; j >= 0; j = M.parent[j]) {
      float v = 0.f;
      for (int t = 0; t < 6; ++t) v += L[w.ks + j * 6 + t] * F[t];
      L[w.L + i * ND + j] = v;
      L[w.L + j * ND + i] = v;
    }
    float v[6], vJ[6], t6[6];
    E.ld6(w.rv + i * 6, v);
    const float qd = L[s + ND + i];
    for (int t = 0; t < 6; ++t) vJ[t] = si[t] * qd;
    Eng::crm6(v, vJ, t6);
    E.st6(w.ra + i * 6, t6);
  }
  wsync();
  // accelerations a_i = a_par + v_i x (s_i qd_i), a_root's parent = -g
  if (lane < 6) {
    const int t = lane;
    // the base acceleration's component t, formed arithmetically: a lane-
    // dependent index into the parameters (or a select the compiler turns
    // into one) would put the engine object in scratch memory
    const float g0 = E.pr.g[0], g1 = E.pr.g[1], g2 = E.pr.g[2];
    const float base = -(g0 * (float)(t == 3) + g1 * (float)(t == 4) + g2 * (float)(t == 5));
    for (int i = 0; i < nb; ++i) {
      const int par = M.parent[i];
      L[w.ra + i * 6 + t] += par >= 0 ? L[w.ra + par * 6 + t] : base;
    }
  }
  wsync();
  // body forces f_i = I_i a_i + v_i x* (I_i v_i) into rfl and rff
  if (lane < nb) {
    const int i = lane;
    float v[6], acc[6], fl[6], hv[6], t6[6];
    E.ld6(w.rv + i * 6, v);
    E.ld6(w.ra + i * 6, acc);
    E.mul6(w.kI + i * 36, acc, fl);
    E.mul6(w.kI + i * 36, v, hv);
    Eng::crf6(v, hv, t6);
    for (int t = 0; t < 6; ++t) fl[t] += t6[t];
    E.st6(w.rfl + i * 6, fl);
    E.st6(w.rff + i * 6, fl);
  }
  wsync();
  // subtree force sums (one lane per component, up the tree)
  if (lane < 6) {
    for (int i = nb - 1; i > 0; --i) {
      const int par = M.parent[i];
      if (par >= 0) L[w.rff + par * 6 + lane] += L[w.rff + i * 6 + lane];
    }
  }
  wsync();
  // bias torques C_i = s_i . f_i; M~ = M + diag(armature), copied to the
  // M~^-1 buffer for the elimination
  if (lane < nb) {
    const int i = lane;
    float c = 0.f;
    for (int t = 0; t < 6; ++t) c += L[w.ks + i * 6 + t] * L[w.rff + i * 6 + t];
    L[w.lz + i] = c;
    L[w.L + i * ND + i] += L[w.arm + i];
  }
  wsync();
  // Gauss-Jordan elimination without pivoting (M~ is symmetric positive
  // definite), in registers: lane i < 16 holds row i; pivot p's row is read
  // from lane p with readlane (the pivot loop is unrolled, so every register
  // index is a constant); rows and columns past the robot's degrees of
  // freedom are identity and stay so
  if (lane < ND) {
    float a[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) a[k] = L[w.L + lane * ND + k];
    bool degen = false;
#pragma unroll
    for (int p = 0; p < ND; ++p) {
      float prow[ND];
#pragma unroll
      for (int k = 0; k < ND; ++k) prow[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[k]), p));
      float piv = prow[p];
      if (p < nb && !(piv > 0.f)) {
        degen = true;
        piv = 1e-30f;
      }
      const float inv = 1.f / piv;
      const float f = a[p];
      const bool own = lane == p;
#pragma unroll
      for (int k = 0; k < ND; ++k) {
        if (k == p) a[k] = own ? inv : -f * inv;
        else a[k] = own ? prow[k] * inv : a[k] - f * (prow[k] * inv);
      }
    }
    if (degen && lane == 0) E.status |= Eng::MS_DEGENERATE_BIT;
#pragma unroll
    for (int k = 0; k < ND; ++k) L[w.Minv + lane * ND + k] = lane < nb && k < nb ? a[k] : 0.f;
  }
}

// z = M~^-1 (tau - C) from the explicit inverse (lane per DoF)
__device__ __forceinline__ void solve_z_wave(const msa::Eng& E, float* L) {
  const int lane = lane_id();
  const msa::WS& w = E.w;
  if (lane < ND) {
    float z = 0.f;
    for (int k = 0; k < E.nb; ++k) z += L[w.Minv + k * ND + lane] * (L[w.tau + k] - L[w.lz + k]);
    L[w.z + lane] = lane < E.nb ? z : 0.f;
  }
}

// dynamics^T over the lanes (the same adjoint as the engine's dynamics_bar,
// with its recursions written as ancestor / descendant sums)
__device__ __forceinline__ void dynamics_bar_wave(msa::Eng& E, float* L) {
  using namespace msa;
  const int lane = lane_id();
  const WS& w = E.w;
  const DModel& M = *E.sc.M;
  const int nb = E.nb;
  const float h = E.pr.h;
  const long s = w.st, gB = w.gB;
  // vR = qd + h z: qd gets vRbar; lz = M~^-1 h vRbar is tau's adjoint
  if (lane < ND) {
    L[gB + ND + lane] += L[w.vRb + lane];
    float lz = 0.f;
    for (int k = 0; k < nb; ++k) lz += L[w.Minv + k * ND + lane] * (h * L[w.vRb + k]);
    L[w.lz + lane] = lane < nb ? lz : 0.f;
  }
  wsync();
  // M~bar -= lz z^T; drive^T
  for (int idx = lane; idx < ND * ND; idx += 64) {
    const int r = idx / ND, c = idx - ND * (idx / ND);
    if (r < nb && c < nb) L[w.Mb + idx] -= L[w.lz + r] * L[w.z + c];
  }
  if (lane < nb) E.drive_bar_one(lane, L[w.lz + lane]);
  wsync();
  // CRBA^T, per body i: F_i = Ic_i s_i, Fbar_i = sum over the ancestors j of
  // c_ij s_j (c_ii = Mbar_ii, c_ij = Mbar_ij + Mbar_ji), Icbar_i = Fbar_i s_i^T
  if (lane < nb) {
    const int i = lane;
    float si[6], F[6], Fb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    E.ld6(w.ks + i * 6, si);
    E.mul6(w.kIc + i * 36, si, F);
    E.st6(w.tF + i * 6, F);
    for (int j = i; j >= 0; j = M.parent[j]) {
      const float c = j == i ? L[w.Mb + i * ND + i] : L[w.Mb + i * ND + j] + L[w.Mb + j * ND + i];
      for (int t = 0; t < 6; ++t) Fb[t] += c * L[w.ks + j * 6 + t];
    }
    E.st6(w.tFb + i * 6, Fb);
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) L[w.Icb + i * 36 + r * 6 + c] = Fb[r] * si[c];
  }
  wsync();
  // sbar_j = sum over the descendants i of c_ij F_i + Ic_j^T Fbar_j; then
  // RNEA^T: fbar_i = -sum over the ancestors of s_k lz_k, sbar_i -= lz_i f_i
  if (lane < nb) {
    const int j = lane;
    float sb[6], Fb[6];
    E.ld6(w.tFb + j * 6, Fb);
    E.mul6t(w.kIc + j * 36, Fb, sb);
    for (int i = j; i < nb; ++i) {
      if (!((M.anc[i] >> j) & 1)) continue;
      const float c = j == i ? L[w.Mb + i * ND + i] : L[w.Mb + i * ND + j] + L[w.Mb + j * ND + i];
      for (int t = 0; t < 6; ++t) sb[t] += c * L[w.tF + i * 6 + t];
    }
    const float Cb = -L[w.lz + j];
    float fb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k <= j; ++k)
      if ((M.anc[j] >> k) & 1) {
        const float ck = -L[w.lz + k];
        for (int t = 0; t < 6; ++t) fb[t] += L[w.ks + k * 6 + t] * ck;
      }
    E.st6(w.fbar + j * 6, fb);
    for (int t = 0; t < 6; ++t) sb[t] += Cb * L[w.rff + j * 6 + t];
    E.st6(w.sb + j * 6, sb);
  }
  wsync();
  // Ibar_i = Icbar_i + Ibar_par (one lane per entry, down the tree)
  if (lane < 36) {
    for (int i = 0; i < nb; ++i) {
      const int par = M.parent[i];
      L[w.Ib + i * 36 + lane] = L[w.Icb + i * 36 + lane] + (par >= 0 ? L[w.Ib + par * 36 + lane] : 0.f);
    }
  }
  wsync();
  // body terms of f = I a + v x* (I v): Ibar, the own parts of abar and vbar
  if (lane < nb) {
    const int i = lane;
    const long I = w.kI + i * 36;
    float v[6], acc[6], fb[6], t6[6], hv[6];
    E.ld6(w.rv + i * 6, v);
    E.ld6(w.ra + i * 6, acc);
    E.ld6(w.fbar + i * 6, fb);
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) L[w.Ib + i * 36 + r * 6 + c] += fb[r] * acc[c];
    E.mul6t(I, fb, t6);
    E.st6(w.tA + i * 6, t6);
    E.mul6(I, v, hv);
    V om{v[0], v[1], v[2]}, nu{v[3], v[4], v[5]}, hn{hv[0], hv[1], hv[2]}, hf{hv[3], hv[4], hv[5]};
    V fn{fb[0], fb[1], fb[2]}, ff{fb[3], fb[4], fb[5]};
    V omb = cross(hn, fn) + cross(hf, ff), nub = cross(hf, fn);
    V hnb = cross(fn, om), hfb = cross(fn, nu) + cross(ff, om);
    float hb[6] = {hnb.x, hnb.y, hnb.z, hfb.x, hfb.y, hfb.z};
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) L[w.Ib + i * 36 + r * 6 + c] += hb[r] * v[c];
    E.mul6t(I, hb, t6);
    float ov[6] = {omb.x + t6[0], omb.y + t6[1], omb.z + t6[2], nub.x + t6[3], nub.y + t6[4], nub.z + t6[5]};
    E.st6(w.tV + i * 6, ov);
  }
  wsync();
  // abar_i = subtree sum of the own parts (one lane per component, up the
  // tree); then the a = a_par + v x vJ term's share of vbar_i
  if (lane < 6) {
    for (int i = 0; i < nb; ++i) L[w.abar + i * 6 + lane] = L[w.tA + i * 6 + lane];
    for (int i = nb - 1; i > 0; --i) {
      const int par = M.parent[i];
      if (par >= 0) L[w.abar + par * 6 + lane] += L[w.abar + i * 6 + lane];
    }
  }
  wsync();
  if (lane < nb) {
    const int i = lane;
    float ab[6];
    E.ld6(w.abar + i * 6, ab);
    const float qd = L[s + ND + i];
    const float* si = L + w.ks + i * 6;
    V vJw{si[0] * qd, si[1] * qd, si[2] * qd}, vJv{si[3] * qd, si[4] * qd, si[5] * qd};
    V aw{ab[0], ab[1], ab[2]}, av{ab[3], ab[4], ab[5]};
    V omb2 = cross(vJw, aw) + cross(vJv, av), nub2 = cross(vJw, av);
    float o2[6] = {omb2.x, omb2.y, omb2.z, nub2.x, nub2.y, nub2.z};
    E.st6(w.tV2 + i * 6, o2);
  }
  wsync();
  // vbar_i = subtree sum of both own parts (one lane per component, up the
  // tree); the joint velocity's adjoint
  if (lane < 6) {
    for (int i = 0; i < nb; ++i) L[w.vbar + i * 6 + lane] = L[w.tV + i * 6 + lane] + L[w.tV2 + i * 6 + lane];
    for (int i = nb - 1; i > 0; --i) {
      const int par = M.parent[i];
      if (par >= 0) L[w.vbar + par * 6 + lane] += L[w.vbar + i * 6 + lane];
    }
  }
  wsync();
  if (lane < nb) {
    const int i = lane;
    float vb[6];
    E.ld6(w.vbar + i * 6, vb);
    float v[6], ab[6], si[6];
    E.ld6(w.rv + i * 6, v);
    E.ld6(w.abar + i * 6, ab);
    E.ld6(w.ks + i * 6, si);
    V om{v[0], v[1], v[2]}, nu{v[3], v[4], v[5]}, aw{ab[0], ab[1], ab[2]}, av{ab[3], ab[4], ab[5]};
    V vJwb = cross(aw, om) + cross(av, nu), vJvb = cross(av, om);
    float vJb[6] = {vJwb.x + vb[0], vJwb.y + vb[1], vJwb.z + vb[2], vJvb.x + vb[3], vJvb.y + vb[4], vJvb.z + vb[5]};
    const float qd = L[s + ND + i];
    float qdb = 0.f;
    for (int t = 0; t < 6; ++t) {
      L[w.sb + i * 6 + t] += qd * vJb[t];
      qdb += si[t] * vJb[t];
    }
    L[gB + ND + i] += qdb;
  }
  wsync();
  // per body, door / drawer joint and free body
  if (lane < nb) E.body_bar_one(lane);
  if (lane >= ND && lane < ND + E.sc.na) E.aux_dyn_bar_one(lane - ND);
  for (int f = lane; f < E.sc.nf; f += 64) E.free_dyn_bar_one(s, f);
  wsync();
}

// kinematics^T: joint k receives a_k . (Mo - o_k x F + Md) (revolute) or
// a_k . F (prismatic) with F, Mo, Md summed over the subtree of k
__device__ __forceinline__ void kin_bar_wave(const msa::Eng& E, float* L) {
  using namespace msa;
  const int lane = lane_id();
  const WS& w = E.w;
  const DModel& M = *E.sc.M;
  if (lane < E.nb) {
    const int i = lane;
    V F{0.f, 0.f, 0.f}, Mo{0.f, 0.f, 0.f}, Md{0.f, 0.f, 0.f};
    for (int k = i; k < E.nb; ++k)
      if ((M.anc[k] >> i) & 1) {
        F = F + E.v3(w.bacc + k * 9);
        Mo = Mo + E.v3(w.bacc + k * 9 + 3);
        Md = Md + E.v3(w.bacc + k * 9 + 6);
      }
    const V a = E.v3(w.ka + i * 3);
    L[w.gB + i] += M.jtype[i] == 0 ? dot(a, Mo + Md - cross(E.v3(w.ko + i * 3), F)) : dot(a, F);
  }
}

__device__ void bwd_scene(const BwdArgs& a, int s, float* L) {
  using namespace msa;
  const int lane = lane_id();
  const DScene& D = a.scenes[s];
  Eng E;
  E.sc = SceneRef{a.models + D.model, a.free + D.f0, a.statics + 6 * (size_t)D.s0, a.planes + D.p0, a.aux + D.a0,
                  D.hold, D.nf, D.ns, D.np, D.na};
  E.pr = a.pr;
  E.w = a.w;
  E.b = Buf{L, 1};
  E.nb = E.sc.M->nb;
  E.nsph = E.sc.M->nsph;
  E.status = 0;
  E.nc = E.nrob = E.nlim = 0;
  E.cur_s = a.w.st;
  const WS& w = a.w;
  const RecLayout& RL = a.RL;
  const float* rec = a.rec + (size_t)s * RL.total;
  const int nf = D.nf, na = D.na, fm = w.fmax;
  const size_t S = (size_t)a.S;
  const size_t oq = 16 * (size_t)s, oqd = 16 * S + 16 * (size_t)s;
  const size_t ofr = 32 * S + 16 * (size_t)D.f0, oax = 32 * S + 16 * (size_t)a.NF + 4 * (size_t)D.a0;
  const float* u = a.u + 16 * (size_t)s;
  Lv LV = lv_view(L, w);
  const bool prof = a.cycles != nullptr;
  unsigned long long cyc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long tc = prof ? clock64() : 0;
  auto phase = [&](int k) {
    if (prof) {
      unsigned long long t2 = clock64();
      cyc[k] += t2 - tc;
      tc = t2;
    }
  };

  // adjoint of the end state
  zero_lds(L, w.gA, w.ss);
  zero_lds(L, w.ub, ND);
  wsync();
  if (lane < ND) {
    L[w.gA + lane] = a.gxo[oq + lane];
    L[w.gA + ND + lane] = a.gxo[oqd + lane];
  }
  for (int i = lane; i < nf * 16; i += 64) L[w.gA + 32 + i] = a.gxo[ofr + i];
  if (lane < na * 4) L[w.gA + 32 + 16 * fm + lane] = a.gxo[oax + lane];
  wsync();

  for (int si = a.pr.nsub - 1; si >= 0; --si) {
    const float* st0 = rec + (size_t)si * RL.ss;
    const float* st1 = rec + (size_t)(si + 1) * RL.ss;
    const float* cr = rec + RL.con + (size_t)si * RL.cstride;
    // state at the substep start; velocities at its end (after Gauss-Seidel)
    for (int i = lane; i < w.ss; i += 64) L[w.st + i] = st0[i];
    if (lane < ND) L[w.vR + lane] = st1[ND + lane];
    if (lane < na) L[w.vA + lane] = st1[32 + 16 * fm + 4 * lane + 1];
    for (int f = lane; f < nf; f += 64) {
      const float* x = st1 + 32 + 16 * f;
      L[w.vF + f * 6 + 0] = x[8]; L[w.vF + f * 6 + 1] = x[9]; L[w.vF + f * 6 + 2] = x[10];
      L[w.vF + f * 6 + 3] = x[12]; L[w.vF + f * 6 + 4] = x[13]; L[w.vF + f * 6 + 5] = x[14];
    }
    // the substep's contacts as the forward kernel emitted them
    const int NCf = __float_as_int(cr[0]), NL = __float_as_int(cr[1]), NR = __float_as_int(cr[2]);
    const int nc = NCf - NL;
    for (int ci = lane; ci < nc; ci += 64) {
      const float* c = cr + 4 + (size_t)(NL + ci) * CSTR;
      const int info = __float_as_int(c[0]);
      const int key = __float_as_int(c[16]);
      const int aside = info & 0xffff;
      const int akind = (aside >> 8) & 0xff, aidx = aside & 0xff;
      const int osub = key & 0xff, tk = (key >> 8) & 3, ti = key >> 10;
      int ok, oi, ov = 0;
      float r;
      if (akind == 1) {  // robot sphere
        ok = 0;
        oi = osub;
        r = E.sc.M->sph[osub].w;
      } else {  // free body
        oi = aidx;
        if (E.sc.F[aidx].type == 0) {
          ok = 1;
          ov = osub;
          r = 0.f;
        } else {
          ok = 2;
          r = E.sc.F[aidx].half[0];
        }
      }
      const long eo = w.con + (long)ci * CR;
      V n{c[1], c[2], c[3]}, p{c[4], c[5], c[6]};
      L[eo + C_ID] = pack_ids(ok, oi, ov, tk, ti);
      L[eo + C_R] = r;
      L[eo + C_PHI] = c[14];
      bs3(E.b, eo + C_N, n);
      bs3(E.b, eo + C_P, p);
    }
    wsync();
    phase(0);
    // recompute: drive, kinematics, frames and dynamics (without the
    // unconstrained velocities) on one lane; M~^-1 and the contact rows over
    // the lanes; the limit rows and the level schedule on one lane
    E.nc = nc;
    E.nrob = NR;
    recompute_wave(E, L, u);
    phase(1);
    wsync();
    solve_z_wave(E, L);
    rows_wave(E, L);
    if (lane == 0) {
      E.build_lims();
      if (E.nlim != NL) E.status |= MS_ST_RECORD;
      LV.cnt[2] = E.nlim;
      LV.cnt[4] = (int)E.status;
    }
    wsync();
    // level schedule.  Rows are merged into groups first: a run of
    // consecutive rows between one free body and static targets is one group
    // (reversed by one lane, last row first, with the body in registers);
    // every other row is a group of its own.  level(g) = 1 + the largest
    // level of the earlier groups sharing a dynamic node.  Each row's nodes
    // packed per lane; the groups' first rows; one pass over the groups with
    // the last level of node j in lane j's register (read with readlane);
    // then per-level counts, offsets and the order (entries: first row |
    // rows << 16)
    E.nlim = LV.cnt[2];
    {
      const int R = E.nlim + E.nc;
      for (int r = lane; r < R; r += 64) {
        int n1, n2;
        row_nodes(E, r, n1, n2);
        bool robot = false, single = false;
        if (r >= E.nlim) {
          const Ids id = E.ids(w.con + (long)(r - E.nlim) * CR);
          robot = id.ok == 0;
          single = id.ok != 0 && (id.tk == 0 || id.tk == 1);
        }
        LV.lvl[r] = n1 | ((n2 + 1) << 8) | (robot ? 1 << 16 : 0) | (single ? 1 << 17 : 0);
      }
      wsync();
      int G = 0;
      for (int base = 0; base < R; base += 64) {
        const int r = base + lane;
        bool st = false;
        if (r < R) {
          const int pk = LV.lvl[r];
          st = true;
          if (r > 0 && (pk >> 17) & 1) {
            const int pp = LV.lvl[r - 1];
            st = !(((pp >> 17) & 1) && (pp & 0xff) == (pk & 0xff));
          }
        }
        const uint64_t mk = __ballot(st);
        if (st) LV.gfirst[G + __popcll(mk & ((1ull << lane) - 1ull))] = r;
        G += __popcll(mk);
      }
      if (lane == 0) LV.gfirst[G] = R;
      wsync();
      int last = 0, maxl = 0;
      for (int base = 0; base < G; base += 64) {
        const int pkv = base + lane < G ? LV.lvl[LV.gfirst[base + lane]] : 0;
        int mine = 0;
        const int n = G - base < 64 ? G - base : 64;
        for (int k = 0; k < n; ++k) {
          const int pk = __builtin_amdgcn_readlane(pkv, k);
          const int n1 = pk & 0xff, n2 = ((pk >> 8) & 0xff) - 1;
          int lv = __builtin_amdgcn_readlane(last, n1);
          if (n2 >= 0) {
            const int l2 = __builtin_amdgcn_readlane(last, n2);
            lv = l2 > lv ? l2 : lv;
          }
          ++lv;
          if (lane == n1 || lane == n2) last = lv;
          if (lane == k) mine = lv | (pk & (1 << 16));
          maxl = lv > maxl ? lv : maxl;
        }
        wsync();
        // group g's first row is at index >= g, so the packs still to be
        // read (groups past this chunk) are not overwritten
        if (base + lane < G) LV.lvl[base + lane] = mine;
      }
      for (int l = lane; l <= maxl + 1; l += 64) {
        LV.loff[l] = 0;
        LV.rob[l] = -1;
      }
      wsync();
      for (int g = lane; g < G; g += 64) {
        const int v = LV.lvl[g], lv = v & 0xffff;
        if (v >> 16) LV.rob[lv] = LV.gfirst[g];
        else atomicAdd(&LV.loff[lv], 1);
      }
      wsync();
      if (lane == 0) {
        int acc = 0;
        for (int l = 1; l <= maxl; ++l) {
          const int c = LV.loff[l];
          LV.loff[l - 1] = acc;
          acc += c;
        }
        LV.loff[maxl] = acc;
      }
      wsync();
      // fill (groups of one level touch disjoint bodies, so their order
      // within the level does not change any result): loff[l - 1] is the
      // running write position of level l
      for (int g = lane; g < G; g += 64) {
        const int v = LV.lvl[g];
        if (!(v >> 16)) {
          const int r0 = LV.gfirst[g];
          LV.order[atomicAdd(&LV.loff[(v & 0xffff) - 1], 1)] = r0 | ((LV.gfirst[g + 1] - r0) << 16);
        }
      }
      wsync();
      if (lane == 0) {
        // restore the offsets
        int acc = 0;
        for (int l = 1; l <= maxl; ++l) {
          const int end = LV.loff[l - 1];
          LV.loff[l - 1] = acc;
          acc = end;
        }
        LV.loff[maxl] = acc;
        LV.cnt[0] = E.nc;
        LV.cnt[1] = E.nrob;
        LV.cnt[3] = maxl;
      }
    }
    wsync();
    phase(2);
    E.nc = LV.cnt[0];
    E.nrob = LV.cnt[1];
    E.nlim = LV.cnt[2];
    E.status = (uint32_t)LV.cnt[4];
    const int maxl = LV.cnt[3];
    // the tape of this substep's sweeps: two sweeps at a time staged in an
    // LDS ring (sweep it in slot it & 1); the reverse sweep it reads sweeps
    // it and it - 1
    const float* tape_g = rec + RL.tape + (size_t)si * a.pr.K * RL.tsw;
    E.tb = Buf{L + w.tring, 1};
    E.tsw = w.trs;
    E.tmask = 1;
    const int R3 = 3 * (E.nlim + E.nc);
    auto stage = [&](int it) {
      float* dst = L + w.tring + (it & 1) * w.trs;
      const float* src = tape_g + (size_t)it * RL.tsw;
      for (int i = lane; i < R3; i += 64) dst[i] = src[i];
    };
    // a reverse sweep reads its own tape slot and the previous sweep's; the
    // sweep two back is loaded into registers a sweep ahead and written to
    // its slot once that slot is free, so that no sweep waits for the record
    constexpr int TPF = 8;  // tape floats per lane carried in registers (the rest staged directly)
    float pf[TPF];
    auto fetch = [&](int it) {
      const float* src = tape_g + (size_t)it * RL.tsw;
#pragma unroll
      for (int k = 0; k < TPF; ++k) {
        const int i = lane + 64 * k;
        pf[k] = i < R3 ? src[i] : 0.f;
      }
    };
    auto put = [&](int it) {
      float* dst = L + w.tring + (it & 1) * w.trs;
#pragma unroll
      for (int k = 0; k < TPF; ++k) {
        const int i = lane + 64 * k;
        if (i < R3) dst[i] = pf[k];
      }
      const float* src = tape_g + (size_t)it * RL.tsw;
      for (int i = lane + 64 * TPF; i < R3; i += 64) dst[i] = src[i];
    };
    if (a.pr.K > 0) stage(a.pr.K - 1);
    if (a.pr.K > 1) stage(a.pr.K - 2);
    if (a.pr.K > 2) fetch(a.pr.K - 3);
    // adjoint accumulators of this substep
    zero_lds(L, w.gB, w.ss);
    zero_lds(L, w.vRb, ND);
    zero_lds(L, w.vAb, AMAX);
    zero_lds(L, w.vFb, fm * 6);
    zero_lds(L, w.limb, 2 * AMAX);
    zero_lds(L, w.llamb, 2 * AMAX);
    zero_lds(L, w.lamb, 3 * E.nc);
    zero_lds(L, w.conb, E.nc * CB);
    zero_lds(L, w.rJb, E.nrob * 3 * ND);
    zero_lds(L, w.rwb, E.nrob * 3 * ND);
    zero_lds(L, w.fb, fm * FB);
    zero_lds(L, w.xb, AMAX * XB);
    zero_lds(L, w.bacc, ND * 9);
    zero_lds(L, w.Mb, ND * ND);
    wsync();
    // integrate^T: lane per DoF, door / drawer joint and free body
    if (lane < ND) E.integrate_bar_dof(lane);
    if (lane >= ND && lane < ND + AMAX) E.integrate_bar_aux(lane - ND);
    for (int f = lane; f < nf; f += 64) E.integrate_bar_free(w.st, f);
    wsync();
    phase(3);
    // Gauss-Seidel sweeps in reverse, levels in reverse
    for (int it = a.pr.K - 1; it >= 0; --it) {
      if (it >= 1 && it <= a.pr.K - 2) {
        put(it - 1);
        if (it >= 2) fetch(it - 2);
      }
      lds_order();
      for (int lv = maxl; lv >= 1; --lv) {
        const int rr = LV.rob[lv];
        if (rr >= 0) robot_contact_bar(E, it, rr - E.nlim, L);
        const int o0 = LV.loff[lv - 1], o1 = LV.loff[lv];
        for (int k = o0 + lane; k < o1; k += 64) {
          const int ge = LV.order[k], r = ge & 0xffff, gn = ge >> 16;
          if (gn > 1) E.contact_group_bar(it, r - E.nlim, gn);
          else if (r < E.nlim) E.limit_bar(it, r);
          else E.contact_bar(it, r - E.nlim);
        }
        lds_order();
      }
    }
    phase(4);
    // rows^T: robot rows over the lanes; then level by level (rows of a
    // level touch disjoint bodies) the other rows, the robot rows' target
    // sides and the limit rows, one lane each
    robot_rows_bar_wave(E, L);
    for (int lv = 1; lv <= maxl; ++lv) {
      const int rr = LV.rob[lv];
      if (rr >= 0 && lane == 0) E.rows_bar_one(rr - E.nlim, false);
      const int o0 = LV.loff[lv - 1], o1 = LV.loff[lv];
      for (int k = o0 + lane; k < o1; k += 64) {
        const int ge = LV.order[k], r0 = ge & 0xffff, gn = ge >> 16;
        for (int r = r0; r < r0 + gn; ++r) {
          if (r < E.nlim) E.rows_bar_limit(r);
          else E.rows_bar_one(r - E.nlim, false);
        }
      }
      wsync();
    }
    phase(5);
    dynamics_bar_wave(E, L);
    phase(6);
    // contacts^T level by level (rows of a level touch disjoint bodies);
    // frames^T per free body / joint; kinematics^T per joint
    for (int lv = 1; lv <= maxl; ++lv) {
      const int rr = LV.rob[lv];
      if (rr >= 0 && lane == 0) E.contact_geom_bar(rr - E.nlim);
      const int o0 = LV.loff[lv - 1], o1 = LV.loff[lv];
      for (int k = o0 + lane; k < o1; k += 64) {
        const int ge = LV.order[k], r0 = ge & 0xffff, gn = ge >> 16;
        for (int r = r0; r < r0 + gn; ++r)
          if (r >= E.nlim) E.contact_geom_bar(r - E.nlim);
      }
      wsync();
    }
    if (lane == 0) LV.cnt[4] = (int)E.status;
    for (int f = lane; f < E.sc.nf; f += 64) E.free_frame_bar(w.st, f);
    if (lane >= ND && lane < ND + E.sc.na) E.aux_frame_bar(lane - ND);
    kin_bar_wave(E, L);
    wsync();
    for (int i = lane; i < w.ss; i += 64) L[w.gA + i] = L[w.gB + i];
    wsync();
    phase(7);
  }
  if (lane < ND) {
    a.gxi[oq + lane] = L[w.gA + lane];
    a.gxi[oqd + lane] = L[w.gA + ND + lane];
    a.gu[16 * (size_t)s + lane] = L[w.ub + lane];
  }
  for (int i = lane; i < nf * 16; i += 64) a.gxi[ofr + i] = L[w.gA + 32 + i];
  if (lane < na * 4) a.gxi[oax + lane] = L[w.gA + 32 + 16 * fm + lane];
  if (lane == 0 && LV.cnt[4]) a.status[s] |= (uint32_t)LV.cnt[4];
  if (prof && lane == 0)
    for (int k = 0; k < 8; ++k) a.cycles[(size_t)s * 8 + k] = cyc[k];
}

// does every substep's contact list of scene s hold at most cc contacts and
// rc robot contacts?  cost: the sum over the substeps of contacts + 64 robot
// contacts (the reverse sweeps take about that many contact reversals)
__device__ bool rec_fits(const float* rec, const RecLayout& RL, int nsub, int s, int cc, int rc, int* cost = nullptr) {
  const float* cr = rec + (size_t)s * RL.total + RL.con;
  bool ok = true;
  int c = 0;
  for (int si = 0; si < nsub; ++si, cr += RL.cstride) {
    const int NCf = __float_as_int(cr[0]), NL = __float_as_int(cr[1]), NR = __float_as_int(cr[2]);
    ok = ok && NL >= 0 && NL <= 2 * AMAX && NCf - NL <= cc && NR <= rc;
    c += (NCf - NL) + 64 * NR;
  }
  if (cost) *cost = c;
  return ok;
}

// wave-level inclusive prefix sum
__device__ __forceinline__ int wave_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

}  // namespace

// the LDS layout must hold the scene's lists (else the scene is flagged and
// left out)
__device__ void bwd_checked(const BwdArgs& a, int s, float* lds) {
  if (!rec_fits(a.rec, a.RL, a.pr.nsub, s, a.w.ccap, a.w.rcap)) {
    if (lane_id() == 0) a.status[s] |= MS_ST_RECORD;
    return;
  }
  bwd_scene(a, s, lds);
}

__global__ __launch_bounds__(64) void k_step_bwd_wave(BwdArgs a) {
  extern __shared__ float lds[];
  // mode 2 loops over the first *n_over positions; modes 0 and 1 take one
  // position each (one call site keeps the scene's code inlined)
  const bool loop = a.fit_mode == 2;
  const int end = loop ? *a.n_over : a.S;
  const int step = loop ? (int)gridDim.x : a.S;
  for (int pos = (a.fit_mode == 1 ? *a.n_over : 0) + (int)blockIdx.x; pos < end; pos += step) {
    bwd_checked(a, a.order[pos], lds);
    wsync();
  }
}

// sort slot of each scene: group * NKEY + (NKEY - 1 - key), the cost key
// clamped to [0, NKEY), group 0 for the scenes that overflow (fit_c, fit_r)
constexpr int NKEY = 4096;
__global__ __launch_bounds__(256) void k_bwd_keys(const float* rec, RecLayout RL, int S, int nsub, int fit_c,
                                                  int fit_r, int* slot) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= S) return;
  int c = 0;
  const bool fits = rec_fits(rec, RL, nsub, s, fit_c, fit_r, &c);
  const int g = fit_c > 0 && !fits ? 0 : 1;
  const int k = c < 0 ? 0 : (c >= NKEY ? NKEY - 1 : c);
  slot[s] = g * NKEY + (NKEY - 1 - k);
}

// counting sort of the scenes by their slots: one workgroup
__global__ __launch_bounds__(1024) void k_bwd_order(const int* slot, int S, int* order, int* n_over) {
  __shared__ int cnt[2 * NKEY];
  __shared__ int wsum[16];
  const int t = threadIdx.x;
  for (int i = t; i < 2 * NKEY; i += 1024) cnt[i] = 0;
  __syncthreads();
  auto slot_of = [&](int s) { return slot[s]; };
  for (int s = t; s < S; s += 1024) atomicAdd(&cnt[slot_of(s)], 1);
  __syncthreads();
  // exclusive scan: thread t owns entries 8t .. 8t + 7
  int loc[8], sum = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    loc[i] = cnt[8 * t + i];
    sum += loc[i];
  }
  const int inc = wave_scan(sum);
  if ((t & 63) == 63) wsum[t >> 6] = inc;
  __syncthreads();
  int base = inc - sum;
  for (int wv = 0; wv < (t >> 6); ++wv) base += wsum[wv];
  // thread NKEY / 8 owns the first entry of group 1
  if (t == NKEY / 8) *n_over = base;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    cnt[8 * t + i] = base;
    base += loc[i];
  }
  __syncthreads();
  for (int s = t; s < S; s += 1024) order[atomicAdd(&cnt[slot_of(s)], 1)] = s;
}

// one wavefront that waits about `ticks` of the 100 MHz wall clock (a
// bounded wait: the clock always advances)
__global__ __launch_bounds__(64) void k_delay(long long ticks) {
  const long long t0 = (long long)wall_clock64();
  while ((long long)wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(2);
}

void launch_delay(long long ticks, hipStream_t st) { hipLaunchKernelGGL(k_delay, dim3(1), dim3(64), 0, st, ticks); }

void launch_bwd_order(const float* rec, const RecLayout& RL, int S, int nsub, int fit_c, int fit_r, int* slot,
                      int* order, int* n_over, hipStream_t st) {
  hipLaunchKernelGGL(k_bwd_keys, dim3((S + 255) / 256), dim3(256), 0, st, rec, RL, S, nsub, fit_c, fit_r, slot);
  hipLaunchKernelGGL(k_bwd_order, dim3(1), dim3(1024), 0, st, slot, S, order, n_over);
}

void launch_step_bwd_wave(const BwdArgs& a, size_t lds_bytes, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_step_bwd_wave, dim3(grid), dim3(64), lds_bytes, st, a);
}
const void* step_bwd_wave_ptr() { return reinterpret_cast<const void*>(&k_step_bwd_wave); }

}  // namespace msk
