// ms_tasks.hip -- subtask success predicates, event labels and trajectory
// categories (App. A.2 subtask definitions, App. A.3 event labeling and
// success / failure modes) for every scene of a batch, one lane per scene.
//
// The work per scene is a forward-kinematics walk along two ancestor chains
// and a few comparisons: latency-bound bookkeeping that runs once per control
// step next to the physics step.
#include "ms_tasks.h"

namespace msk {
namespace {

struct f3t {
  float x, y, z;
};
__device__ __forceinline__ f3t rmul(const float* R, f3t v) {
  return {R[0] * v.x + R[1] * v.y + R[2] * v.z, R[3] * v.x + R[4] * v.y + R[5] * v.z,
          R[6] * v.x + R[7] * v.y + R[8] * v.z};
}
__device__ __forceinline__ void mmul(const float* A, const float* B, float* C) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) C[r * 3 + c] = A[r * 3] * B[c] + A[r * 3 + 1] * B[3 + c] + A[r * 3 + 2] * B[6 + c];
}

// world pose (R, p) of body `body`: composes the joint transforms of its
// ancestors in index order (a parent always precedes its children)
__device__ void body_pose(const DModel& M, const float* q, int body, float* R, f3t& p) {
  for (int t = 0; t < 9; ++t) R[t] = (t % 4 == 0) ? 1.f : 0.f;
  p = {0.f, 0.f, 0.f};
  const int anc = M.anc[body];
  for (int j = 0; j < M.nb; ++j) {
    if (!((anc >> j) & 1)) continue;
    float Rj[9];
    mmul(R, M.xtR[j], Rj);
    const f3t xo = rmul(R, f3t{M.xtp[j][0], M.xtp[j][1], M.xtp[j][2]});
    p = {p.x + xo.x, p.y + xo.y, p.z + xo.z};
    const f3t ax{M.axis[j][0], M.axis[j][1], M.axis[j][2]};
    if (M.jtype[j] == 0) {
      // rotation by q about the unit axis (Rodrigues)
      float sn, cs;
      sincosf(q[j], &sn, &cs);
      const float c1 = 1.f - cs;
      const float Rr[9] = {cs + ax.x * ax.x * c1,        ax.x * ax.y * c1 - ax.z * sn, ax.x * ax.z * c1 + ax.y * sn,
                           ax.y * ax.x * c1 + ax.z * sn, cs + ax.y * ax.y * c1,        ax.y * ax.z * c1 - ax.x * sn,
                           ax.z * ax.x * c1 - ax.y * sn, ax.z * ax.y * c1 + ax.x * sn, cs + ax.z * ax.z * c1};
      mmul(Rj, Rr, R);
    } else {
      const f3t a = rmul(Rj, ax);
      p = {p.x + a.x * q[j], p.y + a.y * q[j], p.z + a.z * q[j]};
      for (int t = 0; t < 9; ++t) R[t] = Rj[t];
    }
  }
}

struct Lim {
  float ee, arm, torso, col;  // end-effector distance, arm and torso joint error, collision force
};
// success limits per subtask (App. A.2)
__device__ __forceinline__ Lim limits(int kind) {
  if (kind == MS_TASK_PICK) return {0.05f, 0.6f, 1e30f, 5000.f};
  if (kind == MS_TASK_PLACE) return {0.05f, 0.2f, 0.01f, 7500.f};
  return {0.05f, 0.2f, 0.01f, 10000.f};
}

__global__ __launch_bounds__(64) void k_task_eval(TaskArgs a) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= a.S) return;
  const bool begin = a.robot_force == nullptr;
  if (begin && a.mask && !a.mask[s]) return;
  ms_episode& E = a.ep[s];
  if (!begin && E.ind == 0xffffffffu) return;  // the episode did not start
  const ms_task T = a.tasks[s];
  const DScene& D = a.scenes[s];
  const DModel& M = a.models[D.model];
  const ms_task_robot& R = a.robot;
  const size_t S = (size_t)a.S;
  const float* q = a.x + 16 * (size_t)s;
  const float* qd = a.x + 16 * S + 16 * (size_t)s;
  const bool obj = T.kind == MS_TASK_PICK || T.kind == MS_TASK_PLACE;
  const bool art = T.kind == MS_TASK_OPEN || T.kind == MS_TASK_CLOSE;
  if (!(obj || art) || T.target < 0 || (obj && T.target >= D.nf) || (art && T.target >= D.na) ||
      (art && !a.aux[D.a0 + T.target].has_limit)) {
    E.ind = 0xffffffffu;
    return;
  }
  // end effector in the base frame
  float Re[9], Rb[9];
  f3t pe, pb;
  body_pose(M, q, R.ee_body, Re, pe);
  body_pose(M, q, R.base_body, Rb, pb);
  const f3t eo = rmul(Re, f3t{R.ee_offset[0], R.ee_offset[1], R.ee_offset[2]});
  const f3t dw{pe.x + eo.x - pb.x, pe.y + eo.y - pb.y, pe.z + eo.z - pb.z};
  const f3t eb{Rb[0] * dw.x + Rb[3] * dw.y + Rb[6] * dw.z, Rb[1] * dw.x + Rb[4] * dw.y + Rb[7] * dw.z,
               Rb[2] * dw.x + Rb[5] * dw.y + Rb[8] * dw.z};
  const f3t de{eb.x - R.ee_rest[0], eb.y - R.ee_rest[1], eb.z - R.ee_rest[2]};
  const float d_ee = sqrtf(de.x * de.x + de.y * de.y + de.z * de.z);
  float j_arm = 0.f, qd_arm = 0.f;
  for (int i = R.arm0; i < R.arm0 + R.narm; ++i) {
    j_arm = fmaxf(j_arm, fabsf(q[i] - R.q_rest[i]));
    qd_arm = fmaxf(qd_arm, fabsf(qd[i]));
  }
  const float j_tor = R.torso >= 0 ? fabsf(q[R.torso] - R.q_rest[R.torso]) : 0.f;
  const bool stat = qd_arm <= 0.2f && fabsf(qd[R.base_x]) <= 0.05f && fabsf(qd[R.base_y]) <= 0.05f &&
                    fabsf(qd[R.base_yaw]) <= 0.05f;
  // the target's contact data and position
  const size_t row = obj ? (size_t)D.f0 + T.target : (size_t)a.NF + D.a0 + T.target;
  const float f_ee = a.grip ? a.grip[2 * row] / (float)a.n_sub : 0.f;
  const float f_fing = a.grip ? a.grip[2 * row + 1] : 0.f;
  const bool grasped = obj && f_fing >= R.grasp_force;
  float d_goal = 0.f, aq = 0.f;
  if (obj) {
    const float* xf = a.x + 32 * S + 16 * row;
    const float gx = xf[0] - T.goal[0], gy = xf[1] - T.goal[1], gz = xf[2] - T.goal[2];
    d_goal = sqrtf(gx * gx + gy * gy + gz * gz);
  } else {
    aq = a.x[32 * S + 16 * (size_t)a.NF + 4 * ((size_t)D.a0 + T.target)];
  }
  const float cum = begin ? 0.f : E.cumcol + a.robot_force[s] / (float)a.n_sub;
  const float aq0 = begin ? aq : E.aq0;
  const Lim lim = limits(T.kind);
  const bool rest = d_ee <= lim.ee && j_arm <= lim.arm && j_tor <= lim.torso && stat && cum <= lim.col;
  uint32_t ind = 0;
  if (grasped) ind |= MS_IND_GRASPED;
  if (f_ee > 0.f) ind |= MS_IND_CONTACT;
  if (cum > lim.col) ind |= MS_IND_EXCESSIVE;
  bool succ = false;
  if (T.kind == MS_TASK_PICK) {
    succ = grasped && rest;
  } else if (T.kind == MS_TASK_PLACE) {
    if (d_goal <= 0.15f) ind |= MS_IND_AT_GOAL;
    succ = !grasped && d_goal <= 0.15f && rest;
  } else {
    const DAux& X = a.aux[D.a0 + T.target];
    const float span = X.hi - X.lo;
    bool st, sl;
    if (T.kind == MS_TASK_OPEN) {
      st = aq >= T.open_frac * span + X.lo;
      sl = aq >= 0.1f * span + X.lo;
    } else {
      st = aq <= 0.01f * span + X.lo;
      sl = aq < aq0 - 0.05f * span;
    }
    if (st) ind |= MS_IND_OPEN;
    if (sl) ind |= MS_IND_SLIGHT;
    succ = st && rest;
  }
  if (succ) ind |= MS_IND_SUCCESS;
  if (a.pred) {
    float* o = a.pred + 8 * (size_t)s;
    o[MS_PRED_D_EE] = d_ee;
    o[MS_PRED_J_ARM] = j_arm;
    o[MS_PRED_J_TORSO] = j_tor;
    o[MS_PRED_QD_MAX] = qd_arm;
    o[MS_PRED_D_GOAL] = d_goal;
    o[MS_PRED_AQ] = aq;
    o[MS_PRED_F_EE] = f_ee;
    o[MS_PRED_F_FINGER] = f_fing;
  }
  if (begin) {
    E.cumcol = 0.f;
    E.aq0 = aq;
    E.d0 = d_goal;
    E.ind = ind;
    E.t = 0;
    E.n = 0;
    for (int k = 0; k < 8; ++k) E.last[k] = -1;
    for (int k = 0; k < MS_EP_LIST; ++k) E.list[k] = 0;
    return;
  }
  // events of this step, in the appendix's order
  const uint32_t p = E.ind;
  auto was = [&](uint32_t b) { return (p & b) != 0; };
  auto is = [&](uint32_t b) { return (ind & b) != 0; };
  auto rise = [&](uint32_t b) { return !was(b) && is(b); };
  auto fall = [&](uint32_t b) { return was(b) && !is(b); };
  int n = E.n;
  auto add = [&](bool happened, int code) {
    if (!happened) return;
    if (n < MS_EP_LIST) E.list[n] = (uint8_t)code;
    E.last[code] = n;
    ++n;
  };
  if (T.kind == MS_TASK_PICK) {
    add(rise(MS_IND_CONTACT), MS_EV_PICK_CONTACT);
    add(rise(MS_IND_GRASPED), MS_EV_PICK_GRASPED);
    add(fall(MS_IND_GRASPED), MS_EV_PICK_DROPPED);
    add(rise(MS_IND_SUCCESS), MS_EV_PICK_SUCCESS);
    add(rise(MS_IND_EXCESSIVE), MS_EV_PICK_EXCESSIVE);
  } else if (T.kind == MS_TASK_PLACE) {
    add(rise(MS_IND_GRASPED), MS_EV_PLACE_GRASPED);
    add(rise(MS_IND_AT_GOAL), MS_EV_PLACE_AT_GOAL);
    add(is(MS_IND_AT_GOAL) && fall(MS_IND_GRASPED), MS_EV_PLACE_RELEASED_AT_GOAL);
    add(!is(MS_IND_AT_GOAL) && fall(MS_IND_GRASPED), MS_EV_PLACE_RELEASED_OUTSIDE);
    add(fall(MS_IND_AT_GOAL), MS_EV_PLACE_LEFT_GOAL);
    add(rise(MS_IND_SUCCESS), MS_EV_PLACE_SUCCESS);
    add(rise(MS_IND_EXCESSIVE), MS_EV_PLACE_EXCESSIVE);
  } else {
    // open: opened / slightly opened / closed; close: closed / slightly closed / opened
    add(rise(MS_IND_CONTACT), 0);
    add(rise(MS_IND_OPEN), 1);
    add(rise(MS_IND_SLIGHT), 2);
    add(fall(MS_IND_OPEN), 3);
    add(rise(MS_IND_SUCCESS), 4);
    add(rise(MS_IND_EXCESSIVE), 5);
  }
  E.n = n;
  E.cumcol = cum;
  E.ind = ind;
  E.t += 1;
}

// ------------------------------------------------------------ categories
struct Ev {
  const ms_episode& E;
  __device__ bool in(int c) const { return E.last[c] >= 0; }
  __device__ int at(int c) const { return E.last[c]; }
  // the list equals (c0, c1, ...) of length len
  __device__ bool eq(int len, int c0 = -1, int c1 = -1, int c2 = -1) const {
    if (E.n != len) return false;
    const int c[3] = {c0, c1, c2};
    for (int k = 0; k < len && k < 3; ++k)
      if (E.list[k] != c[k]) return false;
    return true;
  }
};

__device__ int mode_pick(const Ev& v) {
  const ms_episode& E = v.E;
  const bool exc = v.in(MS_EV_PICK_EXCESSIVE);
  const bool drop_last = v.in(MS_EV_PICK_DROPPED) && v.at(MS_EV_PICK_DROPPED) > v.at(MS_EV_PICK_GRASPED);
  if (v.in(MS_EV_PICK_SUCCESS)) {
    if (exc) return 4;
    if (drop_last) return 3;
    if (v.eq(3, MS_EV_PICK_CONTACT, MS_EV_PICK_GRASPED, MS_EV_PICK_SUCCESS)) return 1;
    if (E.n > 3 && E.list[0] == MS_EV_PICK_CONTACT && E.list[1] == MS_EV_PICK_GRASPED) return 2;
    return 0;
  }
  if (exc) return 5;
  if (E.n == 0) return 6;
  if (v.eq(1, MS_EV_PICK_CONTACT)) return 7;
  if (drop_last) return 8;
  if (v.in(MS_EV_PICK_GRASPED) && v.at(MS_EV_PICK_GRASPED) > v.at(MS_EV_PICK_DROPPED)) return 9;
  return 0;
}

__device__ int mode_place(const Ev& v) {
  const ms_episode& E = v.E;
  const bool exc = v.in(MS_EV_PLACE_EXCESSIVE);
  const int i_at = v.at(MS_EV_PLACE_AT_GOAL), i_left = v.at(MS_EV_PLACE_LEFT_GOAL);
  const int i_ra = v.at(MS_EV_PLACE_RELEASED_AT_GOAL), i_ro = v.at(MS_EV_PLACE_RELEASED_OUTSIDE);
  const int i_gr = v.at(MS_EV_PLACE_GRASPED);
  const bool near0 = E.d0 <= 0.15f;
  if (v.in(MS_EV_PLACE_SUCCESS)) {
    if (exc) return 5;
    if (E.n <= 4 && (i_ra >= 0 || near0) && i_left <= i_at) return 1;
    if (E.n <= 4 && (i_ro >= 0 || !near0) && i_left <= i_at) return 2;
    if (i_at < i_left) return 3;
    if (E.n > 4 && i_at > i_left) return 4;
    return 0;
  }
  if (exc) return 6;
  if (E.n == 0) return 7;
  if (i_at < 0) return 8;
  const bool placed_latest = (E.n <= 2 && near0) || (i_ra > i_ro && i_ra > i_gr);
  const bool dropped_latest = (E.n <= 2 && !near0) || (i_ro > i_ra && i_ro > i_gr);
  if (placed_latest && i_left > i_at) return 9;
  if (dropped_latest && i_left > i_at) return 10;
  if (i_gr > i_ra && i_gr > i_ro) return 11;
  return 12;
}

// open and close share their event numbering: 0 contact, 1 the goal state
// reached (opened / closed), 2 slightly there, 3 the goal state left
// (closed / opened), 4 success, 5 excessive collisions
__device__ int mode_art(const Ev& v, bool open) {
  const bool exc = v.in(5);
  const int i_reach = v.at(1), i_slight = v.at(2), i_leave = v.at(3);
  if (v.in(4)) {
    if (exc) return 3;
    if (i_reach > i_leave) return 1;
    if (i_reach < i_leave) return 2;
    return 0;
  }
  if (exc) return 4;
  if (!v.in(0)) return 5;
  // open: closed after opening; close: opened after closing
  const bool undone = open ? (v.in(3) && i_leave > i_reach && i_leave > i_slight)
                           : (v.in(1) && i_leave > i_reach && i_leave > i_slight);
  if (undone) return 6;
  if (i_slight > i_reach && i_slight > i_leave) return 7;
  if (v.in(1)) return 8;
  return 9;
}

__global__ __launch_bounds__(64) void k_task_categorize(const ms_task* tasks, const ms_episode* ep, int32_t* mode,
                                                        int S) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= S) return;
  const ms_episode& E = ep[s];
  const Ev v{E};
  const int kind = tasks[s].kind;
  int m = 0;
  if (E.ind == 0xffffffffu) m = 0;
  else if (kind == MS_TASK_PICK) m = mode_pick(v);
  else if (kind == MS_TASK_PLACE) m = mode_place(v);
  else if (kind == MS_TASK_OPEN || kind == MS_TASK_CLOSE) m = mode_art(v, kind == MS_TASK_OPEN);
  mode[s] = m;
}

}  // namespace

void launch_task_eval(const TaskArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_task_eval, dim3((a.S + 63) / 64), dim3(64), 0, st, a);
}
void launch_task_categorize(const ms_task* tasks, const ms_episode* ep, int32_t* mode, int S, hipStream_t st) {
  hipLaunchKernelGGL(k_task_categorize, dim3((S + 63) / 64), dim3(64), 0, st, tasks, ep, mode, S);
}

}  // namespace msk
