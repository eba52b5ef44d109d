// ms_pack.h -- host-side validation and packing of a scene description into
// the device layout of ms_internal.h (used by the C ABI at batch creation).
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ms_phys.h"
#include "ms_internal.h"

namespace mspack {
using namespace msk;

inline thread_local std::string g_err;

inline ms_status fail(ms_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}



inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Counts {
  int S, M, NF, NS, NP, NA;
  int fmax, smax, pmax, amax;
  int nsph_max;  // most robot spheres of a model
};

inline ms_status validate(const ms_batch_desc* d, const ms_scene_desc* sc, Counts& c) {
  if (!d || !sc) return fail(MS_E_INVALID, "null desc or scene description");
  if (d->n_scenes <= 0) return fail(MS_E_INVALID, "n_scenes must be positive (got %d)", d->n_scenes);
  if (d->n_substeps <= 0 || d->n_substeps > 1000) return fail(MS_E_INVALID, "n_substeps out of range");
  if (d->pgs_iters < 0 || d->pgs_iters > 1000) return fail(MS_E_INVALID, "pgs_iters out of range");
  if (d->control_mode < 0 || d->control_mode > 3) return fail(MS_E_INVALID, "unknown control_mode %d", d->control_mode);
  if (d->control_mode == MS_CTRL_ACTIONS && sc && (!sc->model_act_kind || !sc->model_act_scale))
    return fail(MS_E_INVALID, "MS_CTRL_ACTIONS needs model_act_kind and model_act_scale");
  if (d->contact_cap <= 0 || d->contact_cap > 4096) return fail(MS_E_INVALID, "contact_cap out of range (1..4096)");
  if (d->robot_contact_cap < 0 || d->robot_contact_cap > d->contact_cap)
    return fail(MS_E_INVALID, "robot_contact_cap out of range (0..contact_cap)");
  if (!(d->h > 0.f) || !(d->mu >= 0.f) || !(d->margin >= 0.f) || !(d->baumgarte >= 0.f))
    return fail(MS_E_INVALID, "h must be > 0 and mu, margin, baumgarte >= 0");
  const void* req[] = {sc->model_nb, sc->model_parent, sc->model_jtype, sc->model_axis, sc->model_xt_rot,
                       sc->model_xt_pos, sc->model_mass, sc->model_com, sc->model_inertia, sc->model_kp,
                       sc->model_kd, sc->model_veldof, sc->model_armature, sc->model_damping, sc->model_nsph,
                       sc->model_sph_body, sc->model_sph, sc->model_sph_flags, sc->scene_model, sc->free_off,
                       sc->static_off, sc->plane_off, sc->aux_off, sc->scene_hold};
  for (const void* p : req)
    if (!p) return fail(MS_E_INVALID, "a required scene array is null");
  c.S = d->n_scenes;
  c.M = sc->n_models;
  c.nsph_max = 0;
  if (c.M <= 0) return fail(MS_E_INVALID, "n_models must be positive");
  for (int m = 0; m < c.M; ++m) {
    int nb = sc->model_nb[m], ns = sc->model_nsph[m];
    if (nb < 0 || nb > ND) return fail(MS_E_INVALID, "model %d: %d bodies (max %d)", m, nb, ND);
    if (ns < 0 || ns > SPH) return fail(MS_E_INVALID, "model %d: %d spheres (max %d)", m, ns, SPH);
    c.nsph_max = std::max(c.nsph_max, ns);
    for (int i = 0; i < nb; ++i) {
      int p = sc->model_parent[m * ND + i];
      if (p >= i || p < -1) return fail(MS_E_INVALID, "model %d body %d: parent %d must precede it", m, i, p);
      int jt = sc->model_jtype[m * ND + i];
      if (jt != 0 && jt != 1) return fail(MS_E_INVALID, "model %d body %d: joint type %d", m, i, jt);
    }
    if (sc->model_act_kind)
      for (int i = 0; i < nb; ++i) {
        int ak = sc->model_act_kind[m * ND + i];
        if (ak < 0 || ak > 4) return fail(MS_E_INVALID, "model %d DoF %d: action channel %d", m, i, ak);
      }
    int prev = 0;
    for (int k = 0; k < ns; ++k) {
      int b = sc->model_sph_body[m * SPH + k];
      if (b < 0 || b >= nb) return fail(MS_E_INVALID, "model %d sphere %d: body %d out of range", m, k, b);
      if (b < prev) return fail(MS_E_INVALID, "model %d: spheres must be sorted by body", m);
      prev = b;
    }
  }
  const int32_t* offs[4] = {sc->free_off, sc->static_off, sc->plane_off, sc->aux_off};
  const char* names[4] = {"free_off", "static_off", "plane_off", "aux_off"};
  int maxc[4] = {FMAXL, 1 << 20, PMAX, AMAX};
  int cnt[4], mx[4];
  for (int t = 0; t < 4; ++t) {
    if (offs[t][0] != 0) return fail(MS_E_INVALID, "%s[0] must be 0", names[t]);
    mx[t] = 0;
    for (int s = 0; s < c.S; ++s) {
      int n = offs[t][s + 1] - offs[t][s];
      if (n < 0) return fail(MS_E_INVALID, "%s not monotone at scene %d", names[t], s);
      if (n > maxc[t]) return fail(MS_E_INVALID, "scene %d: %d entries in %s (max %d)", s, n, names[t], maxc[t]);
      mx[t] = std::max(mx[t], n);
    }
    cnt[t] = offs[t][c.S];
  }
  c.NF = cnt[0]; c.NS = cnt[1]; c.NP = cnt[2]; c.NA = cnt[3];
  c.fmax = mx[0]; c.smax = mx[1]; c.pmax = mx[2]; c.amax = mx[3];
  // a contact's target index is stored in 16 bits by the adjoint
  if (c.smax > 65535) return fail(MS_E_INVALID, "a scene has %d furniture boxes (at most 65535)", c.smax);
  for (int s = 0; s < c.S; ++s) {
    int m = sc->scene_model[s];
    if (m < 0 || m >= c.M) return fail(MS_E_INVALID, "scene %d: model %d out of range", s, m);
  }
  if (c.NF > 0 && (!sc->free_type || !sc->free_size || !sc->free_mass || !sc->free_inertia))
    return fail(MS_E_INVALID, "free-body arrays are null");
  for (int f = 0; f < c.NF; ++f) {
    if (sc->free_type[f] != 0 && sc->free_type[f] != 1) return fail(MS_E_INVALID, "free body %d: bad type", f);
    if (!(sc->free_mass[f] > 0.f)) return fail(MS_E_INVALID, "free body %d: mass must be > 0", f);
    for (int t = 0; t < 3; ++t)
      if (!(sc->free_inertia[f * 3 + t] > 0.f)) return fail(MS_E_INVALID, "free body %d: inertia must be > 0", f);
  }
  if (c.NS > 0 && !sc->static_box) return fail(MS_E_INVALID, "static_box is null");
  if (c.NP > 0 && !sc->plane) return fail(MS_E_INVALID, "plane is null");
  if (c.NA > 0 && (!sc->aux_type || !sc->aux_rot || !sc->aux_pos || !sc->aux_axis || !sc->aux_box ||
                   !sc->aux_mass || !sc->aux_inertia || !sc->aux_limit))
    return fail(MS_E_INVALID, "aux arrays are null");
  for (int x = 0; x < c.NA; ++x)
    if (!(sc->aux_mass[x] > 0.f)) return fail(MS_E_INVALID, "aux joint %d: mass must be > 0", x);
  return MS_OK;
}

inline void quat_R(const float* q, float* R) {
  float w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}

struct ParamLayout {
  size_t models, scenes, free, statics, sgrid, planes, aux, order, free_off, aux_off, total;
  int sg_nw;  // 64-bit words per furniture grid cell
};

inline ParamLayout param_layout(const Counts& c) {
  ParamLayout p;
  size_t o = 0;
  p.models = o; o = align256(o + sizeof(DModel) * c.M);
  p.scenes = o; o = align256(o + sizeof(DScene) * c.S);
  p.free = o; o = align256(o + sizeof(DFree) * std::max(c.NF, 1));
  p.statics = o; o = align256(o + sizeof(float) * 6 * std::max(c.NS, 1));
  p.sg_nw = std::max((c.smax + 63) / 64, 1);
  p.sgrid = o; o = align256(o + sizeof(float) * (size_t)sgrid_floats(p.sg_nw) * c.S);
  p.planes = o; o = align256(o + sizeof(float4) * std::max(c.NP, 1));
  p.aux = o; o = align256(o + sizeof(DAux) * std::max(c.NA, 1));
  p.order = o; o = align256(o + sizeof(int) * c.S);
  p.free_off = o; o = align256(o + sizeof(int) * (c.S + 1));
  p.aux_off = o; o = align256(o + sizeof(int) * (c.S + 1));
  p.total = o;
  return p;
}

struct ScratchLayout {
  size_t queue, status, debug, cycles, act, actb, bwd_order, bwd_nover, bwd_slot, fwd_cost, fwd_order, fwd_maxc,
      fwd_nover, fwd_retry, total;
};
inline ScratchLayout scratch_layout(const Counts& c, int n_sub) {
  ScratchLayout s;
  size_t o = 0;
  s.queue = o; o = align256(o + 256);
  s.status = o; o = align256(o + sizeof(uint32_t) * c.S);
  s.debug = o; o = align256(o + sizeof(uint32_t) * 4 * (size_t)c.S * n_sub);
  s.cycles = o; o = align256(o + sizeof(unsigned long long) * 8 * (size_t)c.S);
  s.act = o; o = align256(o + sizeof(float) * 16 * (size_t)c.S);
  s.actb = o; o = align256(o + sizeof(float) * 16 * (size_t)c.S);
  s.bwd_order = o; o = align256(o + sizeof(int) * (size_t)c.S);
  s.bwd_nover = o; o = align256(o + 256);
  s.bwd_slot = o; o = align256(o + sizeof(int) * (size_t)c.S);
  s.fwd_cost = o; o = align256(o + sizeof(int) * (size_t)c.S);
  s.fwd_order = o; o = align256(o + sizeof(int) * (size_t)c.S);
  s.fwd_maxc = o; o = align256(o + sizeof(int) * (size_t)c.S);
  s.fwd_nover = o; o = align256(o + 256);
  s.fwd_retry = o; o = align256(o + sizeof(int) * (1 + (size_t)c.S));
  s.total = o;
  return s;
}

inline int lds_ccap(const ms_batch_desc* d) { return d->contact_cap; }

inline LdsLayout lds_for(const ms_batch_desc* d, const Counts& c, bool stage_static, bool force = false) {
  return make_layout(std::max(c.fmax, 1), c.smax, lds_ccap(d), std::max(d->robot_contact_cap, 1), stage_static ? 1 : 0,
                     force ? 1 : 0, std::max(c.nsph_max, 1));
}


// Pack the scene description into host (pl.total bytes, zero-filled); also
// returns the cost-sorted scene order in host.
inline void pack_params(const ms_scene_desc* sc, const Counts& c, const ParamLayout& pl, char* hostp) {
  struct HostView {
    char* p;
    char* data() { return p; }
  } host{hostp};
  // robot models
  DModel* models = reinterpret_cast<DModel*>(host.data() + pl.models);
  for (int m = 0; m < c.M; ++m) {
    DModel& M = models[m];
    M.nb = sc->model_nb[m];
    M.nsph = sc->model_nsph[m];
    for (int i = 0; i < ND; ++i) {
      int k = m * ND + i;
      M.parent[i] = i < M.nb ? sc->model_parent[k] : -1;
      M.jtype[i] = sc->model_jtype[k];
      M.veldof[i] = sc->model_veldof[k];
      int anc = 0;
      if (i < M.nb)
        for (int j = i; j >= 0; j = sc->model_parent[m * ND + j]) anc |= 1 << j;
      M.anc[i] = anc;
      for (int t = 0; t < 3; ++t) {
        M.axis[i][t] = sc->model_axis[k * 3 + t];
        M.xtp[i][t] = sc->model_xt_pos[k * 3 + t];
        M.com[i][t] = sc->model_com[k * 3 + t];
      }
      quat_R(sc->model_xt_rot + k * 4, M.xtR[i]);
      M.mass[i] = sc->model_mass[k];
      for (int t = 0; t < 6; ++t) M.Ic[i][t] = sc->model_inertia[k * 6 + t];
      M.kp[i] = sc->model_kp[k];
      M.kd[i] = sc->model_kd[k];
      M.arm[i] = sc->model_armature[k];
      M.damp[i] = sc->model_damping[k];
      M.act_kind[i] = sc->model_act_kind ? sc->model_act_kind[k] : 0;
      M.act_scale[i] = sc->model_act_scale ? sc->model_act_scale[k] : 0.f;
    }
    M.act_x = M.act_yaw = -1;
    for (int i = 0; i < M.nb; ++i) {
      if (M.act_kind[i] == MS_ACT_BASE_FWD_X) M.act_x = i;
      if (M.act_kind[i] == MS_ACT_BASE_YAW) M.act_yaw = i;
    }
    for (int k = 0; k < SPH; ++k) {
      const float* sp = sc->model_sph + (m * SPH + k) * 4;
      M.sph[k] = make_float4(sp[0], sp[1], sp[2], sp[3]);
      M.sph_body[k] = sc->model_sph_body[m * SPH + k];
      M.sph_flags[k] = sc->model_sph_flags[m * SPH + k];
    }
    // per-body sphere ranges and bounding spheres (centre = mean of the
    // sphere centres, radius = max distance + sphere radius)
    for (int i = 0; i < ND; ++i) {
      M.sph_first[i] = 0;
      M.sph_count[i] = 0;
      M.bsph[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    for (int k = M.nsph - 1; k >= 0; --k) {
      int bi = M.sph_body[k];
      M.sph_first[bi] = k;
      M.sph_count[bi] += 1;
    }
    for (int i = 0; i < M.nb; ++i) {
      if (M.sph_count[i] == 0) continue;
      double c[3] = {0, 0, 0};
      for (int k = M.sph_first[i]; k < M.sph_first[i] + M.sph_count[i]; ++k) {
        c[0] += M.sph[k].x; c[1] += M.sph[k].y; c[2] += M.sph[k].z;
      }
      for (int t = 0; t < 3; ++t) c[t] /= M.sph_count[i];
      double r = 0.0;
      for (int k = M.sph_first[i]; k < M.sph_first[i] + M.sph_count[i]; ++k) {
        double dx = M.sph[k].x - c[0], dy = M.sph[k].y - c[1], dz = M.sph[k].z - c[2];
        r = std::max(r, std::sqrt(dx * dx + dy * dy + dz * dz) + M.sph[k].w);
      }
      M.bsph[i] = make_float4((float)c[0], (float)c[1], (float)c[2], (float)r);
    }
  }
  DScene* scenes = reinterpret_cast<DScene*>(host.data() + pl.scenes);
  std::vector<std::pair<long, int>> cost(c.S);
  for (int s = 0; s < c.S; ++s) {
    DScene& S = scenes[s];
    S.model = sc->scene_model[s];
    S.f0 = sc->free_off[s]; S.nf = sc->free_off[s + 1] - S.f0;
    S.s0 = sc->static_off[s]; S.ns = sc->static_off[s + 1] - S.s0;
    S.p0 = sc->plane_off[s]; S.np = sc->plane_off[s + 1] - S.p0;
    S.a0 = sc->aux_off[s]; S.na = sc->aux_off[s + 1] - S.a0;
    int nown = 0;
    for (int f = 0; f < S.nf; ++f) nown += sc->free_type[S.f0 + f] == 0 ? 8 : 1;
    S.nown = nown;
    long nt = S.np + S.ns + S.na + S.nf;
    long owners = sc->model_nsph[S.model] + nown;
    S.cost = (int)std::min<long>(owners * nt, 1 << 30);
    for (int j = 0; j < ND; ++j) S.hold[j] = sc->scene_hold[s * ND + j];
    cost[s] = {-(long)S.cost, s};
  }
  DFree* fr = reinterpret_cast<DFree*>(host.data() + pl.free);
  for (int f = 0; f < c.NF; ++f) {
    fr[f].type = sc->free_type[f];
    for (int t = 0; t < 3; ++t) {
      fr[f].half[t] = sc->free_size[f * 3 + t];
      fr[f].Ib[t] = sc->free_inertia[f * 3 + t];
    }
    fr[f].mass = sc->free_mass[f];
  }
  if (c.NS > 0) std::memcpy(host.data() + pl.statics, sc->static_box, sizeof(float) * 6 * c.NS);
  // furniture grids (see KArgs::sgrid): cells over the xy extent of the
  // scene's boxes; a box goes into every cell its xy extent grown by 1 mm
  // overlaps (double arithmetic, so the float query on the device, which
  // grows its own extent by more, never misses one)
  for (int s = 0; s < c.S; ++s) {
    float* g = reinterpret_cast<float*>(host.data() + pl.sgrid) + (size_t)sgrid_floats(pl.sg_nw) * s;
    const int s0 = sc->static_off[s], ns = sc->static_off[s + 1] - s0;
    double lo[2] = {0.0, 0.0}, hi[2] = {1.0, 1.0};
    for (int i = 0; i < ns; ++i)
      for (int d = 0; d < 2; ++d) {
        const double a = (double)sc->static_box[(s0 + i) * 6 + d] - sc->static_box[(s0 + i) * 6 + 3 + d];
        const double b = (double)sc->static_box[(s0 + i) * 6 + d] + sc->static_box[(s0 + i) * 6 + 3 + d];
        lo[d] = i == 0 ? a : std::min(lo[d], a);
        hi[d] = i == 0 ? b : std::max(hi[d], b);
      }
    double inv[2];
    for (int d = 0; d < 2; ++d) inv[d] = SGRID / std::max(hi[d] - lo[d], 1e-3);
    g[0] = (float)lo[0];
    g[1] = (float)lo[1];
    g[2] = (float)inv[0];
    g[3] = (float)inv[1];
    uint64_t* cells = reinterpret_cast<uint64_t*>(g + 4);
    for (int i = 0; i < ns; ++i) {
      int c0[2], c1[2];
      for (int d = 0; d < 2; ++d) {
        const double ctr = sc->static_box[(s0 + i) * 6 + d], half = sc->static_box[(s0 + i) * 6 + 3 + d];
        c0[d] = std::max(0, std::min(SGRID - 1, (int)std::floor((ctr - half - 1e-3 - lo[d]) * inv[d])));
        c1[d] = std::max(0, std::min(SGRID - 1, (int)std::floor((ctr + half + 1e-3 - lo[d]) * inv[d])));
      }
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int x = c0[0]; x <= c1[0]; ++x) cells[(y * SGRID + x) * pl.sg_nw + i / 64] |= 1ull << (i % 64);
    }
  }
  if (c.NP > 0) std::memcpy(host.data() + pl.planes, sc->plane, sizeof(float) * 4 * c.NP);
  DAux* ax = reinterpret_cast<DAux*>(host.data() + pl.aux);
  for (int x = 0; x < c.NA; ++x) {
    ax[x].type = sc->aux_type[x];
    quat_R(sc->aux_rot + x * 4, ax[x].R0);
    for (int t = 0; t < 3; ++t) {
      ax[x].p0[t] = sc->aux_pos[x * 3 + t];
      ax[x].axis[t] = sc->aux_axis[x * 3 + t];
      ax[x].bc[t] = sc->aux_box[x * 6 + t];
      ax[x].bh[t] = sc->aux_box[x * 6 + 3 + t];
      ax[x].Ib[t] = sc->aux_inertia[x * 3 + t];
    }
    ax[x].mass = sc->aux_mass[x];
    ax[x].lo = sc->aux_limit[x * 2];
    ax[x].hi = sc->aux_limit[x * 2 + 1];
    ax[x].has_limit = ax[x].lo <= ax[x].hi ? 1 : 0;
  }
  // scene order: most expensive first (stable), so the tail of the launch holds small scenes
  std::stable_sort(cost.begin(), cost.end());
  int* order = reinterpret_cast<int*>(host.data() + pl.order);
  for (int s = 0; s < c.S; ++s) order[s] = cost[s].second;
  std::memcpy(host.data() + pl.free_off, sc->free_off, sizeof(int) * (c.S + 1));
  std::memcpy(host.data() + pl.aux_off, sc->aux_off, sizeof(int) * (c.S + 1));

}

}  // namespace mspack
