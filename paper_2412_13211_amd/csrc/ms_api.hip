// ms_api.hip -- host side of the C ABI declared in include/ms_phys.h.
//
// Validates and packs the scene description into the caller's params buffer,
// owns the schedule (grid shape, persistent queue, per-substep launches, LDS
// staging of furniture boxes), captures a control step as a hipGraph and
// replays it, and times the candidate schedules (autotuner).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ms_phys.h"
#include "ms_internal.h"

using namespace msk;

namespace {

thread_local std::string g_err;

ms_status fail(ms_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(MS_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Counts {
  int S, M, NF, NS, NP, NA;
  int fmax, smax, pmax, amax;
};

ms_status validate(const ms_batch_desc* d, const ms_scene_desc* sc, Counts& c) {
  if (!d || !sc) return fail(MS_E_INVALID, "null desc or scene description");
  if (d->n_scenes <= 0) return fail(MS_E_INVALID, "n_scenes must be positive (got %d)", d->n_scenes);
  if (d->n_substeps <= 0 || d->n_substeps > 1000) return fail(MS_E_INVALID, "n_substeps out of range");
  if (d->pgs_iters < 0 || d->pgs_iters > 1000) return fail(MS_E_INVALID, "pgs_iters out of range");
  if (d->control_mode < 0 || d->control_mode > 2) return fail(MS_E_INVALID, "unknown control_mode %d", d->control_mode);
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
  if (c.M <= 0) return fail(MS_E_INVALID, "n_models must be positive");
  for (int m = 0; m < c.M; ++m) {
    int nb = sc->model_nb[m], ns = sc->model_nsph[m];
    if (nb < 0 || nb > ND) return fail(MS_E_INVALID, "model %d: %d bodies (max %d)", m, nb, ND);
    if (ns < 0 || ns > SPH) return fail(MS_E_INVALID, "model %d: %d spheres (max %d)", m, ns, SPH);
    for (int i = 0; i < nb; ++i) {
      int p = sc->model_parent[m * ND + i];
      if (p >= i || p < -1) return fail(MS_E_INVALID, "model %d body %d: parent %d must precede it", m, i, p);
      int jt = sc->model_jtype[m * ND + i];
      if (jt != 0 && jt != 1) return fail(MS_E_INVALID, "model %d body %d: joint type %d", m, i, jt);
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

void quat_R(const float* q, float* R) {
  float w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}

struct ParamLayout {
  size_t models, scenes, free, statics, planes, aux, order, free_off, aux_off, total;
};

ParamLayout param_layout(const Counts& c) {
  ParamLayout p;
  size_t o = 0;
  p.models = o; o = align256(o + sizeof(DModel) * c.M);
  p.scenes = o; o = align256(o + sizeof(DScene) * c.S);
  p.free = o; o = align256(o + sizeof(DFree) * std::max(c.NF, 1));
  p.statics = o; o = align256(o + sizeof(float) * 6 * std::max(c.NS, 1));
  p.planes = o; o = align256(o + sizeof(float4) * std::max(c.NP, 1));
  p.aux = o; o = align256(o + sizeof(DAux) * std::max(c.NA, 1));
  p.order = o; o = align256(o + sizeof(int) * c.S);
  p.free_off = o; o = align256(o + sizeof(int) * (c.S + 1));
  p.aux_off = o; o = align256(o + sizeof(int) * (c.S + 1));
  p.total = o;
  return p;
}

struct ScratchLayout {
  size_t queue, status, debug, cycles, total;
};
ScratchLayout scratch_layout(const Counts& c, int n_sub) {
  ScratchLayout s;
  size_t o = 0;
  s.queue = o; o = align256(o + 256);
  s.status = o; o = align256(o + sizeof(uint32_t) * c.S);
  s.debug = o; o = align256(o + sizeof(uint32_t) * 4 * (size_t)c.S * n_sub);
  s.cycles = o; o = align256(o + sizeof(unsigned long long) * 8 * (size_t)c.S);
  s.total = o;
  return s;
}

int lds_ccap(const ms_batch_desc* d) { return d->contact_cap; }

LdsLayout lds_for(const ms_batch_desc* d, const Counts& c, bool stage_static) {
  return make_layout(std::max(c.fmax, 1), c.smax, lds_ccap(d), std::max(d->robot_contact_cap, 1), stage_static ? 1 : 0);
}

}  // namespace

struct ms_batch {
  ms_batch_desc desc;
  Counts cnt;
  ParamLayout pl;
  ScratchLayout sl;
  char* params;
  char* scratch;
  char* tape;
  int device;
  int n_cu;
  size_t max_lds;
  std::vector<int32_t> free_off, aux_off;
  ms_schedule sched;
  bool debug_on;
  bool profile_on;
  hipStream_t cap_stream;
  // graphs keyed by (x_in, u, x_out)
  std::map<std::tuple<const void*, const void*, void*>, hipGraphExec_t> graphs;
  std::map<std::tuple<const void*, const void*, void*>, hipGraph_t> graph_defs;
};

namespace {

void drop_graphs(ms_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : b->graph_defs) (void)hipGraphDestroy(kv.second);
  b->graphs.clear();
  b->graph_defs.clear();
}

KArgs make_args(const ms_batch* b, const void* x_in, const float* u, void* x_out) {
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.models = reinterpret_cast<const DModel*>(b->params + b->pl.models);
  a.scenes = reinterpret_cast<const DScene*>(b->params + b->pl.scenes);
  a.free = reinterpret_cast<const DFree*>(b->params + b->pl.free);
  a.statics = reinterpret_cast<const float*>(b->params + b->pl.statics);
  a.planes = reinterpret_cast<const float4*>(b->params + b->pl.planes);
  a.aux = reinterpret_cast<const DAux*>(b->params + b->pl.aux);
  a.order = reinterpret_cast<const int*>(b->params + b->pl.order);
  a.x_in = static_cast<const float*>(x_in);
  a.x_out = static_cast<float*>(x_out);
  a.u = u;
  a.status = reinterpret_cast<uint32_t*>(b->scratch + b->sl.status);
  a.debug = b->debug_on ? reinterpret_cast<uint32_t*>(b->scratch + b->sl.debug) : nullptr;
  a.phase_cycles = b->profile_on ? reinterpret_cast<unsigned long long*>(b->scratch + b->sl.cycles) : nullptr;
  a.queue = reinterpret_cast<int*>(b->scratch + b->sl.queue);
  a.S = b->cnt.S;
  a.NF = b->cnt.NF;
  a.NA = b->cnt.NA;
  a.n_sub = b->desc.n_substeps;
  a.sub0 = 0;
  a.n_sub_total = b->desc.n_substeps;
  a.K = b->desc.pgs_iters;
  a.mode = b->desc.control_mode;
  a.ccap = b->desc.contact_cap;
  a.rcap = b->desc.robot_contact_cap;
  a.stage_static = (b->sched.flags & MS_SCHED_STAGE_STATIC) ? 1 : 0;
  a.cull = (b->sched.flags & MS_SCHED_CULL) ? 1 : 0;
  a.persistent = (b->sched.flags & MS_SCHED_PERSISTENT) ? 1 : 0;
  a.h = b->desc.h;
  a.mu = b->desc.mu;
  a.beta = b->desc.baumgarte;
  a.margin = b->desc.margin;
  for (int t = 0; t < 3; ++t) a.g[t] = b->desc.gravity[t];
  a.L = lds_for(&b->desc, b->cnt, a.stage_static);
  return a;
}

size_t lds_bytes_of(const KArgs& a) { return (size_t)a.L.total * sizeof(float); }

int persistent_grid(const ms_batch* b, size_t lds) {
  if (b->sched.grid > 0) return b->sched.grid;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, step_kernel_ptr(), WAVE, lds) != hipSuccess || per_cu <= 0)
    per_cu = 1;
  return std::min(b->cnt.S, per_cu * b->n_cu);
}

// Enqueue one control step with the current schedule (no graph).
ms_status enqueue_step(ms_batch* b, const void* x_in, const float* u, void* x_out, hipStream_t st) {
  KArgs a = make_args(b, x_in, u, x_out);
  size_t lds = lds_bytes_of(a);
  if (lds > b->max_lds)
    return fail(MS_E_UNSUPPORTED, "scene working set needs %zu B of LDS (device limit %zu B); lower contact_cap "
                "or robot_contact_cap or disable furniture staging", lds, b->max_lds);
  const bool per_sub = (b->sched.flags & MS_SCHED_PER_SUBSTEP) != 0;
  const int launches = per_sub ? b->desc.n_substeps : 1;
  for (int k = 0; k < launches; ++k) {
    KArgs ak = a;
    if (per_sub) {
      ak.n_sub = 1;
      ak.sub0 = k;
      if (k > 0) ak.x_in = ak.x_out;
    }
    int grid = b->cnt.S;
    if (ak.persistent) {
      launch_reset_queue(ak.queue, st);
      grid = persistent_grid(b, lds);
    }
    launch_step(ak, grid, lds, st);
    HIP_TRY(hipGetLastError());
  }
  return MS_OK;
}

}  // namespace

extern "C" {

const char* ms_last_error(void) { return g_err.c_str(); }

ms_status ms_state_floats(const ms_scene_desc* sc, int32_t n_scenes, size_t* out) {
  if (!sc || !out || n_scenes <= 0 || !sc->free_off || !sc->aux_off) return fail(MS_E_INVALID, "bad arguments");
  *out = (size_t)n_scenes * 32 + (size_t)sc->free_off[n_scenes] * 16 + (size_t)sc->aux_off[n_scenes] * 4;
  return MS_OK;
}

ms_status ms_query_sizes(const ms_batch_desc* d, const ms_scene_desc* sc, ms_sizes* out) {
  if (!out) return fail(MS_E_INVALID, "null output");
  Counts c;
  ms_status st = validate(d, sc, c);
  if (st != MS_OK) return st;
  out->params = param_layout(c).total;
  out->state = ((size_t)c.S * 32 + (size_t)c.NF * 16 + (size_t)c.NA * 4) * sizeof(float);
  out->scratch = scratch_layout(c, d->n_substeps).total;
  out->tape = 0;
  out->lds = (size_t)lds_for(d, c, true).total * sizeof(float);
  return MS_OK;
}

ms_status ms_create_batch(const ms_batch_desc* d, const ms_scene_desc* sc, void* params_dev, void* scratch_dev,
                          void* tape_dev, void* hip_stream, ms_batch** out) {
  if (!out) return fail(MS_E_INVALID, "null output");
  *out = nullptr;
  Counts c;
  ms_status st = validate(d, sc, c);
  if (st != MS_OK) return st;
  if (!params_dev || !scratch_dev) return fail(MS_E_INVALID, "params_dev and scratch_dev are required");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(MS_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
  ParamLayout pl = param_layout(c);
  std::vector<char> host(pl.total, 0);
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

  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  HIP_TRY(hipMemcpyAsync(params_dev, host.data(), pl.total, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));

  ms_batch* b = new ms_batch();
  b->desc = *d;
  b->cnt = c;
  b->pl = pl;
  b->sl = scratch_layout(c, d->n_substeps);
  b->params = static_cast<char*>(params_dev);
  b->scratch = static_cast<char*>(scratch_dev);
  b->tape = static_cast<char*>(tape_dev);
  b->device = dev;
  b->n_cu = prop.multiProcessorCount;
  b->max_lds = prop.sharedMemPerBlock;
  size_t opt = 0;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && v > 0) opt = v;
  b->max_lds = std::max(b->max_lds, opt);
  b->free_off.assign(sc->free_off, sc->free_off + c.S + 1);
  b->aux_off.assign(sc->aux_off, sc->aux_off + c.S + 1);
  b->sched.flags = MS_SCHED_STAGE_STATIC | MS_SCHED_CULL;
  b->sched.grid = 0;
  b->debug_on = false;
  b->profile_on = false;
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return fail(MS_E_HIP, "hipStreamCreateWithFlags failed");
  }
  // allow the kernel the whole LDS of a workgroup
  (void)hipFuncSetAttribute(step_kernel_ptr(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->max_lds);
  // status starts at zero
  hipError_t e = hipMemsetAsync(b->scratch + b->sl.status, 0, sizeof(uint32_t) * c.S, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return fail(MS_E_HIP, "status init: %s", hipGetErrorString(e));
  }
  *out = b;
  return MS_OK;
}

ms_status ms_destroy_batch(ms_batch* b) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  drop_graphs(b);
  (void)hipStreamDestroy(b->cap_stream);
  delete b;
  return MS_OK;
}

ms_status ms_set_schedule(ms_batch* b, const ms_schedule* s) {
  if (!b || !s) return fail(MS_E_INVALID, "null argument");
  const int known = MS_SCHED_PERSISTENT | MS_SCHED_GRAPH | MS_SCHED_PER_SUBSTEP | MS_SCHED_STAGE_STATIC | MS_SCHED_CULL;
  if (s->flags & ~known) return fail(MS_E_INVALID, "unknown schedule flags 0x%x", s->flags);
  if (s->grid < 0) return fail(MS_E_INVALID, "grid must be >= 0");
  KArgs a = make_args(b, nullptr, nullptr, nullptr);
  a.L = lds_for(&b->desc, b->cnt, (s->flags & MS_SCHED_STAGE_STATIC) != 0);
  if (lds_bytes_of(a) > b->max_lds)
    return fail(MS_E_UNSUPPORTED, "schedule needs %zu B of LDS per scene (limit %zu)", lds_bytes_of(a), b->max_lds);
  drop_graphs(b);
  b->sched = *s;
  return MS_OK;
}

ms_status ms_get_schedule(const ms_batch* b, ms_schedule* out) {
  if (!b || !out) return fail(MS_E_INVALID, "null argument");
  *out = b->sched;
  return MS_OK;
}

ms_status ms_enable_debug(ms_batch* b, int32_t on) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if ((bool)on != b->debug_on) drop_graphs(b);
  b->debug_on = on != 0;
  return MS_OK;
}

ms_status ms_step(ms_batch* b, const void* x_in, const float* u, void* x_out, void* hip_stream) {
  if (!b || !x_in || !u || !x_out) return fail(MS_E_INVALID, "null batch, state or controls");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (!(b->sched.flags & MS_SCHED_GRAPH)) return enqueue_step(b, x_in, u, x_out, st);
  auto key = std::make_tuple(x_in, static_cast<const void*>(u), x_out);
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    if (b->graphs.size() >= 8) drop_graphs(b);
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    ms_status rs = enqueue_step(b, x_in, u, x_out, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rs != MS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rs;
    }
    if (e != hipSuccess) return fail(MS_E_HIP, "graph capture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(MS_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    b->graph_defs[key] = g;
    it = b->graphs.emplace(key, ex).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, st));
  return MS_OK;
}

ms_status ms_step_backward(ms_batch* b, const void* x_in, const float* u, const void* gx_out, void* gx_in,
                           float* gu, void* hip_stream) {
  (void)x_in; (void)u; (void)gx_out; (void)gx_in; (void)gu; (void)hip_stream;
  if (!b) return fail(MS_E_INVALID, "null batch");
  return fail(MS_E_UNSUPPORTED, "ms_step_backward: adjoint kernels not built into this library");
}

ms_status ms_get_state(const ms_batch* b, const void* x, ms_state_view* out) {
  if (!b || !x || !out) return fail(MS_E_INVALID, "null argument");
  float* base = const_cast<float*>(static_cast<const float*>(x));
  const int S = b->cnt.S;
  out->q = base;
  out->qd = base + (size_t)S * ND;
  out->free_body = base + (size_t)S * 2 * ND;
  out->aux = base + (size_t)S * 2 * ND + (size_t)b->cnt.NF * 16;
  out->free_off_host = b->free_off.data();
  out->aux_off_host = b->aux_off.data();
  out->n_scenes = S;
  out->n_free = b->cnt.NF;
  out->n_aux = b->cnt.NA;
  return MS_OK;
}

ms_status ms_set_state(ms_batch* b, void* x, const void* src, const uint8_t* mask, void* hip_stream) {
  if (!b || !x || !src) return fail(MS_E_INVALID, "null argument");
  launch_masked_copy(static_cast<float*>(x), static_cast<const float*>(src), mask, b->cnt.S, b->cnt.NF, b->cnt.NA,
                     reinterpret_cast<const int*>(b->params + b->pl.free_off),
                     reinterpret_cast<const int*>(b->params + b->pl.aux_off), static_cast<hipStream_t>(hip_stream));
  HIP_TRY(hipGetLastError());
  return MS_OK;
}

ms_status ms_scene_status(const ms_batch* b, uint32_t* out) {
  if (!b || !out) return fail(MS_E_INVALID, "null argument");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out, b->scratch + b->sl.status, sizeof(uint32_t) * b->cnt.S, hipMemcpyDeviceToHost));
  for (int s = 0; s < b->cnt.S; ++s)
    if (out[s] & (MS_ST_NONFINITE | MS_ST_DEGENERATE)) return MS_E_NUMERIC;
  return MS_OK;
}

ms_status ms_enable_phase_profile(ms_batch* b, int32_t on) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if ((bool)on != b->profile_on) drop_graphs(b);
  b->profile_on = on != 0;
  return MS_OK;
}

ms_status ms_phase_cycles(const ms_batch* b, unsigned long long* out) {
  if (!b || !out) return fail(MS_E_INVALID, "null argument");
  if (!b->profile_on) return fail(MS_E_STATE, "phase profile is off (ms_enable_phase_profile)");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out, b->scratch + b->sl.cycles, sizeof(unsigned long long) * 8 * (size_t)b->cnt.S,
                    hipMemcpyDeviceToHost));
  return MS_OK;
}

ms_status ms_debug_contacts(const ms_batch* b, uint32_t* out) {
  if (!b || !out) return fail(MS_E_INVALID, "null argument");
  if (!b->debug_on) return fail(MS_E_STATE, "debug output is off (ms_enable_debug)");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out, b->scratch + b->sl.debug, sizeof(uint32_t) * 4 * (size_t)b->cnt.S * b->desc.n_substeps,
                    hipMemcpyDeviceToHost));
  return MS_OK;
}

ms_status ms_autotune(ms_batch* b, const void* x, const float* u, void* tmp, int32_t reps, void* hip_stream,
                      ms_schedule* chosen, float* ms_per_step) {
  if (!b || !x || !u || !tmp) return fail(MS_E_INVALID, "null argument");
  if (reps <= 0) reps = 5;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const ms_schedule saved = b->sched;
  const int base_flags[] = {MS_SCHED_GRAPH | MS_SCHED_CULL, MS_SCHED_GRAPH | MS_SCHED_PERSISTENT | MS_SCHED_CULL};
  const int stage_opts[] = {MS_SCHED_STAGE_STATIC, 0};
  ms_schedule best = saved;
  float best_ms = 1e30f;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  size_t bytes = ((size_t)b->cnt.S * 32 + (size_t)b->cnt.NF * 16 + (size_t)b->cnt.NA * 4) * sizeof(float);
  for (int bf : base_flags)
    for (int so : stage_opts) {
      ms_schedule s{bf | so, 0};
      if (ms_set_schedule(b, &s) != MS_OK) continue;
      if (hipMemcpyAsync(tmp, x, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) continue;
      if (ms_step(b, tmp, u, tmp, st) != MS_OK) continue;  // warm-up (and capture)
      (void)hipEventRecord(e0, st);
      bool ok = true;
      for (int r = 0; r < reps && ok; ++r) ok = ms_step(b, tmp, u, tmp, st) == MS_OK;
      (void)hipEventRecord(e1, st);
      if (!ok || hipEventSynchronize(e1) != hipSuccess) continue;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      if (ms < best_ms) {
        best_ms = ms;
        best = s;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ms_status rs = ms_set_schedule(b, best_ms < 1e29f ? &best : &saved);
  if (chosen) *chosen = b->sched;
  if (ms_per_step) *ms_per_step = best_ms;
  return rs;
}

}  // extern "C"
