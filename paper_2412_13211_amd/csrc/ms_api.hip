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
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ms_phys.h"
#include "ms_internal.h"
#include "ms_pack.h"
#include "ms_backward.h"
#include "ms_tasks.h"

using namespace msk;

using namespace mspack;

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(MS_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

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
  float* frc_robot;
  float* frc_body;
  std::vector<int> model_nb;
  bool task_robot_set;
  ms_task_robot task_robot;
  float* grip;
  hipStream_t cap_stream;
  // split adjoint launches: contact caps of the smaller LDS layout (0: no
  // split), the stream of the full-size launch and the fork / join events
  int split_c, split_r;
  // the forward's smaller layout: contact cap per (furniture staging, force
  // outputs), -1 until computed, 0 for none; a forced cap (>= 0) or -1
  int fsplit[2][2];
  int fsplit_force;
  hipStream_t bwd_stream;
  hipEvent_t ev_fork, ev_join;
  // graphs keyed by (x_in, u, x_out)
  std::map<std::tuple<const void*, const void*, void*>, hipGraphExec_t> graphs;
  std::map<std::tuple<const void*, const void*, void*>, hipGraph_t> graph_defs;
  // autotuner: device architecture (e.g. gfx950), cache file ("" = none),
  // whether the last ms_autotune / ms_autotune_backward took its choice from it
  std::string arch;
  std::string tune_cache;
  bool fwd_from_cache, bwd_from_cache;
};

namespace {

void release_handles(ms_batch* b) {
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->bwd_stream) (void)hipStreamDestroy(b->bwd_stream);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
}

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
  a.sgrid = reinterpret_cast<const float*>(b->params + b->pl.sgrid);
  a.sg_nw = b->pl.sg_nw;
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
  a.L = lds_for(&b->desc, b->cnt, a.stage_static, b->frc_robot != nullptr || b->grip != nullptr);
  a.frc_robot = b->frc_robot;
  a.frc_body = b->frc_body;
  a.grip = b->grip;
  a.grip_ee = b->task_robot.ee_bodies;
  a.grip_fl = b->task_robot.finger_l;
  a.grip_fr = b->task_robot.finger_r;
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

// MS_CTRL_ACTIONS: the PD targets of the control step (in scratch), computed
// from the actions and the step's start state; other modes pass u through.
const float* control_targets(ms_batch* b, const void* x_in, const float* u, hipStream_t st) {
  if (b->desc.control_mode != MS_CTRL_ACTIONS) return u;
  float* tgt = reinterpret_cast<float*>(b->scratch + b->sl.act);
  launch_actions(reinterpret_cast<const DModel*>(b->params + b->pl.models),
                 reinterpret_cast<const DScene*>(b->params + b->pl.scenes), static_cast<const float*>(x_in), u, tgt,
                 b->cnt.S, st);
  return tgt;
}
int step_mode(const ms_batch* b) { return b->desc.control_mode == MS_CTRL_ACTIONS ? MS_CTRL_PD : b->desc.control_mode; }

// robot contacts of the forward's smaller layout: the batch's cap.  (A lower
// one saves 192 B of LDS per robot contact, but a scene whose robot contacts
// jump past it within a step is retried after the join, adding about one
// scene's step time to the control step.)
int fwd_split_rcap(const ms_batch* b) { return std::max(b->desc.robot_contact_cap, 1); }

// Enqueue one control step with the current schedule (no graph).
// the order of a step's scenes: by the scene times the previous step wrote
// (a counting sort that also zeroes the work counters), the scenes routed to
// the full layout first when fit_c > 0; or the static order
void set_step_order(ms_batch* b, KArgs& a, hipStream_t st, int fit_c) {
  a.cost = reinterpret_cast<int*>(b->scratch + b->sl.fwd_cost);
  a.maxc = reinterpret_cast<int*>(b->scratch + b->sl.fwd_maxc);
  if (b->sched.flags & MS_SCHED_STATIC_ORDER) {
    if (a.persistent) launch_reset_queue(a.queue, st);
    return;
  }
  int* ord = reinterpret_cast<int*>(b->scratch + b->sl.fwd_order);
  a.n_over = reinterpret_cast<int*>(b->scratch + b->sl.fwd_nover);
  a.retry = reinterpret_cast<int*>(b->scratch + b->sl.fwd_retry);
  launch_cost_order(a.cost, a.maxc, b->cnt.S, fit_c, fwd_split_rcap(b), ord,
                    const_cast<int*>(a.n_over), a.persistent ? a.queue : nullptr, a.retry, st);
  a.order = ord;
}

// Workgroups of the forward kernel per CU at an LDS size (the occupancy
// query, capped by the measured LDS rule of bwd_per_cu)
int fwd_per_cu(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel_ptr(), WAVE, lds) != hipSuccess) n = 0;
  return std::min(n, (int)(size_t{163840} / (lds + 1024)));
}

// rc < 0: the batch's robot contact cap
LdsLayout fwd_layout(const ms_batch* b, int cc, int stage, int force, int rc = -1) {
  const Counts& c = b->cnt;
  return make_layout(std::max(c.fmax, 1), c.smax, cc, rc < 0 ? std::max(b->desc.robot_contact_cap, 1) : rc, stage,
                     force, std::max(c.nsph_max, 1));
}


// Contact cap of the forward's smaller layout: among the caps from 3/4 of the
// batch's up, the largest one of the highest workgroups-per-CU count above the
// full layout's, 0 for none.  Scenes whose last contact counts leave room
// under it run in it; a scene that overflows it anyway is stepped again in
// the full layout.  (The autotuner also tries the lower caps down to half.)
int fwd_split_cap(ms_batch* b, int stage, int force) {
  if (b->fsplit_force >= 0) return b->fsplit_force;
  int& v = b->fsplit[stage][force];
  if (v >= 0) return v;
  v = 0;
  const int cap = b->desc.contact_cap;
  const size_t full = (size_t)fwd_layout(b, cap, stage, force).total * sizeof(float);
  const int occ = fwd_per_cu(full);
  if (occ <= 0) return v;
  int best = occ;
  for (int k = cap - 1; k >= std::max((3 * cap) / 4, 1); --k) {
    const int o = fwd_per_cu((size_t)fwd_layout(b, k, stage, force, fwd_split_rcap(b)).total * sizeof(float));
    if (o > best) {
      best = o;
      v = k;
    }
  }
  return v;
}

// One fused launch of a control step (persistent or not), or the split form:
// the scenes routed to the full layout on st (a grid of one per CU looping
// over them), the others in the smaller layout on the second stream after a
// 15 us wait (as in the adjoint's split), joined back; then a retry launch
// for the scenes that overflowed the smaller layout.  Not while st is being
// captured: a replayed graph runs the two branches one after the other.
ms_status launch_fused(ms_batch* b, KArgs& a, size_t lds, hipStream_t st) {
  const int force = (b->frc_robot != nullptr || b->grip != nullptr) ? 1 : 0;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(st, &cap));
  const int fc = (a.persistent && cap == hipStreamCaptureStatusNone &&
                  !(b->sched.flags & (MS_SCHED_STATIC_ORDER | MS_SCHED_FWD_ONE_LAUNCH)))
                     ? fwd_split_cap(b, a.stage_static, force)
                     : 0;
  set_step_order(b, a, st, fc);
  HIP_TRY(hipGetLastError());
  if (fc <= 0) {
    launch_step(a, a.persistent ? persistent_grid(b, lds) : b->cnt.S, lds, st);
    HIP_TRY(hipGetLastError());
    return MS_OK;
  }
  KArgs big = a, small = a, rt = a;
  big.fit_mode = 2;
  small.fit_mode = 1;
  small.L = fwd_layout(b, fc, a.stage_static, force, fwd_split_rcap(b));
  small.rcap = std::min(a.rcap, small.L.rcap);  // a scene with more robot contacts gives up (status 8) and is retried
  rt.fit_mode = 3;
  const size_t lds_s = lds_bytes_of(small);
  HIP_TRY(hipEventRecord(b->ev_fork, st));
  HIP_TRY(hipStreamWaitEvent(b->bwd_stream, b->ev_fork, 0));
  launch_step(big, std::min(b->cnt.S, b->n_cu), lds, st);
  HIP_TRY(hipGetLastError());
  launch_delay(1500, b->bwd_stream);
  launch_step(small, persistent_grid(b, lds_s), lds_s, b->bwd_stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(b->ev_join, b->bwd_stream));
  HIP_TRY(hipStreamWaitEvent(st, b->ev_join, 0));
  launch_step(rt, std::min(b->cnt.S, b->n_cu), lds, st);
  HIP_TRY(hipGetLastError());
  return MS_OK;
}

ms_status enqueue_step(ms_batch* b, const void* x_in, const float* u, void* x_out, hipStream_t st) {
  u = control_targets(b, x_in, u, st);
  HIP_TRY(hipGetLastError());
  KArgs a = make_args(b, x_in, u, x_out);
  a.mode = step_mode(b);
  size_t lds = lds_bytes_of(a);
  if (lds > b->max_lds)
    return fail(MS_E_UNSUPPORTED, "scene working set needs %zu B of LDS (device limit %zu B); lower contact_cap "
                "or robot_contact_cap or disable furniture staging", lds, b->max_lds);
  const bool per_sub = (b->sched.flags & MS_SCHED_PER_SUBSTEP) != 0;
  if (!per_sub) return launch_fused(b, a, lds, st);
  const int launches = b->desc.n_substeps;
  set_step_order(b, a, st, 0);
  HIP_TRY(hipGetLastError());
  for (int k = 0; k < launches; ++k) {
    KArgs ak = a;
    if (per_sub) {
      ak.n_sub = 1;
      ak.sub0 = k;
      if (k > 0) ak.x_in = ak.x_out;
    }
    int grid = b->cnt.S;
    if (ak.persistent) {
      if (k > 0) launch_reset_queue(ak.queue, st);
      grid = persistent_grid(b, lds);
    }
    launch_step(ak, grid, lds, st);
    HIP_TRY(hipGetLastError());
  }
  return MS_OK;
}

msa::WS bwd_ws(const ms_batch_desc* d, const Counts& c) {
  const int ntmax = c.pmax + c.smax + c.amax + std::max(c.fmax, 1);
  return msa::ws_layout(std::max(c.fmax, 1), ntmax, d->contact_cap, std::max(d->robot_contact_cap, 1), d->pgs_iters,
                    d->n_substeps);
}

// LDS block of the wavefront adjoint kernel, for the batch's contact caps or
// for smaller ones (cc contacts, rc robot contacts)
msa::WS bwd_ws_wave(const ms_batch_desc* d, const Counts& c, int cc = -1, int rc = -1) {
  const int ntmax = c.pmax + c.smax + c.amax + std::max(c.fmax, 1);
  return msa::ws_layout(std::max(c.fmax, 1), ntmax, cc < 0 ? d->contact_cap : cc,
                        rc < 0 ? std::max(d->robot_contact_cap, 1) : rc, d->pgs_iters, d->n_substeps, true);
}

// Workgroups of the wavefront adjoint per CU at an LDS size.  Near the
// thresholds gfx950 fits fewer single-wave workgroups than the occupancy
// query reports (timed: three fit at 53760 B but not at 53768 B, five at
// 32000 B but not at 32064 B, while the query allows 54528 B and 32768 B);
// n workgroups are counted as fitting only when n (size + 1 KiB) stays
// within the CU's 160 KiB, which stays below every measured threshold.
int bwd_per_cu(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_bwd_wave_ptr(), 64, lds) != hipSuccess) n = 0;
  const int by_size = (int)(size_t{163840} / (lds + 1024));
  return std::min(n, by_size);
}

// Contact caps of a second, smaller LDS layout of the wavefront adjoint that
// fits more workgroups per CU: at most 8 robot contacts and the largest
// contact count (not below half the batch's cap) that raises the occupancy.
// Scenes whose lists fit it run at that occupancy; the rest run beside them
// in a launch sized for the batch's caps.  0, 0 when no such layout exists.
void choose_bwd_split(const ms_batch* b, int& cc, int& rc) {
  cc = rc = 0;
  const ms_batch_desc* d = &b->desc;
  const size_t full = (size_t)bwd_ws_wave(d, b->cnt).total * sizeof(float);
  if (full > b->max_lds) return;
  const int occ = bwd_per_cu(full);
  if (occ <= 0) return;
  const int r = std::min(std::max(d->robot_contact_cap, 1), 8);
  for (int k = d->contact_cap; k >= std::max(d->contact_cap / 2, 1); --k) {
    if (k == d->contact_cap && r == std::max(d->robot_contact_cap, 1)) continue;
    if (bwd_per_cu((size_t)bwd_ws_wave(d, b->cnt, k, r).total * sizeof(float)) > occ) {
      cc = k;
      rc = r;
      return;
    }
  }
}

// record of a control step written by the forward kernel for the wavefront adjoint kernel
RecLayout bwd_rec(const ms_batch_desc* d, const Counts& c) {
  return rec_layout(std::max(c.fmax, 1), d->contact_cap, d->pgs_iters, d->n_substeps);
}

// the tape buffer holds either the record (wavefront kernel) or the
// interleaved workspace of the lane kernel
size_t bwd_bytes(const ms_batch_desc* d, const Counts& c) {
  size_t lane = (size_t)bwd_ws(d, c).total * (size_t)bwd_stride(c.S) * sizeof(float);
  size_t rec = (size_t)bwd_rec(d, c).total * (size_t)c.S * sizeof(float);
  return std::max(lane, rec);
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
  out->tape = bwd_bytes(d, c);
  out->lds = (size_t)lds_for(d, c, true).total * sizeof(float);
  out->record = (size_t)bwd_rec(d, c).total * (size_t)c.S * sizeof(float);
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
  pack_params(sc, c, pl, host.data());
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
  b->frc_robot = nullptr;
  b->frc_body = nullptr;
  b->model_nb.assign(sc->model_nb, sc->model_nb + c.M);
  b->task_robot_set = false;
  std::memset(&b->task_robot, 0, sizeof b->task_robot);
  b->task_robot.finger_l = b->task_robot.finger_r = -1;
  b->grip = nullptr;
  b->cap_stream = b->bwd_stream = nullptr;
  for (int i = 0; i < 4; ++i) b->fsplit[i / 2][i % 2] = -1;
  b->fsplit_force = -1;
  b->ev_fork = b->ev_join = nullptr;
  b->arch = prop.gcnArchName;
  if (b->arch.find(':') != std::string::npos) b->arch = b->arch.substr(0, b->arch.find(':'));
  b->fwd_from_cache = b->bwd_from_cache = false;
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&b->bwd_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess) {
    release_handles(b);
    delete b;
    return fail(MS_E_HIP, "stream / event creation failed");
  }
  // allow the kernels the whole LDS of a workgroup
  (void)hipFuncSetAttribute(step_kernel_ptr(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->max_lds);
  (void)hipFuncSetAttribute(step_rec_kernel_ptr(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->max_lds);
  (void)hipFuncSetAttribute(step_frc_kernel_ptr(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->max_lds);
  (void)hipFuncSetAttribute(spawn_check_kernel_ptr(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->max_lds);
  (void)hipFuncSetAttribute(step_bwd_wave_ptr(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->max_lds);
  choose_bwd_split(b, b->split_c, b->split_r);
  // status starts at zero; the first step's scene times (which order the
  // step) decrease along the static order
  std::vector<int> cost0(c.S);
  {
    const int* ord = reinterpret_cast<const int*>(host.data() + pl.order);
    for (int p = 0; p < c.S; ++p) cost0[ord[p]] = (int)std::min<long long>(4096LL * (c.S - p), 0x7fffffffLL);
  }
  hipError_t e = hipMemsetAsync(b->scratch + b->sl.status, 0, sizeof(uint32_t) * c.S, stream);
  if (e == hipSuccess) e = hipMemsetAsync(b->scratch + b->sl.fwd_maxc, 0, sizeof(int) * c.S, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->scratch + b->sl.fwd_cost, cost0.data(), sizeof(int) * c.S, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    release_handles(b);
    delete b;
    return fail(MS_E_HIP, "status init: %s", hipGetErrorString(e));
  }
  *out = b;
  return MS_OK;
}

ms_status ms_destroy_batch(ms_batch* b) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  drop_graphs(b);
  release_handles(b);
  delete b;
  return MS_OK;
}

ms_status ms_set_schedule(ms_batch* b, const ms_schedule* s) {
  if (!b || !s) return fail(MS_E_INVALID, "null argument");
  const int known = MS_SCHED_PERSISTENT | MS_SCHED_GRAPH | MS_SCHED_PER_SUBSTEP | MS_SCHED_STAGE_STATIC | MS_SCHED_CULL |
                    MS_SCHED_BWD_REFERENCE | MS_SCHED_BWD_ONE_LAUNCH | MS_SCHED_STATIC_ORDER |
                    MS_SCHED_FWD_ONE_LAUNCH;
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

ms_status ms_set_backward_split(ms_batch* b, int32_t contact_cap, int32_t robot_contact_cap) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if (contact_cap < 0) {
    choose_bwd_split(b, b->split_c, b->split_r);
    return MS_OK;
  }
  if (contact_cap == 0) {
    b->split_c = b->split_r = 0;
    return MS_OK;
  }
  if (contact_cap > b->desc.contact_cap || robot_contact_cap < 1 ||
      robot_contact_cap > std::max(b->desc.robot_contact_cap, 1))
    return fail(MS_E_INVALID, "split caps %d / %d outside [1, %d] / [1, %d]", contact_cap, robot_contact_cap,
                b->desc.contact_cap, std::max(b->desc.robot_contact_cap, 1));
  b->split_c = contact_cap;
  b->split_r = robot_contact_cap;
  return MS_OK;
}

ms_status ms_set_forward_split(ms_batch* b, int32_t contact_cap) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if (contact_cap >= b->desc.contact_cap)
    return fail(MS_E_INVALID, "forward split cap %d must be below the batch's contact_cap %d", contact_cap,
                b->desc.contact_cap);
  drop_graphs(b);
  b->fsplit_force = contact_cap < 0 ? -1 : contact_cap;
  return MS_OK;
}

ms_status ms_get_forward_split(ms_batch* b, int32_t* contact_cap, int32_t* n_full, int32_t* n_retry) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  const int force = (b->frc_robot != nullptr || b->grip != nullptr) ? 1 : 0;
  const int stage = (b->sched.flags & MS_SCHED_STAGE_STATIC) ? 1 : 0;
  if (contact_cap) *contact_cap = fwd_split_cap(b, stage, force);
  if (n_full || n_retry) {
    int v[2] = {0, 0};
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(&v[0], b->scratch + b->sl.fwd_nover, sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&v[1], b->scratch + b->sl.fwd_retry, sizeof(int), hipMemcpyDeviceToHost));
    if (n_full) *n_full = v[0];
    if (n_retry) *n_retry = v[1];
  }
  return MS_OK;
}

ms_status ms_get_backward_split(const ms_batch* b, int32_t* contact_cap, int32_t* robot_contact_cap) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if (contact_cap) *contact_cap = b->split_c;
  if (robot_contact_cap) *robot_contact_cap = b->split_r;
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

// ------------------------------------------------------ allocation-free step
//
// ms_step_noalloc keeps the step's scratch -- the persistent work counter and,
// for normalized actions, the control step's PD targets -- in the library's
// own device array instead of the batch's scratch buffer, and enqueues only
// kernels: no allocation, no graph, no split launch.

}  // extern "C"

namespace {
constexpr int NOALLOC_MAX_SCENES = 16384;
constexpr size_t NOALLOC_QUEUE_BYTES = 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_QUEUE_BYTES + sizeof(float) * 16 * (size_t)NOALLOC_MAX_SCENES;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

// each device holds its own copy (1 MiB + 256 B) until the process ends; host
// code uses only the address hipGetSymbolAddress gives for the current device
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
// the device address of `scratch` on device dev (current), looked up once
ms_status noalloc_scratch(int dev, char** out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(MS_E_UNSUPPORTED, "device %d beyond %d", dev, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(MS_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_noalloc_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return MS_OK;
}
}  // namespace

extern "C" {

ms_status ms_step_noalloc(ms_batch* b, const void* x_in, const float* u, void* x_out, void* hip_stream) {
  if (!b || !x_in || !u || !x_out) return fail(MS_E_INVALID, "null batch, state or controls");
  if (b->cnt.S > NOALLOC_MAX_SCENES)
    return fail(MS_E_INVALID, "ms_step_noalloc: %d scenes exceed its limit of %d (use ms_step)", b->cnt.S,
                NOALLOC_MAX_SCENES);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != b->device) return fail(MS_E_INVALID, "ms_step_noalloc: current device %d, batch on %d", dev, b->device);
  char* base = nullptr;
  ms_status rs = noalloc_scratch(dev, &base);
  if (rs != MS_OK) return rs;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int* queue = reinterpret_cast<int*>(base);
  const float* uu = u;
  if (b->desc.control_mode == MS_CTRL_ACTIONS) {
    float* tgt = reinterpret_cast<float*>(base + NOALLOC_QUEUE_BYTES);
    launch_actions(reinterpret_cast<const DModel*>(b->params + b->pl.models),
                   reinterpret_cast<const DScene*>(b->params + b->pl.scenes), static_cast<const float*>(x_in), u,
                   tgt, b->cnt.S, st);
    HIP_TRY(hipGetLastError());
    uu = tgt;
  }
  KArgs a = make_args(b, x_in, uu, x_out);
  a.mode = step_mode(b);
  a.queue = queue;
  a.cost = nullptr;   // the static scene order: no cost keys, no split
  a.maxc = nullptr;
  a.debug = nullptr;
  a.phase_cycles = nullptr;
  const size_t lds = lds_bytes_of(a);
  if (lds > b->max_lds)
    return fail(MS_E_UNSUPPORTED, "scene working set needs %zu B of LDS (device limit %zu B)", lds, b->max_lds);
  if (a.persistent) {
    launch_reset_queue(queue, st);   // the counter keeps the last call's value
    HIP_TRY(hipGetLastError());
  }
  launch_step(a, a.persistent ? persistent_grid(b, lds) : b->cnt.S, lds, st);
  HIP_TRY(hipGetLastError());
  return MS_OK;
}

// The forward kernel in record mode: one fused launch per control step (the
// batch's persistent / staging / culling choices), no state output.
ms_status enqueue_record(ms_batch* b, const void* x_in, const float* u, float* rec, hipStream_t st,
                         void* x_out = nullptr) {
  KArgs a = make_args(b, x_in, u, x_out);
  a.mode = step_mode(b);
  a.debug = nullptr;
  a.phase_cycles = nullptr;
  a.frc_robot = nullptr;
  a.frc_body = nullptr;
  a.grip = nullptr;
  a.rec = rec;
  a.RL = bwd_rec(&b->desc, b->cnt);
  size_t lds = lds_bytes_of(a);
  if (lds > b->max_lds) return fail(MS_E_UNSUPPORTED, "scene working set needs %zu B of LDS", lds);
  return launch_fused(b, a, lds, st);
}

ms_status ms_reset_robots(ms_batch* b, void* x, const uint8_t* mask, const float* base, const float* noise,
                          const float* clip, void* hip_stream) {
  if (!b || !x || !base || !noise || !clip) return fail(MS_E_INVALID, "ms_reset_robots: null argument");
  for (int j = 0; j < ND; ++j)
    if (!(clip[j] >= 0.f)) return fail(MS_E_INVALID, "ms_reset_robots: clip[%d] must be >= 0", j);
  launch_reset_robots(static_cast<float*>(x), mask, base, noise, clip, b->cnt.S, static_cast<hipStream_t>(hip_stream));
  HIP_TRY(hipGetLastError());
  return MS_OK;
}

ms_status ms_spawn_check(ms_batch* b, const void* x, uint8_t* collide, void* hip_stream) {
  if (!b || !x || !collide) return fail(MS_E_INVALID, "ms_spawn_check: null argument");
  // the kernel loads a scene like a step does; the control slot reads the scratch targets
  KArgs a = make_args(b, x, reinterpret_cast<const float*>(b->scratch + b->sl.act), nullptr);
  a.debug = nullptr;
  a.phase_cycles = nullptr;
  size_t lds = lds_bytes_of(a);
  if (lds > b->max_lds) return fail(MS_E_UNSUPPORTED, "scene working set needs %zu B of LDS", lds);
  launch_spawn_check(a, collide, lds, static_cast<hipStream_t>(hip_stream));
  HIP_TRY(hipGetLastError());
  return MS_OK;
}

ms_status ms_set_force_outputs(ms_batch* b, float* robot_force, float* body_force) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if ((robot_force == nullptr) != (body_force == nullptr))
    return fail(MS_E_INVALID, "ms_set_force_outputs: give both outputs or neither");
  drop_graphs(b);
  b->frc_robot = robot_force;
  b->frc_body = body_force;
  return MS_OK;
}

ms_status ms_set_task_robot(ms_batch* b, const ms_task_robot* r) {
  if (!b || !r) return fail(MS_E_INVALID, "ms_set_task_robot: null argument");
  for (size_t m = 0; m < b->model_nb.size(); ++m) {
    const int nb = b->model_nb[m];
    auto in = [&](int i) { return i >= 0 && i < nb; };
    if (!in(r->ee_body) || !in(r->base_body) || !in(r->finger_l) || !in(r->finger_r))
      return fail(MS_E_INVALID, "ms_set_task_robot: body index out of range for model %zu (%d bodies)", m, nb);
    if (!in(r->base_x) || !in(r->base_y) || !in(r->base_yaw) || (r->torso != -1 && !in(r->torso)))
      return fail(MS_E_INVALID, "ms_set_task_robot: DoF index out of range for model %zu (%d DoFs)", m, nb);
    if (r->narm < 0 || (r->narm > 0 && (!in(r->arm0) || !in(r->arm0 + r->narm - 1))))
      return fail(MS_E_INVALID, "ms_set_task_robot: arm DoFs out of range for model %zu", m);
    if (nb < 32 && (r->ee_bodies >> nb) != 0u)
      return fail(MS_E_INVALID, "ms_set_task_robot: ee_bodies names a body past model %zu's %d", m, nb);
  }
  if (!(r->grasp_force >= 0.f)) return fail(MS_E_INVALID, "ms_set_task_robot: grasp_force must be >= 0");
  drop_graphs(b);
  b->task_robot = *r;
  b->task_robot_set = true;
  return MS_OK;
}

ms_status ms_set_grip_outputs(ms_batch* b, float* grip) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if (grip && !b->task_robot_set) return fail(MS_E_STATE, "ms_set_grip_outputs: call ms_set_task_robot first");
  drop_graphs(b);
  b->grip = grip;
  return MS_OK;
}

}  // extern "C"

namespace {
ms_status task_eval(ms_batch* b, const void* x, const ms_task* tasks, const float* robot_force, const float* grip,
                    ms_episode* ep, const uint8_t* mask, float* pred, void* hip_stream) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if (!x || !tasks || !ep) return fail(MS_E_INVALID, "task call: null state, tasks or episode buffer");
  if (!b->task_robot_set) return fail(MS_E_STATE, "task call: call ms_set_task_robot first");
  TaskArgs a;
  std::memset(&a, 0, sizeof a);
  a.models = reinterpret_cast<const DModel*>(b->params + b->pl.models);
  a.scenes = reinterpret_cast<const DScene*>(b->params + b->pl.scenes);
  a.aux = reinterpret_cast<const DAux*>(b->params + b->pl.aux);
  a.x = static_cast<const float*>(x);
  a.tasks = tasks;
  a.robot_force = robot_force;
  a.grip = grip;
  a.mask = mask;
  a.ep = ep;
  a.pred = pred;
  a.robot = b->task_robot;
  a.S = b->cnt.S;
  a.NF = b->cnt.NF;
  a.n_sub = b->desc.n_substeps;
  launch_task_eval(a, static_cast<hipStream_t>(hip_stream));
  HIP_TRY(hipGetLastError());
  return MS_OK;
}
}  // namespace

extern "C" {

ms_status ms_task_begin(ms_batch* b, const void* x, const ms_task* tasks, const float* grip, ms_episode* ep,
                        const uint8_t* mask, float* pred, void* hip_stream) {
  return task_eval(b, x, tasks, nullptr, grip, ep, mask, pred, hip_stream);
}

ms_status ms_task_update(ms_batch* b, const void* x, const ms_task* tasks, const float* robot_force, const float* grip,
                         ms_episode* ep, float* pred, void* hip_stream) {
  if (!robot_force) return fail(MS_E_INVALID, "ms_task_update: robot_force_dev is required");
  return task_eval(b, x, tasks, robot_force, grip, ep, nullptr, pred, hip_stream);
}

ms_status ms_task_categorize(ms_batch* b, const ms_task* tasks, const ms_episode* ep, int32_t* mode, void* hip_stream) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if (!tasks || !ep || !mode) return fail(MS_E_INVALID, "ms_task_categorize: null buffer");
  launch_task_categorize(tasks, ep, mode, b->cnt.S, static_cast<hipStream_t>(hip_stream));
  HIP_TRY(hipGetLastError());
  return MS_OK;
}

ms_status ms_step_record(ms_batch* b, const void* x_in, const float* u, void* x_out, void* record, void* hip_stream) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if (!x_in || !u || !x_out || !record) return fail(MS_E_INVALID, "ms_step_record: null buffer");
  if (reinterpret_cast<uintptr_t>(record) % sizeof(float)) return fail(MS_E_INVALID, "ms_step_record: misaligned record");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const float* ut = control_targets(b, x_in, u, st);
  HIP_TRY(hipGetLastError());
  return enqueue_record(b, x_in, ut, static_cast<float*>(record), st, x_out);
}

static ms_status step_backward_impl(ms_batch* b, const void* x_in, const float* u, const float* given_rec,
                             const void* gx_out, void* gx_in, float* gu, void* hip_stream) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  if (!x_in || !u || !gx_out || !gx_in || !gu) return fail(MS_E_INVALID, "ms_step_backward: null buffer");
  if (!b->tape && (!given_rec || (b->sched.flags & MS_SCHED_BWD_REFERENCE)))
    return fail(MS_E_STATE, "ms_step_backward: the batch was created without a tape buffer");
  const Counts& c = b->cnt;
  const ms_batch_desc* d = &b->desc;
  BwdArgs a;
  std::memset(&a, 0, sizeof a);
  a.models = reinterpret_cast<const DModel*>(b->params + b->pl.models);
  a.scenes = reinterpret_cast<const DScene*>(b->params + b->pl.scenes);
  a.free = reinterpret_cast<const DFree*>(b->params + b->pl.free);
  a.statics = reinterpret_cast<const float*>(b->params + b->pl.statics);
  a.planes = reinterpret_cast<const float4*>(b->params + b->pl.planes);
  a.aux = reinterpret_cast<const DAux*>(b->params + b->pl.aux);
  a.order = reinterpret_cast<const int*>(b->params + b->pl.order);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const bool actions = d->control_mode == MS_CTRL_ACTIONS;
  const float* ut = control_targets(b, x_in, u, st);
  HIP_TRY(hipGetLastError());
  a.x = static_cast<const float*>(x_in);
  a.u = ut;
  a.gxo = static_cast<const float*>(gx_out);
  a.gxi = static_cast<float*>(gx_in);
  a.gu = actions ? reinterpret_cast<float*>(b->scratch + b->sl.actb) : gu;
  a.status = reinterpret_cast<uint32_t*>(b->scratch + b->sl.status);
  a.cycles = b->profile_on ? reinterpret_cast<unsigned long long*>(b->scratch + b->sl.cycles) : nullptr;
  a.ws = reinterpret_cast<float*>(b->tape);
  a.S = c.S;
  a.NF = c.NF;
  a.stride = bwd_stride(c.S);
  a.pr = msa::Prm{d->h, d->mu, d->baumgarte, d->margin, {d->gravity[0], d->gravity[1], d->gravity[2]},
                  d->pgs_iters, step_mode(b), d->contact_cap, std::max(d->robot_contact_cap, 1), d->n_substeps};
  const msa::WS ww = bwd_ws_wave(d, c);
  const size_t lds = (size_t)ww.total * sizeof(float);
  if ((b->sched.flags & MS_SCHED_BWD_REFERENCE) || lds > b->max_lds) {
    a.w = bwd_ws(d, c);
    launch_step_bwd(a, st);
  } else {
    const float* rec = given_rec;
    if (!rec) {
      float* tr = reinterpret_cast<float*>(b->tape);
      ms_status rs = enqueue_record(b, x_in, ut, tr, st);
      if (rs != MS_OK) return rs;
      rec = tr;
    }
    a.rec = rec;
    a.RL = bwd_rec(d, c);
    a.w = ww;
    // scene order by the cost the record shows (overflowing scenes first)
    const bool split = b->split_c > 0 && !(b->sched.flags & MS_SCHED_BWD_ONE_LAUNCH);
    int* bord = reinterpret_cast<int*>(b->scratch + b->sl.bwd_order);
    int* nover = reinterpret_cast<int*>(b->scratch + b->sl.bwd_nover);
    int* bslot = reinterpret_cast<int*>(b->scratch + b->sl.bwd_slot);
    launch_bwd_order(rec, a.RL, c.S, d->n_substeps, split ? b->split_c : 0, split ? b->split_r : 0, bslot, bord, nover,
                     st);
    HIP_TRY(hipGetLastError());
    a.order = bord;
    a.n_over = nover;
    if (!split) {
      a.fit_mode = 0;
      launch_step_bwd_wave(a, lds, c.S, st);
    } else {
      // fork: the scenes that overflow the smaller layout (the costliest
      // ones) on st in the full layout, a fixed grid looping over them; the
      // others on the second stream at the higher occupancy, joined back
      // onto st.  The second stream first waits 15 us so that the full-size
      // workgroups are resident before the smaller ones fill the CUs (they
      // would otherwise wait for two free slots on one CU).
      BwdArgs big = a;
      big.fit_mode = 2;
      a.fit_mode = 1;
      a.w = bwd_ws_wave(d, c, b->split_c, b->split_r);
      HIP_TRY(hipEventRecord(b->ev_fork, st));
      HIP_TRY(hipStreamWaitEvent(b->bwd_stream, b->ev_fork, 0));
      launch_step_bwd_wave(big, lds, std::min(c.S, 2 * b->n_cu), st);
      HIP_TRY(hipGetLastError());
      launch_delay(1500, b->bwd_stream);
      launch_step_bwd_wave(a, (size_t)a.w.total * sizeof(float), c.S, b->bwd_stream);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipEventRecord(b->ev_join, b->bwd_stream));
      HIP_TRY(hipStreamWaitEvent(st, b->ev_join, 0));
    }
  }
  if (actions)
    launch_actions_bwd(a.models, a.scenes, a.x, u, a.gu, gu, a.gxi, c.S, st);
  HIP_TRY(hipGetLastError());
  return MS_OK;
}

ms_status ms_step_backward(ms_batch* b, const void* x_in, const float* u, const void* gx_out, void* gx_in, float* gu,
                           void* hip_stream) {
  return step_backward_impl(b, x_in, u, nullptr, gx_out, gx_in, gu, hip_stream);
}

ms_status ms_step_backward_recorded(ms_batch* b, const void* x_in, const float* u, const void* record,
                                    const void* gx_out, void* gx_in, float* gu, void* hip_stream) {
  if (!record) return fail(MS_E_INVALID, "ms_step_backward_recorded: null record");
  if (reinterpret_cast<uintptr_t>(record) % sizeof(float))
    return fail(MS_E_INVALID, "ms_step_backward_recorded: misaligned record");
  return step_backward_impl(b, x_in, u, static_cast<const float*>(record), gx_out, gx_in, gu, hip_stream);
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

// ---------------------------------------------------------------- autotuner
//
// Forward: the forms (persistent split launch, persistent one launch, graph
// replay of the persistent step, graph replay of one workgroup per scene),
// each with and without the furniture staged in LDS, the persistent grid
// (every resident slot, or one workgroup per CU fewer) and, for the split
// form, the smaller layout's contact cap at each step of the occupancy it
// gives, down to 3/4 of the batch's cap (below it, the scenes whose lists
// grow over a rollout would crowd the full-layout launch, which a few timed
// steps from one state do not show).  Backward: the adjoint's smaller layout (none, or each contact cap
// at a step of its occupancy, with 4 or 8 robot contacts).  Choices are
// cached per (device architecture, configuration hash) in a JSON-lines file
// when one is set.

}  // extern "C"

namespace {

#ifndef MS_SOURCE_HASH
#define MS_SOURCE_HASH "unversioned"
#endif

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

std::string tune_key(const ms_batch* b, const char* what) {
  const ms_batch_desc& d = b->desc;
  const Counts& c = b->cnt;
  const int iv[] = {d.n_scenes, d.n_substeps, d.pgs_iters, d.control_mode, d.contact_cap, d.robot_contact_cap,
                    c.S, c.M, c.NF, c.NS, c.NP, c.NA, c.fmax, c.smax, c.pmax, c.amax, c.nsph_max, b->n_cu,
                    (b->frc_robot != nullptr || b->grip != nullptr) ? 1 : 0};
  const float fv[] = {d.h, d.mu, d.baumgarte, d.margin};
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, iv, sizeof iv);
  h = fnv1a(h, fv, sizeof fv);
  h = fnv1a(h, MS_SOURCE_HASH, std::strlen(MS_SOURCE_HASH));
  char buf[128];
  std::snprintf(buf, sizeof buf, "%s:%s:%016llx", b->arch.c_str(), what, (unsigned long long)h);
  return buf;
}

// integer field `name` of a cache line, or false
bool cache_int(const char* line, const char* name, long& v) {
  char pat[64];
  std::snprintf(pat, sizeof pat, "\"%s\": ", name);
  const char* p = std::strstr(line, pat);
  if (!p) return false;
  return std::sscanf(p + std::strlen(pat), "%ld", &v) == 1;
}

// the last line of the cache file whose key is `key`
bool cache_lookup(const std::string& path, const std::string& key, std::string& line_out) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  const std::string pat = "\"key\": \"" + key + "\"";
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof line, f))
    if (std::strstr(line, pat.c_str())) {
      line_out = line;
      found = true;
    }
  std::fclose(f);
  return found;
}

void cache_append(const std::string& path, const std::string& line) {
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fputs(line.c_str(), f);
  std::fputc('\n', f);
  std::fclose(f);
}

float cache_ms(const std::string& line) {
  const char* p = std::strstr(line.c_str(), "\"ms_per_step\": ");
  float v = -1.f;
  if (p) std::sscanf(p + 15, "%f", &v);
  return v;
}

// contact caps below `cap` (down to `lowest`) at which the occupancy per CU
// of the layout steps up: the largest cap of each occupancy above full's
template <class PerCu>
std::vector<int> occupancy_steps(int cap, PerCu per_cu, int lowest) {
  std::vector<int> out;
  int last = per_cu(cap);
  for (int k = cap - 1; k >= std::max(lowest, 1); --k) {
    const int o = per_cu(k);
    if (o > last) {
      out.push_back(k);
      last = o;
    }
  }
  return out;
}

// time `reps` calls of fn on st after two untimed ones; ms per call or < 0
template <class F>
float time_calls(hipStream_t st, int reps, F fn) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.f;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.f;
  }
  bool ok = fn() && fn();
  (void)hipEventRecord(e0, st);
  for (int r = 0; r < reps && ok; ++r) ok = fn();
  (void)hipEventRecord(e1, st);
  float ms = -1.f;
  if (ok && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) ms /= reps;
  else ms = -1.f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

}  // namespace

extern "C" {

ms_status ms_set_autotune_cache(ms_batch* b, const char* path) {
  if (!b) return fail(MS_E_INVALID, "null batch");
  b->tune_cache = path ? path : "";
  return MS_OK;
}

ms_status ms_autotune_key(const ms_batch* b, int32_t backward, char* out, size_t n, int32_t* from_cache) {
  if (!b || !out || n == 0) return fail(MS_E_INVALID, "null argument");
  const std::string k = tune_key(b, backward ? "bwd" : "fwd");
  if (k.size() + 1 > n) return fail(MS_E_INVALID, "ms_autotune_key: buffer of %zu bytes, %zu needed", n, k.size() + 1);
  std::memcpy(out, k.c_str(), k.size() + 1);
  if (from_cache) *from_cache = backward ? b->bwd_from_cache : b->fwd_from_cache;
  return MS_OK;
}

ms_status ms_autotune(ms_batch* b, const void* x, const float* u, void* tmp, int32_t reps, void* hip_stream,
                      ms_schedule* chosen, float* ms_per_step) {
  if (!b || !x || !u || !tmp) return fail(MS_E_INVALID, "null argument");
  if (reps <= 0) reps = 5;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const std::string key = tune_key(b, "fwd");
  b->fwd_from_cache = false;
  if (!b->tune_cache.empty()) {
    std::string line;
    long fl = 0, gr = 0, fs = -1;
    if (cache_lookup(b->tune_cache, key, line) && cache_int(line.c_str(), "flags", fl) &&
        cache_int(line.c_str(), "grid", gr) && cache_int(line.c_str(), "fwd_split", fs)) {
      ms_schedule s{(int32_t)fl, (int32_t)gr};
      if (ms_set_schedule(b, &s) == MS_OK && ms_set_forward_split(b, (int32_t)fs) == MS_OK) {
        b->fwd_from_cache = true;
        if (chosen) *chosen = b->sched;
        if (ms_per_step) *ms_per_step = cache_ms(line);
        return MS_OK;
      }
    }
  }
  const ms_schedule saved = b->sched;
  const int saved_fs = b->fsplit_force;
  const int P = MS_SCHED_PERSISTENT, G = MS_SCHED_GRAPH, CU = MS_SCHED_CULL;
  const int forms[] = {P | CU, P | CU | MS_SCHED_FWD_ONE_LAUNCH, G | P | CU, G | CU};
  const int force = (b->frc_robot != nullptr || b->grip != nullptr) ? 1 : 0;
  struct Cand { int flags, grid, fsplit; };
  std::vector<Cand> cands;
  for (int stage : {(int)MS_SCHED_STAGE_STATIC, 0}) {
    const int si = stage ? 1 : 0;
    const size_t full = (size_t)fwd_layout(b, b->desc.contact_cap, si, force).total * sizeof(float);
    if (full > b->max_lds) continue;
    for (int form : forms) {
      const int fl = form | stage;
      std::vector<int> splits{-1};
      if (form == (P | CU)) {
        // the full layout's occupancy, then the smaller layout's at each cap
        splits = occupancy_steps(b->desc.contact_cap, [&](int k) {
          const int rc = k == b->desc.contact_cap ? -1 : fwd_split_rcap(b);
          return fwd_per_cu((size_t)fwd_layout(b, k, si, force, rc).total * sizeof(float));
        }, (3 * b->desc.contact_cap) / 4);
        if (splits.empty()) continue;   // no smaller layout: the same as one launch
      }
      for (int fs : splits) {
        std::vector<int> grids{0};
        if (form & P) {
          const size_t lds = fs > 0 ? (size_t)fwd_layout(b, fs, si, force, fwd_split_rcap(b)).total * sizeof(float)
                                    : full;
          const int per_cu = fwd_per_cu(lds);
          if (per_cu > 1 && b->n_cu * (per_cu - 1) < b->cnt.S) grids.push_back(b->n_cu * (per_cu - 1));
        }
        for (int g : grids) cands.push_back({fl, g, fs});
      }
    }
  }
  const size_t bytes = ((size_t)b->cnt.S * 32 + (size_t)b->cnt.NF * 16 + (size_t)b->cnt.NA * 4) * sizeof(float);
  Cand best{saved.flags, saved.grid, saved_fs};
  float best_ms = 1e30f;
  for (const Cand& c : cands) {
    ms_schedule s{c.flags, c.grid};
    if (ms_set_schedule(b, &s) != MS_OK) continue;
    if (ms_set_forward_split(b, c.fsplit) != MS_OK) continue;
    if (hipMemcpyAsync(tmp, x, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) continue;
    const float ms = time_calls(st, reps, [&] { return ms_step(b, tmp, u, tmp, st) == MS_OK; });
    if (ms > 0.f && ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  ms_schedule bs{best.flags, best.grid};
  ms_status rs = ms_set_schedule(b, &bs);
  if (rs == MS_OK) rs = ms_set_forward_split(b, best.fsplit);
  if (rs != MS_OK) {
    (void)ms_set_schedule(b, &saved);
    (void)ms_set_forward_split(b, saved_fs);
    return rs;
  }
  if (chosen) *chosen = b->sched;
  if (ms_per_step) *ms_per_step = best_ms;
  if (!b->tune_cache.empty() && best_ms < 1e29f) {
    char line[512];
    std::snprintf(line, sizeof line,
                  "{\"key\": \"%s\", \"flags\": %d, \"grid\": %d, \"fwd_split\": %d, \"ms_per_step\": %.5f, "
                  "\"candidates\": %zu}",
                  key.c_str(), best.flags, best.grid, best.fsplit, best_ms, cands.size());
    cache_append(b->tune_cache, line);
  }
  return MS_OK;
}

ms_status ms_autotune_backward(ms_batch* b, const void* x, const float* u, const void* gx_out, void* gx_in,
                               float* gu, int32_t reps, void* hip_stream, int32_t* split_c, int32_t* split_r,
                               float* ms_per_step) {
  if (!b || !x || !u || !gx_out || !gx_in || !gu) return fail(MS_E_INVALID, "null argument");
  if (!b->tape) return fail(MS_E_STATE, "ms_autotune_backward: the batch has no tape buffer");
  if (reps <= 0) reps = 3;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const std::string key = tune_key(b, "bwd");
  b->bwd_from_cache = false;
  if (!b->tune_cache.empty()) {
    std::string line;
    long c = 0, r = 0;
    if (cache_lookup(b->tune_cache, key, line) && cache_int(line.c_str(), "split_c", c) &&
        cache_int(line.c_str(), "split_r", r) && ms_set_backward_split(b, (int32_t)c, (int32_t)r) == MS_OK) {
      b->bwd_from_cache = true;
      if (split_c) *split_c = b->split_c;
      if (split_r) *split_r = b->split_r;
      if (ms_per_step) *ms_per_step = cache_ms(line);
      return MS_OK;
    }
  }
  const int sc0 = b->split_c, sr0 = b->split_r;
  const ms_batch_desc* d = &b->desc;
  std::vector<std::pair<int, int>> cands{{0, 0}};
  const int rfull = std::max(d->robot_contact_cap, 1);
  for (int r : {std::min(rfull, 8), std::min(rfull, 4)}) {
    std::vector<int> ks = occupancy_steps(d->contact_cap + 1, [&](int k) {
      const int kk = std::min(k, d->contact_cap);
      return bwd_per_cu((size_t)bwd_ws_wave(d, b->cnt, kk, k > d->contact_cap ? rfull : r).total * sizeof(float));
    }, (d->contact_cap + 1) / 2);
    for (int k : ks)
      if (std::find(cands.begin(), cands.end(), std::make_pair(k, r)) == cands.end()) cands.push_back({k, r});
  }
  // the candidates time the adjoint launches alone, from one record of this
  // step in the tape buffer (the record does not depend on the split: timed
  // with it, the candidates' differences drowned in the recording's time);
  // the reference path, or a workspace beyond LDS, records in each call
  const float* rec = nullptr;
  {
    const msa::WS ww = bwd_ws_wave(d, b->cnt);
    if (!(b->sched.flags & MS_SCHED_BWD_REFERENCE) && (size_t)ww.total * sizeof(float) <= b->max_lds) {
      const float* ut = control_targets(b, x, u, st);
      HIP_TRY(hipGetLastError());
      const ms_status rs = enqueue_record(b, x, ut, reinterpret_cast<float*>(b->tape), st);
      if (rs != MS_OK) return rs;
      rec = reinterpret_cast<const float*>(b->tape);
    }
  }
  // two rounds over the candidates, each kept at its faster round: the
  // candidates are a few percent apart, about the spread of one timing
  std::pair<int, int> best{sc0, sr0};
  float best_ms = 1e30f;
  std::vector<float> cand_ms(cands.size(), 1e30f);
  std::vector<std::pair<int, int>> applied(cands);
  for (int round = 0; round < 2; ++round)
    for (size_t i = 0; i < cands.size(); ++i) {
      const auto& c = cands[i];
      if (c.first == 0) b->split_c = b->split_r = 0;
      else if (ms_set_backward_split(b, c.first, c.second) != MS_OK) continue;
      applied[i] = {b->split_c, b->split_r};
      const float ms =
          time_calls(st, reps, [&] { return step_backward_impl(b, x, u, rec, gx_out, gx_in, gu, st) == MS_OK; });
      if (ms > 0.f) cand_ms[i] = std::min(cand_ms[i], ms);
    }
  for (size_t i = 0; i < cands.size(); ++i)
    if (cand_ms[i] < best_ms) {
      best_ms = cand_ms[i];
      best = applied[i];
    }
  // within 2 % of the fastest, the split with the most robot contacts in its
  // smaller layout: the tuning step is one state, and a horizon whose robot
  // contacts grow sends fewer scenes to the full layout with it
  for (size_t i = 0; i < cands.size(); ++i)
    if (cand_ms[i] <= 1.02f * best_ms && applied[i].first > 0 &&
        (best.first == 0 || applied[i].second > best.second)) {
      best = applied[i];
      best_ms = cand_ms[i];
    }
  b->split_c = best.first;
  b->split_r = best.second;
  if (split_c) *split_c = b->split_c;
  if (split_r) *split_r = b->split_r;
  if (ms_per_step) *ms_per_step = best_ms;
  if (!b->tune_cache.empty() && best_ms < 1e29f) {
    char line[512];
    std::snprintf(line, sizeof line,
                  "{\"key\": \"%s\", \"split_c\": %d, \"split_r\": %d, \"ms_per_step\": %.5f, \"candidates\": %zu}",
                  key.c_str(), best.first, best.second, best_ms, cands.size());
    cache_append(b->tune_cache, line);
  }
  return MS_OK;
}

}  // extern "C"
