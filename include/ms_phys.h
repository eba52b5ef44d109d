/* ms_phys.h -- C ABI of the batched rigid-body physics step on MI355X (gfx950).
 *
 * The step advances S independent scenes by one control step: n_substeps
 * physics substeps with the controls held (zero-order hold).  It is the
 * physics part of the environment dynamics T: S x A -> S that the paper's
 * many-environment simulation evaluates for every environment at once
 * (MDP formulation, Sec. 3; 100 Hz simulation under 20 Hz control and up to
 * 4096 parallel environments, Sec. 4.2).  Each substep: drive (torque or
 * implicit PD), forward kinematics, sphere-decomposed contacts, articulated-
 * body dynamics, contact rows, projected Gauss-Seidel with a friction disk in
 * a fixed level-scheduled order, semi-implicit Euler.  The paper does not
 * describe its solver; every numerical choice is documented with the oracle.
 *
 * Conventions
 *   - All functions are extern "C", never throw, and return ms_status
 *     (0 = MS_OK, negative = error).  ms_last_error() gives a message.
 *   - "_dev" pointers are device memory on the batch's device; "host" ones
 *     are host memory.  The caller owns every buffer; the library allocates
 *     no device memory (it binds the params / scratch / tape buffers the
 *     caller allocated from ms_query_sizes) and keeps only host objects: HIP
 *     graphs, a capture stream, and a second stream with two events for
 *     split launches (all at default priority).
 *   - Stream-ordered calls (ms_step, ms_step_record, ms_step_backward,
 *     ms_step_backward_recorded, ms_set_state) enqueue work on hip_stream (a
 *     hipStream_t, may be null = default stream) and return without
 *     synchronising.  A split launch runs part of the work on the library's
 *     second stream, forked from and joined back onto hip_stream with events,
 *     so later work on hip_stream sees all of it; calls on one batch from
 *     several streams at once are not supported.  Argument errors are
 *     detected before anything is enqueued and leave all buffers untouched.
 *   - Numeric faults are per scene: status bits, read with ms_scene_status.
 *
 * State layout (float32, one flat buffer of ms_state_floats() floats):
 *   q[S][16], qd[S][16]            robot joint positions / velocities (padded to 16)
 *   free[NF][16]                   per free body: pos xyz, 0, quat wxyz,
 *                                  linvel xyz, 0, angvel xyz, 0 (world frame)
 *   aux[NA][4]                     per door / drawer joint: q, qd, 0, 0
 * with NF = free_off[S], NA = aux_off[S] (CSR offsets of the scene description).
 * Controls: float32 [S][16] (torques, PD targets, or torques added to a PD hold,
 * by control_mode).
 */
#ifndef MS_PHYS_H
#define MS_PHYS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ms_status;
enum {
  MS_OK = 0,
  MS_E_INVALID = -1,     /* bad argument, shape or pointer; nothing was done */
  MS_E_NOMEM = -2,       /* a caller buffer is smaller than ms_query_sizes asked for */
  MS_E_HIP = -3,         /* a HIP runtime call failed (message in ms_last_error) */
  MS_E_STATE = -4,       /* call not valid in the batch's current state */
  MS_E_NUMERIC = -5,     /* at least one scene has a numeric status bit set */
  MS_E_UNSUPPORTED = -6  /* device or configuration not supported (e.g. not gfx950) */
};

/* control modes: joint torques; PD targets (position, or velocity for base
 * DoFs); torques added to a PD hold of scene_hold; normalized actions in
 * [-1, 1] mapped per DoF to PD targets once per control step (joint delta
 * position for arm, torso and head, base linear and angular velocity,
 * gripper opening: the action space of Sec. 4.1, see model_act_kind) */
enum { MS_CTRL_TORQUE = 0, MS_CTRL_PD = 1, MS_CTRL_TORQUE_HOLD = 2, MS_CTRL_ACTIONS = 3 };
/* normalized-action channel of a DoF (a = the action clipped to [-1, 1],
 * q = the state at the control step's start, s = model_act_scale) */
enum {
  MS_ACT_DELTA = 0,       /* position target q + a s */
  MS_ACT_BASE_FWD_X = 1,  /* velocity target a s cos(yaw) (yaw: the MS_ACT_BASE_YAW DoF's position) */
  MS_ACT_BASE_FWD_Y = 2,  /* velocity target a_x s sin(yaw) (a_x: the MS_ACT_BASE_FWD_X DoF's action) */
  MS_ACT_BASE_YAW = 3,    /* velocity target a s */
  MS_ACT_ABSOLUTE = 4     /* position target (a + 1) / 2 s */
};

/* per-scene status bits (ms_scene_status) */
enum {
  MS_ST_NONFINITE = 1u,       /* non-finite value in the scene's state after the step */
  MS_ST_OVERFLOW = 2u,        /* more contacts than contact_cap (extra contacts dropped) */
  MS_ST_DEGENERATE = 4u,      /* a row with effective mass below 1e-12 was skipped */
  MS_ST_ROBOT_OVERFLOW = 8u   /* more robot contacts than robot_contact_cap (dropped) */
};

/* schedule flags */
enum {
  MS_SCHED_PERSISTENT = 1,    /* fixed grid pulling cost-sorted scenes from a queue */
  MS_SCHED_GRAPH = 2,         /* replay one control step as a captured hipGraph */
  MS_SCHED_PER_SUBSTEP = 4,   /* one launch per substep (state round trip through HBM) */
  MS_SCHED_STAGE_STATIC = 8,  /* stage each scene's furniture boxes in LDS */
  MS_SCHED_CULL = 16,         /* bounding-sphere pre-test before sphere-pair tests */
  MS_SCHED_BWD_REFERENCE = 32, /* ms_step_backward on the lane-per-scene kernel that
                                  recomputes everything itself (slow; a cross-check) */
  MS_SCHED_STATIC_ORDER = 128,  /* process the scenes in the order fixed at creation
                                   (by static size) instead of by decreasing time as the
                                   previous step measured it for each scene */
  MS_SCHED_FWD_ONE_LAUNCH = 256, /* the persistent step in one launch sized for the contact
                                    caps.  Without it, when a smaller contact cap fits more
                                    workgroups per CU, the scenes whose previous-step contact
                                    counts leave room under it run in that layout and the
                                    others in the full one (side by side, the second on a
                                    library-owned stream joined back); a scene that
                                    overflows the smaller layout anyway is stepped again in
                                    the full one.  The results are the same bit for bit */
  MS_SCHED_BWD_ONE_LAUNCH = 64  /* ms_step_backward in one wavefront launch sized for the
                                  contact caps.  Without it the scenes whose contact
                                  lists fit a smaller LDS layout (more workgroups per
                                  CU) run in one launch and the rest in a second launch
                                  on a library-owned stream, joined back onto the
                                  caller's stream; the results are the same bit for bit */
};

typedef struct {
  int32_t n_scenes;
  int32_t n_substeps;          /* substeps per control step (zero-order hold) */
  int32_t pgs_iters;           /* Gauss-Seidel sweeps per substep */
  int32_t control_mode;        /* MS_CTRL_* */
  int32_t contact_cap;         /* contacts kept per scene per substep (first in canonical order) */
  int32_t robot_contact_cap;   /* robot-owned contacts kept per scene per substep */
  float h;                     /* substep length, s */
  float mu;                    /* friction coefficient */
  float baumgarte;             /* penetration correction factor beta */
  float margin;                /* speculative contact margin delta, m */
  float gravity[3];            /* m/s^2 */
} ms_batch_desc;

/* Host arrays describing the scenes (same layout as the scene generator
 * writes; ownership stays with the caller, read only during ms_query_sizes /
 * ms_create_batch).  M robot models, S scenes, NF free bodies, NS static
 * boxes, NP planes, NA door / drawer joints. */
typedef struct {
  int32_t n_models;
  const int32_t* model_nb;        /* [M] bodies (= DoFs) of the robot, <= 16 */
  const int32_t* model_parent;    /* [M][16] parent body, -1 = world; parents precede children */
  const int32_t* model_jtype;     /* [M][16] 0 revolute, 1 prismatic */
  const float* model_axis;        /* [M][16][3] unit joint axis in the joint frame */
  const float* model_xt_rot;      /* [M][16][4] joint frame rotation in the parent body frame (wxyz) */
  const float* model_xt_pos;      /* [M][16][3] joint frame origin in the parent body frame */
  const float* model_mass;        /* [M][16] */
  const float* model_com;         /* [M][16][3] centre of mass, body frame */
  const float* model_inertia;     /* [M][16][6] about the COM, body axes: xx yy zz xy xz yz */
  const float* model_kp;          /* [M][16] PD stiffness */
  const float* model_kd;          /* [M][16] PD damping */
  const int32_t* model_veldof;    /* [M][16] 1: the PD target is a velocity (planar base) */
  const float* model_armature;    /* [M][16] rotor inertia */
  const float* model_damping;     /* [M][16] viscous joint damping */
  const int32_t* model_act_kind;  /* [M][16] MS_ACT_* channel (read by MS_CTRL_ACTIONS only; may be null) */
  const float* model_act_scale;   /* [M][16] its scale (may be null with model_act_kind) */
  const int32_t* model_nsph;      /* [M] collision spheres, <= 128 */
  const int32_t* model_sph_body;  /* [M][128] body of each sphere (sorted by body) */
  const float* model_sph;         /* [M][128][4] centre in the body frame, radius */
  const int32_t* model_sph_flags; /* [M][128] bit0: no contact with the scene's first plane */
  const int32_t* scene_model;     /* [S] */
  const int32_t* free_off;        /* [S+1] CSR offsets into the free-body arrays */
  const int32_t* static_off;      /* [S+1] into static_box */
  const int32_t* plane_off;       /* [S+1] into plane */
  const int32_t* aux_off;         /* [S+1] into the aux arrays */
  const float* scene_hold;        /* [S][16] hold targets (MS_CTRL_TORQUE_HOLD) */
  const int32_t* free_type;       /* [NF] 0 box, 1 sphere */
  const float* free_size;         /* [NF][3] half extents, or radius */
  const float* free_mass;         /* [NF] */
  const float* free_inertia;      /* [NF][3] principal moments (box axes) */
  const float* static_box;        /* [NS][6] centre, half extents (axis aligned) */
  const float* plane;             /* [NP][4] unit normal n and d with n.x = d */
  const int32_t* aux_type;        /* [NA] 0 revolute (door), 1 prismatic (drawer) */
  const float* aux_rot;           /* [NA][4] joint frame in the world (wxyz) */
  const float* aux_pos;           /* [NA][3] */
  const float* aux_axis;          /* [NA][3] joint axis, joint frame */
  const float* aux_box;           /* [NA][6] box centre in the moving frame, half extents */
  const float* aux_mass;          /* [NA] */
  const float* aux_inertia;       /* [NA][3] principal moments about the box centre */
  const float* aux_limit;         /* [NA][2] lower, upper joint limit (lower > upper: none) */
} ms_scene_desc;

typedef struct {
  size_t params;   /* device bytes: packed scene description (uploaded by ms_create_batch) */
  size_t state;    /* device bytes of one state buffer */
  size_t scratch;  /* device bytes: queue counters, schedule tables, per-scene status, debug */
  size_t tape;     /* device bytes of the adjoint workspace ms_step_backward needs */
  size_t lds;      /* LDS bytes per scene workgroup (information only) */
  size_t record;   /* device bytes of one control step's record (ms_step_record) */
} ms_sizes;

typedef struct {
  float* q;          /* [S][16] */
  float* qd;         /* [S][16] */
  float* free_body;  /* [NF][16] */
  float* aux;        /* [NA][4] */
  const int32_t* free_off_host;  /* [S+1] (owned by the batch) */
  const int32_t* aux_off_host;   /* [S+1] (owned by the batch) */
  int32_t n_scenes, n_free, n_aux;
} ms_state_view;

typedef struct {
  int32_t flags;        /* MS_SCHED_* */
  int32_t grid;         /* persistent grid size (0 = automatic) */
} ms_schedule;

typedef struct ms_batch ms_batch;

/* Byte sizes of the buffers a batch needs.  Validates desc and scenes
 * (shapes, CSR monotonicity, model sizes); MS_E_INVALID on any violation. */
ms_status ms_query_sizes(const ms_batch_desc* desc, const ms_scene_desc* scenes, ms_sizes* out);

/* Number of floats of one state buffer. */
ms_status ms_state_floats(const ms_scene_desc* scenes, int32_t n_scenes, size_t* out);

/* Create a batch on the current HIP device.  params_dev / scratch_dev /
 * tape_dev must hold at least the sizes from ms_query_sizes (tape_dev may be
 * null when ms_step_backward is never called).  Uploads the scene
 * description synchronously on hip_stream.  Requires a gfx950 device. */
ms_status ms_create_batch(const ms_batch_desc* desc, const ms_scene_desc* scenes, void* params_dev,
                          void* scratch_dev, void* tape_dev, void* hip_stream, ms_batch** out);

/* Destroy the host-side batch object and its graphs (no device frees). */
ms_status ms_destroy_batch(ms_batch* b);

/* Choose how ms_step runs (see MS_SCHED_*).  Drops captured graphs. */
ms_status ms_set_schedule(ms_batch* b, const ms_schedule* sched);
ms_status ms_get_schedule(const ms_batch* b, ms_schedule* out);

/* Contact caps of the smaller LDS layout of the split ms_step_backward (see
 * MS_SCHED_BWD_ONE_LAUNCH): scenes whose contact lists hold at most
 * contact_cap contacts and robot_contact_cap robot contacts in every substep
 * of the step run in the smaller layout, the others in the full one.  At
 * creation the library picks the caps that raise the number of workgroups per
 * CU (contact_cap 0: no such caps, one launch).  contact_cap 0 turns the
 * split off; contact_cap < 0 restores the library's choice.  Error
 * MS_E_INVALID when a cap exceeds the batch's.  Either output may be null. */
ms_status ms_set_backward_split(ms_batch* b, int32_t contact_cap, int32_t robot_contact_cap);
ms_status ms_get_backward_split(const ms_batch* b, int32_t* contact_cap, int32_t* robot_contact_cap);

/* Contact cap of the smaller layout of the persistent step (see
 * MS_SCHED_FWD_ONE_LAUNCH); contact_cap 0 turns the split off, < 0 restores
 * the library's choice.  Error MS_E_INVALID when contact_cap is not below
 * the batch's.  Drops captured graphs. */
ms_status ms_set_forward_split(ms_batch* b, int32_t contact_cap);
/* The cap in use for the current schedule and output settings, and (if
 * n_full or n_retry is non-null; synchronises the device) how many scenes
 * the last split step routed to the full layout and stepped again after
 * overflowing the smaller one.  Any output may be null. */
ms_status ms_get_forward_split(ms_batch* b, int32_t* contact_cap, int32_t* n_full, int32_t* n_retry);

/* Forward autotuner (the batched step's launch schedule, Sec. 4.2's many
 * parallel environments on one device): times every candidate schedule on
 * the given state / controls (the state is not modified: a copy in
 * tmp_state_dev is stepped; each candidate runs 2 + reps steps) and keeps the
 * fastest.  Candidates: the persistent split launch (for each contact cap of
 * the smaller layout at which its workgroups per CU step up), the persistent
 * one launch, the graph replay of the persistent step and of one workgroup
 * per scene; each with and without furniture staged in LDS; persistent forms
 * with the grid filling every resident slot or one workgroup per CU fewer.
 * With a cache file set (ms_set_autotune_cache) a cached choice for the same
 * key is applied without timing, and a new choice is appended.  Synchronises
 * the stream.  Writes the chosen schedule (its forward split cap: see
 * ms_get_forward_split) and its time in ms per control step (the cached
 * time on a cache hit).  On error the previous schedule is kept. */
ms_status ms_autotune(ms_batch* b, const void* state_dev, const float* controls_dev, void* tmp_state_dev,
                      int32_t reps, void* hip_stream, ms_schedule* chosen, float* ms_per_step);

/* Backward autotuner: records the control step from the given state /
 * controls once into the tape buffer, then times the adjoint launches of
 * ms_step_backward from that record with the given state adjoint (gx_in_dev,
 * gu_dev: outputs it may overwrite; gx_out_dev must not alias gx_in_dev) for
 * the adjoint's layouts: one launch in the full layout, or the split launch
 * with each smaller contact cap at which the workgroups per CU step up (4 or
 * 8 robot contacts), each in two rounds of reps calls (the faster round
 * counts); keeps the fastest, or within 2 % of it the split with the most
 * robot contacts in its smaller layout (ms_get_backward_split reads it back),
 * and writes
 * it to split_c / split_r (0 / 0: no split) with its time per call.  Needs
 * the tape buffer (MS_E_STATE otherwise).  Cached like ms_autotune. */
ms_status ms_autotune_backward(ms_batch* b, const void* state_dev, const float* controls_dev,
                               const void* gx_out_dev, void* gx_in_dev, float* gu_dev, int32_t reps,
                               void* hip_stream, int32_t* split_c, int32_t* split_r, float* ms_per_step);

/* Autotune cache: a JSON-lines file (one object per tuned configuration:
 * "key", the choice, "ms_per_step"), read and appended by ms_autotune and
 * ms_autotune_backward; path null or "" turns caching off (the default).
 * The key is the device architecture (e.g. gfx950), "fwd" or "bwd", and a
 * 64-bit hash of the batch description, the scene-content counts, the CU
 * count, the force-output setting and the library's source version.
 * Processes sharing one file must not tune at the same time. */
ms_status ms_set_autotune_cache(ms_batch* b, const char* path);
/* The cache key of the forward (backward != 0: backward) tuning of this
 * batch, NUL-terminated into out (n bytes, 128 suffice), and whether the last
 * tuning took its choice from the cache (from_cache may be null). */
ms_status ms_autotune_key(const ms_batch* b, int32_t backward, char* out, size_t n, int32_t* from_cache);

/* One control step of every scene: state_out = T(state_in, controls).
 * state_out may alias state_in.  controls_dev: float32 [S][16]. */
ms_status ms_step(ms_batch* b, const void* state_in_dev, const float* controls_dev, void* state_out_dev,
                  void* hip_stream);

/* ms_step for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same control
 * step, bit for bit, in its one-launch form (the batch's persistent and
 * staging / culling choices; scenes in the order fixed at creation; no graph
 * replay and no split launch), calling no allocating routine.  Its scratch
 * -- the persistent work counter and, with MS_CTRL_ACTIONS, the control
 * step's PD targets -- is a device array of the library (1 MiB + 256 B per
 * device, held until the process ends), not the batch's scratch buffer; the
 * scene status words, force and gripper outputs still go to the batch's
 * buffers.  At most 16384 scenes (MS_E_INVALID beyond).  The calling thread's
 * current device must be the batch's.  Every call on one device shares that
 * array: calls that overlap on one device (other streams, other batches)
 * race; calls ordered on one stream do not.  Debug and phase-profile outputs
 * are not written. */
ms_status ms_step_noalloc(ms_batch* b, const void* state_in_dev, const float* controls_dev, void* state_out_dev,
                          void* hip_stream);

/* Vector-Jacobian product of exactly one ms_step (the adjoint of the step
 * T: S x A -> S of Sec. 3, recomputed internally): given dL/dstate_out
 * (float32, state layout), writes dL/dstate_in (state layout) and
 * dL/dcontrols (float32 [S][16]).  The contact set and the Gauss-Seidel
 * active set are those of the recomputed step; at a kink the derivative of
 * max(0, y) is taken as 0 at y = 0 and a disk projection exactly on the
 * boundary counts as inside.  Needs the batch to have been created with a
 * tape buffer of ms_query_sizes().tape bytes (else MS_E_STATE); the buffer is
 * scratch owned by the caller and overwritten by every call.
 * grad_state_in_dev may alias grad_state_out_dev.  Stream-ordered; OR-s the
 * MS_ST_* bits it meets into the scene status words. */
ms_status ms_step_backward(ms_batch* b, const void* state_in_dev, const float* controls_dev,
                           const void* grad_state_out_dev, void* grad_state_in_dev, float* grad_controls_dev,
                           void* hip_stream);

/* ms_step that also writes the step's record into record_dev (caller-owned
 * device memory of ms_query_sizes().record bytes, float-aligned): the state
 * at every substep start and at the end, each substep's contact list and the
 * pre-projection value of every Gauss-Seidel row update -- what the adjoint
 * of Sec. 3's step T needs, so that ms_step_backward_recorded need not run
 * the step again.  state_out_dev is the same, bit for bit, as ms_step's (it
 * may alias state_in_dev; record_dev may not alias either).  Runs the
 * step's fused launch whatever the schedule (no graph, no per-substep
 * launches).  Stream-ordered. */
ms_status ms_step_record(ms_batch* b, const void* state_in_dev, const float* controls_dev, void* state_out_dev,
                         void* record_dev, void* hip_stream);

/* ms_step_backward from the record ms_step_record wrote for the same
 * (state_in, controls): the same results bit for bit, without running the
 * step again and without the tape buffer (unless MS_SCHED_BWD_REFERENCE is
 * set: then the record is not read and the tape buffer is needed).  The
 * record is only read. */
ms_status ms_step_backward_recorded(ms_batch* b, const void* state_in_dev, const float* controls_dev,
                                    const void* record_dev, const void* grad_state_out_dev, void* grad_state_in_dev,
                                    float* grad_controls_dev, void* hip_stream);

/* Typed device views into a state buffer (no copy, no device work). */
ms_status ms_get_state(const ms_batch* b, const void* state_dev, ms_state_view* out);

/* Copy scene s of src_dev into state_dev wherever scene_mask_dev[s] != 0
 * (mask null: every scene). */
ms_status ms_set_state(ms_batch* b, void* state_dev, const void* src_dev, const uint8_t* scene_mask_dev,
                       void* hip_stream);

/* Contact-force outputs (the inputs of contact-based task predicates: the
 * robot's cumulative collision force and per-object contact forces, Sec. 4.3
 * and App. A).  When both pointers are non-null, every following ms_step
 * also writes, for its control step:
 *   robot_force_dev[S]       sum over the substeps of the robot's total
 *                            normal contact force (sum of its normal impulses
 *                            / h), N;
 *   body_force_dev[NF][4]    per free body, sum over the substeps of the force
 *                            the robot's contacts exert on it (x, y, z; then 0).
 * Divide by n_substeps for the mean over the control step.  Both null: off
 * (the default).  Device float32 buffers owned by the caller; only one
 * non-null is MS_E_INVALID.  Drops captured graphs. */
ms_status ms_set_force_outputs(ms_batch* b, float* robot_force_dev, float* body_force_dev);

/* Per-scene robot resets (the episode initialisation of App. A.1: rest pose
 * plus clipped Gaussian noise on the arm joints, base position and base
 * rotation).  For every scene with mask_dev[s] != 0 (mask null: all):
 * q[s][j] = base_dev[s][j] + clip(noise_dev[s][j], -clip_host[j], clip_host[j])
 * and qd[s][j] = 0; free bodies and doors / drawers are left as they are.
 * base_dev, noise_dev: device float32 [S][16] (the noise is drawn by the
 * caller, e.g. N(0, 0.1) arm and base position, N(0, 0.25) base yaw);
 * clip_host: host float32 [16].  Stream-ordered. */
ms_status ms_reset_robots(ms_batch* b, void* state_dev, const uint8_t* mask_dev, const float* base_dev,
                          const float* noise_dev, const float* clip_host, void* hip_stream);

/* Spawn check for rejection sampling of resets (spawn without collisions,
 * App. A.2): collide_dev[s] (uint8, device) = 1 where a robot sphere
 * penetrates (phi < 0) a plane (the base's spheres not the floor), a
 * furniture box, a door / drawer box or a free body; 0 otherwise.
 * Stream-ordered. */
ms_status ms_spawn_check(ms_batch* b, const void* state_dev, uint8_t* collide_dev, void* hip_stream);

/* ---------------------------------------------------------------- tasks
 * Success predicates, event labels and trajectory categories of the four
 * rearrangement subtasks (App. A.2 subtask definitions; App. A.3 event
 * labeling and success / failure modes), evaluated for every scene after
 * each control step.  Readings of points the appendix leaves open:
 *   - distances d are Euclidean norms in m;
 *   - is_static compares absolute values: max |qd_arm| <= 0.2 and |qd| <= 0.05
 *     for the base x, y and yaw DoFs;
 *   - the cumulative robot collision force C_t adds, per control step, the
 *     mean over its substeps of the robot's total normal contact force;
 *   - grasped(x): each of the two finger bodies presses on x with a normal
 *     force >= grasp_force in the last substep of the control step;
 *   - F_ee,x (contact events): the mean over the control step of the normal
 *     force the end effector's bodies exert on x; "contact" is 0 -> > 0;
 *   - an event index i_e is the position of e's latest occurrence in the
 *     event list (-1 absent); modes are tested in the order given with
 *     ms_task_categorize, the first that holds wins. */
enum { MS_TASK_PICK = 0, MS_TASK_PLACE = 1, MS_TASK_OPEN = 2, MS_TASK_CLOSE = 3 };

/* the robot as the predicates see it (body / DoF indices of the model) */
typedef struct {
  int32_t ee_body;          /* body carrying the end effector */
  int32_t base_body;        /* body whose frame is the base frame */
  int32_t base_x, base_y, base_yaw;  /* DoFs of the base's x, y and yaw velocity */
  int32_t arm0, narm;       /* arm DoFs arm0 .. arm0 + narm - 1 */
  int32_t torso;            /* torso DoF, -1: none */
  int32_t finger_l, finger_r;        /* finger bodies (grasp test) */
  uint32_t ee_bodies;       /* bit b set: body b belongs to the end effector */
  float ee_offset[3];       /* end-effector point in ee_body's frame */
  float ee_rest[3];         /* its rest position in the base frame (the caller's
                               choice, e.g. the point at q_rest) */
  float q_rest[16];         /* resting joint positions */
  float grasp_force;        /* N */
} ms_task_robot;

/* one scene's subtask (device array [S]) */
typedef struct {
  int32_t kind;             /* MS_TASK_* */
  int32_t target;           /* scene-local free body (pick, place) or door / drawer joint (open, close) */
  float goal[3];            /* place: goal position, world */
  float open_frac;          /* open: 0.75 for a fridge, 0.9 otherwise */
} ms_task;

/* indicator bits of ms_episode.ind (values after the last evaluated step) */
enum {
  MS_IND_GRASPED = 1u, MS_IND_SUCCESS = 2u, MS_IND_OPEN = 4u /* open (open task) / closed (close task) */,
  MS_IND_SLIGHT = 8u /* slightly opened / slightly closed */, MS_IND_AT_GOAL = 16u, MS_IND_CONTACT = 32u,
  MS_IND_EXCESSIVE = 64u /* C_t above the subtask's limit: the failure condition */
};
/* event codes, in the order the appendix evaluates them per step */
enum { MS_EV_PICK_CONTACT = 0, MS_EV_PICK_GRASPED, MS_EV_PICK_DROPPED, MS_EV_PICK_SUCCESS, MS_EV_PICK_EXCESSIVE };
enum {
  MS_EV_PLACE_GRASPED = 0, MS_EV_PLACE_AT_GOAL, MS_EV_PLACE_RELEASED_AT_GOAL, MS_EV_PLACE_RELEASED_OUTSIDE,
  MS_EV_PLACE_LEFT_GOAL, MS_EV_PLACE_SUCCESS, MS_EV_PLACE_EXCESSIVE
};
enum { MS_EV_OPEN_CONTACT = 0, MS_EV_OPEN_OPENED, MS_EV_OPEN_SLIGHT, MS_EV_OPEN_CLOSED, MS_EV_OPEN_SUCCESS,
       MS_EV_OPEN_EXCESSIVE };
enum { MS_EV_CLOSE_CONTACT = 0, MS_EV_CLOSE_CLOSED, MS_EV_CLOSE_SLIGHT, MS_EV_CLOSE_OPENED, MS_EV_CLOSE_SUCCESS,
       MS_EV_CLOSE_EXCESSIVE };

#define MS_EP_LIST 16
/* per-scene episode record (device array [S], caller-owned; written by
 * ms_task_begin / ms_task_update) */
typedef struct {
  float cumcol;             /* C_t, N */
  float aq0;                /* door / drawer position at the episode start */
  float d0;                 /* place: object-goal distance at the start */
  uint32_t ind;             /* MS_IND_* bits of the last evaluated step */
  int32_t t;                /* control steps evaluated since the start */
  int32_t n;                /* events so far (list keeps the first MS_EP_LIST) */
  int32_t last[8];          /* list index of each event code's latest occurrence, -1: none */
  uint8_t list[MS_EP_LIST]; /* event codes in chronological order */
} ms_episode;

/* predicate values written per scene when pred_dev is non-null: float32 [S][8] */
enum { MS_PRED_D_EE = 0, MS_PRED_J_ARM, MS_PRED_J_TORSO, MS_PRED_QD_MAX, MS_PRED_D_GOAL, MS_PRED_AQ,
       MS_PRED_F_EE, MS_PRED_F_FINGER };

/* Sets the robot description used by the task calls and the gripper outputs
 * (copied; host struct).  Indices are checked against every model of the
 * batch.  Drops captured graphs. */
ms_status ms_set_task_robot(ms_batch* b, const ms_task_robot* robot_host);

/* Gripper contact outputs: when grip_dev is non-null, every following
 * ms_step writes float32 [NF + NA][2]: rows 0 .. NF-1 the free bodies, rows
 * NF .. NF+NA-1 the door / drawer joints; [0] the normal force the end
 * effector's bodies exert on it, summed over the substeps (N; divide by
 * n_substeps for the mean), [1] the smaller of the two fingers' normal
 * forces on it in the last substep (N).  Needs ms_set_task_robot first
 * (else MS_E_STATE).  Null: off.  Drops captured graphs. */
ms_status ms_set_grip_outputs(ms_batch* b, float* grip_dev);

/* Starts the episodes of the scenes with mask_dev[s] != 0 (null: all) at
 * state_dev: C = 0, t = 0, empty event list, the indicators of the start
 * state (grip_dev as written by ms_set_grip_outputs, or null: no contact and
 * not grasped), aq0 and d0.  pred_dev: optional predicate values.
 * Stream-ordered; MS_E_STATE without ms_set_task_robot; an out-of-range task
 * kind or target, or an open / close target without joint limits, leaves
 * that scene's record with ind = 0xffffffff (also after ms_task_update). */
ms_status ms_task_begin(ms_batch* b, const void* state_dev, const ms_task* tasks_dev, const float* grip_dev,
                        ms_episode* ep_dev, const uint8_t* mask_dev, float* pred_dev, void* hip_stream);

/* Evaluates the predicates after one control step (state_dev the state it
 * produced, robot_force_dev and grip_dev its force outputs; grip_dev may be
 * null), adds the step's events to every scene's list in the appendix's
 * order, and advances t.  Stream-ordered. */
ms_status ms_task_update(ms_batch* b, const void* state_dev, const ms_task* tasks_dev, const float* robot_force_dev,
                         const float* grip_dev, ms_episode* ep_dev, float* pred_dev, void* hip_stream);

/* Success / failure mode of every scene's trajectory (App. A.3), int32
 * mode_dev[S]: the appendix's roman numeral (pick: i-iv success, v-ix
 * failure; place: i-v success, vi-xii failure; open and close: i-iii
 * success, iv-ix failure) as 1, 2, ...; 0 when no mode's condition holds.
 * Modes are tested in this order, the first that holds wins:
 *   pick success: iv, iii, i, ii; failure: v, vi, vii, viii, ix;
 *   place success: v, i, ii, iii, iv; failure: vi, vii, viii, ix, x, xi, xii;
 *   open / close success: iii, i, ii; failure: iv, v, vi, vii, viii, ix.
 * The success modes "success then excessive collisions" are read with
 * e_excessive in the list.  Stream-ordered. */
ms_status ms_task_categorize(ms_batch* b, const ms_task* tasks_dev, const ms_episode* ep_dev, int32_t* mode_dev,
                             void* hip_stream);

/* Synchronise and read the per-scene status words of the last step
 * (bits MS_ST_*) into status_host[S].  Returns MS_E_NUMERIC if any scene
 * has MS_ST_NONFINITE or MS_ST_DEGENERATE set, MS_OK otherwise. */
ms_status ms_scene_status(const ms_batch* b, uint32_t* status_host);

/* Diagnostics of the last ms_step (synchronises): per scene and substep the
 * number of contacts, the number of robot-owned contacts and the 64-bit sum
 * of mixed contact keys (owner key << 32 | target key, mixed by the
 * SplitMix64 finaliser), written as uint32 [S][n_substeps][4]:
 * count, robot count, key-sum low, key-sum high.  Enabled by ms_enable_debug. */
ms_status ms_enable_debug(ms_batch* b, int32_t on);
ms_status ms_debug_contacts(const ms_batch* b, uint32_t* out_host);

/* Per-phase shader-clock cycles of the last ms_step, summed over its
 * substeps (synchronises): uint64 [S][8] for the phases drive+kinematics,
 * contacts, dynamics, rows, level schedule, Gauss-Seidel, integration, and
 * load/store.  Enabled by ms_enable_phase_profile (adds clock reads). */
ms_status ms_enable_phase_profile(ms_batch* b, int32_t on);
ms_status ms_phase_cycles(const ms_batch* b, unsigned long long* out_host);

/* Measurement probes: the achievable rates of the device as this library is
 * built, the second denominators of the step's rooflines next to the
 * published peaks (8 TB/s HBM, 157.3 TFLOP/s FP32 vector).  Both enqueue one
 * kernel on hip_stream; the caller times it (e.g. with HIP events).
 *   ms_probe_copy: a streaming copy of `bytes` (multiple of 16) from src_dev
 *     to dst_dev (both 16-byte aligned, not overlapping); 2 x bytes of HBM
 *     traffic when the buffers exceed the on-chip caches.
 *   ms_probe_fma: `blocks` workgroups of 256 lanes, each lane running eight
 *     independent FP32 FMA chains of 16 x iters FMAs; out_dev: a device
 *     scratch of 1024 floats (written only in a case that never occurs);
 *     *flops (host, may be null) receives the FLOPs the launch executes
 *     (2 per FMA).
 * Invalid sizes or alignment return MS_E_INVALID before anything is enqueued. */
ms_status ms_probe_copy(const void* src_dev, void* dst_dev, size_t bytes, void* hip_stream);
ms_status ms_probe_fma(void* out_dev, int32_t blocks, int32_t iters, void* hip_stream, double* flops);

/* Message of the last failed call on this thread (empty if none). */
const char* ms_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MS_PHYS_H */
