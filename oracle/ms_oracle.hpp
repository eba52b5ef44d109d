// ms_oracle.hpp -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow FP64 CPU reference of one batched rigid-body control step and
// of its vector-Jacobian product.  Only the tests, the package smoke check and
// the benchmark's CPU-baseline leg may load it; the GPU library shares no code,
// header or table with it.
//
// What it computes (the paper delegates its physics to a GPU simulator and
// describes no solver: Sec. 1 and Sec. 4.1; it fixes 100 Hz simulation under
// 20 Hz control in Sec. 4.2).  Each scene is advanced by n_sub substeps of:
//   1. drive: joint torques held over the control step, or implicit joint PD,
//      plus rotor inertia and implicit viscous damping (diagonal
//      a = armature + h (kd + damping) + h^2 kp added to the mass matrix);
//   2. forward kinematics of every articulation (world-frame spatial algebra);
//   3. sphere-decomposed contact generation against planes, axis-aligned
//      boxes, articulated boxes and free boxes / spheres (brute force over all
//      allowed pairs, emitted when the signed distance is below the margin);
//   4. unconstrained velocities: CRBA mass matrix, RNEA bias, Cholesky solve;
//      free bodies by Newton-Euler with an explicit gyroscopic term;
//   5. contact rows (normal + two tangents of the Duff et al. 2017 basis),
//      effective masses and speculative / Baumgarte biases;
//   6. K sweeps of projected Gauss-Seidel in the canonical row order, with an
//      isotropic friction disk;
//   7. semi-implicit Euler (quaternion exponential map for free bodies).
// The result is defined as the K-sweep iterate from zero impulses; it is not
// "the" LCP solution.  Every silent point of the paper is read as stated in
// the design notes that accompany this repository.
#pragma once
#include <stdint.h>

extern "C" {

// Host arrays of one scene batch (layout produced by the scene generator).
typedef struct {
  int32_t n_scenes, n_models;
  const int32_t* model_nb;        // [M]
  const int32_t* model_parent;    // [M][16]
  const int32_t* model_jtype;     // [M][16] 0 revolute, 1 prismatic
  const float* model_axis;        // [M][16][3]
  const float* model_xt_rot;      // [M][16][4] wxyz
  const float* model_xt_pos;      // [M][16][3]
  const float* model_mass;        // [M][16]
  const float* model_com;         // [M][16][3]
  const float* model_inertia;     // [M][16][6] xx yy zz xy xz yz
  const float* model_kp;          // [M][16]
  const float* model_kd;          // [M][16]
  const int32_t* model_veldof;    // [M][16]
  const float* model_armature;    // [M][16]
  const float* model_damping;     // [M][16]
  const int32_t* model_act_kind;  // [M][16] normalized-action channel
  const float* model_act_scale;   // [M][16]
  const int32_t* model_nsph;      // [M]
  const int32_t* model_sph_body;  // [M][128]
  const float* model_sph;         // [M][128][4]
  const int32_t* model_sph_flags; // [M][128]
  const int32_t* scene_model;     // [S]
  const int32_t* free_off;        // [S+1]
  const int32_t* static_off;      // [S+1]
  const int32_t* plane_off;       // [S+1]
  const int32_t* aux_off;         // [S+1]
  const float* scene_hold;        // [S][16]
  const int32_t* free_type;       // [NF]
  const float* free_size;         // [NF][3]
  const float* free_mass;         // [NF]
  const float* free_inertia;      // [NF][3]
  const float* static_box;        // [NS][6]
  const float* plane;             // [NP][4]
  const int32_t* aux_type;        // [NA]
  const float* aux_rot;           // [NA][4]
  const float* aux_pos;           // [NA][3]
  const float* aux_axis;          // [NA][3]
  const float* aux_box;           // [NA][6]
  const float* aux_mass;          // [NA]
  const float* aux_inertia;       // [NA][3]
  const float* aux_limit;         // [NA][2]
} or_scene;

typedef struct {
  double h, mu, baumgarte, margin, gravity[3];
  int32_t n_sub, pgs_iters, control_mode;
  int32_t contact_cap;        // contacts kept per scene and substep (first in canonical order)
  int32_t robot_contact_cap;  // robot-owned contacts kept per scene and substep; the
                              // robot's later contacts are dropped before the total cap
} or_params;

// Optional per-scene diagnostics (any pointer may be null).
typedef struct {
  uint32_t* status;        // [S] bit0 non-finite, bit1 contact overflow, bit2 degenerate row,
                           // bit3 robot contact overflow
  int32_t* n_contacts;     // [S][n_sub]
  uint64_t* key_hash;      // [S][n_sub] sum of mixed contact keys
  uint64_t* act_hash;      // [S][n_sub] hash of the PGS active set (clamps / projections)
  int32_t dump_cap;        // contacts dumped per scene (last substep)
  uint64_t* dump_keys;     // [S][dump_cap]
  double* dump_phi;        // [S][dump_cap]
  double* dump_lambda;     // [S][dump_cap][3] final impulses
  double* dump_y;          // [S][pgs_iters][dump_cap][3] pre-projection value of every
                           // Gauss-Seidel row update in the last substep (limit rows
                           // first, then contacts; normal, tangent 1, tangent 2)
  double* robot_force;     // [S] sum over substeps of robot-owned normal impulses / h
  double* robot_body_force;  // [NF][3] sum over substeps of the force the robot's
                             // contacts exert on each free body (impulse / h)
  uint32_t grip_ee;          // robot bodies of the end effector (bit mask)
  int32_t grip_finger_l, grip_finger_r;  // finger bodies
  double* grip;              // [NF + NA][2] end-effector normal force on each free body /
                             // door-drawer joint summed over substeps; smaller finger
                             // normal force on it in the last substep
} or_debug;

// One control step for every scene.  x_in / x_out: flat state
// (q[S][16], qd[S][16], free[NF][16], aux[NA][4]); u: controls [S][16].
// x_out may alias x_in.  threads <= 0 uses all hardware threads.
int or_step(const or_scene* sc, const or_params* pr, const double* x_in, const double* u,
            double* x_out, int threads, or_debug* dbg);

// The same control step evaluated with float intermediates (FP32 error floor).
int or_step_f32(const or_scene* sc, const or_params* pr, const double* x_in, const double* u,
                double* x_out, int threads, or_debug* dbg);

// Vector-Jacobian product of one control step: given gx_out = dL/dx_out,
// returns dL/dx_in (gx_in) and dL/du (gu), by reverse-mode differentiation of
// exactly the arithmetic of or_step.
int or_vjp(const or_scene* sc, const or_params* pr, const double* x_in, const double* u,
           const double* gx_out, double* gx_in, double* gu, int threads);

// Jacobian-vector product (forward mode): dx_out = J_x dx_in + J_u du.
int or_jvp(const or_scene* sc, const or_params* pr, const double* x_in, const double* u,
           const double* dx_in, const double* du, double* dx_out, int threads);

// Floating-point operation count of one control step per scene (adds, muls,
// divides, square roots and transcendental calls each count as one).
int or_flops(const or_scene* sc, const or_params* pr, const double* x_in, const double* u,
             double* flops_per_scene);

// Spawn check of a reset: collide[s] = 1 where a robot sphere penetrates
// (phi < 0) a plane (the base's spheres not the first plane), a furniture
// box, a door / drawer box or a free body; brute force over every pair.
// min_phi (may be null): per scene the smallest signed distance over those pairs.
int or_spawn_check(const or_scene* sc, const double* x, int32_t* collide, double* min_phi, int threads);

// ---- single-function probes used by the closed-form tests ----
// Robot model m: world sphere centres [nsph][3] and body origins [nb][3].
int or_fk(const or_scene* sc, int model, const double* q, double* sph_out, double* origin_out,
          double* rot_out);
// Mass matrix (CRBA, no armature) [16][16] and bias C(q, qd) [16] (RNEA, gravity g).
int or_dynamics(const or_scene* sc, int model, const double* q, const double* qd, const double* g,
                double* M_out, double* C_out);
// Forward dynamics by FP64 articulated-body algorithm (world frame) with
// armature: qdd = (M + diag(arm))^-1 (tau - C).
int or_aba(const or_scene* sc, int model, const double* q, const double* qd, const double* tau,
           const double* arm, const double* g, double* qdd_out);
// Kinetic energy from link velocities: sum 1/2 m |v_c|^2 + 1/2 w^T I w.
double or_kinetic_energy(const or_scene* sc, int model, const double* q, const double* qd);
// Sphere (c, r) vs primitive: kind 0 plane (n, d), 1 box (centre, half, quat wxyz),
// 2 sphere (centre, radius).  Writes phi, n[3], p[3].
int or_pair(int kind, const double* c, double r, const double* prim, double* out7);
// Duff et al. orthonormal basis from a unit normal: t1[3], t2[3].
void or_onb(const double* n, double* t1, double* t2);
// Quaternion exponential-map update: Q' = normalize(exp(h w) (x) Q).
void or_quat_update(const double* Q, const double* w, double h, double* out);

}  // extern "C"
