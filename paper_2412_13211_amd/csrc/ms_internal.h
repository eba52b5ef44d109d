// ms_internal.h -- device-side data layout of the batched physics step (gfx950).
//
// The scene description is packed once into one device buffer ("params"):
//   [DModel x M][DScene x S][DFree x NF][static boxes 6 floats x NS]
//   [planes float4 x NP][DAux x NA][scene order int x S]
// Every scene is processed by one 64-lane wavefront (one workgroup); all of
// a scene's working data lives in that workgroup's LDS for the whole control
// step, so HBM traffic is the state in/out, the controls and the scene
// description.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msk {

constexpr int ND = 16;        // padded robot DoFs (one DoF per body)
constexpr int SPH = 128;      // max robot collision spheres
constexpr int WAVE = 64;
constexpr int AMAX = 4;       // max door / drawer joints per scene
constexpr int PMAX = 8;       // max planes per scene
constexpr int FMAXL = 58;     // max free bodies per scene (node ids 1 + AMAX + f < 63)

struct DModel {
  int nb, nsph, pad0, pad1;
  int parent[ND];
  int jtype[ND];
  int veldof[ND];
  int anc[ND];          // bit k set: body k is body i or one of its ancestors
  float axis[ND][3];
  float xtR[ND][9];
  float xtp[ND][3];
  float mass[ND];
  float com[ND][3];
  float Ic[ND][6];      // xx yy zz xy xz yz about the COM, body axes
  float kp[ND], kd[ND], arm[ND], damp[ND];
  int act_kind[ND];     // normalized-action channel of each DoF
  float act_scale[ND];
  int act_x, act_yaw;   // DoF of the base forward action and of the base heading (-1: none)
  int pad2, pad3;
  float4 sph[SPH];      // centre (body frame), radius
  int sph_body[SPH];
  int sph_flags[SPH];
  int sph_first[ND];    // spheres of body i: [sph_first, sph_first + sph_count)
  int sph_count[ND];
  float4 bsph[ND];      // bounding sphere of body i's spheres (body frame centre, radius)
};

struct DScene {
  int model, f0, nf, s0, ns, p0, np, a0, na, nown, cost, pad;
  float hold[ND];
};

struct DFree {
  int type;            // 0 box, 1 sphere
  float half[3];       // half extents or (radius, 0, 0)
  float mass;
  float Ib[3];         // principal moments
};

struct DAux {
  int type;            // 0 revolute, 1 prismatic
  float R0[9];         // joint frame rotation (world)
  float p0[3];
  float axis[3];
  float bc[3];         // box centre in the moving frame
  float bh[3];         // half extents
  float mass;
  float Ib[3];
  float lo, hi;
  int has_limit;
  int pad;
};

// Offsets (in floats) of the regions of one scene's LDS block.
struct LdsLayout {
  int fmax, smax, ccap, rcap, owners, ntmax;
  int robot, sph, fr, aux, stat, plane, own, con, rows, dyn, cmask, nch, lvl, cand, frc, total;
};

__host__ __device__ inline int lds_align4(int x) { return (x + 3) & ~3; }

// Robot block (persistent over a substep): q qd tau arm u [5*16]; R[16*9]
// p[16*3] s[16*6]; Minv[16*16].
constexpr int ROBOT_FLOATS = 5 * ND + ND * 9 + ND * 3 + ND * 6 + ND * ND;
// Dynamics scratch (only inside the dynamics phase, which runs before the
// contacts are generated, so it shares the space of the contact list and the
// robot contact rows): per body COM, mass and world inertia about the COM
// [16*BI_FLOATS], velocity-product accelerations and body forces [2*16*6],
// M~ [16*16], tau - C [16].
constexpr int BI_FLOATS = 11;       // odd stride
constexpr int DSUM_FLOATS = 17;     // odd stride: a_i (6), composite inertia (10) / subtree force (6), G_i (6)
constexpr int DYN_FLOATS = ND * BI_FLOATS + 2 * ND * 6 + ND * ND + ND + ND * DSUM_FLOATS;
constexpr int FREE_FLOATS = 37;     // per free body (odd stride: conflict-free LDS banks)
constexpr int FSTR = FREE_FLOATS;
constexpr int AUX_FLOATS = 32;      // per aux joint
constexpr int FRC_FLOATS = 5;       // per free body, force-output mode: force on it (3), end-effector and finger force
constexpr int CON_FLOATS = 17;      // per contact (odd stride)
constexpr int CSTR = CON_FLOATS;
constexpr int ROW_FLOATS = 3 * ND;  // per robot contact: J [3][16] (normal, two tangents)

__host__ __device__ inline LdsLayout make_layout(int fmax, int smax, int ccap, int rcap, int stage_static,
                                                 int force = 0, int nsph = SPH) {
  LdsLayout L;
  L.fmax = fmax;
  L.smax = stage_static ? smax : 0;
  L.ccap = ccap;
  L.rcap = rcap;
  L.owners = fmax * 8;
  L.ntmax = PMAX + smax + AMAX + fmax;
  int o = 0;
  L.robot = o; o += lds_align4(ROBOT_FLOATS);
  L.sph = o;   o += nsph * 4;   // world sphere centres and radii of the robot
  L.fr = o;    o += lds_align4((fmax + 1) * FREE_FLOATS);  // + a zero record (static side)
  L.aux = o;   o += AMAX * AUX_FLOATS;
  L.stat = o;  o += lds_align4(L.smax * 6);
  L.plane = o; o += PMAX * 4;
  L.own = o;   o += lds_align4((L.owners + 1) / 2);        // uint16 owner table
  L.con = o;
  L.dyn = o;
  L.rows = o + lds_align4(ccap * CON_FLOATS);
  // the culling masks (per robot or free body and 64-target chunk, 64 bits)
  // live in the robot rows' space: the contact phase fills them before the
  // rows phase builds the rows
  L.nch = (L.ntmax + WAVE - 1) / WAVE;
  L.cmask = L.rows;
  {
    // masks, then the robot's or the free bodies' bounding spheres (4 floats each)
    const int rw = lds_align4(rcap * ROW_FLOATS),
              mk = lds_align4((fmax > ND ? fmax : ND) * L.nch * 2) + (fmax > ND ? fmax : ND) * 4;
    const int cr = lds_align4(ccap * CON_FLOATS) + (rw > mk ? rw : mk);
    o += cr > DYN_FLOATS ? cr : DYN_FLOATS;
  }
  // level schedule: uint16 group offsets and robot row per level [ccap + 2]
  // each, the groups by level (uint32) [ccap], each group's level [ccap] and
  // first row [ccap + 1] (uint16)
  L.lvl = o;   o += lds_align4((6 * ccap + 5 + 1) / 2);
  // two uint16 candidate lists; after the contact phase the level schedule's
  // per-node row masks (64-bit, per node and 64-row chunk)
  {
    const int masks = (1 + AMAX + fmax) * ((ccap + WAVE - 1) / WAVE) * 2;
    L.cand = o;  o += lds_align4(L.ntmax > masks ? L.ntmax : masks);
  }
  L.frc = o;   o += force ? lds_align4(fmax * FRC_FLOATS) : 0;  // force-output accumulators
  L.total = o;
  return L;
}

// Record of one control step written by the forward kernel for the adjoint
// (floats, per scene, contiguous): the state at every substep start and at the
// end (each 32 + 16 fmax + 4 AMAX floats: q, qd, free bodies, door/drawer),
// per substep the contact list (header NC, NL, NR, 0, then NC records of
// CSTR floats), and per substep the pre-projection value of every
// Gauss-Seidel row update (sweep-major, 3 slots per list entry).
struct RecLayout {
  int ss, con, cstride, tape, tsw, total;
};
__host__ __device__ inline RecLayout rec_layout(int fmax, int ccap, int K, int nsub) {
  RecLayout r;
  r.ss = 32 + 16 * fmax + 4 * AMAX;
  r.con = (nsub + 1) * r.ss;
  r.cstride = 4 + ccap * CSTR;
  r.tape = r.con + nsub * r.cstride;
  r.tsw = 3 * ccap;
  r.total = (r.tape + nsub * K * r.tsw + 3) & ~3;
  return r;
}

// Per-scene grid over the furniture (xy, SGRID x SGRID cells): a header of
// four floats (x0, y0, 1 / cell width, 1 / cell depth) then per cell a bit
// mask over the scene's furniture boxes (sg_nw 64-bit words) of the boxes
// whose xy extent (grown by 1 mm) overlaps the cell.  A query over the cells
// a sphere's xy extent overlaps finds every box it can come near.
constexpr int SGRID = 8;
__host__ __device__ inline int sgrid_floats(int nw) { return 4 + SGRID * SGRID * nw * 2; }

struct KArgs {
  const DModel* models;
  const DScene* scenes;
  const DFree* free;
  const float* statics;
  const float* sgrid;      // [S][sgrid_floats(sg_nw)]
  int sg_nw;
  const float4* planes;
  const DAux* aux;
  const int* order;        // scene processing order (cost-sorted)
  const float* x_in;
  float* x_out;
  const float* u;
  uint32_t* status;        // [S]
  uint32_t* debug;         // [S][n_sub][4] or null
  unsigned long long* phase_cycles;  // [S][8] shader-clock cycles per phase, or null
  int* queue;              // work counter (persistent schedule)
  int* cost;               // [S] each scene's time in the step (shader clock / 16), for the next step's order, or null
  int* maxc;               // [S] largest contact count | largest robot-contact count << 16 over the step's substeps, or null
  // split launches (persistent only): 0 takes every position of the order;
  // 1 the positions from *n_over on, leaving a scene whose contact lists
  // overflow the launch's layout whole to the retry list; 2 the first
  // *n_over positions; 3 the retry list.  Work counters queue[0], [1], [2].
  int fit_mode;
  const int* n_over;
  int* retry;              // [1 + S]: count, then scene indices
  int S, NF, NA;
  int n_sub, sub0, n_sub_total;  // substeps in this launch, index of the first, substeps per control step
  int K, mode, ccap, rcap;
  int persistent, stage_static, cull;
  float h, mu, beta, margin;
  float g[3];
  LdsLayout L;
  float* rec;              // record of the control step for the adjoint, or null
  RecLayout RL;
  float* frc_robot;        // [S] contact-force outputs, or null
  float* frc_body;         // [NF][4]
  float* grip;             // [NF + NA][2] gripper contact outputs, or null
  uint32_t grip_ee;        // robot bodies of the end effector (bit mask)
  int grip_fl, grip_fr;    // finger bodies
};

void launch_step(const KArgs& a, int grid, size_t lds_bytes, hipStream_t st);
void launch_reset_queue(int* q, hipStream_t st);
// order = the scenes by decreasing cost (a scene time; keyed by its logarithm),
// those whose last contact counts (maxc) do not leave 8 contacts and 2 robot
// contacts of room under (fit_c, fit_r) first (fit_c = 0: none), *n_over
// their count; also zeroes the work counters q[0..2] and the retry count
// (each pointer may be null)
void launch_cost_order(const int* cost, const int* maxc, int S, int fit_c, int fit_r, int* order, int* n_over, int* q,
                       int* retry, hipStream_t st);
void launch_actions(const DModel* models, const DScene* scenes, const float* x, const float* a, float* tgt, int S,
                    hipStream_t st);
void launch_actions_bwd(const DModel* models, const DScene* scenes, const float* x, const float* a,
                        const float* gtgt, float* ga, float* gx, int S, hipStream_t st);
void launch_masked_copy(float* dst, const float* src, const uint8_t* mask, int S, int NF, int NA,
                        const int* free_off, const int* aux_off, hipStream_t st);
const void* step_kernel_ptr();
const void* step_rec_kernel_ptr();
const void* step_frc_kernel_ptr();
const void* spawn_check_kernel_ptr();
void launch_spawn_check(const KArgs& a, uint8_t* collide, size_t lds_bytes, hipStream_t st);
void launch_reset_robots(float* x, const uint8_t* mask, const float* base, const float* noise, const float* clip,
                         int S, hipStream_t st);

}  // namespace msk
