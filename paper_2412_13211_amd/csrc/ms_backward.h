// ms_backward.h -- launch interface of the adjoint (vector-Jacobian product)
// of one control step; the arithmetic is in ms_adjoint.h.
//
// Two kernels compute it:
//   k_step_bwd_wave  one wavefront per scene.  It reads the record of the
//                    control step that the forward kernel writes in record
//                    mode (substep states, contact lists, pre-projection
//                    values of the Gauss-Seidel updates), keeps the scene's
//                    adjoint workspace in LDS and reverses the Gauss-Seidel
//                    sweeps level by level (rows of one level touch disjoint
//                    bodies, so they are reversed in parallel);
//   k_step_bwd       one lane per scene, recomputing everything itself with
//                    the workspace interleaved in global memory (the
//                    reference the wavefront kernel is tested against).
#pragma once
#include "ms_adjoint.h"

namespace msk {

struct BwdArgs {
  const DModel* models;
  const DScene* scenes;
  const DFree* free;
  const float* statics;
  const float4* planes;
  const DAux* aux;
  const int* order;       // scene processing order (slot -> scene)
  const float* x;         // state in
  const float* u;         // controls [S][16]
  const float* gxo;       // adjoint of the state out
  float* gxi;             // adjoint of the state in (may alias gxo)
  float* gu;              // adjoint of the controls [S][16]
  uint32_t* status;       // [S], bits OR-ed in
  unsigned long long* cycles;  // [S][8] shader-clock cycles per phase of the wavefront kernel, or null
  float* ws;              // lane kernel: workspace, w.total floats per slot, interleaved with stride `stride`
  const float* rec;       // wavefront kernel: forward record, RL.total floats per scene
  RecLayout RL;
  int S, NF, stride;
  msa::Prm pr;
  msa::WS w;              // lane kernel: global layout; wavefront kernel: LDS layout
  // wavefront kernel, with the order from launch_bwd_order: 0 reverses
  // every scene, slot by slot; 1 the scenes after the first *n_over of the
  // order (those whose contact lists fit the smaller layout), slot by slot;
  // 2 the first *n_over, a fixed grid looping over them
  int fit_mode;
  const int* n_over;
};

inline int bwd_stride(int S) { return (S + 63) & ~63; }
void launch_step_bwd(const BwdArgs& a, hipStream_t st);
void launch_step_bwd_wave(const BwdArgs& a, size_t lds_bytes, int grid, hipStream_t st);
// one wavefront waiting about `ticks` of the 100 MHz wall clock
void launch_delay(long long ticks, hipStream_t st);
// the adjoint's scene order from the record (scenes overflowing fit_c
// contacts or fit_r robot contacts in some substep first, fit_c = 0: none;
// each group by decreasing estimated cost) and the size of the first group;
// slot: [S] ints of scratch
void launch_bwd_order(const float* rec, const RecLayout& RL, int S, int nsub, int fit_c, int fit_r, int* slot,
                      int* order, int* n_over, hipStream_t st);
const void* step_bwd_wave_ptr();

// status bit set when the record and the recomputed joint-limit rows disagree
constexpr uint32_t MS_ST_RECORD = 16u;

}  // namespace msk
