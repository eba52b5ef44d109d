// ms_backward.h -- launch interface of the adjoint (vector-Jacobian product)
// of one control step; the arithmetic is in ms_adjoint.h.
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
  float* ws;              // workspace, w.total floats per slot, interleaved with stride `stride`
  int S, NF, stride;
  msa::Prm pr;
  msa::WS w;
};

inline int bwd_stride(int S) { return (S + 63) & ~63; }
inline msa::WS bwd_layout(int fmax, int ntmax, int ccap, int rcap, int K, int nsub) {
  return msa::ws_layout(fmax, ntmax, ccap, rcap, K, nsub);
}
void launch_step_bwd(const BwdArgs& a, hipStream_t st);

}  // namespace msk
