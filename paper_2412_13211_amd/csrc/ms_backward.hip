// ms_backward.hip -- the adjoint of one control step on gfx950: one lane per
// scene (scenes taken in the cost-sorted order so that a wavefront holds
// scenes of similar size), workspace interleaved across the lanes.
#include "ms_backward.h"

namespace msk {

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

}  // namespace msk
