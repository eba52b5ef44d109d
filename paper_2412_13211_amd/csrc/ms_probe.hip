// ms_probe.hip -- measurement probes: the achievable HBM copy bandwidth and
// FP32 FMA rate of the device this library runs on, as built (the second
// denominators of the step's rooflines next to the published peaks).
#include <hip/hip_runtime.h>

#include "../../include/ms_phys.h"
#include "ms_pack.h"

namespace {

// Streaming copy, 16 B per lane per access, grid-stride.
__global__ void k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

// Eight independent FMA chains per lane (enough to cover the VALU's
// dependency latency); the result is stored only when it equals a value it
// never takes, so the chains stay live without memory traffic.
__global__ void k_probe_fma(float* out, int iters, float seed) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  float a0 = seed + t * 1e-9f, a1 = a0 + 1e-3f, a2 = a0 + 2e-3f, a3 = a0 + 3e-3f;
  float a4 = a0 + 4e-3f, a5 = a0 + 5e-3f, a6 = a0 + 6e-3f, a7 = a0 + 7e-3f;
  const float m = 0.999999f, c = 1e-6f;
#pragma unroll 1
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      a0 = fmaf(a0, m, c); a1 = fmaf(a1, m, c); a2 = fmaf(a2, m, c); a3 = fmaf(a3, m, c);
      a4 = fmaf(a4, m, c); a5 = fmaf(a5, m, c); a6 = fmaf(a6, m, c); a7 = fmaf(a7, m, c);
    }
  }
  const float s = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
  if (s == -1.2345f) out[t & 1023] = s;
}

}  // namespace

extern "C" {

ms_status ms_probe_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
  using mspack::fail;
  if (!src || !dst) return fail(MS_E_INVALID, "null argument");
  if (bytes % 16 != 0 || ((uintptr_t)src % 16) != 0 || ((uintptr_t)dst % 16) != 0)
    return fail(MS_E_INVALID, "copy probe: bytes and both pointers must be 16-byte aligned");
  const size_t n4 = bytes / 16;
  if (n4 == 0) return MS_OK;
  const int block = 256;
  const size_t want = (n4 + block - 1) / block;
  const int grid = (int)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(block), 0, static_cast<hipStream_t>(hip_stream),
                     static_cast<const float4*>(src), static_cast<float4*>(dst), n4);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MS_E_HIP, "copy probe: %s", hipGetErrorString(e));
  return MS_OK;
}

ms_status ms_probe_fma(void* out_dev, int32_t blocks, int32_t iters, void* hip_stream, double* flops) {
  using mspack::fail;
  if (!out_dev) return fail(MS_E_INVALID, "null argument");
  if (blocks <= 0 || iters <= 0) return fail(MS_E_INVALID, "FMA probe: blocks and iters must be positive");
  const int block = 256;
  hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(block), 0, static_cast<hipStream_t>(hip_stream),
                     static_cast<float*>(out_dev), iters, 1.0f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MS_E_HIP, "FMA probe: %s", hipGetErrorString(e));
  if (flops) *flops = 2.0 * 8 * 16 * (double)iters * (double)blocks * block;
  return MS_OK;
}

}  // extern "C"
