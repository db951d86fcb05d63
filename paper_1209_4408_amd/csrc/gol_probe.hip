// VALU issue-rate probe: the per-instruction lane rates behind the ALU
// roofline of the tile pass.  Every thread runs eight independent chains of
// one instruction kind (no chain waits on another), so with 32768 waves in
// flight the issue rate, not latency, sets the time.  Register-only: the
// plain ops are written as inline asm so the compiler cannot fold repeated
// applications; the DPP move uses the builtin so the compiler inserts the
// wait states DPP needs after a VALU write.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gol_internal.h"
#include "gol_runtime.h"

namespace gol {

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocks = 8192;  // 32768 waves
constexpr int kProbeChains = 8;
constexpr int kProbeIters = 2048;

// kinds: 0 v_xor_b32, 1 v_bitop3_b32 (three VGPR sources), 2 v_alignbit_b32,
// 3 v_mov_b32 with DPP (wave_shr:1), 4 v_add_u32
template <int KIND>
__global__ __launch_bounds__(kProbeThreads) void k_valu_probe(uint32_t* out, int iters) {
  const uint32_t t = blockIdx.x * kProbeThreads + threadIdx.x;
  uint32_t a[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) a[c] = t * 2654435761u + (uint32_t)c;
  const uint32_t k1 = t | 1u, k2 = t ^ 0x5bd1e995u;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) {
      if constexpr (KIND == 0) {
        asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[c]) : "v"(k1));
      } else if constexpr (KIND == 1) {
        asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[c]) : "v"(k1), "v"(k2));
      } else if constexpr (KIND == 2) {
        asm volatile("v_alignbit_b32 %0, %0, %1, 31" : "+v"(a[c]) : "v"(k1));
      } else if constexpr (KIND == 3) {
        a[c] = (uint32_t)__builtin_amdgcn_mov_dpp((int)a[c], 0x138 /* wave_shr:1 */, 0xF, 0xF,
                                                  false);
      } else {
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[c]) : "v"(k1));
      }
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) r ^= a[c];
  out[t] = r;  // keeps every chain live
}

static hipError_t launch_probe(int kind, uint32_t* out, int iters, hipStream_t st) {
  const dim3 grid(kProbeBlocks), block(kProbeThreads);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_valu_probe<0>, grid, block, 0, st, out, iters); break;
    case 1: hipLaunchKernelGGL(k_valu_probe<1>, grid, block, 0, st, out, iters); break;
    case 2: hipLaunchKernelGGL(k_valu_probe<2>, grid, block, 0, st, out, iters); break;
    case 3: hipLaunchKernelGGL(k_valu_probe<3>, grid, block, 0, st, out, iters); break;
    default: hipLaunchKernelGGL(k_valu_probe<4>, grid, block, 0, st, out, iters); break;
  }
  return hipGetLastError();
}

}  // namespace gol

extern "C" int gol_debug_valu_rate(int kind, void* stream, double* lane_ops_per_second) {
  using namespace gol;
  if (kind < 0 || kind > 4 || !lane_ops_per_second)
    return set_error(GOL_EINVAL, "kind must be 0..4 and the result pointer non-null");
  const hipStream_t st = (hipStream_t)stream;
  const size_t bytes = (size_t)kProbeBlocks * kProbeThreads * sizeof(uint32_t);
  void* out = nullptr;
  int rc = scratch_alloc(&out, bytes, st);
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch_probe(kind, (uint32_t*)out, kProbeIters, st);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = launch_probe(kind, (uint32_t*)out, kProbeIters, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  scratch_free(out, st);
  if (e != hipSuccess) return hip_error(e, "valu probe");
  const double ops = (double)kProbeBlocks * kProbeThreads * kProbeIters * kProbeChains;
  *lane_ops_per_second = ops / ((double)ms * 1e-3);
  return GOL_OK;
}
