// Placement probe: records where the workgroups of a stream run (XCC, SE, CU)
// to verify the CU partition of the co-scheduling streams.
#include <hip/hip_runtime.h>

#include <vector>

#include "vuda.h"
#include "vuda_runtime.h"

namespace {

// HW_ID register (gfx9 layout): CU_ID bits 11:8, SH_ID bit 12, SE_ID bits 15:13.
// XCC_ID register: bits 3:0.
__global__ void probe_kernel(int32_t* out, long long spin_cycles) {
  if (threadIdx.x != 0) return;
  const unsigned hw = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4);
  const unsigned xcc = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 20);
  const long long t0 = clock64();
  while (clock64() - t0 < spin_cycles) {
  }
  out[3 * blockIdx.x + 0] = (int32_t)(xcc & 0xF);
  out[3 * blockIdx.x + 1] = (int32_t)((hw >> 13) & 0x7);
  out[3 * blockIdx.x + 2] = (int32_t)((hw >> 8) & 0xF);
}

}  // namespace

extern "C" int vuda_probe_placement(vuda_world* w, int32_t phase, int32_t n_blocks, int32_t spin_us,
                                    int32_t* out) {
  if (!w || !out || n_blocks <= 0 || n_blocks > (1 << 20) || spin_us < 0 || spin_us > 100000)
    return vuda::fail(VUDA_EINVAL, "probe arguments");
  hipStream_t s = phase == VUDA_PHASE_STEP ? w->s_sim : (phase == VUDA_PHASE_RENDER ? w->s_render : nullptr);
  if (!s) return vuda::fail(VUDA_EINVAL, "phase %d", phase);
  int32_t* d = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(int32_t) * 3 * (size_t)n_blocks);
  if (e != hipSuccess) return vuda::hip_fail(e, "hipMalloc");
  // clock64 counts shader clocks (~2.4 GHz on MI355X)
  hipLaunchKernelGGL(probe_kernel, dim3(n_blocks), dim3(64), 0, s, d, (long long)spin_us * 2400);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess)
    e = hipMemcpy(out, d, sizeof(int32_t) * 3 * (size_t)n_blocks, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return e == hipSuccess ? VUDA_OK : vuda::hip_fail(e, "probe");
}
