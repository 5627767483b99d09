// Linear (metric) depth from the 24-bit depth images.
//
// A camera's view-projection maps a point to clip z and w with z = alpha w +
// beta for a perspective of the usual form (its third row is alpha times its
// fourth plus beta in the translation column), so the stored depth
// z_ndc = D / (2^24 - 1) gives back the view depth w = beta / (z_ndc - alpha):
// the distance along the camera axis of the surface seen at the pixel.  The
// conversion runs in float64 (z_ndc - alpha loses about 6 digits at the far
// plane in float32) and rounds once to float32.
#include <algorithm>

#include "vuda_runtime.h"

namespace vuda {
namespace {

__global__ __launch_bounds__(256) void depth_metric_kernel(const uint32_t* depth, const MetricCam* cams,
                                                           float* out) {
  const MetricCam c = cams[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < c.npix; i += (int64_t)gridDim.x * 256) {
    const uint32_t D = depth[c.pix_off + i];
    float v = __builtin_inff();  // background: no surface
    if (D != 0xFFFFFFFFu) v = (float)(c.beta / ((double)D / 16777215.0 - c.alpha));
    out[c.out_off + i] = v;
  }
}

}  // namespace

hipError_t launch_depth_metric(const uint32_t* depth, const MetricCam* cams, int32_t ncams, int64_t max_pix,
                               float* out, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((max_pix + 255) / 256, 64);
  for (int32_t c0 = 0; c0 < ncams; c0 += 65535) {
    const int32_t n = std::min(ncams - c0, 65535);
    hipLaunchKernelGGL(depth_metric_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1), n), dim3(256), 0, s, depth,
                       cams + c0, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vuda
