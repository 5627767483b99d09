// MLP policy phase for gfx950: a rendered frame per env in, actions out.
//
// The paper's RL rollouts run an MLP policy beside physics and rendering on
// the same GPU (Evaluation, RL Training, MLP-based RL).  The observation of an
// env is its camera 0 frame as K = 4 W H integers 0..255: the RGB bytes in
// memory order, then the top byte of each 24-bit depth.  Layers:
//   h1 = relu(x W1 + b1)   W1 bfloat16 [K][H], given transposed as [H][K]
//   h2 = relu(h1 W2 + b2)  float32
//   y  = h2 W3 + b3        float32, A = 3 B outputs
//   a  = a_max clamp(y, -1, 1): the force on body b is a[3b .. 3b+2]
// Layer 1 is the one dense contraction of the step loop (K = 65,536 at
// 128x128); it runs on MFMA (v_mfma_f32_16x16x32_bf16): every observation
// value is an 8-bit integer, exact in bfloat16, so each product is exact and
// only the float32 accumulation rounds.  K is split over workgroups (partial
// sums in float32, added in a fixed order by the head), so that a batch of a
// few hundred envs still fills 256 CUs.  Layers 2 and 3 are small (H^2 and
// H A per env) and run on the VALU in the head kernel, one workgroup per env.
#include "vuda_internal.h"

#pragma clang fp contract(off)

namespace vuda {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRows = 64;      // envs per layer-1 workgroup
constexpr int kCols = 256;     // hidden units per layer-1 workgroup (64 per wave)
constexpr int kKStep = 32;     // k per MFMA step
constexpr int kLdsRow = 40;    // bfloat16 per staged row (32 + 8 padding against bank conflicts)

// bfloat16 bits of the integers in the four bytes of w (exact: 8-bit values)
__device__ __forceinline__ uint2 bytes_to_bf16(uint32_t w) {
  // (the compiler turns these into v_cvt_f32_ubyte0..3)
  const uint32_t f0 = __float_as_uint((float)(w & 0xFFu));
  const uint32_t f1 = __float_as_uint((float)((w >> 8) & 0xFFu));
  const uint32_t f2 = __float_as_uint((float)((w >> 16) & 0xFFu));
  const uint32_t f3 = __float_as_uint((float)(w >> 24));
  // the upper halves of (f1, f0) and (f3, f2)
  return make_uint2(__builtin_amdgcn_perm(f1, f0, 0x07060302u), __builtin_amdgcn_perm(f3, f2, 0x07060302u));
}

// 8 observation values x[k .. k+7] of one frame as bfloat16 (k a multiple of
// 8; the RGB part ends at 3 W H, a multiple of 32)
__device__ __forceinline__ uint4 obs8(const uint8_t* rgb, const uint32_t* depth, int k, int krgb) {
  if (k < krgb) {
    const uint2 b = *(const uint2*)(rgb + k);
    const uint2 lo = bytes_to_bf16(b.x), hi = bytes_to_bf16(b.y);
    return make_uint4(lo.x, lo.y, hi.x, hi.y);
  }
  const uint4 d0 = *(const uint4*)(depth + (k - krgb));
  const uint4 d1 = *(const uint4*)(depth + (k - krgb) + 4);
  // byte 2 of each depth word: its top byte (background 0xFFFFFFFF gives 255)
  const uint32_t w0 = __builtin_amdgcn_perm(d0.y, d0.x, 0x0c0c0602u) | (__builtin_amdgcn_perm(d0.w, d0.z, 0x0c0c0602u) << 16);
  const uint32_t w1 = __builtin_amdgcn_perm(d1.y, d1.x, 0x0c0c0602u) | (__builtin_amdgcn_perm(d1.w, d1.z, 0x0c0c0602u) << 16);
  const uint2 lo = bytes_to_bf16(w0), hi = bytes_to_bf16(w1);
  return make_uint4(lo.x, lo.y, hi.x, hi.y);
}

// Layer 1: partial sums over k in [s Kc, (s+1) Kc) for kRows envs and kCols
// hidden units.  Wave w owns units n0 + 64 w .. + 63, all kRows envs: 4 x 4
// blocks of 16 x 16, one MFMA each per k step.
__global__ __launch_bounds__(256) void policy_l1_kernel(WorldDev W, PolicyLaunch L) {
  __shared__ __align__(16) uint16_t sA[2][kRows * kLdsRow];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m0 = blockIdx.x * kRows;
  const int n0 = blockIdx.y * kCols + 64 * wave;
  const int s = blockIdx.z;
  const int K = L.K, krgb = L.krgb, Kc = L.kchunk;
  const int kbeg = s * Kc;
  const int nsteps = Kc / kKStep;
  // staging role: row r = tid / 4, k offset 8 (tid % 4) of each step
  const int r = tid >> 2, kq = 8 * (tid & 3);
  const uint8_t* rgb = nullptr;
  const uint32_t* dep = nullptr;
  const bool rvalid = m0 + r < L.M;
  if (rvalid) {
    const CamDev cam = W.cams[W.envs[L.envs[m0 + r]].cam_off];
    rgb = W.rgb + 3 * cam.pix_off;
    dep = W.depth + cam.pix_off;
  }
  // B fragments: lane (column n0 + 16 cb + lane % 16, k + 8 (lane / 16) .. + 7)
  const uint16_t* bcol[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int n = min(n0 + 16 * cb + (lane & 15), L.H - 1);
    bcol[cb] = L.w1t + (int64_t)n * K + 8 * (lane >> 4);
  }
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  uint4 stage = rvalid ? obs8(rgb, dep, kbeg + kq, krgb) : make_uint4(0, 0, 0, 0);
  *(uint4*)&sA[0][r * kLdsRow + kq] = stage;
  // W1 fragments run one step ahead of the MFMAs that use them
  uint4 bn[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) bn[cb] = *(const uint4*)(bcol[cb] + kbeg);
  __syncthreads();
  for (int t = 0; t < nsteps; ++t) {
    const int k = kbeg + t * kKStep;
    const int buf = t & 1;
    bf16x8 b[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) b[cb] = __builtin_bit_cast(bf16x8, bn[cb]);
    // next step's W1 fragments and observation values, in flight while this
    // step multiplies
    if (t + 1 < nsteps) {
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) bn[cb] = *(const uint4*)(bcol[cb] + k + kKStep);
      stage = rvalid ? obs8(rgb, dep, k + kKStep + kq, krgb) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const bf16x8 a = __builtin_bit_cast(bf16x8, *(const uint4*)&sA[buf][(16 * rb + (lane & 15)) * kLdsRow + 8 * (lane >> 4)]);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[cb], acc[rb][cb], 0, 0, 0);
    }
    if (t + 1 < nsteps) *(uint4*)&sA[buf ^ 1][r * kLdsRow + kq] = stage;
    __syncthreads();
  }
  // D layout: lane holds rows 4 (lane / 16) + i of a block, column lane % 16
  float* P = L.partial + (int64_t)s * L.M * L.H;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int n = n0 + 16 * cb + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + 16 * rb + 4 * (lane >> 4) + i;
        if (m < L.M && n < L.H) P[(int64_t)m * L.H + n] = acc[rb][cb][i];
      }
    }
}

// Layers 2 and 3, one workgroup per env (blockDim = H rounded up to 64,
// at most 1024): the split-K partials added in split order, then every unit
// on its own lane, its dot product in index order.
__global__ __launch_bounds__(1024) void policy_head_kernel(WorldDev W, PolicyLaunch L) {
  extern __shared__ float sh[];  // h1 [H], h2 [H]
  const int m = blockIdx.x;
  if (m >= L.M) return;
  const int env = L.envs[m];
  const int j = threadIdx.x, H = L.H;
  float* h1 = sh;
  float* h2 = sh + H;
  // loads go out eight at a time; the sums still run in index order
  if (j < H) {
    const float* p = L.partial + (int64_t)m * H + j;
    const int64_t stride = (int64_t)L.M * H;
    float s1 = 0.0f;
    int s = 0;
    for (; s + 8 <= L.splits; s += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[(s + u) * stride];
#pragma unroll
      for (int u = 0; u < 8; ++u) s1 = s1 + v[u];
    }
    for (; s < L.splits; ++s) s1 = s1 + p[s * stride];
    s1 = s1 + L.b1[j];
    h1[j] = s1 > 0.0f ? s1 : 0.0f;
  }
  __syncthreads();
  if (j < H) {
    float s2 = 0.0f;
    int i = 0;
    for (; i + 8 <= H; i += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = L.w2[(int64_t)(i + u) * H + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) s2 = s2 + h1[i + u] * v[u];
    }
    for (; i < H; ++i) s2 = s2 + h1[i] * L.w2[(int64_t)i * H + j];
    s2 = s2 + L.b2[j];
    h2[j] = s2 > 0.0f ? s2 : 0.0f;
  }
  __syncthreads();
  for (int q = j; q < L.A; q += blockDim.x) {
    float y = 0.0f;
    int i = 0;
    for (; i + 8 <= H; i += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = L.w3[(int64_t)(i + u) * L.A + q];
#pragma unroll
      for (int u = 0; u < 8; ++u) y = y + h2[i + u] * v[u];
    }
    for (; i < H; ++i) y = y + h2[i] * L.w3[(int64_t)i * L.A + q];
    y = y + L.b3[q];
    const float c = __builtin_amdgcn_fmed3f(y, -1.0f, 1.0f);  // y is finite: the clamp
    W.actions[(int64_t)env * L.A + q] = L.a_max * c;
  }
  if (j == 0) W.act_on[env] = 1;
}

}  // namespace

hipError_t launch_policy(const WorldDev& w, const PolicyLaunch& l, hipStream_t s) {
  if (l.M <= 0) return hipSuccess;
  const dim3 g1((l.M + kRows - 1) / kRows, (l.H + kCols - 1) / kCols, l.splits);
  hipLaunchKernelGGL(policy_l1_kernel, g1, dim3(256), 0, s, w, l);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int threads = (l.H + 63) / 64 * 64;
  hipLaunchKernelGGL(policy_head_kernel, dim3(l.M), dim3(threads), 2 * l.H * sizeof(float), s, w, l);
  return hipGetLastError();
}

}  // namespace vuda
