// MLP policy phase for gfx950: a rendered frame per env in, actions out.
//
// The paper's RL rollouts run an MLP policy beside physics and rendering on
// the same GPU (Evaluation, RL Training, MLP-based RL).  The observation of an
// env is its camera 0 frame as K = 4 W H integers 0..255: the RGB bytes in
// memory order, then the top byte of each 24-bit depth.  Layers:
//   h1 = relu(x W1 + b1)   W1 bfloat16 [K][H], held as panels [K / 32][H][32]
//   h2 = relu(h1 W2 + b2)  float32
//   y  = h2 W3 + b3        float32, A = 3 B outputs
//   a  = a_max clamp(y, -1, 1): the force on body b is a[3b .. 3b+2]
// Layer 1 is the one dense contraction of the step loop (K = 65,536 at
// 128x128); it runs on MFMA (v_mfma_f32_16x16x32_bf16): every observation
// value is an 8-bit integer, exact in bfloat16, so each product is exact and
// only the float32 accumulation rounds.  K is split over workgroups (partial
// sums in float32, added in a fixed order by the head), so that a batch of a
// few hundred envs still fills 256 CUs.  Up to H = 1024, layers 2 and 3 are
// small (H^2 and H A per env) and run on the VALU in one head kernel, one
// workgroup per env.  Wider policies (H = 4096: 16.8 M multiply-adds per env
// in layer 2) run layers 2 and 3 as batched products over all envs on
// float32 MFMA (v_mfma_f32_16x16x4_f32), each split over K like layer 1,
// with small kernels that add the splits in order and apply the bias and the
// activation.
#include "vuda_internal.h"

#include <type_traits>

#pragma clang fp contract(off)

namespace vuda {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRows = 64;      // envs per layer-1 workgroup
constexpr int kCols = 256;     // hidden units per layer-1 workgroup (64 per wave)
constexpr int kKStep = 32;     // k per MFMA step
constexpr int kLdsRow = 40;    // bfloat16 per staged row (32 + 8 padding against bank conflicts)

constexpr int kXcds = 8;        // accelerator complex dies, each with its own L2

// Position of this workgroup in the grid's logical order (x fastest, then
// y, then z).  The dispatcher deals workgroups to the XCDs round-robin in
// launch order; renumbered like this, each XCD takes one contiguous run of
// the logical order, so that the row tiles that share a weight slice (and
// the column tiles that share rows) meet in one L2 instead of eight.
__device__ __forceinline__ int3 xcd_tile() {
  const int total = gridDim.x * gridDim.y * gridDim.z;
  int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  if (total % kXcds == 0) b = (b % kXcds) * (total / kXcds) + b / kXcds;
  return make_int3(b % gridDim.x, (b / gridDim.x) % gridDim.y, b / (gridDim.x * gridDim.y));
}

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

// The bytes behind 8 observation values x[k .. k+7] of one frame (k a
// multiple of 8): 8 RGB bytes while k is in the RGB part (which ends at
// 3 W H, a multiple of 32, so a whole 32-k step is on one side), else 8
// depth words; only the members of that kind are loaded and read.  They are
// loaded a step ahead and converted only after that step's MFMAs, so that
// the wait for them does not come before the MFMAs.
struct ObsRaw {
  uint2 c;       // RGB bytes
  uint4 d0, d1;  // depth words
};

// kRgb: the bytes at rgb[k ..]; else the words at depth[kd ..]
template <bool kRgb>
__device__ __forceinline__ void obs_load(ObsRaw& r, const uint8_t* rgb, const uint32_t* depth, int k, int kd) {
  if constexpr (kRgb) {
    r.c = *(const uint2*)(rgb + k);
  } else {
    r.d0 = *(const uint4*)(depth + kd);
    r.d1 = *(const uint4*)(depth + kd + 4);
  }
}

// the 8 values as bfloat16
template <bool kRgb>
__device__ __forceinline__ uint4 obs_convert(const ObsRaw& r) {
  uint32_t w0, w1;
  if constexpr (kRgb) {
    w0 = r.c.x;
    w1 = r.c.y;
  } else {
    // byte 2 of each depth word: its top byte (background 0xFFFFFFFF gives 255)
    w0 = __builtin_amdgcn_perm(r.d0.y, r.d0.x, 0x0c0c0602u) | (__builtin_amdgcn_perm(r.d0.w, r.d0.z, 0x0c0c0602u) << 16);
    w1 = __builtin_amdgcn_perm(r.d1.y, r.d1.x, 0x0c0c0602u) | (__builtin_amdgcn_perm(r.d1.w, r.d1.z, 0x0c0c0602u) << 16);
  }
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
  const int3 tile = xcd_tile();
  const int m0 = tile.x * kRows;
  const int n0 = tile.y * kCols + 64 * wave;
  const int s = tile.z;
  const int krgb = L.krgb, Kc = L.kchunk;
  const int kbeg = s * Kc;
  const int nsteps = Kc / kKStep;
  // staging role: row r = tid / 4, k offset 8 (tid % 4) of each step
  const int r = tid >> 2, kq = 8 * (tid & 3);
  // rows past M (a ragged last tile) read row m0's frame: a row of A only
  // reaches the same row of the product, and those rows are not stored
  const CamDev cam = W.cams[W.envs[L.envs[min(m0 + r, L.M - 1)]].cam_off];
  const uint8_t* rgb = W.rgb + 3 * cam.pix_off;
  const uint32_t* dep = W.depth + cam.pix_off;
  // B fragments: lane (column n0 + 16 cb + lane % 16, k + 8 (lane / 16) .. + 7),
  // in the panel of step k at (k / 32) 32 H
  const uint16_t* bcol[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int n = min(n0 + 16 * cb + (lane & 15), L.H - 1);
    bcol[cb] = L.w1t + (int64_t)n * kKStep + 8 * (lane >> 4);
  }
  const int64_t panel = (int64_t)kKStep * L.H;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  const int kend = kbeg + Kc;
  {
    ObsRaw raw;
    uint4 v;
    if (kbeg < krgb) {
      obs_load<true>(raw, rgb, dep, kbeg + kq, 0);
      v = obs_convert<true>(raw);
    } else {
      obs_load<false>(raw, rgb, dep, 0, kbeg + kq - krgb);
      v = obs_convert<false>(raw);
    }
    *(uint4*)&sA[0][r * kLdsRow + kq] = v;
  }
  // W1 fragments run one step ahead of the MFMAs that use them
  uint4 bn[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) bn[cb] = *(const uint4*)(bcol[cb] + (kbeg / kKStep) * panel);
  __syncthreads();
  // One step: the next step's W1 fragments and observation bytes (of the
  // kind the template argument names) go out, this step's MFMAs run, then
  // the bytes are converted and staged.  No branch surrounds a load, so no
  // register copy of a loaded value (and no wait for it) lands before the
  // MFMAs.  The last step reloads itself (in bounds, unused).
  auto step = [&](auto next_rgb, int t) {
    constexpr bool kNextRgb = decltype(next_rgb)::value;
    const int k = kbeg + t * kKStep;
    const int knext = min(k + kKStep, kend - kKStep);
    const int buf = t & 1;
    bf16x8 b[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) b[cb] = __builtin_bit_cast(bf16x8, bn[cb]);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) bn[cb] = *(const uint4*)(bcol[cb] + (knext / kKStep) * panel);
    ObsRaw raw;
    // (a depth load for a step still in the RGB part reads depth word 0 on)
    obs_load<kNextRgb>(raw, rgb, dep, knext + kq, max(knext + kq - krgb, 0));
    // the loads go out before the MFMAs
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const bf16x8 a = __builtin_bit_cast(bf16x8, *(const uint4*)&sA[buf][(16 * rb + (lane & 15)) * kLdsRow + 8 * (lane >> 4)]);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[cb], acc[rb][cb], 0, 0, 0);
    }
    // nothing below moves above the MFMAs
    __builtin_amdgcn_sched_barrier(0);
    *(uint4*)&sA[buf ^ 1][r * kLdsRow + kq] = obs_convert<kNextRgb>(raw);
    __syncthreads();
  };
  // steps whose successor is in the RGB part, then the rest
  const int t_rgb = min(max((krgb - kbeg) / kKStep, 0), nsteps);  // steps in the RGB part
  int t = 0;
  for (; t < t_rgb - 1; ++t) step(std::true_type{}, t);
  for (; t < nsteps; ++t) step(std::false_type{}, t);
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

// sum_{s < n} p[s * stride], in s order; the loads go out kBatch at a time
// (independent, so their latencies overlap), the additions stay in order
template <int kBatch>
__device__ __forceinline__ float ordered_strided_sum(const float* p, int64_t stride, int n) {
  float acc = 0.0f;
  int s = 0;
  for (; s + kBatch <= n; s += kBatch) {
    float v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) v[u] = p[(s + u) * stride];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) acc = acc + v[u];
  }
  for (; s < n; ++s) acc = acc + p[s * stride];
  return acc;
}

// sum_{i < n} x[i] w[i * stride] in i order (x in LDS), loads kBatch at a time
template <int kBatch>
__device__ __forceinline__ float ordered_dot(const float* x, const float* w, int64_t stride, int n) {
  float acc = 0.0f;
  int i = 0;
  for (; i + kBatch <= n; i += kBatch) {
    float v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) v[u] = w[(i + u) * stride];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) acc = acc + x[i + u] * v[u];
  }
  for (; i < n; ++i) acc = acc + x[i] * w[i * stride];
  return acc;
}

__device__ __forceinline__ float relu(float v) { return v > 0.0f ? v : 0.0f; }

// a_max clamp(y, -1, 1) for a finite y
__device__ __forceinline__ float action_of(float y, float a_max) {
  return a_max * __builtin_amdgcn_fmed3f(y, -1.0f, 1.0f);
}

// Layers 2 and 3, one workgroup per env (blockDim = H rounded up to 64,
// at most 1024): the split-K partials added in split order, then every unit
// on its own lane, its dot product in index order.  (Splitting each sum over
// more lanes, to put more loads in flight, was slower: the weight reads from
// L2 bound this kernel, not their latency.)
__global__ __launch_bounds__(1024) void policy_head_kernel(WorldDev W, PolicyLaunch L) {
  extern __shared__ float sh[];  // h1 [H], h2 [H]
  const int m = blockIdx.x;
  if (m >= L.M) return;
  const int env = L.envs[m];
  const int j = threadIdx.x, H = L.H;
  float* h1 = sh;
  float* h2 = sh + H;
  if (j < H) {
    const float s1 = ordered_strided_sum<16>(L.partial + (int64_t)m * H + j, (int64_t)L.M * H, L.splits);
    h1[j] = relu(s1 + L.b1[j]);
  }
  __syncthreads();
  if (j < H) h2[j] = relu(ordered_dot<32>(h1, L.w2 + j, H, H) + L.b2[j]);
  __syncthreads();
  for (int q = j; q < L.A; q += blockDim.x)
    W.actions[(int64_t)env * L.A + q] = action_of(ordered_dot<32>(h2, L.w3 + q, L.A, H) + L.b3[q], L.a_max);
  if (j == 0) W.act_on[env] = 1;
}

// ---- layers 2 and 3 as batched products (H > 1024) ----

// out[m][j] = relu(sum_s P[s][m][j] + b[j]) for j < N, P with row stride N
__global__ __launch_bounds__(256) void policy_hidden_kernel(const float* P, int splits, int M, int N, const float* b,
                                                            float* out) {
  const int m = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (m >= M || j >= N) return;
  const int64_t at = (int64_t)m * N + j;
  out[at] = relu(ordered_strided_sum<16>(P + at, (int64_t)M * N, splits) + b[j]);
}

// actions of row m: a_max clamp(sum_s P[s][m][q] + b3[q]) for q < A, P with
// row stride ldp; and the env's force flag
__global__ __launch_bounds__(256) void policy_act_kernel(WorldDev W, PolicyLaunch L, const float* P, int splits,
                                                         int ldp) {
  const int m = blockIdx.x;
  if (m >= L.M) return;
  const int env = L.envs[m];
  for (int q = threadIdx.x; q < L.A; q += blockDim.x) {
    const float y = ordered_strided_sum<16>(P + (int64_t)m * ldp + q, (int64_t)L.M * ldp, splits);
    W.actions[(int64_t)env * L.A + q] = action_of(y + L.b3[q], L.a_max);
  }
  if (threadIdx.x == 0) W.act_on[env] = 1;
}

constexpr int kDTile = 64;   // rows and columns of a dense-product workgroup tile
constexpr int kDStep = 16;   // k per staged step
constexpr int kAPitch = 20;  // floats per staged A row (16 + 4: lanes of one read hit distinct banks)
constexpr int kBPitch = 80;  // floats per staged B row (64 + 16)

// P[s][m][n] = sum_{k in chunk s} X[m][k] B[k][n] for m < M, n < ldb: X is
// [M][K] and B [K][ldb] row-major float32, K and ldb multiples of 64, chunk
// a multiple of kDStep.  Workgroup: a 64 x 64 tile of one chunk; wave w
// owns the 32 x 32 quadrant (w & 1, w >> 1), 2 x 2 blocks of 16 x 16.
__global__ __launch_bounds__(256) void policy_dense_kernel(const float* X, const float* B, int M, int K, int ldb,
                                                           int kchunk, float* P) {
  __shared__ __align__(16) float sA[2][kDTile * kAPitch];
  __shared__ __align__(16) float sB[2][kDStep * kBPitch];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int3 tile = xcd_tile();
  const int m0 = tile.x * kDTile, n0 = tile.y * kDTile, s = tile.z;
  const int wm = 32 * (wave & 1), wn = 32 * (wave >> 1);
  const int kbeg = s * kchunk, nsteps = kchunk / kDStep;
  // staging roles: X row ar, columns ac .. ac+3; B row br, columns bc .. bc+3
  const int ar = tid >> 2, ac = 4 * (tid & 3);
  const int br = tid >> 4, bc = 4 * (tid & 15);
  // rows past M read row M - 1: a row of X only reaches the same row of
  // the product, and those rows are not stored
  const float* xa = X + (int64_t)min(m0 + ar, M - 1) * K + ac;
  const float* bb = B + (int64_t)br * ldb + n0 + bc;
  float4 ra = *(const float4*)(xa + kbeg);
  float4 rb = *(const float4*)(bb + (int64_t)kbeg * ldb);
  *(float4*)&sA[0][ar * kAPitch + ac] = ra;
  *(float4*)&sB[0][br * kBPitch + bc] = rb;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  __syncthreads();
  for (int t = 0; t < nsteps; ++t) {
    const int buf = t & 1;
    if (t + 1 < nsteps) {
      const int k = kbeg + (t + 1) * kDStep;
      ra = *(const float4*)(xa + k);
      rb = *(const float4*)(bb + (int64_t)k * ldb);
    }
    // operands of v_mfma_f32_16x16x4_f32: lane l holds A[l % 16][l / 16]
    // and B[l / 16][l % 16] of the 16 x 4 and 4 x 16 blocks
#pragma unroll
    for (int kk = 0; kk < kDStep; kk += 4) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sA[buf][(wm + 16 * i + (lane & 15)) * kAPitch + kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sB[buf][(kk + (lane >> 4)) * kBPitch + wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (t + 1 < nsteps) {
      *(float4*)&sA[buf ^ 1][ar * kAPitch + ac] = ra;
      *(float4*)&sB[buf ^ 1][br * kBPitch + bc] = rb;
    }
    __syncthreads();
  }
  // D layout: lane holds rows 4 (lane / 16) + r of a block, column lane % 16
  float* Ps = P + (int64_t)s * M * ldb;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + 16 * j + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        if (m < M) Ps[(int64_t)m * ldb + n] = acc[i][j][r];
      }
    }
}

}  // namespace

hipError_t launch_policy(const WorldDev& w, const PolicyLaunch& l, hipStream_t s, LaunchEvents* ev) {
  if (l.M <= 0) return hipSuccess;
  const dim3 g1((l.M + kRows - 1) / kRows, (l.H + kCols - 1) / kCols, l.splits);
  timed_launch(ev, true, false, policy_l1_kernel, g1, dim3(256), 0, s, w, l);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!l.layered) {
    const int threads = (l.H + 63) / 64 * 64;
    timed_launch(ev, false, true, policy_head_kernel, dim3(l.M), dim3(threads), (uint32_t)(2 * l.H * sizeof(float)), s,
                 w, l);
    return hipGetLastError();
  }
  // h1, then layer 2 into the partials (free again once h1 is made), h2,
  // layer 3, the actions
  const int mt = (l.M + kDTile - 1) / kDTile;
  const dim3 gh((l.H + 255) / 256, l.M);
  hipLaunchKernelGGL(policy_hidden_kernel, gh, dim3(256), 0, s, l.partial, l.splits, l.M, l.H, l.b1, l.h1);
  hipLaunchKernelGGL(policy_dense_kernel, dim3(mt, l.H / kDTile, l.s2), dim3(256), 0, s, l.h1, l.w2, l.M, l.H, l.H,
                     l.H / l.s2, l.partial);
  hipLaunchKernelGGL(policy_hidden_kernel, gh, dim3(256), 0, s, l.partial, l.s2, l.M, l.H, l.b2, l.h2);
  hipLaunchKernelGGL(policy_dense_kernel, dim3(mt, l.Ap / kDTile, l.s3), dim3(256), 0, s, l.h2, l.w3p, l.M, l.H,
                     l.Ap, l.H / l.s3, l.partial);
  timed_launch(ev, false, true, policy_act_kernel, dim3(l.M), dim3(256), 0, s, w, l, (const float*)l.partial, l.s3, l.Ap);
  return hipGetLastError();
}

}  // namespace vuda
