// Internal layout of a world in device memory, shared by the host runtime and
// the HIP kernels of libvuda.  Everything here is structure-of-arrays over a
// global body index (env-major, contiguous per env) so that the lane that
// owns a body reads and writes its components with coalesced accesses.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vuda {

constexpr int kStateComps = 13;  // px py pz vx vy vz qw qx qy qz wx wy wz
enum StateComp { PX = 0, PY, PZ, VX, VY, VZ, QW, QX, QY, QZ, WX, WY, WZ };

constexpr int kMaxBodies = 128;     // bodies per env
constexpr int kMaxTplVerts = 64;    // vertices per template
constexpr int kMaxTplFaces = 128;   // faces per template
constexpr int kMaxGroundVerts = 8;
constexpr int kMaxGroundFaces = 8;
constexpr int kGroundPair = 0xFFFF;
constexpr int kTile = 16;           // default raster tile edge in pixels
constexpr int kTileShiftMin = 3, kTileShiftMax = 5;  // tile edges 8, 16 and 32

// env flags (device-side, sticky until fetched)
constexpr uint32_t kFlagNonFinite = 1u;
constexpr uint32_t kFlagContactOverflow = 2u;
constexpr uint32_t kFlagBinOverflow = 4u;
constexpr uint32_t kFlagClipOverflow = 8u;  // an image cut more near-plane pieces than kClipRecs

struct EnvDev {
  int32_t body_off;   // first global body id
  int32_t n_bodies;   // 0 = free slot
  int32_t cam_off;    // first global camera id
  int32_t n_cams;
  int32_t n_verts;    // template vertices of all bodies + ground
  int32_t n_tris;     // primitives: ground faces + template faces of all bodies
  int64_t prim_map;   // offset of the env's primitive -> body map
  int64_t vert_map;   // offset of the env's vertex -> body map
};

// Uniform loads of data that no wave writes while the kernel runs (launch
// tables, descriptors, what an earlier kernel wrote): read through the
// constant address space, so that they are scalar loads into scalar
// registers.  uniform_copy takes a whole struct, a word at a time.
template <class T>
__device__ __forceinline__ T uniform_ld(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}

__device__ __forceinline__ int2 uniform_ld(const int2* p) {
  const uint64_t v = uniform_ld((const uint64_t*)p);
  return make_int2((int32_t)(uint32_t)v, (int32_t)(uint32_t)(v >> 32));
}

template <class T>
__device__ __forceinline__ T uniform_copy(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  T v;
  const uint32_t* s = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) {
    const uint32_t x = uniform_ld(s + i);
    __builtin_memcpy(reinterpret_cast<char*>(&v) + 4 * i, &x, 4);
  }
  return v;
}

constexpr uint8_t kGroundBody = 0xFF;  // body id of ground primitives in the maps

struct CamDev {
  float vp[16];
  int32_t w, h;
  int64_t pix_off;    // first pixel of the image in the image arena
  int32_t env;
  int32_t n_tris;     // primitives of the env (sizes the raster scratch)
  int64_t rs_off;     // byte offset of the image's raster scratch (two layouts, one per state buffer)
  int32_t rs_recs, rs_bins, rs_total;  // rs_layout(n_tris, tiles): offsets and size of one layout
  int32_t rs_attr;                     // smooth shading: the attribute records
  int32_t rs_tuv;                      // textured worlds: the texture-coordinate records
};

// Raster scratch of one camera image and state buffer (two per camera, one
// for each state buffer), written by the setup kernel and read by the tile
// kernel: a header (record count, binned flag), the tile table
// (bin offset, bin count per 16x16 tile), the setup records (kRecBytes each,
// room for every primitive of the env and kClipRecs pieces of triangles cut
// by the near plane) and the bins (u16 record ids, bit 15 set when the
// triangle covers the whole tile).
constexpr int kRecWords = 16;  // X0 Y0 X1 Y1 | X2 Y2 key z0 | z1 z2 invA rgb | box x, box y, flags, 0
constexpr int kRecBytes = 4 * kRecWords;
constexpr int kBinsPerTri = 4;  // bin capacity of an image, per primitive
constexpr int kClipRecs = 64;   // records an image keeps for pieces of triangles cut by the near plane

// Smooth shading: per record an attribute record of 16 floats, the world
// normals of its vertices in edge order (9), their reciprocal clip w (3) and
// the albedo (3).
constexpr int kAttrWords = 16;

// Textured worlds: per record the texture coordinates of its vertices in
// edge order (6 floats) and a flag (1: textured), padded to 8 floats.
constexpr int kTuvWords = 8;

struct RsLayout {
  int64_t tiles, recs, bins, attr, tuv, total;
  int32_t bin_cap;
};

__host__ __device__ inline int64_t rs_align(int64_t x) { return (x + 255) & ~(int64_t)255; }

__host__ __device__ inline RsLayout rs_layout(int32_t ntris, int32_t ntiles, bool smooth = false,
                                              bool textured = false) {
  RsLayout r;
  r.tiles = 64;
  r.recs = rs_align(64 + 8 * (int64_t)ntiles);
  r.bins = r.recs + rs_align((int64_t)kRecBytes * (ntris + kClipRecs));
  r.bin_cap = kBinsPerTri * (ntris + kClipRecs);
  r.attr = r.bins + rs_align(2 * (int64_t)r.bin_cap);
  r.tuv = r.attr + (smooth ? rs_align((int64_t)4 * kAttrWords * (ntris + kClipRecs)) : 0);
  r.total = r.tuv + (textured ? rs_align((int64_t)4 * kTuvWords * (ntris + kClipRecs)) : 0);
  return r;
}

// tiles of edge 1 << shift covering a w x h image
__host__ __device__ inline int32_t tiles_of(int32_t w, int32_t h, int shift = 4) {
  const int t = 1 << shift;
  return ((w + t - 1) >> shift) * ((h + t - 1) >> shift);
}

// Mesh templates and shading constants (device copy of the descriptor).
struct alignas(16) Templates {
  float sphere_v[kMaxTplVerts][3];
  float cube_v[kMaxTplVerts][3];
  float ground_v[kMaxGroundVerts][3];
  uint8_t sphere_f[kMaxTplFaces][3];
  uint8_t cube_f[kMaxTplFaces][3];
  uint8_t ground_f[kMaxGroundFaces][3];
  float sphere_n[kMaxTplFaces][3];
  float cube_n[kMaxTplFaces][3];
  int32_t sphere_nv, sphere_nf, cube_nv, cube_nf, ground_nv, ground_nf;
  float light[3];
  float palette[8][3];
  float ground_albedo;
  float near_w;
  float guard;
  // textured worlds: texture size (0: untextured) and the ground's texture
  // repeats per metre
  int32_t tex_w, tex_h;
  float ground_uv_scale;
};

struct PhysConsts {
  float h;        // dt / substeps
  float hh;       // h / 2
  float k, c;
  float g[3];
  int32_t substeps;
  float mu, v_eps;  // regularized Coulomb friction (mu = 0: none)
  int32_t edge;     // box-box edge-edge points (separating-axis test)
};

// Pointers into the world arena used by the kernels.
struct WorldDev {
  EnvDev* envs;
  CamDev* cams;
  // static per body
  const uint8_t* type;
  const uint8_t* albedo;
  const float* size;
  const float* rbound;
  const float* inv_m;
  const float* inv_I;
  const float* box;          // per body [6]: half-extents xyz, principal moments xyz (boxes)
  const int32_t* prim_base;  // env-local primitive id of the body's first face
  const int32_t* vert_base;  // env-local vertex index of the body's first vertex
  const uint8_t* prim_body;  // per env: body of each primitive (kGroundBody: ground)
  const uint8_t* vert_body;  // per env: body of each template vertex
  // dynamic state: state[buf][comp * cap_bodies + body]
  float* state[2];
  int64_t cap_bodies;
  // images
  uint8_t* rgb;
  uint32_t* depth;
  int32_t* winners;    // debug only (nullable)
  int32_t* coverage;   // debug only (nullable)
  // debug contact sets: per env [substeps][1 + 2*pair_cap]
  int32_t* contacts;   // nullable
  int32_t pair_cap;
  uint32_t* env_flags;
  const Templates* tpl;
  const uint8_t* texture;   // textured worlds: RGB8 texels [tex_h][tex_w][3]; nullptr: none
  unsigned char* rscratch;  // raster scratch of every camera (CamDev::rs_off)
  // policy actions: per env act_dim floats, the force on body b in
  // [3b, 3b + 3); act_on[env] != 0 once the policy has acted on the env
  float* actions;           // nullable (no policy)
  uint8_t* act_on;
  int32_t act_dim;
};

// Host-side launchers (implemented next to the kernels).
struct PhysLaunch {
  const int32_t* work;     // env ids, LPT order
  int32_t n_work;
  int32_t max_bodies;      // over the listed envs
  int32_t parity;          // buffer read; writes 1 - parity
  int32_t nsteps;
  int32_t persistent;      // 0: one workgroup per env; >0: that many resident workgroups
  int32_t* queue;          // persistent work counter (one int), nullable otherwise
  int32_t prio;            // wave issue priority 0..3 (s_setprio) of the physics waves
  int32_t broadphase;      // 0 auto, 1 uniform grid hash, 2 all pairs
  int32_t pack;            // envs per wave when every env has at most 32 bodies (1 or 2)
};

// Tile-kernel job: the camera id in the low bits, the number of the row's
// tiles the workgroup takes, less one, above them.
constexpr int kJobWavesShift = 28;
constexpr int32_t kJobCamMask = (1 << kJobWavesShift) - 1;

struct RasterLaunch {
  const int32_t* work;     // camera ids, LPT order (setup kernel, one workgroup each)
  int32_t n_work;
  const int2* tiles;       // tile kernel: per workgroup (camera | (n - 1) << kJobWavesShift,
                           // tx | ty << 16): the n <= tile_waves tiles tx .. tx + n - 1 of
                           // tile row ty; -1 for padding entries
  int32_t n_tile_groups;
  int32_t max_verts;       // over the listed cameras' envs
  int32_t max_tiles;
  int32_t max_bodies;
  int32_t max_tris;
  int32_t parity;          // state buffer rendered
  int32_t threads;         // setup workgroup size (multiple of 64)
  int32_t bin_limit;       // bin entries an image may use (0: its whole capacity)
  int32_t persistent;      // setup kernel: resident workgroups pulling images
  int32_t* queue;
  int32_t prio;            // setup and tile kernels: wave issue priority 0..3 (s_setprio)
  int32_t near_clip;       // setup kernel: cut triangles crossing the near plane
  int32_t smooth;          // per-pixel shading of interpolated vertex normals
  int32_t tile_shift;      // raster tiles of edge 1 << tile_shift (8, 16 or 32 pixels)
  int32_t tile_waves;      // tile kernel: tiles (one per wave) per workgroup, 1, 2 or 4
  // fused kernel only (raster_fused_plan): LDS bytes reserved for the tile
  // pass's z-buffers, compact records and bin entries an image keeps in LDS
  int32_t lds_zone0, lrec_cap, lbin_cap;
};

// Timing events of one launch (a kernel or a chain of them): `start` is
// recorded when its first kernel begins and `stop` when its last one ends,
// through HIP's extended launch, so that the span is the kernels' own time.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  bool started = false, stopped = false;
};

template <typename K, typename... A>
inline void timed_launch(LaunchEvents* ev, bool first, bool last, K kernel, dim3 grid, dim3 block, uint32_t lds,
                         hipStream_t s, A... args) {
  hipEvent_t e0 = (ev && first && !ev->started) ? ev->start : nullptr;
  hipEvent_t e1 = (ev && last) ? ev->stop : nullptr;
  if (!e0 && !e1) {
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    return;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, lds, s, e0, e1, 0, args...);
  if (e0) ev->started = true;
  if (e1) ev->stopped = true;
}

hipError_t launch_physics(const WorldDev& w, const PhysConsts& pc, const PhysLaunch& l,
                          hipStream_t s, LaunchEvents* ev = nullptr);

// The policy over M envs: layer 1 split over `splits` chunks of `kchunk`
// observation values (MFMA), then layers 2 and 3 and the actions.
struct PolicyLaunch {
  const int32_t* envs;     // env ids, one per row
  int32_t M;               // rows
  int32_t K;               // observation length 4 W H
  int32_t krgb;            // 3 W H: start of the depth bytes
  int32_t H, A;            // hidden units, actions
  int32_t splits, kchunk;  // K = splits kchunk, kchunk a multiple of 32
  const uint16_t* w1t;     // [K / 32][H][32] bfloat16: W1 in panels of one MFMA k step
  const float* b1;
  const float* w2;         // [H][H]
  const float* b2;
  const float* w3;         // [H][A]
  const float* b3;
  float a_max;
  float* partial;          // [splits][M][H]; layered: also layer 2's [s2][M][H] and layer 3's [s3][M][Ap]
  // layers 2 and 3 as batched products (H a multiple of 64) instead of the
  // per-env head
  int32_t layered;
  int32_t s2, s3;          // K splits of layers 2 and 3 (each divides H / 16)
  int32_t Ap;              // A rounded up to a multiple of 64
  const float* w3p;        // [H][Ap]: W3 with zero columns beyond A
  float* h1;               // [M][H]
  float* h2;               // [M][H]
};
hipError_t launch_policy(const WorldDev& w, const PolicyLaunch& l, hipStream_t s, LaunchEvents* ev = nullptr);
// The render work of a state buffer: setup (geometry, records, bins) into the
// cameras' scratch of that buffer, then the tiles (pixels) from it.
hipError_t launch_raster_setup(const WorldDev& w, const RasterLaunch& l, hipStream_t s, LaunchEvents* ev = nullptr);
hipError_t launch_raster_tiles(const WorldDev& w, const RasterLaunch& l, hipStream_t s, LaunchEvents* ev = nullptr);
size_t raster_lds_bytes(const RasterLaunch& l);
hipError_t raster_configure(size_t lds_bytes);
// Fused setup + tiles, one workgroup of l.threads per image (flat shading, no
// near-plane clipping): raster_fused_plan fills the LDS fields of l (at most
// max_recs records in LDS when max_recs > 0) and returns the dynamic LDS
// bytes (0: the images do not fit in LDS).
constexpr size_t kFusedLdsMax = 160 * 1024;
size_t raster_fused_plan(RasterLaunch* l, bool debug, int max_recs);
hipError_t raster_fused_configure(size_t lds_bytes);
hipError_t launch_raster_fused(const WorldDev& w, const RasterLaunch& l, size_t lds, hipStream_t s,
                               LaunchEvents* ev = nullptr);
hipError_t launch_reset_queue(int32_t* q, hipStream_t s);

// Workgroups of `kernel` (threads per workgroup, dynamic LDS bytes) that the
// current device holds at once: its occupancy per CU times the CU count.
// Cached per (device, kernel, shape); *out is 0 on failure.
hipError_t resident_workgroups(const void* kernel, int threads, size_t dyn_lds, int* out);

// The grid of a persistent launch of `items` work items: `persistent` > 0
// workgroups, or (< 0) the resident count from resident_workgroups, at most
// `items` either way.
hipError_t persistent_grid(int persistent, int items, const void* kernel, int threads, size_t dyn_lds,
                           int* grid);

}  // namespace vuda
