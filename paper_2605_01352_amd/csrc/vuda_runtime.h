// Host-side state of a world (internal to libvuda).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "vuda.h"
#include "vuda_internal.h"

namespace vuda {

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
// Checks of an env batch against the limits of the ABI (sizes, arrays
// present, body types, boxes' extents, primitive counts); fills the body,
// camera and pixel totals.
int validate_batch(const vuda_env_batch& b, const vuda_render_desc& r, int64_t* nb_out, int32_t* nc_out,
                   int64_t* npix_out);

// First-fit allocator of index ranges in [0, cap).
class RangeAlloc {
 public:
  void init(int64_t cap) {
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  int64_t alloc(int64_t n);
  void release(int64_t start, int64_t n);
  // mark [start, start + n) as used (it must be free)
  void take(int64_t start, int64_t n) {
    if (n <= 0) return;
    auto it = free_.upper_bound(start);
    --it;
    const int64_t s = it->first, e = it->second;
    free_.erase(it);
    if (s < start) free_[s] = start;
    if (start + n < e) free_[start + n] = e;
  }
  int64_t free_total() const {
    int64_t t = 0;
    for (auto& kv : free_) t += kv.second - kv.first;
    return t;
  }

 private:
  std::map<int64_t, int64_t> free_;  // start -> end
};

// Device storage of one version of a work list.  A rebuilt list goes into
// the other version; a version is written again only after the fence events
// recorded when it was replaced have completed, so launches already enqueued
// keep reading the list they were given.
struct ListBuf {
  int32_t* dptr = nullptr;
  int32_t cap = 0;
  int2* tptr = nullptr;
  int32_t tcap = 0;
  hipEvent_t fence[2] = {nullptr, nullptr};
  int nfence = 0;  // fence events pending (0: free)
};

struct WorkList {
  ListBuf buf[2];
  int cur = 0;
  bool built = false;
  const int32_t* dptr = nullptr;  // the current version
  const int2* tptr = nullptr;     // render: tile-kernel jobs (camera and tile count, first tile)
  int32_t n_groups = 0;
  bool dirty = true;   // rebuild before the next use
  int32_t n = 0;
  int32_t max_bodies = 0;
  int32_t max_verts = 0;
  int32_t max_tris = 0;
  int32_t max_tiles = 0;
};

struct Tuning {
  int32_t raster_threads = 256;
  int32_t rec_cap = 0;  // bin entries an image may use (0: its whole capacity)
  int32_t phys_persistent = 0;
  int32_t raster_persistent = 0;
  bool graphs = false;
  int32_t phys_prio = 0;
  int32_t broadphase = 0;
  bool timing = false;
  bool presetup = true;
  bool policy_layered = false;  // layers 2-3 as batched products at any hidden size
  int32_t phys_pack = 1;         // envs of at most 32 bodies per physics wave (1 or 2)
  int32_t tile_shift = 4;        // raster tile edge 1 << tile_shift pixels
  int32_t tile_waves = 2;        // tiles (one per wave) per tile-kernel workgroup: 1, 2 or 4
  int32_t tile_prio = 0;         // wave issue priority 0..3 of the tile kernel
  bool raster_fused = false;     // setup and tiles in one kernel, records in LDS
  int32_t fused_recs = 0;        // records a fused image keeps in LDS at most (0: automatic)
};

// kernels of the step loop (index of their timing events)
constexpr int kKernelPhysics = 0, kKernelSetup = 1, kKernelTiles = 2, kKernelPolicy = 3, kKernelFused = 4;
constexpr int kKernelKinds = 5;

// Metric depth of one camera image: out[out_off + i] for its npix pixels
// from depth[pix_off + i], view depth = beta / (D / (2^24 - 1) - alpha).
struct MetricCam {
  int64_t pix_off, out_off, npix;
  double alpha, beta;
};
hipError_t launch_depth_metric(const uint32_t* depth, const MetricCam* cams, int32_t ncams, int64_t max_pix,
                               float* out, hipStream_t s);

// Hidden sizes: up to kPolicyHeadMax the per-env head kernel runs layers 2
// and 3; above it (multiples of 64) they run as batched products.
constexpr int32_t kPolicyHeadMax = 1024, kPolicyHiddenMax = 8192;

// The MLP policy of a world (device copies of its weights).
struct Policy {
  bool set = false;
  int32_t in_w = 0, in_h = 0, H = 0, A = 0;
  float a_max = 0.0f;
  uint16_t* w1t = nullptr;  // [K / 32][H][32] bfloat16
  float* wf = nullptr;      // b1 [H], w2 [H][H], b2 [H], w3 [H][A], b3 [A]
  float* w3p = nullptr;     // [H][A rounded up to 64] (hidden a multiple of 64)
  float* partial = nullptr;
  int64_t partial_cap = 0;  // floats
};

}  // namespace vuda

struct vuda_world {
  int device = -1;
  vuda_phys_params phys{};
  vuda::PhysConsts pc{};
  vuda::Templates tpl{};
  bool debug = false;
  bool near_clip = false;  // VUDA_FLAG_NEAR_CLIP
  bool smooth = false;     // VUDA_FLAG_SMOOTH
  bool textured = false;   // VUDA_FLAG_TEXTURE
  int32_t pair_cap = 1024;
  int32_t cap_envs = 0, cap_cams = 0;
  int64_t cap_bodies = 0, cap_pixels = 0;
  uint64_t hbm_budget = 0;
  int32_t n_envs_hi = 0;

  // device arena
  unsigned char* arena = nullptr;
  size_t arena_bytes = 0;
  vuda_allocator allocator{};
  bool has_allocator = false;
  struct {
    size_t envs, cams, type, albedo, size, rbound, inv_m, inv_I, box, prim_base, vert_base, prim_body, vert_body, state0,
        state1, rgb, depth, flags, tpl, texture, queues, winners, coverage, contacts, rs;
  } off_{};
  vuda::WorldDev dev{};
  int32_t* queues = nullptr;

  // host mirrors
  std::vector<vuda::EnvDev> env_host;
  std::vector<uint8_t> env_parity;
  std::vector<uint8_t> env_active;
  std::vector<uint8_t> env_retired;  // retired, not yet released
  std::vector<vuda::CamDev> cam_host;
  vuda::RangeAlloc slots, bodies, camslots, pixels, primspace, vertspace;
  vuda::RangeAlloc rsspace;  // raster scratch, in 256-byte units
  int64_t cap_prims = 0, cap_verts = 0, cap_rs = 0;

  // streams: mode 0 serialized (s_sim == s_render == s_serial), 1 CU-masked
  // (a partition), 2 streams over every CU (masks of all CUs, for hardware
  // queues of their own)
  hipStream_t s_serial = nullptr, s_sim = nullptr, s_render = nullptr;
  hipStream_t s_setup = nullptr;  // raster setup of the pipelined schedule (the step's CUs)
  int mode = 0;
  float cu_split = 0.0f;

  // dependency events per env: the last step, and the last render of each
  // buffer; render_state_ev: the last render of each buffer whose kernels
  // read the state buffer itself (its own raster setup, or the fused kernel)
  std::vector<int64_t> step_ev;
  std::vector<int64_t> render_ev[2];
  std::vector<int64_t> render_state_ev[2];
  std::vector<hipEvent_t> evpool;
  int64_t next_event = 0;

  // launch timing: per kernel (kKernel*) and launch, an event before and one
  // after; tev_used[k] launches recorded since the last read
  std::vector<hipEvent_t> tev[vuda::kKernelKinds];
  size_t tev_used[vuda::kKernelKinds] = {0, 0, 0, 0, 0};
  // per env: the raster scratch of its current state buffer holds that
  // state's setup
  std::vector<uint8_t> setup_ok;
  // policy: weights, and per env its actions (WorldDev::actions, act_on)
  vuda::Policy pol;
  float* actions = nullptr;
  uint8_t* act_on = nullptr;
  // metric-depth fetches: camera table and float staging, grown on demand
  vuda::MetricCam* metric_cams = nullptr;
  int64_t metric_cams_cap = 0;
  float* metric_buf = nullptr;
  int64_t metric_buf_cap = 0;

  std::map<std::tuple<int, int32_t, int32_t>, vuda::WorkList> lists;
  std::map<std::tuple<int, int32_t, int32_t, int>, hipGraphExec_t> graphs;
  vuda::Tuning tune;
  size_t lds_configured = 64 * 1024;

  int alloc_arena(const vuda_allocator* a);
  int upload(const vuda_env_batch& b, int32_t e0, int64_t b0, int32_t c0, int64_t p0, int64_t m0,
             int64_t v0, int64_t r0, int parity, hipStream_t s);
  void map_sizes(const vuda_env_batch& b, int64_t* prims, int64_t* verts) const;
  int64_t rs_units(const vuda_env_batch& b) const;
  int32_t env_tris(const vuda_env_batch& b, int32_t e) const;
  void free_all();
  int make_streams(float split);
  void destroy_streams();
  int drain();
  // Host-synchronous copy and fill that do not wait for the world's work
  // streams.  Streams with a CU mask (every co-scheduled mode) are blocking
  // streams, which any operation on the null stream waits for; outside the
  // serialized mode these go through the serial stream, which is then idle
  // and non-blocking.
  hipError_t copy_now(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
  hipError_t fill_now(void* dst, int value, size_t bytes);
  int init_events();
  int new_event(hipStream_t s, int64_t* id);
  int reserve_event(int64_t* id, hipEvent_t* ev);
  int wait_event(hipStream_t s, int64_t id);
  void invalidate_lists();
  int get_list(int phase, int32_t lo, int32_t hi, const vuda::WorkList** out);
  int range_parity(int32_t lo, int32_t hi, int* parity);
  int check_range(int32_t lo, int32_t hi);
  int enqueue_physics(const vuda::WorkList& L, int parity, hipStream_t s, vuda::LaunchEvents* ev = nullptr);
  int raster_launch_of(const vuda::WorkList& L, int parity, int32_t* queue, vuda::RasterLaunch* out);
  // the fused raster launch of a render list; *lds = 0 when the two-kernel
  // path renders it (fused off, smooth shading, near-plane clipping, or an
  // env too large for LDS)
  int fused_launch_of(const vuda::WorkList& L, int parity, int32_t* queue, vuda::RasterLaunch* out, size_t* lds);
  size_t lds_fused_configured = 64 * 1024;
  int enqueue_kernel(int kind, const vuda::WorkList& L, int parity, hipStream_t s, int32_t* queue,
                     vuda::LaunchEvents* ev = nullptr);
  int run_kernel(int kind, const vuda::WorkList& L, int parity, int32_t lo, int32_t hi, hipStream_t s,
                 int32_t* queue, hipEvent_t done = nullptr);
  // the launch itself: direct, timed, or through a captured graph
  int launch_kernel(int kind, const vuda::WorkList& L, int parity, int32_t lo, int32_t hi, hipStream_t s,
                    int32_t* queue);
  int check_flags();
  int32_t active_midpoint();
  // events that complete when everything enqueued so far on the world's
  // streams has run (one per stream in use); returns how many were recorded
  int mark(hipEvent_t ev[2]);
  // retire envs [first, first + n): no later launch includes them, their
  // memory stays allocated until vuda_release
  int retire(int32_t first, int32_t n);
  void free_policy();
  int policy_launch_of(const vuda::WorkList& L, vuda::PolicyLaunch* out);
};
