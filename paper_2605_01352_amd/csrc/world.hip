// Host runtime of libvuda: world arena, env/camera tables, streams and the
// co-scheduling switch, per-env dependency tracking, fetch and admission.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "vuda.h"
#include "vuda_internal.h"
#include "vuda_runtime.h"

using namespace vuda;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

int vuda::fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int vuda::hip_fail(hipError_t e, const char* what) {
  return fail(VUDA_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e__ = (x);                           \
    if (e__ != hipSuccess) return hip_fail(e__, #x); \
  } while (0)

extern "C" const char* vuda_strerror(int code) {
  switch (code) {
    case VUDA_OK: return "ok";
    case VUDA_EINVAL: return "invalid argument";
    case VUDA_ENOMEM: return "out of device memory or over the HBM budget";
    case VUDA_EHIP: return "HIP runtime error";
    case VUDA_ENUMERIC: return "non-finite physics state";
    case VUDA_EOVERFLOW: return "contact or bin capacity exceeded";
    case VUDA_EBUSY: return "no free slots or budget";
    default: return "unknown error";
  }
}

extern "C" const char* vuda_last_error_message(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// range allocator (first fit over [0, cap))
// ---------------------------------------------------------------------------

int64_t RangeAlloc::alloc(int64_t n) {
  if (n == 0) return 0;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second - it->first >= n) {
      const int64_t s = it->first;
      const int64_t e = it->second;
      free_.erase(it);
      if (s + n < e) free_[s + n] = e;
      return s;
    }
  }
  return -1;
}

void RangeAlloc::release(int64_t s, int64_t n) {
  if (n == 0) return;
  int64_t e = s + n;
  auto nx = free_.lower_bound(s);
  if (nx != free_.end() && nx->first == e) {
    e = nx->second;
    free_.erase(nx);
  }
  auto it = free_.lower_bound(s);
  if (it != free_.begin()) {
    auto pv = std::prev(it);
    if (pv->second == s) {
      pv->second = e;
      return;
    }
  }
  free_[s] = e;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int vuda::validate_batch(const vuda_env_batch& b, const vuda_render_desc& r, int64_t* nb_out,
                   int32_t* nc_out, int64_t* npix_out) {
  if (b.n_envs < 0) return fail(VUDA_EINVAL, "n_envs < 0");
  if (b.n_envs == 0) {
    *nb_out = 0; *nc_out = 0; *npix_out = 0;
    return VUDA_OK;
  }
  if (!b.body_off || !b.cam_off) return fail(VUDA_EINVAL, "body_off / cam_off missing");
  if (b.body_off[0] != 0 || b.cam_off[0] != 0) return fail(VUDA_EINVAL, "offsets must start at 0");
  for (int e = 0; e < b.n_envs; ++e) {
    const int nb = b.body_off[e + 1] - b.body_off[e];
    if (nb < 0 || nb > kMaxBodies) return fail(VUDA_EINVAL, "env %d: %d bodies (0..%d)", e, nb, kMaxBodies);
    const int nc = b.cam_off[e + 1] - b.cam_off[e];
    if (nc < 0) return fail(VUDA_EINVAL, "env %d: negative camera count", e);
  }
  const int64_t nb = b.body_off[b.n_envs];
  const int32_t nc = b.cam_off[b.n_envs];
  if (nb > 0 && (!b.type || !b.size || !b.rbound || !b.inv_m || !b.inv_I || !b.albedo || !b.pos ||
                 !b.vel || !b.quat || !b.omega))
    return fail(VUDA_EINVAL, "body arrays missing");
  if (nc > 0 && (!b.cam_vp || !b.cam_w || !b.cam_h)) return fail(VUDA_EINVAL, "camera arrays missing");
  for (int64_t i = 0; i < nb; ++i) {
    if (b.type[i] > 2) return fail(VUDA_EINVAL, "body %lld: type %d", (long long)i, (int)b.type[i]);
    if (b.type[i] == 2) {
      if (!b.ext || !b.inertia) return fail(VUDA_EINVAL, "body %lld: a box needs ext and inertia", (long long)i);
      for (int k = 0; k < 3; ++k)
        if (!(b.ext[3 * i + k] > 0.0f) || !std::isfinite(b.ext[3 * i + k]) || !(b.inertia[3 * i + k] > 0.0f) ||
            !std::isfinite(b.inertia[3 * i + k]))
          return fail(VUDA_EINVAL, "body %lld: box extents/inertia", (long long)i);
    }
    if (b.albedo[i] > 7) return fail(VUDA_EINVAL, "body %lld: albedo %d", (long long)i, (int)b.albedo[i]);
    if (!(b.size[i] > 0.0f) || !(b.rbound[i] >= b.size[i]))
      return fail(VUDA_EINVAL, "body %lld: size/rbound", (long long)i);
  }
  int64_t npix = 0;
  for (int32_t c = 0; c < nc; ++c) {
    if (b.cam_w[c] < 1 || b.cam_h[c] < 1 || b.cam_w[c] > 4096 || b.cam_h[c] > 4096)
      return fail(VUDA_EINVAL, "camera %d: size %dx%d", c, b.cam_w[c], b.cam_h[c]);
    npix += (int64_t)b.cam_w[c] * b.cam_h[c];
  }
  // primitive ids must fit 16 bits
  for (int e = 0; e < b.n_envs; ++e) {
    int64_t tris = r.ground_nf;
    for (int32_t i = b.body_off[e]; i < b.body_off[e + 1]; ++i) tris += b.type[i] ? r.cube_nf : r.sphere_nf;
    if (tris > 65535) return fail(VUDA_EINVAL, "env %d: %lld primitives (max 65535)", e, (long long)tris);
  }
  *nb_out = nb;
  *nc_out = nc;
  *npix_out = npix;
  return VUDA_OK;
}

static int validate_render(const vuda_render_desc& r) {
  if (!r.sphere_v || !r.sphere_f || !r.sphere_n || !r.cube_v || !r.cube_f || !r.cube_n ||
      !r.ground_v || !r.ground_f)
    return fail(VUDA_EINVAL, "render templates missing");
  if (r.sphere_nv < 3 || r.sphere_nv > kMaxTplVerts || r.cube_nv < 3 || r.cube_nv > kMaxTplVerts ||
      r.ground_nv < 3 || r.ground_nv > kMaxGroundVerts)
    return fail(VUDA_EINVAL, "template vertex counts");
  if (r.sphere_nf < 1 || r.sphere_nf > kMaxTplFaces || r.cube_nf < 1 || r.cube_nf > kMaxTplFaces ||
      r.ground_nf < 1 || r.ground_nf > kMaxGroundFaces)
    return fail(VUDA_EINVAL, "template face counts");
  auto chk = [](const int32_t* f, int nf, int nv) {
    for (int i = 0; i < 3 * nf; ++i)
      if (f[i] < 0 || f[i] >= nv) return false;
    return true;
  };
  if (!chk(r.sphere_f, r.sphere_nf, r.sphere_nv) || !chk(r.cube_f, r.cube_nf, r.cube_nv) ||
      !chk(r.ground_f, r.ground_nf, r.ground_nv))
    return fail(VUDA_EINVAL, "template face index out of range");
  if (!(r.near_w > 0.0f) || !(r.guard > 0.0f) || r.guard > 65536.0f)
    return fail(VUDA_EINVAL, "near_w / guard");
  return VUDA_OK;
}

static void fill_templates(Templates& t, const vuda_render_desc& r) {
  memset(&t, 0, sizeof(t));
  for (int i = 0; i < r.sphere_nv; ++i)
    for (int k = 0; k < 3; ++k) t.sphere_v[i][k] = r.sphere_v[3 * i + k];
  for (int i = 0; i < r.cube_nv; ++i)
    for (int k = 0; k < 3; ++k) t.cube_v[i][k] = r.cube_v[3 * i + k];
  for (int i = 0; i < r.ground_nv; ++i)
    for (int k = 0; k < 3; ++k) t.ground_v[i][k] = r.ground_v[3 * i + k];
  for (int i = 0; i < r.sphere_nf; ++i)
    for (int k = 0; k < 3; ++k) {
      t.sphere_f[i][k] = (uint8_t)r.sphere_f[3 * i + k];
      t.sphere_n[i][k] = r.sphere_n[3 * i + k];
    }
  for (int i = 0; i < r.cube_nf; ++i)
    for (int k = 0; k < 3; ++k) {
      t.cube_f[i][k] = (uint8_t)r.cube_f[3 * i + k];
      t.cube_n[i][k] = r.cube_n[3 * i + k];
    }
  for (int i = 0; i < r.ground_nf; ++i)
    for (int k = 0; k < 3; ++k) t.ground_f[i][k] = (uint8_t)r.ground_f[3 * i + k];
  t.sphere_nv = r.sphere_nv; t.sphere_nf = r.sphere_nf;
  t.cube_nv = r.cube_nv; t.cube_nf = r.cube_nf;
  t.ground_nv = r.ground_nv; t.ground_nf = r.ground_nf;
  for (int k = 0; k < 3; ++k) t.light[k] = r.light[k];
  for (int i = 0; i < 8; ++i)
    for (int k = 0; k < 3; ++k) t.palette[i][k] = r.palette[3 * i + k];
  t.ground_albedo = r.ground_albedo;
  t.near_w = r.near_w;
  t.guard = r.guard;
  t.tex_w = t.tex_h = 0;
  t.ground_uv_scale = r.ground_uv_scale;
}

// ---------------------------------------------------------------------------
// world lifetime
// ---------------------------------------------------------------------------

int vuda_world::alloc_arena(const vuda_allocator* a) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  const int64_t B = std::max<int64_t>(cap_bodies, 1);
  const int64_t P = std::max<int64_t>(cap_pixels, 1);
  const int64_t E = std::max<int32_t>(cap_envs, 1);
  const int64_t C = std::max<int32_t>(cap_cams, 1);
  off_.envs = take(sizeof(EnvDev) * E);
  off_.cams = take(sizeof(CamDev) * C);
  off_.type = take(B);
  off_.albedo = take(B);
  off_.size = take(4 * B);
  off_.rbound = take(4 * B);
  off_.inv_m = take(4 * B);
  off_.inv_I = take(4 * B);
  off_.box = take(4 * 6 * B);
  off_.prim_base = take(4 * B);
  off_.vert_base = take(4 * B);
  off_.prim_body = take(std::max<int64_t>(cap_prims, 1));
  off_.vert_body = take(std::max<int64_t>(cap_verts, 1));
  off_.state0 = take(4 * (size_t)kStateComps * B);
  off_.state1 = take(4 * (size_t)kStateComps * B);
  off_.rgb = take(3 * P + 16);
  off_.depth = take(4 * P);
  off_.flags = take(4 * E + 4);
  off_.tpl = take(sizeof(Templates));
  off_.texture = take(textured ? 3 * (size_t)tpl.tex_w * (size_t)tpl.tex_h : 0);
  off_.queues = take(64);
  off_.rs = take(256 * (size_t)std::max<int64_t>(cap_rs, 1));
  if (debug) {
    off_.winners = take(4 * P);
    off_.coverage = take(4 * P);
    off_.contacts = take(4 * (size_t)E * phys.substeps * (1 + 2 * (size_t)pair_cap));
  }
  arena_bytes = o;
  if (hbm_budget && arena_bytes > hbm_budget)
    return fail(VUDA_ENOMEM, "arena of %zu bytes exceeds the HBM budget of %llu", arena_bytes,
                (unsigned long long)hbm_budget);
  if (a && a->alloc) {
    allocator = *a;
    has_allocator = true;
    arena = (unsigned char*)a->alloc(arena_bytes, a->ctx);
    if (!arena) return fail(VUDA_ENOMEM, "allocator returned NULL for %zu bytes", arena_bytes);
  } else {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, arena_bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(VUDA_ENOMEM, "hipMalloc(%zu): %s", arena_bytes, hipGetErrorString(e));
    }
    arena = (unsigned char*)p;
  }
  HIPCHK(hipMemset(arena, 0, arena_bytes));
  dev.envs = (EnvDev*)(arena + off_.envs);
  dev.cams = (CamDev*)(arena + off_.cams);
  dev.type = arena + off_.type;
  dev.albedo = arena + off_.albedo;
  dev.size = (float*)(arena + off_.size);
  dev.rbound = (float*)(arena + off_.rbound);
  dev.inv_m = (float*)(arena + off_.inv_m);
  dev.inv_I = (float*)(arena + off_.inv_I);
  dev.box = (float*)(arena + off_.box);
  dev.prim_base = (int32_t*)(arena + off_.prim_base);
  dev.vert_base = (int32_t*)(arena + off_.vert_base);
  dev.prim_body = arena + off_.prim_body;
  dev.vert_body = arena + off_.vert_body;
  dev.state[0] = (float*)(arena + off_.state0);
  dev.state[1] = (float*)(arena + off_.state1);
  dev.cap_bodies = B;
  dev.rgb = arena + off_.rgb;
  dev.depth = (uint32_t*)(arena + off_.depth);
  dev.env_flags = (uint32_t*)(arena + off_.flags);
  dev.tpl = (const Templates*)(arena + off_.tpl);
  dev.texture = textured ? arena + off_.texture : nullptr;
  dev.rscratch = arena + off_.rs;
  queues = (int32_t*)(arena + off_.queues);
  dev.winners = debug ? (int32_t*)(arena + off_.winners) : nullptr;
  dev.coverage = debug ? (int32_t*)(arena + off_.coverage) : nullptr;
  dev.contacts = debug ? (int32_t*)(arena + off_.contacts) : nullptr;
  dev.pair_cap = pair_cap;
  return VUDA_OK;
}

// Upload a batch of envs into slots [e0, e0 + n), bodies from b0, cameras
// from c0, pixels from p0; state goes to buffer `parity`.
// Per-env primitive and vertex maps start on 16-byte boundaries so that the
// raster kernel can copy them with 16-byte loads.
static int64_t map_round(int64_t n) { return (n + 15) & ~(int64_t)15; }

void vuda_world::map_sizes(const vuda_env_batch& b, int64_t* prims, int64_t* verts) const {
  int64_t np = 0, nv = 0;
  for (int e = 0; e < b.n_envs; ++e) {
    int64_t ep = tpl.ground_nf, ev = tpl.ground_nv;
    for (int32_t i = b.body_off[e]; i < b.body_off[e + 1]; ++i) {
      ep += b.type[i] ? tpl.cube_nf : tpl.sphere_nf;
      ev += b.type[i] ? tpl.cube_nv : tpl.sphere_nv;
    }
    np += map_round(ep);
    nv += map_round(ev);
  }
  *prims = np;
  *verts = nv;
}

int32_t vuda_world::env_tris(const vuda_env_batch& b, int32_t e) const {
  int32_t n = tpl.ground_nf;
  for (int32_t i = b.body_off[e]; i < b.body_off[e + 1]; ++i) n += b.type[i] ? tpl.cube_nf : tpl.sphere_nf;
  return n;
}

// Raster scratch of a batch's cameras, in 256-byte units.
int64_t vuda_world::rs_units(const vuda_env_batch& b) const {
  int64_t u = 0;
  for (int32_t e = 0; e < b.n_envs; ++e) {
    const int32_t nt = env_tris(b, e);
    for (int32_t c = b.cam_off[e]; c < b.cam_off[e + 1]; ++c)
      u += 2 * (rs_layout(nt, tiles_of(b.cam_w[c], b.cam_h[c], kTileShiftMin), smooth, textured).total / 256);
  }
  return u;
}

int vuda_world::upload(const vuda_env_batch& b, int32_t e0, int64_t b0, int32_t c0, int64_t p0,
                       int64_t m0, int64_t v0, int64_t r0, int parity, hipStream_t s) {
  const int64_t nb = b.n_envs ? b.body_off[b.n_envs] : 0;
  const int32_t nc = b.n_envs ? b.cam_off[b.n_envs] : 0;
  std::vector<EnvDev> envs(b.n_envs);
  std::vector<int32_t> pbase(nb), vbase(nb);
  std::vector<uint8_t> pmap, vmap;
  for (int e = 0; e < b.n_envs; ++e) {
    EnvDev& d = envs[e];
    d.body_off = (int32_t)(b0 + b.body_off[e]);
    d.n_bodies = b.body_off[e + 1] - b.body_off[e];
    d.cam_off = c0 + b.cam_off[e];
    d.n_cams = b.cam_off[e + 1] - b.cam_off[e];
    d.prim_map = m0 + (int64_t)pmap.size();
    d.vert_map = v0 + (int64_t)vmap.size();
    pmap.insert(pmap.end(), tpl.ground_nf, kGroundBody);
    vmap.insert(vmap.end(), tpl.ground_nv, kGroundBody);
    int32_t pv = tpl.ground_nf, vv = tpl.ground_nv;
    for (int32_t i = b.body_off[e]; i < b.body_off[e + 1]; ++i) {
      pbase[i] = pv;
      vbase[i] = vv;
      const int nf = b.type[i] ? tpl.cube_nf : tpl.sphere_nf;
      const int nvt = b.type[i] ? tpl.cube_nv : tpl.sphere_nv;
      pmap.insert(pmap.end(), nf, (uint8_t)(i - b.body_off[e]));
      vmap.insert(vmap.end(), nvt, (uint8_t)(i - b.body_off[e]));
      pv += nf;
      vv += nvt;
    }
    d.n_tris = pv;
    d.n_verts = vv;
    pmap.resize(map_round((int64_t)pmap.size()), kGroundBody);
    vmap.resize(map_round((int64_t)vmap.size()), kGroundBody);
  }
  std::vector<CamDev> cams(nc);
  int64_t po = p0, ro = 256 * r0;
  for (int e = 0; e < b.n_envs; ++e) {
    const int32_t nt = envs[e].n_tris;
    for (int32_t c = b.cam_off[e]; c < b.cam_off[e + 1]; ++c) {
      CamDev& d = cams[c];
      memcpy(d.vp, b.cam_vp + 16 * (size_t)c, sizeof(d.vp));
      d.w = b.cam_w[c];
      d.h = b.cam_h[c];
      d.pix_off = po;
      d.env = e0 + e;
      d.n_tris = nt;
      d.rs_off = ro;
      // the tile table has room for the smallest tiles
      const RsLayout rl = rs_layout(nt, tiles_of(d.w, d.h, kTileShiftMin), smooth, textured);
      d.rs_recs = (int32_t)rl.recs;
      d.rs_bins = (int32_t)rl.bins;
      d.rs_total = (int32_t)rl.total;
      d.rs_attr = (int32_t)rl.attr;
      d.rs_tuv = (int32_t)rl.tuv;
      po += (int64_t)d.w * d.h;
      ro += 2 * rl.total;
    }
  }
  std::vector<float> st((size_t)kStateComps * nb);
  for (int64_t i = 0; i < nb; ++i) {
    for (int k = 0; k < 3; ++k) {
      st[(PX + k) * nb + i] = b.pos[3 * i + k];
      st[(VX + k) * nb + i] = b.vel[3 * i + k];
      st[(WX + k) * nb + i] = b.omega[3 * i + k];
    }
    for (int k = 0; k < 4; ++k) st[(QW + k) * nb + i] = b.quat[4 * i + k];
  }
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  HIPCHK(up(dev.envs + e0, envs.data(), sizeof(EnvDev) * envs.size()));
  HIPCHK(up(dev.cams + c0, cams.data(), sizeof(CamDev) * cams.size()));
  HIPCHK(up((void*)(dev.type + b0), b.type, nb));
  HIPCHK(up((void*)(dev.albedo + b0), b.albedo, nb));
  HIPCHK(up((void*)(dev.size + b0), b.size, 4 * nb));
  HIPCHK(up((void*)(dev.rbound + b0), b.rbound, 4 * nb));
  HIPCHK(up((void*)(dev.inv_m + b0), b.inv_m, 4 * nb));
  HIPCHK(up((void*)(dev.inv_I + b0), b.inv_I, 4 * nb));
  // per body: half-extents and principal moments; (a, a, a) and unused
  // moments for a sphere or a cube of size a
  std::vector<float> box6((size_t)(6 * nb), 0.0f);
  for (int64_t i = 0; i < nb; ++i)
    for (int k = 0; k < 3; ++k) {
      box6[(size_t)(6 * i + k)] = b.type[i] == 2 ? b.ext[3 * i + k] : b.size[i];
      box6[(size_t)(6 * i + 3 + k)] = b.type[i] == 2 ? b.inertia[3 * i + k] : 0.0f;
    }
  HIPCHK(up((void*)(dev.box + 6 * b0), box6.data(), 4 * box6.size()));
  HIPCHK(up((void*)(dev.prim_base + b0), pbase.data(), 4 * nb));
  HIPCHK(up((void*)(dev.vert_base + b0), vbase.data(), 4 * nb));
  HIPCHK(up((void*)(dev.prim_body + m0), pmap.data(), pmap.size()));
  HIPCHK(up((void*)(dev.vert_body + v0), vmap.data(), vmap.size()));
  for (int k = 0; k < kStateComps; ++k)
    HIPCHK(up(dev.state[parity] + k * dev.cap_bodies + b0, st.data() + k * nb, 4 * nb));
  // flags of the new envs start clear
  std::vector<uint32_t> zero(b.n_envs, 0u);
  HIPCHK(up(dev.env_flags + e0, zero.data(), 4 * zero.size()));
  // host mirrors
  for (int e = 0; e < b.n_envs; ++e) {
    env_host[e0 + e] = envs[e];
    env_parity[e0 + e] = (uint8_t)parity;
    env_active[e0 + e] = 1;
  }
  for (int32_t c = 0; c < nc; ++c) cam_host[c0 + c] = cams[c];
  HIPCHK(hipStreamSynchronize(s));  // host vectors die at return
  invalidate_lists();
  return VUDA_OK;
}

static int noalloc_init(int device);

extern "C" int vuda_create_world(const vuda_world_desc* d, const vuda_allocator* a, vuda_world** out) {
  if (!d || !out) return fail(VUDA_EINVAL, "null descriptor or output");
  *out = nullptr;
  if (!(d->phys.dt > 0.0f) || d->phys.substeps < 1 || d->phys.substeps > 64 ||
      !(d->phys.k_contact >= 0.0f) || !(d->phys.c_damp >= 0.0f))
    return fail(VUDA_EINVAL, "physics parameters");
  if (!(d->phys.mu >= 0.0f) || !std::isfinite(d->phys.mu) ||
      (d->phys.mu > 0.0f && (!(d->phys.v_eps > 0.0f) || !std::isfinite(d->phys.v_eps))))
    return fail(VUDA_EINVAL, "friction parameters mu %g, v_eps %g", d->phys.mu, d->phys.v_eps);
  if (d->phys.edge_contacts != 0 && d->phys.edge_contacts != 1)
    return fail(VUDA_EINVAL, "edge_contacts %d", (int)d->phys.edge_contacts);
  int rc = validate_render(d->render);
  if (rc) return rc;
  int64_t nb = 0, npix = 0;
  int32_t nc = 0;
  rc = validate_batch(d->initial, d->render, &nb, &nc, &npix);
  if (rc) return rc;
  if ((d->flags & VUDA_FLAG_SMOOTH) && (d->flags & VUDA_FLAG_NEAR_CLIP))
    return fail(VUDA_EINVAL, "VUDA_FLAG_SMOOTH does not combine with VUDA_FLAG_NEAR_CLIP");
  if (d->flags & VUDA_FLAG_TEXTURE) {
    if (!(d->flags & VUDA_FLAG_SMOOTH)) return fail(VUDA_EINVAL, "VUDA_FLAG_TEXTURE needs VUDA_FLAG_SMOOTH");
    const vuda_render_desc& r = d->render;
    if (!r.texture || r.texture_w < 1 || r.texture_w > 4096 || r.texture_h < 1 || r.texture_h > 4096)
      return fail(VUDA_EINVAL, "texture %p of %d x %d texels", (const void*)r.texture, (int)r.texture_w,
                  (int)r.texture_h);
    if (!std::isfinite(r.ground_uv_scale)) return fail(VUDA_EINVAL, "ground_uv_scale %g", r.ground_uv_scale);
  }
  vuda_world* w = new (std::nothrow) vuda_world();
  if (!w) return fail(VUDA_ENOMEM, "host allocation");
  HIPCHK(hipGetDevice(&w->device));
  w->phys = d->phys;
  w->debug = (d->flags & VUDA_FLAG_DEBUG) != 0;
  w->near_clip = (d->flags & VUDA_FLAG_NEAR_CLIP) != 0;
  w->smooth = (d->flags & VUDA_FLAG_SMOOTH) != 0;
  w->textured = (d->flags & VUDA_FLAG_TEXTURE) != 0;
  w->pair_cap = d->pair_cap > 0 ? d->pair_cap : 1024;
  w->cap_envs = std::max(d->cap_envs, d->initial.n_envs);
  w->cap_bodies = std::max(d->cap_bodies, nb);
  w->cap_cams = std::max(d->cap_cams, nc);
  w->cap_pixels = std::max(d->cap_pixels, npix);
  w->hbm_budget = d->hbm_budget;
  fill_templates(w->tpl, d->render);
  if (w->textured) {
    w->tpl.tex_w = d->render.texture_w;
    w->tpl.tex_h = d->render.texture_h;
  }
  int64_t init_prims = 0, init_verts = 0;
  w->map_sizes(d->initial, &init_prims, &init_verts);
  {
    // room for the maps of envs admitted later: every body at its largest template
    const int64_t mf = std::max(w->tpl.sphere_nf, w->tpl.cube_nf);
    const int64_t mv = std::max(w->tpl.sphere_nv, w->tpl.cube_nv);
    const int64_t spare_b = w->cap_bodies - nb, spare_e = (int64_t)w->cap_envs - d->initial.n_envs;
    w->cap_prims = init_prims + spare_b * mf + spare_e * (w->tpl.ground_nf + 15);
    w->cap_verts = init_verts + spare_b * mv + spare_e * (w->tpl.ground_nv + 15);
    // raster scratch of cameras admitted later.  Per camera and state buffer
    // (rs_layout) it is at most per_prim (n_tris + kClipRecs) + 8 tiles + 64
    // bytes + 255 of alignment per region, and a camera of W x H pixels
    // (W, H <= 4096) has at most W H / 64 + 1025 tiles of the smallest edge;
    // envs are assumed to carry no more cameras each than the initial
    // batch's most (at least 1).
    int32_t kcam = 1;
    for (int32_t e = 0; e < d->initial.n_envs; ++e)
      kcam = std::max(kcam, d->initial.cam_off[e + 1] - d->initial.cam_off[e]);
    const int64_t per_prim = kRecBytes + 2 * kBinsPerTri + (w->smooth ? 4 * kAttrWords : 0) +
                             (w->textured ? 4 * kTuvWords : 0);
    const int64_t spare_c = (int64_t)w->cap_cams - nc, spare_p = w->cap_pixels - npix;
    const int64_t spare_bytes = 2 * (per_prim * kcam * (w->cap_prims - init_prims) + spare_p / 8 +
                                     (64 + 5 * 255 + 8 * 1025 + per_prim * kClipRecs) * spare_c);
    w->cap_rs = w->rs_units(d->initial) + (spare_bytes + 255) / 256;
  }
  w->pc.h = d->phys.dt / (float)d->phys.substeps;
  w->pc.hh = 0.5f * w->pc.h;
  w->pc.k = d->phys.k_contact;
  w->pc.c = d->phys.c_damp;
  for (int k = 0; k < 3; ++k) w->pc.g[k] = d->phys.gravity[k];
  w->pc.substeps = d->phys.substeps;
  w->pc.mu = d->phys.mu;
  w->pc.v_eps = d->phys.mu > 0.0f ? d->phys.v_eps : 1.0f;
  w->pc.edge = d->phys.edge_contacts;
  rc = w->alloc_arena(a);
  if (rc) {
    w->free_all();
    delete w;
    return rc;
  }
  w->env_host.assign(w->cap_envs, EnvDev{});
  w->env_parity.assign(w->cap_envs, 0);
  w->env_active.assign(w->cap_envs, 0);
  w->env_retired.assign(w->cap_envs, 0);
  w->cam_host.assign(w->cap_cams, CamDev{});
  w->step_ev.assign(w->cap_envs, -1);
  w->setup_ok.assign(w->cap_envs, 0);
  w->render_ev[0].assign(w->cap_envs, -1);
  w->render_ev[1].assign(w->cap_envs, -1);
  w->render_state_ev[0].assign(w->cap_envs, -1);
  w->render_state_ev[1].assign(w->cap_envs, -1);
  w->slots.init(w->cap_envs);
  w->bodies.init(w->cap_bodies);
  w->camslots.init(w->cap_cams);
  w->pixels.init(w->cap_pixels);
  w->primspace.init(w->cap_prims);
  w->vertspace.init(w->cap_verts);
  w->rsspace.init(w->cap_rs);
  rc = w->make_streams(0.0f);
  // set-up with the device current: the workspace address of the
  // allocation-free policy launch, and the event pool (created here, so
  // that enqueueing never creates one)
  if (rc == VUDA_OK) rc = noalloc_init(w->device);
  if (rc == VUDA_OK) rc = w->init_events();
  if (rc == VUDA_OK) {
    hipError_t e = hipMemcpy((void*)w->dev.tpl, &w->tpl, sizeof(Templates), hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = hip_fail(e, "template upload");
  }
  if (rc == VUDA_OK && w->textured) {
    hipError_t e = hipMemcpy((void*)w->dev.texture, d->render.texture,
                             3 * (size_t)w->tpl.tex_w * (size_t)w->tpl.tex_h, hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = hip_fail(e, "texture upload");
  }
  if (rc == VUDA_OK && d->initial.n_envs > 0) {
    w->slots.take(0, d->initial.n_envs);
    w->bodies.take(0, nb);
    w->camslots.take(0, nc);
    w->pixels.take(0, npix);
    w->primspace.take(0, init_prims);
    w->vertspace.take(0, init_verts);
    w->rsspace.take(0, w->rs_units(d->initial));
    rc = w->upload(d->initial, 0, 0, 0, 0, 0, 0, 0, 0, w->s_serial);
    w->n_envs_hi = d->initial.n_envs;
  }
  if (rc) {
    w->free_all();
    delete w;
    return rc;
  }
  *out = w;
  return VUDA_OK;
}

void vuda_world::free_all() {
  if (device >= 0) (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  for (auto& kv : lists) {
    for (ListBuf& b : kv.second.buf) {
      if (b.dptr) (void)hipFree(b.dptr);
      if (b.tptr) (void)hipFree(b.tptr);
      for (hipEvent_t e : b.fence)
        if (e) (void)hipEventDestroy(e);
    }
  }
  lists.clear();
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
  graphs.clear();
  if (metric_cams) (void)hipFree(metric_cams);
  if (metric_buf) (void)hipFree(metric_buf);
  metric_cams = nullptr;
  metric_buf = nullptr;
  metric_cams_cap = metric_buf_cap = 0;
  destroy_streams();
  if (s_serial) (void)hipStreamDestroy(s_serial);
  s_serial = nullptr;
  for (auto& e : evpool) (void)hipEventDestroy(e);
  evpool.clear();
  for (auto& v : tev) {
    for (auto& e : v) (void)hipEventDestroy(e);
    v.clear();
  }
  free_policy();
  if (arena) {
    if (has_allocator) allocator.free(arena, allocator.ctx);
    else (void)hipFree(arena);
  }
  arena = nullptr;
}

extern "C" int vuda_destroy_world(vuda_world* w) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  w->free_all();
  delete w;
  return VUDA_OK;
}

extern "C" int vuda_world_info(vuda_world* w, int32_t* n_envs, int64_t* n_bodies, int32_t* n_cams,
                               int64_t* n_pixels, uint64_t* arena_bytes) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  if (n_envs) *n_envs = w->n_envs_hi;
  if (n_bodies) *n_bodies = w->cap_bodies;
  if (n_cams) *n_cams = w->cap_cams;
  if (n_pixels) *n_pixels = w->cap_pixels;
  if (arena_bytes) *arena_bytes = w->arena_bytes;
  return VUDA_OK;
}

// ---------------------------------------------------------------------------
// streams, CU masks, events
// ---------------------------------------------------------------------------

void vuda_world::destroy_streams() {
  if (s_sim && s_sim != s_serial) (void)hipStreamDestroy(s_sim);
  if (s_render && s_render != s_serial) (void)hipStreamDestroy(s_render);
  if (s_setup && s_setup != s_serial) (void)hipStreamDestroy(s_setup);
  s_sim = s_render = s_setup = nullptr;
}

// Bit i of a HIP CU mask selects a CU of XCD (i mod n_xcd), then of shader
// engine round-robin within it, so a contiguous run of bits spreads evenly
// over the XCDs and engines; the step phase takes bits [0, k), the render
// phase [k, n_cu).
static void cu_masks(int n_cu, float split, std::vector<uint32_t>& sim, std::vector<uint32_t>& ren) {
  const int words = (n_cu + 31) / 32;
  sim.assign(words, 0u);
  ren.assign(words, 0u);
  int k = (int)(split * (float)n_cu + 0.5f);
  k = std::max(1, std::min(n_cu - 1, k));
  for (int i = 0; i < n_cu; ++i) {
    if (i < k) sim[i / 32] |= 1u << (i % 32);
    else ren[i / 32] |= 1u << (i % 32);
  }
}

int vuda_world::make_streams(float split) {
  HIPCHK(hipSetDevice(device));
  if (!s_serial) HIPCHK(hipStreamCreateWithFlags(&s_serial, hipStreamNonBlocking));
  destroy_streams();
  mode = 0;
  cu_split = 0.0f;
  if (split > 0.0f && split < 1.0f) {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    std::vector<uint32_t> ms, mr;
    cu_masks(prop.multiProcessorCount, split, ms, mr);
    HIPCHK(hipExtStreamCreateWithCUMask(&s_sim, (uint32_t)ms.size(), ms.data()));
    HIPCHK(hipExtStreamCreateWithCUMask(&s_render, (uint32_t)mr.size(), mr.data()));
    HIPCHK(hipExtStreamCreateWithCUMask(&s_setup, (uint32_t)ms.size(), ms.data()));
    mode = 1;
    cu_split = split;
  } else if (split == 2.0f) {
    // Unmasked, but created with a mask of every CU all the same: a masked
    // stream gets a hardware queue of its own, while plain streams share the
    // runtime's small pool of queues (four by default) with every other
    // stream of the process, and two streams on one queue run one after the
    // other.  Measured at 1,024 envs: the pipelined schedule of a fresh world
    // 8.9 M env-steps/s on pooled queues (its third stream landed on a busy
    // one), 11.1-11.3 M on queues of its own.
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    std::vector<uint32_t> all((prop.multiProcessorCount + 31) / 32, 0u);
    for (int i = 0; i < prop.multiProcessorCount; ++i) all[i / 32] |= 1u << (i % 32);
    HIPCHK(hipExtStreamCreateWithCUMask(&s_sim, (uint32_t)all.size(), all.data()));
    HIPCHK(hipExtStreamCreateWithCUMask(&s_render, (uint32_t)all.size(), all.data()));
    HIPCHK(hipExtStreamCreateWithCUMask(&s_setup, (uint32_t)all.size(), all.data()));
    mode = 2;
    cu_split = split;
  } else {
    s_sim = s_serial;
    s_render = s_serial;
    s_setup = s_serial;
  }
  return VUDA_OK;
}

hipError_t vuda_world::copy_now(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  if (mode == 0 || !s_serial) return hipMemcpy(dst, src, bytes, kind);
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, s_serial);
  return e == hipSuccess ? hipStreamSynchronize(s_serial) : e;
}

hipError_t vuda_world::fill_now(void* dst, int value, size_t bytes) {
  if (mode == 0 || !s_serial) return hipMemset(dst, value, bytes);
  hipError_t e = hipMemsetAsync(dst, value, bytes, s_serial);
  return e == hipSuccess ? hipStreamSynchronize(s_serial) : e;
}

int vuda_world::drain() {
  HIPCHK(hipSetDevice(device));
  if (s_sim) HIPCHK(hipStreamSynchronize(s_sim));
  if (s_render) HIPCHK(hipStreamSynchronize(s_render));
  if (s_setup) HIPCHK(hipStreamSynchronize(s_setup));
  if (s_serial) HIPCHK(hipStreamSynchronize(s_serial));
  return VUDA_OK;
}

int vuda_world::mark(hipEvent_t ev[2]) {
  hipStream_t ss[2] = {s_sim ? s_sim : s_serial, s_render};
  const int n = (mode != 0 && s_render && s_render != ss[0]) ? 2 : 1;
  for (int k = 0; k < n; ++k) {
    if (!ev[k] && hipEventCreateWithFlags(&ev[k], hipEventDisableTiming) != hipSuccess) {
      hip_fail(hipGetLastError(), "hipEventCreateWithFlags");
      return -1;
    }
    if (hipEventRecord(ev[k], ss[k]) != hipSuccess) {
      hip_fail(hipGetLastError(), "hipEventRecord");
      return -1;
    }
  }
  return n;
}

int vuda_world::retire(int32_t first, int32_t n) {
  if (first < 0 || n <= 0 || first + n > cap_envs) return fail(VUDA_EINVAL, "range");
  for (int32_t e = first; e < first + n; ++e)
    if (!env_active[e]) return fail(VUDA_EINVAL, "env %d is not admitted", e);
  for (int32_t e = first; e < first + n; ++e) {
    env_active[e] = 0;
    env_retired[e] = 1;
    setup_ok[e] = 0;
  }
  invalidate_lists();
  return VUDA_OK;
}

extern "C" int vuda_cosched(vuda_world* w, float cu_split) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  if (!(cu_split <= 0.0f || (cu_split > 0.0f && cu_split < 1.0f) || cu_split == 1.0f || cu_split == 2.0f))
    return fail(VUDA_EINVAL, "cu_split %g: use (0,1), 2, or <=0 / 1", (double)cu_split);
  int rc = w->drain();
  if (rc) return rc;
  for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.second);
  w->graphs.clear();
  rc = w->make_streams(cu_split == 1.0f ? 0.0f : cu_split);
  // every earlier event has completed (drained): forget them
  std::fill(w->step_ev.begin(), w->step_ev.end(), -1);
  for (int q = 0; q < 2; ++q) {
    std::fill(w->render_ev[q].begin(), w->render_ev[q].end(), -1);
    std::fill(w->render_state_ev[q].begin(), w->render_state_ev[q].end(), -1);
  }
  return rc;
}

// Event pool: ids grow monotonically; slot id % size is reused after making
// sure the event it held has completed.
int vuda_world::init_events() {
  const size_t kPool = 512;
  if (evpool.empty()) {
    evpool.resize(kPool, nullptr);
    for (auto& e : evpool) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  return VUDA_OK;
}

// An id of the pool and its event, for the caller to record (run_kernel can
// bind it to the end of a launch instead of a separate record).
int vuda_world::reserve_event(int64_t* id, hipEvent_t* ev) {
  const size_t kPool = 512;
  int rc = init_events();
  if (rc) return rc;
  const int64_t nid = next_event++;
  hipEvent_t e = evpool[nid % kPool];
  if (nid >= (int64_t)kPool) HIPCHK(hipEventSynchronize(e));
  *id = nid;
  *ev = e;
  return VUDA_OK;
}

int vuda_world::new_event(hipStream_t s, int64_t* id) {
  hipEvent_t e;
  int rc = reserve_event(id, &e);
  if (rc) return rc;
  HIPCHK(hipEventRecord(e, s));
  return VUDA_OK;
}

int vuda_world::wait_event(hipStream_t s, int64_t id) {
  const int64_t kPool = (int64_t)evpool.size();
  if (id < 0 || id < next_event - kPool) return VUDA_OK;  // none, or recycled: already complete
  HIPCHK(hipStreamWaitEvent(s, evpool[id % kPool], 0));
  return VUDA_OK;
}

// ---------------------------------------------------------------------------
// work lists (LPT order) cached per range
// ---------------------------------------------------------------------------

// Mark every cached work list for a rebuild (after admission or release,
// which drain the world first, so no kernel still reads a list).
void vuda_world::invalidate_lists() {
  for (auto& kv : lists) kv.second.dirty = true;
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
  graphs.clear();
}

int vuda_world::get_list(int phase, int32_t lo, int32_t hi, const WorkList** out) {
  const auto key = std::make_tuple(phase, lo, hi);
  WorkList& L = lists[key];
  *out = &L;
  if (!L.dirty) return VUDA_OK;
  if (L.built) {
    // every launch reading the current version is enqueued: fence it and
    // build into the other version
    ListBuf& old = L.buf[L.cur];
    const int nf = mark(old.fence);
    if (nf < 0) return VUDA_EHIP;
    old.nfence = nf;
    L.cur ^= 1;
  }
  ListBuf& B = L.buf[L.cur];
  for (int k = 0; k < B.nfence; ++k) HIPCHK(hipEventSynchronize(B.fence[k]));
  B.nfence = 0;
  L.n = 0;
  L.max_bodies = L.max_verts = L.max_tris = L.max_tiles = 0;
  std::vector<std::pair<int64_t, int32_t>> items;
  for (int32_t e = lo; e < hi; ++e) {
    if (!env_active[e]) continue;
    const EnvDev& d = env_host[e];
    if (phase == VUDA_PHASE_STEP) {
      if (d.n_bodies == 0) continue;
      items.push_back({(int64_t)d.n_bodies * d.n_bodies + 8 * d.n_bodies, e});
      L.max_bodies = std::max(L.max_bodies, d.n_bodies);
    } else {
      for (int32_t c = d.cam_off; c < d.cam_off + d.n_cams; ++c) {
        const CamDev& cd = cam_host[c];
        const int tiles = tiles_of(cd.w, cd.h, tune.tile_shift);
        items.push_back({(int64_t)cd.w * cd.h + 64LL * d.n_tris, c});
        L.max_bodies = std::max(L.max_bodies, d.n_bodies);
        L.max_verts = std::max(L.max_verts, d.n_verts);
        L.max_tris = std::max(L.max_tris, d.n_tris);
        L.max_tiles = std::max(L.max_tiles, tiles);
      }
    }
  }
  // longest processing time first; ties by id for a deterministic order
  std::stable_sort(items.begin(), items.end(), [](const auto& a, const auto& b) {
    return a.first > b.first || (a.first == b.first && a.second < b.second);
  });
  std::vector<int32_t> ids(items.size());
  for (size_t i = 0; i < items.size(); ++i) ids[i] = items[i].second;
  if ((int32_t)ids.size() > B.cap) {
    if (B.dptr) HIPCHK(hipFree(B.dptr));
    B.dptr = nullptr;
    B.cap = 0;
    const int32_t want = std::max<int32_t>((int32_t)ids.size(), 64);
    HIPCHK(hipMalloc(&B.dptr, 4 * (size_t)want));
    B.cap = want;
  }
  if (!ids.empty()) HIPCHK(copy_now(B.dptr, ids.data(), 4 * ids.size(), hipMemcpyHostToDevice));
  L.dptr = B.dptr;
  L.n = (int32_t)ids.size();
  L.n_groups = 0;
  if (phase == VUDA_PHASE_RENDER && !ids.empty()) {
    // Tile-kernel jobs of tile_waves tiles of a row.  Workgroups are handed to the 8 XCDs
    // round-robin, so the setup workgroup of image i runs on XCD i mod 8;
    // its tiles get job indices of the same residue, where that XCD's L2
    // still holds the image's records and bins.
    constexpr int kXcd = 8;
    std::vector<std::vector<int2>> per(kXcd);
    for (size_t i = 0; i < ids.size(); ++i) {
      const CamDev& cd = cam_host[ids[i]];
      const int ts = 1 << tune.tile_shift;
      const int32_t ntx = (cd.w + ts - 1) >> tune.tile_shift, nty = (cd.h + ts - 1) >> tune.tile_shift;
      if (ids[i] > kJobCamMask) return fail(VUDA_EINVAL, "camera id %d beyond the tile job's range", ids[i]);
      for (int32_t ty = 0; ty < nty; ++ty)
        for (int32_t tx = 0; tx < ntx; tx += tune.tile_waves) {
          const int32_t n = std::min(tune.tile_waves, ntx - tx);
          per[i % kXcd].push_back(make_int2(ids[i] | ((n - 1) << kJobWavesShift), tx | (ty << 16)));
        }
    }
    size_t len = 0;
    for (auto& v : per) len = std::max(len, v.size());
    std::vector<int2> jobs(kXcd * len, make_int2(-1, 0));
    for (int x = 0; x < kXcd; ++x)
      for (size_t q = 0; q < per[x].size(); ++q) jobs[kXcd * q + x] = per[x][q];
    if ((int64_t)jobs.size() > B.tcap) {
      if (B.tptr) HIPCHK(hipFree(B.tptr));
      B.tptr = nullptr;
      B.tcap = 0;
      const int32_t want = std::max<int32_t>((int32_t)jobs.size(), 64);
      HIPCHK(hipMalloc(&B.tptr, sizeof(int2) * (size_t)want));
      B.tcap = want;
    }
    HIPCHK(copy_now(B.tptr, jobs.data(), sizeof(int2) * jobs.size(), hipMemcpyHostToDevice));
    L.n_groups = (int32_t)jobs.size();
  }
  L.tptr = B.tptr;
  L.built = true;
  L.dirty = false;
  return VUDA_OK;
}

// ---------------------------------------------------------------------------
// step / render / wait
// ---------------------------------------------------------------------------

int vuda_world::range_parity(int32_t lo, int32_t hi, int* parity) {
  int p = -1;
  for (int32_t e = lo; e < hi; ++e) {
    if (!env_active[e]) continue;
    if (p < 0) p = env_parity[e];
    else if (p != env_parity[e])
      return fail(VUDA_EINVAL, "envs %d..%d have different step parity", lo, hi - 1);
  }
  *parity = p < 0 ? 0 : p;
  return VUDA_OK;
}

int vuda_world::check_range(int32_t lo, int32_t hi) {
  if (lo < 0 || hi > cap_envs || lo > hi) return fail(VUDA_EINVAL, "env range [%d,%d) of %d", lo, hi, cap_envs);
  return VUDA_OK;
}

int vuda_world::enqueue_physics(const WorkList& L, int parity, hipStream_t s, LaunchEvents* ev) {
  PhysLaunch pl;
  pl.work = L.dptr;
  pl.n_work = L.n;
  pl.max_bodies = L.max_bodies;
  pl.parity = parity;
  pl.nsteps = 1;
  pl.persistent = tune.phys_persistent;
  pl.queue = queues;
  pl.prio = tune.phys_prio;
  pl.broadphase = tune.broadphase;
  pl.pack = tune.phys_pack;
  HIPCHK(launch_physics(dev, pc, pl, s, ev));
  return VUDA_OK;
}

int vuda_world::raster_launch_of(const WorkList& L, int parity, int32_t* queue, RasterLaunch* out) {
  RasterLaunch rl;
  rl.work = L.dptr;
  rl.n_work = L.n;
  rl.tiles = L.tptr;
  rl.n_tile_groups = L.n_groups;
  rl.max_verts = std::max(L.max_verts, 1);
  rl.max_tiles = std::max(L.max_tiles, 1);
  rl.max_bodies = L.max_bodies;
  rl.max_tris = std::max(L.max_tris, 1);
  rl.parity = parity;
  rl.threads = tune.raster_threads;
  rl.bin_limit = tune.rec_cap;
  rl.persistent = tune.raster_persistent;
  rl.queue = queue;
  rl.prio = 0;
  rl.near_clip = near_clip ? 1 : 0;
  rl.smooth = smooth ? 1 : 0;
  rl.tile_shift = tune.tile_shift;
  rl.tile_waves = tune.tile_waves;
  rl.lds_zone0 = rl.lrec_cap = rl.lbin_cap = 0;
  const size_t lds = raster_lds_bytes(rl);
  const size_t kLdsMax = 160 * 1024;
  if (lds > kLdsMax)
    return fail(VUDA_EOVERFLOW, "raster setup needs %zu bytes of LDS (max %zu)", lds, kLdsMax);
  if (lds > lds_configured) {
    HIPCHK(raster_configure(lds));
    lds_configured = lds;
  }
  *out = rl;
  return VUDA_OK;
}

int vuda_world::fused_launch_of(const WorkList& L, int parity, int32_t* queue, RasterLaunch* out, size_t* lds) {
  *lds = 0;
  // vertex-cache indices and primitives travel in 16 bits of a compact record
  if (!tune.raster_fused || near_clip || smooth || L.max_verts > 65536 || L.max_tris > 65536) return VUDA_OK;
  RasterLaunch rl;
  int rc = raster_launch_of(L, parity, queue, &rl);
  if (rc) return rc;
  const size_t need = raster_fused_plan(&rl, dev.winners != nullptr, tune.fused_recs);
  if (need == 0) return VUDA_OK;
  if (need > lds_fused_configured) {
    HIPCHK(raster_fused_configure(need));
    lds_fused_configured = need;
  }
  *out = rl;
  *lds = need;
  return VUDA_OK;
}

int vuda_world::enqueue_kernel(int kind, const WorkList& L, int parity, hipStream_t s, int32_t* queue,
                               LaunchEvents* ev) {
  if (kind == kKernelPhysics) return enqueue_physics(L, parity, s, ev);
  if (kind == kKernelFused) {
    RasterLaunch rl;
    size_t lds;
    int rc = fused_launch_of(L, parity, queue, &rl, &lds);
    if (rc) return rc;
    if (lds == 0) return fail(VUDA_EINVAL, "fused raster launch does not apply");
    HIPCHK(launch_raster_fused(dev, rl, lds, s, ev));
    return VUDA_OK;
  }
  if (kind == kKernelPolicy) {
    PolicyLaunch pl;
    int rc = policy_launch_of(L, &pl);
    if (rc) return rc;
    HIPCHK(launch_policy(dev, pl, s, ev));
    return VUDA_OK;
  }
  RasterLaunch rl;
  int rc = raster_launch_of(L, parity, queue, &rl);
  if (rc) return rc;
  // the setup that ends a step (its own queue slot) runs at the step's priority
  if (kind == kKernelSetup) rl.prio = queue == queues + 1 ? tune.phys_prio : 0;
  if (kind == kKernelTiles) rl.prio = tune.tile_prio;
  if (kind == kKernelSetup) HIPCHK(launch_raster_setup(dev, rl, s, ev));
  else HIPCHK(launch_raster_tiles(dev, rl, s, ev));
  return VUDA_OK;
}

// Launch one kernel over a work list, through a captured graph when graph mode
// is on, between timing events when timing is on.
// done (optional): an event recorded when the launch has ended.  A direct
// launch without timing binds it to its last kernel (the extended launch's
// end event: no separate marker on the stream); otherwise it is recorded
// after the launch.
int vuda_world::run_kernel(int kind, const WorkList& L, int parity, int32_t lo, int32_t hi, hipStream_t s,
                           int32_t* queue, hipEvent_t done) {
  if (done && !tune.timing && !tune.graphs) {
    LaunchEvents le;
    le.stop = done;
    int rc = enqueue_kernel(kind, L, parity, s, queue, &le);
    if (rc) return rc;
    if (!le.stopped) HIPCHK(hipEventRecord(done, s));  // nothing was launched
    return VUDA_OK;
  }
  const int rc0 = launch_kernel(kind, L, parity, lo, hi, s, queue);
  if (rc0 || !done) return rc0;
  HIPCHK(hipEventRecord(done, s));
  return VUDA_OK;
}

int vuda_world::launch_kernel(int kind, const WorkList& L, int parity, int32_t lo, int32_t hi, hipStream_t s,
                              int32_t* queue) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (tune.timing) {
    std::vector<hipEvent_t>& ev = tev[kind];
    const size_t i = 2 * tev_used[kind];
    while (ev.size() < i + 2) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      ev.push_back(e);
    }
    e0 = ev[i];
    e1 = ev[i + 1];
    // a replayed graph is timed from events around it; a direct launch from
    // events bound to its kernels (their own span, without the launch gap)
    if (tune.graphs) HIPCHK(hipEventRecord(e0, s));
  }
  int rc = VUDA_OK;
  if (!tune.graphs) {
    LaunchEvents le;
    le.start = e0;
    le.stop = e1;
    rc = enqueue_kernel(kind, L, parity, s, queue, e0 ? &le : nullptr);
    if (rc) return rc;
    if (e0 && !le.started) HIPCHK(hipEventRecord(e0, s));  // nothing was launched
    if (e1 && le.stopped) {
      ++tev_used[kind];
      return VUDA_OK;
    }
  } else {
    // the queue slot is part of the launch: it tells the two setup launch sites apart
    const int slot = queue ? (int)(queue - queues) : 0;
    const auto key = std::make_tuple(4 * kind + slot, lo, hi, parity);
    auto it = graphs.find(key);
    if (it == graphs.end()) {
      // A stream of its own for the capture, released right after: a
      // stream kept alive holds one of the process's few hardware queues,
      // which the world's own streams then share (and serialize on).
      hipStream_t cs = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
      }
      rc = enqueue_kernel(kind, L, parity, cs, queue);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cs, &g);
      (void)hipStreamDestroy(cs);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
      hipGraphExec_t ge = nullptr;
      e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
      it = graphs.emplace(key, ge).first;
    }
    HIPCHK(hipGraphLaunch(it->second, s));
  }
  if (rc) return rc;
  if (e1) {
    HIPCHK(hipEventRecord(e1, s));
    ++tev_used[kind];
  }
  return VUDA_OK;
}

extern "C" int vuda_step(vuda_world* w, int32_t lo, int32_t hi, int32_t nsteps) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  int rc = w->check_range(lo, hi);
  if (rc) return rc;
  if (nsteps < 0) return fail(VUDA_EINVAL, "nsteps < 0");
  if (nsteps == 0 || lo == hi) return VUDA_OK;
  int parity;
  rc = w->range_parity(lo, hi, &parity);
  if (rc) return rc;
  const WorkList* L;
  rc = w->get_list(VUDA_PHASE_STEP, lo, hi, &L);
  if (rc) return rc;
  // With presetup the raster setup of the new state (vertex transform,
  // triangle setup, binning -- it reads nothing but that state) follows the
  // last physics step on this stream, and the render phase keeps the pixels.
  const WorkList* LR = nullptr;
  if (w->tune.presetup) {
    rc = w->get_list(VUDA_PHASE_RENDER, lo, hi, &LR);
    if (rc) return rc;
    // a fused render sets up its images itself
    RasterLaunch rl;
    size_t lds;
    rc = w->fused_launch_of(*LR, 0, nullptr, &rl, &lds);
    if (rc) return rc;
    if (lds) LR = nullptr;
  }
  hipStream_t s = w->s_sim;
  for (int t = 0; t < nsteps; ++t) {
    const int p = (parity + t) & 1;
    if (w->mode != 0) {
      // WAR: the renders whose kernels read the state buffer this step
      // overwrites (their own setup, or the fused kernel).  A render whose
      // setup ran here with the step (presetup) has its tiles read only the
      // raster scratch, so the step does not wait for them; the setup below,
      // which rewrites that scratch, does.  Earlier steps are on this same
      // stream (RAW is implicit); events of one stream complete in order, so
      // the latest one covers the others.
      int64_t last = -1;
      const int64_t* rev = w->render_state_ev[p ^ 1].data();
      for (int32_t e = lo; e < hi; ++e) last = rev[e] > last ? rev[e] : last;
      rc = w->wait_event(s, last);
      if (rc) return rc;
    }
    // the step's event, bound to the end of its last kernel
    int64_t id = -1;
    hipEvent_t done = nullptr;
    if (w->mode != 0) {
      rc = w->reserve_event(&id, &done);
      if (rc) return rc;
    }
    const bool setup = LR && t == nsteps - 1;
    rc = w->run_kernel(kKernelPhysics, *L, p, lo, hi, s, w->queues, setup ? nullptr : done);
    if (rc) return rc;
    if (setup) {
      if (w->mode != 0) {
        // WAR: the renders of this buffer read its raster scratch
        int64_t last = -1;
        const int64_t* rev = w->render_ev[p ^ 1].data();
        for (int32_t e = lo; e < hi; ++e) last = rev[e] > last ? rev[e] : last;
        rc = w->wait_event(s, last);
        if (rc) return rc;
      }
      rc = w->run_kernel(kKernelSetup, *LR, p ^ 1, lo, hi, s, w->queues + 1, done);
      if (rc) return rc;
    }
    for (int32_t e = lo; e < hi; ++e) {
      if (!w->env_active[e]) continue;
      w->env_parity[e] ^= 1;
      w->step_ev[e] = id;
    }
  }
  for (int32_t e = lo; e < hi; ++e) w->setup_ok[e] = LR ? 1 : 0;
  return VUDA_OK;
}

extern "C" int vuda_render(vuda_world* w, int32_t lo, int32_t hi) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  int rc = w->check_range(lo, hi);
  if (rc) return rc;
  if (lo == hi) return VUDA_OK;
  int parity;
  rc = w->range_parity(lo, hi, &parity);
  if (rc) return rc;
  const WorkList* L;
  rc = w->get_list(VUDA_PHASE_RENDER, lo, hi, &L);
  if (rc) return rc;
  hipStream_t s = w->s_render;
  if (w->mode != 0) {
    // RAW: the latest step that wrote the state rendered (and its setup)
    int64_t last = -1;
    const int64_t* sev = w->step_ev.data();
    for (int32_t e = lo; e < hi; ++e) last = sev[e] > last ? sev[e] : last;
    rc = w->wait_event(s, last);
    if (rc) return rc;
  }
  RasterLaunch rl;
  size_t lds;
  rc = w->fused_launch_of(*L, parity, w->queues + 2, &rl, &lds);
  if (rc) return rc;
  // the event after the last kernel of this render that reads the state
  // buffer (the step that overwrites the buffer waits for it): the fused
  // kernel, or the raster setup
  int64_t state_id = -1;
  bool reads_state = false;
  if (lds) {
    reads_state = true;
  } else {
    bool need_setup = false;
    for (int32_t e = lo; e < hi; ++e) need_setup |= w->env_active[e] && !w->setup_ok[e];
    if (need_setup) {
      hipEvent_t sdone = nullptr;
      if (w->mode != 0) {
        rc = w->reserve_event(&state_id, &sdone);
        if (rc) return rc;
      }
      rc = w->run_kernel(kKernelSetup, *L, parity, lo, hi, s, w->queues + 2, sdone);
      if (rc) return rc;
      for (int32_t e = lo; e < hi; ++e) w->setup_ok[e] = 1;
    }
  }
  // the render's event, bound to the end of its last kernel
  int64_t id = -1;
  hipEvent_t done = nullptr;
  if (w->mode != 0) {
    rc = w->reserve_event(&id, &done);
    if (rc) return rc;
  }
  if (lds) {
    rc = w->run_kernel(kKernelFused, *L, parity, lo, hi, s, w->queues + 2, done);
    if (rc) return rc;
  } else {
    rc = w->run_kernel(kKernelTiles, *L, parity, lo, hi, s, nullptr, done);
    if (rc) return rc;
  }
  if (w->mode != 0) {
    if (reads_state) state_id = id;
    for (int32_t e = lo; e < hi; ++e) {
      if (!w->env_active[e]) continue;
      w->render_ev[parity][e] = id;
      if (state_id >= 0) w->render_state_ev[parity][e] = state_id;
    }
  }
  return VUDA_OK;
}

int vuda_world::check_flags() {
  uint32_t any = 0;
  std::vector<uint32_t> fl(cap_envs);
  HIPCHK(copy_now(fl.data(), dev.env_flags, 4 * (size_t)cap_envs, hipMemcpyDeviceToHost));
  int first = -1;
  for (int32_t e = 0; e < cap_envs; ++e) {
    if (fl[e] && first < 0) first = e;
    any |= fl[e];
  }
  if (any & kFlagNonFinite) return fail(VUDA_ENUMERIC, "non-finite state (first env %d)", first);
  if (any & (kFlagContactOverflow | kFlagBinOverflow | kFlagClipOverflow))
    return fail(VUDA_EOVERFLOW, "capacity overflow, flags 0x%x (first env %d)", any, first);
  return VUDA_OK;
}

extern "C" int vuda_wait(vuda_world* w, int32_t phase) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  if (phase < 1 || phase > 3) return fail(VUDA_EINVAL, "phase %d", phase);
  HIPCHK(hipSetDevice(w->device));
  if (phase & VUDA_PHASE_STEP) HIPCHK(hipStreamSynchronize(w->s_sim));
  if (phase & VUDA_PHASE_RENDER) HIPCHK(hipStreamSynchronize(w->s_render));
  return w->check_flags();
}

extern "C" int vuda_get_stream(vuda_world* w, int32_t phase, void** s) {
  if (!w || !s) return fail(VUDA_EINVAL, "null argument");
  if (phase == VUDA_PHASE_STEP) *s = (void*)w->s_sim;
  else if (phase == VUDA_PHASE_RENDER) *s = (void*)w->s_render;
  else return fail(VUDA_EINVAL, "phase %d", phase);
  return VUDA_OK;
}

// ---------------------------------------------------------------------------
// policy
// ---------------------------------------------------------------------------

void vuda_world::free_policy() {
  if (pol.w1t) (void)hipFree(pol.w1t);
  if (pol.wf) (void)hipFree(pol.wf);
  if (pol.w3p) (void)hipFree(pol.w3p);
  if (pol.partial) (void)hipFree(pol.partial);
  if (actions) (void)hipFree(actions);
  if (act_on) (void)hipFree(act_on);
  pol = Policy{};
  actions = nullptr;
  act_on = nullptr;
  dev.actions = nullptr;
  dev.act_on = nullptr;
  dev.act_dim = 0;
}

// K split of a product over `tiles` output tiles: enough workgroups to fill
// the chip once (layer 1: two per CU, as many as its registers let stay
// resident), each chunk at least min_steps steps long (layer 1: 4 MFMA
// steps of 32; layers 2 and 3: 8 steps of 16); the count divides `steps`.
static int split_count(int64_t tiles, int32_t steps, int32_t min_steps) {
  int s = 1;
  while (tiles * s < 512 && steps % (2 * s) == 0 && steps / (2 * s) >= min_steps) s *= 2;
  return s;
}

// Launch shape of the policy over M envs: splits, whether layers 2 and 3 run
// as batched products, and the float32 workspace that takes
struct PolicyPlan {
  int32_t splits = 1, s2 = 1, s3 = 1, Ap = 0;
  bool layered = false;
  int64_t partial_floats = 0;  // partials (and h1, h2 when layered)
};

static int policy_plan(const Policy& pol, bool force_layered, int32_t M, PolicyPlan* out) {
  PolicyPlan p;
  const int32_t K = 4 * pol.in_w * pol.in_h, H = pol.H;
  p.splits = split_count((int64_t)((M + 63) / 64) * ((H + 255) / 256), K / 32, 4);
  p.layered = force_layered || H > kPolicyHeadMax;
  p.partial_floats = (int64_t)p.splits * M * H;
  if (p.layered) {
    if (H % 64 != 0) return fail(VUDA_EINVAL, "policy hidden %d: layers 2-3 as products need a multiple of 64", H);
    const int64_t mt = (M + 63) / 64;
    p.Ap = (pol.A + 63) / 64 * 64;
    p.s2 = split_count(mt * (H / 64), H / 16, 8);
    p.s3 = split_count(mt * (p.Ap / 64), H / 16, 8);
    const int64_t most = std::max({(int64_t)p.splits * H, (int64_t)p.s2 * H, (int64_t)p.s3 * p.Ap});
    p.partial_floats = most * M + 2 * (int64_t)M * H;
  }
  *out = p;
  return VUDA_OK;
}

// The policy launch over the M envs listed at `envs`, with `partial`
// (`cap` floats) as its workspace.
static int policy_launch(const Policy& pol, bool layered, const int32_t* envs, int32_t M, float* partial,
                         int64_t cap, PolicyLaunch* out) {
  PolicyPlan plan;
  int rc = policy_plan(pol, layered, M, &plan);
  if (rc) return rc;
  const int32_t K = 4 * pol.in_w * pol.in_h;
  PolicyLaunch pl;
  pl.envs = envs;
  pl.M = M;
  pl.K = K;
  pl.krgb = 3 * pol.in_w * pol.in_h;
  pl.H = pol.H;
  pl.A = pol.A;
  pl.splits = plan.splits;
  pl.kchunk = K / pl.splits;
  pl.w1t = pol.w1t;
  pl.b1 = pol.wf;
  pl.w2 = pl.b1 + pol.H;
  pl.b2 = pl.w2 + (int64_t)pol.H * pol.H;
  pl.w3 = pl.b2 + pol.H;
  pl.b3 = pl.w3 + (int64_t)pol.H * pol.A;
  pl.a_max = pol.a_max;
  if (plan.partial_floats > cap) return fail(VUDA_EINVAL, "policy partials unsized");
  pl.partial = partial;
  pl.layered = plan.layered ? 1 : 0;
  pl.s2 = plan.s2;
  pl.s3 = plan.s3;
  pl.Ap = plan.Ap;
  pl.w3p = pol.w3p;
  pl.h1 = pl.h2 = nullptr;
  if (plan.layered) {
    if (!pol.w3p) return fail(VUDA_EINVAL, "policy without padded W3");
    // h1 and h2 sit after the largest partial block
    pl.h1 = partial + (plan.partial_floats - 2 * (int64_t)M * pol.H);
    pl.h2 = pl.h1 + (int64_t)M * pol.H;
  }
  *out = pl;
  return VUDA_OK;
}

int vuda_world::policy_launch_of(const WorkList& L, PolicyLaunch* out) {
  return policy_launch(pol, tune.policy_layered, L.dptr, L.n, pol.partial, pol.partial_cap, out);
}

extern "C" int vuda_policy_set(vuda_world* w, const vuda_policy_desc* d) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  HIPCHK(hipSetDevice(w->device));
  int rc = w->drain();
  if (rc) return rc;
  // launches captured with the old action buffers are stale
  for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.second);
  w->graphs.clear();
  w->free_policy();
  if (!d) return VUDA_OK;
  const int64_t px = (int64_t)d->in_w * d->in_h;
  if (d->in_w < 1 || d->in_h < 1 || px % 32 != 0 || 4 * px > (int64_t)1 << 30)
    return fail(VUDA_EINVAL, "policy frame %dx%d (pixels a multiple of 32)", d->in_w, d->in_h);
  if (d->hidden < 1 || d->hidden > kPolicyHiddenMax || (d->hidden > kPolicyHeadMax && d->hidden % 64 != 0))
    return fail(VUDA_EINVAL, "policy hidden %d (1..%d, a multiple of 64 above %d)", d->hidden, kPolicyHiddenMax,
                kPolicyHeadMax);
  if (d->act_bodies < 1 || d->act_bodies > 1024) return fail(VUDA_EINVAL, "policy act_bodies %d", d->act_bodies);
  if (!(d->a_max >= 0.0f) || !std::isfinite(d->a_max)) return fail(VUDA_EINVAL, "policy a_max");
  if (!d->w1 || !d->b1 || !d->w2 || !d->b2 || !d->w3 || !d->b3) return fail(VUDA_EINVAL, "null policy weights");
  Policy p;
  p.in_w = d->in_w;
  p.in_h = d->in_h;
  p.H = d->hidden;
  p.A = 3 * d->act_bodies;
  p.a_max = d->a_max;
  const int64_t K = 4 * px, H = p.H, A = p.A;
  // W1 [K][H] -> [K / 32][H][32]: the 32 weights of a unit for one MFMA
  // step of k are contiguous, and one step's weights of all units form one
  // contiguous panel (in 64 x 64 blocks: both sides stay in cache at H = 4096)
  std::vector<uint16_t> w1t((size_t)(K * H));
  for (int64_t k0 = 0; k0 < K; k0 += 64)
    for (int64_t h0 = 0; h0 < H; h0 += 64)
      for (int64_t k = k0; k < std::min(K, k0 + 64); ++k)
        for (int64_t h = h0; h < std::min(H, h0 + 64); ++h)
          w1t[(size_t)(((k >> 5) * H + h) * 32 + (k & 31))] = d->w1[k * H + h];
  std::vector<float> wf;
  wf.insert(wf.end(), d->b1, d->b1 + H);
  wf.insert(wf.end(), d->w2, d->w2 + H * H);
  wf.insert(wf.end(), d->b2, d->b2 + H);
  wf.insert(wf.end(), d->w3, d->w3 + H * A);
  wf.insert(wf.end(), d->b3, d->b3 + A);
  for (float v : wf)
    if (!std::isfinite(v)) return fail(VUDA_EINVAL, "non-finite policy weight");
  // W3 with its columns padded to a multiple of 64, for layers 2-3 as
  // batched products (hidden a multiple of 64)
  std::vector<float> w3p;
  const int64_t Ap = (A + 63) / 64 * 64;
  if (H % 64 == 0) {
    w3p.assign((size_t)(H * Ap), 0.0f);
    for (int64_t i = 0; i < H; ++i)
      for (int64_t q = 0; q < A; ++q) w3p[(size_t)(i * Ap + q)] = d->w3[i * A + q];
  }
  hipError_t e = hipMalloc(&p.w1t, 2 * w1t.size());
  if (e == hipSuccess) e = hipMalloc(&p.wf, 4 * wf.size());
  if (e == hipSuccess && !w3p.empty()) e = hipMalloc(&p.w3p, 4 * w3p.size());
  if (e == hipSuccess) e = hipMalloc(&w->actions, 4 * (size_t)w->cap_envs * A);
  if (e == hipSuccess) e = hipMalloc(&w->act_on, (size_t)w->cap_envs);
  w->pol = p;  // freed by free_policy on any failure below
  if (e != hipSuccess) {
    w->free_policy();
    return fail(VUDA_ENOMEM, "policy buffers: %s", hipGetErrorString(e));
  }
  HIPCHK(hipMemcpy(w->pol.w1t, w1t.data(), 2 * w1t.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(w->pol.wf, wf.data(), 4 * wf.size(), hipMemcpyHostToDevice));
  if (!w3p.empty()) HIPCHK(hipMemcpy(w->pol.w3p, w3p.data(), 4 * w3p.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(w->actions, 0, 4 * (size_t)w->cap_envs * A));
  HIPCHK(hipMemset(w->act_on, 0, (size_t)w->cap_envs));
  w->pol.set = true;
  w->dev.actions = w->actions;
  w->dev.act_on = w->act_on;
  w->dev.act_dim = (int32_t)A;
  return VUDA_OK;
}

extern "C" int vuda_act(vuda_world* w, int32_t lo, int32_t hi) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  int rc = w->check_range(lo, hi);
  if (rc) return rc;
  if (!w->pol.set) return fail(VUDA_EINVAL, "no policy (vuda_policy_set)");
  if (lo == hi) return VUDA_OK;
  for (int32_t e = lo; e < hi; ++e) {
    if (!w->env_active[e]) continue;
    const EnvDev& d = w->env_host[e];
    if (d.n_cams < 1) return fail(VUDA_EINVAL, "env %d has no camera", e);
    const CamDev& c = w->cam_host[d.cam_off];
    if (c.w != w->pol.in_w || c.h != w->pol.in_h)
      return fail(VUDA_EINVAL, "env %d: camera 0 is %dx%d, the policy reads %dx%d", e, c.w, c.h, w->pol.in_w,
                  w->pol.in_h);
    if (c.pix_off % 8 != 0) return fail(VUDA_EINVAL, "env %d: frame offset %lld not a multiple of 8", e,
                                        (long long)c.pix_off);
  }
  const WorkList* L;
  rc = w->get_list(VUDA_PHASE_STEP, lo, hi, &L);
  if (rc) return rc;
  {
    // layer-1 partial sums: grown here, outside any graph capture; graphs
    // that hold the old buffer go with it
    PolicyPlan plan;
    rc = policy_plan(w->pol, w->tune.policy_layered, L->n, &plan);
    if (rc) return rc;
    const int64_t need = plan.partial_floats;
    if (need > w->pol.partial_cap) {
      rc = w->drain();
      if (rc) return rc;
      for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.second);
      w->graphs.clear();
      if (w->pol.partial) HIPCHK(hipFree(w->pol.partial));
      w->pol.partial = nullptr;
      w->pol.partial_cap = 0;
      HIPCHK(hipMalloc(&w->pol.partial, 4 * (size_t)need));
      w->pol.partial_cap = need;
    }
  }
  hipStream_t s = w->s_sim;
  if (w->mode != 0) {
    // RAW: the renders that wrote the frames read here (of each env's
    // current state buffer)
    int64_t last = -1;
    for (int32_t e = lo; e < hi; ++e)
      if (w->env_active[e]) last = std::max(last, w->render_ev[w->env_parity[e]][e]);
    rc = w->wait_event(s, last);
    if (rc) return rc;
  }
  rc = w->run_kernel(kKernelPolicy, *L, 0, lo, hi, s, nullptr);
  if (rc) return rc;
  if (w->mode != 0) {
    // a later render of these envs overwrites the frames read here: it
    // waits for this event as for a step's
    int64_t id;
    rc = w->new_event(s, &id);
    if (rc) return rc;
    for (int32_t e = lo; e < hi; ++e)
      if (w->env_active[e]) w->step_ev[e] = id;
  }
  return VUDA_OK;
}

// ---------------------------------------------------------------------------
// the policy without allocation: a static device workspace
// ---------------------------------------------------------------------------

// Workspace of vuda_act_noalloc, one copy per GPU, held while the library is
// loaded: the env ids of the launch (up to 16,384), then the layer-1 partial
// sums (and h1, h2 of the layered head), 64 MiB.
constexpr size_t kNoAllocIdBytes = (size_t)64 << 10;
constexpr size_t kNoAllocPartialBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocIdBytes + kNoAllocPartialBytes];

// Device address of `scratch` on each GPU (the array's name is a host-side
// stand-in), taken once per device by noalloc_init.
constexpr int kMaxDevices = 64;
static unsigned char* g_scratch[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// With `device` current: record the device address of its copy of scratch.
static int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(VUDA_EINVAL, "device %d", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return VUDA_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  g_scratch[device] = (unsigned char*)p;
  return VUDA_OK;
}

__global__ void fill_env_ids_kernel(int32_t* ids, int32_t lo, int32_t n) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) ids[i] = lo + i;
}

extern "C" int vuda_act_noalloc(vuda_world* w, int32_t lo, int32_t hi) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  int rc = w->check_range(lo, hi);
  if (rc) return rc;
  if (!w->pol.set) return fail(VUDA_EINVAL, "no policy (vuda_policy_set)");
  if (lo == hi) return VUDA_OK;
  for (int32_t e = lo; e < hi; ++e) {
    if (!w->env_active[e]) return fail(VUDA_EINVAL, "env %d is not active (every env of the range must be)", e);
    const EnvDev& d = w->env_host[e];
    if (d.n_cams < 1) return fail(VUDA_EINVAL, "env %d has no camera", e);
    const CamDev& c = w->cam_host[d.cam_off];
    if (c.w != w->pol.in_w || c.h != w->pol.in_h)
      return fail(VUDA_EINVAL, "env %d: camera 0 is %dx%d, the policy reads %dx%d", e, c.w, c.h, w->pol.in_w,
                  w->pol.in_h);
    if (c.pix_off % 8 != 0) return fail(VUDA_EINVAL, "env %d: frame offset %lld not a multiple of 8", e,
                                        (long long)c.pix_off);
  }
  const int32_t M = hi - lo;
  PolicyPlan plan;
  rc = policy_plan(w->pol, w->tune.policy_layered, M, &plan);
  if (rc) return rc;
  if ((size_t)M * 4 > kNoAllocIdBytes || (size_t)plan.partial_floats * 4 > kNoAllocPartialBytes)
    return fail(VUDA_EINVAL,
                "%d envs at hidden %d need %lld bytes of workspace; vuda_act_noalloc holds %zu (and %zu env ids)",
                M, w->pol.H, (long long)plan.partial_floats * 4, kNoAllocPartialBytes, kNoAllocIdBytes / 4);
  unsigned char* base = (w->device >= 0 && w->device < kMaxDevices) ? g_scratch[w->device] : nullptr;
  if (!base) return fail(VUDA_EINVAL, "no workspace address for device %d", w->device);
  int32_t* ids = (int32_t*)base;
  float* partial = (float*)(base + kNoAllocIdBytes);
  PolicyLaunch pl;
  rc = policy_launch(w->pol, w->tune.policy_layered, ids, M, partial, (int64_t)(kNoAllocPartialBytes / 4), &pl);
  if (rc) return rc;
  hipStream_t s = w->s_sim;
  if (w->mode != 0) {
    // RAW: the renders that wrote the frames read here
    int64_t last = -1;
    for (int32_t e = lo; e < hi; ++e) last = std::max(last, w->render_ev[w->env_parity[e]][e]);
    rc = w->wait_event(s, last);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(fill_env_ids_kernel, dim3((M + 255) / 256), dim3(256), 0, s, ids, lo, M);
  HIPCHK(hipGetLastError());
  HIPCHK(launch_policy(w->dev, pl, s, nullptr));
  if (w->mode != 0) {
    int64_t id;
    rc = w->new_event(s, &id);
    if (rc) return rc;
    for (int32_t e = lo; e < hi; ++e) w->step_ev[e] = id;
  }
  return VUDA_OK;
}

// ---------------------------------------------------------------------------
// fetch / load
// ---------------------------------------------------------------------------

static int env_runs(vuda_world* w, int32_t lo, int32_t hi, int what, std::vector<std::pair<int64_t, int64_t>>& runs,
                    int64_t* total) {
  // contiguous element runs [start, count) of the selected data over envs lo..hi
  runs.clear();
  *total = 0;
  for (int32_t e = lo; e < hi; ++e) {
    if (!w->env_active[e]) continue;
    const EnvDev& d = w->env_host[e];
    int64_t s = 0, n = 0;
    if (what == VUDA_FETCH_STATE) {
      s = d.body_off;
      n = d.n_bodies;
    } else if (what == VUDA_FETCH_CONTACTS || what == VUDA_FETCH_FLAGS || what == VUDA_FETCH_ACTIONS) {
      s = e;
      n = 1;
    } else {
      if (d.n_cams == 0) continue;
      const CamDev& c0 = w->cam_host[d.cam_off];
      const CamDev& c1 = w->cam_host[d.cam_off + d.n_cams - 1];
      s = c0.pix_off;
      n = c1.pix_off + (int64_t)c1.w * c1.h - s;
    }
    if (n == 0) continue;
    if (!runs.empty() && runs.back().first + runs.back().second == s) runs.back().second += n;
    else runs.push_back({s, n});
    *total += n;
  }
  return VUDA_OK;
}

static size_t elem_bytes(vuda_world* w, int what) {
  switch (what) {
    case VUDA_FETCH_STATE: return 4 * kStateComps;
    case VUDA_FETCH_RGB: return 3;
    case VUDA_FETCH_DEPTH: return 4;
    case VUDA_FETCH_WINNERS: return 4;
    case VUDA_FETCH_COVERAGE: return 4;
    case VUDA_FETCH_CONTACTS: return 4 * (size_t)w->phys.substeps * (1 + 2 * (size_t)w->pair_cap);
    case VUDA_FETCH_FLAGS: return 4;
    case VUDA_FETCH_ACTIONS: return w->pol.set ? 4 * (size_t)w->pol.A : 0;
    case VUDA_FETCH_DEPTH_METRIC: return 4;
    default: return 0;
  }
}

extern "C" int vuda_fetch_bytes(vuda_world* w, int32_t what, int32_t lo, int32_t hi, size_t* bytes) {
  if (!w || !bytes) return fail(VUDA_EINVAL, "null argument");
  int rc = w->check_range(lo, hi);
  if (rc) return rc;
  if (elem_bytes(w, what) == 0) return fail(VUDA_EINVAL, "fetch selector %d", what);
  std::vector<std::pair<int64_t, int64_t>> runs;
  int64_t total;
  env_runs(w, lo, hi, what, runs, &total);
  *bytes = (size_t)total * elem_bytes(w, what);
  return VUDA_OK;
}

// Maximal runs of active envs in [lo, hi) whose bodies are contiguous and
// whose state sits in the same buffer: {parity, first body, body count}.
struct StateRun {
  int parity;
  int64_t b0, nb;
};
static void state_runs(const vuda_world* w, int32_t lo, int32_t hi, std::vector<StateRun>& runs) {
  runs.clear();
  for (int32_t e = lo; e < hi; ++e) {
    if (!w->env_active[e]) continue;
    const EnvDev& d = w->env_host[e];
    if (d.n_bodies == 0) continue;
    const int par = w->env_parity[e];
    if (!runs.empty() && runs.back().parity == par && runs.back().b0 + runs.back().nb == d.body_off)
      runs.back().nb += d.n_bodies;
    else
      runs.push_back({par, d.body_off, d.n_bodies});
  }
}

// Metric depth of the cameras of the active envs in [lo, hi), in fetch
// order, through the conversion kernel (into dst when it is device memory,
// else into a staging buffer copied out).  Each camera's view-projection
// must be a perspective of the usual form: row 2 = alpha row 3 + beta e_4.
static int fetch_depth_metric(vuda_world* w, int32_t lo, int32_t hi, float* dst, int64_t total, int32_t on_device) {
  std::vector<MetricCam> cams;
  int64_t pos = 0, max_pix = 0;
  for (int32_t e = lo; e < hi; ++e) {
    if (!w->env_active[e]) continue;
    const EnvDev& d = w->env_host[e];
    for (int32_t k = 0; k < d.n_cams; ++k) {
      const CamDev& c = w->cam_host[d.cam_off + k];
      const float* m = c.vp;
      double r2r3 = 0.0, r3r3 = 0.0, r2r2 = 0.0;
      for (int j = 0; j < 3; ++j) {
        r2r3 += (double)m[8 + j] * m[12 + j];
        r3r3 += (double)m[12 + j] * m[12 + j];
        r2r2 += (double)m[8 + j] * m[8 + j];
      }
      MetricCam mc;
      mc.alpha = r3r3 > 0.0 ? r2r3 / r3r3 : 0.0;
      mc.beta = (double)m[11] - mc.alpha * m[15];
      double off = 0.0;  // row 2 minus alpha row 3, first three columns
      for (int j = 0; j < 3; ++j) {
        const double t = (double)m[8 + j] - mc.alpha * m[12 + j];
        off += t * t;
      }
      if (!(r3r3 > 0.0) || off > 1e-12 * (r2r2 + 1.0) || !(mc.beta != 0.0))
        return fail(VUDA_EINVAL, "env %d camera %d: view-projection is not a perspective of the usual form", e, k);
      mc.pix_off = c.pix_off;
      mc.out_off = pos;
      mc.npix = (int64_t)c.w * c.h;
      pos += mc.npix;
      max_pix = std::max(max_pix, mc.npix);
      cams.push_back(mc);
    }
  }
  if (pos != total) return fail(VUDA_EINVAL, "metric depth: %lld pixels, expected %lld", (long long)pos,
                                (long long)total);
  if (cams.empty()) return VUDA_OK;
  HIPCHK(hipSetDevice(w->device));
  if ((int64_t)cams.size() > w->metric_cams_cap) {
    if (w->metric_cams) HIPCHK(hipFree(w->metric_cams));
    w->metric_cams = nullptr;
    w->metric_cams_cap = 0;
    HIPCHK(hipMalloc(&w->metric_cams, sizeof(MetricCam) * cams.size()));
    w->metric_cams_cap = (int64_t)cams.size();
  }
  float* out = dst;
  if (!on_device) {
    if (total > w->metric_buf_cap) {
      if (w->metric_buf) HIPCHK(hipFree(w->metric_buf));
      w->metric_buf = nullptr;
      w->metric_buf_cap = 0;
      HIPCHK(hipMalloc(&w->metric_buf, 4 * (size_t)total));
      w->metric_buf_cap = total;
    }
    out = w->metric_buf;
  }
  HIPCHK(hipMemcpy(w->metric_cams, cams.data(), sizeof(MetricCam) * cams.size(), hipMemcpyHostToDevice));
  HIPCHK(launch_depth_metric(w->dev.depth, w->metric_cams, (int32_t)cams.size(), max_pix, out, w->s_render));
  HIPCHK(hipStreamSynchronize(w->s_render));
  if (!on_device) HIPCHK(hipMemcpy(dst, out, 4 * (size_t)total, hipMemcpyDeviceToHost));
  return w->check_flags();
}

extern "C" int vuda_fetch(vuda_world* w, int32_t what, int32_t lo, int32_t hi, void* dst,
                          size_t dst_bytes, int32_t on_device) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  int rc = w->check_range(lo, hi);
  if (rc) return rc;
  const size_t eb = elem_bytes(w, what);
  if (eb == 0) return fail(VUDA_EINVAL, "fetch selector %d", what);
  if (!w->debug && (what == VUDA_FETCH_CONTACTS || what == VUDA_FETCH_WINNERS || what == VUDA_FETCH_COVERAGE))
    return fail(VUDA_EINVAL, "selector %d needs a world created with VUDA_FLAG_DEBUG", what);
  std::vector<std::pair<int64_t, int64_t>> runs;
  int64_t total;
  env_runs(w, lo, hi, what, runs, &total);
  if ((size_t)total * eb > dst_bytes)
    return fail(VUDA_EINVAL, "dst holds %zu bytes, need %zu", dst_bytes, (size_t)total * eb);
  if (total && !dst) return fail(VUDA_EINVAL, "null dst");
  rc = w->drain();
  if (rc) return rc;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  unsigned char* out = (unsigned char*)dst;
  if (what == VUDA_FETCH_STATE) {
    // gather [13][B] SoA into [n][13], from each env's current buffer
    std::vector<StateRun> sr;
    state_runs(w, lo, hi, sr);
    int64_t pos = 0;
    std::vector<float> tmp, aos;
    for (const StateRun& r : sr) {
      const float* src = w->dev.state[r.parity];
      tmp.resize((size_t)kStateComps * r.nb);
      for (int k = 0; k < kStateComps; ++k)
        HIPCHK(hipMemcpy(tmp.data() + (size_t)k * r.nb, src + k * w->dev.cap_bodies + r.b0, 4 * (size_t)r.nb,
                         hipMemcpyDeviceToHost));
      aos.resize((size_t)kStateComps * r.nb);
      for (int64_t i = 0; i < r.nb; ++i)
        for (int k = 0; k < kStateComps; ++k) aos[(size_t)i * kStateComps + k] = tmp[(size_t)k * r.nb + i];
      HIPCHK(hipMemcpy(out + pos * eb, aos.data(), aos.size() * 4,
                       on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
      pos += r.nb;
    }
    return w->check_flags();
  }
  if (what == VUDA_FETCH_DEPTH_METRIC) return fetch_depth_metric(w, lo, hi, (float*)dst, total, on_device);
  const unsigned char* base = nullptr;
  switch (what) {
    case VUDA_FETCH_RGB: base = w->dev.rgb; break;
    case VUDA_FETCH_DEPTH: base = (const unsigned char*)w->dev.depth; break;
    case VUDA_FETCH_WINNERS: base = (const unsigned char*)w->dev.winners; break;
    case VUDA_FETCH_COVERAGE: base = (const unsigned char*)w->dev.coverage; break;
    case VUDA_FETCH_CONTACTS: base = (const unsigned char*)w->dev.contacts; break;
    case VUDA_FETCH_FLAGS: base = (const unsigned char*)w->dev.env_flags; break;
    case VUDA_FETCH_ACTIONS: base = (const unsigned char*)w->actions; break;
  }
  int64_t pos = 0;
  for (auto& r : runs) {
    HIPCHK(hipMemcpy(out + pos * eb, base + r.first * eb, (size_t)r.second * eb, kind));
    pos += r.second;
  }
  if (what == VUDA_FETCH_FLAGS) return VUDA_OK;
  return w->check_flags();
}

extern "C" int vuda_load_state(vuda_world* w, int32_t lo, int32_t hi, const float* src, size_t src_bytes) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  int rc = w->check_range(lo, hi);
  if (rc) return rc;
  int64_t need = 0;
  for (int32_t e = lo; e < hi; ++e)
    if (w->env_active[e]) need += w->env_host[e].n_bodies;
  if ((size_t)need * 4 * kStateComps > src_bytes || (need && !src))
    return fail(VUDA_EINVAL, "src holds %zu bytes, need %zu", src_bytes, (size_t)need * 4 * kStateComps);
  rc = w->drain();
  if (rc) return rc;
  // one copy per state component for each run of contiguous envs
  std::vector<StateRun> sr;
  state_runs(w, lo, hi, sr);
  int64_t pos = 0;
  std::vector<float> soa;
  for (const StateRun& r : sr) {
    soa.resize((size_t)kStateComps * r.nb);
    for (int64_t i = 0; i < r.nb; ++i)
      for (int k = 0; k < kStateComps; ++k)
        soa[(size_t)k * r.nb + i] = src[(pos + i) * kStateComps + k];
    float* dstp = w->dev.state[r.parity];
    for (int k = 0; k < kStateComps; ++k)
      HIPCHK(hipMemcpy(dstp + k * w->dev.cap_bodies + r.b0, soa.data() + (size_t)k * r.nb, 4 * (size_t)r.nb,
                       hipMemcpyHostToDevice));
    pos += r.nb;
  }
  // the reloaded state has no raster setup yet
  for (int32_t e = lo; e < hi; ++e) w->setup_ok[e] = 0;
  // clear sticky flags of the reloaded envs
  std::vector<uint32_t> zero(hi - lo, 0u);
  if (hi > lo) HIPCHK(w->copy_now(w->dev.env_flags + lo, zero.data(), 4 * zero.size(), hipMemcpyHostToDevice));
  return VUDA_OK;
}

// ---------------------------------------------------------------------------
// admission (serving)
// ---------------------------------------------------------------------------

extern "C" int vuda_admit(vuda_world* w, const vuda_env_batch* b, int32_t parity, int32_t* first_env) {
  if (!w || !b || !first_env) return fail(VUDA_EINVAL, "null argument");
  if (parity != 0 && parity != 1) return fail(VUDA_EINVAL, "parity %d", parity);
  vuda_render_desc rd{};
  rd.ground_nf = w->tpl.ground_nf;
  rd.sphere_nf = w->tpl.sphere_nf;
  rd.cube_nf = w->tpl.cube_nf;
  int64_t nb, npix;
  int32_t nc;
  int rc = validate_batch(*b, rd, &nb, &nc, &npix);
  if (rc) return rc;
  if (b->n_envs == 0) return fail(VUDA_EINVAL, "empty request");
  // The new envs take free slots and free memory: launches already enqueued
  // read neither, and work lists are rebuilt into a fresh version.  Captured
  // graphs hold the old lists and are destroyed below, after they have run.
  if (!w->graphs.empty()) {
    rc = w->drain();
    if (rc) return rc;
  }
  const int64_t e0 = w->slots.alloc(b->n_envs);
  if (e0 < 0) return fail(VUDA_EBUSY, "no run of %d free env slots", b->n_envs);
  int64_t nprim, nvert;
  w->map_sizes(*b, &nprim, &nvert);
  const int64_t b0 = w->bodies.alloc(nb);
  const int64_t c0 = b0 < 0 ? -1 : w->camslots.alloc(nc);
  const int64_t p0 = c0 < 0 ? -1 : w->pixels.alloc(npix);
  const int64_t m0 = p0 < 0 ? -1 : w->primspace.alloc(nprim);
  const int64_t v0 = m0 < 0 ? -1 : w->vertspace.alloc(nvert);
  const int64_t nrs = w->rs_units(*b);
  const int64_t r0 = v0 < 0 ? -1 : w->rsspace.alloc(nrs);
  if (r0 < 0) {
    w->slots.release(e0, b->n_envs);
    if (b0 >= 0) w->bodies.release(b0, nb);
    if (c0 >= 0) w->camslots.release(c0, nc);
    if (p0 >= 0) w->pixels.release(p0, npix);
    if (m0 >= 0) w->primspace.release(m0, nprim);
    if (v0 >= 0) w->vertspace.release(v0, nvert);
    return fail(VUDA_EBUSY, "no room for %lld bodies / %d cameras / %lld pixels", (long long)nb, nc,
                (long long)npix);
  }
  rc = w->upload(*b, (int32_t)e0, b0, (int32_t)c0, p0, m0, v0, r0, parity, w->s_serial);
  if (rc) {
    w->slots.release(e0, b->n_envs);
    w->bodies.release(b0, nb);
    w->camslots.release(c0, nc);
    w->pixels.release(p0, npix);
    w->primspace.release(m0, nprim);
    w->vertspace.release(v0, nvert);
    w->rsspace.release(r0, nrs);
    return rc;
  }
  for (int e = 0; e < b->n_envs; ++e) {
    w->setup_ok[e0 + e] = 0;
    w->step_ev[e0 + e] = -1;
    w->render_ev[0][e0 + e] = -1;
    w->render_ev[1][e0 + e] = -1;
    w->render_state_ev[0][e0 + e] = -1;
    w->render_state_ev[1][e0 + e] = -1;
  }
  // a reused slot starts without the policy's forces of its last env
  if (w->act_on) HIPCHK(w->fill_now(w->act_on + e0, 0, (size_t)b->n_envs));
  w->n_envs_hi = std::max<int32_t>(w->n_envs_hi, (int32_t)(e0 + b->n_envs));
  *first_env = (int32_t)e0;
  return VUDA_OK;
}

extern "C" int vuda_release(vuda_world* w, int32_t first, int32_t n) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  if (first < 0 || n <= 0 || first + n > w->cap_envs) return fail(VUDA_EINVAL, "range");
  for (int32_t e = first; e < first + n; ++e)
    if (!w->env_active[e] && !w->env_retired[e]) return fail(VUDA_EINVAL, "env %d is not admitted", e);
  // Wait for the released envs' own work before their memory is reused:
  // their last step and last renders (events complete in stream order).
  // One stream (serialized), a policy or captured graphs: wait for all.
  int rc = VUDA_OK;
  if (w->mode == 0 || w->pol.set || !w->graphs.empty()) {
    rc = w->drain();
  } else {
    int64_t last[3] = {-1, -1, -1};
    for (int32_t e = first; e < first + n; ++e) {
      last[0] = std::max(last[0], w->step_ev[e]);
      last[1] = std::max(last[1], w->render_ev[0][e]);
      last[2] = std::max(last[2], w->render_ev[1][e]);
    }
    const int64_t kPool = (int64_t)w->evpool.size();
    for (int64_t id : last)
      if (id >= 0 && id >= w->next_event - kPool) HIPCHK(hipEventSynchronize(w->evpool[id % kPool]));
  }
  if (rc) return rc;
  // the request's bodies, cameras and pixels are contiguous
  const EnvDev& d0 = w->env_host[first];
  const EnvDev& d1 = w->env_host[first + n - 1];
  const int64_t nb = (int64_t)d1.body_off + d1.n_bodies - d0.body_off;
  const int32_t nc = d1.cam_off + d1.n_cams - d0.cam_off;
  int64_t p0 = 0, np = 0, r0 = 0, nr = 0;
  if (nc > 0) {
    const CamDev& c0 = w->cam_host[d0.cam_off];
    const CamDev& c1 = w->cam_host[d0.cam_off + nc - 1];
    p0 = c0.pix_off;
    np = c1.pix_off + (int64_t)c1.w * c1.h - p0;
    r0 = c0.rs_off / 256;
    nr = (c1.rs_off + 2 * rs_layout(c1.n_tris, tiles_of(c1.w, c1.h, kTileShiftMin), w->smooth, w->textured).total) /
             256 - r0;
  }
  std::vector<EnvDev> empty(n, EnvDev{});
  HIPCHK(w->copy_now(w->dev.envs + first, empty.data(), sizeof(EnvDev) * n, hipMemcpyHostToDevice));
  w->bodies.release(d0.body_off, nb);
  w->camslots.release(d0.cam_off, nc);
  w->pixels.release(p0, np);
  w->rsspace.release(r0, nr);
  // each env's maps were allocated rounded up to 16 bytes
  w->primspace.release(d0.prim_map, d1.prim_map + map_round(d1.n_tris) - d0.prim_map);
  w->vertspace.release(d0.vert_map, d1.vert_map + map_round(d1.n_verts) - d0.vert_map);
  w->slots.release(first, n);
  for (int32_t e = first; e < first + n; ++e) {
    w->setup_ok[e] = 0;
    w->env_active[e] = 0;
    w->env_retired[e] = 0;
    w->env_host[e] = EnvDev{};
  }
  w->invalidate_lists();
  return VUDA_OK;
}

// ---------------------------------------------------------------------------
// tuning knobs
// ---------------------------------------------------------------------------

extern "C" int vuda_set_tuning(vuda_world* w, int32_t key, int32_t value) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  switch (key) {
    case VUDA_TUNE_RASTER_THREADS:
      if (value < 64 || value > 1024 || value % 64) return fail(VUDA_EINVAL, "raster threads %d", value);
      w->tune.raster_threads = value;
      break;
    case VUDA_TUNE_REC_CAP:
      if (value < 0) return fail(VUDA_EINVAL, "bin limit %d", value);
      w->tune.rec_cap = value;
      break;
    case VUDA_TUNE_PHYS_PERSISTENT:
      if (value < VUDA_PERSISTENT_RESIDENT) return fail(VUDA_EINVAL, "persistent %d", value);
      w->tune.phys_persistent = value;
      break;
    case VUDA_TUNE_RASTER_PERSISTENT:
      if (value < VUDA_PERSISTENT_RESIDENT) return fail(VUDA_EINVAL, "persistent %d", value);
      w->tune.raster_persistent = value;
      break;
    case VUDA_TUNE_GRAPHS:
      w->tune.graphs = value != 0;
      break;
    case VUDA_TUNE_PHYS_PRIORITY:
      if (value < 0 || value > 3) return fail(VUDA_EINVAL, "priority %d", value);
      w->tune.phys_prio = value;
      break;
    case VUDA_TUNE_BROADPHASE:
      if (value < 0 || value > 2) return fail(VUDA_EINVAL, "broadphase %d", value);
      w->tune.broadphase = value;
      break;
    case VUDA_TUNE_TIMING:
      if (value < 0 || value > 1) return fail(VUDA_EINVAL, "timing %d", value);
      w->tune.timing = value != 0;
      return VUDA_OK;  // placement of the events only: graphs stay valid
    case VUDA_TUNE_PRESETUP:
      if (value < 0 || value > 1) return fail(VUDA_EINVAL, "presetup %d", value);
      w->tune.presetup = value != 0;
      return VUDA_OK;
    case VUDA_TUNE_POLICY_LAYERED:
      if (value < 0 || value > 1) return fail(VUDA_EINVAL, "policy layered %d", value);
      w->tune.policy_layered = value != 0;
      break;
    case VUDA_TUNE_PHYS_ENVS_PER_WAVE:
      if (value != 1 && value != 2) return fail(VUDA_EINVAL, "envs per wave %d (1 or 2)", value);
      w->tune.phys_pack = value;
      break;
    case VUDA_TUNE_RASTER_FUSED:
      if (value < 0 || value > 1) return fail(VUDA_EINVAL, "raster fused %d", value);
      // a step set up for the two-kernel path renders correctly either way;
      // one stepped in fused mode has no setup, so its render sets up
      w->tune.raster_fused = value != 0;
      break;
    case VUDA_TUNE_TILE_PRIORITY:
      if (value < 0 || value > 3) return fail(VUDA_EINVAL, "tile priority %d", value);
      w->tune.tile_prio = value;
      break;
    case VUDA_TUNE_TILE_WAVES:
      if (value != 1 && value != 2 && value != 4) return fail(VUDA_EINVAL, "tile waves %d (1, 2 or 4)", value);
      if (value != w->tune.tile_waves) {
        w->tune.tile_waves = value;
        w->invalidate_lists();  // the tile jobs group tile_waves tiles
      }
      break;
    case VUDA_TUNE_FUSED_LDS_RECORDS:
      if (value < 0) return fail(VUDA_EINVAL, "fused LDS records %d", value);
      w->tune.fused_recs = value;
      break;
    case VUDA_TUNE_TILE_SIZE: {
      if (value != 8 && value != 16 && value != 32) return fail(VUDA_EINVAL, "tile size %d (8, 16 or 32)", value);
      const int sh = value == 8 ? 3 : (value == 16 ? 4 : 5);
      if (sh != w->tune.tile_shift) {
        // tile jobs and the setups of the states already set up change
        int rc = w->drain();
        if (rc) return rc;
        w->tune.tile_shift = sh;
        std::fill(w->setup_ok.begin(), w->setup_ok.end(), 0);
        w->invalidate_lists();
      }
      return VUDA_OK;
    }
    default:
      return fail(VUDA_EINVAL, "tuning key %d", key);
  }
  for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.second);
  w->graphs.clear();
  return VUDA_OK;
}

extern "C" int vuda_get_tuning(vuda_world* w, int32_t key, int32_t* value) {
  if (!w || !value) return fail(VUDA_EINVAL, "null argument");
  switch (key) {
    case VUDA_TUNE_RASTER_THREADS: *value = w->tune.raster_threads; break;
    case VUDA_TUNE_REC_CAP: *value = w->tune.rec_cap; break;
    case VUDA_TUNE_PHYS_PERSISTENT: *value = w->tune.phys_persistent; break;
    case VUDA_TUNE_RASTER_PERSISTENT: *value = w->tune.raster_persistent; break;
    case VUDA_TUNE_GRAPHS: *value = w->tune.graphs ? 1 : 0; break;
    case VUDA_TUNE_PHYS_PRIORITY: *value = w->tune.phys_prio; break;
    case VUDA_TUNE_BROADPHASE: *value = w->tune.broadphase; break;
    case VUDA_TUNE_TIMING: *value = w->tune.timing ? 1 : 0; break;
    case VUDA_TUNE_PRESETUP: *value = w->tune.presetup ? 1 : 0; break;
    case VUDA_TUNE_POLICY_LAYERED: *value = w->tune.policy_layered ? 1 : 0; break;
    case VUDA_TUNE_PHYS_ENVS_PER_WAVE: *value = w->tune.phys_pack; break;
    case VUDA_TUNE_TILE_SIZE: *value = 1 << w->tune.tile_shift; break;
    case VUDA_TUNE_RASTER_FUSED: *value = w->tune.raster_fused ? 1 : 0; break;
    case VUDA_TUNE_FUSED_LDS_RECORDS: *value = w->tune.fused_recs; break;
    case VUDA_TUNE_TILE_WAVES: *value = w->tune.tile_waves; break;
    case VUDA_TUNE_TILE_PRIORITY: *value = w->tune.tile_prio; break;
    default: return fail(VUDA_EINVAL, "tuning key %d", key);
  }
  return VUDA_OK;
}

extern "C" int vuda_kernel_times(vuda_world* w, int32_t kernel, int64_t* launches, double* total_ms,
                                 double* max_ms) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  if (kernel < VUDA_KERNEL_PHYSICS || kernel > VUDA_KERNEL_RASTER_FUSED) return fail(VUDA_EINVAL, "kernel %d", kernel);
  const int k = kernel - VUDA_KERNEL_PHYSICS;
  const size_t n = w->tev_used[k];
  double sum = 0.0, mx = 0.0;
  if (n) {
    HIPCHK(hipSetDevice(w->device));
    HIPCHK(hipEventSynchronize(w->tev[k][2 * n - 1]));
    for (size_t i = 0; i < n; ++i) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, w->tev[k][2 * i], w->tev[k][2 * i + 1]));
      sum += ms;
      mx = ms > mx ? ms : mx;
    }
  }
  w->tev_used[k] = 0;
  if (launches) *launches = (int64_t)n;
  if (total_ms) *total_ms = sum;
  if (max_ms) *max_ms = mx;
  return VUDA_OK;
}

// ---------------------------------------------------------------------------
// schedules over every active env
// ---------------------------------------------------------------------------

// Slot index splitting the active envs into two halves of equal count.
int32_t vuda_world::active_midpoint() {
  int32_t total = 0;
  for (int32_t e = 0; e < n_envs_hi; ++e) total += env_active[e];
  int32_t seen = 0;
  for (int32_t e = 0; e < n_envs_hi; ++e) {
    if (seen * 2 >= total) return e;
    seen += env_active[e];
  }
  return n_envs_hi;
}

// Three-stage pipeline: iteration k rasterizes the tiles of S_k on the render
// stream, sets up S_k+1 on the setup stream and steps S_k+1 -> S_k+2 on the
// step stream, each waiting only for work of iteration k - 1: the setup of
// S_k+1 for the step that produced it and for the tiles of S_k-1 (which read
// the raster scratch of its parity), the tiles of S_k for its setup, the step
// for the setup of S_k (which reads the state buffer the step overwrites).
// After `iters` iterations the frames show S_iters-1 and the state is
// S_iters with its setup done, as after the inter-step schedule.  On one
// stream, or with the fused raster (a render that sets itself up), the
// inter-step order runs instead.
static int run_pipelined(vuda_world* w, int32_t iters) {
  const int32_t hi = w->n_envs_hi;
  int parity;
  int rc = w->range_parity(0, hi, &parity);
  if (rc) return rc;
  const WorkList *LS, *LR;
  rc = w->get_list(VUDA_PHASE_STEP, 0, hi, &LS);
  if (!rc) rc = w->get_list(VUDA_PHASE_RENDER, 0, hi, &LR);
  if (rc) return rc;
  RasterLaunch rl;
  size_t lds;
  rc = w->fused_launch_of(*LR, parity, nullptr, &rl, &lds);
  if (rc) return rc;
  if (w->mode == 0 || lds) {
    for (int32_t t = 0; t < iters; ++t) {
      rc = vuda_render(w, 0, hi);
      if (!rc) rc = vuda_step(w, 0, hi, 1);
      if (rc) return rc;
    }
    return VUDA_OK;
  }
  hipStream_t ss = w->s_sim, su = w->s_setup, sr = w->s_render;
  // every stage starts after all earlier work of these envs (the step
  // events are on the step stream, the render events on the render stream:
  // the latest of each covers the others)
  int64_t ls = -1, lr = -1;
  bool need_setup = false;
  for (int32_t e = 0; e < hi; ++e) {
    if (!w->env_active[e]) continue;
    ls = std::max(ls, w->step_ev[e]);
    lr = std::max({lr, w->render_ev[0][e], w->render_ev[1][e]});
    need_setup |= !w->setup_ok[e];
  }
  for (hipStream_t s : {ss, su, sr}) {
    if ((rc = w->wait_event(s, ls)) || (rc = w->wait_event(s, lr))) return rc;
  }
  // each stage's event is bound to the end of its kernel (run_kernel)
  const auto run_ev = [&](int kind, const WorkList& L, int p, hipStream_t s, int32_t* q, int64_t* id) {
    hipEvent_t done;
    int r = w->reserve_event(id, &done);
    return r ? r : w->run_kernel(kind, L, p, 0, hi, s, q, done);
  };
  int64_t ev_setup = -1, ev_phys = -1, ev_tiles_prev = -1;
  if (need_setup) {
    if ((rc = run_ev(kKernelSetup, *LR, parity, su, w->queues + 1, &ev_setup))) return rc;
  }
  if ((rc = run_ev(kKernelPhysics, *LS, parity, ss, w->queues, &ev_phys))) return rc;
  for (int32_t k = 0; k < iters; ++k) {
    const int pk = parity ^ (k & 1);  // state buffer and scratch parity of S_k
    // tiles of S_k
    if ((rc = w->wait_event(sr, ev_setup))) return rc;
    int64_t ev_tiles;
    if ((rc = run_ev(kKernelTiles, *LR, pk, sr, nullptr, &ev_tiles))) return rc;
    // setup of S_k+1
    if ((rc = w->wait_event(su, ev_phys)) || (rc = w->wait_event(su, ev_tiles_prev))) return rc;
    int64_t ev_setup_next;
    if ((rc = run_ev(kKernelSetup, *LR, pk ^ 1, su, w->queues + 1, &ev_setup_next))) return rc;
    // step S_k+1 -> S_k+2, into the buffer of S_k
    if (k + 2 <= iters) {
      if ((rc = w->wait_event(ss, ev_setup))) return rc;
      if ((rc = run_ev(kKernelPhysics, *LS, pk ^ 1, ss, w->queues, &ev_phys))) return rc;
    }
    ev_setup = ev_setup_next;
    ev_tiles_prev = ev_tiles;
  }
  // the step and render streams take over the last setup; their events then
  // cover everything enqueued here
  if ((rc = w->wait_event(ss, ev_setup)) || (rc = w->wait_event(sr, ev_setup))) return rc;
  int64_t sid, rid;
  if ((rc = w->new_event(ss, &sid)) || (rc = w->new_event(sr, &rid))) return rc;
  for (int32_t e = 0; e < hi; ++e) {
    if (!w->env_active[e]) continue;
    if (iters & 1) w->env_parity[e] ^= 1;
    w->step_ev[e] = sid;
    w->render_ev[0][e] = w->render_ev[1][e] = rid;
    w->render_state_ev[0][e] = w->render_state_ev[1][e] = rid;
    w->setup_ok[e] = 1;
  }
  return VUDA_OK;
}

extern "C" int vuda_run(vuda_world* w, int32_t schedule, int32_t iters) {
  if (!w) return fail(VUDA_EINVAL, "null world");
  if (iters < 0 || schedule < VUDA_SCHED_SERIAL || schedule > VUDA_SCHED_PIPELINED)
    return fail(VUDA_EINVAL, "schedule %d / iters %d", schedule, iters);
  if (schedule == VUDA_SCHED_PIPELINED) return iters ? run_pipelined(w, iters) : VUDA_OK;
  const int32_t hi = w->n_envs_hi;
  const int32_t mid = schedule == VUDA_SCHED_INTERTRAJ ? w->active_midpoint() : 0;
  for (int32_t t = 0; t < iters; ++t) {
    int rc = VUDA_OK;
    switch (schedule) {
      case VUDA_SCHED_SERIAL:
        rc = vuda_step(w, 0, hi, 1);
        if (!rc) rc = vuda_render(w, 0, hi);
        break;
      case VUDA_SCHED_INTERSTEP:  // render S_t while S_t -> S_t+1 runs beside it
        rc = vuda_render(w, 0, hi);
        if (!rc) rc = vuda_step(w, 0, hi, 1);
        break;
      case VUDA_SCHED_INTERTRAJ:  // step(A) | render(B), then step(B) | render(A)
        rc = vuda_step(w, 0, mid, 1);
        if (!rc) rc = vuda_render(w, mid, hi);
        if (!rc) rc = vuda_step(w, mid, hi, 1);
        if (!rc) rc = vuda_render(w, 0, mid);
        break;
    }
    if (rc) return rc;
  }
  return VUDA_OK;
}
