// Tiled software rasterizer for gfx950: one workgroup per camera image.
//
// Per image:
//   1. bodies: pose from the physics state buffer (read in place, no copy)
//      and R(q) into LDS;
//   2. vertices: every template vertex of every body (and the ground) is
//      transformed once -- world = p + R (s v), clip = VP world, perspective
//      divide, viewport, snap to 24.8 fixed point -- and cached in LDS;
//   3. triangles: culled if a vertex is behind the near plane or outside the
//      guard band, if back-facing or degenerate (integer area <= 0); the
//      survivors are binned into 16x16-pixel tiles with LDS atomics, a
//      prefix scan of the tile counts and a scatter of triangle ids;
//   4. tiles: each wave takes one tile at a time, four pixels per lane, and
//      walks the tile's bin.  Edge functions are evaluated exactly (integer
//      values held in fp64, which represents them without rounding); a pixel
//      is covered if every edge value is > 0, or == 0 on a top-left edge.
//      Depth is interpolated in fp32, quantised to 24 bits, and the minimum
//      of (depth << 32 | primitive) wins, which makes the result independent
//      of bin order;
//   5. Lambert shading of the winner and RGB8 + u32 depth stores.
// When a tile range's bins do not fit the LDS budget, tiles are processed
// in consecutive groups that do, re-binning per group.
#include "vuda_internal.h"

#pragma clang fp contract(off)

namespace vuda {
namespace {

constexpr int kMaxTileWindow = 1024;

struct RasterLayout {
  // byte offsets into dynamic LDS
  int body, verts, tiles, bins, misc, total;
  int nmax, vmax, tw, bin_cap;
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline RasterLayout make_layout(int max_bodies, int max_verts, int max_tiles,
                                                    int bin_cap) {
  RasterLayout L;
  L.nmax = max_bodies + 1;
  L.vmax = max_verts;
  L.tw = max_tiles < kMaxTileWindow ? max_tiles : kMaxTileWindow;
  L.bin_cap = bin_cap;
  int o = 0;
  L.body = o;   o += align16(4 * 18 * L.nmax);
  L.verts = o;  o += align16(12 * L.vmax);
  L.tiles = o;  o += align16(4 * (3 * L.tw + 1));
  L.bins = o;   o += align16(4 * L.bin_cap);
  L.misc = o;   o += 64;
  L.total = o;
  return L;
}

struct BodyLDS {
  float* p;       // [3][nmax]
  float* R;       // [9][nmax]
  float* s;       // [nmax]
  int32_t* type;  // [nmax]
  int32_t* vb;    // [nmax] vertex base (env-local), vb[n] = total verts
  int32_t* pb;    // [nmax] primitive base, pb[n] = total prims
  int32_t* alb;   // [nmax]
};

__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float* m) {
  const float xx = x * x, yy = y * y, zz = z * z;
  const float xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  m[0] = 1.0f - 2.0f * (yy + zz);
  m[1] = 2.0f * (xy - wz);
  m[2] = 2.0f * (xz + wy);
  m[3] = 2.0f * (xy + wz);
  m[4] = 1.0f - 2.0f * (xx + zz);
  m[5] = 2.0f * (yz - wx);
  m[6] = 2.0f * (xz - wy);
  m[7] = 2.0f * (yz + wx);
  m[8] = 1.0f - 2.0f * (xx + yy);
}

constexpr int32_t kInvalid = (int32_t)0x80000000;

// Snapped screen-space triangle in edge order (vertices 0, 2, 1 of the face).
struct Tri {
  int32_t X[3], Y[3];
  float z[3];
  bool ok;
};

__device__ __forceinline__ int body_of(const int32_t* base, int n, int idx) {
  // largest b in [0, n) with base[b] <= idx
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= idx) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// vertex indices (env-local) of primitive `prim`; body = -1 for the ground
__device__ __forceinline__ void prim_vertices(const Templates* tp, const BodyLDS& B, int n,
                                              int prim, int* body, int* face, int vid[3]) {
  if (prim < tp->ground_nf) {
    *body = -1;
    *face = prim;
#pragma unroll
    for (int k = 0; k < 3; ++k) vid[k] = tp->ground_f[prim][k];
    return;
  }
  const int b = body_of(B.pb, n, prim);
  const int f = prim - B.pb[b];
  *body = b;
  *face = f;
  const uint8_t* fi = B.type[b] ? tp->cube_f[f] : tp->sphere_f[f];
#pragma unroll
  for (int k = 0; k < 3; ++k) vid[k] = B.vb[b] + fi[k];
}

__device__ __forceinline__ Tri load_tri(const int32_t* VX, const int32_t* VY, const float* VZ,
                                        const int vid[3]) {
  Tri t;
  const int ord[3] = {0, 2, 1};
  t.ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int v = vid[ord[k]];
    t.X[k] = VX[v];
    t.Y[k] = VY[v];
    t.z[k] = VZ[v];
    if (t.X[k] == kInvalid) t.ok = false;
  }
  return t;
}

__device__ __forceinline__ int64_t tri_area(const Tri& t) {
  return (int64_t)(t.X[1] - t.X[0]) * (int64_t)(t.Y[2] - t.Y[0]) -
         (int64_t)(t.Y[1] - t.Y[0]) * (int64_t)(t.X[2] - t.X[0]);
}

// Pixel range whose centres 256p+128 lie inside the bounding box, clipped
// to the image; returns false if empty.
__device__ __forceinline__ bool tri_pixels(const Tri& t, int W, int H, int* x0, int* x1, int* y0,
                                           int* y1) {
  const int xmin = min(t.X[0], min(t.X[1], t.X[2])), xmax = max(t.X[0], max(t.X[1], t.X[2]));
  const int ymin = min(t.Y[0], min(t.Y[1], t.Y[2])), ymax = max(t.Y[0], max(t.Y[1], t.Y[2]));
  *x0 = max(0, (xmin + 127) >> 8);
  *x1 = min(W - 1, (xmax - 128) >> 8);
  *y0 = max(0, (ymin + 127) >> 8);
  *y1 = min(H - 1, (ymax - 128) >> 8);
  return *x0 <= *x1 && *y0 <= *y1;
}

__device__ __forceinline__ bool top_left(int32_t dx, int32_t dy) {
  return dy < 0 || (dy == 0 && dx > 0);
}

__device__ void raster_image(unsigned char* lds, const RasterLayout& Lo, const WorldDev& W,
                             const RasterLaunch& L, int cam_id) {
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const CamDev cam = W.cams[cam_id];
  const EnvDev ed = W.envs[cam.env];
  const int n = ed.n_bodies;
  const int Wd = cam.w, Ht = cam.h;
  const Templates* tp = W.tpl;
  const int64_t cap = W.cap_bodies;
  const float* st = W.state[L.parity];

  BodyLDS B;
  float* bf = (float*)(lds + Lo.body);
  B.p = bf;
  B.R = bf + 3 * Lo.nmax;
  B.s = bf + 12 * Lo.nmax;
  B.type = (int32_t*)(bf + 13 * Lo.nmax);
  B.vb = (int32_t*)(bf + 14 * Lo.nmax);
  B.pb = (int32_t*)(bf + 15 * Lo.nmax);
  B.alb = (int32_t*)(bf + 16 * Lo.nmax);
  int32_t* VX = (int32_t*)(lds + Lo.verts);
  int32_t* VY = VX + Lo.vmax;
  float* VZ = (float*)(VY + Lo.vmax);
  int32_t* tcount = (int32_t*)(lds + Lo.tiles);
  int32_t* toff = tcount + Lo.tw;  // tw + 1 entries
  int32_t* tfill = toff + Lo.tw + 1;
  uint32_t* bins = (uint32_t*)(lds + Lo.bins);
  int32_t* misc = (int32_t*)(lds + Lo.misc);

  // 1. bodies
  for (int b = tid; b < n; b += nthr) {
    const int g = ed.body_off + b;
    B.p[b] = st[PX * cap + g];
    B.p[Lo.nmax + b] = st[PY * cap + g];
    B.p[2 * Lo.nmax + b] = st[PZ * cap + g];
    float m[9];
    quat_rot(st[QW * cap + g], st[QX * cap + g], st[QY * cap + g], st[QZ * cap + g], m);
#pragma unroll
    for (int k = 0; k < 9; ++k) B.R[k * Lo.nmax + b] = m[k];
    B.s[b] = W.size[g];
    B.type[b] = W.type[g];
    B.vb[b] = W.vert_base[g];
    B.pb[b] = W.prim_base[g];
    B.alb[b] = W.albedo[g];
  }
  if (tid == 0) {
    B.vb[n] = ed.n_verts;
    B.pb[n] = ed.n_tris;
  }
  __syncthreads();

  // 2. vertices
  const float* vp = cam.vp;
  const float fW = (float)Wd, fH = (float)Ht;
  for (int vi = tid; vi < ed.n_verts; vi += nthr) {
    float wx, wy, wz;
    if (vi < tp->ground_nv) {
      wx = tp->ground_v[vi][0];
      wy = tp->ground_v[vi][1];
      wz = tp->ground_v[vi][2];
    } else {
      const int b = body_of(B.vb, n, vi);
      const int lv = vi - B.vb[b];
      const float* tv = B.type[b] ? tp->cube_v[lv] : tp->sphere_v[lv];
      const float s = B.s[b];
      const float sx = s * tv[0], sy = s * tv[1], sz = s * tv[2];
      const float* R = B.R + b;
      const int S = Lo.nmax;
      wx = B.p[b] + ((R[0] * sx + R[S] * sy) + R[2 * S] * sz);
      wy = B.p[S + b] + ((R[3 * S] * sx + R[4 * S] * sy) + R[5 * S] * sz);
      wz = B.p[2 * S + b] + ((R[6 * S] * sx + R[7 * S] * sy) + R[8 * S] * sz);
    }
    const float cx = ((vp[0] * wx + vp[1] * wy) + vp[2] * wz) + vp[3];
    const float cy = ((vp[4] * wx + vp[5] * wy) + vp[6] * wz) + vp[7];
    const float cz = ((vp[8] * wx + vp[9] * wy) + vp[10] * wz) + vp[11];
    const float cw = ((vp[12] * wx + vp[13] * wy) + vp[14] * wz) + vp[15];
    int32_t X = kInvalid, Y = kInvalid;
    float z = 0.0f;
    if (!(cw < tp->near_w)) {
      const float nx = cx / cw, ny = cy / cw, nz = cz / cw;
      const float px = (nx * 0.5f + 0.5f) * fW;
      const float py = (0.5f - ny * 0.5f) * fH;
      if (!(fabsf(px) > tp->guard || fabsf(py) > tp->guard)) {
        X = (int32_t)rintf(px * 256.0f);
        Y = (int32_t)rintf(py * 256.0f);
        z = nz;
      }
    }
    VX[vi] = X;
    VY[vi] = Y;
    VZ[vi] = z;
  }
  __syncthreads();

  const int ntx = (Wd + kTile - 1) / kTile, nty = (Ht + kTile - 1) / kTile;
  const int ntiles = ntx * nty;
  const int ntris = ed.n_tris;
  const int nwaves = nthr >> 6;
  const int wave = tid >> 6, lane = tid & 63;
  bool overflow = false;

  for (int w0 = 0; w0 < ntiles; w0 += Lo.tw) {
    const int w1 = min(ntiles, w0 + Lo.tw);
    for (int t = tid; t < w1 - w0; t += nthr) tcount[t] = 0;
    __syncthreads();
    // 3a. count
    for (int pr = tid; pr < ntris; pr += nthr) {
      int body, face, vid[3];
      prim_vertices(tp, B, n, pr, &body, &face, vid);
      const Tri t = load_tri(VX, VY, VZ, vid);
      if (!t.ok || tri_area(t) <= 0) continue;
      int x0, x1, y0, y1;
      if (!tri_pixels(t, Wd, Ht, &x0, &x1, &y0, &y1)) continue;
      for (int ty = y0 >> 4; ty <= (y1 >> 4); ++ty)
        for (int tx = x0 >> 4; tx <= (x1 >> 4); ++tx) {
          const int ti = ty * ntx + tx - w0;
          if (ti >= 0 && ti < w1 - w0) atomicAdd(&tcount[ti], 1);
        }
    }
    __syncthreads();
    if (tid == 0) {
      int acc = 0;
      for (int t = 0; t < w1 - w0; ++t) {
        toff[t] = acc;
        acc += tcount[t];
      }
      toff[w1 - w0] = acc;
    }
    __syncthreads();
    // 3b/4. groups of consecutive tiles whose bins fit
    int g0 = 0;
    while (g0 < w1 - w0) {
      if (tid == 0) {
        int g1 = g0 + 1;
        while (g1 < w1 - w0 && toff[g1 + 1] - toff[g0] <= Lo.bin_cap) ++g1;
        misc[0] = g1;
        misc[1] = toff[g1] - toff[g0] > Lo.bin_cap ? 1 : 0;
      }
      __syncthreads();
      const int g1 = misc[0];
      if (misc[1]) overflow = true;
      const int base = toff[g0];
      for (int t = g0 + tid; t < g1; t += nthr) tfill[t] = 0;
      __syncthreads();
      for (int pr = tid; pr < ntris; pr += nthr) {
        int body, face, vid[3];
        prim_vertices(tp, B, n, pr, &body, &face, vid);
        const Tri t = load_tri(VX, VY, VZ, vid);
        if (!t.ok || tri_area(t) <= 0) continue;
        int x0, x1, y0, y1;
        if (!tri_pixels(t, Wd, Ht, &x0, &x1, &y0, &y1)) continue;
        const uint32_t entry = (uint32_t)pr | ((uint32_t)(body + 1) << 16);
        for (int ty = y0 >> 4; ty <= (y1 >> 4); ++ty)
          for (int tx = x0 >> 4; tx <= (x1 >> 4); ++tx) {
            const int ti = ty * ntx + tx - w0;
            if (ti >= g0 && ti < g1) {
              const int slot = toff[ti] - base + atomicAdd(&tfill[ti], 1);
              if (slot < Lo.bin_cap) bins[slot] = entry;
            }
          }
      }
      __syncthreads();
      // 4. raster the group's tiles, one tile per wave at a time
      for (int ti = g0 + wave; ti < g1; ti += nwaves) {
        const int tile = w0 + ti;
        const int tx = tile % ntx, ty = tile / ntx;
        const int px = tx * kTile + (lane & 15);
        const int py0 = ty * kTile + (lane >> 4);
        const double Px = (double)(256 * px + 128);
        uint64_t key[4];
        int cover[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) { key[r] = ~0ull; cover[r] = 0; }
        const int k0 = toff[ti] - base, k1 = min(toff[ti + 1] - base, Lo.bin_cap);
        for (int k = k0; k < k1; ++k) {
          const uint32_t entry = __builtin_amdgcn_readfirstlane(bins[k]);
          const int pr = (int)(entry & 0xFFFFu);
          int body, face, vid[3];
          prim_vertices(tp, B, n, pr, &body, &face, vid);
          const Tri t = load_tri(VX, VY, VZ, vid);
          const int64_t A = tri_area(t);
          const float invA = 1.0f / (float)A;
          // edge k runs from vertex k+1 to vertex k+2; it weights vertex k
          double ea[3], eb[3], E[3];
          bool tl[3];
#pragma unroll
          for (int e = 0; e < 3; ++e) {
            const int a = (e + 1) % 3, b = (e + 2) % 3;
            const int32_t dx = t.X[b] - t.X[a], dy = t.Y[b] - t.Y[a];
            ea[e] = (double)dx;
            eb[e] = (double)dy;
            tl[e] = top_left(dx, dy);
            E[e] = ea[e] * (double)(256 * py0 + 128 - t.Y[a]) - eb[e] * (Px - (double)t.X[a]);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const bool in0 = E[0] > 0.0 || (E[0] == 0.0 && tl[0]);
            const bool in1 = E[1] > 0.0 || (E[1] == 0.0 && tl[1]);
            const bool in2 = E[2] > 0.0 || (E[2] == 0.0 && tl[2]);
            if (in0 && in1 && in2) {
              cover[r] += 1;
              const float zz = (((float)E[0] * t.z[0] + (float)E[1] * t.z[1]) + (float)E[2] * t.z[2]) * invA;
              const uint32_t D = (uint32_t)rintf(fminf(fmaxf(zz, 0.0f), 1.0f) * 16777215.0f);
              const uint64_t kk = ((uint64_t)D << 32) | entry;
              if (kk < key[r]) key[r] = kk;
            }
#pragma unroll
            for (int e = 0; e < 3; ++e) E[e] += ea[e] * 1024.0;  // next row of this lane: +4 px
          }
        }
        // 5. shade and store
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int py = py0 + 4 * r;
          if (px >= Wd || py >= Ht) continue;
          const int64_t pix = cam.pix_off + (int64_t)py * Wd + px;
          uint8_t rgb[3] = {0, 0, 0};
          uint32_t D = 0xFFFFFFFFu;
          int32_t win = -1;
          if (key[r] != ~0ull) {
            const uint32_t e = (uint32_t)(key[r] & 0xFFFFFFFFu);
            D = (uint32_t)(key[r] >> 32);
            win = (int32_t)(e & 0xFFFFu);
            const int body = (int)(e >> 16) - 1;
            float nx, ny, nz, al[3];
            if (body < 0) {
              nx = 0.0f; ny = 0.0f; nz = 1.0f;
              al[0] = al[1] = al[2] = tp->ground_albedo;
            } else {
              const int f = win - B.pb[body];
              const float* nf = B.type[body] ? tp->cube_n[f] : tp->sphere_n[f];
              const float* R = B.R + body;
              const int S = Lo.nmax;
              nx = (R[0] * nf[0] + R[S] * nf[1]) + R[2 * S] * nf[2];
              ny = (R[3 * S] * nf[0] + R[4 * S] * nf[1]) + R[5 * S] * nf[2];
              nz = (R[6 * S] * nf[0] + R[7 * S] * nf[1]) + R[8 * S] * nf[2];
              const int ai = B.alb[body];
              al[0] = tp->palette[ai][0];
              al[1] = tp->palette[ai][1];
              al[2] = tp->palette[ai][2];
            }
            const float l = fmaxf(0.0f, (nx * tp->light[0] + ny * tp->light[1]) + nz * tp->light[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const float col = al[c] * (0.2f + 0.8f * l);
              rgb[c] = (uint8_t)fminf(255.0f, rintf(col * 255.0f));
            }
          }
          W.rgb[3 * pix] = rgb[0];
          W.rgb[3 * pix + 1] = rgb[1];
          W.rgb[3 * pix + 2] = rgb[2];
          W.depth[pix] = D;
          if (W.winners) W.winners[pix] = win;
          if (W.coverage) W.coverage[pix] = cover[r];
        }
      }
      __syncthreads();
      g0 = g1;
    }
  }
  if (overflow && tid == 0) atomicOr(&W.env_flags[cam.env], kFlagBinOverflow);
}

__global__ void raster_kernel(WorldDev W, RasterLaunch L) {
  extern __shared__ __align__(16) unsigned char lds[];
  const RasterLayout Lo = make_layout(L.max_bodies, L.max_verts, L.max_tiles, L.bin_cap);
  if (L.persistent == 0) {
    if ((int)blockIdx.x >= L.n_work) return;
    raster_image(lds, Lo, W, L, L.work[blockIdx.x]);
    return;
  }
  int32_t* slot = (int32_t*)(lds + Lo.misc) + 4;
  for (;;) {
    if (threadIdx.x == 0) *slot = atomicAdd(L.queue, 1);
    __syncthreads();
    const int wi = *slot;
    __syncthreads();
    if (wi >= L.n_work) return;
    raster_image(lds, Lo, W, L, L.work[wi]);
    __syncthreads();
  }
}

}  // namespace

size_t raster_lds_bytes(const RasterLaunch& l) {
  return (size_t)make_layout(l.max_bodies, l.max_verts, l.max_tiles, l.bin_cap).total;
}

hipError_t raster_configure(size_t lds_bytes) {
  return hipFuncSetAttribute((const void*)raster_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t launch_raster(const WorldDev& w, const RasterLaunch& l, hipStream_t s) {
  if (l.n_work <= 0) return hipSuccess;
  const size_t lds = raster_lds_bytes(l);
  const int grid = l.persistent > 0 ? (l.persistent < l.n_work ? l.persistent : l.n_work) : l.n_work;
  if (l.persistent > 0) {
    hipError_t e = launch_reset_queue(l.queue, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(raster_kernel, dim3(grid), dim3(l.threads), lds, s, w, l);
  return hipGetLastError();
}

}  // namespace vuda
