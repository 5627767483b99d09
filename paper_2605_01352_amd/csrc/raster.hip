// Tiled software rasterizer for gfx950: one workgroup per camera image.
//
// Per image:
//   1. bodies: pose from the physics state buffer (read in place, no copy)
//      and R(q) into LDS; template vertex and face tables into LDS;
//   2. vertices: every template vertex of every body (and the ground) is
//      transformed once -- world = p + R (s v), clip = VP world, perspective
//      divide, viewport, snap to 24.8 fixed point -- and cached in LDS;
//   3. triangle setup: a triangle is culled if a vertex is behind the near
//      plane or outside the guard band, if it is back-facing or degenerate
//      (integer area <= 0), or if its bounding box holds no pixel centre;
//      survivors get a setup record in LDS (snapped vertices in edge order,
//      depths, 1/area, primitive key and its flat Lambert colour) and are
//      binned into 16x16-pixel tiles with LDS atomics, a workgroup prefix
//      scan of the tile counts and a scatter;
//   4. tiles: each wave takes one tile at a time and keeps the tile's
//      z-buffer of 64-bit keys (depth << 32 | primitive << 16 | record) in
//      LDS.  Small triangles (box within the tile <= 64 pixels) are packed as
//      fragments, one pixel per lane across several triangles; large ones run
//      one lane per four pixels.  Edge functions are exact (integer values
//      carried in fp64, which represents them without rounding); a pixel is
//      covered if every edge value is > 0, or == 0 on a top-left edge.  Depth
//      is interpolated in fp32 and quantised to 24 bits; the minimum key wins,
//      so the result does not depend on bin order or on which lane tests
//      which pixel;
//   5. the winner's colour from its record, RGB8 + u32 depth stores.
// Images whose records or bins do not fit the LDS budget take a slower path
// that re-derives each triangle from the vertex cache per tile and bins
// tiles in groups that fit; both paths produce identical bits.
#include <cstddef>

#include "vuda_internal.h"

#pragma clang fp contract(off)

namespace vuda {
namespace {

constexpr int kMaxTileWindow = 1024;
constexpr int kRecWords = 12;  // X0 Y0 X1 Y1 | X2 Y2 key z0 | z1 z2 invA rgb
// per wave: tile z-buffer (256 x u64), coverage counts (256 x i32), fragment owners (64 x i32)
constexpr int kWaveBytes = 256 * 8 + 256 * 4 + 64 * 4;

// The template vertex and face tables (the leading members of Templates)
// are copied into LDS per workgroup; normals and shading constants, used once
// per visible triangle, stay in global memory.
struct TplLDS {
  float sphere_v[kMaxTplVerts][3];
  float cube_v[kMaxTplVerts][3];
  float ground_v[kMaxGroundVerts][3];
  uint8_t sphere_f[kMaxTplFaces][3];
  uint8_t cube_f[kMaxTplFaces][3];
  uint8_t ground_f[kMaxGroundFaces][3];
};
constexpr int kTplBytes = ((int)sizeof(TplLDS) + 15) & ~15;
static_assert(offsetof(Templates, sphere_v) == offsetof(TplLDS, sphere_v) &&
              offsetof(Templates, ground_f) == offsetof(TplLDS, ground_f) &&
              kTplBytes <= (int)sizeof(Templates), "template tables lead Templates");

struct RasterLayout {
  // byte offsets into dynamic LDS
  int tpl, maps, body, verts, recs, tiles, waves, misc, total;
  int nmax, vmax, tw, rec_cap, bin_cap_fast, bin_cap_slow, nwaves;
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline RasterLayout make_layout(int max_bodies, int max_verts, int max_tiles,
                                                    int max_tris, int rec_cap, int threads) {
  RasterLayout L;
  L.nmax = max_bodies + 1;
  L.vmax = max_verts;
  L.tw = max_tiles < kMaxTileWindow ? max_tiles : kMaxTileWindow;
  L.rec_cap = rec_cap;
  L.nwaves = threads / 64;
  const int vb = align16(12 * L.vmax), bb = align16(8 * rec_cap);
  const int vbytes = vb > bb ? vb : bb;
  L.bin_cap_fast = vbytes / 2;                // u16 record ids in the vertex region
  L.bin_cap_slow = kRecWords * rec_cap;       // u32 entries in the record region
  int o = 0;
  L.tpl = o;    o += align16(kTplBytes);
  L.maps = o;   o += align16(max_tris) + align16(max_verts);  // prim and vertex -> body
  L.body = o;   o += align16(4 * 18 * L.nmax);
  L.verts = o;  o += vbytes;
  L.recs = o;   o += align16(4 * kRecWords * rec_cap);
  L.tiles = o;  o += align16(4 * (3 * L.tw + 1));
  L.waves = o;  o += L.nwaves * kWaveBytes;
  L.misc = o;   o += 128;  // scalars [0, 8), per-wave scan totals [8, 24)
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

// vertex indices (env-local) of primitive `prim`; body = -1 for the ground
__device__ __forceinline__ void prim_vertices(const TplLDS* T, const BodyLDS& B, const uint8_t* pmap,
                                              int prim, int* body, int vid[3]) {
  const int b = pmap[prim];
  if (b == kGroundBody) {
    *body = -1;
#pragma unroll
    for (int k = 0; k < 3; ++k) vid[k] = T->ground_f[prim][k];
    return;
  }
  const int f = prim - B.pb[b];
  *body = b;
  const uint8_t* fi = B.type[b] ? T->cube_f[f] : T->sphere_f[f];
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

__device__ __forceinline__ int64_t tri_area(const int32_t* X, const int32_t* Y) {
  return (int64_t)(X[1] - X[0]) * (int64_t)(Y[2] - Y[0]) -
         (int64_t)(Y[1] - Y[0]) * (int64_t)(X[2] - X[0]);
}

// Pixel range whose centres 256p+128 lie inside the bounding box, clipped
// to the image; returns false if empty.
__device__ __forceinline__ bool tri_pixels(const int32_t* X, const int32_t* Y, int W, int H, int* x0,
                                           int* x1, int* y0, int* y1) {
  const int xmin = min(X[0], min(X[1], X[2])), xmax = max(X[0], max(X[1], X[2]));
  const int ymin = min(Y[0], min(Y[1], Y[2])), ymax = max(Y[0], max(Y[1], Y[2]));
  *x0 = max(0, (xmin + 127) >> 8);
  *x1 = min(W - 1, (xmax - 128) >> 8);
  *y0 = max(0, (ymin + 127) >> 8);
  *y1 = min(H - 1, (ymax - 128) >> 8);
  return *x0 <= *x1 && *y0 <= *y1;
}

__device__ __forceinline__ bool top_left(int32_t dx, int32_t dy) {
  return dy < 0 || (dy == 0 && dx > 0);
}

// Classify the pixel centres of the tile block [x0..x1] x [y0..y1] against
// the edges of a snapped triangle (edge order): 0 none can be covered, 1 some
// may be, 2 all are.  Edge values are affine in the pixel centre, so their
// extremes over the block are at its corners; all values are exact in fp64.
__device__ __forceinline__ int tile_class(const int32_t* X, const int32_t* Y, int x0, int x1, int y0,
                                          int y1) {
  const double Px = (double)(256 * x0 + 128), Py = (double)(256 * y0 + 128);
  const double wx = (double)(256 * (x1 - x0)), wy = (double)(256 * (y1 - y0));
  bool all = true;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int a = (e + 1) % 3, b = (e + 2) % 3;
    const int32_t dx = X[b] - X[a], dy = Y[b] - Y[a];
    const double E = (double)dx * (Py - (double)Y[a]) - (double)dy * (Px - (double)X[a]);
    const double ax = -(double)dy * wx, ay = (double)dx * wy;
    const double emin = E + fmin(0.0, ax) + fmin(0.0, ay);
    const double emax = E + fmax(0.0, ax) + fmax(0.0, ay);
    const bool tl = top_left(dx, dy);
    if (emax < 0.0 || (emax == 0.0 && !tl)) return 0;
    if (!(emin > 0.0 || (emin == 0.0 && tl))) all = false;
  }
  return all ? 2 : 1;
}

// Flat Lambert colour of face `face` of body `body` (-1: ground), RGB8 packed.
__device__ __forceinline__ uint32_t face_color(const Templates* tp, const BodyLDS& B, int nmax,
                                               int body, int face) {
  float nx, ny, nz, al[3];
  if (body < 0) {
    nx = 0.0f; ny = 0.0f; nz = 1.0f;
    al[0] = al[1] = al[2] = tp->ground_albedo;
  } else {
    const float* nf = B.type[body] ? tp->cube_n[face] : tp->sphere_n[face];
    const float* R = B.R + body;
    const int S = nmax;
    nx = (R[0] * nf[0] + R[S] * nf[1]) + R[2 * S] * nf[2];
    ny = (R[3 * S] * nf[0] + R[4 * S] * nf[1]) + R[5 * S] * nf[2];
    nz = (R[6 * S] * nf[0] + R[7 * S] * nf[1]) + R[8 * S] * nf[2];
    const int ai = B.alb[body];
    al[0] = tp->palette[ai][0];
    al[1] = tp->palette[ai][1];
    al[2] = tp->palette[ai][2];
  }
  const float l = fmaxf(0.0f, (nx * tp->light[0] + ny * tp->light[1]) + nz * tp->light[2]);
  uint32_t rgb = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float col = al[c] * (0.2f + 0.8f * l);
    rgb |= (uint32_t)fminf(255.0f, rintf(col * 255.0f)) << (8 * c);
  }
  return rgb;
}

__device__ __forceinline__ void store_pixel(const WorldDev& W, int64_t pix, uint32_t rgb, uint32_t D,
                                            int32_t win, int cover) {
  W.rgb[3 * pix] = (uint8_t)(rgb & 0xFF);
  W.rgb[3 * pix + 1] = (uint8_t)((rgb >> 8) & 0xFF);
  W.rgb[3 * pix + 2] = (uint8_t)((rgb >> 16) & 0xFF);
  W.depth[pix] = D;
  if (W.winners) W.winners[pix] = win;
  if (W.coverage) W.coverage[pix] = cover;
}

struct Rec {
  int32_t X[3], Y[3];
  uint32_t key;
  float z[3];
  float invA;
};

__device__ __forceinline__ Rec load_rec(const int32_t* recs, int r) {
  const int4* p = (const int4*)(recs + kRecWords * r);
  const int4 a = p[0], b = p[1], c = p[2];
  Rec R;
  R.X[0] = a.x; R.Y[0] = a.y; R.X[1] = a.z; R.Y[1] = a.w;
  R.X[2] = b.x; R.Y[2] = b.y; R.key = (uint32_t)b.z; R.z[0] = __int_as_float(b.w);
  R.z[1] = __int_as_float(c.x); R.z[2] = __int_as_float(c.y); R.invA = __int_as_float(c.z);
  return R;
}

__device__ __forceinline__ void store_rec(int32_t* recs, int r, const Tri& t, uint32_t key, float invA,
                                          uint32_t rgb) {
  int4* p = (int4*)(recs + kRecWords * r);
  p[0] = make_int4(t.X[0], t.Y[0], t.X[1], t.Y[1]);
  p[1] = make_int4(t.X[2], t.Y[2], (int32_t)key, __float_as_int(t.z[0]));
  p[2] = make_int4(__float_as_int(t.z[1]), __float_as_int(t.z[2]), __float_as_int(invA), (int32_t)rgb);
}

// Coverage and key of one pixel centre (Px, Py in 24.8 units) for a record.
__device__ __forceinline__ bool pixel_key(const Rec& R, int Px, int Py, uint64_t* key) {
  double E[3];
  bool in = true;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int a = (e + 1) % 3, b = (e + 2) % 3;
    const int32_t dx = R.X[b] - R.X[a], dy = R.Y[b] - R.Y[a];
    E[e] = (double)dx * (double)(Py - R.Y[a]) - (double)dy * (double)(Px - R.X[a]);
    in = in && (E[e] > 0.0 || (E[e] == 0.0 && top_left(dx, dy)));
  }
  if (!in) return false;
  const float zz = (((float)E[0] * R.z[0] + (float)E[1] * R.z[1]) + (float)E[2] * R.z[2]) * R.invA;
  const uint32_t D = (uint32_t)rintf(fminf(fmaxf(zz, 0.0f), 1.0f) * 16777215.0f);
  *key = ((uint64_t)D << 32) | R.key;
  return true;
}

// Inclusive wave64 scans with DPP row shifts and row broadcasts: each step is
// a VALU operation reading a neighbour lane, with no LDS round trip.  Lanes
// whose source is outside the row read the identity (0; values are >= 0).
__device__ __forceinline__ int wave_incl_add(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}
__device__ __forceinline__ int wave_incl_max(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
  return x;
}

struct ImageCtx {
  int Wd, Ht, ntx, nty, ntiles;
  int64_t pix_off;
  int env;
};

// Exclusive prefix sum over the workgroup of one value per thread.
__device__ __forceinline__ int wg_excl_scan(int v, int32_t* tmp, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  int base = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    const int t = tmp[k];
    base += k < wave ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// toff[t] = sum of cnt[0..t), toff[n] = total, with every thread of the group.
__device__ __forceinline__ int tile_scan(const int32_t* cnt, int32_t* toff, int n, int32_t* tmp) {
  const int nthr = blockDim.x;
  const int per = (n + nthr - 1) / nthr;
  const int t0 = min(n, (int)threadIdx.x * per), t1 = min(n, t0 + per);
  int s = 0;
  for (int t = t0; t < t1; ++t) s += cnt[t];
  int total;
  int acc = wg_excl_scan(s, tmp, &total);
  for (int t = t0; t < t1; ++t) {
    toff[t] = acc;
    acc += cnt[t];
  }
  if (threadIdx.x == 0) toff[n] = total;
  __syncthreads();
  return total;
}

// Fast path, step 4: one tile by one wave, from setup records.
__device__ void raster_tile_fast(const WorldDev& W, const ImageCtx& im, const int32_t* recs,
                                 const uint16_t* bins, int k0, int k1, int tile, uint64_t* zb,
                                 int32_t* cov) {
  int32_t* own = cov + 256;  // 64 fragment-owner marks of this wave
  const int lane = threadIdx.x & 63;
  const int tx = tile % im.ntx, ty = tile / im.ntx;
  const int tx0 = tx * kTile, ty0 = ty * kTile;
  const int tx1 = min(tx0 + kTile - 1, im.Wd - 1), ty1 = min(ty0 + kTile - 1, im.Ht - 1);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    zb[lane + 64 * r] = ~0ull;
    cov[lane + 64 * r] = 0;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  // this lane's four pixels for the large-triangle path
  const int px = tx0 + (lane & 15);
  const int py0 = ty0 + (lane >> 4);
  uint64_t kreg[4];
  int creg[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) { kreg[r] = ~0ull; creg[r] = 0; }

  for (int kb = k0; kb < k1; kb += 64) {
    const int k = kb + lane;
    int rec = 0, fx0 = 0, fy0 = 0, bw = 1, area = 0, full = 0;
    if (k < k1) {
      const int entry = bins[k];
      rec = entry & 0x7FFF;
      full = entry >> 15;
      const Rec R = load_rec(recs, rec);
      int x0, x1, y0, y1;
      tri_pixels(R.X, R.Y, im.Wd, im.Ht, &x0, &x1, &y0, &y1);
      fx0 = max(x0, tx0);
      fy0 = max(y0, ty0);
      bw = min(x1, tx1) - fx0 + 1;
      const int bh = min(y1, ty1) - fy0 + 1;
      area = (bw > 0 && bh > 0) ? bw * bh : 0;
      if (bw < 1) bw = 1;
    }
    const bool big = area > 64;
    // small triangles: fragments packed over lanes.  Fragment f belongs to
    // the lane j with off_j <= f < off_j + a_j; per window of 64 fragments
    // each owner marks where its range starts and a max-scan spreads it.
    const int a = big ? 0 : area;
    const int incl = wave_incl_add(a);
    const int F = __builtin_amdgcn_readlane(incl, 63);
    const int off = incl - a;
    int carry = 0;  // owner + 1 of the fragment before the window
    for (int f0 = 0; f0 < F; f0 += 64) {
      own[lane] = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      if (a > 0 && off >= f0 && off < f0 + 64) own[off - f0] = lane + 1;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      int o = own[lane];
      if (lane == 0) o = max(o, carry);
      o = wave_incl_max(o);
      carry = __builtin_amdgcn_readlane(o, 63);
      const int j = o - 1;  // >= 0 for every fragment below F
      const int f = f0 + lane;
      const int jrec = __shfl(rec, j, 64);
      const int jx0 = __shfl(fx0, j, 64), jy0 = __shfl(fy0, j, 64);
      const int jbw = __shfl(bw, j, 64), joff = __shfl(off, j, 64);
      if (f < F) {
        const int rr = f - joff;
        // rr / jbw exactly: rr < 64 and jbw <= 16 leave a margin far above the rounding
        const int qy = (int)(((float)rr + 0.5f) * (1.0f / (float)jbw));
        const int qx = rr - qy * jbw;
        const int ppx = jx0 + qx, ppy = jy0 + qy;
        const int p = (ppy - ty0) * kTile + (ppx - tx0);
        const Rec R = load_rec(recs, jrec);
        uint64_t kk;
        if (p >= 0 && p < 256 && pixel_key(R, 256 * ppx + 128, 256 * ppy + 128, &kk)) {
          atomicMin((unsigned long long*)&zb[p], (unsigned long long)kk);
          atomicAdd(&cov[p], 1);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    }
    // large triangles: one lane per four pixels, the record uniform
    uint64_t m = __ballot(big);
    while (m) {
      const int j = __ffsll((unsigned long long)m) - 1;
      m &= m - 1ull;
      const int jrec = __builtin_amdgcn_readfirstlane(__shfl(rec, j, 64));
      const bool jfull = __builtin_amdgcn_readfirstlane(__shfl(full, j, 64)) != 0;
      const Rec R = load_rec(recs, jrec);
      // E is an integer held exactly in fp64; inside the edge means E > 0, or
      // E == 0 on a top-left edge, i.e. E + tl > 0 with tl in {0, 1}.
      double ea[3], E[3], tb[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const int a0 = (e + 1) % 3, b0 = (e + 2) % 3;
        const int32_t dx = R.X[b0] - R.X[a0], dy = R.Y[b0] - R.Y[a0];
        ea[e] = (double)dx * 1024.0;  // 4 pixel rows down
        tb[e] = top_left(dx, dy) ? 1.0 : 0.0;
        E[e] = (double)dx * (double)(256 * py0 + 128 - R.Y[a0]) - (double)dy * (double)(256 * px + 128 - R.X[a0]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double m = fmin(fmin(E[0] + tb[0], E[1] + tb[1]), E[2] + tb[2]);
        const float zz = (((float)E[0] * R.z[0] + (float)E[1] * R.z[1]) + (float)E[2] * R.z[2]) * R.invA;
        const uint32_t D = (uint32_t)rintf(fminf(fmaxf(zz, 0.0f), 1.0f) * 16777215.0f);
        const uint64_t kk = ((uint64_t)D << 32) | R.key;
        const bool in = jfull || m > 0.0;
        creg[r] += in ? 1 : 0;
        kreg[r] = (in && kk < kreg[r]) ? kk : kreg[r];
#pragma unroll
        for (int e = 0; e < 3; ++e) E[e] += ea[e];
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int py = py0 + 4 * r;
    if (px > tx1 || py > ty1) continue;
    const int p = lane + 64 * r;
    const uint64_t z = zb[p];
    const uint64_t key = z < kreg[r] ? z : kreg[r];
    const int64_t pix = im.pix_off + (int64_t)py * im.Wd + px;
    uint32_t rgb = 0, D = 0xFFFFFFFFu;
    int32_t win = -1;
    if (key != ~0ull) {
      const uint32_t lo = (uint32_t)key;
      D = (uint32_t)(key >> 32);
      win = (int32_t)(lo >> 16);
      rgb = (uint32_t)recs[kRecWords * (lo & 0xFFFFu) + 11];
    }
    store_pixel(W, pix, rgb, D, win, cov[p] + creg[r]);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Slow path: re-derive triangles from the vertex cache, tiles in groups whose
// bins fit the record region.  Keys: depth << 32 | (body + 1) << 16 | prim.
__device__ void raster_slow(unsigned char* lds, const RasterLayout& Lo, const WorldDev& W,
                            const TplLDS* T, const BodyLDS& B, const uint8_t* pmap, int ntris,
                            const ImageCtx& im, bool* overflow) {
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const Templates* tp = W.tpl;
  const int32_t* VX = (const int32_t*)(lds + Lo.verts);
  const int32_t* VY = VX + Lo.vmax;
  const float* VZ = (const float*)(VY + Lo.vmax);
  int32_t* tcount = (int32_t*)(lds + Lo.tiles);
  int32_t* toff = tcount + Lo.tw;
  int32_t* tfill = toff + Lo.tw + 1;
  uint32_t* bins = (uint32_t*)(lds + Lo.recs);
  int32_t* misc = (int32_t*)(lds + Lo.misc);
  const int bin_cap = Lo.bin_cap_slow;
  const int nwaves = nthr >> 6;
  const int wave = tid >> 6, lane = tid & 63;

  for (int w0 = 0; w0 < im.ntiles; w0 += Lo.tw) {
    const int w1 = min(im.ntiles, w0 + Lo.tw);
    for (int t = tid; t < w1 - w0; t += nthr) tcount[t] = 0;
    __syncthreads();
    for (int pr = tid; pr < ntris; pr += nthr) {
      int body, vid[3];
      prim_vertices(T, B, pmap, pr, &body, vid);
      const Tri t = load_tri(VX, VY, VZ, vid);
      if (!t.ok || tri_area(t.X, t.Y) <= 0) continue;
      int x0, x1, y0, y1;
      if (!tri_pixels(t.X, t.Y, im.Wd, im.Ht, &x0, &x1, &y0, &y1)) continue;
      for (int ty = y0 >> 4; ty <= (y1 >> 4); ++ty)
        for (int tx = x0 >> 4; tx <= (x1 >> 4); ++tx) {
          const int ti = ty * im.ntx + tx - w0;
          if (ti >= 0 && ti < w1 - w0) atomicAdd(&tcount[ti], 1);
        }
    }
    __syncthreads();
    tile_scan(tcount, toff, w1 - w0, misc + 8);
    int g0 = 0;
    while (g0 < w1 - w0) {
      if (tid == 0) {
        int g1 = g0 + 1;
        while (g1 < w1 - w0 && toff[g1 + 1] - toff[g0] <= bin_cap) ++g1;
        misc[0] = g1;
        misc[1] = toff[g1] - toff[g0] > bin_cap ? 1 : 0;
      }
      __syncthreads();
      const int g1 = misc[0];
      if (misc[1]) *overflow = true;
      const int base = toff[g0];
      for (int t = g0 + tid; t < g1; t += nthr) tfill[t] = 0;
      __syncthreads();
      for (int pr = tid; pr < ntris; pr += nthr) {
        int body, vid[3];
        prim_vertices(T, B, pmap, pr, &body, vid);
        const Tri t = load_tri(VX, VY, VZ, vid);
        if (!t.ok || tri_area(t.X, t.Y) <= 0) continue;
        int x0, x1, y0, y1;
        if (!tri_pixels(t.X, t.Y, im.Wd, im.Ht, &x0, &x1, &y0, &y1)) continue;
        const uint32_t entry = (uint32_t)pr | ((uint32_t)(body + 1) << 16);
        for (int ty = y0 >> 4; ty <= (y1 >> 4); ++ty)
          for (int tx = x0 >> 4; tx <= (x1 >> 4); ++tx) {
            const int ti = ty * im.ntx + tx - w0;
            if (ti >= g0 && ti < g1) {
              const int slot = toff[ti] - base + atomicAdd(&tfill[ti], 1);
              if (slot < bin_cap) bins[slot] = entry;
            }
          }
      }
      __syncthreads();
      for (int ti = g0 + wave; ti < g1; ti += nwaves) {
        const int tile = w0 + ti;
        const int tx = tile % im.ntx, ty = tile / im.ntx;
        const int px = tx * kTile + (lane & 15);
        const int py0 = ty * kTile + (lane >> 4);
        uint64_t key[4];
        int cover[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) { key[r] = ~0ull; cover[r] = 0; }
        const int k0 = toff[ti] - base, k1 = min(toff[ti + 1] - base, bin_cap);
        for (int k = k0; k < k1; ++k) {
          const uint32_t entry = __builtin_amdgcn_readfirstlane(bins[k]);
          int body, vid[3];
          prim_vertices(T, B, pmap, (int)(entry & 0xFFFFu), &body, vid);
          const Tri t = load_tri(VX, VY, VZ, vid);
          Rec R;
#pragma unroll
          for (int q = 0; q < 3; ++q) { R.X[q] = t.X[q]; R.Y[q] = t.Y[q]; R.z[q] = t.z[q]; }
          R.key = entry;
          R.invA = 1.0f / (float)(double)tri_area(t.X, t.Y);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            uint64_t kk;
            if (pixel_key(R, 256 * px + 128, 256 * (py0 + 4 * r) + 128, &kk)) {
              cover[r] += 1;
              if (kk < key[r]) key[r] = kk;
            }
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int py = py0 + 4 * r;
          if (px >= im.Wd || py >= im.Ht) continue;
          uint32_t rgb = 0, D = 0xFFFFFFFFu;
          int32_t win = -1;
          if (key[r] != ~0ull) {
            const uint32_t e = (uint32_t)key[r];
            D = (uint32_t)(key[r] >> 32);
            win = (int32_t)(e & 0xFFFFu);
            const int body = (int)(e >> 16) - 1;
            rgb = face_color(tp, B, Lo.nmax, body, body < 0 ? win : win - B.pb[body]);
          }
          store_pixel(W, im.pix_off + (int64_t)py * im.Wd + px, rgb, D, win, cover[r]);
        }
      }
      __syncthreads();
      g0 = g1;
    }
  }
}

constexpr int kWide = 8;

// Bin record r into tile (tx, ty) unless its edges miss the tile; flag the
// entry when the triangle covers every pixel of the tile.
__device__ __forceinline__ void bin_tile(const Rec& R, int r, int tx, int ty, int x0, int x1, int y0,
                                         int y1, bool classify, const ImageCtx& im, const int32_t* toff,
                                         int32_t* tfill, uint16_t* bins) {
  const int bx0 = max(x0, tx * kTile), bx1 = min(x1, tx * kTile + kTile - 1);
  const int by0 = max(y0, ty * kTile), by1 = min(y1, ty * kTile + kTile - 1);
  const int cls = classify ? tile_class(R.X, R.Y, bx0, bx1, by0, by1) : 1;
  if (cls == 0) return;
  const bool whole = bx0 == tx * kTile && by0 == ty * kTile &&
                     bx1 == min(im.Wd - 1, tx * kTile + kTile - 1) &&
                     by1 == min(im.Ht - 1, ty * kTile + kTile - 1);
  const int ti = ty * im.ntx + tx;
  bins[toff[ti] + atomicAdd(&tfill[ti], 1)] = (uint16_t)(r | ((cls == 2 && whole) ? 0x8000 : 0));
}

__device__ void raster_image(unsigned char* lds, const RasterLayout& Lo, const WorldDev& W,
                             const RasterLaunch& L, int cam_id) {
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const CamDev cam = W.cams[cam_id];
  const EnvDev ed = W.envs[cam.env];
  const int n = ed.n_bodies;
  const int64_t cap = W.cap_bodies;
  const float* st = W.state[L.parity];
  const uint8_t* gpmap = W.prim_body + ed.prim_map;
  const uint8_t* gvmap = W.vert_body + ed.vert_map;
  ImageCtx im;
  im.Wd = cam.w;
  im.Ht = cam.h;
  im.ntx = (im.Wd + kTile - 1) / kTile;
  im.nty = (im.Ht + kTile - 1) / kTile;
  im.ntiles = im.ntx * im.nty;
  im.pix_off = cam.pix_off;
  im.env = cam.env;

  TplLDS* T = (TplLDS*)(lds + Lo.tpl);
  const Templates* tp = W.tpl;
  uint8_t* pmap = lds + Lo.maps;
  uint8_t* vmap = pmap + align16(L.max_tris);
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
  int32_t* recs = (int32_t*)(lds + Lo.recs);
  int32_t* tcount = (int32_t*)(lds + Lo.tiles);
  int32_t* toff = tcount + Lo.tw;
  int32_t* tfill = toff + Lo.tw + 1;
  int32_t* misc = (int32_t*)(lds + Lo.misc);

  // 1. bodies and templates
  {
    const int4* src = (const int4*)W.tpl;
    int4* dst = (int4*)T;
    for (int i = tid; i < kTplBytes / 16; i += nthr) dst[i] = src[i];
    for (int i = tid; i < (ed.n_tris + 15) / 16; i += nthr) ((int4*)pmap)[i] = ((const int4*)gpmap)[i];
    for (int i = tid; i < (ed.n_verts + 15) / 16; i += nthr) ((int4*)vmap)[i] = ((const int4*)gvmap)[i];
  }
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
  if (tid == 0) misc[2] = 0;  // records
  const bool fast_tiles = im.ntiles <= Lo.tw;
  if (fast_tiles)
    for (int t = tid; t < im.ntiles; t += nthr) tcount[t] = 0;
  __syncthreads();

  // 2. vertices
  const float* vp = cam.vp;
  const float fW = (float)im.Wd, fH = (float)im.Ht;
  for (int vi = tid; vi < ed.n_verts; vi += nthr) {
    float wx, wy, wz;
    const int b = vmap[vi];
    if (b == kGroundBody) {
      wx = T->ground_v[vi][0];
      wy = T->ground_v[vi][1];
      wz = T->ground_v[vi][2];
    } else {
      const int lv = vi - B.vb[b];
      const float* tv = B.type[b] ? T->cube_v[lv] : T->sphere_v[lv];
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

  // 3. setup records (with the face colour) and tile counts.  A triangle
  // whose box spans more than kWide tiles is binned by its whole wave, one
  // tile per lane, so that one lane never walks a long tile list alone.
  const int ntris = ed.n_tris;
  const int lane = tid & 63;
  for (int base = 0; base < ntris; base += nthr) {
    const int pr = base + tid;
    int tx0 = 0, ty0 = 0, nx = 0, ntl = 0;
    if (pr < ntris) {
      int body, vid[3];
      prim_vertices(T, B, pmap, pr, &body, vid);
      const Tri t = load_tri(VX, VY, VZ, vid);
      int x0, x1, y0, y1;
      if (t.ok) {
        const int64_t A = tri_area(t.X, t.Y);
        if (A > 0 && tri_pixels(t.X, t.Y, im.Wd, im.Ht, &x0, &x1, &y0, &y1)) {
          const int slot = atomicAdd(&misc[2], 1);
          if (slot < Lo.rec_cap) {
            const uint32_t rgb = face_color(tp, B, Lo.nmax, body, body < 0 ? pr : pr - B.pb[body]);
            store_rec(recs, slot, t, ((uint32_t)pr << 16) | (uint32_t)slot, 1.0f / (float)(double)A, rgb);
          }
          tx0 = x0 >> 4;
          ty0 = y0 >> 4;
          nx = (x1 >> 4) - tx0 + 1;
          ntl = nx * ((y1 >> 4) - ty0 + 1);
        }
      }
    }
    if (!fast_tiles) continue;
    if (ntl <= kWide)
      for (int q = 0; q < ntl; ++q) {
        const int qy = q / nx;
        atomicAdd(&tcount[(ty0 + qy) * im.ntx + tx0 + (q - qy * nx)], 1);
      }
    uint64_t m = __ballot(ntl > kWide);
    while (m) {
      const int j = __ffsll((unsigned long long)m) - 1;
      m &= m - 1ull;
      const int jx0 = __shfl(tx0, j, 64), jy0 = __shfl(ty0, j, 64);
      const int jnx = __shfl(nx, j, 64), jn = __shfl(ntl, j, 64);
      for (int q = lane; q < jn; q += 64) {
        const int qy = q / jnx;
        atomicAdd(&tcount[(jy0 + qy) * im.ntx + jx0 + (q - qy * jnx)], 1);
      }
    }
  }
  __syncthreads();
  const int nrec = misc[2];
  bool fast = fast_tiles && nrec <= Lo.rec_cap;
  if (fast) {
    const int total = tile_scan(tcount, toff, im.ntiles, misc + 8);
    if (total > Lo.bin_cap_fast) fast = false;
  }

  bool overflow = false;
  if (fast) {
    // scatter record ids into the bins (the vertex cache is no longer needed)
    uint16_t* bins = (uint16_t*)(lds + Lo.verts);
    for (int t = tid; t < im.ntiles; t += nthr) tfill[t] = 0;
    __syncthreads();
    for (int base = 0; base < nrec; base += nthr) {
      const int r = base + tid;
      int x0 = 0, x1 = 0, y0 = 0, y1 = 0, nx = 0, ntl = 0;
      Rec R;
      if (r < nrec) {
        R = load_rec(recs, r);
        tri_pixels(R.X, R.Y, im.Wd, im.Ht, &x0, &x1, &y0, &y1);
        nx = (x1 >> 4) - (x0 >> 4) + 1;
        ntl = nx * ((y1 >> 4) - (y0 >> 4) + 1);
      }
      if (ntl <= kWide)
        for (int q = 0; q < ntl; ++q) {
          const int qy = q / nx;
          bin_tile(R, r, (x0 >> 4) + (q - qy * nx), (y0 >> 4) + qy, x0, x1, y0, y1, ntl > 1, im, toff,
                   tfill, bins);
        }
      uint64_t m = __ballot(ntl > kWide);
      while (m) {
        const int j = __ffsll((unsigned long long)m) - 1;
        m &= m - 1ull;
        const int jr = __builtin_amdgcn_readfirstlane(__shfl(r, j, 64));
        const Rec J = load_rec(recs, jr);
        int jx0, jx1, jy0, jy1;
        tri_pixels(J.X, J.Y, im.Wd, im.Ht, &jx0, &jx1, &jy0, &jy1);
        const int jnx = (jx1 >> 4) - (jx0 >> 4) + 1;
        const int jn = jnx * ((jy1 >> 4) - (jy0 >> 4) + 1);
        for (int q = lane; q < jn; q += 64) {
          const int qy = q / jnx;
          bin_tile(J, jr, (jx0 >> 4) + (q - qy * jnx), (jy0 >> 4) + qy, jx0, jx1, jy0, jy1, true, im,
                   toff, tfill, bins);
        }
      }
    }
    __syncthreads();
    const int wave = tid >> 6;
    uint64_t* zb = (uint64_t*)(lds + Lo.waves + wave * kWaveBytes);
    int32_t* cov = (int32_t*)(zb + 256);
    for (int ti = wave; ti < im.ntiles; ti += Lo.nwaves)
      raster_tile_fast(W, im, recs, bins, toff[ti], toff[ti] + tfill[ti], ti, zb, cov);
  } else {
    raster_slow(lds, Lo, W, T, B, pmap, ntris, im, &overflow);
  }
  if (overflow && tid == 0) atomicOr(&W.env_flags[cam.env], kFlagBinOverflow);
}

__global__ void raster_kernel(WorldDev W, RasterLaunch L) {
  extern __shared__ __align__(16) unsigned char lds[];
  const RasterLayout Lo = make_layout(L.max_bodies, L.max_verts, L.max_tiles, L.max_tris, L.rec_cap, blockDim.x);
  if (L.persistent == 0) {
    if ((int)blockIdx.x >= L.n_work) return;
    raster_image(lds, Lo, W, L, L.work[blockIdx.x]);
    return;
  }
  int32_t* slot = (int32_t*)(lds + Lo.misc) + 4;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(L.queue, 1);
    __syncthreads();
    const int wi = *slot;
    if (wi >= L.n_work) return;
    raster_image(lds, Lo, W, L, L.work[wi]);
  }
}

}  // namespace

size_t raster_lds_bytes(const RasterLaunch& l) {
  return (size_t)make_layout(l.max_bodies, l.max_verts, l.max_tiles, l.max_tris, l.rec_cap, l.threads).total;
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
