// Tiled software rasterizer for gfx950: two kernels per render launch.
//
// raster_setup_kernel, one workgroup per camera image:
//   1. body poses, read in place from the physics state buffer, with R(q),
//      and the mesh templates go to LDS;
//   2. every template vertex of every body (and the ground) is transformed
//      once -- world = p + R (s v), clip = VP world, perspective divide,
//      viewport, snap to 24.8 fixed point -- into an LDS vertex cache;
//   3. culling: a triangle is dropped if a vertex in front of the near plane
//      is outside the guard band, if it is back-facing or degenerate (integer
//      area <= 0), or if its bounding box holds no pixel centre; one that
//      crosses the near plane is cut along it into one or two pieces (the
//      polygon in front, split as a fan), each culled the same way;
//      survivors are compacted into lists;
//   4. each survivor gets a setup record in the image's raster scratch
//      (snapped vertices in edge order, depths, 1/area, primitive and flat Lambert
//      colour) and the tiles of its box are counted with LDS atomics;
//   5. a workgroup prefix scan of the counts places each 16x16 tile's bin; a
//      scatter pass appends each triangle's record id to the bins of the
//      tiles of its box, after an exact corner test of the edge functions
//      where its box in the tile is large, flagged when the triangle covers
//      the whole tile.
// raster_tile_kernel, one wave per tile and one, two or four tiles of a row
//   per workgroup; a lane owns four horizontally adjacent pixels.  The bin is read in batches of 64
//   records.  Small triangles (at most 64 pixels of their box in the tile)
//   are expanded into fragments, one pixel per lane across several
//   triangles, whose keys meet in an LDS z-buffer through atomic minimum;
//   large ones are tested by every lane on its own four pixels, keeping the
//   minimum in registers.  Edge functions are exact (integer values carried
//   in fp64); a pixel centre is covered if every edge value is > 0, or == 0
//   on a top-left edge.  Depth is interpolated in fp32 and quantised to 24
//   bits, and the minimum key (depth << 40 | primitive << 24 | RGB8) wins,
//   so the result depends neither on bin order nor on which lane tests which
//   pixel.  The winner's colour comes from its record; depth and RGB8 leave
//   in 16- and 4-byte stores.
// An image whose bins exceed their capacity, or whose tile table does not fit
// the setup kernel's LDS, is marked unbinned: each of its tiles then tests
// every record of the image -- slower, with the same output.
#include <cstddef>

#include <type_traits>

#include "vuda_internal.h"

#pragma clang fp contract(off)

namespace vuda {
namespace {

constexpr int kMaxLdsTiles = 4096;  // tile table held in the setup kernel's LDS
constexpr int kSmallMax = 64;       // box pixels in the tile of a fragment-packed triangle
constexpr int kWide = 8;            // triangles over more tiles are binned by their whole wave
constexpr int kTplBytes = (int)((sizeof(Templates) + 15) & ~(size_t)15);

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

struct SetupLayout {
  // byte offsets into the setup (or fused) kernel's dynamic LDS
  int tpl, body, verts, vis, cvis, pmap, vmap, tiles, misc, lrec, lbin, total;
  int nmax, vmax, tw, rec_cap, bin_cap;
};

// The regions the setup alone uses (templates, poses, survivor lists, maps)
// come first, and at least zone0 bytes are reserved for them: the fused
// kernel's tile pass keeps its z-buffers there once the setup is done.  Then
// the vertex cache, the tile table and counters, and (fused kernel) rec_cap
// compact records and bin_cap bin entries.
__host__ __device__ inline SetupLayout setup_layout(int max_bodies, int max_verts, int max_tiles,
                                                    int max_tris, bool near_clip, int zone0 = 0,
                                                    int rec_cap = 0, int bin_cap = 0) {
  SetupLayout L;
  L.nmax = max_bodies + 1;
  L.vmax = max_verts;
  L.tw = max_tiles < kMaxLdsTiles ? max_tiles : kMaxLdsTiles;
  L.rec_cap = rec_cap;
  L.bin_cap = bin_cap;
  int o = 0;
  L.tpl = o;    o += kTplBytes;
  L.body = o;   o += align16(4 * 20 * L.nmax);
  L.vis = o;    o += align16(2 * max_tris);
  L.cvis = o;   o += near_clip ? align16(40 * kClipRecs) : 0;  // near-plane pieces: X[3] Y[3] z[3], primitive
  L.pmap = o;   o += align16(max_tris);   // primitive -> body map of the env
  L.vmap = o;   o += align16(L.vmax);     // vertex -> body map of the env
  if (o < zone0) o = align16(zone0);
  L.verts = o;  o += 16 * L.vmax;         // (X, Y, z, 0) per vertex
  L.tiles = o;  o += align16(4 * (3 * L.tw + 1));
  L.misc = o;   o += 128;  // [2] record count, [3] near-plane pieces, [4] queue slot,
                           // [5] a vertex behind the near plane, [6] fused: bit 0 records
                           // and bins in LDS, bit 1 binned; [8, 24) scan totals
  L.lrec = o;   o += 16 * rec_cap;
  L.lbin = o;   o += align16(2 * bin_cap);
  L.total = o;
  return L;
}

struct BodyLDS {
  float* p;       // [3][nmax]
  float* R;       // [9][nmax]
  float4* e;      // [nmax] half-extents along the body axes (x, y, z, 0); a radius thrice for a sphere
  int32_t* type;  // [nmax]
  int32_t* vb;    // [nmax] vertex base (env-local)
  int32_t* pb;    // [nmax] primitive base
  int32_t* alb;   // [nmax]
};

// Rotation matrix of a unit quaternion, row-major, element k at m[k * stride]
__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float* m, int stride) {
  const float xx = x * x, yy = y * y, zz = z * z;
  const float xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  m[0] = 1.0f - 2.0f * (yy + zz);
  m[stride] = 2.0f * (xy - wz);
  m[2 * stride] = 2.0f * (xz + wy);
  m[3 * stride] = 2.0f * (xy + wz);
  m[4 * stride] = 1.0f - 2.0f * (xx + zz);
  m[5 * stride] = 2.0f * (yz - wx);
  m[6 * stride] = 2.0f * (xz - wy);
  m[7 * stride] = 2.0f * (yz + wx);
  m[8 * stride] = 1.0f - 2.0f * (xx + yy);
}

constexpr int32_t kInvalid = (int32_t)0x80000000;  // in front, outside the guard band
constexpr int32_t kBehind = (int32_t)0x80000001;   // behind the near plane (clip w < near)

// Snapped screen-space triangle in edge order (vertices 0, 2, 1 of the face).
struct Tri {
  int32_t X[3], Y[3];
  float z[3];
  bool ok;
};

// vertex indices (env-local) of primitive `prim` whose body (from the map) is
// b; *body = -1 for the ground
__device__ __forceinline__ void prim_vertices(const Templates* T, const BodyLDS& B, int b, int prim,
                                              int* body, int vid[3]) {
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

__device__ __forceinline__ Tri load_tri(const int4* V, const int vid[3]) {
  Tri t;
  const int ord[3] = {0, 2, 1};
  t.ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int4 q = V[vid[ord[k]]];
    t.X[k] = q.x;
    t.Y[k] = q.y;
    t.z[k] = __int_as_float(q.z);
    if (t.X[k] <= kBehind) t.ok = false;  // kInvalid or kBehind
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

// Viewport transform and 24.8 snap of clip coordinates c: X = kBehind when
// near_test and c.w < near, kInvalid outside the guard band.
__device__ __forceinline__ void snap_clip(float4 c, float fW, float fH, const Templates* T, bool near_test,
                                          int32_t* X, int32_t* Y, float* z) {
  *X = kInvalid;
  *Y = kInvalid;
  *z = 0.0f;
  if (near_test && c.w < T->near_w) {
    *X = *Y = kBehind;
    return;
  }
  const float nx = c.x / c.w, ny = c.y / c.w, nz = c.z / c.w;
  const float px = (nx * 0.5f + 0.5f) * fW;
  const float py = (0.5f - ny * 0.5f) * fH;
  if (!(fabsf(px) > T->guard || fabsf(py) > T->guard)) {
    *X = (int32_t)rintf(px * 256.0f);
    *Y = (int32_t)rintf(py * 256.0f);
    *z = nz;
  }
}

// The point where the edge from a (in front) to b (behind) meets the plane
// w = near, taken from the vertex in front so that both triangles sharing
// the edge cut it at the same point.
__device__ __forceinline__ float4 near_cut(float4 a, float4 b, float near_w) {
  const float t = (near_w - a.w) / (b.w - a.w);
  return make_float4(a.x + t * (b.x - a.x), a.y + t * (b.y - a.y), a.z + t * (b.z - a.z), a.w + t * (b.w - a.w));
}

// Piece s (0 or 1) of the part of a triangle in front of the near plane (c:
// clip coordinates of its vertices in face order, at least one in front and
// none in front outside the guard band): the polygon in front, in face
// order, split as a fan from its first vertex; the piece in edge order.
// Returns false if there is no piece s; t->ok is false if a cut point falls
// outside the guard band.
__device__ __forceinline__ bool near_piece(const float4 c[3], int s, float fW, float fH, const Templates* T,
                                           Tri* t) {
  // the polygon's candidate points in cycle order: vertex k (if in front),
  // then the cut of edge k -> k+1 (if it crosses); selected with static
  // indices only, so that everything stays in registers
  float4 val[6];
  bool has[6], cut[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k1 = k == 2 ? 0 : k + 1;
    const bool ik = !(c[k].w < T->near_w), ik1 = !(c[k1].w < T->near_w);
    val[2 * k] = c[k];
    has[2 * k] = ik;
    cut[2 * k] = false;
    val[2 * k + 1] = ik ? near_cut(c[k], c[k1], T->near_w) : near_cut(c[k1], c[k], T->near_w);
    has[2 * k + 1] = ik != ik1;
    cut[2 * k + 1] = true;
  }
  int m = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) m += has[j] ? 1 : 0;
  if (s + 2 >= m) return false;
  const int want[3] = {0, s + 2, s + 1};  // the piece (q0, q[s+1], q[s+2]) in edge order
  t->ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float4 q = val[0];
    bool qc = false;
    int n = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (has[j] && n == want[k]) {
        q = val[j];
        qc = cut[j];
      }
      n += has[j] ? 1 : 0;
    }
    snap_clip(q, fW, fH, T, !qc, &t->X[k], &t->Y[k], &t->z[k]);
    if (t->X[k] == kInvalid || t->X[k] == kBehind) t->ok = false;
  }
  return true;
}

__device__ __forceinline__ bool top_left(int32_t dx, int32_t dy) {
  return dy < 0 || (dy == 0 && dx > 0);
}

// Classify the pixel centres of the block [x0..x1] x [y0..y1] against the
// edges of a snapped triangle (edge order): 0 none can be covered, 1 some may
// be, 2 all are.  Edge values are affine in the pixel centre, so their
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

// Exclusive prefix sum over the workgroup of one value per thread.
__device__ __forceinline__ int wg_excl_scan(int v, int32_t* tmp, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int x = wave_incl_add(v);
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

// A small triangle's edge values over its box, in 32-bit integers: when the
// triangle spans at most kNarrow units (120 pixels) on both axes, every edge
// value at a pixel centre in its box is at most 2 kNarrow^2 < 2^31 in
// magnitude and the steps per pixel, 256 dx and 256 dy, stay below 2^23, so
// 24-bit multiply-adds are exact.
constexpr int kNarrow = 120 * 256;

// Flags of a triangle's setup record: bit e set when edge e is not top-left
// (a pixel centre on it is outside), bit 3 set when the triangle is narrow.
__device__ __forceinline__ int rec_flags(const Tri& t) {
  int flags = 0;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int a0 = (e + 1) % 3, b0 = (e + 2) % 3;
    if (!top_left(t.X[b0] - t.X[a0], t.Y[b0] - t.Y[a0])) flags |= 1 << e;
  }
  const bool narrow = max(t.X[0], max(t.X[1], t.X[2])) - min(t.X[0], min(t.X[1], t.X[2])) <= kNarrow &&
                      max(t.Y[0], max(t.Y[1], t.Y[2])) - min(t.Y[0], min(t.Y[1], t.Y[2])) <= kNarrow;
  if (narrow) flags |= 8;
  return flags;
}

// Setup record of a triangle in the image's raster scratch (64 bytes): what
// every tile it is binned to needs, so that the tile kernel recomputes none
// of it.  Word 2 of the last quad holds the flags.
__device__ __forceinline__ void store_rec(int4* recs, int r, const Tri& t, int prim, float invA,
                                          uint32_t rgb, int x0, int x1, int y0, int y1) {
  const int flags = rec_flags(t);
  int4* p = recs + 4 * r;
  p[0] = make_int4(t.X[0], t.Y[0], t.X[1], t.Y[1]);
  p[1] = make_int4(t.X[2], t.Y[2], prim, __float_as_int(t.z[0]));
  p[2] = make_int4(__float_as_int(t.z[1]), __float_as_int(t.z[2]), __float_as_int(invA), (int32_t)rgb);
  p[3] = make_int4(x0 | (x1 << 16), y0 | (y1 << 16), flags, 0);
}

// Append record r to the bin of tile (tx, ty) unless its edges miss the tile;
// flag the entry when the triangle covers every pixel of the tile.  Only a
// box of more than kSmallMax pixels in the tile is classified (the tile
// kernel rasterizes it pixel by pixel over the whole tile, where the flag and
// the rejection pay); a smaller one is expanded into its box's pixels there
// anyway.
__device__ __forceinline__ void bin_tile(const Tri& t, int r, int tx, int ty, int x0, int x1, int y0,
                                         int y1, bool classify, int Wd, int Ht, int ntx, int TS,
                                         const int32_t* toff, int32_t* tfill, uint16_t* bins) {
  const int bx0 = max(x0, tx * TS), bx1 = min(x1, tx * TS + TS - 1);
  const int by0 = max(y0, ty * TS), by1 = min(y1, ty * TS + TS - 1);
  const bool large = (bx1 - bx0 + 1) * (by1 - by0 + 1) > kSmallMax;
  const int cls = (classify && large) ? tile_class(t.X, t.Y, bx0, bx1, by0, by1) : 1;
  if (cls == 0) return;
  const bool whole = bx0 == tx * TS && by0 == ty * TS &&
                     bx1 == min(Wd - 1, tx * TS + TS - 1) &&
                     by1 == min(Ht - 1, ty * TS + TS - 1);
  const int ti = ty * ntx + tx;
  bins[toff[ti] + atomicAdd(&tfill[ti], 1)] = (uint16_t)(r | ((cls == 2 && whole) ? 0x8000 : 0));
}

// ---------------------------------------------------------------------------
// setup kernel
// ---------------------------------------------------------------------------

// Clip coordinates of env-local vertex vi: the body's pose applied to the
// scaled template vertex (the ground's vertices as they are), then the
// camera's view-projection (row dot products summed left to right, then the
// translation).
__device__ __forceinline__ float4 vertex_clip(const Templates* T, const BodyLDS& B, int S, const uint8_t* gvmap,
                                              int vi, const float* vp) {
  float wx, wy, wz;
  const int b = gvmap[vi];
  if (b == kGroundBody) {
    wx = T->ground_v[vi][0];
    wy = T->ground_v[vi][1];
    wz = T->ground_v[vi][2];
  } else {
    const int lv = vi - B.vb[b];
    const float* tv = B.type[b] ? T->cube_v[lv] : T->sphere_v[lv];
    const float4 e = B.e[b];
    const float sx = e.x * tv[0], sy = e.y * tv[1], sz = e.z * tv[2];
    const float* R = B.R + b;
    wx = B.p[b] + ((R[0] * sx + R[S] * sy) + R[2 * S] * sz);
    wy = B.p[S + b] + ((R[3 * S] * sx + R[4 * S] * sy) + R[5 * S] * sz);
    wz = B.p[2 * S + b] + ((R[6 * S] * sx + R[7 * S] * sy) + R[8 * S] * sz);
  }
  return make_float4(((vp[0] * wx + vp[1] * wy) + vp[2] * wz) + vp[3], ((vp[4] * wx + vp[5] * wy) + vp[6] * wz) + vp[7],
                     ((vp[8] * wx + vp[9] * wy) + vp[10] * wz) + vp[11],
                     ((vp[12] * wx + vp[13] * wy) + vp[14] * wz) + vp[15]);
}

// Attribute record r of a triangle for smooth shading (face `face` of body
// `body`, -1 the ground; vid its vertices in face order): the world normal
// and the reciprocal clip w of each vertex in edge order (face vertices 0, 2,
// 1), and the albedo.  A sphere's vertex normal is its unit template vertex
// turned by R, a cube's or box's the face normal, the ground's +z.
__device__ __forceinline__ void store_attr(float4* ga, float4* gt, int r, const Templates* T, const BodyLDS& B,
                                           int S, const uint8_t* gvmap, int body, int face, const int vid[3],
                                           const float* vp) {
  const int ord[3] = {0, 2, 1};
  float n[3][3], iw[3], al[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int v = vid[ord[k]];
    iw[k] = 1.0f / vertex_clip(T, B, S, gvmap, v, vp).w;
    if (body < 0) {
      n[k][0] = 0.0f;
      n[k][1] = 0.0f;
      n[k][2] = 1.0f;
    } else {
      const float* nb = B.type[body] ? T->cube_n[face] : T->sphere_v[v - B.vb[body]];
      const float* R = B.R + body;
      n[k][0] = (R[0] * nb[0] + R[S] * nb[1]) + R[2 * S] * nb[2];
      n[k][1] = (R[3 * S] * nb[0] + R[4 * S] * nb[1]) + R[5 * S] * nb[2];
      n[k][2] = (R[6 * S] * nb[0] + R[7 * S] * nb[1]) + R[8 * S] * nb[2];
    }
  }
  if (body < 0) {
    al[0] = al[1] = al[2] = T->ground_albedo;
  } else {
    const int ai = B.alb[body];
    al[0] = T->palette[ai][0];
    al[1] = T->palette[ai][1];
    al[2] = T->palette[ai][2];
  }
  float4* p = ga + 4 * r;
  p[0] = make_float4(n[0][0], n[0][1], n[0][2], n[1][0]);
  p[1] = make_float4(n[1][1], n[1][2], n[2][0], n[2][1]);
  p[2] = make_float4(n[2][2], iw[0], iw[1], iw[2]);
  p[3] = make_float4(al[0], al[1], al[2], 0.0f);
  if (!gt) return;
  // textured worlds: the texture coordinates of the vertices in edge order
  // (the ground: world x, y scaled; a cube or box face: the unit square over
  // the face's tangent axes of the body frame) and whether to sample
  float uv[3][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}};
  float textured = 0.0f;
  if (body < 0) {
    textured = 1.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int v = vid[ord[k]];
      uv[k][0] = T->ground_v[v][0] * T->ground_uv_scale;
      uv[k][1] = T->ground_v[v][1] * T->ground_uv_scale;
    }
  } else if (B.type[body]) {
    textured = 1.0f;
    const float* fn = T->cube_n[face];
    const int a = fabsf(fn[0]) > 0.5f ? 0 : (fabsf(fn[1]) > 0.5f ? 1 : 2);
    const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float* tv = T->cube_v[vid[ord[k]] - B.vb[body]];
      uv[k][0] = (tv[t0] + 1.0f) * 0.5f;
      uv[k][1] = (tv[t1] + 1.0f) * 0.5f;
    }
  }
  float4* q = gt + 2 * r;
  q[0] = make_float4(uv[0][0], uv[0][1], uv[1][0], uv[1][1]);
  q[1] = make_float4(uv[2][0], uv[2][1], textured, 0.0f);
}

// CLIP: cut triangles crossing the near plane (else they are culled whole,
// and none of that code is compiled in).  FUSED: the fused kernel's setup,
// which keeps the image's records and bins in LDS when they fit (16-byte
// records: the vertex-cache indices of the corners in edge order, the
// primitive, 1/area, RGB8 and the flags), else writes them to the raster
// scratch as the setup kernel does; the tile table stays in LDS either way.
template <bool CLIP, bool FUSED>
__device__ void setup_image(unsigned char* lds, const SetupLayout& Lo, const WorldDev& W,
                            const RasterLaunch& L, int cam_id) {
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int lane = tid & 63;
  const CamDev cam = uniform_copy(W.cams + cam_id);
  const EnvDev ed = uniform_copy(W.envs + cam.env);
  const int n = ed.n_bodies;
  const int ntris = ed.n_tris;
  const int64_t cap = W.cap_bodies;
  const float* st = W.state[L.parity];
  // the env's primitive and vertex maps (16-byte aligned and padded), read
  // once into LDS: every phase below looks them up per triangle or vertex
  const uint8_t* gpmap = (const uint8_t*)(lds + Lo.pmap);
  const uint8_t* gvmap = (const uint8_t*)(lds + Lo.vmap);
  const int Wd = cam.w, Ht = cam.h;
  const int tsh = L.tile_shift, TS = 1 << tsh;  // tile edge in pixels
  const int ntx = (Wd + TS - 1) >> tsh;
  const int ntiles = tiles_of(Wd, Ht, tsh);
  // the image's scratch as the host laid it out (a tile table with room
  // for the smallest tiles)
  unsigned char* rs = W.rscratch + cam.rs_off + (int64_t)L.parity * cam.rs_total;  // one scratch per state buffer
  int32_t* hdr = (int32_t*)rs;
  int32_t* ttab = (int32_t*)(rs + 64);
  int4* grec = (int4*)(rs + cam.rs_recs);
  uint16_t* bins = (uint16_t*)(rs + cam.rs_bins);
  const int rs_bin_cap = kBinsPerTri * (cam.n_tris + kClipRecs);
  const int bin_cap = (L.bin_limit > 0 && L.bin_limit < rs_bin_cap) ? L.bin_limit : rs_bin_cap;

  Templates* T = (Templates*)(lds + Lo.tpl);
  BodyLDS B;
  float* bf = (float*)(lds + Lo.body);
  B.p = bf;
  B.R = bf + 3 * Lo.nmax;
  B.e = (float4*)(bf + 12 * Lo.nmax);
  B.type = (int32_t*)(bf + 16 * Lo.nmax);
  B.vb = (int32_t*)(bf + 17 * Lo.nmax);
  B.pb = (int32_t*)(bf + 18 * Lo.nmax);
  B.alb = (int32_t*)(bf + 19 * Lo.nmax);
  int4* V = (int4*)(lds + Lo.verts);
  uint16_t* vis = (uint16_t*)(lds + Lo.vis);
  int32_t* cvis = (int32_t*)(lds + Lo.cvis);  // 10 words per piece
  int32_t* tcount = (int32_t*)(lds + Lo.tiles);
  int32_t* toff = tcount + Lo.tw;
  int32_t* tfill = toff + Lo.tw + 1;
  int32_t* misc = (int32_t*)(lds + Lo.misc);

  // 1. templates, maps and bodies
  {
    const int4* src = (const int4*)W.tpl;
    int4* dst = (int4*)T;
    for (int i = tid; i < kTplBytes / 16; i += nthr) dst[i] = src[i];
    const int4* ps = (const int4*)(W.prim_body + ed.prim_map);
    int4* pd = (int4*)(lds + Lo.pmap);
    for (int i = tid; i < (ntris + 15) / 16; i += nthr) pd[i] = ps[i];
    const int4* vs = (const int4*)(W.vert_body + ed.vert_map);
    int4* vd = (int4*)(lds + Lo.vmap);
    for (int i = tid; i < (ed.n_verts + 15) / 16; i += nthr) vd[i] = vs[i];
  }
  for (int b = tid; b < n; b += nthr) {
    const int g = ed.body_off + b;
    B.p[b] = st[PX * cap + g];
    B.p[Lo.nmax + b] = st[PY * cap + g];
    B.p[2 * Lo.nmax + b] = st[PZ * cap + g];
    quat_rot(st[QW * cap + g], st[QX * cap + g], st[QY * cap + g], st[QZ * cap + g], B.R + b, Lo.nmax);
    const float* bx = W.box + 6 * (int64_t)g;
    B.e[b] = make_float4(bx[0], bx[1], bx[2], 0.0f);
    B.type[b] = W.type[g];
    B.vb[b] = W.vert_base[g];
    B.pb[b] = W.prim_base[g];
    B.alb[b] = W.albedo[g];
  }
  const bool tiled = ntiles <= Lo.tw;
  if (tid == 0) misc[2] = misc[3] = misc[5] = 0;
  if (tiled)
    for (int t = tid; t < ntiles; t += nthr) tcount[t] = 0;
  __syncthreads();

  // 2. vertices
  const float* vp = cam.vp;
  const float fW = (float)Wd, fH = (float)Ht;
  for (int vi = tid; vi < ed.n_verts; vi += nthr) {
    int32_t X, Y;
    float z;
    snap_clip(vertex_clip(T, B, Lo.nmax, gvmap, vi, vp), fW, fH, T, true, &X, &Y, &z);
    if (CLIP && X == kBehind) misc[5] = 1;  // some vertex of the image is behind the near plane
    V[vi] = make_int4(X, Y, __float_as_int(z), 0);
  }
  __syncthreads();

  // 3. visibility.  A triangle survives if every vertex is in front of the
  // near plane and inside the guard band, its integer area is > 0 (front
  // facing, not degenerate) and its box holds a pixel centre.  Survivors are
  // compacted into vis (a wave ballot and one atomic per wave), so that the
  // costlier steps below run on full waves.  A triangle that crosses the
  // near plane (and has no vertex in front outside the guard band) is cut
  // along it: its surviving pieces go to cvis, and become the records after
  // the whole triangles.
  // (two versions of the pass: images with no vertex behind the near plane,
  // nearly all of them, run the one without the cut)
  const auto visibility = [&](auto cut_tag) {
  for (int base = 0; base < ntris; base += nthr) {
    const int pr = base + tid;
    bool keep = false;
    if (pr < ntris) {
      int body, vid[3];
      prim_vertices(T, B, gpmap[pr], pr, &body, vid);
      const Tri t = load_tri(V, vid);
      int x0, x1, y0, y1;
      keep = t.ok && tri_area(t.X, t.Y) > 0 && tri_pixels(t.X, t.Y, Wd, Ht, &x0, &x1, &y0, &y1);
      if constexpr (decltype(cut_tag)::value) {
      int behind = 0, outside = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        behind += t.X[k] == kBehind;
        outside += t.X[k] == kInvalid;
      }
      if (behind > 0 && behind < 3 && outside == 0) {
        float4 c[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) c[k] = vertex_clip(T, B, Lo.nmax, gvmap, vid[k], vp);
        for (int sp = 0; sp < 2; ++sp) {
          Tri q;
          q.ok = false;
          if (near_piece(c, sp, fW, fH, T, &q) && q.ok && tri_area(q.X, q.Y) > 0 &&
              tri_pixels(q.X, q.Y, Wd, Ht, &x0, &x1, &y0, &y1)) {
            // the piece itself is kept, so that the record and binning
            // passes need not cut again
            const int slot = atomicAdd(&misc[3], 1);
            if (slot < kClipRecs) {
              int32_t* o = cvis + 10 * slot;
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                o[k] = q.X[k];
                o[3 + k] = q.Y[k];
                o[6 + k] = __float_as_int(q.z[k]);
              }
              o[9] = pr;
            }
          }
        }
      }
      }
    }
    const uint64_t m = __ballot(keep);
    int wbase = 0;
    if (lane == 0 && m) wbase = atomicAdd(&misc[2], __popcll(m));
    wbase = __builtin_amdgcn_readfirstlane(wbase);
    const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
    if (keep) vis[wbase + below] = (uint16_t)pr;
  }
  };
  if constexpr (CLIP) {
    if (misc[5]) visibility(std::true_type{});
    else visibility(std::false_type{});
  } else {
    visibility(std::false_type{});
  }
  __syncthreads();
  const int nwhole = misc[2];
  const int npieces = min(misc[3], kClipRecs);
  const int nrec = nwhole + npieces;
  if (tid == 0 && misc[3] > kClipRecs) atomicOr(&W.env_flags[cam.env], kFlagClipOverflow);
  // record r: whole triangle vis[r], or piece cvis[r - nwhole]; vid its
  // face's vertices in face order
  const auto record_tri = [&](int r, int* pr, int* body, int vid[3], Tri* t) {
    if (!CLIP || r < nwhole) {
      *pr = vis[r];
      prim_vertices(T, B, gpmap[*pr], *pr, body, vid);
      *t = load_tri(V, vid);
      return;
    }
    const int32_t* o = cvis + 10 * (r - nwhole);
    *pr = o[9];
    prim_vertices(T, B, gpmap[*pr], *pr, body, vid);
    t->ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      t->X[k] = o[k];
      t->Y[k] = o[3 + k];
      t->z[k] = __int_as_float(o[6 + k]);
    }
  };

  // 4. tile counts, one surviving triangle per lane.  A triangle whose box
  // spans more than kWide tiles is counted by its whole wave, one tile per
  // lane, so that one lane never walks a long tile list alone.
  if (tiled) {
    for (int base = 0; base < nrec; base += nthr) {
      const int r = base + tid;
      int tx0 = 0, ty0 = 0, nx = 0, ny = 0;
      if (r < nrec) {
        int pr, body, vid[3];
        Tri t;
        record_tri(r, &pr, &body, vid, &t);
        int x0, x1, y0, y1;
        tri_pixels(t.X, t.Y, Wd, Ht, &x0, &x1, &y0, &y1);
        tx0 = x0 >> tsh;
        ty0 = y0 >> tsh;
        nx = (x1 >> tsh) - tx0 + 1;
        ny = (y1 >> tsh) - ty0 + 1;
      }
      const bool wide = nx * ny > kWide;
      if (!wide)
        for (int qy = 0; qy < ny; ++qy)
          for (int qx = 0; qx < nx; ++qx) atomicAdd(&tcount[(ty0 + qy) * ntx + tx0 + qx], 1);
      uint64_t m = __ballot(wide);
      while (m) {
        const int j = __ffsll((unsigned long long)m) - 1;
        m &= m - 1ull;
        const int jx0 = __shfl(tx0, j, 64), jy0 = __shfl(ty0, j, 64);
        const int jnx = __shfl(nx, j, 64), jn = jnx * __shfl(ny, j, 64);
        for (int q = lane; q < jn; q += 64) {
          const int qy = q / jnx;
          atomicAdd(&tcount[(jy0 + qy) * ntx + jx0 + (q - qy * jnx)], 1);
        }
      }
    }
  }
  __syncthreads();
  // bin entries hold 15-bit record ids
  bool binned = tiled && nrec <= 32768;
  int total = 0;
  if (binned) total = tile_scan(tcount, toff, ntiles, misc + 8);
  bool local = false;
  if constexpr (FUSED) local = nrec <= Lo.rec_cap && (!binned || total <= Lo.bin_cap);
  if (binned && total > (local ? Lo.bin_cap : bin_cap)) binned = false;
  int4* lrec = (int4*)(lds + Lo.lrec);
  uint16_t* bout = local ? (uint16_t*)(lds + Lo.lbin) : bins;
  if (binned) {
    for (int t = tid; t < ntiles; t += nthr) tfill[t] = 0;
    __syncthreads();
  }

  // 5. a setup record (with the face colour) per surviving triangle, and its
  // record id scattered into the bins, from the vertex cache.  Record slots
  // differ from run to run; they appear in no key, which orders by depth,
  // then primitive.
  for (int base = 0; base < nrec; base += nthr) {
    const int r = base + tid;
    int x0 = 0, x1 = 0, y0 = 0, y1 = 0, nx = 0, ny = 0;
    Tri t{};
    if (r < nrec) {
      int pr, body, vid[3];
      record_tri(r, &pr, &body, vid, &t);
      tri_pixels(t.X, t.Y, Wd, Ht, &x0, &x1, &y0, &y1);
      const int64_t A = tri_area(t.X, t.Y);
      const int face = body < 0 ? pr : pr - B.pb[body];
      uint32_t rgb;
      if (L.smooth) {
        // the key carries the record instead of a colour; the pixel's colour
        // comes from the record's attributes in the tile kernel
        rgb = (uint32_t)r;
        store_attr((float4*)(rs + cam.rs_attr), W.texture ? (float4*)(rs + cam.rs_tuv) : nullptr, r, T, B,
                   Lo.nmax, gvmap, body, face, vid, vp);
      } else {
        rgb = face_color(T, B, Lo.nmax, body, face);
      }
      const float invA = 1.0f / (float)(double)A;
      if (FUSED && local)
        lrec[r] = make_int4((int32_t)((uint32_t)vid[0] | ((uint32_t)vid[2] << 16)),
                            (int32_t)((uint32_t)vid[1] | ((uint32_t)pr << 16)), __float_as_int(invA),
                            (int32_t)(rgb | ((uint32_t)rec_flags(t) << 24)));
      else
        store_rec(grec, r, t, pr, invA, rgb, x0, x1, y0, y1);
      nx = (x1 >> tsh) - (x0 >> tsh) + 1;
      ny = (y1 >> tsh) - (y0 >> tsh) + 1;
    }
    if (!binned) continue;
    const bool wide = nx * ny > kWide;
    if (!wide)
      for (int qy = 0; qy < ny; ++qy)
        for (int qx = 0; qx < nx; ++qx)
          bin_tile(t, r, (x0 >> tsh) + qx, (y0 >> tsh) + qy, x0, x1, y0, y1, nx * ny > 1, Wd, Ht, ntx, TS,
                   toff, tfill, bout);
    // a wide triangle is binned by the whole wave, one tile per lane; its
    // snapped vertices and pixel box come from its lane's registers
    uint64_t m = __ballot(wide);
    while (m) {
      const int j = __ffsll((unsigned long long)m) - 1;
      m &= m - 1ull;
      const int jr = __builtin_amdgcn_readlane(r, j);
      Tri J{};
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        J.X[v] = __builtin_amdgcn_readlane(t.X[v], j);
        J.Y[v] = __builtin_amdgcn_readlane(t.Y[v], j);
      }
      const int jx0 = __builtin_amdgcn_readlane(x0, j), jx1 = __builtin_amdgcn_readlane(x1, j);
      const int jy0 = __builtin_amdgcn_readlane(y0, j), jy1 = __builtin_amdgcn_readlane(y1, j);
      const int jnx = (jx1 >> tsh) - (jx0 >> tsh) + 1;
      const int jn = jnx * ((jy1 >> tsh) - (jy0 >> tsh) + 1);
      for (int q = lane; q < jn; q += 64) {
        const int qy = q / jnx;
        bin_tile(J, jr, (jx0 >> tsh) + (q - qy * jnx), (jy0 >> tsh) + qy, jx0, jx1, jy0, jy1, true, Wd, Ht,
                 ntx, TS, toff, tfill, bout);
      }
    }
  }
  if constexpr (FUSED) {
    // the tile pass reads the table from LDS after the caller's barrier
    if (tid == 0) misc[6] = (local ? 1 : 0) | (binned ? 2 : 0);
    return;
  }
  __syncthreads();
  if (binned)
    for (int t = tid; t < ntiles; t += nthr) {
      ttab[2 * t] = toff[t];
      ttab[2 * t + 1] = tfill[t];
    }
  if (tid == 0) {
    hdr[0] = nrec;
    hdr[1] = binned ? 1 : 0;
  }
}

// Held to 80 VGPRs (six waves per SIMD; left alone the compiler takes 134,
// mostly fp64 edge terms of the tile classification hoisted out of the
// binning loops, and is capped at 128).  The spills this costs (about 50
// VGPRs to scratch) slow the kernel by about 1.5% when it runs alone, but
// its waves then fit beside the tile and physics waves that hold the rest of
// a SIMD's register file when the render overlaps the next step: about 4%
// more steps per second co-scheduled, at 1024 envs of 32 bodies and at 4096
// envs of 64 (7 and 8 waves per SIMD, 72 and 64 VGPRs, spill more and lose).
template <bool CLIP>
__global__ void __attribute__((amdgpu_waves_per_eu(6))) raster_setup_kernel(WorldDev W, RasterLaunch L) {
  extern __shared__ __align__(16) unsigned char lds[];
  // At the end of a step this kernel shares CUs with the render's tile
  // waves; a higher issue priority keeps its chains of dependent steps moving.
  switch (L.prio) {
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    case 3: __builtin_amdgcn_s_setprio(3); break;
    default: break;
  }
  const SetupLayout Lo = setup_layout(L.max_bodies, L.max_verts, L.max_tiles, L.max_tris, CLIP);
  if (L.persistent == 0) {
    if ((int)blockIdx.x >= L.n_work) return;
    setup_image<CLIP, false>(lds, Lo, W, L, uniform_ld(L.work + blockIdx.x));
    return;
  }
  int32_t* slot = (int32_t*)(lds + Lo.misc) + 4;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(L.queue, 1);
    __syncthreads();
    const int wi = *slot;
    if (wi >= L.n_work) return;
    setup_image<CLIP, false>(lds, Lo, W, L, uniform_ld(L.work + wi));
  }
}

// ---------------------------------------------------------------------------
// tile kernel
// ---------------------------------------------------------------------------

// A tile of TS x TS pixels per wave: each lane owns a block of BW x BH
// pixels, BW adjacent in a row (4, or 1 for 8x8 tiles), BH rows (4 for
// 32x32 tiles, else 1).
template <int TS>
struct TileGeo {
  static constexpr int BW = TS >= 16 ? 4 : 1;
  static constexpr int LPR = TS / BW;              // lanes per row of blocks
  static constexpr int BH = TS * TS / (64 * BW);
  static constexpr int NPX = BW * BH;              // pixels per lane
  static_assert(LPR * (64 / LPR) == 64 && (64 / LPR) * BH == TS, "tile shape");
};

template <int TS>
struct TileWaveLDS {
  uint64_t zb[TS * TS];  // z-buffer of the small-triangle fragments
  int32_t own[64];       // fragment owner marks
};

// Key of a primitive's fragment below its depth: primitive << 24 | RGB8.
// Primitives number at most 65535 per env, so no key equals the empty ~0.
__device__ __forceinline__ uint64_t prim_key(int prim, uint32_t rgb) {
  return ((uint64_t)(uint32_t)prim << 24) | (uint64_t)(rgb & 0xFFFFFFu);
}

// Quantised depth key of a covered pixel from its three edge values; the
// 24-bit depth decides, then the primitive (unique in an image), so the
// colour carried in the low bits never does.
__device__ __forceinline__ uint64_t depth_key(float e0, float e1, float e2, float z0, float z1, float z2,
                                              float invA, uint64_t key) {
  const float zz = ((e0 * z0 + e1 * z1) + e2 * z2) * invA;
  // the interpolated depth is finite, so the median equals the clamp to [0, 1]
  const uint32_t D = (uint32_t)rintf(__builtin_amdgcn_fmed3f(zz, 0.0f, 1.0f) * 16777215.0f);
  return ((uint64_t)D << 40) | key;
}

// Smooth shading of pixel (px, py) won by record r: the attribute record's
// vertex normals interpolated with weights E_k / w_k at the pixel centre
// (exact edge values), normalized, and Lambert-shaded; RGB8 packed.
__device__ __forceinline__ uint32_t smooth_color(const int4* grec, const float4* gattr, const float4* gtuv,
                                                 const uint8_t* tex, const Templates* T, int r, int px, int py) {
  const int4 a = grec[4 * r], b = grec[4 * r + 1];
  const float4 g0 = gattr[4 * r], g1 = gattr[4 * r + 1], g2 = gattr[4 * r + 2], g3 = gattr[4 * r + 3];
  const int32_t X[3] = {a.x, a.z, b.x}, Y[3] = {a.y, a.w, b.y};
  const float iw[3] = {g2.y, g2.z, g2.w};
  const int Px = 256 * px + 128, Py = 256 * py + 128;
  float u[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int a0 = (e + 1) % 3, b0 = (e + 2) % 3;
    const int32_t dx = X[b0] - X[a0], dy = Y[b0] - Y[a0];
    const double E = fma(-(double)dy, (double)(Px - X[a0]), (double)dx * (double)(Py - Y[a0]));
    u[e] = (float)E * iw[e];
  }
  const float mx = (u[0] * g0.x + u[1] * g0.w) + u[2] * g1.z;
  const float my = (u[0] * g0.y + u[1] * g1.x) + u[2] * g1.w;
  const float mz = (u[0] * g0.z + u[1] * g1.y) + u[2] * g2.x;
  const float l2 = (mx * mx + my * my) + mz * mz;
  float nx = 0.0f, ny = 0.0f, nz = 0.0f;
  if (l2 > 0.0f) {
    const float l = sqrtf(l2);
    nx = mx / l;
    ny = my / l;
    nz = mz / l;
  }
  const float lam = fmaxf(0.0f, (nx * T->light[0] + ny * T->light[1]) + nz * T->light[2]);
  float al[3] = {g3.x, g3.y, g3.z};
  if (gtuv) {
    // textured worlds: the albedo times the texel (nearest, repeating) at
    // the texture coordinates interpolated with the weights above
    const float4 t0 = gtuv[2 * r], t1 = gtuv[2 * r + 1];
    if (t1.z != 0.0f) {
      const float s = (u[0] + u[1]) + u[2];
      float U = 0.0f, V = 0.0f;
      if (s > 0.0f) {
        U = ((u[0] * t0.x + u[1] * t0.z) + u[2] * t1.x) / s;
        V = ((u[0] * t0.y + u[1] * t0.w) + u[2] * t1.y) / s;
      }
      float fu = U - floorf(U), fv = V - floorf(V);
      if (!(fu >= 0.0f)) fu = 0.0f;
      if (!(fv >= 0.0f)) fv = 0.0f;
      const int i = min((int)(fu * (float)T->tex_w), T->tex_w - 1);
      const int j = min((int)(fv * (float)T->tex_h), T->tex_h - 1);
      const uint8_t* p = tex + 3 * ((int64_t)j * T->tex_w + i);
#pragma unroll
      for (int c = 0; c < 3; ++c) al[c] = al[c] * ((float)p[c] / 255.0f);
    }
  }
  uint32_t rgb = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float col = al[c] * (0.2f + 0.8f * lam);
    rgb |= (uint32_t)fminf(255.0f, rintf(col * 255.0f)) << (8 * c);
  }
  return rgb;
}

// Where the tile pass finds an image's records and bins.  GlobalRecs: the
// 64-byte records and the bins in the raster scratch.  LdsRecs (fused
// kernel): 16-byte records and bins in LDS, the corners read from the
// vertex cache and the pixel box recomputed, so that fetch() returns the
// four quads of the 64-byte record.
struct GlobalRecs {
  const int4* rec;
  const uint16_t* bins;
  __device__ __forceinline__ int bin(int k) const { return bins[k]; }
  __device__ __forceinline__ void fetch(int r, int4& a, int4& b, int4& c, int4& d) const {
    a = rec[4 * r];
    b = rec[4 * r + 1];
    c = rec[4 * r + 2];
    d = rec[4 * r + 3];
  }
};

struct LdsRecs {
  const int4* rec;
  const int4* V;
  const uint16_t* bins;
  int w, h;
  __device__ __forceinline__ int bin(int k) const { return bins[k]; }
  __device__ __forceinline__ void fetch(int r, int4& a, int4& b, int4& c, int4& d) const {
    const int4 q = rec[r];
    const int4 v0 = V[q.x & 0xFFFF], v1 = V[(uint32_t)q.x >> 16], v2 = V[q.y & 0xFFFF];
    a = make_int4(v0.x, v0.y, v1.x, v1.y);
    b = make_int4(v2.x, v2.y, (int32_t)((uint32_t)q.y >> 16), v0.z);
    c = make_int4(v1.z, v2.z, q.z, q.w & 0xFFFFFF);
    const int32_t X[3] = {v0.x, v1.x, v2.x}, Y[3] = {v0.y, v1.y, v2.y};
    int x0, x1, y0, y1;
    tri_pixels(X, Y, w, h, &x0, &x1, &y0, &y1);
    d = make_int4(x0 | (x1 << 16), y0 | (y1 << 16), (int32_t)((uint32_t)q.w >> 24), 0);
  }
};

// One tile of an image: records k0 .. k1 of the tile's bin (binned), or
// every record k0 .. k1 of the image.  rs: the image's raster scratch (smooth
// shading reads its attribute records there).
template <bool DBG, bool SMOOTH, int TS, class Src>
__device__ __forceinline__ void raster_tile(const WorldDev& W, const CamDev& cam, const Src& src, bool binned,
                                            int k0, int k1, int tx, int ty, TileWaveLDS<TS>& S, int32_t* cov,
                                            const unsigned char* rs) {
  using G = TileGeo<TS>;
  constexpr int BW = G::BW, BH = G::BH, NPX = G::NPX;
  const int lane = threadIdx.x & 63;
  const int Wd = cam.w, Ht = cam.h;
  const int tx0 = tx * TS, ty0 = ty * TS;
  const int tx1 = min(tx0 + TS - 1, Wd - 1), ty1 = min(ty0 + TS - 1, Ht - 1);
  // this lane's pixels: (px0 + i, py0 + j) for i < BW, j < BH, z-buffer
  // entries zrow (j) + i
  const int bx = lane % G::LPR, by = lane / G::LPR;
  const int px0 = tx0 + BW * bx, py0 = ty0 + BH * by;
  const auto zidx = [&](int i, int j) { return (BH * by + j) * TS + BW * bx + i; };
  uint64_t* zb = S.zb;
  // The LDS z-buffer is only for small triangles' fragments: it is cleared
  // before the first fragment window and read back only if it was.  A tile
  // whose bin is empty (a third of them in a settled scene) or holds large
  // triangles alone, such as the open ground, never touches it.
  bool zused = false;
  if (DBG) {
#pragma unroll
    for (int j = 0; j < BH; ++j)
#pragma unroll
      for (int i = 0; i < BW; ++i) cov[zidx(i, j)] = 0;
  }
  uint64_t kreg[NPX];
  int creg[NPX];
#pragma unroll
  for (int q = 0; q < NPX; ++q) {
    kreg[q] = ~0ull;
    creg[q] = 0;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");

  for (int kb = k0; kb < k1; kb += 64) {
    // One record per lane, kept in registers: a small triangle's fragments
    // fetch their owner's values with cross-lane reads (ds_bpermute, which
    // needs no LDS of its own), a large triangle's record is read uniformly
    // with readlane.  So the tile keeps little LDS, and the step's waves
    // find room beside it on the CU.
    const int k = kb + lane;
    int full = 0, area = 0, fx0 = 0, fy0 = 0, bw = 1;
    bool big = false;
    int4 ra = make_int4(0, 0, 0, 0), rb = ra, rc = ra;
    int E0[3] = {0, 0, 0}, sr[3] = {0, 0, 0}, sc[3] = {0, 0, 0}, thr = 0;
    if (k < k1) {
      int rec = k;
      if (binned) {
        const int e = src.bin(k);
        rec = e & 0x7FFF;
        full = e >> 15;
      }
      int4 rd;
      src.fetch(rec, ra, rb, rc, rd);
      const int32_t X[3] = {ra.x, ra.z, rb.x}, Y[3] = {ra.y, ra.w, rb.y};
      // the triangle's pixel box (never empty) clipped to the tile
      fx0 = max(rd.x & 0xFFFF, tx0);
      fy0 = max(rd.y & 0xFFFF, ty0);
      bw = min(rd.x >> 16, tx1) - fx0 + 1;
      const int bh = min(rd.y >> 16, ty1) - fy0 + 1;
      area = ((bw > 0) & (bh > 0)) ? bw * bh : 0;
      if (bw < 1) bw = 1;
      const bool narrow = (rd.z & 8) != 0;
      big = area > kSmallMax || (area > 0 && !narrow);
      if (!big && area > 0) {
        // edge values at the centre of pixel (fx0, fy0), steps per row and
        // column; (E > 0 or E == 0 on a top-left edge) == (E >= thr bit)
        const int Px = 256 * fx0 + 128, Py = 256 * fy0 + 128;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int a0 = (e + 1) % 3, b0 = (e + 2) % 3;
          const int32_t dx = X[b0] - X[a0], dy = Y[b0] - Y[a0];
          E0[e] = __mul24(dx, Py - Y[a0]) - __mul24(dy, Px - X[a0]);
          sr[e] = 256 * dx;
          sc[e] = -256 * dy;
        }
        thr = rd.z & 7;
      }
    }
    // small triangles: fragments packed over lanes.  Fragment f belongs to
    // the lane j with off_j <= f < off_j + a_j; per window of 64 fragments
    // each owner marks where its range starts and a max-scan spreads it.
    const int a = big ? 0 : area;
    const int incl = wave_incl_add(a);
    const int F = __builtin_amdgcn_readlane(incl, 63);
    const int off = incl - a;
    const int mxy = fx0 | (fy0 << 16), mob = off | (bw << 16);
    int carry = 0;  // owner + 1 of the fragment before the window
    if (F > 0 && !zused) {
#pragma unroll
      for (int j = 0; j < BH; ++j)
#pragma unroll
        for (int i = 0; i < BW; ++i) zb[zidx(i, j)] = ~0ull;
      zused = true;
    }
    for (int f0 = 0; f0 < F; f0 += 64) {
      S.own[lane] = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      if (a > 0 && off >= f0 && off < f0 + 64) S.own[off - f0] = lane + 1;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      int o = S.own[lane];
      if (lane == 0) o = max(o, carry);
      o = wave_incl_max(o);
      carry = __builtin_amdgcn_readlane(o, 63);
      const int f = f0 + lane;
      // the owner's values (lanes past F read lane 63's, unused)
      const int j = (o - 1) & 63;
      const int jxy = __shfl(mxy, j, 64), job = __shfl(mob, j, 64);
      const int rr = f - (job & 0xFFFF), jbw = job >> 16;
      // rr / jbw exactly: rr < 64 and jbw <= 32 (a box in a tile of at
      // most 32 pixels) keep the quotient's fraction at least 1/64 away
      // from an integer, far above the reciprocal's rounding
      const int qy = (int)(((float)rr + 0.5f) * __builtin_amdgcn_rcpf((float)jbw));
      const int qx = rr - qy * jbw;
      const int e0 = __shfl(E0[0], j, 64) + __mul24(__shfl(sr[0], j, 64), qy) + __mul24(__shfl(sc[0], j, 64), qx);
      const int e1 = __shfl(E0[1], j, 64) + __mul24(__shfl(sr[1], j, 64), qy) + __mul24(__shfl(sc[1], j, 64), qx);
      const int e2 = __shfl(E0[2], j, 64) + __mul24(__shfl(sr[2], j, 64), qy) + __mul24(__shfl(sc[2], j, 64), qx);
      const int jthr = __shfl(thr, j, 64);
      const float z0 = __int_as_float(__shfl(rb.w, j, 64)), z1 = __int_as_float(__shfl(rc.x, j, 64));
      const float z2 = __int_as_float(__shfl(rc.y, j, 64)), invA = __int_as_float(__shfl(rc.z, j, 64));
      const int jprim = __shfl(rb.z, j, 64), jrgb = __shfl(rc.w, j, 64);
      if ((f < F) & (e0 >= (jthr & 1)) & (e1 >= ((jthr >> 1) & 1)) & (e2 >= (jthr >> 2))) {
        const uint64_t kk = depth_key((float)e0, (float)e1, (float)e2, z0, z1, z2, invA,
                                      prim_key(jprim, (uint32_t)jrgb));
        const int p = (jxy >> 16) + qy - ty0;  // row in the tile
        const int pp = p * TS + (jxy & 0xFFFF) + qx - tx0;
        atomicMin((unsigned long long*)&zb[pp], (unsigned long long)kk);
        if (DBG) atomicAdd(&cov[pp], 1);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    }
    // large triangles: every lane on its four pixels, the record uniform
    uint64_t m = __ballot(big);
    while (m) {
      const int j = __ffsll((unsigned long long)m) - 1;
      m &= m - 1ull;
      const bool jfull = __builtin_amdgcn_readlane(full, j) != 0;  // uniform
      const int32_t X[3] = {__builtin_amdgcn_readlane(ra.x, j), __builtin_amdgcn_readlane(ra.z, j),
                            __builtin_amdgcn_readlane(rb.x, j)};
      const int32_t Y[3] = {__builtin_amdgcn_readlane(ra.y, j), __builtin_amdgcn_readlane(ra.w, j),
                            __builtin_amdgcn_readlane(rb.y, j)};
      const float z0 = __int_as_float(__builtin_amdgcn_readlane(rb.w, j));
      const float z1 = __int_as_float(__builtin_amdgcn_readlane(rc.x, j));
      const float z2 = __int_as_float(__builtin_amdgcn_readlane(rc.y, j));
      const float invA = __int_as_float(__builtin_amdgcn_readlane(rc.z, j));
      const uint64_t key = prim_key(__builtin_amdgcn_readlane(rb.z, j), (uint32_t)__builtin_amdgcn_readlane(rc.w, j));
      // edge values at the lane's first pixel, one pixel right, one row
      // down: exact integers in fp64, so stepping is exact
      double Er[3], step[3], down[3], thr[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const int a0 = (e + 1) % 3, b0 = (e + 2) % 3;
        const int32_t dx = X[b0] - X[a0], dy = Y[b0] - Y[a0];
        Er[e] = fma(-(double)dy, (double)(256 * px0 + 128 - X[a0]), (double)dx * (double)(256 * py0 + 128 - Y[a0]));
        step[e] = -(double)dy * 256.0;
        down[e] = (double)dx * 256.0;
        thr[e] = top_left(dx, dy) ? 0.0 : 1.0;
      }
#pragma unroll
      for (int j = 0; j < BH; ++j) {
        double E[3] = {Er[0], Er[1], Er[2]};
        if (jfull) {
          // every pixel of the tile is covered
#pragma unroll
          for (int i = 0; i < BW; ++i) {
            const int q = j * BW + i;
            const uint64_t kk = depth_key((float)E[0], (float)E[1], (float)E[2], z0, z1, z2, invA, key);
            kreg[q] = kk < kreg[q] ? kk : kreg[q];
            if (DBG) creg[q] += 1;
#pragma unroll
            for (int e = 0; e < 3; ++e) E[e] += step[e];
          }
        } else {
#pragma unroll
          for (int i = 0; i < BW; ++i) {
            const int q = j * BW + i;
            const bool in = (E[0] >= thr[0]) & (E[1] >= thr[1]) & (E[2] >= thr[2]);
            const uint64_t kk = depth_key((float)E[0], (float)E[1], (float)E[2], z0, z1, z2, invA, key);
            kreg[q] = (in & (kk < kreg[q])) ? kk : kreg[q];
            if (DBG) creg[q] += in ? 1 : 0;
#pragma unroll
            for (int e = 0; e < 3; ++e) E[e] += step[e];
          }
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) Er[e] += down[e];
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // resolve: the fragment z-buffer against the registers, then the winners'
  // colours and the stores, one row of the lane's block at a time
#pragma unroll
  for (int j = 0; j < BH; ++j) {
    const int py = py0 + j;
    uint32_t D[BW], rgb[BW];
    int32_t win[BW];
#pragma unroll
    for (int i = 0; i < BW; ++i) {
      const int q = j * BW + i;
      const uint64_t zk = zused ? zb[zidx(i, j)] : ~0ull;
      const uint64_t key = zk < kreg[q] ? zk : kreg[q];
      const bool hit = key != ~0ull;
      D[i] = hit ? (uint32_t)(key >> 40) : 0xFFFFFFFFu;
      rgb[i] = hit ? (uint32_t)key & 0xFFFFFFu : 0u;  // the winner's colour travels in its key
      win[i] = hit ? (int32_t)((key >> 24) & 0xFFFFu) : -1;
      if constexpr (SMOOTH) {
        // the key's low bits name the winning record
        if (hit)
          rgb[i] = smooth_color(src.rec, (const float4*)(rs + cam.rs_attr),
                                W.texture ? (const float4*)(rs + cam.rs_tuv) : nullptr, W.texture, W.tpl,
                                (int)rgb[i], px0 + i, py);
      }
    }
    if (py > ty1) continue;
    const int64_t pix = cam.pix_off + (int64_t)py * Wd + px0;
    if constexpr (BW == 4) {
      if (px0 + 3 <= tx1 && (pix & 3) == 0) {
        *(uint4*)(W.depth + pix) = make_uint4(D[0], D[1], D[2], D[3]);
        uint32_t* c = (uint32_t*)(W.rgb + 3 * pix);  // 3 pix is a multiple of 12
        c[0] = rgb[0] | (rgb[1] << 24);
        c[1] = (rgb[1] >> 8) | (rgb[2] << 16);
        c[2] = (rgb[2] >> 16) | (rgb[3] << 8);
      } else {
#pragma unroll
        for (int i = 0; i < BW; ++i) {
          if (px0 + i > tx1) continue;
          W.depth[pix + i] = D[i];
          W.rgb[3 * (pix + i)] = (uint8_t)(rgb[i] & 0xFF);
          W.rgb[3 * (pix + i) + 1] = (uint8_t)((rgb[i] >> 8) & 0xFF);
          W.rgb[3 * (pix + i) + 2] = (uint8_t)((rgb[i] >> 16) & 0xFF);
        }
      }
    } else {
      if (px0 <= tx1) {
        W.depth[pix] = D[0];
        W.rgb[3 * pix] = (uint8_t)(rgb[0] & 0xFF);
        W.rgb[3 * pix + 1] = (uint8_t)((rgb[0] >> 8) & 0xFF);
        W.rgb[3 * pix + 2] = (uint8_t)((rgb[0] >> 16) & 0xFF);
      }
    }
    if (DBG) {
#pragma unroll
      for (int i = 0; i < BW; ++i) {
        if (px0 + i > tx1) continue;
        W.winners[pix + i] = win[i];
        W.coverage[pix + i] = cov[zidx(i, j)] + creg[j * BW + i];
      }
    }
  }
}

// TW tiles of a row per workgroup, one per wave
template <bool DBG, bool SMOOTH, int TS, int TW>
__global__ void __launch_bounds__(64 * TW) raster_tile_kernel(WorldDev W, RasterLaunch L) {
  __shared__ TileWaveLDS<TS> S[TW];
  __shared__ int32_t C[DBG ? TW : 1][DBG ? TS * TS : 1];
  // beside the step's kernels, a higher issue priority keeps the render
  // (the longer phase) from stretching
  switch (L.prio) {
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    case 3: __builtin_amdgcn_s_setprio(3); break;
    default: break;
  }
  // The tile's bookkeeping is uniform and takes three rounds of loads (the
  // job, the camera, then the image's header and the tile's bin range
  // together) before the first bin entry is read.
  const int2 job = uniform_ld(L.tiles + blockIdx.x);
  if (job.x < 0) return;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (wave > (job.x >> kJobWavesShift)) return;  // past the row's last tile; no workgroup barrier follows
  const CamDev* cp = W.cams + (job.x & kJobCamMask);
  CamDev cam;  // the fields the tile pass reads
  cam.w = uniform_ld(&cp->w);
  cam.h = uniform_ld(&cp->h);
  cam.pix_off = uniform_ld(&cp->pix_off);
  cam.rs_off = uniform_ld(&cp->rs_off);
  cam.rs_recs = uniform_ld(&cp->rs_recs);
  cam.rs_bins = uniform_ld(&cp->rs_bins);
  cam.rs_total = uniform_ld(&cp->rs_total);
  cam.rs_attr = uniform_ld(&cp->rs_attr);
  cam.rs_tuv = uniform_ld(&cp->rs_tuv);
  const int ntx = (cam.w + TS - 1) / TS;
  const int tx = (job.y & 0xFFFF) + wave, ty = job.y >> 16;
  const unsigned char* rs = W.rscratch + cam.rs_off + (int64_t)L.parity * cam.rs_total;
  // the tile table has room for the image's tiles at the smallest tile
  // edge, so its entry is read before the header says the image is binned
  const int2 hdr = uniform_ld((const int2*)rs);
  const int2 te = uniform_ld((const int2*)(rs + 64) + (ty * ntx + tx));
  const bool binned = hdr.y != 0;
  const int k0 = binned ? te.x : 0, k1 = binned ? te.x + te.y : hdr.x;
  const GlobalRecs src{(const int4*)(rs + cam.rs_recs), (const uint16_t*)(rs + cam.rs_bins)};
  raster_tile<DBG, SMOOTH, TS>(W, cam, src, binned, k0, k1, tx, ty, S[wave], DBG ? C[wave] : nullptr, rs);
}

// The tiles wave, wave + nw, ... of an image whose setup is done, from
// records and bins in src.
template <bool DBG, int TS, class Src>
__device__ __forceinline__ void fused_tiles(const WorldDev& W, const CamDev& cam, const Src& src, bool binned,
                                            int nrec, const int32_t* toff, const int32_t* tfill, int wave,
                                            int nw, TileWaveLDS<TS>* S, int32_t* C, const unsigned char* rs) {
  const int ntx = (cam.w + TS - 1) / TS, ntiles = ntx * ((cam.h + TS - 1) / TS);
  for (int t = wave; t < ntiles; t += nw) {
    const int k0 = binned ? toff[t] : 0, k1 = binned ? k0 + tfill[t] : nrec;
    raster_tile<DBG, false, TS>(W, cam, src, binned, k0, k1, t % ntx, t / ntx, S[wave],
                                DBG ? C + wave * TS * TS : nullptr, rs);
  }
}

// Setup and tiles of one image per workgroup (flat shading, no near-plane
// clipping): the setup pass as above, then every wave rasterizes tiles
// wave, wave + nw, ... of the image from the records and bins in LDS, its
// z-buffer in the setup-only region.  Records and bins that do not fit go
// through the raster scratch instead, with the same results.
template <bool DBG, int TS>
__global__ void __launch_bounds__(1024) raster_fused_kernel(WorldDev W, RasterLaunch L) {
  extern __shared__ __align__(16) unsigned char lds[];
  const SetupLayout Lo = setup_layout(L.max_bodies, L.max_verts, L.max_tiles, L.max_tris, false, L.lds_zone0,
                                      L.lrec_cap, L.lbin_cap);
  const int nw = (int)(blockDim.x >> 6);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  TileWaveLDS<TS>* S = (TileWaveLDS<TS>*)lds;
  int32_t* C = (int32_t*)(lds + nw * sizeof(TileWaveLDS<TS>));  // debug coverage, TS * TS per wave
  int32_t* misc = (int32_t*)(lds + Lo.misc);
  const int32_t* toff = (const int32_t*)(lds + Lo.tiles) + Lo.tw;
  const int32_t* tfill = toff + Lo.tw + 1;
  int wi = (int)blockIdx.x;
  for (;;) {
    if (L.persistent > 0) {
      __syncthreads();
      if (threadIdx.x == 0) misc[4] = atomicAdd(L.queue, 1);
      __syncthreads();
      wi = misc[4];
    }
    if (wi >= L.n_work) return;
    const int cam_id = uniform_ld(L.work + wi);
    setup_image<false, true>(lds, Lo, W, L, cam_id);
    __syncthreads();
    const CamDev cam = uniform_copy(W.cams + cam_id);
    const int nrec = misc[2], mode = misc[6];
    const bool binned = (mode & 2) != 0;
    const unsigned char* rs = W.rscratch + cam.rs_off + (int64_t)L.parity * cam.rs_total;
    if (mode & 1) {
      const LdsRecs src{(const int4*)(lds + Lo.lrec), (const int4*)(lds + Lo.verts),
                        (const uint16_t*)(lds + Lo.lbin), cam.w, cam.h};
      fused_tiles<DBG, TS>(W, cam, src, binned, nrec, toff, tfill, wave, nw, S, C, rs);
    } else {
      const GlobalRecs src{(const int4*)(rs + cam.rs_recs), (const uint16_t*)(rs + cam.rs_bins)};
      fused_tiles<DBG, TS>(W, cam, src, binned, nrec, toff, tfill, wave, nw, S, C, rs);
    }
    if (L.persistent == 0) return;
    __syncthreads();  // the next image's setup reuses the LDS
  }
}

}  // namespace

size_t raster_lds_bytes(const RasterLaunch& l) {
  return (size_t)setup_layout(l.max_bodies, l.max_verts, l.max_tiles, l.max_tris, l.near_clip != 0).total;
}

// The fused kernel's LDS for workgroups of l.threads: the tile pass's
// z-buffers (and debug coverage) over the setup-only region, and as many
// compact records as LDS allows up to half the primitives plus 64 (a convex
// closed mesh seen from outside shows at most about half its faces), with
// four bin entries each (at most max_recs records if max_recs > 0); 0 if
// fewer than min(64, max_recs) fit.
size_t raster_fused_plan(RasterLaunch* l, bool debug, int max_recs) {
  const int ts = 1 << l->tile_shift;
  const int nw = l->threads / 64;
  const size_t wave_lds = ts == 8 ? sizeof(TileWaveLDS<8>) : ts == 32 ? sizeof(TileWaveLDS<32>)
                                                                       : sizeof(TileWaveLDS<16>);
  l->lds_zone0 = (int32_t)(nw * (wave_lds + (debug ? 4 * ts * ts : 0)));
  int cap = (l->max_tris + 1) / 2 + 64;
  if (max_recs > 0 && max_recs < cap) cap = max_recs;
  for (const int least = cap < 64 ? cap : 64; cap >= least; cap /= 2) {
    const SetupLayout Lo = setup_layout(l->max_bodies, l->max_verts, l->max_tiles, l->max_tris, false,
                                        l->lds_zone0, cap, 4 * cap);
    if (Lo.total <= kFusedLdsMax) {
      l->lrec_cap = cap;
      l->lbin_cap = 4 * cap;
      return (size_t)Lo.total;
    }
  }
  return 0;
}

hipError_t raster_fused_configure(size_t lds_bytes) {
  const void* k[] = {(const void*)raster_fused_kernel<false, 8>, (const void*)raster_fused_kernel<false, 16>,
                     (const void*)raster_fused_kernel<false, 32>, (const void*)raster_fused_kernel<true, 8>,
                     (const void*)raster_fused_kernel<true, 16>, (const void*)raster_fused_kernel<true, 32>};
  for (const void* f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool DBG>
static const void* fused_fn(int tile_shift) {
  if (tile_shift == 3) return (const void*)raster_fused_kernel<DBG, 8>;
  if (tile_shift == 5) return (const void*)raster_fused_kernel<DBG, 32>;
  return (const void*)raster_fused_kernel<DBG, 16>;
}

template <bool DBG>
static void launch_fused(const WorldDev& w, const RasterLaunch& l, int grid, size_t lds, hipStream_t s,
                         LaunchEvents* ev) {
  const dim3 g(grid), b(l.threads);
  if (l.tile_shift == 3) timed_launch(ev, true, true, raster_fused_kernel<DBG, 8>, g, b, (uint32_t)lds, s, w, l);
  else if (l.tile_shift == 5) timed_launch(ev, true, true, raster_fused_kernel<DBG, 32>, g, b, (uint32_t)lds, s, w, l);
  else timed_launch(ev, true, true, raster_fused_kernel<DBG, 16>, g, b, (uint32_t)lds, s, w, l);
}

hipError_t launch_raster_fused(const WorldDev& w, const RasterLaunch& l0, size_t lds, hipStream_t s,
                               LaunchEvents* ev) {
  if (l0.n_work <= 0) return hipSuccess;
  RasterLaunch l = l0;
  int grid = l.n_work;
  if (l.persistent != 0) {
    hipError_t e = persistent_grid(l.persistent, l.n_work, w.winners ? fused_fn<true>(l.tile_shift)
                                                                     : fused_fn<false>(l.tile_shift),
                                   l.threads, lds, &grid);
    if (e != hipSuccess) return e;
    l.persistent = grid;  // the kernel only tells 0 from the rest
    e = launch_reset_queue(l.queue, s);
    if (e != hipSuccess) return e;
  }
  if (w.winners) launch_fused<true>(w, l, grid, lds, s, ev);
  else launch_fused<false>(w, l, grid, lds, s, ev);
  return hipGetLastError();
}

hipError_t raster_configure(size_t lds_bytes) {
  const hipError_t e = hipFuncSetAttribute((const void*)raster_setup_kernel<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)raster_setup_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds_bytes);
}

hipError_t launch_raster_setup(const WorldDev& w, const RasterLaunch& l0, hipStream_t s, LaunchEvents* ev) {
  if (l0.n_work <= 0) return hipSuccess;
  RasterLaunch l = l0;
  const size_t lds = raster_lds_bytes(l);
  int grid = l.n_work;
  if (l.persistent != 0) {
    hipError_t e = persistent_grid(l.persistent, l.n_work,
                                   l.near_clip ? (const void*)raster_setup_kernel<true>
                                               : (const void*)raster_setup_kernel<false>,
                                   l.threads, lds, &grid);
    if (e != hipSuccess) return e;
    l.persistent = grid;  // the kernel only tells 0 from the rest
    e = launch_reset_queue(l.queue, s);
    if (e != hipSuccess) return e;
  }
  if (l.near_clip)
    timed_launch(ev, true, true, raster_setup_kernel<true>, dim3(grid), dim3(l.threads), (uint32_t)lds, s, w, l);
  else
    timed_launch(ev, true, true, raster_setup_kernel<false>, dim3(grid), dim3(l.threads), (uint32_t)lds, s, w, l);
  return hipGetLastError();
}

template <int TS, int TW>
static void launch_tiles(const WorldDev& w, const RasterLaunch& l, hipStream_t s, LaunchEvents* ev) {
  const dim3 g(l.n_tile_groups), b(64 * TW);
  if (l.smooth) {
    if (w.winners) timed_launch(ev, true, true, raster_tile_kernel<true, true, TS, TW>, g, b, 0, s, w, l);
    else timed_launch(ev, true, true, raster_tile_kernel<false, true, TS, TW>, g, b, 0, s, w, l);
  } else {
    if (w.winners) timed_launch(ev, true, true, raster_tile_kernel<true, false, TS, TW>, g, b, 0, s, w, l);
    else timed_launch(ev, true, true, raster_tile_kernel<false, false, TS, TW>, g, b, 0, s, w, l);
  }
}

template <int TS>
static void launch_tiles(const WorldDev& w, const RasterLaunch& l, hipStream_t s, LaunchEvents* ev) {
  if (l.tile_waves == 1) launch_tiles<TS, 1>(w, l, s, ev);
  else if (l.tile_waves == 2) launch_tiles<TS, 2>(w, l, s, ev);
  else launch_tiles<TS, 4>(w, l, s, ev);
}

hipError_t launch_raster_tiles(const WorldDev& w, const RasterLaunch& l, hipStream_t s, LaunchEvents* ev) {
  if (l.n_tile_groups <= 0) return hipSuccess;
  if (l.tile_shift == 3) launch_tiles<8>(w, l, s, ev);
  else if (l.tile_shift == 5) launch_tiles<32>(w, l, s, ev);
  else launch_tiles<16>(w, l, s, ev);
  return hipGetLastError();
}

}  // namespace vuda
