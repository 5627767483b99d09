// Rigid-body physics step for gfx950: one workgroup per env, one lane per body.
//
// One launch advances every listed env by one step of `substeps` substeps,
// reading state buffer `parity` and writing buffer 1 - parity once; the
// substeps run out of LDS and registers.  Per substep:
//   1. publish p, v, omega and R(q) of every body to LDS;
//   2. broadphase on a uniform grid hashed into 2^ceil(log2 2N) buckets
//      (Teschner et al. 2003 XOR-prime hash).  A bucket is a bitset of
//      bodies; each body ORs the buckets of its cell and the 13 cells of the
//      half shell, tests the distance of every body found and records the
//      pair (i < j) in a per-row bitset;
//   3. candidate rows are compacted into a pair list sorted by (i, j) with a
//      workgroup prefix scan of the row popcounts;
//   4. narrowphase: a pair with a sphere (one contact point at most) on one
//      lane; a cube-cube pair's 16 vertex-in-box tests on 16 lanes, then its
//      point terms summed in point order, one component per lane; likewise
//      the 8 corners of a cube near the ground.  A pair in contact gets a
//      slot holding its summed force and both bodies' torques;
//   5. each body gathers its pairs in sorted order (pairs (i, b) for i < b,
//      then (b, j), then the ground), so every sum is formed in a fixed
//      order independent of scheduling;
//   6. semi-implicit Euler.
// No floating-point atomics are used; results are bit-reproducible.
#include <map>
#include <mutex>
#include <tuple>

#include "vuda_internal.h"

#pragma clang fp contract(off)

namespace vuda {
namespace {

struct f3 {
  float x, y, z;
};
__device__ __forceinline__ f3 mk(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ f3 add(f3 a, f3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ f3 sub(f3 a, f3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ f3 mul(f3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ f3 neg(f3 a) { return mk(-a.x, -a.y, -a.z); }
__device__ __forceinline__ float dot(f3 a, f3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

struct M3 {
  float m[9];
};
__device__ __forceinline__ f3 rot(const M3& R, f3 v) {
  return mk((R.m[0] * v.x + R.m[1] * v.y) + R.m[2] * v.z,
            (R.m[3] * v.x + R.m[4] * v.y) + R.m[5] * v.z,
            (R.m[6] * v.x + R.m[7] * v.y) + R.m[8] * v.z);
}
__device__ __forceinline__ f3 rotT(const M3& R, f3 v) {
  return mk((R.m[0] * v.x + R.m[3] * v.y) + R.m[6] * v.z,
            (R.m[1] * v.x + R.m[4] * v.y) + R.m[7] * v.z,
            (R.m[2] * v.x + R.m[5] * v.y) + R.m[8] * v.z);
}
__device__ __forceinline__ M3 quat_to_rot(float w, float x, float y, float z) {
  const float xx = x * x, yy = y * y, zz = z * z;
  const float xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  M3 R;
  R.m[0] = 1.0f - 2.0f * (yy + zz);
  R.m[1] = 2.0f * (xy - wz);
  R.m[2] = 2.0f * (xz + wy);
  R.m[3] = 2.0f * (xy + wz);
  R.m[4] = 1.0f - 2.0f * (xx + zz);
  R.m[5] = 2.0f * (yz - wx);
  R.m[6] = 2.0f * (xz - wy);
  R.m[7] = 2.0f * (yz + wx);
  R.m[8] = 1.0f - 2.0f * (xx + yy);
  return R;
}

// LDS image of one env of up to N bodies (N = 32, 64 or 128 lanes): NW =
// 64-bit words per body bitset row = waves per env.
template <int N_>
struct PhysLDS {
  static constexpr int N = N_;
  static constexpr int NW = N_ > 64 ? N_ / 64 : 1;
  static constexpr int CAPC = 4 * N;  // candidate pairs
  static_assert(CAPC <= 1024 && N <= 2048, "cube-cube queue packing");
  static constexpr int CAPK = 2 * N;  // pairs in contact
  float4 pr[N];  // position and bounding radius (the substep-start position of every phase)
  float v[3][N];
  float w[3][N];
  float R[9][N];
  float size[N];
  float4 ext[N];   // half-extents along the body axes, 0 ((a, a, a) for a cube)
  float inert[3][N];  // principal moments of a box
  float rb[N];
  int32_t type[N];
  // arrays of disjoint phases of a substep share their storage: the grid
  // buckets (broadphase), the sorted candidate pairs (compaction and the
  // narrowphase of pairs with a sphere) and the per-lane point terms of the
  // box-pair and ground groups; a barrier separates each from the next
  union alignas(16) {
    uint64_t bucket[2 * N][NW];
    uint32_t cand[CAPC];    // candidate pairs i | j << 16, sorted
    float stage[9][N];      // one contact point's terms per lane, before the ordered sum
  };
  uint64_t rowCand[N][NW];
  uint64_t rowC[N][NW];
  uint64_t colC[N][NW];
  int32_t cstart[N];      // candidate-list start of each row
  int32_t gflag[N];       // body touches the ground
  uint16_t kslot[CAPC];   // slot of each candidate in contact
  uint32_t ccl[CAPC];     // candidates whose bodies are both cubes: k | i << 10 | j << 21
  int32_t gcl[N];         // cubes closer to the ground than their bounding radius
  float kres[9][CAPK];    // SF xyz, Ti xyz, Tj xyz of each pair in contact
  float estage[9][N / 16];        // terms of the edge-edge point of each 16-lane group
  float gres[6][N];       // ground force and torque of each body
  int32_t scan[NW + 1];
  float red[NW];
  int32_t work;
  int32_t kcnt, ncc, ngc;
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Exclusive prefix sum over the workgroup (thread order); *total gets the sum.
// Inclusive wave64 prefix sum with DPP row shifts and row broadcasts (VALU
// only); lanes reading outside their row take 0.
__device__ __forceinline__ int wave_incl_add(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

// Inclusive prefix sum within each 32-lane half of the wave (row shifts and
// the broadcast of row 0 into row 1, row 2 into row 3).
__device__ __forceinline__ int half_incl_add(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  return x;
}

// Exclusive prefix sum over the N lanes of one env (thread order); *total
// gets the env's sum.
template <int N>
__device__ __forceinline__ int block_excl_scan(int v, int32_t* tmp, int* total) {
  constexpr int NW = N > 64 ? N / 64 : 1;
  const int lane = lane_id();
  if (N == 32) {
    const int x = half_incl_add(v);
    *total = __shfl(x, (lane & 32) + 31, 64);
    return x - v;
  }
  const int x = wave_incl_add(v);
  if (NW == 1) {
    *total = __builtin_amdgcn_readlane(x, 63);
    return x - v;
  }
  const int wv = threadIdx.x >> 6;
  if (lane == 63) tmp[wv] = x;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    int t = tmp[k];
    if (k < wv) base += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

template <int N>
__device__ __forceinline__ float block_max(float v, float* tmp) {
  constexpr int NW = N > 64 ? N / 64 : 1;
  float x = v;
#pragma unroll
  for (int d = (N < 64 ? N / 2 : 32); d >= 1; d >>= 1) x = fmaxf(x, __shfl_xor(x, d, 64));
  if (NW == 1) return x;
  if (lane_id() == 0) tmp[threadIdx.x >> 6] = x;
  __syncthreads();
  float m = tmp[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) m = fmaxf(m, tmp[k]);
  __syncthreads();
  return m;
}

__device__ __forceinline__ uint32_t grid_hash(int cx, int cy, int cz, uint32_t mask) {
  return ((uint32_t)cx * 73856093u ^ (uint32_t)cy * 19349663u ^ (uint32_t)cz * 83492791u) & mask;
}

struct Point {
  f3 n;
  float delta;
  f3 xc;
};

template <int N>
__device__ __forceinline__ f3 ldsP(const PhysLDS<N>& s, int b) {
  const float4 q = s.pr[b];
  return mk(q.x, q.y, q.z);
}
template <int N>
__device__ __forceinline__ f3 ldsV(const PhysLDS<N>& s, int b) {
  return mk(s.v[0][b], s.v[1][b], s.v[2][b]);
}
template <int N>
__device__ __forceinline__ f3 ldsW(const PhysLDS<N>& s, int b) {
  return mk(s.w[0][b], s.w[1][b], s.w[2][b]);
}
template <int N>
__device__ __forceinline__ M3 ldsR(const PhysLDS<N>& s, int b) {
  M3 R;
#pragma unroll
  for (int k = 0; k < 9; ++k) R.m[k] = s.R[k][b];
  return R;
}

// Sum of one pair's contact forces, accumulated in point order.
struct PairAcc {
  f3 SF, Ti, Tj;
  int npts;
};

// Force of one contact point on the pair's first body and the torques it
// exerts on both bodies; a_first: body A (pushed along +n) is the pair's
// first body.
struct PointTerms {
  f3 Fi, ti, tj;
};
// FR: friction on (a separate instantiation, so that the frictionless
// kernel keeps its registers and needs no stack)
template <bool FR>
__device__ __forceinline__ PointTerms point_terms(const Point& pt, bool a_first, f3 pi, f3 vi, f3 wi,
                                                  f3 pj, f3 vj, f3 wj, bool ground,
                                                  const PhysConsts& pc) {
  const f3 pa = a_first ? pi : pj, va = a_first ? vi : vj, wa = a_first ? wi : wj;
  const f3 pb = a_first ? pj : pi, vb = a_first ? vj : vi, wb = a_first ? wj : wi;
  const f3 velA = add(va, cross(wa, sub(pt.xc, pa)));
  f3 vrel;
  if (ground) {
    vrel = velA;
  } else {
    const f3 velB = add(vb, cross(wb, sub(pt.xc, pb)));
    vrel = sub(velA, velB);
  }
  const float vn = dot(vrel, pt.n);
  float f = pc.k * pt.delta - pc.c * vn;
  if (f < 0.0f) f = 0.0f;
  f3 F = mul(pt.n, f);
  if constexpr (FR) {
    // regularized Coulomb friction against the tangential slip v_t
    const f3 vt = sub(vrel, mul(pt.n, vn));
    const float st = sqrtf(dot(vt, vt));
    const float ft = (pc.mu * f) / (st > pc.v_eps ? st : pc.v_eps);
    F = sub(F, mul(vt, ft));
  }
  PointTerms r;
  r.Fi = a_first ? F : neg(F);
  r.ti = cross(sub(pt.xc, pi), r.Fi);
  r.tj = ground ? mk(0.0f, 0.0f, 0.0f) : cross(sub(pt.xc, pj), neg(r.Fi));
  return r;
}

// Add the force of one contact point to its pair's sums.
template <bool FR>
__device__ __forceinline__ void add_point(PairAcc& acc, const Point& pt, bool a_first, f3 pi,
                                          f3 vi, f3 wi, f3 pj, f3 vj, f3 wj, bool ground,
                                          const PhysConsts& pc) {
  const PointTerms t = point_terms<FR>(pt, a_first, pi, vi, wi, pj, vj, wj, ground, pc);
  acc.SF = add(acc.SF, t.Fi);
  acc.Ti = add(acc.Ti, t.ti);
  if (!ground) acc.Tj = add(acc.Tj, t.tj);
  acc.npts += 1;
}

template <int N>
__device__ __forceinline__ f3 ldsE(const PhysLDS<N>& s, int b) {
  const float4 e = s.ext[b];
  return mk(e.x, e.y, e.z);
}

// Corner k of a box of half-extents e (sign + on axis t iff bit t of k is
// set): p + R w with w = (+-e.x, +-e.y, +-e.z).
__device__ __forceinline__ f3 corner_vertex(f3 p, const M3& R, f3 e, int k) {
  return add(p, rot(R, mk((k & 1) ? e.x : -e.x, (k & 2) ? e.y : -e.y, (k & 4) ? e.z : -e.z)));
}

// argmin over axes of (e_axis - |u_axis|), lowest axis on ties
__device__ __forceinline__ int min_axis(f3 u, f3 e, float* depth) {
  const float d0 = e.x - fabsf(u.x), d1 = e.y - fabsf(u.y), d2 = e.z - fabsf(u.z);
  int m = 0;
  float dm = d0;
  if (d1 < dm) { m = 1; dm = d1; }
  if (d2 < dm) { m = 2; dm = d2; }
  *depth = dm;
  return m;
}

__device__ __forceinline__ f3 axis_unit(int m, float sgn) {
  return mk(m == 0 ? sgn : 0.0f, m == 1 ? sgn : 0.0f, m == 2 ? sgn : 0.0f);
}

__device__ __forceinline__ float pick(f3 u, int m) { return m == 0 ? u.x : (m == 1 ? u.y : u.z); }

// Sphere (centre c, radius r) against box (p, R, half-extents a); normal
// from the box to the sphere.  Returns true on contact.
__device__ __forceinline__ bool sphere_cube(f3 c, float r, f3 p, const M3& R, f3 a, Point* pt) {
  const f3 u = rotT(R, sub(c, p));
  const f3 e = mk(fminf(fmaxf(u.x, -a.x), a.x), fminf(fmaxf(u.y, -a.y), a.y), fminf(fmaxf(u.z, -a.z), a.z));
  const f3 rv = sub(u, e);
  const float L2 = dot(rv, rv);
  if (!(L2 < r * r)) return false;
  f3 nl;
  float delta;
  if (L2 > 0.0f) {
    const float L = sqrtf(L2);
    nl = mk(rv.x / L, rv.y / L, rv.z / L);
    delta = r - L;
  } else {
    float dm;
    const int m = min_axis(u, a, &dm);
    nl = axis_unit(m, pick(u, m) >= 0.0f ? 1.0f : -1.0f);
    delta = r + dm;
  }
  pt->n = rot(R, nl);
  pt->delta = delta;
  pt->xc = add(p, rot(R, e));
  return true;
}

// Narrowphase + force sum of body pair (i, j), i < j, one of them a sphere.
template <int N, bool FR>
__device__ __noinline__ PairAcc pair_forces(const PhysLDS<N>& s, int i, int j,
                                            const PhysConsts& pc) {
  PairAcc acc;
  acc.SF = mk(0.0f, 0.0f, 0.0f);
  acc.Ti = acc.SF;
  acc.Tj = acc.SF;
  acc.npts = 0;
  const f3 pi = ldsP(s, i), pj = ldsP(s, j);
  const f3 vi = ldsV(s, i), vj = ldsV(s, j);
  const f3 wi = ldsW(s, i), wj = ldsW(s, j);
  const int ti = s.type[i], tj = s.type[j];
  const float si = s.size[i], sj = s.size[j];
  Point pt;
  if (ti == 0 && tj == 0) {
    const f3 d = sub(pi, pj);
    const float d2 = dot(d, d);
    const float sr = si + sj;
    if (d2 < sr * sr) {
      const float L = sqrtf(d2);
      pt.n = L > 0.0f ? mk(d.x / L, d.y / L, d.z / L) : mk(0.0f, 0.0f, 1.0f);
      pt.delta = sr - L;
      pt.xc = add(pj, mul(pt.n, sj - 0.5f * pt.delta));
      add_point<FR>(acc, pt, true, pi, vi, wi, pj, vj, wj, false, pc);
    }
  } else if (ti == 0 || tj == 0) {
    // one path for both orders: the sphere is body i (pushed along +n, the
    // pair's first body) or body j
    const bool sfirst = ti == 0;
    const int cb = sfirst ? j : i;
    const M3 Rc = ldsR(s, cb);
    if (sphere_cube(sfirst ? pi : pj, sfirst ? si : sj, sfirst ? pj : pi, Rc, ldsE(s, cb), &pt))
      add_point<FR>(acc, pt, sfirst, pi, vi, wi, pj, vj, wj, false, pc);
  }
  return acc;
}

// Two boxes (centres pa, pb, rotations Ra, Rb, half-extents ea, eb) that
// are apart along one of their six face axes by more than a rounding margin.
// Then no vertex of either lies inside the other and the separating-axis
// test of edge-edge points finds them apart too, so the pair has no contact
// point.  Along the axis a_k of A (column k of Ra) the boxes reach
// ea_k + sum_l eb_l |a_k . b_l| from their centres, along b_l of B
// sum_k ea_k |a_k . b_l| + eb_l.  The margin, 1e-5 of the coordinate and
// extent magnitudes, is over ten times the float32 error of the corner and
// containment arithmetic, so a vertex the corner test would place inside
// is never skipped.
__device__ __forceinline__ bool face_separated(f3 pa, const M3& Ra, f3 ea, f3 pb, const M3& Rb, f3 eb) {
  const f3 d = sub(pa, pb);
  const f3 da = rotT(Ra, d), db = rotT(Rb, d);
  float C[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      C[k][l] = fabsf((Ra.m[k] * Rb.m[l] + Ra.m[3 + k] * Rb.m[3 + l]) + Ra.m[6 + k] * Rb.m[6 + l]);
  const float mag = ((fabsf(pa.x) + fabsf(pa.y)) + fabsf(pa.z)) + ((fabsf(pb.x) + fabsf(pb.y)) + fabsf(pb.z)) +
                    2.0f * (((ea.x + ea.y) + ea.z) + ((eb.x + eb.y) + eb.z));
  const float tol = 1.0e-5f * mag;
  const float eA[3] = {ea.x, ea.y, ea.z}, eB[3] = {eb.x, eb.y, eb.z};
  const float dA[3] = {da.x, da.y, da.z}, dB[3] = {db.x, db.y, db.z};
  bool sep = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float rb = (eB[0] * C[k][0] + eB[1] * C[k][1]) + eB[2] * C[k][2];
    sep |= fabsf(dA[k]) > (eA[k] + rb) + tol;
    const float ra = (eA[0] * C[0][k] + eA[1] * C[1][k]) + eA[2] * C[2][k];
    sep |= fabsf(dB[k]) > (ra + eB[k]) + tol;
  }
  return sep;
}

// Corner k of box A strictly inside box B: the contact point, pushed out of
// B along the normal of B's nearest face.
__device__ __forceinline__ bool corner_in_box(f3 pa, const M3& Ra, f3 aa, int k, f3 pb, const M3& Rb,
                                              f3 ab, Point* pt) {
  const f3 vtx = corner_vertex(pa, Ra, aa, k);
  const f3 u = rotT(Rb, sub(vtx, pb));
  if (!(fabsf(u.x) < ab.x && fabsf(u.y) < ab.y && fabsf(u.z) < ab.z)) return false;
  float dm;
  const int m = min_axis(u, ab, &dm);
  pt->n = rot(Rb, axis_unit(m, pick(u, m) >= 0.0f ? 1.0f : -1.0f));
  pt->delta = dm;
  pt->xc = vtx;
  return true;
}

// Axis k (0..2) of a rotation (row-major): its column k, selected without
// indexing the registers.
__device__ __forceinline__ f3 axis_of(const M3& R, int k) {
  return k == 0 ? mk(R.m[0], R.m[3], R.m[6]) : (k == 1 ? mk(R.m[1], R.m[4], R.m[7]) : mk(R.m[2], R.m[5], R.m[8]));
}

// Half-width of a box (rotation R, half-extents e) along direction L.
__device__ __forceinline__ float box_radius(const M3& R, f3 e, f3 L) {
  const f3 u = rotT(R, L);
  return (e.x * fabsf(u.x) + e.y * fabsf(u.y)) + e.z * fabsf(u.z);
}

// The step's candidate superset: pairs within their bounding radii plus
// kSupMargin (m) at substep 0; retested alone while no body has moved more
// than kSupMargin / 4 (kSupMove2 is its square).
constexpr float kSupMargin = 0.04f;
constexpr float kSupMove2 = 1.0e-4f;
constexpr float kEdgeParallel = 1.0e-6f;  // squared length below which a cross product is no axis
constexpr float kEdgeBias = 0.95f;        // an edge axis wins below this fraction of the least face overlap

// Edge-edge point of the box pair (i, j), i < j, by the separating-axis
// test, evaluated by the 16-lane group of the calling lane (every lane of
// the wave calls it; `live` is uniform over a group).  Lane r < 15 takes
// candidate axis r: the 3 axes of i, the 3 of j, then (axis a of i) x
// (axis b of j) at 6 + 3a + b.  The group reduces the least face overlap
// and the least edge overlap (lowest axis on ties); if no axis separates
// and the edge overlap is below kEdgeBias times the face one, lane 15
// stages the point's terms in estage.  Returns that decision, the same on
// every lane of the group.
template <int N, bool FR>
__device__ __forceinline__ bool edge_point(PhysLDS<N>& s, bool live, int r, int lane, int i, int j,
                                           const PhysConsts& pc) {
  const M3 Ri = ldsR(s, i), Rj = ldsR(s, j);
  const f3 ei = ldsE(s, i), ej = ldsE(s, j);
  const f3 pi = ldsP(s, i), pj = ldsP(s, j);
  const f3 d = sub(pi, pj);
  f3 L = mk(0.0f, 0.0f, 0.0f);
  bool valid = false;
  if (live && r < 15) {
    if (r < 3) {
      L = axis_of(Ri, r);
      valid = true;
    } else if (r < 6) {
      L = axis_of(Rj, r - 3);
      valid = true;
    } else {
      L = cross(axis_of(Ri, (r - 6) / 3), axis_of(Rj, (r - 6) % 3));
      const float l2 = dot(L, L);
      valid = l2 >= kEdgeParallel;
      if (valid) {
        const float l = sqrtf(l2);
        L = mk(L.x / l, L.y / l, L.z / l);
      }
    }
  }
  float o = INFINITY;
  if (valid) o = (box_radius(Ri, ei, L) + box_radius(Rj, ej, L)) - fabsf(dot(d, L));
  const int g0 = lane & 48;
  const bool sep = ((__ballot(valid && !(o > 0.0f)) >> g0) & 0xFFFFull) != 0ull;
  float fo = r < 6 ? o : INFINITY;
  float eo = r < 6 ? INFINITY : o;
  int ek = r;
#pragma unroll
  for (int m = 1; m < 16; m <<= 1) {
    const float fo2 = __shfl_xor(fo, m, 64);
    const float eo2 = __shfl_xor(eo, m, 64);
    const int ek2 = __shfl_xor(ek, m, 64);
    fo = fminf(fo, fo2);
    if (eo2 < eo || (eo2 == eo && ek2 < ek)) {
      eo = eo2;
      ek = ek2;
    }
  }
  const bool has = live && !sep && eo < kEdgeBias * fo;
  // the winning axis, as its lane computed it
  const int src = g0 + ek;
  const f3 eL = mk(__shfl(L.x, src, 64), __shfl(L.y, src, 64), __shfl(L.z, src, 64));
  if (has && r == 15) {
    const int a = (ek - 6) / 3, b = (ek - 6) % 3;
    const f3 n = dot(eL, d) < 0.0f ? neg(eL) : eL;  // from j to i
    // the edge of i along its axis a deepest toward j (along -n) and the
    // edge of j along its axis b deepest toward i (along +n): their centres
    const f3 ui = rotT(Ri, n), uj = rotT(Rj, n);
    const f3 wi = mk(a == 0 ? 0.0f : (ui.x > 0.0f ? -ei.x : ei.x), a == 1 ? 0.0f : (ui.y > 0.0f ? -ei.y : ei.y),
                     a == 2 ? 0.0f : (ui.z > 0.0f ? -ei.z : ei.z));
    const f3 wj = mk(b == 0 ? 0.0f : (uj.x > 0.0f ? ej.x : -ej.x), b == 1 ? 0.0f : (uj.y > 0.0f ? ej.y : -ej.y),
                     b == 2 ? 0.0f : (uj.z > 0.0f ? ej.z : -ej.z));
    const f3 ci = add(pi, rot(Ri, wi)), cj = add(pj, rot(Rj, wj));
    // closest points of the two edge lines, each clamped to its edge
    const f3 da = axis_of(Ri, a), db = axis_of(Rj, b);
    const f3 w = sub(ci, cj);
    const float bb = dot(da, db), dd = dot(da, w), ee = dot(db, w);
    const float den = 1.0f - bb * bb;
    float sa = (bb * ee - dd) / den, tb = (ee - bb * dd) / den;
    const float ha = pick(ei, a), hb = pick(ej, b);
    sa = fminf(fmaxf(sa, -ha), ha);
    tb = fminf(fmaxf(tb, -hb), hb);
    Point pt;
    pt.n = n;
    pt.delta = eo;
    pt.xc = mul(add(add(ci, mul(da, sa)), add(cj, mul(db, tb))), 0.5f);
    const PointTerms pq = point_terms<FR>(pt, true, pi, ldsV(s, i), ldsW(s, i), pj, ldsV(s, j), ldsW(s, j), false, pc);
    const int gi = ((int)threadIdx.x % N) >> 4;
    s.estage[0][gi] = pq.Fi.x; s.estage[1][gi] = pq.Fi.y; s.estage[2][gi] = pq.Fi.z;
    s.estage[3][gi] = pq.ti.x; s.estage[4][gi] = pq.ti.y; s.estage[5][gi] = pq.ti.z;
    s.estage[6][gi] = pq.tj.x; s.estage[7][gi] = pq.tj.y; s.estage[8][gi] = pq.tj.z;
  }
  return has;
}

// Lanes of this wave below the calling lane whose bit is set in m.
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Ordered sum, over the set bits l of the group mask gm (ascending), of
// stage[c][base + l] for l < G: the terms of one pair's contact points in
// point order.  The G values are loaded first, then added where selected.
template <int G, int N>
__device__ __forceinline__ float ordered_sum(const PhysLDS<N>& s, int c, int base, uint32_t gm) {
  float v[G];
  const float4* src = (const float4*)&s.stage[c][base];
#pragma unroll
  for (int l = 0; l < G / 4; ++l) {
    const float4 x = src[l];
    v[4 * l] = x.x; v[4 * l + 1] = x.y; v[4 * l + 2] = x.z; v[4 * l + 3] = x.w;
  }
  float acc = 0.0f;
#pragma unroll
  for (int l = 0; l < G; ++l)
    if ((gm >> l) & 1u) acc = acc + v[l];
  return acc;
}

__device__ __forceinline__ uint64_t below_mask(int b) {
  return b >= 64 ? ~0ull : ((1ull << b) - 1ull);
}

template <int NW>
__device__ __forceinline__ int popc_below(const uint64_t* row, int b) {
  int c = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) c += __popcll(row[k] & below_mask(b - 64 * k < 0 ? 0 : b - 64 * k));
  return c;
}

template <int N, bool FR, bool EE, bool SUP>
__device__ void step_env(PhysLDS<N>& s, const WorldDev& W, const PhysConsts& pc, int env,
                         int parity, int broadphase) {
  constexpr int NW = PhysLDS<N>::NW;
  // Lanes of this env: N consecutive threads.  At N = 32 two envs share a
  // wave, each in one half: their compactions count within the half, a
  // half's first lane does its atomics, and every loop holding a wave-wide
  // operation runs the larger of the two halves' trip counts.
  constexpr int LW = N < 64 ? N : 64;  // lanes of this env in one wave
  const int tid = (int)threadIdx.x % N;
  const int lane = lane_id();
  const int lbase = lane & ~(LW - 1);  // this env's first lane in the wave
  const auto half = [&](uint64_t m) -> uint64_t { return N < 64 ? ((m >> lbase) & 0xFFFFFFFFull) : m; };
  const auto below = [&](uint64_t m) -> int {
    return __popcll(half(m) & ((1ull << (lane - lbase)) - 1ull));
  };
  const auto wmax = [&](int x) -> int { return N < 64 ? max(x, __shfl_xor(x, 32, 64)) : x; };
  EnvDev ed{};
  if (env >= 0) ed = uniform_copy(W.envs + env);  // a scalar load where the env is the wave's
  const int n = ed.n_bodies;
  if (N >= 64 && n <= 0) return;  // a whole workgroup; a half-wave env of no bodies does nothing below
  const int b0 = ed.body_off;
  const bool own = tid < n;
  const int64_t cap = W.cap_bodies;
  const float* in = W.state[parity];
  float* out = W.state[parity ^ 1];
  const int gb = b0 + (own ? tid : 0);

  // owned body state in registers
  f3 p = mk(0, 0, 0), v = p, w = p;
  float qw = 1.0f, qx = 0.0f, qy = 0.0f, qz = 0.0f;
  float inv_m = 0.0f, inv_I = 0.0f, a = 0.0f, rbv = 0.0f, ex = 0.0f, ey = 0.0f, ez = 0.0f;
  int ty = 0;
  if (own) {
    p = mk(in[PX * cap + gb], in[PY * cap + gb], in[PZ * cap + gb]);
    v = mk(in[VX * cap + gb], in[VY * cap + gb], in[VZ * cap + gb]);
    qw = in[QW * cap + gb]; qx = in[QX * cap + gb]; qy = in[QY * cap + gb]; qz = in[QZ * cap + gb];
    w = mk(in[WX * cap + gb], in[WY * cap + gb], in[WZ * cap + gb]);
    inv_m = W.inv_m[gb];
    inv_I = W.inv_I[gb];
    a = W.size[gb];
    rbv = W.rbound[gb];
    ty = W.type[gb];
    s.size[tid] = a;
    ex = ey = ez = a;
    if (ty == 2) {
      const float* bx = W.box + 6 * (int64_t)gb;
      ex = bx[0];
      ey = bx[1];
      ez = bx[2];
      s.ext[tid] = make_float4(ex, ey, ez, 0.0f);
      s.inert[0][tid] = bx[3];
      s.inert[1][tid] = bx[4];
      s.inert[2][tid] = bx[5];
    } else {
      s.ext[tid] = make_float4(a, a, a, 0.0f);
    }
    s.rb[tid] = rbv;
    s.type[tid] = ty;
  }
  // the policy's force on this body, held over the substeps
  f3 fx = mk(0.0f, 0.0f, 0.0f);
  bool has_fx = false;
  if (W.actions && own && tid < W.act_dim / 3 && W.act_on[env]) {
    const float* fa = W.actions + (int64_t)env * W.act_dim + 3 * tid;
    fx = mk(fa[0], fa[1], fa[2]);
    has_fx = true;
  }
  // grid cell edge: a little above the largest bounding diameter
  const float rmax = block_max<N>(own ? rbv : 0.0f, s.red);
  const float inv_c = 1.0f / (2.0f * rmax * 1.000244140625f);
  int tbits = 1;
  while ((1 << tbits) < 2 * n) ++tbits;
  const int T = 1 << tbits;
  const uint32_t hmask = (uint32_t)(T - 1);
  const f3 gvec = mk(pc.g[0], pc.g[1], pc.g[2]);
  bool bad = false;
  // broadphase choice: 0 auto (grid above 64 bodies), 1 grid, 2 all-pairs
  const bool use_grid = broadphase == 1 || (broadphase == 0 && n > 64);
  // the step's candidate superset (all-pairs path): pairs found at substep 0
  // within their bounding radii plus kSupMargin, by the lane that found them
  const f3 p0 = p;
  uint64_t supM = 0ull;

  for (int sub_i = 0; sub_i < pc.substeps; ++sub_i) {
    // 1. publish substep-start state
    M3 R = quat_to_rot(qw, qx, qy, qz);
    if (own) {
      s.pr[tid] = make_float4(p.x, p.y, p.z, rbv);
      s.v[0][tid] = v.x; s.v[1][tid] = v.y; s.v[2][tid] = v.z;
      s.w[0][tid] = w.x; s.w[1][tid] = w.y; s.w[2][tid] = w.z;
#pragma unroll
      for (int k = 0; k < 9; ++k) s.R[k][tid] = R.m[k];
    }
    for (int k = tid; k < T; k += N)
#pragma unroll
      for (int q = 0; q < NW; ++q) s.bucket[k][q] = 0ull;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      s.rowCand[tid][q] = 0ull;
      s.rowC[tid][q] = 0ull;
      s.colC[tid][q] = 0ull;
    }
    if (tid == 0) {
      s.kcnt = 0;
      s.ncc = 0;
      s.ngc = 0;
    }
    // 2. broadphase.  The candidate set is exactly {(i, j): i < j,
    // |p_i - p_j|^2 <= (R_i + R_j)^2}; two ways produce it.  All-pairs: every
    // lane tests every body, reading it with one broadcast LDS load (no
    // divergence) -- the faster choice for one wave.  Grid: bodies hashed into
    // bitset buckets by cell, each lane ORs its own and the 13 half-shell
    // neighbour buckets and tests only the bodies found.  Cells far from the
    // origin fall back to all-pairs.
    int cx = 0, cy = 0, cz = 0, far_cell = 0;
    if (use_grid && own) {
      const float fx = floorf(p.x * inv_c), fy = floorf(p.y * inv_c), fz = floorf(p.z * inv_c);
      far_cell = !(fabsf(fx) < 1000.0f && fabsf(fy) < 1000.0f && fabsf(fz) < 1000.0f);
      cx = (int)fx; cy = (int)fy; cz = (int)fz;
    }
    // the barrier that publishes the substep state also ORs the far-cell
    // test over every wave of the env
    const bool grid = (__syncthreads_or(far_cell) == 0) && use_grid;
    if (!grid && N <= 64) {
      // Substeps after the first retest only the step's superset while every
      // body of the env is within a quarter of the margin of its step-start
      // position: a pair in contact range now was then within the sum of
      // its radii plus half the margin, and the other half covers rounding
      // (positions under 1000 m, where it is below 0.1 mm).  The retest is
      // the same expression, so the candidate set is the same bits.
      // Only where a lane has more than one batch of eight rotations: below
      // that the retest saves nothing.
      const int groups = n <= N / 2 ? 2 : 1;
      const int i = groups == 2 ? (tid & (N / 2 - 1)) : tid;
      const int g = groups == 2 ? tid / (N / 2) : 0;
      const int R = n / 2;
      const bool use_sup = SUP && (R + groups - 1) / groups > 8;
      bool retest = false;
      if constexpr (SUP) {
        bool risky = true;
        if (sub_i > 0 && use_sup) {
          risky = false;
          if (own) {
            const f3 dp = sub(p, p0);
            risky = dot(dp, dp) > kSupMove2 ||
                    !(fabsf(p.x) < 1000.0f && fabsf(p.y) < 1000.0f && fabsf(p.z) < 1000.0f);
          }
        }
        retest = half(__ballot(risky)) == 0;
      }
      // one wave: lane l tests body i against body (i + r) mod n for its
      // share of the rotations r = 1 .. n/2 (two groups of 32 lanes when
      // n <= 32).  Every unordered pair is one rotation away from one of its
      // bodies; at r = n/2 (n even) both see it and the lower one keeps it.
      // The test is symmetric in the two bodies, bit for bit.
      // Eight rotations per batch: their loads issue back to back.
      const bool build = sub_i == 0 && use_sup;
      if (i < n && retest) {
        // eight members of the superset per batch: their loads issue together
        const float4 me = s.pr[i];
        uint64_t m = supM;
        while (m) {
          float4 o[8];
          int jj[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            jj[u] = m ? __ffsll((unsigned long long)m) - 1 : -1;
            m &= m - 1ull;
            o[u] = s.pr[jj[u] < 0 ? i : jj[u]];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int j = jj[u];
            const f3 d = mk(me.x - o[u].x, me.y - o[u].y, me.z - o[u].z);
            const float rs = me.w + o[u].w;
            if ((j >= 0) & (dot(d, d) <= rs * rs)) {
              const int lo = i < j ? i : j, hi = i < j ? j : i;
              atomicOr((unsigned long long*)&s.rowCand[lo][0], 1ull << hi);
            }
          }
        }
      } else if (i < n) {
        const float4 me = s.pr[i];
        if (build) supM = 0ull;
        for (int r0 = 1 + g; r0 <= R; r0 += 8 * groups) {
          float4 o[8];
          int jj[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int r = r0 + u * groups;
            int j = i + r;
            if (j >= n) j -= n;
            jj[u] = r <= R ? j : i;
            o[u] = s.pr[jj[u]];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int r = r0 + u * groups, j = jj[u];
            const f3 d = mk(me.x - o[u].x, me.y - o[u].y, me.z - o[u].z);
            const float rs = me.w + o[u].w;
            const float d2 = dot(d, d);
            const bool mine = (r <= R) & !((2 * r == n) & (i > j));
            if (mine & (d2 <= rs * rs)) {
              const int lo = i < j ? i : j, hi = i < j ? j : i;
              atomicOr((unsigned long long*)&s.rowCand[lo][0], 1ull << hi);
            }
            if (build) {
              const float rm = rs + kSupMargin;
              if (mine & (d2 <= rm * rm)) supM |= 1ull << j;
            }
          }
        }
      }
    } else if (!grid) {
      if (own) {
        uint64_t row[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) row[q] = 0ull;
        const float4 me = s.pr[tid];
        // j is the same in every lane: s.pr[j] is one broadcast load
#pragma unroll 4
        for (int j = 0; j < n; ++j) {
          const float4 o = s.pr[j];
          const f3 d = mk(me.x - o.x, me.y - o.y, me.z - o.z);
          const float rs = me.w + o.w;
          if (j > tid && dot(d, d) <= rs * rs) {
#pragma unroll
            for (int q = 0; q < NW; ++q)
              if (q == (j >> 6)) row[q] |= 1ull << (j & 63);
          }
        }
#pragma unroll
        for (int q = 0; q < NW; ++q) s.rowCand[tid][q] = row[q];
      }
    } else {
      if (own) {
        const uint32_t h = grid_hash(cx, cy, cz, hmask);
        atomicOr((unsigned long long*)&s.bucket[h][tid >> 6], 1ull << (tid & 63));
      }
      __syncthreads();
      if (own) {
        uint64_t M[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) M[q] = 0ull;
        // own cell and the 13 neighbours of the half shell
#pragma unroll
        for (int o = 0; o < 14; ++o) {
          int dx, dy, dz;
          if (o == 0) { dx = 0; dy = 0; dz = 0; }
          else if (o <= 9) { dx = 1; dy = (o - 1) / 3 - 1; dz = (o - 1) % 3 - 1; }
          else if (o <= 12) { dx = 0; dy = 1; dz = o - 11; }
          else { dx = 0; dy = 0; dz = 1; }
          const uint32_t h = grid_hash(cx + dx, cy + dy, cz + dz, hmask);
#pragma unroll
          for (int q = 0; q < NW; ++q) M[q] |= s.bucket[h][q];
        }
#pragma unroll
        for (int q = 0; q < NW; ++q)
          if (q == (tid >> 6)) M[q] &= ~(1ull << (tid & 63));
#pragma unroll
        for (int q = 0; q < NW; ++q) {
          uint64_t m = M[q];
          while (m) {
            const int j = 64 * q + __ffsll((unsigned long long)m) - 1;
            m &= m - 1ull;
            const int lo = tid < j ? tid : j, hi = tid < j ? j : tid;
            const float4 a4 = s.pr[lo], b4 = s.pr[hi];
            const f3 d = mk(a4.x - b4.x, a4.y - b4.y, a4.z - b4.z);
            const float rs = a4.w + b4.w;
            if (dot(d, d) <= rs * rs)
              atomicOr((unsigned long long*)&s.rowCand[lo][hi >> 6], 1ull << (hi & 63));
          }
        }
      }
    }
    __syncthreads();
    // 3. compaction of candidate rows into the sorted pair list
    int ccount = 0;
    if (own) {
#pragma unroll
      for (int q = 0; q < NW; ++q) ccount += __popcll(s.rowCand[tid][q]);
    }
    int ctotal;
    const int cstart = block_excl_scan<N>(ccount, s.scan, &ctotal);
    s.cstart[tid] = cstart;
    if (own) {
      int pos = cstart;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        uint64_t m = s.rowCand[tid][q];
        while (m) {
          const int j = 64 * q + __ffsll((unsigned long long)m) - 1;
          m &= m - 1ull;
          if (pos < PhysLDS<N>::CAPC) s.cand[pos] = (uint32_t)tid | ((uint32_t)j << 16);
          ++pos;
        }
      }
    }
    if (ctotal > PhysLDS<N>::CAPC) bad = true;
    __syncthreads();
    // 4a. narrowphase of the pairs with a sphere, one candidate per lane;
    // cube-cube pairs are queued.  A pair in contact takes the next free
    // slot (handed out per wave) and its candidate remembers it, so the
    // order of the slots affects no sum.
    const int nc = ctotal < PhysLDS<N>::CAPC ? ctotal : PhysLDS<N>::CAPC;
    const int ncw = wmax(nc);
    for (int c0 = 0; c0 < ncw; c0 += N) {
      const int k = c0 + tid;
      bool contact = false, cc = false;
      PairAcc acc;
      int i = 0, j = 0;
      if (k < nc) {
        const uint32_t pr = s.cand[k];
        i = (int)(pr & 0xFFFFu);
        j = (int)(pr >> 16);
        cc = (s.type[i] != 0) & (s.type[j] != 0);
        if (!cc) {
          acc = pair_forces<N, FR>(s, i, j, pc);
          contact = acc.npts > 0;
        } else {
          // box pairs apart along a face axis have no point: not queued
          cc = !face_separated(ldsP(s, i), ldsR(s, i), ldsE(s, i), ldsP(s, j), ldsR(s, j), ldsE(s, j));
        }
      }
      const uint64_t cm = __ballot(contact), qm = __ballot(cc);
      int kb = 0, qb = 0;
      if (lane == lbase) {
        if (half(cm)) kb = atomicAdd(&s.kcnt, __popcll(half(cm)));
        if (half(qm)) qb = atomicAdd(&s.ncc, __popcll(half(qm)));
      }
      kb = __shfl(kb, lbase, 64);
      qb = __shfl(qb, lbase, 64);
      if (contact) {
        const int slot = kb + below(cm);
        s.kslot[k] = (uint16_t)slot;
        if (slot < PhysLDS<N>::CAPK) {
          s.kres[0][slot] = acc.SF.x; s.kres[1][slot] = acc.SF.y; s.kres[2][slot] = acc.SF.z;
          s.kres[3][slot] = acc.Ti.x; s.kres[4][slot] = acc.Ti.y; s.kres[5][slot] = acc.Ti.z;
          s.kres[6][slot] = acc.Tj.x; s.kres[7][slot] = acc.Tj.y; s.kres[8][slot] = acc.Tj.z;
        }
        atomicOr((unsigned long long*)&s.rowC[i][j >> 6], 1ull << (j & 63));
        atomicOr((unsigned long long*)&s.colC[j][i >> 6], 1ull << (i & 63));
      }
      if (cc) s.ccl[qb + below(qm)] = (uint32_t)k | ((uint32_t)i << 10) | ((uint32_t)j << 21);
    }
    // ground: a sphere's single point on its own lane; cubes are queued
    bool gsph = false;
    PairAcc gs;
    if (own && p.z < rbv && ty == 0) {
      const f3 z3 = mk(0.0f, 0.0f, 0.0f);
      Point pt;
      gs.SF = z3;
      gs.Ti = z3;
      gs.Tj = z3;
      gs.npts = 0;
      if (p.z < a) {
        pt.n = mk(0.0f, 0.0f, 1.0f);
        pt.delta = a - p.z;
        pt.xc = mk(p.x, p.y, p.z - a);
        add_point<FR>(gs, pt, true, p, v, w, z3, z3, z3, true, pc);
        gsph = true;
      }
    }
    {
      // a cube is queued for the 8-lane corner terms only if one of its
      // corners is below the ground: the same z of each corner as the
      // corner test computes, p.z + row 2 of R times (+-e)
      bool gq = false;
      if (own && p.z < rbv && ty != 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float wx = (k & 1) ? ex : -ex, wy = (k & 2) ? ey : -ey, wz = (k & 4) ? ez : -ez;
          gq |= p.z + ((R.m[6] * wx + R.m[7] * wy) + R.m[8] * wz) < 0.0f;
        }
      }
      const uint64_t gm = __ballot(gq);
      int gb = 0;
      if (lane == lbase && half(gm)) gb = atomicAdd(&s.ngc, __popcll(half(gm)));
      gb = __shfl(gb, lbase, 64);
      if (gq) s.gcl[gb + below(gm)] = tid;
      s.gflag[tid] = gsph ? 1 : 0;
      if (gsph) {
        s.gres[0][tid] = gs.SF.x; s.gres[1][tid] = gs.SF.y; s.gres[2][tid] = gs.SF.z;
        s.gres[3][tid] = gs.Ti.x; s.gres[4][tid] = gs.Ti.y; s.gres[5][tid] = gs.Ti.z;
      }
    }
    __syncthreads();
    // 4b. cube-cube pairs, 16 lanes each: lane r of a group tests corner
    // r & 7 of cube i inside cube j (r < 8), then of j inside i -- the
    // oracle's point order -- and lanes 0..8 of the group then sum one
    // component each over the points found, in that order.
    const int ncc = s.ncc;
    const int nccw = wmax(ncc);
    for (int t0 = 0; t0 < 16 * nccw; t0 += N) {
      const int t = t0 + tid;
      const int r = lane & 15;
      bool hit = false;
      int k = 0, i = 0, j = 0;
      if (t < 16 * ncc) {
        const uint32_t e = s.ccl[t >> 4];
        k = (int)(e & 0x3FFu);
        i = (int)((e >> 10) & 0x7FFu);
        j = (int)(e >> 21);
        const int A = r < 8 ? i : j, B = r < 8 ? j : i;
        const f3 pA = ldsP(s, A), pB = ldsP(s, B);
        const M3 RA = ldsR(s, A), RB = ldsR(s, B);
        const f3 aA = ldsE(s, A), aB = ldsE(s, B);
        const f3 vi = ldsV(s, i), wi = ldsW(s, i), vj = ldsV(s, j), wj = ldsW(s, j);
        Point pt;
        hit = corner_in_box(pA, RA, aA, r & 7, pB, RB, aB, &pt);
        if (hit) {
          const f3 pi = r < 8 ? pA : pB, pj = r < 8 ? pB : pA;
          const PointTerms pq = point_terms<FR>(pt, r < 8, pi, vi, wi, pj, vj, wj, false, pc);
          s.stage[0][tid] = pq.Fi.x; s.stage[1][tid] = pq.Fi.y; s.stage[2][tid] = pq.Fi.z;
          s.stage[3][tid] = pq.ti.x; s.stage[4][tid] = pq.ti.y; s.stage[5][tid] = pq.ti.z;
          s.stage[6][tid] = pq.tj.x; s.stage[7][tid] = pq.tj.y; s.stage[8][tid] = pq.tj.z;
        }
      }
      // edge-edge point (after the 16 vertex points in the pair's order)
      bool ehit = false;
      if constexpr (EE) ehit = edge_point<N, FR>(s, t < 16 * ncc, r, lane, i, j, pc);
      const uint64_t hm = __ballot(hit);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const int g0 = lane & 48;  // the group's first lane in the wave
      const uint32_t gm = (uint32_t)(hm >> g0) & 0xFFFFu;
      float sum = 0.0f;
      if (r < 9) sum = ordered_sum<16, N>(s, r, tid - r, gm);
      if constexpr (EE) {
        if (ehit && r < 9) sum = sum + s.estage[r][tid >> 4];
      }
      const bool any = gm != 0 || ehit;
      const uint64_t lead = __ballot(r == 0 && any);
      int kb = 0;
      if (lane == lbase && half(lead)) kb = atomicAdd(&s.kcnt, __popcll(half(lead)));
      kb = __shfl(kb, lbase, 64);
      if (any) {
        const int slot = kb + __popcll(half(lead) & ((1ull << (g0 - lbase)) - 1ull));
        if (r < 9 && slot < PhysLDS<N>::CAPK) s.kres[r][slot] = sum;
        if (r == 0) {
          s.kslot[k] = (uint16_t)slot;
          atomicOr((unsigned long long*)&s.rowC[i][j >> 6], 1ull << (j & 63));
          atomicOr((unsigned long long*)&s.colC[j][i >> 6], 1ull << (i & 63));
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    // 4c. cubes near the ground, 8 lanes each: lane r tests corner r, and
    // lanes 0..5 sum the force and torque components in corner order
    const int ngc = s.ngc;
    const int ngcw = wmax(ngc);
    for (int t0 = 0; t0 < 8 * ngcw; t0 += N) {
      const int t = t0 + tid;
      const int r = lane & 7;
      bool hit = false;
      int b = 0;
      if (t < 8 * ngc) {
        b = s.gcl[t >> 3];
        const f3 pb = ldsP(s, b), vb = ldsV(s, b), wb = ldsW(s, b);
        const f3 vtx = corner_vertex(pb, ldsR(s, b), ldsE(s, b), r);
        if (vtx.z < 0.0f) {
          hit = true;
          const f3 z3 = mk(0.0f, 0.0f, 0.0f);
          Point pt;
          pt.n = mk(0.0f, 0.0f, 1.0f);
          pt.delta = -vtx.z;
          pt.xc = vtx;
          const PointTerms pq = point_terms<FR>(pt, true, pb, vb, wb, z3, z3, z3, true, pc);
          s.stage[0][tid] = pq.Fi.x; s.stage[1][tid] = pq.Fi.y; s.stage[2][tid] = pq.Fi.z;
          s.stage[3][tid] = pq.ti.x; s.stage[4][tid] = pq.ti.y; s.stage[5][tid] = pq.ti.z;
        }
      }
      const uint64_t hm = __ballot(hit);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const uint32_t gm = (uint32_t)(hm >> (lane & 56)) & 0xFFu;
      if (gm != 0 && r < 6) {
        s.gres[r][b] = ordered_sum<8, N>(s, r, tid - r, gm);
        if (r == 0) s.gflag[b] = 1;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    __syncthreads();
    if (s.kcnt > PhysLDS<N>::CAPK) bad = true;
    // 5. gather in sorted pair order, then the ground, then integrate.
    // Contacts are taken four at a time so that each level of lookups
    // (candidate index, slot, sums) issues its loads together.
    if (own) {
      f3 F = mk(0.0f, 0.0f, 0.0f), Tq = F;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        // pairs (i, tid), i ascending: the candidate index of (i, tid) is
        // the start of row i plus the rank of tid in that row
        uint64_t m = s.colC[tid][q];
        while (m) {
          int ii[4], idx[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            ii[u] = m ? 64 * q + __ffsll((unsigned long long)m) - 1 : -1;
            m &= m - 1ull;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = ii[u] < 0 ? 0 : ii[u];
            idx[u] = s.kslot[s.cstart[i] + popc_below<NW>(s.rowCand[i], tid)];
            if (ii[u] < 0 || idx[u] >= PhysLDS<N>::CAPK) idx[u] = -1;
          }
          float kv[4][6];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int x = idx[u] < 0 ? 0 : idx[u];
            kv[u][0] = s.kres[0][x]; kv[u][1] = s.kres[1][x]; kv[u][2] = s.kres[2][x];
            kv[u][3] = s.kres[6][x]; kv[u][4] = s.kres[7][x]; kv[u][5] = s.kres[8][x];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (idx[u] >= 0) {
              F = sub(F, mk(kv[u][0], kv[u][1], kv[u][2]));
              Tq = add(Tq, mk(kv[u][3], kv[u][4], kv[u][5]));
            }
          }
        }
      }
      {
        // pairs (tid, j), j ascending: candidates of row tid in contact
        int c = cstart;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
          uint64_t m = s.rowCand[tid][q];
          const uint64_t mc = s.rowC[tid][q];
          uint64_t mk_ = mc;
          while (mk_) {
            // candidate index of each of the next four contacts: the row
            // start plus its rank among the row's candidates
            int idx[4];
            bool ok[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              ok[u] = mk_ != 0ull;
              const int j = ok[u] ? __ffsll((unsigned long long)mk_) - 1 : 0;
              mk_ &= mk_ - 1ull;
              idx[u] = s.kslot[c + __popcll(m & below_mask(j))];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (!ok[u] || idx[u] >= PhysLDS<N>::CAPK) idx[u] = -1;
            float kv[4][6];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int x = idx[u] < 0 ? 0 : idx[u];
              kv[u][0] = s.kres[0][x]; kv[u][1] = s.kres[1][x]; kv[u][2] = s.kres[2][x];
              kv[u][3] = s.kres[3][x]; kv[u][4] = s.kres[4][x]; kv[u][5] = s.kres[5][x];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (idx[u] >= 0) {
                F = add(F, mk(kv[u][0], kv[u][1], kv[u][2]));
                Tq = add(Tq, mk(kv[u][3], kv[u][4], kv[u][5]));
              }
            }
          }
          c += __popcll(m);
        }
      }
      if (s.gflag[tid]) {
        F = add(F, mk(s.gres[0][tid], s.gres[1][tid], s.gres[2][tid]));
        Tq = add(Tq, mk(s.gres[3][tid], s.gres[4][tid], s.gres[5][tid]));
      }
      if (has_fx) F = add(F, fx);  // external force, after the contacts
      // semi-implicit Euler
      const f3 acc = add(mul(F, inv_m), gvec);
      v = add(v, mul(acc, pc.h));
      p = add(p, mul(v, pc.h));
      if (ty == 2) {
        // a box: Euler's equations in the body frame with the gyroscopic
        // term, R of the substep start: w_b = R^T w,
        // dw_b = (R^T T - w_b x (I w_b)) / I, w = R (w_b + h dw_b)
        const M3 Rs = ldsR(s, tid);
        const f3 I = mk(s.inert[0][tid], s.inert[1][tid], s.inert[2][tid]);
        const f3 wb = rotT(Rs, w), tb = rotT(Rs, Tq);
        const f3 gy = cross(wb, mk(I.x * wb.x, I.y * wb.y, I.z * wb.z));
        const f3 dwb = mk((tb.x - gy.x) / I.x, (tb.y - gy.y) / I.y, (tb.z - gy.z) / I.z);
        w = rot(Rs, add(wb, mul(dwb, pc.h)));
      } else {
        w = add(w, mul(mul(Tq, inv_I), pc.h));
      }
      const float dw = (-w.x * qx - w.y * qy) - w.z * qz;
      const float dx = (w.x * qw + w.y * qz) - w.z * qy;
      const float dy = (w.y * qw + w.z * qx) - w.x * qz;
      const float dz = (w.z * qw + w.x * qy) - w.y * qx;
      qw = qw + pc.hh * dw;
      qx = qx + pc.hh * dx;
      qy = qy + pc.hh * dy;
      qz = qz + pc.hh * dz;
      const float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
      const float inv = 1.0f / sqrtf(n2);
      qw = qw * inv; qx = qx * inv; qy = qy * inv; qz = qz * inv;
    }
    __syncthreads();
    if (W.contacts) {
      // pairs of row tid in ascending j, then (tid, ground)
      int cnt = 0;
      bool gc = false;
      if (own) {
        gc = s.gflag[tid] != 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) cnt += __popcll(s.rowC[tid][q]);
        cnt += gc ? 1 : 0;
      }
      int tot;
      const int off = block_excl_scan<N>(cnt, s.scan, &tot);
      int32_t* dst = W.contacts + ((int64_t)(env < 0 ? 0 : env) * pc.substeps + sub_i) * (1 + 2 * W.pair_cap);
      if (tid == 0 && env >= 0) dst[0] = tot;
      if (own) {
        int pos = off;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
          uint64_t m = s.rowC[tid][q];
          while (m) {
            const int j = 64 * q + __ffsll((unsigned long long)m) - 1;
            m &= m - 1ull;
            if (pos < W.pair_cap) { dst[1 + 2 * pos] = tid; dst[2 + 2 * pos] = j; }
            ++pos;
          }
        }
        if (gc && pos < W.pair_cap) { dst[1 + 2 * pos] = tid; dst[2 + 2 * pos] = kGroundPair; }
      }
    }
    __syncthreads();
  }
  if (own) {
    out[PX * cap + gb] = p.x; out[PY * cap + gb] = p.y; out[PZ * cap + gb] = p.z;
    out[VX * cap + gb] = v.x; out[VY * cap + gb] = v.y; out[VZ * cap + gb] = v.z;
    out[QW * cap + gb] = qw; out[QX * cap + gb] = qx; out[QY * cap + gb] = qy; out[QZ * cap + gb] = qz;
    out[WX * cap + gb] = w.x; out[WY * cap + gb] = w.y; out[WZ * cap + gb] = w.z;
    const bool fin = isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(v.x) &&
                     isfinite(v.y) && isfinite(v.z) && isfinite(w.x) && isfinite(w.y) &&
                     isfinite(w.z) && isfinite(qw) && isfinite(qx) && isfinite(qy) && isfinite(qz);
    if (!fin) atomicOr(&W.env_flags[env], kFlagNonFinite);
  }
  if (bad && tid == 0 && env >= 0) atomicOr(&W.env_flags[env], kFlagContactOverflow);
}

// FR: friction; EE: edge-edge points of box pairs; SUP: the step's candidate
// superset on the all-pairs path (compiled in only for launches whose envs
// exceed 32 bodies, where it pays).  N lanes per env: a workgroup of 64
// threads holds two envs at N = 32, one at N = 64; two waves hold one env at
// N = 128.  Work item w takes envs P w .. P w + P - 1 of the list (P envs per
// workgroup).
template <int N, bool FR, bool EE, bool SUP>
__global__ __launch_bounds__(N < 64 ? 64 : N) void physics_kernel(WorldDev W, PhysConsts pc, PhysLaunch L) {
  constexpr int P = N < 64 ? 64 / N : 1;
  __shared__ PhysLDS<N> sh[P];
  const int sub = (int)threadIdx.x / N;
  // The step is latency-bound; a higher issue priority shortens it when it
  // shares CUs with the render phase.
  switch (L.prio) {
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    case 3: __builtin_amdgcn_s_setprio(3); break;
    default: break;
  }
  if (L.persistent == 0) {
    const int wi = blockIdx.x;
    if (P * wi >= L.n_work) return;
    const int item = P * wi + sub;
    step_env<N, FR, EE, SUP>(sh[sub], W, pc, item < L.n_work ? uniform_ld(L.work + item) : -1, L.parity, L.broadphase);
    return;
  }
  for (;;) {
    if (threadIdx.x == 0) sh[0].work = atomicAdd(L.queue, 1);
    __syncthreads();
    const int wi = sh[0].work;
    __syncthreads();
    if (P * wi >= L.n_work) return;
    const int item = P * wi + sub;
    step_env<N, FR, EE, SUP>(sh[sub], W, pc, item < L.n_work ? uniform_ld(L.work + item) : -1, L.parity, L.broadphase);
  }
}

__global__ void reset_queue_kernel(int32_t* q) { *q = 0; }

}  // namespace

hipError_t launch_reset_queue(int32_t* q, hipStream_t s) {
  hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(1), 0, s, q);
  return hipGetLastError();
}

hipError_t resident_workgroups(const void* kernel, int threads, size_t dyn_lds, int* out) {
  *out = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int, size_t>, int> cache;
  const auto key = std::make_tuple(dev, kernel, threads, dyn_lds);
  {
    std::lock_guard<std::mutex> g(mu);
    const auto it = cache.find(key);
    if (it != cache.end()) {
      *out = it->second;
      return hipSuccess;
    }
  }
  int per_cu = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, dyn_lds);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int n = per_cu * cus;
  if (n <= 0) return hipErrorInvalidConfiguration;
  std::lock_guard<std::mutex> g(mu);
  cache[key] = n;
  *out = n;
  return hipSuccess;
}

hipError_t persistent_grid(int persistent, int items, const void* kernel, int threads, size_t dyn_lds,
                           int* grid) {
  int n = persistent;
  if (n < 0) {
    const hipError_t e = resident_workgroups(kernel, threads, dyn_lds, &n);
    if (e != hipSuccess) return e;
  }
  *grid = n < items ? n : items;
  return hipSuccess;
}

template <int N, bool SUP>
static const void* physics_fn(bool fr, bool ee) {
  if (!fr && !ee) return (const void*)physics_kernel<N, false, false, SUP>;
  if (!ee) return (const void*)physics_kernel<N, true, false, SUP>;
  if (!fr) return (const void*)physics_kernel<N, false, true, SUP>;
  return (const void*)physics_kernel<N, true, true, SUP>;
}

template <int N, bool SUP>
static void launch_n(bool fr, bool ee, LaunchEvents* ev, bool first, bool last, dim3 g, hipStream_t s,
                     const WorldDev& w, const PhysConsts& pc, const PhysLaunch& lt) {
  const dim3 b(N < 64 ? 64 : N);
  if (!fr && !ee) timed_launch(ev, first, last, physics_kernel<N, false, false, SUP>, g, b, 0, s, w, pc, lt);
  else if (!ee) timed_launch(ev, first, last, physics_kernel<N, true, false, SUP>, g, b, 0, s, w, pc, lt);
  else if (!fr) timed_launch(ev, first, last, physics_kernel<N, false, true, SUP>, g, b, 0, s, w, pc, lt);
  else timed_launch(ev, first, last, physics_kernel<N, true, true, SUP>, g, b, 0, s, w, pc, lt);
}

hipError_t launch_physics(const WorldDev& w, const PhysConsts& pc, const PhysLaunch& l,
                          hipStream_t s, LaunchEvents* ev) {
  if (l.n_work <= 0) return hipSuccess;
  // lanes per env: two envs of at most 32 bodies share a wave when packing
  // is on; one wave for up to 64 bodies; two for up to 128
  const int N = (l.max_bodies <= 32 && l.pack == 2) ? 32 : (l.max_bodies <= 64 ? 64 : 128);
  const int P = N < 64 ? 64 / N : 1;
  const int items = (l.n_work + P - 1) / P;
  const bool fr = pc.mu > 0.0f, ee = pc.edge != 0;
  int grid = items;
  if (l.persistent != 0) {
    const void* fn = N == 32 ? physics_fn<32, false>(fr, ee)
                     : N == 64 ? (l.max_bodies > 32 ? physics_fn<64, true>(fr, ee) : physics_fn<64, false>(fr, ee))
                               : physics_fn<128, false>(fr, ee);
    const hipError_t e = persistent_grid(l.persistent, items, fn, N < 64 ? 64 : N, 0, &grid);
    if (e != hipSuccess) return e;
  }
  for (int t = 0; t < l.nsteps; ++t) {
    PhysLaunch lt = l;
    lt.parity = (l.parity + t) & 1;
    lt.persistent = l.persistent != 0 ? grid : 0;  // the kernel only tells 0 from the rest
    if (l.persistent != 0) {
      hipError_t e = launch_reset_queue(l.queue, s);
      if (e != hipSuccess) return e;
    }
    const bool first = t == 0, last = t == l.nsteps - 1;
    if (N == 32) launch_n<32, false>(fr, ee, ev, first, last, dim3(grid), s, w, pc, lt);
    else if (N == 64 && l.max_bodies > 32) launch_n<64, true>(fr, ee, ev, first, last, dim3(grid), s, w, pc, lt);
    else if (N == 64) launch_n<64, false>(fr, ee, ev, first, last, dim3(grid), s, w, pc, lt);
    else launch_n<128, false>(fr, ee, ev, first, last, dim3(grid), s, w, pc, lt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vuda
