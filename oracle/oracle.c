/*
 * CPU oracle: physics step and rasterizer, single-threaded per env.
 *
 * TEST INFRASTRUCTURE ONLY -- see oracle.h.  Compiled with -ffp-contract=off
 * and no fast-math; every floating-point expression is evaluated exactly in
 * the order written.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef struct { float x, y, z; } v3;

static v3 mk(float x, float y, float z) { v3 r = {x, y, z}; return r; }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(v3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
static v3 neg(v3 a) { return mk(-a.x, -a.y, -a.z); }
/* dot product, summed left to right */
static float dot(v3 a, v3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static v3 cross(v3 a, v3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static float comp(v3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

/* Rotation matrix of a quaternion (w,x,y,z), row-major m[3*r+c]; the
 * standard unit-quaternion formula, evaluated as written. */
static void quat_mat(const float* q, float* m) {
  float w = q[0], x = q[1], y = q[2], z = q[3];
  float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  float wx = w * x, wy = w * y, wz = w * z;
  m[0] = 1.0f - 2.0f * (yy + zz); m[1] = 2.0f * (xy - wz);        m[2] = 2.0f * (xz + wy);
  m[3] = 2.0f * (xy + wz);        m[4] = 1.0f - 2.0f * (xx + zz); m[5] = 2.0f * (yz - wx);
  m[6] = 2.0f * (xz - wy);        m[7] = 2.0f * (yz + wx);        m[8] = 1.0f - 2.0f * (xx + yy);
}
/* R v (rows dotted with v) */
static v3 mat_vec(const float* m, v3 v) {
  return mk((m[0] * v.x + m[1] * v.y) + m[2] * v.z,
            (m[3] * v.x + m[4] * v.y) + m[5] * v.z,
            (m[6] * v.x + m[7] * v.y) + m[8] * v.z);
}
/* R^T v (columns dotted with v) */
static v3 mat_tvec(const float* m, v3 v) {
  return mk((m[0] * v.x + m[3] * v.y) + m[6] * v.z,
            (m[1] * v.x + m[4] * v.y) + m[7] * v.z,
            (m[2] * v.x + m[5] * v.y) + m[8] * v.z);
}

static v3 load3(const float* a, int32_t i) { return mk(a[3 * i], a[3 * i + 1], a[3 * i + 2]); }

/* Corner k of a cube of half-extent a: sign + on axis t iff bit t of k set. */
/* Corner k of a box of half-extents e (a cube: e = (a, a, a)): sign + on
 * axis t iff bit t of k is set. */
static v3 cube_vertex(v3 p, const float* R, v3 e, int k) {
  v3 w = mk((k & 1) ? e.x : -e.x, (k & 2) ? e.y : -e.y, (k & 4) ? e.z : -e.z);
  return add(p, mat_vec(R, w));
}

/* Deepest-face axis of a local point strictly inside a box of half-extents
 * e: argmin over axes of (e_axis - |u_axis|), lowest axis on ties. */
static int min_axis(v3 u, v3 e, float* depth) {
  float d0 = e.x - fabsf(u.x), d1 = e.y - fabsf(u.y), d2 = e.z - fabsf(u.z);
  int m = 0;
  float dm = d0;
  if (d1 < dm) { m = 1; dm = d1; }
  if (d2 < dm) { m = 2; dm = d2; }
  *depth = dm;
  return m;
}

static v3 axis_dir(int m, float s) {
  return mk(m == 0 ? s : 0.0f, m == 1 ? s : 0.0f, m == 2 ? s : 0.0f);
}

/* ---------------------------------------------------------------------------
 * Narrowphase.  "Contact" means penetration strictly greater than zero.
 * Each point names the body "A" pushed along +n.
 * ------------------------------------------------------------------------- */

static int np_sphere_sphere(v3 pi, float ri, v3 pj, float rj, oracle_point* out) {
  v3 d = sub(pi, pj);
  float d2 = dot(d, d);
  float s = ri + rj;
  if (!(d2 < s * s)) return 0;
  float L = sqrtf(d2);
  v3 n = L > 0.0f ? mk(d.x / L, d.y / L, d.z / L) : mk(0.0f, 0.0f, 1.0f);
  float delta = s - L;
  v3 xc = add(pj, scl(n, rj - 0.5f * delta));
  out->n[0] = n.x; out->n[1] = n.y; out->n[2] = n.z;
  out->delta = delta;
  out->xc[0] = xc.x; out->xc[1] = xc.y; out->xc[2] = xc.z;
  out->a_is_first = 1;
  return 1;
}

/* sphere (centre c, radius r) against box (p, R, half-extents a); normal
 * from the box to the sphere */
static int np_sphere_cube(v3 c, float r, v3 p, const float* R, v3 a, int sphere_first,
                          oracle_point* out) {
  v3 u = mat_tvec(R, sub(c, p));
  v3 e = mk(fminf(fmaxf(u.x, -a.x), a.x), fminf(fmaxf(u.y, -a.y), a.y), fminf(fmaxf(u.z, -a.z), a.z));
  v3 rv = sub(u, e);
  float L2 = dot(rv, rv);
  if (!(L2 < r * r)) return 0;
  v3 nl;
  float delta;
  if (L2 > 0.0f) {
    float L = sqrtf(L2);
    nl = mk(rv.x / L, rv.y / L, rv.z / L);
    delta = r - L;
  } else {
    float dm;
    int m = min_axis(u, a, &dm);
    nl = axis_dir(m, comp(u, m) >= 0.0f ? 1.0f : -1.0f);
    delta = r + dm;
  }
  v3 n = mat_vec(R, nl);
  v3 xc = add(p, mat_vec(R, e));
  out->n[0] = n.x; out->n[1] = n.y; out->n[2] = n.z;
  out->delta = delta;
  out->xc[0] = xc.x; out->xc[1] = xc.y; out->xc[2] = xc.z;
  out->a_is_first = sphere_first;
  return 1;
}

/* vertices of box A (pa, Ra, half-extents aa) strictly inside box B (pb, Rb, ab) */
static int np_vertices_in_box(v3 pa, const float* Ra, v3 aa, v3 pb, const float* Rb, v3 ab,
                              int a_first, oracle_point* out) {
  int cnt = 0;
  for (int k = 0; k < 8; ++k) {
    v3 v = cube_vertex(pa, Ra, aa, k);
    v3 u = mat_tvec(Rb, sub(v, pb));
    if (fabsf(u.x) < ab.x && fabsf(u.y) < ab.y && fabsf(u.z) < ab.z) {
      float dm;
      int m = min_axis(u, ab, &dm);
      v3 n = mat_vec(Rb, axis_dir(m, comp(u, m) >= 0.0f ? 1.0f : -1.0f));
      oracle_point* o = &out[cnt++];
      o->n[0] = n.x; o->n[1] = n.y; o->n[2] = n.z;
      o->delta = dm;
      o->xc[0] = v.x; o->xc[1] = v.y; o->xc[2] = v.z;
      o->a_is_first = a_first;
    }
  }
  return cnt;
}

/* ---------------------------------------------------------------------------
 * Edge-edge contact of two boxes by the separating-axis test (optional).
 * Candidate axes, in this order: the three axes of box i, the three of box
 * j, then the nine cross products (axis a of i) x (axis b of j), a major;
 * a cross product shorter than sqrt(ORACLE_EDGE_PARALLEL) (near-parallel
 * edges) is no axis.  Along a unit axis L the boxes overlap by
 * o(L) = r_i(L) + r_j(L) - |(p_i - p_j) . L|, r(L) = sum_k e_k |u_k . L|.
 * Some o <= 0: separated, no point.  Otherwise, if the least overlap over
 * the cross-product axes is below ORACLE_EDGE_BIAS times the least over the
 * face axes (faces are preferred: their contacts are the vertex points),
 * one point is added where the two supporting edges pass closest: normal
 * that axis pointing from j to i, depth that overlap.
 * ------------------------------------------------------------------------- */

/* Column k of a row-major rotation: the body's axis k in the world. */
static v3 mat_col(const float* R, int k) { return mk(R[k], R[3 + k], R[6 + k]); }

/* Half-width of a box (rotation R, half-extents e) along direction L. */
static float box_radius(const float* R, v3 e, v3 L) {
  v3 u = mat_tvec(R, L);
  return (e.x * fabsf(u.x) + e.y * fabsf(u.y)) + e.z * fabsf(u.z);
}

static int np_edge_edge(v3 pi, const float* Ri, v3 ei, v3 pj, const float* Rj, v3 ej, oracle_point* out) {
  v3 d = sub(pi, pj);
  float fmin = INFINITY, emin = INFINITY;
  int ek = -1;
  v3 eL = mk(0.0f, 0.0f, 0.0f);
  for (int k = 0; k < 15; ++k) {
    v3 L;
    if (k < 3) {
      L = mat_col(Ri, k);
    } else if (k < 6) {
      L = mat_col(Rj, k - 3);
    } else {
      L = cross(mat_col(Ri, (k - 6) / 3), mat_col(Rj, (k - 6) % 3));
      float l2 = dot(L, L);
      if (!(l2 >= ORACLE_EDGE_PARALLEL)) continue;
      float l = sqrtf(l2);
      L = mk(L.x / l, L.y / l, L.z / l);
    }
    float o = (box_radius(Ri, ei, L) + box_radius(Rj, ej, L)) - fabsf(dot(d, L));
    if (!(o > 0.0f)) return 0; /* a separating axis */
    if (k < 6) {
      if (o < fmin) fmin = o;
    } else if (o < emin) {
      emin = o;
      ek = k;
      eL = L;
    }
  }
  if (ek < 0 || !(emin < ORACLE_EDGE_BIAS * fmin)) return 0;
  int a = (ek - 6) / 3, b = (ek - 6) % 3;
  v3 n = dot(eL, d) < 0.0f ? neg(eL) : eL; /* from j to i */
  /* the edge of i along its axis a deepest toward j (along -n), and the
   * edge of j along its axis b deepest toward i (along +n): their centres */
  v3 ui = mat_tvec(Ri, n), uj = mat_tvec(Rj, n);
  v3 wi = mk(a == 0 ? 0.0f : (ui.x > 0.0f ? -ei.x : ei.x), a == 1 ? 0.0f : (ui.y > 0.0f ? -ei.y : ei.y),
             a == 2 ? 0.0f : (ui.z > 0.0f ? -ei.z : ei.z));
  v3 wj = mk(b == 0 ? 0.0f : (uj.x > 0.0f ? ej.x : -ej.x), b == 1 ? 0.0f : (uj.y > 0.0f ? ej.y : -ej.y),
             b == 2 ? 0.0f : (uj.z > 0.0f ? ej.z : -ej.z));
  v3 ci = add(pi, mat_vec(Ri, wi)), cj = add(pj, mat_vec(Rj, wj));
  /* closest points of the lines ci + s da and cj + t db (unit directions),
   * each clamped to its edge */
  v3 da = mat_col(Ri, a), db = mat_col(Rj, b);
  v3 w = sub(ci, cj);
  float bb = dot(da, db), dd = dot(da, w), ee = dot(db, w);
  float den = 1.0f - bb * bb;
  float sa = (bb * ee - dd) / den, tb = (ee - bb * dd) / den;
  float ha = comp(ei, a), hb = comp(ej, b);
  sa = fminf(fmaxf(sa, -ha), ha);
  tb = fminf(fmaxf(tb, -hb), hb);
  v3 xc = scl(add(add(ci, scl(da, sa)), add(cj, scl(db, tb))), 0.5f);
  out->n[0] = n.x; out->n[1] = n.y; out->n[2] = n.z;
  out->delta = emin;
  out->xc[0] = xc.x; out->xc[1] = xc.y; out->xc[2] = xc.z;
  out->a_is_first = 1;
  return 1;
}

/* Half-extents of body i: its own for a box (type 2), (a, a, a) for a cube
 * or a sphere of size a. */
static v3 body_ext(int32_t i, const uint8_t* type, const float* size, const float* ext) {
  if (type[i] == 2 && ext) return load3(ext, i);
  return mk(size[i], size[i], size[i]);
}

static int np_ground(int32_t i, const uint8_t* type, const float* size, const float* ext, const float* pos,
                     const float* quat, oracle_point* out) {
  v3 p = load3(pos, i);
  float a = size[i];
  if (type[i] == 0) {
    if (!(p.z < a)) return 0;
    out->n[0] = 0.0f; out->n[1] = 0.0f; out->n[2] = 1.0f;
    out->delta = a - p.z;
    out->xc[0] = p.x; out->xc[1] = p.y; out->xc[2] = p.z - a;
    out->a_is_first = 1;
    return 1;
  }
  float R[9];
  quat_mat(quat + 4 * i, R);
  v3 e = body_ext(i, type, size, ext);
  int cnt = 0;
  for (int k = 0; k < 8; ++k) {
    v3 v = cube_vertex(p, R, e, k);
    if (v.z < 0.0f) {
      oracle_point* o = &out[cnt++];
      o->n[0] = 0.0f; o->n[1] = 0.0f; o->n[2] = 1.0f;
      o->delta = -v.z;
      o->xc[0] = v.x; o->xc[1] = v.y; o->xc[2] = v.z;
      o->a_is_first = 1;
    }
  }
  return cnt;
}

static int narrowphase(int32_t i, int32_t j, const uint8_t* type, const float* size, const float* ext,
                       const float* pos, const float* quat, int edge, oracle_point* pts) {
  if (j == ORACLE_GROUND) return np_ground(i, type, size, ext, pos, quat, pts);
  v3 pi = load3(pos, i), pj = load3(pos, j);
  float Ri[9], Rj[9];
  quat_mat(quat + 4 * i, Ri);
  quat_mat(quat + 4 * j, Rj);
  v3 ei = body_ext(i, type, size, ext), ej = body_ext(j, type, size, ext);
  if (type[i] == 0 && type[j] == 0) return np_sphere_sphere(pi, size[i], pj, size[j], pts);
  if (type[i] == 0) return np_sphere_cube(pi, size[i], pj, Rj, ej, 1, pts);
  if (type[j] == 0) return np_sphere_cube(pj, size[j], pi, Ri, ei, 0, pts);
  int c = np_vertices_in_box(pi, Ri, ei, pj, Rj, ej, 1, pts);
  c += np_vertices_in_box(pj, Rj, ej, pi, Ri, ei, 0, pts + c);
  if (edge) c += np_edge_edge(pi, Ri, ei, pj, Rj, ej, pts + c);
  return c;
}

int oracle_narrowphase(int32_t i, int32_t j, const uint8_t* type, const float* size,
                       const float* pos, const float* quat, oracle_point* pts) {
  return narrowphase(i, j, type, size, NULL, pos, quat, 0, pts);
}

int oracle_narrowphase_box(int32_t i, int32_t j, const uint8_t* type, const float* size, const float* ext,
                           const float* pos, const float* quat, int32_t edge, oracle_point* pts) {
  return narrowphase(i, j, type, size, ext, pos, quat, edge, pts);
}

/* ---------------------------------------------------------------------------
 * Physics step
 * ------------------------------------------------------------------------- */

typedef struct { v3 F, T; } acc_t;

static int finite3(v3 a) { return isfinite(a.x) && isfinite(a.y) && isfinite(a.z); }

int oracle_step_env(int32_t n, const uint8_t* type, const float* size, const float* rbound,
                    const float* inv_m, const float* inv_I, float* pos, float* vel,
                    float* quat, float* omega, const oracle_phys_params* prm,
                    int32_t* pairs, int32_t pair_cap, int32_t* npairs) {
  return oracle_step_env_ext(n, type, size, rbound, inv_m, inv_I, pos, vel, quat, omega, prm, pairs,
                             pair_cap, npairs, NULL);
}

int oracle_step_env_ext(int32_t n, const uint8_t* type, const float* size, const float* rbound,
                        const float* inv_m, const float* inv_I, float* pos, float* vel,
                        float* quat, float* omega, const oracle_phys_params* prm,
                        int32_t* pairs, int32_t pair_cap, int32_t* npairs, const float* fext) {
  return oracle_step_env_box(n, type, size, NULL, NULL, rbound, inv_m, inv_I, pos, vel, quat, omega, prm, pairs,
                             pair_cap, npairs, fext);
}

int oracle_step_env_box(int32_t n, const uint8_t* type, const float* size, const float* ext,
                        const float* inertia, const float* rbound, const float* inv_m, const float* inv_I,
                        float* pos, float* vel, float* quat, float* omega, const oracle_phys_params* prm,
                        int32_t* pairs, int32_t pair_cap, int32_t* npairs, const float* fext) {
  const float h = prm->dt / (float)prm->substeps;
  const float hh = 0.5f * h;
  const v3 g = mk(prm->g[0], prm->g[1], prm->g[2]);
  acc_t* acc = (acc_t*)malloc(sizeof(acc_t) * (size_t)(n > 0 ? n : 1));
  oracle_point pts[ORACLE_MAX_POINTS];
  int status = 0;

  for (int s = 0; s < prm->substeps; ++s) {
    int32_t np = 0;
    for (int32_t b = 0; b < n; ++b) { acc[b].F = mk(0, 0, 0); acc[b].T = mk(0, 0, 0); }

    /* Walk pairs in sorted (i, j) order, the ground last in each row; all
     * tests use the substep-start state. */
    for (int32_t i = 0; i < n; ++i) {
      v3 pi = load3(pos, i);
      for (int32_t j = i + 1; j <= n; ++j) {
        int32_t jj = (j == n) ? ORACLE_GROUND : j;
        int cand;
        if (jj == ORACLE_GROUND) {
          cand = pi.z < rbound[i];
        } else {
          v3 d = sub(pi, load3(pos, j));
          float rs = rbound[i] + rbound[j];
          cand = dot(d, d) <= rs * rs;
        }
        if (!cand) continue;
        int cnt = narrowphase(i, jj, type, size, ext, pos, quat, prm->edge, pts);
        if (cnt == 0) continue;
        if (pairs) {
          if (np >= pair_cap) { status = -1; }
          else {
            pairs[(size_t)s * pair_cap * 2 + 2 * np] = i;
            pairs[(size_t)s * pair_cap * 2 + 2 * np + 1] = jj;
          }
        }
        ++np;
        /* Forces of the pair's points, summed per pair in point order, then
         * added to each body in pair order. */
        v3 pA = pi, vA = load3(vel, i), wA = load3(omega, i);
        v3 pB = mk(0, 0, 0), vB = mk(0, 0, 0), wB = mk(0, 0, 0);
        if (jj != ORACLE_GROUND) { pB = load3(pos, jj); vB = load3(vel, jj); wB = load3(omega, jj); }
        v3 SF = mk(0, 0, 0), Ti = mk(0, 0, 0), Tj = mk(0, 0, 0);
        for (int k = 0; k < cnt; ++k) {
          v3 nrm = mk(pts[k].n[0], pts[k].n[1], pts[k].n[2]);
          v3 xc = mk(pts[k].xc[0], pts[k].xc[1], pts[k].xc[2]);
          /* body A of this point is pushed along +n */
          v3 pa = pts[k].a_is_first ? pA : pB, va = pts[k].a_is_first ? vA : vB;
          v3 wa = pts[k].a_is_first ? wA : wB;
          v3 pb = pts[k].a_is_first ? pB : pA, vb = pts[k].a_is_first ? vB : vA;
          v3 wb = pts[k].a_is_first ? wB : wA;
          v3 velA = add(va, cross(wa, sub(xc, pa)));
          v3 vrel;
          if (jj == ORACLE_GROUND) {
            vrel = velA; /* the ground does not move */
          } else {
            v3 velB = add(vb, cross(wb, sub(xc, pb)));
            vrel = sub(velA, velB);
          }
          float vn = dot(vrel, nrm);
          float f = prm->k * pts[k].delta - prm->c * vn;
          if (f < 0.0f) f = 0.0f;
          v3 F = scl(nrm, f);
          if (prm->mu > 0.0f) {
            /* friction: -mu f v_t / max(|v_t|, v_eps), v_t the slip of A on B
             * (regularized Coulomb: at most mu f, opposing the slip) */
            v3 vt = sub(vrel, scl(nrm, vn));
            float st = sqrtf(dot(vt, vt));
            float den = st > prm->v_eps ? st : prm->v_eps;
            float ft = (prm->mu * f) / den;
            F = sub(F, scl(vt, ft));
          }
          v3 Fi = pts[k].a_is_first ? F : neg(F); /* force on the pair's first body */
          SF = add(SF, Fi);
          Ti = add(Ti, cross(sub(xc, pA), Fi));
          if (jj != ORACLE_GROUND) Tj = add(Tj, cross(sub(xc, pB), neg(Fi)));
        }
        acc[i].F = add(acc[i].F, SF);
        acc[i].T = add(acc[i].T, Ti);
        if (jj != ORACLE_GROUND) {
          acc[jj].F = sub(acc[jj].F, SF);
          acc[jj].T = add(acc[jj].T, Tj);
        }
      }
    }
    if (npairs) npairs[s] = np;

    /* Semi-implicit Euler: v then p (with the new v); omega then q. */
    for (int32_t b = 0; b < n; ++b) {
      v3 v = load3(vel, b), p = load3(pos, b), w = load3(omega, b);
      v3 F = acc[b].F;
      if (fext) F = add(F, load3(fext, b)); /* external force, after the contacts */
      v3 a = add(scl(F, inv_m[b]), g);
      v = add(v, scl(a, h));
      p = add(p, scl(v, h));
      if (type[b] == 2 && inertia) {
        /* a box: Euler's equations in the body frame, with the gyroscopic
         * term, R the orientation at the start of the substep:
         * w_b = R^T w, dw_b = (R^T T - w_b x (I w_b)) / I, w = R (w_b + h dw_b) */
        float R[9];
        quat_mat(quat + 4 * b, R);
        v3 I = load3(inertia, b);
        v3 wb = mat_tvec(R, w), tb = mat_tvec(R, acc[b].T);
        v3 L = mk(I.x * wb.x, I.y * wb.y, I.z * wb.z);
        v3 gy = cross(wb, L);
        v3 dwb = mk((tb.x - gy.x) / I.x, (tb.y - gy.y) / I.y, (tb.z - gy.z) / I.z);
        w = mat_vec(R, add(wb, scl(dwb, h)));
      } else {
        w = add(w, scl(scl(acc[b].T, inv_I[b]), h));
      }
      float* q = quat + 4 * b;
      float qw = q[0], qx = q[1], qy = q[2], qz = q[3];
      /* dq = (0, w) (x) q, Hamilton product */
      float dw = (-w.x * qx - w.y * qy) - w.z * qz;
      float dx = (w.x * qw + w.y * qz) - w.z * qy;
      float dy = (w.y * qw + w.z * qx) - w.x * qz;
      float dz = (w.z * qw + w.x * qy) - w.y * qx;
      qw = qw + hh * dw; qx = qx + hh * dx; qy = qy + hh * dy; qz = qz + hh * dz;
      float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
      float inv = 1.0f / sqrtf(n2);
      q[0] = qw * inv; q[1] = qx * inv; q[2] = qy * inv; q[3] = qz * inv;
      vel[3 * b] = v.x; vel[3 * b + 1] = v.y; vel[3 * b + 2] = v.z;
      pos[3 * b] = p.x; pos[3 * b + 1] = p.y; pos[3 * b + 2] = p.z;
      omega[3 * b] = w.x; omega[3 * b + 1] = w.y; omega[3 * b + 2] = w.z;
      if (status == 0 && !(finite3(v) && finite3(p) && finite3(w) && isfinite(q[0]) &&
                           isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3])))
        status = 2;
    }
  }
  free(acc);
  return status;
}

/* ---------------------------------------------------------------------------
 * Rasterizer
 * ------------------------------------------------------------------------- */

int oracle_setup_triangle(const float* w0, const float* w1, const float* w2, const float* vp,
                          int32_t W, int32_t H, float near_w, float guard,
                          int32_t* X, int32_t* Y, float* z, int64_t* area) {
  const float* wv[3] = {w0, w1, w2};
  int32_t Xs[3], Ys[3];
  float zs[3];
  for (int k = 0; k < 3; ++k) {
    float x = wv[k][0], y = wv[k][1], zz = wv[k][2];
    float c[4];
    for (int r = 0; r < 4; ++r)
      c[r] = ((vp[4 * r] * x + vp[4 * r + 1] * y) + vp[4 * r + 2] * zz) + vp[4 * r + 3];
    if (c[3] < near_w) return 0;
    float nx = c[0] / c[3], ny = c[1] / c[3], nz = c[2] / c[3];
    float sx = (nx * 0.5f + 0.5f) * (float)W;
    float sy = (0.5f - ny * 0.5f) * (float)H;
    if (fabsf(sx) > guard || fabsf(sy) > guard) return 0;
    Xs[k] = (int32_t)rintf(sx * 256.0f);
    Ys[k] = (int32_t)rintf(sy * 256.0f);
    zs[k] = nz;
  }
  /* A triangle counter-clockwise in y-up NDC is clockwise in y-down screen
   * space; taking the vertices in the order (0, 2, 1) makes its signed area
   * positive. */
  const int ord[3] = {0, 2, 1};
  for (int k = 0; k < 3; ++k) { X[k] = Xs[ord[k]]; Y[k] = Ys[ord[k]]; z[k] = zs[ord[k]]; }
  int64_t A = (int64_t)(X[1] - X[0]) * (int64_t)(Y[2] - Y[0]) -
              (int64_t)(Y[1] - Y[0]) * (int64_t)(X[2] - X[0]);
  *area = A;
  return A > 0;
}

/* Clip coordinates of a world-space point (the row dot products summed left
 * to right, then the translation). */
static void clip_coords(const float* wv, const float* vp, float* c) {
  float x = wv[0], y = wv[1], zz = wv[2];
  for (int r = 0; r < 4; ++r)
    c[r] = ((vp[4 * r] * x + vp[4 * r + 1] * y) + vp[4 * r + 2] * zz) + vp[4 * r + 3];
}

/* Viewport transform and 24.8 snap of clip coordinates; 0 outside the
 * guard band. */
static int snap_clip(const float* c, int32_t W, int32_t H, float guard, int32_t* X, int32_t* Y, float* z) {
  float nx = c[0] / c[3], ny = c[1] / c[3], nz = c[2] / c[3];
  float sx = (nx * 0.5f + 0.5f) * (float)W;
  float sy = (0.5f - ny * 0.5f) * (float)H;
  if (fabsf(sx) > guard || fabsf(sy) > guard) return 0;
  *X = (int32_t)rintf(sx * 256.0f);
  *Y = (int32_t)rintf(sy * 256.0f);
  *z = nz;
  return 1;
}

/* The point where the edge from `in` (w >= near) to `out` (w < near) meets
 * the plane w = near, always taken from the vertex in front, so that the two
 * triangles sharing an edge cut it at the same point. */
static void near_cut(const float* in, const float* out, float near_w, float* c) {
  float t = (near_w - in[3]) / (out[3] - in[3]);
  for (int r = 0; r < 4; ++r) c[r] = in[r] + t * (out[r] - in[r]);
}

int oracle_setup_clipped(const float* w0, const float* w1, const float* w2, const float* vp,
                         int32_t W, int32_t H, float near_w, float guard,
                         int32_t* X, int32_t* Y, float* z, int64_t* area) {
  const float* wv[3] = {w0, w1, w2};
  float c[3][4];
  int in[3], n_in = 0;
  for (int k = 0; k < 3; ++k) {
    clip_coords(wv[k], vp, c[k]);
    in[k] = !(c[k][3] < near_w);
    n_in += in[k];
  }
  if (n_in == 0) return 0;
  /* a vertex in front but outside the guard band culls the whole triangle */
  int32_t vx[3], vy[3];
  float vz[3];
  for (int k = 0; k < 3; ++k)
    if (in[k] && !snap_clip(c[k], W, H, guard, &vx[k], &vy[k], &vz[k])) return 0;
  /* the polygon in front of the near plane, in the triangle's vertex order:
   * 3 vertices (all in front, or one) or 4 (two in front) */
  float q[4][4];
  int32_t qx[4], qy[4];
  float qz[4];
  int qok[4], m = 0;
  for (int k = 0; k < 3; ++k) {
    int k1 = (k + 1) % 3;
    if (in[k]) {
      memcpy(q[m], c[k], sizeof(q[m]));
      qx[m] = vx[k]; qy[m] = vy[k]; qz[m] = vz[k]; qok[m] = 1;
      ++m;
    }
    if (in[k] != in[k1]) {
      if (in[k]) near_cut(c[k], c[k1], near_w, q[m]);
      else near_cut(c[k1], c[k], near_w, q[m]);
      qok[m] = snap_clip(q[m], W, H, guard, &qx[m], &qy[m], &qz[m]);
      ++m;
    }
  }
  /* fan from the first vertex: (q0, q1, q2), then (q0, q2, q3); each in the
   * order (0, 2, 1) (positive area for a front face) */
  int n = 0;
  for (int s = 0; s + 2 < m; ++s) {
    int idx[3] = {0, s + 2, s + 1};
    if (!(qok[idx[0]] && qok[idx[1]] && qok[idx[2]])) continue;
    int32_t* Xo = X + 3 * n;
    int32_t* Yo = Y + 3 * n;
    float* zo = z + 3 * n;
    for (int k = 0; k < 3; ++k) { Xo[k] = qx[idx[k]]; Yo[k] = qy[idx[k]]; zo[k] = qz[idx[k]]; }
    int64_t A = (int64_t)(Xo[1] - Xo[0]) * (int64_t)(Yo[2] - Yo[0]) -
                (int64_t)(Yo[1] - Yo[0]) * (int64_t)(Xo[2] - Xo[0]);
    if (A <= 0) continue;
    area[n] = A;
    ++n;
  }
  return n;
}

static int64_t edge_fn(int32_t xa, int32_t ya, int32_t xb, int32_t yb, int64_t px, int64_t py) {
  return (int64_t)(xb - xa) * (py - ya) - (int64_t)(yb - ya) * (px - xa);
}

/* top-left edge in y-down screen space, for triangles of positive area */
static int top_left(int32_t xa, int32_t ya, int32_t xb, int32_t yb) {
  int32_t dx = xb - xa, dy = yb - ya;
  return dy < 0 || (dy == 0 && dx > 0);
}

static int edge_in(int64_t E, int32_t xa, int32_t ya, int32_t xb, int32_t yb) {
  return E > 0 || (E == 0 && top_left(xa, ya, xb, yb));
}

int oracle_covers(const int32_t* X, const int32_t* Y, int32_t px, int32_t py) {
  int64_t Px = 256 * (int64_t)px + 128, Py = 256 * (int64_t)py + 128;
  int64_t E0 = edge_fn(X[1], Y[1], X[2], Y[2], Px, Py);
  int64_t E1 = edge_fn(X[2], Y[2], X[0], Y[0], Px, Py);
  int64_t E2 = edge_fn(X[0], Y[0], X[1], Y[1], Px, Py);
  return edge_in(E0, X[1], Y[1], X[2], Y[2]) && edge_in(E1, X[2], Y[2], X[0], Y[0]) &&
         edge_in(E2, X[0], Y[0], X[1], Y[1]);
}

static void raster_snapped(const int32_t* X, const int32_t* Y, const float* z, int64_t A, uint32_t prim,
                           int32_t W, int32_t Hh, uint64_t* keys, int32_t* cover, int32_t* tri_of, int32_t t);

/* A triangle, or with near_clip the part of it in front of the near plane
 * (one or two triangles with the triangle's primitive id). */
static void raster_tri(const float* w0, const float* w1, const float* w2, uint32_t prim,
                       const float* vp, int32_t W, int32_t Hh, const oracle_render_params* rp,
                       uint64_t* keys, int32_t* cover) {
  int32_t X[6], Y[6];
  float z[6];
  int64_t A[2];
  int n;
  if (rp->near_clip) n = oracle_setup_clipped(w0, w1, w2, vp, W, Hh, rp->near_w, rp->guard, X, Y, z, A);
  else n = oracle_setup_triangle(w0, w1, w2, vp, W, Hh, rp->near_w, rp->guard, X, Y, z, A);
  for (int s = 0; s < n; ++s)
    raster_snapped(X + 3 * s, Y + 3 * s, z + 3 * s, A[s], prim, W, Hh, keys, cover, NULL, 0);
}

/* ---------------------------------------------------------------------------
 * Smooth shading (a reading: the paper's renderer shades meshes, the
 * interpolation of attributes across a triangle is the perspective-correct
 * one of any rasterizer).  A visible triangle keeps its snapped vertices in
 * setup order, the reciprocal clip w of each and a normal per vertex (world
 * space).  At a pixel centre with edge values E_k (E_k weights vertex k),
 * the perspective-correct weights are proportional to E_k / w_k; the
 * interpolated normal is their weighted sum, normalized (the common factor
 * cancels), and the pixel takes Lambert shading of it.
 * ------------------------------------------------------------------------- */

typedef struct {
  int32_t X[3], Y[3];
  float iw[3];      /* 1 / clip w of each vertex, setup order */
  float n[3][3];    /* world normal of each vertex, setup order */
  float alb[3];
  float uv[3][2];   /* texture coordinates of each vertex, setup order */
  int32_t textured;
} smooth_tri;

/* Perspective-correct interpolation at the centre of pixel (px, py) of a
 * triangle covering it: the unit normal there (zero if the weighted sum
 * vanishes). */
void oracle_smooth_normal(const int32_t* X, const int32_t* Y, const float* iw, const float* n, int32_t px,
                          int32_t py, float* out) {
  int64_t Px = 256 * (int64_t)px + 128, Py = 256 * (int64_t)py + 128;
  int64_t E[3];
  E[0] = edge_fn(X[1], Y[1], X[2], Y[2], Px, Py);
  E[1] = edge_fn(X[2], Y[2], X[0], Y[0], Px, Py);
  E[2] = edge_fn(X[0], Y[0], X[1], Y[1], Px, Py);
  float u[3];
  for (int k = 0; k < 3; ++k) u[k] = (float)E[k] * iw[k];
  v3 m = mk((u[0] * n[0] + u[1] * n[3]) + u[2] * n[6], (u[0] * n[1] + u[1] * n[4]) + u[2] * n[7],
            (u[0] * n[2] + u[1] * n[5]) + u[2] * n[8]);
  float l2 = dot(m, m);
  if (l2 > 0.0f) {
    float l = sqrtf(l2);
    out[0] = m.x / l; out[1] = m.y / l; out[2] = m.z / l;
  } else {
    out[0] = out[1] = out[2] = 0.0f;
  }
}

/* Texture coordinates, a reading of the paper's textured meshes: the
 * coordinates of a pixel are interpolated with the same perspective-correct
 * weights as the normal, E_k / w_k, here normalized by their sum. */
void oracle_smooth_uv(const int32_t* X, const int32_t* Y, const float* iw, const float* uv, int32_t px,
                      int32_t py, float* out) {
  int64_t Px = 256 * (int64_t)px + 128, Py = 256 * (int64_t)py + 128;
  int64_t E[3];
  E[0] = edge_fn(X[1], Y[1], X[2], Y[2], Px, Py);
  E[1] = edge_fn(X[2], Y[2], X[0], Y[0], Px, Py);
  E[2] = edge_fn(X[0], Y[0], X[1], Y[1], Px, Py);
  float u[3];
  for (int k = 0; k < 3; ++k) u[k] = (float)E[k] * iw[k];
  float s = (u[0] + u[1]) + u[2];
  if (!(s > 0.0f)) {
    out[0] = out[1] = 0.0f;
    return;
  }
  out[0] = ((u[0] * uv[0] + u[1] * uv[2]) + u[2] * uv[4]) / s;
  out[1] = ((u[0] * uv[1] + u[1] * uv[3]) + u[2] * uv[5]) / s;
}

void oracle_cube_face_uv(const oracle_render_params* rp, int32_t f, float* uv) {
  const float* n = rp->cube_n + 3 * f;
  /* the face normal's axis; the other two, in order, are the tangent axes */
  int a = fabsf(n[0]) > 0.5f ? 0 : (fabsf(n[1]) > 0.5f ? 1 : 2);
  int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
  for (int k = 0; k < 3; ++k) {
    const float* v = rp->cube_v + 3 * rp->cube_f[3 * f + k];
    uv[2 * k] = (v[t0] + 1.0f) * 0.5f;
    uv[2 * k + 1] = (v[t1] + 1.0f) * 0.5f;
  }
}

/* The texel under (U, V): the fractional parts select the texel, nearest,
 * the texture repeating in both directions; its RGB / 255. */
static void texel_at(const oracle_render_params* rp, float U, float V, float* t) {
  float fu = U - floorf(U), fv = V - floorf(V);
  if (!(fu >= 0.0f)) fu = 0.0f; /* not a number (coordinates beyond float range) */
  if (!(fv >= 0.0f)) fv = 0.0f;
  int32_t i = (int32_t)(fu * (float)rp->tex_w), j = (int32_t)(fv * (float)rp->tex_h);
  if (i > rp->tex_w - 1) i = rp->tex_w - 1;
  if (j > rp->tex_h - 1) j = rp->tex_h - 1;
  const uint8_t* p = rp->texture + 3 * ((size_t)j * (size_t)rp->tex_w + (size_t)i);
  for (int c = 0; c < 3; ++c) t[c] = (float)p[c] / 255.0f;
}

static void raster_snapped(const int32_t* X, const int32_t* Y, const float* z, int64_t A, uint32_t prim,
                           int32_t W, int32_t Hh, uint64_t* keys, int32_t* cover, int32_t* tri_of, int32_t t) {
  int32_t xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0];
  for (int k = 1; k < 3; ++k) {
    if (X[k] < xmin) xmin = X[k];
    if (X[k] > xmax) xmax = X[k];
    if (Y[k] < ymin) ymin = Y[k];
    if (Y[k] > ymax) ymax = Y[k];
  }
  /* a superset of the pixels whose centres can lie in the bounding box */
  int32_t px0 = (xmin >> 8) - 1, px1 = (xmax >> 8) + 1;
  int32_t py0 = (ymin >> 8) - 1, py1 = (ymax >> 8) + 1;
  if (px0 < 0) px0 = 0;
  if (py0 < 0) py0 = 0;
  if (px1 > W - 1) px1 = W - 1;
  if (py1 > Hh - 1) py1 = Hh - 1;
  float invA = 1.0f / (float)A;
  for (int32_t py = py0; py <= py1; ++py) {
    for (int32_t px = px0; px <= px1; ++px) {
      int64_t Px = 256 * (int64_t)px + 128, Py = 256 * (int64_t)py + 128;
      int64_t E0 = edge_fn(X[1], Y[1], X[2], Y[2], Px, Py);
      int64_t E1 = edge_fn(X[2], Y[2], X[0], Y[0], Px, Py);
      int64_t E2 = edge_fn(X[0], Y[0], X[1], Y[1], Px, Py);
      if (!(edge_in(E0, X[1], Y[1], X[2], Y[2]) && edge_in(E1, X[2], Y[2], X[0], Y[0]) &&
            edge_in(E2, X[0], Y[0], X[1], Y[1])))
        continue;
      size_t pix = (size_t)py * W + px;
      if (cover) cover[pix] += 1;
      /* E0 weights vertex 0, E1 vertex 1, E2 vertex 2 */
      float zz = (((float)E0 * z[0] + (float)E1 * z[1]) + (float)E2 * z[2]) * invA;
      uint32_t D = (uint32_t)rintf(fminf(fmaxf(zz, 0.0f), 1.0f) * 16777215.0f);
      uint64_t key = ((uint64_t)D << 32) | prim;
      if (key < keys[pix]) {
        keys[pix] = key;
        if (tri_of) tri_of[pix] = t;
      }
    }
  }
}

/* Setup and raster of one triangle (world vertices w0..w2 in face order,
 * their normals nv) for smooth shading: the triangle table keeps its
 * snapped vertices, 1 / clip w and normals in setup order (0, 2, 1). */
static int smooth_tri_raster(const float* w0, const float* w1, const float* w2, const float* const nv[3],
                             const float* alb, const float* uvf, uint32_t prim, const float* vp, int32_t W, int32_t H,
                             const oracle_render_params* rp, uint64_t* keys, int32_t* cover, int32_t* tri_of,
                             smooth_tri** tris, int32_t* ntri, int32_t* tcap) {
  int32_t X[3], Y[3];
  float z[3];
  int64_t A;
  if (!oracle_setup_triangle(w0, w1, w2, vp, W, H, rp->near_w, rp->guard, X, Y, z, &A)) return 0;
  if (*ntri == *tcap) {
    smooth_tri* nt = (smooth_tri*)realloc(*tris, sizeof(smooth_tri) * (size_t)(2 * *tcap));
    if (!nt) return -1;
    *tris = nt;
    *tcap *= 2;
  }
  smooth_tri* st = &(*tris)[*ntri];
  const float* wv[3] = {w0, w1, w2};
  const int ord[3] = {0, 2, 1};
  for (int k = 0; k < 3; ++k) {
    float c[4];
    clip_coords(wv[ord[k]], vp, c);
    st->X[k] = X[k];
    st->Y[k] = Y[k];
    st->iw[k] = 1.0f / c[3];
    for (int r = 0; r < 3; ++r) st->n[k][r] = nv[ord[k]][r];
    st->uv[k][0] = uvf ? uvf[2 * ord[k]] : 0.0f;
    st->uv[k][1] = uvf ? uvf[2 * ord[k] + 1] : 0.0f;
  }
  st->textured = uvf != NULL;
  for (int c = 0; c < 3; ++c) st->alb[c] = alb[c];
  raster_snapped(X, Y, z, A, prim, W, H, keys, cover, tri_of, *ntri);
  ++*ntri;
  return 0;
}

int oracle_render_image(int32_t n, const uint8_t* type, const float* size,
                        const uint8_t* albedo, const float* pos, const float* quat,
                        const float* vp, int32_t W, int32_t H, const oracle_render_params* rp,
                        uint8_t* rgb, uint32_t* depth, int32_t* winner, int32_t* cover) {
  return oracle_render_image_box(n, type, size, NULL, albedo, pos, quat, vp, W, H, rp, rgb, depth, winner, cover);
}

int oracle_render_image_box(int32_t n, const uint8_t* type, const float* size, const float* ext,
                            const uint8_t* albedo, const float* pos, const float* quat,
                            const float* vp, int32_t W, int32_t H, const oracle_render_params* rp,
                            uint8_t* rgb, uint32_t* depth, int32_t* winner, int32_t* cover) {
  size_t npix = (size_t)W * (size_t)H;
  if (rp->smooth && rp->near_clip) return -2;
  if (rp->texture && (!rp->smooth || rp->tex_w < 1 || rp->tex_h < 1)) return -2;
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (npix ? npix : 1));
  if (!keys) return -1;
  for (size_t i = 0; i < npix; ++i) keys[i] = UINT64_MAX;
  if (cover) memset(cover, 0, sizeof(int32_t) * npix);
  /* smooth shading: each pixel's winning triangle, and the triangles */
  int32_t* tri_of = NULL;
  smooth_tri* tris = NULL;
  int32_t ntri = 0, tcap = 0;
  if (rp->smooth) {
    tri_of = (int32_t*)malloc(sizeof(int32_t) * (npix ? npix : 1));
    tcap = 64;
    tris = (smooth_tri*)malloc(sizeof(smooth_tri) * (size_t)tcap);
    if (!tri_of || !tris) { free(keys); free(tri_of); free(tris); return -1; }
    for (size_t i = 0; i < npix; ++i) tri_of[i] = -1;
  }

  /* prim ids: 0..ground_nf-1 the ground, then each body's faces in order */
  uint32_t prim = 0;
  for (int f = 0; f < rp->ground_nf; ++f, ++prim) {
    const int32_t* fi = rp->ground_f + 3 * f;
    if (rp->smooth) {
      const float up[3] = {0.0f, 0.0f, 1.0f};
      const float* nv[3] = {up, up, up};
      const float ga[3] = {rp->ground_albedo, rp->ground_albedo, rp->ground_albedo};
      /* the ground's texture coordinates: its world (x, y) scaled */
      float guv[6];
      for (int k = 0; k < 3; ++k) {
        guv[2 * k] = rp->ground_v[3 * fi[k]] * rp->ground_uv_scale;
        guv[2 * k + 1] = rp->ground_v[3 * fi[k] + 1] * rp->ground_uv_scale;
      }
      if (smooth_tri_raster(rp->ground_v + 3 * fi[0], rp->ground_v + 3 * fi[1], rp->ground_v + 3 * fi[2], nv, ga,
                            rp->texture ? guv : NULL, prim, vp, W, H, rp, keys, cover, tri_of, &tris, &ntri,
                            &tcap)) {
        free(keys); free(tri_of); free(tris); return -1;
      }
      continue;
    }
    raster_tri(rp->ground_v + 3 * fi[0], rp->ground_v + 3 * fi[1], rp->ground_v + 3 * fi[2],
               prim, vp, W, H, rp, keys, cover);
  }
  for (int32_t b = 0; b < n; ++b) {
    float R[9];
    quat_mat(quat + 4 * b, R);
    v3 p = load3(pos, b);
    v3 e = body_ext(b, type, size, ext); /* the unit template scaled per axis */
    const float* tv = type[b] ? rp->cube_v : rp->sphere_v;
    const int32_t* tf = type[b] ? rp->cube_f : rp->sphere_f;
    int32_t nf = type[b] ? rp->cube_nf : rp->sphere_nf;
    for (int f = 0; f < nf; ++f, ++prim) {
      float wv[3][3];
      for (int k = 0; k < 3; ++k) {
        v3 t = load3(tv, tf[3 * f + k]);
        v3 w = add(p, mat_vec(R, mk(t.x * e.x, t.y * e.y, t.z * e.z)));
        wv[k][0] = w.x; wv[k][1] = w.y; wv[k][2] = w.z;
      }
      if (rp->smooth) {
        /* vertex normals: a sphere's template vertex (a point of the unit
         * sphere) turned by R; a cube's or box's face normal at every vertex */
        float nvw[3][3];
        for (int k = 0; k < 3; ++k) {
          v3 nb = type[b] ? load3(rp->cube_n, f) : load3(tv, tf[3 * f + k]);
          v3 nw = mat_vec(R, nb);
          nvw[k][0] = nw.x; nvw[k][1] = nw.y; nvw[k][2] = nw.z;
        }
        const float* nv[3] = {nvw[0], nvw[1], nvw[2]};
        float al[3];
        for (int c = 0; c < 3; ++c) al[c] = rp->palette[3 * albedo[b] + c];
        /* cube and box faces are textured over the face's unit square */
        float fuv[6];
        if (type[b]) oracle_cube_face_uv(rp, f, fuv);
        if (smooth_tri_raster(wv[0], wv[1], wv[2], nv, al, (rp->texture && type[b]) ? fuv : NULL, prim, vp, W, H,
                              rp, keys, cover, tri_of, &tris, &ntri, &tcap)) {
          free(keys); free(tri_of); free(tris); return -1;
        }
        continue;
      }
      raster_tri(wv[0], wv[1], wv[2], prim, vp, W, H, rp, keys, cover);
    }
  }

  /* Lambert shading of each pixel's winner */
  v3 L = mk(rp->light[0], rp->light[1], rp->light[2]);
  for (size_t i = 0; i < npix; ++i) {
    uint64_t key = keys[i];
    if (key == UINT64_MAX) {
      rgb[3 * i] = rgb[3 * i + 1] = rgb[3 * i + 2] = 0;
      depth[i] = 0xFFFFFFFFu;
      if (winner) winner[i] = -1;
      continue;
    }
    uint32_t pr = (uint32_t)(key & 0xFFFFFFFFu);
    depth[i] = (uint32_t)(key >> 32);
    if (winner) winner[i] = (int32_t)pr;
    v3 nrm;
    float alb[3];
    if (pr < (uint32_t)rp->ground_nf) {
      nrm = mk(0.0f, 0.0f, 1.0f);
      alb[0] = alb[1] = alb[2] = rp->ground_albedo;
    } else {
      uint32_t rem = pr - (uint32_t)rp->ground_nf;
      int32_t b = 0;
      for (;;) {
        uint32_t nf = (uint32_t)(type[b] ? rp->cube_nf : rp->sphere_nf);
        if (rem < nf) break;
        rem -= nf;
        ++b;
      }
      float R[9];
      quat_mat(quat + 4 * b, R);
      nrm = mat_vec(R, load3(type[b] ? rp->cube_n : rp->sphere_n, (int32_t)rem));
      for (int c = 0; c < 3; ++c) alb[c] = rp->palette[3 * albedo[b] + c];
    }
    if (rp->smooth) {
      /* the winning triangle's interpolated normal at this pixel centre */
      const smooth_tri* st = &tris[tri_of[i]];
      float nn[3];
      oracle_smooth_normal(st->X, st->Y, st->iw, &st->n[0][0], (int32_t)(i % (size_t)W), (int32_t)(i / (size_t)W),
                           nn);
      nrm = mk(nn[0], nn[1], nn[2]);
      for (int c = 0; c < 3; ++c) alb[c] = st->alb[c];
      if (st->textured) {
        /* the albedo times the texel at the pixel's coordinates */
        float uv[2], t[3];
        oracle_smooth_uv(st->X, st->Y, st->iw, &st->uv[0][0], (int32_t)(i % (size_t)W), (int32_t)(i / (size_t)W),
                         uv);
        texel_at(rp, uv[0], uv[1], t);
        for (int c = 0; c < 3; ++c) alb[c] = alb[c] * t[c];
      }
    }
    float l = fmaxf(0.0f, dot(nrm, L));
    for (int c = 0; c < 3; ++c) {
      float col = alb[c] * (0.2f + 0.8f * l);
      rgb[3 * i + c] = (uint8_t)fminf(255.0f, rintf(col * 255.0f));
    }
  }
  free(keys);
  free(tri_of);
  free(tris);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Multi-threaded batch driver (whole envs per thread)
 * ------------------------------------------------------------------------- */

typedef struct {
  int32_t tid, nthreads, n_envs, n_steps, do_render;
  const int32_t* body_off; const uint8_t* type; const float *size, *rbound, *inv_m, *inv_I;
  const uint8_t* albedo; float *pos, *vel, *quat, *omega;
  const oracle_phys_params* prm;
  const int32_t* cam_off; const float* cam_vp; const int32_t *cam_w, *cam_h;
  const int64_t* img_off; const oracle_render_params* rp; uint8_t* rgb; uint32_t* depth;
  int status;
} batch_job;

static void* batch_worker(void* arg) {
  batch_job* j = (batch_job*)arg;
  for (int32_t e = j->tid; e < j->n_envs; e += j->nthreads) {
    int32_t b0 = j->body_off[e], nb = j->body_off[e + 1] - b0;
    for (int32_t t = 0; t < j->n_steps; ++t) {
      int st = oracle_step_env(nb, j->type + b0, j->size + b0, j->rbound + b0, j->inv_m + b0,
                               j->inv_I + b0, j->pos + 3 * b0, j->vel + 3 * b0,
                               j->quat + 4 * b0, j->omega + 3 * b0, j->prm, NULL, 0, NULL);
      if (st && !j->status) j->status = st;
      if (!j->do_render) continue;
      for (int32_t c = j->cam_off[e]; c < j->cam_off[e + 1]; ++c) {
        int64_t o = j->img_off[c];
        oracle_render_image(nb, j->type + b0, j->size + b0, j->albedo + b0, j->pos + 3 * b0,
                            j->quat + 4 * b0, j->cam_vp + 16 * c, j->cam_w[c], j->cam_h[c],
                            j->rp, j->rgb + 3 * o, j->depth + o, NULL, NULL);
      }
    }
  }
  return NULL;
}

int oracle_run_batch(int32_t n_envs, const int32_t* body_off, const uint8_t* type,
                     const float* size, const float* rbound, const float* inv_m,
                     const float* inv_I, const uint8_t* albedo, float* pos, float* vel,
                     float* quat, float* omega, const oracle_phys_params* prm,
                     const int32_t* cam_off, const float* cam_vp, const int32_t* cam_w,
                     const int32_t* cam_h, const int64_t* img_off,
                     const oracle_render_params* rp, uint8_t* rgb, uint32_t* depth,
                     int32_t n_steps, int32_t nthreads, int32_t do_render) {
  if (nthreads < 1) nthreads = 1;
  batch_job* jobs = (batch_job*)calloc((size_t)nthreads, sizeof(batch_job));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  for (int t = 0; t < nthreads; ++t) {
    batch_job* j = &jobs[t];
    j->tid = t; j->nthreads = nthreads; j->n_envs = n_envs; j->n_steps = n_steps;
    j->do_render = do_render;
    j->body_off = body_off; j->type = type; j->size = size; j->rbound = rbound;
    j->inv_m = inv_m; j->inv_I = inv_I; j->albedo = albedo; j->pos = pos; j->vel = vel;
    j->quat = quat; j->omega = omega; j->prm = prm; j->cam_off = cam_off; j->cam_vp = cam_vp;
    j->cam_w = cam_w; j->cam_h = cam_h; j->img_off = img_off; j->rp = rp; j->rgb = rgb;
    j->depth = depth;
    pthread_create(&th[t], NULL, batch_worker, j);
  }
  int status = 0;
  for (int t = 0; t < nthreads; ++t) {
    pthread_join(th[t], NULL);
    if (jobs[t].status && !status) status = jobs[t].status;
  }
  free(jobs);
  free(th);
  return status;
}
