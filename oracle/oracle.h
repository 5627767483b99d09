/*
 * CPU oracle of the batched embodied-AI step: a rigid-body physics step and a
 * software rasterizer, plain single-threaded C, IEEE binary32 throughout.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference
 * that the HIP path is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product library
 * never does.  It shares no code with the HIP path.
 *
 * Build: gcc -O2 -ffp-contract=off (no fast-math): every expression is
 * evaluated exactly as written, left to right, with correctly rounded
 * division and square root and round-to-nearest-even rintf.
 *
 * The paper (VUDA, arXiv 2605.01352) treats the physics engine and the
 * renderer as black boxes (Background, Workload Characterization) and states
 * no algorithm for either; the computation here follows the readings listed
 * in the project's design notes: penalty (spring-dashpot) contact with
 * semi-implicit Euler, and an edge-function rasterizer with 24.8 fixed point,
 * a top-left fill rule and a (depth, primitive id) z-test.
 */
#ifndef VUDA_ORACLE_H
#define VUDA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_GROUND 0xFFFF
#define ORACLE_MAX_POINTS 17
/* Edge-edge contacts: cross products with squared length below this are no
 * axis; an edge axis wins only below this fraction of the least face
 * overlap. */
#define ORACLE_EDGE_PARALLEL 1.0e-6f
#define ORACLE_EDGE_BIAS 0.95f

/* Physics parameters: dt, substeps, contact stiffness k, damping c, gravity;
 * friction coefficient mu (0: none) and the slip speed v_eps below which
 * the regularized Coulomb friction is linear in the slip; edge != 0 adds
 * the separating-axis edge-edge point to box-box contacts. */
typedef struct {
  float dt;
  int32_t substeps;
  float k;
  float c;
  float g[3];
  float mu;
  float v_eps;
  int32_t edge;
} oracle_phys_params;

/* Mesh templates (unit size) and shading constants. */
typedef struct {
  const float* sphere_v; const int32_t* sphere_f; const float* sphere_n;
  int32_t sphere_nv, sphere_nf;
  const float* cube_v; const int32_t* cube_f; const float* cube_n;
  int32_t cube_nv, cube_nf;
  const float* ground_v; const int32_t* ground_f;
  int32_t ground_nf;
  float light[3];
  float palette[24];
  float ground_albedo;
  float near_w;     /* cull a triangle if any vertex has clip w below this */
  float guard;      /* cull a triangle if any |screen coord| exceeds this  */
  int32_t near_clip; /* nonzero: cut triangles crossing w = near_w instead
                        (oracle_setup_clipped) */
  int32_t smooth;    /* nonzero: Lambert shading per pixel of the normal
                        interpolated perspective-correctly from the
                        triangle's vertex normals (not with near_clip) */
  /* Texture (smooth shading only; NULL: none): RGB8 texels [tex_h][tex_w][3].
   * The ground takes texture coordinates (x, y) * ground_uv_scale of its
   * world vertices; a cube or box face takes the unit square over its two
   * tangent axes of the body frame; spheres are not textured.  A textured
   * pixel's albedo is multiplied by its texel (nearest, repeat wrap) / 255
   * at the perspective-correct coordinates (oracle_smooth_uv). */
  const uint8_t* texture;
  int32_t tex_w, tex_h;
  float ground_uv_scale;
} oracle_render_params;

/* One contact point as the narrowphase reports it. */
typedef struct {
  float n[3];      /* unit normal; pushes body "A" along +n */
  float delta;     /* penetration depth, > 0                */
  float xc[3];     /* contact point                         */
  int32_t a_is_first; /* 1 if A is the pair's first body     */
} oracle_point;

/*
 * Advance one env by one step (`substeps` substeps).  Body arrays are the
 * env's slices: pos/vel/omega [n][3], quat [n][4] (w,x,y,z), updated in place.
 * If pairs != NULL, the sorted contact-pair set of every substep is written:
 * pairs[s*pair_cap*2 + 2*k + {0,1}] = (i, j), j = ORACLE_GROUND for ground,
 * and npairs[s] = its size.
 * Returns 0; -1 if a pair list exceeds pair_cap; 2 if the new state holds a
 * non-finite value.
 */
int oracle_step_env(int32_t n, const uint8_t* type, const float* size, const float* rbound,
                    const float* inv_m, const float* inv_I, float* pos, float* vel,
                    float* quat, float* omega, const oracle_phys_params* prm,
                    int32_t* pairs, int32_t pair_cap, int32_t* npairs);

/* The same step with an external force fext[b] (3 floats per body, held over
 * the step's substeps) on every body: it joins the body's force after the
 * contact and ground sums, before the division by the mass.  fext = NULL
 * is the step above. */
int oracle_step_env_ext(int32_t n, const uint8_t* type, const float* size, const float* rbound,
                        const float* inv_m, const float* inv_I, float* pos, float* vel,
                        float* quat, float* omega, const oracle_phys_params* prm,
                        int32_t* pairs, int32_t pair_cap, int32_t* npairs, const float* fext);

/* As oracle_step_env_ext, with boxes: body type 2 is a box of half-extents
 * ext[3b .. 3b+2] (body frame) and principal moments of inertia
 * inertia[3b .. 3b+2]; its angular velocity follows Euler's equations in
 * the body frame, gyroscopic term included (the isotropic sphere and cube
 * keep w += h T inv_I).  ext and inertia may be NULL when there is no box. */
int oracle_step_env_box(int32_t n, const uint8_t* type, const float* size, const float* ext,
                        const float* inertia, const float* rbound, const float* inv_m, const float* inv_I,
                        float* pos, float* vel, float* quat, float* omega, const oracle_phys_params* prm,
                        int32_t* pairs, int32_t pair_cap, int32_t* npairs, const float* fext);

/* Narrowphase of one body pair (i < j) or of body i with the ground
 * (j = ORACLE_GROUND), evaluated on the given state.  Returns the number of
 * contact points written to pts (at most ORACLE_MAX_POINTS). */
int oracle_narrowphase(int32_t i, int32_t j, const uint8_t* type, const float* size,
                       const float* pos, const float* quat, oracle_point* pts);
/* As oracle_narrowphase, with boxes (ext as in oracle_step_env_box, may be
 * NULL) and, for edge != 0, the edge-edge point of two boxes. */
int oracle_narrowphase_box(int32_t i, int32_t j, const uint8_t* type, const float* size, const float* ext,
                           const float* pos, const float* quat, int32_t edge, oracle_point* pts);

/*
 * Render one camera of one env.  rgb [H][W][3] u8, depth [H][W] u32 (24-bit
 * unorm depth, 0xFFFFFFFF background).  winner [H][W] (prim id or -1) and
 * cover [H][W] (number of covering, non-culled triangles) may be NULL.
 */
int oracle_render_image(int32_t n, const uint8_t* type, const float* size,
                        const uint8_t* albedo, const float* pos, const float* quat,
                        const float* vp, int32_t W, int32_t H, const oracle_render_params* rp,
                        uint8_t* rgb, uint32_t* depth, int32_t* winner, int32_t* cover);

/* As oracle_render_image, with boxes (type 2: the cube template scaled by
 * the half-extents ext[3b .. 3b+2]); ext may be NULL when there is no box. */
/* Smooth shading: the unit normal at the centre of pixel (px, py) of a
 * triangle (snapped vertices X, Y in setup order, 1 / clip w per vertex,
 * world normals n[3][3]) interpolated perspective-correctly; zero if the
 * weighted sum vanishes. */
void oracle_smooth_normal(const int32_t* X, const int32_t* Y, const float* iw, const float* n, int32_t px,
                          int32_t py, float* out);

/* Texture coordinates at the centre of pixel (px, py) of a triangle (setup
 * order, 1 / clip w and (u, v) per vertex, uv[3][2]) interpolated
 * perspective-correctly: the weights E_k / w_k normalized by their sum;
 * (0, 0) if the sum is not positive. */
void oracle_smooth_uv(const int32_t* X, const int32_t* Y, const float* iw, const float* uv, int32_t px,
                      int32_t py, float* out);

/* The face-corner texture coordinates of face f of the cube template
 * (corner k of the face in face order): the corner's template coordinates
 * on the two tangent axes of the face normal (y, z for x faces; x, z for y
 * faces; x, y for z faces), mapped from [-1, 1] to [0, 1]. */
void oracle_cube_face_uv(const oracle_render_params* rp, int32_t f, float* uv);

int oracle_render_image_box(int32_t n, const uint8_t* type, const float* size, const float* ext,
                            const uint8_t* albedo, const float* pos, const float* quat,
                            const float* vp, int32_t W, int32_t H, const oracle_render_params* rp,
                            uint8_t* rgb, uint32_t* depth, int32_t* winner, int32_t* cover);

/* Screen-space setup of one triangle given world-space vertices: writes the
 * snapped 24.8 vertices (in edge order) and depths; returns 1 if the triangle
 * survives culling, 0 otherwise.  Exposed for the coverage pins. */
int oracle_setup_triangle(const float* w0, const float* w1, const float* w2, const float* vp,
                          int32_t W, int32_t H, float near_w, float guard,
                          int32_t* X, int32_t* Y, float* z, int64_t* area);

/* Setup with near-plane clipping: the part of the triangle (world-space
 * vertices in template order) in front of the plane clip w = near_w, as 0,
 * 1 or 2 triangles of positive area.  A vertex in front but outside the
 * guard band culls the whole triangle; an edge crossing the plane is cut at
 * in + t (out - in), t = (near_w - w_in) / (w_out - w_in), from its vertex in
 * front; the polygon is split as a fan from its first vertex, and a piece
 * with a cut point outside the guard band is dropped.  Writes triangle s to
 * X, Y, z [3 s .. 3 s + 2] (edge order) and area[s]; returns their count. */
int oracle_setup_clipped(const float* w0, const float* w1, const float* w2, const float* vp,
                         int32_t W, int32_t H, float near_w, float guard,
                         int32_t* X, int32_t* Y, float* z, int64_t* area);

/* Coverage of one snapped triangle (vertices in edge order, area > 0) at a
 * pixel centre (256*px+128, 256*py+128).  Returns 1 if covered. */
int oracle_covers(const int32_t* X, const int32_t* Y, int32_t px, int32_t py);

/*
 * Whole-batch driver for the CPU baseline: runs n_steps of (physics step of
 * every env, then render every camera of every env), sharding whole envs over
 * nthreads POSIX threads; the per-env work is the single-threaded code above.
 * Body arrays are global (env-major) with offsets body_off[E+1]; cameras
 * cam_off[E+1], cam_vp [C][16], cam_w/cam_h [C]; image outputs are packed at
 * pixel offsets img_off[C].  Returns 0 or the first nonzero per-env status.
 */
int oracle_run_batch(int32_t n_envs, const int32_t* body_off, const uint8_t* type,
                     const float* size, const float* rbound, const float* inv_m,
                     const float* inv_I, const uint8_t* albedo, float* pos, float* vel,
                     float* quat, float* omega, const oracle_phys_params* prm,
                     const int32_t* cam_off, const float* cam_vp, const int32_t* cam_w,
                     const int32_t* cam_h, const int64_t* img_off,
                     const oracle_render_params* rp, uint8_t* rgb, uint32_t* depth,
                     int32_t n_steps, int32_t nthreads, int32_t do_render);

#ifdef __cplusplus
}
#endif
#endif
