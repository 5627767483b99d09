/*
 * vuda.h -- C ABI of the MI355X co-scheduled physics + render step loop.
 *
 * The loop being accelerated is the phased step of a batched embodied-AI
 * simulator: a physics step (compute) followed by a camera render of every
 * environment (graphics), which the paper shows leaves one kind of GPU
 * resource idle in each phase (Background, Workload Characterization).  Its
 * remedy is to run the two phases spatially side by side on one GPU over a
 * shared address space with no copy between them (Introduction; System
 * Mechanisms).  On gfx950 both phases are HIP kernels in one process: the
 * render kernel reads the physics state buffer in place, and the spatial
 * partition is a pair of CU-masked HIP streams.
 *
 * The entry points mirror the paper's interface table (VUDA Programming
 * Interface, API Surface, Table 1):
 *   vuda_cosched(split)        ~ CUstream_bind / CUstream_unbind
 *   vuda_step / vuda_render    ~ step_async / render_async (enqueue, return)
 *   vuda_wait(phase)           ~ wait_step / wait_render
 * and add world creation, result fetch and the serving admission calls.
 *
 * Conventions shared by every call:
 *  - Return value: VUDA_OK (0) or a negative VUDA_E* code; the thread-local
 *    detail is vuda_last_error_message().  No C++ exception crosses the ABI.
 *  - Device faults and kernel-detected conditions (non-finite state, contact
 *    or bin capacity overflow) are asynchronous and surface at the next
 *    vuda_wait / vuda_fetch of the world.
 *  - A world is used from one host thread at a time.
 *  - Host pointers passed in are read during the call only; the library
 *    copies what it keeps.
 */
#ifndef VUDA_H
#define VUDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define VUDA_OK         0
#define VUDA_EINVAL    -1  /* malformed argument or descriptor              */
#define VUDA_ENOMEM    -2  /* device allocation failed or HBM budget exceeded */
#define VUDA_EHIP      -3  /* a HIP runtime call failed (code in message)    */
#define VUDA_ENUMERIC  -4  /* a physics step produced a non-finite state     */
#define VUDA_EOVERFLOW -5  /* contact-pair, bin or near-plane piece capacity exceeded */
#define VUDA_EBUSY     -6  /* slots or budget not available right now        */

/* ---- phases (vuda_wait, vuda_get_stream) ------------------------------- */
#define VUDA_PHASE_STEP   1
#define VUDA_PHASE_RENDER 2
#define VUDA_PHASE_ALL    3

/* ---- vuda_fetch selectors ---------------------------------------------- */
#define VUDA_FETCH_STATE    0 /* float [n_bodies][13]: px py pz vx vy vz qw qx qy qz wx wy wz */
#define VUDA_FETCH_RGB      1 /* uint8 per camera [H][W][3], cameras in order           */
#define VUDA_FETCH_DEPTH    2 /* uint32 per camera [H][W] (24-bit unorm; 0xFFFFFFFF = none) */
#define VUDA_FETCH_CONTACTS 3 /* int32 per env [substeps][1 + 2*pair_cap]: count, then
                                 (i, j) pairs sorted, ground j = 0xFFFF (debug worlds)   */
#define VUDA_FETCH_WINNERS  4 /* int32 per camera [H][W]: winning primitive id, -1 none
                                 (debug worlds)                                        */
#define VUDA_FETCH_COVERAGE 5 /* int32 per camera [H][W]: covering triangles (debug)    */
#define VUDA_FETCH_FLAGS    6 /* uint32 per env: bit0 non-finite, bit1 contact overflow,
                                 bit2 bin overflow, bit3 more than 64 near-plane pieces
                                 in one image                                          */
#define VUDA_FETCH_ACTIONS  7 /* float per env [3 act_bodies]: the policy's last actions
                                 (zeros before the first vuda_act); needs a policy     */
#define VUDA_FETCH_DEPTH_METRIC 8 /* float per camera [H][W]: view depth [m] along the
                                 camera axis, +inf where no surface (vuda_fetch)        */

/* ---- world flags -------------------------------------------------------- */
#define VUDA_FLAG_DEBUG 1u  /* keep contact sets, winners and coverage for fetch */
#define VUDA_FLAG_NEAR_CLIP 2u /* cut triangles that cross the near plane into the
                                  part in front (one or two pieces, at most 64 per
                                  image, else VUDA_EOVERFLOW) instead of culling
                                  them whole; images are otherwise unchanged    */
#define VUDA_FLAG_SMOOTH 4u    /* smooth shading: each pixel takes Lambert shading
                                  of the vertex normals of its winning triangle
                                  interpolated perspective-correctly (weights
                                  E_k / w_k: edge value over clip w), normalized;
                                  a sphere's vertex normal is its template vertex
                                  turned by the body's rotation, a cube's or box's
                                  the face normal, the ground's +z.  Winners,
                                  depth and coverage are those of flat shading.
                                  Not with VUDA_FLAG_NEAR_CLIP (VUDA_EINVAL)     */
#define VUDA_FLAG_TEXTURE 8u   /* with VUDA_FLAG_SMOOTH: the render description's
                                  texture on the ground and on cube and box
                                  faces.  A textured pixel's albedo is multiplied
                                  by the texel (nearest, repeating) / 255 at the
                                  pixel centre's texture coordinates, interpolated
                                  with the same perspective-correct weights
                                  E_k / w_k normalized by their sum.  The ground's
                                  coordinates are its world (x, y) times
                                  ground_uv_scale; a cube or box face spans the
                                  unit square over its two tangent axes of the
                                  body frame (y, z for x faces; x, z for y faces;
                                  x, y for z faces, each mapped from [-1, 1]);
                                  spheres are not textured.  Without
                                  VUDA_FLAG_SMOOTH, or without a valid texture:
                                  VUDA_EINVAL                                   */

typedef struct vuda_world vuda_world;

/* Optional device allocator (e.g. PyTorch's caching allocator).  alloc
 * returns device memory of at least `bytes` (256-byte aligned) or NULL. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} vuda_allocator;

/* Physics constants: step dt [s] split in `substeps` substeps of dt/substeps;
 * penalty contact f = max(0, k*delta - c*v_n); gravity [m/s^2].  Friction
 * (regularized Coulomb): at each contact point the tangential relative
 * velocity v_t adds -mu f v_t / max(|v_t|, v_eps) to the normal force f n,
 * so that |F_t| <= mu f, reached once the point slides faster than v_eps;
 * mu = 0 turns it off (the frictionless step, bit for bit).  The force is
 * explicit in each substep: below v_eps it acts as a viscous drag of slope
 * mu f / v_eps, stable for v_eps above about 4 mu |g| h (h the substep;
 * 0.05 m/s covers mu <= 1 at h = 1/960 s), while a body on a slope of
 * angle theta < atan(mu) creeps at v_eps tan(theta) / mu.  VUDA_EINVAL
 * for mu negative or non-finite, or v_eps not positive and finite while
 * mu > 0.
 *
 * edge_contacts = 1 adds, to the vertex-in-box points of two boxes or
 * cubes, one edge-edge point found by the separating-axis test over the
 * 15 axes of the pair (each box's 3 axes, then the 9 cross products of an
 * axis of the first with one of the second, skipped when the two axes are
 * within 1e-3 rad of parallel).  No axis may separate the boxes, and the
 * least overlap over the cross products must be below 0.95 times the least
 * over the face axes; the point is where the two supporting edges pass
 * closest, with that overlap as depth and that axis as normal (pointing
 * from the second body to the first).  0 keeps vertex-only box contacts,
 * which miss two edges crossing with no vertex inside the other box.
 * Other values: VUDA_EINVAL. */
typedef struct {
  float dt;
  int32_t substeps;
  float k_contact;
  float c_damp;
  float gravity[3];
  float mu;     /* friction coefficient (0: none)                  */
  float v_eps;  /* [m/s] slip speed below which friction is linear */
  int32_t edge_contacts;  /* 1: box-box edge-edge points (0: off) */
} vuda_phys_params;

/* Unit mesh templates and shading constants.  Faces are vertex-index
 * triples wound counter-clockwise seen from outside; normals are per face. */
typedef struct {
  const float* sphere_v; int32_t sphere_nv;   /* [nv][3], nv <= 64         */
  const int32_t* sphere_f; const float* sphere_n; int32_t sphere_nf; /* nf <= 128 */
  const float* cube_v; int32_t cube_nv;       /* [nv][3], nv <= 64         */
  const int32_t* cube_f; const float* cube_n; int32_t cube_nf;
  const float* ground_v; int32_t ground_nv;   /* world-space ground polygon    */
  const int32_t* ground_f; int32_t ground_nf;
  float light[3];        /* unit direction towards the light */
  float palette[24];     /* 8 RGB albedos, indexed by body albedo index */
  float ground_albedo;
  float near_w;          /* triangles with a vertex at clip w < near_w are culled */
  float guard;           /* ... or with |screen coordinate| > guard (pixels)      */
  /* VUDA_FLAG_TEXTURE only (else ignored): RGB8 texels [texture_h][texture_w][3],
   * row-major, copied at creation; 1 <= texture_w, texture_h <= 4096;
   * ground_uv_scale: texture repeats per metre of ground (finite) */
  const uint8_t* texture;
  int32_t texture_w, texture_h;
  float ground_uv_scale;
} vuda_render_desc;

/*
 * Per-env content.  Bodies of env e are body_off[e] .. body_off[e+1]-1
 * (at most 128 per env); cameras cam_off[e] .. cam_off[e+1]-1.
 * Body arrays: type (0 sphere, 1 cube, 2 box), size (radius, half-extent,
 * or a box's largest half-extent), rbound (bounding-sphere radius), inv_m,
 * inv_I (isotropic; unused for a box), albedo (palette index 0..7),
 * pos/vel/omega [B][3], quat [B][4] (w,x,y,z).  Boxes also need ext [B][3]
 * (half-extents along the body axes) and inertia [B][3] (principal moments
 * about them); their rows for other bodies are not read, and both may be
 * NULL when there is no box.  A box's spin follows Euler's equations in the
 * body frame, gyroscopic term included.
 * Cameras: vp [C][16] row-major view-projection (clip = vp * [x y z 1]^T,
 * depth in [0,1]), w/h in pixels (1..4096).
 */
typedef struct {
  int32_t n_envs;
  const int32_t* body_off;
  const uint8_t* type; const float* size; const float* rbound;
  const float* inv_m; const float* inv_I; const uint8_t* albedo;
  const float* pos; const float* vel; const float* quat; const float* omega;
  const int32_t* cam_off; const float* cam_vp; const int32_t* cam_w; const int32_t* cam_h;
  const float* ext; const float* inertia;
} vuda_env_batch;

/*
 * World descriptor.  `initial` holds the envs created with the world (may
 * have n_envs = 0 for a serving world that admits envs later).  The
 * capacities reserve room for envs admitted later: 0 means "exactly the
 * initial envs".  hbm_budget (bytes, 0 = unlimited) bounds the device arena.
 * pair_cap is the per-env, per-substep capacity of the debug contact sets.
 */
typedef struct {
  vuda_phys_params phys;
  vuda_render_desc render;
  vuda_env_batch initial;
  uint32_t flags;          /* VUDA_FLAG_* */
  int32_t cap_envs;        /* max env slots                  */
  int64_t cap_bodies;      /* max bodies over all slots      */
  int32_t cap_cams;        /* max cameras over all slots     */
  int64_t cap_pixels;      /* max pixels over all cameras    */
  int32_t pair_cap;        /* debug contact-set capacity (default 1024) */
  uint64_t hbm_budget;
} vuda_world_desc;

/* Create a world: validates the descriptor, allocates one device arena
 * (through `alloc` if non-NULL, else hipMalloc), uploads static data and
 * the initial state, and creates its streams on the current HIP device.
 * Errors: VUDA_EINVAL (descriptor), VUDA_ENOMEM (allocation or budget), no
 * partial world is left behind. */
int vuda_create_world(const vuda_world_desc* desc, const vuda_allocator* alloc, vuda_world** out);

/* Wait for all work of the world, then free its device memory and streams. */
int vuda_destroy_world(vuda_world* w);

/*
 * Co-scheduling switch (the paper's stream bind/unbind).  0 < cu_split < 1:
 * the step phase runs on a stream restricted to that fraction of the CUs and
 * the render phase on a stream restricted to the rest (hipExtStreamCreate-
 * WithCUMask, balanced over the XCDs); cu_split == 2 runs them on streams
 * over every CU (masks of all CUs, so that each stream has a hardware queue
 * of its own); cu_split <= 0 or == 1 restores the serialized path (one
 * stream, every phase in enqueue order).  Changing it only moves work
 * between CUs: outputs are bit-identical in every mode.  Drains the world
 * before switching.  The co-scheduled streams are blocking streams: work
 * the caller puts on the null stream waits for them.
 */
int vuda_cosched(vuda_world* w, float cu_split);

/*
 * Enqueue `nsteps` physics steps of envs [env_lo, env_hi) and return (the
 * paper's step_async).  Step t of an env reads its state buffer t%2 and
 * writes (t+1)%2.  Dependencies are stream-ordered: the step waits for the
 * last enqueued step of the world (state read) and the last enqueued render
 * (which may read the buffer being overwritten).  All envs of the range must
 * have taken the same number of steps modulo 2 (VUDA_EINVAL otherwise).
 */
int vuda_step(vuda_world* w, int32_t env_lo, int32_t env_hi, int32_t nsteps);

/*
 * Enqueue the render of every camera of envs [env_lo, env_hi) from their
 * latest enqueued state (the paper's render_async): waits for the last
 * enqueued step that writes that state; may overlap a later step that only
 * reads it (inter-step pipelining).  Outputs RGB8 and 24-bit depth.
 */
int vuda_render(vuda_world* w, int32_t env_lo, int32_t env_hi);

/* Block until the enqueued work of `phase` (VUDA_PHASE_*) is complete, then
 * report asynchronous errors (VUDA_ENUMERIC, VUDA_EOVERFLOW, VUDA_EHIP). */
int vuda_wait(vuda_world* w, int32_t phase);

/*
 * Copy results of envs [env_lo, env_hi) into dst (`dst_bytes` long; host
 * memory, or device memory if dst_on_device).  Stream-ordered after all
 * enqueued work, and synchronous on return.  The layout is given with the
 * VUDA_FETCH_* selectors; fetch size queries: vuda_fetch_bytes.
 *
 * VUDA_FETCH_DEPTH_METRIC converts the 24-bit depth on the GPU: a camera
 * whose view-projection rows satisfy row2 = alpha row3 + beta e4 (every
 * perspective of the usual form, Vulkan or OpenGL depth) gives the view
 * depth w = beta / (D / (2^24 - 1) - alpha) in float64, rounded to float32.
 * Its error is the 24-bit quantization of D: about d^2 / |beta| 2^-24 at
 * depth d.  VUDA_EINVAL for a camera of another form.  A host dst goes
 * through a device staging buffer that the world keeps (grown as needed).
 */
int vuda_fetch(vuda_world* w, int32_t what, int32_t env_lo, int32_t env_hi, void* dst,
               size_t dst_bytes, int32_t dst_on_device);
int vuda_fetch_bytes(vuda_world* w, int32_t what, int32_t env_lo, int32_t env_hi, size_t* bytes);

/* Overwrite the current state of envs [env_lo, env_hi) with `src` (host,
 * float [n][13] as VUDA_FETCH_STATE); used for checkpoint/resume and for
 * parity checks from an identical input state. */
int vuda_load_state(vuda_world* w, int32_t env_lo, int32_t env_hi, const float* src,
                    size_t src_bytes);

/* The HIP stream (hipStream_t) of a phase, for interop (e.g. an external
 * stream object in PyTorch).  Valid until the next vuda_cosched call. */
int vuda_get_stream(vuda_world* w, int32_t phase, void** hip_stream);

/*
 * Serving: admit the envs of one request into free slots of a world created
 * with spare capacity.  The request's envs take `batch->n_envs` consecutive
 * slots starting at *first_env; their state is written to buffer `parity`
 * (so that they step in lockstep with envs of that parity).  Returns
 * VUDA_EBUSY if no run of free slots, bodies or pixels is large enough or
 * the HBM budget would be exceeded; nothing is changed then.
 */
int vuda_admit(vuda_world* w, const vuda_env_batch* batch, int32_t parity, int32_t* first_env);

/* Free the slots [first_env, first_env + n_envs) of an admitted request
 * (stream-ordered after all enqueued work on them). */
int vuda_release(vuda_world* w, int32_t first_env, int32_t n_envs);

/* World shape queries. */
int vuda_world_info(vuda_world* w, int32_t* n_envs, int64_t* n_bodies, int32_t* n_cams,
                    int64_t* n_pixels, uint64_t* arena_bytes);

/*
 * Launch-shape knobs (the autotuner's search space).  Keys:
 *   VUDA_TUNE_RASTER_THREADS   raster workgroup size, multiple of 64 (default 256)
 *   VUDA_TUNE_REC_CAP          tile-bin entries an image may use (0: its whole
 *                              capacity, 4 per primitive of its env); an image
 *                              needing more is rendered without bins, each
 *                              tile testing every visible triangle (slower,
 *                              same output)
 *   VUDA_TUNE_PHYS_PERSISTENT  0: one workgroup per env; n > 0: n resident
 *                              workgroups pulling envs from a device queue;
 *                              VUDA_PERSISTENT_RESIDENT (-1): as many
 *                              workgroups as the GPU holds at once (the
 *                              kernel's occupancy per CU times the CU count)
 *   VUDA_TUNE_RASTER_PERSISTENT  the same for camera images
 *   VUDA_TUNE_GRAPHS           1: each (phase, env range, parity) launch is
 *                              captured once into a hipGraph and replayed
 *   VUDA_TUNE_PHYS_PRIORITY    0..3: instruction-issue priority of the step's
 *                              waves (physics, and the raster setup that ends
 *                              a step with VUDA_TUNE_PRESETUP) relative to the
 *                              render's tile waves on shared CUs
 *   VUDA_TUNE_BROADPHASE       0 automatic (all pairs up to 64 bodies, uniform
 *                              grid hash above), 1 grid hash, 2 all pairs;
 *                              both give the same candidate set
 *   VUDA_TUNE_TIMING           1: record a HIP event pair around every kernel
 *                              launch on the stream it runs on (read with
 *                              vuda_kernel_times); 0: off (default)
 *   VUDA_TUNE_PRESETUP         1 (default): vuda_step ends with the raster
 *                              setup of the state it produced, on the step
 *                              stream, so that vuda_render only rasterizes;
 *                              0: vuda_render does both.  A render of a state
 *                              without setup (after creation, vuda_load_state
 *                              or a step with this off) does its own setup
 *   VUDA_TUNE_POLICY_LAYERED   1: layers 2 and 3 of the policy run as batched
 *                              float32 MFMA products over all envs at any
 *                              hidden size (a multiple of 64; vuda_act returns
 *                              VUDA_EINVAL otherwise); 0 (default): only above
 *                              hidden 1024, the per-env head kernel below.
 *                              Changes the float32 summation order of layers
 *                              2 and 3 (the actions stay within the same
 *                              error bound of the exact ones)
 *   VUDA_TUNE_PHYS_ENVS_PER_WAVE  1 (default) or 2: envs of at most 32 bodies
 *                              per physics wave (two envs share a wave, one
 *                              in each half, when every env of a launch has
 *                              at most 32 bodies)
 *   VUDA_TUNE_TILE_SIZE        8, 16 (default) or 32: edge in pixels of the
 *                              raster tiles (binning and one tile-kernel wave
 *                              per tile); changing it waits for queued work
 *                              and redoes the raster setup of current states
 *   VUDA_TUNE_RASTER_FUSED     1: vuda_render runs setup and tiles of an image
 *                              in one workgroup (VUDA_TUNE_RASTER_THREADS
 *                              threads) that keeps its setup records, bins and
 *                              tile table in LDS, so that they never reach
 *                              HBM, and vuda_step does no raster setup; worlds
 *                              with smooth shading or near-plane clipping, and
 *                              envs too large for LDS, keep the two kernels.
 *                              0 (default): setup and tile kernels
 *   VUDA_TUNE_FUSED_LDS_RECORDS  fused raster: 0 (default) keeps up to half
 *                              the env's primitives plus 64 records of an
 *                              image in LDS (less if LDS is short), n > 0 at
 *                              most n (with 4 bin entries each; less LDS per
 *                              workgroup); an image with more records or bin
 *                              entries passes them through the raster scratch
 *   VUDA_TUNE_TILE_WAVES       1, 2 (default) or 4: tiles of a row per tile-kernel
 *                              workgroup, one per wave (smaller workgroups fit
 *                              beside the step's on shared CUs)
 *   VUDA_TUNE_TILE_PRIORITY    0..3: instruction-issue priority of the tile
 *                              kernel's waves relative to the step's
 * None of the others changes any output bit.  Returns VUDA_EINVAL for unknown keys
 * or out-of-range values.
 */
#define VUDA_TUNE_RASTER_THREADS 1
#define VUDA_TUNE_REC_CAP 2
#define VUDA_TUNE_PHYS_PERSISTENT 3
#define VUDA_TUNE_RASTER_PERSISTENT 4
#define VUDA_PERSISTENT_RESIDENT (-1) /* persistent grid sized to the GPU's resident workgroups */
#define VUDA_TUNE_GRAPHS 5
#define VUDA_TUNE_PHYS_PRIORITY 6
#define VUDA_TUNE_BROADPHASE 7
#define VUDA_TUNE_TIMING 8
#define VUDA_TUNE_PRESETUP 9
#define VUDA_TUNE_POLICY_LAYERED 10
#define VUDA_TUNE_PHYS_ENVS_PER_WAVE 11
#define VUDA_TUNE_TILE_SIZE 12
#define VUDA_TUNE_RASTER_FUSED 13
#define VUDA_TUNE_FUSED_LDS_RECORDS 14
#define VUDA_TUNE_TILE_WAVES 15
#define VUDA_TUNE_TILE_PRIORITY 16
int vuda_set_tuning(vuda_world* w, int32_t key, int32_t value);
int vuda_get_tuning(vuda_world* w, int32_t key, int32_t* value);

/*
 * Kernel durations recorded while VUDA_TUNE_TIMING is on.  `kernel` is
 * VUDA_KERNEL_PHYSICS (the step), VUDA_KERNEL_RASTER_SETUP (vertex
 * transform, triangle setup and tile binning of a state; part of the step
 * with VUDA_TUNE_PRESETUP, else of the render) or VUDA_KERNEL_RASTER_TILES
 * (the pixels, part of the render) or VUDA_KERNEL_POLICY (layer 1 and the
 * head of vuda_act) or VUDA_KERNEL_RASTER_FUSED (setup and pixels in one
 * kernel, the render with VUDA_TUNE_RASTER_FUSED).  Waits for the last recorded launch of
 * that kernel, then returns the number of launches since the previous call
 * for it and the sum and maximum of their durations in milliseconds -- GPU
 * time between an event recorded on the launch's stream just before the
 * kernel (after the stream's waits were satisfied) and one just after it
 * (including its queue reset when persistent) -- and starts a new count.
 * Any output pointer may be NULL.
 */
#define VUDA_KERNEL_PHYSICS 1
#define VUDA_KERNEL_RASTER_SETUP 2
#define VUDA_KERNEL_RASTER_TILES 3
#define VUDA_KERNEL_POLICY 4
#define VUDA_KERNEL_RASTER_FUSED 5
int vuda_kernel_times(vuda_world* w, int32_t kernel, int64_t* launches, double* total_ms,
                      double* max_ms);

/*
 * MLP policy: the RL rollout's third phase beside physics and rendering
 * (paper: Evaluation, RL Training, MLP-based RL; the paper gives no
 * architecture, the one here is a reading).  The observation of an env is
 * its camera 0 frame as K = 4 in_w in_h integers 0..255: the RGB bytes in
 * memory order (row-major pixels, R G B), then the top byte of each pixel's
 * 24-bit depth (background: 255).  Then
 *   h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3,
 *   a = a_max clamp(y, -1, 1),
 * and a[3b .. 3b+2] is an external force (N) on body b (b < act_bodies and
 * below the env's body count), added to the body's contact forces on every
 * substep of each following vuda_step until the next vuda_act.  Layer 1 runs
 * in bfloat16 products (exact: 8-bit inputs) with float32 sums; layers 2 and
 * 3 in float32 (per env up to hidden 1024, as batched MFMA products above,
 * and at any hidden size with VUDA_TUNE_POLICY_LAYERED).
 *
 * vuda_policy_set copies the weights (the caller keeps ownership of desc and
 * its arrays) and clears every env's actions; desc = NULL removes the policy
 * and the forces.  It waits for the world's queued work.  VUDA_EINVAL for a
 * frame whose pixel count is not a multiple of 32, hidden outside 1..8192
 * or above 1024 and not a multiple of 64, act_bodies outside 1..1024, a_max negative or non-finite, null arrays or
 * non-finite weights; VUDA_ENOMEM when the device buffers (weights, and
 * cap_envs x 3 act_bodies floats of actions) do not fit.  vuda_act grows
 * the policy's float32 workspace when a launch needs more (draining the
 * world's queued work first): layer-1 partial sums, splits x envs x H
 * floats, splits chosen so that the launch fills the GPU once, plus for the
 * layered head h1 and h2 (2 x envs x H).
 *
 * vuda_act enqueues the policy on the active envs in [env_lo, env_hi), on
 * the step stream after the renders of their current state, and returns;
 * a later render of those envs waits for it.  Every such env needs a camera
 * 0 of in_w x in_h pixels whose frame starts at a pixel offset that is a
 * multiple of 8 (VUDA_EINVAL otherwise, or without a policy).
 */
typedef struct {
  int32_t in_w, in_h;        /* camera-0 frame the policy reads                   */
  int32_t hidden;            /* H                                                 */
  int32_t act_bodies;        /* B: 3 B actions                                    */
  float a_max;               /* force bound (N)                                   */
  const uint16_t* w1;        /* bfloat16 bits, [4 in_w in_h][H] row-major          */
  const float* b1;           /* [H]                                               */
  const float* w2;           /* [H][H] row-major                                  */
  const float* b2;           /* [H]                                               */
  const float* w3;           /* [H][3 B] row-major                                */
  const float* b3;           /* [3 B]                                             */
} vuda_policy_desc;
int vuda_policy_set(vuda_world* w, const vuda_policy_desc* desc);
int vuda_act(vuda_world* w, int32_t env_lo, int32_t env_hi);

/*
 * vuda_act without allocation, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid it).  Same policy, same kernels and the same actions bit for bit as
 * vuda_act over the same envs; it calls no hipMalloc or hipFree.  Its
 * workspace is a static device array of the library, one per GPU, held from
 * the first world on that GPU until the process ends: up to 16,384 env ids
 * and 64 MiB of float32 layer-1 partial sums (with h1 and h2 of the layered
 * head) -- enough for 1,024 envs at 128x128 and hidden 4096, or 4,096 envs
 * at 256x256 and hidden 256.  A launch that needs more returns VUDA_EINVAL
 * (use vuda_act).  Every env in [env_lo, env_hi) must be active (else
 * VUDA_EINVAL).  Calls of this function on one GPU share the workspace: two
 * of them in flight at once on different streams (two worlds, or two
 * threads) race; one world's calls are ordered on its step stream.
 */
int vuda_act_noalloc(vuda_world* w, int32_t env_lo, int32_t env_hi);

/*
 * Placement probe: launches n_blocks one-wave workgroups on the stream of
 * `phase` (VUDA_PHASE_STEP or VUDA_PHASE_RENDER), each spinning for about
 * spin_us microseconds so that they spread over the CUs the stream may use,
 * and writes per block the hardware XCC id, shader-engine id and CU id into
 * out[3*i .. 3*i+2] (host memory, 3*n_blocks int32).  Used to verify the CU
 * partition of vuda_cosched.  Synchronous.
 */
int vuda_probe_placement(vuda_world* w, int32_t phase, int32_t n_blocks, int32_t spin_us,
                         int32_t* out);

/* ---- schedules (vuda_run, autotuner, serving) -------------------------- */
#define VUDA_SCHED_SERIAL    0  /* step then render, one stream                    */
#define VUDA_SCHED_INTERSTEP 1  /* render S_t beside step S_t -> S_t+1 (double
                                   buffered), the paper's inter-step pipelining     */
#define VUDA_SCHED_INTERTRAJ 2  /* envs split in two halves: step(A) beside
                                   render(B), then step(B) beside render(A), the
                                   paper's inter-trajectory parallelism             */
#define VUDA_SCHED_PIPELINED 3  /* three stages on three streams: tiles of S_t
                                   beside the raster setup of S_t+1 beside the
                                   step S_t+1 -> S_t+2, each stage waiting only
                                   for the previous iteration; the same steps
                                   and frames as VUDA_SCHED_INTERSTEP (inter-step
                                   order on one stream or with the fused raster) */

/*
 * Enqueue `iters` iterations of a schedule over every active env: each
 * iteration advances every env one step and renders it once (Parallelism
 * Patterns: inter-step and inter-trajectory overlap).  Uses the current
 * co-scheduling mode; with VUDA_SCHED_SERIAL the phases follow each other.
 * After the call the frames show the state before the last step (the
 * inter-step and pipelined schedules) or after it (serial; inter-trajectory:
 * after it for the first half of the envs, before it for the second).
 * All active envs must have the same step parity.
 */
int vuda_run(vuda_world* w, int32_t schedule, int32_t iters);

/*
 * Autotuner: searches the launch shapes (schedule, CU split, physics and
 * raster persistent grids and workgroup shapes, raster tile size, physics
 * envs per wave, fused raster, tile-kernel workgroup, hipGraph replay,
 * physics and tile priorities, broadphase, presetup) for the highest
 * co-scheduled env-steps/s on this world.  A trial of a candidate is the
 * median of three runs of `steps_per_trial` iterations, each from the
 * current state after 3 warmup iterations (the state is saved before and
 * restored after, so results are unchanged); a candidate replaces the
 * incumbent only when faster by more than 1%.  Coordinate descent over
 * all of them, then a second descent per schedule over its split, workgroup
 * shapes, envs per wave and priorities; each schedule's result, the first
 * descent's and the serialized baseline are timed again, three trials each,
 * and the best median is chosen (VUDA_SCHED_SERIAL where nothing
 * co-scheduled beats it; its rate is reported as cosched_env_steps_per_s).
 * A world's unmasked streams (split 2) have hardware queues of their own, so
 * the choice does not depend on what other streams the process holds.  It
 * applies the best, and
 * records it in the text file `cache_path` (may be NULL) keyed by the GPU
 * architecture and the world's shape; a later call with the same key applies
 * the cached choice without trials.  Also reports the best serialized rate.
 */
typedef struct {
  float cu_split;            /* chosen split: (0,1) CU-masked, 2 every CU on each stream */
  int32_t schedule;          /* VUDA_SCHED_* */
  int32_t raster_threads, rec_cap, phys_persistent, raster_persistent, phys_priority, broadphase;
  double cosched_env_steps_per_s;
  double serial_env_steps_per_s;
  int32_t serial_raster_threads, serial_phys_persistent;
  int32_t trials;            /* 0 when taken from the cache */
  int32_t presetup;          /* VUDA_TUNE_PRESETUP chosen */
  int32_t graphs;            /* VUDA_TUNE_GRAPHS chosen */
  int32_t phys_envs_per_wave; /* VUDA_TUNE_PHYS_ENVS_PER_WAVE chosen */
  int32_t tile_size;         /* VUDA_TUNE_TILE_SIZE chosen */
  int32_t raster_fused;      /* VUDA_TUNE_RASTER_FUSED chosen */
  int32_t tile_waves;        /* VUDA_TUNE_TILE_WAVES chosen */
  int32_t tile_priority;     /* VUDA_TUNE_TILE_PRIORITY chosen */
} vuda_tune_result;
int vuda_autotune(vuda_world* w, int32_t steps_per_trial, const char* cache_path, vuda_tune_result* out);

/*
 * Serving with continuous batching.  A server owns a world created with spare
 * capacity (desc->initial may be empty).  Requests (envs + horizon) are
 * queued by vuda_serve_submit, which refuses (VUDA_EINVAL) a request that is
 * malformed or larger than the world's capacity or the budget.  Each
 * vuda_serve_tick:
 *   1. completes the ticks enqueued earlier that have finished on the GPU
 *      (and waits for the oldest one while two are in flight): their
 *      env-steps count as served, and the requests whose last step they
 *      held complete, their memory released;
 *   2. admits queued requests in FIFO order while env slots, bodies,
 *      cameras and pixels are free and the reserved bytes stay within
 *      desc->hbm_budget; admission does not wait for running work;
 *   3. enqueues k co-scheduled iterations (every running env steps and is
 *      rendered k times), k = the fewest steps a running request has left,
 *      at most 8, and returns without waiting for them.  A request whose
 *      last step is enqueued leaves every later launch; with keep_results its
 *      final state and a frame of it are fetched then (that fetch waits).
 * Latency is completion time (the host sees its last tick finished) minus
 * submit time (host monotonic clock).  A request that admission refuses for
 * a reason other than capacity is dropped and counted in `rejected`.
 */
typedef struct vuda_server vuda_server;
typedef struct {
  int64_t submitted, admitted, completed, queued, active_requests, active_envs;
  int64_t env_steps;             /* env-steps served so far                    */
  int64_t ticks;
  double busy_s;                 /* time inside vuda_serve_tick               */
  double latency_p50_s, latency_p99_s, latency_max_s, latency_mean_s;
  double queue_p50_s, queue_p99_s; /* submit -> admission                     */
  uint64_t reserved_bytes, peak_reserved_bytes;
  int64_t rejected;              /* dropped at admission (malformed)          */
} vuda_serve_stats_t;
int vuda_serve_create(const vuda_world_desc* desc, float cu_split, int32_t schedule,
                      int32_t keep_results, vuda_server** out);
int vuda_serve_destroy(vuda_server* s);
int vuda_serve_submit(vuda_server* s, int64_t request_id, const vuda_env_batch* envs, int32_t horizon);
int vuda_serve_tick(vuda_server* s, int32_t* n_completed);
/* Pop up to cap completed request ids (and their latencies, seconds). */
int vuda_serve_completed(vuda_server* s, int64_t* ids, double* latency_s, int32_t cap, int32_t* n);
/* Kept result of a completed request: what = VUDA_FETCH_STATE, _RGB or _DEPTH;
 * *need receives the size; dst may be NULL to query it. */
int vuda_serve_result(vuda_server* s, int64_t request_id, int32_t what, void* dst, size_t bytes,
                      size_t* need);
int vuda_serve_stats(vuda_server* s, vuda_serve_stats_t* out);
/* The server's world (for tuning knobs and the autotuner). */
int vuda_serve_world(vuda_server* s, vuda_world** w);

const char* vuda_strerror(int code);
const char* vuda_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif
