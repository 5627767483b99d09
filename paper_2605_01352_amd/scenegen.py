"""Seeded synthetic scene generator: the inputs of the step loop.

This module produces input data only -- initial body state, static body
parameters, mesh templates, cameras and light -- and holds none of the
physics or raster arithmetic.  Both the CPU oracle and the HIP path consume
exactly the arrays built here.

The paper runs ManiSkill3 scenes on SAPIEN/PhysX (Evaluation, Experimental
Setup); those assets are not available, so seeded synthetic drops of spheres
and cubes of the same batch shapes stand in for them.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw k of a stream keyed by (config seed, global env id, stream id)
is mix64(x0 + (k+1)*GAMMA).  An env's content therefore never depends on its
position in a batch.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

SPHERE = 0
CUBE = 1
BOX = 2

# random streams per env
ST_SHAPE, ST_POS, ST_ROT, ST_CAM, ST_COUNT, ST_RES, ST_BOX, ST_TEX = 0, 1, 2, 3, 4, 5, 6, 7


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser (vectorised, wrapping uint64 arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, env_gid, stream: int) -> np.ndarray:
    """Initial SplitMix64 state of the stream (seed, env, stream)."""
    e = np.asarray(env_gid, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = (np.uint64(seed) << np.uint64(40)) ^ (e << np.uint64(8)) ^ np.uint64(stream)
        return mix64(x)


def draw_u64(key: np.ndarray, counter) -> np.ndarray:
    """Draw number `counter` (0-based) of the stream with state `key`."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + (c + np.uint64(1)) * GAMMA)


def draw_unit(key, counter) -> np.ndarray:
    """Uniform double in [0, 1) from the top 53 bits of a draw."""
    return (draw_u64(key, counter) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# --------------------------------------------------------------------------
# Mesh templates
# --------------------------------------------------------------------------

def _orient_outward(verts: np.ndarray, faces: List[tuple]) -> List[tuple]:
    out = []
    for a, b, c in faces:
        n = np.cross(verts[b] - verts[a], verts[c] - verts[a])
        cen = (verts[a] + verts[b] + verts[c]) / 3.0
        out.append((a, b, c) if np.dot(n, cen) > 0 else (a, c, b))
    return out


def icosphere_template():
    """Unit icosphere: icosahedron with one midpoint subdivision (42 v, 80 f).

    Vertices lie on the unit sphere; faces wind counter-clockwise seen from
    outside.  Returns (verts f64 [42,3], faces int [80,3]).
    """
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    base = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            base.append((0.0, s1, s2 * phi))
            base.append((s1, s2 * phi, 0.0))
            base.append((s2 * phi, 0.0, s1))
    v = np.array(base, dtype=np.float64)
    nv = len(v)
    tris = []
    for a in range(nv):
        for b in range(a + 1, nv):
            if abs(np.linalg.norm(v[a] - v[b]) - 2.0) > 1e-9:
                continue
            for c in range(b + 1, nv):
                if (abs(np.linalg.norm(v[a] - v[c]) - 2.0) < 1e-9
                        and abs(np.linalg.norm(v[b] - v[c]) - 2.0) < 1e-9):
                    tris.append((a, b, c))
    assert len(tris) == 20
    tris = _orient_outward(v, tris)
    verts = [tuple(x) for x in v]
    mid: Dict[tuple, int] = {}

    def midpoint(i, j):
        key = (min(i, j), max(i, j))
        if key not in mid:
            m = (np.array(verts[i]) + np.array(verts[j])) / 2.0
            verts.append(tuple(m))
            mid[key] = len(verts) - 1
        return mid[key]

    faces = []
    for a, b, c in tris:
        ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
        faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
    vv = np.array(verts, dtype=np.float64)
    vv /= np.linalg.norm(vv, axis=1, keepdims=True)
    faces = _orient_outward(vv, faces)
    return vv, np.array(faces, dtype=np.int32)


def cube_template():
    """Unit cube (+-1)^3: vertex k has sign +1 on axis a iff bit a of k is set.

    12 faces, counter-clockwise seen from outside.
    """
    v = np.array([[1.0 if (k >> a) & 1 else -1.0 for a in range(3)] for k in range(8)])
    faces = []
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            quad = [k for k in range(8) if v[k, axis] == sgn]
            o = [a for a in range(3) if a != axis]
            # order the 4 corners around the face centre
            ang = [math.atan2(v[k, o[1]], v[k, o[0]]) for k in quad]
            quad = [q for _, q in sorted(zip(ang, quad))]
            faces += [(quad[0], quad[1], quad[2]), (quad[0], quad[2], quad[3])]
    faces = _orient_outward(v, faces)
    return v, np.array(faces, dtype=np.int32)


def ground_template():
    """Ground quad [-1,1]^2 at z = 0, two triangles facing +z."""
    v = np.array([[-1.0, -1.0, 0.0], [1.0, -1.0, 0.0], [1.0, 1.0, 0.0], [-1.0, 1.0, 0.0]])
    f = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return v, f


def face_normals(v: np.ndarray, f: np.ndarray) -> np.ndarray:
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


@dataclasses.dataclass
class Templates:
    sphere_v: np.ndarray  # f32 [42,3]
    sphere_f: np.ndarray  # i32 [80,3]
    sphere_n: np.ndarray  # f32 [80,3]
    cube_v: np.ndarray    # f32 [8,3]
    cube_f: np.ndarray    # i32 [12,3]
    cube_n: np.ndarray    # f32 [12,3]
    ground_v: np.ndarray  # f32 [4,3]
    ground_f: np.ndarray  # i32 [2,3]


_TEMPLATES: Optional[Templates] = None


def templates() -> Templates:
    global _TEMPLATES
    if _TEMPLATES is None:
        sv, sf = icosphere_template()
        cv, cf = cube_template()
        gv, gf = ground_template()
        _TEMPLATES = Templates(
            sv.astype(np.float32), sf, face_normals(sv, sf).astype(np.float32),
            cv.astype(np.float32), cf, face_normals(cv, cf).astype(np.float32),
            gv.astype(np.float32), gf)
    return _TEMPLATES


# --------------------------------------------------------------------------
# Cameras
# --------------------------------------------------------------------------

NEAR = 0.05
FAR = 10.0
FOVY_DEG = 60.0
TARGET = (0.0, 0.0, 0.3)
FIXED_EYE = (1.5, 0.0, 1.0)


def view_proj(eye, target=TARGET, up=(0.0, 0.0, 1.0), fovy_deg=FOVY_DEG,
              aspect=1.0, near=NEAR, far=FAR) -> np.ndarray:
    """Right-handed look-at times a perspective with Vulkan [0,1] depth.

    Computed in double and rounded to f32, row-major, acting on column
    vectors (clip = VP @ [x, y, z, 1]).  NDC y points up; depth is
    z_ndc = far*(d-near) / (d*(far-near)) for view distance d.
    """
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, np.asarray(up, np.float64))
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    V = np.eye(4)
    V[0, :3], V[1, :3], V[2, :3] = s, u, -f
    V[0, 3], V[1, 3], V[2, 3] = -s @ eye, -u @ eye, f @ eye
    fy = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    P = np.zeros((4, 4))
    P[0, 0] = fy / aspect
    P[1, 1] = fy
    P[2, 2] = -far / (far - near)
    P[2, 3] = -far * near / (far - near)
    P[3, 2] = -1.0
    return (P @ V).astype(np.float32)


LIGHT = (np.array([0.4, -0.3, 0.866]) / np.linalg.norm([0.4, -0.3, 0.866])).astype(np.float32)
PALETTE = np.array([
    [0.90, 0.20, 0.20], [0.20, 0.75, 0.25], [0.20, 0.35, 0.90], [0.95, 0.80, 0.15],
    [0.80, 0.30, 0.85], [0.15, 0.80, 0.80], [0.95, 0.55, 0.15], [0.70, 0.70, 0.70],
], dtype=np.float32)
GROUND_ALBEDO = np.float32(0.6)
GUARD_BAND = 8192.0


# --------------------------------------------------------------------------
# Scene container
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Scene:
    """A batch of envs, structure-of-arrays over a global body index.

    Bodies of env e are body_off[e] .. body_off[e+1]-1 (env-major);
    cameras of env e are cam_off[e] .. cam_off[e+1]-1.
    """
    body_off: np.ndarray   # i32 [E+1]
    btype: np.ndarray      # u8 [B]  0 sphere, 1 cube
    size: np.ndarray       # f32 [B] radius or cube half-extent
    rbound: np.ndarray     # f32 [B] bounding-sphere radius
    inv_m: np.ndarray      # f32 [B]
    inv_I: np.ndarray      # f32 [B]
    albedo: np.ndarray     # u8 [B] palette index
    pos: np.ndarray        # f32 [B,3]
    vel: np.ndarray        # f32 [B,3]
    quat: np.ndarray       # f32 [B,4] (w, x, y, z)
    omega: np.ndarray      # f32 [B,3]
    cam_off: np.ndarray    # i32 [E+1]
    cam_vp: np.ndarray     # f32 [C,16] row-major
    cam_w: np.ndarray      # i32 [C]
    cam_h: np.ndarray      # i32 [C]
    dt: float = 1.0 / 240.0
    substeps: int = 4
    k_contact: float = 1.0e4
    c_damp: float = 10.0
    gravity: tuple = (0.0, 0.0, -9.81)
    mu: float = 0.0        # regularized Coulomb friction coefficient (0: none)
    v_eps: float = 0.05    # [m/s] slip speed below which friction is linear
    edge_contacts: bool = False  # box-box edge-edge points (separating-axis test)
    near_clip: bool = False  # cut triangles crossing the near plane instead of culling them
    smooth: bool = False  # per-pixel Lambert shading of the interpolated vertex normal
    # texture (with smooth): RGB8 texels [h, w, 3] on the ground and on cube and box faces
    texture: Optional[np.ndarray] = None
    ground_uv_scale: float = 1.0  # texture repeats per metre of ground
    # boxes (type 2): half-extents and principal moments of inertia, body frame
    ext: Optional[np.ndarray] = None      # f32 [B,3] (rows of other bodies unused)
    inertia: Optional[np.ndarray] = None  # f32 [B,3]
    name: str = ""
    seed: int = 0
    env_gid0: int = 0

    @property
    def n_envs(self) -> int:
        return len(self.body_off) - 1

    @property
    def n_bodies(self) -> int:
        return int(self.body_off[-1])

    @property
    def n_cams(self) -> int:
        return int(self.cam_off[-1])

    def counts(self) -> np.ndarray:
        return np.diff(self.body_off)

    def state(self) -> Dict[str, np.ndarray]:
        return dict(pos=self.pos.copy(), vel=self.vel.copy(),
                    quat=self.quat.copy(), omega=self.omega.copy())

    def subset(self, envs: Sequence[int]) -> "Scene":
        """Scene restricted to the given envs (same per-env content)."""
        envs = list(envs)
        bsel = np.concatenate([np.arange(self.body_off[e], self.body_off[e + 1]) for e in envs]) \
            if envs else np.zeros(0, np.int64)
        csel = np.concatenate([np.arange(self.cam_off[e], self.cam_off[e + 1]) for e in envs]) \
            if envs else np.zeros(0, np.int64)
        nb = np.array([0] + [self.body_off[e + 1] - self.body_off[e] for e in envs]).cumsum()
        nc = np.array([0] + [self.cam_off[e + 1] - self.cam_off[e] for e in envs]).cumsum()
        return dataclasses.replace(
            self, body_off=nb.astype(np.int32), btype=self.btype[bsel], size=self.size[bsel],
            rbound=self.rbound[bsel], inv_m=self.inv_m[bsel], inv_I=self.inv_I[bsel],
            albedo=self.albedo[bsel], pos=self.pos[bsel].copy(), vel=self.vel[bsel].copy(),
            quat=self.quat[bsel].copy(), omega=self.omega[bsel].copy(),
            cam_off=nc.astype(np.int32), cam_vp=self.cam_vp[csel], cam_w=self.cam_w[csel],
            cam_h=self.cam_h[csel], ext=None if self.ext is None else self.ext[bsel],
            inertia=None if self.inertia is None else self.inertia[bsel])

    @staticmethod
    def concat(scenes: Sequence["Scene"]) -> "Scene":
        s0 = scenes[0]
        nb = np.concatenate([[0]] + [s.counts() for s in scenes]).cumsum().astype(np.int32)
        nc = np.concatenate([[0]] + [np.diff(s.cam_off) for s in scenes]).cumsum().astype(np.int32)
        cat = lambda f: np.concatenate([getattr(s, f) for s in scenes])
        boxes = any(s.ext is not None for s in scenes)
        cat3 = lambda f: np.concatenate([getattr(s, f) if getattr(s, f) is not None
                                         else np.zeros((s.n_bodies, 3), np.float32) for s in scenes])
        return dataclasses.replace(
            s0, body_off=nb, btype=cat("btype"), size=cat("size"), rbound=cat("rbound"),
            inv_m=cat("inv_m"), inv_I=cat("inv_I"), albedo=cat("albedo"), pos=cat("pos"),
            vel=cat("vel"), quat=cat("quat"), omega=cat("omega"), cam_off=nc,
            cam_vp=cat("cam_vp"), cam_w=cat("cam_w"), cam_h=cat("cam_h"), name="concat",
            ext=cat3("ext") if boxes else None, inertia=cat3("inertia") if boxes else None)


# --------------------------------------------------------------------------
# Generators
# --------------------------------------------------------------------------

SQRT3 = math.sqrt(3.0)


def _shapes(seed, gids, counts, mixed: bool):
    """Per-body type, size, bounding radius, inverse mass and inertia."""
    E = len(gids)
    B = int(counts.sum())
    env_of = np.repeat(np.arange(E), counts)
    local = np.arange(B) - np.repeat(np.concatenate([[0], np.cumsum(counts)[:-1]]), counts)
    key = stream_key(seed, np.asarray(gids, np.uint64)[env_of], ST_SHAPE)
    u = draw_unit(key, local.astype(np.uint64))
    btype = np.where(mixed & (local % 2 == 1), CUBE, SPHERE).astype(np.uint8)
    size64 = np.where(btype == SPHERE, 0.05 + 0.10 * u, 0.03 + 0.09 * u)
    size = size64.astype(np.float32)
    s = size.astype(np.float64)
    # bounding radius slightly inflated so rounding of R(q) never leaves it
    rb = np.where(btype == SPHERE, s, s * SQRT3 * (1.0 + 1e-6)).astype(np.float32)
    inv_m = np.ones(B, np.float32)
    inv_I = np.where(btype == SPHERE, 1.0 / (0.4 * s * s), 1.0 / ((2.0 / 3.0) * s * s)).astype(np.float32)
    albedo = (local % 8).astype(np.uint8)
    return env_of, local, btype, size, rb, inv_m, inv_I, albedo


def _place(seed, gids, counts, rb, env_of, local, box_h_min: float = 1.0, batch: int = 32):
    """Rejection-sample non-overlapping centres in a box, per env.

    x, y ~ U[-0.5+R, 0.5-R], z ~ U[R, H-R]; H = max(1, V_bound/0.25); after
    1000 failed tries for one body H grows by 0.25 m.  Tries consume three
    draws each, in order; `batch` tries are evaluated at once and the first
    acceptable one is kept, which gives the same result as trying one by one.
    """
    E = len(gids)
    B = len(rb)
    off = np.concatenate([[0], np.cumsum(counts)])
    rb64 = rb.astype(np.float64)
    vol = np.zeros(E)
    np.add.at(vol, env_of, 4.0 / 3.0 * math.pi * rb64 ** 3)
    H = np.maximum(box_h_min, vol / 0.25)
    key = stream_key(seed, np.asarray(gids, np.uint64), ST_POS)
    native = _placement_lib()
    if native is not None and E:
        import ctypes as C
        pos = np.zeros((B, 3))
        a = lambda x, t: np.ascontiguousarray(x, t)
        off64, cnt64 = a(off[:-1], np.int64), a(counts, np.int64)
        keys, H0, R = a(key, np.uint64), a(H, np.float64), a(rb64, np.float64)
        ptr = lambda x: x.ctypes.data_as(C.c_void_p)
        native.place_envs(C.c_int64(E), ptr(off64), ptr(cnt64), ptr(keys), ptr(H0), ptr(R), ptr(pos))
        return pos.astype(np.float32)
    ctr = np.zeros(E, np.uint64)
    pos = np.zeros((B, 3))
    nmax = int(counts.max()) if E else 0
    tries = np.zeros(E, np.int64)
    for k in range(nmax):
        pending = np.nonzero(counts > k)[0]
        tries[pending] = 0
        while len(pending):
            n = len(pending)
            T = np.minimum(batch, 1000 - tries[pending])          # tries before H may grow
            t_idx = np.arange(batch)[None, :]
            c0 = ctr[pending][:, None] + np.uint64(3) * t_idx.astype(np.uint64)
            kk = key[pending][:, None]
            ux, uy, uz = draw_unit(kk, c0), draw_unit(kk, c0 + np.uint64(1)), draw_unit(kk, c0 + np.uint64(2))
            bi = off[pending] + k
            R = rb64[bi][:, None]
            cand = np.stack([-0.5 + R + (1.0 - 2.0 * R) * ux,
                             -0.5 + R + (1.0 - 2.0 * R) * uy,
                             R + (H[pending][:, None] - 2.0 * R) * uz], axis=2)   # [n, batch, 3]
            ok = t_idx < T[:, None]
            if k > 0:
                idx = off[pending][:, None] + np.arange(k)[None, :]
                diff = pos[idx][:, None, :, :] - cand[:, :, None, :]
                d2 = np.einsum("ntkc,ntkc->ntk", diff, diff)
                rs = rb64[idx][:, None, :] + R[:, :, None]
                ok &= np.all(d2 > rs * rs, axis=2)
            anyok = ok.any(axis=1)
            first = np.argmax(ok, axis=1)
            used = np.where(anyok, first + 1, T)
            ctr[pending] += np.uint64(3) * used.astype(np.uint64)
            tries[pending] += used
            acc = pending[anyok]
            pos[off[acc] + k] = cand[np.nonzero(anyok)[0], first[anyok]]
            fail = pending[~anyok]
            grow = tries[fail] >= 1000
            H[fail[grow]] += 0.25
            tries[fail[grow]] = 0
            pending = fail
    return pos.astype(np.float32)


_PLACE_LIB = []


def _placement_lib():
    """The compiled placement (placement.c, same draws and arithmetic as the
    numpy loop below), if it has been built; else None."""
    if not _PLACE_LIB:
        import ctypes as C
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libplace.so")
        lib = None
        if os.path.exists(path) and not os.environ.get("VUDA_NUMPY_PLACEMENT"):
            lib = C.CDLL(path)
            lib.place_envs.restype = None
        _PLACE_LIB.append(lib)
    return _PLACE_LIB[0]


def _place_chunk(args):
    seed, gids, counts, rb, env_of, local = args
    return _place(seed, gids, counts, rb, env_of, local)


def _place_parallel(seed, gids, counts, rb, env_of, local, workers: int):
    """_place over contiguous chunks of envs in `workers` processes.  Each
    env draws from its own stream, so the result equals _place's.  The
    processes are started fresh (spawn), never forked from the caller."""
    import concurrent.futures as cf
    import multiprocessing as mp
    E = len(gids)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    bounds = np.linspace(0, E, workers + 1).astype(np.int64)
    jobs = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        if b > a:
            sl = slice(int(off[a]), int(off[b]))
            jobs.append((seed, gids[a:b], counts[a:b], rb[sl], env_of[sl] - a, local[sl]))
    with cf.ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_place_chunk, jobs))
    return np.concatenate(parts) if parts else np.zeros((0, 3), np.float32)


def _orientations(seed, gids, btype, env_of, local):
    """Shoemake uniform random rotations for cubes; identity for spheres."""
    key = stream_key(seed, np.asarray(gids, np.uint64)[env_of], ST_ROT)
    c = (local.astype(np.uint64) * np.uint64(3))
    u1, u2, u3 = draw_unit(key, c), draw_unit(key, c + np.uint64(1)), draw_unit(key, c + np.uint64(2))
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([b * np.cos(2 * math.pi * u3), a * np.sin(2 * math.pi * u2),
                  a * np.cos(2 * math.pi * u2), b * np.sin(2 * math.pi * u3)], axis=1)
    q[btype == SPHERE] = (1.0, 0.0, 0.0, 0.0)
    return q.astype(np.float32)


def make_scene(seed: int, counts, res, mixed: bool, cams_per_env: int = 1,
               ring: bool = False, env_gid0: int = 0, name: str = "", workers: int = 1) -> Scene:
    """Build a scene of len(counts) envs.

    counts: bodies per env; res: per-env square resolution (int or array).
    ring: cameras at seeded poses on a 1.5 m ring (else one fixed pose).
    workers: processes for the rejection-sampled placement when the compiled
    placement is not built (same result).
    """
    counts = np.asarray(counts, np.int64)
    E = len(counts)
    gids = np.arange(env_gid0, env_gid0 + E, dtype=np.uint64)
    res = np.broadcast_to(np.asarray(res, np.int64), (E,))
    env_of, local, btype, size, rb, inv_m, inv_I, albedo = _shapes(seed, gids, counts, mixed)
    if workers > 1 and E >= 2 * workers and _placement_lib() is None:
        pos = _place_parallel(seed, gids, counts, rb, env_of, local, workers)
    else:
        pos = _place(seed, gids, counts, rb, env_of, local)
    quat = _orientations(seed, gids, btype, env_of, local)
    B = len(btype)
    C = E * cams_per_env
    vps = np.zeros((C, 16), np.float32)
    if ring:
        key = stream_key(seed, gids, ST_CAM)
        for c in range(cams_per_env):
            th = 2.0 * math.pi * draw_unit(key, np.full(E, 2 * c, np.uint64))
            hh = 0.5 + draw_unit(key, np.full(E, 2 * c + 1, np.uint64))
            for e in range(E):
                eye = (1.5 * math.cos(th[e]), 1.5 * math.sin(th[e]), hh[e])
                vps[e * cams_per_env + c] = view_proj(eye).reshape(16)
    else:
        vps[:] = view_proj(FIXED_EYE).reshape(16)
    cw = np.repeat(res, cams_per_env).astype(np.int32)
    return Scene(
        body_off=np.concatenate([[0], np.cumsum(counts)]).astype(np.int32),
        btype=btype, size=size, rbound=rb, inv_m=inv_m, inv_I=inv_I, albedo=albedo,
        pos=pos, vel=np.zeros((B, 3), np.float32), quat=quat,
        omega=np.zeros((B, 3), np.float32),
        cam_off=(np.arange(E + 1) * cams_per_env).astype(np.int32),
        cam_vp=vps, cam_w=cw, cam_h=cw.copy(), name=name, seed=seed, env_gid0=env_gid0)


def poisson_knuth(key, lam: float) -> np.ndarray:
    """Knuth's multiplicative Poisson sampler, vectorised over streams."""
    L = math.exp(-lam)
    n = len(key)
    k = np.zeros(n, np.int64)
    p = np.ones(n)
    ctr = np.zeros(n, np.uint64)
    alive = np.ones(n, bool)
    while alive.any():
        idx = np.nonzero(alive)[0]
        p[idx] *= draw_unit(key[idx], ctr[idx])
        ctr[idx] += np.uint64(1)
        done = p[idx] <= L
        k[idx[~done]] += 1
        alive[idx[done]] = False
    return k


# Seeds per config: config i uses 1000 + i.
CONFIG_SEEDS = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005}
CONFIG_STEPS = {1: 100, 2: 500, 3: 200, 4: 300}


def config_scene(cfg: int, n_envs: Optional[int] = None, env_gid0: int = 0, workers: int = 1) -> Scene:
    """The synthetic workloads (optionally only the first n_envs envs).

    1: 16 envs x 8 spheres, one 64x64 camera, fixed pose.
    2: 1024 envs x 32 bodies (half spheres, half cubes), 128x128, fixed pose.
    3: 4096 envs x 64 bodies, two 256x256 ring cameras per env.
    4: 2048 envs, bodies ~ clamp(Poisson(24), 4, 128), res in {64,128,256}.
    """
    seed = CONFIG_SEEDS[cfg]
    full = {1: 16, 2: 1024, 3: 4096, 4: 2048}[cfg]
    E = full if n_envs is None else n_envs
    gids = np.arange(env_gid0, env_gid0 + E, dtype=np.uint64)
    if cfg == 1:
        return make_scene(seed, np.full(E, 8), 64, mixed=False, env_gid0=env_gid0, name="c1")
    if cfg == 2:
        return make_scene(seed, np.full(E, 32), 128, mixed=True, env_gid0=env_gid0, name="c2", workers=workers)
    if cfg == 3:
        return make_scene(seed, np.full(E, 64), 256, mixed=True, cams_per_env=2, ring=True,
                          env_gid0=env_gid0, name="c3", workers=workers)
    if cfg == 4:
        kc = stream_key(seed, gids, ST_COUNT)
        counts = np.clip(poisson_knuth(kc, 24.0), 4, 128)
        kr = stream_key(seed, gids, ST_RES)
        res = np.array([64, 128, 256])[(draw_unit(kr, np.zeros(E, np.uint64)) * 3).astype(np.int64)]
        return make_scene(seed, counts, res, mixed=True, env_gid0=env_gid0, name="c4", workers=workers)
    raise ValueError(f"no scene for config {cfg}")


def with_boxes(scene: Scene, every: int = 2, seed: int = 2029) -> Scene:
    """The scene with every `every`-th cube (in body order) made a box.

    A cube of half-extent a becomes a box of half-extents (a, a s1, a s2),
    s1, s2 uniform in [0.4, 1), in its body axes, with the principal moments
    of a solid box of the cube's mass; its bounding radius shrinks to the
    box's half-diagonal, so the placement stays overlap-free.
    """
    B = scene.n_bodies
    cubes = np.flatnonzero(scene.btype == CUBE)[::every]
    key = stream_key(seed, np.arange(B, dtype=np.uint64), ST_BOX)
    s1 = 0.4 + 0.6 * draw_unit(key, np.zeros(B, np.uint64))
    s2 = 0.4 + 0.6 * draw_unit(key, np.ones(B, np.uint64))
    a = scene.size.astype(np.float64)
    btype = scene.btype.copy()
    btype[cubes] = BOX
    ext = np.stack([a, a * s1, a * s2], 1)
    ext[btype != BOX] = a[btype != BOX, None]
    m = 1.0 / scene.inv_m.astype(np.float64)
    e2 = ext ** 2
    inertia = m[:, None] / 3.0 * np.stack([e2[:, 1] + e2[:, 2], e2[:, 0] + e2[:, 2], e2[:, 0] + e2[:, 1]], 1)
    rb = scene.rbound.copy()
    rb[cubes] = (np.linalg.norm(ext[cubes], axis=1) * (1.0 + 1e-6)).astype(np.float32)
    return dataclasses.replace(scene, btype=btype, rbound=rb, ext=ext.astype(np.float32),
                               inertia=inertia.astype(np.float32), name=scene.name + "+boxes")


def procedural_texture(w: int = 32, h: int = 32, seed: int = 2031) -> np.ndarray:
    """A seeded RGB8 texture [h, w, 3]: a checkerboard of 4x4-texel cells in
    two tones with per-texel noise, so that any texel off by one is seen."""
    i = np.arange(w)[None, :]
    j = np.arange(h)[:, None]
    check = ((i // 4 + j // 4) % 2).astype(np.float64)
    key = stream_key(seed, np.arange(h * w, dtype=np.uint64), ST_TEX)
    noise = np.stack([draw_unit(key, np.full(h * w, c, np.uint64)) for c in range(3)], 1).reshape(h, w, 3)
    base = np.where(check[..., None] > 0, [[[0.95, 0.85, 0.55]]], [[[0.35, 0.45, 0.75]]])
    return np.clip(np.rint(255.0 * (0.8 * base + 0.2 * noise)), 0, 255).astype(np.uint8)


def with_texture(scene: Scene, texture: Optional[np.ndarray] = None, ground_uv_scale: float = 2.0) -> Scene:
    """The scene rendered textured: smooth shading, the given (or the
    procedural) texture on the ground and on cube and box faces."""
    tex = procedural_texture() if texture is None else np.ascontiguousarray(texture, np.uint8)
    return dataclasses.replace(scene, smooth=True, texture=tex, ground_uv_scale=float(ground_uv_scale),
                               name=scene.name + "+texture")


@dataclasses.dataclass
class RequestSpec:
    """One rollout request of the serving workload."""
    rid: int
    arrival_s: float
    n_envs: int
    n_bodies: int
    res: int
    horizon: int


def serving_requests(duration_s: float = 120.0, rate: float = 50.0, seed: int = 1005,
                     max_requests: Optional[int] = None) -> List[RequestSpec]:
    """Poisson arrivals; envs log-uniform in [16,512]; 8-64 bodies; horizon
    U{50..500}; resolution from {64,128,256}."""
    out = []
    t = 0.0
    r = 0
    while True:
        key = stream_key(seed, np.array([r], np.uint64), 7)
        u = draw_unit(key, np.arange(6, dtype=np.uint64))
        t += -math.log(1.0 - u[0]) / rate
        if t > duration_s or (max_requests is not None and r >= max_requests):
            break
        n_envs = int(math.floor(math.exp(math.log(16) + u[1] * (math.log(512) - math.log(16)))))
        n_envs = min(max(n_envs, 16), 512)
        nb = 8 + int(u[2] * 57)
        res = (64, 128, 256)[int(u[3] * 3)]
        hor = 50 + int(u[4] * 451)
        out.append(RequestSpec(r, t, n_envs, nb, res, hor))
        r += 1
    return out


def request_scene(req: RequestSpec, seed: int = 1005) -> Scene:
    """Envs of one serving request (homogeneous within the request)."""
    gid0 = req.rid << 12
    return make_scene(seed, np.full(req.n_envs, req.n_bodies), req.res, mixed=True,
                      env_gid0=gid0, name=f"req{req.rid}")


def _bf16_bits(x: np.ndarray) -> np.ndarray:
    """16-bit patterns of float32 values rounded to bfloat16 (nearest, ties
    to even)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + (((u >> 16) & 1) + 0x7FFF)) >> 16).astype(np.uint16)


def policy_weights(seed: int, in_w: int, in_h: int, hidden: int, act_bodies: int,
                   a_max: float = 2.0, zero: bool = False) -> Dict:
    """Seeded random weights of an MLP policy over a camera-0 frame of
    in_w x in_h pixels (observation length K = 4 in_w in_h), scaled so that
    every layer's values are of order one: W1 ~ N(0, 1/(sqrt(K) 128)) in
    bfloat16, W2 and W3 ~ N(0, 1/hidden), biases of order 0.1 to 0.5.
    zero: every weight matrix zero and b3 drawn from {-2, -0.5, 0.5, 2}, so
    that the actions are a_max clamp(b3) exactly."""
    rng = np.random.default_rng(seed)
    K, H, A = 4 * in_w * in_h, hidden, 3 * act_bodies
    P = dict(in_w=in_w, in_h=in_h, act_bodies=act_bodies, a_max=np.float32(a_max))
    if zero:
        P.update(w1_bf16=np.zeros((K, H), np.uint16), b1=np.zeros(H, np.float32),
                 w2=np.zeros((H, H), np.float32), b2=np.zeros(H, np.float32),
                 w3=np.zeros((H, A), np.float32),
                 b3=rng.choice(np.array([-2.0, -0.5, 0.5, 2.0], np.float32), A))
        return P
    P.update(w1_bf16=_bf16_bits(rng.normal(0.0, 1.0 / (math.sqrt(K) * 128.0), (K, H))),
             b1=rng.normal(0.0, 0.1, H).astype(np.float32),
             w2=rng.normal(0.0, 1.0 / H, (H, H)).astype(np.float32),
             b2=rng.normal(0.0, 0.5, H).astype(np.float32),
             w3=rng.normal(0.0, 1.0 / H, (H, A)).astype(np.float32),
             b3=rng.normal(0.0, 0.3, A).astype(np.float32))
    return P
