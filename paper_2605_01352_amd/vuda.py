"""Python binding of libvuda (the C ABI in include/vuda.h).

Argument marshalling only: every step of the physics and render path runs in
the library's HIP kernels.  Importing this module does not touch the GPU; the
first World() loads lib/libvuda.so and raises if it has not been built
(there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libvuda.so")
DEFAULT_LIB_PATH = LIB_PATH

OK, EINVAL, ENOMEM, EHIP, ENUMERIC, EOVERFLOW, EBUSY = 0, -1, -2, -3, -4, -5, -6
PHASE_STEP, PHASE_RENDER, PHASE_ALL = 1, 2, 3
FETCH_STATE, FETCH_RGB, FETCH_DEPTH, FETCH_CONTACTS, FETCH_WINNERS, FETCH_COVERAGE, FETCH_FLAGS, FETCH_ACTIONS, \
    FETCH_DEPTH_METRIC = range(9)
FLAG_DEBUG = 1
FLAG_NEAR_CLIP = 2
FLAG_SMOOTH = 4
FLAG_TEXTURE = 8
TUNE_RASTER_THREADS, TUNE_REC_CAP, TUNE_PHYS_PERSISTENT, TUNE_RASTER_PERSISTENT, TUNE_GRAPHS = 1, 2, 3, 4, 5
PERSISTENT_RESIDENT = -1  # persistent grid of the workgroups the GPU holds at once
TUNE_PHYS_PRIORITY = 6
TUNE_BROADPHASE = 7
TUNE_TIMING = 8
TUNE_PRESETUP = 9
TUNE_POLICY_LAYERED = 10
TUNE_PHYS_ENVS_PER_WAVE = 11
TUNE_TILE_SIZE = 12
TUNE_RASTER_FUSED = 13
TUNE_FUSED_LDS_RECORDS = 14
TUNE_TILE_WAVES = 15
TUNE_TILE_PRIORITY = 16
KERNEL_PHYSICS, KERNEL_RASTER_SETUP, KERNEL_RASTER_TILES, KERNEL_POLICY, KERNEL_RASTER_FUSED = 1, 2, 3, 4, 5
GROUND = 0xFFFF

EXPORTS = [
    "vuda_create_world", "vuda_destroy_world", "vuda_cosched", "vuda_step", "vuda_render",
    "vuda_wait", "vuda_fetch", "vuda_fetch_bytes", "vuda_load_state", "vuda_get_stream",
    "vuda_admit", "vuda_release", "vuda_world_info", "vuda_set_tuning", "vuda_get_tuning",
    "vuda_probe_placement", "vuda_strerror", "vuda_last_error_message", "vuda_run",
    "vuda_autotune", "vuda_serve_create", "vuda_serve_destroy", "vuda_serve_submit",
    "vuda_serve_tick", "vuda_serve_completed", "vuda_serve_result", "vuda_serve_stats",
    "vuda_serve_world", "vuda_kernel_times", "vuda_policy_set", "vuda_act", "vuda_act_noalloc",
]
SCHED_SERIAL, SCHED_INTERSTEP, SCHED_INTERTRAJ, SCHED_PIPELINED = 0, 1, 2, 3
SCHED_NAMES = {SCHED_SERIAL: "serial", SCHED_INTERSTEP: "interstep", SCHED_INTERTRAJ: "intertraj",
               SCHED_PIPELINED: "pipelined"}


class VudaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class PhysParams(C.Structure):
    _fields_ = [("dt", C.c_float), ("substeps", C.c_int32), ("k_contact", C.c_float),
                ("c_damp", C.c_float), ("gravity", C.c_float * 3), ("mu", C.c_float), ("v_eps", C.c_float),
                ("edge_contacts", C.c_int32)]


class RenderDesc(C.Structure):
    _fields_ = [
        ("sphere_v", C.c_void_p), ("sphere_nv", C.c_int32), ("sphere_f", C.c_void_p),
        ("sphere_n", C.c_void_p), ("sphere_nf", C.c_int32),
        ("cube_v", C.c_void_p), ("cube_nv", C.c_int32), ("cube_f", C.c_void_p),
        ("cube_n", C.c_void_p), ("cube_nf", C.c_int32),
        ("ground_v", C.c_void_p), ("ground_nv", C.c_int32), ("ground_f", C.c_void_p),
        ("ground_nf", C.c_int32),
        ("light", C.c_float * 3), ("palette", C.c_float * 24), ("ground_albedo", C.c_float),
        ("near_w", C.c_float), ("guard", C.c_float),
        ("texture", C.c_void_p), ("texture_w", C.c_int32), ("texture_h", C.c_int32),
        ("ground_uv_scale", C.c_float)]


class EnvBatch(C.Structure):
    _fields_ = [
        ("n_envs", C.c_int32), ("body_off", C.c_void_p),
        ("type", C.c_void_p), ("size", C.c_void_p), ("rbound", C.c_void_p),
        ("inv_m", C.c_void_p), ("inv_I", C.c_void_p), ("albedo", C.c_void_p),
        ("pos", C.c_void_p), ("vel", C.c_void_p), ("quat", C.c_void_p), ("omega", C.c_void_p),
        ("cam_off", C.c_void_p), ("cam_vp", C.c_void_p), ("cam_w", C.c_void_p), ("cam_h", C.c_void_p),
        ("ext", C.c_void_p), ("inertia", C.c_void_p)]


class WorldDesc(C.Structure):
    _fields_ = [("phys", PhysParams), ("render", RenderDesc), ("initial", EnvBatch),
                ("flags", C.c_uint32), ("cap_envs", C.c_int32), ("cap_bodies", C.c_int64),
                ("cap_cams", C.c_int32), ("cap_pixels", C.c_int64), ("pair_cap", C.c_int32),
                ("hbm_budget", C.c_uint64)]


class TuneResult(C.Structure):
    _fields_ = [("cu_split", C.c_float), ("schedule", C.c_int32), ("raster_threads", C.c_int32),
                ("rec_cap", C.c_int32), ("phys_persistent", C.c_int32),
                ("raster_persistent", C.c_int32), ("phys_priority", C.c_int32),
                ("broadphase", C.c_int32), ("cosched_env_steps_per_s", C.c_double),
                ("serial_env_steps_per_s", C.c_double), ("serial_raster_threads", C.c_int32),
                ("serial_phys_persistent", C.c_int32), ("trials", C.c_int32), ("presetup", C.c_int32),
                ("graphs", C.c_int32), ("phys_envs_per_wave", C.c_int32), ("tile_size", C.c_int32),
                ("raster_fused", C.c_int32), ("tile_waves", C.c_int32), ("tile_priority", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PolicyDesc(C.Structure):
    _fields_ = [("in_w", C.c_int32), ("in_h", C.c_int32), ("hidden", C.c_int32), ("act_bodies", C.c_int32),
                ("a_max", C.c_float), ("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p),
                ("b2", C.c_void_p), ("w3", C.c_void_p), ("b3", C.c_void_p)]


class ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("queued", C.c_int64), ("active_requests", C.c_int64), ("active_envs", C.c_int64),
                ("env_steps", C.c_int64), ("ticks", C.c_int64), ("busy_s", C.c_double),
                ("latency_p50_s", C.c_double), ("latency_p99_s", C.c_double),
                ("latency_max_s", C.c_double), ("latency_mean_s", C.c_double),
                ("queue_p50_s", C.c_double), ("queue_p99_s", C.c_double),
                ("reserved_bytes", C.c_uint64), ("peak_reserved_bytes", C.c_uint64),
                ("rejected", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def stale_sources():
    """Sources whose bytes differ from what the in-tree library was built from
    (its manifest, written by build.py); ['(no manifest)'] without one."""
    from . import build as _build
    try:
        with open(_build.MANIFEST) as f:
            built = json.load(f)["sources"]
    except (OSError, ValueError, KeyError):
        return ["(no manifest)"]
    now = _build.source_digests()
    return sorted(k for k in set(built) | set(now) if built.get(k) != now.get(k))


def lib():
    """Load libvuda.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2605_01352_amd/build.py "
                               f"(or __graft_entry__.build())")
        if LIB_PATH == DEFAULT_LIB_PATH:
            stale = stale_sources()
            if stale:
                raise RuntimeError(f"{LIB_PATH} was built from other sources than the tree holds "
                                   f"({', '.join(stale[:4])}{' ...' if len(stale) > 4 else ''}); rebuild it "
                                   f"(paper_2605_01352_amd/build.py or __graft_entry__.build())")
        # PyTorch ships its own HIP runtime and loads it under another name; it
        # has to be loaded first so that libvuda binds to that same runtime and
        # the process holds one (streams and events are then shared with it).
        try:
            import torch  # noqa: F401
        except Exception:
            pass
        L = C.CDLL(LIB_PATH)
        for name in EXPORTS:
            getattr(L, name)  # raises AttributeError if missing
        L.vuda_strerror.restype = C.c_char_p
        L.vuda_serve_submit.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32]
        L.vuda_serve_result.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_size_t,
                                        C.c_void_p]
        L.vuda_last_error_message.restype = C.c_char_p
        _lib = L
    return _lib


def check(code: int):
    if code != 0:
        L = lib()
        raise VudaError(code, L.vuda_last_error_message().decode(errors="replace"))
    return code


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Keep:
    """Holds contiguous copies of arrays referenced by a ctypes struct."""

    def __init__(self):
        self.arrs = []

    def __call__(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.arrs.append(a)
        return a


def render_desc(keep: _Keep, light=None, palette=None, ground_albedo=None, near=None, guard=None, texture=None,
                ground_uv_scale=1.0):
    from . import scenegen as sg
    t = sg.templates()
    sv, sf, sn = keep(t.sphere_v, np.float32), keep(t.sphere_f, np.int32), keep(t.sphere_n, np.float32)
    cv, cf, cn = keep(t.cube_v, np.float32), keep(t.cube_f, np.int32), keep(t.cube_n, np.float32)
    gv, gf = keep(t.ground_v, np.float32), keep(t.ground_f, np.int32)
    light = sg.LIGHT if light is None else light
    palette = sg.PALETTE if palette is None else palette
    return RenderDesc(
        _p(sv), len(sv), _p(sf), _p(sn), len(sf), _p(cv), len(cv), _p(cf), _p(cn), len(cf),
        _p(gv), len(gv), _p(gf), len(gf),
        (C.c_float * 3)(*np.asarray(light, np.float32).tolist()),
        (C.c_float * 24)(*np.asarray(palette, np.float32).reshape(-1).tolist()),
        float(sg.GROUND_ALBEDO if ground_albedo is None else ground_albedo),
        float(sg.NEAR if near is None else near), float(sg.GUARD_BAND if guard is None else guard),
        None if texture is None else _p(keep(texture, np.uint8)),
        0 if texture is None else int(np.shape(texture)[1]), 0 if texture is None else int(np.shape(texture)[0]),
        float(np.float32(ground_uv_scale)))


def env_batch(keep: _Keep, scene, state: Optional[Dict[str, np.ndarray]] = None) -> EnvBatch:
    st = scene.state() if state is None else state
    if scene.n_envs == 0:
        return EnvBatch(0)
    return EnvBatch(
        scene.n_envs, _p(keep(scene.body_off, np.int32)), _p(keep(scene.btype, np.uint8)),
        _p(keep(scene.size, np.float32)), _p(keep(scene.rbound, np.float32)),
        _p(keep(scene.inv_m, np.float32)), _p(keep(scene.inv_I, np.float32)),
        _p(keep(scene.albedo, np.uint8)), _p(keep(st["pos"], np.float32)),
        _p(keep(st["vel"], np.float32)), _p(keep(st["quat"], np.float32)),
        _p(keep(st["omega"], np.float32)), _p(keep(scene.cam_off, np.int32)),
        _p(keep(scene.cam_vp, np.float32)), _p(keep(scene.cam_w, np.int32)),
        _p(keep(scene.cam_h, np.int32)),
        None if scene.ext is None else _p(keep(scene.ext, np.float32)),
        None if scene.inertia is None else _p(keep(scene.inertia, np.float32)))


def state_to_aos(st: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([st["pos"], st["vel"], st["quat"], st["omega"]], axis=1).astype(np.float32)


def aos_to_state(a: np.ndarray) -> Dict[str, np.ndarray]:
    a = np.asarray(a, np.float32).reshape(-1, 13)
    return dict(pos=a[:, 0:3].copy(), vel=a[:, 3:6].copy(), quat=a[:, 6:10].copy(),
                omega=a[:, 10:13].copy())


class World:
    """A batch of envs resident on the current HIP device."""

    def __init__(self, scene=None, debug: bool = False, cap_envs: int = 0, cap_bodies: int = 0,
                 cap_cams: int = 0, cap_pixels: int = 0, pair_cap: int = 1024,
                 hbm_budget: int = 0, phys=None, render_kw=None):
        L = lib()
        keep = _Keep()
        from . import scenegen as sg
        ref = scene
        dt = (ref.dt if ref is not None else 1.0 / 240.0)
        sub = (ref.substeps if ref is not None else 4)
        k = (ref.k_contact if ref is not None else 1.0e4)
        c = (ref.c_damp if ref is not None else 10.0)
        g = (ref.gravity if ref is not None else (0.0, 0.0, -9.81))
        mu = (ref.mu if ref is not None else 0.0)
        v_eps = (ref.v_eps if ref is not None else 0.05)
        edge = bool(ref.edge_contacts) if ref is not None else False
        if phys:
            dt, sub, k, c, g = phys.get("dt", dt), phys.get("substeps", sub), phys.get("k", k), \
                phys.get("c", c), phys.get("g", g)
            mu, v_eps = phys.get("mu", mu), phys.get("v_eps", v_eps)
            edge = phys.get("edge_contacts", edge)
        desc = WorldDesc()
        desc.phys = PhysParams(float(np.float32(dt)), int(sub), float(k), float(c),
                               (C.c_float * 3)(*[float(x) for x in g]), float(mu), float(v_eps), int(edge))
        rkw = dict(render_kw or {})
        if getattr(ref, "texture", None) is not None:
            rkw.setdefault("texture", ref.texture)
            rkw.setdefault("ground_uv_scale", getattr(ref, "ground_uv_scale", 1.0))
        desc.render = render_desc(keep, **rkw)
        desc.initial = env_batch(keep, scene) if scene is not None else EnvBatch(0)
        desc.flags = (FLAG_DEBUG if debug else 0) | (FLAG_NEAR_CLIP if getattr(ref, "near_clip", False) else 0) | \
            (FLAG_SMOOTH if getattr(ref, "smooth", False) else 0) | \
            (FLAG_TEXTURE if getattr(ref, "texture", None) is not None else 0)
        desc.cap_envs, desc.cap_bodies, desc.cap_cams, desc.cap_pixels = cap_envs, cap_bodies, cap_cams, cap_pixels
        desc.pair_cap = pair_cap
        desc.hbm_budget = hbm_budget
        self._w = C.c_void_p()
        check(L.vuda_create_world(C.byref(desc), None, C.byref(self._w)))
        self.scene = scene
        self.debug = debug
        self.substeps = int(sub)
        self.pair_cap = pair_cap
        self.n_envs = scene.n_envs if scene is not None else 0

    # -- lifetime --------------------------------------------------------
    def close(self):
        if self._w:
            check(lib().vuda_destroy_world(self._w))
            self._w = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- the loop ---------------------------------------------------------
    def cosched(self, split: float):
        check(lib().vuda_cosched(self._w, C.c_float(split)))

    def step(self, lo: int = 0, hi: Optional[int] = None, nsteps: int = 1):
        hi = self.n_envs if hi is None else hi
        check(lib().vuda_step(self._w, lo, hi, nsteps))

    def render(self, lo: int = 0, hi: Optional[int] = None):
        hi = self.n_envs if hi is None else hi
        check(lib().vuda_render(self._w, lo, hi))

    def set_policy(self, policy: Optional[Dict]):
        """Install an MLP policy (keys in_w, in_h, act_bodies, a_max,
        w1_bf16 [K, H] uint16 bfloat16 bits, b1, w2, b2, w3, b3), or remove
        it (None)."""
        if policy is None:
            check(lib().vuda_policy_set(self._w, None))
            return
        P = policy
        keep = [np.ascontiguousarray(P["w1_bf16"], np.uint16)]
        keep += [np.ascontiguousarray(P[k], np.float32) for k in ("b1", "w2", "b2", "w3", "b3")]
        d = PolicyDesc(int(P["in_w"]), int(P["in_h"]), int(keep[1].shape[0]), int(P["act_bodies"]),
                       float(P["a_max"]), *[a.ctypes.data for a in keep])
        check(lib().vuda_policy_set(self._w, C.byref(d)))

    def act(self, lo: int = 0, hi: Optional[int] = None):
        """Enqueue the policy on envs [lo, hi): actions for their next steps."""
        hi = self.n_envs if hi is None else hi
        check(lib().vuda_act(self._w, lo, hi))

    def act_noalloc(self, lo: int = 0, hi: Optional[int] = None):
        """vuda_act through the library's static workspace (no allocation)."""
        hi = self.n_envs if hi is None else hi
        check(lib().vuda_act_noalloc(self._w, lo, hi))

    def wait(self, phase: int = PHASE_ALL):
        check(lib().vuda_wait(self._w, phase))

    def run(self, schedule: int = SCHED_INTERSTEP, iters: int = 1):
        """Enqueue iterations of a schedule over every active env."""
        check(lib().vuda_run(self._w, schedule, iters))

    def autotune(self, steps: int = 30, cache: Optional[str] = None) -> Dict:
        r = TuneResult()
        check(lib().vuda_autotune(self._w, steps, cache.encode() if cache else None, C.byref(r)))
        return r.as_dict()

    def set_tuning(self, key: int, value: int):
        check(lib().vuda_set_tuning(self._w, key, int(value)))

    def get_tuning(self, key: int) -> int:
        v = C.c_int32()
        check(lib().vuda_get_tuning(self._w, key, C.byref(v)))
        return v.value

    def kernel_times(self, kernel: int) -> Dict:
        """Launch count, total and max duration (ms) of a kernel (KERNEL_*)
        recorded with TUNE_TIMING on since the previous call for it."""
        n, tot, mx = C.c_int64(), C.c_double(), C.c_double()
        check(lib().vuda_kernel_times(self._w, kernel, C.byref(n), C.byref(tot), C.byref(mx)))
        return {"launches": n.value, "total_ms": tot.value, "max_ms": mx.value}

    def stream(self, phase: int) -> int:
        p = C.c_void_p()
        check(lib().vuda_get_stream(self._w, phase, C.byref(p)))
        return p.value or 0

    def probe_placement(self, phase: int, n_blocks: int, spin_us: int = 200) -> np.ndarray:
        out = np.zeros((n_blocks, 3), np.int32)
        check(lib().vuda_probe_placement(self._w, phase, n_blocks, spin_us, _p(out)))
        return out

    # -- results ------------------------------------------------------------
    def fetch_bytes(self, what: int, lo: int = 0, hi: Optional[int] = None) -> int:
        hi = self.n_envs if hi is None else hi
        n = C.c_size_t()
        check(lib().vuda_fetch_bytes(self._w, what, lo, hi, C.byref(n)))
        return n.value

    def fetch(self, what: int, lo: int = 0, hi: Optional[int] = None, out=None):
        """Copy results into a numpy array (or a torch CUDA tensor given as out)."""
        hi = self.n_envs if hi is None else hi
        nbytes = self.fetch_bytes(what, lo, hi)
        if out is not None and hasattr(out, "data_ptr"):
            if out.numel() * out.element_size() < nbytes:
                raise ValueError("output tensor too small")
            check(lib().vuda_fetch(self._w, what, lo, hi, C.c_void_p(out.data_ptr()),
                                   C.c_size_t(nbytes), 1 if out.is_cuda else 0))
            return out
        dt = {FETCH_STATE: np.float32, FETCH_RGB: np.uint8, FETCH_DEPTH: np.uint32,
              FETCH_CONTACTS: np.int32, FETCH_WINNERS: np.int32, FETCH_COVERAGE: np.int32,
              FETCH_FLAGS: np.uint32, FETCH_ACTIONS: np.float32, FETCH_DEPTH_METRIC: np.float32}[what]
        buf = np.zeros(nbytes // np.dtype(dt).itemsize, dt)
        check(lib().vuda_fetch(self._w, what, lo, hi, _p(buf), C.c_size_t(nbytes), 0))
        return buf

    def state(self, lo: int = 0, hi: Optional[int] = None) -> Dict[str, np.ndarray]:
        return aos_to_state(self.fetch(FETCH_STATE, lo, hi))

    def load_state(self, st: Dict[str, np.ndarray], lo: int = 0, hi: Optional[int] = None):
        hi = self.n_envs if hi is None else hi
        a = np.ascontiguousarray(state_to_aos(st))
        check(lib().vuda_load_state(self._w, lo, hi, _p(a), C.c_size_t(a.nbytes)))

    def images(self, what: int, scene=None, lo: int = 0, hi: Optional[int] = None):
        """List of per-camera images of envs [lo, hi)."""
        scene = self.scene if scene is None else scene
        hi = self.n_envs if hi is None else hi
        flat = self.fetch(what, lo, hi)
        out, pos = [], 0
        for c in range(int(scene.cam_off[lo]), int(scene.cam_off[hi])):
            w, h = int(scene.cam_w[c]), int(scene.cam_h[c])
            ch = 3 if what == FETCH_RGB else 1
            img = flat[pos:pos + w * h * ch]
            out.append(img.reshape(h, w, 3) if ch == 3 else img.reshape(h, w))
            pos += w * h * ch
        return out

    def contacts(self, lo: int = 0, hi: Optional[int] = None):
        """Per env, per substep: sorted (i, j) pair arrays."""
        hi = self.n_envs if hi is None else hi
        flat = self.fetch(FETCH_CONTACTS, lo, hi).reshape(hi - lo, self.substeps, 1 + 2 * self.pair_cap)
        res = []
        for e in range(hi - lo):
            per = []
            for s in range(self.substeps):
                n = int(flat[e, s, 0])
                if n > self.pair_cap:
                    raise VudaError(EOVERFLOW, f"env {lo + e}: {n} contact pairs > pair_cap")
                per.append(flat[e, s, 1:1 + 2 * n].reshape(n, 2).copy())
            res.append(per)
        return res

    # -- serving -----------------------------------------------------------
    def admit(self, scene, parity: int = 0) -> int:
        keep = _Keep()
        b = env_batch(keep, scene)
        first = C.c_int32()
        check(lib().vuda_admit(self._w, C.byref(b), parity, C.byref(first)))
        self.n_envs = max(self.n_envs, first.value + scene.n_envs)
        return first.value

    def try_admit(self, scene, parity: int = 0) -> Optional[int]:
        keep = _Keep()
        b = env_batch(keep, scene)
        first = C.c_int32()
        rc = lib().vuda_admit(self._w, C.byref(b), parity, C.byref(first))
        if rc == EBUSY:
            return None
        check(rc)
        self.n_envs = max(self.n_envs, first.value + scene.n_envs)
        return first.value

    def release(self, first: int, n: int):
        check(lib().vuda_release(self._w, first, n))

    def info(self):
        ne, nb, nc, npx, ab = C.c_int32(), C.c_int64(), C.c_int32(), C.c_int64(), C.c_uint64()
        check(lib().vuda_world_info(self._w, C.byref(ne), C.byref(nb), C.byref(nc), C.byref(npx), C.byref(ab)))
        return dict(n_envs=ne.value, cap_bodies=nb.value, cap_cams=nc.value, cap_pixels=npx.value,
                    arena_bytes=ab.value)


def world_desc(keep: _Keep, scene=None, debug: bool = False, cap_envs: int = 0, cap_bodies: int = 0,
               cap_cams: int = 0, cap_pixels: int = 0, pair_cap: int = 1024, hbm_budget: int = 0,
               phys=None) -> WorldDesc:
    dt, sub, k, c, g = 1.0 / 240.0, 4, 1.0e4, 10.0, (0.0, 0.0, -9.81)
    mu, v_eps, edge = 0.0, 0.05, False
    if scene is not None:
        dt, sub, k, c, g = scene.dt, scene.substeps, scene.k_contact, scene.c_damp, scene.gravity
        mu, v_eps, edge = scene.mu, scene.v_eps, bool(scene.edge_contacts)
    if phys:
        dt, sub, k, c, g = phys.get("dt", dt), phys.get("substeps", sub), phys.get("k", k), \
            phys.get("c", c), phys.get("g", g)
        mu, v_eps = phys.get("mu", mu), phys.get("v_eps", v_eps)
        edge = phys.get("edge_contacts", edge)
    d = WorldDesc()
    d.phys = PhysParams(float(np.float32(dt)), int(sub), float(k), float(c),
                        (C.c_float * 3)(*[float(x) for x in g]), float(mu), float(v_eps), int(edge))
    tex = getattr(scene, "texture", None)
    d.render = render_desc(keep, texture=tex, ground_uv_scale=getattr(scene, "ground_uv_scale", 1.0))
    d.initial = env_batch(keep, scene) if scene is not None else EnvBatch(0)
    d.flags = (FLAG_DEBUG if debug else 0) | (FLAG_NEAR_CLIP if getattr(scene, "near_clip", False) else 0) | \
        (FLAG_SMOOTH if getattr(scene, "smooth", False) else 0) | (FLAG_TEXTURE if tex is not None else 0)
    d.cap_envs, d.cap_bodies, d.cap_cams, d.cap_pixels = cap_envs, cap_bodies, cap_cams, cap_pixels
    d.pair_cap = pair_cap
    d.hbm_budget = hbm_budget
    return d


class Server:
    """Serving loop with continuous batching (vuda_serve_*)."""

    def __init__(self, cap_envs: int, cap_bodies: int, cap_cams: int, cap_pixels: int,
                 hbm_budget: int = 0, cu_split: float = 2.0, schedule: int = SCHED_INTERSTEP,
                 keep_results: bool = False):
        L = lib()
        keep = _Keep()
        d = world_desc(keep, None, cap_envs=cap_envs, cap_bodies=cap_bodies, cap_cams=cap_cams,
                       cap_pixels=cap_pixels, hbm_budget=hbm_budget)
        self._s = C.c_void_p()
        check(L.vuda_serve_create(C.byref(d), C.c_float(cu_split), schedule, int(keep_results),
                                  C.byref(self._s)))

    def close(self):
        if self._s:
            check(lib().vuda_serve_destroy(self._s))
            self._s = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def world_handle(self):
        w = C.c_void_p()
        check(lib().vuda_serve_world(self._s, C.byref(w)))
        return w

    def set_tuning(self, key: int, value: int):
        check(lib().vuda_set_tuning(self.world_handle(), key, int(value)))

    def submit(self, request_id: int, scene, horizon: int):
        keep = _Keep()
        b = env_batch(keep, scene)
        check(lib().vuda_serve_submit(self._s, int(request_id), C.byref(b), int(horizon)))

    def tick(self) -> int:
        n = C.c_int32()
        check(lib().vuda_serve_tick(self._s, C.byref(n)))
        return n.value

    def completed(self, cap: int = 4096):
        ids = np.zeros(cap, np.int64)
        lat = np.zeros(cap, np.float64)
        n = C.c_int32()
        check(lib().vuda_serve_completed(self._s, _p(ids), _p(lat), cap, C.byref(n)))
        return list(zip(ids[:n.value].tolist(), lat[:n.value].tolist()))

    def result(self, request_id: int, what: int) -> np.ndarray:
        need = C.c_size_t()
        check(lib().vuda_serve_result(self._s, int(request_id), what, None, 0, C.byref(need)))
        dt = {FETCH_STATE: np.float32, FETCH_RGB: np.uint8, FETCH_DEPTH: np.uint32}[what]
        out = np.zeros(need.value // np.dtype(dt).itemsize, dt)
        check(lib().vuda_serve_result(self._s, int(request_id), what, _p(out), C.c_size_t(need.value),
                                      C.byref(need)))
        return out

    def stats(self) -> Dict:
        st = ServeStats()
        check(lib().vuda_serve_stats(self._s, C.byref(st)))
        return st.as_dict()
