"""Hand-built tiny scenes for the oracle pins and parity edge cases."""
import dataclasses
import math

import numpy as np

from paper_2605_01352_amd import scenegen as sg


def tiny_scene(bodies, gravity=(0.0, 0.0, -9.81), res=64, vp=None, envs=1, k=1.0e4, c=10.0, mu=0.0,
               v_eps=0.05):
    """bodies: list of dicts(type, size, pos, [quat], [vel], [omega], [mass]).

    The same bodies are repeated in every env.
    """
    n = len(bodies)
    f32 = lambda x: np.asarray(x, np.float32)
    bt = np.array([b["type"] for b in bodies], np.uint8)
    # a box (type 2) has half-extents "ext"; its size is the largest of them
    ext64 = np.array([b.get("ext", (b.get("size", 0.0),) * 3) for b in bodies], np.float64).reshape(n, 3)
    size = f32([b["size"] if "size" in b else max(b["ext"]) for b in bodies])
    s64 = size.astype(np.float64)
    m = np.array([b.get("mass", 1.0) for b in bodies])
    rb = np.where(bt == 0, s64, s64 * math.sqrt(3.0) * (1 + 1e-6))
    rb = np.where(bt == 2, np.linalg.norm(ext64, axis=1) * (1 + 1e-6), rb).astype(np.float32)
    inv_I = np.where(bt == 0, 1.0 / (0.4 * m * s64 ** 2), 1.0 / ((2.0 / 3.0) * m * s64 ** 2)).astype(np.float32)
    e2 = ext64 ** 2
    inertia = (m[:, None] / 3.0 * np.stack([e2[:, 1] + e2[:, 2], e2[:, 0] + e2[:, 2], e2[:, 0] + e2[:, 1]], 1))
    has_box = bool(np.any(bt == 2))
    rep = lambda a: np.concatenate([a] * envs)
    pos = f32([b["pos"] for b in bodies]).reshape(n, 3)
    quat = f32([b.get("quat", (1, 0, 0, 0)) for b in bodies]).reshape(n, 4)
    vel = f32([b.get("vel", (0, 0, 0)) for b in bodies]).reshape(n, 3)
    om = f32([b.get("omega", (0, 0, 0)) for b in bodies]).reshape(n, 3)
    if vp is None:
        vp = sg.view_proj(sg.FIXED_EYE)
    return sg.Scene(
        body_off=(np.arange(envs + 1) * n).astype(np.int32), btype=rep(bt), size=rep(size),
        rbound=rep(rb), inv_m=rep((1.0 / m).astype(np.float32)), inv_I=rep(inv_I),
        albedo=rep((np.arange(n) % 8).astype(np.uint8)), pos=rep(pos), vel=rep(vel),
        quat=rep(quat), omega=rep(om), cam_off=np.arange(envs + 1).astype(np.int32),
        cam_vp=np.repeat(np.asarray(vp, np.float32).reshape(1, 16), envs, axis=0),
        cam_w=np.full(envs, res, np.int32), cam_h=np.full(envs, res, np.int32),
        gravity=gravity, k_contact=k, c_damp=c, mu=mu, v_eps=v_eps, name="tiny",
        ext=rep(ext64.astype(np.float32)) if has_box else None, inertia=rep(inertia.astype(np.float32)) if has_box else None)


def quat_axis_angle(axis, ang):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    return (math.cos(ang / 2), *(a * math.sin(ang / 2)))
