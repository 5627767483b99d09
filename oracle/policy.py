"""Policy oracle: the MLP that maps a rendered frame to actions, and the
external forces the actions become.  Test infrastructure only, like the rest
of this package: nothing on the product path imports it.

The paper's RL rollouts (Evaluation, RL Training, MLP-based RL) run an MLP
policy on the same GPU as physics and rendering, at 128x128 frames and hidden
sizes 256 and 4096, but do not define its input or its action space.  The
readings taken here:

  * observation of an env: camera 0's frame as K = 4 W H integers in
    0..255 -- first the RGB bytes in memory order (row-major pixels, R G B),
    then the top byte of each pixel's 24-bit depth (background 255);
  * h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3, with W1
    given in bfloat16 (K x H) and everything else in float32;
  * action a = a_max clamp(y, -1, 1), A = 3 B outputs: the force on body b
    (b < B and b < the env's body count) is (a[3b], a[3b+1], a[3b+2]) N, held
    over the next step.

Everything here is evaluated in float64 from the exact inputs: products of
integers and bfloat16 weights are exact, so layer 1 is the exact sum up to
float64 rounding.
"""
from typing import Dict, Tuple

import numpy as np


def bf16_to_f64(bits: np.ndarray) -> np.ndarray:
    """Values of bfloat16 numbers given by their 16-bit patterns."""
    u = (np.asarray(bits, np.uint32) & 0xFFFF) << 16
    return u.view(np.float32).astype(np.float64)


def f32_to_bf16_rne(x: np.ndarray) -> np.ndarray:
    """16-bit patterns of float32 values rounded to bfloat16 (round to
    nearest, ties to even; inputs are finite)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u >> 16) & 1) + 0x7FFF
    return ((u + r) >> 16).astype(np.uint16)


def observation(rgb: np.ndarray, depth: np.ndarray) -> np.ndarray:
    """Observation vector (float64, K = 4 W H) of one frame: rgb [H, W, 3]
    uint8, depth [H, W] uint32 (24-bit values, 0xFFFFFFFF = background)."""
    rgb = np.asarray(rgb, np.uint8).reshape(-1)
    d = np.asarray(depth, np.uint32).reshape(-1)
    top = np.where(d == 0xFFFFFFFF, 255, (d >> 16) & 0xFF)
    return np.concatenate([rgb.astype(np.float64), top.astype(np.float64)])


def prepare(P: Dict) -> Dict:
    """P with the float64 values of W1 and their magnitudes added (keys w1,
    w1abs), for repeated calls."""
    w1 = bf16_to_f64(P["w1_bf16"])
    return dict(P, w1=w1, w1abs=np.abs(w1))


def _w1(P: Dict) -> np.ndarray:
    return P["w1"] if "w1" in P else bf16_to_f64(P["w1_bf16"])


def _w1abs(P: Dict) -> np.ndarray:
    return P["w1abs"] if "w1abs" in P else np.abs(_w1(P))


def forward(x: np.ndarray, P: Dict[str, np.ndarray]) -> Tuple[np.ndarray, Dict[str, np.ndarray]]:
    """Actions of one observation under policy P (keys w1_bf16 [K, H] uint16,
    b1 [H], w2 [H, H], b2 [H], w3 [H, A], b3 [A], a_max).  Also returns the
    layer values (pre-activations s1, s2, y; activations h1, h2) for error
    bounds."""
    s1 = x @ _w1(P) + P["b1"].astype(np.float64)
    h1 = np.maximum(s1, 0.0)
    s2 = h1 @ P["w2"].astype(np.float64) + P["b2"].astype(np.float64)
    h2 = np.maximum(s2, 0.0)
    y = h2 @ P["w3"].astype(np.float64) + P["b3"].astype(np.float64)
    a = float(P["a_max"]) * np.clip(y, -1.0, 1.0)
    return a, dict(s1=s1, h1=h1, s2=s2, h2=h2, y=y)


def error_bound(x: np.ndarray, P: Dict[str, np.ndarray], inner: Dict[str, np.ndarray],
                lam: float = 8.0) -> np.ndarray:
    """Bound on |a_computed - a| for an evaluation in float32 arithmetic in
    any summation order: the exact products of layer 1 accumulated in float32,
    layers 2 and 3 with float32 products and sums.  A dot product of n terms
    is taken to carry at most lam sqrt(n) u sum |terms| of its own rounding,
    the probabilistic bound of Higham and Mary (SIAM J. Sci. Comput. 41, 2019)
    for independent rounding errors, which fails with probability at most
    2 exp(-lam^2 (1 - u)^2 / 2) (about 2.5e-14 at lam = 8); u = 2^-23 covers
    rounding toward zero as well as to nearest.  Errors of a layer's inputs
    pass on through the absolute weights (relu and clamp are 1-Lipschitz)."""
    u = 2.0 ** -23
    g = lambda n: lam * np.sqrt(n) * u
    W1 = _w1abs(P)
    W2 = np.abs(P["w2"].astype(np.float64))
    W3 = np.abs(P["w3"].astype(np.float64))
    K, H = W1.shape
    A = W3.shape[1]
    e1 = g(K + 1) * (np.abs(x) @ W1 + np.abs(P["b1"]))
    e2 = e1 @ W2 + g(H + 1) * ((inner["h1"] + e1) @ W2 + np.abs(P["b2"]))
    e3 = e2 @ W3 + g(H + 1) * ((inner["h2"] + e2) @ W3 + np.abs(P["b3"]))
    return float(P["a_max"]) * e3 + 4 * u * float(P["a_max"]) * np.ones(A)


def forces(a: np.ndarray, n_bodies: int, act_bodies: int) -> np.ndarray:
    """External forces [n_bodies, 3] of one env from its actions."""
    f = np.zeros((n_bodies, 3), np.float32)
    m = min(n_bodies, act_bodies)
    f[:m] = np.asarray(a, np.float32).reshape(-1, 3)[:m]
    return f
