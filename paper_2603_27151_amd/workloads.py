"""Seeded synthetic inputs for the triangle-soup rasterization step.

This module builds *inputs only*: triangle soups, per-triangle feature grids,
MLP parameters, cameras and target images. It holds none of the rasterizer's
arithmetic, so that the CPU oracle and the GPU path can both draw their inputs
from it without sharing any of the method's code.

Shapes and distributions follow the five workloads the method is exercised on:

* ``tiny``     : 64 triangles, vertices U[-1,1]^3, one 128x128 view, 4x4x8
                 features, MLP 8->16->4.
* ``single``   : 10,000 triangles (centres uniform in the unit ball, equilateral
                 with side exp(N(-3, 0.5^2)), random orientation), one 800x800
                 view, 8x8x16 features, MLP 16->32->32->4.
* ``batched``  : 50,000 triangles as in ``single``; 64 views on a Fibonacci
                 sphere of radius 3, each view's resolution drawn from
                 {256, 512, 800, 1024}^2.
* ``serving``  : four resident soups of 20k/40k/70k/100k triangles; requests
                 at 640x360, 1280x720 or 1920x1080 from random directions.
* ``large``    : 200,000 triangles in 16 Gaussian blobs (sigma 0.15), 16 views
                 at 1920x1080, 8x8x32 features, MLP 32->64->64->4.

Features are N(0, 0.1^2) (0.1 read as the standard deviation), MLP weights are
Glorot-uniform with a = sqrt(6 / (fan_in + fan_out)) and zero biases (the
paper's Xavier initialisation, Supplement B.3). The triangle soup itself is
the paper's representation of Section 3.1: |T| independent triangles of nine
floats each (Supplement B.6).

Cameras are pinhole cameras with a 60 degree vertical field of view that look
at the origin with +y up (+z when the view direction is within 0.99 of +-y),
near 0.1 and far 100, OpenGL clip-space convention. Matrices are built in
float64 and rounded once to float32; both implementations receive the same
float32 matrix.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# cameras
# ---------------------------------------------------------------------------

NEAR = 0.1
FAR = 100.0
VFOV_DEG = 60.0


def look_at(eye: Sequence[float], target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """World->camera matrix (float64), camera looking down its -z axis."""
    eye = np.asarray(eye, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    f = target - eye
    f = f / np.linalg.norm(f)
    up = np.asarray(up, dtype=np.float64)
    if abs(float(np.dot(f, up / np.linalg.norm(up)))) > 0.99:
        up = np.array([0.0, 0.0, 1.0])
    s = np.cross(f, up)
    s = s / np.linalg.norm(s)
    u = np.cross(s, f)
    m = np.eye(4)
    m[0, :3] = s
    m[1, :3] = u
    m[2, :3] = -f
    m[0, 3] = -np.dot(s, eye)
    m[1, 3] = -np.dot(u, eye)
    m[2, 3] = np.dot(f, eye)
    return m


def perspective(vfov_deg: float, aspect: float, near: float = NEAR, far: float = FAR) -> np.ndarray:
    """OpenGL-style projection matrix (float64): NDC z in [-1, 1]."""
    t = 1.0 / math.tan(math.radians(vfov_deg) / 2.0)
    p = np.zeros((4, 4))
    p[0, 0] = t / aspect
    p[1, 1] = t
    p[2, 2] = (far + near) / (near - far)
    p[2, 3] = 2.0 * far * near / (near - far)
    p[3, 2] = -1.0
    return p


def view_proj(eye, width: int, height: int, vfov_deg: float = VFOV_DEG) -> np.ndarray:
    """float32 [4,4] row-major matrix M with clip = M @ [x, y, z, 1]."""
    m = perspective(vfov_deg, width / height) @ look_at(eye)
    return m.astype(np.float32)


def fibonacci_sphere(n: int, radius: float = 3.0) -> np.ndarray:
    """n points on a sphere (float64 [n,3]) by the golden-angle spiral."""
    i = np.arange(n, dtype=np.float64)
    y = 1.0 - 2.0 * (i + 0.5) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - y * y))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([r * np.cos(phi), y, r * np.sin(phi)], axis=1)


# ---------------------------------------------------------------------------
# scene pieces
# ---------------------------------------------------------------------------

def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly random rotation matrices [n,3,3] from random unit quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r = np.empty((n, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def uniform_ball(rng: np.random.Generator, n: int, radius: float = 1.0) -> np.ndarray:
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    return d * r[:, None]


def equilateral_soup(rng: np.random.Generator, centres: np.ndarray,
                     log_mean: float = -3.0, log_sigma: float = 0.5) -> np.ndarray:
    """Equilateral triangles with side exp(N(log_mean, log_sigma^2)), random
    orientation, centred at ``centres``. Returns float32 [T,3,3]."""
    n = centres.shape[0]
    side = np.exp(rng.normal(log_mean, log_sigma, n))
    circ = side / math.sqrt(3.0)
    ang = np.array([0.0, 2.0 * math.pi / 3.0, 4.0 * math.pi / 3.0])
    local = np.stack([np.cos(ang), np.sin(ang), np.zeros(3)], axis=1)  # [3,3]
    rot = random_rotations(rng, n)
    v = np.einsum('nij,kj->nki', rot, local) * circ[:, None, None] + centres[:, None, :]
    return v.astype(np.float32)


def glorot_mlp(rng: np.random.Generator, dims: Sequence[int]) -> np.ndarray:
    """Flattened parameters [W0 (d1 x d0), b0 (d1), W1, b1, ...], float32."""
    parts = []
    for fan_in, fan_out in zip(dims[:-1], dims[1:]):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-a, a, (fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def mlp_param_count(dims: Sequence[int]) -> int:
    return int(sum(o * i + o for i, o in zip(dims[:-1], dims[1:])))


# ---------------------------------------------------------------------------
# containers
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Scene:
    verts: np.ndarray          # float32 [T,3,3]
    feats: np.ndarray          # float32 [T,G,G,C]
    mlp: np.ndarray            # float32 [P]
    dims: List[int]            # [C, h1, ..., 4]

    @property
    def T(self) -> int:
        return int(self.verts.shape[0])

    @property
    def G(self) -> int:
        return int(self.feats.shape[1])

    @property
    def C(self) -> int:
        return int(self.feats.shape[3])


@dataclasses.dataclass
class View:
    width: int
    height: int
    view_id: int
    M: np.ndarray              # float32 [4,4]


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    views: List[View]
    seed: int                  # Philox key
    step: int = 0
    targets: Optional[List[np.ndarray]] = None   # float32 [H,W,3] per view

    @property
    def pixels(self) -> int:
        return int(sum(v.width * v.height for v in self.views))


def random_scene(rng, verts, G, C, dims) -> Scene:
    feats = rng.normal(0.0, 0.1, (verts.shape[0], G, G, C)).astype(np.float32)
    mlp = glorot_mlp(rng, dims)
    return Scene(verts=np.ascontiguousarray(verts, dtype=np.float32), feats=feats,
                 mlp=mlp, dims=list(dims))


def _targets(rng, views):
    return [rng.random((v.height, v.width, 3)).astype(np.float32) for v in views]


CONFIG_SEEDS = {"tiny": 1001, "single": 1002, "batched": 1003, "serving": 1004, "large": 1005, "paper": 1006}
PHILOX_SEEDS = {k: 0x5EED0000 + i + 1 for i, k in enumerate(CONFIG_SEEDS)}


def tiny(with_targets: bool = True) -> Workload:
    rng = np.random.Generator(np.random.PCG64(CONFIG_SEEDS["tiny"]))
    verts = rng.uniform(-1.0, 1.0, (64, 3, 3)).astype(np.float32)
    scene = random_scene(rng, verts, 4, 8, [8, 16, 4])
    views = [View(128, 128, 0, view_proj((0.0, 0.0, 3.0), 128, 128))]
    t = _targets(rng, views) if with_targets else None
    return Workload("tiny", scene, views, PHILOX_SEEDS["tiny"], 0, t)


def single(with_targets: bool = True, ball_radius: float = 1.0, T: int = 10_000,
           res: int = 800) -> Workload:
    rng = np.random.Generator(np.random.PCG64(CONFIG_SEEDS["single"]))
    verts = equilateral_soup(rng, uniform_ball(rng, T, ball_radius))
    scene = random_scene(rng, verts, 8, 16, [16, 32, 32, 4])
    views = [View(res, res, 0, view_proj((0.0, 0.0, 3.0), res, res))]
    t = _targets(rng, views) if with_targets else None
    return Workload("single", scene, views, PHILOX_SEEDS["single"], 0, t)


# Radius of the ball of triangle centres at which the single-view workload has
# a depth complexity of 8 (mean fragments per covered pixel), the figure the
# configuration quotes but its unit ball does not give (2.97): bisection on the
# radius with the oracle's fragment statistics gives 7.997 at this radius.
DC8_RADIUS = 0.5736


def single_dc8(with_targets: bool = True) -> Workload:
    """The single-view workload with its centres in a ball of radius
    DC8_RADIUS, for a depth complexity of 8."""
    w = single(with_targets=with_targets, ball_radius=DC8_RADIUS)
    w.name = "single_dc8"
    return w


BATCHED_RES = (256, 512, 800, 1024)


def batched(with_targets: bool = True, n_views: int = 64, T: int = 50_000) -> Workload:
    rng = np.random.Generator(np.random.PCG64(CONFIG_SEEDS["batched"]))
    verts = equilateral_soup(rng, uniform_ball(rng, T))
    scene = random_scene(rng, verts, 8, 16, [16, 32, 32, 4])
    eyes = fibonacci_sphere(n_views, 3.0)
    res = rng.choice(np.array(BATCHED_RES), size=n_views)
    views = [View(int(r), int(r), i, view_proj(eyes[i], int(r), int(r))) for i, r in enumerate(res)]
    t = _targets(rng, views) if with_targets else None
    return Workload("batched", scene, views, PHILOX_SEEDS["batched"], 0, t)


def large(with_targets: bool = True, n_views: int = 16, blobs: int = 16,
          per_blob: int = 12_500, width: int = 1920, height: int = 1080) -> Workload:
    rng = np.random.Generator(np.random.PCG64(CONFIG_SEEDS["large"]))
    centres_b = uniform_ball(rng, blobs)
    centres = np.concatenate([rng.normal(centres_b[b], 0.15, (per_blob, 3)) for b in range(blobs)])
    verts = equilateral_soup(rng, centres)
    scene = random_scene(rng, verts, 8, 32, [32, 64, 64, 4])
    eyes = fibonacci_sphere(n_views, 3.0)
    views = [View(width, height, i, view_proj(eyes[i], width, height)) for i in range(n_views)]
    t = _targets(rng, views) if with_targets else None
    return Workload("large", scene, views, PHILOX_SEEDS["large"], 0, t)


SERVING_SOUPS = (20_000, 40_000, 70_000, 100_000)
SERVING_RES = ((640, 360), (1280, 720), (1920, 1080))


def serving_soups() -> List[Scene]:
    rng = np.random.Generator(np.random.PCG64(CONFIG_SEEDS["serving"]))
    out = []
    for T in SERVING_SOUPS:
        verts = equilateral_soup(rng, uniform_ball(rng, T))
        out.append(random_scene(rng, verts, 8, 16, [16, 32, 32, 4]))
    return out


@dataclasses.dataclass
class Request:
    arrival_s: float
    soup: int
    view: View


def serving_requests(rate_hz: float, duration_s: float, seed: int = 1004_1) -> List[Request]:
    """Poisson arrivals; soup uniform; resolution uniform; camera direction
    uniform on the sphere of radius 3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    i = 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        soup = int(rng.integers(0, len(SERVING_SOUPS)))
        w, h = SERVING_RES[int(rng.integers(0, len(SERVING_RES)))]
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        out.append(Request(t, soup, View(w, h, i, view_proj(3.0 * d, w, h))))
        i += 1
    return out


# ---------------------------------------------------------------------------
# paper form: mesh-colour texture levels and the deferred-shading MLP
# ---------------------------------------------------------------------------

PF_MLP_DIMS = [16, 16, 16, 3]       # 7 features + 9 harmonics -> 16 -> 16 -> RGB
PF_CHANNELS = 8                     # 7 colour features, then the opacity


def mc_vertices(R: int) -> int:
    """Grid vertices of a level-R mesh-colour grid (n = 2^R segments per edge)."""
    n = 1 << R
    return (n + 1) * (n + 2) // 2


def inv_view_proj(M: np.ndarray) -> np.ndarray:
    """The inverse of a float32 view-projection matrix, taken in float64 and
    rounded once to float32 (an input of the deferred shading)."""
    return np.linalg.inv(np.asarray(M, np.float64)).astype(np.float32)


@dataclasses.dataclass
class PScene:
    """A paper-form scene: per-triangle activated texture tex [T, V(R), 8] in
    [0, 1] (grid vertex (i, j) of the level-R grid at row-major index
    j (n + 1) - j (j - 1) / 2 + i) and the shading MLP's flat parameters."""
    verts: np.ndarray          # float32 [T,3,3]
    tex: np.ndarray            # float32 [T,V(R),8]
    mlp: np.ndarray            # float32 [P]
    R: int

    @property
    def T(self) -> int:
        return int(self.verts.shape[0])


@dataclasses.dataclass
class PLevels:
    """The learnable texture levels Rmin..Rtop ([T, V(level), 8] each, before
    the sigmoid) accumulated on the level-Rmax grid."""
    raw: List[np.ndarray]
    Rmin: int
    Rmax: int

    @property
    def Rtop(self) -> int:
        return self.Rmin + len(self.raw) - 1


def random_pscene(rng, verts, R: int = 5, lo: float = 0.05, hi: float = 0.95) -> PScene:
    """Activated texture values U[lo, hi] per grid vertex and channel, Glorot
    MLP with small random biases."""
    T = verts.shape[0]
    tex = rng.uniform(lo, hi, (T, mc_vertices(R), PF_CHANNELS)).astype(np.float32)
    mlp = glorot_mlp(rng, PF_MLP_DIMS)
    nW = [o * i for i, o in zip(PF_MLP_DIMS[:-1], PF_MLP_DIMS[1:])]
    at = 0
    for l, w in enumerate(nW):
        at += w
        o = PF_MLP_DIMS[l + 1]
        mlp[at:at + o] = rng.normal(0.0, 0.1, o)
        at += o
    return PScene(np.ascontiguousarray(verts, np.float32), tex, mlp, R)


def random_levels(rng, T: int, Rmin: int, Rtop: int, Rmax: int, sd: float = 0.5) -> PLevels:
    """Raw texture levels N(0, sd^2) (the paper starts them at zero; random
    values make every level's contribution visible)."""
    raw = [rng.normal(0.0, sd, (T, mc_vertices(R), PF_CHANNELS)).astype(np.float32)
           for R in range(Rmin, Rtop + 1)]
    return PLevels(raw, Rmin, Rmax)


@dataclasses.dataclass
class PWorkload:
    """The paper form's training step: a soup, its learnable texture levels
    Rmin..Rmax-1 accumulated on the level-Rmax grid, the shading MLP, views
    and targets."""
    name: str
    verts: np.ndarray
    levels: PLevels
    mlp: np.ndarray
    views: List[View]
    seed: int
    step: int = 0
    targets: Optional[List[np.ndarray]] = None

    @property
    def pixels(self) -> int:
        return int(sum(v.width * v.height for v in self.views))

    @property
    def T(self) -> int:
        return int(self.verts.shape[0])


def paper(with_targets: bool = True, T: int = 50_000, n_views: int = 4, res: int = 800, Rmin: int = 2,
          Rmax: int = 5) -> PWorkload:
    """The paper form at the paper's second training stage (levels 2..4 onto
    the level-5 grid, 561 vertices per triangle) and its batch of four
    views, on the batched workload's kind of soup: 50,000 triangles, views of
    800 x 800 on a sphere of radius 3."""
    rng = np.random.Generator(np.random.PCG64(CONFIG_SEEDS["paper"]))
    verts = equilateral_soup(rng, uniform_ball(rng, T))
    levels = random_levels(rng, T, Rmin, Rmax - 1, Rmax)
    mlp = random_pscene(rng, verts[:1], 0).mlp
    eyes = fibonacci_sphere(n_views, 3.0)
    views = [View(res, res, i, view_proj(eyes[i], res, res)) for i in range(n_views)]
    t = _targets(rng, views) if with_targets else None
    return PWorkload("paper", verts, levels, mlp, views, PHILOX_SEEDS["paper"], 0, t)


def by_name(name: str, **kw) -> Workload:
    return {"tiny": tiny, "single": single, "single_dc8": single_dc8, "batched": batched,
            "large": large}[name](**kw)


# ---------------------------------------------------------------------------
# small hand-built scenes used by the tests
# ---------------------------------------------------------------------------

def identity_mlp_dims(C: int = 8, H: int = 16) -> List[int]:
    return [C, H, 4]


def passthrough_mlp(C: int = 8, H: int = 16) -> np.ndarray:
    """MLP C->H->4 whose outputs equal features 1,2,3 (RGB logits) and
    feature 0 (opacity logit) exactly: hidden units carry +x_k and -x_k through
    the ReLU and the output layer subtracts them."""
    assert H >= 8
    W0 = np.zeros((H, C), np.float32)
    b0 = np.zeros(H, np.float32)
    W1 = np.zeros((4, H), np.float32)
    b1 = np.zeros(4, np.float32)
    src = [1, 2, 3, 0]       # output j reads feature src[j]
    for j, k in enumerate(src):
        W0[2 * j, k] = 1.0
        W0[2 * j + 1, k] = -1.0
        W1[j, 2 * j] = 1.0
        W1[j, 2 * j + 1] = -1.0
    return np.concatenate([W0.ravel(), b0, W1.ravel(), b1]).astype(np.float32)
