"""Seeded synthetic inputs for the dual-quaternion Julia ray-march workloads.

This module is the only code shared by the FP64 oracle and the GPU path. It
holds parameter records and seeded generators and none of the method's
arithmetic: no algebra, no iteration, no camera basis, no ray or shading maths.
Every floating-point parameter is drawn in FP64 and rounded once to FP32, so
both sides receive bit-identical values and any difference between them comes
from arithmetic alone.

Conventions fixed here (both sides read them from these records):

* A dual quaternion is 8 reals ``[r0 r1 r2 r3 | d0 d1 d2 d3]``: the real
  quaternion first, the dual quaternion second, slot 0 of each the scalar
  (the iteration formula of Eq. quatsq squares its first slot as the scalar;
  the paper's printed constants write a complex number as ``(re, im, 0, 0)``).
* The default 3D slice maps a world point ``(X, Y, Z)`` to
  ``(X, Y, Z, 0 | 0, 0, 0, 0)``: five components held constant at zero
  (section "Dimension Reduction").
* The camera is a pinhole at radius 3 looking at the origin, 60 degree
  vertical field of view, pixel centres, row 0 at the top.
* Lighting is one directional light towards ``(1, 1, 1)`` with
  ``k_a = 0.1`` and ``k_d = 0.9`` (the ambient and diffuse terms of Eq. phong).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

NORM_EUCLID8 = 0      # escape on the sum of all 8 squares (default reading)
NORM_REALPART = 1     # escape on the real quaternion's 4 squares only

PREC_FP32 = 0
PREC_SPLIT = 1
PREC_FP64 = 2

MARCH_FIXED = 0       # S fixed steps over the box segment, then bisection
MARCH_DE = 1          # distance-estimate steps (the paper's own march)

ALGEBRA_DUAL = 0           # (a + b e)^2 = a^2 + (ab + ba) e, the product rule
ALGEBRA_COMPONENTWISE = 1  # a^2 + b^2 e, the form printed with the iteration

NORMAL_POTENTIAL = 0    # central differences of the escape potential
NORMAL_NEIGHBOUR4 = 1   # from the four neighbouring pixels' hit points


def f32(x: float) -> float:
    """Round one FP64 value to the nearest FP32 value (returned as a Python float)."""
    return float(np.float32(x))


def f32v(xs: Sequence[float]) -> List[float]:
    return [f32(x) for x in xs]


def default_eye(radius: float = 3.0, azimuth_deg: float = 30.0,
                elevation_deg: float = 20.0) -> List[float]:
    """Camera position on a sphere of ``radius`` around the origin (input recipe only)."""
    az = math.radians(azimuth_deg)
    el = math.radians(elevation_deg)
    return f32v([radius * math.cos(el) * math.sin(az),
                 radius * math.sin(el),
                 radius * math.cos(el) * math.cos(az)])


def identity_slice():
    """(X, Y, Z) -> (X, Y, Z, 0 | 0, 0, 0, 0)."""
    origin = [0.0] * 8
    axes = [[0.0] * 8 for _ in range(3)]
    axes[0][0] = 1.0
    axes[1][1] = 1.0
    axes[2][2] = 1.0
    return origin, axes


@dataclasses.dataclass
class Params:
    """One render request. Field meanings follow the C ABI's ``dqj_params``.

    All floats are already FP32-representable (see module docstring).
    """
    c: List[float]
    width: int
    height: int
    max_iter: int
    march_steps: int
    bisect_steps: int
    escape_radius: float = 4.0
    slice_origin: List[float] = dataclasses.field(default_factory=lambda: identity_slice()[0])
    slice_axes: List[List[float]] = dataclasses.field(default_factory=lambda: identity_slice()[1])
    box_min: List[float] = dataclasses.field(default_factory=lambda: [-1.5, -1.5, -1.5])
    box_max: List[float] = dataclasses.field(default_factory=lambda: [1.5, 1.5, 1.5])
    eye: List[float] = dataclasses.field(default_factory=default_eye)
    target: List[float] = dataclasses.field(default_factory=lambda: [0.0, 0.0, 0.0])
    up: List[float] = dataclasses.field(default_factory=lambda: [0.0, 1.0, 0.0])
    fov_y_deg: float = 60.0
    norm: int = NORM_EUCLID8
    precision: int = PREC_FP32
    fp64_window: int = 2
    normal_h: float = 1e-3
    light_dir: List[float] = dataclasses.field(default_factory=lambda: [1.0, 1.0, 1.0])
    k_ambient: float = 0.1
    k_diffuse: float = 0.9
    march: int = MARCH_FIXED
    de_hit_eps: float = 1e-4
    de_min_step: float = 1e-4
    de_max_step: float = 0.25
    algebra: int = ALGEBRA_DUAL
    normal_mode: int = NORMAL_POTENTIAL
    k_specular: float = 0.0
    shininess: float = 16.0
    cull_radius: float = 0.0
    fiber: Optional[np.ndarray] = None   # projection: F x 8 offsets in R^8 (None: slice)

    def __post_init__(self):
        self.c = f32v(self.c)
        self.escape_radius = f32(self.escape_radius)
        self.slice_origin = f32v(self.slice_origin)
        self.slice_axes = [f32v(a) for a in self.slice_axes]
        self.box_min = f32v(self.box_min)
        self.box_max = f32v(self.box_max)
        self.eye = f32v(self.eye)
        self.target = f32v(self.target)
        self.up = f32v(self.up)
        self.fov_y_deg = f32(self.fov_y_deg)
        self.normal_h = f32(self.normal_h)
        self.light_dir = f32v(self.light_dir)
        self.k_ambient = f32(self.k_ambient)
        self.k_diffuse = f32(self.k_diffuse)
        self.de_hit_eps = f32(self.de_hit_eps)
        self.de_min_step = f32(self.de_min_step)
        self.de_max_step = f32(self.de_max_step)
        self.k_specular = f32(self.k_specular)
        self.shininess = f32(self.shininess)
        self.cull_radius = f32(self.cull_radius)
        if self.fiber is not None:
            a = np.asarray(self.fiber, dtype=np.float64).reshape(-1, 8)
            self.fiber = np.ascontiguousarray(a.astype(np.float32).astype(np.float64))

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)

    @property
    def pixels(self) -> int:
        return self.width * self.height


def seeded_c(seed: int, real_amp: float = 0.6, dual_amp: float = 0.5) -> List[float]:
    """Dual-quaternion constant from a seed: real comps U[-a, a], dual comps U[-0.5, 0.5]."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(-real_amp, real_amp, 4)
    d = rng.uniform(-dual_amp, dual_amp, 4)
    return f32v(list(r) + list(d))


# Constants printed in the paper's figure captions (Fig. test2, Fig. highres2,
# Fig. highres). The first caption's "-023" is read as -0.23.
PAPER_C = [
    [-0.10, 0.8, -0.26, 0.15, -0.23, -0.38, -0.86, 0.64],
    [-0.67, -0.54, -0.07, 0.02, 0.06, -0.53, 0.15, -0.27],
    [-0.98, 0.27, 0.40, 0.20, -0.37, -0.41, -0.24, -0.34],
    [0.35, 0.78, 0.85, -0.57, -0.22, 0.06, -0.46, 0.05],
    [-0.17, -0.28, 0.11, 0.8, 0.06, 0.44, -0.66, 0.06],
    [-0.04, 0.95, 0.4, -0.43, 0.09, -0.45, -0.27, -0.31],
    [-0.04, 0.95, 0.4, -0.43, 0.09, -0.35, -0.27, -0.31],   # Fig. highres2, n = 15
    [-0.39054, -0.58679, 0.0, 0.0, 0.0, 0.5632, 0.0, 0.05],  # Fig. highres, n = 15
]


# --------------------------------------------------------------------------
# The five workloads. Each returns a list of Params (one per frame/request).
# --------------------------------------------------------------------------

def plain_128(seed: int = 0) -> List[Params]:
    """128x128 FP32, max_iter 12, 128 march steps, 8 bisection steps."""
    return [Params(c=seeded_c(seed, 0.6), width=128, height=128, max_iter=12,
                   march_steps=128, bisect_steps=8)]


def plain_1024(seeds: Sequence[int] = (0, 1, 2)) -> List[Params]:
    """1024x1024 FP32, 3 seeded c, max_iter 24, 512 march steps, 10 bisection steps."""
    return [Params(c=seeded_c(s, 0.6), width=1024, height=1024, max_iter=24,
                   march_steps=512, bisect_steps=10) for s in seeds]


def split_1080p(seeds: Sequence[int] = tuple(range(8))) -> List[Params]:
    """1920x1080 split precision: FP16 512-step march, FP32 12-step bisection, FP64 window 2."""
    return [Params(c=seeded_c(s, 0.6), width=1920, height=1080, max_iter=32,
                   march_steps=512, bisect_steps=12, precision=PREC_SPLIT,
                   fp64_window=2) for s in seeds]


def sweep_256(n: int = 4096, first_seed: int = 0) -> List[Params]:
    """Parameter sweep: n seeded c (real comps U[-0.8, 0.8]), each 256x256, max_iter 16."""
    return [Params(c=seeded_c(first_seed + i, 0.8), width=256, height=256, max_iter=16,
                   march_steps=256, bisect_steps=8) for i in range(n)]


def voxel_grid(n: int, c: Optional[Sequence[float]] = None, max_iter: int = 15,
               algebra: int = ALGEBRA_DUAL) -> Tuple[Params, Tuple[int, int, int]]:
    """Dense voxel grid over the box [-1.5, 1.5]^3: n^3 voxel centres, identity slice,
    R = 4. Default constant and max_iter: the paper's high-detail figure (PAPER_C[7],
    n = 15), whose set fills about 3.6% of the box. Returns (params, (nx, ny, nz))."""
    return (Params(c=list(c) if c is not None else list(PAPER_C[7]), width=64, height=64,
                   max_iter=max_iter, march_steps=64, bisect_steps=0, algebra=algebra),
            (n, n, n))


def voxel_100() -> Tuple[Params, Tuple[int, int, int]]:
    """The paper's larger voxel prototype size, 100^3."""
    return voxel_grid(100)


def voxel_1024() -> Tuple[Params, Tuple[int, int, int]]:
    """1024^3 voxels (1.07e9) of the high-detail constant: the throughput case."""
    return voxel_grid(1024)


def animated_slices(n: int = 16, side: int = 256) -> List[Params]:
    """An animated slice (section "Dimension Reduction"): n frames of the paper's
    high-detail constant (PAPER_C[7], n = 15) whose third slice axis turns from the real
    k axis into the dual part's scalar axis, W = cos(theta) e2 + sin(theta) e4 with
    theta = f/(n-1) * pi/2, so the last frame slices (X, Y, d0). Each frame is an ordinary
    render; a batch renders the sequence."""
    out: List[Params] = []
    for f in range(n):
        th = 0.5 * math.pi * f / max(n - 1, 1)
        w = [0.0] * 8
        w[2], w[4] = math.cos(th), math.sin(th)
        axes = [[1.0, 0, 0, 0, 0, 0, 0, 0], [0, 1.0, 0, 0, 0, 0, 0, 0], w]
        out.append(Params(c=list(PAPER_C[7]), width=side, height=side, max_iter=15,
                          march_steps=256, bisect_steps=8, slice_axes=axes))
    return out


SERVE_SIDES = (128, 256, 512, 1024, 2048)


@dataclasses.dataclass
class Arrival:
    t: float          # scheduled arrival time, seconds from stream start
    params: Params


def serve_stream(duration_s: float = 60.0, rate_hz: float = 200.0, seed: int = 5,
                 first_request_seed: int = 100000, precision: int = PREC_SPLIT,
                 sides: Sequence[int] = SERVE_SIDES) -> List[Arrival]:
    """Poisson request stream: exponential inter-arrival times of mean 1/rate.

    Request i: c from seed ``first_request_seed + i`` (real amp 0.6), square side
    uniform over ``sides``, max_iter uniform integer in [8, 64], march steps
    2 * max_iter * 8, 10 bisection steps.
    """
    rng = np.random.default_rng(seed)
    out: List[Arrival] = []
    t = 0.0
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        side = int(sides[int(rng.integers(0, len(sides)))])
        n_iter = int(rng.integers(8, 65))
        p = Params(c=seeded_c(first_request_seed + i, 0.6), width=side, height=side,
                   max_iter=n_iter, march_steps=2 * n_iter * 8, bisect_steps=10,
                   precision=precision)
        out.append(Arrival(t=t, params=p))
        i += 1
    return out


def de_128(seed: int = 0) -> List[Params]:
    """plain_128 marched by distance estimates (at most 128 steps)."""
    return [p.replace(march=MARCH_DE) for p in plain_128(seed)]


def de_1024(seeds: Sequence[int] = (0, 1, 2)) -> List[Params]:
    """plain_1024 marched by distance estimates: the same frames, at most 512 steps,
    hit below 1e-4, steps clamped to [1e-4, 0.25]."""
    return [p.replace(march=MARCH_DE) for p in plain_1024(seeds)]


def fiber_ball(count: int, radius: float, seed: int) -> np.ndarray:
    """count offsets in R^8 for a projection of the identity slice: the zero offset, then
    seeded points uniform in the ball of the given radius in the five collapsed
    coordinates (a3 and b0..b3)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count, 8))
    for f in range(1, count):
        while True:
            v = rng.uniform(-radius, radius, 5)
            if float(v @ v) <= radius * radius:
                break
        out[f, 3:] = v
    return out


def project_128(seed: int = 0, fibers: int = 8) -> List[Params]:
    """A projection (section "Dimension Reduction", approach 2) of plain_128's set: the
    shadow of the set on the identity slice's 3D space, its fibre sampled by `fibers`
    offsets (the zero offset and points of the 5-ball of radius 0.5)."""
    return [p.replace(fiber=fiber_ball(fibers, 0.5, 100 + seed)) for p in plain_128(seed)]


PROJECT_C = (7, 0, 4)   # the paper's printed constants whose sets fill the view


def project_512(fibers: int = 16) -> List[Params]:
    """Three 512x512 shadows of sets of the paper's printed constants (PAPER_C[7], [0],
    [4]; max_iter 15, 256 march steps, 10 bisection steps), each fibre sampled by 16
    offsets (zero and 15 points of the 5-ball of radius 0.5)."""
    return [Params(c=list(PAPER_C[ci]), width=512, height=512, max_iter=15, march_steps=256,
                   bisect_steps=10, fiber=fiber_ball(fibers, 0.5, 100 + f))
            for f, ci in enumerate(PROJECT_C)]


def scene_extent(p: Params) -> float:
    """Length of the box diagonal: the scale the depth tolerance is quoted in."""
    return math.sqrt(sum((b - a) ** 2 for a, b in zip(p.box_min, p.box_max)))


WORKLOADS = {
    "plain_128": plain_128,
    "plain_1024": plain_1024,
    "de_128": de_128,
    "de_1024": de_1024,
    "voxel_100": voxel_100,
    "voxel_1024": voxel_1024,
    "split_1080p": split_1080p,
    "sweep_256": sweep_256,
    "project_128": project_128,
    "project_512": project_512,
}
