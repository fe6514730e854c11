"""Seeded synthetic workloads (grids, constraints, loads, crack segments).

Problem definitions only -- no part of the method's arithmetic lives here -- so that
the GPU library and the CPU oracle are driven by identical inputs.  Random arrays
come from numpy's PCG64 seeded with [config_id, case_id].

The paper measures on parametric plates and blocks described in prose (Sec. 5);
these stand in for them at the sizes the benchmark configurations name:
  plate32   2D static, 32 x 32, delta = 3h, u = 0 on a delta-wide layer on all sides
  plate512  2D static, 512 x 512, delta = 3h, left layer fixed, band load at the right
  crack1024 2D dynamic, 1024 x 1024, delta = 4h, 30-degree pre-crack, opposing edge loads
  cube128   3D static, 128^3, delta = 3h, z = 0 layer fixed, 16 load cases
  plates64  2D differentiable batch of 64 plates of sizes {64..384}^2
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


def rng(config_id: int, case_id: int = 0) -> np.random.Generator:
    return np.random.default_rng([config_id, case_id])


def alpha_plane(E: float, delta: float, thickness: float = 1.0) -> float:
    """Micromodulus scale of a 2D plate, 9E/(pi delta^3 t) (material constant, Sec. 2.1)."""
    return 9.0 * E / (math.pi * delta ** 3 * thickness)


def alpha_solid(E: float, delta: float) -> float:
    """Micromodulus scale of a 3D body, 12E/(pi delta^4) (Sec. 2.1)."""
    return 12.0 * E / (math.pi * delta ** 4)


def node_index_grids(n: Sequence[int]):
    """Per-axis integer node index arrays, flattened in node order (x fastest)."""
    idx = np.unravel_index(np.arange(int(np.prod(n))), tuple(n)[::-1])
    return [idx[len(n) - 1 - a] for a in range(len(n))]


def layer_mask(n: Sequence[int], M: int, faces: Sequence[tuple]) -> np.ndarray:
    """Constrained-DOF mask [dim][N]: nodes whose centre lies within delta = M h of one of
    the listed faces (axis, side), side 0 = low, 1 = high; all components constrained."""
    d = len(n)
    ix = node_index_grids(n)
    m = np.zeros(int(np.prod(n)), dtype=bool)
    for axis, side in faces:
        m |= (ix[axis] < M) if side == 0 else (ix[axis] >= n[axis] - M)
    return np.repeat(m[None], d, axis=0)


ALL_SIDES_2D = [(0, 0), (0, 1), (1, 0), (1, 1)]


@dataclass
class Workload:
    name: str
    n: tuple
    h: float
    M: int
    alpha: float
    rho: float = 1.0
    infl: tuple = ()
    fixed: Optional[np.ndarray] = None     # [dim][N] bool
    b: Optional[np.ndarray] = None         # [B][dim][N] float64
    g: Optional[np.ndarray] = None         # [B][dim][N] float64 or None
    cracks: Optional[np.ndarray] = None    # [ns][4] segments
    dt: float = 0.0
    steps: int = 0
    tol: float = 1e-10
    extra: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def batch(self) -> int:
        return 1 if self.b is None else self.b.shape[0]

    @property
    def dofs(self) -> int:
        return self.dim * self.N


def plate32() -> Workload:
    n, M = (32, 32), 3
    h = 1.0 / 32
    r = rng(1)
    return Workload("plate32", n, h, M, alpha_plane(1.0, M * h),
                    fixed=layer_mask(n, M, ALL_SIDES_2D),
                    b=r.standard_normal((1, 2, 32 * 32)), tol=1e-10)


def plate512() -> Workload:
    n, M = (512, 512), 3
    h = 1.0 / 512
    r = rng(2)
    b = 0.1 * r.standard_normal((1, 2, 512 * 512))
    ix = node_index_grids(n)
    b[0, 0, ix[0] == n[0] - 1] += 1.0 / h          # band of width h at the right edge
    return Workload("plate512", n, h, M, alpha_plane(1.0, M * h),
                    fixed=layer_mask(n, M, [(0, 0)]), b=b, tol=1e-10)


def crack_segment(center=(0.5, 0.5), length=0.3, angle_deg=30.0) -> np.ndarray:
    c, s = math.cos(math.radians(angle_deg)), math.sin(math.radians(angle_deg))
    hl = 0.5 * length
    return np.array([[center[0] - hl * c, center[1] - hl * s, center[0] + hl * c, center[1] + hl * s]])


def crack1024(n_side: int = 1024, steps: int = 1000) -> Workload:
    n, M = (n_side, n_side), 4
    h = 1.0 / n_side
    delta = M * h
    c = alpha_plane(1.0, delta)
    ix = node_index_grids(n)
    b = np.zeros((1, 2, n_side * n_side))
    b[0, 1, ix[1] >= n_side - M] = 1.0                # +y on the top M rows
    b[0, 1, ix[1] < M] = -1.0                         # -y on the bottom M rows
    dt = 0.5 * h / math.sqrt(c * delta * delta)
    return Workload("crack1024", n, h, M, c, rho=1.0, b=b, cracks=crack_segment(), dt=dt, steps=steps)


def cube128(batch: int = 16, n_side: int = 128) -> Workload:
    n, M = (n_side,) * 3, 3
    h = 1.0 / n_side
    N = n_side ** 3
    b = np.empty((batch, 3, N))
    for c in range(batch):
        b[c] = rng(4, c).standard_normal((3, N))
    return Workload("cube128", n, h, M, alpha_solid(1.0, M * h),
                    fixed=layer_mask(n, M, [(2, 0)]), b=b, tol=1e-8)


def plates64(count: int = 64, sizes=(64, 128, 192, 256, 384), n_infl: int = 8) -> List[Workload]:
    """64 plates, sizes drawn uniformly, omega = sum_k a_k (r/delta)^k with a_k ~ U[0,1),
    Dirichlet layer on all sides, b ~ N(0,1); target coefficients a'_k = max(0, a_k(1 + 0.05 z))."""
    r = rng(5)
    pick = r.integers(0, len(sizes), size=count)
    out = []
    for i in range(count):
        s = int(sizes[pick[i]])
        rc = rng(5, i + 1)
        a = rc.uniform(0.0, 1.0, size=n_infl)
        at = np.maximum(0.0, a * (1.0 + 0.05 * rc.standard_normal(n_infl)))
        n, M, h = (s, s), 3, 1.0 / s
        w = Workload("plates64[%d]" % i, n, h, M, alpha_plane(1.0, M * h), infl=tuple(a),
                     fixed=layer_mask(n, M, ALL_SIDES_2D), b=rc.standard_normal((1, 2, s * s)),
                     tol=1e-10)
        w.extra["infl_target"] = tuple(at)
        out.append(w)
    return out


def small(dim: int, n: Sequence[int], M: int, seed: int, fixed: str = "none", crack: bool = False,
          batch: int = 1, infl: tuple = (), E: float = 1.0) -> Workload:
    """Small seeded case for parity tests: ragged sizes, optional constraints and crack."""
    n = tuple(int(x) for x in n)
    h = 1.0 / max(n)
    r = rng(100 + seed)
    alpha = alpha_plane(E, M * h) if dim == 2 else alpha_solid(E, M * h)
    if fixed == "all":
        faces = [(a, s) for a in range(dim) for s in (0, 1)]
    elif fixed == "left":
        faces = [(0, 0)]
    elif fixed == "bottom":
        faces = [(dim - 1, 0)]
    else:
        faces = []
    fx = layer_mask(n, M, faces) if faces else None
    if fixed == "mixed":
        # Remark 2: x constrained on the left layer, y free there
        fx = layer_mask(n, M, [(0, 0)])
        fx[1:] = False
    N = int(np.prod(n))
    cracks = None
    if crack and dim == 2:
        W, Hh = n[0] * h, n[1] * h
        cracks = np.array([[0.2 * W + 0.013 * h, 0.35 * Hh + 0.007 * h, 0.7 * W + 0.011 * h, 0.62 * Hh + 0.003 * h]])
    return Workload("small%dd_%s" % (dim, "x".join(map(str, n))), n, h, M, alpha, infl=tuple(infl),
                    fixed=fx, b=r.standard_normal((batch, dim, N)), cracks=cracks)
