"""CPU oracle for the linear bond-based peridynamic model, FP64.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the GPU library; only the seeded input generators are common to both.

Every function is the plain definition of what the paper's method reproduces
exactly ("without loss of accuracy", Sec. 1): the meshfree sum of eq. (mat:f1)
evaluated bond by bond (``oracle_core.c``), the dense stiffness matrix of
eqs. (matrix)/(mae:e1), and the model equations built on it:

* ``force``/``apply``      -- f = A u, eq. (mat:f1); constrained rows reported as 0
                              (their content is arbitrary, Remark 1); optionally with
                              the surface correction of Remark 3 / eq. (scr).
* ``surface_volume_factors`` -- per-node factors nu_p = (full-horizon volume) / (volume
                              of the horizon inside the grid), partial volumes lambda.
* ``assemble_dense``       -- A, eq. (matrix); used at small sizes only.
* ``solve_dense``          -- static model eq. (mat:e2): K = -A, K_FF u_F =
                              b_F - K_FC g_C, u_C = g_C (Sec. 3.4, eq. (up));
                              dense Cholesky.
* ``solve_cg``             -- the same system by conjugate gradients with the
                              bond-sum apply (for grids too big to factor).
* ``vv``                   -- velocity Verlet, Alg. 2, with a = (A u + b)/rho and
                              constrained DOFs overwritten after each update (eq. (up)).
* ``energy``, ``energy_parts`` -- kinetic + elastic - external work of the discrete system
                              (and the three terms on their own).
* ``adr_step``/``adr``     -- the quasi-static model by adaptive dynamic relaxation (Sec. 2.2,
                              eq. (ADR:e1), Alg. 1, CDEI) with the fictitious density and the
                              adaptive damping of the cited ADR method (Kilic and Madenci):
                              one update, and a run of updates.
* ``grad_dense``           -- exact gradient of ||u - u_t||^2 w.r.t. the body force
                              and the influence coefficients a_k (omega = sum_k a_k (r/delta)^k).
* ``grad_cg``              -- the same gradient with the two solves by CG (large plates).
* ``crack_to_bonds``       -- broken set of eq. (mu) for a pre-crack: a bond is broken
                              iff its segment properly crosses a crack segment.
* ``bond_stretch``         -- s of eq. (fra:s1) for given bonds, from node coordinates.
* ``crack_update``         -- the new broken set of eq. (mu): every unbroken bond with
                              s >= s0, brute force over every bond of the horizon.
* ``generating_blocks``    -- the d x d blocks G(o) of the Toeplitz generating array
                              (Sec. 3.2 / 4), read off the bond-sum force of a unit
                              displacement at the centre of a (2M+1)^d grid.
* ``periodic_apply``       -- the L-periodic operator with that generating array, by
                              direct convolution (for pins).
* ``fft_setup``/``fft_apply`` -- f = A u by the paper's fast method itself on the CPU (the
                              assembly of spectra and D^e; then Alg. 3 / Alg. 4 with D^e and
                              D^f, Sec. 3.3-3.6), with scipy's FFT: a timing reference for the
                              CPU baseline, pinned to ``apply``.
* ``precond_apply``        -- the circulant preconditioner of the preconditioned solver
                              (prior fast methods cited in Sec. 1; not part of MSBFM):
                              z = Pi_F E^T (K_per + s I)^{-1} E r, K_per = -A_per,
                              inverted per frequency with numpy's FFT.

Parity of the paper's own displacement results is unpinned (they are figures
only and are absent from the text); the tests pin this oracle with
invariants and closed forms instead.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_core.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile ``oracle_core.c`` with gcc (IEEE FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_oracle(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_force_rows.argtypes = [ctypes.c_int, P, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_int, P, P, P, P, P,
                                          ctypes.c_int64, P, P]
        lib.oracle_force_rows.restype = None
        lib.oracle_assemble_dense.argtypes = [ctypes.c_int, P, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_int, P, P, P, P]
        lib.oracle_assemble_dense.restype = None
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Problem:
    """Uniform-grid linear BB-PD problem (Sec. 3 for 2D, Sec. 4 for 3D).

    n      -- nodes per axis (nx, ny) or (nx, ny, nz); node (i,j,k) at ((i+1/2)h, ...)
    h      -- grid spacing; node volume V = h^dim
    M      -- horizon in cells, delta = M h
    alpha  -- micromodulus scale of eq. (ker:e1) (caller computes it, Sec. 2.1)
    infl   -- influence coefficients a_k, omega(r) = sum_k a_k (r/delta)^k; empty -> 1
    rho    -- mass density (dynamic model, eq. (mat:e1))
    """
    n: Sequence[int]
    h: float
    M: int
    alpha: float
    infl: Sequence[float] = field(default_factory=tuple)
    rho: float = 1.0

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def delta(self) -> float:
        return self.M * self.h

    def node_coords(self) -> np.ndarray:
        """[dim][N] node coordinates x = (i + 1/2) h, node id (k*ny + j)*nx + i."""
        axes = [(np.arange(m) + 0.5) * self.h for m in self.n]
        grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
        return np.stack([g.reshape(-1) for g in grids])


def alpha_2d(E: float, delta: float, thickness: float = 1.0) -> float:
    """alpha = 9E / (pi delta^3 t), plane stress/strain (Sec. 2.1)."""
    return 9.0 * E / (math.pi * delta ** 3 * thickness)


def alpha_3d(E: float, delta: float) -> float:
    """alpha = 12E / (pi delta^4) (Sec. 2.1)."""
    return 12.0 * E / (math.pi * delta ** 4)


def broken_csr(N: int, pairs: Optional[np.ndarray]):
    """Per-node sorted neighbour lists of the broken set (mu = 0, eq. (mu))."""
    if pairs is None or len(pairs) == 0:
        return None, None
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    src = np.concatenate([pairs[:, 0], pairs[:, 1]])
    dst = np.concatenate([pairs[:, 1], pairs[:, 0]])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    ptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(ptr, src + 1, 1)
    ptr = np.cumsum(ptr)
    return np.ascontiguousarray(ptr), np.ascontiguousarray(dst)


def _infl_arr(prob: Problem):
    a = np.ascontiguousarray(np.asarray(prob.infl, dtype=np.float64))
    return a, len(a)


def force(prob: Problem, u: np.ndarray, broken=None, rows: Optional[np.ndarray] = None,
          nu: Optional[np.ndarray] = None) -> np.ndarray:
    """f = A u evaluated bond by bond, eq. (mat:f1), on every row (or on ``rows``).

    nu: per-node surface-correction factors [N] (Remark 3, eq. (scr)): rows of nodes
    within M of a face scale each bond by (nu_p + nu_q) / 2.
    u: [dim][N] (or flat).  Returns [dim][N] (or [dim][len(rows)])."""
    lib = _load()
    d, N = prob.dim, prob.N
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(d, N))
    n = np.array(list(prob.n) + [1] * (3 - d), dtype=np.int64)
    ptr, idx = broken_csr(N, broken)
    infl, ni = _infl_arr(prob)
    if rows is not None:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        nr = len(rows)
    else:
        nr = N
    f = np.empty((d, nr), dtype=np.float64)
    nuv = None if nu is None else np.ascontiguousarray(np.asarray(nu, dtype=np.float64).reshape(N))
    lib.oracle_force_rows(d, _ptr(n), prob.h, prob.M, prob.alpha, ni,
                          _ptr(infl) if ni else None, _ptr(u), _ptr(ptr), _ptr(idx),
                          _ptr(rows), nr, _ptr(nuv), _ptr(f))
    return f


def apply(prob: Problem, u: np.ndarray, fixed: Optional[np.ndarray] = None, broken=None,
          nu: Optional[np.ndarray] = None) -> np.ndarray:
    """f = A u with rows of constrained DOFs reported as 0 (Remark 1)."""
    f = force(prob, u, broken, nu=nu)
    if fixed is not None:
        f[np.asarray(fixed, dtype=bool).reshape(f.shape)] = 0.0
    return f


def assemble_dense(prob: Problem, broken=None) -> np.ndarray:
    """Dense A (dim*N square), eq. (matrix); row/column index c*N + p."""
    lib = _load()
    d, N = prob.dim, prob.N
    n = np.array(list(prob.n) + [1] * (3 - d), dtype=np.int64)
    ptr, idx = broken_csr(N, broken)
    infl, ni = _infl_arr(prob)
    A = np.empty((d * N, d * N), dtype=np.float64)
    lib.oracle_assemble_dense(d, _ptr(n), prob.h, prob.M, prob.alpha, ni,
                              _ptr(infl) if ni else None, _ptr(ptr), _ptr(idx), _ptr(A))
    return A


def _split(prob: Problem, fixed):
    d, N = prob.dim, prob.N
    if fixed is None:
        fx = np.zeros(d * N, dtype=bool)
    else:
        fx = np.asarray(fixed, dtype=bool).reshape(-1)
    return fx


def solve_dense(prob: Problem, b, fixed=None, g=None, broken=None, A=None) -> np.ndarray:
    """Static model eq. (mat:e2) by dense Cholesky.

    K = -A; K_FF u_F = b_F - K_FC g_C; u_C = g_C (eq. (up), Sec. 3.4).  Returns [dim][N]."""
    import scipy.linalg as sla
    d, N = prob.dim, prob.N
    fx = _split(prob, fixed)
    F, C = ~fx, fx
    if A is None:
        A = assemble_dense(prob, broken)
    K = -A
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    gv = np.zeros(d * N) if g is None else np.asarray(g, dtype=np.float64).reshape(-1)
    rhs = b[F] - K[np.ix_(F, C)] @ gv[C]
    cf = sla.cho_factor(K[np.ix_(F, F)], lower=True)
    u = np.zeros(d * N)
    u[F] = sla.cho_solve(cf, rhs)
    u[C] = gv[C]
    return u.reshape(d, N)


def lifted_rhs(prob: Problem, b, fixed=None, g=None, broken=None) -> np.ndarray:
    """b_F - K_FC g_C on free DOFs (0 on constrained), via the bond-sum apply."""
    d, N = prob.dim, prob.N
    fx = _split(prob, fixed)
    b = np.asarray(b, dtype=np.float64).reshape(-1).copy()
    if g is not None:
        gc = np.where(fx, np.asarray(g, dtype=np.float64).reshape(-1), 0.0)
        b += force(prob, gc, broken).reshape(-1)   # -K_FC g_C = A_FC g_C
    b[fx] = 0.0
    return b.reshape(d, N)


def solve_cg(prob: Problem, b, fixed=None, g=None, broken=None, tol: float = 1e-14,
             maxit: int = 100000, x0=None):
    """Static model eq. (mat:e2) by plain conjugate gradients on the free DOFs.

    Operator v -> -(A v) restricted to free DOFs (v is zero on constrained DOFs);
    stops when ||r||_2 <= tol ||b'||_2.  Returns (u [dim][N], iterations, rel_residual)."""
    d, N = prob.dim, prob.N
    fx = _split(prob, fixed)

    def K(v):
        w = -force(prob, v, broken).reshape(-1)
        w[fx] = 0.0
        return w

    bp = lifted_rhs(prob, b, fixed, g, broken).reshape(-1)
    x = np.zeros(d * N) if x0 is None else np.where(fx, 0.0, np.asarray(x0).reshape(-1))
    r = bp - K(x)
    p = r.copy()
    rr = r @ r
    bn = math.sqrt(bp @ bp)
    it = 0
    while math.sqrt(rr) > tol * bn and it < maxit:
        q = K(p)
        a = rr / (p @ q)
        x += a * p
        r -= a * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    rtrue = bp - K(x)
    u = x.copy()
    if g is not None:
        u[fx] = np.asarray(g, dtype=np.float64).reshape(-1)[fx]
    return u.reshape(d, N), it, math.sqrt(rtrue @ rtrue) / bn


def vv(prob: Problem, u0, v0, b, dt: float, nsteps: int, fixed=None, g=None, broken=None,
       energy_every: int = 0, nu=None):
    """Velocity Verlet, Alg. 2, with acceleration a = (A u + b)/rho (eq. (mat:e1)).

    Constrained DOFs are overwritten with g after each displacement update
    (eq. (up)); their velocity and acceleration are held at 0.
    Returns (u, v, a, energies) with energies sampled after every
    ``energy_every`` steps (empty when 0)."""
    d, N = prob.dim, prob.N
    fx = _split(prob, fixed).reshape(d, N)
    b = np.asarray(b, dtype=np.float64).reshape(d, N)
    u = np.asarray(u0, dtype=np.float64).reshape(d, N).copy()
    v = np.asarray(v0, dtype=np.float64).reshape(d, N).copy()
    gv = None if g is None else np.asarray(g, dtype=np.float64).reshape(d, N)
    if gv is not None:
        u[fx] = gv[fx]
    v[fx] = 0.0

    def accel(uu):
        a = (force(prob, uu, broken, nu=nu) + b) / prob.rho
        a[fx] = 0.0
        return a

    a = accel(u)
    energies = []
    for n in range(1, nsteps + 1):
        u = u + dt * v + 0.5 * dt * dt * a
        if gv is not None:
            u[fx] = gv[fx]
        a_new = accel(u)
        v = v + 0.5 * dt * (a + a_new)
        v[fx] = 0.0
        a = a_new
        if energy_every and n % energy_every == 0:
            energies.append(energy(prob, u, v, b, fixed, broken))
    return u, v, a, np.array(energies)


def energy_parts(prob: Problem, u, v, b, fixed=None, broken=None):
    """(kinetic, elastic, load) = (1/2 rho V sum v^2, -1/2 V sum u (A u), -V sum b u)
    over free DOFs; their sum is the energy below."""
    d, N = prob.dim, prob.N
    fx = _split(prob, fixed)
    F = ~fx
    V = prob.h ** d
    u = np.asarray(u, dtype=np.float64).reshape(-1)
    v = np.asarray(v, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    Au = force(prob, u, broken).reshape(-1)
    return (float(0.5 * prob.rho * V * (v[F] @ v[F])), float(-0.5 * V * (u[F] @ Au[F])),
            float(-V * (b[F] @ u[F])))


def energy(prob: Problem, u, v, b, fixed=None, broken=None) -> float:
    """H = 1/2 rho V sum v^2 - 1/2 V sum u (A u) - V sum b u over free DOFs.

    -A is symmetric positive semidefinite, so this is the conserved energy of
    rho u'' = A u + b (eq. (mat:e1)) and VV keeps it bounded."""
    kin, el, load = energy_parts(prob, u, v, b, fixed, broken)
    return float(kin + el + load)


def grad_dense(prob: Problem, b, u_target, fixed=None, g=None, broken=None):
    """Loss L = ||u - u_t||^2 (all DOFs) of the static solution and its exact gradient.

    u solves K(a) u = b on free DOFs, K = -A(a), A(a) = sum_k a_k A_k with A_k the
    stiffness built with omega = (r/delta)^k.  Adjoint: K_FF symmetric, so
    w = K_FF^{-1} dL/du_F; dL/db_F = w; dL/da_k = w . (A_k u)_F (u including g).
    Returns (L, u, dL/db [dim][N] (0 on constrained), dL/da [n_infl])."""
    d, N = prob.dim, prob.N
    fx = _split(prob, fixed)
    F = ~fx
    A = assemble_dense(prob, broken)
    u = solve_dense(prob, b, fixed, g, broken, A=A).reshape(-1)
    ut = np.asarray(u_target, dtype=np.float64).reshape(-1)
    L = float((u - ut) @ (u - ut))
    import scipy.linalg as sla
    cf = sla.cho_factor(-A[np.ix_(F, F)], lower=True)
    w = np.zeros(d * N)
    w[F] = sla.cho_solve(cf, 2.0 * (u - ut)[F])
    ga = np.zeros(len(prob.infl))
    for k in range(len(prob.infl)):
        e = np.zeros(len(prob.infl))
        e[k] = 1.0
        pk = Problem(prob.n, prob.h, prob.M, prob.alpha, tuple(e), prob.rho)
        Aku = force(pk, u, broken).reshape(-1)
        ga[k] = w[F] @ Aku[F]
    return L, u.reshape(d, N), w.reshape(d, N), ga


def grad_cg(prob: Problem, b, u_target, fixed=None, g=None, broken=None, tol: float = 1e-13,
            maxit: int = 200000):
    """The gradient of ``grad_dense`` with both solves by conjugate gradients (plates too
    big to factor): u solves K(a) u = b on free DOFs (u = g on constrained), the adjoint
    w solves K_FF w_F = 2 (u - u_t)_F (K_FF symmetric), dL/db_F = w and
    dL/da_k = w . (A_k u)_F.  Returns (L, u, dL/db, dL/da, (iterations of u, of w),
    (relative residuals of u, of w))."""
    d, N = prob.dim, prob.N
    fx = _split(prob, fixed)
    F = ~fx
    u, itu, resu = solve_cg(prob, b, fixed, g, broken, tol=tol, maxit=maxit)
    u = u.reshape(-1)
    ut = np.asarray(u_target, dtype=np.float64).reshape(-1)
    L = float((u - ut) @ (u - ut))
    rhs = np.where(fx, 0.0, 2.0 * (u - ut))
    w, itw, resw = solve_cg(prob, rhs, fixed, None, broken, tol=tol, maxit=maxit)
    w = w.reshape(-1)
    ga = np.zeros(len(prob.infl))
    for k in range(len(prob.infl)):
        e = np.zeros(len(prob.infl))
        e[k] = 1.0
        pk = Problem(prob.n, prob.h, prob.M, prob.alpha, tuple(e), prob.rho)
        Aku = force(pk, u, broken).reshape(-1)
        ga[k] = w[F] @ Aku[F]
    return L, u.reshape(d, N), w.reshape(d, N), ga, (itu, itw), (resu, resw)


def crack_to_bonds(prob: Problem, segments) -> np.ndarray:
    """Broken bonds of a 2D pre-crack: {p, q} (p < q, inside each other's horizon)
    is broken iff the closed segment [x_p, x_q] properly crosses a crack segment,
    i.e. both orientation pairs have strictly opposite signs (FP64; touching or
    collinear does not count).  Brute force over every bond.  Returns [nb][2]."""
    assert prob.dim == 2
    nx, ny = prob.n
    M = prob.M
    xs = prob.node_coords()
    out = []
    segs = np.asarray(segments, dtype=np.float64).reshape(-1, 4)
    ids = np.arange(prob.N).reshape(ny, nx)

    def orient(ax, ay, bx, by, cx, cy):
        return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)

    for oy in range(0, M + 1):
        for ox in range(-M, M + 1):
            if oy == 0 and ox <= 0:
                continue                         # each undirected bond once
            if ox * ox + oy * oy > M * M:
                continue
            i0, i1 = max(0, -ox), min(nx, nx - ox)
            j0, j1 = 0, ny - oy
            if i0 >= i1 or j0 >= j1:
                continue
            P = ids[j0:j1, i0:i1].reshape(-1)
            Q = ids[j0 + oy:j1 + oy, i0 + ox:i1 + ox].reshape(-1)
            px, py = xs[0][P], xs[1][P]
            qx, qy = xs[0][Q], xs[1][Q]
            cut = np.zeros(len(P), dtype=bool)
            for (c0x, c0y, c1x, c1y) in segs:
                d1 = orient(c0x, c0y, c1x, c1y, px, py)
                d2 = orient(c0x, c0y, c1x, c1y, qx, qy)
                d3 = orient(px, py, qx, qy, c0x, c0y)
                d4 = orient(px, py, qx, qy, c1x, c1y)
                cut |= (((d1 > 0) & (d2 < 0)) | ((d1 < 0) & (d2 > 0))) & \
                       (((d3 > 0) & (d4 < 0)) | ((d3 < 0) & (d4 > 0)))
            if cut.any():
                pp, qq = P[cut], Q[cut]
                out.append(np.stack([np.minimum(pp, qq), np.maximum(pp, qq)], axis=1))
    if not out:
        return np.zeros((0, 2), dtype=np.int64)
    pairs = np.concatenate(out)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    return np.ascontiguousarray(pairs[order])


# ---------------------------------------------------------------- circulant preconditioner
def generating_blocks(prob: Problem) -> np.ndarray:
    """G(o) for every offset o in [-M, M]^d: the block A_{p,q} with p - q = o of the
    unbroken operator (translation invariant away from the boundary, eqs. (matrix),
    (mae:e1)).  Read off f = A e_c for a unit displacement e_c in component c at the
    centre of a (2M+1)^d grid, whose horizon lies inside the grid: G(o)[a, c] =
    f[a, centre + o].  Returns [d][d][2M+1]...[2M+1] (axes z, y, x reversed like the
    node ids: index [a][c][oz+M][oy+M][ox+M])."""
    d, M = prob.dim, prob.M
    m = 2 * M + 1
    small = Problem(tuple([m] * d), prob.h, M, prob.alpha, tuple(prob.infl), prob.rho)
    centre = sum(M * m ** a for a in range(d))
    G = np.zeros((d, d) + (m,) * d)
    for c in range(d):
        u = np.zeros((d, small.N))
        u[c, centre] = 1.0
        f = force(small, u)
        for a in range(d):
            G[a, c] = f[a].reshape((m,) * d)
    return G


def _grid_shape(n):
    return tuple(int(x) for x in reversed(list(n)))


def periodic_apply(prob: Problem, L: Sequence[int], v: np.ndarray, G: Optional[np.ndarray] = None) -> np.ndarray:
    """A_per v on the L-periodic grid: (A_per v)_p = sum_o G(o) v_{p - o} (indices mod L),
    by direct summation over the offsets.  v: [d][prod L] (node id x fastest)."""
    d, M = prob.dim, prob.M
    if G is None:
        G = generating_blocks(prob)
    shp = _grid_shape(L)
    v = np.asarray(v, dtype=np.float64).reshape((d,) + shp)
    out = np.zeros_like(v)
    rng = range(-M, M + 1)
    offs = [(o,) for o in rng] if d == 1 else (
        [(oy, ox) for oy in rng for ox in rng] if d == 2 else [(oz, oy, ox) for oz in rng for oy in rng for ox in rng])
    for o in offs:
        blk = G[(slice(None), slice(None)) + tuple(x + M for x in o)]
        if not blk.any():
            continue
        shifted = np.roll(v, shift=o, axis=tuple(range(1, d + 1)))   # shifted_p = v_{p - o}
        out += np.einsum("ac,c...->a...", blk, shifted)
    return out.reshape(d, -1)


def fft_setup(prob: Problem, L: Optional[Sequence[int]] = None, workers: Optional[int] = None,
              G: Optional[np.ndarray] = None) -> dict:
    """The assembly of the fast method (Sec. 3.3): the spectra of the full-horizon generating
    array G (Sec. 3.2 / 4) wrapped onto a zero-padded grid of lengths L >= N + M per axis
    (default N + M; the paper pads to 2N), and the D^e blocks: a node whose horizon leaves the
    grid keeps in its diagonal block only the bonds inside the grid while G(0) sums all of them,
    so D^e_p = sum of W(o) = G(o) over the offsets o != 0 with p + o outside (eq. (mat:se))."""
    import scipy.fft as sfft
    d, M = prob.dim, prob.M
    shp = _grid_shape(prob.n)                       # (z,) y, x
    if L is None:
        L = tuple(reversed([n + M for n in shp]))  # x fastest, like prob.n
    Ls = _grid_shape(L)
    if any(a < n + M for a, n in zip(Ls, shp)):
        raise ValueError("padded lengths must be >= N + M per axis")
    if G is None:
        G = generating_blocks(prob)
    m = 2 * M + 1
    arr = np.zeros((d, d) + Ls)                     # G(o) at index o mod L
    idx = np.ix_(*[[(o - M) % Lk for o in range(m)] for Lk in Ls])
    for a in range(d):
        for c in range(d):
            arr[(a, c) + idx] = G[a, c]
    Gh = sfft.fftn(arr, axes=tuple(range(2, d + 2)), workers=workers)
    De = np.zeros((d, d) + shp)
    coords = np.meshgrid(*[np.arange(n) for n in shp], indexing="ij")
    for o in np.ndindex(*([m] * d)):
        off = tuple(k - M for k in o)
        blk = G[(slice(None), slice(None)) + o]
        if not any(off) or not blk.any():
            continue
        out = np.zeros(shp, dtype=bool)
        for k in range(d):
            out |= (coords[k] + off[k] < 0) | (coords[k] + off[k] >= shp[k])
        if out.any():
            De[:, :, out] += blk[:, :, None]
    return {"L": Ls, "Gh": Gh, "De": De, "G": G}


def fft_apply(prob: Problem, u: np.ndarray, fixed: Optional[np.ndarray] = None, broken=None,
              L: Optional[Sequence[int]] = None, workers: Optional[int] = None, setup: Optional[dict] = None):
    """f = A u by the matrix-structure-based fast method (Sec. 3.3-3.6) on the CPU.

    The Toeplitz part: u embedded in the zero-padded grid, forward FFT, the d x d block
    product with the spectra of G, inverse FFT, cropped to the grid (Alg. 3 in 2D, Alg. 4 in
    3D).  Then D^e u (``fft_setup``), and D^f: each broken bond's term W(q - p)(u_q - u_p)
    removed from both ends (eq. (df) / (tea:fr)).  Rows of constrained DOFs reported as 0, as
    ``apply``.  workers: scipy's FFT threads; setup: ``fft_setup``'s result (else built)."""
    import scipy.fft as sfft
    d, M = prob.dim, prob.M
    if setup is None:
        setup = fft_setup(prob, L, workers)
    Ls, Gh, De, G = setup["L"], setup["Gh"], setup["De"], setup["G"]
    shp = _grid_shape(prob.n)
    sp = tuple(range(1, d + 1))
    inner = (slice(None),) + tuple(slice(0, n) for n in shp)
    u = np.asarray(u, dtype=np.float64).reshape((d,) + shp)
    uu = np.zeros((d,) + Ls)
    uu[inner] = u
    uh = sfft.fftn(uu, axes=sp, workers=workers)
    fh = np.einsum("ac...,c...->a...", Gh, uh)
    f = sfft.ifftn(fh, axes=sp, workers=workers).real[inner]
    f += np.einsum("ac...,c...->a...", De, u)
    if broken is not None and len(broken):
        pr = np.asarray(broken, dtype=np.int64).reshape(-1, 2)
        uf = u.reshape(d, -1)
        ff = f.reshape(d, -1)
        nx = list(prob.n) + [1, 1]

        def zyx(node):
            return [node // (nx[0] * nx[1]), (node // nx[0]) % nx[1], node % nx[0]][3 - d:]
        cp, cq = zyx(pr[:, 0]), zyx(pr[:, 1])
        for e in range(len(pr)):
            p_, q_ = pr[e]
            o = tuple(int(cq[k][e] - cp[k][e]) + M for k in range(d))      # q - p, per (z,) y, x
            om = tuple(2 * M - k for k in o)                               # p - q
            du = uf[:, q_] - uf[:, p_]
            ff[:, p_] -= G[(slice(None), slice(None)) + o] @ du
            ff[:, q_] += G[(slice(None), slice(None)) + om] @ du
        f = ff.reshape((d,) + shp)
    f = f.reshape(d, -1)
    if fixed is not None:
        f[np.asarray(fixed, dtype=bool).reshape(f.shape)] = 0.0
    return f


def precond_symbol(prob: Problem, L: Sequence[int], G: Optional[np.ndarray] = None):
    """Khat(k) = -sum_o G(o) exp(-2 pi i k.o / L) for every frequency of the L grid (real:
    G(o) = G(-o)), and the shift s = 1e-3 * max over k of the largest row sum of
    |Khat(k)| (1e-3 if that is 0).  Returns (Khat [d][d][shape L reversed], s)."""
    d, M = prob.dim, prob.M
    if G is None:
        G = generating_blocks(prob)
    shp = _grid_shape(L)
    arr = np.zeros((d, d) + shp)
    rng = range(-M, M + 1)
    idx = np.stack(np.meshgrid(*([np.arange(-M, M + 1)] * d), indexing="ij"), axis=-1).reshape(-1, d)
    for o in idx:
        arr[(slice(None), slice(None)) + tuple(int(x) % l for x, l in zip(o, shp))] += \
            G[(slice(None), slice(None)) + tuple(int(x) + M for x in o)]
    Gh = np.fft.fftn(arr, axes=tuple(range(2, d + 2)))
    Kh = -Gh.real
    bound = np.abs(Kh).sum(axis=1).max()
    s = 1e-3 * (bound if bound > 0 else 1.0)
    return Kh, s


def precond_apply(prob: Problem, r: np.ndarray, L: Sequence[int], fixed=None) -> np.ndarray:
    """z = Pi_F E^T (K_per + s I)^{-1} E r: zero-pad r ([d][N]) to the L grid, solve the
    d x d system of every frequency, transform back, keep the N-grid, zero constrained
    DOFs.  Returns [d][N]."""
    d, N = prob.dim, prob.N
    Kh, s = precond_symbol(prob, L)
    shp = _grid_shape(L)
    nshp = _grid_shape(prob.n)
    full = np.zeros((d,) + shp)
    full[(slice(None),) + tuple(slice(0, m) for m in nshp)] = np.asarray(r, dtype=np.float64).reshape((d,) + nshp)
    rh = np.fft.fftn(full, axes=tuple(range(1, d + 1)))
    C = np.moveaxis(Kh, (0, 1), (-2, -1)) + s * np.eye(d)
    zh = np.linalg.solve(C, np.moveaxis(rh, 0, -1)[..., None])[..., 0]
    zf = np.fft.ifftn(np.moveaxis(zh, -1, 0), axes=tuple(range(1, d + 1))).real
    z = zf[(slice(None),) + tuple(slice(0, m) for m in nshp)].reshape(d, N).copy()
    if fixed is not None:
        z[np.asarray(fixed, dtype=bool).reshape(d, N)] = 0.0
    return z


def precond_apply_periodic(prob: Problem, L: Sequence[int], v: np.ndarray) -> np.ndarray:
    """(K_per + s I)^{-1} v on the whole L-periodic grid (for pins).  v: [d][prod L]."""
    d = prob.dim
    Kh, s = precond_symbol(prob, L)
    shp = _grid_shape(L)
    vh = np.fft.fftn(np.asarray(v, dtype=np.float64).reshape((d,) + shp), axes=tuple(range(1, d + 1)))
    C = np.moveaxis(Kh, (0, 1), (-2, -1)) + s * np.eye(d)
    zh = np.linalg.solve(C, np.moveaxis(vh, 0, -1)[..., None])[..., 0]
    return np.fft.ifftn(np.moveaxis(zh, -1, 0), axes=tuple(range(1, d + 1))).real.reshape(d, -1)


# ---------------------------------------------------------------- crack propagation
def all_bonds(prob: Problem) -> np.ndarray:
    """Every bond {p, q} of the discrete horizon (integer offsets 0 < |o|^2 <= M^2, q inside
    the grid), as [n][2] pairs p < q sorted by (p, q)."""
    d, M = prob.dim, prob.M
    n = list(prob.n)
    ids = np.arange(prob.N).reshape(tuple(reversed(n)))
    out = []
    rng = range(-M, M + 1)
    offs = [(ox, oy, 0) for oy in rng for ox in rng] if d == 2 else \
        [(ox, oy, oz) for oz in rng for oy in rng for ox in rng]
    for o in offs:
        o = o[:d]
        s2 = sum(x * x for x in o)
        if s2 == 0 or s2 > M * M:
            continue
        src = tuple(slice(max(0, -x), m - max(0, x)) for x, m in zip(reversed(o), reversed(n)))
        dst = tuple(slice(max(0, x), m - max(0, -x)) for x, m in zip(reversed(o), reversed(n)))
        P, Q = ids[src].reshape(-1), ids[dst].reshape(-1)
        keep = P < Q
        out.append(np.stack([P[keep], Q[keep]], axis=1))
    pairs = np.concatenate(out) if out else np.zeros((0, 2), dtype=np.int64)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    return np.ascontiguousarray(pairs[order].astype(np.int64))


def bond_stretch(prob: Problem, u: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """s = (|x_q + u_q - x_p - u_p| - |x_q - x_p|) / |x_q - x_p|, eq. (fra:s1), FP64."""
    d = prob.dim
    x = prob.node_coords()
    u = np.asarray(u, dtype=np.float64).reshape(d, prob.N)
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    P, Q = pairs[:, 0], pairs[:, 1]
    xi = x[:, Q] - x[:, P]
    eta = u[:, Q] - u[:, P]
    ref = np.sqrt((xi * xi).sum(axis=0))
    cur = np.sqrt(((xi + eta) ** 2).sum(axis=0))
    return (cur - ref) / ref


def crack_update(prob: Problem, u: np.ndarray, s0: float, broken=None):
    """Eq. (mu): mu drops to 0 for good once s >= s0.  Returns (new [k][2] pairs p < q sorted,
    the updated broken set [n][2] sorted, the stretches of every bond of all_bonds)."""
    bonds = all_bonds(prob)
    s = bond_stretch(prob, u, bonds)
    old = set() if broken is None or len(broken) == 0 else \
        {(int(a), int(b)) for a, b in np.asarray(broken, dtype=np.int64).reshape(-1, 2)}
    new = [(int(a), int(b)) for (a, b), si in zip(bonds, s) if si >= s0 and (int(a), int(b)) not in old]
    allb = sorted(old | set(new))
    as_arr = lambda v: np.array(v, dtype=np.int64).reshape(-1, 2)
    return as_arr(new), as_arr(allb), s


# ---------------------------------------------------------------- surface correction
def surface_volume_factors(prob: Problem) -> np.ndarray:
    """nu_p = sum over the full discrete horizon of lambda(o) V / the same sum over the
    neighbours inside the grid (the volume reading of the surface-correction factor,
    Remark 3); 1 on nodes with a complete horizon.  lambda as in eq. (fac:e1):
    1 for |o|^2 <= M^2 - M, else M + 1/2 - |o|."""
    d, M = prob.dim, prob.M
    n = list(prob.n)
    shp = tuple(reversed(n))
    full = 0.0
    inside = np.zeros(shp)
    for o in np.ndindex(*([2 * M + 1] * d)):
        o = np.array(o) - M
        s2 = int((o * o).sum())
        if s2 == 0 or s2 > M * M:
            continue
        lam = 1.0 if s2 <= M * M - M else M + 0.5 - math.sqrt(s2)
        full += lam
        ok = np.ones(shp, dtype=bool)
        for a in range(d):   # axis a of the node grid is array axis d - 1 - a
            idx = np.arange(n[a]) + o[a]
            good = (idx >= 0) & (idx < n[a])
            sh = [1] * d
            sh[d - 1 - a] = n[a]
            ok &= good.reshape(sh)
        inside += lam * ok
    return (full / inside).reshape(-1)


# ---------------------------------------------------------------- adaptive dynamic relaxation
def adr_density(prob: Problem, broken=None) -> np.ndarray:
    """Fictitious diagonal density of the cited ADR method: D_ii = 1/4 sum_j |K_ij| (a
    Gershgorin bound, time step 1), K = -A assembled densely (every row and column, broken
    bonds removed).  Returns [dim][N]."""
    K = -assemble_dense(prob, broken)
    return (0.25 * np.abs(K).sum(axis=1)).reshape(prob.dim, prob.N)


def adr_step(prob: Problem, u, v, F, Fprev, b, D, fixed=None, g=None, broken=None, Dc=None):
    """One update of Alg. 1 (time step 1) from u^n with F = F(u^n), the velocity v^{n-1/2}
    and F^{n-1} (Fprev None: the first update, v^{1/2} = D^{-1} F^0 / 2):

        c^n        = 2 sqrt(u^T K1 u / u^T u) over the free DOFs, K1_ii = -(F^n_i - F^{n-1}_i) /
                     (D_ii v^{n-1/2}_i) (0 where v = 0); c^n = 0 when the quotient is not positive
        v^{n+1/2}  = ((2 - c^n) v^{n-1/2} + 2 D^{-1} F^n) / (2 + c^n)
        u^{n+1}    = u^n + v^{n+1/2}

    F = A u + b on free DOFs, 0 on constrained ones (u held at g there).  Dc: the density in
    K1 when it differs from D (the one in force when F^n was evaluated, for a step right
    after the operator changed).  Returns (u^{n+1}, v^{n+1/2}, F(u^{n+1}), c^n or None for the
    first update)."""
    d, N = prob.dim, prob.N
    fx = _split(prob, fixed).reshape(d, N)
    free = ~fx
    b = np.asarray(b, dtype=np.float64).reshape(d, N)
    u = np.asarray(u, dtype=np.float64).reshape(d, N)
    F = np.asarray(F, dtype=np.float64).reshape(d, N)
    c = None
    if Fprev is None:
        vn = np.where(free, 0.5 * F / D, 0.0)
    else:
        v = np.asarray(v, dtype=np.float64).reshape(d, N)
        Fp = np.asarray(Fprev, dtype=np.float64).reshape(d, N)
        with np.errstate(divide="ignore", invalid="ignore"):
            k1 = np.where(free & (v != 0.0), -(F - Fp) / ((D if Dc is None else Dc) * v), 0.0)
        num = float((u[free] * k1[free] * u[free]).sum())
        den = float((u[free] * u[free]).sum())
        c = 2.0 * math.sqrt(num / den) if den > 0 and num > 0 else 0.0
        vn = np.where(free, ((2.0 - c) * v + 2.0 * F / D) / (2.0 + c), 0.0)
    un = u + vn
    if g is not None:
        un[fx] = np.asarray(g, dtype=np.float64).reshape(d, N)[fx]
    Fn = force(prob, un, broken) + b
    Fn[fx] = 0.0
    return un, vn, Fn, c


def adr(prob: Problem, u0, b, nsteps: int, fixed=None, g=None, broken=None):
    """Alg. 1 (CDEI) for D u'' + c D u' = f + b (eq. (ADR:e1)): nsteps updates of
    ``adr_step`` from u0 (u held at g on constrained DOFs), D from ``adr_density``.
    Returns (u, the last velocity, F(u), list of c^n)."""
    d, N = prob.dim, prob.N
    fx = _split(prob, fixed).reshape(d, N)
    D = adr_density(prob, broken)
    b = np.asarray(b, dtype=np.float64).reshape(d, N)
    u = np.asarray(u0, dtype=np.float64).reshape(d, N).copy()
    u[fx] = 0.0 if g is None else np.asarray(g, dtype=np.float64).reshape(d, N)[fx]
    F = force(prob, u, broken) + b
    F[fx] = 0.0
    v, Fprev, cs = np.zeros((d, N)), None, []
    for _ in range(nsteps):
        un, v, Fn, c = adr_step(prob, u, v, F, Fprev, b, D, fixed, g, broken)
        if c is not None:
            cs.append(c)
        u, Fprev, F = un, F, Fn
    return u, v, F, cs
