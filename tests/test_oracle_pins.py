"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-derives the oracle's own formula: each checks a property
(symmetry, invariance, a continuum closed form, a decoupling identity, a
closed-form count or trajectory, finite differences) that a dropped term, a
wrong sign or index or a transposed operand in the oracle would break.
"""
import math
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _prob2(nx, ny, M, E=1.0, h=None, infl=()):
    h = h or 1.0 / max(nx, ny)
    return O.Problem((nx, ny), h, M, O.alpha_2d(E, M * h), infl)


def _prob3(nx, ny, nz, M, E=1.0, h=None):
    h = h or 1.0 / max(nx, ny, nz)
    return O.Problem((nx, ny, nz), h, M, O.alpha_3d(E, M * h))


def _random_bonds(prob, nb, seed):
    """A random set of in-horizon node pairs (p < q) to mark broken."""
    rng = np.random.default_rng(seed)
    d, M = prob.dim, prob.M
    out = set()
    n = list(prob.n)
    while len(out) < nb:
        ip = [rng.integers(0, m) for m in n]
        o = rng.integers(-M, M + 1, size=d)
        s2 = int((o * o).sum())
        if s2 == 0 or s2 > M * M:
            continue
        iq = [a + b for a, b in zip(ip, o)]
        if any(c < 0 or c >= m for c, m in zip(iq, n)):
            continue

        def nid(ix):
            idx = 0
            for a in reversed(range(d)):
                idx = idx * n[a] + ix[a]
            return idx
        p, q = nid(ip), nid(iq)
        out.add((min(p, q), max(p, q)))
    return np.array(sorted(out), dtype=np.int64)


# ---------------------------------------------------------------- golden stencil

def test_golden_stencil_entries_2d():
    """Hand-worked entries of eq. (frb:e1) with lambda of eq. (fac:e1), M = 3."""
    M, n = 3, 7
    p = O.Problem((n, n), 1.0, M, 1.0)
    A = O.assemble_dense(p)
    N = p.N
    c = M * n + M
    comp = {"xx": (0, 0), "yy": (1, 1), "xy": (0, 1)}
    rows = [l.split() for l in open(os.path.join(GOLDEN, "stencil_M3_2d.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 10
    for ox, oy, cname, val in rows:
        a, b = comp[cname]
        q = (M + int(oy)) * n + (M + int(ox))
        got = A[a * N + c, b * N + q]
        assert got == pytest.approx(float(val), rel=1e-14, abs=1e-15), (ox, oy, cname)


# ---------------------------------------------------------------- symmetry (P1)

@pytest.mark.parametrize("dim", [2, 3])
def test_symmetry_bitwise(dim):
    """A^{yx} = A^{xy} and A_pq = A_qp (Sec. 4, from the kernel's symmetry), bitwise."""
    p = _prob2(9, 7, 3) if dim == 2 else _prob3(5, 4, 6, 2)
    br = _random_bonds(p, 25, seed=1)
    A = O.assemble_dense(p, br)
    assert np.array_equal(A, A.T)


# ------------------------------------------------------- rigid motions (P2, P3)

@pytest.mark.parametrize("dim", [2, 3])
def test_rigid_translation_gives_zero_force(dim):
    """Diagonal = minus the row sum over in-domain, unbroken bonds (eq. (matrix),
    (Oe:e2), Sec. 3.6): a uniform translation produces no force on any row,
    including incomplete-horizon and broken-bond rows."""
    p = _prob2(11, 9, 3) if dim == 2 else _prob3(6, 5, 7, 2)
    br = _random_bonds(p, 30, seed=2)
    c = np.array([0.7, -1.3, 0.4][:dim])
    u = np.repeat(c[:, None], p.N, axis=1)
    f = O.force(p, u, br)
    A = O.assemble_dense(p, br)
    assert np.abs(f).max() <= 1e-14 * np.abs(A).max() * np.abs(u).max() * 50


@pytest.mark.parametrize("dim", [2, 3])
def test_infinitesimal_rotation_gives_zero_force(dim):
    """C(xi) = alpha xi(x)xi/|xi|^3 (eq. (ker:e1)) annihilates xi-perpendicular
    relative displacements: u = w x x gives zero force on every row."""
    p = _prob2(10, 8, 3) if dim == 2 else _prob3(6, 6, 5, 2)
    br = _random_bonds(p, 20, seed=3)
    x = p.node_coords()
    if dim == 2:
        u = 0.01 * np.stack([-x[1], x[0]])
    else:
        w = np.array([0.3, -0.2, 0.5])
        u = np.cross(w, x.T).T
    f = O.force(p, u, br)
    scale = np.abs(O.force(p, np.stack([x[0]] + [0 * x[0]] * (dim - 1)))).max()
    assert scale > 1.0                                  # the probe itself is not degenerate
    assert np.abs(f).max() <= 1e-13 * scale


def test_transpose_of_rotation_is_not_zero():
    """Guard: the transposed rotation u = (y, x) (a symmetric strain) does produce force
    near the boundary, so the rotation test above discriminates."""
    p = _prob2(10, 8, 3)
    x = p.node_coords()
    f = O.force(p, np.stack([x[1], x[0]]))
    assert np.abs(f).max() > 1.0


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_field_zero_on_full_horizon_rows(dim):
    """Rows of Omega_in (full horizon, no broken bond) depend only on the offset
    (eqs. (frb:e1)-(frb:e4)): a symmetric stencil applied to an affine field gives 0.
    Incomplete-horizon rows (Omega_e) do not."""
    rng = np.random.default_rng(4)
    p = _prob2(13, 12, 3) if dim == 2 else _prob3(9, 8, 9, 2)
    x = p.node_coords()
    F = rng.standard_normal((dim, dim))
    u = F @ x + rng.standard_normal((dim, 1))
    f = O.force(p, u)
    M = p.M
    idx = np.stack(np.unravel_index(np.arange(p.N), tuple(p.n)[::-1]))[::-1]
    interior = np.ones(p.N, dtype=bool)
    for a in range(dim):
        interior &= (idx[a] >= M) & (idx[a] < p.n[a] - M)
    scale = np.abs(f).max()
    assert scale > 1.0
    assert np.abs(f[:, interior]).max() <= 1e-12 * scale
    assert np.abs(f[:, ~interior]).max() > 1e-3 * scale


# ---------------------------------------------------------- continuum limit (P5)

def _limits():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "continuum_limits.txt"))
            if l.strip() and not l.startswith("#")]
    return {k: float(v) for k, v in rows}


def _centre_force(p, u):
    M = p.M
    n = p.n[0]
    c = sum((M * n ** a) for a in range(p.dim))
    return O.force(p, u, rows=np.array([c]))[:, 0]


def test_continuum_limit_2d():
    """alpha = 9E/(pi delta^3) (Sec. 2.1) makes the nonlocal operator tend to the
    plane-stress Navier operator with nu = 1/3 as the horizon holds more nodes:
    u = (x^2, 0) -> f_x = 9E/4, u = (y^2, 0) -> 3E/4, u = (0, xy) -> f_x = 3E/4,
    and -tr(A_pp) delta^2 -> alpha * int 1/r dA * delta^2 = 18E (closed forms of
    the continuum integral of eq. (ker:e1) over the disk; see tests/golden)."""
    E = 2.0
    g = _limits()
    lim = {k: g["2d_" + k] * E for k in ("xx", "yy", "xy", "tr")}
    errs = {k: [] for k in lim}
    for M in (3, 8, 16, 32, 64):
        n = 2 * M + 1
        p = O.Problem((n, n), 1.0 / n, M, O.alpha_2d(E, M / n))
        x = p.node_coords()
        z = 0 * x[0]
        vals = {"xx": _centre_force(p, np.stack([x[0] ** 2, z]))[0],
                "yy": _centre_force(p, np.stack([x[1] ** 2, z]))[0],
                "xy": _centre_force(p, np.stack([z, x[0] * x[1]]))[0]}
        c = M * n + M
        ex = np.zeros((2, p.N)); ex[0, c] = 1
        ey = np.zeros((2, p.N)); ey[1, c] = 1
        tr = O.force(p, ex, rows=np.array([c]))[0, 0] + O.force(p, ey, rows=np.array([c]))[1, 0]
        vals["tr"] = -tr * (M / n) ** 2
        for k in lim:
            errs[k].append(abs(vals[k] - lim[k]) / lim[k])
    for k in lim:
        e = errs[k]
        assert all(b < a for a, b in zip(e, e[1:])), (k, e)   # converging
        assert e[-1] < 0.015, (k, e)


def test_continuum_limit_3d():
    """alpha = 12E/(pi delta^4) (Sec. 2.1): u = (x^2, 0, 0) -> f_x = 12E/5 (Navier,
    nu = 1/4) and -tr(A_pp) delta^2 -> 24E."""
    E = 1.0
    ex_f, ex_t = [], []
    for M in (3, 6, 12, 24, 48):
        n = 2 * M + 1
        p = O.Problem((n, n, n), 1.0 / n, M, O.alpha_3d(E, M / n))
        x = p.node_coords()
        z = 0 * x[0]
        fx = _centre_force(p, np.stack([x[0] ** 2, z, z]))[0]
        c = (M * n + M) * n + M
        tr = 0.0
        for a in range(3):
            e = np.zeros((3, p.N)); e[a, c] = 1
            tr += O.force(p, e, rows=np.array([c]))[a, 0]
        g = _limits()
        ex_f.append(abs(fx - g["3d_xx"] * E) / (g["3d_xx"] * E))
        ex_t.append(abs(-tr * (M / n) ** 2 - g["3d_tr"] * E) / (g["3d_tr"] * E))
    assert all(b < a for a, b in zip(ex_f, ex_f[1:])), ex_f
    assert all(b < a for a, b in zip(ex_t, ex_t[1:])), ex_t
    assert ex_f[-1] < 0.02 and ex_t[-1] < 0.02


# ------------------------------------------------------- brute force (tiny grids)

def test_banded_loop_equals_all_pairs_double_loop():
    """The banded offset loop (eq. (band)) equals a literal all-pairs double loop over
    every node pair, horizon decided by |x_q - x_p| <= delta (exact here: h = 1)."""
    nx, ny, M = 6, 5, 2
    p = O.Problem((nx, ny), 1.0, M, 3.0)
    br = _random_bonds(p, 6, seed=5)
    bset = {tuple(b) for b in br.tolist()}
    N = p.N
    xs = p.node_coords().T
    A = np.zeros((2 * N, 2 * N))
    for a in range(N):
        for b in range(N):
            if a == b or (min(a, b), max(a, b)) in bset:
                continue
            xi = xs[b] - xs[a]
            r = math.hypot(*xi)
            if r > M:                       # delta = M h with h = 1
                continue
            lam = 1.0 if r <= M - 0.5 else M + 0.5 - r
            for c in range(2):
                for e in range(2):
                    w = p.alpha * lam * xi[c] * xi[e] / r ** 3
                    A[c * N + a, e * N + b] += w
                    A[c * N + a, e * N + a] -= w
    B = O.assemble_dense(p, br)
    assert np.allclose(A, B, rtol=1e-14, atol=1e-14 * np.abs(B).max())


# ------------------------------------------------------------- broken bonds (P10)

def test_full_cut_decouples_the_plate():
    """A crack cutting the plate in two (mu = 0 on every crossing bond, eq. (mu)) gives
    exactly the stiffness of two separate plates: the D^f bookkeeping of eq. (df)
    is then the incomplete-horizon correction of eq. (mat:se)."""
    nx, ny, M, cut = 12, 8, 3, 5          # crack between columns 5 and 6
    h = 1.0 / 16
    p = O.Problem((nx, ny), h, M, O.alpha_2d(1.0, M * h))
    xc = (cut + 1) * h
    br = O.crack_to_bonds(p, [[xc, -1.0, xc, 2.0]])
    A = O.assemble_dense(p, br)
    left = O.Problem((cut + 1, ny), h, M, p.alpha)
    right = O.Problem((nx - cut - 1, ny), h, M, p.alpha)
    AL, AR = O.assemble_dense(left), O.assemble_dense(right)
    N = p.N
    ids = np.arange(N).reshape(ny, nx)
    L_ids = ids[:, :cut + 1].reshape(-1)
    R_ids = ids[:, cut + 1:].reshape(-1)
    for sub, Asub in ((L_ids, AL), (R_ids, AR)):
        rows = np.concatenate([sub, sub + N])
        assert np.allclose(A[np.ix_(rows, rows)], Asub, rtol=1e-13, atol=1e-13 * np.abs(Asub).max())
    rowsL = np.concatenate([L_ids, L_ids + N])
    rowsR = np.concatenate([R_ids, R_ids + N])
    assert np.abs(A[np.ix_(rowsL, rowsR)]).max() == 0.0


def test_crack_count_vertical_closed_form():
    """A vertical crack between two node columns, longer than the plate, cuts exactly
    the bonds whose ends lie on opposite sides: sum over offsets ox > 0 of ox*(ny-|oy|)."""
    nx, ny, M = 20, 14, 4
    h = 1.0 / 20
    p = O.Problem((nx, ny), h, M, 1.0)
    xc = 10 * h                            # between columns 9 and 10
    br = O.crack_to_bonds(p, [[xc, -0.5, xc, 1.5]])
    expect = sum(ox * (ny - abs(oy)) for ox in range(1, M + 1) for oy in range(-M, M + 1)
                 if ox * ox + oy * oy <= M * M)
    assert len(br) == expect
    xs = p.node_coords()
    assert np.all((xs[0][br[:, 0]] - xc) * (xs[0][br[:, 1]] - xc) < 0)


def test_crack_along_node_row_closed_form():
    """A crack lying exactly on a node row: bonds with an end on the row are not
    properly crossed; bonds whose ends straddle the row are, wherever they pass
    (including through a node on it): sum over oy >= 2 of (oy-1)*(nx-|ox|)."""
    nx, ny, M = 15, 15, 3
    h = 1.0 / 15
    p = O.Problem((nx, ny), h, M, 1.0)
    yc = (7 + 0.5) * h                      # row j = 7
    br = O.crack_to_bonds(p, [[-1.0, yc, 2.0, yc]])
    expect = sum((oy - 1) * (nx - abs(ox)) for oy in range(2, M + 1) for ox in range(-M, M + 1)
                 if ox * ox + oy * oy <= M * M)
    assert len(br) == expect


def test_crack_mirror_symmetry():
    """Mirroring the crack about the plate's vertical mid-line mirrors the broken set."""
    nx, ny, M = 24, 18, 3
    h = 1.0 / 24
    p = O.Problem((nx, ny), h, M, 1.0)
    seg = np.array([0.31, 0.22, 0.71, 0.53])
    br = O.crack_to_bonds(p, [seg])
    W = nx * h
    br_m = O.crack_to_bonds(p, [[W - seg[0], seg[1], W - seg[2], seg[3]]])
    assert len(br) > 10

    def mirror(q):
        j, i = np.divmod(q, nx)
        return j * nx + (nx - 1 - i)
    m = np.sort(np.stack([mirror(br[:, 0]), mirror(br[:, 1])], 1), axis=1)
    m = m[np.lexsort((m[:, 1], m[:, 0]))]
    assert np.array_equal(m, br_m)


# ----------------------------------------------------------------- static (P8)

def _dirichlet_layer(p, sides="all"):
    """Fixed mask [dim][N]: nodes whose centre is within delta of a constrained face."""
    idx = np.stack(np.unravel_index(np.arange(p.N), tuple(p.n)[::-1]))[::-1]
    m = np.zeros(p.N, dtype=bool)
    for a in range(p.dim):
        m |= (idx[a] < p.M) | (idx[a] >= p.n[a] - p.M)
    return np.repeat(m[None], p.dim, axis=0)


def test_dense_solve_recovers_manufactured_solution():
    """K = -A (eq. (mat:e2)); with u* given, b_F = (K u*)_F and the solve returns u*."""
    rng = np.random.default_rng(6)
    p = _prob2(14, 12, 3)
    br = _random_bonds(p, 10, seed=7)
    fixed = _dirichlet_layer(p)
    g = np.where(fixed, rng.standard_normal(fixed.shape), 0.0)
    ustar = np.where(fixed, g, rng.standard_normal(fixed.shape))
    b = -O.force(p, ustar, br)
    u = O.solve_dense(p, b, fixed, g, br)
    assert np.abs(u - ustar).max() <= 1e-10 * np.abs(ustar).max()


def test_cg_agrees_with_cholesky():
    rng = np.random.default_rng(8)
    p = _prob2(16, 16, 3)
    fixed = _dirichlet_layer(p)
    b = rng.standard_normal((2, p.N))
    u1 = O.solve_dense(p, b, fixed)
    u2, it, res = O.solve_cg(p, b, fixed, tol=1e-14)
    assert res <= 1e-13
    assert np.linalg.norm(u2 - u1) <= 1e-11 * np.linalg.norm(u1)


# ------------------------------------------------------------------ dynamic (P9)

def test_vv_constant_force_is_exact():
    """No bonds (alpha = 0): Alg. 2 integrates u'' = b/rho exactly,
    u(t) = u0 + v0 t + b t^2 / (2 rho)."""
    rng = np.random.default_rng(9)
    p = O.Problem((5, 4), 0.1, 2, 0.0, rho=2.5)
    u0, v0, b = (rng.standard_normal((2, p.N)) for _ in range(3))
    dt, n = 0.01, 50
    u, v, a, _ = O.vv(p, u0, v0, b, dt, n)
    t = dt * n
    assert np.allclose(u, u0 + v0 * t + 0.5 * b / p.rho * t * t, rtol=1e-12, atol=1e-12)
    assert np.allclose(v, v0 + b / p.rho * t, rtol=1e-12, atol=1e-12)


def test_vv_two_node_oscillator_closed_form():
    """Two nodes one cell apart with M = 1 share one bond of stiffness
    k = alpha * lambda * h^(d-1) with lambda = 1/2 (eq. (fac:e1) at |xi| = delta).
    The relative x-displacement y obeys y'' = -(2k/rho) y, and Alg. 2 reproduces
    the leapfrog solution y_n = A cos(n th) + B sin(n th), cos th = 1 - dt^2 w^2/2;
    the y-components move freely."""
    h, alpha, rho = 1.0, 3.0, 2.0
    p = O.Problem((2, 1), h, 1, alpha, rho=rho)
    k = alpha * 0.5 * h
    w2 = 2 * k / rho
    dt, n = 0.05, 400
    u0 = np.array([[0.1, -0.2], [0.0, 0.0]])
    v0 = np.array([[0.3, 0.05], [0.2, 0.2]])
    b = np.zeros((2, 2))
    y0 = u0[0, 1] - u0[0, 0]
    wv0 = v0[0, 1] - v0[0, 0]
    y1 = y0 + dt * wv0 - 0.5 * dt * dt * w2 * y0
    th = math.acos(1 - 0.5 * dt * dt * w2)
    B = (y1 - y0 * math.cos(th)) / math.sin(th)
    for steps in (1, 17, n):
        u, v, _, _ = O.vv(p, u0, v0, b, dt, steps)
        y = u[0, 1] - u[0, 0]
        assert y == pytest.approx(y0 * math.cos(steps * th) + B * math.sin(steps * th), abs=1e-12)
        assert u[0, 0] + u[0, 1] == pytest.approx(u0[0].sum() + v0[0].sum() * dt * steps, abs=1e-12)
        assert np.allclose(u[1], u0[1] + v0[1] * dt * steps, atol=1e-12)


def test_vv_energy_drift_is_second_order():
    """Velocity Verlet is symplectic and second order: the energy error is bounded
    and shrinks about 4x when dt halves."""
    rng = np.random.default_rng(10)
    p = _prob2(10, 10, 3)
    p.rho = 1.0
    u0 = 1e-3 * rng.standard_normal((2, p.N))
    v0 = np.zeros((2, p.N))
    b = rng.standard_normal((2, p.N))
    A = O.assemble_dense(p)
    lam_max = np.linalg.eigvalsh(-A).max()
    T = 20.0 / math.sqrt(lam_max)
    drifts = []
    for ns in (200, 400):
        dt = T / ns
        E0 = O.energy(p, u0, v0, b)
        _, _, _, Es = O.vv(p, u0, v0, b, dt, ns, energy_every=ns // 20)
        drifts.append(np.abs(Es - E0).max() / abs(E0))
    assert drifts[0] < 0.2
    assert 2.5 < drifts[0] / drifts[1] < 6.0


# ----------------------------------------------------------------- gradient (P11)

def test_gradient_matches_central_differences():
    """Adjoint gradient of ||u - u_t||^2 w.r.t. the influence coefficients a_k and
    the body force equals central finite differences of the solve."""
    rng = np.random.default_rng(11)
    nx, M = 9, 2
    a = rng.uniform(0.2, 1.0, size=4)
    h = 1.0 / nx
    p = O.Problem((nx, nx), h, M, O.alpha_2d(1.0, M * h), tuple(a))
    fixed = _dirichlet_layer(p)
    b = rng.standard_normal((2, p.N))
    ut = np.where(fixed, 0.0, 1e-3 * rng.standard_normal((2, p.N)))
    L, u, gb, ga = O.grad_dense(p, b, ut, fixed)
    for k in range(len(a)):
        eps = 1e-4 * a[k]
        ap, am = a.copy(), a.copy()
        ap[k] += eps
        am[k] -= eps
        Lp = O.grad_dense(O.Problem(p.n, h, M, p.alpha, tuple(ap)), b, ut, fixed)[0]
        Lm = O.grad_dense(O.Problem(p.n, h, M, p.alpha, tuple(am)), b, ut, fixed)[0]
        assert ga[k] == pytest.approx((Lp - Lm) / (2 * eps), rel=1e-6)
    free = np.flatnonzero(~fixed.reshape(-1))
    for idx in free[[0, 7, 40, len(free) - 1]]:
        eps = 1e-3
        bp, bm = b.copy().reshape(-1), b.copy().reshape(-1)
        bp[idx] += eps
        bm[idx] -= eps
        Lp = O.grad_dense(p, bp, ut, fixed)[0]
        Lm = O.grad_dense(p, bm, ut, fixed)[0]
        assert gb.reshape(-1)[idx] == pytest.approx((Lp - Lm) / (2 * eps), rel=1e-6)
    assert np.all(gb[fixed] == 0)


def test_cg_gradient_equals_dense_gradient_small_plates():
    """The CG form of the adjoint gradient (two CG solves, the derivative products)
    equals the dense-Cholesky gradient (itself pinned by finite differences above) on
    plates with a crack, prescribed displacements and all eight coefficients."""
    rng = np.random.default_rng(12)
    for nx, ny, M, crack in ((13, 11, 2, False), (17, 15, 3, True)):
        a = rng.uniform(0.1, 1.0, size=8)
        h = 1.0 / max(nx, ny)
        p = O.Problem((nx, ny), h, M, O.alpha_2d(1.0, M * h), tuple(a))
        fixed = _dirichlet_layer(p)
        br = O.crack_to_bonds(p, [[0.2, 0.3, 0.8, 0.7]]) if crack else None
        b = rng.standard_normal((2, p.N))
        g = np.where(fixed, 1e-3 * rng.standard_normal((2, p.N)), 0.0)
        ut = np.where(fixed, g, 1e-3 * rng.standard_normal((2, p.N)))
        Ld, ud, gbd, gad = O.grad_dense(p, b, ut, fixed, g, br)
        Lc, uc, gbc, gac, its, res = O.grad_cg(p, b, ut, fixed, g, br, tol=1e-14)
        assert res[0] <= 1e-14 and res[1] <= 1e-14
        assert Lc == pytest.approx(Ld, rel=1e-10)
        assert np.abs(gac - gad).max() <= 1e-9 * np.abs(gad).max()
        assert np.abs(gbc - gbd).max() <= 1e-9 * np.abs(gbd).max()


def test_cg_gradient_equals_dense_gradient_on_a_64x64_plate():
    """The 64 x 64 member of the 64-plate batch (omega = sum_k a_k (r/delta)^k, all sides
    fixed, target from the perturbed coefficients): dense and CG gradients agree."""
    from paper_2301_11828_amd import workloads as W
    ws = W.plates64()
    w = next(x for x in ws if x.n[0] == 64)
    p = O.Problem(w.n, w.h, w.M, w.alpha, w.infl)
    pt = O.Problem(w.n, w.h, w.M, w.alpha, w.extra["infl_target"])
    ut, _, _ = O.solve_cg(pt, w.b[0], w.fixed, tol=1e-14)
    Ld, _, gbd, gad = O.grad_dense(p, w.b[0], ut, w.fixed)
    Lc, _, gbc, gac, its, res = O.grad_cg(p, w.b[0], ut, w.fixed, tol=1e-13)
    assert Lc == pytest.approx(Ld, rel=1e-9)
    assert np.abs(gac - gad).max() <= 1e-8 * np.abs(gad).max()
    assert np.abs(gbc - gbd).max() <= 1e-8 * np.abs(gbd).max()


def test_energy_parts_sum_to_the_energy():
    """Kinetic, elastic and load terms: their sum is the energy; at u = 0 only the
    kinetic term 1/2 rho V v.v remains (free DOFs); elastic = -1/2 V u.(A u) >= 0."""
    rng = np.random.default_rng(13)
    p = _prob2(11, 9, 3)
    p.rho = 1.7
    fixed = _dirichlet_layer(p)
    u, v, b = (rng.standard_normal((2, p.N)) for _ in range(3))
    kin, el, load = O.energy_parts(p, u, v, b, fixed)
    assert kin + el + load == O.energy(p, u, v, b, fixed)
    assert el >= 0.0 and kin >= 0.0
    V = p.h ** 2
    F = ~fixed.reshape(-1)
    k0, e0, l0 = O.energy_parts(p, np.zeros((2, p.N)), v, b, fixed)
    assert e0 == 0.0 and l0 == 0.0
    assert k0 == pytest.approx(0.5 * p.rho * V * float(v.reshape(-1)[F] @ v.reshape(-1)[F]), rel=1e-15)


def test_lift_equals_dense_block():
    """b_F - K_FC g_C computed with the bond-sum apply equals the dense block product."""
    rng = np.random.default_rng(12)
    p = _prob2(12, 10, 3)
    fixed = _dirichlet_layer(p).reshape(-1)
    g = np.where(fixed, rng.standard_normal(fixed.shape), 0.0)
    b = rng.standard_normal(fixed.shape)
    A = O.assemble_dense(p)
    F, C = ~fixed, fixed
    ref = b[F] + A[np.ix_(F, C)] @ g[C]
    got = O.lifted_rhs(p, b, fixed, g).reshape(-1)
    assert np.allclose(got[F], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert np.all(got[C] == 0)


# ---------------------------------------------------------------- circulant preconditioner

def test_generating_blocks_match_golden_stencil():
    """G(o) read off the unit-displacement force equals the hand-worked entries of
    eq. (frb:e1) (A_{p, p+o} = G(-o) = G(o))."""
    M = 3
    p = O.Problem((7, 7), 1.0, M, 1.0)
    G = O.generating_blocks(p)
    comp = {"xx": (0, 0), "yy": (1, 1), "xy": (0, 1)}
    rows = [l.split() for l in open(os.path.join(GOLDEN, "stencil_M3_2d.txt"))
            if l.strip() and not l.startswith("#")]
    for ox, oy, cname, val in rows:
        a, b = comp[cname]
        for sgn in (1, -1):
            got = G[a, b, M + sgn * int(oy), M + sgn * int(ox)]
            assert got == pytest.approx(float(val), rel=1e-14, abs=1e-15), (ox, oy, cname)


@pytest.mark.parametrize("dim", [2, 3])
def test_generating_blocks_symmetries(dim):
    """Sum over o of G(o) = 0 (rigid translation), G(o) = G(-o), symmetric blocks, and
    G(o) = 0 outside the horizon |o| > M."""
    p = _prob2(9, 9, 3) if dim == 2 else _prob3(5, 5, 5, 2)
    G = O.generating_blocks(p)
    M = p.M
    scale = np.abs(G).max()
    assert np.abs(G.sum(axis=tuple(range(2, dim + 2)))).max() <= 1e-13 * scale
    flip = G[(slice(None), slice(None)) + (slice(None, None, -1),) * dim]
    assert np.abs(G - flip).max() <= 1e-15 * scale
    assert np.array_equal(G, np.swapaxes(G, 0, 1))
    o = np.stack(np.meshgrid(*([np.arange(-M, M + 1)] * dim), indexing="ij"))
    outside = (o ** 2).sum(axis=0) > M * M
    assert np.all(G[:, :, outside] == 0.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_apply_equals_bounded_apply_in_interior(dim):
    """For u on the N grid zero-padded to L >= N + M, the periodic operator agrees with the
    bond sum of eq. (mat:f1) on every node whose horizon lies inside the domain."""
    rng = np.random.default_rng(31 + dim)
    if dim == 2:
        p, L = _prob2(14, 11, 3), (18, 15)
    else:
        p, L = _prob3(8, 7, 6, 2), (11, 9, 8)
    M, d = p.M, dim
    u = rng.standard_normal((d, p.N))
    nshp = tuple(reversed(p.n))
    full = np.zeros((d,) + tuple(reversed(L)))
    full[(slice(None),) + tuple(slice(0, m) for m in nshp)] = u.reshape((d,) + nshp)
    ap = O.periodic_apply(p, L, full.reshape(d, -1)).reshape(full.shape)
    ap = ap[(slice(None),) + tuple(slice(0, m) for m in nshp)]
    ab = O.force(p, u).reshape((d,) + nshp)
    inner = (slice(None),) + (slice(M, -M),) * d
    assert np.abs(ap[inner] - ab[inner]).max() <= 1e-12 * np.abs(ab).max()
    # the boundary rows differ (incomplete horizons: the D^e correction)
    assert np.abs(ap - ab).max() > 1e-3 * np.abs(ab).max()


def _dense_periodic(p, L):
    n = int(np.prod(L)) * p.dim
    C = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        C[:, j] = -O.periodic_apply(p, L, e.reshape(p.dim, -1)).reshape(-1)
    return C


@pytest.mark.parametrize("dim", [2, 3])
def test_precond_equals_dense_inverse(dim):
    """Brute force on tiny grids: z = Pi_F E^T (K_per + s I)^{-1} E r with K_per assembled
    column by column from the direct convolution and inverted densely; s = 1e-3 x the
    largest absolute row sum over the frequency blocks."""
    rng = np.random.default_rng(41 + dim)
    if dim == 2:
        p, L = _prob2(5, 4, 2), (8, 7)
    else:
        p, L = _prob3(3, 3, 2, 2), (6, 5, 5)
    d = p.dim
    K = _dense_periodic(p, L)
    assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert ev.min() >= -1e-12 * ev.max()            # positive semi-definite, translations in the kernel
    Kh, s = O.precond_symbol(p, L)
    # the Gershgorin bound of every block is at least its largest eigenvalue
    assert 1e-3 * ev.max() <= s * (1 + 1e-12)
    Cinv = np.linalg.inv(K + s * np.eye(K.shape[0]))
    fixed = np.zeros((d, p.N), dtype=bool)
    fixed[:, :p.n[0]] = True                          # first grid row constrained
    r = rng.standard_normal((d, p.N))
    # explicit padding: node id i + nx (j + ny k) -> i + Lx (j + Ly k)
    ids = np.arange(p.N)
    coords = []
    rem = ids.copy()
    for m in p.n:
        coords.append(rem % m)
        rem //= m
    pid = np.zeros(p.N, dtype=np.int64)
    for a in reversed(range(d)):
        pid = pid * L[a] + coords[a]
    nL = int(np.prod(L))
    E = np.zeros((d * nL, d * p.N))
    for c in range(d):
        E[c * nL + pid, c * p.N + ids] = 1.0
    ref = (E.T @ Cinv @ E @ r.reshape(-1)).reshape(d, p.N)
    ref[fixed] = 0.0
    got = O.precond_apply(p, r, L, fixed)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
    # constant fields are the k = 0 mode: (K_per + s I)^{-1} c = c / s
    const = np.ones((d, nL)) * np.arange(1, d + 1)[:, None]
    assert np.allclose(O.precond_apply_periodic(p, L, const), const / s, rtol=1e-12)


def test_precond_is_spd_on_free_dofs():
    rng = np.random.default_rng(51)
    p, L = _prob2(20, 17, 3), (24, 20)
    fixed = np.zeros((2, p.N), dtype=bool)
    fixed[:, ::20] = True                              # left column
    r1 = np.where(fixed, 0.0, rng.standard_normal((2, p.N)))
    r2 = np.where(fixed, 0.0, rng.standard_normal((2, p.N)))
    z1, z2 = O.precond_apply(p, r1, L, fixed), O.precond_apply(p, r2, L, fixed)
    assert abs((r1 * z2).sum() - (r2 * z1).sum()) <= 1e-13 * abs((r1 * z1).sum())
    assert (r1 * z1).sum() > 0 and (r2 * z2).sum() > 0


# ---------------------------------------------------------------- crack propagation (eq. (mu))

@pytest.mark.parametrize("dim", [2, 3])
def test_all_bonds_equals_pair_double_loop(dim):
    p = _prob2(9, 7, 3) if dim == 2 else _prob3(5, 4, 4, 2)
    got = {tuple(b) for b in O.all_bonds(p)}
    n = list(p.n)
    coords = [np.unravel_index(i, tuple(reversed(n)))[::-1] for i in range(p.N)]
    want = set()
    for a in range(p.N):
        for b in range(a + 1, p.N):
            if sum((x - y) ** 2 for x, y in zip(coords[a], coords[b])) <= p.M ** 2:
                want.add((a, b))
    assert got == want


@pytest.mark.parametrize("dim", [2, 3])
def test_stretch_zero_under_rigid_motion(dim):
    """Translations and finite rotations leave every bond length unchanged (eq. (fra:s1)
    is the nonlinear stretch), so nothing breaks at any s0 > 1e-12."""
    p = _prob2(12, 10, 3) if dim == 2 else _prob3(6, 5, 5, 2)
    x = p.node_coords()
    t = 0.7
    if dim == 2:
        R = np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])
    else:
        R = np.array([[1, 0, 0], [0, math.cos(t), -math.sin(t)], [0, math.sin(t), math.cos(t)]])
    for u in (np.ones((dim, p.N)) * np.arange(1, dim + 1)[:, None], R @ x - x):
        s = O.bond_stretch(p, u, O.all_bonds(p))
        assert np.abs(s).max() <= 1e-13
        new, allb, _ = O.crack_update(p, u, 1e-12)
        assert len(new) == 0 and len(allb) == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_stretch_breaks_the_closed_form_set(dim):
    """u = eps x_1 e_1: a bond at angle theta to e_1 has s = sqrt((1+eps)^2 cos^2 + sin^2) - 1,
    so it breaks iff cos^2(theta) >= ((1+s0)^2 - 1) / ((1+eps)^2 - 1); the number of broken
    bonds is the sum over those offsets o of prod_a (n_a - |o_a|)."""
    p = _prob2(14, 11, 3) if dim == 2 else _prob3(7, 6, 5, 2)
    eps, s0 = 0.05, 0.03
    x = p.node_coords()
    u = np.zeros_like(x)
    u[0] = eps * x[0]
    thresh = ((1 + s0) ** 2 - 1) / ((1 + eps) ** 2 - 1)
    M = p.M
    want = 0
    for o in np.ndindex(*([2 * M + 1] * dim)):
        o = np.array(o) - M
        s2 = int((o * o).sum())
        if s2 == 0 or s2 > M * M:
            continue
        lex = next((v for v in o[::-1] if v != 0), 0)   # count each bond once: o > 0 in (z, y, x) order
        if lex < 0:
            continue
        c2 = o[0] ** 2 / s2
        assert abs(c2 - thresh) > 1e-6                  # no direction at the threshold
        if c2 >= thresh:
            want += int(np.prod([m - abs(v) for m, v in zip(p.n, o)]))
    new, allb, s = O.crack_update(p, u, s0)
    assert len(new) == want and want > 0
    # history: bonds already broken are not reported again, the union is kept
    half = new[: len(new) // 2]
    new2, allb2, _ = O.crack_update(p, u, s0, half)
    assert len(new2) == want - len(half)
    assert np.array_equal(allb2, allb)


# ---------------------------------------------------------------- surface correction (Remark 3)

def _omega_e(p):
    """Nodes within M of a face (incomplete horizon)."""
    n = list(p.n)
    coords = np.stack(np.unravel_index(np.arange(p.N), tuple(reversed(n)))[::-1])
    on = np.zeros(p.N, dtype=bool)
    for a in range(p.dim):
        on |= (coords[a] < p.M) | (coords[a] >= n[a] - p.M)
    return on


@pytest.mark.parametrize("dim", [2, 3])
def test_surface_constant_factor_scales_edge_rows(dim):
    """nu = c everywhere: v_pq = c on the rows of Omega_e, so those rows are c f and every
    other row is f; nu = 1 is the plain sum."""
    rng = np.random.default_rng(61 + dim)
    p = _prob2(13, 11, 3) if dim == 2 else _prob3(8, 7, 7, 2)
    br = _random_bonds(p, 15, 62)
    u = rng.standard_normal((dim, p.N))
    f = O.force(p, u, br)
    assert np.array_equal(O.force(p, u, br, nu=np.ones(p.N)), f)
    fc = O.force(p, u, br, nu=np.full(p.N, 1.7))
    on = _omega_e(p)
    assert np.allclose(fc[:, on], 1.7 * f[:, on], rtol=1e-13, atol=1e-13 * np.abs(f).max())
    assert np.array_equal(fc[:, ~on], f[:, ~on])
    assert on.any() and (~on).any()


def test_surface_rigid_translation_and_interior_rows():
    """Any factors: a translation still gives zero force (each bond term has u_q - u_p),
    and rows off Omega_e are untouched."""
    rng = np.random.default_rng(63)
    p = _prob2(14, 12, 3)
    nu = rng.uniform(0.5, 2.0, p.N)
    t = np.ones((2, p.N)) * np.array([[0.3], [-1.1]])
    assert np.abs(O.force(p, t, nu=nu)).max() <= 1e-12 * np.abs(O.force(p, rng.standard_normal((2, p.N)))).max()
    u = rng.standard_normal((2, p.N))
    on = _omega_e(p)
    assert np.array_equal(O.force(p, u, nu=nu)[:, ~on], O.force(p, u)[:, ~on])


def test_surface_volume_factors_closed_form():
    """M = 1 (4 neighbours, lambda = 1/2 each): corner 4/2 = 2, edge 4/3, interior 1.
    M = 3: a node at distance 2 from one face lacks only the offset (-3, 0) of weight 1/2."""
    p = _prob2(5, 4, 1)
    nu = O.surface_volume_factors(p).reshape(4, 5)
    assert nu[0, 0] == 2.0 and nu[3, 4] == 2.0 and nu[0, 2] == pytest.approx(4 / 3, abs=1e-15)
    assert nu[1, 2] == 1.0
    p3 = _prob2(12, 12, 3)
    nu3 = O.surface_volume_factors(p3).reshape(12, 12)
    lam = [1.0 if s2 <= 6 else 3.5 - math.sqrt(s2)
           for s2 in (ox * ox + oy * oy for oy in range(-3, 4) for ox in range(-3, 4)) if 0 < s2 <= 9]
    full = sum(lam)
    assert nu3[5, 2] == pytest.approx(full / (full - 0.5), rel=1e-14)


def _surface_entry(p, nu, pi, qi, a, b):
    """A[a p, b q] of the surface-corrected operator, read off the force of a unit
    displacement of DOF (b, q) at row p."""
    e = np.zeros((p.dim, p.N))
    e[b, qi] = 1.0
    return O.force(p, e, nu=nu, rows=np.array([pi]))[a, 0]


def test_surface_golden_rows():
    """Hand-worked rows (tests/golden/surface_rows_M2_2d.txt): one bond coefficient
    v_pq = (nu_p + nu_q)/2 per bond on the rows of Omega_e, with non-constant nu, so a
    factor taken from p alone (or from q alone) changes the entries."""
    n, M = 7, 2
    p = O.Problem((n, n), 1.0, M, 1.0)
    ix = np.arange(p.N) % n
    nu = 1.0 + ix / 10.0
    comp = {"xx": (0, 0), "yy": (1, 1), "xy": (0, 1)}
    rows = [l.split() for l in open(os.path.join(GOLDEN, "surface_rows_M2_2d.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 15
    for px, py, qx, qy, cname, val in rows:
        a, b = comp[cname]
        got = _surface_entry(p, nu, int(py) * n + int(px), int(qy) * n + int(qx), a, b)
        assert got == pytest.approx(float(val), rel=1e-14, abs=1e-15), (px, py, qx, qy, cname)


def test_surface_block_symmetric_on_omega_e():
    """A bond's micromodulus belongs to the pair, so the scaled block is symmetric
    between two rows of Omega_e (A_pq = A_qp for p, q both in Omega_e); across the edge of
    Omega_e it is not (the row of the node off Omega_e is unscaled)."""
    rng = np.random.default_rng(64)
    p = _prob2(9, 8, 3)
    nu = rng.uniform(0.6, 1.8, p.N)
    on = _omega_e(p)
    A = np.stack([O.force(p, np.eye(2 * p.N)[j].reshape(2, p.N), nu=nu).reshape(-1) for j in range(2 * p.N)], 1)
    idx = np.concatenate([np.flatnonzero(on), p.N + np.flatnonzero(on)])
    Ae = A[np.ix_(idx, idx)]
    assert np.allclose(Ae, Ae.T, rtol=0, atol=1e-13 * np.abs(Ae).max())
    off = np.concatenate([np.flatnonzero(~on), p.N + np.flatnonzero(~on)])
    cross = A[np.ix_(idx, off)]
    assert np.abs(cross - A[np.ix_(off, idx)].T).max() > 1e-3 * np.abs(Ae).max()


# ---------------------------------------------------------------- adaptive dynamic relaxation (Alg. 1)

def test_adr_converges_to_the_dense_solution():
    """The damped relaxation of eq. (ADR:e1) has the static solution of eq. (mat:e2) as its
    fixed point: clamped plate with a crack and prescribed displacements, and a cantilever."""
    from paper_2301_11828_amd import workloads as W
    for (n, fixed, crack, steps, tol) in (((20, 16), "all", True, 200, 1e-12), ((16, 12), "left", False, 500, 1e-10)):
        w = W.small(2, n, 3, seed=71, fixed=fixed, crack=crack)
        p = O.Problem(w.n, w.h, w.M, w.alpha)
        br = None if w.cracks is None else O.crack_to_bonds(p, w.cracks)
        g = np.where(w.fixed, 0.01 * np.random.default_rng(72).standard_normal((2, p.N)), 0.0)
        ref = O.solve_dense(p, w.b[0], w.fixed, g, br)
        u, v, F, cs = O.adr(p, np.zeros((2, p.N)), w.b[0], steps, w.fixed, g, br)
        err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
        assert err <= tol, (fixed, err)
        assert np.array_equal(u[w.fixed], g[w.fixed])
        assert all(c >= 0 for c in cs)


@pytest.mark.parametrize("dim", [2, 3])
def test_adr_density_bounds_the_spectrum_and_interior_closed_form(dim):
    """D = 1/4 Gershgorin: the eigenvalues of D^-1 K lie in [0, 4]; on a node with a full
    horizon D_aa = 1/4 (sum_b |sum_o G_ab(o)| over the diagonal block + sum_o sum_b |G_ab(o)|)
    with the generating blocks G read off the unit-displacement force."""
    p = _prob2(9, 8, 2) if dim == 2 else _prob3(6, 5, 5, 1)
    K = -O.assemble_dense(p)
    D = O.adr_density(p)
    ev = np.linalg.eigvals(K / D.reshape(-1)[:, None]).real
    assert ev.min() >= -1e-12 and ev.max() <= 4.0 + 1e-12
    G = O.generating_blocks(p)
    M = p.M
    ctr = tuple([M] * dim)
    off = G.copy()
    off[(slice(None), slice(None)) + ctr] = 0.0
    diag = -G[(slice(None), slice(None)) + ctr]       # K_pp = -A_pp
    node = sum((M + 1) * int(np.prod(p.n[:a])) for a in range(dim))   # index (M+1, ..., M+1): full horizon
    for a in range(dim):
        want = 0.25 * (np.abs(diag[a]).sum() + np.abs(off[a]).sum())
        assert D[a, node] == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_fft_apply_equals_bond_sum(dim):
    """The fast method on the CPU (zero-padded embedding, FFT block product, D^e, D^f) equals
    the bond-by-bond sum of eq. (mat:f1) on every row, with broken bonds, constrained DOFs,
    influence coefficients and both the N + M and the paper's 2N padding; leaving out the
    broken bonds breaks it (the periodic pin above shows the rows D^e changes)."""
    rng = np.random.default_rng(51 + dim)
    if dim == 2:
        p = _prob2(17, 13, 3, infl=(0.6, 0.3, 0.1))
    else:
        p = _prob3(8, 7, 6, 2)
    broken = _random_bonds(p, 40, 52 + dim)
    fixed = np.zeros((dim, p.N), dtype=bool)
    fixed[0, : p.n[0]] = True
    u = rng.standard_normal((dim, p.N))
    ref = O.apply(p, u, fixed, broken)
    scale = np.abs(ref).max()
    for L in (None, tuple(2 * n for n in p.n)):
        f = O.fft_apply(p, u, fixed, broken, L=L)
        assert np.abs(f - ref).max() <= 1e-12 * scale
    # without the broken-bond term, or on a product without D^e (interior-only agreement)
    f_nob = O.fft_apply(p, u, fixed, None)
    assert np.abs(f_nob - ref).max() > 1e-3 * scale
    assert np.abs(f_nob - O.apply(p, u, fixed, None)).max() <= 1e-12 * scale
