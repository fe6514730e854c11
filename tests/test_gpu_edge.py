"""Degenerate shapes for the solvers and corrections: horizons wider than the grid (every
column within M of a face), single-row and single-column grids, and empty updates, each
against the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2301_11828_amd import workloads as W
from helpers import gpu_apply, gpu_plan, log, oracle_bonds, oracle_problem, rel_err, to_dev

pytestmark = pytest.mark.gpu

# solvable shapes (K_FF positive definite)
SOLVE_SHAPES = [
    (2, (6, 5), 4, "left"),       # horizon wider than the grid in both directions
    (3, (4, 3, 5), 3, "bottom"),  # every node of a 3D block within M of a face
]
# single-row / single-column grids: every bond is parallel to the grid line, so the
# transverse block of K vanishes (singular for solves); products and corrections only
SHAPES = SOLVE_SHAPES + [
    (2, (1, 17), 2, "none"),
    (2, (19, 1), 2, "left"),
]


def _ids(c):
    return "%dd-%s-M%d-%s" % (c[0], "x".join(map(str, c[1])), c[2], c[3])


@pytest.mark.parametrize("case", SOLVE_SHAPES, ids=_ids)
def test_pcg_and_cg_degenerate_shapes(case):
    dim, n, M, fixed = case
    w = W.small(dim, n, M, seed=601, fixed=fixed, batch=2)
    plan = gpu_plan(w)
    for pre in (False, True):
        u, info = plan.solve(to_dev(w.b), precision="fp64", tol=1e-13, precond=pre, check=False)
        for c in range(2):
            ref = O.solve_dense(oracle_problem(w), w.b[c], w.fixed)
            err = rel_err(u.cpu().numpy()[c], ref)
            log("%s precond=%d case %d: status %d, %d it, rel err %.2e" % (_ids(case), pre, c, info[c].status,
                                                                            info[c].inner_iters, err))
            assert info[c].status == 0 and err <= 1e-11


@pytest.mark.parametrize("case", SHAPES, ids=_ids)
def test_precond_and_surface_degenerate_shapes(case):
    dim, n, M, fixed = case
    w = W.small(dim, n, M, seed=602, fixed=fixed)
    plan = gpu_plan(w)
    p = oracle_problem(w)
    z = plan.apply_precond(to_dev(w.b)).cpu().numpy()[0]
    ez = rel_err(z, O.precond_apply(p, w.b[0], plan.padded_lengths, w.fixed))
    nu = plan.surface_volume_factors()
    assert np.abs(nu - O.surface_volume_factors(p)).max() <= 1e-14 * nu.max()
    plan.set_surface(nu)
    f = gpu_apply(plan, to_dev(w.b)).cpu().numpy()[0]
    ef = rel_err(f, O.apply(p, w.b[0], w.fixed, None, nu=nu))
    log("%s: preconditioner rel err %.2e, surface-corrected product rel err %.2e" % (_ids(case), ez, ef))
    assert ez <= 1e-12 and ef <= 1e-12


@pytest.mark.parametrize("case", SHAPES, ids=_ids)
def test_crack_update_degenerate_shapes(case):
    dim, n, M, fixed = case
    w = W.small(dim, n, M, seed=603, fixed=fixed)
    plan = gpu_plan(w)
    p = oracle_problem(w)
    ur = 1e-2 * w.h * np.random.default_rng(604).standard_normal((1, w.dim, w.N))
    bonds = O.all_bonds(p)
    s = np.sort(O.bond_stretch(p, ur[0], bonds))
    i = (3 * len(s)) // 4                 # upper quartile: a positive critical stretch
    s0 = 0.5 * (s[i - 1] + s[i])
    assert s0 > 0 and np.abs(s - s0).min() > 1e-9 * s0
    new_ref, all_ref, _ = O.crack_update(p, ur[0], s0)
    nn = plan.crack_update(to_dev(ur), s0)
    log("%s: %d bonds, %d break (oracle %d)" % (_ids(case), len(bonds), nn, len(new_ref)))
    assert nn == len(new_ref) > 0 and np.array_equal(plan.bonds(), all_ref)
    f = gpu_apply(plan, to_dev(w.b)).cpu().numpy()[0]
    assert rel_err(f, O.apply(p, w.b[0], w.fixed, all_ref)) <= 1e-12


@pytest.mark.parametrize("case", SOLVE_SHAPES, ids=_ids)
def test_adr_degenerate_shapes(case):
    import torch
    dim, n, M, fixed = case
    w = W.small(dim, n, M, seed=603, fixed=fixed)
    plan = gpu_plan(w)
    p = oracle_problem(w)
    # ADR: zero updates only evaluates F; then relax to the fixed point
    u = torch.zeros((1, w.dim, w.N), dtype=torch.float64, device="cuda")
    v, F = torch.zeros_like(u), torch.zeros_like(u)
    res0 = plan.adr_run(0, u, v, F, to_dev(w.b), residual=True)
    F0 = w.b[0] * ~w.fixed
    assert rel_err(F.cpu().numpy()[0], F0) <= 1e-15 and abs(res0[0] - np.linalg.norm(F0)) <= 1e-12 * np.linalg.norm(F0)
    plan.adr_run(3000, u, v, F, to_dev(w.b), restart=False)
    ref = O.solve_dense(p, w.b[0], w.fixed)
    ea = rel_err(u.cpu().numpy()[0], ref)
    log("%s: ADR 3000 updates, rel err vs Cholesky %.2e" % (_ids(case), ea))
    assert ea <= 1e-9


# the largest padded lengths a workgroup's LDS holds in FP64 (x pass: twiddles and two
# buffers of one complex row, 48 L bytes; 2D line pass: twiddles and two buffers of the
# two components of one line, 80 L bytes; both within 159 KiB): L_x = 3375 and L_y = 2025
MAX_SHAPES = [((3300, 6), 3375), ((6, 2022), 2025)]


@pytest.mark.parametrize("n,L", MAX_SHAPES, ids=["x3375", "y2025"])
def test_largest_lengths_the_lds_holds(n, L):
    import torch
    w = W.small(2, n, 3, seed=611, fixed="left")
    plan = gpu_plan(w)
    assert max(plan.padded_lengths) == L
    p = oracle_problem(w)
    for prec, dt, tol in (("fp64", torch.float64, 1e-12), ("fp32", torch.float32, 2e-6)):
        u = w.b if prec == "fp64" else w.b.astype(np.float32).astype(np.float64)
        f = gpu_apply(plan, to_dev(w.b, dt)).double().cpu().numpy()[0]
        err = rel_err(f, O.apply(p, u[0], w.fixed))
        log("grid %s, padded %s, %s product rel err %.2e" % (n, plan.padded_lengths, prec, err))
        assert err <= tol


@pytest.mark.parametrize("n", [(3400, 6), (6, 2040)], ids=["x3456", "y2048"])
def test_lengths_beyond_lds_are_rejected(n):
    """One 5-smooth length further (3456, 2048) no longer fits: plan creation fails with
    MSB_EUNSUPPORTED instead of a launch failing later."""
    import paper_2301_11828_amd as msb
    w = W.small(2, n, 3, seed=612)
    with pytest.raises(msb.MsbError) as e:
        gpu_plan(w)
    assert e.value.status == msb.MSB_EUNSUPPORTED


@pytest.mark.parametrize("dim", [2, 3])
def test_single_node_grid(dim):
    """One node and no bonds: the product is zero (up to the rounding of the transform's
    centre term against D^e, which cancel exactly in exact arithmetic), the crack update
    finds nothing, and the preconditioner is the oracle's (the shifted periodic symbol)."""
    w = W.small(dim, (1,) * dim, 1, seed=621, batch=2)
    plan = gpu_plan(w)
    p = oracle_problem(w)
    assert np.array_equal(O.apply(p, w.b[0], w.fixed), np.zeros((dim, 1)))
    f = gpu_apply(plan, to_dev(w.b)).cpu().numpy()
    scale = np.abs(w.b).max() * max(1.0, w.alpha * w.h ** dim)   # |u| x the stencil's weight scale
    log("%dD single node: |f| %.2e (scale %.2e)" % (dim, np.abs(f).max(), scale))
    assert np.abs(f).max() <= 1e-13 * scale
    z = plan.apply_precond(to_dev(w.b)).cpu().numpy()
    for c in range(2):
        ez = rel_err(z[c], O.precond_apply(p, w.b[c], plan.padded_lengths, w.fixed))
        log("%dD single node: preconditioner case %d rel err %.2e" % (dim, c, ez))
        assert ez <= 1e-12
    if dim == 2:   # the crack update takes single-case plans
        p1 = gpu_plan(w, batch=1)
        assert p1.crack_update(to_dev(w.b[:1]), 1e-3) == 0 and len(p1.bonds()) == 0
