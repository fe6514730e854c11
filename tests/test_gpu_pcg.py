"""Preconditioned CG: the circulant preconditioner (prior fast methods cited in Sec. 1)
applied on its own against the oracle's Fourier-space inverse, and preconditioned static
solves of eq. (mat:e2) against the oracle's dense Cholesky solve."""
import numpy as np
import pytest

import oracle as O
from paper_2301_11828_amd import workloads as W
from helpers import gpu_plan, log, oracle_bonds, oracle_problem, rel_err, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-6


def _dense(w, c=0, g=None):
    return O.solve_dense(oracle_problem(w), w.b[c], w.fixed, None if g is None else g[c], oracle_bonds(w))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_apply_precond_matches_oracle(prec, dim):
    import torch
    if dim == 2:
        w = W.small(2, (45, 38), 3, seed=201, fixed="left", crack=True, batch=2)
    else:
        w = W.small(3, (14, 11, 9), 2, seed=202, fixed="bottom", batch=2)
    plan = gpu_plan(w)
    dt = torch.float64 if prec == "fp64" else torch.float32
    r = w.b if prec == "fp64" else w.b.astype(np.float32).astype(np.float64)
    z = plan.apply_precond(to_dev(w.b, dt), torch.full((w.batch, w.dim, w.N), float("nan"), dtype=dt,
                                                       device="cuda")).double().cpu().numpy()
    L = plan.padded_lengths
    for c in range(w.batch):
        ref = O.precond_apply(oracle_problem(w), r[c], L, w.fixed)
        err = rel_err(z[c], ref)
        log("precond %dD %s L=%s case %d rel err %.2e" % (dim, prec, L, c, err))
        assert err <= (FP64_TOL if prec == "fp64" else FP32_TOL)


def test_apply_precond_per_case_and_after_set_infl():
    """Per-case influence coefficients give each case its own C; new coefficients rebuild it."""
    w = W.small(2, (33, 29), 3, seed=203, fixed="all", batch=3)
    plan = gpu_plan(w)
    L = plan.padded_lengths
    infl = np.array([[1.0, 0.0], [0.3, 0.8], [0.6, -0.2]])
    plan.apply_precond(to_dev(w.b))        # builds C for the shared coefficients first
    plan.set_infl(infl, per_case=True)
    z = plan.apply_precond(to_dev(w.b)).cpu().numpy()
    for c in range(3):
        ref = O.precond_apply(oracle_problem(w, infl=tuple(infl[c])), w.b[c], L, w.fixed)
        err = rel_err(z[c], ref)
        log("per-case precond case %d rel err %.2e" % (c, err))
        assert err <= FP64_TOL
    plan.set_infl((0.5, 0.5))
    z = plan.apply_precond(to_dev(w.b)).cpu().numpy()
    for c in range(3):
        err = rel_err(z[c], O.precond_apply(oracle_problem(w, infl=(0.5, 0.5)), w.b[c], L, w.fixed))
        assert err <= FP64_TOL


@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
def test_pcg_matches_cholesky_2d_crack_and_lift(prec):
    w = W.small(2, (30, 26), 3, seed=204, fixed="all", crack=True, batch=2)
    g = np.where(w.fixed[None], np.random.default_rng(205).standard_normal((2, 2, w.N)), 0.0)
    plan = gpu_plan(w)
    u, info = plan.solve(to_dev(w.b), g=to_dev(g), precision=prec, tol=1e-13, precond=True)
    uu = u.cpu().numpy()
    for c in range(2):
        err = rel_err(uu[c], _dense(w, c, g))
        log("pcg %s case %d: %d outer %d inner, residual %.2e, rel err %.2e" %
            (prec, c, info[c].outer_iters, info[c].inner_iters, info[c].rel_residual, err))
        assert info[c].status == 0
        assert err <= (1e-11 if prec == "fp64" else 1e-10)
        assert np.array_equal(uu[c][w.fixed], g[c][w.fixed])


@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
def test_pcg_matches_cholesky_3d(prec):
    w = W.small(3, (13, 11, 9), 2, seed=206, fixed="bottom", batch=2)
    plan = gpu_plan(w)
    u, info = plan.solve(to_dev(w.b), precision=prec, tol=1e-13, precond=True)
    for c in range(2):
        err = rel_err(u.cpu().numpy()[c], _dense(w, c))
        log("pcg 3D %s case %d: %d inner, rel err %.2e" % (prec, c, info[c].inner_iters, err))
        assert info[c].status == 0 and err <= (1e-11 if prec == "fp64" else 1e-10)


def test_pcg_plain_fp32_error_stated():
    w = W.small(2, (40, 36), 3, seed=207, fixed="left")
    plan = gpu_plan(w)
    u, info = plan.solve(to_dev(w.b), precision="fp32", tol=1e-5, precond=True, check=False)
    err = rel_err(u.cpu().numpy()[0], _dense(w))
    log("pcg plain fp32 to 1e-5: %d it, FP64 residual %.2e, rel err %.2e" % (info[0].inner_iters,
                                                                            info[0].rel_residual, err))
    assert err <= 1e-4


def test_pcg_cuts_iterations():
    """On a 128 x 128 plate clamped on one side the preconditioner cuts the CG iteration
    count several times over; both solves agree with each other and with the oracle's
    bond-sum residual."""
    w = W.small(2, (128, 128), 3, seed=208, fixed="left")
    plan = gpu_plan(w)
    u0, i0 = plan.solve(to_dev(w.b), precision="fp64", tol=1e-10)
    u1, i1 = plan.solve(to_dev(w.b), precision="fp64", tol=1e-10, precond=True)
    a = u1.cpu().numpy()[0]
    p = oracle_problem(w)
    free = ~w.fixed
    r = (w.b[0] + O.apply(p, a, w.fixed))[free]
    rel = np.linalg.norm(r) / np.linalg.norm(w.b[0][free])
    d = rel_err(a, u0.cpu().numpy()[0])
    log("128^2: CG %d it, PCG %d it, oracle residual %.2e, PCG vs CG %.2e" %
        (i0[0].inner_iters, i1[0].inner_iters, rel, d))
    assert i0[0].status == 0 and i1[0].status == 0
    assert 3 * i1[0].inner_iters <= i0[0].inner_iters
    assert rel <= 2e-10 and d <= 1e-7


def test_pcg_graph_blocks_equal_plain():
    w = W.small(2, (40, 33), 3, seed=209, fixed="left", batch=2)
    plan = gpu_plan(w)
    a, ia = plan.solve(to_dev(w.b), precision="fp64", tol=1e-12, precond=True)
    b, ib = plan.solve(to_dev(w.b), precision="fp64", tol=1e-12, precond=True, graph_block=8)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert [x.inner_iters for x in ia] == [x.inner_iters for x in ib]


def test_pcg_many_tiles_per_case():
    """More than 1024 x-tiles per case: the case sums of both chains come from the
    per-case reduction kernel; the result matches the fused path and the oracle."""
    w = W.small(2, (24, 1100), 3, seed=210, fixed="left", batch=2)
    plan = gpu_plan(w)
    plan.set_config("fp64", rows_per_wg=1, team_x=0)
    u1, info1 = plan.solve(to_dev(w.b), precision="fp64", tol=1e-11, maxit=20000, precond=True)
    plan.set_config("fp64", rows_per_wg=8, team_x=0)
    u2, info2 = plan.solve(to_dev(w.b), precision="fp64", tol=1e-11, maxit=20000, precond=True)
    a, bb = u1.cpu().numpy(), u2.cpu().numpy()
    p = oracle_problem(w)
    for c in range(2):
        free = ~w.fixed
        r = (w.b[c] + O.apply(p, a[c], w.fixed))[free]
        rel = np.linalg.norm(r) / np.linalg.norm(w.b[c][free])
        d = rel_err(a[c], bb[c])
        log("pcg 1100 tiles/case: case %d %d vs %d it, oracle residual %.2e, vs fused %.2e" %
            (c, info1[c].inner_iters, info2[c].inner_iters, rel, d))
        assert info1[c].status == 0 and info2[c].status == 0
        assert rel <= 1e-10 and d <= 1e-8


@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("tiled", [False, True])
def test_reliable_update_matches_cholesky(precond, tiled):
    """FP32 CG inside FP64 refinement that keeps its search direction across residual
    replacements (plain and preconditioned; chain and tiled products), with a crack, a lift
    and three cases, against each case's dense Cholesky solve; certified residual <= tol."""
    w = W.small(2, (34, 27), 3, seed=211, fixed="left", crack=True, batch=3)
    rng = np.random.default_rng(212)
    g = np.where(w.fixed[None], 1e-2 * rng.standard_normal((w.batch, 2, w.N)), 0.0)
    plan = gpu_plan(w)
    if tiled:
        for f in ("fp64", "fp32"):
            plan.set_config(f, tile=16, tile_regs=1, tile_run=1)
    tol = 1e-11
    u, info = plan.solve(to_dev(w.b), to_dev(g), precision="fp32_refined", tol=tol, reliable_update=1,
                         precond=precond)
    _, info_r = plan.solve(to_dev(w.b), to_dev(g), precision="fp32_refined", tol=tol, precond=precond)
    uu = u.cpu().numpy()
    for c in range(w.batch):
        ref = O.solve_dense(oracle_problem(w), w.b[c], w.fixed, g[c], oracle_bonds(w))
        err = rel_err(uu[c], ref)
        log("reliable updates precond=%d tiled=%d case %d: %d outer %d inner (restarted: %d outer %d inner), "
            "residual %.2e, rel err %.2e" % (precond, tiled, c, info[c].outer_iters, info[c].inner_iters,
                                             info_r[c].outer_iters, info_r[c].inner_iters, info[c].rel_residual, err))
        assert info[c].status == 0 and info[c].rel_residual <= tol
        assert err <= 1e-9


def test_plate512_pcg_at_the_benchmark_tuning_certified_by_oracle():
    """Full size, the bench's recorded tuning: FP64 and FP32-refined preconditioned solves to
    1e-10, each certified by the oracle's bond-sum residual."""
    import json
    import os
    rec = json.load(open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                                      "plate512_tuning.json")))
    w = W.plate512()
    plan = gpu_plan(w)
    plan.set_lengths(rec["padded"])
    plan.set_config("fp64", **rec["fp64"])
    plan.set_config("fp32", **rec["fp32"])
    p = oracle_problem(w)
    bp = O.lifted_rhs(p, w.b[0], w.fixed).reshape(-1)
    for prec in ("fp64", "fp32_refined"):
        u, info = plan.solve(to_dev(w.b), precision=prec, tol=1e-10, maxit=200000, precond=True)
        r = bp + O.apply(p, u.cpu().numpy()[0], w.fixed).reshape(-1)
        res = np.linalg.norm(r) / np.linalg.norm(bp)
        log("plate512 PCG %s: %d it, oracle residual %.2e" % (prec, info[0].inner_iters, res))
        assert info[0].status == 0 and res <= 1.05e-10


@pytest.mark.parametrize("precond", [False, True])
def test_refined_graph_blocks_reused_across_solves_equal_plain(precond):
    """The refinement loop's inner solves replay one captured block of iterations (kept in the
    plan's workspace across calls): every solve equals its plain-launch twin bit for bit,
    also after new coefficients and after a configuration change (a new capture)."""
    import torch
    w = W.small(2, (40, 31), 3, seed=221, fixed="left", crack=True, batch=2, infl=(0.7, 0.2))
    plan = gpu_plan(w)
    rng = np.random.default_rng(222)
    steps = [None, dict(infl=(0.5, 0.4)), dict(cfg=dict(tile=16, tile_regs=1, tile_run=1)), None]
    for k, step in enumerate(steps):
        if step and "infl" in step:
            plan.set_infl(np.array(step["infl"]))
        if step and "cfg" in step:
            for f in ("fp64", "fp32"):
                plan.set_config(f, **step["cfg"])
        b = to_dev(rng.standard_normal((w.batch, 2, w.N)))
        for rel in (0, 1):
            a, ia = plan.solve(b, precision="fp32_refined", tol=1e-11, graph_block=8, precond=precond,
                               reliable_update=rel)
            a = a.clone()
            c, ic = plan.solve(b, precision="fp32_refined", tol=1e-11, graph_block=0, precond=precond,
                               reliable_update=rel)
            log("graph reuse step %d reliable %d: %s vs %s iterations" % (k, rel, [x.inner_iters for x in ia],
                                                                        [x.inner_iters for x in ic]))
            assert torch.equal(a, c)
            assert [x.inner_iters for x in ia] == [x.inner_iters for x in ic]
