"""CG steps fused into the frame-16 register kernel: the update of the previous step is
applied on each block's patch as it loads (r, p, q ping-pong between two vector sets), q = K p
and its partial sums follow in the same launch.  Checked against the oracle's dense Cholesky
solve of eq. (mat:e2), against hipGraph-block replays bit for bit, with cases that stop at
different steps (zero right-hand side, early convergence, iteration cap)."""
import numpy as np
import pytest

import oracle as O
from paper_2301_11828_amd import workloads as W
from helpers import gpu_plan, log, oracle_bonds, oracle_problem, rel_err, to_dev

pytestmark = pytest.mark.gpu

FUSED = dict(tile=16, tile_regs=1, tile_run=1)


def _plan(w):
    plan = gpu_plan(w)
    for f in ("fp64", "fp32"):
        plan.set_config(f, **FUSED)
    return plan


@pytest.mark.parametrize("prec,rel", [("fp64", 0), ("fp32_refined", 0), ("fp32_refined", 1)])
def test_fused_cg_matches_cholesky(prec, rel):
    w = W.small(2, (44, 37), 3, seed=801, fixed="left", batch=3, infl=(0.8, 0.3))
    rng = np.random.default_rng(802)
    g = np.where(w.fixed[None], 1e-2 * rng.standard_normal((w.batch, 2, w.N)), 0.0)
    b = w.b.copy()
    b[1] *= 1e-3          # a case with a smaller load (its own stop threshold)
    plan = _plan(w)
    tol = 1e-11
    u, info = plan.solve(to_dev(b), to_dev(g), precision=prec, tol=tol, reliable_update=rel, graph_block=8)
    chain = gpu_plan(w)   # the same solve on the three-pass chain (unfused steps)
    _, info_c = chain.solve(to_dev(b), to_dev(g), precision=prec, tol=tol, reliable_update=rel)
    uu = u.cpu().numpy()
    for c in range(w.batch):
        ref = O.solve_dense(oracle_problem(w), b[c], w.fixed, g[c], oracle_bonds(w))
        err = rel_err(uu[c], ref)
        log("fused CG %s reliable %d case %d: %d it (chain %d), residual %.2e, rel err %.2e" %
            (prec, rel, c, info[c].inner_iters, info_c[c].inner_iters, info[c].rel_residual, err))
        assert info[c].status == 0 and info[c].rel_residual <= tol
        assert err <= 100 * tol   # condition number of these plates below 100
        if prec == "fp64":   # FP32 iteration counts follow the product's rounding, not a pin
            assert abs(info[c].inner_iters - info_c[c].inner_iters) <= max(3, 0.02 * info_c[c].inner_iters)


@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
def test_fused_cg_graph_blocks_equal_plain(prec):
    """A zero right-hand side (stopped before the first step), a small load and two ordinary
    cases: graph-block replays equal plain launches bit for bit."""
    import torch
    w = W.small(2, (40, 33), 3, seed=811, fixed="left", batch=4)
    b = w.b.copy()
    b[0] = 0.0
    b[2] *= 1e-4
    plan = _plan(w)
    a, ia = plan.solve(to_dev(b), precision=prec, tol=1e-11, graph_block=8)
    a = a.clone()
    c, ic = plan.solve(to_dev(b), precision=prec, tol=1e-11, graph_block=0)
    log("fused graph vs plain %s: %s / %s iterations" % (prec, [x.inner_iters for x in ia], [x.inner_iters for x in ic]))
    assert torch.equal(a, c)
    assert [x.inner_iters for x in ia] == [x.inner_iters for x in ic]
    assert ia[0].status == 0 and float(a[0].abs().max()) == 0.0
    for k in range(1, 4):
        ref = O.solve_dense(oracle_problem(w), b[k], w.fixed, None, oracle_bonds(w))
        assert rel_err(a.cpu().numpy()[k], ref) <= (1e-11 if prec == "fp64" else 1e-9)


def test_fused_cg_iteration_cap():
    """Capped runs (the final update-only step through the fused kernel): the iterate after
    k steps equals the unfused chain's to rounding, graph and plain launches alike."""
    import torch
    import paper_2301_11828_amd as msb
    w = W.small(2, (36, 29), 3, seed=821, fixed="left", batch=2)
    plan = _plan(w)
    chain = gpu_plan(w)
    for k in (1, 2, 7, 16):
        a, ia = plan.solve(to_dev(w.b), precision="fp64", tol=1e-14, maxit=k, graph_block=4, check=False)
        a = a.clone()
        c, ic = plan.solve(to_dev(w.b), precision="fp64", tol=1e-14, maxit=k, graph_block=0, check=False)
        d, idd = chain.solve(to_dev(w.b), precision="fp64", tol=1e-14, maxit=k, check=False)
        err = rel_err(a.cpu().numpy(), d.cpu().numpy())
        log("fused capped at %d: status %s, vs chain rel diff %.2e" % (k, [x.status for x in ia], err))
        assert torch.equal(a, c)
        assert all(x.status == msb.MSB_ENOCONV for x in ia) and all(x.inner_iters == k for x in ia)
        assert err <= 1e-10


@pytest.mark.parametrize("prec,rel,tile", [("fp64", 0, 16), ("fp64", 0, 32), ("fp32_refined", 0, 32),
                                           ("fp32_refined", 1, 16)])
def test_group_fused_cg_equals_members_and_cholesky(prec, rel, tile):
    """Plan groups fuse the steps too when every member can (no crack, no surface factors):
    members of different sizes stop at different steps and leave the work list; each member's
    solution equals its own fused solve bit for bit and the dense Cholesky solution."""
    import torch
    import paper_2301_11828_amd as msb
    ws = [W.small(2, (40, 31), 3, seed=831, fixed="left", batch=2),
          W.small(2, (18, 23), 3, seed=832, fixed="all", batch=1, infl=(0.5, 0.2)),
          W.small(2, (57, 12), 3, seed=833, fixed="bottom", batch=2)]
    cfg = dict(tile=tile, tile_regs=1, tile_run=1)
    plans = [gpu_plan(w) for w in ws]
    grp = msb.PlanGroup(plans)
    for f in ("fp64", "fp32"):
        grp.set_config(f, **cfg)
    tol = 1e-11
    bs = [to_dev(w.b) for w in ws]
    us, infos = grp.solve(bs, precision=prec, tol=tol, reliable_update=rel, graph_block=8)
    us = [u.clone() for u in us]
    us0, _ = grp.solve(bs, precision=prec, tol=tol, reliable_update=rel, graph_block=0)
    for i, (w, p) in enumerate(zip(ws, plans)):
        assert torch.equal(us[i], us0[i]), "member %d: graph blocks differ from plain launches" % i
        for f in ("fp64", "fp32"):
            p.set_config(f, **grp.get_config(f))
        own, own_info = p.solve(bs[i], precision=prec, tol=tol, reliable_update=rel)
        if prec == "fp64":
            assert torch.equal(us[i], own), "member %d differs from its own fused solve" % i
        for c in range(w.batch):
            ref = O.solve_dense(oracle_problem(w), w.b[c], w.fixed, None, oracle_bonds(w))
            err = rel_err(us[i].cpu().numpy()[c], ref)
            log("group fused %s rel %d t%d member %d case %d: %d it (own %d), residual %.2e, rel err %.2e" %
                (prec, rel, tile, i, c, infos[i][c].inner_iters, own_info[c].inner_iters, infos[i][c].rel_residual, err))
            assert infos[i][c].status == 0 and infos[i][c].rel_residual <= tol
            assert err <= 100 * tol


@pytest.mark.parametrize("prec,rel", [("fp64", 0), ("fp32_refined", 0), ("fp32_refined", 1)])
def test_fused_pcg_matches_cholesky_and_graphs(prec, rel):
    """Preconditioned CG with its stiffness step fused (p = z + beta p on the patches, p
    alternating between two vectors): cases stopping at different steps (a zero and a small
    load), against dense Cholesky, graph-block replays bit for bit, and FP64 iteration counts
    of the unfused chain."""
    import torch
    w = W.small(2, (46, 35), 3, seed=841, fixed="left", batch=4, infl=(0.7, 0.4))
    b = w.b.copy()
    b[0] = 0.0
    b[2] *= 1e-3
    plan = _plan(w)
    tol = 1e-11
    u, info = plan.solve(to_dev(b), precision=prec, tol=tol, reliable_update=rel, precond=True, graph_block=8)
    u = u.clone()
    u0, info0 = plan.solve(to_dev(b), precision=prec, tol=tol, reliable_update=rel, precond=True, graph_block=0)
    assert torch.equal(u, u0)
    assert [x.inner_iters for x in info] == [x.inner_iters for x in info0]
    chain = gpu_plan(w)
    _, info_c = chain.solve(to_dev(b), precision=prec, tol=tol, reliable_update=rel, precond=True)
    for c in range(w.batch):
        ref = O.solve_dense(oracle_problem(w), b[c], w.fixed, None, oracle_bonds(w))
        err = rel_err(u.cpu().numpy()[c], ref) if c else float(u[c].abs().max())
        log("fused PCG %s rel %d case %d: %d it (chain %d), residual %.2e, err %.2e" %
            (prec, rel, c, info[c].inner_iters, info_c[c].inner_iters, info[c].rel_residual, err))
        assert info[c].status == 0 and info[c].rel_residual <= tol
        assert err <= 100 * tol
        if prec == "fp64":
            assert abs(info[c].inner_iters - info_c[c].inner_iters) <= 3
