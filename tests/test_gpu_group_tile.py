"""Plan groups with the tiled 2D product: one launch of the overlap-save block kernel over
the blocks of every member (register-resident and LDS frames), in products, plain and
preconditioned group CG, refinement and the adjoint gradient, against each member's own
tiled product, the oracle's bond sums (eq. (mat:f1)) and its dense Cholesky solve of
eq. (mat:e2)."""
import numpy as np
import pytest

import oracle as O
from paper_2301_11828_amd import workloads as W
from helpers import gpu_plan, log, oracle_bonds, oracle_problem, rel_err, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-6

# frame 16/32/64 register kernels; LDS frames of 24 (composite-free radices) and 40 (radix cap 8)
TILED = [dict(tile=16, tile_regs=1, tile_run=1), dict(tile=32, tile_regs=1, tile_run=1),
         dict(tile=64, tile_regs=1, tile_run=1), dict(tile=24, tile_regs=0, tile_run=1, threads_tile=256),
         dict(tile=40, tile_regs=0, tile_run=1, threads_tile=128, max_radix=8)]


def _members():
    # different sizes, a crack, several cases, influence coefficients; the last member has
    # more blocks per case than grid rows at frame 16 (12 x 1 blocks, 6 rows)
    return [W.small(2, (37, 30), 3, seed=701, fixed="left", crack=True, batch=2),
            W.small(2, (20, 17), 3, seed=702, fixed="all", batch=1, infl=(0.4, 0.3, 0.2)),
            W.small(2, (64, 50), 3, seed=703, fixed="mixed", batch=3),
            W.small(2, (117, 6), 3, seed=704, fixed="left", batch=1)]


def _oracle_apply(w, u):
    p = oracle_problem(w)
    br = oracle_bonds(w)
    return np.stack([O.apply(p, u[c], w.fixed, br) for c in range(u.shape[0])])


def _key(cfg):
    return "t%d%s" % (cfg["tile"], "r" if cfg["tile_regs"] else "")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("cfg", TILED, ids=_key)
def test_group_tiled_apply_equals_members_and_oracle(prec, cfg):
    import torch
    import paper_2301_11828_amd as msb
    ws = _members()
    plans = [gpu_plan(w) for w in ws]
    grp = msb.PlanGroup(plans)
    grp.set_config(prec, **cfg)
    got = grp.get_config(prec)
    assert all(got[k] == v for k, v in cfg.items())
    dt = torch.float64 if prec == "fp64" else torch.float32
    us = [to_dev(w.b, dt) for w in ws]
    fs = [f.double().cpu().numpy() for f in grp.apply(us, [torch.full_like(u, float("nan")) for u in us])]
    for i, (w, p) in enumerate(zip(ws, plans)):
        p.set_config(prec, **got)   # the member alone, same block kernel: identical arithmetic
        own = p.apply(us[i], torch.full_like(us[i], float("nan"))).double().cpu().numpy()
        assert np.array_equal(fs[i], own), "member %d differs from its own tiled product" % i
        u = w.b if prec == "fp64" else w.b.astype(np.float32).astype(np.float64)
        err = rel_err(fs[i], _oracle_apply(w, u))
        log("tiled group %s %s member %d (%s x%d) rel err %.2e" % (_key(cfg), prec, i, "x".join(map(str, w.n)),
                                                                w.batch, err))
        assert err <= (FP64_TOL if prec == "fp64" else FP32_TOL)


@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("cfg", [TILED[0], TILED[3]], ids=_key)
def test_group_tiled_solve_matches_cholesky(prec, precond, cfg):
    """Group CG with the tiled product (a transform-free x pass carries the CG update, the
    block kernel forms q = K p and its partial sums; the preconditioners' chains stay
    untiled), with lifts, against each member's dense Cholesky solve."""
    import paper_2301_11828_amd as msb
    ws = [W.small(2, (25, 22), 3, seed=711, fixed="left", crack=True, batch=2),
          W.small(2, (14, 18), 3, seed=712, fixed="all", batch=1, infl=(0.5, 0.2)),
          W.small(2, (117, 6), 3, seed=713, fixed="bottom", batch=2)]   # 12 blocks per case, 6 rows
    rng = np.random.default_rng(714)
    gs = [np.where(w.fixed[None], 1e-2 * rng.standard_normal((w.batch, 2, w.N)), 0.0) for w in ws]
    gs[1] = None
    plans = [gpu_plan(w) for w in ws]
    grp = msb.PlanGroup(plans)
    for f in ("fp64", "fp32"):
        grp.set_config(f, **cfg)
    us, infos = grp.solve([to_dev(w.b) for w in ws], [None if g is None else to_dev(g) for g in gs],
                          precision=prec, tol=1e-13, precond=precond)
    for i, w in enumerate(ws):
        uu = us[i].cpu().numpy()
        for c in range(w.batch):
            ref = O.solve_dense(oracle_problem(w), w.b[c], w.fixed, None if gs[i] is None else gs[i][c], oracle_bonds(w))
            err = rel_err(uu[c], ref)
            log("tiled group solve %s %s precond=%d member %d case %d: %d outer %d inner, residual %.2e, rel err %.2e"
                % (_key(cfg), prec, precond, i, c, infos[i][c].outer_iters, infos[i][c].inner_iters,
                   infos[i][c].rel_residual, err))
            assert infos[i][c].status == 0
            assert err <= (1e-11 if prec == "fp64" else 1e-10)


def test_group_tiled_graph_blocks_equal_plain():
    import paper_2301_11828_amd as msb
    ws = [W.small(2, (40, 33), 3, seed=721, fixed="left", batch=2), W.small(2, (17, 26), 3, seed=722, fixed="all")]
    plans = [gpu_plan(w) for w in ws]
    grp = msb.PlanGroup(plans)
    grp.set_config("fp64", **TILED[0])
    bs = [to_dev(w.b) for w in ws]
    for precond in (False, True):
        a, ia = grp.solve(bs, precision="fp64", tol=1e-12, precond=precond)
        b, ib = grp.solve(bs, precision="fp64", tol=1e-12, graph_block=8, precond=precond)
        for i in range(2):
            assert np.array_equal(a[i].cpu().numpy(), b[i].cpu().numpy())
            assert [x.inner_iters for x in ia[i]] == [x.inner_iters for x in ib[i]]


def test_group_tiled_adjoint_gradient_matches_oracle():
    """dL/db and dL/da through the tiled group solve and its adjoint against the oracle's
    exact dense gradient of each member."""
    import torch
    import paper_2301_11828_amd as msb
    rng = np.random.default_rng(731)
    ws, uts, refs = [], [], []
    for i, (n, crack) in enumerate((((20, 17), True), ((15, 12), False), ((24, 9), False))):
        a = tuple(rng.uniform(0.2, 1.0, size=4))
        w = W.small(2, n, 3, seed=732 + i, fixed="all", crack=crack, infl=a)
        ut = np.where(w.fixed, 0.0, 1e-3 * rng.standard_normal((2, w.N)))
        refs.append(O.grad_dense(oracle_problem(w), w.b[0], ut, w.fixed, None, oracle_bonds(w)))
        ws.append(w)
        uts.append(ut)
    plans = [gpu_plan(w) for w in ws]
    grp = msb.PlanGroup(plans, precond=True)
    grp.set_config("fp64", **TILED[0])
    GSolve = msb.make_group_solve_function()
    bs = [to_dev(w.b).requires_grad_(True) for w in ws]
    infls = [torch.tensor(w.infl, dtype=torch.float64, requires_grad=True) for w in ws]
    us = GSolve.apply(grp, "fp64", 1e-13, *bs, *infls)
    loss = sum(((u - to_dev(ut[None])) ** 2).sum() for u, ut in zip(us, uts))
    loss.backward()
    for i, (L, uref, gb_ref, ga_ref) in enumerate(refs):
        eb = rel_err(bs[i].grad.cpu().numpy()[0], gb_ref)
        ea = rel_err(infls[i].grad.numpy(), ga_ref)
        log("tiled group adjoint member %d: rel err dL/db %.2e, dL/da %.2e" % (i, eb, ea))
        assert eb <= 1e-9 and ea <= 1e-9


def test_group_tiled_configuration_rules():
    """Runs of blocks are refused for groups (a run would cross members), so is a 3D tiled
    group; a member's tiled configuration carries over at one block per workgroup; new
    coefficients (which drop the members' frame spectra) leave the group's products right."""
    import paper_2301_11828_amd as msb
    ws = _members()[:3]
    plans = [gpu_plan(w) for w in ws]
    grp = msb.PlanGroup(plans)
    with pytest.raises(msb.MsbError) as e:
        grp.set_config("fp64", tile=16, tile_regs=1, tile_run=2)
    assert e.value.status == msb.MSB_EINVAL
    assert grp.get_config("fp64")["tile"] == 0
    p3 = [gpu_plan(W.small(3, (10, 9, 8), 2, seed=741)), gpu_plan(W.small(3, (7, 8, 6), 2, seed=742))]
    g3 = msb.PlanGroup(p3)
    with pytest.raises(msb.MsbError):
        g3.set_config("fp64", tile=16)
    g3.close()
    big = max(range(len(ws)), key=lambda i: ws[i].N * ws[i].batch)
    plans[big].set_config("fp64", tile=32, tile_regs=1, tile_run=4)
    g2 = msb.PlanGroup(plans)
    c2 = g2.get_config("fp64")
    assert (c2["tile"], c2["tile_regs"], c2["tile_run"]) == (32, 1, 1)
    rng = np.random.default_rng(743)
    coeffs = [rng.uniform(0.2, 1.0, 4) for _ in ws]
    g2.set_infl(coeffs)
    fs = g2.apply([to_dev(w.b) for w in ws])
    for i, w in enumerate(ws):
        ref = np.stack([O.apply(oracle_problem(w, infl=tuple(coeffs[i])), w.b[c], w.fixed, oracle_bonds(w))
                        for c in range(w.batch)])
        err = rel_err(fs[i].cpu().numpy(), ref)
        log("tiled group after set_infl member %d rel err %.2e" % (i, err))
        assert err <= FP64_TOL
    g2.close()
    grp.close()


@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("cfg", [None, TILED[0]], ids=["chain", "t16r"])
def test_group_reliable_update_matches_cholesky(precond, cfg):
    """Group refinement that keeps every member's search direction across the FP64 residual
    replacements (plain and preconditioned, chain and tiled products) against each member's
    dense Cholesky solve; certified residual <= tol."""
    import paper_2301_11828_amd as msb
    ws = [W.small(2, (25, 22), 3, seed=751, fixed="left", crack=True, batch=2),
          W.small(2, (14, 18), 3, seed=752, fixed="all", batch=1, infl=(0.5, 0.2)),
          W.small(2, (117, 6), 3, seed=753, fixed="bottom", batch=2)]
    rng = np.random.default_rng(754)
    gs = [np.where(w.fixed[None], 1e-2 * rng.standard_normal((w.batch, 2, w.N)), 0.0) for w in ws]
    plans = [gpu_plan(w) for w in ws]
    grp = msb.PlanGroup(plans)
    if cfg:
        for f in ("fp64", "fp32"):
            grp.set_config(f, **cfg)
    tol = 1e-11
    us, infos = grp.solve([to_dev(w.b) for w in ws], [to_dev(g) for g in gs], precision="fp32_refined", tol=tol,
                          precond=precond, reliable_update=1, graph_block=8)
    _, infos_r = grp.solve([to_dev(w.b) for w in ws], [to_dev(g) for g in gs], precision="fp32_refined", tol=tol,
                           precond=precond)
    for i, w in enumerate(ws):
        uu = us[i].cpu().numpy()
        for c in range(w.batch):
            ref = O.solve_dense(oracle_problem(w), w.b[c], w.fixed, gs[i][c], oracle_bonds(w))
            err = rel_err(uu[c], ref)
            log("group reliable %s precond=%d member %d case %d: %d outer %d inner (restarted %d), residual %.2e, "
                "rel err %.2e" % ("chain" if cfg is None else "t16r", precond, i, c, infos[i][c].outer_iters,
                                  infos[i][c].inner_iters, infos_r[i][c].inner_iters, infos[i][c].rel_residual, err))
            assert infos[i][c].status == 0 and infos[i][c].rel_residual <= tol
            assert err <= 1e-9
