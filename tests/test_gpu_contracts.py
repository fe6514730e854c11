"""Contracts of the C ABI beyond the arithmetic: argument validation of the broken-bond
list, the certified stop test of the static solvers, plan groups whose members change
their padded lengths, and an adjoint solve after the plan's operator changed."""
import numpy as np
import pytest

import oracle as O
from paper_2301_11828_amd import workloads as W
from helpers import gpu_apply, gpu_plan, log, oracle_bonds, oracle_problem, rel_err, to_dev

pytestmark = pytest.mark.gpu


def test_set_bonds_rejects_invalid_lists_and_keeps_the_old_one():
    """msb_plan_set_bonds returns MSB_EINVAL on an id outside the grid, p == q, a pair
    outside the horizon or a duplicate (either order), and leaves the broken set as it was."""
    import paper_2301_11828_amd as msb
    w = W.small(2, (21, 18), 3, seed=301, fixed="left", crack=True)
    plan = gpu_plan(w)
    u = to_dev(np.random.default_rng(302).standard_normal((1, 2, w.N)))
    f0 = gpu_apply(plan, u).cpu().numpy()
    good = plan.bonds()
    assert len(good) > 0
    nx = w.n[0]
    bad_lists = {
        "id out of range": [[0, 1], [w.N - 1, w.N]],
        "negative id": [[-1, 0]],
        "p == q": [[5, 5]],
        "outside the horizon (x)": [[0, 4]],
        "outside the horizon (|o|^2 > M^2)": [[0, 2 * nx + 3]],
        "duplicate": [[0, 1], [1, 0]],
    }
    for name, pairs in bad_lists.items():
        with pytest.raises(msb.MsbError) as ei:
            plan.set_bonds(np.array(pairs, dtype=np.int64))
        assert ei.value.status == msb.MSB_EINVAL, name
        log("set_bonds %s: %s" % (name, ei.value))
        assert np.array_equal(plan.bonds(), good), name
        assert np.array_equal(gpu_apply(plan, u).cpu().numpy(), f0), name
    # a valid list after the rejected ones still takes effect
    plan.set_bonds(None)
    ref = O.apply(oracle_problem(w), u.cpu().numpy()[0], w.fixed)
    assert rel_err(gpu_apply(plan, u).cpu().numpy()[0], ref) <= 1e-12


@pytest.mark.parametrize("prec,precond", [("fp64", False), ("fp64", True), ("fp32_refined", False),
                                          ("fp32_refined", True)])
def test_ok_status_means_certified_residual_within_tol(prec, precond):
    """MSB_OK promises ||b' - K u|| <= tol ||b'|| with the FP64 product: every case with
    status 0 must report a certified residual at or below tol (single plan and group)."""
    import paper_2301_11828_amd as msb
    ws = [W.small(2, (48, 40), 3, seed=303, fixed="left", batch=3),
          W.small(2, (33, 29), 3, seed=304, fixed="all", crack=True, batch=2)]
    for tol in (1e-10, 1e-12):
        for w in ws:
            plan = gpu_plan(w)
            _, info = plan.solve(to_dev(w.b), precision=prec, tol=tol, precond=precond, check=False)
            for c, i in enumerate(info):
                log("%s pre=%d tol %.0e %s case %d: status %d, residual %.3e, %d it" %
                    (prec, precond, tol, w.n, c, i.status, i.rel_residual, i.inner_iters))
                assert i.status != 0 or i.rel_residual <= tol
                assert i.status == 0
        plans = [gpu_plan(w) for w in ws]
        grp = msb.PlanGroup(plans)
        _, infos = grp.solve([to_dev(w.b) for w in ws], precision=prec, tol=tol, precond=precond, check=False)
        for m, ii in enumerate(infos):
            for c, i in enumerate(ii):
                assert i.status == 0 and i.rel_residual <= tol, (m, c, i)
        grp.close()


def test_group_follows_a_member_relayout():
    """A member whose padded lengths change after the group was built (msb_plan_set_lengths)
    is launched with its new tile counts and LDS sizes: the group product still matches the
    oracle, and so does a group solve."""
    import torch
    import paper_2301_11828_amd as msb
    ws = [W.small(2, (37, 30), 3, seed=305, fixed="left", crack=True, batch=2),
          W.small(2, (20, 17), 3, seed=306, fixed="all", batch=1)]
    plans = [gpu_plan(w) for w in ws]
    grp = msb.PlanGroup(plans)
    rng = np.random.default_rng(307)
    us = [rng.standard_normal((w.batch, 2, w.N)) for w in ws]
    for L in ((80, 72), (45, 36)):          # longer, then shorter than the default
        plans[0].set_lengths(L)
        fs = grp.apply([to_dev(u) for u in us])
        for w, u, f in zip(ws, us, fs):
            p, br = oracle_problem(w), oracle_bonds(w)
            for c in range(w.batch):
                err = rel_err(f.cpu().numpy()[c], O.apply(p, u[c], w.fixed, br))
                log("group after relayout L=%s member %s case %d: rel err %.2e" % (L, w.n, c, err))
                assert err <= 1e-12
    xs, infos = grp.solve([to_dev(w.b) for w in ws], precision="fp64", tol=1e-12)
    for w, x in zip(ws, xs):
        for c in range(w.batch):
            ref = O.solve_dense(oracle_problem(w), w.b[c], w.fixed, None, oracle_bonds(w))
            assert rel_err(x.cpu().numpy()[c], ref) <= 1e-9
    grp.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("group", [False, True])
def test_adjoint_after_the_plan_operator_changed(group):
    """The config-5 loss computes its target with perturbed coefficients on the same plan.
    When that happens between the forward solve and backward, the adjoint must still use
    the forward solve's coefficients: the gradient equals the oracle's."""
    import torch
    import paper_2301_11828_amd as msb
    rng = np.random.default_rng(308)
    a = tuple(rng.uniform(0.2, 1.0, size=4))
    w = W.small(2, (19, 16), 3, seed=309, fixed="all", crack=True, infl=a)
    ut = np.where(w.fixed, 0.0, 1e-3 * rng.standard_normal((2, w.N)))
    L, _, gb_ref, ga_ref = O.grad_dense(oracle_problem(w), w.b[0], ut, w.fixed, None, oracle_bonds(w))
    plan = gpu_plan(w)
    b = to_dev(w.b).requires_grad_(True)
    infl = torch.tensor(a, dtype=torch.float64, requires_grad=True)
    other = np.asarray(a) * 1.3
    if group:
        grp = msb.PlanGroup([plan])
        (u,) = msb.make_group_solve_function().apply(grp, "fp64", 1e-13, b, infl)
        grp.set_infl([other])
    else:
        u = msb.make_solve_function().apply(plan, b, infl, "fp64", 1e-13, False)
        plan.set_infl(other)
    loss = ((u - to_dev(ut[None])) ** 2).sum()
    loss.backward()
    eb = rel_err(b.grad.cpu().numpy()[0], gb_ref)
    ea = rel_err(infl.grad.numpy(), ga_ref)
    log("adjoint after set_infl (group=%d): rel err dL/db %.2e, dL/da %.2e" % (group, eb, ea))
    assert eb <= 1e-9 and ea <= 1e-9
    # the coefficients set after the forward solve are in force again
    assert np.array_equal(plan._infl_state[0], other)
    # a structural change cannot be undone: backward refuses it
    b2 = to_dev(w.b).requires_grad_(True)
    infl2 = torch.tensor(a, dtype=torch.float64, requires_grad=True)
    u2 = msb.make_solve_function().apply(plan, b2, infl2, "fp64", 1e-13, False)
    plan.set_constraints(None)
    with pytest.raises(RuntimeError):
        (u2 ** 2).sum().backward()
