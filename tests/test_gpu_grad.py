"""Adjoint gradient of a static solve w.r.t. influence coefficients and load, on the GPU,
vs the oracle's exact dense gradient (which the CPU suite pins to finite differences)."""
import numpy as np
import pytest

import oracle as O
from paper_2301_11828_amd import workloads as W
from helpers import gpu_plan, log, oracle_bonds, oracle_problem, rel_err, to_dev

pytestmark = pytest.mark.gpu


def test_apply_dinfl_matches_oracle():
    w = W.small(2, (25, 22), 3, seed=41, fixed="all", crack=True, infl=(0.3, 0.5, 0.1, 0.7))
    plan = gpu_plan(w)
    u = np.random.default_rng(3).standard_normal((1, 2, w.N))
    for k in range(4):
        f = plan.apply_dinfl(k, to_dev(u)).cpu().numpy()[0]
        e = np.zeros(k + 1)
        e[k] = 1.0
        ref = O.apply(oracle_problem(w, infl=tuple(e)), u[0], w.fixed, oracle_bonds(w))
        err = rel_err(f, ref)
        log("dA/da_%d rel err %.2e" % (k, err))
        assert err <= 1e-12


@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
def test_adjoint_gradient_matches_oracle(prec, precond):
    rng = np.random.default_rng(42)
    a = tuple(rng.uniform(0.2, 1.0, size=5))
    w = W.small(2, (20, 17), 3, seed=43, fixed="all", crack=True, infl=a)
    ut = np.where(w.fixed, 0.0, 1e-3 * rng.standard_normal((2, w.N)))
    L, uref, gb_ref, ga_ref = O.grad_dense(oracle_problem(w), w.b[0], ut, w.fixed, None, oracle_bonds(w))
    import torch
    import paper_2301_11828_amd as msb
    plan = gpu_plan(w)
    Solve = msb.make_solve_function()
    b = to_dev(w.b).requires_grad_(True)
    infl = torch.tensor(a, dtype=torch.float64, requires_grad=True)
    u = Solve.apply(plan, b, infl, prec, 1e-13, precond)
    loss = ((u - to_dev(ut[None])) ** 2).sum()
    loss.backward()
    eb = rel_err(b.grad.cpu().numpy()[0], gb_ref)
    ea = rel_err(infl.grad.numpy(), ga_ref)
    log("adjoint %s precond=%d: loss %.6e (oracle %.6e), rel err dL/db %.2e, dL/da %.2e" %
        (prec, precond, loss.item(), L, eb, ea))
    assert abs(loss.item() - L) <= 1e-8 * L
    assert eb <= 1e-9 and ea <= 1e-9


def test_per_case_influence_batch():
    rng = np.random.default_rng(44)
    a = rng.uniform(0.1, 1.0, size=(3, 4))
    w = W.small(2, (18, 16), 3, seed=45, fixed="all", batch=3, infl=tuple(a[0]))
    import paper_2301_11828_amd as msb
    plan = gpu_plan(w)
    plan.set_infl(a, per_case=True)
    u, info = plan.solve(to_dev(w.b), precision="fp64", tol=1e-13)
    uu = u.cpu().numpy()
    for c in range(3):
        p = oracle_problem(w, infl=tuple(a[c]))
        ref = O.solve_dense(p, w.b[c], w.fixed)
        err = rel_err(uu[c], ref)
        log("per-case infl case %d rel err %.2e" % (c, err))
        assert err <= 1e-11
    wv = np.where(w.fixed[None], 0.0, rng.standard_normal((3, 2, w.N)))
    ga = plan.grad_infl(u, to_dev(wv))
    for c in range(3):
        for k in range(4):
            e = np.zeros(k + 1)
            e[k] = 1.0
            Aku = O.force(oracle_problem(w, infl=tuple(e)), uu[c])
            ref = (wv[c] * Aku)[~w.fixed].sum()
            assert ga[c, k] == pytest.approx(ref, rel=1e-11, abs=1e-12 * abs(ref) + 1e-300)


def _plates64_group(tuning_path=None):
    """The benchmark's 64-plate batch as one plan group, at the recorded group tuning."""
    import json
    import os
    import paper_2301_11828_amd as msb
    ws = W.plates64()
    plans = []
    for w in ws:
        pl = msb.Plan(w.n, w.h, w.M, w.alpha, infl=w.infl, batch=1)
        pl.set_constraints(w.fixed)
        plans.append(pl)
    grp = msb.PlanGroup(plans)
    path = tuning_path or os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                                       "plates64_tuning.json")
    if os.path.exists(path):
        rec = json.load(open(path))
        grp.set_config("fp64", **rec["fp64"])
        grp.set_config("fp32", **rec["fp32"])
    return ws, plans, grp


def _oracle_rows():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plates64_grad_oracle.txt")
    rows = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows[int(f[0])] = dict(size=int(f[1]), L=float(f[2]), ga=np.array([float(x) for x in f[3:11]]))
    return rows


@pytest.mark.parametrize("tol", [1e-11, 1e-10])
def test_plates64_member_gradients_vs_oracle_cg(tol):
    """The benchmark's pipeline (target solve with the perturbed coefficients, forward
    solve, loss, group adjoint solve, dL/da) on the 64-plate group at its recorded tuning,
    FP32-refined: the first member of every size (64^2 ... 384^2) against the oracle's CG
    gradient (tests/golden/plates64_grad_oracle.txt, written by make_plates64_grad.py from
    the oracle alone; its solves to 1e-13, the adjoint's true residual 1e-13 ... 8e-12).  Error
    bound from the solve tolerances: the gradient error is about kappa (tol + 1e-11) with
    kappa <= 2e4 at 384^2 (1e-11 is near the FP64 residual floor eps kappa of that plate)."""
    import torch
    import paper_2301_11828_amd as msb
    rows = _oracle_rows()
    ws, plans, grp = _plates64_group()
    bs = [torch.from_numpy(w.b).cuda().requires_grad_(True) for w in ws]
    as_ = [torch.tensor(w.infl, dtype=torch.float64, requires_grad=True) for w in ws]
    grp.set_infl([np.asarray(w.extra["infl_target"]) for w in ws])
    uts, infos = grp.solve([b.detach() for b in bs], precision="fp32_refined", tol=tol)
    us = msb.make_group_solve_function().apply(grp, "fp32_refined", tol, *bs, *as_)
    losses = [((u - ut) ** 2).sum() for u, ut in zip(us, uts)]
    sum(losses).backward()
    worst = 0.0
    for i, r in sorted(rows.items()):
        g = as_[i].grad.numpy()
        err = np.abs(g - r["ga"]).max() / np.abs(r["ga"]).max()
        el = abs(losses[i].item() - r["L"]) / r["L"]
        log("plates64[%d] %d^2 tol %.0e: dL/da max rel err %.2e, loss rel err %.2e" % (i, r["size"], tol, err, el))
        worst = max(worst, err)
        assert err <= (1e-6 if tol <= 1e-11 else 1e-5) and el <= (1e-6 if tol <= 1e-11 else 1e-5)
    assert len(rows) == 5
    grp.close()
