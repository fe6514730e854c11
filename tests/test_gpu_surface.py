"""Surface correction (Remark 3, eq. (scr)): products and Verlet runs with per-node
factors against the oracle's bond-by-bond sum with the same factors."""
import numpy as np
import pytest

import oracle as O
from paper_2301_11828_amd import workloads as W
from helpers import gpu_apply, gpu_plan, log, oracle_bonds, oracle_problem, rel_err, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-6


def _oracle_apply(w, u, nu):
    p = oracle_problem(w)
    br = oracle_bonds(w)
    return np.stack([O.apply(p, u[c], w.fixed, br, nu=nu) for c in range(u.shape[0])])


@pytest.mark.parametrize("team", ["block", "wave"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_surface_apply_matches_oracle(dim, prec, team):
    import torch
    if dim == 2:
        w = W.small(2, (41, 35), 3, seed=401, fixed="left", crack=True, batch=2)
    else:
        w = W.small(3, (13, 10, 9), 2, seed=402, fixed="bottom", batch=2)
    plan = gpu_plan(w)
    if team == "wave":
        plan.set_config(prec, team_x=1, slots_fwd=2, slots_inv=2, rows_per_wg=4)
    nu = np.random.default_rng(403).uniform(0.5, 2.0, w.N)
    plan.set_surface(nu)
    dt = torch.float64 if prec == "fp64" else torch.float32
    u = w.b if prec == "fp64" else w.b.astype(np.float32).astype(np.float64)
    f = gpu_apply(plan, to_dev(w.b, dt)).double().cpu().numpy()
    ref = _oracle_apply(w, u, nu if prec == "fp64" else nu.astype(np.float32).astype(np.float64))
    err = max(rel_err(f[c], ref[c]) for c in range(w.batch))
    plain = _oracle_apply(w, u, None)
    log("surface %dD %s %s: rel err %.2e (correction changes f by %.2e)" %
        (dim, prec, team, err, rel_err(ref, plain)))
    assert err <= (FP64_TOL if prec == "fp64" else FP32_TOL)
    assert rel_err(ref, plain) > 1e-3
    plan.set_surface(None)
    f0 = gpu_apply(plan, to_dev(w.b, dt)).double().cpu().numpy()
    assert max(rel_err(f0[c], plain[c]) for c in range(w.batch)) <= (FP64_TOL if prec == "fp64" else FP32_TOL)


@pytest.mark.parametrize("dim", [2, 3])
def test_surface_volume_factors_match_oracle(dim):
    w = W.small(2, (23, 19), 3, seed=404) if dim == 2 else W.small(3, (9, 8, 7), 2, seed=405)
    plan = gpu_plan(w)
    nu = plan.surface_volume_factors()
    ref = O.surface_volume_factors(oracle_problem(w))
    log("volume factors %dD: max |diff| %.1e, range [%.3f, %.3f]" % (dim, np.abs(nu - ref).max(), nu.min(), nu.max()))
    assert np.abs(nu - ref).max() <= 1e-14 * ref.max()
    plan.set_surface(nu)
    f = gpu_apply(plan, to_dev(w.b)).cpu().numpy()
    assert rel_err(f[0], O.apply(oracle_problem(w), w.b[0], w.fixed, None, nu=ref)) <= FP64_TOL


def test_surface_verlet_matches_oracle():
    w = W.small(2, (36, 30), 3, seed=406, fixed="left", crack=True)
    plan = gpu_plan(w)
    nu = plan.surface_volume_factors()
    plan.set_surface(nu)
    r = np.random.default_rng(407)
    u0 = np.where(w.fixed[None], 0.0, 1e-4 * r.standard_normal((1, w.dim, w.N)))
    v0 = np.where(w.fixed[None], 0.0, 1e-3 * r.standard_normal((1, w.dim, w.N)))
    dt, n = 0.2 * w.h / np.sqrt(w.alpha * (w.M * w.h) ** 2), 50
    u, v, b = to_dev(u0), to_dev(v0), to_dev(w.b)
    a = plan.vv_init(u, b)
    plan.vv_run(dt, n, u, v, a, b)
    uo, vo, ao, _ = O.vv(oracle_problem(w), u0[0], v0[0], w.b[0], dt, n, w.fixed, None, oracle_bonds(w), nu=nu)
    eu, ev = rel_err(u.cpu().numpy()[0], uo), rel_err(v.cpu().numpy()[0], vo)
    log("surface-corrected VV 50 steps: rel err u %.2e v %.2e" % (eu, ev))
    assert eu <= 1e-12 and ev <= 1e-12


def test_surface_rejects_cg_and_group_solve_and_keeps_group_apply():
    import torch
    import paper_2301_11828_amd as msb
    ws = [W.small(2, (21, 18), 3, seed=408, fixed="left"), W.small(2, (15, 12), 3, seed=409, fixed="all")]
    plans = [gpu_plan(w) for w in ws]
    nu = plans[0].surface_volume_factors()
    plans[0].set_surface(nu)
    with pytest.raises(msb.MsbError) as e:
        plans[0].solve(to_dev(ws[0].b))
    assert e.value.status == msb.MSB_EUNSUPPORTED
    grp = msb.PlanGroup(plans)
    with pytest.raises(msb.MsbError) as e:
        grp.solve([to_dev(w.b) for w in ws])
    assert e.value.status == msb.MSB_EUNSUPPORTED
    fs = grp.apply([to_dev(w.b) for w in ws], [torch.full((1, 2, w.N), float("nan"), dtype=torch.float64,
                                                          device="cuda") for w in ws])
    cfg = grp.get_config("fp64")
    for i, (w, pl) in enumerate(zip(ws, plans)):
        pl.set_config("fp64", **cfg)
        own = gpu_apply(pl, to_dev(w.b)).cpu().numpy()
        assert np.array_equal(fs[i].cpu().numpy(), own)
    err = rel_err(fs[0].cpu().numpy()[0], O.apply(oracle_problem(ws[0]), ws[0].b[0], ws[0].fixed, None, nu=nu))
    log("group member with surface correction: rel err %.2e" % err)
    assert err <= FP64_TOL
