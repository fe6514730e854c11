"""Dynamic model eq. (mat:e1) by velocity Verlet (Alg. 2) on the GPU vs the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2301_11828_amd import workloads as W
from helpers import gpu_plan, log, oracle_bonds, oracle_problem, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _setup(w, seed):
    r = np.random.default_rng(seed)
    u0 = 1e-4 * r.standard_normal((1, w.dim, w.N))
    v0 = 1e-3 * r.standard_normal((1, w.dim, w.N))
    return u0, v0


def _stable_dt(w):
    # explicit step well inside the stability limit of the bond stiffness
    return 0.2 * w.h / np.sqrt(w.alpha * (w.M * w.h) ** 2)


@pytest.mark.parametrize("dim", [2, 3])
def test_vv_fp64_matches_oracle(dim):
    if dim == 2:
        w = W.small(2, (36, 30), 3, seed=31, fixed="left", crack=True)
    else:
        w = W.small(3, (10, 9, 8), 2, seed=32, fixed="bottom")
    w.rho = 1.7
    u0, v0 = _setup(w, 1)
    g = np.where(w.fixed[None], 1e-4, 0.0) if w.fixed is not None else None
    if g is not None:
        u0 = np.where(w.fixed[None], g, u0)
        v0 = np.where(w.fixed[None], 0.0, v0)
    dt, n, every = _stable_dt(w), 60, 10
    plan = gpu_plan(w)
    u, v = to_dev(u0), to_dev(v0)
    b = to_dev(w.b)
    a = plan.vv_init(u, b)
    en = plan.vv_run(dt, n, u, v, a, b, g=None if g is None else to_dev(g), energy_every=every)
    p = oracle_problem(w)
    uo, vo, ao, eo = O.vv(p, u0[0], v0[0], w.b[0], dt, n, w.fixed, None if g is None else g[0],
                          oracle_bonds(w), energy_every=every)
    eu, ev, ea = rel_err(u.cpu().numpy()[0], uo), rel_err(v.cpu().numpy()[0], vo), rel_err(a.cpu().numpy()[0], ao)
    ee = np.abs(en - eo).max() / np.abs(eo).max()
    log("VV fp64 %dD %d steps: rel err u %.2e v %.2e a %.2e energy %.2e" % (dim, n, eu, ev, ea, ee))
    assert eu <= 1e-12 and ev <= 1e-12 and ea <= 1e-12 and ee <= 1e-11


def test_vv_fp32_error_stated():
    w = W.small(2, (64, 60), 4, seed=33, crack=True)
    u0, v0 = _setup(w, 2)
    dt, n = _stable_dt(w), 100
    import torch
    plan = gpu_plan(w)
    u, v, b = to_dev(u0, torch.float32), to_dev(v0, torch.float32), to_dev(w.b, torch.float32)
    a = plan.vv_init(u, b)
    plan.vv_run(dt, n, u, v, a, b)
    p = oracle_problem(w)
    uo, vo, _, _ = O.vv(p, u0[0].astype(np.float32).astype(np.float64), v0[0].astype(np.float32).astype(np.float64),
                        w.b[0].astype(np.float32).astype(np.float64), dt, n, None, None, oracle_bonds(w))
    eu, ev = rel_err(u.double().cpu().numpy()[0], uo), rel_err(v.double().cpu().numpy()[0], vo)
    log("VV fp32 vs FP64 oracle after %d steps: rel err u %.2e v %.2e" % (n, eu, ev))
    assert eu <= 1e-4 and ev <= 1e-4


def test_crack1024_fp32_short_run_vs_oracle():
    """Benchmark shape (1024^2, delta = 4h, pre-crack, opposing edge loads) for 20 steps, in
    the default launch configuration and in the benchmark's (the recorded tuning): FP32 state
    against the FP64 oracle trajectory; error stated."""
    import json
    import os
    import torch
    w = W.crack1024(steps=20)
    plan = gpu_plan(w)
    assert plan.n_bonds == 12654
    p = oracle_problem(w)
    uo, vo, _, _ = O.vv(p, np.zeros((2, w.N)), np.zeros((2, w.N)), w.b[0], w.dt, w.steps, None, None, oracle_bonds(w))
    rec = json.load(open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                                      "crack1024_tuning.json")))
    for name in ("default", "recorded"):
        if name == "recorded":
            plan.set_lengths(rec["padded"])
            plan.set_config("fp32", **rec["fp32"])
        u = torch.zeros((1, 2, w.N), dtype=torch.float32, device="cuda")
        v = torch.zeros_like(u)
        b = to_dev(w.b, torch.float32)
        a = plan.vv_init(u, b)
        plan.vv_run(w.dt, w.steps, u, v, a, b)
        eu, ev = rel_err(u.double().cpu().numpy()[0], uo), rel_err(v.double().cpu().numpy()[0], vo)
        log("crack1024 FP32 VV %d steps (%s configuration) vs FP64 oracle: rel err u %.2e v %.2e" %
            (w.steps, name, eu, ev))
        assert eu <= 1e-4 and ev <= 1e-4


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_crack1024_1000_steps_vs_oracle(prec):
    """The benchmark's dynamic run (1024^2, delta = 4h, 12,654 pre-broken bonds, opposing
    edge loads, 1000 Verlet steps, Alg. 2) at the recorded tuning, against the oracle's FP64
    trajectory sampled at 4096 seeded DOFs after 10, 100 and 1000 steps
    (tests/golden/crack1024_vv_oracle.npz, written by make_crack1024_vv.py from the oracle
    alone), and the energy every 10 steps against the oracle's.  The errors are stated;
    FP64 keeps the 1e-12 parity bar at every sample, FP32 state is bounded at 1e-4."""
    import json
    import os
    import torch
    here = os.path.dirname(os.path.abspath(__file__))
    g = np.load(os.path.join(here, "golden", "crack1024_vv_oracle.npz"))
    w = W.crack1024(steps=1000)
    assert abs(float(g["dt"]) - w.dt) <= 1e-15 * w.dt
    plan = gpu_plan(w)
    assert plan.n_bonds == int(g["n_bonds"])
    rec = json.load(open(os.path.join(os.path.dirname(here), "profiles", "crack1024_tuning.json")))
    plan.set_lengths(rec["padded"])
    plan.set_config("fp32", **rec["fp32"])
    dt_ = torch.float32 if prec == "fp32" else torch.float64
    u = torch.zeros((1, 2, w.N), dtype=dt_, device="cuda")
    v = torch.zeros_like(u)
    b = to_dev(w.b, dt_)
    a = plan.vv_init(u, b)
    idx = torch.from_numpy(g["idx"]).cuda()
    en, done = [], 0
    for n in (10, 100, 1000):
        en.append(plan.vv_run(w.dt, n - done, u, v, a, b, energy_every=10))
        done = n
        us = u.reshape(-1)[idx].double().cpu().numpy()
        vs = v.reshape(-1)[idx].double().cpu().numpy()
        eu, ev = rel_err(us, g["u%d" % n]), rel_err(vs, g["v%d" % n])
        log("crack1024 %s VV step %d vs FP64 oracle (4096 sampled DOFs): rel err u %.2e v %.2e" % (prec, n, eu, ev))
        assert eu <= (1e-4 if prec == "fp32" else 1e-12) and ev <= (1e-4 if prec == "fp32" else 1e-12)
    en = np.concatenate(en)
    parts = g["energy_parts"]
    eo = parts.sum(axis=1)
    scale = max(parts[:, 0].max(), parts[:, 1].max())     # max kinetic, max elastic over the run
    de = np.abs(en - eo).max() / scale
    drift = np.abs(eo - eo[0]).max() / scale
    log("crack1024 %s energy vs oracle: max |dE| / max(kinetic, elastic) %.2e; oracle's own energy drift over "
        "1000 steps %.2e of that scale (max kinetic %.3e, max elastic %.3e)" %
        (prec, de, drift, parts[:, 0].max(), parts[:, 1].max()))
    assert len(en) == 100 and de <= (1e-3 if prec == "fp32" else 1e-10)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("cfg", [None, dict(tile=16, tile_regs=1, tile_run=1), dict(tile=32, tile_regs=1, tile_run=1),
                                 dict(tile=24, tile_regs=0, tile_run=1)], ids=["chain", "t16r", "t32r", "t24"])
@pytest.mark.parametrize("nsteps", [1, 2, 7, 8])
def test_vv_steps_in_one_call_equal_single_steps(prec, cfg, nsteps):
    """After the first step of a call, each step's epilogue forms the next displacement
    (Alg. 2's update) into a second vector and the next product runs without a prologue
    pass: n steps in one call equal n calls of one step bit for bit (crack, constraints with
    prescribed g, energies), for odd and even n, on the chain and the tiled kernels."""
    import torch
    w = W.small(2, (41, 33), 3, seed=37, fixed="left", crack=True, batch=2)
    w.rho = 1.3
    u0, v0 = _setup(w, 3)
    g = np.where(w.fixed[None], 1e-4, 0.0)
    u0 = np.where(w.fixed[None], g, u0)
    dt = _stable_dt(w)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    plan = gpu_plan(w)
    if cfg:
        plan.set_config(prec, **cfg)
    b, gd = to_dev(w.b, dtype), to_dev(np.broadcast_to(g, (w.batch, 2, w.N)).copy(), dtype)
    res = []
    for one_call in (True, False):
        u, v = to_dev(np.broadcast_to(u0, (w.batch, 2, w.N)).copy(), dtype), to_dev(np.broadcast_to(v0, (w.batch, 2, w.N)).copy(), dtype)
        a = plan.vv_init(u, b)
        if one_call:
            en = plan.vv_run(dt, nsteps, u, v, a, b, g=gd, energy_every=1)
        else:
            en = np.concatenate([plan.vv_run(dt, 1, u, v, a, b, g=gd, energy_every=1) for _ in range(nsteps)])
        res.append((u.clone(), v.clone(), a.clone(), en))
    (u1, v1, a1, e1), (u2, v2, a2, e2) = res
    log("VV %s %s %d steps one call vs single steps: max |du| %.1e" % (prec, cfg, nsteps, float((u1 - u2).abs().max())))
    assert torch.equal(u1, u2) and torch.equal(v1, v2) and torch.equal(a1, a2)
    assert np.array_equal(e1, e2)
