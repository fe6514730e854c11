"""The tiled single-pass 2D product (launch configuration `tile` > 0): overlap-save
blocks of tile - 2M nodes, each transformed in LDS with its M-wide halo, multiplied by the
spectra of the generating array wrapped to tile x tile (Alg. 3 on the patch) and
transformed back, with D^e, D^f, the surface correction, the mask and the fused solver
epilogues applied in the same launch.  Checked against the oracle's bond-by-bond sum
(eq. (mat:f1)), dense Cholesky (eq. (mat:e2)), the oracle's Verlet trajectory (Alg. 2),
its relaxation map (Alg. 1) and its exact adjoint gradient."""
import numpy as np
import pytest

import oracle as O
from paper_2301_11828_amd import workloads as W
from helpers import gpu_apply, gpu_plan, log, oracle_bonds, oracle_problem, rel_err, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-6


def _oracle_apply(w, u, nu=None):
    p = oracle_problem(w)
    br = oracle_bonds(w)
    return np.stack([O.apply(p, u[c], w.fixed, br, nu=nu) for c in range(u.shape[0])])


def _tiled(plan, tl, prec="fp64", threads=256, radix=None):
    kw = dict(tile=tl, threads_tile=threads)
    if radix:
        kw["max_radix"] = radix
    plan.set_config(prec, **kw)
    assert plan.get_config(prec)["tile"] == tl


CASES = [
    # n, M, fixed, crack, batch, tile -- several blocks per axis with ragged edges, blocks
    # larger than the grid, a one-column grid, per-DOF constraints
    ((37, 29), 3, "none", False, 1, 16),
    ((64, 50), 4, "left", True, 2, 20),
    ((33, 70), 2, "all", True, 1, 24),
    ((41, 23), 3, "mixed", False, 1, 32),
    ((1, 17), 2, "none", False, 1, 12),
    ((5, 3), 4, "none", False, 3, 16),
    ((90, 77), 3, "left", True, 2, 40),
    ((130, 61), 3, "all", False, 1, 64),
    ((70, 70), 3, "bottom", True, 1, 48),
    ((52, 45), 1, "mixed", True, 1, 10),
]


def _cid(c):
    return "%s-M%d-%s%s-b%d-t%d" % ("x".join(map(str, c[0])), c[1], c[2], "-crack" if c[3] else "", c[4], c[5])


@pytest.mark.parametrize("case", CASES, ids=_cid)
def test_tiled_apply_fp64_matches_oracle(case):
    n, M, fixed, crack, batch, tl = case
    log("tiled apply fp64 %s" % (case,))
    w = W.small(2, n, M, seed=500 + CASES.index(case), fixed=fixed, crack=crack, batch=batch)
    plan = gpu_plan(w)
    _tiled(plan, tl)
    f = gpu_apply(plan, to_dev(w.b)).cpu().numpy()
    ref = _oracle_apply(w, w.b)
    for c in range(batch):
        err = rel_err(f[c], ref[c])
        log("  case %d rel err %.3e" % (c, err))
        assert err <= FP64_TOL
    if w.fixed is not None:
        assert np.all(f[:, w.fixed] == 0.0)


@pytest.mark.parametrize("radix", [8, 16])
@pytest.mark.parametrize("threads", [64, 256, 512])
def test_tiled_launch_shapes_agree(threads, radix):
    """Every frame length the autotuner tries, at several workgroup sizes and radix caps,
    against the oracle and against the global chain."""
    w = W.small(2, (83, 67), 3, seed=520, fixed="left", crack=True, batch=2)
    plan = gpu_plan(w)
    u = to_dev(w.b)
    chain = gpu_apply(plan, u).cpu().numpy()
    ref = _oracle_apply(w, w.b)
    for tl in (16, 20, 24, 30, 32, 36, 40, 48, 60, 64):
        _tiled(plan, tl, threads=threads, radix=radix)
        f = gpu_apply(plan, u).cpu().numpy()
        e1 = max(rel_err(f[c], ref[c]) for c in range(2))
        e2 = max(rel_err(f[c], chain[c]) for c in range(2))
        log("tile %d threads %d radix %d: vs oracle %.2e, vs chain %.2e" % (tl, threads, radix, e1, e2))
        assert e1 <= FP64_TOL and e2 <= FP64_TOL


@pytest.mark.parametrize("tl", [24, 40, 64, 96])
def test_tiled_apply_fp32_error_bounded(tl):
    import torch
    w = W.small(2, (75, 66), 4, seed=521, fixed="left", crack=True, batch=2)
    plan = gpu_plan(w)
    _tiled(plan, tl, "fp32")
    f = gpu_apply(plan, to_dev(w.b, torch.float32)).double().cpu().numpy()
    ref = _oracle_apply(w, w.b.astype(np.float32).astype(np.float64))
    err = max(rel_err(f[c], ref[c]) for c in range(2))
    log("tiled fp32 tile %d rel err vs FP64 oracle %.3e" % (tl, err))
    assert err <= FP32_TOL


def test_tiled_exhaustive_unit_vectors_reproduce_dense_A():
    """Every column of A on a 9x9 grid with a crack and mixed constraints, frame 12 (blocks
    of 6 nodes: the grid spans two blocks per axis)."""
    w = W.small(2, (9, 9), 3, seed=3, fixed="mixed", crack=True)
    A = O.assemble_dense(oracle_problem(w), oracle_bonds(w))
    D = 2 * w.N
    plan = gpu_plan(w, batch=D)
    _tiled(plan, 12)
    U = np.eye(D).reshape(D, 2, w.N)
    F = gpu_apply(plan, to_dev(U)).cpu().numpy().reshape(D, D)
    ref = A.T.copy()
    ref[:, w.fixed.reshape(-1)] = 0.0
    err = np.abs(F - ref).max() / np.abs(A).max()
    log("tiled exhaustive max abs err / max|A| = %.3e" % err)
    assert err <= 1e-14 * 50


def test_tiled_batch_equals_single_bitwise_and_deterministic():
    w = W.small(2, (45, 38), 3, seed=11, fixed="left", crack=True, batch=3)
    pb = gpu_plan(w)
    _tiled(pb, 24)
    fb = pb.apply(to_dev(w.b)).cpu().numpy()
    assert np.array_equal(fb, pb.apply(to_dev(w.b)).cpu().numpy())
    w1 = W.small(2, (45, 38), 3, seed=11, fixed="left", crack=True, batch=1)
    p1 = gpu_plan(w1)
    _tiled(p1, 24)
    for c in range(3):
        assert np.array_equal(p1.apply(to_dev(w.b[c:c + 1])).cpu().numpy()[0], fb[c])


def test_tiled_per_case_coefficients_and_derivative_operators():
    """Per-case influence coefficients (one frame spectrum per case) and the a_k-derivative
    operators of the adjoint run tiled like the operator itself."""
    rng = np.random.default_rng(522)
    a = rng.uniform(0.1, 1.0, size=(3, 4))
    w = W.small(2, (47, 40), 3, seed=523, fixed="all", crack=True, batch=3, infl=tuple(a[0]))
    plan = gpu_plan(w)
    plan.set_infl(a, per_case=True)
    _tiled(plan, 32)
    u = rng.standard_normal((3, 2, w.N))
    f = gpu_apply(plan, to_dev(u)).cpu().numpy()
    for c in range(3):
        ref = O.apply(oracle_problem(w, infl=tuple(a[c])), u[c], w.fixed, oracle_bonds(w))
        assert rel_err(f[c], ref) <= FP64_TOL
    for k in range(4):
        fk = plan.apply_dinfl(k, to_dev(u)).cpu().numpy()
        e = np.zeros(k + 1)
        e[k] = 1.0
        for c in range(3):
            ref = O.apply(oracle_problem(w, infl=tuple(e)), u[c], w.fixed, oracle_bonds(w))
            assert rel_err(fk[c], ref) <= FP64_TOL
    # new coefficients rebuild the frame spectra
    plan.set_infl(a[::-1].copy(), per_case=True)
    f2 = gpu_apply(plan, to_dev(u)).cpu().numpy()
    for c in range(3):
        ref = O.apply(oracle_problem(w, infl=tuple(a[2 - c])), u[c], w.fixed, oracle_bonds(w))
        assert rel_err(f2[c], ref) <= FP64_TOL


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tiled_surface_correction(prec):
    import torch
    w = W.small(2, (58, 49), 3, seed=524, fixed="left", crack=True, batch=2)
    plan = gpu_plan(w)
    _tiled(plan, 20, prec)
    nu = np.random.default_rng(525).uniform(0.5, 2.0, w.N)
    plan.set_surface(nu)
    dt = torch.float64 if prec == "fp64" else torch.float32
    u = w.b if prec == "fp64" else w.b.astype(np.float32).astype(np.float64)
    f = gpu_apply(plan, to_dev(w.b, dt)).double().cpu().numpy()
    ref = _oracle_apply(w, u, nu if prec == "fp64" else nu.astype(np.float32).astype(np.float64))
    err = max(rel_err(f[c], ref[c]) for c in range(2))
    log("tiled surface %s rel err %.2e" % (prec, err))
    assert err <= (FP64_TOL if prec == "fp64" else FP32_TOL)


@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
def test_tiled_solves_match_cholesky(prec, precond):
    """CG (fused prologue as its own pass, then the tiled product with the CG epilogue),
    refined FP32 and the preconditioned solver (its preconditioner keeps the chain) reach
    the dense solution, with nonzero prescribed displacements and a crack."""
    w = W.small(2, (44, 37), 3, seed=526, fixed="all", crack=True, batch=2)
    g = np.where(w.fixed[None], np.random.default_rng(527).standard_normal((2, 2, w.N)), 0.0)
    plan = gpu_plan(w)
    _tiled(plan, 24, "fp64")
    _tiled(plan, 32, "fp32")
    u, info = plan.solve(to_dev(w.b), g=to_dev(g), precision=prec, tol=1e-13, precond=precond)
    for c in range(2):
        ref = O.solve_dense(oracle_problem(w), w.b[c], w.fixed, g[c], oracle_bonds(w))
        err = rel_err(u.cpu().numpy()[c], ref)
        log("tiled %s precond=%d case %d: %d it, residual %.2e, rel err %.2e" %
            (prec, precond, c, info[c].inner_iters, info[c].rel_residual, err))
        assert info[c].status == 0 and info[c].rel_residual <= 1e-13
        assert err <= (1e-11 if prec == "fp64" else 1e-10)


def test_tiled_cg_graph_blocks_equal_plain_launches():
    w = W.small(2, (60, 52), 3, seed=528, fixed="left", batch=2)
    plan = gpu_plan(w)
    _tiled(plan, 32)
    u1, i1 = plan.solve(to_dev(w.b), precision="fp64", tol=1e-11, graph_block=0)
    u2, i2 = plan.solve(to_dev(w.b), precision="fp64", tol=1e-11, graph_block=16)
    assert np.array_equal(u1.cpu().numpy(), u2.cpu().numpy())
    assert [i.inner_iters for i in i1] == [i.inner_iters for i in i2]


def test_tiled_verlet_matches_oracle():
    w = W.small(2, (49, 41), 3, seed=529, fixed="left", crack=True)
    w.rho = 1.3
    r = np.random.default_rng(530)
    u0 = 1e-4 * r.standard_normal((1, 2, w.N))
    v0 = 1e-3 * r.standard_normal((1, 2, w.N))
    g = np.where(w.fixed[None], 1e-4, 0.0)
    u0 = np.where(w.fixed[None], g, u0)
    v0 = np.where(w.fixed[None], 0.0, v0)
    dt, n, every = 0.2 * w.h / np.sqrt(w.alpha * (w.M * w.h) ** 2), 50, 10
    plan = gpu_plan(w)
    _tiled(plan, 27)   # odd frame length (row pitch = frame)
    u, v = to_dev(u0), to_dev(v0)
    b = to_dev(w.b)
    a = plan.vv_init(u, b)
    en = plan.vv_run(dt, n, u, v, a, b, g=to_dev(g), energy_every=every)
    uo, vo, ao, eo = O.vv(oracle_problem(w), u0[0], v0[0], w.b[0], dt, n, w.fixed, g[0], oracle_bonds(w),
                          energy_every=every)
    eu, ev, ea = rel_err(u.cpu().numpy()[0], uo), rel_err(v.cpu().numpy()[0], vo), rel_err(a.cpu().numpy()[0], ao)
    ee = np.abs(en - eo).max() / np.abs(eo).max()
    log("tiled VV fp64: rel err u %.2e v %.2e a %.2e energy %.2e" % (eu, ev, ea, ee))
    assert eu <= 1e-12 and ev <= 1e-12 and ea <= 1e-12 and ee <= 1e-11


def test_tiled_relaxation_updates_match_oracle():
    """Each adaptive-relaxation update (prologue pass, then the tiled product with the
    ADR epilogue and its damping partials) against the oracle's one-step map."""
    import torch
    w = W.small(2, (34, 29), 3, seed=531, fixed="left", crack=True)
    plan = gpu_plan(w)
    _tiled(plan, 16)
    u = torch.zeros((1, 2, w.N), dtype=torch.float64, device="cuda")
    v = torch.full_like(u, float("nan"))
    F = torch.full_like(u, float("nan"))
    b = to_dev(w.b)
    plan.adr_run(0, u, v, F, b, restart=True)
    hist = [(u.cpu().numpy(), None, F.cpu().numpy())]
    for k in range(6):
        plan.adr_run(1, u, v, F, b, restart=False)
        hist.append((u.cpu().numpy(), v.cpu().numpy(), F.cpu().numpy()))
    p = oracle_problem(w)
    D = O.adr_density(p, oracle_bonds(w))
    worst = 0.0
    for k in range(1, 7):
        u0, v0, F0 = hist[k - 1]
        Fp = hist[k - 2][2][0] if k >= 2 else None
        uo, vo, Fo, _ = O.adr_step(p, u0[0], None if v0 is None else v0[0], F0[0], Fp, w.b[0], D, w.fixed, None,
                                   oracle_bonds(w))
        u1, v1, F1 = hist[k]
        worst = max(worst, rel_err(u1[0], uo), rel_err(v1[0], vo), rel_err(F1[0], Fo))
    log("tiled ADR worst per-update rel err %.2e" % worst)
    assert worst <= 2e-13


def test_tiled_adjoint_gradient_matches_oracle():
    import torch
    import paper_2301_11828_amd as msb
    rng = np.random.default_rng(532)
    a = tuple(rng.uniform(0.2, 1.0, size=5))
    w = W.small(2, (22, 19), 3, seed=533, fixed="all", crack=True, infl=a)
    ut = np.where(w.fixed, 0.0, 1e-3 * rng.standard_normal((2, w.N)))
    L, _, gb_ref, ga_ref = O.grad_dense(oracle_problem(w), w.b[0], ut, w.fixed, None, oracle_bonds(w))
    plan = gpu_plan(w)
    _tiled(plan, 16)
    b = to_dev(w.b).requires_grad_(True)
    infl = torch.tensor(a, dtype=torch.float64, requires_grad=True)
    u = msb.make_solve_function().apply(plan, b, infl, "fp64", 1e-13, False)
    loss = ((u - to_dev(ut[None])) ** 2).sum()
    loss.backward()
    eb = rel_err(b.grad.cpu().numpy()[0], gb_ref)
    ea = rel_err(infl.grad.numpy(), ga_ref)
    log("tiled adjoint: rel err dL/db %.2e, dL/da %.2e" % (eb, ea))
    assert eb <= 1e-9 and ea <= 1e-9


def test_tiled_profile_and_graph_replay():
    """The tiled product is one kernel (profile reports one pass), and replays of a
    captured hipGraph of products equal the eager product bit for bit on every replay."""
    import torch
    w = W.small(2, (100, 90), 3, seed=534, fixed="left")
    plan = gpu_plan(w)
    _tiled(plan, 40)
    u = to_dev(w.b)
    ms = plan.profile_apply(u, nrep=5)
    assert len(ms) == 1 and ms[0] > 0
    eager = plan.apply(u).clone()
    f = torch.empty_like(u)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr, stream=s):
        for _ in range(3):
            plan.apply(u, f)
    torch.cuda.synchronize()
    for _ in range(3):
        f.fill_(float("nan"))
        gr.replay()
        torch.cuda.synchronize()
        assert torch.equal(f, eager)
        plan.apply(u)
        torch.cuda.synchronize()


def test_tiled_configurations_rejected():
    import paper_2301_11828_amd as msb
    w = W.small(2, (30, 30), 4, seed=535)
    plan = gpu_plan(w)
    for bad in (dict(tile=11), dict(tile=7), dict(tile=10), dict(tile=72), dict(tile=24, threads_tile=96),
                dict(tile=24, threads_tile=1024)):
        with pytest.raises(msb.MsbError) as ei:
            plan.set_config("fp64", **bad)
        assert ei.value.status == msb.MSB_EINVAL, bad
    assert plan.get_config("fp64")["tile"] == 0
    plan.set_config("fp32", tile=72)      # FP32 frames reach 96
    w3 = W.small(3, (10, 9, 8), 2, seed=536)
    p3 = gpu_plan(w3)
    with pytest.raises(msb.MsbError):
        p3.set_config("fp64", tile=16)
    # plan groups take a member's tiled configuration; the limits of a plan apply to them
    _tiled(plan, 24)
    grp = msb.PlanGroup([plan])
    assert grp.get_config("fp64")["tile"] == 24
    for bad in (dict(tile=11), dict(tile=72), dict(tile=24, threads_tile=96)):
        with pytest.raises(msb.MsbError):
            grp.set_config("fp64", **bad)
    assert grp.get_config("fp64")["tile"] == 24
    grp.close()
