"""Parity of the GPU FFT product f = A u (Alg. 3 / Alg. 4 plus D^e, D^f and the
constraint mask) against the oracle's bond-by-bond sum, eq. (mat:f1).

FP64 bar: relative error <= 1e-12 (2-norm over each case), the target the build
states for FP64 displacements; FP32 results are compared with the FP64 oracle and
their error is bounded (and printed) rather than required to match."""
import numpy as np
import pytest

import oracle as O
from paper_2301_11828_amd import workloads as W
from helpers import gpu_apply, gpu_plan, log, oracle_bonds, oracle_problem, rel_err, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-6


def _oracle_apply(w, u):
    p = oracle_problem(w)
    br = oracle_bonds(w)
    return np.stack([O.apply(p, u[c], w.fixed, br) for c in range(u.shape[0])])


CASES = [
    # dim, n, M, fixed, crack, batch -- several tiles per pass and ragged tails
    (2, (37, 29), 3, "none", False, 1),
    (2, (64, 50), 4, "left", True, 2),
    (2, (33, 70), 2, "all", True, 1),
    (2, (41, 23), 3, "mixed", False, 1),
    (2, (1, 17), 2, "none", False, 1),
    (2, (5, 3), 4, "none", False, 3),
    (3, (11, 9, 13), 2, "bottom", False, 1),
    (3, (16, 12, 10), 3, "all", False, 2),
    (3, (7, 5, 6), 3, "none", False, 1),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dd-%s-M%d-%s%s-b%d" % (c[0], "x".join(map(str, c[1])), c[2], c[3], "-crack" if c[4] else "", c[5]))
def test_apply_fp64_matches_oracle(case):
    dim, n, M, fixed, crack, batch = case
    log("apply fp64 %s" % (case,))
    w = W.small(dim, n, M, seed=CASES.index(case), fixed=fixed, crack=crack, batch=batch)
    plan = gpu_plan(w)
    if crack:
        assert plan.n_bonds == len(oracle_bonds(w)) > 0
    f = gpu_apply(plan, to_dev(w.b)).cpu().numpy()
    import paper_2301_11828_amd as msb
    log("  HIP runtime(s): %s" % msb.loaded_hip_runtimes())
    assert len(msb.loaded_hip_runtimes()) == 1
    ref = _oracle_apply(w, w.b)
    for c in range(batch):
        err = rel_err(f[c], ref[c])
        log("  case %d rel err %.3e" % (c, err))
        assert err <= FP64_TOL
    if w.fixed is not None:
        assert np.all(f[:, w.fixed] == 0.0)


@pytest.mark.parametrize("case", [CASES[1], CASES[2], CASES[7]], ids=["2d-crack", "2d-all", "3d"])
def test_apply_fp32_error_bounded(case):
    dim, n, M, fixed, crack, batch = case
    import torch
    w = W.small(dim, n, M, seed=7, fixed=fixed, crack=crack, batch=batch)
    plan = gpu_plan(w)
    f = gpu_apply(plan, to_dev(w.b, torch.float32)).double().cpu().numpy()
    ref = _oracle_apply(w, w.b.astype(np.float32).astype(np.float64))
    for c in range(batch):
        err = rel_err(f[c], ref[c])
        log("fp32 apply %s case %d rel err vs FP64 oracle %.3e" % (case, c, err))
        assert err <= FP32_TOL


@pytest.mark.parametrize("dim", [2, 3])
def test_exhaustive_unit_vectors_reproduce_dense_A(dim):
    """Every column of A on a 9x9 (9x9x9 in 3D, batched) grid with constraints and (2D)
    a crack through the grid: the product equals the oracle's dense matrix."""
    import torch
    n = (9, 9) if dim == 2 else (9, 9, 9)
    M = 3 if dim == 2 else 2
    w = W.small(dim, n, M, seed=3, fixed="mixed" if dim == 2 else "bottom", crack=(dim == 2))
    p = oracle_problem(w)
    A = O.assemble_dense(p, oracle_bonds(w))
    D = dim * w.N
    fixed = w.fixed.reshape(-1)
    plan = gpu_plan(w, batch=D if dim == 2 else 81 * 3)
    cols = np.arange(D) if dim == 2 else np.random.default_rng(0).choice(D, 81 * 3, replace=False)
    U = np.zeros((len(cols), D))
    U[np.arange(len(cols)), cols] = 1.0
    F = gpu_apply(plan, to_dev(U.reshape(len(cols), dim, w.N))).cpu().numpy().reshape(len(cols), D)
    ref = A[:, cols].T.copy()
    ref[:, fixed] = 0.0
    err = np.abs(F - ref).max() / np.abs(A).max()
    log("exhaustive %dD max abs err / max|A| = %.3e" % (dim, err))
    assert err <= 1e-14 * 50


def test_batched_equals_single_bitwise():
    import torch
    w = W.small(2, (45, 38), 3, seed=11, fixed="left", crack=True, batch=3)
    plan_b = gpu_plan(w)
    fb = plan_b.apply(to_dev(w.b)).cpu().numpy()
    w1 = W.small(2, (45, 38), 3, seed=11, fixed="left", crack=True, batch=1)
    plan_1 = gpu_plan(w1)
    for c in range(3):
        f1 = plan_1.apply(to_dev(w.b[c:c + 1])).cpu().numpy()
        assert np.array_equal(f1[0], fb[c])


def test_apply_deterministic():
    w = W.small(3, (12, 10, 9), 3, seed=5, fixed="bottom", batch=2)
    plan = gpu_plan(w)
    u = to_dev(w.b)
    a = gpu_apply(plan, u).cpu().numpy()
    b = gpu_apply(plan, u).cpu().numpy()
    assert np.array_equal(a, b)


def test_rigid_translation_and_rotation_on_gpu():
    """Invariants hold on the GPU product too: translation -> 0 on every row, rotation -> 0."""
    import torch
    w = W.small(2, (40, 31), 3, seed=2, crack=True)
    plan = gpu_plan(w)
    x = oracle_problem(w).node_coords()
    u = np.stack([np.full(w.N, 0.3), np.full(w.N, -0.7)])[None]
    f = gpu_apply(plan, to_dev(u)).cpu().numpy()
    scale = np.abs(gpu_apply(plan, to_dev(np.stack([x[0], 0 * x[0]])[None])).cpu().numpy()).max()
    assert np.abs(f).max() <= 1e-12 * scale
    rot = (1e-2 * np.stack([-x[1], x[0]]))[None]
    fr = gpu_apply(plan, to_dev(rot)).cpu().numpy()
    assert np.abs(fr).max() <= 1e-12 * scale


@pytest.mark.parametrize("name", ["plate32", "plate512", "crack1024"])
def test_apply_at_benchmark_sizes(name):
    """Full-size 2D workloads in the plans' default launch configuration (the crack1024 Verlet bench
    tunes its own; any accepted configuration is exact, see the random-configuration tests)."""
    w = {"plate32": W.plate32, "plate512": W.plate512, "crack1024": lambda: W.crack1024(steps=1)}[name]()
    log("apply at %s" % name)
    plan = gpu_plan(w)
    u = np.random.default_rng(1).standard_normal((1, 2, w.N))
    f = gpu_apply(plan, to_dev(u)).cpu().numpy()
    ref = _oracle_apply(w, u)
    err = rel_err(f, ref)
    log("  %s rel err %.3e" % (name, err))
    assert err <= FP64_TOL


def _cube128_products(w, dt, prec):
    """f = A u of the 128^3 x 16 plan in its default launch configuration and in the one the
    benchmark applies (the recorded tuning)."""
    plan = gpu_plan(w)
    out = {"default": gpu_apply(plan, to_dev(w.b, dt)).double().cpu().numpy()}
    rec = _recorded_tuning("cube128")
    plan.set_lengths(rec["padded"])
    plan.set_config(prec, **rec[prec])
    out["recorded %s" % rec[prec]] = gpu_apply(plan, to_dev(w.b, dt)).double().cpu().numpy()
    return out


def test_apply_cube128_sampled_rows():
    """3D 128^3 batch of 16: compare 3000 sampled nodes per case on 3 cases with the
    oracle's row-by-row sum (all components), in the default and the benchmark's launch
    configuration."""
    import torch
    w = W.cube128(batch=16)
    log("apply cube128 B=16")
    fs = _cube128_products(w, torch.float64, "fp64")
    p = oracle_problem(w)
    rs = np.random.default_rng(3)
    for c in (0, 7, 15):
        rows = np.sort(rs.choice(w.N, 3000, replace=False))
        rows = np.concatenate([rows, [0, w.N - 1, 128 * 128 * 64 + 64 * 128 + 64]])
        ref = O.force(p, w.b[c], rows=rows)
        ref[w.fixed[:, rows]] = 0.0
        for name, f in fs.items():
            err = rel_err(f[c][:, rows], ref)
            log("  case %d %s sampled rel err %.3e" % (c, name, err))
            assert err <= FP64_TOL


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("spw,spwi,lpw", [(1, 1, 1), (2, 1, 1), (1, 2, 2), (4, 2, 2), (3, 3, 3), (2, 4, 1)])
@pytest.mark.parametrize("dim", [2, 3])
def test_wave_owned_signals_match_oracle(prec, spw, spwi, lpw, dim):
    """The wave-owned decomposition (several signals per wavefront, used for large
    batches) on small ragged grids, both precisions, composite radices; the forward
    and inverse x passes take their slots-per-wave independently."""
    import torch
    if dim == 2:
        w = W.small(2, (37, 30), 3, seed=61, fixed="left", crack=True, batch=2)
    else:
        w = W.small(3, (13, 11, 9), 2, seed=62, fixed="bottom", batch=2)
    plan = gpu_plan(w)
    # at most 8 waves per workgroup: 3D rows of 3 components take 5 rows (8 slots) per workgroup
    plan.set_config(prec, rows_per_wg=8 if dim == 2 else 5, team_x=1, slots_fwd=spw, slots_inv=spwi, team_line=1,
                    lines_per_wg=4, lines_per_wave=lpw, max_radix=16)
    dt = torch.float64 if prec == "fp64" else torch.float32
    u = w.b if prec == "fp64" else w.b.astype(np.float32).astype(np.float64)
    f = gpu_apply(plan, to_dev(w.b, dt)).double().cpu().numpy()
    ref = _oracle_apply(w, u)
    for c in range(2):
        err = rel_err(f[c], ref[c])
        log("wave %s spw=%d/%d lpw=%d %dD case %d rel err %.2e" % (prec, spw, spwi, lpw, dim, c, err))
        assert err <= (FP64_TOL if prec == "fp64" else FP32_TOL)


def test_apply_cube128_fp32_sampled_rows():
    """FP32 product at the 128^3 x 16 size (wave-owned, several signals per wave), in the
    default and the benchmark's launch configuration."""
    import torch
    w = W.cube128(batch=16)
    fs = _cube128_products(w, torch.float32, "fp32")
    p = oracle_problem(w)
    rs = np.random.default_rng(4)
    for c in (0, 9):
        rows = np.sort(rs.choice(w.N, 2000, replace=False))
        ref = O.force(p, w.b[c].astype(np.float32).astype(np.float64), rows=rows)
        ref[w.fixed[:, rows]] = 0.0
        for name, f in fs.items():
            err = rel_err(f[c][:, rows], ref)
            log("cube128 fp32 case %d %s sampled rel err %.2e" % (c, name, err))
            assert err <= FP32_TOL


@pytest.mark.parametrize("dim", [2, 3])
def test_profile_apply_times_every_pass_and_leaves_the_product(dim):
    """The measurement helper repeats each pass back to back, then computes f = A u once:
    f must equal the plain product bit for bit."""
    import torch
    if dim == 2:
        w = W.small(2, (40, 33), 3, seed=95, fixed="left", crack=True)
    else:
        w = W.small(3, (12, 9, 8), 2, seed=96, fixed="bottom")
    plan = gpu_plan(w)
    u = to_dev(w.b)
    f = torch.full_like(u, float("nan"))
    ks = plan.profile_apply(u, f, nrep=7)
    log("profile_apply %dD: %s ms" % (dim, ["%.4f" % k for k in ks]))
    assert len(ks) == (3 if dim == 2 else 5) and all(k > 0 for k in ks)
    assert np.array_equal(f.cpu().numpy(), gpu_apply(plan, u).cpu().numpy())


def _recorded_tuning(name="plate512"):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        "%s_tuning.json" % name)
    return json.load(open(path))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plate512_at_the_benchmark_tuning(prec):
    """plate512 in the launch configuration and padded lengths the benchmark applies (the
    recorded tuning), FP64 within 1e-12 of the oracle, FP32 error bounded."""
    import torch
    rec = _recorded_tuning()
    w = W.plate512()
    plan = gpu_plan(w)
    plan.set_lengths(rec["padded"])
    plan.set_config(prec, **rec[prec])
    dt = torch.float64 if prec == "fp64" else torch.float32
    u = np.random.default_rng(11).standard_normal((1, 2, w.N))
    if prec == "fp32":
        u = u.astype(np.float32).astype(np.float64)
    f = gpu_apply(plan, to_dev(u, dt)).double().cpu().numpy()
    err = rel_err(f, _oracle_apply(w, u))
    log("plate512 %s at the recorded tuning %s: rel err %.2e" % (prec, rec["padded"], err))
    assert err <= (FP64_TOL if prec == "fp64" else FP32_TOL)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plate512_written_through_output_equals_plain_stores(prec):
    """The block kernel writes a plain product's output through the L2s when it is at most 8 MB
    (one plate512 case: 4.2 MB in FP64) and with plain stores above (three FP64 cases, five FP32
    ones): case 0 of the larger batch equals the one-case product bit for bit."""
    import torch
    rec = _recorded_tuning()
    w = W.plate512()
    dt = torch.float64 if prec == "fp64" else torch.float32
    big = 3 if prec == "fp64" else 5
    assert big * 2 * w.N * (8 if prec == "fp64" else 4) > 8 << 20 >= 2 * w.N * (8 if prec == "fp64" else 4)
    u = np.random.default_rng(14).standard_normal((big, 2, w.N))
    out = []
    for B in (1, big):
        plan = gpu_plan(w, batch=B)
        plan.set_lengths(rec["padded"])
        plan.set_config(prec, **rec[prec])
        out.append(gpu_apply(plan, to_dev(u[:B], dt)).cpu().numpy())
    log("plate512 %s: one case (written through) vs case 0 of %d (plain stores)" % (prec, big))
    assert np.array_equal(out[0][0], out[1][0])


def test_plate512_batch16_at_the_benchmark_tuning():
    """The bench's 16-case plate512 product in its recorded configuration: sampled rows of
    three cases against the oracle's row-by-row sum."""
    rec = _recorded_tuning()
    w = W.plate512()
    plan = gpu_plan(w, batch=16)
    plan.set_config("fp64", **rec["batch16_fp64"])
    u = np.random.default_rng(12).standard_normal((16, 2, w.N))
    f = gpu_apply(plan, to_dev(u)).cpu().numpy()
    p = oracle_problem(w)
    rs = np.random.default_rng(13)
    for c in (0, 9, 15):
        rows = np.sort(rs.choice(w.N, 2000, replace=False))
        rows = np.concatenate([rows, [0, 511, w.N - 512, w.N - 1]])
        ref = O.force(p, u[c], rows=rows)
        ref[w.fixed[:, rows]] = 0.0
        err = rel_err(f[c][:, rows], ref)
        log("plate512 x16 at the recorded tuning, case %d sampled rel err %.2e" % (c, err))
        assert err <= FP64_TOL


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_products_captured_in_a_hipgraph_replay_exactly(prec, dim):
    """Products captured in a hipGraph on a side stream (as the benchmark times them): every
    replay, with eager products and synchronisations between replays, equals the eager
    product bit for bit."""
    import torch
    if dim == 2:
        w = W.small(2, (45, 38), 3, seed=97, fixed="left", crack=True, batch=2)
    else:
        w = W.small(3, (12, 9, 8), 2, seed=98, fixed="bottom", batch=2)
    plan = gpu_plan(w)
    dt = torch.float64 if prec == "fp64" else torch.float32
    u = to_dev(w.b, dt)
    eager = gpu_apply(plan, u).clone()
    f = torch.full_like(u, float("nan"))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(3):
            plan.apply(u, f)
    torch.cuda.synchronize()
    for r in range(4):
        f.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(f, eager), "replay %d differs from the eager product" % r
        other = gpu_apply(plan, u.flip(-1).contiguous())   # eager work between replays
        torch.cuda.synchronize()
        assert not torch.equal(other, eager)
    ref = _oracle_apply(w, w.b if prec == "fp64" else w.b.astype(np.float32).astype(np.float64))
    assert rel_err(f.double().cpu().numpy(), ref) <= (FP64_TOL if prec == "fp64" else FP32_TOL)
