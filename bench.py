#!/usr/bin/env python3
"""Benchmark of the FFT-BTTB peridynamic product on one MI355X.

Workload (plate512): 2D static linear bond-based peridynamics, 512 x 512 nodes
(524,288 DOF), delta = 3h, plane stress, E = 1, alpha = 9E/(pi delta^3), left
delta-layer constrained, synthetic seeded input.  One step = one FP64 product
f = A u (x-forward pass, y line product pass, x-inverse pass with the D^e/D^f
corrections and the constraint mask), inputs resident in HBM.

Printed JSON line: GDOF/s of the product, per-kernel HIP-event timings with the
roofline of the dominant kernel (algorithmic bytes per launch / mean duration vs
8 TB/s), the FP32 product rate, CG time to a 1e-10 residual in FP64 and in FP32
inside FP64 refinement, and the CPU oracle (bond-by-bond FP64 sum, OpenMP) timed
on a bounded sample of the same product.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def pass_bytes(n, L, d, s):
    """Algorithmic HBM bytes of each kernel of one 2D product (s = bytes per real).

    x-forward: read u (d N reals), write the half spectrum d * Ny * H complex.
    y line   : read + write d * H * Ny complex, read 3 * H * Ly real spectra.
    x-inverse: read d * Ny * H complex, write f (d N reals)."""
    nx, ny = n
    Lx, Ly = L
    H = Lx // 2 + 1
    N = nx * ny
    half = d * ny * H * 2 * s
    return [d * N * s + half, 2 * half + 3 * H * Ly * s, half + d * N * s]


def pass_bytes_3d(n, L, s, nb):
    """Algorithmic HBM bytes of each pass of one 3D product over nb cases (s = bytes per
    real; d = 3; spectra 6 H Ly Lz reals read once per launch).
    x-forward: read u, write T1 [B][d][Nz][H][Ny] complex; y-forward: read T1, write T2
    [B][d][H][Ly][Nz] complex; z line product: read + write T2, read the spectra; y-inverse:
    read T2, write T1; x-inverse: read T1, write f."""
    nx, ny, nz = n
    Lx, Ly, Lz = L
    H = Lx // 2 + 1
    d = 3
    u = nb * d * nx * ny * nz * s
    t1 = nb * d * nz * H * ny * 2 * s
    t2 = nb * d * H * Ly * nz * 2 * s
    spec = 6 * H * Ly * Lz * s
    return [u + t1, t1 + t2, 2 * t2 + spec, t2 + t1, t1 + u]


def tile_bytes(n, d, s, tl, nb=1):
    """Algorithmic HBM bytes of one launch of the tiled single-pass product over nb cases:
    read u and write f (d N reals each per case), the constraint mask (d N bytes, shared),
    the frame spectra (3 tl^2 reals, shared).  Halo re-reads of neighbouring blocks are
    not algorithmic (they come from L2 when neighbouring blocks run on one XCD)."""
    N = n[0] * n[1]
    return nb * 2 * d * N * s + d * N + 3 * tl * tl * s


def model_c_bytes_per_dof(n, M, d, s):
    """Bytes per DOF that a global-embedding FFT product (three HBM passes in 2D) must
    move: s (2 d N + 3 H Ly + 16 H Ny) / (d N) with L the smallest 5-smooth length
    >= N + M per axis and H = Lx / 2 + 1; the reference figure for the primary
    roofline fraction GDOF/s x bytes per DOF / peak."""
    def smooth(x):
        while True:
            m = x
            for q in (2, 3, 5):
                while m % q == 0:
                    m //= q
            if m == 1:
                return x
            x += 1
    Lx, Ly = smooth(n[0] + M), smooth(n[1] + M)
    H = Lx // 2 + 1
    N = n[0] * n[1]
    return s * (2 * d * N + 3 * H * Ly + 16 * H * n[1]) / (d * N)


def product_kernels(plan, prec, n, L, d, s, nb=1):
    """Names and algorithmic bytes per launch of the kernels of one product at the plan's
    configuration: the tiled single-pass kernel, or the three passes of the chain."""
    c = plan.get_config(prec)
    if c["tile"] > 0:
        return ["tile_product"], [tile_bytes(n, d, s, c["tile"], nb)]
    pb = [nb * x for x in pass_bytes(n, L, d, s)]
    pb[1] -= (nb - 1) * 3 * (L[0] // 2 + 1) * L[1] * s      # spectra are read once per launch
    return ["x_forward", "y_line_product", "x_inverse"], pb


def kernel_key(plan, prec, name, n, M, nb=1):
    """The counter summary's key of a product kernel: short name @ workgroups."""
    c = plan.get_config(prec)
    t = "double" if prec == "fp64" else "float"
    if name == "tile_product":
        inner = c["tile"] - 2 * M
        tiles = nb * (-(-n[0] // inner)) * (-(-n[1] // inner))
        if c["tile_regs"]:
            tiles = -(-tiles // c["tile_run"])     # one workgroup per run of blocks
        return "%s<%s>@%d" % ("k_tile_reg" if c["tile_regs"] else "k_tile", t, tiles)
    L = plan.padded_lengths
    wave = c["team_line"] == 1 if name == "y_line_product" else c["team_x"] == 1
    ngroups = (-(-(L[0] // 2 + 1) // c["lines_per_wg"]) if name == "y_line_product"
               else -(-n[1] // c["rows_per_wg"]))
    return "%s<%s%s>@%d" % ({"x_forward": "k_xfwd", "y_line_product": "k_line_y", "x_inverse": "k_xinv"}[name],
                            t, ",wave" if wave else "", nb * ngroups)


def load_traffic(path, kernel):
    """HBM traffic per launch (bytes) of `kernel` from a committed rocprofv3 counter
    summary, or None when absent or taken on a different kernel source."""
    from paper_2301_11828_amd.profiling import source_hash
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    if ("source_hash: %s" % source_hash()) not in lines:
        return None
    for line in lines:
        parts = line.split()
        if len(parts) == 3 and parts[0] == "traffic" and parts[1] == kernel:
            return float(parts[2])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-cg", action="store_true", help="skip the CG time-to-tolerance runs")
    ap.add_argument("--no-copy-bw", action="store_true",
                    help="skip the 1 GiB copy-bandwidth measurement (counter runs: the 64 MiB copy alone "
                         "calibrates FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cube", action="store_true",
                    help="skip the 128^3 x 16 leg of the default run (products, CG to 1e-8 in four variants)")
    ap.add_argument("--graph-block", type=int, default=int(os.environ.get("MSB_BENCH_GRAPH_BLOCK", "32")),
                    help="CG iterations per hipGraph launch in the solves (0: plain launches)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the plans' default launch configurations (skip the autotuner)")
    ap.add_argument("--config", default=os.path.join(ROOT, "profiles", "plate512_tuning.json"),
                    help="JSON file with a recorded plate512 tuning (padded lengths and launch configurations, "
                         "as written by the autotuner) applied instead of tuning; default: the tuning the "
                         "committed plate512 profiles were taken with")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner instead of applying the recorded tunings (profiles/<workload>_tuning.json)")
    ap.add_argument("--workload", default="plate512",
                    choices=["plate512", "crack1024", "cube128", "plates64"],
                    help="plate512 is the headline line; the others measure the remaining workloads")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload != "plate512":
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"crack1024": bench_crack1024, "cube128": bench_cube128,
                          "plates64": bench_plates64}[args.workload](args)), flush=True)
        return

    import numpy as np
    import torch
    import paper_2301_11828_amd as msb
    from paper_2301_11828_amd import workloads as W

    torch.cuda.set_device(0)
    w = W.plate512()
    plan = msb.Plan(w.n, w.h, w.M, w.alpha, batch=1)
    plan.set_constraints(w.fixed)
    tuning = None
    recorded = (json.load(open(args.config)) if args.config and os.path.exists(args.config)
                and not args.retune and not args.no_tune else None)
    if recorded:
        plan.set_lengths(recorded["padded"])
        plan.set_config("fp64", **recorded["fp64"])
        plan.set_config("fp32", **recorded["fp32"])
        tuning = dict(recorded, source=os.path.basename(args.config))
    elif not args.no_tune:
        # launch configuration and padded lengths picked by the library's autotuner
        # (untimed set-up, like the warm-up)
        print("bench: autotune plate512", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        _, ms64 = plan.autotune("fp64", effort=1, lengths=True)
        _, ms32 = plan.autotune("fp32", effort=1)
        tuning = {"seconds": round(time.perf_counter() - t0, 2), "padded": list(plan.padded_lengths),
                  "fp64": plan.get_config("fp64"), "fp32": plan.get_config("fp32"),
                  "product_ms_fp64": round(ms64, 5), "product_ms_fp32": round(ms32, 5)}
    L = plan.padded_lengths
    dofs = w.dofs
    u64 = torch.from_numpy(W.rng(2, 1).standard_normal((1, 2, w.N))).cuda()
    f64 = torch.empty_like(u64)
    u32, f32 = u64.float(), torch.empty_like(u64, dtype=torch.float32)

    def timed(u, f, steps, warmup, graph=0):
        """`steps` products after `warmup` untimed ones: one launch chain per product, or
        (graph > 0, dividing steps) replays of a hipGraph that holds `graph` products."""
        g = None
        if graph:
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                for _ in range(graph):
                    plan.apply(u, f)
            torch.cuda.synchronize()
        per = graph if g is not None else 1

        def run():
            if g is not None:
                g.replay()
            else:
                plan.apply(u, f)
        for _ in range(-(-warmup // per)):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps // per):
            run()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # device time of the same steps between two events, in a pass of its own (the event
        # records stay out of the wall-clock region)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps // per):
            run()
        ev1.record()
        torch.cuda.synchronize()
        return wall, ev0.elapsed_time(ev1) / steps

    # the timed steps replay a hipGraph of G products (the launch gaps between the three
    # kernels of consecutive products shrink); the same steps as plain launches beside it
    G = max([g for g in range(1, 51) if args.steps % g == 0]) if args.steps > 1 else 0
    print("bench: plate512 FP64 product, %d warmup + %d steps (graphs of %d)" % (args.warmup, args.steps, G),
          file=sys.stderr, flush=True)
    wall, ev_ms = timed(u64, f64, args.steps, args.warmup, G)
    ms_step = 1e3 * wall / args.steps
    value = dofs * args.steps / wall / 1e9
    eager = torch.empty_like(f64)
    plan.apply(u64, eager)
    graph_eq = bool(torch.equal(eager, f64))          # the replayed products are the eager one
    wall_plain, ev_plain = timed(u64, f64, args.steps, args.warmup)

    wall32, ev_ms32 = timed(u32, f32, args.steps, args.warmup, G)

    # per-kernel durations (HIP events recorded around the kernels on this stream)
    names, pb = product_kernels(plan, "fp64", w.n, L, 2, 8)
    names32, pb32 = product_kernels(plan, "fp32", w.n, L, 2, 4)
    kms = plan.profile_apply(u64, f64, nrep=max(50, args.steps // 2))
    kms32 = plan.profile_apply(u32, f32, nrep=max(50, args.steps // 2))
    dom = int(np.argmax(kms))
    # the counter summary keys kernels by name and workgroup count (tells this plan's
    # launches from the 16-case plan's)
    kname = kernel_key(plan, "fp64", names[dom], w.n, w.M)
    traffic = load_traffic(os.path.join(ROOT, "profiles", "plate512_fp64_hbm_counters.txt"), kname)
    bpd_c = model_c_bytes_per_dof(w.n, w.M, 2, 8)
    if names[dom] == "tile_product":
        # the survey's per-DOF figure (model C: what a global-embedding FFT product moves per
        # matvec) x the DOFs one launch processes, over the kernel's mean duration; the bytes
        # this kernel itself must move (read u, write f, spectra, mask) reported beside it
        alg = bpd_c * dofs
        model = ("model C: s (2 d N + 3 H Ly + 16 H Ny) at L = 540, the bytes a global-embedding FFT product "
                 "moves per matvec, x the DOFs of one launch")
    else:
        alg = pb[dom]
        model = "the pass's reads and writes of the global-embedding chain"
    achieved = alg / (kms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": names[dom], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "traffic_kind": "L2-fabric bytes per launch (rocprofv3 FETCH_SIZE + "
                                                    "WRITE_SIZE, calibrated with a plain copy)",
                "bytes_per_launch": round(alg), "ms_per_launch": round(kms[dom], 5), "counter_key": kname,
                "bytes_model": model,
                "compulsory": {"bytes_per_launch": pb[dom],
                               "bytes_model": ("read u + write f + frame spectra + constraint mask"
                                               if names[dom] == "tile_product" else "as above"),
                               "achieved_GBs": round(pb[dom] / (kms[dom] * 1e-3) / 1e9, 1),
                               "frac": round(pb[dom] / (kms[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                "primary_frac_model_c": {"B_per_DOF": round(bpd_c, 2), "frac": None,
                                         "definition": "GDOF/s (wall clock) x B_per_DOF / 8 TB/s"}}
    chain_ms = float(sum(kms))
    chain = {"bytes_per_matvec": sum(pb), "kernel_ms_sum": round(chain_ms, 5),
             "achieved_GBs": round(sum(pb) / (chain_ms * 1e-3) / 1e9, 1),
             "frac": round(sum(pb) / (chain_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "event_ms_per_matvec": round(ev_ms, 5)}

    roofline["primary_frac_model_c"]["frac"] = round(value * bpd_c / HBM_PEAK_GBS, 4)
    line = {
        "metric": "BTTB PD matvec GDOF/s (%HBM roofline); CG time-to-1e-10, FP32-refined vs FP64",
        "value": round(value, 3), "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "plate512: 2D static linear BB-PD, 512x512 nodes (524288 DOF), "
                               "delta=3h, left layer constrained, FP64 FFT-BTTB product",
                   "grid": list(w.n), "M": w.M, "dofs": dofs, "padded": list(L)},
        "roofline": roofline,
        "timing": {"graph_products": G, "graph_equals_eager": graph_eq,
                   "plain_launches": {"GDOF_s": round(dofs * args.steps / wall_plain / 1e9, 3),
                                      "ms_per_step": round(1e3 * wall_plain / args.steps, 5),
                                      "event_ms_per_matvec": round(ev_plain, 5)}},
        "kernels_ms": {n: round(float(t), 5) for n, t in zip(names, kms)},
        "kernels_bytes": dict(zip(names, pb)),
        "chain": chain,
        "tuning": tuning,
        "fp32": {"GDOF_s": round(dofs * args.steps / wall32 / 1e9, 3),
                 "kernels_ms": {n: round(float(t), 5) for n, t in zip(names32, kms32)},
                 "chain_frac": round(sum(pb32) / (float(sum(kms32)) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }

    # the same product on 16 load cases at once (one plan, shared spectra): the
    # bandwidth regime, reported beside the single-case latency regime above
    nb = 16
    pb16 = msb.Plan(w.n, w.h, w.M, w.alpha, batch=nb)
    pb16.set_constraints(w.fixed)
    if recorded and "batch16_fp64" in recorded:
        pb16.set_config("fp64", **recorded["batch16_fp64"])
    elif not args.no_tune:
        pb16.autotune("fp64", effort=1)
    if tuning is not None:
        tuning["batch16_fp64"] = pb16.get_config("fp64")
    ub = torch.from_numpy(W.rng(3, 1).standard_normal((nb, 2, w.N))).cuda()
    fb = torch.empty_like(ub)
    for _ in range(5):
        pb16.apply(ub, fb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(50):
        pb16.apply(ub, fb)
    torch.cuda.synchronize()
    sb = (time.perf_counter() - t0) / 50
    kb = pb16.profile_apply(ub, fb, nrep=20)
    names16, bb = product_kernels(pb16, "fp64", w.n, pb16.padded_lengths, 2, 8, nb)
    db = int(np.argmax(kb))
    line["batch16_fp64"] = {"GDOF_s": round(nb * dofs / sb / 1e9, 3), "ms_per_matvec": round(1e3 * sb, 4),
                            "kernels_ms": {n: round(float(t), 5) for n, t in zip(names16, kb)},
                            "counter_key": kernel_key(pb16, "fp64", names16[db], w.n, w.M, nb),
                            "dominant": names16[db],
                            "dominant_frac": round(bb[db] / (kb[db] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "chain_frac": round(sum(bb) / (float(sum(kb)) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    pb16.close()
    del ub, fb

    # calibration for the HBM byte counters: one plain 64 MiB device copy
    src = torch.empty(8 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    # the bandwidth a plain device copy reaches on this GPU (1 GiB read + 1 GiB written per
    # copy, far beyond the 256 MB Infinity Cache), beside the 8 TB/s peak the fractions use
    if not args.no_copy_bw:
        src = torch.empty(128 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(10):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        copy_s = ev0.elapsed_time(ev1) / 10 * 1e-3
        line["hbm_copy"] = {"GB_s": round(2 * src.numel() * 8 / copy_s / 1e9, 1),
                            "bytes_per_copy": 2 * src.numel() * 8,
                            "frac_of_peak": round(2 * src.numel() * 8 / copy_s / 1e9 / HBM_PEAK_GBS, 4)}
        del src, dst

    if not args.no_cg:
        b = torch.from_numpy(w.b).cuda()
        cg = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.apply_precond(b)            # builds the circulant preconditioner (host spectra + upload)
        torch.cuda.synchronize()
        cg["precond_build_seconds"] = round(time.perf_counter() - t0, 4)
        for prec, pre, rel in CG_VARIANTS:
            key = cg_key(prec, pre, rel)
            print("bench: CG %s to 1e-10" % key, file=sys.stderr, flush=True)
            plan.solve(b, precision=prec, tol=1e-10, maxit=200000, graph_block=args.graph_block, precond=pre,
                       reliable_update=rel)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = plan.solve(b, precision=prec, tol=1e-10, maxit=200000, graph_block=args.graph_block,
                                 precond=pre, reliable_update=rel)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            cg[key] = {"seconds": round(dt, 4), "iterations": info[0].inner_iters,
                       "outer": info[0].outer_iters, "rel_residual_fp64": info[0].rel_residual,
                       "status": info[0].status}
        cg_speedups(cg)
        line["cg"] = cg
        # the paper's own static solver: adaptive dynamic relaxation (Alg. 1), FP64, one
        # fused product chain per update; updates/s and the force residual reached
        print("bench: ADR 2000 updates", file=sys.stderr, flush=True)
        ua = torch.zeros_like(b)
        va, Fa = torch.zeros_like(b), torch.zeros_like(b)
        plan.adr_run(20, ua, va, Fa, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.adr_run(0, ua, va, Fa, b)
        res = plan.adr_run(2000, ua, va, Fa, b, restart=False, residual=True)
        torch.cuda.synchronize()
        dta = time.perf_counter() - t0
        bn = float(torch.linalg.vector_norm(b * (1 - torch.from_numpy(w.fixed.astype(np.float64)).cuda())))
        line["adr"] = {"updates": 2000, "seconds": round(dta, 4), "updates_per_s": round(2000 / dta, 1),
                       "rel_force_residual": float(res[0]) / bn,
                       "note": "convergence of the left-clamped plate takes far more updates than CG iterations"}

    if not args.no_cube and not args.no_cg:
        # the bandwidth regime of the method: 128^3 x 16 load cases, both products and the
        # four CG variants to 1e-8 (where refined FP32 is expected to beat FP64)
        print("bench: cube128 x16 leg", file=sys.stderr, flush=True)
        del pb16
        torch.cuda.empty_cache()
        line["cube128"] = bench_cube128(args)

    if not args.no_cpu:
        import oracle as O
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        p = O.Problem(w.n, w.h, w.M, w.alpha)
        u = u64.cpu().numpy()[0]
        O.apply(p, u, w.fixed)           # load / warm
        reps, t0 = 0, time.perf_counter()
        while True:
            O.apply(p, u, w.fixed)
            reps += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        cores = _cpu_cores()
        line["cpu_baseline"] = {"value": round(dofs * reps / dt / 1e9, 5), "unit": "GDOF/s",
                                "cores": cores, "cpu_model": _cpu_model(), "kind": "oracle",
                                "sample": "%d full FP64 bond-by-bond products of plate512 (%.1f s)" % (reps, dt)}
        # context: the paper's fast method itself on the same CPU (the oracle's FFT product,
        # scipy's multithreaded FFT), the FP64 CG time it implies at the GPU's iteration
        # count, and config 1 (32^2 plate) solved by dense Cholesky and by the oracle's CG
        t0 = time.perf_counter()
        fs = O.fft_setup(p, plan.padded_lengths, workers=cores)
        t_setup = time.perf_counter() - t0
        O.fft_apply(p, u, w.fixed, workers=cores, setup=fs)
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 3.0:
            O.fft_apply(p, u, w.fixed, workers=cores, setup=fs)
            reps += 1
        per = (time.perf_counter() - t0) / reps
        its = line.get("cg", {}).get("fp64", {}).get("iterations")
        line["cpu_baseline"]["fft_method"] = {
            "GDOF_s": round(dofs / per / 1e9, 5), "ms_per_product": round(per * 1e3, 2), "threads": cores,
            "assembly_seconds": round(t_setup, 3),
            "sample": "%d FP64 products of plate512 at the GPU's padded lengths" % reps,
            "cg_fp64_seconds_extrapolated": round(per * its, 1) if its else None}
        w1 = W.plate32()
        p1 = O.Problem(w1.n, w1.h, w1.M, w1.alpha)
        t0 = time.perf_counter()
        x1 = O.solve_dense(p1, w1.b[0], w1.fixed)
        t_chol = time.perf_counter() - t0
        t0 = time.perf_counter()
        x2, its1 = O.solve_cg(p1, w1.b[0], w1.fixed, tol=1e-10)[:2]
        t_cg = time.perf_counter() - t0
        line["cpu_baseline"]["config1_plate32"] = {
            "dense_cholesky_seconds": round(t_chol, 4), "cg_to_1e-10_seconds": round(t_cg, 4),
            "cg_iterations": int(its1), "cg_vs_cholesky_rel_diff": float(np.linalg.norm(x2 - x1) / np.linalg.norm(x1))}
    print(json.dumps(line), flush=True)


def _cpu_cores():
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()


def _cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), for the CPU-baseline records."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def recorded_tuning(args, name):
    """The tuning recorded for a workload (padded lengths and launch configurations as the
    autotuner chose them; the parity tests run the same), or None to tune at run time."""
    path = os.path.join(ROOT, "profiles", "%s_tuning.json" % name)
    if args.retune or args.no_tune or not os.path.exists(path):
        return None
    return json.load(open(path))



# CG variants timed to a tolerance: (precision, preconditioned, reliable updates).  The
# refined solver restarts CG after each FP64 residual update, or (reliable) keeps the
# search direction across the replacement.
CG_VARIANTS = (("fp64", False, 0), ("fp32_refined", False, 0), ("fp32_refined", False, 1),
               ("fp64", True, 0), ("fp32_refined", True, 0), ("fp32_refined", True, 1))


def cg_key(prec, pre, rel):
    return prec + ("_reliable" if rel else "") + ("_pcg" if pre else "")


def cg_speedups(cg):
    """FP64 seconds over each other variant's, against the same preconditioning."""
    for k in list(cg):
        if not isinstance(cg[k], dict) or k in ("fp64", "fp64_pcg"):
            continue
        base = "fp64_pcg" if k.endswith("_pcg") else "fp64"
        cg["speedup_%s_vs_%s" % (k, base)] = round(cg[base]["seconds"] / cg[k]["seconds"], 3)
    cg["speedup_fp64_pcg_vs_fp64"] = round(cg["fp64"]["seconds"] / cg["fp64_pcg"]["seconds"], 3)


def bench_crack1024(args):
    """Dynamic pre-crack plate, 1024^2 (2.1M DOF), delta = 4h, 12,654 broken bonds:
    velocity Verlet in FP32 with the FP64 energy every 10 steps; steps/s."""
    import numpy as np
    import torch
    import paper_2301_11828_amd as msb
    from paper_2301_11828_amd import workloads as W
    w = W.crack1024(steps=1000)
    plan = msb.Plan(w.n, w.h, w.M, w.alpha, rho=w.rho)
    plan.set_bonds(msb.crack_to_bonds(w.n, w.h, w.M, w.cracks))
    rec = recorded_tuning(args, "crack1024")
    if rec:
        plan.set_lengths(rec["padded"])
        plan.set_config("fp32", **rec["fp32"])
        tuned = dict(rec["fp32"], source="crack1024_tuning.json")
    else:
        tuned = None if args.no_tune else plan.autotune("fp32", effort=1)[0]
    u = torch.zeros((1, 2, w.N), dtype=torch.float32, device="cuda")
    v = torch.zeros_like(u)
    bf = torch.from_numpy(w.b).float().cuda()
    a = plan.vv_init(u, bf)
    plan.vv_run(w.dt, 20, u.clone(), v.clone(), a.clone(), bf)          # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    en = plan.vv_run(w.dt, w.steps, u, v, a, bf, energy_every=10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # energy on a scale: kinetic 1/2 rho V |v|^2 and elastic -1/2 V u.(A u) of the final
    # state (FP64 product of the FP32 state), the drift of the FP64 energy over the run
    # relative to the larger of the two
    V = w.h ** 2
    u64 = u.double()
    kin = 0.5 * w.rho * V * float((v.double() ** 2).sum())
    ela = -0.5 * V * float((u64 * plan.apply(u64)).sum())
    scale = max(kin, ela)
    out = {"workload": "crack1024: 2D dynamic pre-crack, 1024x1024 (2097152 DOF), delta=4h, "
                       "12654 broken bonds, FP32 velocity Verlet, FP64 energy every 10 steps",
           "steps": w.steps, "seconds": round(dt, 4), "steps_per_s": round(w.steps / dt, 1),
           "GDOF_steps_per_s": round(w.dofs * w.steps / dt / 1e9, 3),
           "energy": {"first": float(en[0]), "last": float(en[-1]), "kinetic_final": kin, "elastic_final": ela,
                      "max_abs_change_over_run_rel_to_max_kinetic_elastic": float(np.abs(en - en[0]).max()) / scale},
           "n_bonds": plan.n_bonds, "tuned_fp32": tuned}
    # crack propagation (eq. (mu)): the stretch pass over all 2.1M x 24 half-stencil bonds
    # plus the count read-back, at a critical stretch no bond reaches (cost of the check);
    # then Verlet with the check after every step
    s0 = 1.0
    plan.crack_update(u, s0)                                             # mask upload, warm
    torch.cuda.synchronize()
    reps = 50
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.crack_update(u, s0)
    per_call = (time.perf_counter() - t0) / reps
    nsteps = 200
    t0 = time.perf_counter()
    for _ in range(nsteps):
        plan.vv_run(w.dt, 1, u, v, a, bf)
        plan.crack_update(u, s0)
    torch.cuda.synchronize()
    dtc = time.perf_counter() - t0
    half = 24   # bonds per node in the half stencil at delta = 4h
    out["crack_update"] = {"s0": s0, "us_per_call": round(1e6 * per_call, 2),
                           "bonds_checked": half * w.N, "Gbond_per_s": round(half * w.N / per_call / 1e9, 2),
                           "verlet_plus_check_steps_per_s": round(nsteps / dtc, 1),
                           "bytes_per_call": 2 * w.N * 4 + 2 * w.N * 8 + w.N * 4}
    # with real breaks: s0 set to the 2000th largest bond stretch of the loaded state (a
    # workload parameter picked from u; the stretches near the crack tips are the largest),
    # so one call breaks about 2000 bonds: the stretch pass, the scan, the emit pass, the
    # host merge into the sorted broken list and the D^f list rebuild, then the product
    # with the longer list
    uu = u.reshape(2, w.n[1], w.n[0]).double()
    top = []
    for oy in range(0, w.M + 1):
        for ox in range(-w.M, w.M + 1):
            if (oy == 0 and ox <= 0) or ox * ox + oy * oy > w.M * w.M:
                continue
            dxu = uu[0, oy:, max(ox, 0):w.n[0] + min(ox, 0)] - uu[0, :w.n[1] - oy, max(-ox, 0):w.n[0] - max(ox, 0)]
            dyu = uu[1, oy:, max(ox, 0):w.n[0] + min(ox, 0)] - uu[1, :w.n[1] - oy, max(-ox, 0):w.n[0] - max(ox, 0)]
            r0 = w.h * (ox * ox + oy * oy) ** 0.5
            st = torch.sqrt((ox * w.h + dxu) ** 2 + (oy * w.h + dyu) ** 2) / r0 - 1.0
            top.append(torch.topk(st.reshape(-1), 2000).values)
    s_break = float(torch.topk(torch.cat(top), 2000).values[-1])
    nb0 = plan.n_bonds
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_new = plan.crack_update(u, s_break)
    torch.cuda.synchronize()
    t_break = time.perf_counter() - t0
    f32 = torch.empty_like(u)
    plan.apply(u, f32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        plan.apply(u, f32)
    torch.cuda.synchronize()
    out["crack_update_with_breaks"] = {
        "s0": s_break, "bonds_before": nb0, "new_broken_bonds": n_new, "bonds_after": plan.n_bonds,
        "ms_per_call": round(1e3 * t_break, 3),
        "note": "one call: stretch pass over every bond, scan, emit of the new pairs, host merge, D^f rebuild",
        "product_us_after": round(1e6 * (time.perf_counter() - t0) / 20, 2)}
    if not args.no_cpu:
        import oracle as O
        p = O.Problem(w.n, w.h, w.M, w.alpha, rho=w.rho)
        br = O.crack_to_bonds(p, w.cracks)
        t0 = time.perf_counter()
        O.vv(p, np.zeros((2, w.N)), np.zeros((2, w.N)), w.b[0], w.dt, 5, None, None, br)
        dtc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(5 / dtc, 3), "unit": "steps/s", "cores": _cpu_cores(),
                               "cpu_model": _cpu_model(),
                               "kind": "oracle", "sample": "5 FP64 Verlet steps of crack1024"}
    return out


def bench_cube128(args):
    """3D block 128^3 x 16 load cases (100.7M DOF): FP32 and FP64 products and
    FP32-refined CG vs FP64 CG to 1e-8."""
    import numpy as np
    import torch
    import paper_2301_11828_amd as msb
    from paper_2301_11828_amd import workloads as W
    w = W.cube128(batch=16)
    plan = msb.Plan(w.n, w.h, w.M, w.alpha, batch=16)
    plan.set_constraints(w.fixed)
    tuning = None
    rec = recorded_tuning(args, "cube128")
    if rec:
        plan.set_lengths(rec["padded"])
        plan.set_config("fp64", **rec["fp64"])
        plan.set_config("fp32", **rec["fp32"])
        tuning = {"fp64": rec["fp64"], "fp32": rec["fp32"], "source": "cube128_tuning.json"}
    elif not args.no_tune:
        t0 = time.perf_counter()
        plan.autotune("fp32_refined", effort=1)
        tuning = {"seconds": round(time.perf_counter() - t0, 2), "fp64": plan.get_config("fp64"),
                  "fp32": plan.get_config("fp32")}
    b = torch.from_numpy(w.b).cuda()
    dofs = w.dofs * 16
    out = {"workload": "cube128: 3D static, 128^3 x 16 cases (100663296 DOF), delta=3h, z=0 layer fixed",
           "padded": list(plan.padded_lengths), "tuning": tuning}
    for dt in (torch.float64, torch.float32):
        u = b.to(dt)
        f = torch.empty_like(u)
        for _ in range(3):
            plan.apply(u, f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            plan.apply(u, f)
        torch.cuda.synchronize()
        s = (time.perf_counter() - t0) / 10
        ks = plan.profile_apply(u, f, nrep=5)
        sz = 8 if dt == torch.float64 else 4
        pb = pass_bytes_3d(w.n, plan.padded_lengths, sz, 16)
        dom = int(np.argmax(ks))
        names = ["x_forward", "y_forward", "z_line_product", "y_inverse", "x_inverse"]
        ach = pb[dom] / (float(ks[dom]) * 1e-3) / 1e9
        out["matvec_" + str(dt)[6:]] = {
            "GDOF_s": round(dofs / s / 1e9, 2), "ms": round(1e3 * s, 3),
            "kernels_ms": dict(zip(names, [round(float(x), 4) for x in ks])),
            "kernels_GBs": dict(zip(names, [round(b / (float(t) * 1e-3) / 1e9, 1) for b, t in zip(pb, ks)])),
            "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": pb[dom],
                         "ms_per_launch": round(float(ks[dom]), 5)},
            "chain_frac": round(sum(pb) / (float(sum(ks)) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del u, f
    # calibration for counter runs of this leg: one plain 64 MiB device copy
    src = torch.empty(8 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    if args.no_cg:
        return out
    cg = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.apply_precond(b)
    torch.cuda.synchronize()
    cg["precond_build_seconds"] = round(time.perf_counter() - t0, 3)
    for prec, pre, rel in CG_VARIANTS:
        key = cg_key(prec, pre, rel)
        print("bench: cube128 CG %s to 1e-8" % key, file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        _, info = plan.solve(b, precision=prec, tol=1e-8, maxit=100000, graph_block=args.graph_block, precond=pre,
                             reliable_update=rel)
        torch.cuda.synchronize()
        cg[key] = {"seconds": round(time.perf_counter() - t0, 3),
                   "iterations_max": max(i.inner_iters for i in info),
                   "max_rel_residual": max(i.rel_residual for i in info),
                   "status": max((i.status for i in info), key=abs)}
    cg_speedups(cg)
    out["cg_to_1e-8"] = cg
    if not args.no_cpu:
        # the oracle's bond-by-bond FP64 product on one case (3 runs), and the CG time it
        # implies: per-case product time x 16 cases x the GPU's FP64 iteration count
        # (extrapolated: the oracle's own CG at this size would take about that long)
        import oracle as O
        p = O.Problem(w.n, w.h, w.M, w.alpha)
        u0 = w.b[0]
        O.apply(p, u0, w.fixed)
        t0 = time.perf_counter()
        for _ in range(3):
            O.apply(p, u0, w.fixed)
        per = (time.perf_counter() - t0) / 3
        out["cpu_baseline"] = {"value": round(w.dofs / per / 1e9, 5), "unit": "GDOF/s", "cores": _cpu_cores(),
                               "cpu_model": _cpu_model(),
                               "kind": "oracle", "sample": "3 FP64 bond-by-bond products of one 128^3 case",
                               "cg_fp64_seconds_extrapolated": round(per * 16 * cg["fp64"]["iterations_max"], 1)}
    return out


def bench_plates64(args):
    """64 plates of uneven size (64^2 .. 384^2), each with its own influence
    coefficients: target solve, forward FP32-refined solve, loss, hand-written adjoint
    solve and influence-coefficient gradient.  Headline: one plan per plate, all 64
    run as one plan group (one launch per pass covers every plate still iterating).
    Beside it: the same 64 plans one after another, and the plates batched per size
    (5 plans with per-case coefficients) one after another."""
    import numpy as np
    import torch
    import paper_2301_11828_amd as msb
    from paper_2301_11828_amd import workloads as W
    ws = W.plates64()
    plans = []
    for w in ws:
        pl = msb.Plan(w.n, w.h, w.M, w.alpha, infl=w.infl, batch=1)
        pl.set_constraints(w.fixed)
        plans.append(pl)
    grp = msb.PlanGroup(plans)
    tuning = None
    rec = recorded_tuning(args, "plates64")
    if rec:
        # the group tuning the gradient parity test runs at
        grp.set_config("fp64", **rec["fp64"])
        grp.set_config("fp32", **rec["fp32"])
        tuning = {"fp64": rec["fp64"], "fp32": rec["fp32"], "source": "plates64_tuning.json"}
    elif not args.no_tune:
        # the group's launch configuration picked by the group autotuner (untimed set-up)
        t0 = time.perf_counter()
        grp.autotune("fp32_refined", effort=1)
        tuning = {"seconds": round(time.perf_counter() - t0, 2), "fp64": grp.get_config("fp64"),
                  "fp32": grp.get_config("fp32")}
    # plain launches: hipGraph blocks of 32 iterations measured 2% slower for this group (its
    # kernels run 30-110 us each and the work list changes as plates converge), and reliable
    # updates 8% slower than restarts (more FP64 residual replacements)
    grp.graph_block = 0
    GSolve = msb.make_group_solve_function()
    Solve = msb.make_solve_function()
    by_size = {}
    for i, w in enumerate(ws):
        by_size.setdefault(w.n[0], []).append(i)
    sizes = sorted(by_size)
    splans = []
    for sz in sizes:
        w0 = ws[by_size[sz][0]]
        pl = msb.Plan(w0.n, w0.h, w0.M, w0.alpha, infl=w0.infl, batch=len(by_size[sz]))
        pl.set_constraints(w0.fixed)
        splans.append(pl)

    def inputs():
        bs = [torch.from_numpy(w.b).cuda().requires_grad_(True) for w in ws]
        as_ = [torch.tensor(w.infl, dtype=torch.float64, requires_grad=True) for w in ws]
        return bs, as_

    def run_group():
        bs, as_ = inputs()
        grp.set_infl([np.asarray(w.extra["infl_target"]) for w in ws])
        uts, _ = grp.solve([b.detach() for b in bs], precision="fp32_refined", tol=1e-10)
        us = GSolve.apply(grp, "fp32_refined", 1e-10, *bs, *as_)
        loss = sum(((u - ut) ** 2).sum() for u, ut in zip(us, uts))
        loss.backward()
        torch.cuda.synchronize()
        return loss.item(), np.stack([a.grad.numpy() for a in as_])

    def run_plans():
        bs, as_ = inputs()
        total = 0.0
        for pl, w, b, a in zip(plans, ws, bs, as_):
            pl.set_infl(np.asarray(w.extra["infl_target"]))
            ut, _ = pl.solve(b.detach(), precision="fp32_refined", tol=1e-10)
            u = Solve.apply(pl, b, a, "fp32_refined", 1e-10)
            loss = ((u - ut) ** 2).sum()
            loss.backward()
            total += loss.item()
        torch.cuda.synchronize()
        return total, np.stack([a.grad.numpy() for a in as_])

    def run_sizes():
        total = 0.0
        grads = np.zeros((len(ws), len(ws[0].infl)))
        for pl, sz in zip(splans, sizes):
            idx = by_size[sz]
            b = torch.from_numpy(np.concatenate([ws[i].b for i in idx])).cuda().requires_grad_(True)
            a = torch.tensor(np.array([ws[i].infl for i in idx]), dtype=torch.float64, requires_grad=True)
            pl.set_infl(np.array([ws[i].extra["infl_target"] for i in idx]), per_case=True)
            ut, _ = pl.solve(b.detach(), precision="fp32_refined", tol=1e-10)
            u = Solve.apply(pl, b, a, "fp32_refined", 1e-10)
            loss = ((u - ut) ** 2).sum()
            loss.backward()
            total += loss.item()
            grads[idx] = a.grad.numpy()
        torch.cuda.synchronize()
        return total, grads

    def timed(fn):
        # one untimed run (first-use set-up: derivative operators, preconditioners, frame
        # spectra), then the faster of two timed runs
        fn()
        best = None
        for _ in range(2):
            t0 = time.perf_counter()
            r = fn()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, r)
        return best

    dt, (loss, grads) = timed(run_group)
    # the same with every member's CG preconditioned by its circulant inverse (each
    # preconditioner is rebuilt when the member's coefficients change: inside the timing)
    grp.precond = True
    dtc, (loss_c, grads_c) = timed(run_group)
    grp.precond = False
    dtp, (loss_p, grads_p) = timed(run_plans)
    dts, (loss_s, grads_s) = timed(run_sizes)

    def gdiff(g, h):
        return float(np.max(np.abs(g - h)) / max(np.max(np.abs(h)), 1e-300))

    dofs = sum(w.dofs for w in ws)
    return {"workload": "plates64: 64 plates, sizes %s, delta=3h, omega=sum_k a_k (r/delta)^k per plate, "
                        "target + forward + adjoint FP32-refined solves to 1e-10 and dL/da" % sizes,
            "plates": len(ws), "dofs_total": dofs, "solves": 3 * len(ws),
            "seconds": round(dt, 3), "mode": "64 plans in one plan group (one launch per pass; a 2D tiled "
                                              "configuration: one launch of the block kernel per product)",
            "graph_block": 0, "refinement": "restarted",
            "graph_block_note": "hipGraph blocks of 32 iterations measured 2% slower for this group and reliable "
                                "updates 8% slower than restarts",
            "work_list": "per-pass group launches over the members still iterating (rebuilt at each flag "
                         "check), not a persistent kernel",
            "seconds_group_pcg": round(dtc, 3), "speedup_group_pcg_vs_group": round(dt / dtc, 2),
            "grad_max_rel_diff_pcg_vs_cg": gdiff(grads_c, grads),
            "seconds_64_plans_one_after_another": round(dtp, 3),
            "seconds_batched_per_size_one_after_another": round(dts, 3),
            "speedup_group_vs_plans": round(dtp / dt, 2), "speedup_group_vs_batched_sizes": round(dts / dt, 2),
            "loss": loss, "grad_max_rel_diff_vs_plans": gdiff(grads, grads_p),
            "grad_max_rel_diff_vs_batched_sizes": gdiff(grads, grads_s),
            "plates_per_size": {int(k): len(v) for k, v in sorted(by_size.items())}, "group_tuning": tuning}


if __name__ == "__main__":
    main()
