"""Test helpers: build the oracle problem and the GPU plan from one seeded workload."""
import numpy as np

import oracle as O
from paper_2301_11828_amd import workloads as W


def oracle_problem(w: W.Workload, infl=None) -> O.Problem:
    return O.Problem(w.n, w.h, w.M, w.alpha, tuple(w.infl if infl is None else infl), w.rho)


def oracle_bonds(w: W.Workload):
    if w.cracks is None:
        return None
    return O.crack_to_bonds(oracle_problem(w), w.cracks)


def gpu_plan(w: W.Workload, batch=None):
    import paper_2301_11828_amd as msb
    plan = msb.Plan(w.n, w.h, w.M, w.alpha, w.infl, w.rho, batch or w.batch)
    if w.fixed is not None:
        plan.set_constraints(w.fixed)
    if w.cracks is not None:
        plan.set_bonds(msb.crack_to_bonds(w.n, w.h, w.M, w.cracks))
    return plan


def rel_err(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def log(msg):
    print(msg, flush=True)


def gpu_apply(plan, u):
    """plan.apply into an output pre-filled with NaN: an element the kernels never
    write shows up as NaN instead of whatever the allocator last left there."""
    import torch
    out = torch.full_like(u, float("nan"))
    return plan.apply(u, out=out)
