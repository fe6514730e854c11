"""Writes plates64_grad_oracle.txt from the CPU oracle alone (run from the repository root:
python tests/golden/make_plates64_grad.py; a few minutes on 8 cores).

For the first plate of each size (64^2 ... 384^2) of the seeded 64-plate batch (omega =
sum_k a_k (r/delta)^k, all sides fixed, b ~ N(0, 1)): the target u_t solved with the
perturbed coefficients a'_k, then the loss L = ||u - u_t||^2 of the solution with a_k and
its gradient dL/da_k = w . (A_k u)_F with the adjoint w = K_FF^{-1} 2 (u - u_t)_F, every
solve by the oracle's CG to a relative residual of 1e-13."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O                                   # noqa: E402
from paper_2301_11828_amd import workloads as W      # noqa: E402


def main():
    ws = W.plates64()
    lines = ["# plate size L dL/da_0..dL/da_7 cg_iterations_u cg_iterations_w rel_residual_u rel_residual_w"]
    done = set()
    for i, w in enumerate(ws):
        s = w.n[0]
        if s in done:
            continue
        done.add(s)
        pt = O.Problem(w.n, w.h, w.M, w.alpha, w.extra["infl_target"])
        ut, _, _ = O.solve_cg(pt, w.b[0], w.fixed, tol=1e-13)
        p = O.Problem(w.n, w.h, w.M, w.alpha, w.infl)
        L, _, _, ga, its, res = O.grad_cg(p, w.b[0], ut, w.fixed, tol=1e-13)
        lines.append("%d %d %.17e %s %d %d %.3e %.3e" % (i, s, L, " ".join("%.17e" % x for x in ga), its[0], its[1],
                                                          res[0], res[1]))
        print(lines[-1], flush=True)
    open(os.path.join(HERE, "plates64_grad_oracle.txt"), "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
