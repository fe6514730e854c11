"""Writes crack1024_vv_oracle.npz from the CPU oracle alone (run from the repository root:
python tests/golden/make_crack1024_vv.py; about 6 minutes on 8 cores).

The 1024 x 1024 pre-crack plate (delta = 4h, 12,654 broken bonds, opposing edge loads,
u = v = 0 at rest; Alg. 2 with a = (A u + b)/rho) advanced 1000 FP64 Verlet steps at the
workload's time step.  Stored: 4096 seeded DOF indices, u and v at those DOFs after 10,
100 and 1000 steps, and the kinetic, elastic and load energies every 10 steps."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O                                   # noqa: E402
from paper_2301_11828_amd import workloads as W      # noqa: E402


def main():
    w = W.crack1024(steps=1000)
    p = O.Problem(w.n, w.h, w.M, w.alpha, rho=w.rho)
    br = O.crack_to_bonds(p, w.cracks)
    idx = np.sort(np.random.default_rng(2301).choice(2 * w.N, size=4096, replace=False))
    u = np.zeros((2, w.N))
    v = np.zeros((2, w.N))
    snaps = {}
    parts = []
    for chunk in range(100):
        u, v, _, _ = O.vv(p, u, v, w.b[0], w.dt, 10, None, None, br)
        n = 10 * (chunk + 1)
        parts.append(O.energy_parts(p, u, v, w.b[0], None, br))
        if n in (10, 100, 1000):
            snaps[n] = (u.reshape(-1)[idx].copy(), v.reshape(-1)[idx].copy())
        print("step %d energy parts %s" % (n, parts[-1]), flush=True)
    np.savez(os.path.join(HERE, "crack1024_vv_oracle.npz"), idx=idx, dt=w.dt, n_bonds=len(br),
             u10=snaps[10][0], v10=snaps[10][1], u100=snaps[100][0], v100=snaps[100][1],
             u1000=snaps[1000][0], v1000=snaps[1000][1], energy_parts=np.array(parts))


if __name__ == "__main__":
    main()
