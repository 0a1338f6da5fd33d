"""Writes ellipses200_oracle_solve.npz: the FP64 oracle's mobility solve of the 200-ellipse
cell (area fraction 0.4, 256 nodes each, N = 51,200, seed 2).

Only the oracle and the seeded input generator run here. The solve is the completed BIE of
Sec. 5 (eq. BIEPerturbed) with the 3x3 near set, the close correction of Sec. 6.3 and the
proxy periodizer of Sec. 6.1-6.2, by the oracle's MGS GMRES from zero to a relative residual
estimate of 1e-12 (tighter than the 1e-10 the device solves stop at, so that the device's
readouts can be compared with it at their own accuracy). Readouts: velocities and angular
velocities at the centroids (Sec. 3 eq. RigidBodyMotion) and mu_eff by the stresslet identity
(Sec. 3 eq. mueff). The file also records the true residual of the stored density through
the oracle's operator.

Run from the repository root:  python tests/golden/make_ellipses200_solve.py
(about 25 minutes on 8 cores: each operator product of the oracle takes about 9 s).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import operator as op      # noqa: E402
from oracle import readout as ro       # noqa: E402
from paper_1912_04501_amd import workloads as W   # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ellipses200_oracle_solve.npz")


def main():
    t0 = time.time()
    wl = W.ellipses_200()
    prob = op.make_problem(wl)
    b = op.rhs(prob)
    count = [0]

    def mv(v):
        count[0] += 1
        if count[0] % 10 == 0:
            print(f"product {count[0]} at {time.time() - t0:.0f} s", flush=True)
        return op.apply(prob, v)

    x, info = op.gmres(mv, b, tol=1e-12, maxiter=500)
    res = float(np.linalg.norm(b - op.apply(prob, x)) / np.linalg.norm(b))
    v, om = ro.velocities(prob, x)
    mu = float(ro.mu_eff(prob, x))
    np.savez_compressed(OUT, sigma=x, vel=v, omega=om, mu_eff=np.array(mu), true_residual=np.array(res),
                        iterations=np.array(info["iterations"]), N=np.array(prob.N),
                        skew=np.array(wl["skew"]))
    print(f"wrote {OUT}: iterations {info['iterations']}, true residual {res:.3e}, mu_eff {mu:.12f}, "
          f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
