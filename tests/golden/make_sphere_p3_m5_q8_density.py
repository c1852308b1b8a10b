"""Writes the oracle's density and potential for the Laplace sphere workload (p=3, m=5, q=8, eta=1.6, Gauss
order 6, data from 4 seeded exterior point charges) to sphere_p3_m5_q8_density.txt.

Calls only the oracle (the FP64 CPU reference) and the seeded input generators: H2 operator with stored
coupling blocks, Jacobi CG to true relative residual 1e-13, potential at the 100 seeded interior points.
Run from the repository root: python3 tests/golden/make_sphere_p3_m5_q8_density.py (a few minutes on 8 cores).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1708_09162_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "sphere_p3_m5_q8_density.txt")


def main():
    cfg = W.config_sphere_h2()
    t0 = time.time()
    P = oracle.Problem(cfg["patches"], p=3, m=5, q=8, eta=1.6, gauss_regular=6)
    P.h2_assemble(store_coupling=True)
    t1 = time.time()
    b = P.rhs(W.laplace_charge_field(P.rhs_points(), *cfg["charges"]))
    w, it, rr = P.solve(b, tol=1e-13, maxit=5000)
    t2 = time.time()
    u = P.potential(P.apply_Tt(w), cfg["eval_points"])
    exact = W.laplace_charge_field(cfg["eval_points"], *cfg["charges"])
    print(f"assembly {t1 - t0:.1f} s, CG {it} iterations to {rr:.2e} in {t2 - t1:.1f} s, "
          f"potential max error {np.abs(u - exact).max():.3e}", flush=True)
    assert rr <= 1e-13
    with open(OUT, "w") as fh:
        fh.write("# Oracle solution of the Laplace sphere workload: 6-patch exact unit sphere, p=3, m=5 (7350 dofs),\n")
        fh.write("# H2 with q=8, eta=1.6, Gauss order 6; data = 4 exterior point charges (seed 2); Jacobi CG from 0\n")
        fh.write(f"# to true relative residual {rr:.3e} ({it} iterations).  Written by make_sphere_p3_m5_q8_density.py\n")
        fh.write("# (oracle only).  Lines: n_dof, then the density coefficients in S order, then n_points, then the\n")
        fh.write("# potential at the 100 seeded interior points (seed 2) computed by the oracle from this density.\n")
        fh.write(f"{len(w)}\n")
        for v in w:
            fh.write(f"{v:.17e}\n")
        fh.write(f"{len(u)}\n")
        for v in u:
            fh.write(f"{v:.17e}\n")


if __name__ == "__main__":
    main()
