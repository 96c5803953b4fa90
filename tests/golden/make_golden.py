"""Writes the stored expected values of the full-size parity tests.

Runs only the oracle (no GPU code): the plane-wave workload on the 16^3 mesh
of order 3 (omega = 8 pi, V(2,2), theta = 1/5), solved by the oracle's PCG to
1e-8 and to 1e-12.  Stores the iteration counts and the solution at 256
seeded sample positions of the canonical trace vector.

    python tests/golden/make_golden.py      # takes a few minutes
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dpg, multigrid  # noqa: E402
from paper_2304_01728_amd import workloads  # noqa: E402


def main():
    from threadpoolctl import threadpool_limits
    w = workloads.plane_wave_16()
    with threadpool_limits(1):
        pr = dpg.Problem(w.N, w.p, w.omega, [dict(u0=dpg.plane_wave_u0(w.omega, w.direction))])
        S, s, _ = pr.condensed()
    rhs = dpg.assemble_vector(pr.edofs, s, pr.num.n)[:, 0]
    H = multigrid.Hierarchy(w.N, w.p, S, theta=w.theta, nu_pre=w.nu_pre, nu_post=w.nu_post)
    x8, it8, rr8 = H.solve(rhs, 1e-8)
    x12, it12, rr12 = H.solve(rhs, 1e-12)
    rng = np.random.default_rng(2024)
    pos = np.sort(rng.choice(pr.num.n, size=256, replace=False))
    out = {
        "workload": w.name,
        "generator": "tests/golden/make_golden.py (oracle only)",
        "n_trace": int(pr.num.n),
        "iters_tol_1e-8": int(it8), "relres_tol_1e-8": float(rr8),
        "iters_tol_1e-12": int(it12), "relres_tol_1e-12": float(rr12),
        "x_inf_norm": float(np.abs(x12).max()),
        "sample_pos": pos.tolist(),
        "x12_sample_re": x12[pos].real.tolist(),
        "x12_sample_im": x12[pos].imag.tolist(),
        "s_sample_re": rhs[pos].real.tolist(),
        "s_sample_im": rhs[pos].imag.tolist(),
    }
    with open(os.path.join(HERE, "plane_wave_16.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("iterations", it8, it12)


if __name__ == "__main__":
    main()
