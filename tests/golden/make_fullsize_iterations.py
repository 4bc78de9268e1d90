"""Writes fullsize_iterations.txt: the oracle's iteration counts and final relative
residuals on the 128^3 lognormal diffusion system (ILU(0); GMRES(30) and BiCGSTAB to
1e-8 from x0 = 0), which the full-size GPU tests compare against.

Calls only the oracle (and the seeded input generator); run from the repository root:
    python tests/golden/make_fullsize_iterations.py
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1606_00545_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_iterations.txt")


def main():
    A, xt = synth.workload_diffusion3d(128, sigma=2.0, seed=2)
    b = O.csr_spmv(A.n, A.Ap, A.Aj, A.Ax, xt)
    F = O.iluk(A.n, A.Ap, A.Aj, A.Ax, 0)
    lines = ["# Oracle on the 128^3 lognormal diffusion system (sigma 2, seed 2), b = A x_true,",
             "# ILU(0), x0 = 0, rtol 1e-8. Written by make_fullsize_iterations.py (oracle only).",
             "# columns: solver iterations rel_res seconds"]
    for name, f in (("gmres30", lambda: O.gmres(A, F, b, restart=30, rtol=1e-8)),
                    ("bicgstab", lambda: O.bicgstab(A, F, b, rtol=1e-8))):
        t0 = time.perf_counter()
        r = f()
        dt = time.perf_counter() - t0
        assert r.status == O.OK, (name, r.status)
        lines.append(f"{name} {r.iterations} {r.rel_res:.6e} {dt:.2f}")
        print(lines[-1], flush=True)
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
