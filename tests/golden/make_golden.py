"""Writes the oracle's reference solutions used by the GPU parity tests and bench.py.

Calls only the CPU oracle (oracle/) and the seeded problem generator.  For each
workload it solves A u = b with the oracle's MGS-GMRES and J^{-1} (dense LU
leaf solves) to a preconditioned residual of 1e-13, then stores u at 4096
seeded sample indices together with ||u||, the true relative residual and the
iteration count:

    python tests/golden/make_golden.py bumps_8x8x8_p10
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import hps_oracle as O  # noqa: E402
from paper_2112_02211_amd import problems as P  # noqa: E402


def main(name: str, tol: float = 1e-13, nsamp: int = 4096):
    prob = P.workload(name)
    t0 = time.time()
    op = O.build(prob)
    u, its, hist = O.solve_gmres(op, tol=tol, restart=prob.restart, maxit=5000)
    r = op.rhs - op.A @ u
    true_rel = float(np.linalg.norm(r) / np.linalg.norm(op.rhs))
    idx = np.sort(np.random.default_rng(123).choice(op.d.N, size=min(nsamp, op.d.N), replace=False))
    out = os.path.join(HERE, f"{name}_oracle.npz")
    np.savez(out, idx=idx, u=u[idx], unorm=np.linalg.norm(u), its=its, tol=tol,
             pcrr=hist[-1], true_rel_res=true_rel, N=op.d.N)
    print(f"{name}: N={op.d.N} its={its} pcrr={hist[-1]:.2e} true_rel={true_rel:.2e} "
          f"{time.time() - t0:.0f}s -> {out}")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "bumps_8x8x8_p10")
