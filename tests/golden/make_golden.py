"""Writes the oracle's reference solutions used by the GPU parity tests and bench.py.

Calls only the CPU oracle (oracle/) and the seeded problem generator.  For each
workload it solves A u = b with the oracle's MGS-GMRES and J^{-1} (dense LU
leaf solves) to a preconditioned residual of 1e-13, then stores u at seeded
sample indices together with ||u||, the true relative residual and the
iteration count:

    python tests/golden/make_golden.py bumps_8x8x8_p10
    python tests/golden/make_golden.py bumps_16x16x16_p12 --bucket 1e-2 --nsamp 8192
    python tests/golden/make_golden.py bumps_16x16x16_p10_64rhs --bucket 1e-2 --rhs 0,31,63 --restart 50
    python tests/golden/make_golden.py request_stream --request 39 --bucket 1e-2

--bucket delta shares one LU factorization among the leaves whose homogenized
lambda round to the same point of a grid of spacing delta kappa^2 (the oracle's
lambda buckets).  That changes only the preconditioner, so GMRES converges to
the same u = A^{-1} b; it keeps the factorizations of 4096 leaves of 1600
unknowns within host memory.  With several --rhs indices (sources of the
workload) the file holds one row of samples per source.  --request RID takes
request RID of the serving stream (problems.request_stream, seed 5) instead
of a named workload and writes request_stream_r<RID>_oracle.npz.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import hps_oracle as O  # noqa: E402
from paper_2112_02211_amd import problems as P  # noqa: E402


def solve_one(prob, op, M, which, tol, restart, t0):
    if which != 0:
        s = P.gaussian_source(prob, op.xyz, which)
        rhs = O.assemble_rhs(op.d, s, np.zeros(op.d.N, dtype=np.complex128))
    else:
        rhs = op.rhs
    step = [0]

    def prec(v):
        step[0] += 1
        if step[0] % 50 == 0:
            print(f"  rhs {which}: {step[0]} preconditioner applications, "
                  f"{time.time() - t0:.0f}s", flush=True)
        return M.apply(v)

    u, its, hist = O.gmres_left(lambda v: op.A @ v, prec, rhs, tol=tol, restart=restart,
                                maxit=20000)
    r = rhs - op.A @ u
    true_rel = float(np.linalg.norm(r) / np.linalg.norm(rhs))
    return u, its, hist[-1], true_rel


def main(name: str, tol: float = 1e-13, nsamp: int = 4096, bucket: float = 0.0,
         rhs=(0,), restart=None, request=None):
    if request is not None:
        prob = P.request_stream(request + 1, rate=1.0, seed=5)[request].prob
        name = f"request_stream_r{request}"
    else:
        prob = P.workload(name)
    t0 = time.time()
    op = O.build(prob)
    print(f"{name}: N={op.d.N} nnz={op.A.nnz} built {time.time() - t0:.0f}s", flush=True)
    M = O.Precond(op.d, op.b_nodes, lambda_bucket=bucket)
    m = prob.restart if restart is None else restart
    idx = np.sort(np.random.default_rng(123).choice(op.d.N, size=min(nsamp, op.d.N), replace=False))
    us, unorms, itss, pcrrs, trues = [], [], [], [], []
    for which in rhs:
        u, its, pcrr, true_rel = solve_one(prob, op, M, which, tol, m, t0)
        us.append(u[idx])
        unorms.append(np.linalg.norm(u))
        itss.append(its)
        pcrrs.append(pcrr)
        trues.append(true_rel)
        print(f"{name} rhs {which}: its={its} pcrr={pcrr:.2e} true_rel={true_rel:.2e} "
              f"{time.time() - t0:.0f}s", flush=True)
    out = os.path.join(HERE, f"{name}_oracle.npz")
    if len(rhs) == 1:
        np.savez(out, idx=idx, u=us[0], unorm=unorms[0], its=itss[0], tol=tol, pcrr=pcrrs[0],
                 true_rel_res=trues[0], N=op.d.N, lambda_bucket=bucket, restart=m)
    else:
        np.savez(out, idx=idx, u=np.stack(us), unorm=np.array(unorms), its=np.array(itss),
                 tol=tol, pcrr=np.array(pcrrs), true_rel_res=np.array(trues), N=op.d.N,
                 rhs_index=np.array(rhs), lambda_bucket=bucket, restart=m)
    print(f"{name}: {time.time() - t0:.0f}s -> {out}", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("name", nargs="?", default="bumps_8x8x8_p10")
    ap.add_argument("--tol", type=float, default=1e-13)
    ap.add_argument("--nsamp", type=int, default=4096)
    ap.add_argument("--bucket", type=float, default=0.0)
    ap.add_argument("--rhs", default="0")
    ap.add_argument("--restart", type=int, default=None)
    ap.add_argument("--request", type=int, default=None)
    a = ap.parse_args()
    main(a.name, a.tol, a.nsamp, a.bucket, tuple(int(v) for v in a.rhs.split(",")), a.restart, a.request)
