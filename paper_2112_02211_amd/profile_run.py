"""Fixed launch sequence for hardware-counter runs of the hot-path kernels.

    python -m paper_2112_02211_amd.profile_run [--workload NAME] [--launches 4]

Sets up the workload (FP64, FP32 and BF16 blocks), then launches: the
operator apply, the preconditioner in each block precision, and a plain
elementwise kernel over --copy-mib MiB (dst = 2 src: each byte read once and
written once; the known-size reference that calibrates the FETCH_SIZE /
WRITE_SIZE counters), each --launches times.  Prints one line per phase with its wall time.
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="bumps_8x8x8_p10")
    ap.add_argument("--launches", type=int, default=4)
    ap.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args()
    import torch
    from paper_2112_02211_amd import hps, problems as P

    prob = P.workload(a.workload)
    ctx = hps.Context.from_problem(prob, block_precs=("fp64", "fp32", "bf16"))
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.standard_normal(ctx.N) + 1j * rng.standard_normal(ctx.N)).cuda()
    y = torch.empty_like(x)
    phases = [("apply", lambda: ctx.apply(x, y))] + \
             [(f"precond_{q}", (lambda q=q: ctx.precond(x, y, prec=q))) for q in ("fp64", "fp32", "bf16")]
    n = a.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    phases.append(("copy", lambda: torch.mul(src, 2.0, out=dst)))
    for name, fn in phases:
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.launches):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.launches
        print(f"{name}: {dt * 1e3:.4f} ms per launch", flush=True)
    print(f"copy bytes read = written = {n * 4}")


if __name__ == "__main__":
    main()
