"""The many-right-hand-side workload at full size: 16^3 leaves, p = 10
(3,670,016 unknowns per right-hand side), kappa = 60, 6 Gaussian bumps and 64
Gaussian sources, all solved in lock step.

Parity against the oracle's own converged solutions of three of the 64
systems (tests/golden, written by make_golden.py: oracle MGS-GMRES to a
preconditioned residual of 1e-13) at the golden's sampled nodes, to 1e-8:
the lock-step FGMRES solve with the block product on the matrix cores in FP32
(true residual 1e-10 for every right-hand side, so that the solution error,
about cond times the residual, stays below 1e-8) and the lock-step left GMRES
with the separable FP64 J^-1 (preconditioned residual 1e-10).
"""
import os

import numpy as np
import pytest

from paper_2112_02211_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
NAME = "bumps_16x16x16_p10_64rhs"
HERE = os.path.dirname(os.path.abspath(__file__))


def _rhs(prob, ctx):
    xyz = ctx.nodes()
    k = prob.nrhs
    S = torch.empty(k * ctx.N, dtype=torch.complex128, device="cuda")
    for r in range(k):
        S[r * ctx.N:(r + 1) * ctx.N] = torch.from_numpy(P.gaussian_source(prob, xyz, r)).cuda()
    return S, torch.zeros_like(S)


@pytest.mark.parametrize("form", ["fp32_blocks", "separable"])
def test_c4_lock_step_solutions_match_the_oracle(form):
    from paper_2112_02211_amd import hps
    prob = P.workload(NAME)
    g = np.load(os.path.join(HERE, "golden", f"{NAME}_oracle.npz"))
    assert float(np.max(g["pcrr"])) <= 1e-13
    if form == "fp32_blocks":
        ctx = hps.Context.from_problem(prob, block_precs=("fp32",))
        kw = dict(solver="batched", precond_prec="fp32")
    else:
        ctx = hps.Context.from_problem(prob, block_precs=("separable",))
        kw = dict(solver="batched")
    S, T = _rhs(prob, ctx)
    U = torch.zeros_like(S)
    # FP32 blocks make the lock-step solve flexible (the workload's restart for it)
    m = prob.flex_restart if form == "fp32_blocks" else prob.restart
    _, st, ok = ctx.gmres(S, T, tol=1e-10, restart=m, u=U, **kw)
    assert ok and max(st["rhs_rel_res"]) <= 1e-10
    N = ctx.N
    idx = g["idx"]
    for row, r in enumerate(g["rhs_index"]):
        u = U[int(r) * N:(int(r) + 1) * N].cpu().numpy()
        want = g["u"][row]
        err = np.linalg.norm(u[idx] - want) / np.linalg.norm(want)
        assert err < 1e-8, (form, int(r), err)
    ctx.free()
