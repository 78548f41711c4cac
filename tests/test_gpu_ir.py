"""Iterative refinement with FP32 inner solves (HPS_SOLVER_IR) and its FP32
inner operators, against the oracle.

The inner operators store vectors in complex FP32 and compute in FP64:
J^-1 A x and J^-1 x on FP32 inputs are compared with the oracle's FP64 route
(sparse A, dense-LU J^-1) applied to the same rounded inputs.  Their error is
the rounding of the FP32 stores (the operator image and the face buffer
between the two kernels, and the output), about 1e-7 relative, amplified by
J^-1; the bound 2e-6 leaves an order of magnitude (an index or sign mistake
gives O(1) errors).  The refinement itself recomputes the residual in FP64,
so its solutions must reach the oracle's direct solution (small meshes) and
its converged solution (8^3 leaves, p = 10) as closely as the FP64 solvers.
"""
import os

import numpy as np
import pytest

from oracle import hps_oracle as O
from paper_2112_02211_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))

# n_elem, p, kappa, bumps, seed: ragged meshes, several orders
CASES = [((1, 1, 1), 4, 3.0, 2, 13), ((2, 1, 2), 5, 6.0, 3, 21), ((3, 2, 2), 7, 9.0, 4, 11),
         ((2, 2, 2), 8, 10.0, 3, 12), ((2, 3, 1), 10, 20.0, 5, 14), ((1, 2, 2), 12, 30.0, 3, 15),
         ((1, 1, 2), 13, 22.0, 2, 23), ((2, 1, 1), 16, 25.0, 2, 16)]


def _ctx(case):
    from paper_2112_02211_amd import hps
    n_elem, p, kappa, nbump, seed = case
    prob = P.bump_problem("ir", n_elem, p, kappa, nbump, 1, seed, 30, 1e-10)
    return prob, hps.Context.from_problem(prob, block_precs=("separable",))


@pytest.mark.parametrize("case", CASES)
def test_fp32_inner_operators_match_oracle(case):
    prob, ctx = _ctx(case)
    op = O.build(prob)
    M = O.Precond(op.d, op.b_nodes)
    rng = np.random.default_rng(31)
    x = (rng.standard_normal((2, op.d.N)) + 1j * rng.standard_normal((2, op.d.N))).astype(np.complex64)
    xd = torch.from_numpy(x.reshape(-1)).cuda()
    yl = ctx.op_left_f32(xd).cpu().numpy().reshape(2, -1)
    yp = ctx.precond_f32(xd).cpu().numpy().reshape(2, -1)
    assert yl.dtype == np.complex64
    for k in range(2):
        x64 = x[k].astype(np.complex128)
        want_l = M.apply(op.A @ x64)
        want_p = M.apply(x64)
        el = np.linalg.norm(yl[k] - want_l) / np.linalg.norm(want_l)
        ep = np.linalg.norm(yp[k] - want_p) / np.linalg.norm(want_p)
        assert el < 2e-6 and ep < 2e-6, (el, ep)
        assert el > 1e-9 and ep > 1e-9     # the outputs are FP32 (not an FP64 path)
    ctx.free()


@pytest.mark.parametrize("case", [CASES[2], CASES[3], CASES[4]])
def test_ir_solve_matches_direct_solve(case):
    prob, ctx = _ctx(case)
    op = O.build(prob)
    ud = O.solve_direct(op)
    s, t = P.rhs_data(prob, ctx.nodes())
    for itol in (1e-3, 1e-5):
        u, st, ok = ctx.gmres(torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda(), tol=1e-12,
                              restart=30, solver="ir", inner_tol=itol)
        assert ok and st["true_rel_res"] <= 1e-12 and st["restarts"] >= 2
        assert np.linalg.norm(u.cpu().numpy() - ud) / np.linalg.norm(ud) < 1e-9, itol
    ctx.free()


def test_ir_resumes_from_an_initial_guess():
    prob, ctx = _ctx(CASES[3])
    s, t = P.rhs_data(prob, ctx.nodes())
    sd, td = torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda()
    u, st, ok = ctx.gmres(sd, td, tol=1e-6, restart=30, solver="ir")
    u2, st2, ok2 = ctx.gmres(sd, td, tol=1e-12, restart=30, solver="ir", u=u.clone(), use_x0=True)
    u3, _, _ = ctx.gmres(sd, td, tol=1e-12, restart=30, solver="ir")
    assert ok and ok2 and st2["true_rel_res"] <= 1e-12
    assert torch.linalg.norm(u2 - u3) / torch.linalg.norm(u3) < 1e-9
    ctx.free()


def test_ir_full_size_against_the_oracle_solution():
    from paper_2112_02211_amd import hps
    name = "bumps_8x8x8_p10"
    prob = P.workload(name)
    ctx = hps.Context.from_problem(prob, block_precs=("separable",))
    s, t = P.rhs_data(prob, ctx.nodes())
    u, st, ok = ctx.gmres(torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda(), tol=1e-10,
                          restart=prob.restart, solver="ir")
    g = np.load(os.path.join(HERE, "golden", f"{name}_oracle.npz"))
    idx = g["idx"]
    err = np.linalg.norm(u.cpu().numpy()[idx] - g["u"]) / np.linalg.norm(g["u"])
    assert ok and st["true_rel_res"] <= 1e-10 and err < 1e-8, err
    ctx.free()


def test_ir_option_errors():
    from paper_2112_02211_amd import hps
    prob = P.workload("plane_2x2x2_p8")
    dense = hps.Context.from_problem(prob)
    s, t = P.rhs_data(prob, dense.nodes())
    sd, td = torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda()
    with pytest.raises(hps.HPSError, match="separable"):
        dense.gmres(sd, td, solver="ir")
    x = torch.zeros(dense.N, dtype=torch.complex64, device="cuda")
    with pytest.raises(hps.HPSError):
        dense.op_left_f32(x)
    sep = hps.Context.from_problem(prob, block_precs=("separable",))
    with pytest.raises(hps.HPSError, match="restart"):
        sep.gmres(sd, td, solver="ir", restart=100)
    with pytest.raises(hps.HPSError, match="inner_tol"):
        sep.gmres(sd, td, solver="ir", inner_tol=2.0)
    dense.free()
    sep.free()
