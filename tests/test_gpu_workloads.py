"""Parity at the full size of the 8x8x8-leaf, p = 10 bump workload (458,752
unknowns), in the launch configuration the benchmark times.

The oracle cannot form every leaf's dense LU quickly at this size, so the
operator and the preconditioner are compared on sampled leaves (a corner, an
edge, a face and an interior leaf and a few seeded ones) where the oracle
computes the rows one leaf at a time; the solve is compared with the oracle's
own converged solution (tests/golden, written by make_golden.py) at 4096
seeded nodes.  Tolerances: FP64 apply 1e-13, FP64 preconditioner 1e-12,
solution 1e-8 relative (GPU GMRES run to 1e-10, two digits below the target).
"""
import os

import numpy as np
import pytest

from oracle import hps_oracle as O
from paper_2112_02211_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
NAME = "bumps_8x8x8_p10"


@pytest.fixture(scope="module")
def c2():
    from paper_2112_02211_amd import hps
    prob = P.workload(NAME)
    ctx = hps.Context.from_problem(prob, block_precs=("fp64", "fp32", "bf16"))
    d = O.make_disc(prob.n_elem, prob.p, prob.kappa, prob.eta, prob.lo, prob.hi)
    xyz = ctx.nodes()
    return prob, ctx, d, xyz


def _sample_leaves(d):
    E1, E2, E3 = d.n_elem
    fixed = [0, E1 - 1, E1 * E2 - 1, d.nl - 1, (E1 * E2 * E3) // 2 + E1 // 2 + E1 * (E2 // 2)]
    rnd = np.random.default_rng(7).choice(d.nl, 3, replace=False).tolist()
    return sorted(set(fixed + rnd))


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_full_size_nodes(c2):
    prob, ctx, d, xyz = c2
    assert np.max(np.abs(xyz - O.node_coords(d))) < 1e-14


def test_full_size_apply_sampled_leaves(c2):
    prob, ctx, d, xyz = c2
    b_nodes = P.bump_field(prob, xyz)
    x = _rand(d.N, 31)
    y = ctx.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    for tau, w in O.apply_elementwise(d, b_nodes, x, _sample_leaves(d)).items():
        got = y[tau * d.n:(tau + 1) * d.n]
        assert np.linalg.norm(got - w) / np.linalg.norm(w) < 1e-13, tau


def test_full_size_precond_sampled_leaves(c2):
    prob, ctx, d, xyz = c2
    b_nodes = P.bump_field(prob, xyz)
    x = _rand(d.N, 32)
    xd = torch.from_numpy(x).cuda()
    z64 = ctx.precond(xd).cpu().numpy()
    z32 = ctx.precond(xd, prec="fp32").cpu().numpy()
    z16 = ctx.precond(xd, prec="bf16").cpu().numpy()
    M = O.Precond(d, b_nodes)
    for tau, w in M.apply_elems(x, _sample_leaves(d)).items():
        sl = slice(tau * d.n, (tau + 1) * d.n)
        nw = np.linalg.norm(w)
        assert np.linalg.norm(z64[sl] - w) / nw < 1e-12, tau
        # reduced-precision blocks (FP32 arithmetic), bounds derived in the design notes
        assert np.linalg.norm(z32[sl] - w) / nw < 2e-6, tau
        assert np.linalg.norm(z16[sl] - w) / nw < 2e-2, tau


def _golden():
    g = np.load(os.path.join(HERE, "golden", f"{NAME}_oracle.npz"))
    assert g["true_rel_res"] < 1e-12
    return g


@pytest.mark.parametrize("solver,prec", [("gmres", "fp64"), ("fgmres", "fp64"),
                                         ("fgmres", "fp32"), ("fgmres", "bf16")])
def test_full_size_solve_matches_oracle(c2, solver, prec):
    prob, ctx, d, xyz = c2
    g = _golden()
    s, t = P.rhs_data(prob, xyz)
    u, st, ok = ctx.gmres(torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda(), tol=1e-10,
                          restart=prob.restart, solver=solver, precond_prec=prec)
    assert ok
    u = u.cpu().numpy()
    err = np.linalg.norm(u[g["idx"]] - g["u"]) / np.linalg.norm(g["u"])
    assert err < 1e-8, err
    assert abs(np.linalg.norm(u) / g["unorm"] - 1.0) < 1e-8


def test_full_size_solve_at_workload_tolerance(c2):
    # the benchmark's own solve (tol 1e-8 on the preconditioned residual)
    prob, ctx, d, xyz = c2
    g = _golden()
    s, t = P.rhs_data(prob, xyz)
    u, st, ok = ctx.gmres(torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda(), tol=prob.tol,
                          restart=prob.restart)
    assert ok and st["true_rel_res"] <= prob.tol
    u = u.cpu().numpy()
    err = np.linalg.norm(u[g["idx"]] - g["u"]) / np.linalg.norm(g["u"])
    assert err < 1e-6, err


def test_full_size_face_system(c2):
    # the face-reduced system with the exact ItI maps at the full size: the
    # operator on sampled leaves (the oracle forms the maps of each sampled
    # leaf's neighbours by dense leaf solves), then the solve against the
    # oracle's converged solution
    prob, ctx, d, xyz = c2
    ctx.iti_build()
    b_nodes = P.bump_field(prob, xyz)
    C = O.c_values(d, b_nodes)
    nb, m = d.nb, d.n1 * d.n1
    f = _rand(d.nl * nb, 33)
    y = ctx.iti_apply(torch.from_numpy(f).cuda()).cpu().numpy()
    for tau in _sample_leaves(d)[:5]:
        want = f[tau * nb:(tau + 1) * nb].copy()
        for face in range(6):
            nbr = O.neighbour(d, tau, face)
            if nbr < 0:
                continue
            Rn = O.iti_map(d, C[nbr * d.n:nbr * d.n + d.ni], homogenized=False)
            fp = O.PARTNER[face]
            want[face * m:(face + 1) * m] += (Rn @ f[nbr * nb:(nbr + 1) * nb])[fp * m:(fp + 1) * m]
        got = y[tau * nb:(tau + 1) * nb]
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-12, tau
    g = _golden()
    s, t = P.rhs_data(prob, xyz)
    u, st, ok = ctx.gmres(torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda(), tol=1e-10,
                          restart=prob.restart, solver="iti")
    assert ok
    u = u.cpu().numpy()
    err = np.linalg.norm(u[g["idx"]] - g["u"]) / np.linalg.norm(g["u"])
    assert err < 1e-8, err
    ctx.trim()
