"""Block GMRES (all right-hand sides in one block Krylov space) on the GPU.

The solutions of several right-hand sides are checked against the oracle's
direct solves (1e-9, solves to PCRR 1e-11) with the stored FP64 blocks and
with the separable J^-1; one right-hand side reduces to GMRES (the same
iterate up to rounding); the block space needs no more block steps than the
lock-step solver needs steps; dependent right-hand sides are reported as a
breakdown; wrong options are rejected.
"""
import numpy as np
import pytest

from oracle import hps_oracle as O
from paper_2112_02211_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def hps_mod():
    from paper_2112_02211_amd import hps
    hps.lib()
    return hps


def _problem(nrhs, seed=31, n_elem=(2, 2, 2), p=8, kappa=14.0):
    return P.bump_problem("bg", n_elem, p, kappa, 4, nrhs, seed, 20, 1e-11)


def _rhs(prob, xyz, nrhs):
    S = np.concatenate([P.rhs_data(prob, xyz, r)[0] for r in range(nrhs)])
    return S, np.zeros_like(S)


@pytest.mark.parametrize("precs", [("fp64",), ("separable",)])
def test_block_gmres_matches_direct_solves(hps_mod, precs):
    k = 5
    prob = _problem(k)
    ctx = hps_mod.Context.from_problem(prob, block_precs=precs)
    op = O.build(prob)
    S, T = _rhs(prob, ctx.nodes(), k)
    u, st, ok = ctx.gmres(dev(S), dev(T), tol=1e-11, restart=20, solver="block_gmres")
    assert ok and st["true_rel_res"] <= 1e-11
    U = host(u).reshape(k, -1)
    for r in range(k):
        rhs = O.assemble_rhs(op.d, S[r * op.d.N:(r + 1) * op.d.N], np.zeros(op.d.N))
        assert rel(U[r], O.solve_direct(op, rhs)) < 1e-9, r
    # lock-step: one Krylov space per right-hand side; the block space takes
    # no more block steps than that takes steps
    u2, st2, ok2 = ctx.gmres(dev(S), dev(T), tol=1e-11, restart=20, solver="batched")
    assert ok2 and st["iters"] <= st2["iters"]
    assert rel(host(u), host(u2)) < 1e-9


def test_block_gmres_restarts_and_ragged_mesh(hps_mod):
    # a restart length well below the step count, odd p, unequal leaf counts
    k = 3
    prob = P.bump_problem("bgr", (3, 2, 1), 7, 11.0, 4, k, 12, 4, 1e-11)
    ctx = hps_mod.Context.from_problem(prob, block_precs=("separable",))
    op = O.build(prob)
    S, T = _rhs(prob, ctx.nodes(), k)
    u, st, ok = ctx.gmres(dev(S), dev(T), tol=1e-11, restart=4, solver="block_gmres")
    assert ok and st["restarts"] > 1
    U = host(u).reshape(k, -1)
    for r in range(k):
        rhs = O.assemble_rhs(op.d, S[r * op.d.N:(r + 1) * op.d.N], np.zeros(op.d.N))
        assert rel(U[r], O.solve_direct(op, rhs)) < 1e-9, r


def test_block_gmres_one_rhs_is_gmres(hps_mod):
    prob = _problem(1, seed=33)
    ctx = hps_mod.Context.from_problem(prob)
    s, t = P.rhs_data(prob, ctx.nodes())
    ub, stb, okb = ctx.gmres(dev(s), dev(t), tol=1e-11, restart=20, solver="block_gmres")
    ug, stg, okg = ctx.gmres(dev(s), dev(t), tol=1e-11, restart=20)
    assert okb and okg
    # the delayed-reorthogonalization GMRES sees step j's residual one step
    # late and polls it one step after that, so it may take two more steps
    assert 0 <= stg["iters"] - stb["iters"] <= 2
    assert rel(host(ub), host(ug)) < 1e-9


def test_block_gmres_dependent_rhs_and_bad_options(hps_mod):
    prob = _problem(2, seed=34)
    ctx = hps_mod.Context.from_problem(prob, block_precs=("fp64", "bf16"))
    s, t = P.rhs_data(prob, ctx.nodes())
    S = np.concatenate([s, s])
    with pytest.raises(hps_mod.HPSError) as e:
        ctx.gmres(dev(S), dev(np.zeros_like(S)), tol=1e-10, restart=10, solver="block_gmres")
    assert e.value.code == hps_mod.HPS_ERR_BREAKDOWN
    S2, T2 = _rhs(prob, ctx.nodes(), 2)
    with pytest.raises(hps_mod.HPSError):
        ctx.gmres(dev(S2), dev(T2), solver="block_gmres", precond_prec="bf16")
    grp = hps_mod.Context.group([_problem(1, seed=35), _problem(1, seed=36)])
    with pytest.raises(hps_mod.HPSError):
        grp.gmres(dev(S2), dev(T2), solver="block_gmres")


def test_block_gmres_long_vectors_split_products(hps_mod):
    # 1.55 million unknowns: the block products V^H W and the Gram matrices
    # run split over chunks of the vector length (partials summed); the block
    # solve agrees with the lock-step one
    k = 3
    prob = P.bump_problem("bgl", (12, 12, 12), 10, 30.0, 6, k, 41, 30, 1e-10)
    ctx = hps_mod.Context.from_problem(prob, block_precs=("separable",))
    assert ctx.N > 256 * 4096
    S, T = _rhs(prob, ctx.nodes(), k)
    ub, stb, okb = ctx.gmres(dev(S), dev(T), tol=1e-10, restart=30, solver="block_gmres")
    ul, stl, okl = ctx.gmres(dev(S), dev(T), tol=1e-10, restart=30, solver="batched")
    assert okb and okl and stb["true_rel_res"] <= 1e-10
    Ub, Ul = host(ub).reshape(k, -1), host(ul).reshape(k, -1)
    for r in range(k):
        assert rel(Ub[r], Ul[r]) < 1e-7, r


def test_block_gmres_resumes_from_an_initial_guess(hps_mod):
    # a bounded first call (not converged), then the same solve resumed from
    # its iterate: the result matches the direct solves
    k = 4
    prob = _problem(k, seed=37)
    ctx = hps_mod.Context.from_problem(prob, block_precs=("separable",))
    op = O.build(prob)
    S, T = _rhs(prob, ctx.nodes(), k)
    u, st, ok = ctx.gmres(dev(S), dev(T), tol=1e-11, restart=6, max_iters=6, solver="block_gmres")
    assert not ok and st["iters"] == 6
    u, st2, ok2 = ctx.gmres(dev(S), dev(T), tol=1e-11, restart=6, u=u, use_x0=True, solver="block_gmres")
    assert ok2 and st2["true_rel_res"] <= 1e-11
    U = host(u).reshape(k, -1)
    for r in range(k):
        rhs = O.assemble_rhs(op.d, S[r * op.d.N:(r + 1) * op.d.N], np.zeros(op.d.N))
        assert rel(U[r], O.solve_direct(op, rhs)) < 1e-9, r
