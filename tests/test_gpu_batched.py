"""Many right-hand sides: the preconditioner's block product as a GEMM on the
matrix cores, and lock-step GMRES over several right-hand sides.

Parity: every column of the batched J^{-1} against the oracle's dense-LU leaf
inverse (FP64 blocks: 1e-12) and against the bounds of the reduced-precision
blocks; batched solves against the oracle's direct solve per right-hand side.
Cases cover several row panels with a ragged last panel (p = 12: 600 face
rows), odd n1 (p = 7, 9: padded BF16 column groups) and more than one
64-column panel (70 right-hand sides).
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


def rand_block(n, k, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n))


@pytest.fixture(scope="module")
def hps_mod():
    from paper_2112_02211_amd import hps
    hps.lib()
    return hps


CASES = [((2, 2, 1), 7, 9.0, 3, 21, 5), ((2, 2, 2), 10, 20.0, 4, 22, 8), ((1, 1, 2), 12, 25.0, 3, 23, 6),
         ((2, 1, 1), 9, 11.0, 2, 24, 70)]


@pytest.mark.parametrize("case", CASES)
def test_batched_precond_columns_match_oracle(hps_mod, case):
    n_elem, p, kappa, nbump, seed, k = case
    prob = P.bump_problem("b", n_elem, p, kappa, nbump, 1, seed, 30, 1e-10)
    ctx = hps_mod.Context.from_problem(prob, block_precs=("fp64", "fp32", "bf16"))
    op = O.build(prob, with_matrix=False)
    X = rand_block(ctx.N, k, seed)
    xd = dev(X.reshape(-1))
    M = O.Precond(op.d, op.b_nodes)
    want = np.stack([M.apply(X[r]) for r in range(k)])
    bounds = {"fp64": 1e-12, "fp32": 2e-6, "bf16": 2e-2}
    for prec, tol in bounds.items():
        Z = host(ctx.precond(xd, prec=prec)).reshape(k, -1)
        for r in range(k):
            e = np.linalg.norm(Z[r] - want[r]) / np.linalg.norm(want[r])
            assert e < tol, (prec, r, e)


def test_batched_precond_equals_single_column_path_fp64(hps_mod):
    # the GEMM path (>= 4 columns) and the single-column path compute the same
    # FP64 product; they differ only in summation order
    prob = P.bump_problem("b", (2, 2, 2), 8, 10.0, 3, 1, 25, 30, 1e-10)
    ctx = hps_mod.Context.from_problem(prob)
    X = rand_block(ctx.N, 6, 5)
    Z = host(ctx.precond(dev(X.reshape(-1)))).reshape(6, -1)
    for r in range(6):
        z1 = host(ctx.precond(dev(X[r])))
        assert np.linalg.norm(Z[r] - z1) / np.linalg.norm(z1) < 1e-14


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_lockstep_solves_match_direct_solves(hps_mod, prec):
    prob = P.bump_problem("lb", (2, 2, 2), 8, 12.0, 4, 6, 26, 30, 1e-10)
    ctx = hps_mod.Context.from_problem(prob, block_precs=("fp64", "fp32", "bf16"))
    op = O.build(prob)
    xyz = ctx.nodes()
    S = np.stack([P.rhs_data(prob, xyz, r)[0] for r in range(6)])
    T = np.zeros_like(S)
    u, st, ok = ctx.gmres(dev(S.reshape(-1)), dev(T.reshape(-1)), tol=1e-11, restart=20,
                          solver="batched", precond_prec=prec)
    assert ok and st["converged"] == 1
    U = host(u).reshape(6, -1)
    for r in range(6):
        b = O.assemble_rhs(op.d, S[r], T[r])
        ud = O.solve_direct(op, b)
        assert np.linalg.norm(U[r] - ud) / np.linalg.norm(ud) < 1e-8, r


def test_lockstep_equals_individual_solves(hps_mod):
    # each right-hand side gives the same solution alone and in the batch
    prob = P.bump_problem("lb2", (2, 2, 2), 8, 12.0, 4, 5, 27, 30, 1e-10)
    ctx = hps_mod.Context.from_problem(prob)
    xyz = ctx.nodes()
    S = np.stack([P.rhs_data(prob, xyz, r)[0] for r in range(5)])
    T = np.zeros_like(S)
    u, st, ok = ctx.gmres(dev(S.reshape(-1)), dev(T.reshape(-1)), tol=1e-11, restart=20,
                          solver="batched")
    U = host(u).reshape(5, -1)
    for r in range(5):
        u1, st1, ok1 = ctx.gmres(dev(S[r]), dev(T[r]), tol=1e-11, restart=20)
        u1 = host(u1)
        assert np.linalg.norm(U[r] - u1) / np.linalg.norm(u1) < 1e-9


def test_kernel_timing_counts_launches(hps_mod):
    # regression: the event-timing API over the single-column and the batched paths
    prob = P.bump_problem("kt", (2, 2, 1), 8, 10.0, 3, 1, 28, 30, 1e-10)
    ctx = hps_mod.Context.from_problem(prob, block_precs=("fp64", "fp32"))
    ctx.set_timing(True)
    ctx.kernel_times(reset=True)
    x1 = dev(rand_block(ctx.N, 1, 1).reshape(-1))
    x6 = dev(rand_block(ctx.N, 6, 2).reshape(-1))
    for _ in range(3):
        ctx.apply(x1)
        ctx.precond(x1)
        ctx.precond(x6, prec="fp32")
    kt = ctx.kernel_times(reset=True)
    ctx.set_timing(False)
    assert kt["apply_launches"] == 3 and kt["precond_launches"] == 6 and kt["gemm_launches"] == 3
    assert kt["apply_ms"] > 0 and kt["precond_ms"] > kt["gemm_ms"] > 0
    assert ctx.kernel_times()["precond_launches"] == 0


@pytest.mark.parametrize("nrhs", [4, 17, 40, 64])
def test_gemm_tile_shapes_give_identical_results(nrhs):
    # every tile shape accumulates the inner index in the same order: J^-1 on a
    # ragged number of right-hand sides is bit-identical whichever shape runs
    from paper_2112_02211_amd import hps
    prob = P.bump_problem("sh", (2, 2, 2), 8, 12.0, 3, 1, 44, 20, 1e-10)
    ctx = hps.Context.from_problem(prob, block_precs=("fp64", "fp32", "bf16"))
    rng = np.random.default_rng(nrhs)
    X = rng.standard_normal(nrhs * ctx.N) + 1j * rng.standard_normal(nrhs * ctx.N)
    x = torch.from_numpy(X).cuda()
    for prec in ("fp64", "fp32", "bf16"):
        outs = []
        for sh in range(len(hps.GEMM_SHAPES)):
            hps.autotune_set(prob.p, prec, nrhs, sh)
            y = ctx.precond(x, prec=prec)
            torch.cuda.synchronize()
            outs.append(y.cpu().numpy())
        hps.autotune_set(prob.p, prec, nrhs, -1)
        for sh, o in enumerate(outs[1:], 1):
            assert np.array_equal(o, outs[0]), (prec, sh)


def test_autotune_picks_and_records_a_shape():
    from paper_2112_02211_amd import hps
    prob = P.bump_problem("at", (3, 3, 2), 8, 12.0, 3, 1, 45, 20, 1e-10)
    ctx = hps.Context.from_problem(prob, block_precs=("fp32",))
    sh = ctx.autotune(12, "fp32", reps=2)
    assert 0 <= sh < len(hps.GEMM_SHAPES)
    assert hps.autotune_get(prob.p, "fp32", 12) == sh
    hps.autotune_set(prob.p, "fp32", 12, -1)
    with pytest.raises(hps.HPSError):
        ctx.autotune(12, "bf16")          # BF16 blocks were not built
