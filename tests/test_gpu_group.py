"""Operator groups: several problems on one mesh with their own wave number,
impedance parameter and medium, built into one context so that every launch
of the solve covers all of them ([op][N] vectors, one right-hand side per
operator).

Each operator's part of the group's A x, J^{-1} x and J^{-1} A x is bit-equal
to what a context of that problem alone computes (the same kernels read that
operator's C, eta, lambda and blocks); lock-step group solves match the
separate solves (1e-9) and the oracle's direct solves (1e-9).
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


def _probs(n_elem=(2, 2, 2), p=8, kappas=(10.0, 13.0, 16.5), seeds=(31, 32, 33)):
    return [P.bump_problem(f"g{i}", n_elem, p, k, 4, 1, s, 30, 1e-10)
            for i, (k, s) in enumerate(zip(kappas, seeds))]


@pytest.mark.parametrize("shape", [((2, 2, 2), 8), ((3, 2, 1), 10), ((1, 1, 2), 5)])
def test_group_operators_equal_separate_contexts(hps_mod, shape):
    n_elem, p = shape
    probs = _probs(n_elem, p)
    grp = hps_mod.Context.group(probs, block_precs=("fp64", "bf16"))
    one = [hps_mod.Context.from_problem(pr, block_precs=("fp64", "bf16")) for pr in probs]
    assert grp.n_ops == 3 and grp.N == one[0].N
    N = grp.N
    rng = np.random.default_rng(5)
    X = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    xd = dev(X.reshape(-1))
    outs = {"apply": host(grp.apply(xd)), "precond": host(grp.precond(xd)),
            "op_left": host(grp.op_left(xd)), "bf16": host(grp.precond(xd, prec="bf16"))}
    for k in range(3):
        xk = dev(X[k])
        want = {"apply": host(one[k].apply(xk)), "precond": host(one[k].precond(xk)),
                "op_left": host(one[k].op_left(xk)), "bf16": host(one[k].precond(xk, prec="bf16"))}
        for name, got in outs.items():
            assert np.array_equal(got[k * N:(k + 1) * N], want[name]), (name, k)
    assert np.array_equal(grp.lambdas(), np.concatenate([c.lambdas() for c in one]))


@pytest.mark.parametrize("solver,prec", [("gmres", "fp64"), ("fgmres", "bf16")])
def test_group_solves_match_separate_solves_and_oracle(hps_mod, solver, prec):
    probs = _probs()
    grp = hps_mod.Context.group(probs, block_precs=("fp64", "bf16"))
    xyz = grp.nodes()
    S = np.concatenate([P.rhs_data(pr, xyz)[0] for pr in probs])
    T = np.zeros_like(S)
    U, st, ok = grp.gmres(dev(S), dev(T), tol=1e-11, restart=30, solver=solver, precond_prec=prec)
    assert ok and len(st["rhs_rel_res"]) == 3
    U = host(U).reshape(3, -1)
    N = grp.N
    for k, pr in enumerate(probs):
        ck = hps_mod.Context.from_problem(pr, block_precs=("fp64", "bf16"))
        uk, _, okk = ck.gmres(dev(S[k * N:(k + 1) * N]), dev(T[k * N:(k + 1) * N]), tol=1e-11, restart=30,
                              solver=solver, precond_prec=prec)
        assert okk
        assert rel(U[k], host(uk)) < 1e-9, k
    op = O.build(probs[1])
    assert rel(U[1], O.solve_direct(op, O.assemble_rhs(op.d, S[N:2 * N], T[N:2 * N]))) < 1e-9


def test_group_with_complex_and_zero_media(hps_mod):
    # one absorbing medium makes C complex for the whole group; a plane-wave
    # problem (b = 0) in the same group
    probs = _probs()
    probs[0].bump_amps = probs[0].bump_amps + 0.3j
    pw = P.plane_wave_problem((2, 2, 2), 8, 11.0)
    probs = probs + [pw]
    grp = hps_mod.Context.group(probs)
    one = [hps_mod.Context.from_problem(pr) for pr in probs]
    N = grp.N
    X = np.random.default_rng(6).standard_normal((4, N)) + 0j
    Y = host(grp.apply(dev(X.reshape(-1)))).reshape(4, -1)
    Z = host(grp.precond(dev(X.reshape(-1)))).reshape(4, -1)
    for k in range(4):
        assert rel(Y[k], host(one[k].apply(dev(X[k])))) < 1e-15, k
        assert rel(Z[k], host(one[k].precond(dev(X[k])))) < 1e-15, k


def test_group_rejects_wrong_right_hand_side_counts(hps_mod):
    probs = _probs()
    grp = hps_mod.Context.group(probs)
    x = dev(np.zeros(grp.N, dtype=np.complex128))
    with pytest.raises(hps_mod.HPSError):
        grp.apply(x)
    with pytest.raises(hps_mod.HPSError):
        grp.precond(x)
    with pytest.raises(hps_mod.HPSError):
        grp.gmres(x, x)
    with pytest.raises(hps_mod.HPSError):
        grp.iti_build()
    with pytest.raises(ValueError):
        hps_mod.Context.group([probs[0], P.bump_problem("x", (2, 2, 1), 8, 10.0, 4, 1, 3, 30, 1e-10)])
