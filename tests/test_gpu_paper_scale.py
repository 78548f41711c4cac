"""Parity at paper scale with shared blocks: 32^3 leaves at n_c = 16 (128,450,560
unknowns, kappa = 96 pi), lambda buckets of spacing 1e-2 kappa^2 (per-leaf
blocks would need 725 GB).  Index arithmetic over 2 GB vectors and 32768
leaves is what this size adds over the small bucket tests.

On sampled leaves (corners, the centre, two leaves inside bumps, seeded others) the oracle computes
the rows of A x leaf by leaf and the bucketed J^{-1} x by a dense LU of the
homogenized leaf matrix at the rounded lambda.  Tolerances as at small size:
apply 1e-13, J^{-1} 1e-12 relative per leaf; rounded lambdas exact (away from
rounding ties).  The separable J^{-1} (no blocks) at every leaf's exact lambda is
checked the same way against the oracle's dense LU at the unrounded lambda.
"""

import numpy as np
import pytest

from oracle import hps_oracle as O
from paper_2112_02211_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAME = "bumps_32x32x32_p16"


@pytest.fixture(scope="module")
def big():
    from paper_2112_02211_amd import hps
    prob = P.workload(NAME)
    ctx = hps.Context.from_problem(prob)
    d = O.make_disc(prob.n_elem, prob.p, prob.kappa, prob.eta, prob.lo, prob.hi)
    E = d.n_elem[0]
    # corners, the centre, the leaves holding two bump centres, seeded others
    ix = np.minimum((np.asarray(prob.bump_centres[:2]) / d.h).astype(int), E - 1)
    in_bumps = {int(i + E * (j + E * k)) for i, j, k in ix}
    leaves = sorted({0, d.nl - 1, (E // 2) * (1 + E + E * E), E - 1} | in_bumps |
                    set(np.random.default_rng(11).choice(d.nl, 2, replace=False).tolist()))
    near = set(leaves)
    for tau in leaves:
        near |= {O.neighbour(d, tau, f) for f in range(6)} - {-1}
    xyz = O.node_coords(d)
    b_nodes = np.zeros(d.N, dtype=np.complex128)      # b where the oracle reads it
    for tau in near:
        sl = slice(tau * d.n, (tau + 1) * d.n)
        b_nodes[sl] = P.bump_field(prob, xyz[sl])
    rng = np.random.default_rng(12)
    x = rng.standard_normal(d.N) + 1j * rng.standard_normal(d.N)
    return prob, ctx, d, leaves, xyz, b_nodes, x


def test_paper_scale_sizes_and_lambdas(big):
    prob, ctx, d, leaves, xyz, b_nodes, x = big
    assert ctx.N == d.N == 128_450_560
    assert 1 < ctx.n_blocks < 1000
    lam = ctx.lambdas()
    C = O.c_values(d, b_nodes)
    h = prob.lambda_bucket * d.kappa * d.kappa
    for tau in leaves:
        Ci = C[tau * d.n:tau * d.n + d.ni]
        exact = O.homog_lambda(d, Ci)[0]
        v = np.array([exact.real, exact.imag]) / h + 0.5
        if np.all(np.abs(v - np.floor(v + 0.5)) > 1e-9):
            assert lam[tau] == O.homog_lambda(d, Ci, delta=prob.lambda_bucket)[0], tau
    nodes = ctx.nodes()
    for tau in leaves:
        sl = slice(tau * d.n, (tau + 1) * d.n)
        assert np.max(np.abs(nodes[sl] - xyz[sl])) < 1e-14


def test_paper_scale_apply_and_bucketed_precond_sampled_leaves(big):
    prob, ctx, d, leaves, xyz, b_nodes, x = big
    xd = torch.from_numpy(x).cuda()
    y = ctx.apply(xd).cpu().numpy()
    for tau, w in O.apply_elementwise(d, b_nodes, x, leaves).items():
        got = y[tau * d.n:(tau + 1) * d.n]
        assert np.linalg.norm(got - w) / np.linalg.norm(w) < 1e-13, tau
    del y
    z = ctx.precond(xd).cpu().numpy()
    M = O.Precond(d, b_nodes, lambda_bucket=prob.lambda_bucket)
    for tau, w in M.apply_elems(x, leaves).items():
        got = z[tau * d.n:(tau + 1) * d.n]
        assert np.linalg.norm(got - w) / np.linalg.norm(w) < 1e-12, tau


def test_paper_scale_separable_precond_sampled_leaves(big):
    # the separable J^-1 at every leaf's exact lambda (no blocks, 0.7 GB of setup
    # instead of 725 GB of per-leaf blocks) against the oracle's dense-LU inverse
    from paper_2112_02211_amd import hps
    prob, _, d, leaves, xyz, b_nodes, x = big
    sctx = hps.Context.from_problem(prob, block_precs=("separable",), lambda_bucket=0.0)
    try:
        lam = sctx.lambdas()
        C = O.c_values(d, b_nodes)
        for tau in leaves:
            assert abs(lam[tau] - O.homog_lambda(d, C[tau * d.n:tau * d.n + d.ni])[0]) <= \
                1e-12 * abs(lam[tau]), tau
        z = sctx.precond(torch.from_numpy(x).cuda()).cpu().numpy()
        M = O.Precond(d, b_nodes)
        for tau, w in M.apply_elems(x, leaves).items():
            got = z[tau * d.n:(tau + 1) * d.n]
            assert np.linalg.norm(got - w) / np.linalg.norm(w) < 1e-12, tau
    finally:
        sctx.free()


def test_paper_scale_short_basis_arnoldi(big):
    # GMRES(8) on 2 GB vectors: every reduction of the delayed-reorthogonalization
    # Arnoldi covers at most 8 basis vectors of at least 2^24 entries, the case
    # whose tiles are split over wavefronts.  After the same 8 and 16 steps the
    # GMRES iterate is the same vector whatever the orthogonalization, so it is
    # compared with classical Gram-Schmidt twice (other kernels throughout).
    from paper_2112_02211_amd import hps
    prob, _, d, leaves, xyz, b_nodes, x = big
    sctx = hps.Context.from_problem(prob, block_precs=("separable",), lambda_bucket=0.0)
    try:
        s = torch.from_numpy(P.gaussian_source(prob, xyz)).cuda()
        prev = None
        for steps in (8, 16):
            out = {}
            for orth in ("dcgs", "cgs2"):
                u, st, ok = sctx.gmres(s, None, tol=1e-12, restart=8, max_iters=steps, orth=orth)
                assert st["iters"] == steps
                out[orth] = (u, st["true_rel_res"])
            ud, uc = out["dcgs"][0], out["cgs2"][0]
            assert float(torch.linalg.norm(ud - uc) / torch.linalg.norm(uc)) < 1e-9
            assert abs(out["dcgs"][1] - out["cgs2"][1]) < 1e-8 * out["cgs2"][1]
            del ud, uc, out
            res = sctx.gmres(s, None, tol=1e-12, restart=8, max_iters=steps)[1]["true_rel_res"]
            assert res < 0.5 and (prev is None or res < 0.8 * prev)
            prev = res
    finally:
        sctx.free()
