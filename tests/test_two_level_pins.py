"""Pins of the two-level preconditioner prototype (oracle/two_level.py): the
coarse-grid correction with block-Jacobi smoothing that the paper's concluding
section proposes.  Each pin checks the prototype against a fact of
interpolation or linear algebra, not against its own formulas.
"""
import numpy as np
import pytest

from oracle import hps_oracle as O
from oracle import two_level as T
from paper_2112_02211_amd import problems as P


@pytest.mark.parametrize("pf, pt", [(6, 10), (8, 12), (10, 6)])
def test_lagrange_interpolation_is_exact_on_polynomials(pf, pt):
    src, dst = T.interior_nodes(pf), T.interior_nodes(pt)
    L = T.lagrange_matrix(src, dst)
    for k in range(pf - 2):      # degree <= (p_from - 2) - 1
        assert np.max(np.abs(L @ src ** k - dst ** k)) < 1e-12
    # and not beyond (so the pin is not vacuous)
    k = pf - 2
    assert np.max(np.abs(L @ src ** k - dst ** k)) > 1e-6


def test_transfer_at_equal_order_is_the_identity():
    assert np.max(np.abs(T.leaf_transfer(8, 8) - np.eye(6 * 6 * 12))) < 1e-13


@pytest.mark.parametrize("pc, pf", [(4, 8), (6, 10)])
def test_restriction_after_prolongation_is_the_identity(pc, pf):
    R, Pm = T.transfer(3, pf, pc), T.transfer(3, pc, pf)
    assert abs(R @ Pm - np.eye(R.shape[0])).max() < 1e-12


@pytest.mark.parametrize("pc, pf", [(5, 8), (6, 10)])
def test_prolongation_reproduces_a_smooth_field_at_the_fine_nodes(pc, pf):
    # a polynomial of degree p_c - 3 in each variable (not symmetric in x, y, z,
    # so a misordered Kronecker factor fails) sampled at the coarse nodes of each
    # discretization's own node table
    prob = P.plane_wave_problem((2, 1, 2), pf)
    dc = O.make_disc(prob.n_elem, pc, prob.kappa, prob.eta, prob.lo, prob.hi)
    df = O.make_disc(prob.n_elem, pf, prob.kappa, prob.eta, prob.lo, prob.hi)
    deg = pc - 3
    rng = np.random.default_rng(3)
    coef = rng.standard_normal((deg + 1, deg + 1, deg + 1))

    def u(xyz):
        x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
        return sum(coef[a, b, c] * x ** a * y ** b * z ** c
                   for a in range(deg + 1) for b in range(deg + 1) for c in range(deg + 1))

    Pm = T.transfer(df.nl, pc, pf)
    uc, uf = u(O.node_coords(dc)), u(O.node_coords(df))
    assert np.max(np.abs(Pm @ uc - uf)) < 1e-11 * np.max(np.abs(uf))


def test_two_level_at_equal_order_is_the_exact_inverse():
    prob = P.bump_problem("tl", (2, 2, 1), 6, 8.0, 3, 1, 4, 30, 1e-10)
    tl = T.TwoLevel(prob, prob.p)
    x = np.random.default_rng(7).standard_normal(tl.op.d.N) + 0j
    assert np.linalg.norm(tl.apply(tl.op.A @ x) - x) < 1e-10 * np.linalg.norm(x)


def test_two_level_gmres_reaches_the_direct_solution():
    prob = P.bump_problem("tl", (2, 2, 2), 8, 12.0, 4, 1, 5, 30, 1e-10)
    tl = T.TwoLevel(prob, 5)
    op = tl.op
    x, its, _ = O.gmres_left(lambda v: op.A @ v, tl.apply, op.rhs, tol=1e-12, restart=30)
    ud = O.solve_direct(op)
    assert np.linalg.norm(x - ud) < 1e-9 * np.linalg.norm(ud)
