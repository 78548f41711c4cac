"""The separable form of the homogenized leaf solve, on the CPU: the table the
library builds on the host (hps_separable_table: the complex eigendecomposition
of the line operator and the 2 x 2 face system of a line) and the sequence of
steps the GPU kernel applies with it, replayed here in NumPy, against the
oracle's dense LU of the whole homogenized leaf matrix (eq. (block_pc)).

What this pins: the derivation (the homogenized leaf matrix is separable along
grid lines including its impedance rows, so its inverse is a 2 x 2 elimination
per line plus a complex fast diagonalization) and the host tables, for every
p = 4 ... 16 with real and complex lambda.  Tolerance 1e-12 relative at
moderate kappa h (the dense LU itself carries cond(A) * 1e-16, cond(A) <= 1e5
here).
"""
import ctypes

import numpy as np
import pytest

from oracle import hps_oracle as O
from paper_2112_02211_amd import hps


def _line_operator(d):
    """Lt and Fi from the oracle's differentiation matrices (independent of the library)."""
    p = d.p
    D, D2 = O.phys_tables(d)
    e = p - 1
    Fbb = np.array([[-D[0, 0] + 1j * d.eta, -D[0, e]], [D[e, 0], D[e, e] + 1j * d.eta]])
    Fi = np.linalg.inv(Fbb)
    Fbi = np.vstack([-D[0, 1:-1], D[e, 1:-1]])
    Lt = D2[1:-1, 1:-1] - D2[1:-1][:, [0, e]] @ Fi @ Fbi
    return Lt, Fi


def _separable_solve(d, lam, x, table, split=False):
    """The kernel's steps: g = Fi [x_lo, x_hi] per line; r = x_i - A_ib g;
    u_i = (Vc x Vc x Vc) diag(1 / (-Ec_sum - lambda)) (Wc x Wc x Wc) r;
    u_b = g - Fi Fbi1 u_line.  Leaf layout [interior, x fastest | faces 1..6]."""
    Wc, Vc, Ec, Fi = table
    p, n1 = d.p, d.n1
    L, NI = n1 * n1, n1 ** 3
    D, D2 = O.phys_tables(d)
    Dlo, Dhi = D[0, 1:-1], D[p - 1, 1:-1]
    C0, C1 = D2[1:-1, 0], D2[1:-1, p - 1]
    G = x[NI:].reshape(6, n1, n1).copy()           # [face][b][a], position a + n1 b
    for ax in range(3):
        lo, hi = G[2 * ax].copy(), G[2 * ax + 1].copy()
        G[2 * ax] = Fi[0, 0] * lo + Fi[0, 1] * hi
        G[2 * ax + 1] = Fi[1, 0] * lo + Fi[1, 1] * hi
    T = x[:NI].reshape(n1, n1, n1).copy()          # [k][j][i]
    T += C0[None, None, :] * G[0][:, :, None] + C1[None, None, :] * G[1][:, :, None]
    T += C0[None, :, None] * G[2][:, None, :] + C1[None, :, None] * G[3][:, None, :]
    T += C0[:, None, None] * G[4][None, :, :] + C1[:, None, None] * G[5][None, :, :]

    def modes(M, A):
        A = np.einsum("oi,kji->kjo", M, A)
        A = np.einsum("oj,kji->koi", M, A)
        return np.einsum("ok,kji->oji", M, A)

    Es = Ec[:, None, None] + Ec[None, :, None] + Ec[None, None, :]
    if split:
        U = _split_modes(Vc, _split_modes(Wc, T, False) / (-Es - lam), True)
    else:
        U = modes(Vc, modes(Wc, T) / (-Es - lam))
    out = np.zeros(d.n, dtype=complex)
    out[:NI] = U.reshape(-1)
    # lines along x through (j, k): U[k, j, :]; along y through (i, k): U[k, :, i]; along z: U[:, j, i]
    lines = (U, np.transpose(U, (0, 2, 1)), np.transpose(U, (1, 2, 0)))
    for ax in range(3):
        slo, shi = -(lines[ax] @ Dlo), lines[ax] @ Dhi       # [b][a]
        out[NI + 2 * ax * L:NI + (2 * ax + 1) * L] = (G[2 * ax] - (Fi[0, 0] * slo + Fi[0, 1] * shi)).reshape(-1)
        out[NI + (2 * ax + 1) * L:NI + (2 * ax + 2) * L] = (G[2 * ax + 1] - (Fi[1, 0] * slo + Fi[1, 1] * shi)).reshape(-1)
    return out


def _split_modes(M, A, inverse):
    """The even / odd mode products of the p = 12 kernel along the three axes
    of A ([k][j][i]), with modes 0 .. H-1 even and H .. n1-1 odd.  Forward
    (M = Wc): fold each line, v_i + v_{n1-1-i} for the even modes and v_i -
    v_{n1-1-i} for the odd ones, and take H terms per output.  Inverse (M = Vc):
    A_i from the even modes at position i, B_i from the odd modes at n1-1-i,
    then the butterflies (A + B, A - B) along all three axes."""
    n1 = M.shape[0]
    H = n1 // 2
    for ax in (2, 1, 0):       # x, y, z in turn (A is [k][j][i])
        X = np.moveaxis(A, ax, -1)
        out = np.empty_like(X)
        if not inverse:
            lo, hi = X[..., :H], X[..., ::-1][..., :H]
            out[..., :H] = (lo + hi) @ M[:H, :H].T
            out[..., H:] = (lo - hi) @ M[H:, :H].T
        else:
            out[..., :H] = X[..., :H] @ M[:H, :H].T
            out[..., ::-1][..., :H] = X[..., H:] @ M[:H, H:].T
        A = np.moveaxis(out, -1, ax)
    if inverse:
        for ax in range(3):
            X = np.moveaxis(A, ax, -1)
            a, b = X[..., :H].copy(), X[..., ::-1][..., :H].copy()
            X[..., :H] = a + b
            X[..., ::-1][..., :H] = a - b
    return A


@pytest.mark.parametrize("p", [4, 6, 8, 10, 12, 14, 16])
def test_even_odd_mode_products_equal_the_full_ones(p):
    # the kernel's even / odd form (fold, half products, deferred butterflies)
    # against the plain fast diagonalization on the same table, and with it
    # against the oracle's dense LU of the leaf matrix
    rng = np.random.default_rng(100 + p)
    kappa, h = 40.0, 0.125
    d = O.make_disc((1, 1, 1), p, kappa, kappa, (0, 0, 0), (h, h, h))
    Wc, Vc, Ec, Fi = hps.separable_table(p, h, kappa)
    n1 = p - 2
    r = rng.standard_normal((n1, n1, n1)) + 1j * rng.standard_normal((n1, n1, n1))
    lam = kappa ** 2 * (0.7 + 0.05j)
    Es = Ec[:, None, None] + Ec[None, :, None] + Ec[None, None, :]

    def full(M, A):
        A = np.einsum("oi,kji->kjo", M, A)
        A = np.einsum("oj,kji->koi", M, A)
        return np.einsum("ok,kji->oji", M, A)

    want = full(Vc, full(Wc, r) / (-Es - lam))
    got = _split_modes(Vc, _split_modes(Wc, r, False) / (-Es - lam), True)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-13
    # and the whole leaf solve with it
    ops = O.local_ops(d)
    A, _ = O.leaf_matrices(d, np.full(d.ni, lam), ops)
    x = rng.standard_normal(d.n) + 1j * rng.standard_normal(d.n)
    sol = np.linalg.solve(A, x)
    out = _separable_solve(d, lam, x, (Wc, Vc, Ec, Fi), split=True)
    assert np.linalg.norm(out - sol) / np.linalg.norm(sol) < 1e-12


@pytest.mark.parametrize("p", list(range(4, 17)))
def test_table_is_an_eigendecomposition_of_the_line_operator(p):
    kappa, h = 40.0, 0.125
    d = O.make_disc((1, 1, 1), p, kappa, kappa, (0, 0, 0), (h, h, h))
    Wc, Vc, Ec, Fi = hps.separable_table(p, h, kappa)
    Lt, Fi_o = _line_operator(d)
    n1 = p - 2
    assert np.max(np.abs(Wc @ Vc - np.eye(n1))) < 1e-12
    assert np.max(np.abs(Vc @ np.diag(Ec) @ Wc - Lt)) < 1e-11 * np.max(np.abs(Lt))
    assert np.max(np.abs(Fi - Fi_o)) < 1e-13 * np.max(np.abs(Fi_o))
    # the spectrum is that of Lt
    ev = np.linalg.eigvals(Lt)
    ev = ev[np.lexsort((ev.imag, ev.real))]
    got = Ec[np.lexsort((Ec.imag, Ec.real))]
    assert np.max(np.abs(got - ev)) < 1e-10 * np.max(np.abs(ev))
    if n1 % 2 == 0:
        # Lt commutes with the flip of a line (its two faces mirror each other):
        # modes 0 .. n1/2-1 are even, the rest odd, exactly (the p = 12 kernel
        # takes half the terms of each mode product from this)
        H, J = n1 // 2, np.eye(n1)[::-1]
        assert np.max(np.abs(J @ Lt @ J - Lt)) < 1e-13 * np.max(np.abs(Lt))
        par = np.r_[np.ones(H), -np.ones(H)]
        assert np.array_equal(J @ Vc, Vc * par)
        assert np.array_equal(Wc @ J, par[:, None] * Wc)
    else:
        assert np.array_equal(Ec, Ec[np.lexsort((Ec.imag, Ec.real))])


@pytest.mark.parametrize("p", list(range(4, 17)))
def test_separable_steps_invert_the_homogenized_leaf_matrix(p):
    rng = np.random.default_rng(p)
    for kappa, h in ((10.0, 0.5), (40.0, 0.125)):
        d = O.make_disc((1, 1, 1), p, kappa, kappa, (0, 0, 0), (h, h, h))
        table = hps.separable_table(p, h, kappa)
        ops = O.local_ops(d)
        for lam in (0.9 * kappa ** 2, kappa ** 2 * (0.7 + 0.05j)):
            A, _ = O.leaf_matrices(d, np.full(d.ni, lam), ops)
            x = rng.standard_normal(d.n) + 1j * rng.standard_normal(d.n)
            want = np.linalg.solve(A, x)
            got = _separable_solve(d, lam, x, table)
            assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-12, (kappa, lam)


def test_separable_table_errors():
    out = (ctypes.c_double * 8)()
    L = hps.lib()
    assert L.hps_separable_table(3, 0.1, 1.0, out) == hps.HPS_ERR_UNSUPPORTED
    assert L.hps_separable_table(8, 0.1, 0.0, out) == hps.HPS_ERR_ARG
    assert L.hps_separable_table(8, -0.1, 1.0, out) == hps.HPS_ERR_ARG
    assert L.hps_separable_table(8, 0.1, 1.0, None) == hps.HPS_ERR_ARG


@pytest.mark.parametrize("p", [4, 7, 10])
def test_leaf_matrix_couples_along_grid_lines_only(p):
    # the structure the separable form rests on, read off the oracle's leaf
    # matrix: an interior row couples only nodes on the three grid lines through
    # its node; a face row (eq. (flux) plus i eta) only nodes on the normal line
    # of its face node, which ends at a node of the opposite face
    d = O.make_disc((1, 1, 1), p, 10.0, 10.0)
    A, _ = O.leaf_matrices(d, np.full(d.ni, 50.0), O.local_ops(d))
    ref = O.leaf_nodes_ref(d)          # (n, 3) grid indices of the local nodes
    for row in range(d.n):
        cols = np.nonzero(A[row])[0]
        diff = ref[cols] != ref[row]     # coordinates that differ from the row's node
        if row < d.ni:
            assert np.all(diff.sum(axis=1) <= 1), row
        else:
            f = (row - d.ni) // (d.n1 ** 2)
            ax = f // 2
            assert np.all(diff.sum(axis=1) <= 1) and not np.any(np.delete(diff, ax, axis=1)), row
            ends = cols[(ref[cols][:, ax] == 0) | (ref[cols][:, ax] == p - 1)]
            assert len(ends) == 2, row     # its own node and the opposite face's
