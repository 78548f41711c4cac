"""CPU prototype of a two-level preconditioner for the HPS system: the
block-Jacobi preconditioner as smoother around a coarse-grid correction (the
multi-level solver that the concluding section of the paper proposes as future
work; the paper leaves the coarse solver open).

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: nothing in the product path
imports it.  It is the reference a GPU version would be checked against, and
it measures whether the idea pays before any kernel is written.

Construction (all FP64, dense per-leaf tensor products, scipy sparse globally):
  * coarse grid: the same leaves discretized by HPS at a lower order p_c < p
    (the same equations, eq. (leaf) and eq. (outgoingimpedance), rebuilt at
    p_c by hps_oracle), A_c its global matrix;
  * prolongation P (coarse -> fine), leaf by leaf: interior values by the
    tensor product of the 1D Lagrange interpolation from the p_c - 2 interior
    Chebyshev-Lobatto nodes to the p - 2 fine ones, face values by the 2D
    tensor product of the same on each face (the face nodes are the interior
    nodes of the face, Sec. 2.1);
  * restriction R (fine -> coarse): the same construction from the fine nodes
    to the coarse ones; R P = I because the fine interpolant of a coarse
    polynomial is that polynomial;
  * one application, for a residual r: x1 = J^-1 r; x2 = x1 + P A_c^-1 R (r -
    A x1); x = x2 + J^-1 (r - A x2) (pre-smoothing, coarse correction,
    post-smoothing), with A_c^-1 by a sparse LU.
With p_c = p, P = R = I and A_c = A, so the application is A^-1 r exactly.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import hps_oracle as O


def interior_nodes(p: int) -> np.ndarray:
    """The p - 2 interior Chebyshev-Lobatto nodes on [-1, 1], ascending."""
    return O.cheb_nodes(p)[1:-1]


def lagrange_matrix(src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """L[i, j] = l_j(dst[i]): values at dst of the Lagrange basis on the nodes src."""
    L = np.ones((len(dst), len(src)))
    for j, xj in enumerate(src):
        for m, xm in enumerate(src):
            if m != j:
                L[:, j] *= (dst - xm) / (xj - xm)
    return L


def leaf_transfer(p_from: int, p_to: int) -> np.ndarray:
    """Dense (n_to, n_from) map of one leaf's nodal values (interior block, then
    faces 1..6, local order of hps_oracle) from order p_from to order p_to."""
    L = lagrange_matrix(interior_nodes(p_from), interior_nodes(p_to))
    m_from, m_to = p_from - 2, p_to - 2
    # interior: x fastest, so the x-factor is the right-most Kronecker factor
    Ti = np.kron(L, np.kron(L, L))
    # a face: its two tangential axes, lower axis fastest
    Tf = np.kron(L, L)
    n_from = m_from ** 3 + 6 * m_from ** 2
    n_to = m_to ** 3 + 6 * m_to ** 2
    T = np.zeros((n_to, n_from))
    T[:m_to ** 3, :m_from ** 3] = Ti
    for f in range(6):
        r0 = m_to ** 3 + f * m_to ** 2
        c0 = m_from ** 3 + f * m_from ** 2
        T[r0:r0 + m_to ** 2, c0:c0 + m_from ** 2] = Tf
    return T


def transfer(nl: int, p_from: int, p_to: int) -> sp.csr_matrix:
    """The leaf map on every leaf (block diagonal)."""
    return sp.block_diag([sp.csr_matrix(leaf_transfer(p_from, p_to))] * nl, format="csr")


class TwoLevel:
    """The two-level preconditioner of one problem (a problems.Problem) at
    fine order prob.p and coarse order p_c."""

    def __init__(self, prob, p_c: int, op: O.OracleProblem | None = None):
        from paper_2112_02211_amd import problems as P   # seeded input data only
        if not 3 <= p_c <= prob.p:
            raise ValueError("need 3 <= p_c <= p")
        self.op = O.build(prob) if op is None else op
        d = self.op.d
        self.dc = O.make_disc(prob.n_elem, p_c, prob.kappa, prob.eta, prob.lo, prob.hi)
        xyz_c = O.node_coords(self.dc)
        b_c = np.zeros(self.dc.N, dtype=np.complex128) if prob.plane_dir is not None \
            else P.bump_field(prob, xyz_c)
        self.Ac = O.assemble_global(self.dc, b_c)
        self.lu = spla.splu(self.Ac.tocsc())
        self.P = transfer(d.nl, p_c, d.p)
        self.R = transfer(d.nl, d.p, p_c)
        self.J = O.Precond(d, self.op.b_nodes)

    def coarse(self, r: np.ndarray) -> np.ndarray:
        """P A_c^-1 R r."""
        return self.P @ self.lu.solve(self.R @ r)

    def apply(self, r: np.ndarray) -> np.ndarray:
        A = self.op.A
        x = self.J.apply(r)
        x = x + self.coarse(r - A @ x)
        return x + self.J.apply(r - A @ x)
