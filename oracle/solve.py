"""Oracle linear solves: elimination + LAPACK banded Cholesky, dense Cholesky, the paper's
Lagrange-multiplier system, and extended-precision iterative refinement.

Paper: Sec. 2.2.1-2.2.2 -- K u = f (Eq. (1)); supports enter through Lagrange multipliers,
[[K, V^T], [V, 0]] [u; mu] = [f; b] (Eq. (2)) with V u = b (Eq. (3)); the paper solves it with a
dense LU or with sparse direct solvers.  The oracle eliminates the constrained DOFs instead,
u_c = b_c and K_ff u_f = f_f - K_fc b_c, which gives the identical u, and solves the symmetric
positive definite K_ff with a banded Cholesky in natural node order.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp


def free_dofs(mesh):
    return np.flatnonzero(mesh.fixed.reshape(-1) == 0)


def _to_banded_upper(A):
    """Upper banded storage ab[u + i - j, j] = A[i, j] for i <= j (scipy/LAPACK convention)."""
    A = sp.triu(A.tocoo())
    u = int(np.max(A.col - A.row)) if A.nnz else 0
    ab = np.zeros((u + 1, A.shape[0]), dtype=A.dtype)
    ab[u + A.row - A.col, A.col] = A.data
    return ab


def residual_ld(A, x, b):
    """b - A x computed with every product and sum in numpy longdouble (80-bit on x86)."""
    A = A.tocsr()
    ld = np.longdouble
    prod = A.data.astype(ld) * x.astype(ld)[A.indices]
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    Ax = np.zeros(A.shape[0], dtype=ld)
    np.add.at(Ax, rows, prod)
    return b.astype(ld) - Ax


class SPDSolver:
    """Banded Cholesky of an SPD sparse matrix with refinement against the original matrix."""

    def __init__(self, A, dense_limit=3000):
        self.A = A.tocsr()
        n = A.shape[0]
        if n <= dense_limit:
            self.kind = "dense"
            self.L = la.cholesky(self.A.toarray(), lower=True)
        else:
            self.kind = "banded"
            self.cb = la.cholesky_banded(_to_banded_upper(self.A), lower=False)

    def _solve_once(self, b):
        if self.kind == "dense":
            return la.cho_solve((self.L, True), b)
        return la.cho_solve_banded((self.cb, False), b)

    def solve(self, b, refine=2):
        x = self._solve_once(b)
        for _ in range(refine):
            r = residual_ld(self.A, x, b)
            x = x + self._solve_once(np.asarray(r, dtype=np.float64))
        return x


def prescribed(mesh):
    """The prescribed displacement vector b [n_dof] (Eq. (3)): mesh.u_prescribed at the
    constrained DOFs, 0 at the free ones; None when the mesh prescribes none."""
    up = getattr(mesh, "u_prescribed", None)
    if up is None:
        return None
    fixed = mesh.fixed.reshape(-1) != 0
    return np.where(fixed, np.asarray(up, dtype=float).reshape(-1), 0.0)


def solve_eliminated(mesh, K, f, refine=2, solver=None, b=None):
    """u with u_c = b_c on constrained DOFs (0 when b is None) and
    K_ff u_f = f_f - K_fc b_c on the free ones.

    Returns (u, solver) so that the adjoint can reuse the factorisation."""
    F = free_dofs(mesh)
    K = K.tocsr()
    if solver is None:
        solver = SPDSolver(K[F][:, F])
    rhs = np.asarray(f, dtype=float)[F]
    u = np.zeros(mesh.n_dof)
    if b is not None:
        C = np.flatnonzero(mesh.fixed.reshape(-1) != 0)
        u[C] = b[C]
        rhs = rhs - K[F][:, C] @ b[C]
    u[F] = solver.solve(rhs, refine)
    return u, solver


def solve_lagrange(mesh, K, f, b=None):
    """The paper's augmented system (Eq. (2)) with dense LU: returns (u, mu).

    V selects the constrained DOFs (one row per fixed flag); b are the prescribed values."""
    n = mesh.n_dof
    C = np.flatnonzero(mesh.fixed.reshape(-1) != 0)
    V = np.zeros((len(C), n))
    V[np.arange(len(C)), C] = 1.0
    b = np.zeros(len(C)) if b is None else b
    Kaug = np.block([[K.toarray(), V.T], [V, np.zeros((len(C), len(C)))]])
    sol = np.linalg.solve(Kaug, np.concatenate([f, b]))
    return sol[:n], sol[n:]
