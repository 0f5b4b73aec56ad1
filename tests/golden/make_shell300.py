"""Write tests/golden/shell300_oracle.npz: the oracle's reference solution of the 300 x 300
continuous shell (90,601 nodes, 543,606 DOF, seed 2), for the full-size parity test.

Calls only ``oracle`` and ``meshgen`` (nothing of the HIP path):

* K as the plain sum of element matrices (``assembly.assemble_coo``), f from the load lumping;
* u by elimination of the constrained DOFs, LAPACK banded Cholesky (natural node order,
  half-bandwidth 6 (m + 2) + 5) and iterative refinement with long-double residuals
  (Sec. 2.2.1, Eqs. (1)-(3));
* the compliance c = f^T u and its adjoint gradient (lambda = u) with respect to every nodal
  coordinate, quad thickness and quad stiffness scale, element terms by the complex step,
  gathered in ascending element order (Sec. 2.3.1, Eqs. (5)-(6));
* kappa_eff = ||K_ff||_2 ||u||_2 / ||f||_2 (largest eigenvalue by Lanczos), the bound
  kappa_eff * eps_64 on the relative residual that rounding u to FP64 alone can cause, and the
  measured relative residuals of the stored FP64 u, evaluated once exactly (long double) and
  once in plain FP64 arithmetic (the floor of an FP64 residual evaluation).

Run from the repository root: ``python tests/golden/make_shell300.py`` (about 10 minutes and
25 GB of host memory on 8 cores).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import meshgen  # noqa: E402
from oracle import assembly, sensitivity, solve  # noqa: E402

OUT = os.path.join(HERE, "shell300_oracle.npz")
CHUNK = 6000   # quads per complex-step batch (bounds the host memory of the element terms)


def log(msg, t0=[time.perf_counter()]):
    print(f"[{time.perf_counter() - t0[0]:7.1f} s] {msg}", flush=True)


def main():
    import scipy.sparse.linalg as sla
    mesh = meshgen.shell_300()
    log(f"mesh: {mesh.n_nodes} nodes, {mesh.n_quads} quads, {mesh.n_dof} DOF")
    K = assembly.assemble_coo(mesh)
    f = assembly.load_vector(mesh)
    log(f"K assembled: nnz {K.nnz}")
    F = solve.free_dofs(mesh)
    u, solver = solve.solve_eliminated(mesh, K, f, refine=3)
    log("u solved (banded Cholesky, 3 long-double refinement steps)")
    Kff = K.tocsr()[F][:, F]
    del solver
    ff = f[F]
    r_ld = solve.residual_ld(Kff, u[F], ff)
    rel_ld = float(np.sqrt(np.sum(r_ld * r_ld)) / np.sqrt(np.sum(ff.astype(np.longdouble) ** 2)))
    rel_64 = float(np.linalg.norm(ff - Kff @ u[F]) / np.linalg.norm(ff))
    log(f"residual of the stored u: exact {rel_ld:.3e}, FP64 evaluation {rel_64:.3e}")
    lam_max = float(sla.eigsh(Kff, k=1, which="LA", tol=1e-4, return_eigenvectors=False)[0])
    kappa = lam_max * np.linalg.norm(u) / np.linalg.norm(ff)
    log(f"||K_ff||_2 = {lam_max:.6e}, kappa_eff = {kappa:.4e}, "
        f"kappa_eff * eps = {kappa * np.finfo(float).eps:.3e}")
    c = float(f[F] @ u[F])
    gq = np.zeros((mesh.n_quads, 14))
    for lo in range(0, mesh.n_quads, CHUNK):
        hi = min(mesh.n_quads, lo + CHUNK)
        sub = mesh.copy(quad_nodes=mesh.quad_nodes[lo:hi], quad_prop=mesh.quad_prop[lo:hi],
                        quad_scale=None if mesh.quad_scale is None else
                        mesh.quad_scale[lo:hi])
        _, gq[lo:hi] = sensitivity.element_terms(sub, u, u, 1.0, 1.0)
        log(f"element terms {hi}/{mesh.n_quads}")
    gx, gt, gs = sensitivity.gather(mesh, np.zeros((0, 6)), gq)
    log(f"compliance {c:.12e}")
    np.savez_compressed(OUT, u=u, grad_xyz=gx, grad_t=gt, grad_scale=gs, c=c,
                        kappa_eff=kappa, norm_K2=lam_max, rel_residual_exact=rel_ld,
                        rel_residual_fp64=rel_64)
    log(f"wrote {OUT}")


if __name__ == "__main__":
    main()
