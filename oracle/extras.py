"""Oracle for the optimisation extras of the paper's examples: the penalised material volume of
the size optimisation (Sec. 3.3) with its adjoint gradient, the self-adaptive penalty update,
and the hat filter applied to sensitivities (Sec. 3.1-3.2).  TEST INFRASTRUCTURE ONLY.

Readings (the paper states the formulas but not every detail):
* c(p) = sum over nodes of max(0, |u_z| / u_max - 1), with u_z the vertical displacement (the
  example applies the limit to Z); dc/du_z = sign(u_z) / u_max where the term is active, 0
  elsewhere (also at the kink).
* W(p) = sum_i A_i t_i + sum_i max(0, (t_min - t_i) / t_min) over the quads, A_i the element
  area used for the loads, |d13 x d24| / 2; dW/dt_i = A_i - 1/t_min where t_i < t_min.
* g = (1 + eps1 c) W and dg/dp = eps1 W dc/dp + (1 + eps1 c) dW/dp, dc/dp by the adjoint
  (Eqs. 5-6) with dg/du = dc/du.
* hat filter: g_i <- sum_j w_ij g_j / sum_j w_ij with w_ij = max(0, r - |X_i - X_j|) over the
  design nodes (3-D distance of the current coordinates); the weighted average normalised per
  row (the density-filter form of topology optimisation).
"""
from __future__ import annotations

import numpy as np

from . import elements, sensitivity

CS_STEP = 1.0e-30


def displacement_violation(u, u_max):
    """c = sum_j max(0, |u_jz| / u_max - 1) and dc/du [n_dof]."""
    uz = np.asarray(u).reshape(-1, 6)[:, 2]
    v = np.abs(uz) / u_max - 1.0
    active = v > 0.0
    c = float(np.sum(np.where(active, v, 0.0)))
    dcdu = np.zeros(np.asarray(u).size)
    dcdu[6 * np.flatnonzero(active) + 2] = np.sign(uz[active]) / u_max
    return c, dcdu


def penalised_volume(mesh, t_min, xyz=None, quad_t=None):
    """W, dW/dxyz [n_nodes, 3] (gathered per node in ascending element order) and dW/dt."""
    xyz = mesh.xyz if xyz is None else xyz
    t = mesh.quad_prop[:, 0] if quad_t is None else quad_t
    X = xyz[mesh.quad_nodes]
    A = elements.shell_area(X)
    below = t < t_min
    W = float(np.sum(A * t) + np.sum(np.where(below, (t_min - t) / t_min, 0.0)))
    dt = A - np.where(below, 1.0 / t_min, 0.0)
    gq = np.zeros((mesh.n_quads, 12))
    for d in range(12):
        Xc = X.astype(complex)
        Xc[:, d // 3, d % 3] += 1j * CS_STEP
        gq[:, d] = t * np.imag(elements.shell_area(Xc)) / CS_STEP
    gx = np.zeros((mesh.n_nodes, 3))
    for e in range(mesh.n_quads):
        for a in range(4):
            gx[mesh.quad_nodes[e, a]] += gq[e, 3 * a:3 * a + 3]
    return W, gx, dt


def size_objective(mesh, eps1, u_max, t_min, pat=None):
    """g = (1 + eps1 c) W with its gradient with respect to nodal coordinates and thickness."""
    fw = sensitivity.forward(mesh, pat=pat)
    c, dcdu = displacement_violation(fw["u"], u_max)
    r = sensitivity.analyze(mesh, "user", dg_du=dcdu, pat=pat)
    W, wx, wt = penalised_volume(mesh, t_min)
    g = (1.0 + eps1 * c) * W
    gx = eps1 * W * r["grad_xyz"] + (1.0 + eps1 * c) * wx
    gt = eps1 * W * r["grad_t"] + (1.0 + eps1 * c) * wt
    return dict(g=g, c=c, W=W, u=fw["u"], grad_xyz=gx, grad_t=gt, dc_dxyz=r["grad_xyz"],
                dc_dt=r["grad_t"])


def size_objective_value(mesh, eps1, u_max, t_min, xyz=None, quad_t=None, pat=None):
    fw = sensitivity.forward(mesh, pat=pat, xyz=xyz, quad_t=quad_t)
    c, _ = displacement_violation(fw["u"], u_max)
    W, _, _ = penalised_volume(mesh, t_min, xyz=xyz, quad_t=quad_t)
    return (1.0 + eps1 * c) * W


def update_eps1(eps1, violated, kappa=1.015):
    """Self-adaptive penalty coefficient: times kappa after a violation, divided by it after none."""
    return eps1 * kappa if violated else eps1 / kappa


def hat_filter(xyz, nodes, g, radius):
    """Filtered sensitivities of the design nodes, a plain double loop in ascending j."""
    P = np.asarray(xyz)[np.asarray(nodes)]
    g = np.asarray(g, dtype=float)
    out = np.zeros(len(nodes))
    for i in range(len(nodes)):
        num = 0.0
        den = 0.0
        for j in range(len(nodes)):
            d = np.sqrt(np.sum((P[i] - P[j]) ** 2))
            w = max(0.0, radius - d)
            num += w * g[j]
            den += w
        out[i] = num / den
    return out
