"""Oracle objectives, adjoint solve and gradients with respect to nodal coordinates, quad
thickness and quad stiffness scale.

Paper: Sec. 2.3.1 -- minimise g(u, p) subject to K(p) u = f(p); the adjoint equation
K^T lambda = (dg/du)^T (Eq. (5)) and the adjoint sensitivity
dg/dp = dg/dp|_explicit - lambda^T (dK/dp u - df/dp) (Eq. (6)).  Objectives: the paper's
"strain energy" g = f^T u / 2 (Sec. 2.2.3 and 2.3.2), compliance f^T u (the loss of the neural
network example, Sec. 3.6), a linear functional a^T u, or any g whose dg/du the caller provides.
Design parameters: nodal Z (and X, Y) coordinates (Sec. 2.3.1 listing, NodeParameter(node, 2))
and shell thickness (Sec. 3.3), plus the per-element stiffness scale that carries the SIMP
density (Sec. 3.4, Eq. (13)).

Element derivatives dK_e/dp and df_e/dp are taken by the complex step,
dK_e/dp = Im K_e(p + i h) / h with h = 1e-30 (exact to rounding, independent of any dual or
reverse-mode code).  The element terms are gathered per node over incident elements in ascending
element order (beams first, then quads).
"""
from __future__ import annotations

import numpy as np

from . import assembly, elements, solve

CS_STEP = 1.0e-30
FD_STEP = 1.0e-6

OBJECTIVES = ("compliance", "strain_energy", "linear", "user")


def forward(mesh, pat=None, xyz=None, quad_t=None, quad_scale=None, refine=2):
    """Assemble, mask and solve.  Returns a dict with K (unconstrained), Km, f, fm, u, solver."""
    K = assembly.assemble(mesh, pat, xyz, quad_t, quad_scale)
    f = assembly.load_vector(mesh, xyz, quad_t)
    Km, fm = assembly.masked_system(mesh, K, f)
    b = solve.prescribed(mesh)
    u, solver = solve.solve_eliminated(mesh, K, f, refine, b=b)
    return dict(K=K, Km=Km, f=f, fm=fm, u=u, solver=solver, b=b)


def objective_value(kind, f, u, a=None):
    """g(u): compliance f^T u, strain energy f^T u / 2 (f masked: the applied load on the free
    DOFs), or linear a^T u."""
    if kind == "compliance":
        return float(f @ u)
    if kind == "strain_energy":
        return 0.5 * float(f @ u)
    if kind == "linear":
        return float(a @ u)
    raise ValueError(kind)


def _quad_inputs(mesh, xyz, quad_t, quad_scale):
    X = xyz[mesh.quad_nodes].astype(complex)
    prop = mesh.quad_prop.astype(complex)
    prop[:, 0] = quad_t
    scale = np.ones(mesh.n_quads, complex) if quad_scale is None else quad_scale.astype(complex)
    return X, prop, scale


def element_terms(mesh, u, lam, c_lam, c_u, xyz=None, quad_t=None, quad_scale=None):
    """Per-element adjoint terms g_e,p = c_lam (lam_e^T df_e/dp - lam_e^T dK_e/dp u_e)
    + c_u u_e^T df_e/dp, the last with u_e zero at constrained DOFs (the objectives use the
    load on the free DOFs only; this matters with prescribed displacements).

    Returns beam terms [nb, 6] (3 coordinates of each end node) and quad terms [nq, 14]
    (12 coordinates of the 4 corners, then t, then the stiffness scale)."""
    xyz = mesh.xyz if xyz is None else xyz
    quad_t = mesh.quad_prop[:, 0] if quad_t is None else quad_t
    quad_scale = mesh.quad_scale if quad_scale is None else quad_scale
    bd, qd = assembly.element_dofs(mesh)
    h = CS_STEP
    gb = np.zeros((mesh.n_beams, 6))
    if mesh.n_beams:
        X = xyz[mesh.beam_nodes].astype(complex)
        ue, le = u[bd], lam[bd]
        for d in range(6):
            Xp = X.copy()
            Xp[:, d // 3, d % 3] += 1j * h
            dK = np.imag(elements.beam_K(Xp, mesh.beam_prop)) / h
            gb[:, d] = -c_lam * np.einsum("na,nab,nb->n", le, dK, ue)
    gq = np.zeros((mesh.n_quads, 14))
    if mesh.n_quads:
        X, prop, scale = _quad_inputs(mesh, xyz, quad_t, quad_scale)
        ue, le = u[qd], lam[qd]
        ux = np.where(mesh.fixed.reshape(-1)[qd] != 0, 0.0, ue)
        for d in range(14):
            Xp, pp, sp_ = X.copy(), prop.copy(), scale.copy()
            if d < 12:
                Xp[:, d // 3, d % 3] += 1j * h
            elif d == 12:
                pp[:, 0] += 1j * h
            else:
                sp_ += 1j * h
            dK = np.imag(elements.shell_K(Xp, pp, sp_)) / h
            dfe = np.imag(elements.shell_load(Xp, pp[:, 0], mesh.unit_weight,
                                              mesh.surface_load)) / h
            gq[:, d] = (c_lam * (np.einsum("na,na->n", le, dfe)
                                 - np.einsum("na,nab,nb->n", le, dK, ue))
                        + c_u * np.einsum("na,na->n", ux, dfe))
    return gb, gq


def gather(mesh, gb, gq):
    """dg/dxyz [n_nodes, 3] summed over incident elements in ascending element order, plus
    dg/dt [nq] and dg/dscale [nq] taken directly from the quad terms."""
    g = np.zeros((mesh.n_nodes, 3))
    for e in range(mesh.n_beams):
        for a in range(2):
            g[mesh.beam_nodes[e, a]] += gb[e, 3 * a:3 * a + 3]
    for e in range(mesh.n_quads):
        for a in range(4):
            g[mesh.quad_nodes[e, a]] += gq[e, 3 * a:3 * a + 3]
    return g, gq[:, 12].copy(), gq[:, 13].copy()


def analyze(mesh, objective="compliance", a=None, dg_du=None, refine=2, pat=None):
    """Forward solve, objective, adjoint and gradient.

    objective: 'compliance' (f^T u), 'strain_energy' (f^T u / 2), 'linear' (a^T u, a given) or
    'user' (dg/du given; dg/dp then omits any explicit dependence of g on p)."""
    fw = forward(mesh, pat=pat, refine=refine)
    u, fm = fw["u"], fw["fm"]
    fixed = mesh.fixed.reshape(-1).astype(bool)
    if objective in ("compliance", "strain_energy"):
        c = 1.0 if objective == "compliance" else 0.5
        g = objective_value(objective, fm, u)
        if fw["b"] is None:
            lam = u.copy()        # K lam = f has the solution lam = u
        else:
            # with prescribed displacements u solves the lifted system, so lam != u
            lam, _ = solve.solve_eliminated(mesh, fw["K"], fm, refine, solver=fw["solver"])
        c_lam, c_u = c, c
    else:
        rhs = np.asarray(a if objective == "linear" else dg_du, dtype=float)
        g = objective_value("linear", fm, u, rhs) if objective == "linear" else None
        rhs = np.where(fixed, 0.0, rhs)
        lam, _ = solve.solve_eliminated(mesh, fw["K"], rhs, refine, solver=fw["solver"])
        c_lam, c_u = 1.0, 0.0
    gb, gq = element_terms(mesh, u, lam, c_lam, c_u)
    gx, gt, gs = gather(mesh, gb, gq)
    out = dict(fw)
    out.update(g=g, lam=lam, grad_xyz=gx, grad_t=gt, grad_scale=gs, gb=gb, gq=gq)
    return out


def objective_at(mesh, objective, a=None, xyz=None, quad_t=None, quad_scale=None, pat=None):
    fw = forward(mesh, pat=pat, xyz=xyz, quad_t=quad_t, quad_scale=quad_scale)
    return objective_value(objective, fw["fm"], fw["u"], a)


def objective_and_grad_fd(mesh, objective, params, a=None, h=FD_STEP, pat=None):
    """Central finite differences of the whole pipeline, (g(p + h) - g(p - h)) / 2h.

    params: list of ('xyz', node, comp) | ('t', quad) | ('scale', quad)."""
    pat = assembly.pattern(mesh) if pat is None else pat
    t0 = mesh.quad_prop[:, 0].copy()
    s0 = np.ones(mesh.n_quads) if mesh.quad_scale is None else mesh.quad_scale.copy()
    out = []
    for p in params:
        vals = []
        for sgn in (1.0, -1.0):
            xyz, t, s = mesh.xyz.copy(), t0.copy(), s0.copy()
            if p[0] == "xyz":
                xyz[p[1], p[2]] += sgn * h
            elif p[0] == "t":
                t[p[1]] += sgn * h
            else:
                s[p[1]] += sgn * h
            vals.append(objective_at(mesh, objective, a, xyz, t, s, pat))
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)
