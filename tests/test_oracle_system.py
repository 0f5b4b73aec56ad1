"""System-level pins of the oracle: supports, equilibrium, invariance, pattern closed forms,
adjoint gradients against central finite differences, gradient invariants and the paper's own
printed sensitivity (soft)."""
import json
import os

import numpy as np
import pytest

import meshgen
import oracle
from oracle import assembly, sensitivity, solve
from structures import plate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def small_shell(m=6, seed=11):
    return meshgen.shell(m, L=6.0, seed=seed)


# --------------------------------------------------------------------------- supports

@pytest.mark.parametrize("which", ["grid", "shell"])
def test_lagrange_system_equals_elimination(which):
    """The paper's augmented system [[K, V^T], [V, 0]] [u; mu] = [f; 0] gives the eliminated
    u, and the multipliers are the support reactions f - K u on the constrained DOFs."""
    m = meshgen.gridshell(5, seed=2) if which == "grid" else small_shell(4)
    K = assembly.assemble(m)
    f = assembly.load_vector(m)
    u_el, _ = solve.solve_eliminated(m, K, f)
    u_lg, mu = solve.solve_lagrange(m, K, f)
    np.testing.assert_allclose(u_lg, u_el, rtol=0, atol=1e-10 * np.abs(u_el).max())
    C = np.flatnonzero(m.fixed.reshape(-1))
    reac = (f - K @ u_el)[C]
    np.testing.assert_allclose(mu, reac, rtol=0, atol=1e-9 * np.abs(f).max())


def test_masked_system_solution_equals_elimination():
    m = small_shell(5)
    K = assembly.assemble(m)
    f = assembly.load_vector(m)
    Km, fm = assembly.masked_system(m, K, f)
    u_mask = np.linalg.solve(Km.toarray(), fm)
    u_el, _ = solve.solve_eliminated(m, K, f)
    np.testing.assert_allclose(u_mask, u_el, rtol=0, atol=1e-11 * np.abs(u_el).max())


@pytest.mark.parametrize("which", ["grid", "shell"])
def test_equilibrium_of_reactions_and_loads(which):
    m = meshgen.gridshell(7, seed=4) if which == "grid" else small_shell(6)
    K = assembly.assemble(m)
    f = assembly.load_vector(m)
    u, _ = solve.solve_eliminated(m, K, f)
    r = (K @ u - f).reshape(-1, 6)            # support reactions on the structure, 0 elsewhere
    F = f.reshape(-1, 6)
    free = m.fixed == 0
    assert np.abs(r[free]).max() <= 1e-9 * np.abs(f).max()
    force = (r[:, :3] + F[:, :3]).sum(0)       # applied + support forces on the structure
    mom = (np.cross(m.xyz, r[:, :3] + F[:, :3]) + (r[:, 3:] + F[:, 3:])).sum(0)
    scale = np.abs(F[:, :3]).sum() * (1 + np.abs(m.xyz).max())
    assert np.abs(force).max() <= 1e-10 * scale
    assert np.abs(mom).max() <= 1e-10 * scale
    assert np.abs(r[~free]).max() > 1e-3 * np.abs(F).max()     # supports do carry load


def test_long_double_refinement_reduces_residual():
    m = meshgen.shell(12, seed=5)
    K = assembly.assemble(m)
    f = assembly.load_vector(m)
    F = solve.free_dofs(m)
    A = K.tocsr()[F][:, F]
    s = solve.SPDSolver(A, dense_limit=0)
    x0 = s.solve(f[F], refine=0)
    x2 = s.solve(f[F], refine=2)
    r0 = np.abs(solve.residual_ld(A, x0, f[F])).max()
    r2 = np.abs(solve.residual_ld(A, x2, f[F])).max()
    assert r2 <= r0
    # best attainable for an FP64 x: a few ulps of |A| |x| per row
    floor = (abs(A) @ np.abs(x2)).max() * np.finfo(float).eps
    assert r2 <= 4 * floor


# --------------------------------------------------------------------------- invariance

def _rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


@pytest.mark.parametrize("which", ["grid", "shell"])
def test_rigid_motion_invariance(which):
    """Rotating and translating the whole model with its loads leaves the compliance unchanged
    and rotates u.  Beams use Iy = Iz (the member roll rule refers to global Z)."""
    m = meshgen.gridshell(5, seed=6) if which == "grid" else small_shell(4, seed=3)
    rng = np.random.default_rng(1)
    m.f_nodal = np.zeros_like(m.f_nodal)
    m.f_nodal[m.fixed[:, 0] == 0] = rng.normal(size=((m.fixed[:, 0] == 0).sum(), 6)) * 1e3
    m.unit_weight = m.surface_load = 0.0
    Q = _rotation(5)
    m2 = m.copy()
    m2.xyz = np.ascontiguousarray(m.xyz @ Q.T + np.array([3.0, -1.0, 2.0]))
    m2.f_nodal = np.ascontiguousarray(np.concatenate([m.f_nodal[:, :3] @ Q.T,
                                                      m.f_nodal[:, 3:] @ Q.T], 1))
    r1 = sensitivity.forward(m)
    r2 = sensitivity.forward(m2)
    c1, c2 = r1["fm"] @ r1["u"], r2["fm"] @ r2["u"]
    assert c2 == pytest.approx(c1, rel=1e-10)
    u1 = r1["u"].reshape(-1, 6)
    u2 = r2["u"].reshape(-1, 6)
    np.testing.assert_allclose(u2[:, :3], u1[:, :3] @ Q.T, atol=1e-10 * np.abs(u1).max())
    np.testing.assert_allclose(u2[:, 3:], u1[:, 3:] @ Q.T, atol=1e-10 * np.abs(u1).max())


# --------------------------------------------------------------------------- pattern

@pytest.mark.parametrize("n", [3, 6, 11])
def test_gridshell_pattern_closed_form(n):
    m = meshgen.gridshell(n)
    pat = assembly.pattern(m)
    nblocks = len(pat["col"]) // 36
    assert nblocks == n * n + 4 * n * (n - 1)
    _check_pattern(m, pat)


@pytest.mark.parametrize("mm", [1, 4, 9])
def test_quad_pattern_closed_form(mm):
    m = meshgen.shell(mm, seed=0)
    pat = assembly.pattern(m)
    assert len(pat["col"]) // 36 == (3 * mm + 1) ** 2
    _check_pattern(m, pat)


def _check_pattern(m, pat):
    rp, col = pat["row_ptr"], pat["col"]
    n = m.n_dof
    A = np.zeros((n, n), bool)
    for r in range(n):
        cs = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(cs) > 0)           # sorted, unique
        A[r, cs] = True
    assert np.array_equal(A, A.T)                # structurally symmetric
    # perm is the stable key sort; S[perm] is non-decreasing and seg delimits equal slots
    S, perm, seg = pat["S"], pat["perm"], pat["seg"]
    assert np.all(np.diff(S[perm]) >= 0)
    for s in range(0, len(col), max(1, len(col) // 97)):
        ks = perm[seg[s]:seg[s + 1]]
        assert np.all(S[ks] == s)
        assert np.all(np.diff(ks) > 0)           # stable: ascending COO index within a slot
    assert seg[-1] == len(S)


def test_mixed_beams_and_quads_pattern():
    m = meshgen.shell(3, seed=0)
    m.beam_nodes = np.array([[0, 15], [5, 10]], np.int32)
    m.beam_prop = np.tile([2e11, 8e10, 1e-3, 1e-6, 1e-6, 2e-6], (2, 1))
    pat = assembly.pattern(m)
    _check_pattern(m, pat)
    assert pat["perm"].shape[0] == 2 * 144 + 9 * 576


# --------------------------------------------------------------------------- gradients

def _fd_params(m, k, seed):
    rng = np.random.default_rng(seed)
    ps = []
    for _ in range(k):
        ps.append(("xyz", int(rng.integers(m.n_nodes)), int(rng.integers(3))))
    if m.n_quads:
        for _ in range(k // 2):
            ps.append(("t", int(rng.integers(m.n_quads))))
            ps.append(("scale", int(rng.integers(m.n_quads))))
    return ps


def _check_fd(m, r, objective, ps, a=None):
    fd = sensitivity.objective_and_grad_fd(m, objective, ps, a=a)
    gref = np.abs(np.concatenate([r["grad_xyz"].ravel(), r["grad_t"], r["grad_scale"]])).max()
    for p, v in zip(ps, fd):
        g = r["grad_xyz"][p[1], p[2]] if p[0] == "xyz" else (
            r["grad_t"][p[1]] if p[0] == "t" else r["grad_scale"][p[1]])
        assert abs(g - v) <= 1e-5 * max(abs(v), 1e-3 * gref), (p, g, v)


@pytest.mark.parametrize("objective", ["compliance", "strain_energy"])
def test_gridshell_gradient_vs_fd(objective):
    m = meshgen.grid_shell_11()
    r = oracle.analyze(m, objective)
    _check_fd(m, r, objective, _fd_params(m, 20, 0))


@pytest.mark.parametrize("objective", ["compliance", "linear"])
def test_shell_gradient_vs_fd(objective):
    m = small_shell(6)
    m.quad_scale = np.random.default_rng(2).uniform(0.2, 1.0, m.n_quads) ** 3
    a = None
    if objective == "linear":
        a = np.zeros(m.n_dof)
        a[6 * (m.n_nodes // 2) + 2] = 1.0
    r = oracle.analyze(m, objective, a=a)
    _check_fd(m, r, objective, _fd_params(m, 20, 1), a=a)


def test_user_objective_matches_linear():
    m = small_shell(5)
    a = np.random.default_rng(3).normal(size=m.n_dof)
    r1 = oracle.analyze(m, "linear", a=a)
    r2 = oracle.analyze(m, "user", dg_du=a)
    np.testing.assert_allclose(r2["grad_xyz"], r1["grad_xyz"], rtol=1e-12, atol=0)


def test_translation_invariance_of_coordinate_gradient():
    for m in (meshgen.grid_shell_11(), small_shell(6)):
        r = oracle.analyze(m, "compliance")
        g = r["grad_xyz"]
        assert np.abs(g.sum(0)).max() <= 1e-9 * np.abs(g).max() * np.sqrt(m.n_nodes)


def test_scale_homogeneity():
    """K_e scales with s_e and loads do not depend on s: sum_e s_e dc/ds_e = -c; with
    s = rho^3, sum_e rho_e dc/drho_e = -3 c."""
    m = small_shell(6)
    rho = np.random.default_rng(4).uniform(0.3, 1.0, m.n_quads)
    m.quad_scale = rho**3
    r = oracle.analyze(m, "compliance")
    assert (m.quad_scale * r["grad_scale"]).sum() == pytest.approx(-r["g"], rel=1e-10)
    dc_drho = r["grad_scale"] * 3 * rho**2
    assert (rho * dc_drho).sum() == pytest.approx(-3 * r["g"], rel=1e-10)


def test_flat_plate_vertical_load_has_zero_z_gradient():
    p = plate(6, a=4.0, t=0.1, E=3e10, nu=0.2, q=2e3)
    bnd = np.isclose(p.xyz[:, 0], 0) | np.isclose(p.xyz[:, 0], 4) | \
        np.isclose(p.xyz[:, 1], 0) | np.isclose(p.xyz[:, 1], 4)
    p.fixed[bnd] = [1, 1, 1, 0, 0, 0]
    r = oracle.analyze(p, "compliance")
    assert np.abs(r["grad_xyz"][:, 2]).max() <= 1e-9 * np.abs(r["grad_xyz"]).max()
    assert r["g"] > 0


def test_compliance_is_energy_norm():
    m = small_shell(5)
    r = oracle.analyze(m, "compliance")
    c_energy = r["u"] @ (r["Km"] @ r["u"])
    assert r["g"] == pytest.approx(c_energy, rel=1e-10)
    assert r["g"] > 0


# --------------------------------------------------------------------------- paper values

def test_paper_arch_centre_sensitivity_soft():
    """Soft pin (within 2%): the 2D parabolic arch of the FEA validation and the centre-node
    dSE/dz printed by the paper.  The node spacing (uniform in x) is a reading; the two nodes
    nearest mid-span give the same value by symmetry."""
    gv = json.load(open(GOLDEN))["arch_2d"]
    n = gv["n_beams"] + 1
    L, hgt = gv["span_m"], gv["rise_m"]
    x = np.linspace(0.0, L, n)
    z = 4 * hgt / L**2 * x * (L - x)
    xyz = np.ascontiguousarray(np.stack([x, np.zeros(n), z], 1))
    fixed = np.zeros((n, 6), np.uint8)
    fixed[0] = fixed[-1] = gv["support_flags"]
    f = np.zeros((n, 6))
    f[:, 2] = -gv["nodal_load_N"]
    bn = np.stack([np.arange(n - 1), np.arange(1, n)], 1).astype(np.int32)
    E, nu = gv["E_Pa"], gv["nu"]
    prop = np.tile([E, E / (2 * (1 + nu)), gv["A_m2"], gv["Iy_m4"], gv["Iz_m4"],
                    gv["Iy_m4"] + gv["Iz_m4"]], (n - 1, 1))
    m = meshgen.Mesh(xyz=xyz, fixed=fixed, f_nodal=f, beam_nodes=bn, beam_prop=prop)
    r = oracle.analyze(m, "strain_energy")
    g = r["grad_xyz"][n // 2 - 1, 2]
    assert r["grad_xyz"][n // 2, 2] == pytest.approx(g, rel=1e-8)
    assert g == pytest.approx(gv["dSE_dz_centre_adjoint"], rel=0.02)


@pytest.mark.parametrize("which", ["grid11", "shell8"])
def test_displacement_parity_bar_is_attainable(which):
    """kappa_eff = ||K||_2 ||u||_2 / ||f||_2 of the masked system: the 1e-10 relative bar on u is
    within reach of a backward-stable FP64 solve only where kappa_eff * eps64 is below it."""
    import scipy.sparse.linalg as sla
    m = meshgen.grid_shell_11() if which == "grid11" else meshgen.shell(8, L=8.0, seed=3)
    r = oracle.analyze(m, "compliance")
    lmax = sla.eigsh(r["Km"].tocsr(), k=1, which="LA", return_eigenvectors=False)[0]
    k_eff = lmax * np.linalg.norm(r["u"]) / np.linalg.norm(r["fm"])
    print(f"{which}: kappa_eff = {k_eff:.3e}, kappa_eff * eps = {k_eff * np.finfo(float).eps:.2e}")
    assert k_eff * np.finfo(float).eps < 1e-10


def test_assemble_coo_equals_dictionary_assembly():
    """The duplicate-summing COO route (used for the 300 x 300 reference) gives the K of the
    dictionary-scatter route, up to the order of a slot's at most four additions."""
    import scipy.sparse as sp
    for mesh in (meshgen.gridshell(7, seed=3), meshgen.shell(6, L=6.0, seed=4)):
        K1 = assembly.assemble(mesh).tocsr()
        K2 = assembly.assemble_coo(mesh)
        d = abs(K1 - K2)
        assert d.max() <= 1e-14 * abs(K1).max()
        assert K2.nnz == K1.nnz


@pytest.mark.slow
def test_shell300_reference_solution_properties():
    """The stored reference of the 300 x 300 shell against what fixes it at any size: its
    residual under the element-by-element operator, c = f^T u, translation invariance of the
    coordinate gradient and homogeneity of c in the stiffness scale."""
    import os
    z = np.load(os.path.join(os.path.dirname(__file__), "golden", "shell300_oracle.npz"))
    mesh = meshgen.shell_300()
    u = z["u"]
    f = assembly.load_vector(mesh)
    free = mesh.fixed.reshape(-1) == 0
    r = (f - assembly.apply_K_elementwise(mesh, u))[free]
    assert np.linalg.norm(r) / np.linalg.norm(f[free]) <= 2e-10
    assert np.all(u[~free] == 0.0)
    c = float(z["c"])
    assert c == pytest.approx(float(f[free] @ u[free]), rel=1e-13)
    gx = z["grad_xyz"]
    for k in range(3):
        assert abs(gx[:, k].sum()) <= 1e-9 * np.abs(gx[:, k]).sum()
    assert z["grad_scale"].sum() == pytest.approx(-c, rel=1e-10)
    assert float(z["kappa_eff"]) * np.finfo(float).eps > 1e-10
