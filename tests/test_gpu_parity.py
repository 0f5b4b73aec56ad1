"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: pattern, permutation and segments bit-exact; K and f within 1e-13 of the matrix scale;
u within 1e-10 relative (2-norm) when PCG runs to the residual floor; gradients within 1e-8
relative (inf-norm) of the oracle adjoint and within the finite-difference bound
|g - fd| <= 1e-5 max(|fd|, 1e-3 |g|_inf) at central differences h = 1e-6."""
import numpy as np
import pytest

import meshgen
import oracle
from oracle import assembly, sensitivity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _sso():
    import paper_2407_20026_amd as sso
    return sso


def small_shell(m=8, seed=3, scaled=True):
    s = meshgen.shell(m, L=8.0, seed=seed)
    if scaled:
        s.quad_scale = np.random.default_rng(seed).uniform(0.2, 1.0, s.n_quads) ** 3
    return s


def mixed_mesh():
    s = meshgen.shell(5, L=5.0, seed=2)
    s.beam_nodes = np.array([[0, 14], [3, 20], [7, 35], [30, 11]], np.int32)
    s.beam_prop = np.tile([2.1e11, 8.1e10, 2e-3, 3e-6, 5e-6, 4e-6], (4, 1)).astype(np.float64)
    s.f_nodal = np.zeros_like(s.f_nodal)
    s.f_nodal[s.fixed[:, 0] == 0, 2] = -5e3
    return s


def hub_mesh(n_spokes=20):
    """A hub node joined to a ring of n_spokes nodes (spokes + ring members): the hub's block row
    has n_spokes + 1 blocks, more than the padded layout takes (the block order of K is used)."""
    ang = np.linspace(0.0, 2 * np.pi, n_spokes, endpoint=False)
    ring = np.column_stack([5 * np.cos(ang), 5 * np.sin(ang), 0.3 * np.sin(3 * ang)])
    xyz = np.vstack([[0.0, 0.0, 1.5], ring])
    n = len(xyz)
    spokes = [[0, 1 + k] for k in range(n_spokes)]
    hoop = [[1 + k, 1 + (k + 1) % n_spokes] for k in range(n_spokes)]
    fixed = np.zeros((n, 6), np.uint8)
    fixed[1::4, :3] = 1
    f = np.zeros((n, 6))
    f[:, 2] = -1e4
    f[0, 0] = 3e3
    beams = np.array(spokes + hoop, np.int32)
    prop = np.tile([2.1e11, 8.1e10, 1e-3, 1e-6, 1.5e-6, 2e-6], (len(beams), 1))
    return meshgen.Mesh(xyz=xyz, fixed=fixed, f_nodal=f, beam_nodes=beams, beam_prop=prop,
                        quad_nodes=np.zeros((0, 4), np.int32), quad_prop=np.zeros((0, 5)),
                        name="hub")


def cantilever_beam():
    """One member, one workgroup with a single active row pair: node 0 clamped, a skew tip load."""
    xyz = np.array([[0.0, 0.0, 0.0], [3.0, 0.4, 0.7]])
    fixed = np.zeros((2, 6), np.uint8)
    fixed[0] = 1
    f = np.zeros((2, 6))
    f[1, :3] = [2e3, -1e3, -5e3]
    f[1, 5] = 4e2
    return meshgen.Mesh(xyz=xyz, fixed=fixed, f_nodal=f,
                        beam_nodes=np.array([[0, 1]], np.int32),
                        beam_prop=np.array([[2.1e11, 8.1e10, 1e-3, 1e-6, 2e-6, 1.5e-6]]),
                        name="cantilever")


def one_quad():
    """One warped shell element clamped along one edge, loaded at the free corners."""
    xyz = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.1], [2.1, 1.8, -0.05], [0.0, 2.0, 0.0]])
    fixed = np.zeros((4, 6), np.uint8)
    fixed[[0, 3]] = 1
    f = np.zeros((4, 6))
    f[1, 2] = -3e3
    f[2, 2] = -2e3
    f[2, 0] = 1e3
    return meshgen.Mesh(xyz=xyz, fixed=fixed, f_nodal=f,
                        quad_nodes=np.array([[0, 1, 2, 3]], np.int32),
                        quad_prop=np.array([[0.12, 30e9, 0.2, 1.0, 1.0]]),
                        quad_scale=np.array([0.7]), name="one_quad")


CASES = {
    "cantilever": cantilever_beam,
    "one_quad": one_quad,
    "grid11": meshgen.grid_shell_11,
    "hub": hub_mesh,
    "grid_ragged": lambda: meshgen.gridshell(13, seed=5),
    "shell8": small_shell,
    "mixed": mixed_mesh,
    "shell60": meshgen.shell_60,
    "arch6": lambda: meshgen.arch_bridge(6),
}

TIGHT = dict(rtol=1e-13, max_it=50000)


@pytest.fixture(scope="module")
def refs():
    cache = {}

    def get(name):
        if name not in cache:
            mesh = CASES[name]()
            pat = assembly.pattern(mesh)
            r = oracle.analyze(mesh, "compliance", pat=pat)
            cache[name] = (mesh, pat, r)
        return cache[name]
    return get


def _problem(mesh, **opts):
    sso = _sso()
    o = sso.Options(**{**TIGHT, **opts})
    return sso.Problem(mesh, o)


def _solve_tight(p):
    u, st = p.solve(check=False)
    sso = _sso()
    # converged, or stagnated at the rounding floor (reported as not converged).  The true
    # residual floor of an FP64 solution is about eps * |K| |u| / |f| (1e-11 .. 1e-10 here), so
    # the parity bar is on u itself, not on the residual.
    assert p.last_status in (sso.SSO_OK, sso.SSO_ENOTCONV), p.last_status
    assert st["rel_residual"] < 1e-9, st
    return u, st


@pytest.mark.parametrize("name", list(CASES))
def test_pattern_bit_exact(refs, name):
    mesh, pat, _ = refs(name)
    print(f"[gpu] pattern {name}", flush=True)
    with _problem(mesh) as p:
        g = {k: v.cpu().numpy().astype(np.int64) for k, v in p.pattern().items()}
    for k in ("row_ptr", "col", "perm", "seg"):
        assert g[k].shape == pat[k].shape, k
        assert np.array_equal(g[k], pat[k]), k


@pytest.mark.parametrize("name", list(CASES))
def test_stiffness_and_load(refs, name):
    mesh, pat, r = refs(name)
    print(f"[gpu] K/f {name}", flush=True)
    with _problem(mesh) as p:
        _solve_tight(p)
        vals, f = p.matrix()
    vals = vals.cpu().numpy()
    Kref = r["Km"].tocsr()
    Kref.sort_indices()
    ref = Kref.data
    assert vals.shape == ref.shape
    scale = np.abs(ref).max()
    assert np.abs(vals - ref).max() <= 1e-13 * scale
    np.testing.assert_allclose(f.cpu().numpy().ravel(), r["fm"], rtol=0,
                               atol=1e-14 * np.abs(r["fm"]).max())
    # bitwise symmetric: an entry below the diagonal is summed from its transposed entry's
    # element contributions, which the products that read only the upper triangle rely on
    n = mesh.n_dof
    import scipy.sparse as sp
    Kg = sp.csr_matrix((vals, pat["col"], pat["row_ptr"]), shape=(n, n))
    assert abs(Kg - Kg.T).max() == 0.0


@pytest.mark.parametrize("name", list(CASES))
def test_displacement(refs, name):
    mesh, _, r = refs(name)
    print(f"[gpu] u {name}", flush=True)
    with _problem(mesh) as p:
        u, st = _solve_tight(p)
        c = p.objective("compliance")
        se = p.objective("strain_energy")
    u = u.cpu().numpy().ravel()
    err = np.linalg.norm(u - r["u"]) / np.linalg.norm(r["u"])
    print(f"  iters={st['iters']} rel_res={st['rel_residual']:.2e} |du|/|u|={err:.2e}")
    assert err <= 1e-10
    assert c == pytest.approx(r["g"], rel=1e-10)
    assert se == pytest.approx(0.5 * r["g"], rel=1e-10)


def _grad_err(g, ref):
    scale = max(np.abs(ref).max(), 1e-300)
    return np.abs(g - ref).max() / scale


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("objective", ["compliance", "strain_energy"])
def test_gradient_energy_objectives(refs, name, objective):
    mesh, pat, r0 = refs(name)
    print(f"[gpu] grad {name} {objective}", flush=True)
    r = r0 if objective == "compliance" else oracle.analyze(mesh, objective, pat=pat)
    with _problem(mesh) as p:
        _solve_tight(p)
        g = p.adjoint(objective)
    gx = g["dg_dxyz"].cpu().numpy()
    assert _grad_err(gx, r["grad_xyz"]) <= 1e-8
    if mesh.n_quads:
        assert _grad_err(g["dg_dt"].cpu().numpy(), r["grad_t"]) <= 1e-8
        assert _grad_err(g["dg_dscale"].cpu().numpy(), r["grad_scale"]) <= 1e-8


@pytest.mark.parametrize("name", ["grid11", "shell8", "mixed"])
@pytest.mark.parametrize("objective", ["linear", "user"])
def test_gradient_general_objective(refs, name, objective):
    mesh, pat, _ = refs(name)
    print(f"[gpu] grad {name} {objective}", flush=True)
    rng = np.random.default_rng(9)
    if objective == "linear":
        a = np.zeros(mesh.n_dof)
        a[6 * (mesh.n_nodes // 2) + 2] = 1.0
    else:
        a = rng.normal(size=mesh.n_dof)
    r = oracle.analyze(mesh, objective, a=a, dg_du=a, pat=pat)
    # the adjoint solve runs to the problem's rtol on the true residual, so it must be above
    # the FP64 floor (~3e-11 on the grid-shell) for the call to report success
    with _problem(mesh, rtol=1e-10) as p:
        _solve_tight(p)
        if objective == "linear":
            assert p.objective("linear", a) == pytest.approx(r["g"], rel=1e-9)
        g = p.adjoint(objective, dg_du=a)
    assert _grad_err(g["dg_dxyz"].cpu().numpy(), r["grad_xyz"]) <= 1e-8
    if mesh.n_quads:
        assert _grad_err(g["dg_dt"].cpu().numpy(), r["grad_t"]) <= 1e-8
        assert _grad_err(g["dg_dscale"].cpu().numpy(), r["grad_scale"]) <= 1e-8


@pytest.mark.parametrize("name", ["grid11", "shell8", "mixed"])
@pytest.mark.parametrize("objective", ["compliance", "strain_energy", "linear"])
def test_prescribed_displacements(refs, name, objective):
    """Nonzero prescribed support displacements (Eq. 3 with b != 0): u equals b exactly on the
    constrained DOFs and the oracle's eliminated solution elsewhere (bar as for u); objective
    and gradients (for the energy objectives through a separate adjoint solve) as for the other
    gradients."""
    mesh0, pat, _ = refs(name)
    rng = np.random.default_rng(17)
    mesh = mesh0.copy(u_prescribed=1e-3 * rng.standard_normal((mesh0.n_nodes, 6)))
    a = None
    if objective == "linear":
        a = np.zeros(mesh.n_dof)
        a[6 * (mesh.n_nodes // 2) + 2] = 1.0
    print(f"[gpu] prescribed displacements {name} {objective}", flush=True)
    r = oracle.analyze(mesh, objective, a=a, pat=pat)
    sso = _sso()
    with _problem(mesh) as p:
        u, st = _solve_tight(p)
        g_val = p.objective(objective, a)
        # the adjoint solve stops on the true residual, above the FP64 floor
        p.set_options(sso.Options(rtol=1e-10, max_it=50000))
        g = p.adjoint(objective, dg_du=a)
    u = u.cpu().numpy().ravel()
    fixed = mesh.fixed.reshape(-1) != 0
    np.testing.assert_array_equal(u[fixed], mesh.u_prescribed.reshape(-1)[fixed])
    err = np.linalg.norm(u - r["u"]) / np.linalg.norm(r["u"])
    print(f"  iters={st['iters']} |du|/|u|={err:.2e} adjoint iters={g['stats']['iters']}")
    assert err <= 1e-10
    assert g_val == pytest.approx(r["g"], rel=1e-10)
    assert _grad_err(g["dg_dxyz"].cpu().numpy(), r["grad_xyz"]) <= 1e-8
    if mesh.n_quads:
        assert _grad_err(g["dg_dt"].cpu().numpy(), r["grad_t"]) <= 1e-8
        assert _grad_err(g["dg_dscale"].cpu().numpy(), r["grad_scale"]) <= 1e-8


@pytest.mark.parametrize("name", ["grid11", "shell8"])
def test_gradient_vs_central_differences(refs, name):
    """The GPU gradient against the oracle's central differences (h = 1e-6) of the whole
    pipeline, 20 sampled parameters."""
    mesh, pat, _ = refs(name)
    print(f"[gpu] fd {name}", flush=True)
    rng = np.random.default_rng(21)
    params = [("xyz", int(rng.integers(mesh.n_nodes)), int(rng.integers(3))) for _ in range(14)]
    if mesh.n_quads:
        params += [("t", int(rng.integers(mesh.n_quads))) for _ in range(3)]
        params += [("scale", int(rng.integers(mesh.n_quads))) for _ in range(3)]
    fd = sensitivity.objective_and_grad_fd(mesh, "compliance", params, pat=pat)
    with _problem(mesh) as p:
        _solve_tight(p)
        g = p.adjoint("compliance")
    gx = g["dg_dxyz"].cpu().numpy()
    gt = g["dg_dt"].cpu().numpy() if mesh.n_quads else None
    gs = g["dg_dscale"].cpu().numpy() if mesh.n_quads else None
    gmax = max(np.abs(gx).max(), np.abs(gt).max() if gt is not None else 0,
               np.abs(gs).max() if gs is not None else 0)
    for prm, v in zip(params, fd):
        gv = gx[prm[1], prm[2]] if prm[0] == "xyz" else (gt if prm[0] == "t" else gs)[prm[1]]
        assert abs(gv - v) <= 1e-5 * max(abs(v), 1e-3 * gmax), (prm, gv, v)


@pytest.mark.parametrize("name", ["shell8", "shell60"])
def test_bitwise_determinism(refs, name):
    mesh, _, _ = refs(name)
    print(f"[gpu] determinism {name}", flush=True)
    outs = []
    for _ in range(2):
        with _problem(mesh, rtol=1e-8) as p:
            u, _ = p.solve()
            vals, _ = p.matrix()
            g = p.adjoint("compliance")
            outs.append([u.cpu().numpy(), vals.cpu().numpy(), g["dg_dxyz"].cpu().numpy(),
                         g["dg_dt"].cpu().numpy()])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("solver", ["standard", "fused", "wg"])
@pytest.mark.parametrize("name", ["grid11", "hub", "mixed", "shell60"])
def test_both_recurrences(refs, name, solver):
    """Standard, single-reduction (fused) and one-workgroup PCG, each chosen explicitly: u and
    the gradients at the parity bars, the recurrence reported back, and two runs bitwise
    equal."""
    sso = _sso()
    mesh, _, r = refs(name)
    code = {"standard": sso.SOLVER_STANDARD, "fused": sso.SOLVER_FUSED,
            "wg": sso.SOLVER_WG}[solver]
    print(f"[gpu] recurrences {name} {solver}", flush=True)
    outs = []
    for _ in range(2):
        with _problem(mesh, solver=code) as p:
            u, st = _solve_tight(p)
            g = p.adjoint("compliance")
            outs.append((u.cpu().numpy().ravel(), g["dg_dxyz"].cpu().numpy()))
        assert st["solver"] == code
    u, gx = outs[0]
    assert np.linalg.norm(u - r["u"]) / np.linalg.norm(r["u"]) <= 1e-10
    assert _grad_err(gx, r["grad_xyz"]) <= 1e-8
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_update_changes_design_and_matches_fresh_problem():
    mesh = small_shell(6, seed=4)
    print("[gpu] update", flush=True)
    rng = np.random.default_rng(0)
    xyz2 = mesh.xyz + rng.normal(0, 0.01, mesh.xyz.shape)
    t2 = mesh.quad_prop[:, 0] * 1.1
    s2 = mesh.quad_scale * 0.9
    m2 = mesh.copy()
    m2.xyz = np.ascontiguousarray(xyz2)
    m2.quad_prop[:, 0] = t2
    m2.quad_scale = s2
    with _problem(mesh) as p:
        p.solve()
        p.update(xyz=xyz2, quad_t=t2, quad_scale=s2)
        u1, _ = p.solve()
        g1 = p.adjoint("compliance")
    with _problem(m2) as q:
        u2, _ = q.solve()
        g2 = q.adjoint("compliance")
    assert torch.equal(u1, u2)
    assert torch.equal(g1["dg_dxyz"], g2["dg_dxyz"])


def test_zero_load_gives_zero_solution():
    mesh = small_shell(4, seed=1)
    mesh.unit_weight = mesh.surface_load = 0.0
    with _problem(mesh) as p:
        u, st = p.solve()
    assert torch.count_nonzero(u).item() == 0
    assert st["iters"] == 0


def test_invalid_inputs_are_rejected():
    sso = _sso()
    print("[gpu] errors", flush=True)
    bad = small_shell(3)
    bad.quad_nodes = bad.quad_nodes.copy()
    bad.quad_nodes[2, 1] = bad.quad_nodes[2, 0]          # repeated node
    with pytest.raises(sso.SSOError) as e:
        _problem(bad)
    assert e.value.status == sso.SSO_EINVAL
    bad = small_shell(3)
    bad.quad_nodes = bad.quad_nodes.copy()
    bad.quad_nodes[0, 0] = bad.n_nodes + 5               # index out of range
    with pytest.raises(sso.SSOError) as e:
        _problem(bad)
    assert e.value.status == sso.SSO_EINVAL
    g = meshgen.gridshell(4)
    g.xyz = g.xyz.copy()
    g.xyz[1] = g.xyz[0]                                   # zero-length member
    with _problem(g) as p:
        with pytest.raises(sso.SSOError) as e:
            p.solve()
        assert e.value.status == sso.SSO_EINVAL
    s = small_shell(3)
    s.quad_prop = s.quad_prop.copy()
    s.quad_prop[0, 3] = 2.0                               # kx != 1
    with _problem(s) as p:
        with pytest.raises(sso.SSOError) as e:
            p.solve()
        assert e.value.status == sso.SSO_EINVAL
    # a concave (dart-shaped) quad: its third corner pulled (in all three coordinates, so that
    # the dart survives the projection onto the element's mean plane of this curved shell) to a
    # tenth of the way from the first; det J at the four Gauss points of the element's frame is
    # then 1.23, 0.19, 0.19, -0.85, though the diagonals still give a positive area (0.76)
    s = small_shell(3)
    s.xyz = s.xyz.copy()
    a, b, c, d = s.quad_nodes[4]
    s.xyz[c] = s.xyz[a] + 0.1 * (s.xyz[c] - s.xyz[a])
    with _problem(s) as p:
        with pytest.raises(sso.SSOError) as e:
            p.solve()
        assert e.value.status == sso.SSO_EINVAL


def test_every_dof_fixed_gives_zero_solution():
    """Degenerate supports (no free DOF): the masked system is the identity with a zero
    right-hand side, so u, the compliance and its gradients are exactly zero."""
    sso = _sso()
    g = meshgen.gridshell(4)
    g.fixed = np.ones_like(g.fixed)
    print("[gpu] every DOF fixed", flush=True)
    with _problem(g) as p:
        u, st = p.solve()
        assert p.last_status == sso.SSO_OK
        assert st["iters"] == 0
        assert not torch.any(u != 0)
        assert p.objective("compliance") == 0.0
        grads = p.adjoint("compliance")
        assert not torch.any(grads["dg_dxyz"] != 0)


def test_unsupported_structure_reports_failure():
    """No supports: K is singular; PCG must stop with breakdown or non-convergence."""
    sso = _sso()
    g = meshgen.gridshell(4)
    g.fixed = np.zeros_like(g.fixed)
    with _problem(g, rtol=1e-12, max_it=400) as p:
        _, st = p.solve(check=False)
        assert p.last_status in (sso.SSO_ENOTCONV, sso.SSO_EBREAKDOWN)
        assert st["iters"] <= 400


def test_debug_mode_checks_every_pattern(monkeypatch):
    """HIPSSO_DEBUG: the GPU-built pattern, permutation and padded rows of every parity structure
    pass the host-side check, and the debug problem's solve is bitwise the plain one's."""
    sso = _sso()
    print("[gpu] debug-mode pattern checks", flush=True)
    for name, make in CASES.items():
        mesh = make()
        monkeypatch.setenv("HIPSSO_DEBUG", "1")
        with _problem(mesh, rtol=1e-10) as p:
            u_dbg, _ = p.solve(check=False)
            u_dbg = u_dbg.cpu()
        monkeypatch.delenv("HIPSSO_DEBUG")
        with _problem(mesh, rtol=1e-10) as q:
            u, _ = q.solve(check=False)
        assert torch.equal(u_dbg, u.cpu()), name


def test_pool_trim_between_solves_changes_nothing():
    """Destroyed problems' memory stays in the library's pool; trimming it back to the driver
    and solving again gives bitwise the same displacements."""
    import paper_2407_20026_amd as sso
    print("[gpu] pool trim", flush=True)
    mesh = meshgen.shell(12, seed=5)
    us = []
    for trim in (False, True, False):
        with sso.Problem(mesh, sso.Options(rtol=1e-10)) as p:
            u, _ = p.solve()
            us.append(u.cpu())
        torch.cuda.synchronize()
        if trim:
            sso.pool_trim(0, 0)
    assert torch.equal(us[0], us[1]) and torch.equal(us[0], us[2])
