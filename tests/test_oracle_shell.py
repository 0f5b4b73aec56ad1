"""Pins of the oracle's 4-node flat shell (Q4 membrane + MITC4 plate + drilling + warp offset).

Closed forms used:
* rigid-body null space of the unconstrained K (6 modes, translations and rotations);
* membrane and bending patch tests (constant strain / constant curvature reproduced exactly);
* uniaxial tension of a free strip: u = sigma L / E, lateral contraction -nu sigma / E;
* Navier series for the simply supported square Kirchhoff plate under uniform load
  (Timoshenko & Woinowsky-Krieger): w(a/2, a/2) = 16 q a^4 / (pi^6 D) sum_{m,n odd}
  (-1)^((m+n)/2-1) / (m n (m^2 + n^2)^2) ~ 0.00406 q a^4 / D;
* Marcus-moment relation for the hard simply supported Mindlin plate:
  w_M = w_K + M / (kappa G t), with M the solution of -lap M = q, M = 0 on the edge;
* complex-step element derivatives against central differences, and the thickness derivative
  against its closed form dK/dt = (K_m + K_s + K_d) / t + 3 K_b / t.
"""
import numpy as np
import pytest

from oracle import assembly, elements, solve
from structures import boundary_nodes, plate, rigid_body_modes, solve_prescribed


def _series(m_terms=399):
    sK = sM = 0.0
    for i in range(1, m_terms, 2):
        for j in range(1, m_terms, 2):
            sg = (-1.0) ** ((i + j) // 2 - 1)
            sK += sg / (i * j * (i * i + j * j) ** 2)
            sM += sg / (i * j * (i * i + j * j))
    return sK, sM


def _centre(mm):
    return (mm // 2) * (mm + 1) + mm // 2


SHAPES = {
    "flat": None,
    "cylinder": lambda x, y: np.sqrt(4.0 - (x - 0.5) ** 2) - 2.0,
    "warped": lambda x, y: 0.3 * np.sin(2 * x) * np.cos(1.5 * y) + 0.2 * x * y,
}


@pytest.mark.parametrize("shape", list(SHAPES))
def test_rigid_body_null_space_and_symmetry(shape):
    m = plate(4, a=1.5, t=0.05, jitter=0.25, seed=1, z=SHAPES[shape])
    K = assembly.assemble(m).toarray()
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    nK = np.linalg.norm(K, 2)
    for r in rigid_body_modes(m.xyz):
        assert np.linalg.norm(K @ r) <= 1e-11 * nK * np.linalg.norm(r)
    ev = np.linalg.eigvalsh(K)
    assert np.all(np.abs(ev[:6]) < 1e-12 * ev[-1])
    assert ev[6] > 1e-8 * ev[-1]


def test_single_warped_element_rigid_modes():
    X = np.array([[[0.0, 0.0, 0.1], [1.1, -0.1, -0.05], [1.0, 0.9, 0.12], [-0.1, 1.0, -0.08]]])
    prop = np.array([[0.02, 3e10, 0.2, 1.0, 1.0]])
    K = elements.shell_K(X, prop)[0]
    modes = rigid_body_modes(X[0])
    for r in modes:
        assert np.linalg.norm(K @ r) <= 1e-12 * np.linalg.norm(K, 2) * np.linalg.norm(r)


def _patch(m=2):
    p = plate(m, a=1.0, t=0.01, E=2e9, nu=0.25, jitter=0.3, seed=7)
    return p


def test_membrane_patch_constant_strain():
    p = _patch(3)
    K = assembly.assemble(p)
    a0, a1, a2, b0, b1, b2 = 1e-3, 2e-3, -1.5e-3, -2e-3, 0.7e-3, 1.1e-3
    x, y = p.xyz[:, 0], p.xyz[:, 1]
    exact = np.zeros((p.n_nodes, 6))
    exact[:, 0] = a0 + a1 * x + a2 * y
    exact[:, 1] = b0 + b1 * x + b2 * y
    exact[:, 5] = 0.5 * (b1 - a2)
    presc = {}
    for nd in boundary_nodes(3):
        for c in range(6):
            presc[6 * nd + c] = exact[nd, c]
    for nd in range(p.n_nodes):      # out-of-plane DOFs held at the exact (zero) value
        for c in (2, 3, 4):
            presc[6 * nd + c] = 0.0
    u = solve_prescribed(K, np.zeros(p.n_dof), presc).reshape(-1, 6)
    np.testing.assert_allclose(u, exact, rtol=0, atol=1e-10 * np.abs(exact).max())


def test_bending_patch_constant_curvature():
    p = _patch(3)
    K = assembly.assemble(p)
    c1, c2, c3, d0, d1, d2 = 2e-3, -1e-3, 1.5e-3, 1e-4, -2e-4, 3e-4
    x, y = p.xyz[:, 0], p.xyz[:, 1]
    w = 0.5 * (c1 * x * x + c2 * y * y + c3 * x * y) + d0 + d1 * x + d2 * y
    wx = c1 * x + 0.5 * c3 * y + d1
    wy = c2 * y + 0.5 * c3 * x + d2
    exact = np.zeros((p.n_nodes, 6))
    exact[:, 2] = w
    exact[:, 3] = wy          # theta_x = -beta_y = w,y
    exact[:, 4] = -wx         # theta_y = beta_x = -w,x
    presc = {}
    for nd in boundary_nodes(3):
        for c in range(6):
            presc[6 * nd + c] = exact[nd, c]
    for nd in range(p.n_nodes):
        for c in (0, 1, 5):
            presc[6 * nd + c] = 0.0
    u = solve_prescribed(K, np.zeros(p.n_dof), presc).reshape(-1, 6)
    np.testing.assert_allclose(u, exact, rtol=0, atol=1e-10 * np.abs(exact).max())


def test_uniaxial_tension_membrane_modulus():
    """Strip [0, a]^2, left edge held in x (one node also in y), right edge pulled with the
    consistent nodal forces of a uniform traction sigma; free contraction."""
    mm, a, t, E, nu, sig = 4, 2.0, 0.05, 3e10, 0.2, 1e6
    p = plate(mm, a=a, t=t, E=E, nu=nu)
    x = p.xyz[:, 0]
    left = np.flatnonzero(np.isclose(x, 0))
    right = np.flatnonzero(np.isclose(x, a))
    p.fixed[:, 2:5] = 1                       # out-of-plane held
    p.fixed[left, 0] = 1
    p.fixed[left[0], 1] = 1
    f = np.zeros((p.n_nodes, 6))
    edge_force = sig * t * a / mm
    for nd in right:
        yv = p.xyz[nd, 1]
        f[nd, 0] = edge_force * (0.5 if np.isclose(yv, 0) or np.isclose(yv, a) else 1.0)
    K = assembly.assemble(p)
    u, _ = solve.solve_eliminated(p, K, f.reshape(-1))
    u = u.reshape(-1, 6)
    np.testing.assert_allclose(u[:, 0], sig / E * x, rtol=0, atol=1e-12 * sig / E * a)
    np.testing.assert_allclose(u[:, 1], -nu * sig / E * p.xyz[:, 1], rtol=0,
                               atol=1e-12 * sig / E * a)


@pytest.mark.parametrize("mm,tol", [(10, 4e-3), (20, 1e-3), (40, 2.5e-4)])
def test_navier_thin_plate(mm, tol):
    a, t, E, nu, q = 1.0, 1e-3, 1e9, 0.3, 1.0
    p = plate(mm, a=a, t=t, E=E, nu=nu, q=q)
    p.fixed[boundary_nodes(mm)] = [1, 1, 1, 0, 0, 0]
    K = assembly.assemble(p)
    u, _ = solve.solve_eliminated(p, K, assembly.load_vector(p))
    D = E * t**3 / (12 * (1 - nu**2))
    sK, _ = _series()
    w = 16 * q * a**4 / (np.pi**6 * D) * sK
    assert w == pytest.approx(0.00406 * q * a**4 / D, rel=1e-3)
    err = abs(-u[6 * _centre(mm) + 2] - w) / w
    assert err < tol


@pytest.mark.parametrize("mm,tol", [(10, 4e-3), (20, 1e-3)])
def test_mindlin_hard_simply_supported_plate(mm, tol):
    a, t, E, nu, q = 1.0, 0.1, 1e9, 0.3, 1.0
    p = plate(mm, a=a, t=t, E=E, nu=nu, q=q)
    p.fixed[boundary_nodes(mm)] = [1, 1, 1, 0, 0, 0]
    x, y = p.xyz[:, 0], p.xyz[:, 1]
    p.fixed[np.isclose(x, 0) | np.isclose(x, a), 3] = 1     # tangential rotation held
    p.fixed[np.isclose(y, 0) | np.isclose(y, a), 4] = 1
    K = assembly.assemble(p)
    u, _ = solve.solve_eliminated(p, K, assembly.load_vector(p))
    D = E * t**3 / (12 * (1 - nu**2))
    G = E / (2 * (1 + nu))
    sK, sM = _series()
    wK = 16 * q * a**4 / (np.pi**6 * D) * sK
    M = 16 * q * a**2 / np.pi**4 * sM
    assert M == pytest.approx(0.0736713 * q * a**2, rel=1e-5)
    wM = wK + M / (5.0 / 6.0 * G * t)
    err = abs(-u[6 * _centre(mm) + 2] - wM) / wM
    assert err < tol


def _random_quads(n, seed=0):
    rng = np.random.default_rng(seed)
    base = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], float)
    X = base[None] * rng.uniform(0.5, 2.0, (n, 1, 1)) + rng.uniform(-0.15, 0.15, (n, 4, 3))
    prop = np.stack([rng.uniform(0.05, 0.3, n), np.full(n, 3e10), np.full(n, 0.2),
                     np.ones(n), np.ones(n)], 1)
    return X, prop


def test_shell_complex_step_matches_central_difference():
    X, prop = _random_quads(6)
    scale = np.linspace(0.5, 1.5, 6)
    for d in range(13):
        Xc, pc = X.astype(complex), prop.astype(complex)
        if d < 12:
            Xc[:, d // 3, d % 3] += 1e-30j
        else:
            pc[:, 0] += 1e-30j
        cs = np.imag(elements.shell_K(Xc, pc, scale.astype(complex))) / 1e-30
        h = 1e-6
        Xp, Xm, pp, pm = X.copy(), X.copy(), prop.copy(), prop.copy()
        if d < 12:
            Xp[:, d // 3, d % 3] += h
            Xm[:, d // 3, d % 3] -= h
        else:
            pp[:, 0] += h
            pm[:, 0] -= h
        fd = (elements.shell_K(Xp, pp, scale) - elements.shell_K(Xm, pm, scale)) / (2 * h)
        np.testing.assert_allclose(cs, fd, rtol=0, atol=2e-7 * np.abs(cs).max())


def test_thickness_derivative_closed_form():
    X, prop = _random_quads(5, seed=3)
    Km, Kb, Ks, Kd = elements.shell_K_parts(X, prop)
    t = prop[:, 0][:, None, None]
    closed = (Km + Ks + Kd) / t + 3 * Kb / t
    pc = prop.astype(complex)
    pc[:, 0] += 1e-30j
    cs = np.imag(elements.shell_K(X.astype(complex), pc)) / 1e-30
    np.testing.assert_allclose(cs, closed, rtol=0, atol=1e-13 * np.abs(closed).max())


def test_load_lumping_total_equals_area_times_pressure():
    p = plate(5, a=3.0, t=0.2, q=2e3, jitter=0.3)
    p.unit_weight = 25e3
    f = assembly.load_vector(p).reshape(-1, 6)
    total = -(25e3 * 0.2 + 2e3) * 9.0
    assert f[:, 2].sum() == pytest.approx(total, rel=1e-13)
    assert np.all(f[:, [0, 1, 3, 4, 5]] == 0)


def test_area_of_planar_quad_is_exact():
    X = np.array([[[0.0, 0, 0], [2.0, 0, 0], [2.5, 1.5, 0], [0.2, 1.0, 0]]])
    # shoelace area of the polygon
    x, y = X[0, :, 0], X[0, :, 1]
    shoelace = 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))
    assert elements.shell_area(X)[0] == pytest.approx(shoelace, rel=1e-15)


def test_dart_quad_of_a_curved_shell_has_a_negative_gauss_jacobian():
    """The inverted-element input of the GPU error tests: on the curved 3x3 shell, the centre
    quad's third corner pulled in all three coordinates to a tenth of the way from the first
    gives det J < 0 at a Gauss point of the mean-plane frame with a positive area; pulled in x
    and y only, the corner keeps its height and the projected quad stays convex."""
    import meshgen
    base = meshgen.shell(3, L=8.0, seed=3)
    a, b, c, d = base.quad_nodes[4]
    for full, negative in ((True, True), (False, False)):
        xyz = base.xyz.copy()
        k = slice(None) if full else slice(0, 2)
        xyz[c, k] = xyz[a, k] + 0.1 * (xyz[c, k] - xyz[a, k])
        _, x, y, _, area = elements.shell_frame(xyz[[a, b, c, d]][None])
        assert area[0] > 0.0
        assert (elements.min_gauss_detJ(x, y)[0] < 0.0) == negative
