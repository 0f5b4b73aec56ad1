"""Pins of the oracle's 12-DOF space-frame element against closed forms.

Cantilever formulas (Euler-Bernoulli, end loads -- for which cubic Hermite elements are exact):
tip deflection P L^3 / (3 E I), tip slope P L^2 / (2 E I), axial P L / (E A), twist T L / (G J),
end moment M: deflection M L^2 / (2 E I), slope M L / (E I)."""
import numpy as np
import pytest

import meshgen
from oracle import assembly, elements, sensitivity, solve
from structures import cantilever, rigid_body_modes

DIRECTIONS = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 2, 3), (-2, 0.5, 1), (0.3, -1, -0.2)]


def _tip_response(mesh, load6):
    f = np.zeros(mesh.n_dof)
    f[-6:] = load6
    K = assembly.assemble(mesh)
    u, _ = solve.solve_eliminated(mesh, K, f)
    return u[-6:]


@pytest.mark.parametrize("d", DIRECTIONS)
@pytest.mark.parametrize("n_el", [1, 5])
def test_cantilever_axial_torsion_isotropic_bending(d, n_el):
    """Iy = Iz: bending is orientation-free, so any load perpendicular to the axis works."""
    E, nu, A, I, J, L = 200e9, 0.3, 3e-3, 4e-6, 7e-6, 2.5
    G = E / (2 * (1 + nu))
    m = cantilever(d, L=L, n_el=n_el, E=E, nu=nu, A=A, Iy=I, Iz=I, J=J)
    e1 = np.asarray(d, float) / np.linalg.norm(d)
    perp = np.cross(e1, [0.3, 0.7, -0.4])
    perp /= np.linalg.norm(perp)
    P, T, M = 1234.0, 567.0, 890.0
    # axial
    r = _tip_response(m, np.r_[P * e1, 0, 0, 0])
    np.testing.assert_allclose(r[:3], P * L / (E * A) * e1, rtol=1e-12, atol=1e-20)
    # torsion
    r = _tip_response(m, np.r_[0, 0, 0, T * e1])
    np.testing.assert_allclose(r[3:], T * L / (G * J) * e1, rtol=1e-12, atol=1e-20)
    # transverse tip force
    r = _tip_response(m, np.r_[P * perp, 0, 0, 0])
    np.testing.assert_allclose(r[:3], P * L**3 / (3 * E * I) * perp, rtol=1e-12, atol=1e-20)
    np.testing.assert_allclose(r[3:], P * L**2 / (2 * E * I) * np.cross(e1, perp), rtol=1e-12,
                               atol=1e-20)
    # tip moment about perp
    r = _tip_response(m, np.r_[0, 0, 0, M * perp])
    np.testing.assert_allclose(r[3:], M * L / (E * I) * perp, rtol=1e-12, atol=1e-20)
    np.testing.assert_allclose(r[:3], M * L**2 / (2 * E * I) * np.cross(perp, e1), rtol=1e-12,
                               atol=1e-20)


@pytest.mark.parametrize("n_el", [1, 4])
def test_cantilever_axis_assignment(n_el):
    """Member along +X: local y = +Y (bending uses Iz), local z = +Z (bending uses Iy)."""
    E, Iy, Iz, L = 70e9, 2e-6, 9e-6, 3.0
    m = cantilever((1, 0, 0), L=L, n_el=n_el, E=E, Iy=Iy, Iz=Iz)
    P = 1000.0
    r = _tip_response(m, np.r_[0, P, 0, 0, 0, 0])
    assert r[1] == pytest.approx(P * L**3 / (3 * E * Iz), rel=1e-12)
    assert r[5] == pytest.approx(P * L**2 / (2 * E * Iz), rel=1e-12)
    r = _tip_response(m, np.r_[0, 0, P, 0, 0, 0])
    assert r[2] == pytest.approx(P * L**3 / (3 * E * Iy), rel=1e-12)
    assert r[4] == pytest.approx(-P * L**2 / (2 * E * Iy), rel=1e-12)


def test_vertical_member_uses_global_y_as_local_y():
    """Vertical member: local y = global Y (bending about local z uses Iz)."""
    E, Iy, Iz, L = 70e9, 2e-6, 9e-6, 3.0
    m = cantilever((0, 0, 1), L=L, n_el=2, E=E, Iy=Iy, Iz=Iz)
    P = 1000.0
    r = _tip_response(m, np.r_[0, P, 0, 0, 0, 0])
    assert r[1] == pytest.approx(P * L**3 / (3 * E * Iz), rel=1e-12)
    r = _tip_response(m, np.r_[P, 0, 0, 0, 0, 0])
    assert r[0] == pytest.approx(P * L**3 / (3 * E * Iy), rel=1e-12)


def test_local_matrix_is_singular_with_six_rigid_modes():
    L = np.array([1.7])
    k = elements.beam_local_k(np.array([2e11]), np.array([8e10]), np.array([1e-3]),
                              np.array([2e-6]), np.array([3e-6]), np.array([4e-6]), L)[0]
    ev = np.linalg.eigvalsh(k)
    assert np.all(np.abs(ev[:6]) < 1e-9 * ev[-1])
    assert ev[6] > 1e-6 * ev[-1]
    np.testing.assert_array_equal(k, k.T)


def test_gridshell_rigid_body_and_symmetry():
    m = meshgen.gridshell(5, seed=3)
    K = assembly.assemble(m).toarray()
    np.testing.assert_allclose(K, K.T, rtol=0, atol=1e-9 * np.abs(K).max())
    modes = rigid_body_modes(m.xyz)
    for r in modes:
        assert np.linalg.norm(K @ r) <= 1e-11 * np.linalg.norm(K, 2) * np.linalg.norm(r)
    ev = np.linalg.eigvalsh(K)
    assert ev[6] > 1e-8 * ev[-1]


def test_beam_complex_step_matches_central_difference():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(7, 2, 3))
    prop = np.tile([2e11, 8e10, 1e-3, 2e-6, 3e-6, 4e-6], (7, 1))
    for d in range(6):
        Xc = X.astype(complex)
        Xc[:, d // 3, d % 3] += 1e-30j
        cs = np.imag(elements.beam_K(Xc, prop)) / 1e-30
        h = 1e-6
        Xp, Xm = X.copy(), X.copy()
        Xp[:, d // 3, d % 3] += h
        Xm[:, d // 3, d % 3] -= h
        fd = (elements.beam_K(Xp, prop) - elements.beam_K(Xm, prop)) / (2 * h)
        np.testing.assert_allclose(cs, fd, rtol=1e-6, atol=1e-8 * np.abs(cs).max())
