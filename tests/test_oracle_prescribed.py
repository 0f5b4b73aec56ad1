"""Pins of the oracle with nonzero prescribed support displacements (Sec. 2.2.1, Eqs. 2-3 with
V u = b): the paper's Lagrange-multiplier system with b, a support motion that is a rigid-body
mode (it must add the mode to the displacement and change nothing else), superposition of
load and support motion, and the adjoint gradient against central differences of the whole
pipeline (with b the compliance is no longer self-adjoint, so lambda needs its own solve)."""
import numpy as np
import pytest

import meshgen
import oracle
from oracle import assembly, sensitivity, solve
from structures import rigid_body_modes
from test_oracle_system import _check_fd, _fd_params


def _mesh(which):
    if which == "grid":
        return meshgen.gridshell(5, seed=2)
    return meshgen.shell(4, L=6.0, seed=11)


def _with_b(m, seed=3, scale=1e-3):
    rng = np.random.default_rng(seed)
    return m.copy(u_prescribed=scale * rng.standard_normal((m.n_nodes, 6)))


@pytest.mark.parametrize("which", ["grid", "shell"])
def test_lagrange_system_with_prescribed_values_equals_elimination(which):
    m = _with_b(_mesh(which))
    K = assembly.assemble(m)
    f = assembly.load_vector(m)
    b = solve.prescribed(m)
    C = np.flatnonzero(m.fixed.reshape(-1))
    u_el, _ = solve.solve_eliminated(m, K, f, b=b)
    u_lg, _ = solve.solve_lagrange(m, K, f, b[C])
    np.testing.assert_allclose(u_lg, u_el, rtol=0, atol=1e-10 * np.abs(u_el).max())
    np.testing.assert_array_equal(u_el[C], b[C])


@pytest.mark.parametrize("which", ["grid", "shell"])
@pytest.mark.parametrize("mode", range(6))
def test_rigid_support_motion_adds_the_mode(which, mode):
    m0 = _mesh(which)
    rb = 1e-3 * rigid_body_modes(m0.xyz)[mode]
    m = m0.copy(u_prescribed=rb.reshape(-1, 6))
    u0 = oracle.analyze(m0, "compliance")["u"]
    u = sensitivity.forward(m)["u"]
    np.testing.assert_allclose(u - rb, u0, rtol=0,
                               atol=1e-9 * max(np.abs(u0).max(), np.abs(rb).max()))


@pytest.mark.parametrize("which", ["grid", "shell"])
def test_superposition_of_load_and_support_motion(which):
    m = _with_b(_mesh(which), seed=5)
    u_both = sensitivity.forward(m)["u"]
    u_load = sensitivity.forward(m.copy(u_prescribed=None))["u"]
    unloaded = m.copy(f_nodal=np.zeros_like(m.f_nodal), unit_weight=0.0, surface_load=0.0)
    u_motion = sensitivity.forward(unloaded)["u"]
    np.testing.assert_allclose(u_both, u_load + u_motion, rtol=0,
                               atol=1e-10 * np.abs(u_both).max())


@pytest.mark.parametrize("objective", ["compliance", "linear"])
def test_gradient_with_prescribed_displacements_vs_fd(objective):
    m = _with_b(meshgen.shell(5, L=6.0, seed=11), seed=7, scale=2e-3)
    m.quad_scale = np.random.default_rng(2).uniform(0.2, 1.0, m.n_quads) ** 3
    a = None
    if objective == "linear":
        a = np.zeros(m.n_dof)
        a[6 * (m.n_nodes // 2) + 2] = 1.0
    r = oracle.analyze(m, objective, a=a)
    if objective == "compliance":
        # not self-adjoint any more: lambda solves K lambda = f with homogeneous supports
        assert np.abs(r["lam"] - r["u"]).max() > 1e-3 * np.abs(r["u"]).max()
    _check_fd(m, r, objective, _fd_params(m, 16, 4), a=a)


def test_grid_gradient_with_prescribed_displacements_vs_fd():
    m = _with_b(meshgen.gridshell(7, seed=4), seed=9, scale=5e-3)
    r = oracle.analyze(m, "strain_energy")
    _check_fd(m, r, "strain_energy", _fd_params(m, 16, 5))
