"""Pins of the oracle's optimisation extras: the penalised material volume of the size
optimisation example (Sec. 3.3) against closed forms on a flat plate and, with its adjoint
displacement penalty, against central differences of the whole pipeline; the self-adaptive
penalty rule; the sensitivity hat filter (Sec. 3.1) against hand-computed weights and its
invariants."""
import numpy as np
import pytest

import meshgen
from oracle import extras, sensitivity
from structures import plate


def test_volume_of_flat_plate_closed_form():
    m, a = 4, 2.0
    p = plate(m, a=a)
    t = np.random.default_rng(1).uniform(0.02, 0.08, m * m)
    p.quad_prop[:, 0] = t
    t_min = 0.05
    W, gx, gt = extras.penalised_volume(p, t_min)
    h2 = (a / m) ** 2
    assert W == pytest.approx(h2 * t.sum() + np.sum(np.maximum(0.0, (t_min - t) / t_min)),
                              rel=1e-14)
    np.testing.assert_allclose(gt, h2 - (t < t_min) / t_min, rtol=1e-14)
    # flat plate: moving a node out of plane leaves every area unchanged to first order
    np.testing.assert_allclose(gx[:, 2], 0.0, atol=1e-15)


def test_volume_gradient_at_corner_and_interior_nodes():
    """Square elements of side h: moving the corner node (0, 0) along x by d shrinks its quad's
    area |d13 x d24| / 2 by h d / 2; an interior node of a uniform-thickness regular grid moves
    no volume to first order (its four quads cancel)."""
    m, a, t = 3, 3.0, 0.1
    p = plate(m, a=a, t=t)
    _, gx, _ = extras.penalised_volume(p, 0.01)
    h = a / m
    assert gx[0, 0] == pytest.approx(-t * h / 2, rel=1e-13)
    assert gx[0, 1] == pytest.approx(-t * h / 2, rel=1e-13)
    interior = (m + 1) + 1
    np.testing.assert_allclose(gx[interior], 0.0, atol=1e-15)


def _size_case():
    m = meshgen.shell(5, L=6.0, seed=11)
    m.quad_prop[:, 0] = np.random.default_rng(4).uniform(0.05, 0.3, m.n_quads)
    u = sensitivity.forward(m)["u"].reshape(-1, 6)[:, 2]
    u_max = 0.5 * np.abs(u).max()
    t_min = float(np.median(m.quad_prop[:, 0]))
    # stay away from the kinks of max(0, .) for the finite differences
    assert np.min(np.abs(np.abs(u) / u_max - 1.0)) > 1e-3
    return m, u_max, t_min


def test_size_objective_gradient_vs_fd():
    m, u_max, t_min = _size_case()
    t = m.quad_prop[:, 0]
    # thickness parameters away from t_min (the median itself sits on the kink)
    cand = np.flatnonzero(np.abs(t - t_min) > 1e-3)[:6]
    eps1 = 0.7
    r = extras.size_objective(m, eps1, u_max, t_min)
    assert r["c"] > 0.0
    h = 1e-6
    rng = np.random.default_rng(3)
    params = [("t", int(e)) for e in cand] + \
        [("xyz", int(n), int(k)) for n, k in zip(rng.integers(0, m.n_nodes, 8),
                                                 rng.integers(0, 3, 8))]
    scale = max(np.abs(r["grad_xyz"]).max(), np.abs(r["grad_t"]).max())
    for p in params:
        vals = []
        for s in (1.0, -1.0):
            xyz, tt = m.xyz.copy(), t.copy()
            if p[0] == "t":
                tt[p[1]] += s * h
            else:
                xyz[p[1], p[2]] += s * h
            vals.append(extras.size_objective_value(m, eps1, u_max, t_min, xyz=xyz, quad_t=tt))
        fd = (vals[0] - vals[1]) / (2 * h)
        g = r["grad_t"][p[1]] if p[0] == "t" else r["grad_xyz"][p[1], p[2]]
        assert abs(g - fd) <= 1e-5 * max(abs(fd), 1e-3 * scale), (p, g, fd)


def test_size_objective_without_violation_is_the_volume():
    m, _, t_min = _size_case()
    r = extras.size_objective(m, 2.0, 1e3, t_min)
    W, gx, gt = extras.penalised_volume(m, t_min)
    assert r["c"] == 0.0 and r["g"] == W
    np.testing.assert_array_equal(r["grad_t"], gt)
    np.testing.assert_array_equal(r["grad_xyz"], gx)


def test_self_adaptive_penalty_rule():
    assert extras.update_eps1(2.0, True) == pytest.approx(2.03)
    assert extras.update_eps1(2.03, False) == pytest.approx(2.0)
    assert extras.update_eps1(1.0, True, kappa=1.1) == pytest.approx(1.1)


def test_hat_filter_hand_computed_weights():
    xyz = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0], [9.0, 9.0, 9.0]])
    out = extras.hat_filter(xyz, [0, 1, 2], [1.0, 2.0, 4.0], 1.5)
    # weights max(0, 1.5 - d): row 0 (1.5, 0.5, 0), row 1 (0.5, 1.5, 0.5), row 2 (0, 0.5, 1.5)
    np.testing.assert_allclose(out, [2.5 / 2.0, 5.5 / 2.5, 7.0 / 2.0], rtol=1e-15)


def test_hat_filter_invariants():
    rng = np.random.default_rng(5)
    xyz = rng.uniform(0.0, 10.0, (60, 3))
    nodes = rng.permutation(60)[:40]
    g = rng.normal(size=40)
    # constant sensitivities stay constant; a radius below the smallest spacing is the identity
    np.testing.assert_allclose(extras.hat_filter(xyz, nodes, np.full(40, 3.0), 4.0), 3.0,
                               rtol=1e-14)
    P = xyz[nodes]
    dmin = min(np.linalg.norm(P[i] - P[j]) for i in range(40) for j in range(i))
    np.testing.assert_array_equal(extras.hat_filter(xyz, nodes, g, 0.9 * dmin), g)
    # relabelling the design nodes relabels the result
    perm = rng.permutation(40)
    a = extras.hat_filter(xyz, nodes, g, 3.0)
    b = extras.hat_filter(xyz, nodes[perm], g[perm], 3.0)
    np.testing.assert_allclose(b, a[perm], rtol=1e-13)
    # a weighted average: inside the range of the inputs
    assert np.all(a <= g.max() + 1e-12) and np.all(a >= g.min() - 1e-12)
