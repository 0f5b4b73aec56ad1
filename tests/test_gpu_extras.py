"""Optimisation extras on the GPU against the oracle: the penalised material volume of the size
optimisation (Sec. 3.3) with its gradient, and the sensitivity hat filter (Sec. 3.1-3.2).

Bars: W and its gradient (no solve involved) within 1e-12; g, c and the full gradient, which
go through the solve and the adjoint at rtol 1e-10, within 1e-8 relative (inf-norm) like the
other adjoint gradients; the filter within 1e-12 relative per entry."""
import numpy as np
import pytest

import meshgen
from oracle import extras, sensitivity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mesh():
    m = meshgen.shell(8, L=8.0, seed=3)
    m.quad_prop[:, 0] = np.random.default_rng(4).uniform(0.05, 0.3, m.n_quads)
    return m


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("case", ["violated", "inactive"])
def test_size_objective_matches_oracle(case):
    import paper_2407_20026_amd as sso
    m = _mesh()
    uz = sensitivity.forward(m)["u"].reshape(-1, 6)[:, 2]
    u_max = 0.5 * np.abs(uz).max() if case == "violated" else 1e3
    t_min = float(np.median(m.quad_prop[:, 0]))
    eps1 = 0.7
    r = extras.size_objective(m, eps1, u_max, t_min)
    print(f"[gpu] size objective {case}: c={r['c']:.4e} W={r['W']:.6e}", flush=True)
    with sso.Problem(m, sso.Options(rtol=1e-10, max_it=50000)) as p:
        p.solve()
        out = p.size_objective(eps1, u_max, t_min)
    assert out["W"] == pytest.approx(r["W"], rel=1e-12)
    assert out["c"] == pytest.approx(r["c"], rel=1e-8, abs=0.0)
    assert out["g"] == pytest.approx(r["g"], rel=1e-8)
    gx, gt = out["dg_dxyz"].cpu().numpy(), out["dg_dt"].cpu().numpy()
    tol = 1e-12 if case == "inactive" else 1e-8
    print(f"  grad errors xyz {_rel(gx, r['grad_xyz']):.2e} t {_rel(gt, r['grad_t']):.2e}")
    assert _rel(gx, r["grad_xyz"]) <= tol
    assert _rel(gt, r["grad_t"]) <= tol
    if case == "inactive":
        assert out["c"] == 0.0


def test_size_objective_rejects_bad_parameters():
    import paper_2407_20026_amd as sso
    with sso.Problem(_mesh()) as p:
        p.solve()
        for args in ((-1.0, 0.01, 0.1), (1.0, 0.0, 0.1), (1.0, 0.01, -0.1),
                     (1.0, float("nan"), 0.1)):
            with pytest.raises(sso.SSOError):
                p.size_objective(*args)


@pytest.mark.parametrize("which", ["design_nodes", "all_nodes"])
def test_hat_filter_matches_oracle(which):
    import paper_2407_20026_amd as sso
    m = meshgen.shell(20, seed=5)          # 441 nodes: two tiles of 256, the second ragged
    rng = np.random.default_rng(8)
    if which == "design_nodes":
        nodes = np.flatnonzero(m.fixed[:, 2] == 0).astype(np.int32)
    else:
        nodes = np.arange(m.n_nodes, dtype=np.int32)
    g = rng.normal(size=len(nodes))
    ref = extras.hat_filter(m.xyz, nodes, g, 2.5)
    print(f"[gpu] hat filter {which}: {len(nodes)} nodes", flush=True)
    with sso.Problem(m) as p:
        out = p.hat_filter(g, 2.5, nodes=None if which == "all_nodes" else nodes)
    out = out.cpu().numpy()
    err = np.abs(out - ref) / np.maximum(np.abs(ref), 1e-300)
    print(f"  max rel err {err.max():.2e}")
    assert np.all(err <= 1e-12)


def test_hat_filter_rejects_out_of_range_nodes():
    import paper_2407_20026_amd as sso
    m = meshgen.shell(4, seed=5)
    with sso.Problem(m) as p:
        with pytest.raises(sso.SSOError):
            p.hat_filter(np.ones(3), 1.0, nodes=np.array([0, m.n_nodes, 1], np.int32))
        with pytest.raises(sso.SSOError):
            p.hat_filter(np.ones(3), 0.0)
        # the problem stays usable
        out = p.hat_filter(np.ones(3), 1.0, nodes=np.array([0, 1, 2], np.int32))
    np.testing.assert_allclose(out.cpu().numpy(), 1.0, rtol=1e-15)
