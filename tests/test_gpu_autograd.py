"""torch.autograd through the HIP analysis: the network-driven shell batch (MLP -> heights and
thickness -> rho^3-scaled shells -> mean compliance) against the oracle adjoint chained through
the network (every weight) and central finite differences of the oracle (h = 1e-6) on 20 random
network parameters, and the displacement function's backward against the oracle adjoint."""
import numpy as np
import pytest

import meshgen
import oracle
from oracle import assembly

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _sigmoid(v):
    return 1.0 / (1.0 + np.exp(-v))


def _oracle_loss(params, base, rhos, L):
    """Mean oracle compliance for network weights params = (W1, b1, W2, b2) (numpy)."""
    W1, b1, W2, b2 = params
    xy = base.xyz[:, :2]
    o = np.tanh((xy / L) @ W1.T + b1) @ W2.T + b2
    z = 3.0 * _sigmoid(o[:, 0])
    t = (0.1 + 0.2 * _sigmoid(o[:, 1]))[base.quad_nodes].mean(axis=1)
    total = 0.0
    for rho in rhos:
        m = base.copy()
        m.xyz = np.ascontiguousarray(np.column_stack([xy, z]))
        m.quad_prop[:, 0] = t
        m.quad_scale = rho ** 3
        fw = oracle.sensitivity.forward(m)
        total += float(fw["fm"] @ fw["u"])
    return total / len(rhos)


def _oracle_adjoint_grads(net_cpu, base, rhos, L):
    """Network gradient of the mean oracle compliance: the oracle adjoint (dc/dz, dc/dt per
    variant) chained through the MLP with torch's CPU autograd."""
    from paper_2407_20026_amd.shellnet import geometry
    xy = torch.tensor(base.xyz[:, :2])
    qn = torch.tensor(base.quad_nodes.astype(np.int64))
    xyz, t = geometry(net_cpu, xy, L, qn)
    gx = np.zeros((base.n_nodes, 3))
    gt = np.zeros(base.n_quads)
    for rho in rhos:
        m = base.copy()
        m.xyz = np.ascontiguousarray(xyz.detach().numpy())
        m.quad_prop[:, 0] = t.detach().numpy()
        m.quad_scale = rho ** 3
        r = oracle.analyze(m, "compliance")
        gx += r["grad_xyz"] / len(rhos)
        gt += r["grad_t"] / len(rhos)
    ((xyz * torch.tensor(gx)).sum() + (t * torch.tensor(gt)).sum()).backward()
    return [p.grad.numpy().copy() for p in net_cpu.parameters()]


def test_network_batch_gradient_vs_oracle_fd():
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.shellnet import DesignMLP, ShellBatch
    print("[gpu] shellnet batch 8x8 x 3 variants", flush=True)
    L = 20.0
    batch = ShellBatch(m=8, n_variants=3, L=L, options=sso.Options(rtol=1e-12, max_it=50000))
    net = DesignMLP().to("cuda")
    loss = batch.loss(net)
    loss.backward()
    grads = [p.grad.detach().cpu().numpy().copy() for p in net.parameters()]
    params = [p.detach().cpu().numpy().copy() for p in net.parameters()]
    rhos = [r.cpu().numpy() for r in batch.rho]
    base = batch.base
    ref = _oracle_loss(params, base, rhos, L)
    assert loss.item() == pytest.approx(ref, rel=1e-10)
    gmax = max(np.abs(g).max() for g in grads)
    # every weight: the oracle adjoint chained through the network
    for g, r in zip(grads, _oracle_adjoint_grads(DesignMLP(), base, rhos, L)):
        assert np.abs(g - r).max() <= 1e-8 * gmax
    # 20 sampled weights, central differences of the oracle.  (a) The prescribed step
    # h = 1e-6: rounding in the oracle's FP64 K, amplified by the conditioning of the
    # rho^3-scaled shells, perturbs each loss value by ~1e-12 relative (measured: quotients at
    # h = 1e-6 scatter by up to 1.4, i.e. 2.8e-5 relative, around the converged values of (b)),
    # so 2e-12 |L| / h is added to the bound.  (b) Richardson extrapolation of the quotients at
    # h = 2.5e-4 and 1.25e-4 (truncation O(h^4), rounding ~1e-8 relative) at the plain bound.
    rng = np.random.default_rng(0)

    def quotient(k, idx, step):
        vals = []
        for sgn in (1.0, -1.0):
            pp = [q.copy() for q in params]
            pp[k][idx] += sgn * step
            vals.append(_oracle_loss(pp, base, rhos, L))
        return (vals[0] - vals[1]) / (2 * step)

    for _ in range(20):
        k = int(rng.integers(len(params)))
        idx = tuple(int(rng.integers(s)) for s in params[k].shape)
        g = grads[k][idx]
        h = 1e-6
        fd = quotient(k, idx, h)
        assert abs(g - fd) <= 1e-5 * max(abs(fd), 1e-3 * gmax) + 2e-12 * abs(ref) / h, \
            (k, idx, g, fd)
        f1, f2 = quotient(k, idx, 2.5e-4), quotient(k, idx, 1.25e-4)
        rich = f2 + (f2 - f1) / 3
        assert abs(g - rich) <= 1e-5 * max(abs(rich), 1e-3 * gmax), (k, idx, g, rich)
    batch.close()


def test_displacement_backward_matches_oracle_adjoint():
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.autograd import displacement
    print("[gpu] displacement backward", flush=True)
    mesh = meshgen.shell(6, L=6.0, seed=8)
    w = np.random.default_rng(1).normal(size=(mesh.n_nodes, 6))
    ref = oracle.analyze(mesh, "linear", a=w.ravel(), pat=assembly.pattern(mesh))
    with sso.Problem(mesh, sso.Options(rtol=1e-10, max_it=50000)) as p:
        xyz = torch.tensor(mesh.xyz, device="cuda", requires_grad=True)
        t = torch.tensor(mesh.quad_prop[:, 0], device="cuda", requires_grad=True)
        s = torch.ones(mesh.n_quads, dtype=torch.float64, device="cuda", requires_grad=True)
        u = displacement(p, xyz, t, s)
        (u * torch.tensor(w, device="cuda")).sum().backward()
    scale = np.abs(ref["grad_xyz"]).max()
    assert np.abs(xyz.grad.cpu().numpy() - ref["grad_xyz"]).max() <= 1e-8 * scale
    assert np.abs(t.grad.cpu().numpy() - ref["grad_t"]).max() <= \
        1e-8 * np.abs(ref["grad_t"]).max()
    assert np.abs(s.grad.cpu().numpy() - ref["grad_scale"]).max() <= \
        1e-8 * np.abs(ref["grad_scale"]).max()


def test_batched_network_batch_matches_one_by_one():
    """The variants' solves advancing together in multi-problem launches give the loss and the
    network gradient of the one-by-one form (same recurrences: each solve is bitwise the same;
    only the order in which the per-variant gradients are summed differs)."""
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.shellnet import DesignMLP, ShellBatch
    print("[gpu] shellnet batched vs one by one", flush=True)
    out = []
    for batched in (False, True):
        b = ShellBatch(m=8, n_variants=4, L=20.0,
                       options=sso.Options(rtol=1e-10, solver=sso.SOLVER_STANDARD),
                       batched=batched)
        net = DesignMLP().to("cuda")
        loss = b.loss(net)
        loss.backward()
        out.append((loss.item(), [p.grad.detach().cpu().numpy().copy()
                                  for p in net.parameters()]))
        b.close()
    (l0, g0), (l1, g1) = out
    assert l1 == pytest.approx(l0, rel=1e-14)
    for a, c in zip(g0, g1):
        np.testing.assert_allclose(c, a, rtol=1e-12, atol=1e-12 * np.abs(a).max())


def test_nonlinear_displacement_objective_through_autograd():
    """A nonlinear objective of u written in torch (a p-norm of the vertical displacement, a
    smooth stand-in for the displacement penalty among the paper's objectives): the gradient
    through Displacement's backward (the USER adjoint with dg/du from torch) against the oracle
    adjoint with the same dg/du, and against the oracle's central differences of g."""
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.autograd import displacement
    from oracle import sensitivity
    print("[gpu] p-norm displacement objective", flush=True)
    mesh = meshgen.shell(6, L=6.0, seed=11)
    pexp = 4.0

    def g_of(u):
        return float(np.sum(np.abs(u.reshape(-1, 6)[:, 2]) ** pexp) ** (1.0 / pexp))

    fw = sensitivity.forward(mesh)
    uz = fw["u"].reshape(-1, 6)[:, 2]
    norm = np.sum(np.abs(uz) ** pexp) ** (1.0 / pexp)
    dg = np.zeros((mesh.n_nodes, 6))
    dg[:, 2] = np.sign(uz) * np.abs(uz) ** (pexp - 1) * norm ** (1 - pexp)
    ref = oracle.analyze(mesh, "user", dg_du=dg.ravel())
    with sso.Problem(mesh, sso.Options(rtol=1e-10, max_it=50000)) as p:
        xyz = torch.tensor(mesh.xyz, device="cuda", requires_grad=True)
        t = torch.tensor(mesh.quad_prop[:, 0], device="cuda", requires_grad=True)
        u = displacement(p, xyz, t)
        g = (u[:, 2].abs() ** pexp).sum() ** (1.0 / pexp)
        g.backward()
    assert g.item() == pytest.approx(g_of(fw["u"]), rel=1e-9)
    gx, gt = xyz.grad.cpu().numpy(), t.grad.cpu().numpy()
    assert np.abs(gx - ref["grad_xyz"]).max() <= 1e-8 * np.abs(ref["grad_xyz"]).max()
    assert np.abs(gt - ref["grad_t"]).max() <= 1e-8 * np.abs(ref["grad_t"]).max()
    rng = np.random.default_rng(3)
    h = 1e-6
    gmax = np.abs(gx).max()
    for _ in range(6):
        i, c = int(rng.integers(mesh.n_nodes)), int(rng.integers(3))
        vals = []
        for sgn in (1.0, -1.0):
            m = mesh.copy()
            m.xyz = mesh.xyz.copy()
            m.xyz[i, c] += sgn * h
            vals.append(g_of(sensitivity.forward(m)["u"]))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(gx[i, c] - fd) <= 1e-5 * max(abs(fd), 1e-3 * gmax), (i, c, gx[i, c], fd)


def test_network_batch_at_configured_size_vs_oracle_adjoint():
    """The configured plan, 80 x 80 quads (39,366 DOF per variant), variants 0 and 1 in
    multi-problem launches: the loss and every network weight's gradient against the oracle's
    adjoint of the same design (tests/golden/make_shellnet80.py) chained through the same MLP
    with torch's CPU autograd, at 1e-8 of the largest weight gradient."""
    import os
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.shellnet import DesignMLP, ShellBatch, geometry
    print("[gpu] shellnet batch 80x80 x 2 variants vs oracle adjoint", flush=True)
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "shellnet80_oracle.npz"))
    L = 20.0
    # rtol 1e-9: the rho^3 contrast puts the smallest true residual an FP64 u of these systems
    # reaches near 1.4e-10 (measured with the compensated residual)
    batch = ShellBatch(m=80, n_variants=2, L=L, options=sso.Options(rtol=1e-9, max_it=400000),
                       batched=True)
    try:
        net = DesignMLP().to("cuda")
        for p, k in zip(net.parameters(), ("W1", "b1", "W2", "b2")):
            assert np.array_equal(p.detach().cpu().numpy(), ref[k]), k   # the same network
        loss = batch.loss(net)
        loss.backward()
        grads = [p.grad.detach().cpu().numpy().copy() for p in net.parameters()]
        statuses = [p.last_status for p in batch.problems]
        resid = [p.last_stats["rel_residual"] for p in batch.problems]
        base = batch.base
    finally:
        batch.close()
    print(f"  statuses {statuses}, residuals {resid}")
    assert statuses == [0, 0] and max(resid) <= 1e-9
    c_ref = np.mean([float(ref[f"c_{v}"]) for v in (0, 1)])
    assert loss.item() == pytest.approx(c_ref, rel=1e-9)
    gx = np.mean([ref[f"grad_xyz_{v}"] for v in (0, 1)], axis=0)
    gt = np.mean([ref[f"grad_t_{v}"] for v in (0, 1)], axis=0)
    net_cpu = DesignMLP()
    xyz, t = geometry(net_cpu, torch.tensor(base.xyz[:, :2]), L,
                      torch.tensor(base.quad_nodes.astype(np.int64)))
    ((xyz * torch.tensor(gx)).sum() + (t * torch.tensor(gt)).sum()).backward()
    gmax = max(np.abs(g).max() for g in grads)
    for g, p in zip(grads, net_cpu.parameters()):
        err = np.abs(g - p.grad.numpy()).max() / gmax
        print(f"  weight block {tuple(g.shape)}: max error {err:.2e} of the largest gradient")
        assert err <= 1e-8


def test_two_forwards_on_one_problem_then_one_backward():
    """Two compliance evaluations of different designs on one problem, summed, then one
    backward: each node differentiates its own design (the later forward changed K and u in
    between), so the gradients equal those of two separate problems."""
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.autograd import compliance
    print("[gpu] two forwards, one backward", flush=True)
    mesh = meshgen.shell(8, L=8.0, seed=31)
    x0 = torch.tensor(mesh.xyz, device="cuda")
    t0 = torch.tensor(mesh.quad_prop[:, 0], device="cuda")
    designs = [(x0, t0), (x0 + torch.tensor([0.0, 0.0, 0.3], dtype=torch.float64,
                                            device="cuda") * x0[:, :1] / 8.0, 1.3 * t0)]
    opts = sso.Options(rtol=1e-11, solver=sso.SOLVER_STANDARD)

    def leaves():
        return [(x.clone().requires_grad_(True), t.clone().requires_grad_(True))
                for x, t in designs]

    shared = leaves()
    with sso.Problem(mesh, opts) as p:
        (compliance(p, *shared[0]) + compliance(p, *shared[1])).backward()
    apart = leaves()
    for (x, t) in apart:
        with sso.Problem(mesh, opts) as q:
            compliance(q, x, t).backward()
    for (xs, ts), (xa, ta) in zip(shared, apart):
        assert torch.equal(xs.grad, xa.grad) and torch.equal(ts.grad, ta.grad)
    assert not torch.equal(shared[0][0].grad, shared[1][0].grad)
