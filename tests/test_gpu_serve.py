"""Continuous batching: requests of mixed sizes admitted by slots and device-memory budget run
concurrently on separate streams; every result equals the same request solved alone."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _requests(n, seed=0, rate=2000.0):
    from paper_2407_20026_amd.serve import Request, poisson_arrivals
    rng = np.random.default_rng(seed)
    t = poisson_arrivals(n, rate, seed)
    out = []
    for i in range(n):
        if i % 2 == 0:
            mesh = meshgen.gridshell(int(rng.integers(8, 15)), seed=int(rng.integers(1 << 30)))
        else:
            mesh = meshgen.shell(int(rng.integers(10, 17)), seed=int(rng.integers(1 << 30)))
        out.append(Request(i, mesh, float(t[i])))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_results_in_the_mix_equal_results_alone(precision):
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.serve import Server, run_one
    print(f"[gpu] serve mix precision={precision}", flush=True)
    opts = sso.Options(precision=precision, rtol=1e-10)
    reqs = _requests(12, seed=precision)
    stats = Server(slots=4, options=opts).run(reqs)
    assert stats.n == len(reqs)
    assert stats.peak_inflight >= 2          # work did overlap
    for r, req in zip(stats.results, reqs):
        alone = run_one(req, opts)
        assert r.g == pytest.approx(alone.g, rel=1e-12)
        np.testing.assert_allclose(r.grad_xyz, alone.grad_xyz, rtol=0,
                                   atol=1e-12 * np.abs(alone.grad_xyz).max())
        # deterministic kernels and identical launch shapes: bitwise equal by design
        assert r.g == alone.g and np.array_equal(r.grad_xyz, alone.grad_xyz)
    print(f"  solves/s={stats.solves_per_s:.1f} p50={stats.p50_ms:.2f} ms "
          f"p99={stats.p99_ms:.2f} ms peak in flight={stats.peak_inflight}")


@pytest.mark.parametrize("solver", ["standard", "fused"])
def test_batched_loop_results_equal_results_alone(solver):
    """Multi-problem launches: each request keeps its own workgroup decomposition, so its
    arithmetic, and its result, is bitwise that of the request solved alone with the same
    recurrences."""
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.serve import BatchedServer, run_one
    print(f"[gpu] batched serve mix {solver}", flush=True)
    code = {"standard": sso.SOLVER_STANDARD, "fused": sso.SOLVER_FUSED}[solver]
    opts = sso.Options(rtol=1e-10, solver=code)
    reqs = _requests(16, seed=7, rate=5000.0)
    stats = BatchedServer(slots=8, options=opts, chunk=16).run(reqs)
    assert stats.n == len(reqs)
    assert stats.peak_inflight >= 4
    for r, req in zip(stats.results, reqs):
        alone = run_one(req, opts)
        assert r.g == alone.g
        assert np.array_equal(r.grad_xyz, alone.grad_xyz)
    print(f"  solves/s={stats.solves_per_s:.1f} p50={stats.p50_ms:.2f} ms "
          f"p99={stats.p99_ms:.2f} ms peak in flight={stats.peak_inflight}")


def test_batched_auto_matches_single_auto_within_tolerance():
    """Under SSO_SOLVER_AUTO a request in the mix runs the standard recurrences and alone the
    single-reduction ones (below 20,000 nodes): equal within the solve tolerance."""
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.serve import BatchedServer, run_one
    print("[gpu] batched serve auto", flush=True)
    opts = sso.Options(rtol=1e-10)
    reqs = _requests(8, seed=9, rate=5000.0)
    stats = BatchedServer(slots=8, options=opts, chunk=16).run(reqs)
    for r, req in zip(stats.results, reqs):
        alone = run_one(req, opts)
        assert r.g == pytest.approx(alone.g, rel=1e-9)
        np.testing.assert_allclose(r.grad_xyz, alone.grad_xyz, rtol=0,
                                   atol=1e-7 * np.abs(alone.grad_xyz).max())


def test_memory_budget_limits_admission():
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.serve import Server, footprint_bytes
    print("[gpu] serve budget", flush=True)
    reqs = _requests(8, seed=5, rate=1e6)
    big = max(footprint_bytes(r.mesh) for r in reqs)
    budget = int(2.2 * big)
    stats = Server(slots=6, hbm_budget=budget, options=sso.Options(rtol=1e-8)).run(reqs)
    assert stats.n == 8
    assert stats.peak_bytes <= budget
    assert stats.peak_inflight <= 6


def test_batch_mixing_both_recurrences_matches_solves_alone():
    """One multi-problem launcher with problems on the standard and on the single-reduction
    recurrences: each result is bitwise the same as its own sso_solve; a problem listed twice
    is rejected."""
    import paper_2407_20026_amd as sso
    print("[gpu] batch with both recurrences", flush=True)
    meshes = [meshgen.gridshell(9, seed=11), meshgen.shell(10, seed=12),
              meshgen.shell(12, seed=13), meshgen.gridshell(12, seed=14)]
    solvers = [sso.SOLVER_STANDARD, sso.SOLVER_FUSED, sso.SOLVER_STANDARD, sso.SOLVER_FUSED]
    stream = torch.cuda.Stream()
    batch = sso.Batch(stream)
    probs = [sso.Problem(m, sso.Options(rtol=1e-10, solver=k), stream=stream)
             for m, k in zip(meshes, solvers)]
    try:
        for p in probs:
            p.solve_begin()
        with pytest.raises(sso.SSOError):
            batch.iterate([probs[0], probs[0]], 1)
        done = [False] * len(probs)
        for _ in range(10000):
            done = batch.iterate(probs, 16)
            if all(done):
                break
        assert all(done)
        got = []
        for p in probs:
            u, st = p.solve_end()
            got.append((u.cpu().numpy(), st["solver"]))
    finally:
        for p in probs:
            p.close()
        batch.close()
    for m, k, (u, used) in zip(meshes, solvers, got):
        assert used == k
        with sso.Problem(m, sso.Options(rtol=1e-10, solver=k)) as q:
            ua, _ = q.solve()
        assert np.array_equal(u, ua.cpu().numpy())


@pytest.mark.parametrize("solver", ["standard", "fused"])
def test_batched_mixed_precision_matches_solves_alone(solver):
    """Mixed precision in multi-problem launches (FP32 inner iterations, FP64 refinement between
    them): every request bitwise equal to the same request solved alone with sso_solve and the
    same recurrences."""
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.serve import BatchedServer, run_one
    print(f"[gpu] batched serve mixed precision {solver}", flush=True)
    code = {"standard": sso.SOLVER_STANDARD, "fused": sso.SOLVER_FUSED}[solver]
    opts = sso.Options(precision=sso.PREC_MIXED, rtol=1e-8, solver=code)
    reqs = _requests(12, seed=21, rate=5000.0)
    stats = BatchedServer(slots=6, options=opts, chunk=16).run(reqs)
    assert stats.n == len(reqs)
    assert stats.peak_inflight >= 3
    for r, req in zip(stats.results, reqs):
        alone = run_one(req, opts)
        assert r.g == alone.g
        assert np.array_equal(r.grad_xyz, alone.grad_xyz)


def test_batch_with_prescribed_displacements_matches_solves_alone():
    """Problems with nonzero prescribed support displacements iterating in one multi-problem
    launcher (both recurrences): each u is bitwise its own sso_solve's, with u = b exactly on
    the constrained DOFs."""
    import paper_2407_20026_amd as sso
    print("[gpu] batch with prescribed displacements", flush=True)
    rng = np.random.default_rng(23)
    meshes = [meshgen.shell(10, seed=31), meshgen.gridshell(10, seed=32)]
    meshes = [m.copy(u_prescribed=1e-3 * rng.standard_normal((m.n_nodes, 6))) for m in meshes]
    solvers = [sso.SOLVER_FUSED, sso.SOLVER_STANDARD]
    stream = torch.cuda.Stream()
    batch = sso.Batch(stream)
    probs = [sso.Problem(m, sso.Options(rtol=1e-10, solver=k), stream=stream)
             for m, k in zip(meshes, solvers)]
    try:
        for p in probs:
            p.solve_begin()
        done = [False] * len(probs)
        for _ in range(10000):
            done = batch.iterate(probs, 16)
            if all(done):
                break
        assert all(done)
        got = [p.solve_end()[0].cpu().numpy() for p in probs]
    finally:
        for p in probs:
            p.close()
        batch.close()
    for m, k, u in zip(meshes, solvers, got):
        fixed = m.fixed.reshape(-1) != 0
        np.testing.assert_array_equal(u.reshape(-1)[fixed], m.u_prescribed.reshape(-1)[fixed])
        with sso.Problem(m, sso.Options(rtol=1e-10, solver=k)) as q:
            ua, _ = q.solve()
        assert np.array_equal(u, ua.cpu().numpy())
