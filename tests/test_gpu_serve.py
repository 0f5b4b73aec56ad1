"""Continuous batching: requests of mixed sizes admitted by slots and device-memory budget run
concurrently on separate streams; every result equals the same request solved alone, and a
sample of the served stream, its largest sizes included, matches the oracle."""
import os

import numpy as np
import pytest

import meshgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "served_sample_oracle.npz")

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
        assert r.status == sso.SSO_OK and r.rel_residual <= opts.rtol
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
        assert r.status == sso.SSO_OK and r.rel_residual <= opts.rtol
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


def test_batch_reading_the_upper_triangle_matches_full_products_alone():
    """Three 120 x 120 shells (37.5 MB of K each) and a 100 x 100 one (26.1 MB) iterate in one
    multi-problem launch, whose K (138.6 MB together) is past the 128 MiB at which the products
    read only K's upper triangle; alone, each reads all of K.  Only the problems still running
    are launched, and any three of them hold less than 128 MiB, so once the first converges
    (the smaller shell, hundreds of iterations earlier) the launches read all of K again: the
    others change product form mid-solve.  K is assembled bitwise symmetric and both forms sum
    the same values in the same order, so each u is bitwise its solve alone."""
    import paper_2407_20026_amd as sso
    print("[gpu] batch of upper-triangle products against full products alone", flush=True)
    meshes = [meshgen.shell(120, seed=s) for s in (41, 42, 43)] + [meshgen.shell(100, seed=44)]
    opts = sso.Options(rtol=1e-8, solver=sso.SOLVER_STANDARD)
    stream = torch.cuda.Stream()
    batch = sso.Batch(stream)
    probs = [sso.Problem(m, opts, stream=stream) for m in meshes]
    try:
        for p in probs:
            p.solve_begin()
        running, sizes = list(probs), []
        for _ in range(1000):
            sizes.append(len(running))
            flags = batch.iterate(running, 16)
            running = [p for p, f in zip(running, flags) if not f]
            if not running:
                break
        assert not running
        assert sizes[0] == 4 and min(sizes) < 4   # both product forms ran
        got = [p.solve_end()[0].cpu().numpy() for p in probs]
    finally:
        for p in probs:
            p.close()
        batch.close()
    for m, u in zip(meshes, got):
        with sso.Problem(m, opts) as q:
            ua, st = q.solve()
        assert st["sym_products"] == 0   # alone: 37.5 MB of K, the full product
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
        assert r.status == sso.SSO_OK and r.rel_residual <= opts.rtol
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


@pytest.fixture(scope="module")
def served_sample():
    """Requests 0, 1, 2, 3, 4, 6, 10, 11 and 51 of the served stream (shells 55, 54, 25, 16 and
    120 -- the stream's largest -- and grid-shells 26, 41, 13 and 60, the largest) and the
    oracle's c and gradients of each (tests/golden/make_served_sample.py)."""
    from paper_2407_20026_amd import Options, PREC_FP64, PREC_MIXED
    from paper_2407_20026_amd.serve import BatchedServer, Request
    ref = np.load(GOLDEN)
    rids = [int(i) for i in ref["rids"]]
    reqs = [Request(i, meshgen.served_request(i), 0.002 * k) for k, i in enumerate(rids)]
    for q in reqs:
        assert q.mesh.name == str(ref[f"name_{q.rid}"])
    out = {}
    for name, prec in (("fp64", PREC_FP64), ("mixed", PREC_MIXED)):
        print(f"[gpu] served sample vs oracle: {name}, {len(reqs)} requests", flush=True)
        opts = Options(precision=prec, rtol=1e-10, max_it=400000)
        out[name] = BatchedServer(slots=16, options=opts, chunk=32).run(reqs)
    return ref, reqs, out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_served_results_match_the_oracle(served_sample, precision):
    """Each served result (in the mix, multi-problem launches, rtol 1e-10) against the oracle:
    c within 1e-10 relative, every entry of dc/dxyz and dc/dt within 1e-8 of the largest."""
    ref, reqs, out = served_sample
    stats = out[precision]
    assert stats.n == len(reqs)
    assert stats.peak_inflight >= 4
    for r in stats.results:
        assert r.status == 0 and r.rel_residual <= 1e-10, (r.rid, r.status, r.rel_residual)
        g_ref = float(ref[f"g_{r.rid}"])
        gx_ref, gt_ref = ref[f"grad_xyz_{r.rid}"], ref[f"grad_t_{r.rid}"]
        eg = abs(r.g - g_ref) / abs(g_ref)
        ex = np.abs(r.grad_xyz - gx_ref).max() / np.abs(gx_ref).max()
        et = (np.abs(r.grad_t - gt_ref).max() / np.abs(gt_ref).max()
              if gt_ref.size else 0.0)
        print(f"  {precision} request {r.rid} ({str(ref[f'name_{r.rid}'])}, {r.n_dof} DOF): "
              f"c {eg:.2e}, dc/dxyz {ex:.2e}, dc/dt {et:.2e}, residual {r.rel_residual:.2e}")
        assert eg <= 1e-10 and ex <= 1e-8 and et <= 1e-8, r.rid


def test_mixed_served_results_report_their_error_against_fp64(served_sample):
    """The served mixed-precision form reports, per result, its error against the FP64 path
    (the same requests served in FP64); here every one is within the parity bars."""
    from paper_2407_20026_amd.serve import errors_against
    _, reqs, out = served_sample
    errs = errors_against(out["mixed"].results, out["fp64"].results)
    assert [e["rid"] for e in errs] == sorted(q.rid for q in reqs)
    for e in errs:
        assert e["g_rel"] <= 1e-10 and e["dg_dxyz_rel_inf"] <= 1e-8
        assert e.get("dg_dt_rel_inf", 0.0) <= 1e-8
    print("  mixed vs FP64: max g", max(e["g_rel"] for e in errs), "max dc/dxyz",
          max(e["dg_dxyz_rel_inf"] for e in errs))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_footprint_bounds_what_the_library_allocates(precision):
    """Admission's footprint estimate against the library's own count of the device memory a
    problem holds after its forward and adjoint (sso_problem_bytes): an upper bound, and not a
    gross one, on a sample of the stream's sizes (both element kinds, smallest to largest)."""
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.serve import footprint_bytes
    print(f"[gpu] footprint vs allocation, {precision}", flush=True)
    mixed = precision == "mixed"
    opts = sso.Options(rtol=1e-8, precision=sso.PREC_MIXED if mixed else sso.PREC_FP64)
    for i in (0, 1, 3, 4, 6, 10, 11, 51):
        mesh = meshgen.served_request(i)
        with sso.Problem(mesh, opts) as p:
            p.solve(check=False)
            p.adjoint("compliance")
            held = p.device_bytes()
        est = footprint_bytes(mesh, mixed)
        print(f"  {mesh.name}: held {held / 2**20:.2f} MiB, estimate {est / 2**20:.2f} MiB")
        assert 0 < held <= est <= 1.6 * held + (2 << 20), mesh.name


def test_problems_sharing_a_pattern_match_problems_with_their_own():
    """sso_problem_create_like: a problem of the same topology shares the first one's pattern and
    gives bitwise the same results as one created on its own, whichever of the two is destroyed
    first; a different connectivity or size is rejected."""
    import paper_2407_20026_amd as sso
    print("[gpu] shared patterns", flush=True)
    a_mesh, b_mesh = meshgen.shell(14, seed=41), meshgen.shell(14, seed=42)
    opts = sso.Options(rtol=1e-10)
    with sso.Problem(b_mesh, opts) as own:
        u_own, _ = own.solve()
        g_own = own.adjoint("compliance")["dg_dxyz"].cpu()
        u_own = u_own.cpu()
    first = sso.Problem(a_mesh, opts)
    second = sso.Problem(b_mesh, opts, like=first)
    first.close()                       # the pattern outlives the problem that built it
    u, _ = second.solve()
    g = second.adjoint("compliance")["dg_dxyz"].cpu()
    assert torch.equal(u.cpu(), u_own) and torch.equal(g, g_own)
    third = sso.Problem(a_mesh, opts, like=second)
    second.close()
    third.solve()
    third.close()
    other = meshgen.shell(14, seed=43)
    other.quad_nodes = other.quad_nodes[:, [1, 2, 3, 0]].copy()   # same counts, other connectivity
    with sso.Problem(a_mesh, opts) as base:
        with pytest.raises(sso.SSOError) as e:
            sso.Problem(other, opts, like=base)
        assert e.value.status == sso.SSO_EINVAL
        with pytest.raises(sso.SSOError):
            sso.Problem(meshgen.shell(13, seed=44), opts, like=base)


def test_batched_server_with_shared_patterns_matches_solves_alone():
    """The batched loop shares patterns between requests of one topology in flight: each result
    is still bitwise that of the request solved alone with the same recurrences."""
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.serve import BatchedServer, Request, run_one
    print("[gpu] batched serve with shared patterns", flush=True)
    opts = sso.Options(rtol=1e-10, solver=sso.SOLVER_STANDARD)
    reqs = [Request(i, meshgen.shell(12, seed=60 + i) if i % 2 else meshgen.gridshell(10, seed=i),
                    0.0) for i in range(10)]
    stats = BatchedServer(slots=10, options=opts, chunk=16).run(reqs)
    for r, req in zip(stats.results, reqs):
        alone = run_one(req, opts)
        assert r.g == alone.g and np.array_equal(r.grad_xyz, alone.grad_xyz)


def test_asynchronous_launch_protocol():
    """sso_batch_launch / sso_batch_wait: the wait must name the launched list, one launch is
    pending at a time, a pending problem may not move streams or end, and a launch + wait gives
    bitwise what sso_batch_iterate gives."""
    import paper_2407_20026_amd as sso
    print("[gpu] batch launch/wait protocol", flush=True)
    meshes = [meshgen.shell(10, seed=71), meshgen.gridshell(9, seed=72)]
    stream = torch.cuda.Stream()
    other = torch.cuda.Stream()
    opts = sso.Options(rtol=1e-10, solver=sso.SOLVER_STANDARD)
    outs = []
    for mode in ("iterate", "launch"):
        batch = sso.Batch(stream)
        probs = [sso.Problem(m, opts, stream=stream) for m in meshes]
        try:
            for p in probs:
                p.solve_begin()
            done = [False] * len(probs)
            while not all(done):
                if mode == "iterate":
                    done = batch.iterate(probs, 8)
                    continue
                batch.launch(probs, 8)
                with pytest.raises(sso.SSOError):
                    batch.launch(probs, 8)                 # one pending launch at a time
                with pytest.raises(sso.SSOError):
                    batch.wait(probs[::-1])                # not the launched list
                with pytest.raises(sso.SSOError):
                    probs[0].set_stream(other)             # pending: may not move
                with pytest.raises(sso.SSOError):
                    probs[0].solve_end()                   # pending: may not end
                done = batch.wait(probs)
            outs.append([p.solve_end()[0].cpu() for p in probs])
        finally:
            for p in probs:
                p.close()
            batch.close()
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_overlapped_and_plain_loops_give_the_same_results():
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.serve import BatchedServer
    print("[gpu] overlapped vs plain batched loop", flush=True)
    reqs = _requests(12, seed=8, rate=5000.0)
    opts = sso.Options(rtol=1e-10, solver=sso.SOLVER_STANDARD)
    a = BatchedServer(slots=6, options=opts, chunk=16, overlap=True).run(reqs)
    b = BatchedServer(slots=6, options=opts, chunk=16, overlap=False).run(reqs)
    for ra, rb in zip(a.results, b.results):
        assert ra.rid == rb.rid and ra.g == rb.g and np.array_equal(ra.grad_xyz, rb.grad_xyz)


def test_one_workgroup_problems_in_a_batch_match_solves_alone():
    """The one-workgroup solver (SSO_SOLVER_WG) in multi-problem launches beside standard
    problems: its kernel resumes from the state record at every launch (8 x 16 iterations
    here), against one launch for the whole solve alone; u, the iteration count and the
    gradient must be bitwise the same."""
    import paper_2407_20026_amd as sso
    print("[gpu] one-workgroup problems in a batch", flush=True)
    meshes = [meshgen.gridshell(8, seed=81), meshgen.shell(10, seed=82),
              meshgen.gridshell(13, seed=83), meshgen.shell(14, seed=84)]
    kinds = [sso.SOLVER_WG, sso.SOLVER_WG, sso.SOLVER_STANDARD, sso.SOLVER_WG]
    alone = []
    for m, k in zip(meshes, kinds):
        with sso.Problem(m, sso.Options(rtol=1e-10, solver=k)) as p:
            u, st = p.solve()
            g = p.adjoint("compliance")
            assert st["solver"] == k
            alone.append((u.cpu(), st["iters"], g["dg_dxyz"].cpu()))
    stream = torch.cuda.Stream()
    batch = sso.Batch(stream)
    probs = [sso.Problem(m, sso.Options(rtol=1e-10, solver=k), stream=stream)
             for m, k in zip(meshes, kinds)]
    try:
        for p in probs:
            p.solve_begin()
        done = [False] * len(probs)
        launches = 0
        while not all(done):
            done = batch.iterate(probs, 8)
            launches += 1
        assert launches > 2
        for p, (u0, it0, g0) in zip(probs, alone):
            u, st = p.solve_end()
            g = p.adjoint("compliance")
            assert st["iters"] == it0
            assert torch.equal(u.cpu(), u0)
            assert torch.equal(g["dg_dxyz"].cpu(), g0)
    finally:
        for p in probs:
            p.close()
        batch.close()


def test_one_workgroup_solver_rejects_mixed_precision():
    import paper_2407_20026_amd as sso
    with pytest.raises(sso.SSOError):
        sso.Problem(meshgen.gridshell(6), sso.Options(solver=sso.SOLVER_WG,
                                                      precision=sso.PREC_MIXED))


def _timed_batch(sso, meshes, opts, stream, every, span, chunk=8):
    batch = sso.Batch(stream)
    probs = [sso.Problem(m, opts, stream=stream) for m in meshes]
    try:
        if every:
            batch.profile(every, span)
        for p in probs:
            p.solve_begin()
        calls = 0
        done = [False] * len(probs)
        while not all(done):
            done = batch.iterate(probs, chunk)
            calls += 1
        timing = batch.timing()
        us = [p.solve_end()[0].cpu() for p in probs]
        per_it = [(36 * 8 + 4) * p.n_blocks + 4 * (p.n_nodes + 1) + 4 * 8 * 6 * p.n_nodes +
                  (4 + 3.5 + 3) * 8 * 6 * p.n_nodes for p in probs]
    finally:
        for p in probs:
            p.close()
        batch.close()
    return timing, calls, us, per_it


def test_batch_timing_samples_count_the_iterations_they_time():
    """sso_batch_profile / sso_batch_timing.  Each problem alone with whole chunks timed gives
    its batch iteration count as bytes / (bytes per iteration, all of K); three together with
    the first 4 of every 8 iterations timed then give 4 timed iterations per launch and, per
    problem, min(4, iterations left) of each chunk's iterations in the bytes; results are bitwise
    those of an unsampled batch."""
    import paper_2407_20026_amd as sso
    print("[gpu] batch timing samples", flush=True)
    meshes = [meshgen.shell(12, seed=91), meshgen.gridshell(10, seed=92),
              meshgen.shell(16, seed=93)]
    opts = sso.Options(rtol=1e-10, solver=sso.SOLVER_STANDARD)
    stream = torch.cuda.Stream()
    counts = []
    for m in meshes:
        t, calls, _, (per_it,) = _timed_batch(sso, [m], opts, stream, 1, 8)
        n = t["bytes"] / per_it
        assert n == round(n) and 8 * (calls - 1) <= n <= 8 * calls
        assert t["iters"] == 8 * calls
        counts.append(int(round(n)))
    t0, _, u0, _ = _timed_batch(sso, meshes, opts, stream, 0, 0)
    assert t0 == {"us": 0.0, "iters": 0, "bytes": 0.0, "bytes_read": 0.0}
    t1, calls, u1, per_it = _timed_batch(sso, meshes, opts, stream, 1, 4)
    assert t1["iters"] == 4 * calls and t1["us"] > 0
    want = sum(w * sum(min(4, max(0, n - 8 * c)) for c in range(calls))
               for n, w in zip(counts, per_it))
    assert t1["bytes"] == pytest.approx(want, rel=1e-12)
    assert t1["bytes_read"] == pytest.approx(want, rel=1e-12)   # small K: all of it read
    for a, b in zip(u0, u1):
        assert torch.equal(a, b)
    batch = sso.Batch(stream)
    try:
        with pytest.raises(sso.SSOError):
            batch.profile(1, 0)
    finally:
        batch.close()
