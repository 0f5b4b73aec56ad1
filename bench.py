"""Benchmark: forward + adjoint structural analyses per second on one MI355X.

One step = one forward analysis (element stiffness, loads, assembly, masking, block-Jacobi, PCG
to 1e-8 relative residual) + the objective + its adjoint gradient with respect to every nodal
coordinate, every shell thickness and every stiffness scale, for the 60 x 60 continuous shell
(22,326 DOF, compliance; the adjoint of compliance is lambda = u, no second solve).  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

The dominant kernel of the PCG -- k_cg1_iter1, one whole single-reduction iteration (the
default up to 20,000 nodes), or k_spmv_dir, the direction + SpMV kernel of the standard
recurrences -- is timed live
with HIP events on the problem's stream for every n-th launch; its roofline uses the algorithmic
bytes of one launch.  The CPU baseline
is the FP64 oracle timed on the host on one forward + adjoint of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import meshgen  # noqa: E402

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and WRITE_SIZE counters
# (KiB per dispatch, mean over working launches) scaled by what they read for a plain 256 MiB
# copy (FETCH x 2.000, WRITE x 1.000).  Valid only for the kernel code they were taken on: an
# entry is removed when that kernel changes.
MEASURED_TRAFFIC = {
    ("shell60", "fp64", "k_cg1_iter1"): (6570.6 * 2.000 + 954.4 * 1.000) * 1024,
    ("shell300", "fp64", "k_spmv_dir"): (131735.3 * 2.000 + 8554.7 * 1.000) * 1024,
}
METRIC = "forward+adjoint solves/s & DOF/s at 1e-8 residual; p50/p99 latency, mixed sizes"

WORKLOADS = {
    "shell60": ("60x60 continuous shell, 22,326 DOF, FP64, compliance, seed 1", meshgen.shell_60),
    "grid11": ("11x11 grid-shell, 726 DOF, FP64, compliance, seed 0", meshgen.grid_shell_11),
    "shell300": ("300x300 continuous shell, 543,606 DOF, FP64, compliance, seed 2",
                 meshgen.shell_300),
}


# the workload's generator at another seed (for the batched measurement)
SEEDED = {
    "shell60": lambda seed: meshgen.shell(60, seed=seed),
    "grid11": lambda seed: meshgen.gridshell(11, seed=seed),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="shell60", choices=list(WORKLOADS))
    ap.add_argument("--objective", default="compliance",
                    choices=["compliance", "strain_energy", "linear"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--inner-max-it", type=int, default=0,
                    help="mixed precision: iteration cap of each FP32 inner solve (0 = none)")
    ap.add_argument("--refine-steps", type=int, default=20,
                    help="mixed precision: outer (FP64 flexible CG) step limit")
    ap.add_argument("--solver", default="auto", choices=["auto", "standard", "fused"])
    ap.add_argument("--profile-every", type=int, default=64,
                    help="time every n-th iteration kernel with HIP events "
                         "(16: ~5 %% overhead, 64: ~1.5 %%, 0: off)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the mixed-size served stream (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--batch", type=int, default=16,
                    help="also time this many problems of the workload (seeds 1..n) advancing "
                         "together in multi-problem launches (0: skip)")
    ap.add_argument("--general-steps", type=int, default=5,
                    help="also time this many steps with a linear objective (second PCG "
                         "for the adjoint; 0: skip)")
    ap.add_argument("--shellnet", type=int, default=0,
                    help="also time one loss + backward of the network-driven batch of this "
                         "many 80 x 80 shells (0: skip)")
    ap.add_argument("--arch", default="2,6,10,20,30,80",
                    help="elements per span of the arch-bridge rows to time ('' = none)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="before the workload, copy a float64 tensor of this many MiB 3 times "
                         "(a plain copy kernel of known size for scaling HBM counters)")
    return ap.parse_args()


def _oracle_rate(mesh, objective, budget_s, threads):
    import numpy as np
    import oracle
    from threadpoolctl import threadpool_limits
    a = None
    if objective == "linear":
        a = np.zeros(mesh.n_dof)
        a[6 * (mesh.n_nodes // 2) + 2] = 1.0
    n, t0 = 0, time.perf_counter()
    with threadpool_limits(limits=threads):
        while True:
            oracle.analyze(mesh, objective, a=a)
            n += 1
            log(f"cpu baseline ({threads} BLAS threads): oracle analysis {n} done")
            el = time.perf_counter() - t0
            if el >= budget_s or el * (n + 1) / n > 1.5 * budget_s:
                break
    return n, el


def cpu_baseline(mesh, objective, budget_s):
    """The oracle as it stands, one forward + adjoint at a time, for about budget_s seconds with
    one BLAS thread (the reported value), then for about budget_s / 2 seconds with every host
    core given to BLAS (the banded Cholesky is the threaded part), and one SciPy sparse direct
    solve of the same system (SuperLU) for context."""
    import numpy as np
    import scipy.sparse.linalg as sla
    from oracle import assembly, solve
    n, el = _oracle_rate(mesh, objective, budget_s, 1)
    rate = n / el
    # the host cores this process may use (the thread limit of the environment when it sets one)
    all_cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or os.cpu_count() or 1
    n2, el2 = _oracle_rate(mesh, objective, budget_s / 2, all_cores)
    K = assembly.assemble(mesh)
    f = assembly.load_vector(mesh)
    F = solve.free_dofs(mesh)
    Kff = K.tocsc()[F][:, F]
    t0 = time.perf_counter()
    sla.spsolve(Kff, np.asarray(f)[F])
    t_sp = time.perf_counter() - t0
    log(f"cpu baseline: SciPy spsolve {t_sp:.2f} s")
    return {"value": rate, "unit": "solves/s", "dof_per_s": rate * mesh.n_dof, "cores": 1,
            "kind": "oracle",
            "sample": f"{n} forward+adjoint analyses (pattern, assembly, banded Cholesky, "
                      f"complex-step adjoint) of the benchmark workload in {el:.1f} s, "
                      f"BLAS threads 1, host cpus {all_cores}",
            "all_cores": {"value": n2 / el2, "unit": "solves/s", "cores": all_cores,
                          "sample": f"{n2} analyses in {el2:.1f} s"},
            "scipy_spsolve_s": t_sp}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def serve_bench(n, slots, precision, solver, inner_max_it=0, refine_steps=20):
    """Mixed-size served stream: grid-shells (n x n nodes, n ~ U{8..60}) and shells (m x m quads,
    m ~ U{10..120}) with per-request seeds, rtol 1e-8 on the FP64 true residual, all requests in
    flight iterating in shared multi-problem launches; FP64 or mixed precision (FP32 inner
    iterations).  A closed-loop pass measures the capacity; the timed pass uses Poisson arrivals
    at 0.8 x capacity."""
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.serve import BatchedServer, Request, poisson_arrivals
    meshes = [meshgen.served_request(i) for i in range(n)]
    # multi-problem launches take the standard recurrences under AUTO; mixed precision may cap
    # each FP32 inner solve
    opts = sso.Options(rtol=1e-8, precision=sso.PREC_MIXED if precision == "mixed" else
                       sso.PREC_FP64,
                       solver=solver if precision == "fp64" else sso.SOLVER_AUTO,
                       inner_max_it=inner_max_it if precision == "mixed" else 0,
                       refine_steps=refine_steps)
    srv = BatchedServer(slots=slots, options=opts)
    n_cl = min(n, 64)
    cl = srv.run([Request(i, meshes[i], 0.0) for i in range(n_cl)])
    log(f"serving {precision} closed loop: {cl.solves_per_s:.1f} solves/s")
    lam = 0.8 * cl.solves_per_s
    t = poisson_arrivals(n, lam, seed=3)
    st = srv.run([Request(i, meshes[i], float(t[i])) for i in range(n)])
    log(f"serving {precision} Poisson stream: {st.solves_per_s:.1f} solves/s "
        f"p99 {st.p99_ms:.1f} ms")
    return {"requests": st.n, "slots": slots, "precision": precision, "rtol": 1e-8,
            "closed_loop_solves_per_s": cl.solves_per_s, "arrival_rate_per_s": lam,
            "solves_per_s": st.solves_per_s, "dof_per_s": st.dof_per_s,
            "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_queue_ms": st.mean_queue_ms,
            "peak_inflight": st.peak_inflight,
            "not_converged": st.not_converged + cl.not_converged,
            "max_rel_residual": max(st.max_rel_residual, cl.max_rel_residual),
            "mean_dof": float(np.mean([m.n_dof for m in meshes])),
            "closed_loop_phase_s": {k: round(v, 4) for k, v in cl.host_s.items()},
            "phase_s": {k: round(v, 4) for k, v in st.host_s.items()}}


def batch_bench(gen_seed, n_problems, rtol, objective, solver):
    """n problems of the workload with seeds 1..n, all iterating together in multi-problem
    launches (one launch per kernel for all of them), forward + adjoint each."""
    import torch
    import paper_2407_20026_amd as sso
    meshes = [gen_seed(k + 1) for k in range(n_problems)]
    stream = torch.cuda.Stream()
    batch = sso.Batch(stream)
    probs = [sso.Problem(m, sso.Options(rtol=rtol, max_it=400000, solver=solver), stream=stream)
             for m in meshes]

    def one_pass():
        for p in probs:
            p.solve_begin()
        done = [False] * len(probs)
        while not all(done):
            done = batch.iterate(probs, 32)
        for p in probs:
            p.solve_end()
            p.objective(objective)
            p.adjoint(objective)

    try:
        one_pass()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one_pass()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        for p in probs:
            p.close()
        batch.close()
    log(f"batched: {n_problems} problems in {1000 * el:.1f} ms")
    return {"problems": n_problems, "solves_per_s": n_problems / el,
            "dof_per_s": sum(m.n_dof for m in meshes) / el, "wall_ms": 1000 * el,
            "note": "same generator, seeds 1..n; all problems in flight together"}


def general_objective_bench(mesh, opts, steps):
    """The same workload with a linear objective g = u_z at the centre node: its adjoint is a
    second PCG solve (K lambda = a), unlike compliance where lambda = u."""
    import torch
    import paper_2407_20026_amd as sso
    a = torch.zeros(mesh.n_dof, dtype=torch.float64, device="cuda")
    a[6 * (mesh.n_nodes // 2) + 2] = 1.0
    adj = []
    with sso.Problem(mesh, opts) as prob:
        def step():
            prob.solve(check=False)
            if prob.last_status not in (sso.SSO_OK, sso.SSO_ENOTCONV):
                raise sso.SSOError(prob.last_status, "sso_solve")
            prob.objective("linear", a)
            adj.append(prob.adjoint("linear", dg_du=a)["stats"]["iters"])
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    log(f"general objective: {1000 * el / steps:.2f} ms/step")
    return {"objective": "linear (u_z at the centre node)", "solves_per_s": steps / el,
            "ms_per_step": 1000 * el / steps, "adjoint_pcg_iters": int(np.median(adj))}


# FEA time of the paper's performance table (seconds, best column: SciPy sparse with GPU
# assembly, A100 + Xeon 6342) for the 100-span arch bridge, by DOF; context only.
PAPER_ARCH_FEA_S = {1206: 0.006, 3606: 0.006, 6006: 0.007, 12006: 0.038, 18006: 0.044,
                    48006: 0.072}


def arch_bench(rows, reps=3):
    """The paper's performance-study structure (100 parabolic arch spans, beam elements only):
    FEA (elements, assembly, block-Jacobi PCG to 1e-8) and sensitivity (FEA + adjoint of the
    strain energy) wall time per row, beside the paper's best FEA time for the same DOF."""
    import torch
    import meshgen
    import paper_2407_20026_amd as sso
    out = []
    for n_el in rows:
        mesh = meshgen.arch_bridge(n_el)
        with sso.Problem(mesh, sso.Options(rtol=1e-8, max_it=400000)) as prob:
            def fea():
                _, st = prob.solve(check=False)
                if prob.last_status not in (sso.SSO_OK, sso.SSO_ENOTCONV):
                    raise sso.SSOError(prob.last_status, "sso_solve")
                return st

            def sens():
                st = fea()
                prob.adjoint("strain_energy")
                return st
            st = sens()
            times = {}
            for name, fn in (("fea", fea), ("sensitivity", sens)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    fn()
                torch.cuda.synchronize()
                times[name] = (time.perf_counter() - t0) / reps
        out.append({"elements_per_span": n_el, "dof": mesh.n_dof, "pcg_iters": st["iters"],
                    "rel_residual": st["rel_residual"], "fea_ms": 1000 * times["fea"],
                    "sensitivity_ms": 1000 * times["sensitivity"],
                    "paper_best_fea_s": PAPER_ARCH_FEA_S.get(mesh.n_dof)})
        log(f"arch {n_el} elements/span ({mesh.n_dof} DOF): {st['iters']} iterations, "
            f"FEA {1000 * times['fea']:.2f} ms, sensitivity {1000 * times['sensitivity']:.2f} ms")
    return out


def shellnet_bench(n_variants, solver, m=80):
    """The network-driven batch: n_variants shells on an m x m plan, heights and thickness from
    the MLP, element stiffness scaled by rho^3; one loss (mean compliance) + backward into the
    network weights, the variants' PCG iterations advancing together in multi-problem launches.
    Timed: the second of two passes."""
    import torch
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.shellnet import DesignMLP, ShellBatch
    t0 = time.perf_counter()
    b = ShellBatch(m=m, n_variants=n_variants, options=sso.Options(rtol=1e-8, solver=solver),
                   batched=True)
    log(f"shellnet: {n_variants} problems created in {time.perf_counter() - t0:.1f} s")
    net = DesignMLP().to("cuda")
    try:
        times = []
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            net.zero_grad()
            loss = b.loss(net)
            loss.backward()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            log(f"shellnet: loss + backward {times[-1]:.2f} s")
        iters = [p.last_stats["iters"] for p in b.problems]
        rres = [p.last_stats["rel_residual"] for p in b.problems]
        not_conv = sum(1 for p in b.problems if p.last_status != 0)
        n_dof = b.problems[0].n_dof
    finally:
        b.close()
    return {"variants": n_variants, "mesh": f"{m}x{m} quads", "n_dof_per_variant": n_dof,
            "loss_and_backward_s": times[-1], "solves_per_s": n_variants / times[-1],
            "dof_per_s": n_variants * n_dof / times[-1], "loss": float(loss.item()),
            "pcg_iters_median": int(np.median(iters)), "pcg_iters_max": int(max(iters)),
            "not_converged": not_conv, "max_rel_residual": float(max(rres))}


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 x {mib} MiB")


def measured_copy_bandwidth(mib=1024, reps=10):
    """HBM bandwidth a plain device copy reaches on this GPU (bytes read + written per second,
    GB/s), the measured ceiling beside the datasheet peak."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    log(f"measured copy bandwidth: {gbs:.0f} GB/s")
    return gbs


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent problems shard whole across GPUs; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2407_20026_amd as sso

    desc, gen = WORKLOADS[args.workload]
    mesh = gen()
    torch.cuda.set_device(0)
    if args.copy_mib > 0:
        copy_calibration(args.copy_mib)
    a = None
    if args.objective == "linear":
        a = torch.zeros(mesh.n_dof, dtype=torch.float64, device="cuda")
        a[6 * (mesh.n_nodes // 2) + 2] = 1.0
    prec = sso.PREC_MIXED if args.precision == "mixed" else sso.PREC_FP64
    solver = {"auto": sso.SOLVER_AUTO, "standard": sso.SOLVER_STANDARD,
              "fused": sso.SOLVER_FUSED}[args.solver]
    opts = sso.Options(precision=prec, rtol=args.rtol, max_it=400000,
                       profile_every=args.profile_every, solver=solver,
                       refine_steps=args.refine_steps, inner_max_it=args.inner_max_it)
    prob = sso.Problem(mesh, opts)
    u_out = torch.empty((mesh.n_nodes, 6), dtype=torch.float64, device="cuda")

    spmv_us, spmv_n, iters, resid, adj_iters, outer = [], [], [], [], [], []
    last_g = []

    statuses = []

    def step():
        _, st = prob.solve(u_out, check=False)
        if prob.last_status not in (sso.SSO_OK, sso.SSO_ENOTCONV):
            raise sso.SSOError(prob.last_status, "sso_solve")
        statuses.append(prob.last_status)
        prob.objective(args.objective, a) if args.objective == "linear" else \
            prob.objective(args.objective)
        g = prob.adjoint(args.objective, dg_du=a)
        last_g[:] = [g]
        iters.append(st["iters"])
        outer.append(st["refine_steps"])
        resid.append(st["rel_residual"])
        adj_iters.append(g["stats"]["iters"])
        if st["spmv_samples"]:
            spmv_us.append(st["spmv_us"] * st["spmv_samples"])
            spmv_n.append(st["spmv_samples"])
        return st

    log(f"{desc}: problem created")
    for _ in range(args.warmup):
        step()
    log("warmup done")
    spmv_us.clear(); spmv_n.clear(); iters.clear(); resid.clear(); adj_iters.clear()
    statuses.clear()
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        st = step()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log(f"timed {args.steps} steps: {1000 * el / args.steps:.2f} ms/step")
    vs_fp64 = None
    if args.precision == "mixed":
        # the error of u and of the gradients against the FP64 path, same mesh and rtol
        u_mx, g_mx = u_out.clone(), last_g[0]
        with sso.Problem(mesh, sso.Options(rtol=args.rtol, max_it=400000,
                                           solver=solver)) as ref:
            u_ref, _ = ref.solve(check=False)
            g_ref = ref.adjoint(args.objective, dg_du=a)

        def rel_inf(x, y):
            return float((x - y).abs().max() / y.abs().max())
        vs_fp64 = {"u_rel_2norm": float((u_mx - u_ref).norm() / u_ref.norm()),
                   "dg_dxyz_rel_inf": rel_inf(g_mx["dg_dxyz"], g_ref["dg_dxyz"]),
                   "dg_dt_rel_inf": rel_inf(g_mx["dg_dt"], g_ref["dg_dt"])
                   if g_ref["dg_dt"] is not None and g_ref["dg_dt"].numel() else None}
        log(f"mixed vs FP64: {vs_fp64}")
    ms = 1000.0 * el / args.steps
    rate = args.steps / el
    spmv_bytes = st["spmv_bytes"]
    spmv_avg_us = sum(spmv_us) / max(1, sum(spmv_n))
    achieved = spmv_bytes / (spmv_avg_us * 1e-6) / 1e9 if spmv_avg_us > 0 else 0.0
    kernel = "k_cg1_iter1" if st["solver"] == sso.SOLVER_FUSED else "k_spmv_dir"
    solver_name = "fused single-reduction" if st["solver"] == sso.SOLVER_FUSED else "standard"

    out = {
        "metric": METRIC,
        "value": rate,
        "unit": "solves/s",
        "dof_per_s": rate * mesh.n_dof,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "p50_ms": 1000.0 * float(np.percentile(lat, 50)),
        "p99_ms": 1000.0 * float(np.percentile(lat, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 inner / f64 flexible CG",
        "data": "synthetic (seeded generator)",
        "config": {"workload": desc, "n_dof": mesh.n_dof, "objective": args.objective,
                   "rtol": args.rtol, "precision": args.precision, "pcg": solver_name,
                   **({"inner_max_it": args.inner_max_it, "outer_steps": int(np.median(outer)),
                       "vs_fp64": vs_fp64} if args.precision == "mixed" else {}),
                   "pcg_iters": int(np.median(iters)),
                   "adjoint_pcg_iters": int(np.median(adj_iters)),
                   "rel_residual": float(np.max(resid)), "n_blocks": prob.n_blocks,
                   "status": "converged" if all(v == sso.SSO_OK for v in statuses) else
                   "stopped above rtol (FP64 residual floor)"},
        "roofline": {"bound": "hbm", "kernel": kernel, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": MEASURED_TRAFFIC.get((args.workload, args.precision, kernel)),
                     "bytes_per_launch": spmv_bytes,
                     "avg_launch_us": spmv_avg_us, "samples": int(sum(spmv_n))},
    }
    prob.close()
    copy_gbs = measured_copy_bandwidth()
    out["roofline"]["measured_copy_gbs"] = copy_gbs
    out["roofline"]["frac_of_measured"] = achieved / copy_gbs
    if args.objective != "linear" and args.general_steps > 0:
        out["general_objective"] = general_objective_bench(mesh, opts, args.general_steps)
    if args.batch > 0 and args.workload in SEEDED and args.objective != "linear":
        out["batched"] = batch_bench(SEEDED[args.workload], args.batch, args.rtol,
                                     args.objective, solver)
    if args.shellnet > 0:
        out["shellnet"] = shellnet_bench(args.shellnet, solver)
    if args.serve_requests > 0:
        out["serving"] = {prec: serve_bench(args.serve_requests, args.serve_slots, prec, solver,
                                            args.inner_max_it, args.refine_steps)
                          for prec in ("fp64", "mixed")}
    if args.arch:
        out["arch_replay"] = arch_bench([int(v) for v in args.arch.split(",")])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh, args.objective, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
