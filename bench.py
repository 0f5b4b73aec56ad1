"""Benchmark: forward + adjoint structural analyses per second on one MI355X.

Headline (the default): the mixed-size served stream.  2,000 forward + adjoint requests, each a
grid-shell (n x n nodes, n ~ U{8..60}) or a quad shell (m x m elements, m ~ U{10..120}) with its
own seed (``meshgen.served_request``), compliance, rtol 1e-8, served by continuous batching
(``serve.BatchedServer``: admission by slots and device-memory footprint, all requests in flight
iterating in shared multi-problem launches).  A "step" is one request.  The headline runs in
mixed precision (FP32 inner PCG solves inside an FP64 flexible CG) with plain FP64 beside it:

* value (solves/s) and DOF/s: all requests queued at once (closed loop), wall time of the whole
  stream -- the throughput the server sustains on this mix of sizes;
* p50/p99 latency (arrival to result): the same 2,000 requests arriving as a Poisson process at
  0.8 times the smaller of the two precisions' closed-loop capacities;
* per request, the error of the mixed result against the FP64 result (g, dg/dxyz, dg/dt).

Inputs are resident in HBM before each request's timed work starts: a request's mesh is uploaded
when it is admitted, which is part of serving it.

Legs: the 300 x 300 shell (543,606 DOF) at rtol 1e-10 in FP64 and mixed precision, whose PCG
iteration (k_spmv_dir_single + k_update_single, timed live with HIP events on the problem's stream) gives the
roofline; the 60 x 60 shell; a linear objective (second PCG for the adjoint); the network batch
(256 variants of the 80 x 80 shell through the MLP); the paper's arch-bridge rows; the measured
HBM and FP64 ceilings; the oracle timed on the host on a sample of the stream's requests.
Prints one JSON line.
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

# HBM bytes per PCG iteration, from rocprofv3 FETCH_SIZE and WRITE_SIZE counters (KiB per
# dispatch, mean over working launches, summed over the iteration's kernels) scaled by what they
# read for a plain copy of known size (FETCH x 2.000, WRITE x 1.000).  Valid only for the kernel
# code they were taken on: an entry is removed when one of its kernels changes.
MEASURED_TRAFFIC = {
    ("shell60", "fp64", "k_cg1_iter1"): (6340.9 * 2.000 + 939.9 * 1.000) * 1024,
    ("shell300", "fp64", "k_spmv_dir_single<sym> + k_update_single"):
        (83791.4 * 2.000 + 8692.7 * 1.000 + 17524.3 * 2.000 + 12775.4 * 1.000) * 1024,
    ("shell500", "fp64", "k_spmv_dir_single<sym> + k_update_single"):
        (243043.5 * 2.000 + 25219.8 * 1.000 + 45718.6 * 2.000 + 35349.3 * 1.000) * 1024,
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
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps: requests of the stream (default 2000), or solves of a "
                         "single-problem workload (default 20)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 32 requests of other seeds, or 3 solves)")
    ap.add_argument("--workload", default="stream", choices=["stream", *WORKLOADS])
    ap.add_argument("--objective", default="compliance",
                    choices=["compliance", "strain_energy", "linear"])
    ap.add_argument("--rtol", type=float, default=None,
                    help="relative residual target (default 1e-8; 1e-10 for shell300)")
    ap.add_argument("--precision", default=None, choices=["auto", "fp64", "mixed"],
                    help="headline precision (default: auto for the stream -- FP32 inner "
                         "solves where the problem's K outgrows the caches -- fp64 otherwise)")
    ap.add_argument("--inner-max-it", type=int, default=0,
                    help="mixed precision: iteration cap of each FP32 inner solve (0 = none)")
    ap.add_argument("--refine-steps", type=int, default=20,
                    help="mixed precision: outer (FP64 flexible CG) step limit")
    ap.add_argument("--solver", default="auto", choices=["auto", "standard", "fused"])
    ap.add_argument("--stream-beside", default="fp64,mixed",
                    help="stream: precisions timed beside the headline (comma-separated; '' = "
                         "the headline alone, and no error-against-FP64 summary)")
    ap.add_argument("--no-poisson", action="store_true",
                    help="stream: closed loop only (p50/p99 then from the closed loop, all "
                         "requests arriving at once; for profiling one pass)")
    ap.add_argument("--slots", type=int, default=32, help="stream: requests in flight at most")
    ap.add_argument("--chunk", type=int, default=32,
                    help="stream: iterations per multi-problem launch sequence between polls")
    ap.add_argument("--profile-every", type=int, default=64,
                    help="time every n-th PCG iteration with HIP events "
                         "(16: ~5 %% overhead, 64: ~1.5 %%, 0: off)")
    ap.add_argument("--legs", default="large,large500,shell60,general,network,arch,ceilings",
                    help="comma-separated extra measurements ('' = none): large (300x300 shell, "
                         "FP64 + mixed, rtol 1e-10, the roofline), large500 (the 500x500 "
                         "shell's iteration, out of the Infinity Cache), shell60, general (linear "
                         "objective), batch (16 60x60 shells in one launch), network (the MLP "
                         "batch), arch (the paper's arch-bridge rows), ceilings")
    ap.add_argument("--network-variants", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--arch", default="2,6,10,20,30,80",
                    help="elements per span of the arch-bridge rows to time")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="before the workload, copy a float64 buffer of this many MiB 3 times "
                         "with the library's copy kernel (a known size for scaling HBM counters)")
    args = ap.parse_args()
    stream = args.workload == "stream"
    if args.steps is None:
        args.steps = 2000 if stream else 20
    if args.warmup is None:
        args.warmup = 32 if stream else 3
    if args.precision is None:
        args.precision = "auto" if stream else "fp64"
    if args.rtol is None:
        args.rtol = 1e-10 if args.workload == "shell300" else 1e-8
    return args


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---- CPU baseline: the oracle on the host ---------------------------------------------------

def _threads(n):
    from threadpoolctl import threadpool_limits
    return threadpool_limits(limits=n)


def _oracle_analyses(meshes, objective, budget_s, threads):
    """Forward + adjoint analyses of meshes[0], meshes[1], ... by the oracle until about
    budget_s seconds have passed (at least one); returns (count, DOF, seconds)."""
    import oracle
    n, dof, t0 = 0, 0, time.perf_counter()
    with _threads(threads):
        for mesh in meshes:
            a = None
            if objective == "linear":
                a = np.zeros(mesh.n_dof)
                a[6 * (mesh.n_nodes // 2) + 2] = 1.0
            oracle.analyze(mesh, objective, a=a)
            n += 1
            dof += mesh.n_dof
            el = time.perf_counter() - t0
            log(f"cpu baseline ({threads} BLAS threads): {n} analyses, {el:.1f} s")
            if el >= budget_s or el * (n + 1) / n > 1.5 * budget_s:
                break
    return n, dof, time.perf_counter() - t0


def cpu_baseline(meshes, objective, budget_s, what):
    """The oracle as it stands on a bounded sample: forward + adjoint analyses of `meshes` in
    order for about budget_s seconds with one BLAS thread (the reported value), then about
    budget_s / 2 seconds with every host core given to BLAS (the banded Cholesky is the threaded
    part)."""
    all_cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or os.cpu_count() or 1
    n, dof, el = _oracle_analyses(meshes, objective, budget_s, 1)
    n2, dof2, el2 = _oracle_analyses(meshes, objective, budget_s / 2, all_cores)
    return {"value": n / el, "unit": "solves/s", "dof_per_s": dof / el, "cores": 1,
            "kind": "oracle",
            "sample": f"the first {n} {what} ({dof} DOF in all), one forward + adjoint "
                      f"analysis each (pattern, assembly, banded Cholesky with long-double "
                      f"refinement, complex-step adjoint) in {el:.1f} s, 1 BLAS thread; host "
                      f"cpus {all_cores}",
            "all_cores": {"value": n2 / el2, "unit": "solves/s", "dof_per_s": dof2 / el2,
                          "cores": all_cores, "sample": f"{n2} analyses in {el2:.1f} s"}}


# ---- the served stream ----------------------------------------------------------------------

PRECISIONS = {"auto": "PREC_AUTO", "fp64": "PREC_FP64", "mixed": "PREC_MIXED"}


def _stream_options(sso, precision, rtol, args):
    return sso.Options(rtol=rtol, max_it=400000, precision=getattr(sso, PRECISIONS[precision]),
                       inner_max_it=args.inner_max_it if precision == "mixed" else 0,
                       refine_steps=args.refine_steps)


def _size_buckets(results, meshes):
    """p50/p99 latency per DOF quartile of the stream (Poisson pass)."""
    dof = np.array([meshes[r.rid].n_dof for r in results])
    lat = np.array([r.latency for r in results]) * 1000.0
    edges = np.percentile(dof, [0, 25, 50, 75, 100])
    out = []
    for k in range(4):
        sel = (dof >= edges[k]) & ((dof <= edges[k + 1]) if k == 3 else (dof < edges[k + 1]))
        if np.any(sel):
            out.append({"dof_range": [int(edges[k]), int(edges[k + 1])], "n": int(sel.sum()),
                        "p50_ms": float(np.percentile(lat[sel], 50)),
                        "p99_ms": float(np.percentile(lat[sel], 99))})
    return out


def _error_summary(errs):
    def one(key):
        v = np.array([e.get(key, 0.0) for e in errs])
        return {"max": float(v.max()), "p99": float(np.percentile(v, 99)),
                "p50": float(np.percentile(v, 50))}
    return {"requests": len(errs), "g_rel": one("g_rel"),
            "dg_dxyz_rel_inf": one("dg_dxyz_rel_inf"), "dg_dt_rel_inf": one("dg_dt_rel_inf")}


def stream_headline(args):
    """The served stream in the headline precision (the AUTO policy by default) and plain FP64:
    closed-loop capacity, then Poisson arrivals at 0.8 of the smaller capacity; FP32 inner
    solves forced on every request (mixed precision regardless of size) in a closed loop
    beside them."""
    import paper_2407_20026_amd as sso
    from paper_2407_20026_amd.serve import (BatchedServer, Request, errors_against,
                                            poisson_arrivals)
    n = args.steps
    meshes = [meshgen.served_request(i) for i in range(n)]
    warm = [meshgen.served_request(i, base_seed=2 * 10**6) for i in range(args.warmup)]
    log(f"stream: {n} requests, {sum(m.n_dof for m in meshes)} DOF in all")
    head = args.precision
    beside = [p for p in args.stream_beside.split(",") if p]
    order = [head] + [p for p in ("fp64", "mixed") if p != head and p in beside]
    closed, poisson, servers = {}, {}, {}
    for prec in order:
        # the first 8 iterations of every 4th chunk of FP64 standard problems timed with HIP
        # events (the dominant kernel pair of the stream, live; the same kernels)
        srv = BatchedServer(slots=args.slots, options=_stream_options(sso, prec, args.rtol, args),
                            chunk=args.chunk, profile_every=4, profile_span=8)
        servers[prec] = srv
        if warm:
            srv.run([Request(i, m, 0.0) for i, m in enumerate(warm)])
        torch.cuda.synchronize()
        st = srv.run([Request(i, m, 0.0) for i, m in enumerate(meshes)])
        closed[prec] = st
        log(f"stream {prec} closed loop: {st.solves_per_s:.1f} solves/s, "
            f"{st.dof_per_s / 1e6:.2f} M DOF/s, {st.wall_s:.1f} s")
    timed = [p for p in (head, "fp64") if p in closed][:2]
    lam = 0.8 * min(closed[p].solves_per_s for p in timed)
    if args.no_poisson:
        timed = []
    t_arr = poisson_arrivals(n, lam, seed=3)
    for prec in timed:
        st = servers[prec].run([Request(i, m, float(t_arr[i])) for i, m in enumerate(meshes)])
        poisson[prec] = st
        log(f"stream {prec} Poisson at {lam:.1f}/s: {st.solves_per_s:.1f} solves/s, "
            f"p50 {st.p50_ms:.1f} ms, p99 {st.p99_ms:.1f} ms")

    def leg(prec):
        c = closed[prec]
        out = {"closed_loop": {"solves_per_s": c.solves_per_s, "dof_per_s": c.dof_per_s,
                               "wall_s": c.wall_s, "peak_inflight": c.peak_inflight,
                               "iteration_gbs": c.iteration_bytes_per_s / 1e9,
                               "phase_s": {k: round(v, 3) for k, v in c.host_s.items()}},
               "not_converged": c.not_converged, "max_rel_residual": c.max_rel_residual,
               "iters_median": int(np.median([r.iters for r in c.results])),
               "mixed_requests": int(sum(1 for r in c.results if r.outer_steps > 0))}
        if c.iteration_timing and c.iteration_timing["iters"] > 0:
            out["closed_loop"]["iteration_timing"] = c.iteration_timing
        if prec in poisson:
            q = poisson[prec]
            out["poisson"] = {"arrival_rate_per_s": lam, "solves_per_s": q.solves_per_s,
                              "dof_per_s": q.dof_per_s, "p50_ms": q.p50_ms, "p99_ms": q.p99_ms,
                              "mean_queue_ms": q.mean_queue_ms,
                              "peak_inflight": q.peak_inflight,
                              "by_size": _size_buckets(q.results, meshes)}
            out["not_converged"] += q.not_converged
            out["max_rel_residual"] = max(out["max_rel_residual"], q.max_rel_residual)
        return out

    c = closed[head]
    q = poisson.get(head, c)
    nc = sum(leg(p)["not_converged"] for p in order)
    out = {
        "value": c.solves_per_s,
        "dof_per_s": c.dof_per_s,
        "ms_per_step": 1000.0 * c.wall_s / n,
        "p50_ms": q.p50_ms,
        "p99_ms": q.p99_ms,
        "dtype": {"auto": "f64, f32 inner PCG above the size crossover", "fp64": "f64",
                  "mixed": "f32 inner PCG / f64 flexible CG"}[head],
        "config": {
            "workload": (f"served stream: {n} forward+adjoint requests (grid-shells n~U{{8..60}}, "
                         f"shells m~U{{10..120}}, per-request seeds 10^6+i), compliance, "
                         f"rtol {args.rtol:g}, precision {head}; value = closed-loop solves/s, "
                         + ("p50/p99 of the closed loop (all requests at t = 0)"
                            if args.no_poisson else
                            f"p50/p99 from arrival under Poisson arrivals at {lam:.1f}/s")),
            "requests": n, "mean_dof": float(np.mean([m.n_dof for m in meshes])),
            "slots": args.slots, "chunk": args.chunk, "rtol": args.rtol, "precision": head,
            "arrival_rate_per_s": lam,
            "status": "converged" if nc == 0 else f"{nc} requests stopped above rtol",
        },
        "stream": {p: leg(p) for p in order},
        "errors_vs_fp64": {p: _error_summary(errors_against(closed[p].results,
                                                            closed["fp64"].results))
                           for p in order if p != "fp64" and "fp64" in closed},
        "_timing": c.iteration_timing,
    }
    return out, meshes


# ---- one problem, repeated ------------------------------------------------------------------

def problem_run(mesh, opts, steps, warmup, objective="compliance", with_grad=True):
    """Forward + objective + adjoint of one problem, `steps` times after `warmup`; returns the
    timings, PCG statistics, live iteration timing and the last u and gradients."""
    import paper_2407_20026_amd as sso
    a = None
    if objective == "linear":
        a = torch.zeros(mesh.n_dof, dtype=torch.float64, device="cuda")
        a[6 * (mesh.n_nodes // 2) + 2] = 1.0
    rec = dict(it_us=[], it_n=[], iters=[], resid=[], adj=[], outer=[], status=[], lat=[])
    with sso.Problem(mesh, opts) as prob:
        u_out = torch.empty((mesh.n_nodes, 6), dtype=torch.float64, device="cuda")
        last = {}

        def step(keep):
            _, st = prob.solve(u_out, check=False)
            if prob.last_status not in (sso.SSO_OK, sso.SSO_ENOTCONV):
                raise sso.SSOError(prob.last_status, "sso_solve")
            prob.objective(objective, a)
            g = prob.adjoint(objective, dg_du=a) if with_grad else None
            if keep:
                rec["iters"].append(st["iters"])
                rec["outer"].append(st["refine_steps"])
                rec["resid"].append(st["rel_residual"])
                rec["status"].append(prob.last_status)
                rec["adj"].append(g["stats"]["iters"] if g else 0)
                if st["spmv_samples"]:
                    rec["it_us"].append(st["spmv_us"] * st["spmv_samples"])
                    rec["it_n"].append(st["spmv_samples"])
            last.update(st=st, g=g)

        for _ in range(warmup):
            step(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            step(True)
            rec["lat"].append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        n_blocks = prob.n_blocks
        u = u_out.clone()
    st = last["st"]
    it_us = sum(rec["it_us"]) / max(1, sum(rec["it_n"]))
    return {"wall_s": el, "steps": steps, "solves_per_s": steps / el,
            "dof_per_s": steps * mesh.n_dof / el, "ms_per_step": 1000.0 * el / steps,
            "p50_ms": 1000.0 * float(np.percentile(rec["lat"], 50)),
            "p99_ms": 1000.0 * float(np.percentile(rec["lat"], 99)),
            "pcg_iters": int(np.median(rec["iters"])),
            "adjoint_pcg_iters": int(np.median(rec["adj"])),
            "outer_steps": int(np.median(rec["outer"])),
            "rel_residual": float(np.max(rec["resid"])),
            "status": "converged" if all(v == sso.SSO_OK for v in rec["status"]) else
                      "stopped above rtol",
            "solver": "fused single-reduction" if st["solver"] == sso.SOLVER_FUSED else
                      "standard",
            "n_blocks": n_blocks, "n_nodes": mesh.n_nodes,
            "iteration": {"kernels": "k_cg1_iter1" if st["solver"] == sso.SOLVER_FUSED else
                          "k_spmv_dir_single<sym> + k_update_single" if st["sym_products"] else
                          "k_spmv_dir_single + k_update_single", "bytes": st["spmv_bytes"],
                          "avg_us": it_us, "samples": int(sum(rec["it_n"]))},
            "_u": u, "_g": last["g"]}


def algorithmic_iteration_bytes(n_nodes, n_blocks, precision, symmetric=False):
    """Algorithmic HBM bytes of one standard PCG iteration by the scope table's accounting:
    the BSR values, block columns and row pointers once; twelve vector passes (p read and Ap
    written by the product; x, r, p, Ap read and x, r, z written by the update; z and p read
    and p written for the direction); the 6 x 6 block-Jacobi inverse of every node (36 values).
    The library moves fewer than that (the direction is formed inside the product, the inverse
    is stored packed, 21 values), so this is an upper bound of what the kernels need.
    symmetric: what a product that reads only K's upper triangle must fetch (the diagonal blocks
    and half the others, with an 8-byte (column, value slot) pair per block in place of the
    4-byte column): the bytes-read figure reported beside the scope table's one."""
    v = 4.0 if precision == "mixed" else 8.0
    n_dof = 6.0 * n_nodes
    if symmetric:
        k_bytes = 36.0 * v * 0.5 * (n_blocks + n_nodes) + 8.0 * n_blocks
    else:
        k_bytes = (36.0 * v + 4.0) * n_blocks
    return k_bytes + 4.0 * (n_nodes + 1) + 12.0 * v * n_dof + 36.0 * v * n_nodes


def roofline_of(run, workload, precision, ceilings=None):
    it = run["iteration"]
    sym_read = None
    if it["kernels"].startswith("k_spmv_dir"):
        # the unit of work is one PCG iteration on this K, counted by the scope table (all of K
        # read); the upper-triangle product fetches less, which is reported beside it
        if "<sym>" in it["kernels"]:
            sym_read = algorithmic_iteration_bytes(run["n_nodes"], run["n_blocks"], precision,
                                                   symmetric=True)
        it = dict(it, library_bytes=it["bytes"],
                  bytes=algorithmic_iteration_bytes(run["n_nodes"], run["n_blocks"], precision))
    achieved = it["bytes"] / (it["avg_us"] * 1e-6) / 1e9 if it["avg_us"] > 0 else 0.0
    out = {"bound": "hbm", "kernel": it["kernels"], "workload": workload,
           "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS,
           "traffic": MEASURED_TRAFFIC.get((workload, precision, it["kernels"])),
           "bytes_per_launch": it["bytes"], "avg_launch_us": it["avg_us"],
           "samples": it["samples"]}
    if "library_bytes" in it:
        out["library_bytes_per_launch"] = it["library_bytes"]
    if sym_read is not None and it["avg_us"] > 0:
        out["bytes_read_per_launch"] = sym_read
        out["frac_on_bytes_read"] = sym_read / (it["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
    if ceilings:
        out["measured_read_gbs"] = ceilings["read_gbs"]
        out["measured_copy_gbs"] = ceilings["copy_gbs"]
        out["frac_of_measured_read"] = achieved / ceilings["read_gbs"]
    return out


def stream_roofline(timing, ceilings=None):
    """Roofline of the served stream's dominant kernels, the multi-problem FP64 standard pair
    (product kernel + k_update over every problem in flight), from the closed loop's HIP-event
    samples: algorithmic bytes of the problem-iterations inside the timed spans (all of K
    counted, as for the single-problem roofline) over the spans' event time."""
    if not timing or timing["iters"] <= 0 or timing["us"] <= 0:
        return None
    us = timing["us"] / timing["iters"]
    achieved = timing["bytes"] / (timing["us"] * 1e-6) / 1e9
    out = {"bound": "hbm", "kernel": "k_spmv_dir_sym / k_spmv_dir + k_update (multi-problem)",
           "workload": "served stream, closed loop", "achieved": achieved,
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "traffic": None, "bytes_per_launch": timing["bytes"] / timing["iters"],
           "avg_launch_us": us, "samples": timing["iters"],
           "bytes_read_per_launch": timing["bytes_read"] / timing["iters"],
           "frac_on_bytes_read": timing["bytes_read"] / (timing["us"] * 1e-6) / 1e9 / HBM_PEAK_GBS}
    if ceilings:
        out["measured_read_gbs"] = ceilings["read_gbs"]
        out["frac_of_measured_read"] = achieved / ceilings["read_gbs"]
    return out


def _public(run):
    return {k: v for k, v in run.items() if not k.startswith("_")}


def large_leg(args):
    """The 300 x 300 shell at rtol 1e-10: FP64 (whose iteration gives the roofline; AUTO's choice
    at this size and tolerance) and mixed precision with AUTO's inner cap of 30 iterations, with
    the mixed result's error against the FP64 one."""
    import paper_2407_20026_amd as sso
    mesh = meshgen.shell_300()
    out = {}
    runs = {}
    for prec in ("fp64", "mixed"):
        opts = sso.Options(rtol=1e-10, max_it=400000, profile_every=args.profile_every,
                           precision=sso.PREC_MIXED if prec == "mixed" else sso.PREC_FP64,
                           refine_steps=20000, inner_max_it=30 if prec == "mixed" else 0)
        runs[prec] = problem_run(mesh, opts, steps=2, warmup=1)
        log(f"300x300 shell {prec}: {runs[prec]['ms_per_step']:.1f} ms per forward + adjoint, "
            f"iteration {runs[prec]['iteration']['avg_us']:.2f} us")
        out[prec] = _public(runs[prec])
    u64, umx = runs["fp64"]["_u"], runs["mixed"]["_u"]
    g64, gmx = runs["fp64"]["_g"], runs["mixed"]["_g"]

    def rel_inf(x, y):
        return float((x - y).abs().max() / y.abs().max())
    out["mixed"]["vs_fp64"] = {"u_rel_2norm": float((umx - u64).norm() / u64.norm()),
                               "dg_dxyz_rel_inf": rel_inf(gmx["dg_dxyz"], g64["dg_dxyz"]),
                               "dg_dt_rel_inf": rel_inf(gmx["dg_dt"], g64["dg_dt"])}
    out["workload"] = "300x300 continuous shell, 543,606 DOF, compliance, rtol 1e-10, seed 2"
    out["mixed"]["precision"] = "mixed (inner solves capped at 30, as AUTO runs it)"
    out["auto_precision"] = "fp64 (K of 234 MB, below the 256 MiB at which AUTO takes mixed " \
                            "precision for rtol 1e-9 or tighter)"
    if out["mixed"].get("outer_steps", 0) == 0:
        raise RuntimeError("mixed precision ran no outer steps on the 300 x 300 shell")
    return out, runs["fp64"]


def out_of_cache_leg(args):
    """The upper-triangle iteration of the single-solve FP64 kernels on a 500 x 500 shell
    (1,506,006 DOF; K 650 MB, the upper triangle 596 MB per iteration: no part of the working set
    stays in the 256 MB Infinity Cache between iterations).  Only the iteration is measured:
    3,000 iterations timed live with HIP events (every 16th, samples of 8 back-to-back
    iterations), the solve stopping at that limit."""
    import paper_2407_20026_amd as sso
    mesh = meshgen.shell(500, seed=5)
    opts = sso.Options(precision=sso.PREC_FP64, rtol=1e-10, max_it=3000, profile_every=16)
    with sso.Problem(mesh, opts) as prob:
        for _ in range(2):   # the first solve pays the pattern, the second is the one kept
            prob.solve(check=False)
        st = prob.last_stats
        n_blocks = prob.n_blocks
    run = {"n_nodes": mesh.n_nodes, "n_blocks": n_blocks,
           "iteration": {"kernels": "k_spmv_dir_single<sym> + k_update_single"
                         if st["sym_products"] else "k_spmv_dir_single + k_update_single",
                         "bytes": st["spmv_bytes"], "avg_us": st["spmv_us"],
                         "samples": st["spmv_samples"]}}
    log(f"500x500 shell: iteration {st['spmv_us']:.2f} us over {st['spmv_samples']} samples")
    return run


def shell60_leg(args):
    import paper_2407_20026_amd as sso
    mesh = meshgen.shell_60()
    opts = sso.Options(rtol=1e-8, max_it=400000, profile_every=args.profile_every)
    run = problem_run(mesh, opts, steps=20, warmup=3)
    log(f"60x60 shell: {run['ms_per_step']:.2f} ms per forward + adjoint")
    out = _public(run)
    out["workload"] = "60x60 continuous shell, 22,326 DOF, FP64, compliance, rtol 1e-8, seed 1"
    return out, run


def general_leg(args):
    """The 60 x 60 shell with a linear objective g = u_z at the centre node: its adjoint is a
    second PCG solve (K lambda = a), unlike compliance where lambda = u."""
    import paper_2407_20026_amd as sso
    run = problem_run(meshgen.shell_60(), sso.Options(rtol=1e-8, max_it=400000), steps=5,
                      warmup=1, objective="linear")
    log(f"general objective: {run['ms_per_step']:.2f} ms per forward + adjoint")
    return {"objective": "linear (u_z at the centre node)", "workload": "60x60 shell",
            "solves_per_s": run["solves_per_s"], "ms_per_step": run["ms_per_step"],
            "pcg_iters": run["pcg_iters"], "adjoint_pcg_iters": run["adjoint_pcg_iters"]}


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
    """Three copies of a float64 buffer of `mib` MiB by the library's copy kernel: a plain copy
    of known size for scaling the HBM counters of a profiled run."""
    from paper_2407_20026_amd import ceiling
    ceiling.measure(mib=mib, reps=3)
    log(f"copy calibration: {mib} MiB")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent problems shard whole across GPUs; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    global torch
    import torch
    import paper_2407_20026_amd as sso

    torch.cuda.set_device(0)
    legs = {x.strip() for x in args.legs.split(",") if x.strip()}
    if args.copy_mib > 0:
        copy_calibration(args.copy_mib)
    ceilings = None

    out = {"metric": METRIC, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic (seeded generators)"}
    roof_of = None   # (run, workload, precision) of the roofline, taken once the ceilings are in
    stream_timing = None
    if args.workload == "stream":
        head, meshes = stream_headline(args)
        stream_timing = head.pop("_timing", None)
        out.update(head)
        cpu_meshes, cpu_what = meshes, "requests of the stream"
    else:
        desc, gen = WORKLOADS[args.workload]
        mesh = gen()
        prec = getattr(sso, PRECISIONS[args.precision])
        solver = {"auto": sso.SOLVER_AUTO, "standard": sso.SOLVER_STANDARD,
                  "fused": sso.SOLVER_FUSED}[args.solver]
        opts = sso.Options(precision=prec, rtol=args.rtol, max_it=400000,
                           profile_every=args.profile_every, solver=solver,
                           refine_steps=args.refine_steps, inner_max_it=args.inner_max_it)
        run = problem_run(mesh, opts, args.steps, args.warmup, args.objective)
        out.update(value=run["solves_per_s"], dof_per_s=run["dof_per_s"],
                   ms_per_step=run["ms_per_step"], p50_ms=run["p50_ms"], p99_ms=run["p99_ms"],
                   dtype={"fp64": "f64", "mixed": "f32 inner PCG / f64 flexible CG",
                          "auto": "f64, f32 inner PCG above the size crossover"}[args.precision],
                   config={"workload": desc, "n_dof": mesh.n_dof, "objective": args.objective,
                           "rtol": args.rtol, "precision": args.precision,
                           **{k: v for k, v in _public(run).items()
                              if k in ("pcg_iters", "adjoint_pcg_iters", "outer_steps",
                                       "rel_residual", "status", "solver", "n_blocks")}})
        roof_of = (run, args.workload, args.precision)
        cpu_meshes, cpu_what = [mesh] * 1000, f"analyses of the {desc}"
    if "large" in legs:
        out["large"], run300 = large_leg(args)
        if roof_of is None:
            roof_of = (run300, "shell300", "fp64")
    run500 = None
    if "large500" in legs:
        run500 = out_of_cache_leg(args)
    run60 = None
    if "shell60" in legs:
        out["shell60"], run60 = shell60_leg(args)
    if "general" in legs:
        out["general_objective"] = general_leg(args)
    if "batch" in legs:
        out["batched"] = batch_bench(SEEDED["shell60"], 16, 1e-8, "compliance",
                                     sso.SOLVER_AUTO)
    if "network" in legs and args.network_variants > 0:
        out["network"] = shellnet_bench(args.network_variants, sso.SOLVER_AUTO)
    if "arch" in legs and args.arch:
        out["arch_replay"] = arch_bench([int(v) for v in args.arch.split(",")])
    # last of the GPU work: the ceilings' 4 GiB of torch buffers and the cache release after
    # them were measured to slow the host calls of a stream that follows (about 2.7 ms per
    # request)
    if "ceilings" in legs:
        from paper_2407_20026_amd import ceiling
        ceilings = ceiling.measure()
        log(f"ceilings: read {ceilings['read_gbs']:.0f} GB/s, copy {ceilings['copy_gbs']:.0f} "
            f"GB/s, FP64 FMA {ceilings['fp64_fma_tflops']:.1f} TFLOP/s")
    if run60 is not None:
        out["shell60"]["roofline"] = roofline_of(run60, "shell60", "fp64", ceilings)
        out["shell60"]["roofline"]["note"] = ("9.4 MB of K: resident in the 256 MB Infinity "
                                              "Cache, not an HBM figure")
    if roof_of is not None:
        out["roofline"] = roofline_of(*roof_of, ceilings)
    if run500 is not None:
        out["shell500_roofline"] = roofline_of(run500, "shell500", "fp64", ceilings)
        out["shell500_roofline"]["note"] = (
            "500x500 shell, 1,506,006 DOF, seed 5: the same kernels with no working set in the "
            "Infinity Cache; iteration only (3,000 iterations, the solve stops at that limit)")
    if args.workload == "stream":
        sr = stream_roofline(stream_timing, ceilings)
        if sr is not None:
            out["stream_roofline"] = sr
    if ceilings:
        out["ceilings"] = ceilings
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cpu_meshes, args.objective, args.cpu_seconds,
                                           cpu_what)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
