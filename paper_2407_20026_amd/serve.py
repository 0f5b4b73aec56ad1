"""Continuous-batching request loops for forward + adjoint analyses of mixed-size structures.

Requests (a structure and an objective) arrive over time.  A request is admitted as soon as a
slot is free and its device-memory footprint fits in the remaining budget; a finished request
frees its slot and its memory at once and the next waiting request is admitted.  Per request
the loops record arrival, admission and completion times, so p50/p99 latency (arrival to
result) and throughput (solves/s, DOF/s) are reported side by side.

* :class:`BatchedServer` -- one host thread: every admitted request's PCG iterations run in
  shared launches on one stream (``sso_batch_launch`` / ``sso_batch_wait``: one launch per
  kernel for all requests in flight, each request on its own range of workgroups); requests are
  admitted and finished on a second stream while the next chunk runs, and join and leave the
  iterations at the chunk boundaries.  FP64, mixed precision (FP32 inner iterations, FP64
  refinement) or AUTO.
* :class:`Server` -- one host thread and one HIP stream per slot, each slot solving its request
  with ``sso_solve``.

Every number comes from the HIP library; K, the preconditioner and u stay on the device for a
request's lifetime.
"""
from __future__ import annotations

import collections
import hashlib
import threading
import time
from dataclasses import dataclass, field, replace

import numpy as np
import torch

from . import PREC_MIXED, SOLVER_AUTO, SOLVER_WG, Options, Problem


# sso_solve's automatic choice of the single-reduction recurrences (which keep B = K M beside
# K) stops at this many nodes (include/hipsso.h, SSO_SOLVER_AUTO)
FUSED_MAX_NODES = 8192


ARENA_CHUNK = 2 << 20      # the library's chunk size for the buffers of one owner


def _arena_bound(bufs) -> int:
    """Device memory an owner holds for buffers of the given byte sizes: a buffer above a
    quarter chunk has a chunk of its own, smaller ones share chunks that are left only when
    less than a quarter chunk is free (so each but the last is at least 3/4 used)."""
    big = sum(-(-b // 256) * 256 for b in bufs if b > ARENA_CHUNK // 4)
    small = sum(-(-b // 256) * 256 for b in bufs if b <= ARENA_CHUNK // 4)
    chunks = 0 if small == 0 else int(small * 4 / 3 // ARENA_CHUNK) + 1
    return big + chunks * ARENA_CHUNK


def footprint_bytes(mesh, mixed: bool | None = False) -> int:
    """Upper bound of the device memory one problem holds after its forward and adjoint
    (mesh copies, pattern, element list, K, packed preconditioner, B = K M of the
    single-reduction PCG or the FP32 copies of mixed precision, solver vectors, gradients),
    in the chunks the library carves them from.  mixed=None: the precision is picked by the
    library (AUTO), either bound.  Checked against the library's own count (sso_problem_bytes)
    in the serving tests."""
    if mixed is None:
        return max(footprint_bytes(mesh, False), footprint_bytes(mesh, True))
    nn, nb, nq = mesh.n_nodes, mesh.n_beams, mesh.n_quads
    blocks = nn + 2 * nb + 12 * nq                  # diagonal + off-diagonal blocks (bound)
    padded = 12 * nn                                # padded block rows, 12 slots at most
    nbcoo = 4 * nb + 16 * nq
    ndof = 6 * nn
    dinv = 21 * (nn + 63) // 64 * 64                # packed inverses, whole groups of 64
    pattern = [4 * nbcoo] * 3 + [4 * blocks] * 3 + [4 * (nn + 1)] * 4 + [4 * padded]
    bufs = [24 * nn, 6 * nn, 48 * nn, 8 * nb, 48 * nb, 16 * nq, 40 * nq, 8 * nq]   # mesh copies
    bufs += [8 * (144 * nb + 576 * nq), 8 * nq]                                    # elements
    bufs += [288 * blocks, 8 * dinv]                                               # K, Dinv
    bufs += [8 * ndof] * 14 + [8 * 6 * nb, 8 * 14 * nq]                            # vectors, grads
    bufs += [8 * 11 * 1024, 4096, 64]                                              # partials
    if mixed:
        bufs += [144 * max(blocks, padded), 4 * dinv] + [4 * ndof] * 11
    elif nn <= FUSED_MAX_NODES:
        bufs += [288 * max(blocks, padded)]  # B = K M in FP64 (single-reduction recurrences)
    return int(1.05 * (_arena_bound(pattern) + _arena_bound(bufs))) + (1 << 20)


@dataclass
class Request:
    rid: int
    mesh: object
    arrival: float                      # seconds from the start of the stream
    objective: str = "compliance"


@dataclass
class Result:
    rid: int
    n_dof: int
    g: float
    grad_xyz: np.ndarray
    grad_t: np.ndarray | None
    iters: int
    arrival: float
    admitted: float
    done: float
    status: int = 0              # SSO_OK, or SSO_ENOTCONV (stopped above rtol)
    rel_residual: float = 0.0    # true relative residual of the solve
    outer_steps: int = 0         # FP64 outer steps (> 0: the request ran in mixed precision)
    iter_bytes: float = 0.0      # algorithmic bytes of its PCG iterations (iters x per iteration)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServeStats:
    n: int
    wall_s: float
    solves_per_s: float
    dof_per_s: float
    p50_ms: float
    p99_ms: float
    mean_queue_ms: float
    peak_inflight: int
    peak_bytes: int
    results: list = field(repr=False, default_factory=list)
    host_s: dict = field(default_factory=dict)   # BatchedServer: wall time per phase
    not_converged: int = 0         # requests that stopped above rtol (status SSO_ENOTCONV)
    max_rel_residual: float = 0.0  # largest true relative residual over the requests
    iteration_bytes_per_s: float = 0.0   # the requests' algorithmic PCG iteration bytes / wall
    streams_overlap: bool | None = None  # BatchedServer: its two streams ran concurrently
    # BatchedServer(profile_every > 0): sums of the timed FP64 standard iteration spans
    # (Batch.timing: event us, iterations, algorithmic bytes all-K and as read)
    iteration_timing: dict | None = None


def _convergence(results) -> dict:
    """How many requests stopped above rtol, and the largest true residual."""
    return {"not_converged": sum(1 for r in results if r.status != 0),
            "max_rel_residual": max((r.rel_residual for r in results), default=0.0)}


def topology_key(mesh):
    """Requests with equal keys have the same node, member and quad counts and connectivity,
    so one problem's pattern can be shared with the next (sso_problem_create_like)."""
    h = hashlib.blake2b(digest_size=16)
    for a in (mesh.beam_nodes, mesh.quad_nodes):
        h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
    return (int(mesh.n_nodes), int(mesh.beam_nodes.shape[0]), int(mesh.quad_nodes.shape[0]),
            h.hexdigest())


def errors_against(results, reference) -> list[dict]:
    """Per request, the error of each result against the same request's result in a reference
    run (e.g. the plain FP64 path): relative error of g, and max-norm relative errors of dg/dxyz
    and dg/dt.  Requests are matched by id; ids missing from the reference are skipped."""
    ref = {r.rid: r for r in reference}
    out = []
    for r in results:
        q = ref.get(r.rid)
        if q is None:
            continue
        e = {"rid": r.rid, "n_dof": r.n_dof,
             "g_rel": abs(r.g - q.g) / max(abs(q.g), 1e-300),
             "dg_dxyz_rel_inf": float(np.abs(r.grad_xyz - q.grad_xyz).max() /
                                      max(np.abs(q.grad_xyz).max(), 1e-300))}
        if r.grad_t is not None and q.grad_t is not None and q.grad_t.size:
            e["dg_dt_rel_inf"] = float(np.abs(r.grad_t - q.grad_t).max() /
                                       max(np.abs(q.grad_t).max(), 1e-300))
        out.append(e)
    return out


def run_one(req: Request, options: Options, stream=None, device="cuda") -> Result:
    """Forward + adjoint of one request on ``stream`` (used by the loop and to check results
    alone)."""
    t0 = time.perf_counter()
    with Problem(req.mesh, options, device=device, stream=stream) as p:
        _, st = p.solve(check=False)
        if p.last_status not in (0, -4):
            raise RuntimeError(f"request {req.rid}: solve status {p.last_status}")
        g = p.objective(req.objective)
        gr = p.adjoint(req.objective)
        gx = gr["dg_dxyz"].cpu().numpy()
        gt = gr["dg_dt"].cpu().numpy() if gr["dg_dt"] is not None else None
    t1 = time.perf_counter()
    return Result(req.rid, req.mesh.n_dof, g, gx, gt, st["iters"], 0.0, t0, t1,
                  p.last_status, st["rel_residual"], st["refine_steps"])


class Server:
    """Admission by slot count and device-memory budget; one host thread and one HIP stream
    per slot."""

    def __init__(self, slots: int = 4, hbm_budget: int = 64 << 30, options: Options | None = None,
                 device="cuda"):
        self.slots = slots
        self.budget = hbm_budget
        self.options = options or Options()
        self.device = torch.device(device)
        # FP64, mixed, or AUTO (the library picks per problem: either footprint)
        self.mixed = {0: False, 1: True}.get(self.options.precision)

    def run(self, requests: list[Request]) -> ServeStats:
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            if footprint_bytes(r.mesh, self.mixed) > self.budget:
                raise ValueError(f"request {r.rid} can never be admitted: footprint above budget")
        cond = threading.Condition()
        waiting = collections.deque()
        results: list[Result] = []
        state = dict(free=self.budget, inflight=0, peak_inflight=0, peak_bytes=0,
                     arrived=0, finished=0, error=None)
        t_start = time.perf_counter()

        def clock():
            return time.perf_counter() - t_start

        def arrivals():
            for r in reqs:
                delay = r.arrival - clock()
                if delay > 0:
                    time.sleep(delay)
                with cond:
                    waiting.append(r)
                    state["arrived"] += 1
                    cond.notify_all()

        def worker(stream):
            while True:
                with cond:
                    while True:
                        if state["error"] is not None:
                            return
                        if waiting and footprint_bytes(waiting[0].mesh, self.mixed) <= \
                                state["free"]:
                            req = waiting.popleft()
                            need = footprint_bytes(req.mesh, self.mixed)
                            state["free"] -= need
                            state["inflight"] += 1
                            state["peak_inflight"] = max(state["peak_inflight"],
                                                         state["inflight"])
                            state["peak_bytes"] = max(state["peak_bytes"],
                                                      self.budget - state["free"])
                            break
                        if state["arrived"] == len(reqs) and not waiting:
                            return
                        cond.wait()
                admitted = clock()
                try:
                    res = run_one(req, self.options, stream=stream, device=self.device)
                except Exception as e:  # stop the loop, report the first failure
                    with cond:
                        state["error"] = e
                        cond.notify_all()
                    return
                res.arrival, res.admitted, res.done = req.arrival, admitted, clock()
                with cond:
                    results.append(res)
                    state["free"] += need
                    state["inflight"] -= 1
                    state["finished"] += 1
                    cond.notify_all()

        streams = [torch.cuda.Stream(device=self.device) for _ in range(self.slots)]
        threads = [threading.Thread(target=worker, args=(s,), daemon=True) for s in streams]
        feeder = threading.Thread(target=arrivals, daemon=True)
        for t in threads:
            t.start()
        feeder.start()
        feeder.join()
        for t in threads:
            t.join()
        if state["error"] is not None:
            raise state["error"]
        wall = clock()
        lat = np.array([r.latency for r in results])
        dof = sum(r.n_dof for r in results)
        return ServeStats(
            n=len(results), wall_s=wall, solves_per_s=len(results) / wall, dof_per_s=dof / wall,
            p50_ms=1000 * float(np.percentile(lat, 50)), p99_ms=1000 * float(np.percentile(lat, 99)),
            mean_queue_ms=1000 * float(np.mean([r.admitted - r.arrival for r in results])),
            peak_inflight=state["peak_inflight"], peak_bytes=state["peak_bytes"],
            results=sorted(results, key=lambda r: r.rid), **_convergence(results))


def finish_one(p: Problem, req: Request):
    """Finish a request whose iteration has stopped: FP64 refinement, objective, adjoint."""
    _, st = p.solve_end(check=False)
    if p.last_status not in (0, -4):
        raise RuntimeError(f"request {req.rid}: solve status {p.last_status}")
    g = p.objective(req.objective)
    gr = p.adjoint(req.objective)
    with torch.cuda.stream(p.stream):   # the copies on the problem's stream, after its work
        gx = gr["dg_dxyz"].cpu().numpy()
        gt = gr["dg_dt"].cpu().numpy() if gr["dg_dt"] is not None else None
    return (g, gx, gt, st["iters"], p.last_status, st["rel_residual"], st["refine_steps"],
            st["iters"] * st["spmv_bytes"])


def streams_overlap(a, b, spin_cycles: int = 4_000_000):
    """Whether work enqueued on stream b runs while a kernel on stream a is still running.  The
    runtime maps streams onto a small pool of hardware queues (four by default); two streams on
    one queue run in order, so a second stream only overlaps the first if their queues differ.
    A bounded spin kernel on a, an event after it on a, then an event on b: on separate queues
    b's event completes at once while a's is still pending; on a shared queue b's completes after
    a's.  None if the spin kernel is not available."""
    sleep = getattr(torch.cuda, "_sleep", None)
    if sleep is None:
        return None
    ea, eb = torch.cuda.Event(), torch.cuda.Event()
    with torch.cuda.stream(a):
        sleep(spin_cycles)
    ea.record(a)
    eb.record(b)
    eb.synchronize()
    overlap = not ea.query()
    a.synchronize()
    return overlap


class BatchedServer:
    """Admission by slot count and device-memory budget; the iterations of all requests in
    flight advance together in multi-problem launches on one stream.

    overlap=True (default): requests are admitted (creation, elements, assembly, PCG start) and
    finished (true residual, objective, adjoint, copies) on a second stream while the next chunk
    of iterations runs: the loop launches a chunk (sso_batch_launch), does the host and admission
    work of the requests that stopped at the previous poll or arrived since, then waits for the
    chunk (sso_batch_wait).  A request moves to the launcher's stream when it joins the
    iterations and back when it stops (sso_problem_set_stream).  The kernels and their
    decomposition are the same either way, so every result is bitwise the same."""

    def __init__(self, slots: int = 64, hbm_budget: int = 64 << 30,
                 options: Options | None = None, device="cuda", chunk: int = 32,
                 share_patterns: bool = True, overlap: bool = True, wg_max_nodes: int = 0,
                 profile_every: int = 0, profile_span: int = 8):
        # profile_every > 0: time the first profile_span iterations of every profile_every-th
        # chunk of FP64 standard problems with HIP events (Batch.profile); kernels unchanged
        self.profile_every = profile_every
        self.profile_span = profile_span
        self.share_patterns = share_patterns
        self.overlap = overlap
        self.slots = slots
        self.budget = hbm_budget
        self.options = options or Options()
        # FP64, mixed, or AUTO (the library picks per problem: either footprint)
        self.mixed = {0: False, 1: True}.get(self.options.precision)
        self.device = torch.device(device)
        self.chunk = chunk
        # wg_max_nodes > 0: requests of at most that many nodes run on one workgroup each
        # (SSO_SOLVER_WG) whatever their size in LDS; 0: the library's AUTO choice, which puts the
        # LDS-resident ones (at most 144 nodes) there
        self.wg_max_nodes = wg_max_nodes
        self.options_wg = None
        if wg_max_nodes > 0 and self.options.solver == SOLVER_AUTO and \
                self.options.precision != PREC_MIXED:
            self.options_wg = replace(self.options, solver=SOLVER_WG)

    def options_for(self, mesh) -> Options:
        if self.options_wg is not None and mesh.n_nodes <= self.wg_max_nodes:
            return self.options_wg
        return self.options

    def run(self, requests: list[Request]) -> ServeStats:
        from . import Batch
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            if footprint_bytes(r.mesh, self.mixed) > self.budget:
                raise ValueError(f"request {r.rid} can never be admitted: footprint above budget")
        it_stream = torch.cuda.Stream(device=self.device)
        aux = it_stream
        overlapping = None
        if self.overlap:
            # a second stream that does not share the iteration stream's hardware queue (on a
            # shared one every finishing synchronisation waits for the running chunk: measured
            # 101 against 112 solves/s); the next streams of torch's pool until one overlaps
            for _ in range(8):
                aux = torch.cuda.Stream(device=self.device)
                overlapping = streams_overlap(it_stream, aux)
                if overlapping is not False:
                    break
        batch = Batch(it_stream, self.device)
        if self.profile_every > 0:
            batch.profile(self.profile_every, self.profile_span)
        timing = None
        waiting = collections.deque()
        active = []          # iterating: (problem, request, admitted time, footprint)
        joining = []         # begun on the admission stream, join at the next launch
        finishing = []       # stopped at the last poll, finished on the admission stream
        live = collections.defaultdict(set)   # topology -> problems in flight (shared patterns)
        results: list[Result] = []
        free = self.budget
        peak_inflight = peak_bytes = 0
        nxt = 0
        t_start = time.perf_counter()
        phase = dict(admit=0.0, iterate=0.0, finish=0.0, idle=0.0)

        def clock():
            return time.perf_counter() - t_start

        def admit():
            nonlocal free
            while waiting and len(active) + len(joining) < self.slots and \
                    footprint_bytes(waiting[0].mesh, self.mixed) <= free:
                req = waiting.popleft()
                need = footprint_bytes(req.mesh, self.mixed)
                free -= need
                key = topology_key(req.mesh) if self.share_patterns else None
                like = next(iter(live[key]), None) if key in live else None
                p = Problem(req.mesh, self.options_for(req.mesh), device=self.device, stream=aux,
                            like=like)
                p.topology = key
                if key is not None:
                    live[key].add(p)
                p.solve_begin()
                joining.append((p, req, clock(), need))

        def finish():
            nonlocal free
            for p, req, adm, need in finishing:
                g, gx, gt, iters, status, rres, outer, ib = finish_one(p, req)
                if p.topology is not None:
                    live[p.topology].discard(p)
                p.close()
                free += need
                results.append(Result(req.rid, req.mesh.n_dof, g, gx, gt, iters,
                                      req.arrival, adm, clock(), status, rres, outer, ib))
            finishing.clear()

        try:
            while len(results) < len(reqs):
                now = clock()
                while nxt < len(reqs) and reqs[nxt].arrival <= now:
                    waiting.append(reqs[nxt])
                    nxt += 1
                for item in joining:
                    item[0].set_stream(it_stream)
                    active.append(item)
                joining.clear()
                peak_inflight = max(peak_inflight, len(active))
                peak_bytes = max(peak_bytes, self.budget - free)
                t0 = time.perf_counter()
                if active:
                    batch.launch([a[0] for a in active], self.chunk)
                # while the chunk runs: finish what stopped at the last poll, admit arrivals
                t1 = time.perf_counter()
                finish()
                t2 = time.perf_counter()
                admit()
                t3 = time.perf_counter()
                phase["finish"] += t2 - t1
                phase["admit"] += t3 - t2
                if active:
                    done = batch.wait([a[0] for a in active])
                    still = []
                    for flag, item in zip(done, active):
                        if flag:
                            item[0].set_stream(aux)
                            finishing.append(item)
                        else:
                            still.append(item)
                    active = still
                    phase["iterate"] += (t1 - t0) + (time.perf_counter() - t3)
                elif not joining and not finishing and nxt < len(reqs):
                    time.sleep(max(0.0, reqs[nxt].arrival - clock()))
                    phase["idle"] += time.perf_counter() - t3
            if self.profile_every > 0:
                timing = batch.timing()
        finally:
            for p, *_ in active + joining + finishing:
                p.close()
            batch.close()
        wall = clock()
        lat = np.array([r.latency for r in results])
        dof = sum(r.n_dof for r in results)
        return ServeStats(
            n=len(results), wall_s=wall, solves_per_s=len(results) / wall, dof_per_s=dof / wall,
            p50_ms=1000 * float(np.percentile(lat, 50)), p99_ms=1000 * float(np.percentile(lat, 99)),
            mean_queue_ms=1000 * float(np.mean([r.admitted - r.arrival for r in results])),
            peak_inflight=peak_inflight, peak_bytes=peak_bytes,
            results=sorted(results, key=lambda r: r.rid),
            host_s=phase, iteration_bytes_per_s=sum(r.iter_bytes for r in results) / wall,
            streams_overlap=overlapping, iteration_timing=timing,
            **_convergence(results))


def poisson_arrivals(n: int, rate: float, seed: int = 3) -> np.ndarray:
    """Arrival times (s) of n requests of a Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))
