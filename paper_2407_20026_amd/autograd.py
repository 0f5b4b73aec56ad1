"""torch.autograd bindings of the HIP analysis (argument marshalling only).

The paper couples its differentiable solver to neural networks by chaining the adjoint
sensitivity of the structure into back-propagation (Sec. 2.4, "structural optimization via NN
reparameterization"; the shape-and-topology example of Sec. 3.6 trains an MLP whose outputs are
node heights and element densities, with the structure's compliance as the loss).  Here the
forward pass calls ``sso_problem_update`` + ``sso_solve`` and the backward pass calls
``sso_adjoint``: every number comes from the HIP kernels.

* :class:`Compliance` -- c = f^T u as a function of nodal coordinates, shell thickness and the
  per-element stiffness scale s (SIMP: s = rho^P, Sec. 3.4 Eq. (13); chain the power law in torch).
* :class:`Displacement` -- u as a function of the same inputs; its backward solves the adjoint
  system K lambda = dL/du (Sec. 2.3.1, Eqs. 5-6) with the same K and preconditioner.
* :class:`BatchCompliance` -- the compliances of V problems of one topology that share the
  nodal coordinates and thickness and differ in the stiffness scales, their PCG iterations
  advancing together in multi-problem launches (``sso_batch_iterate``).

A backward pass reads K and u from the problem.  Each forward records the problem's generation
(bumped by every update and solve); if another forward has since run on the same problem (two
losses of one problem summed, say), the backward first restores its own design from the inputs
it saved and solves again, so that every node differentiates the design of its own forward.
"""
from __future__ import annotations

import warnings

import torch

from . import OBJ_COMPLIANCE, OBJ_USER, Problem, SSOError


def _as_f64(x, dev):
    return x.detach().to(device=dev, dtype=torch.float64).contiguous()


def _update(problem: Problem, x, t, s):
    problem.update(xyz=x, quad_t=t, quad_scale=s)


def _restore(ctx, problem: Problem):
    """Bring the problem back to the design of this node's forward if it has moved on."""
    if problem.generation != ctx.gen:
        x, t, s = ctx.saved_tensors
        _update(problem, x, t, s)
        _solve(problem)


def _solve(problem: Problem):
    """Forward solve; a stop above rtol (the FP64 residual floor of an ill-conditioned design
    lies above a very tight rtol) keeps the best iterate and warns, other failures raise."""
    u, st = problem.solve(check=False)
    if problem.last_status == -4:
        warnings.warn(f"PCG stopped at relative residual {st['rel_residual']:.2e} above rtol",
                      RuntimeWarning, stacklevel=3)
    elif problem.last_status != 0:
        raise SSOError(problem.last_status, "sso_solve")
    return u


class Compliance(torch.autograd.Function):
    """c(xyz, t, s) = f^T u for a fixed topology held by ``problem``.

    xyz [n_nodes, 3], t [n_quads], s [n_quads] (float64 tensors on the problem's device).
    Returns a 0-dim float64 tensor on the same device."""

    @staticmethod
    def forward(ctx, problem: Problem, xyz, t, s):
        dev = problem.device
        x = _as_f64(xyz, dev)
        tt = _as_f64(t, dev) if t is not None else None
        ss = _as_f64(s, dev) if s is not None else None
        _update(problem, x, tt, ss)
        _solve(problem)
        c = problem.objective("compliance")
        ctx.problem = problem
        ctx.has_t = t is not None
        ctx.has_s = s is not None
        ctx.gen = problem.generation
        ctx.save_for_backward(x, tt, ss)
        return torch.tensor(c, dtype=torch.float64, device=dev)

    @staticmethod
    def backward(ctx, grad_c):
        _restore(ctx, ctx.problem)
        g = ctx.problem.adjoint(OBJ_COMPLIANCE, want_t=ctx.has_t, want_scale=ctx.has_s)
        w = grad_c.to(torch.float64)
        gx = g["dg_dxyz"] * w
        gt = g["dg_dt"] * w if ctx.has_t else None
        gs = g["dg_dscale"] * w if ctx.has_s else None
        return None, gx, gt, gs


class Displacement(torch.autograd.Function):
    """u(xyz, t, s) [n_nodes, 6]; backward: dL/dp = lambda^T (df/dp - dK/dp u), K lambda = dL/du."""

    @staticmethod
    def forward(ctx, problem: Problem, xyz, t, s):
        dev = problem.device
        x = _as_f64(xyz, dev)
        tt = _as_f64(t, dev) if t is not None else None
        ss = _as_f64(s, dev) if s is not None else None
        _update(problem, x, tt, ss)
        u = _solve(problem)
        ctx.problem = problem
        ctx.has_t = t is not None
        ctx.has_s = s is not None
        ctx.gen = problem.generation
        ctx.save_for_backward(x, tt, ss)
        return u.clone()

    @staticmethod
    def backward(ctx, grad_u):
        _restore(ctx, ctx.problem)
        g = ctx.problem.adjoint(OBJ_USER, dg_du=grad_u.to(torch.float64).contiguous(),
                                want_t=ctx.has_t, want_scale=ctx.has_s)
        return None, g["dg_dxyz"], g["dg_dt"] if ctx.has_t else None, \
            g["dg_dscale"] if ctx.has_s else None


class BatchCompliance(torch.autograd.Function):
    """c_v = f_v^T u_v (v < V) for problems created on ``batch``'s stream; xyz [n_nodes, 3] and
    t [n_quads] shared, s [V, n_quads] per problem.  Returns c [V] (float64, problems' device).
    Backward: dL/dxyz = sum_v dL/dc_v dc_v/dxyz (likewise t), dL/ds_v = dL/dc_v dc_v/ds_v."""

    @staticmethod
    def forward(ctx, batch, problems, chunk, xyz, t, s):
        dev = problems[0].device
        x, tt, ss = _as_f64(xyz, dev), _as_f64(t, dev), _as_f64(s, dev)
        for v, p in enumerate(problems):
            p.update(xyz=x, quad_t=tt, quad_scale=ss[v])
            p.solve_begin()
        done = [False] * len(problems)
        while not all(done):
            done = batch.iterate(problems, chunk)
        c = []
        for p in problems:
            p.solve_end(check=False)
            if p.last_status not in (0, -4):
                raise RuntimeError(f"batched solve failed with status {p.last_status}")
            c.append(p.objective("compliance"))
        ctx.problems = problems
        ctx.gens = [p.generation for p in problems]
        ctx.save_for_backward(x, tt, ss)
        return torch.tensor(c, dtype=torch.float64, device=dev)

    @staticmethod
    def backward(ctx, grad_c):
        w = grad_c.to(torch.float64).cpu().tolist()
        x, tt, ss = ctx.saved_tensors
        gx = gt = None
        gs = []
        for v, (wv, p) in enumerate(zip(w, ctx.problems)):
            if p.generation != ctx.gens[v]:
                _update(p, x, tt, ss[v])
                _solve(p)
            g = p.adjoint(OBJ_COMPLIANCE, want_t=True, want_scale=True)
            with torch.cuda.stream(p.stream):
                gx = g["dg_dxyz"] * wv if gx is None else gx + g["dg_dxyz"] * wv
                gt = g["dg_dt"] * wv if gt is None else gt + g["dg_dt"] * wv
                gs.append(g["dg_dscale"] * wv)
            stream = p.stream
        with torch.cuda.stream(stream):
            gsv = torch.stack(gs)
        torch.cuda.current_stream(gx.device).wait_stream(stream)
        for a in (gx, gt, gsv):
            a.record_stream(torch.cuda.current_stream(gx.device))
        return None, None, None, gx, gt, gsv


def batch_compliance(batch, problems, xyz, t, s, chunk: int = 32):
    return BatchCompliance.apply(batch, problems, chunk, xyz, t, s)


def compliance(problem: Problem, xyz, t=None, s=None):
    return Compliance.apply(problem, xyz, t, s)


def displacement(problem: Problem, xyz, t=None, s=None):
    return Displacement.apply(problem, xyz, t, s)
