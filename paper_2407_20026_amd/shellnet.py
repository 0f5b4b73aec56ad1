"""Differentiable batch of shell variants driven by a neural network.

The paper's physics-in-the-loop workflow (Sec. 2.4; example of Sec. 3.6): an MLP maps the plan
coordinates of every node to the node height and to a shell thickness, the structure is
analysed, and the loss (compliance) is back-propagated through the solver's adjoint into the
network weights.  Here a batch of variants shares the network and the plan; each variant has
its own seeded element density rho, which scales the element stiffness by rho^3 (SIMP with
P = 3, Sec. 3.4 Eq. (13); the loads do not depend on rho).  Network: Linear(2, 64) -> tanh ->
Linear(64, 2); z = 3 sigmoid(o_0) m, nodal t = 0.1 + 0.2 sigmoid(o_1) m, element t = mean of its
4 corners; loss = mean compliance over the variants.

Every structural number comes from the HIP kernels through :mod:`paper_2407_20026_amd.autograd`.
"""
from __future__ import annotations

import numpy as np
import torch

import meshgen

from . import Batch, Options, Problem
from .autograd import batch_compliance, compliance


class DesignMLP(torch.nn.Module):
    def __init__(self, hidden: int = 64, seed: int = 4):
        super().__init__()
        g = torch.random.fork_rng(devices=[])
        with g:
            torch.manual_seed(seed)
            self.l1 = torch.nn.Linear(2, hidden, dtype=torch.float64)
            self.l2 = torch.nn.Linear(hidden, 2, dtype=torch.float64)

    def forward(self, xy):
        return self.l2(torch.tanh(self.l1(xy)))


def geometry(net: DesignMLP, xy: torch.Tensor, L: float, quad_nodes: torch.Tensor):
    """(xyz [n, 3], element thickness [n_quads]) from the network."""
    o = net(xy / L)
    z = 3.0 * torch.sigmoid(o[:, 0])
    t_node = 0.1 + 0.2 * torch.sigmoid(o[:, 1])
    xyz = torch.cat([xy, z[:, None]], dim=1)
    t = t_node[quad_nodes].mean(dim=1)
    return xyz, t


class ShellBatch:
    """n_variants problems on one m x m plan; ``loss(net)`` is differentiable in the weights.
    batched=True: the variants' PCG iterations advance together in multi-problem launches on
    one stream (results bitwise equal to solving them one by one)."""

    def __init__(self, m: int = 80, n_variants: int = 256, L: float = 20.0,
                 options: Options | None = None, device="cuda", density_seed: int = 4000,
                 batched: bool = False):
        self.base = meshgen.shell(m, L=L, seed=density_seed, flat=True)
        self.L = L
        self.device = torch.device(device)
        self.xy = torch.as_tensor(self.base.xyz[:, :2], dtype=torch.float64, device=self.device)
        self.quads = torch.as_tensor(self.base.quad_nodes.astype(np.int64), device=self.device)
        self.rho = [torch.as_tensor(meshgen.density_field(self.base.n_quads, v, density_seed),
                                    dtype=torch.float64, device=self.device)
                    for v in range(n_variants)]
        opts = options or Options(rtol=1e-8)
        self.batched = batched
        self.stream = torch.cuda.Stream(device=self.device) if batched else None
        self.batch = Batch(self.stream, self.device) if batched else None
        self.problems = []
        for v in range(n_variants):
            mv = self.base.copy()
            mv.quad_scale = self.rho[v].cpu().numpy() ** 3
            self.problems.append(Problem(mv, opts, device=self.device, stream=self.stream))

    def loss(self, net: DesignMLP):
        xyz, t = geometry(net, self.xy, self.L, self.quads)
        if self.batched:
            s = torch.stack(self.rho) ** 3
            return batch_compliance(self.batch, self.problems, xyz, t, s).mean()
        total = 0.0
        for prob, rho in zip(self.problems, self.rho):
            total = total + compliance(prob, xyz, t, rho ** 3)
        return total / len(self.problems)

    def close(self):
        for p in self.problems:
            p.close()
        self.problems = []
        if self.batch is not None:
            self.batch.close()
            self.batch = None
