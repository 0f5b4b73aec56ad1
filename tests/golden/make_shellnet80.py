"""Write tests/golden/shellnet80_oracle.npz: the oracle's adjoint of the network-driven shell
batch at its configured plan size, for the GPU test of the network gradient.

The design is that of the differentiable batch: an 80 x 80 quad plan on a 20 m square, node
heights and element thickness from the seed-4 MLP (Linear(2, 64) -> tanh -> Linear(64, 2),
z = 3 sigmoid(o_0), nodal t = 0.1 + 0.2 sigmoid(o_1), element t = mean of its corners), variant
v scaling element stiffness by rho_v^3 with rho_v ~ U[0.01, 1] from seed 4000 + v (SIMP, Sec.
3.4 Eq. (13); the network example of Sec. 3.6).  For variants 0 and 1, ``oracle.analyze`` gives
the compliance and its adjoint gradient with respect to every nodal coordinate and element
thickness (Sec. 2.3.1 Eqs. (5)-(6)); the MLP's parameters are stored with them so that the test
can chain the gradient through the same network.  Nothing of the HIP path is called.

Run from the repository root: ``python tests/golden/make_shellnet80.py`` (about a minute).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import torch  # noqa: E402

import meshgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "shellnet80_oracle.npz")
M, L, VARIANTS, NET_SEED, RHO_SEED = 80, 20.0, (0, 1), 4, 4000


def main():
    t0 = time.perf_counter()
    base = meshgen.shell(M, L=L, seed=RHO_SEED, flat=True)
    g = torch.random.fork_rng(devices=[])
    with g:
        torch.manual_seed(NET_SEED)
        l1 = torch.nn.Linear(2, 64, dtype=torch.float64)
        l2 = torch.nn.Linear(64, 2, dtype=torch.float64)
    params = [p.detach().numpy().copy() for p in (l1.weight, l1.bias, l2.weight, l2.bias)]
    W1, b1, W2, b2 = params
    xy = base.xyz[:, :2]
    o = np.tanh((xy / L) @ W1.T + b1) @ W2.T + b2
    z = 3.0 / (1.0 + np.exp(-o[:, 0]))
    t = (0.1 + 0.2 / (1.0 + np.exp(-o[:, 1])))[base.quad_nodes].mean(axis=1)
    out = {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "variants": np.array(VARIANTS)}
    for v in VARIANTS:
        m = base.copy()
        m.xyz = np.ascontiguousarray(np.column_stack([xy, z]))
        m.quad_prop = m.quad_prop.copy()
        m.quad_prop[:, 0] = t
        m.quad_scale = meshgen.density_field(base.n_quads, v, RHO_SEED) ** 3
        r = oracle.analyze(m, "compliance")
        out[f"c_{v}"] = np.array(r["g"])
        out[f"grad_xyz_{v}"] = r["grad_xyz"]
        out[f"grad_t_{v}"] = r["grad_t"]
        print(f"[{time.perf_counter() - t0:6.1f} s] variant {v}: c = {r['g']:.12e}", flush=True)
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e6:.2f} MB)")


if __name__ == "__main__":
    main()
