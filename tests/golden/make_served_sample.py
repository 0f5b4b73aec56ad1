"""Write tests/golden/served_sample_oracle.npz: the oracle's forward + adjoint results of a
sample of the mixed-size served stream, for the serving parity test.

The sample is requests 0, 1, 2, 3, 4, 6, 10, 11 and 51 of ``meshgen.served_request`` (per-request
seeds 10^6 + i): 55x55, 54x54, 25x25, 16x16 and 120x120 quad shells (120 is the largest size of
the stream) and 26x26, 41x41, 13x13 and 60x60 grid-shells (60 is the largest).  For each,
``oracle.analyze`` gives the compliance c = f^T u and its adjoint gradient with respect to every
nodal coordinate and quad thickness (Sec. 2.2.1 Eqs. (1)-(3), Sec. 2.3.1 Eqs. (5)-(6)); nothing
of the HIP path is called.

Run from the repository root: ``python tests/golden/make_served_sample.py`` (about 3 minutes).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import meshgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "served_sample_oracle.npz")
SAMPLE = (0, 1, 2, 3, 4, 6, 10, 11, 51)


def main():
    out = {"rids": np.array(SAMPLE, np.int64)}
    t0 = time.perf_counter()
    for i in SAMPLE:
        mesh = meshgen.served_request(i)
        r = oracle.analyze(mesh, "compliance")
        out[f"name_{i}"] = np.array(mesh.name)
        out[f"g_{i}"] = np.array(r["g"])
        out[f"grad_xyz_{i}"] = r["grad_xyz"]
        out[f"grad_t_{i}"] = r["grad_t"]
        print(f"[{time.perf_counter() - t0:6.1f} s] request {i}: {mesh.name}, {mesh.n_dof} DOF, "
              f"c = {r['g']:.12e}", flush=True)
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e6:.2f} MB)")


if __name__ == "__main__":
    main()
