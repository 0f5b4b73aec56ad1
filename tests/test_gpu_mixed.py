"""Mixed precision (FP32 inner PCG inside FP64 iterative refinement) against the FP64 oracle.

The FP64 residual is recomputed with the FP64 K, so the refinement reaches the same residual
target as the FP64 path; the error of u and of the gradients against the oracle is checked at
the accuracy that residual implies and printed for the record."""
import numpy as np
import pytest

import meshgen
import oracle
from oracle import assembly

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "grid11": meshgen.grid_shell_11,
    "shell8": lambda: meshgen.shell(8, L=8.0, seed=3),
    "shell60": meshgen.shell_60,
}


@pytest.fixture(scope="module")
def refs():
    cache = {}

    def get(name):
        if name not in cache:
            mesh = CASES[name]()
            cache[name] = (mesh, oracle.analyze(mesh, "compliance", pat=assembly.pattern(mesh)))
        return cache[name]
    return get


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_refinement_reaches_fp64_residual(refs, name):
    import paper_2407_20026_amd as sso
    mesh, r = refs(name)
    print(f"[gpu] mixed {name}", flush=True)
    opts = sso.Options(precision=sso.PREC_MIXED, rtol=1e-10, max_it=200000, refine_steps=30)
    with sso.Problem(mesh, opts) as p:
        u, st = p.solve()
        g = p.adjoint("compliance")
    u = u.cpu().numpy().ravel()
    err_u = np.linalg.norm(u - r["u"]) / np.linalg.norm(r["u"])
    gx = g["dg_dxyz"].cpu().numpy()
    err_g = np.abs(gx - r["grad_xyz"]).max() / np.abs(r["grad_xyz"]).max()
    print(f"  inner iters={st['iters']} refine={st['refine_steps']} "
          f"rel_res={st['rel_residual']:.2e} |du|/|u|={err_u:.2e} grad err={err_g:.2e}")
    assert st["rel_residual"] <= 1e-10
    assert err_u <= 1e-6
    assert err_g <= 1e-5


def test_mixed_and_fp64_agree_on_the_same_gpu():
    import paper_2407_20026_amd as sso
    mesh = meshgen.shell(20, seed=7)
    out = {}
    for prec in (sso.PREC_FP64, sso.PREC_MIXED):
        with sso.Problem(mesh, sso.Options(precision=prec, rtol=1e-10)) as p:
            u, st = p.solve()
            out[prec] = (u.cpu().numpy(), st)
    d = np.linalg.norm(out[0][0] - out[1][0]) / np.linalg.norm(out[0][0])
    print(f"[gpu] fp64 vs mixed: |du|/|u|={d:.2e} iters {out[0][1]['iters']} / "
          f"{out[1][1]['iters']}")
    assert d <= 1e-6


def test_auto_precision_runs_fp64_below_the_crossover():
    """SSO_PREC_AUTO on a problem whose K stays in the caches runs plain FP64: no outer steps,
    and u bitwise that of the FP64 precision."""
    import paper_2407_20026_amd as sso
    print("[gpu] AUTO precision below the crossover", flush=True)
    mesh = meshgen.shell(40, seed=17)
    us = {}
    for name, prec in (("auto", sso.PREC_AUTO), ("fp64", sso.PREC_FP64)):
        with sso.Problem(mesh, sso.Options(rtol=1e-10, precision=prec)) as p:
            u, st = p.solve()
            us[name] = (u.cpu(), st["refine_steps"])
    assert us["auto"][1] == 0
    assert torch.equal(us["auto"][0], us["fp64"][0])
