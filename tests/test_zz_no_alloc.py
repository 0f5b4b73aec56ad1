"""The no-allocation form of the penalised-volume objective (sso_size_objective_noalloc) against
the allocating form (sso_size_objective), through the C ABI: bitwise the same g, c, W and
gradients, on two calls in a row (the second on a smaller problem, so the shared static scratch
holds the first call's larger contents), and a clear error above the scratch's size limit."""
import ctypes

import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _call(p, fn, eps1, u_max, t_min):
    import paper_2407_20026_amd as sso
    gx = torch.full((p.n_nodes, 3), np.nan, dtype=torch.float64, device="cuda")
    gt = torch.full((p.n_quads,), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    res = (ctypes.c_double * 3)()
    st = sso.sso_stats()
    status = fn(p.handle, eps1, u_max, t_min, res, ctypes.c_void_p(gx.data_ptr()),
                ctypes.c_void_p(gt.data_ptr()), ctypes.byref(st))
    return status, list(res), gx.cpu().numpy(), gt.cpu().numpy()


def test_noalloc_size_objective_matches_allocating_form():
    import paper_2407_20026_amd as sso
    lib = sso.load_library()
    print("[gpu] no-allocation size objective: 24x24 shell, then 10x10 shell", flush=True)
    cases = [(meshgen.shell(24, L=12.0, seed=21), 2.0, 1e-4, 0.15),
             (meshgen.shell(10, L=6.0, seed=22), 0.5, 5e-5, 0.2)]
    for mesh, eps1, u_max, t_min in cases:
        with sso.Problem(mesh, sso.Options(rtol=1e-10)) as p:
            p.solve()
            st_a, ra, gxa, gta = _call(p, lib.sso_size_objective, eps1, u_max, t_min)
            st_n, rn, gxn, gtn = _call(p, lib.sso_size_objective_noalloc, eps1, u_max, t_min)
        print(f"  {mesh.name}: status {st_a} / {st_n}, g = {ra[0]:.12e} / {rn[0]:.12e}",
              flush=True)
        assert st_a == sso.SSO_OK and st_n == sso.SSO_OK
        assert ra[1] > 0.0          # some displacement limit is active: the adjoint solve ran
        assert rn == ra             # g, c, W bitwise
        assert np.array_equal(gxn, gxa) and np.array_equal(gtn, gta)
        assert np.all(np.isfinite(gxn)) and np.all(np.isfinite(gtn))


def test_noalloc_rejects_problems_above_the_scratch_limit():
    import paper_2407_20026_amd as sso
    lib = sso.load_library()
    m = 374   # 139,876 quads, above the 139,673 the 16 MiB scratch holds
    assert m * m > sso.NOALLOC_MAX_QUADS
    print(f"[gpu] no-allocation size objective: {m}x{m} shell rejected", flush=True)
    with sso.Problem(meshgen.shell(m, seed=23)) as p:
        res = (ctypes.c_double * 3)()
        status = lib.sso_size_objective_noalloc(p.handle, 1.0, 1e-3, 0.1, res, None, None, None)
    assert status == sso.SSO_ESIZE
    assert "static scratch" in lib.sso_strerror(status).decode()
