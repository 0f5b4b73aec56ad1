"""Host-side logic of the request loop (no GPU): footprint bound and rejection of requests that
can never fit."""
import numpy as np
import pytest

import meshgen


def test_footprint_grows_with_size_and_bounds_the_matrix():
    from paper_2407_20026_amd.serve import footprint_bytes
    small, large = meshgen.shell(10), meshgen.shell(40)
    assert footprint_bytes(large) > footprint_bytes(small)
    # (3m+1)^2 blocks: K and B = K M in FP64 (288 bytes each), or K in FP64 and B in FP32 for
    # mixed precision; element list 4608 bytes per quad
    m = 40
    nb = (3 * m + 1) ** 2
    assert footprint_bytes(large) > 2 * 288 * nb + 4608 * m * m
    assert footprint_bytes(large, mixed=True) > (288 + 144) * nb + 4608 * m * m
    g = meshgen.gridshell(20)
    assert footprint_bytes(g) > 288 * (20 * 20 + 4 * 20 * 19)


def test_request_above_budget_is_rejected_before_any_device_work():
    from paper_2407_20026_amd.serve import Request, Server, footprint_bytes
    mesh = meshgen.shell(20)
    srv = Server(slots=2, hbm_budget=footprint_bytes(mesh) - 1)
    with pytest.raises(ValueError):
        srv.run([Request(0, mesh, 0.0)])


def test_poisson_arrivals_rate():
    from paper_2407_20026_amd.serve import poisson_arrivals
    t = poisson_arrivals(20000, 50.0, seed=1)
    assert np.all(np.diff(t) > 0)
    assert 20000 / t[-1] == pytest.approx(50.0, rel=0.03)
