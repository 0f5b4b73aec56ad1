"""The oracle's one-row-at-a-time evaluations agree with its global pattern and assembly."""
import numpy as np

import meshgen
from oracle import assembly


def test_local_rows_match_global_pattern_and_values():
    m = meshgen.shell(5, seed=3)
    m.beam_nodes = np.array([[0, 14], [7, 20]], np.int32)
    m.beam_prop = np.tile([2e11, 8e10, 1e-3, 1e-6, 2e-6, 3e-6], (2, 1))
    pat = assembly.pattern(m)
    K = assembly.assemble(m, pat).tocsr()
    rp, col, perm, seg, S = pat["row_ptr"], pat["col"], pat["perm"], pat["seg"], pat["S"]
    for I in (0, 3, 7, 14, 18, 35):
        cols = assembly.block_row(m, I)
        rows = assembly.K_block_row(m, I)
        for a in range(6):
            r = 6 * I + a
            expect = [6 * J + b for J in cols for b in range(6)]
            assert list(col[rp[r]:rp[r + 1]]) == expect
            for p in range(rp[r], rp[r + 1]):
                assert list(perm[seg[p]:seg[p + 1]]) == assembly.slot_contributions(m, r, col[p])
                J, b = divmod(int(col[p]), 6)
                assert abs(rows[J][a, b] - K.data[p]) <= 1e-13 * abs(K.data).max()
    u = np.random.default_rng(0).normal(size=m.n_dof)
    np.testing.assert_allclose(assembly.apply_K_elementwise(m, u, chunk=7), K @ u, rtol=1e-12,
                               atol=1e-12 * np.abs(K @ u).max())
    assert S.shape == perm.shape
