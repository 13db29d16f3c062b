"""Monodromy with the paths tracked on the GPU (paper_2112_03444_amd.monodromy):
the 4-view and 3-view triangulation families, from the same seed as the stored
start sets, reach Table 2's 296 and 94 solutions and the oracle's sets."""
import numpy as np
import pytest

import hc_inputs.vision as V

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_views,count", [(4, 296), (3, 94)])
def test_triangulation_monodromy_on_gpu_reproduces_the_oracle_set(n_views, count):
    import paper_2112_03444_amd as hc
    import paper_2112_03444_amd.monodromy as GM
    ctx = hc.Context(0)
    try:
        S = V.triangulation_system(n_views)
        c0, sols = GM.monodromy(ctx, GM.LinearFamily(S), seed=4, stall=10)
    finally:
        ctx.close()
    c0s, sols_s = V.start_instance(n_views)
    # the same fabricated start instance (same seed, same draw order)
    assert np.max(np.abs(c0 - c0s)) <= 1e-12 * np.max(np.abs(c0s))
    assert sols.shape == (count, S.n)
    # the same solutions: each stored one matched, relative 1e-8
    for x in sols_s:
        d = np.max(np.abs(sols - x), axis=1) / np.maximum(1.0, np.max(np.abs(x)))
        assert d.min() <= 1e-8
    assert len(GM.distinct(sols)) == count
