"""5-point relative pose + depth (n = 16, 155 terms of degree <= 3, the
general-degree term-list kind) on the GPU through the C ABI, against the
oracle: parameter homotopy from the 40-solution monodromy start set; per
instance the same finite count and the solution sets within 1e-9 relative, in
FP64 and mixed precision; the 1024-instance batch the benchmark runs, sampled."""
import numpy as np
import pytest

import hc_inputs.fivept as F
import _parity
import oracle

pytestmark = pytest.mark.gpu

REL = 1e-9


@pytest.fixture(scope="module")
def hc():
    import paper_2112_03444_amd as hc
    return hc


@pytest.fixture(scope="module")
def ctx(hc):
    c = hc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def family(hc, ctx):
    S = F.fivept_system()
    p0, sols = F.start_instance()
    return S, F.coefficients(p0), sols, ctx.load_system(S, kind=hc.HC_PARAMETER)


def check_sets(ep_g, st_g, ep_o, st_o, hc):
    """Equal finite counts and a one-to-one pairing within 1e-9 (_parity)."""
    return _parity.check_sets(ep_g, st_g, ep_o, st_o, hc.HC_T_SUCCESS, REL)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fivept_parity(hc, ctx, family, precision):
    S, c0, sols, ps = family
    _, coef, _ = F.fivept_instances(4, seed=7300)
    ep, st, info = ctx.track(ps, coef, start=sols, p_start=c0, opts=hc.default_opts(precision=precision))
    oep, ost, _ = oracle.track(S, coef, start=sols, coef0=c0, kind=oracle.LINEAR)
    for i in range(4):
        check_sets(ep[i], st[i], oep[i], ost[i], hc)
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)


def test_fivept_full_batch_sampled(hc, ctx, family):
    S, c0, sols, ps = family
    _, coef, sc = F.fivept_workload("fivept_batch1024")
    ep, st, info = ctx.track(ps, coef, start=sols, p_start=c0, opts=hc.default_opts(precision="mixed"))
    assert ep.shape == (1024, 40, 16)
    ok = st == hc.HC_T_SUCCESS
    assert ok.mean() >= 0.99, np.bincount(st.ravel(), minlength=7)
    assert np.all(info["residual"][ok] <= 1e-10)
    sample = [0, 511, 1023]
    oep, ost, _ = oracle.track(S, coef[sample], start=sols, coef0=c0, kind=oracle.LINEAR)
    for k, i in enumerate(sample):
        check_sets(ep[i], st[i], oep[k], ost[k], hc)
