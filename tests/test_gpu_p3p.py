"""P3P (section 4, three quadratics in the depths; 8 total-degree paths per
instance, dense kernel tables with n = 3) on the GPU through the C ABI, against
the oracle: per instance the same finite count and the solution sets within
1e-9 relative, in FP64 and in mixed precision; the full 65536-instance batch
the benchmark runs, sampled."""
import numpy as np
import pytest

import hc_inputs.p3p as P
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


def check_sets(ep_g, st_g, ep_o, st_o, hc):
    """Equal finite counts and a one-to-one pairing within 1e-9 (_parity)."""
    return _parity.check_sets(ep_g, st_g, ep_o, st_o, hc.HC_T_SUCCESS, REL)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_p3p_parity(hc, ctx, precision):
    S, coef, gam, _ = P.p3p_instances(64, seed=7100)
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision=precision))
    oep, ost, _ = oracle.track(S, coef, gam)
    for i in range(64):
        check_sets(ep[i], st[i], oep[i], ost[i], hc)
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)


def test_p3p_full_batch_sampled(hc, ctx):
    S, coef, gam, sc = P.p3p_workload("p3p_batch65536")
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision="mixed"))
    assert ep.shape == (65536, 8, 3)
    ok = st == hc.HC_T_SUCCESS
    # a few noisy scenes are near-degenerate (rays or points almost collinear)
    assert ok.mean() >= 0.995, np.bincount(st.ravel(), minlength=7)
    assert np.all(info["residual"][ok] <= 1e-10)
    # the noisy scene's depths lie near one of its positive real roots
    for i in range(0, 65536, 4096):
        f = ep[i][ok[i]]
        d = np.max(np.abs(f - sc["rho"][i]), axis=1) / np.max(sc["rho"][i])
        assert d.min() < 0.05
    sample = [0, 32767, 65535]
    oep, ost, _ = oracle.track(S, coef[sample], gam[sample])
    for k, i in enumerate(sample):
        check_sets(ep[i], st[i], oep[k], ost[k], hc)
