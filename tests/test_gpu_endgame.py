"""The power-series end-game (opts.endgame) on the GPU, through the C ABI, against
the oracle's end-game and against what the systems themselves fix.

Bar: the same statuses as the oracle path by path where the end-game decides
them on known systems; regular roots within 1e-9 (FP64 refinement); singular
endpoints (the end-game's extrapolated estimate, not refined) within 1e-8 of
the exact root and of the oracle's estimate -- the estimate of a root of
multiplicity m carries the extrapolation error of the last samples, about
sigma^3 = s^(3/m) at the last sample's distance s from t = 1, far below 1e-8
for the samples these systems reach."""
import numpy as np
import pytest

import _parity
import hc_inputs
import hc_inputs.vision as V
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import paper_2112_03444_amd as hc
    return hc


@pytest.fixture(scope="module")
def ctx(hc):
    c = hc.Context(0)
    yield c
    c.close()


def poly2(eq, exps):
    return hc_inputs.PolySystem(n=2, term_eq=np.array(eq, np.int32), term_exp=np.array(exps, np.int32))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("m", [2, 3])
def test_multiple_root(hc, ctx, m, precision):
    """F = (x1^m, x2 - 1): all m paths end SINGULAR_END with cycle number m at
    (0, 1), as in the oracle (degree 2: dense tables; 3: term lists)."""
    S = poly2([0, 1, 1], [[m, 0], [0, 1], [0, 0]])
    c = np.array([[1, 1, -1]], np.complex128)
    g = np.array([np.exp(0.3j)])
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, c, g, opts=hc.default_opts(precision=precision, endgame=1))
    oep, ost, oinfo, ocyc = oracle.track(S, c, g, endgame=True)
    assert (st == hc.HC_T_SINGULAR_END).all(), st
    np.testing.assert_array_equal(st, ost)
    assert (info["cycle"] == m).all() and (ocyc == m).all()
    assert np.max(np.abs(ep[0] - np.array([0.0, 1.0]))) <= 1e-8
    assert _parity.match_one_to_one(ep[0], oep[0]) <= 1e-8
    assert (info["refine_its"] == 0).all()
    # without the end-game no path succeeds
    _, st0, _ = ctx.track(sysh, c, g, opts=hc.default_opts(precision=precision))
    assert not (st0 == hc.HC_T_SUCCESS).any()
    ctx.free_system(sysh)


def test_no_finite_root(hc, ctx):
    """F = (x1 x2 - 1, x1 x2 - 2) has no finite root: the plain tracker stops its
    4 paths at the minimum step, the end-game puts them at infinity."""
    S = poly2([0, 0, 1, 1], [[1, 1], [0, 0], [1, 1], [0, 0]])
    c = np.array([[1, -1, 1, -2]], np.complex128)
    g = np.array([np.exp(0.3j)])
    sysh = ctx.load_system(S)
    _, st0, _ = ctx.track(sysh, c, g)
    assert (st0 != hc.HC_T_SUCCESS).all()
    ep, st, info = ctx.track(sysh, c, g, opts=hc.default_opts(endgame=1))
    _, ost, _, ocyc = oracle.track(S, c, g, endgame=True)
    assert (st == hc.HC_T_AT_INFINITY).all() and (ost == oracle.AT_INFINITY).all()
    assert (info["cycle"] >= 1).all()
    assert np.isnan(info["residual"]).all()
    ctx.free_system(sysh)


@pytest.mark.parametrize("n", [3, 4])
def test_every_path_regular(hc, ctx, n):
    """endgame = 2 sends every path through the end-game: regular roots keep
    cycle number 1 and the plain run's endpoint after the same refinement."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 3, seed=60 + n)
    sysh = ctx.load_system(S)
    ep0, st0, _ = ctx.track(sysh, coef, gam)
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(endgame=2))
    assert (st0 == hc.HC_T_SUCCESS).all() and (st == hc.HC_T_SUCCESS).all()
    assert (info["cycle"] == 1).all()
    err = np.max(np.abs(ep - ep0), axis=-1) / np.maximum(1.0, np.max(np.abs(ep0), axis=-1))
    assert err.max() <= 1e-12
    ctx.free_system(sysh)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_triangulation3_failures_resolved(hc, ctx, precision):
    """3-view triangulation targets (8 instances x 94 paths): the plain tracker
    stops ~6% of the paths at the minimum step on their way to infinity; with
    the end-game, per instance the same numbers of finite solutions and of paths
    at infinity as the oracle's end-game, the finite sets one to one within
    1e-9, and fewer than 2% of the paths unresolved."""
    S = V.triangulation_system(3)
    c0, sols = V.start_instance(3)
    _, coef, _ = V.vision_workload("triang3_batch4096")
    k = 8
    sysh = ctx.load_system(S, kind=hc.HC_PARAMETER)
    ep, st, info = ctx.track(sysh, coef[:k], start=sols, p_start=c0,
                             opts=hc.default_opts(precision=precision, endgame=1))
    oep, ost, _, _ = oracle.track(S, coef[:k], start=sols, coef0=c0, kind=oracle.LINEAR, endgame=True)
    for i in range(k):
        for code in (hc.HC_T_SUCCESS, hc.HC_T_AT_INFINITY, hc.HC_T_SINGULAR_END):
            assert np.sum(st[i] == code) == np.sum(ost[i] == code), (i, code, np.bincount(st[i], minlength=8),
                                                                     np.bincount(ost[i], minlength=8))
        ok = st[i] == hc.HC_T_SUCCESS
        assert _parity.match_one_to_one(ep[i][ok], oep[i][ost[i] == oracle.SUCCESS]) <= 1e-9
        assert np.all(info[i]["residual"][ok] <= 1e-10)
    unresolved = np.isin(st, [hc.HC_T_MIN_STEP, hc.HC_T_MAX_STEPS, hc.HC_T_REFINE_FAILED, hc.HC_T_SINGULAR])
    assert unresolved.mean() < 0.02
    ctx.free_system(sysh)


def test_endgame_rejected_where_unavailable(hc, ctx):
    """The batch call and the no-allocation entry point refuse the end-game."""
    import torch
    S, coef, gam = hc_inputs.dense_quadratic_instances(3, 1, seed=7)
    sysh = ctx.load_system(S)
    dev = torch.device("cuda:0")
    p, g = torch.from_numpy(coef).to(dev), torch.from_numpy(gam).to(dev)
    ep = torch.zeros((1, 8, 3), dtype=torch.complex128, device=dev)
    st = torch.zeros((1, 8), dtype=torch.int32, device=dev)
    o = hc.default_opts(endgame=1)
    with pytest.raises(hc.HcError):
        ctx.track_device(sysh, p, g, ep, st, None, opts=o, noalloc=True)
    with pytest.raises(hc.HcError):
        ctx.track_batch_device([dict(sys=sysh, p_target=p, gamma=g, endpoints=ep, status=st)], opts=o)
    ctx.free_system(sysh)
