"""Parity of the term-list layout (section 6 term tables, n <= 16) with the CPU
oracle, on the GPU, through the C ABI.

Bar as in test_gpu_parity: per instance the same number of finite solutions as
the oracle and a one-to-one match of the solution sets within 1e-9 relative
error in FP64 mode; in mixed mode additionally every finite endpoint has
residual <= 1e-10 after the FP64 refinement.
"""
import numpy as np
import pytest

import hc_inputs
import hc_inputs.vision as V
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


def rel_match(a, b):
    """Greedy one-to-one nearest matching of the rows of a onto the rows of b;
    returns the worst relative distance (inf if the sizes differ)."""
    if len(a) != len(b):
        return np.inf
    b = list(b)
    worst = 0.0
    for p in a:
        d = [np.max(np.abs(p - q)) / max(1.0, np.max(np.abs(q))) for q in b]
        j = int(np.argmin(d))
        worst = max(worst, d[j])
        b.pop(j)
    return worst


def check_instance_parity(ep_g, st_g, ep_o, st_o, hc, rel=REL):
    fg = ep_g[st_g == hc.HC_T_SUCCESS]
    fo = ep_o[st_o == oracle.SUCCESS]
    assert len(fg) == len(fo), (np.bincount(st_g, minlength=7), np.bincount(st_o, minlength=7))
    w = rel_match(fg, fo)
    assert w <= rel, w
    return w


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [3, 6, 8])
def test_terms_equal_dense_tables_and_oracle(hc, ctx, n, precision):
    """The same dense quadratic systems through both table layouts: each matches
    the oracle, so the two evaluators compute the same homotopy."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 3, seed=5000 + n)
    o = hc.default_opts(precision=precision)
    dense = ctx.load_system(S, layout=hc.HC_LAYOUT_DENSE)
    terms = ctx.load_system(S, layout=hc.HC_LAYOUT_TERMS)
    epd, std, _ = ctx.track(dense, coef, gam, opts=o)
    ept, stt, infot = ctx.track(terms, coef, gam, opts=o)
    oep, ost, _ = oracle.track(S, coef, gam)
    for i in range(3):
        check_instance_parity(ept[i], stt[i], oep[i], ost[i], hc)
        check_instance_parity(epd[i], std[i], oep[i], ost[i], hc)
    assert np.all(infot["residual"][stt == hc.HC_T_SUCCESS] <= 1e-10)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [9, 10])
def test_dense_quadratic_above_eight_unknowns(hc, ctx, n, precision):
    """n = 9 and 10 total-degree systems (512 and 1024 paths, the serving mix's
    largest dense requests) run on the term lists."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 1, seed=5100 + n)
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision=precision))
    oep, ost, _ = oracle.track(S, coef, gam)
    check_instance_parity(ep[0], st[0], oep[0], ost[0], hc)
    assert (st == hc.HC_T_SUCCESS).mean() >= 0.99
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)


@pytest.fixture(scope="module")
def triang(hc, ctx):
    S = V.triangulation_system()
    c0, sols = V.start_instance()
    ps = ctx.load_system(S, kind=hc.HC_PARAMETER)
    return S, c0, sols, ps


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_triangulation_parity(hc, ctx, triang, precision):
    """4-view triangulation from the monodromy start set (296 paths) to 3 scenes."""
    S, c0, sols, ps = triang
    _, coef, _ = V.triangulation_instances(3, seed=5200)
    ep, st, info = ctx.track(ps, coef, start=sols, p_start=c0, opts=hc.default_opts(precision=precision))
    oep, ost, _ = oracle.track(S, coef, start=sols, coef0=c0, kind=oracle.LINEAR)
    for i in range(3):
        check_instance_parity(ep[i], st[i], oep[i], ost[i], hc)
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)


def check_paths_where_both_succeed(ep_g, st_g, res_g, ep_o, st_o, hc, rel=REL, max_frac=0.01):
    """Path-by-path parity for a mode whose failures need not coincide with the
    oracle's: both sides start path b at the same point, so where both succeed
    they reach the same root (within rel); where only one succeeds, its root is
    a valid root (residual <= 1e-10) distinct from every other success of that
    side; the status disagrees on at most max_frac of the paths."""
    both = (st_g == hc.HC_T_SUCCESS) & (st_o == oracle.SUCCESS)
    for b in np.flatnonzero(both):
        d = np.max(np.abs(ep_g[b] - ep_o[b])) / max(1.0, np.max(np.abs(ep_o[b])))
        assert d <= rel, (b, d)
    only_g = (st_g == hc.HC_T_SUCCESS) & ~both
    only_o = (st_o == oracle.SUCCESS) & ~both
    assert only_g.sum() + only_o.sum() <= max_frac * len(st_g)
    assert np.all(res_g[only_g] <= 1e-10)
    for ep, st, only in ((ep_g, st_g == hc.HC_T_SUCCESS, only_g), (ep_o, st_o == oracle.SUCCESS, only_o)):
        ok = ep[st]
        for b in np.flatnonzero(only):
            d = np.max(np.abs(ok - ep[b]), axis=1) / np.maximum(1.0, np.max(np.abs(ep[b])))
            assert np.sum(d <= 1e-8) == 1, b  # only itself


def test_triangulation_fp64_residual(hc, ctx, triang):
    """Mixed mode with the FP64 Newton right-hand side from the FP64 tables
    (fp64_residual) on the quadratic term lists, parameter homotopy.  The FP64
    right-hand side changes which ill-conditioned paths end at the minimum step,
    so the comparison is path by path (check_paths_where_both_succeed)."""
    S, c0, sols, ps = triang
    _, coef, _ = V.triangulation_instances(2, seed=5250)
    ep, st, info = ctx.track(ps, coef, start=sols, p_start=c0,
                             opts=hc.default_opts(precision="mixed", fp64_residual=1))
    oep, ost, _ = oracle.track(S, coef, start=sols, coef0=c0, kind=oracle.LINEAR)
    for i in range(2):
        check_paths_where_both_succeed(ep[i], st[i], info["residual"][i], oep[i], ost[i], hc)
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)


def test_triangulation_full_batch_sampled(hc, ctx, triang):
    """The full 4096-instance batch (1,212,416 paths) in mixed mode, as the
    benchmark runs it; sampled instances against the oracle, every instance's
    finite endpoints against the KKT residual bound and distinctness."""
    S, c0, sols, ps = triang
    _, coef, _ = V.vision_workload("triang4_batch4096")
    ep, st, info = ctx.track(ps, coef, start=sols, p_start=c0, opts=hc.default_opts(precision="mixed"))
    assert ep.shape == (4096, 296, 14)
    ok = st == hc.HC_T_SUCCESS
    assert np.all(info["residual"][ok] <= 1e-10)
    assert ok.sum(axis=1).min() >= 200
    for i in range(0, 4096, 512):
        f = ep[i][ok[i]]
        d = np.abs(f[:, None, :] - f[None, :, :]).max(-1) + np.eye(len(f)) * 1e9
        assert d.min() > 1e-6
    sample = [0, 2047, 4095]
    oep, ost, _ = oracle.track(S, coef[sample], start=sols, coef0=c0, kind=oracle.LINEAR)
    for k, i in enumerate(sample):
        check_instance_parity(ep[i], st[i], oep[k], ost[k], hc)


@pytest.fixture(scope="module")
def triang3(hc, ctx):
    S = V.triangulation_system(3)
    c0, sols = V.start_instance(3)
    ps = ctx.load_system(S, kind=hc.HC_PARAMETER)
    return S, c0, sols, ps


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_triangulation3_parity(hc, ctx, triang3, precision):
    """3-view triangulation (n = 9) from its 94-solution monodromy start set to
    4 scenes: set parity with equal finite counts in both precisions.  ~6% of
    these paths head for infinity and stop at the minimum step short of the
    bound on |x|; in mixed mode which of them get there first depends on the FP32
    part of the path, so mixed mode runs with the end-game on both sides, which
    classifies them at infinity (path-by-path agreement is checked as well)."""
    S, c0, sols, ps = triang3
    _, coef, _ = V.triangulation_instances(4, seed=5600, n_views=3)
    eg = 1 if precision == "mixed" else 0
    ep, st, info = ctx.track(ps, coef, start=sols, p_start=c0, opts=hc.default_opts(precision=precision, endgame=eg))
    if eg:
        oep, ost, _, _ = oracle.track(S, coef, start=sols, coef0=c0, kind=oracle.LINEAR, endgame=True)
    else:
        oep, ost, _ = oracle.track(S, coef, start=sols, coef0=c0, kind=oracle.LINEAR)
    for i in range(4):
        check_instance_parity(ep[i], st[i], oep[i], ost[i], hc)
        check_paths_where_both_succeed(ep[i], st[i], info["residual"][i], oep[i], ost[i], hc, max_frac=2.5 / 94)
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)


def test_triangulation3_full_batch_sampled(hc, ctx, triang3):
    """The 4096-instance 3-view batch (385,024 paths) in mixed mode, as the
    benchmark runs it; sampled instances against the oracle, every finite
    endpoint's residual, distinctness on a sample."""
    S, c0, sols, ps = triang3
    _, coef, _ = V.vision_workload("triang3_batch4096")
    ep, st, info = ctx.track(ps, coef, start=sols, p_start=c0, opts=hc.default_opts(precision="mixed"))
    assert ep.shape == (4096, 94, 9)
    ok = st == hc.HC_T_SUCCESS
    assert np.all(info["residual"][ok] <= 1e-10)
    assert ok.sum(axis=1).min() >= 60
    for i in range(0, 4096, 512):
        f = ep[i][ok[i]]
        d = np.abs(f[:, None, :] - f[None, :, :]).max(-1) + np.eye(len(f)) * 1e9
        assert d.min() > 1e-6
    sample = [0, 2047, 4095]
    oep, ost, _ = oracle.track(S, coef[sample], start=sols, coef0=c0, kind=oracle.LINEAR)
    for k, i in enumerate(sample):
        check_instance_parity(ep[i], st[i], oep[k], ost[k], hc)


def test_terms_chunked_launches_equal_one_shot(hc, ctx, triang):
    S, c0, sols, ps = triang
    _, coef, _ = V.triangulation_instances(2, seed=5300)
    a = ctx.track(ps, coef, start=sols, p_start=c0, opts=hc.default_opts(precision="mixed"))
    b = ctx.track(ps, coef, start=sols, p_start=c0, opts=hc.default_opts(precision="mixed", steps_per_launch=7))
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])


def test_terms_rejects_lane_layouts(hc, ctx, triang):
    S, c0, sols, ps = triang
    _, coef, _ = V.triangulation_instances(1, seed=5400)
    for lanes in (1, 8):
        with pytest.raises(hc.HcError):
            ctx.track(ps, coef, start=sols, p_start=c0, opts=hc.default_opts(lanes_per_path=lanes))
