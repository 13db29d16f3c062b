"""Serving loop (hc_server_*): continuous batching of solve requests.

A request's results must be bitwise those of tracking it alone with the same
options, whatever else shares its batch or the device."""
import numpy as np
import pytest

import hc_inputs

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


def _mix(rng, n_req):
    out = []
    for k in range(n_req):
        n = int(rng.integers(3, 9))
        n_inst = int(rng.integers(1, 4))
        out.append((n, n_inst, 5000 + k))
    return out


def test_alone_equals_in_the_mix(hc, ctx):
    opts = hc.default_opts(precision="mixed")
    systems = {n: ctx.load_system(hc_inputs.dense_quadratic_system(n)) for n in range(3, 9)}
    srv = hc.Server(ctx, max_inflight=3, max_batch_requests=16, opts=opts)
    # the probe request alone
    S, coef, gam = hc_inputs.dense_quadratic_instances(6, 2, seed=4242)
    t = srv.submit(systems[6], coef, gam, with_info=True)
    alone = srv.wait(t)
    # the same request in a stream of others of uneven n and size
    rng = np.random.default_rng(7)
    tickets = []
    for k, (n, n_inst, seed) in enumerate(_mix(rng, 40)):
        _, c2, g2 = hc_inputs.dense_quadratic_instances(n, n_inst, seed=seed)
        tickets.append((n, c2, g2, srv.submit(systems[n], c2, g2)))
        if k == 20:
            probe = srv.submit(systems[6], coef, gam, with_info=True)
    mixed = srv.wait(probe)
    for a, b in zip(alone, mixed):
        np.testing.assert_array_equal(a, b)
    # and every request equals its own single call
    for n, c2, g2, tk in tickets:
        ep, st, _ = srv.wait(tk)
        rep, rst, _ = ctx.track(systems[n], c2, g2, opts=opts)
        np.testing.assert_array_equal(ep, rep)
        np.testing.assert_array_equal(st, rst)
    stats = srv.stats()
    assert stats["completed"] == 42 and stats["latencies"] == 42
    assert 0 < stats["p50_ms"] <= stats["p99_ms"] <= stats["max_ms"]
    srv.close()


def test_vision_and_large_requests_in_the_mix(hc, ctx):
    """Term-list requests (4-view triangulation parameter homotopies with their
    start points, n = 10 total degree) interleaved with dense n = 8 requests:
    each result equals the same request tracked alone."""
    import hc_inputs.vision as V
    opts = hc.default_opts(precision="mixed")
    tri = ctx.load_system(V.triangulation_system(), kind=hc.HC_PARAMETER)
    c0, sols = V.start_instance()
    _, tcoef, _ = V.triangulation_instances(4, seed=6100)
    s8 = ctx.load_system(hc_inputs.dense_quadratic_system(8))
    s10 = ctx.load_system(hc_inputs.dense_quadratic_system(10))
    srv = hc.Server(ctx, max_inflight=3, max_batch_requests=8, opts=opts)
    reqs = []
    for k in range(4):
        reqs.append(("tri", tcoef[k:k + 1], srv.submit(tri, tcoef[k:k + 1], start=sols, p_start=c0)))
        _, c8, g8 = hc_inputs.dense_quadratic_instances(8, 1, seed=6200 + k)
        reqs.append(("d8", (c8, g8), srv.submit(s8, c8, g8)))
    _, c10, g10 = hc_inputs.dense_quadratic_instances(10, 1, seed=6300)
    reqs.append(("d10", (c10, g10), srv.submit(s10, c10, g10)))
    for kind, data, t in reqs:
        ep, st, _ = srv.wait(t)
        if kind == "tri":
            rep, rst, _ = ctx.track(tri, data, start=sols, p_start=c0, opts=opts)
        else:
            rep, rst, _ = ctx.track(s8 if kind == "d8" else s10, data[0], data[1], opts=opts)
        np.testing.assert_array_equal(ep, rep)
        np.testing.assert_array_equal(st, rst)
    srv.close()


def test_resident_start_set_requests_equal_copied_ones(hc, ctx):
    """Triangulation requests that name a start set kept on the device give,
    request by request, what the same requests with copied start points give,
    and the oracle's roots; a set is refused for another system or with start
    points in the request."""
    import _parity
    import oracle
    import hc_inputs.vision as V
    opts = hc.default_opts(precision="mixed")
    S = V.triangulation_system()
    tri = ctx.load_system(S, kind=hc.HC_PARAMETER)
    c0, sols = V.start_instance()
    _, tcoef, _ = V.triangulation_instances(3, seed=6400)
    srv = hc.Server(ctx, max_inflight=2, max_batch_requests=4, opts=opts)
    rs = srv.add_start_set(tri, sols, p_start=c0)
    a = [srv.submit(tri, tcoef[k:k + 1], start_set=rs) for k in range(3)]
    b = [srv.submit(tri, tcoef[k:k + 1], start=sols, p_start=c0) for k in range(3)]
    oep, ost, _ = oracle.track(S, tcoef, start=sols, coef0=c0, kind=oracle.LINEAR)
    for k in range(3):
        ea, sa, _ = srv.wait(a[k])
        eb, sb, _ = srv.wait(b[k])
        np.testing.assert_array_equal(ea, eb)
        np.testing.assert_array_equal(sa, sb)
        _parity.check_sets(ea[0], sa[0], oep[k], ost[k], hc.HC_T_SUCCESS)
    s8 = ctx.load_system(hc_inputs.dense_quadratic_system(8))
    with pytest.raises(hc.HcError):
        srv.submit(s8, np.ones((1, 360)), start_set=rs)
    with pytest.raises(hc.HcError):
        srv.submit(tri, tcoef[:1], start=sols, start_set=rs)
    srv.close()


def test_tight_budget_still_completes(hc, ctx):
    opts = hc.default_opts(precision="fp64")
    sysh = ctx.load_system(hc_inputs.dense_quadratic_system(7))
    # each request needs ~114 KB of device memory: a 150 KB budget admits one at a time
    srv = hc.Server(ctx, max_inflight=2, max_batch_requests=4, hbm_budget=150 << 10, opts=opts)
    ts = []
    for k in range(6):
        _, c, g = hc_inputs.dense_quadratic_instances(7, 2, seed=6000 + k)
        ts.append((c, g, srv.submit(sysh, c, g)))
    for c, g, t in ts:
        ep, st, _ = srv.wait(t)
        rep, rst, _ = ctx.track(sysh, c, g, opts=opts)
        np.testing.assert_array_equal(ep, rep)
    st = srv.stats()
    assert st["batches"] == 6
    assert 0 < st["peak_bytes"] <= 150 << 10
    srv.close()


def test_server_rejects_bad_requests(hc, ctx):
    s1 = ctx.load_system(hc_inputs.dense_quadratic_system(1))
    srv = hc.Server(ctx)
    with pytest.raises(hc.HcError):
        srv.submit(s1, np.ones((1, 3)))
    s4 = ctx.load_system(hc_inputs.dense_quadratic_system(4))
    with pytest.raises(hc.HcError):
        srv.submit(s4, np.ones((1, 60)), n_start=17)  # more paths than the Bezout number
    srv.close()
