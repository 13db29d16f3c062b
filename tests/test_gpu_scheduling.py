"""Scheduling pieces on the GPU through the C ABI: the crossing check of
instances above the LDS capacity (8192 paths), the autotuner (its choices keyed
by workload shape, persisted to a file, over table layouts and steps per
launch) and hipGraph replay of the multi-job batch entry point."""
import os

import numpy as np
import pytest

import _parity
import hc_inputs
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


@pytest.mark.parametrize("n_start", [4000, 9000])
def test_crossing_check_marks_duplicates_in_large_instances(hc, ctx, n_start):
    """Mixed precision, n = 14 dense quadratics (term lists), start points =
    the first n_start total-degree points with path 1 started at path 0's
    point: both end on one root, so the crossing check (in LDS below 8192
    paths, through global memory above) re-tracks both in FP64; no other path
    is restarted unless it met another path's root."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(14, 1, seed=8800)
    sysh = ctx.load_system(S)
    starts = sysh.total_degree_start(0, n_start)
    starts[1] = starts[0]
    ep, st, info = ctx.track(sysh, coef, gam, start=starts, opts=hc.default_opts(precision="mixed"))
    assert st[0, 0] == st[0, 1] == hc.HC_T_SUCCESS
    np.testing.assert_array_equal(ep[0, 0], ep[0, 1])
    assert info["escalated"][0, 0] == info["escalated"][0, 1] == 1
    # the restarted paths are few: the duplicate pair and genuine crossings
    assert info["escalated"][0].sum() <= 2 + 0.01 * n_start
    # the finite roots other than the planted duplicate are pairwise distinct
    ok = ep[0][st[0] == hc.HC_T_SUCCESS][1:]
    from scipy.spatial import cKDTree
    emb = np.concatenate([ok.real, ok.imag], axis=1)
    d, _ = cKDTree(emb).query(emb, k=2, p=np.inf)
    assert np.all(d[:, 1] > 1e-6)
    # the FP64 run reaches the same set of roots
    e64, s64, _ = ctx.track(sysh, coef, gam, start=starts)
    _parity.check_sets(ep[0][1:], st[0][1:], e64[0][1:], s64[0][1:], hc.HC_T_SUCCESS, 1e-9)


def test_autotune_choice_is_keyed_by_shape_not_address(hc, ctx):
    """A choice made for one system applies to another system of the same
    shape, never to a system of another shape loaded after the first was freed
    (possibly at the same address)."""
    import torch
    dev = torch.device("cuda:0")
    S5, coef5, gam5 = hc_inputs.dense_quadratic_instances(5, 8, seed=8801)
    s5 = ctx.load_system(S5)
    p = torch.from_numpy(coef5).to(dev)
    g = torch.from_numpy(gam5).to(dev)
    ep = torch.zeros((8, 32, 5), dtype=torch.complex128, device=dev)
    st = torch.zeros((8, 32), dtype=torch.int32, device=dev)
    best = ctx.autotune(s5, p, g, ep, st, opts=hc.default_opts(precision="mixed"))
    assert best.lanes_per_path in (1, 8, 16) and best.tracks_per_item >= 1
    assert best.table_layout in (hc.HC_LAYOUT_DENSE, hc.HC_LAYOUT_TERMS)
    ctx.free_system(s5)
    # another shape: n = 6 runs with its defaults and matches the oracle
    S6, coef6, gam6 = hc_inputs.dense_quadratic_instances(6, 2, seed=8802)
    s6 = ctx.load_system(S6)
    ep6, st6, _ = ctx.track(s6, coef6, gam6, opts=hc.default_opts(precision="mixed"))
    oep, ost, _ = oracle.track(S6, coef6, gam6)
    for i in range(2):
        _parity.check_sets(ep6[i], st6[i], oep[i], ost[i], hc.HC_T_SUCCESS)
    # the same shape again: the tuned choice applies and equals the explicit one
    s5b = ctx.load_system(S5)
    auto = ctx.track(s5b, coef5, gam5, opts=hc.default_opts(precision="mixed"))
    explicit = ctx.track(s5b, coef5, gam5, opts=hc.default_opts(
        precision="mixed", lanes_per_path=best.lanes_per_path, tracks_per_item=best.tracks_per_item,
        table_layout=best.table_layout))
    for a, b in zip(auto, explicit):
        np.testing.assert_array_equal(a, b)


def test_table_layout_option_gives_the_same_roots(hc, ctx):
    """A dense-table system tracked on its term-list copy (table_layout) reaches
    the oracle's roots; a layout that cannot hold the system is refused."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(6, 3, seed=8803)
    sysh = ctx.load_system(S)
    oep, ost, _ = oracle.track(S, coef, gam)
    for lay in (hc.HC_LAYOUT_DENSE, hc.HC_LAYOUT_TERMS):
        for prec in ("fp64", "mixed"):
            ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision=prec, table_layout=lay))
            for i in range(3):
                _parity.check_sets(ep[i], st[i], oep[i], ost[i], hc.HC_T_SUCCESS)
    S9, coef9, gam9 = hc_inputs.dense_quadratic_instances(9, 1, seed=8804)
    s9 = ctx.load_system(S9)
    with pytest.raises(hc.HcError):
        ctx.track(s9, coef9, gam9, n_start=4, opts=hc.default_opts(table_layout=hc.HC_LAYOUT_DENSE))


def test_autotune_cache_file_round_trip(hc, ctx, tmp_path):
    """hc_tune_save writes the choices (steps per launch tuned too); a fresh
    context loads them and its calls take the tuned decomposition, whose results
    equal the explicit one's; a malformed file is refused."""
    import torch
    dev = torch.device("cuda:0")
    S, coef, gam = hc_inputs.dense_quadratic_instances(4, 16, seed=8805)
    sysh = ctx.load_system(S)
    p = torch.from_numpy(coef).to(dev)
    g = torch.from_numpy(gam).to(dev)
    ep = torch.zeros((16, 16, 4), dtype=torch.complex128, device=dev)
    st = torch.zeros((16, 16), dtype=torch.int32, device=dev)
    best = ctx.autotune(sysh, p, g, ep, st, opts=hc.default_opts(precision="fp64", steps_per_launch=-1))
    assert best.steps_per_launch in (0, 64, 512)
    path = str(tmp_path / "tune.txt")
    ctx.tune_save(path)
    text = open(path).read()
    assert "n=4" in text and " -> " in text
    c2 = hc.Context(0)
    try:
        assert c2.tune_load(path) >= 1
        s2 = c2.load_system(S)
        auto = c2.track(s2, coef, gam, opts=hc.default_opts(precision="fp64", steps_per_launch=-1))
        explicit = c2.track(s2, coef, gam, opts=hc.default_opts(
            precision="fp64", lanes_per_path=best.lanes_per_path, tracks_per_item=best.tracks_per_item,
            steps_per_launch=best.steps_per_launch, table_layout=best.table_layout))
        for a, b in zip(auto, explicit):
            np.testing.assert_array_equal(a, b)
        bad = tmp_path / "bad.txt"
        bad.write_text("not a tuning line\n")
        with pytest.raises(hc.HcError):
            c2.tune_load(str(bad))
    finally:
        c2.close()


def test_batch_graph_replay_matches_eager(hc, ctx):
    """hc_track_batch_device with use_graph: the first call captures, later calls
    replay; with the inputs changed in place between replays (and eager work in
    between), every replay equals an eager batch on the same inputs."""
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    specs = [(3, 2, 21), (5, 3, 22), (8, 2, 23)]
    jobs, alts, bufs = [], [], []
    for n, n_inst, seed in specs:
        S, coef, gam = hc_inputs.dense_quadratic_instances(n, n_inst, seed=seed)
        _, coef2, _ = hc_inputs.dense_quadratic_instances(n, n_inst, seed=seed + 100)
        sysh = ctx.load_system(S)
        p = torch.from_numpy(coef).to(dev)
        jobs.append(dict(sys=sysh, p_target=p, gamma=torch.from_numpy(gam).to(dev),
                         endpoints=torch.zeros((n_inst, 2 ** n, n), dtype=torch.complex128, device=dev),
                         status=torch.zeros((n_inst, 2 ** n), dtype=torch.int32, device=dev)))
        alts.append((coef, coef2))
    for precision in ("mixed", "fp64"):
        og = hc.default_opts(precision=precision, use_graph=1)
        oe = hc.default_opts(precision=precision)
        for rep in range(4):
            for j, (c1, c2) in zip(jobs, alts):
                j["p_target"].copy_(torch.from_numpy(c1 if rep % 2 == 0 else c2))
            torch.cuda.synchronize()
            ctx.track_batch_device(jobs, opts=og, stream=stream)
            stream.synchronize()
            got = [(j["endpoints"].cpu().numpy(), j["status"].cpu().numpy()) for j in jobs]
            for j in jobs:
                j["endpoints"].zero_()
            ctx.track_batch_device(jobs, opts=oe)
            torch.cuda.synchronize()
            for (ge, gs), j in zip(got, jobs):
                np.testing.assert_array_equal(ge, j["endpoints"].cpu().numpy())
                np.testing.assert_array_equal(gs, j["status"].cpu().numpy())
