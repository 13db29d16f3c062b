"""Parity of the HIP path (through the C ABI) with the CPU oracle, on the GPU.

Parity bar (FP64 mode): per instance the same number of finite solutions as the
oracle and a one-to-one match of the solution sets within 1e-9 relative error
(the tracker may route a path to another root after rounding differences, so the
set is what is unique; per-path agreement is checked as a secondary statistic).
Mixed mode: every finite endpoint has residual <= 1e-10 after FP64 refinement and
the finite solution sets match the FP64 oracle within 1e-9.
"""
import numpy as np
import pytest

import _parity
import hc_inputs
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
    """One-to-one nearest matching of the rows of a (GPU) and b (oracle);
    returns the worst relative distance (inf if the sizes differ)."""
    return _parity.match_one_to_one(a, b)


def finite_set(ep, st, ok):
    return ep[st == ok]


def check_instance_parity(ep_g, st_g, ep_o, st_o, hc, rel=REL):
    fg = finite_set(ep_g, st_g, hc.HC_T_SUCCESS)
    fo = finite_set(ep_o, st_o, oracle.SUCCESS)
    assert len(fg) == len(fo), (np.bincount(st_g, minlength=7), np.bincount(st_o, minlength=7))
    w = rel_match(fg, fo)
    assert w <= rel, w
    return w


def test_config1_single_instance_fp64(hc, ctx):
    S, coef, gam = hc_inputs.workload("dense3_single")
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, coef, gam)
    oep, ost, oinfo = oracle.track(S, coef, gam)
    assert (st == hc.HC_T_SUCCESS).all()
    check_instance_parity(ep[0], st[0], oep[0], ost[0], hc)
    # same start point -> same root, and the same step sequence here
    np.testing.assert_allclose(ep[0], oep[0], rtol=0, atol=1e-12)
    assert (info["steps"] == oinfo["steps"]).all()
    assert (info["rejects"] == oinfo["rejects"]).all()
    assert np.all(info["residual"] <= 1e-13)


@pytest.mark.parametrize("lanes", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_dense_fp64_each_n(hc, ctx, n, lanes):
    """lanes 0: the default layout (a group of 4 or 8 lanes per path, one matrix
    row per lane); lanes 1: one path per lane."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 2, seed=1000 + n)
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(lanes_per_path=lanes))
    oep, ost, oinfo = oracle.track(S, coef, gam)
    for i in range(2):
        check_instance_parity(ep[i], st[i], oep[i], ost[i], hc)
    same = np.max(np.abs(ep - oep), axis=-1) <= 1e-9 * np.maximum(1, np.abs(oep).max(-1))
    assert same.mean() >= 0.95
    ctx.free_system(sysh)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8])
def test_dense_fp64_one_path_per_wavefront(hc, ctx, n):
    """lanes_per_path = 64: one path per wavefront, one Jacobian entry per lane
    (the layout the crossing check's and the end-game's re-tracking use): set
    parity with the oracle, and the same roots as the group layout path by path
    wherever both succeed (same start point, same stage machine)."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 3, seed=1100 + n)
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(lanes_per_path=64))
    ep0, st0, _ = ctx.track(sysh, coef, gam)
    oep, ost, oinfo = oracle.track(S, coef, gam)
    for i in range(3):
        check_instance_parity(ep[i], st[i], oep[i], ost[i], hc)
    both = (st == hc.HC_T_SUCCESS) & (st0 == hc.HC_T_SUCCESS)
    d = np.max(np.abs(ep - ep0), axis=-1) / np.maximum(1.0, np.abs(ep0).max(-1))
    assert d[both].max() <= 1e-9
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-12)
    # the step sequence follows the oracle's (FP64 both, same control)
    assert np.mean(info["steps"] == oinfo["steps"]) >= 0.9
    ctx.free_system(sysh)


def test_one_path_per_wavefront_refused_outside_its_range(hc, ctx):
    S, coef, gam = hc_inputs.dense_quadratic_instances(3, 1, seed=1200)
    sysh = ctx.load_system(S)
    with pytest.raises(hc.HcError):
        ctx.track(sysh, coef, gam, opts=hc.default_opts(lanes_per_path=64, precision="mixed"))
    ctx.free_system(sysh)


@pytest.mark.parametrize("lanes,ir", [(0, 0), (0, 1), (1, 0)])
@pytest.mark.parametrize("n", [3, 6, 8])
def test_mixed_mode_residual_and_sets(hc, ctx, n, lanes, ir):
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 4, seed=2000 + n)
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision="mixed", lanes_per_path=lanes,
                                                                   fp64_residual=ir))
    oep, ost, _ = oracle.track(S, coef, gam)
    ok = st == hc.HC_T_SUCCESS
    assert np.all(info["residual"][ok] <= 1e-10)
    for i in range(4):
        check_instance_parity(ep[i], st[i], oep[i], ost[i], hc)


def test_config2_full_batch_fp64_sampled(hc, ctx):
    """The full 512 x 256 batch in the launch configuration the benchmark times;
    sampled instances are checked against the oracle, every instance against
    Bezout (256 distinct finite roots with tiny residual)."""
    S, coef, gam = hc_inputs.workload("dense8_batch512")
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, coef, gam)
    assert ep.shape == (512, 256, 8)
    frac_ok = (st == hc.HC_T_SUCCESS).mean()
    assert frac_ok >= 0.999, np.bincount(st.ravel(), minlength=7)
    for i in range(512):
        f = ep[i][st[i] == hc.HC_T_SUCCESS]
        d = np.abs(f[:, None, :] - f[None, :, :]).max(-1) + np.eye(len(f)) * 1e9
        assert d.min() > 1e-6
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-12)
    sample = [0, 137, 300, 511]
    oep, ost, _ = oracle.track(S, coef[sample], gam[sample])
    for k, i in enumerate(sample):
        check_instance_parity(ep[i], st[i], oep[k], ost[k], hc)


@pytest.mark.parametrize("ir", [0, 1])
def test_config2_full_batch_mixed_sampled(hc, ctx, ir):
    S, coef, gam = hc_inputs.workload("dense8_batch512")
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision="mixed", fp64_residual=ir))
    ok = st == hc.HC_T_SUCCESS
    assert ok.mean() >= 0.999, np.bincount(st.ravel(), minlength=7)
    assert np.all(info["residual"][ok] <= 1e-10)
    sample = [0, 255, 511]
    oep, ost, _ = oracle.track(S, coef[sample], gam[sample])
    for k, i in enumerate(sample):
        check_instance_parity(ep[i], st[i], oep[k], ost[k], hc)


@pytest.mark.parametrize("lanes", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_chunked_launches_equal_one_shot(hc, ctx, precision, lanes):
    S, coef, gam = hc_inputs.dense_quadratic_instances(6, 3, seed=31)
    sysh = ctx.load_system(S)
    a = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision=precision, lanes_per_path=lanes))
    b = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision=precision, steps_per_launch=7,
                                                        lanes_per_path=lanes))
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])


@pytest.mark.parametrize("lanes", [0, 1])
@pytest.mark.parametrize("tpi", [8, 64, 100, 256])
def test_tracks_per_item_invariance(hc, ctx, tpi, lanes):
    S, coef, gam = hc_inputs.dense_quadratic_instances(8, 2, seed=41)
    sysh = ctx.load_system(S)
    ref = ctx.track(sysh, coef, gam, opts=hc.default_opts(lanes_per_path=lanes))
    got = ctx.track(sysh, coef, gam, opts=hc.default_opts(tracks_per_item=tpi, lanes_per_path=lanes))
    for r, g in zip(ref, got):
        np.testing.assert_array_equal(r, g)


def test_ragged_and_empty(hc, ctx):
    S, coef, gam = hc_inputs.dense_quadratic_instances(7, 3, seed=51)
    sysh = ctx.load_system(S)
    # 100 of the 128 start points: a ragged last work item
    ep, st, info = ctx.track(sysh, coef, gam, n_start=100)
    full, fst, _ = ctx.track(sysh, coef, gam)
    np.testing.assert_array_equal(ep, full[:, :100])
    np.testing.assert_array_equal(st, fst[:, :100])
    # no instances / no paths: nothing to do, no error
    e0, s0, _ = ctx.track(sysh, coef[:0], gam[:0])
    assert e0.shape == (0, 128, 7)
    e1, s1, _ = ctx.track(sysh, coef, gam, n_start=0)
    assert e1.shape == (3, 0, 7)


def test_supplied_start_points_equal_generated(hc, ctx):
    S, coef, gam = hc_inputs.dense_quadratic_instances(5, 2, seed=61)
    sysh = ctx.load_system(S)
    starts = sysh.total_degree_start()
    for b in range(len(starts)):
        np.testing.assert_array_equal(starts[b], oracle.total_degree_start(S, b))
    a = ctx.track(sysh, coef, gam)
    b = ctx.track(sysh, coef, gam, start=starts)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_failure_statuses(hc, ctx):
    S, coef, gam = hc_inputs.dense_quadratic_instances(3, 1, seed=1)
    sysh = ctx.load_system(S)
    bad = coef.copy()
    bad[0, 4] = np.nan
    _, st, _ = ctx.track(sysh, bad, gam)
    assert (st == hc.HC_T_NONFINITE).all()
    _, st, _ = ctx.track(sysh, coef, gam, opts=hc.default_opts(max_steps=1))
    assert (st == hc.HC_T_MAX_STEPS).all()
    _, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(max_newton=0, h_min=0.04))
    assert (st == hc.HC_T_MIN_STEP).all() and (info["rejects"] == 1).all()


def test_path_at_infinity(hc, ctx):
    # F = (x1 x2 - 1, x1 - 2): Bezout 2, one finite root (2, 1/2)
    S = hc_inputs.PolySystem(n=2, term_eq=np.array([0, 0, 1, 1], np.int32),
                             term_exp=np.array([[1, 1], [0, 0], [1, 0], [0, 0]], np.int32))
    c = np.array([[1, -1, 1, -2]], np.complex128)
    g = np.array([np.exp(0.7j)])
    sysh = ctx.load_system(S)
    assert sysh.bezout == 2
    ep, st, _ = ctx.track(sysh, c, g)
    _, ost, _ = oracle.track(S, c, g)
    assert sorted(st[0].tolist()) == sorted(ost[0].tolist()) == [hc.HC_T_SUCCESS, hc.HC_T_AT_INFINITY]
    np.testing.assert_allclose(ep[0][st[0] == 0][0], [2, 0.5], rtol=1e-12)


def test_load_system_errors(hc, ctx):
    assert hc.HC_MAX_N == 32  # the paper's largest Jacobian, 32 x 32 (section 1)
    S33 = hc_inputs.support_system(33, [(1, list(range(33)))] * 33)
    with pytest.raises(hc.HcError):
        ctx.load_system(S33)  # n > HC_MAX_N
    with pytest.raises(hc.HcError):
        ctx.load_system(hc_inputs.dense_quadratic_system(9), layout=hc.HC_LAYOUT_DENSE)  # dense tables: n <= 8
    with pytest.raises(hc.HcError):
        ctx.load_system(hc_inputs.dense_quadratic_system(3), layout=7)
    cubic = hc_inputs.PolySystem(n=1, term_eq=np.array([0], np.int32), term_exp=np.array([[3]], np.int32))
    with pytest.raises(hc.HcError):
        ctx.load_system(cubic)


def test_device_entry_point_matches_host(hc, ctx):
    import torch
    S, coef, gam = hc_inputs.dense_quadratic_instances(6, 4, seed=71)
    sysh = ctx.load_system(S)
    ref = ctx.track(sysh, coef, gam)
    dev = torch.device("cuda:0")
    p = torch.from_numpy(coef).to(dev)
    g = torch.from_numpy(gam).to(dev)
    ep = torch.empty((4, 64, 6), dtype=torch.complex128, device=dev)
    st = torch.empty((4, 64), dtype=torch.int32, device=dev)
    info = torch.empty((4, 64, 32), dtype=torch.uint8, device=dev)
    ctx.track_device(sysh, p, g, ep, st, info)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ep.cpu().numpy(), ref[0])
    np.testing.assert_array_equal(st.cpu().numpy(), ref[1])
    inf = info.cpu().numpy().view(hc.INFO_DTYPE).reshape(4, 64)
    np.testing.assert_array_equal(inf["steps"], ref[2]["steps"])


def test_layouts_agree_on_solution_sets(hc, ctx):
    """The one-path-per-lane and the row-per-lane layouts evaluate and eliminate in
    a different order, so endpoints agree to rounding, not bitwise."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(8, 3, seed=81)
    sysh = ctx.load_system(S)
    a = ctx.track(sysh, coef, gam, opts=hc.default_opts(lanes_per_path=1))
    b = ctx.track(sysh, coef, gam, opts=hc.default_opts(lanes_per_path=8))
    for i in range(3):
        check_instance_parity(a[0][i], a[1][i], b[0][i], b[1][i], hc)


def test_bad_layout_option(hc, ctx):
    S, coef, gam = hc_inputs.dense_quadratic_instances(6, 1, seed=82)
    sysh = ctx.load_system(S)
    with pytest.raises(hc.HcError):
        ctx.track(sysh, coef, gam, opts=hc.default_opts(lanes_per_path=4))  # 4 lanes < 6 rows
    with pytest.raises(hc.HcError):
        ctx.track(sysh, coef, gam, opts=hc.default_opts(lanes_per_path=3))


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_ir"])
@pytest.mark.parametrize("n", [3, 5, 8])
def test_parameter_homotopy(hc, ctx, n, precision):
    """Coefficients interpolated from a solved start instance to two targets
    (section 6): the endpoints are the targets' roots, as the oracle's linear
    homotopy and the total-degree solve of the targets both find."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 3, seed=3000 + n)
    td = ctx.load_system(S)
    ep0, st0, _ = ctx.track(td, coef[:1], gam[:1])
    assert (st0 == hc.HC_T_SUCCESS).all()
    starts = ep0[0]
    ps = ctx.load_system(S, kind=hc.HC_PARAMETER)
    ir = precision == "mixed_ir"
    ep, st, info = ctx.track(ps, coef[1:], start=starts, p_start=coef[0],
                             opts=hc.default_opts(precision="mixed" if ir else precision, fp64_residual=int(ir)))
    oep, ost, _ = oracle.track(S, coef[1:], start=starts, coef0=coef[0], kind=oracle.LINEAR)
    tep, tst, _ = ctx.track(td, coef[1:], gam[1:])
    for i in range(2):
        check_instance_parity(ep[i], st[i], oep[i], ost[i], hc)
        check_instance_parity(ep[i], st[i], tep[i], tst[i], hc)
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)


def test_parameter_homotopy_needs_start(hc, ctx):
    S, coef, gam = hc_inputs.dense_quadratic_instances(4, 2, seed=3100)
    ps = ctx.load_system(S, kind=hc.HC_PARAMETER)
    with pytest.raises(hc.HcError):
        ctx.track(ps, coef[1:], n_start=4)                      # no start points
    with pytest.raises(hc.HcError):
        ctx.track(ps, coef[1:], start=np.ones((4, 4)), p_start=coef[0],
                  opts=hc.default_opts(lanes_per_path=1))    # layout without the blend


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_of_uneven_jobs_equals_single_calls(hc, ctx, precision):
    """One persistent-kernel batch over jobs of different n, kind, path and
    instance counts returns, job by job, what a call on that job alone returns."""
    import torch
    dev = torch.device("cuda:0")
    opts = hc.default_opts(precision=precision)
    specs = [(3, 2, None, 11), (5, 3, 20, 12), (8, 4, None, 13), (6, 1, 50, 14), (2, 5, None, 15)]
    jobs, refs, oracle_in = [], [], []
    for n, n_inst, n_start, seed in specs:
        S, coef, gam = hc_inputs.dense_quadratic_instances(n, n_inst, seed=seed)
        sysh = ctx.load_system(S)
        ns = n_start if n_start is not None else sysh.bezout
        oracle_in.append((S, coef, gam, ns))
        p = torch.from_numpy(coef).to(dev)
        g = torch.from_numpy(gam).to(dev)
        ref = [torch.empty((n_inst, ns, n), dtype=torch.complex128, device=dev),
               torch.empty((n_inst, ns), dtype=torch.int32, device=dev),
               torch.empty((n_inst, ns, 32), dtype=torch.uint8, device=dev)]
        ctx.track_device(sysh, p, g, ref[0], ref[1], ref[2], n_start=ns, opts=opts)
        torch.cuda.synchronize()
        refs.append([r.cpu().numpy() for r in ref])
        jobs.append(dict(sys=sysh, p_target=p, gamma=g, n_start=ns,
                         endpoints=torch.zeros_like(ref[0]), status=torch.zeros_like(ref[1]),
                         info=torch.zeros_like(ref[2])))
    # a parameter-homotopy job: n = 4, start points from a solved instance
    S, coef, gam = hc_inputs.dense_quadratic_instances(4, 3, seed=16)
    td = ctx.load_system(S)
    e0, s0, _ = ctx.track(td, coef[:1], gam[:1])
    ps = ctx.load_system(S, kind=hc.HC_PARAMETER)
    st_pts = torch.from_numpy(np.ascontiguousarray(e0[0])).to(dev)
    p = torch.from_numpy(coef[1:]).to(dev)
    p0 = torch.from_numpy(coef[0]).to(dev)
    ref = [torch.empty((2, 16, 4), dtype=torch.complex128, device=dev),
           torch.empty((2, 16), dtype=torch.int32, device=dev),
           torch.empty((2, 16, 32), dtype=torch.uint8, device=dev)]
    ctx.track_device(ps, p, None, ref[0], ref[1], ref[2], start=st_pts, p_start=p0, opts=opts)
    torch.cuda.synchronize()
    refs.append([r.cpu().numpy() for r in ref])
    jobs.append(dict(sys=ps, p_target=p, start=st_pts, p_start=p0, endpoints=torch.zeros_like(ref[0]),
                     status=torch.zeros_like(ref[1]), info=torch.zeros_like(ref[2])))

    ctx.track_batch_device(jobs, opts=opts)
    torch.cuda.synchronize()
    for j, r in zip(jobs, refs):
        np.testing.assert_array_equal(j["endpoints"].cpu().numpy(), r[0])
        np.testing.assert_array_equal(j["status"].cpu().numpy(), r[1])
        np.testing.assert_array_equal(j["info"].cpu().numpy(), r[2])
    # and every job against the oracle, instance by instance (the same start
    # points: the first n_start total-degree points, or the solved instance's roots)
    for j, (Sj, cj, gj, ns) in zip(jobs, oracle_in):
        starts = np.stack([oracle.total_degree_start(Sj, b) for b in range(ns)])
        oep, ost, _ = oracle.track(Sj, cj, gj, start=starts)
        ep_j, st_j = j["endpoints"].cpu().numpy(), j["status"].cpu().numpy()
        for i in range(len(cj)):
            check_instance_parity(ep_j[i], st_j[i], oep[i], ost[i], hc)
    oep, ost, _ = oracle.track(S, coef[1:], start=e0[0], coef0=coef[0], kind=oracle.LINEAR)
    for i in range(2):
        check_instance_parity(jobs[-1]["endpoints"].cpu().numpy()[i], jobs[-1]["status"].cpu().numpy()[i],
                              oep[i], ost[i], hc)


def test_batch_rejects_unsupported(hc, ctx):
    import torch
    S, coef, gam = hc_inputs.dense_quadratic_instances(1, 1, seed=17)
    s1 = ctx.load_system(S)
    dev = torch.device("cuda:0")
    job = dict(sys=s1, p_target=torch.from_numpy(coef).to(dev),
               endpoints=torch.zeros((1, 2, 1), dtype=torch.complex128, device=dev),
               status=torch.zeros((1, 2), dtype=torch.int32, device=dev))
    with pytest.raises(hc.HcError):
        ctx.track_batch_device([job])  # n = 1 has no group layout
    ctx.track_batch_device([])          # an empty batch is a no-op


def test_graph_replay_matches_eager(hc, ctx):
    """A captured launch sequence, replayed several times with eager work and
    synchronisations in between and with the inputs changed in place, gives the
    eager results every time."""
    import torch
    dev = torch.device("cuda:0")
    S, coef, gam = hc_inputs.dense_quadratic_instances(6, 4, seed=91)
    _, coef2, _ = hc_inputs.dense_quadratic_instances(6, 4, seed=92)
    sysh = ctx.load_system(S)
    stream = torch.cuda.Stream()
    p = torch.from_numpy(coef).to(dev)
    g = torch.from_numpy(gam).to(dev)
    ep = torch.zeros((4, 64, 6), dtype=torch.complex128, device=dev)
    st = torch.zeros((4, 64), dtype=torch.int32, device=dev)
    for precision in ("mixed", "fp64"):
        og = hc.default_opts(precision=precision, use_graph=1)
        for rep in range(4):
            src = coef if rep % 2 == 0 else coef2
            p.copy_(torch.from_numpy(src))
            torch.cuda.synchronize()
            ctx.track_device(sysh, p, g, ep, st, None, opts=og, stream=stream)
            stream.synchronize()
            got = (ep.cpu().numpy(), st.cpu().numpy())
            ep.zero_()                      # eager work between replays
            ref = ctx.track(sysh, src, gam, opts=hc.default_opts(precision=precision))
            np.testing.assert_array_equal(got[0], ref[0])
            np.testing.assert_array_equal(got[1], ref[1])


def test_autotune_choice_is_used_and_exact(hc, ctx):
    import torch
    dev = torch.device("cuda:0")
    S, coef, gam = hc_inputs.dense_quadratic_instances(5, 8, seed=93)
    sysh = ctx.load_system(S)
    p = torch.from_numpy(coef).to(dev)
    g = torch.from_numpy(gam).to(dev)
    ep = torch.zeros((8, 32, 5), dtype=torch.complex128, device=dev)
    st = torch.zeros((8, 32), dtype=torch.int32, device=dev)
    best = ctx.autotune(sysh, p, g, ep, st, opts=hc.default_opts(precision="mixed"))
    assert best.lanes_per_path in (1, 8) and best.tracks_per_item >= 1
    explicit = ctx.track(sysh, coef, gam, opts=hc.default_opts(
        precision="mixed", lanes_per_path=best.lanes_per_path, tracks_per_item=best.tracks_per_item))
    auto = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision="mixed"))
    for a, b in zip(explicit, auto):
        np.testing.assert_array_equal(a, b)
